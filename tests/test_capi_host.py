"""C-ABI checks that need no GPU: the library loads, exports every function
``include/fuglbm.h`` declares, and its host-only logic (lattice-unit
constants, argument validation, buffer sizes) agrees with the oracle."""
import os
import re

import numpy as np
import pytest

from inputs import components as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fuglbm.h")


def _capi():
    from paper_2306_10652_amd import capi
    if not os.path.exists(capi.LIB_PATH):
        from paper_2306_10652_amd.build import build_library
        build_library(verbose=False)
    return capi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fuglbm_[a-z_]+)\s*\(", text)))


def test_header_and_library_export_the_same_functions():
    capi = _capi()
    L = capi.lib()
    names = declared_functions()
    assert names == sorted(capi.EXPORTED)
    for n in names:
        assert hasattr(L, n), n


def test_header_is_plain_c(tmp_path):
    """The boundary is a C ABI: the header compiles as strict C99 (no C++
    constructs, no torch or HIP types) and declares every entry point with
    C linkage for a C++ caller."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include "fuglbm.h"\nint main(void) { fuglbm_diag d; '
                   'const char *(*f)(void) = fuglbm_last_error; (void)d; return f == 0; }\n')
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                        "-I", os.path.dirname(HEADER), "-c", str(src), "-o",
                        str(tmp_path / "use.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    text = open(HEADER).read()
    assert 'extern "C"' in text and "hip" not in re.sub(r"/\*.*?\*/", "", text, flags=re.S).replace(
        "hip_stream", "")


# heavy pseudo-components: PR's alpha branch for omega > 0.49, and the
# split itself (omega = 0.49 takes the first branch on both sides)
HEAVY = [C.TABLE_I["C1"], C.Component("h049", 600.0, 20.0, 0.49, 180.0),
         C.Component("h0491", 610.0, 19.0, 0.4901, 185.0),
         C.Component("h06", 650.0, 17.0, 0.6, 220.0),
         C.Component("h08", 720.0, 14.0, 0.8, 300.0),
         C.Component("h10", 800.0, 12.0, 1.0, 400.0)]


@pytest.mark.parametrize("comps,T,kij_seed", [
    (C.DROPLET_3, 250.0, None),
    (C.N_ALKANES, 325.0, 4),
    ([C.TABLE_I["C1"]], 177.24, None),
    (HEAVY, 450.0, 7),
])
@pytest.mark.parametrize("eos", ["PR", "SRK", "vdW"])
def test_lattice_constants_match_oracle_units(comps, T, kij_seed, eos):
    """The library's own unit conversion (Section III.A anchors, Eq. (6)-(8)
    kappa, alpha(T)) reproduces the oracle's, independently written, for
    each cubic."""
    capi = _capi()
    from inputs.fields import draw_kij
    from oracle.lbm import oracle_mixture
    kij = None if kij_seed is None else draw_kij(len(comps), 0.0, 0.05, kij_seed)
    mix = capi.Mixture.from_components(comps, T, kij, kappa_ref=0.03, tau=0.8, eos=eos)
    om = oracle_mixture(comps, T, kij, kappa_ref=0.03, tau=0.8, eos=eos)
    np.testing.assert_allclose(mix.lattice_constants(), om.lattice_constants(), rtol=1e-13,
                               atol=0)


def test_lattice_constants_with_other_anchors_match_oracle():
    """The three-phase case's own anchors (Section III.D: a_C1 = 0.011550,
    b_C1 = 0.107781, R = 1) and k_ij: the library and the oracle agree."""
    capi = _capi()
    from oracle.lbm import oracle_mixture
    kij = np.array(C.three_phase_kij())
    mix = capi.Mixture.from_components(C.THREE_PHASE, C.THREE_PHASE_T_K, kij,
                                       a_ref=C.THREE_PHASE_A_LU, b_ref=C.THREE_PHASE_B_LU)
    om = oracle_mixture(C.THREE_PHASE, C.THREE_PHASE_T_K, kij, a_lu=C.THREE_PHASE_A_LU,
                        b_lu=C.THREE_PHASE_B_LU)
    np.testing.assert_allclose(mix.lattice_constants(), om.lattice_constants(), rtol=1e-13,
                               atol=0)


def test_mixture_argument_validation():
    capi = _capi()
    c = C.DROPLET_3
    with pytest.raises(capi.FuglbmError) as e:
        capi.Mixture.from_components(c, 250.0, tau=0.5)
    assert e.value.status == 1
    bad = np.zeros((3, 3))
    bad[0, 1] = 0.1
    with pytest.raises(capi.FuglbmError):
        capi.Mixture.from_components(c, 250.0, bad)          # asymmetric
    with pytest.raises(capi.FuglbmError):
        capi.Mixture.from_components(c, -1.0)
    with pytest.raises(capi.FuglbmError):
        capi.Mixture([1.0] * 17, [1.0] * 17, [0.0] * 17, [1.0] * 17, 300.0)
    with pytest.raises(capi.FuglbmError) as e:
        capi.Mixture.from_components(c, 250.0, eos=3)
    assert e.value.status == 1


def test_fields_bytes():
    capi = _capi()
    L = capi.lib()
    b64 = L.fuglbm_fields_bytes(10, capi.D2Q9, capi.FP64, 1024, 1024, 1)
    b32 = L.fuglbm_fields_bytes(10, capi.D2Q9, capi.FP32_STORAGE, 1024, 1024, 1)
    pop64 = 2 * 9 * 10 * 8 * 1024 * 1024
    # FP32 storage: rest populations FP64, the 8 moving ones FP32
    pop32 = 2 * (8 + 8 * 4) * 10 * 1024 * 1024
    # FP64 rows are padded to a pitch of 1024 + 16 (workspace is the same)
    pad64 = 2 * 9 * 10 * 8 * 16 * 1024
    # FP32 arrays are 2^16 + 64 elements apart beyond the grid from 2^20
    # sites on, 64 elements below
    pad32 = 2 * (8 + 8 * 4) * 10 * (65536 + 64)
    assert b64 >= pop64 and b64 - b32 == pop64 + pad64 - pop32 - pad32
    n = 512
    s64 = L.fuglbm_fields_bytes(10, capi.D2Q9, capi.FP64, n, n, 1)
    s32 = L.fuglbm_fields_bytes(10, capi.D2Q9, capi.FP32_STORAGE, n, n, 1)
    assert s64 - s32 == (2 * 9 * 10 * 8 * n * (n + 16)) - 2 * (8 + 8 * 4) * 10 * (n * n + 64)
    assert L.fuglbm_fields_bytes(0, 0, 0, 8, 8, 1) == 0
    assert L.fuglbm_fields_bytes(3, 1, 0, 8, 8, 8) >= 2 * 19 * 3 * 8 * 512
