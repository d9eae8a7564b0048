"""ctypes binding of ``libfuglbm.so`` (the C ABI in ``include/fuglbm.h``).

Argument marshalling only: every step of the method runs in the HIP
kernels.  The functions keep the C names; ``Mixture`` and ``Simulation``
are small owners of the opaque handles.  PyTorch is used for device memory
(borrowed ``dev_buf``) and streams.  The first call into the library on a
machine without the built ``libfuglbm.so`` raises ImportError; there is no
CPU fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfuglbm.so")

FUGLBM_MAX_COMP = 16
D2Q9, D3Q19 = 0, 1
FP64, FP32_STORAGE = 0, 1
EOS_PR, EOS_SRK, EOS_VDW = 0, 1, 2
EOS_CODES = {"PR": EOS_PR, "SRK": EOS_SRK, "vdW": EOS_VDW}
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EUNPHYSICAL",
                5: "ENONFINITE", 6: "ESTATE"}

EXPORTED = [
    "fuglbm_init_mixture", "fuglbm_lattice_constants", "fuglbm_destroy_mixture",
    "fuglbm_fields_bytes", "fuglbm_init_fields", "fuglbm_step_n", "fuglbm_step_many",
    "fuglbm_read_moments", "fuglbm_diagnostics", "fuglbm_read_populations",
    "fuglbm_write_populations", "fuglbm_set_tuning", "fuglbm_get_tuning", "fuglbm_sim_info",
    "fuglbm_poke_population", "fuglbm_destroy_sim", "fuglbm_last_error",
    "fuglbm_step_many_noalloc",
]


class FuglbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class MixtureDesc(ctypes.Structure):
    _fields_ = [("ncomp", ctypes.c_int32),
                ("Tc_K", ctypes.POINTER(ctypes.c_double)),
                ("pc_bar", ctypes.POINTER(ctypes.c_double)),
                ("omega", ctypes.POINTER(ctypes.c_double)),
                ("M_gmol", ctypes.POINTER(ctypes.c_double)),
                ("kij", ctypes.POINTER(ctypes.c_double)),
                ("T_K", ctypes.c_double),
                ("ref_comp", ctypes.c_int32),
                ("a_ref_lu", ctypes.c_double), ("b_ref_lu", ctypes.c_double),
                ("R_lu", ctypes.c_double),
                ("kappa_ref_lu", ctypes.c_double),
                ("tau", ctypes.c_double),
                ("eos", ctypes.c_int32)]


class Diag(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64),
                ("mass", ctypes.c_double * FUGLBM_MAX_COMP),
                ("momentum", ctypes.c_double * 3),
                ("momentum_pop", ctypes.c_double * 3),
                ("residual", ctypes.c_double),
                ("status", ctypes.c_uint32)]

    def as_dict(self, ncomp):
        return dict(step=self.step, mass=np.array(self.mass[:ncomp]),
                    momentum=np.array(self.momentum[:]),
                    momentum_pop=np.array(self.momentum_pop[:]), residual=self.residual,
                    status=self.status)


_lib = None


def lib():
    """Load the library (torch first, so one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library links against)
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfuglbm.so is not built; run `python -m paper_2306_10652_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "fuglbm_init_mixture": ([ctypes.POINTER(MixtureDesc), ctypes.POINTER(vp)], i32),
        "fuglbm_lattice_constants": ([vp, dp, sz], i32),
        "fuglbm_destroy_mixture": ([vp], None),
        "fuglbm_fields_bytes": ([i32, i32, i32, i32, i32, i32], sz),
        "fuglbm_init_fields": ([vp, i32, i32, i32, i32, i32, dp, vp, vp, ctypes.POINTER(vp)], i32),
        "fuglbm_step_n": ([vp, i64, vp], i32),
        "fuglbm_step_many": ([ctypes.POINTER(vp), i32, i64, vp], i32),
        "fuglbm_step_many_noalloc": ([ctypes.POINTER(vp), i32, i64, vp], i32),
        "fuglbm_read_moments": ([vp, dp, dp, ctypes.POINTER(Diag)], i32),
        "fuglbm_diagnostics": ([vp, ctypes.POINTER(Diag)], i32),
        "fuglbm_read_populations": ([vp, dp], i32),
        "fuglbm_write_populations": ([vp, dp, i64], i32),
        "fuglbm_set_tuning": ([vp, i32, i32], i32),
        "fuglbm_get_tuning": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "fuglbm_sim_info": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64),
                             ctypes.POINTER(i64), ctypes.POINTER(i32)], i32),
        "fuglbm_poke_population": ([vp, i32, i32, i64, ctypes.c_double], i32),
        "fuglbm_destroy_sim": ([vp], None),
        "fuglbm_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(status):
    if status != 0:
        msg = lib().fuglbm_last_error().decode()
        raise FuglbmError(status, msg)


def _dp(a):
    if a is None:
        return None
    if a.dtype != np.float64 or not a.flags.c_contiguous:
        raise TypeError("expected a C-contiguous float64 array, got %s" % a.dtype)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Mixture:
    """Owner of a ``fuglbm_mixture`` handle (physical constants in)."""

    def __init__(self, Tc_K, pc_bar, omega, M_gmol, T_K, kij=None, ref_comp=0,
                 kappa_ref=0.02, tau=1.0, a_ref=0.0, b_ref=0.0, R_lu=0.0, eos="PR"):
        self._arrs = [np.ascontiguousarray(np.asarray(v, dtype=np.float64))
                      for v in (Tc_K, pc_bar, omega, M_gmol)]
        n = len(self._arrs[0])
        self.N = n
        self._kij = None if kij is None else np.ascontiguousarray(
            np.asarray(kij, dtype=np.float64).reshape(n * n))
        d = MixtureDesc()
        d.ncomp = n
        d.Tc_K, d.pc_bar, d.omega, d.M_gmol = (_dp(a) for a in self._arrs)
        d.kij = _dp(self._kij) if self._kij is not None else None
        d.T_K = float(T_K)
        d.ref_comp = int(ref_comp)
        d.a_ref_lu, d.b_ref_lu, d.R_lu = float(a_ref), float(b_ref), float(R_lu)
        d.kappa_ref_lu = float(kappa_ref)
        d.tau = float(tau)
        d.eos = EOS_CODES[eos] if isinstance(eos, str) else int(eos)
        h = ctypes.c_void_p()
        check(lib().fuglbm_init_mixture(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    @classmethod
    def from_components(cls, comps, T_K, kij=None, **kw):
        return cls([c.Tc for c in comps], [c.pc for c in comps], [c.omega for c in comps],
                   [c.M for c in comps], T_K, kij, **kw)

    def lattice_constants(self):
        n = 1 + 4 * self.N + self.N * self.N
        out = np.zeros(n)
        check(lib().fuglbm_lattice_constants(self.handle, _dp(out), n))
        return out

    def molar_masses_lu(self):
        c = self.lattice_constants()
        return np.array([c[1 + 4 * i + 3] for i in range(self.N)])

    def close(self):
        if self.handle:
            lib().fuglbm_destroy_mixture(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fields_bytes(ncomp, lattice, precision, nx, ny, nz=1):
    return lib().fuglbm_fields_bytes(ncomp, lattice, precision, nx, ny, nz)


class Simulation:
    """Owner of a ``fuglbm_sim``; device memory is a borrowed torch buffer
    (``device_buffer=True``) or the library's own allocation."""

    def __init__(self, mixture, lattice, precision, shape, rho, stream=None,
                 device_buffer=True):
        import torch
        nx, ny, nz = (tuple(shape) + (1, 1))[:3]
        self.mixture = mixture
        self.N = mixture.N
        self.lattice, self.precision = lattice, precision
        self.nx, self.ny, self.nz = nx, ny, nz
        self.sites = nx * ny * nz
        self.stream = stream
        rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(self.N, self.sites))
        self._buf = None
        dev = None
        if device_buffer:
            nbytes = fields_bytes(self.N, lattice, precision, nx, ny, nz)
            self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            p = self._buf.data_ptr()
            dev = ctypes.c_void_p((p + 255) & ~255)
        h = ctypes.c_void_p()
        check(lib().fuglbm_init_fields(mixture.handle, lattice, precision, nx, ny, nz, _dp(rho),
                                       dev, _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def step_n(self, n, stream=None):
        check(lib().fuglbm_step_n(self.handle, int(n), _stream_ptr(stream or self.stream)))

    def read_moments(self, velocity=True, diag=False):
        rho = np.zeros(self.N * self.sites)
        D = 2 if self.lattice == D2Q9 else 3
        u = np.zeros(D * self.sites) if velocity else None
        dg = Diag() if diag else None
        st = lib().fuglbm_read_moments(self.handle, _dp(rho), _dp(u),
                                       ctypes.byref(dg) if dg is not None else None)
        shp = (self.nz, self.ny, self.nx)
        out = dict(rho=rho.reshape((self.N,) + shp), status=st)
        if u is not None:
            out["u"] = u.reshape((D,) + shp)
        if dg is not None:
            out["diag"] = dg.as_dict(self.N)
        if st not in (0, 5):
            check(st)
        return out

    def diagnostics(self):
        dg = Diag()
        st = lib().fuglbm_diagnostics(self.handle, ctypes.byref(dg))
        if st not in (0, 5):
            check(st)
        d = dg.as_dict(self.N)
        d["rc"] = st
        return d

    def read_populations(self):
        Q = 9 if self.lattice == D2Q9 else 19
        g = np.zeros(self.N * Q * self.sites)
        check(lib().fuglbm_read_populations(self.handle, _dp(g)))
        return g.reshape(self.N, Q, self.sites)

    def write_populations(self, g, step):
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).ravel())
        check(lib().fuglbm_write_populations(self.handle, _dp(g), int(step)))

    def set_tuning(self, kernel=0, rows=0):
        check(lib().fuglbm_set_tuning(self.handle, int(kernel), int(rows)))

    def get_tuning(self):
        k, r = ctypes.c_int32(), ctypes.c_int32()
        check(lib().fuglbm_get_tuning(self.handle, ctypes.byref(k), ctypes.byref(r)))
        return dict(kernel=k.value, rows=r.value)

    def info(self):
        Q, D, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        s, b = ctypes.c_int64(), ctypes.c_int64()
        check(lib().fuglbm_sim_info(self.handle, ctypes.byref(Q), ctypes.byref(D),
                                    ctypes.byref(s), ctypes.byref(b), ctypes.byref(k)))
        return dict(Q=Q.value, D=D.value, sites=s.value, alg_bytes_per_step=b.value,
                    kernel=k.value)

    def poke(self, comp, a, site, value):
        check(lib().fuglbm_poke_population(self.handle, comp, a, site, float(value)))

    def close(self):
        if self.handle:
            lib().fuglbm_destroy_sim(self.handle)
            self.handle = None
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fuglbm_step_many(sims, nsteps, stream=None):
    arr = (ctypes.c_void_p * len(sims))(*[s.handle.value for s in sims])
    return lib().fuglbm_step_many(arr, len(sims), int(nsteps), _stream_ptr(stream))


def step_many(sims, nsteps, stream=None):
    check(fuglbm_step_many(sims, nsteps, stream))


def fuglbm_step_many_noalloc(sims, nsteps, stream=None):
    arr = (ctypes.c_void_p * len(sims))(*[s.handle.value for s in sims])
    return lib().fuglbm_step_many_noalloc(arr, len(sims), int(nsteps), _stream_ptr(stream))


def step_many_noalloc(sims, nsteps, stream=None):
    check(fuglbm_step_many_noalloc(sims, nsteps, stream))
