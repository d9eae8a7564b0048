// Driver for the host-side checks of the C-ABI library under AddressSanitizer
// and UndefinedBehaviorSanitizer (no GPU needed): every entry point that
// does its work on the host, and every argument check that returns before
// the first device call.  Exits non-zero on any unexpected status; the
// sanitizers abort on any out-of-bounds access or undefined arithmetic.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "fuglbm.h"

static int failures = 0;

static void expect(const char *what, fuglbm_status got, fuglbm_status want) {
    if (got != want) {
        std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want,
                     fuglbm_last_error());
        ++failures;
    } else if (want != FUGLBM_OK && std::strlen(fuglbm_last_error()) == 0) {
        std::fprintf(stderr, "%s: no error message\n", what);
        ++failures;
    }
}

struct Comps {
    std::vector<double> Tc, pc, w, M, kij;
};

// n-alkane-like constants, heavier with the index (any positive values do)
static Comps make_comps(int n, bool with_kij) {
    Comps c;
    for (int i = 0; i < n; ++i) {
        c.Tc.push_back(190.6 + 45.0 * i);
        c.pc.push_back(45.99 - 2.4 * i);
        c.w.push_back(0.011 + 0.05 * i);
        c.M.push_back(16.043 + 14.027 * i);
    }
    if (with_kij) {
        c.kij.assign((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                if (i != j) c.kij[(size_t)i * n + j] = 0.01 * ((i + j) % 5);
    }
    return c;
}

static fuglbm_mixture_desc desc_of(const Comps &c, int n, int eos) {
    fuglbm_mixture_desc d;
    std::memset(&d, 0, sizeof(d));
    d.ncomp = n;
    d.Tc_K = c.Tc.data();
    d.pc_bar = c.pc.data();
    d.omega = c.w.data();
    d.M_gmol = c.M.data();
    d.kij = c.kij.empty() ? nullptr : c.kij.data();
    d.T_K = 325.0;
    d.ref_comp = 0;
    d.kappa_ref_lu = 0.02;
    d.tau = 1.0;
    d.eos = eos;
    return d;
}

int main() {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    // valid mixtures: every EOS, N from 1 to the maximum, with and without kij
    for (int eos = 0; eos < 3; ++eos) {
        for (int n : {1, 2, 3, 10, FUGLBM_MAX_COMP}) {
            for (bool kij : {false, true}) {
                Comps c = make_comps(n, kij);
                fuglbm_mixture_desc d = desc_of(c, n, eos);
                fuglbm_mixture *m = nullptr;
                expect("init_mixture", fuglbm_init_mixture(&d, &m), FUGLBM_OK);
                if (!m) continue;
                const size_t need = 1 + 4 * (size_t)n + (size_t)n * n;
                std::vector<double> out(need);
                expect("lattice_constants", fuglbm_lattice_constants(m, out.data(), need), FUGLBM_OK);
                for (double v : out)
                    if (!std::isfinite(v)) {
                        std::fprintf(stderr, "non-finite lattice constant\n");
                        ++failures;
                    }
                expect("lattice_constants short", fuglbm_lattice_constants(m, out.data(), need - 1),
                       FUGLBM_EINVAL);
                expect("lattice_constants null", fuglbm_lattice_constants(m, nullptr, need),
                       FUGLBM_EINVAL);
                // init_fields checks that return before any device work
                const int nx = 7, ny = 5;
                std::vector<double> rho((size_t)n * nx * ny, 0.05);
                fuglbm_sim *s = nullptr;
                expect("init_fields null rho",
                       fuglbm_init_fields(m, FUGLBM_D2Q9, FUGLBM_FP64, nx, ny, 1, nullptr, nullptr,
                                          nullptr, &s), FUGLBM_EINVAL);
                expect("init_fields nz != 1 for D2Q9",
                       fuglbm_init_fields(m, FUGLBM_D2Q9, FUGLBM_FP64, nx, ny, 2, rho.data(), nullptr,
                                          nullptr, &s), FUGLBM_EINVAL);
                expect("init_fields zero size",
                       fuglbm_init_fields(m, FUGLBM_D3Q19, FUGLBM_FP32_STORAGE, nx, 0, 1, rho.data(),
                                          nullptr, nullptr, &s), FUGLBM_EINVAL);
                expect("init_fields bad lattice",
                       fuglbm_init_fields(m, (fuglbm_lattice)7, FUGLBM_FP64, nx, ny, 1, rho.data(),
                                          nullptr, nullptr, &s), FUGLBM_EINVAL);
                expect("init_fields bad precision",
                       fuglbm_init_fields(m, FUGLBM_D2Q9, (fuglbm_precision)3, nx, ny, 1, rho.data(),
                                          nullptr, nullptr, &s), FUGLBM_EINVAL);
                expect("init_fields too large",
                       fuglbm_init_fields(m, FUGLBM_D3Q19, FUGLBM_FP64, 2048, 2048, 1024, rho.data(),
                                          nullptr, nullptr, &s), FUGLBM_EINVAL);
                // unphysical fields: the last site of the last component
                std::vector<double> bad = rho;
                bad.back() = -1.0;
                expect("init_fields negative density",
                       fuglbm_init_fields(m, FUGLBM_D2Q9, FUGLBM_FP64, nx, ny, 1, bad.data(), nullptr,
                                          nullptr, &s), FUGLBM_EUNPHYSICAL);
                bad.back() = nan;
                expect("init_fields NaN density",
                       fuglbm_init_fields(m, FUGLBM_D2Q9, FUGLBM_FP64, nx, ny, 1, bad.data(), nullptr,
                                          nullptr, &s), FUGLBM_EUNPHYSICAL);
                std::vector<double> dense((size_t)n * nx * ny, 1e3);
                expect("init_fields past the co-volume",
                       fuglbm_init_fields(m, FUGLBM_D2Q9, FUGLBM_FP64, nx, ny, 1, dense.data(), nullptr,
                                          nullptr, &s), FUGLBM_EUNPHYSICAL);
                if (s) {
                    std::fprintf(stderr, "init_fields returned a simulation on failure\n");
                    ++failures;
                }
                fuglbm_destroy_mixture(m);
            }
        }
    }
    // invalid mixtures
    {
        Comps c = make_comps(3, true);
        fuglbm_mixture *m = nullptr;
        expect("init_mixture null", fuglbm_init_mixture(nullptr, &m), FUGLBM_EINVAL);
        fuglbm_mixture_desc d = desc_of(c, 3, 0);
        expect("init_mixture null out", fuglbm_init_mixture(&d, nullptr), FUGLBM_EINVAL);
        struct Case {
            const char *name;
            void (*edit)(fuglbm_mixture_desc &, Comps &);
        } cases[] = {
            {"ncomp 0", [](fuglbm_mixture_desc &d, Comps &) { d.ncomp = 0; }},
            {"ncomp 17", [](fuglbm_mixture_desc &d, Comps &) { d.ncomp = FUGLBM_MAX_COMP + 1; }},
            {"ref_comp", [](fuglbm_mixture_desc &d, Comps &) { d.ref_comp = 3; }},
            {"eos", [](fuglbm_mixture_desc &d, Comps &) { d.eos = 5; }},
            {"T", [](fuglbm_mixture_desc &d, Comps &) { d.T_K = 0.0; }},
            {"tau", [](fuglbm_mixture_desc &d, Comps &) { d.tau = 0.5; }},
            {"kappa", [](fuglbm_mixture_desc &d, Comps &) { d.kappa_ref_lu = -1.0; }},
            {"Tc NaN", [](fuglbm_mixture_desc &, Comps &c) { c.Tc[1] = std::nan(""); }},
            {"pc 0", [](fuglbm_mixture_desc &, Comps &c) { c.pc[2] = 0.0; }},
            {"kij asymmetric", [](fuglbm_mixture_desc &, Comps &c) { c.kij[1] = 0.3; }},
            {"kij diagonal", [](fuglbm_mixture_desc &, Comps &c) { c.kij[4] = 0.1; }},
            {"kij 1", [](fuglbm_mixture_desc &, Comps &c) { c.kij[1] = c.kij[3] = 1.0; }},
            {"null Tc", [](fuglbm_mixture_desc &d, Comps &) { d.Tc_K = nullptr; }},
        };
        for (auto &k : cases) {
            Comps cc = make_comps(3, true);
            fuglbm_mixture_desc dd = desc_of(cc, 3, 0);
            k.edit(dd, cc);
            m = nullptr;
            expect(k.name, fuglbm_init_mixture(&dd, &m), FUGLBM_EINVAL);
            if (m) {
                std::fprintf(stderr, "%s: mixture returned on failure\n", k.name);
                ++failures;
                fuglbm_destroy_mixture(m);
            }
        }
    }
    // buffer sizes: monotone in every argument, 0 for invalid arguments
    {
        size_t prev = 0;
        for (int n = 1; n <= FUGLBM_MAX_COMP; ++n) {
            const size_t b = fuglbm_fields_bytes(n, FUGLBM_D2Q9, FUGLBM_FP64, 300, 17, 1);
            if (b <= prev) {
                std::fprintf(stderr, "fields_bytes not increasing in ncomp\n");
                ++failures;
            }
            prev = b;
        }
        if (fuglbm_fields_bytes(10, FUGLBM_D3Q19, FUGLBM_FP32_STORAGE, 64, 64, 64) >=
            fuglbm_fields_bytes(10, FUGLBM_D3Q19, FUGLBM_FP64, 64, 64, 64)) {
            std::fprintf(stderr, "FP32 storage not smaller than FP64\n");
            ++failures;
        }
        if (fuglbm_fields_bytes(0, FUGLBM_D2Q9, FUGLBM_FP64, 8, 8, 1) != 0 ||
            fuglbm_fields_bytes(3, (fuglbm_lattice)2, FUGLBM_FP64, 8, 8, 1) != 0 ||
            fuglbm_fields_bytes(3, FUGLBM_D2Q9, FUGLBM_FP64, 0, 8, 1) != 0) {
            std::fprintf(stderr, "fields_bytes accepted an invalid argument\n");
            ++failures;
        }
    }
    // stepping and read-out checks that return before any device work
    {
        fuglbm_diag dg;
        expect("step_n null", fuglbm_step_n(nullptr, 5, nullptr), FUGLBM_EINVAL);
        expect("step_many negative count", fuglbm_step_many(nullptr, -1, 5, nullptr), FUGLBM_EINVAL);
        expect("step_many null array", fuglbm_step_many(nullptr, 2, 5, nullptr), FUGLBM_EINVAL);
        expect("step_many_noalloc null array", fuglbm_step_many_noalloc(nullptr, 2, 5, nullptr),
               FUGLBM_EINVAL);
        std::vector<fuglbm_sim *> many(300, nullptr);
        expect("step_many_noalloc too many", fuglbm_step_many_noalloc(many.data(), 300, 1, nullptr),
               FUGLBM_EINVAL);
        expect("step_many_noalloc null member", fuglbm_step_many_noalloc(many.data(), 3, 1, nullptr),
               FUGLBM_EINVAL);
        expect("read_moments null", fuglbm_read_moments(nullptr, nullptr, nullptr, &dg), FUGLBM_EINVAL);
        expect("diagnostics null", fuglbm_diagnostics(nullptr, &dg), FUGLBM_EINVAL);
        expect("read_populations null", fuglbm_read_populations(nullptr, nullptr), FUGLBM_EINVAL);
        expect("set_tuning null", fuglbm_set_tuning(nullptr, 0, 0), FUGLBM_EINVAL);
        expect("sim_info null", fuglbm_sim_info(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr),
               FUGLBM_EINVAL);
        fuglbm_destroy_sim(nullptr);
        fuglbm_destroy_mixture(nullptr);
    }
    std::printf("%s\n", failures ? "FAILED" : "OK");
    return failures ? 1 : 0;
}
