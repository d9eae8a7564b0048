// Device-side definitions shared by the gfx950 kernels and the host library:
// per-simulation constant block, lattice velocity sets, the local
// cubic-EOS (Peng-Robinson, SRK, vdW) fugacity and the per-(component,
// direction) collision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FUG_MAXC 16

// Status bits (mirrors FUGLBM_ST_* of the public header).
#define FUG_ST_NONFINITE 1u
#define FUG_ST_COVOLUME 2u
#define FUG_ST_NEGATIVE 4u

// Constants of one simulation, lattice units, FP64.  Lives in device memory
// (one per simulation) and is read with wave-uniform loads.
struct SimConst {
    int32_t N;            // components
    int32_t lattice;      // 0 D2Q9, 1 D3Q19
    int32_t nx, ny, nz;
    int32_t eos;          // 0 Peng-Robinson, 1 SRK, 2 van der Waals
    int64_t nsites;
    double omega;         // 1 / tau
    double fcoef;         // 1 - 1 / (2 tau)
    double RT;
    // cubic p = RT/(v - b) - a alpha/((v + d1 b)(v + d2 b)):  d1, d2,
    // u = d1 + d2, w = d1 d2 (exact per EOS) and dk = 1/(d1 - d2) (0 for vdW)
    double d1, d2, eu, ew, dk;
    double b[FUG_MAXC];
    double M[FUG_MAXC];
    double invM[FUG_MAXC];
    double sqk[FUG_MAXC];     // sqrt(kappa_i)
    double aij[FUG_MAXC * FUG_MAXC];  // (a alpha)_ij, row-major, stride FUG_MAXC
};

// ---------------------------------------------------------------------------
// Velocity sets.  D2Q9 order: rest, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-).
// D3Q19 order: rest, 6 faces, 12 edges; opposite pairs at (a, a+1) for a odd.
// ---------------------------------------------------------------------------
struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    static constexpr bool PULL_X = false;   // see pop_col
    __host__ __device__ static constexpr int ex(int a) {
        return a == 1 || a == 5 || a == 8 ? 1 : (a == 3 || a == 6 || a == 7 ? -1 : 0);
    }
    __host__ __device__ static constexpr int ey(int a) {
        return a == 2 || a == 5 || a == 6 ? 1 : (a == 4 || a == 7 || a == 8 ? -1 : 0);
    }
    __host__ __device__ static constexpr int ez(int) { return 0; }
    __host__ __device__ static constexpr double w(int a) {
        return a == 0 ? 4.0 / 9.0 : (a <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr bool PULL_X = true;    // see pop_col
    // faces: 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z
    // edges: 7 (+x+y) 8 (-x-y) 9 (+x-y) 10 (-x+y) 11 (+x+z) 12 (-x-z)
    //        13 (+x-z) 14 (-x+z) 15 (+y+z) 16 (-y-z) 17 (+y-z) 18 (-y+z)
    __host__ __device__ static constexpr int ex(int a) {
        return (a == 1 || a == 7 || a == 9 || a == 11 || a == 13) ? 1
             : ((a == 2 || a == 8 || a == 10 || a == 12 || a == 14) ? -1 : 0);
    }
    __host__ __device__ static constexpr int ey(int a) {
        return (a == 3 || a == 7 || a == 10 || a == 15 || a == 17) ? 1
             : ((a == 4 || a == 8 || a == 9 || a == 16 || a == 18) ? -1 : 0);
    }
    __host__ __device__ static constexpr int ez(int a) {
        return (a == 5 || a == 11 || a == 14 || a == 15 || a == 18) ? 1
             : ((a == 6 || a == 12 || a == 13 || a == 16 || a == 17) ? -1 : 0);
    }
    __host__ __device__ static constexpr double w(int a) {
        return a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
};

// ---------------------------------------------------------------------------
// Cubic-EOS ln f_i for one component, given mixture sums at a site.
//   eta = b_m rt = sum_j b_j rt_j,  am = sum_ij x_i x_j (a alpha)_ij,
//   Si  = sum_j x_j (a alpha)_ij.
// Returns RT ln f_i in the combined-logarithm form (defined for p <= 0):
//   RT ln(rt_i RT/(1-eta)) + RT (b_i/b_m)(Z-1) - (Lhat/b_m) (2 S_i - a_m b_i / b_m),
//   Lhat = ln[(1 + d1 eta) / (1 + d2 eta)] / (d1 - d2)   (PR: Eq. (12); SRK),
//   Lhat = eta                                           (vdW, the d1 = d2 -> 0 limit),
//   Z - 1 = eta/(1 - eta) - am rt / (RT (1 + u eta + w eta^2)).
// The terms shared by all components are passed in precomputed.
// ---------------------------------------------------------------------------
struct MixSums {
    double rt;         // total molar density
    double inv_bm;     // 1 / b_m
    double zm1;        // Z - 1
    double lam_c;      // Lhat / b_m
    double am;
    double log_pref;   // ln(RT / (1 - eta))
    uint32_t bad;      // status bits
};

// Lhat of the EOS (uniform branch on the EOS kind).
__device__ __forceinline__ double eos_lhat(const SimConst *c, double eta) {
    if (c->eos == 2) return eta;
    return log((1.0 + c->d1 * eta) / (1.0 + c->d2 * eta)) * c->dk;
}

__device__ __forceinline__ MixSums cubic_mixture(const SimConst *c, double rt, double eta,
                                                 double am, double RT) {
    MixSums m;
    m.rt = rt;
    m.am = am;
    const double one_m_eta = 1.0 - eta;
    m.bad = (one_m_eta > 0.0) ? 0u : FUG_ST_COVOLUME;
    const double bm = eta / rt;
    m.inv_bm = 1.0 / bm;
    const double den = 1.0 + c->eu * eta + c->ew * eta * eta;
    // Z - 1 = p / (rt RT) - 1,  p = rt RT/(1 - eta) - am rt^2 / den
    m.zm1 = eta / one_m_eta - am * rt / (RT * den);
    m.lam_c = eos_lhat(c, eta) * m.inv_bm;
    m.log_pref = log(RT / one_m_eta);
    return m;
}

__device__ __forceinline__ double cubic_RTlnf(const MixSums &m, double RT, double rt_i,
                                              double b_i, double S_i) {
    const double bi_bm = b_i * m.inv_bm;
    return RT * (log(rt_i) + m.log_pref + bi_bm * m.zm1)
         - m.lam_c * (2.0 * S_i - m.am * bi_bm);
}

// ---------------------------------------------------------------------------
// Collision of one (component, direction): Eq. (1a) with geq of Eq. (1b)
// (rho^c = 0) and the forcing term of Eq. (1c); cs^2 = 1/3.
// ---------------------------------------------------------------------------
template <class L>
__device__ __forceinline__ double collide_one(int a, double g, double rho, double ux,
                                              double uy, double uz, double Fx, double Fy,
                                              double Fz, double Gx, double Gy, double Gz,
                                              double uu, double Fu, double Gu, double omega,
                                              double fcoef) {
    const double exa = L::ex(a), eya = L::ey(a), eza = L::ez(a);
    const double eu = exa * ux + eya * uy + eza * uz;
    const double eF = exa * Fx + eya * Fy + eza * Fz;
    const double eG = exa * Gx + eya * Gy + eza * Gz;
    const double e2 = exa * exa + eya * eya + eza * eza;
    const double wa = L::w(a);
    const double sq = 3.0 * eu + 4.5 * eu * eu - 1.5 * uu;
    const double geq = (a == 0) ? rho + wa * rho * sq : wa * rho * sq;
    const double Fa = wa * (3.0 * (eF - Fu) + 9.0 * eu * eF)
                    + wa * (-Gu + 3.0 * eu * eG + 0.5 * (3.0 * e2 - (double)L::D) * Gu);
    // (1 - omega) g + omega geq: at omega = 1 (tau = 1) the old population
    // drops out exactly, so a caller may pass g = 0 without reading it
    return fma(1.0 - omega, g, omega * geq) + fcoef * Fa;
}

// Population storage of one buffer.  The rest populations are FP64 in both
// precisions; the moving ones (a >= 1) are stored as ST (double for FP64,
// float for FP32 storage).  In FP32 storage a kernel that writes a site
// stores its rest population as rho minus the FP64 sum of the stored moving
// ones (the collision at tau != 1 of the multi-pass path folds their
// rounding error into it instead), so every component's mass is conserved
// to FP64 rounding.  Moving populations sit at the columns pop_col gives.
//
// FP64: blocked by lattice row (row = y + ny*z).  Row `row` is one
// contiguous block [N][pitch] double (rest) ++ [N][Q-1][pitch] double
// (moving), so a workgroup's row of every component comes from one block;
// the pitch is padded past large power-of-two strides.
// FP32 storage: one array per (component, direction) over the whole grid,
// [N][sites + pad] double (rest) ++ [N][Q-1][sites + pad] float (moving).
// (Both measured fastest for their precision with the fused D2Q9 kernel.)
template <typename ST>
struct PopLayout;

template <>
struct PopLayout<double> {
    int64_t pitch, row_bytes, move_base, Qm;
    __host__ __device__ static int64_t pad_pitch(int nx) {
        return nx >= 256 ? ((int64_t)nx + 15) / 16 * 16 + 16 : nx;
    }
    __host__ __device__ PopLayout(int N, int Q, int nx, int64_t /*rows*/)
        : pitch(pad_pitch(nx)), row_bytes((int64_t)N * pitch * Q * 8),
          move_base((int64_t)N * pitch * 8), Qm(Q - 1) {}
    // byte offsets
    __host__ __device__ int64_t rest(int64_t row, int i, int x) const {
        return row * row_bytes + ((int64_t)i * pitch + x) * 8;
    }
    __host__ __device__ int64_t move(int64_t row, int i, int a, int x) const {
        return row * row_bytes + move_base + (((int64_t)i * Qm + (a - 1)) * pitch + x) * 8;
    }
    // element strides from one row to the next (rest array, moving arrays)
    __host__ __device__ int64_t rest_row_stride() const { return row_bytes / 8; }
    __host__ __device__ int64_t move_row_stride() const { return row_bytes / 8; }
    __host__ __device__ int64_t bytes(int64_t rows) const { return rows * row_bytes; }
};

template <>
struct PopLayout<float> {
    // Elements between consecutive arrays.  The arrays of a large grid are
    // large powers of two; a gap of 64 elements breaks the spacing, but the
    // rows that the 9N (or 19N) streams touch together still start at
    // nearly the same place within the HBM channel interleave.  A gap of
    // 2^16 + 64 elements spreads them (on the 1024^2 ten-component field
    // the fused step's memory skeleton ran 14 % faster, the step 3.6 %);
    // small grids keep 64 elements, where the wide gap would dwarf them.
    __host__ __device__ static int64_t pad(int64_t sites) {
        return sites >= ((int64_t)1 << 20) ? 65536 + 64 : 64;
    }
    int64_t nx, ns, move_base, Qm;       // ns: array stride in elements
    __host__ __device__ PopLayout(int N, int Q, int nx_, int64_t rows)
        : nx(nx_), ns(nx_ * rows + pad(nx_ * rows)),
          move_base((int64_t)N * (nx_ * rows + pad(nx_ * rows)) * 8), Qm(Q - 1) {}
    __host__ __device__ int64_t rest(int64_t row, int i, int x) const {
        return ((int64_t)i * ns + row * nx + x) * 8;
    }
    __host__ __device__ int64_t move(int64_t row, int i, int a, int x) const {
        return move_base + (((int64_t)i * Qm + (a - 1)) * ns + row * nx + x) * 4;
    }
    __host__ __device__ int64_t rest_row_stride() const { return nx; }
    __host__ __device__ int64_t move_row_stride() const { return nx; }
    __host__ __device__ int64_t bytes(int64_t /*rows*/) const { return move_base + move_base / 2 * Qm; }
};

// Column of the stored moving population a (a >= 1) that belongs to column
// x of a row.  D3Q19 keeps each moving population at the column it was
// collided at and moves it along y and z only (push in y and z, pull in
// x): population a of column x sits at column x - e_x(a) of x's row, so a
// collision's stores are whole aligned rows (a 64-wide store shifted by
// one column straddles five cache lines, two of them partly written).
// D2Q9 keeps every population at its own site (the fused D2Q9 kernels
// push in x as well).
template <class L>
__host__ __device__ inline int pop_col(int a, int x, int nx) {
    if (!L::PULL_X) return x;
    const int v = x - L::ex(a);
    return v < 0 ? v + nx : (v >= nx ? v - nx : v);
}

template <typename ST>
__device__ __forceinline__ double ld_pop(const void *buf, const PopLayout<ST> &L, int64_t row,
                                         int i, int a, int x) {
    const char *b = (const char *)buf;
    if (a == 0) return *(const double *)(b + L.rest(row, i, x));
    return (double)*(const ST *)(b + L.move(row, i, a, x));
}
