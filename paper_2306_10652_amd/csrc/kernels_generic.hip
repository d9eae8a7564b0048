// Multi-pass step for any lattice (D2Q9, D3Q19), FP64 or FP32 storage
// (population layout: PopLayout of the common header):
//   pass 1  moments + local cubic-EOS fugacity: rho_i, RT ln f_i, s = sum sqrt(kappa_j) rt_j, j
//   pass 2  psi_i = RT ln f_i - sqrt(kappa_i) lap(s)             (Eq. (4)-(5))
//   pass 3  u = (j + F/2) / rho, F = -sum_i rt_i grad psi_i      (LDS tiles)
//   pass 4  F_i, G_i = grad rho_i, collide (Eq. (1)), push        (LDS tiles)
// One thread per site; fields between passes live in the simulation's
// workspace.  Also: initial populations, the macroscopic read-out and the
// per-block diagnostic partial sums.
#include "generic_tiles.h"

namespace {


template <class L>
__device__ __forceinline__ int64_t nb_site(int x, int y, int z, int a, int nx, int ny, int nz) {
    int xx = x + L::ex(a), yy = y + L::ey(a), zz = z + L::ez(a);
    xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
    yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
    zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
    return (int64_t)xx + (int64_t)nx * ((int64_t)yy + (int64_t)ny * zz);
}

template <class L, typename ST>
__global__ __launch_bounds__(TPB) void k_init(const SimConst *__restrict__ c,
                                              const double *__restrict__ rho,
                                              void *__restrict__ g) {
    const int64_t ns = c->nsites;
    const int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (s >= ns) return;
    const int N = c->N, nx = c->nx;
    const PopLayout<ST> P(N, L::Q, nx, (int64_t)c->ny * c->nz);
    const int64_t row = s / nx;
    const int x = (int)(s - row * nx);
    char *b = (char *)g;
    for (int i = 0; i < N; ++i) {
        *(double *)(b + P.rest(row, i, x)) = rho[(int64_t)i * ns + s];
#pragma unroll
        for (int a = 1; a < L::Q; ++a) *(ST *)(b + P.move(row, i, a, x)) = (ST)0;
    }
}

// Each pass is a device function over one work unit (a block of TPB sites,
// or a tile), called by the kernel of one simulation and by the batched
// kernel, which finds the unit's simulation in a member table.
template <class L, typename ST>
__device__ __forceinline__ void moments_eos_body(const SimConst *__restrict__ c,
                                                 const void *__restrict__ g,
                                                 double *__restrict__ rho_f,
                                                 double *__restrict__ psi_f,
                                                 double *__restrict__ s_f,
                                                 double *__restrict__ j_f,
                                                 uint32_t *__restrict__ status, int64_t blk) {
    const int64_t ns = c->nsites;
    const int64_t s = blk * TPB + threadIdx.x;
    if (s >= ns) return;
    const int N = c->N, nx = c->nx;
    const PopLayout<ST> P(N, L::Q, nx, (int64_t)c->ny * c->nz);
    const int64_t row = s / nx;
    const int xs = (int)(s - row * nx);
    double rt[FUG_MAXC];
    double jx = 0.0, jy = 0.0, jz = 0.0;
    double rtt = 0.0, eta = 0.0, sv = 0.0;
    uint32_t bad = 0;
#pragma unroll
    for (int i = 0; i < FUG_MAXC; ++i) {
        rt[i] = 1.0;
        if (i < N) {
            double r = 0.0;
#pragma unroll
            for (int a = 0; a < L::Q; ++a) {
                const double v = ld_pop<ST>(g, P, row, i, a, a == 0 ? xs : pop_col<L>(a, xs, nx));
                r += v;
                jx += L::ex(a) * v;
                jy += L::ey(a) * v;
                jz += L::ez(a) * v;
            }
            rho_f[(int64_t)i * ns + s] = r;
            rt[i] = r * c->invM[i];
            if (!(rt[i] > 0.0)) bad |= FUG_ST_NEGATIVE;
            rtt += rt[i];
            eta += c->b[i] * rt[i];
            sv += c->sqk[i] * rt[i];
        }
    }
    const double inv_rt = 1.0 / rtt;
    double S[FUG_MAXC];
    double am = 0.0;
#pragma unroll
    for (int i = 0; i < FUG_MAXC; ++i) {
        S[i] = 0.0;
        if (i < N) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < FUG_MAXC; ++j)
                if (j < N) acc += rt[j] * c->aij[i * FUG_MAXC + j];
            S[i] = acc * inv_rt;
            am += rt[i] * inv_rt * S[i];
        }
    }
    const double RT = c->RT;
    const MixSums m = cubic_mixture(c, rtt, eta, am, RT);
    bad |= m.bad;
#pragma unroll
    for (int i = 0; i < FUG_MAXC; ++i) {
        if (i < N) {
            const double v = cubic_RTlnf(m, RT, rt[i], c->b[i], S[i]);
            if (!isfinite(v)) bad |= FUG_ST_NONFINITE;
            psi_f[(int64_t)i * ns + s] = v;
        }
    }
    s_f[s] = sv;
    j_f[s] = jx;
    j_f[ns + s] = jy;
    if (L::D == 3) j_f[2 * ns + s] = jz;
    if (bad) atomicOr(status, bad);
}

template <class L, typename ST>
__global__ __launch_bounds__(TPB) void k_moments_eos(const SimConst *__restrict__ c,
                                                     const void *__restrict__ g,
                                                     double *__restrict__ rho_f,
                                                     double *__restrict__ psi_f,
                                                     double *__restrict__ s_f,
                                                     double *__restrict__ j_f,
                                                     uint32_t *__restrict__ status) {
    moments_eos_body<L, ST>(c, g, rho_f, psi_f, s_f, j_f, status, blockIdx.x);
}

template <class L>
__device__ __forceinline__ void interface_body(const SimConst *__restrict__ c,
                                               const double *__restrict__ s_f,
                                               double *__restrict__ psi_f, int64_t blk) {
    const int64_t ns = c->nsites;
    const int64_t s = blk * TPB + threadIdx.x;
    if (s >= ns) return;
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const int x = (int)(s % nx), y = (int)((s / nx) % ny), z = (int)(s / ((int64_t)nx * ny));
    const double sc = s_f[s];
    double acc = 0.0;
#pragma unroll
    for (int a = 1; a < L::Q; ++a)
        acc = fma(L::w(a), s_f[nb_site<L>(x, y, z, a, nx, ny, nz)] - sc, acc);
    const double lap = 6.0 * acc;
    const int N = c->N;
    // explicit fused operations (here and in the velocity pass), so that
    // the rounding does not depend on the compiler's contraction choices
    for (int i = 0; i < N; ++i) {
        const int64_t k = (int64_t)i * ns + s;
        psi_f[k] = fma(-c->sqk[i], lap, psi_f[k]);
    }
}

template <class L>
__global__ __launch_bounds__(TPB) void k_interface(const SimConst *__restrict__ c,
                                                   const double *__restrict__ s_f,
                                                   double *__restrict__ psi_f) {
    interface_body<L>(c, s_f, psi_f, blockIdx.x);
}


// Collision work unit -> (tile, component).  Units go through the tiles in
// chunks of COLLIDE_CHUNK, each chunk component by component, so the
// tiles that read one another's halos run together while the rows being
// written stay few.
constexpr int COLLIDE_CHUNK = 32;
__device__ __forceinline__ void collide_unit(int unit, int ntiles, int N, int &tile, int &comp) {
    const int t0 = unit / (COLLIDE_CHUNK * N) * COLLIDE_CHUNK;
    const int kk = min(COLLIDE_CHUNK, ntiles - t0);
    const int r = unit - t0 * N;
    comp = r / kk;
    tile = t0 + r % kk;
}


// u = (j + F/2) / rho, F = sum_i F_i, F_i = -rt_i grad psi_i  -> u_f
template <class L>
__device__ __forceinline__ void velocity_body(const SimConst *__restrict__ c,
                                              const double *__restrict__ rho_f,
                                              const double *__restrict__ psi_f,
                                              const double *__restrict__ j_f,
                                              double *__restrict__ u_f, int unit, double *lp) {
    using TG = TileGeom<L, TileV<L>>;
    // padding units leave as a whole workgroup, before any barrier
    if (unit >= TG::count(c->nx, c->ny, c->nz)) return;
    const TG T(c, unit);
    const int64_t ns = c->nsites;
    const int64_t s = T.active ? (int64_t)T.x + (int64_t)c->nx * ((int64_t)T.y + (int64_t)c->ny * T.z) : 0;
    double Fx = 0.0, Fy = 0.0, Fz = 0.0, rhot = 0.0;
    for (int i = 0; i < c->N; ++i) {
        __syncthreads();
        T.stage(c, psi_f + (int64_t)i * ns, lp);
        __syncthreads();
        if (T.active) {
            double gx, gy, gz;
            T.grad(lp, gx, gy, gz);
            const double r = rho_f[(int64_t)i * ns + s];
            const double rt = r * c->invM[i];
            Fx = fma(-rt, gx, Fx);
            Fy = fma(-rt, gy, Fy);
            Fz = fma(-rt, gz, Fz);
            rhot += r;
        }
    }
    if (!T.active) return;
    u_f[s] = fma(0.5, Fx, j_f[s]) / rhot;
    u_f[ns + s] = fma(0.5, Fy, j_f[ns + s]) / rhot;
    if (L::D == 3) u_f[2 * ns + s] = fma(0.5, Fz, j_f[2 * ns + s]) / rhot;
}

template <class L>
__global__ __launch_bounds__(TPB) void k_velocity_t(const SimConst *__restrict__ c,
                                                    const double *__restrict__ rho_f,
                                                    const double *__restrict__ psi_f,
                                                    const double *__restrict__ j_f,
                                                    double *__restrict__ u_f) {
    __shared__ double lp[TileGeom<L, TileV<L>>::NH];
    velocity_body<L>(c, rho_f, psi_f, j_f, u_f, xcd_unit(), lp);
}

// collision (Eq. (1a)-(1c)) and push of one component over one tile
// (collide_unit); u from u_f
// KEEP: tau != 1, so the collision keeps (1 - omega) g of the old population.
template <class L, typename ST, bool KEEP>
__device__ __forceinline__ void collide_body(const SimConst *__restrict__ c,
                                             const void *__restrict__ gs, void *__restrict__ gd,
                                             const double *__restrict__ rho_f,
                                             const double *__restrict__ psi_f,
                                             const double *__restrict__ u_f, int unit, double *lp,
                                             double *lr) {
    using TG = TileGeom<L, TileC<L>>;
    const int N = c->N;
    // padding units leave as a whole workgroup, before any barrier
    const int ntiles = (int)TG::count(c->nx, c->ny, c->nz);
    if (unit >= ntiles * N) return;
    int tile, i;
    collide_unit(unit, ntiles, N, tile, i);
    const TG T(c, tile);
    const int64_t ns = c->nsites;
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const int64_t s = T.active ? (int64_t)T.x + (int64_t)nx * ((int64_t)T.y + (int64_t)ny * T.z) : 0;
    const PopLayout<ST> P(N, L::Q, nx, (int64_t)ny * nz);
    double ux = 0.0, uy = 0.0, uz = 0.0;
    if (T.active) {
        ux = u_f[s];
        uy = u_f[ns + s];
        uz = (L::D == 3) ? u_f[2 * ns + s] : 0.0;
    }
    const double omega = c->omega, fcoef = c->fcoef;
    const char *gsb = (const char *)gs;
    char *gdb = (char *)gd;
    {
        T.stage(c, psi_f + (int64_t)i * ns, lp);
        T.stage(c, rho_f + (int64_t)i * ns, lr);
        __syncthreads();
        if (!T.active) return;
        double gx, gy, gz, Gx, Gy, Gz;
        T.grad(lp, gx, gy, gz);
        T.grad(lr, Gx, Gy, Gz);
        const double r = lr[T.lc];
        const double rt = r * c->invM[i];
        const double Fx = -rt * gx, Fy = -rt * gy, Fz = -rt * gz;
        if constexpr (KEEP)
            collide_push_keep<L, ST>(P, gsb, gdb, i, T.x, T.y, T.z, nx, ny, nz, r, ux, uy, uz, Fx,
                                     Fy, Fz, Gx, Gy, Gz, omega, fcoef);
        else
            collide_push_tau1<L, ST>(P, gdb, i, T.x, T.y, T.z, nx, ny, nz, r, ux, uy, uz, Fx, Fy,
                                     Fz, Gx, Gy, Gz, omega, fcoef);
    }
}

template <class L, typename ST, bool KEEP>
__global__ __launch_bounds__(TPB) void k_collide_t(const SimConst *__restrict__ c,
                                                   const void *__restrict__ gs, void *__restrict__ gd,
                                                   const double *__restrict__ rho_f,
                                                   const double *__restrict__ psi_f,
                                                   const double *__restrict__ u_f) {
    __shared__ double lp[TileGeom<L, TileC<L>>::NH];
    __shared__ double lr[TileGeom<L, TileC<L>>::NH];
    collide_body<L, ST, KEEP>(c, gs, gd, rho_f, psi_f, u_f, xcd_unit(), lp, lr);
}

// ---- batched passes: many simulations per launch (GenMember table) ------
// The member that owns global work unit u of pass p (-1 past the last one)
// and the unit's index within it; uniform per workgroup.
__device__ __forceinline__ int find_member(const GenMember *__restrict__ m, int nm, int p,
                                           int64_t u, int64_t &local) {
    if (u >= m[nm - 1].end[p]) return -1;
    int lo = 0, hi = nm - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (m[mid].end[p] > u)
            hi = mid;
        else
            lo = mid + 1;
    }
    local = u - (lo ? m[lo - 1].end[p] : 0);
    return lo;
}

template <class L, typename ST>
__global__ __launch_bounds__(TPB) void k_moments_eos_b(const GenMember *__restrict__ m, int nm,
                                                       int flip) {
    int64_t local;
    const int k = find_member(m, nm, 0, blockIdx.x, local);
    if (k < 0) return;
    const GenMember &g = m[k];
    moments_eos_body<L, ST>(g.c, g.buf[g.parity ^ flip], g.rho_f, g.psi_f, g.s_f, g.j_f, g.status,
                            local);
}

template <class L>
__global__ __launch_bounds__(TPB) void k_interface_b(const GenMember *__restrict__ m, int nm) {
    int64_t local;
    const int k = find_member(m, nm, 0, blockIdx.x, local);
    if (k < 0) return;
    interface_body<L>(m[k].c, m[k].s_f, m[k].psi_f, local);
}

template <class L>
__global__ __launch_bounds__(TPB) void k_velocity_b(const GenMember *__restrict__ m, int nm) {
    __shared__ double lp[TileGeom<L, TileV<L>>::NH];
    int64_t local;
    const int k = find_member(m, nm, 1, xcd_unit(), local);
    if (k < 0) return;
    const GenMember &g = m[k];
    velocity_body<L>(g.c, g.rho_f, g.psi_f, g.j_f, g.u_f, (int)local, lp);
}

template <class L, typename ST, bool KEEP>
__global__ __launch_bounds__(TPB) void k_collide_b(const GenMember *__restrict__ m, int nm,
                                                   int flip) {
    __shared__ double lp[TileGeom<L, TileC<L>>::NH];
    __shared__ double lr[TileGeom<L, TileC<L>>::NH];
    int64_t local;
    const int k = find_member(m, nm, 2, xcd_unit(), local);
    if (k < 0) return;
    const GenMember &g = m[k];
    collide_body<L, ST, KEEP>(g.c, g.buf[g.parity ^ flip], g.buf[g.parity ^ flip ^ 1], g.rho_f,
                              g.psi_f, g.u_f, (int)local, lp, lr);
}

// Diagnostics from the macroscopic fields of the current state (rho_i,
// j and the force-corrected u written by the fields pass): per-block
// partial sums over a fixed site assignment, then one fixed-order final
// sum per quantity.  Sums within a wavefront go through DPP lane moves in
// a fixed pattern, the four wavefronts of a block are added in wavefront
// order, and no float atomics are used, so the result is bitwise
// reproducible for a given grid.
//
// Groups (blockIdx.y): y < N is component y: [0] sum_r rho_y,
// [1] sum_r |rho_y - snap_y| (and snap_y <- rho_y); y == N is the
// momentum: [0..3) sum_r j, [3..6) sum_r rho u.  part[y][b][6].
constexpr int DIAG_Q = DIAG_QUANT;

template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront (every lane active), the same
// value on every lane: quad_perm [1,0,3,2] and [2,3,0,1] (quads),
// row_half_mirror (8 lanes), row_mirror (16 lanes), then the four rows.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    v += dpp_move<0x140>(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Block sum of DIAG_Q values per thread into out[DIAG_Q] (thread 0).
__device__ __forceinline__ void block_sum(const double (&v)[DIAG_Q], double *out) {
    __shared__ double ws[TPB / 64][DIAG_Q];
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < DIAG_Q; ++q) {
        const double t = wave_sum(v[q]);
        if ((threadIdx.x & 63) == 0) ws[wv][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < DIAG_Q) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < TPB / 64; ++w) t += ws[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

template <int D>
__global__ __launch_bounds__(TPB) void k_diag_part(int N, int64_t ns, const double *__restrict__ rho_f,
                                                   const double *__restrict__ j_f,
                                                   const double *__restrict__ u_f,
                                                   double *__restrict__ snap,
                                                   double *__restrict__ part, int use_snap) {
    const int y = blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * TPB;
    double v[DIAG_Q] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (y < N) {
        const double *r = rho_f + (int64_t)y * ns;
        double *sn = snap + (int64_t)y * ns;
        for (int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x; s < ns; s += stride) {
            const double rv = r[s];
            v[0] += rv;
            if (use_snap) v[1] += fabs(rv - sn[s]);
            sn[s] = rv;
        }
    } else {
        for (int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x; s < ns; s += stride) {
            double rt = 0.0;
            for (int i = 0; i < N; ++i) rt += rho_f[(int64_t)i * ns + s];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                v[d] += j_f[(int64_t)d * ns + s];
                v[3 + d] += rt * u_f[(int64_t)d * ns + s];
            }
        }
    }
    block_sum(v, part + ((int64_t)y * gridDim.x + blockIdx.x) * DIAG_Q);
}

// Final sums: group y adds its nblk block partials, thread t taking blocks
// t, t + TPB, ... in order; out[y][DIAG_Q].
__global__ __launch_bounds__(TPB) void k_diag_final(const double *__restrict__ part, int nblk,
                                                    double *__restrict__ out) {
    const int y = blockIdx.x;
    double v[DIAG_Q] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += TPB) {
        const double *p = part + ((int64_t)y * nblk + b) * DIAG_Q;
#pragma unroll
        for (int q = 0; q < DIAG_Q; ++q) v[q] += p[q];
    }
    block_sum(v, out + (int64_t)y * DIAG_Q);
}

inline unsigned nblocks(int64_t ns) { return (unsigned)((ns + TPB - 1) / TPB); }

template <class L, typename ST>
hipError_t step_generic_t(const SimConst *c, int ncomp, int64_t ns, int nx, int ny, int nz,
                          const void *gs, void *gd, double *rho_f, double *psi_f, double *s_f,
                          double *j_f, double *u_f, uint32_t *status, bool keep,
                          hipStream_t st) {
    const unsigned nb = nblocks(ns);
    const unsigned vb = unit_blocks(TileGeom<L, TileV<L>>::count(nx, ny, nz));
    const unsigned cb = unit_blocks(TileGeom<L, TileC<L>>::count(nx, ny, nz) * ncomp);
    hipLaunchKernelGGL((k_moments_eos<L, ST>), dim3(nb), dim3(TPB), 0, st, c, gs, rho_f, psi_f,
                       s_f, j_f, status);
    hipLaunchKernelGGL((k_interface<L>), dim3(nb), dim3(TPB), 0, st, c, s_f, psi_f);
    hipLaunchKernelGGL((k_velocity_t<L>), dim3(vb), dim3(TPB), 0, st, c, rho_f, psi_f, j_f, u_f);
    if (keep)
        hipLaunchKernelGGL((k_collide_t<L, ST, true>), dim3(cb), dim3(TPB), 0, st, c, gs, gd,
                           rho_f, psi_f, u_f);
    else
        hipLaunchKernelGGL((k_collide_t<L, ST, false>), dim3(cb), dim3(TPB), 0, st, c, gs, gd,
                           rho_f, psi_f, u_f);
    return hipGetLastError();
}

template <class L, typename ST>
hipError_t fields_generic_t(const SimConst *c, int nx, int ny, int nz, const void *g, double *rho_f,
                            double *psi_f, double *s_f, double *j_f, double *u_f,
                            uint32_t *status, hipStream_t st) {
    const unsigned nb = nblocks((int64_t)nx * ny * nz);
    hipLaunchKernelGGL((k_moments_eos<L, ST>), dim3(nb), dim3(TPB), 0, st, c, g, rho_f, psi_f,
                       s_f, j_f, status);
    hipLaunchKernelGGL((k_interface<L>), dim3(nb), dim3(TPB), 0, st, c, s_f, psi_f);
    if (u_f) {
        const unsigned vb = unit_blocks(TileGeom<L, TileV<L>>::count(nx, ny, nz));
        hipLaunchKernelGGL((k_velocity_t<L>), dim3(vb), dim3(TPB), 0, st, c, rho_f, psi_f, j_f,
                           u_f);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init(int lattice, bool fp32, const SimConst *c, int64_t ns, const double *rho,
                       void *g, hipStream_t st) {
    const unsigned nb = nblocks(ns);
    if (lattice == 0) {
        if (fp32) hipLaunchKernelGGL((k_init<D2Q9, float>), dim3(nb), dim3(TPB), 0, st, c, rho, g);
        else hipLaunchKernelGGL((k_init<D2Q9, double>), dim3(nb), dim3(TPB), 0, st, c, rho, g);
    } else {
        if (fp32) hipLaunchKernelGGL((k_init<D3Q19, float>), dim3(nb), dim3(TPB), 0, st, c, rho, g);
        else hipLaunchKernelGGL((k_init<D3Q19, double>), dim3(nb), dim3(TPB), 0, st, c, rho, g);
    }
    return hipGetLastError();
}

hipError_t launch_step_generic(int lattice, bool fp32, const SimConst *c, int ncomp, int nx, int ny,
                               int nz, const void *gs, void *gd, double *rho_f, double *psi_f,
                               double *s_f, double *j_f, double *u_f, uint32_t *status,
                               bool keep_old, hipStream_t st) {
    const int64_t ns = (int64_t)nx * ny * nz;
    const bool k = keep_old;
    if (lattice == 0)
        return fp32 ? step_generic_t<D2Q9, float>(c, ncomp, ns, nx, ny, nz, gs, gd, rho_f, psi_f, s_f, j_f, u_f, status, k, st)
                    : step_generic_t<D2Q9, double>(c, ncomp, ns, nx, ny, nz, gs, gd, rho_f, psi_f, s_f, j_f, u_f, status, k, st);
    return fp32 ? step_generic_t<D3Q19, float>(c, ncomp, ns, nx, ny, nz, gs, gd, rho_f, psi_f, s_f, j_f, u_f, status, k, st)
                : step_generic_t<D3Q19, double>(c, ncomp, ns, nx, ny, nz, gs, gd, rho_f, psi_f, s_f, j_f, u_f, status, k, st);
}

void generic_units(int lattice, int ncomp, int nx, int ny, int nz, int64_t units[3]) {
    units[0] = ((int64_t)nx * ny * nz + TPB - 1) / TPB;
    if (lattice == 0) {
        units[1] = TileGeom<D2Q9, TileV<D2Q9>>::count(nx, ny, nz);
        units[2] = TileGeom<D2Q9, TileC<D2Q9>>::count(nx, ny, nz) * ncomp;
    } else {
        units[1] = TileGeom<D3Q19, TileV<D3Q19>>::count(nx, ny, nz);
        units[2] = TileGeom<D3Q19, TileC<D3Q19>>::count(nx, ny, nz) * ncomp;
    }
}

template <class L, typename ST>
hipError_t step_batch_t(bool keep, const GenMember *m, int nm, const int64_t total[3], int flip,
                        hipStream_t st) {
    const unsigned nb = (unsigned)total[0];
    const unsigned vb = unit_blocks(total[1]);
    const unsigned cb = unit_blocks(total[2]);
    hipLaunchKernelGGL((k_moments_eos_b<L, ST>), dim3(nb), dim3(TPB), 0, st, m, nm, flip);
    hipLaunchKernelGGL((k_interface_b<L>), dim3(nb), dim3(TPB), 0, st, m, nm);
    hipLaunchKernelGGL((k_velocity_b<L>), dim3(vb), dim3(TPB), 0, st, m, nm);
    if (keep)
        hipLaunchKernelGGL((k_collide_b<L, ST, true>), dim3(cb), dim3(TPB), 0, st, m, nm, flip);
    else
        hipLaunchKernelGGL((k_collide_b<L, ST, false>), dim3(cb), dim3(TPB), 0, st, m, nm, flip);
    return hipGetLastError();
}

hipError_t launch_step_generic_batch(int lattice, bool fp32, bool keep_old,
                                     const GenMember *members, int nmembers,
                                     const int64_t total[3], int flip, hipStream_t st) {
    if (nmembers < 1) return hipSuccess;
    if (lattice == 0)
        return fp32 ? step_batch_t<D2Q9, float>(keep_old, members, nmembers, total, flip, st)
                    : step_batch_t<D2Q9, double>(keep_old, members, nmembers, total, flip, st);
    return fp32 ? step_batch_t<D3Q19, float>(keep_old, members, nmembers, total, flip, st)
                : step_batch_t<D3Q19, double>(keep_old, members, nmembers, total, flip, st);
}

hipError_t launch_fields(int lattice, bool fp32, const SimConst *c, int nx, int ny, int nz,
                         const void *g, double *rho_f, double *psi_f, double *s_f, double *j_f,
                         double *u_f, uint32_t *status, hipStream_t st) {
    if (lattice == 0)
        return fp32 ? fields_generic_t<D2Q9, float>(c, nx, ny, nz, g, rho_f, psi_f, s_f, j_f, u_f, status, st)
                    : fields_generic_t<D2Q9, double>(c, nx, ny, nz, g, rho_f, psi_f, s_f, j_f, u_f, status, st);
    return fp32 ? fields_generic_t<D3Q19, float>(c, nx, ny, nz, g, rho_f, psi_f, s_f, j_f, u_f, status, st)
                : fields_generic_t<D3Q19, double>(c, nx, ny, nz, g, rho_f, psi_f, s_f, j_f, u_f, status, st);
}

hipError_t launch_diag(int dim, int ncomp, int64_t ns, const double *rho_f, const double *j_f,
                       const double *u_f, double *snap, double *part, int nblk, double *out,
                       int use_snap, hipStream_t st) {
    const dim3 grid(nblk, ncomp + 1);
    if (dim == 2)
        hipLaunchKernelGGL(k_diag_part<2>, grid, dim3(TPB), 0, st, ncomp, ns, rho_f, j_f, u_f,
                           snap, part, use_snap);
    else
        hipLaunchKernelGGL(k_diag_part<3>, grid, dim3(TPB), 0, st, ncomp, ns, rho_f, j_f, u_f,
                           snap, part, use_snap);
    hipLaunchKernelGGL(k_diag_final, dim3(ncomp + 1), dim3(TPB), 0, st, part, nblk, out);
    return hipGetLastError();
}

int diag_blocks(int64_t ns) {
    const int64_t b = (ns + TPB - 1) / TPB;
    return (int)(b < 1024 ? b : 1024);
}
