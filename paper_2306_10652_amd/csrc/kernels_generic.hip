// Multi-pass step for any lattice (D2Q9, D3Q19), FP64 or FP32 storage
// (population layout: PopLayout of the common header):
//   pass 1  moments + local cubic-EOS fugacity: rho_i, RT ln f_i, s = sum sqrt(kappa_j) rt_j, j
//   pass 2  psi_i = RT ln f_i - sqrt(kappa_i) lap(s)             (Eq. (4)-(5))
//   pass 3  u = (j + F/2) / rho, F = -sum_i rt_i grad psi_i      (LDS tiles)
//   pass 4  F_i, G_i = grad rho_i, collide (Eq. (1)), push        (LDS tiles)
// One thread per site; fields between passes live in the simulation's
// workspace.  Also: initial populations, the macroscopic read-out and the
// per-block diagnostic partial sums.
#include "kernels.h"

namespace {

constexpr int TPB = 256;

template <class L>
__device__ __forceinline__ int64_t nb_site(int x, int y, int z, int a, int nx, int ny, int nz) {
    int xx = x + L::ex(a), yy = y + L::ey(a), zz = z + L::ez(a);
    xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
    yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
    zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
    return (int64_t)xx + (int64_t)nx * ((int64_t)yy + (int64_t)ny * zz);
}

// Lattice gradient in pairwise-difference form; phi(site) read through f.
template <class L, class Fn>
__device__ __forceinline__ void lattice_grad(const int64_t *nb, Fn f, double &gx, double &gy,
                                             double &gz) {
    gx = gy = gz = 0.0;
#pragma unroll
    for (int a = 1; a < L::Q; ++a) {
        // visit each opposite pair once: the member with the first non-zero
        // component positive
        const int fx = L::ex(a), fy = L::ey(a), fz = L::ez(a);
        const bool first = fx > 0 || (fx == 0 && (fy > 0 || (fy == 0 && fz > 0)));
        if (!first) continue;
        int o = 0;
#pragma unroll
        for (int b = 1; b < L::Q; ++b)
            if (L::ex(b) == -fx && L::ey(b) == -fy && L::ez(b) == -fz) o = b;
        const double d = f(nb[a]) - f(nb[o]);
        const double wd = L::w(a) * d;
        gx += fx * wd;
        gy += fy * wd;
        gz += fz * wd;
    }
    gx *= 3.0;
    gy *= 3.0;
    gz *= 3.0;
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

template <class L, typename ST>
__global__ __launch_bounds__(TPB) void k_moments_eos(const SimConst *__restrict__ c,
                                                     const void *__restrict__ g,
                                                     double *__restrict__ rho_f,
                                                     double *__restrict__ psi_f,
                                                     double *__restrict__ s_f,
                                                     double *__restrict__ j_f,
                                                     uint32_t *__restrict__ status) {
    const int64_t ns = c->nsites;
    const int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x;
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
                const double v = ld_pop<ST>(g, P, row, i, a, xs);
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

template <class L>
__global__ __launch_bounds__(TPB) void k_interface(const SimConst *__restrict__ c,
                                                   const double *__restrict__ s_f,
                                                   double *__restrict__ psi_f) {
    const int64_t ns = c->nsites;
    const int64_t s = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (s >= ns) return;
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const int x = (int)(s % nx), y = (int)((s / nx) % ny), z = (int)(s / ((int64_t)nx * ny));
    const double sc = s_f[s];
    double acc = 0.0;
#pragma unroll
    for (int a = 1; a < L::Q; ++a)
        acc += L::w(a) * (s_f[nb_site<L>(x, y, z, a, nx, ny, nz)] - sc);
    const double lap = 6.0 * acc;
    const int N = c->N;
    for (int i = 0; i < N; ++i) psi_f[(int64_t)i * ns + s] -= c->sqk[i] * lap;
}

// ---- LDS-tiled force, velocity and collision --------------------------------
// A workgroup owns a tile of TX x TY x TZ sites (one thread per site) and
// stages psi_i (and rho_i) over the tile plus a one-site halo in LDS, so
// every neighbour value is read from HBM/L2 once per tile instead of once
// per neighbour.
//
// Collision tiles are 64 sites wide: a wavefront covers 64 consecutive x
// sites of one row, so each of its population stores is one 512 B (FP64) /
// 256 B (FP32) run.  The velocity pass only reads, and takes the shape with
// the smallest halo.
//
// Tiles are numbered x-fastest (collision units: collide_unit), and each
// XCD takes a contiguous range of work units
// (workgroups go to the XCDs round-robin).  The units that write a lattice
// row's blocks and the partly written cache lines at tile edges then run
// at the same time on the same L2, and the pages being written at any
// moment are few.
template <class L> struct TileC;
template <> struct TileC<D2Q9> { static constexpr int TX = 64, TY = 4, TZ = 1, HZ = 0; };
template <> struct TileC<D3Q19> { static constexpr int TX = 64, TY = 2, TZ = 2, HZ = 1; };
template <class L> struct TileV;
template <> struct TileV<D2Q9> { static constexpr int TX = 64, TY = 4, TZ = 1, HZ = 0; };
template <> struct TileV<D3Q19> { static constexpr int TX = 16, TY = 4, TZ = 4, HZ = 1; };
constexpr int TILE_XCDS = 8;

// This workgroup's work unit; gridDim.x is a multiple of TILE_XCDS
// (unit_blocks), units at or past the real count are padding.
__device__ __forceinline__ int xcd_unit() {
    const int per = (int)gridDim.x / TILE_XCDS;
    return (int)(blockIdx.x % TILE_XCDS) * per + (int)(blockIdx.x / TILE_XCDS);
}

inline unsigned unit_blocks(int64_t units) {
    return (unsigned)((units + TILE_XCDS - 1) / TILE_XCDS * TILE_XCDS);
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

template <class L, class S>
struct TileGeom {
    static constexpr int TX = S::TX, TY = S::TY, TZ = S::TZ, HZ = S::HZ;
    static constexpr int HX = TX + 2, HY = TY + 2, HZN = TZ + 2 * HZ;
    static constexpr int NH = HX * HY * HZN;   // halo tile points
    static_assert(TX * TY * TZ == TPB, "one thread per tile site");
    int x0, y0, z0, lx, ly, lz, x, y, z;
    bool active;
    int lc;      // LDS index of this thread's site
    __host__ __device__ static int64_t count(int nx, int ny, int nz) {
        return (int64_t)((nx + TX - 1) / TX) * ((ny + TY - 1) / TY) * ((nz + TZ - 1) / TZ);
    }
    // tile b < count(nx, ny, nz), numbered x-fastest
    __device__ TileGeom(const SimConst *c, int b) {
        const int ntx = (c->nx + TX - 1) / TX, nty = (c->ny + TY - 1) / TY;
        x0 = (b % ntx) * TX;
        y0 = ((b / ntx) % nty) * TY;
        z0 = (b / (ntx * nty)) * TZ;
        const int t = threadIdx.x;
        lx = t % TX;
        ly = (t / TX) % TY;
        lz = t / (TX * TY);
        x = x0 + lx;
        y = y0 + ly;
        z = z0 + lz;
        active = x < c->nx && y < c->ny && z < c->nz;
        lc = ((lz + HZ) * HY + (ly + 1)) * HX + (lx + 1);
    }
    __device__ static int lds_off(int a) { return (L::ez(a) * HY + L::ey(a)) * HX + L::ex(a); }
    // periodic image of v >= -1 (a tile can be wider than the grid)
    __device__ static int wrap(int v, int n) {
        v = v < 0 ? v + n : v;
        while (v >= n) v -= n;
        return v;
    }
    // stage field f (one component plane of ns values) into lds[NH]; each
    // thread issues all of its loads before its first LDS write, so the
    // loads are in flight together
    __device__ void stage(const SimConst *c, const double *f, double *lds) const {
        const int nx = c->nx, ny = c->ny, nz = c->nz;
        if constexpr (TX == 64) {
            // a wavefront stages whole halo rows (HX = 66 x sites): one
            // y/z wrap per row, one wrapped x per lane for all rows
            constexpr int NW = TPB / 64;
            const int lane = threadIdx.x & 63;
            const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
            const int gx0 = wrap(x0 - 1 + lane, nx);
            const int gx1 = wrap(x0 + 63 + (lane & 1), nx);   // halo x = 64, 65
            constexpr int NR = (HY * HZN + NW - 1) / NW;   // rows per wavefront
            double v0[NR], v1[NR];
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const int row = wv + j * NW;
                if (row < HY * HZN) {
                    const int hy = row % HY, hz = row / HY;
                    const int gy = wrap(y0 - 1 + hy, ny), gz = wrap(z0 - HZ + hz, nz);
                    const double *fr = f + (int64_t)nx * ((int64_t)gy + (int64_t)ny * gz);
                    v0[j] = fr[gx0];
                    v1[j] = fr[gx1];
                }
            }
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const int row = wv + j * NW;
                if (row < HY * HZN) {
                    lds[row * HX + lane] = v0[j];
                    if (lane < 2) lds[row * HX + 64 + lane] = v1[j];
                }
            }
        } else {
            // NK halo points per thread
            constexpr int NK = (NH + TPB - 1) / TPB;
            double v[NK];
#pragma unroll
            for (int j = 0; j < NK; ++j) {
                const int k = (int)threadIdx.x + j * TPB;
                if (k < NH) {
                    const int hx = k % HX, hy = (k / HX) % HY, hz = k / (HX * HY);
                    const int gx = wrap(x0 - 1 + hx, nx), gy = wrap(y0 - 1 + hy, ny),
                              gz = wrap(z0 - HZ + hz, nz);
                    v[j] = f[(int64_t)gx + (int64_t)nx * ((int64_t)gy + (int64_t)ny * gz)];
                }
            }
#pragma unroll
            for (int j = 0; j < NK; ++j) {
                const int k = (int)threadIdx.x + j * TPB;
                if (k < NH) lds[k] = v[j];
            }
        }
    }
    __device__ void grad(const double *lds, double &gx, double &gy, double &gz) const {
        int nb[L::Q];
#pragma unroll
        for (int a = 0; a < L::Q; ++a) nb[a] = lc + lds_off(a);
        int64_t nb64[L::Q];
#pragma unroll
        for (int a = 0; a < L::Q; ++a) nb64[a] = nb[a];
        lattice_grad<L>(nb64, [&](int64_t t) { return lds[t]; }, gx, gy, gz);
    }
};

// u = (j + F/2) / rho, F = sum_i F_i, F_i = -rt_i grad psi_i  -> u_f
template <class L>
__global__ __launch_bounds__(TPB) void k_velocity_t(const SimConst *__restrict__ c,
                                                    const double *__restrict__ rho_f,
                                                    const double *__restrict__ psi_f,
                                                    const double *__restrict__ j_f,
                                                    double *__restrict__ u_f) {
    using TG = TileGeom<L, TileV<L>>;
    __shared__ double lp[TG::NH];
    const int unit = xcd_unit();
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
            Fx -= rt * gx;
            Fy -= rt * gy;
            Fz -= rt * gz;
            rhot += r;
        }
    }
    if (!T.active) return;
    u_f[s] = (j_f[s] + 0.5 * Fx) / rhot;
    u_f[ns + s] = (j_f[ns + s] + 0.5 * Fy) / rhot;
    if (L::D == 3) u_f[2 * ns + s] = (j_f[2 * ns + s] + 0.5 * Fz) / rhot;
}

// collision (Eq. (1a)-(1c)) and push of one component over one tile
// (collide_unit); u from u_f
// KEEP: tau != 1, so the collision keeps (1 - omega) g of the old population.
template <class L, typename ST, bool KEEP>
__global__ __launch_bounds__(TPB) void k_collide_t(const SimConst *__restrict__ c,
                                                   const void *__restrict__ gs, void *__restrict__ gd,
                                                   const double *__restrict__ rho_f,
                                                   const double *__restrict__ psi_f,
                                                   const double *__restrict__ u_f) {
    using TG = TileGeom<L, TileC<L>>;
    __shared__ double lp[TG::NH];
    __shared__ double lr[TG::NH];
    const int N = c->N;
    const int unit = xcd_unit();
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
    const int64_t row = (int64_t)T.y + (int64_t)ny * T.z;
    double ux = 0.0, uy = 0.0, uz = 0.0;
    if (T.active) {
        ux = u_f[s];
        uy = u_f[ns + s];
        uz = (L::D == 3) ? u_f[2 * ns + s] : 0.0;
    }
    const double uu = ux * ux + uy * uy + uz * uz;
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
        const double Fu = Fx * ux + Fy * uy + Fz * uz;
        const double Gu = Gx * ux + Gy * uy + Gz * uz;
        // moving populations first; in FP32 storage their rounding error
        // goes into the rest population, which stays at this site.  At
        // tau = 1 the collision does not depend on the old populations
        // (their moments came from the first pass): they are not read.
        double err = 0.0;
        // tau = 1: collide_one for a moving direction with the site's terms
        // taken out of the direction loop: g^eq_a - w_a rho = w_a rho sq_a and
        // F_a / w_a = 3 eF + 9 eu eF + 3 eu eG + K, where K depends on |e_a|^2
        // only (weight classes |e|^2 = 1 and 2); the dot products with e_a
        // add only its non-zero components (0 * u is not folded away)
        const double c0 = -1.5 * uu;
        const double K1 = -3.0 * Fu - Gu + 0.5 * (3.0 - (double)L::D) * Gu;
        const double K2 = -3.0 * Fu - Gu + 0.5 * (6.0 - (double)L::D) * Gu;
        const double A1 = omega * L::w(1) * r, A2 = omega * L::w(L::Q - 1) * r;
        const double B1 = fcoef * L::w(1), B2 = fcoef * L::w(L::Q - 1);
        auto edot = [](int a, double x, double y, double z) {
            const int cx = L::ex(a), cy = L::ey(a), cz = L::ez(a);
            const double tx = cx > 0 ? x : -x, ty = cy > 0 ? y : -y, tz = cz > 0 ? z : -z;
            if (cx != 0) return cy != 0 ? tx + ty : (cz != 0 ? tx + tz : tx);
            return cy != 0 ? (cz != 0 ? ty + tz : ty) : tz;
        };
        auto dir = [&](int a) {
            double o;
            if constexpr (KEEP) {
                const double gv = (double)*(const ST *)(gsb + P.move(row, i, a, T.x));
                o = collide_one<L>(a, gv, r, ux, uy, uz, Fx, Fy, Fz, Gx, Gy, Gz, uu, Fu, Gu,
                                   omega, fcoef);
            } else {
                const double eu = edot(a, ux, uy, uz);
                const double eF = edot(a, Fx, Fy, Fz);
                const double eG = edot(a, Gx, Gy, Gz);
                const bool e1 = L::ex(a) * L::ex(a) + L::ey(a) * L::ey(a) +
                                L::ez(a) * L::ez(a) == 1;
                const double sq = fma(eu, fma(4.5, eu, 3.0), c0);
                const double q = fma(eF, fma(9.0, eu, 3.0), fma(3.0 * eu, eG, e1 ? K1 : K2));
                o = fma(e1 ? A1 : A2, sq, (e1 ? B1 : B2) * q);
            }
            const ST v = (ST)o;
            if (sizeof(ST) == 4) err += (double)v - o;
            int xx = T.x + L::ex(a), yy = T.y + L::ey(a), zz = T.z + L::ez(a);
            xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
            yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
            zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
            *(ST *)(gdb + P.move((int64_t)yy + (int64_t)ny * zz, i, a, xx)) = v;
        };
        if constexpr (KEEP) {
            // rolled: unrolled, the compiler hoists every load and the
            // kernel needs 256 registers (one wavefront per SIMD)
#pragma unroll 2
            for (int a = 1; a < L::Q; ++a) dir(a);
        } else {
            // no loads: unrolled, the lattice vectors, weights and
            // destination rows fold to constants per direction
#pragma unroll
            for (int a = 1; a < L::Q; ++a) dir(a);
        }
        const double g0 = KEEP ? *(const double *)(gsb + P.rest(row, i, T.x)) : 0.0;
        const double o0 = collide_one<L>(0, g0, r, ux, uy, uz, Fx, Fy, Fz, Gx, Gy, Gz, uu, Fu, Gu,
                                         omega, fcoef);
        *(double *)(gdb + P.rest(row, i, T.x)) = sizeof(ST) == 4 ? o0 - err : o0;
    }
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
