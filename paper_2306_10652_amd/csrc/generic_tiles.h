// LDS-tiled stencil machinery of the multi-pass kernels: the workgroup
// size, the lattice gradient, tile shapes, XCD-aware work-unit numbering,
// the tile geometry with its halo staging, and the collision-and-push of
// one component at one site.
#pragma once

#include "kernels.h"

namespace {

constexpr int TPB = 256;


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

// Store of one new population.  Where the layout keeps a collision's
// stores in whole aligned rows (L::PULL_X, see pop_col), nontemporal: the
// values are read again only by the next step's moments pass, after the
// whole field has been written (D3Q19 at 128^3 x 10: the step 2.9 % faster
// in FP64, 2.1 % with FP32 storage).  Shifted rows (D2Q9) share their edge
// lines with the neighbouring tiles and rely on L2 to merge those partial
// writes: plain stores.
template <class L, typename T>
__device__ __forceinline__ void put_pop(T *p, T v) {
    if constexpr (L::PULL_X)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Collision of component i at one site at tau = 1, Eq. (1a)-(1c) with
// omega = 1: the old population drops out, so it is not read (its moments
// came from the moments pass), and the terms of the site are taken out of
// the direction loop: g^eq_a - w_a rho = w_a rho sq_a and
// F_a / w_a = 3 eF + 9 eu eF + 3 eu eG + K, where K depends on |e_a|^2 only
// (weight classes |e|^2 = 1 and 2); the dot products with e_a add only its
// non-zero components (0 * u is not folded away).  The moving populations
// are pushed to x + e_a (periodic; in y and z only where pop_col says so),
// the rest one stays.  In FP32 storage the moving populations are computed
// in FP32 arithmetic from the per-site terms rounded once (as in the fused
// D2Q9 kernels), and the rest population is rho minus the FP64 sum of the
// stored moving values (in direction order): the collision conserves each
// component's mass, so this keeps it to FP64 rounding.  The FP32 loop
// stores each direction before computing the next (a scheduling barrier):
// left free, the compiler computes every direction first and holds them
// all (109 VGPRs with FP64 arithmetic; 63 in order with FP32 arithmetic,
// eight wavefronts per SIMD).
template <class L, typename ST>
__device__ __forceinline__ void collide_push_tau1(const PopLayout<ST> &P, char *gdb, int i, int x,
                                                  int y, int z, int nx, int ny, int nz, double r,
                                                  double ux, double uy, double uz, double Fx,
                                                  double Fy, double Fz, double Gx, double Gy,
                                                  double Gz, double omega, double fcoef) {
    // the inputs as plain register values (empty register constraints, no
    // instruction): otherwise a caller that has just computed F_i as a
    // product lets the compiler fuse that product into e_a.F, and the
    // rounding would depend on the caller
    asm volatile("" : "+v"(r), "+v"(ux), "+v"(uy), "+v"(uz), "+v"(Fx), "+v"(Fy), "+v"(Fz),
                 "+v"(Gx), "+v"(Gy), "+v"(Gz));
    const double uu = ux * ux + uy * uy + uz * uz;
    const double Fu = Fx * ux + Fy * uy + Fz * uz;
    const double Gu = Gx * ux + Gy * uy + Gz * uz;
    const double c0 = -1.5 * uu;
    const double K1 = -3.0 * Fu - Gu + 0.5 * (3.0 - (double)L::D) * Gu;
    const double K2 = -3.0 * Fu - Gu + 0.5 * (6.0 - (double)L::D) * Gu;
    const double A1 = omega * L::w(1) * r, A2 = omega * L::w(L::Q - 1) * r;
    const double B1 = fcoef * L::w(1), B2 = fcoef * L::w(L::Q - 1);
    auto edot = [](int a, auto ex, auto ey, auto ez) {
        const int cx = L::ex(a), cy = L::ey(a), cz = L::ez(a);
        const auto tx = cx > 0 ? ex : -ex, ty = cy > 0 ? ey : -ey, tz = cz > 0 ? ez : -ez;
        if (cx != 0) return cy != 0 ? tx + ty : (cz != 0 ? tx + tz : tx);
        return cy != 0 ? (cz != 0 ? ty + tz : ty) : tz;
    };
    // push; in x only where the layout does (pop_col)
    auto store = [&](int a, ST v) {
        int xx = L::PULL_X ? x : x + L::ex(a), yy = y + L::ey(a), zz = z + L::ez(a);
        xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
        put_pop<L>((ST *)(gdb + P.move((int64_t)yy + (int64_t)ny * zz, i, a, xx)), v);
    };
    // no loads: unrolled, the lattice vectors, weights and destination rows
    // fold to constants per direction
    if constexpr (sizeof(ST) == 4) {
        const float fux = (float)ux, fuy = (float)uy, fuz = (float)uz;
        const float fFx = (float)Fx, fFy = (float)Fy, fFz = (float)Fz;
        const float fGx = (float)Gx, fGy = (float)Gy, fGz = (float)Gz;
        const float fc0 = (float)c0, fK1 = (float)K1, fK2 = (float)K2;
        const float fA1 = (float)A1, fA2 = (float)A2, fB1 = (float)B1, fB2 = (float)B2;
        double msum = 0.0;
#pragma unroll
        for (int a = 1; a < L::Q; ++a) {
            const float eu = edot(a, fux, fuy, fuz);
            const float eF = edot(a, fFx, fFy, fFz);
            const float eG = edot(a, fGx, fGy, fGz);
            const bool e1 = L::ex(a) * L::ex(a) + L::ey(a) * L::ey(a) + L::ez(a) * L::ez(a) == 1;
            const float sq = fmaf(eu, fmaf(4.5f, eu, 3.0f), fc0);
            const float q = fmaf(eF, fmaf(9.0f, eu, 3.0f), fmaf(3.0f * eu, eG, e1 ? fK1 : fK2));
            const float v = fmaf(e1 ? fA1 : fA2, sq, (e1 ? fB1 : fB2) * q);
            msum += (double)v;
            store(a, (ST)v);
            __builtin_amdgcn_sched_barrier(0);
        }
        put_pop<L>((double *)(gdb + P.rest((int64_t)y + (int64_t)ny * z, i, x)), r - msum);
    } else {
#pragma unroll
        for (int a = 1; a < L::Q; ++a) {
            const double eu = edot(a, ux, uy, uz);
            const double eF = edot(a, Fx, Fy, Fz);
            const double eG = edot(a, Gx, Gy, Gz);
            const bool e1 = L::ex(a) * L::ex(a) + L::ey(a) * L::ey(a) + L::ez(a) * L::ez(a) == 1;
            const double sq = fma(eu, fma(4.5, eu, 3.0), c0);
            const double q = fma(eF, fma(9.0, eu, 3.0), fma(3.0 * eu, eG, e1 ? K1 : K2));
            store(a, (ST)fma(e1 ? A1 : A2, sq, (e1 ? B1 : B2) * q));
        }
        put_pop<L>((double *)(gdb + P.rest((int64_t)y + (int64_t)ny * z, i, x)),
                   collide_one<L>(0, 0.0, r, ux, uy, uz, Fx, Fy, Fz, Gx, Gy, Gz, uu, Fu, Gu, omega,
                                  fcoef));
    }
}

// Collision of component i at one site at tau != 1 (Eq. (1a)-(1c)): reads
// the old populations of the site (the moving ones at their pop_col
// columns), pushes the new ones as collide_push_tau1 does; in FP32 storage
// the moving populations' rounding error is folded into the rest one.
template <class L, typename ST>
__device__ __forceinline__ void collide_push_keep(const PopLayout<ST> &P, const char *gsb,
                                                  char *gdb, int i, int x, int y, int z, int nx,
                                                  int ny, int nz, double r, double ux, double uy,
                                                  double uz, double Fx, double Fy, double Fz,
                                                  double Gx, double Gy, double Gz, double omega,
                                                  double fcoef) {
    asm volatile("" : "+v"(r), "+v"(ux), "+v"(uy), "+v"(uz), "+v"(Fx), "+v"(Fy), "+v"(Fz),
                 "+v"(Gx), "+v"(Gy), "+v"(Gz));
    const double uu = ux * ux + uy * uy + uz * uz;
    const double Fu = Fx * ux + Fy * uy + Fz * uz;
    const double Gu = Gx * ux + Gy * uy + Gz * uz;
    const int64_t row = (int64_t)y + (int64_t)ny * z;
    double err = 0.0;
    auto dir = [&](int a) {
        const double gv = (double)*(const ST *)(gsb + P.move(row, i, a, pop_col<L>(a, x, nx)));
        const double o = collide_one<L>(a, gv, r, ux, uy, uz, Fx, Fy, Fz, Gx, Gy, Gz, uu, Fu, Gu,
                                        omega, fcoef);
        const ST v = (ST)o;
        if (sizeof(ST) == 4) err += (double)v - o;
        int xx = L::PULL_X ? x : x + L::ex(a), yy = y + L::ey(a), zz = z + L::ez(a);
        xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        zz = zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz);
        put_pop<L>((ST *)(gdb + P.move((int64_t)yy + (int64_t)ny * zz, i, a, xx)), v);
    };
    // rolled: unrolled, the compiler hoists every load and the kernel needs
    // 256 registers (one wavefront per SIMD)
#pragma unroll 2
    for (int a = 1; a < L::Q; ++a) dir(a);
    const double g0 = *(const double *)(gsb + P.rest(row, i, x));
    const double o0 = collide_one<L>(0, g0, r, ux, uy, uz, Fx, Fy, Fz, Gx, Gy, Gz, uu, Fu, Gu,
                                     omega, fcoef);
    put_pop<L>((double *)(gdb + P.rest(row, i, x)), sizeof(ST) == 4 ? o0 - err : o0);
}

}  // namespace
