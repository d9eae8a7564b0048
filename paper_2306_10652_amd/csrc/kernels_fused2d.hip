// Fused one-pass D2Q9 step (moments -> PR fugacity -> interface potential ->
// force -> collide -> push-stream) for gfx950.
//
// Work item = a 64-column strip (60 output columns plus a 2-column halo on
// each side) of one simulation, marching up `rows` output rows.  The
// workgroup has one wavefront per component (lane = column): a lane keeps
// only its own component's 9 populations of the rows in flight, in
// registers.  Sums over components go through LDS.  Per lead row r (output
// row y = r - 2), with three workgroup barriers:
//
//   A  (all)  moments of row r -> LDS: rt_i, j_i
//   B  (all)  row r-1: Sraw_i = sum_j (a alpha)_ij rt_j  -> LDS: rt_i Sraw_i
//             G_i(y) = grad rho_i from the register ring
//   -- barrier --
//   M  (one wave, rotating)  row r: rt, b_m rt, s, rho, j totals -> LDS rings
//             row r-1: a_m and the three mixture coefficients of
//             RT ln f_i = RT ln(rt_i c1) + b_i c2 - c3 Sraw_i      (Eq. (9)-(12))
//   -- barrier --
//   C  (all)  psi_i(r-1) = RT ln f_i - sqrt(kappa_i) lap s     (Eq. (3)-(5))
//   D  (all)  F_i(y) = -rt_i grad psi_i                 -> LDS
//   -- barrier --
//   E  (all)  u(y) = (j + F/2) / rho, collide row y (Eq. (1)), push-store
//
// Every population is read from HBM once per step; the 4 halo columns and
// the 4 warm-up rows of a work item are re-reads that neighbouring items
// issue at about the same time (the item order keeps them on one XCD).
#include "kernels.h"

namespace {

// Address-space-qualified views: constant (scalar loads) and global.
template <class T> using cptr = const __attribute__((address_space(4))) T *;
template <class T> using gptr = const __attribute__((address_space(1))) T *;
template <class T> using gmptr = __attribute__((address_space(1))) T *;

// DPP wavefront shifts (GFX9 family): lane l receives lane l-1 (wave_shr:1)
// or lane l+1 (wave_shl:1).  Lanes 0 / 63 receive 0; only lanes 1..62 use
// shifted values.
__device__ __forceinline__ double from_left(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Pairwise-difference D2Q9 gradient from a 3x3 neighbourhood
// (S = row below, C = own row, N = row above; W/E via lane shifts).
__device__ __forceinline__ void grad3(double S, double C, double N, double &gx, double &gy) {
    const double W = from_left(C), E = from_right(C);
    const double SW = from_left(S), SE = from_right(S);
    const double NW = from_left(N), NE = from_right(N);
    const double d1 = E - W, d2 = N - S, d5 = NE - SW, d6 = NW - SE;
    gx = 3.0 * ((1.0 / 9.0) * d1 + (1.0 / 36.0) * d5 - (1.0 / 36.0) * d6);
    gy = 3.0 * ((1.0 / 9.0) * d2 + (1.0 / 36.0) * d5 + (1.0 / 36.0) * d6);
}

__device__ __forceinline__ double lap3(double S, double C, double N) {
    const double W = from_left(C), E = from_right(C);
    const double SW = from_left(S), SE = from_right(S);
    const double NW = from_left(N), NE = from_right(N);
    const double ax = (E - C) + (N - C) + (W - C) + (S - C);
    const double dg = (NE - C) + (NW - C) + (SW - C) + (SE - C);
    return 6.0 * ((1.0 / 9.0) * ax + (1.0 / 36.0) * dg);
}

template <int NC>
struct FusedLds {
    double rt[2][NC][64];   // molar densities of rows r-1, r (slot = row & 1)
    double jx[NC][64];      // per-component momentum of row r
    double jy[NC][64];
    double xs[NC][64];      // rt_i Sraw_i of row r-1
    double fx[NC][64];      // per-component force of row y
    double fy[NC][64];
    double tot[4][4][64];   // ring over rows (slot = row & 3): s, rho, jx, jy
    double mx[2][2][64];    // ring over rows (slot = row & 1): rt, b_m rt
    double eos[3][64];      // c1, c2, c3 of row r-1
};

template <int NC, typename ST>
struct Fused {
    FusedLds<NC> &L;
    cptr<SimConst> C;
    gptr<ST> src[9];
    gmptr<ST> dst[9];
    int comp, lane, nx, ny, xc, xm, xp, y0, rows;
    bool outl;
    double invM, bi, sqki, rb, RT, omega, fcoef;
    uint32_t bad;

    __device__ __forceinline__ int wrap_row(int r) const {
        r %= ny;
        return r < 0 ? r + ny : r;
    }

    __device__ __forceinline__ void load_row(ST (&g)[9], int r) const {
        const uint32_t off = (uint32_t)(wrap_row(r) * nx + xc);
#pragma unroll
        for (int a = 0; a < 9; ++a) g[a] = src[a][off];
    }

    // One lead row r.  gA = row r-2 (collided), gB = row r-1, gC = row r
    // (loaded), gD = row r+1 (prefetched here).  rh* = rho_i of rows
    // r-3 .. r, ps* = psi_i of rows r-3 .. r-1 (written here).
    __device__ __forceinline__ void body(int r, int rend, ST (&gA)[9], ST (&gC)[9], ST (&gD)[9],
                                         double rhm3, double rhm2, double rhm1, double &rh0,
                                         double psm3, double psm2, double &psm1) {
        const int slot = r & 1;
        if (r < rend) load_row(gD, r + 1);
        // ---- A: moments of row r
        {
            double v[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) v[a] = (double)gC[a];
            v[0] += rb;
            double rho = 0.0;
#pragma unroll
            for (int a = 0; a < 9; ++a) rho += v[a];
            rh0 = rho;
            L.rt[slot][comp][lane] = rho * invM;
            L.jx[comp][lane] = (v[1] - v[3]) + (v[5] - v[7]) + (v[8] - v[6]);
            L.jy[comp][lane] = (v[2] - v[4]) + (v[5] - v[7]) + (v[6] - v[8]);
        }
        // ---- B: Sraw_i of row r-1; G_i of row y
        const bool do_eos = r >= y0;
        const bool do_out = r >= y0 + 2;
        double Sraw = 0.0;
        if (do_eos) {
            cptr<double> arow = C->aij + comp * FUG_MAXC;
#pragma unroll
            for (int j = 0; j < NC; ++j) Sraw += arow[j] * L.rt[slot ^ 1][j][lane];
            L.xs[comp][lane] = rhm1 * invM * Sraw;
        }
        double Gx = 0.0, Gy = 0.0;
        if (do_out) grad3(rhm3, rhm2, rhm1, Gx, Gy);
        __syncthreads();
        // ---- M: one wave computes the per-site sums over components
        if (comp == ((r % NC) + NC) % NC) {
            double rtt = 0.0, eta = 0.0, sv = 0.0, rtot = 0.0, jxt = 0.0, jyt = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const double t = L.rt[slot][j][lane];
                rtt += t;
                eta += C->b[j] * t;
                sv += C->sqk[j] * t;
                rtot += C->M[j] * t;
                jxt += L.jx[j][lane];
                jyt += L.jy[j][lane];
            }
            const int ts = r & 3;
            L.tot[ts][0][lane] = sv;
            L.tot[ts][1][lane] = rtot;
            L.tot[ts][2][lane] = jxt;
            L.tot[ts][3][lane] = jyt;
            L.mx[slot][0][lane] = rtt;
            L.mx[slot][1][lane] = eta;
            if (do_eos) {
                // mixture terms of row r-1 (Eq. (9)-(12), combined-log form)
                const double rt1 = L.mx[slot ^ 1][0][lane];
                const double et1 = L.mx[slot ^ 1][1][lane];
                double xsum = 0.0;
#pragma unroll
                for (int j = 0; j < NC; ++j) xsum += L.xs[j][lane];
                const double inv_rt = 1.0 / rt1;
                const double am = xsum * inv_rt * inv_rt;
                const double ome = 1.0 - et1;
                if (!(ome > 0.0)) bad |= FUG_ST_COVOLUME;
                const double inv_ome = 1.0 / ome;
                const double inv_bm = rt1 / et1;
                const double den = 1.0 + 2.0 * et1 - et1 * et1;
                const double zm1 = et1 * inv_ome - am * rt1 / (RT * den);
                const double s2 = 1.4142135623730951;
                const double lam =
                    log((1.0 + (1.0 + s2) * et1) / (1.0 + (1.0 - s2) * et1));
                const double lam_c = lam * inv_bm * (0.5 / s2);
                L.eos[0][lane] = RT * inv_ome;                       // c1
                L.eos[1][lane] = RT * inv_bm * zm1 + lam_c * am * inv_bm;  // c2
                L.eos[2][lane] = 2.0 * lam_c * inv_rt;               // c3
            }
        }
        __syncthreads();
        // ---- C: psi_i of row r-1
        if (do_eos) {
            const double c1 = L.eos[0][lane], c2 = L.eos[1][lane], c3 = L.eos[2][lane];
            const double rti = rhm1 * invM;
            const double lnf = RT * log(rti * c1) + bi * c2 - c3 * Sraw;
            const double s_m2 = L.tot[(r - 2) & 3][0][lane];
            const double s_m1 = L.tot[(r - 1) & 3][0][lane];
            const double s_0 = L.tot[r & 3][0][lane];
            const double psi = lnf - sqki * lap3(s_m2, s_m1, s_0);
            psm1 = psi;
            if (!(rti > 0.0)) bad |= FUG_ST_NEGATIVE;
            if (!isfinite(psi)) bad |= FUG_ST_NONFINITE;
        }
        // ---- D: force of row y
        double Fx = 0.0, Fy = 0.0;
        if (do_out) {
            double gx, gy;
            grad3(psm3, psm2, psm1, gx, gy);
            const double rty = rhm2 * invM;
            Fx = -rty * gx;
            Fy = -rty * gy;
            L.fx[comp][lane] = Fx;
            L.fy[comp][lane] = Fy;
        }
        __syncthreads();
        // ---- E: velocity, collision and push of row y
        if (do_out) {
            double Fsx = 0.0, Fsy = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                Fsx += L.fx[j][lane];
                Fsy += L.fy[j][lane];
            }
            const int ys = (r - 2) & 3;
            const double inv_rho = 1.0 / L.tot[ys][1][lane];
            const double ux = (L.tot[ys][2][lane] + 0.5 * Fsx) * inv_rho;
            const double uy = (L.tot[ys][3][lane] + 0.5 * Fsy) * inv_rho;
            const double uu = ux * ux + uy * uy;
            const double Fu = Fx * ux + Fy * uy;
            const double Gu = Gx * ux + Gy * uy;
            const double rho = rhm2;
            const int y = r - 2;
            const uint32_t rowm = (uint32_t)(wrap_row(y - 1) * nx);
            const uint32_t row0 = (uint32_t)(wrap_row(y) * nx);
            const uint32_t rowp = (uint32_t)(wrap_row(y + 1) * nx);
            if (outl) {
#pragma unroll
                for (int a = 0; a < 9; ++a) {
                    double gv = (double)gA[a];
                    if (a == 0) gv += rb;
                    double o = collide_one<D2Q9>(a, gv, rho, ux, uy, 0.0, Fx, Fy, 0.0, Gx, Gy,
                                                 0.0, uu, Fu, Gu, omega, fcoef);
                    if (a == 0) o -= rb;
                    const int exa = D2Q9::ex(a), eya = D2Q9::ey(a);
                    const uint32_t xx = (uint32_t)(exa == 0 ? xc : (exa > 0 ? xp : xm));
                    const uint32_t rr = eya == 0 ? row0 : (eya > 0 ? rowp : rowm);
                    dst[a][rr + xx] = (ST)o;
                }
            }
        }
    }
};

template <int NC, typename ST>
__global__ __launch_bounds__(64 * NC) void k_fused_d2q9(const FusedItem *__restrict__ items_,
                                                        const FusedSim *__restrict__ sims_,
                                                        int flip) {
    __shared__ FusedLds<NC> lds;
    cptr<FusedItem> itp = (cptr<FusedItem>)items_ + blockIdx.x;
    const FusedItem it = {itp->sim, itp->x0, itp->y0, itp->rows};
    if (it.sim < 0) return;
    cptr<FusedSim> sm = (cptr<FusedSim>)sims_ + it.sim;
    const int par = (sm->parity ^ flip) & 1;
    cptr<SimConst> C = (cptr<SimConst>)sm->c;
    Fused<NC, ST> f{lds, C};
    f.comp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    f.lane = threadIdx.x & 63;
    f.nx = C->nx;
    f.ny = C->ny;
    const int64_t ns = C->nsites;
    const ST *bsrc = (const ST *)(par ? sm->buf[1] : sm->buf[0]);
    ST *bdst = (ST *)(par ? sm->buf[0] : sm->buf[1]);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        f.src[a] = (gptr<ST>)(bsrc + ((int64_t)f.comp * 9 + a) * ns);
        f.dst[a] = (gmptr<ST>)(bdst + ((int64_t)f.comp * 9 + a) * ns);
    }
    int xc = (it.x0 - 2 + f.lane) % f.nx;
    if (xc < 0) xc += f.nx;
    f.xc = xc;
    f.xm = xc == 0 ? f.nx - 1 : xc - 1;
    f.xp = xc == f.nx - 1 ? 0 : xc + 1;
    f.outl = f.lane >= 2 && f.lane < 62 && (it.x0 + f.lane - 2) < f.nx;
    f.y0 = it.y0;
    f.rows = it.rows;
    f.invM = C->invM[f.comp];
    f.bi = C->b[f.comp];
    f.sqki = C->sqk[f.comp];
    f.rb = C->rhobar[f.comp];
    f.RT = C->RT;
    f.omega = C->omega;
    f.fcoef = C->fcoef;
    f.bad = 0;

    ST g0[9], g1[9], g2[9], g3[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) g0[a] = g1[a] = g3[a] = (ST)0;
    const int rbeg = it.y0 - 2, rend = it.y0 + it.rows + 1;
    f.load_row(g2, rbeg);
    // rho rings (rows r-3..r) and psi rings (rows r-3..r-1), rotated by phase
    double h0 = 0.0, h1 = 0.0, h2 = 0.0, h3 = 0.0;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
    for (int r = rbeg; r <= rend; r += 4) {
        // phase 0: rows r-2,r-1,r,r+1 in g0,g1,g2,g3; rho r-3..r in h1,h2,h3,h0
        f.body(r, rend, g0, g2, g3, h1, h2, h3, h0, p1, p2, p3);
        if (r + 1 > rend) break;
        f.body(r + 1, rend, g1, g3, g0, h2, h3, h0, h1, p2, p3, p0);
        if (r + 2 > rend) break;
        f.body(r + 2, rend, g2, g0, g1, h3, h0, h1, h2, p3, p0, p1);
        if (r + 3 > rend) break;
        f.body(r + 3, rend, g3, g1, g2, h0, h1, h2, h3, p0, p1, p2);
    }
    if (f.bad) atomicOr(sm->status, f.bad);
}

template <int NC>
hipError_t launch_nc(bool fp32, const FusedItem *items, int nitems, const FusedSim *sims,
                     int flip, hipStream_t st) {
    if (fp32)
        hipLaunchKernelGGL((k_fused_d2q9<NC, float>), dim3(nitems), dim3(64 * NC), 0, st, items,
                           sims, flip);
    else
        hipLaunchKernelGGL((k_fused_d2q9<NC, double>), dim3(nitems), dim3(64 * NC), 0, st, items,
                           sims, flip);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fused_d2q9(int ncomp, bool fp32, const FusedItem *items, int nitems,
                             const FusedSim *sims, int flip, hipStream_t st) {
    switch (ncomp) {
        case 1: return launch_nc<1>(fp32, items, nitems, sims, flip, st);
        case 2: return launch_nc<2>(fp32, items, nitems, sims, flip, st);
        case 3: return launch_nc<3>(fp32, items, nitems, sims, flip, st);
        case 4: return launch_nc<4>(fp32, items, nitems, sims, flip, st);
        case 5: return launch_nc<5>(fp32, items, nitems, sims, flip, st);
        case 6: return launch_nc<6>(fp32, items, nitems, sims, flip, st);
        case 7: return launch_nc<7>(fp32, items, nitems, sims, flip, st);
        case 8: return launch_nc<8>(fp32, items, nitems, sims, flip, st);
        case 9: return launch_nc<9>(fp32, items, nitems, sims, flip, st);
        case 10: return launch_nc<10>(fp32, items, nitems, sims, flip, st);
        case 11: return launch_nc<11>(fp32, items, nitems, sims, flip, st);
        case 12: return launch_nc<12>(fp32, items, nitems, sims, flip, st);
        case 13: return launch_nc<13>(fp32, items, nitems, sims, flip, st);
        case 14: return launch_nc<14>(fp32, items, nitems, sims, flip, st);
        case 15: return launch_nc<15>(fp32, items, nitems, sims, flip, st);
        case 16: return launch_nc<16>(fp32, items, nitems, sims, flip, st);
        default: return hipErrorInvalidValue;
    }
}
