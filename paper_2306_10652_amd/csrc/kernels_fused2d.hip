// Fused one-pass D2Q9 step (moments -> PR fugacity -> interface potential ->
// force -> collide -> push-stream) for gfx950.
//
// Work item = a 64-column strip (60 output columns plus a 2-column halo on
// each side) of one simulation, marching up `rows` output rows.  The
// workgroup has one wavefront per component (lane = column): a lane keeps
// only its own component's 9 populations of the rows in flight, in
// registers.  Sums over components go through LDS.  Per lead row r (output
// row y = r - 2), with two workgroup barriers:
//
//   1  (all)  moments of row r -> LDS: rt_i, j_i;  G_i(y) = grad rho_i
//      (helpers A, B) row r-1 mixture coefficients of RT ln f_i   (Eq. (9)-(12))
//   -- barrier --
//   2  (all)  s(r) = sum_j sqrt(kappa_j) rt_j;  psi_i(r-1) = RT ln f_i -
//             sqrt(kappa_i) lap s  (Eq. (3)-(5));  F_i(y) = -rt_i grad psi_i
//             -> LDS;  Sraw_i(r) = sum_j (a alpha)_ij rt_j -> LDS
//      (helpers) row r totals: rt, b_m rt, 1/rho, j -> LDS rings
//   -- barrier --
//   3  (all)  u(y) = (j + F/2) / rho, collide row y (Eq. (1)), push-store
//
// Every population is read from HBM once per step; the 4 halo columns and
// the 4 warm-up rows of a work item are re-reads that neighbouring items
// issue at about the same time (the item order keeps them on one XCD).
#include "fused_common.h"

namespace {

using namespace fused;

template <int NC, typename ST>
struct Fused {
    FusedLds<NC> &L;
    cptr<SimConst> C;
    // Population layout (PopLayout): bases of this component's rest array
    // and of its direction-a arrays (at src[a - 1]) at row 0; row w is
    // w * rsr doubles / w * rsm ST elements further on.
    gptr<double> srcR;
    gmptr<double> dstR;
    gptr<ST> src[8];
    gmptr<ST> dst[8];
    uint32_t rsr, rsm;
    int comp, lane, nx, ny, xc, xm, xp, y0, rows;
    int wm3, wm2, wm1, w0;   // wrapped row indices of rows r-3 .. r (uniform)
    bool outl;
    double invM, bi, sqki, RT, invRT, omega, fcoef;
    uint32_t bad;

    // An empty asm statement that reads every register of a row: the
    // compiler must complete the row's loads before it.
    __device__ __forceinline__ static void wait_row(const PopRow<ST> &g) {
        asm volatile("" ::"v"(g.r), "v"(g.m[0]), "v"(g.m[1]), "v"(g.m[2]), "v"(g.m[3]), "v"(g.m[4]),
                     "v"(g.m[5]), "v"(g.m[6]), "v"(g.m[7]));
    }

    __device__ __forceinline__ void load_row(PopRow<ST> &g, int wrow) const {
        g.r = srcR[(uint32_t)wrow * rsr + (uint32_t)xc];
        const uint32_t off = (uint32_t)wrow * rsm + (uint32_t)xc;
#pragma unroll
        for (int a = 0; a < 8; ++a) g.m[a] = src[a][off];
    }

    // One lead row r.  gA = row r-2 (collided), gC = row r (loaded), gD =
    // row r+1 (prefetched here).  rh* = rho_i of rows r-3 .. r (rh0 written
    // here), ps* = psi_i of rows r-3 .. r-1 (psm1 written here), sv* = s of
    // rows r-2 .. r (sv0 written here), sn / so = Sraw_i of rows r / r-1.
    __device__ __forceinline__ void body(int r, int rend, PopRow<ST> &gA, PopRow<ST> &gC,
                                         PopRow<ST> &gD,
                                         double rhm3, double rhm2, double rhm1, double &rh0,
                                         double psm3, double psm2, double &psm1, double svm2,
                                         double svm1, double &sv0, double &sn, double so) {
        // advance the wrapped row indices (uniform, scalar)
        wm3 = wm2;
        wm2 = wm1;
        wm1 = w0;
        w0 = (r == y0 - 2) ? w0 : (w0 + 1 == ny ? 0 : w0 + 1);
        if (r < rend) load_row(gD, w0 + 1 == ny ? 0 : w0 + 1);
        const bool do_s = r >= y0 - 1;
        const bool do_eos = r >= y0;
        const bool do_out = r >= y0 + 2;
        // ---- phase 1: moments of row r; G_i of row y; mixture terms of row r-1
        {
            double v[9];
            v[0] = gC.r;
#pragma unroll
            for (int a = 1; a < 9; ++a) v[a] = (double)gC.m[a - 1];
            double rho = 0.0;
#pragma unroll
            for (int a = 0; a < 9; ++a) rho += v[a];
            rh0 = rho;
            L.rt[comp][lane] = rho * invM;
            L.jx[comp][lane] = (v[1] - v[3]) + (v[5] - v[7]) + (v[8] - v[6]);
            L.jy[comp][lane] = (v[2] - v[4]) + (v[5] - v[7]) + (v[6] - v[8]);
        }
        double Gx = 0.0, Gy = 0.0;
        if (do_out) grad3(rhm3, rhm2, rhm1, Gx, Gy);
        // Eq. (9)-(12) in combined-log form for row r-1 (any of the cubics,
        // p = RT/(v - b) - a/((v + d1 b)(v + d2 b))),
        //   RT ln f_i = RT ln(rt_i c1) + b_i (c2a + lambda c2b) - lambda c3b Sraw_i,
        // split over two helper waves: A (reciprocals, Z - 1) and B (lambda =
        // ln[(1 + d1 eta)/(1 + d2 eta)] / (d1 - d2), or eta for vdW).
        if (do_eos && comp == helper_wave<NC>(0)) {
            const int ms = (r - 1) & 1;
            const double rt1 = L.mx[ms][0][lane];
            const double et1 = L.mx[ms][1][lane];
            double xsum = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) xsum += L.xs[j][lane];
            const double inv_rt = frcp(rt1);
            const double am = xsum * inv_rt * inv_rt;
            const double ome = 1.0 - et1;
            if (!(ome > 0.0)) bad |= FUG_ST_COVOLUME;
            const double inv_ome = frcp(ome);
            const double inv_bm = rt1 * frcp(et1);
            const double den = 1.0 + C->eu * et1 + C->ew * et1 * et1;
            const double zm1 = et1 * inv_ome - am * rt1 * invRT * frcp(den);
            L.eos[0][lane] = RT * inv_ome;
            L.eos[1][lane] = RT * zm1 * inv_bm;
            L.eos[2][lane] = am * inv_bm * inv_bm;
            L.eos[3][lane] = 2.0 * inv_bm * inv_rt;
        }
        if (do_eos && comp == helper_wave<NC>(1)) {
            const double et1 = L.mx[(r - 1) & 1][1][lane];
            L.eos[4][lane] = C->eos == 2
                                 ? et1
                                 : log((1.0 + C->d1 * et1) * frcp(1.0 + C->d2 * et1)) * C->dk;
        }
        __syncthreads();
        // ---- phase 2: s(r); psi_i(r-1); F_i(y); Sraw_i(r); helper sums of row r
        {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) acc += C->sqk[j] * L.rt[j][lane];
            sv0 = acc;
        }
        if (do_eos) {
            const double c1 = L.eos[0][lane], c2a = L.eos[1][lane], c2b = L.eos[2][lane];
            const double c3b = L.eos[3][lane], lam = L.eos[4][lane];
            const double rti = rhm1 * invM;
            const double lnf = RT * log(rti * c1) + bi * fma(lam, c2b, c2a) - lam * c3b * so;
            const double psi = lnf - sqki * lap3(svm2, svm1, sv0);
            psm1 = psi;
            if (!(rti > 0.0)) bad |= FUG_ST_NEGATIVE;
            if (!isfinite(psi)) bad |= FUG_ST_NONFINITE;
        }
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
        if (do_s) {
            cptr<double> arow = C->aij + comp * FUG_MAXC;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) acc += arow[j] * L.rt[j][lane];
            sn = acc;
            L.xs[comp][lane] = rh0 * invM * acc;
        }
        if (do_s && comp == helper_wave<NC>(2)) {
            double rtt = 0.0, eta = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const double t = L.rt[j][lane];
                rtt += t;
                eta += C->b[j] * t;
            }
            L.mx[r & 1][0][lane] = rtt;
            L.mx[r & 1][1][lane] = eta;
        }
        if (comp == helper_wave<NC>(3)) {
            double rtot = 0.0, jxt = 0.0, jyt = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                rtot += C->M[j] * L.rt[j][lane];
                jxt += L.jx[j][lane];
                jyt += L.jy[j][lane];
            }
            L.tot[r & 3][0][lane] = frcp(rtot);
            L.tot[r & 3][1][lane] = jxt;
            L.tot[r & 3][2][lane] = jyt;
        }
        __syncthreads();
        // Make the prefetched row resident here, before this row's stores:
        // a wait for loads while stores are in flight waits for those
        // stores too, and the ring rotation at the end of the row would
        // otherwise wait for the stores just issued.
        wait_row(gD);
        // ---- phase 3: velocity, collision and push of row y
        if (do_out) {
            double Fsx = 0.0, Fsy = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                Fsx += L.fx[j][lane];
                Fsy += L.fy[j][lane];
            }
            const int ys = (r - 2) & 3;
            const double inv_rho = L.tot[ys][0][lane];
            const double ux = (L.tot[ys][1][lane] + 0.5 * Fsx) * inv_rho;
            const double uy = (L.tot[ys][2][lane] + 0.5 * Fsy) * inv_rho;
            const double orho = omega * rhm2;
            const double A = 3.0 * orho, B = 4.5 * orho;
            const double C9 = 9.0 * fcoef, C3 = 3.0 * fcoef;
            const double omc = 1.0 - omega;
            const double base = -1.5 * orho * (ux * ux + uy * uy) - C3 * (Fx * ux + Fy * uy);
            const double Gu = Gx * ux + Gy * uy;
            const double K1 = fma(-0.5 * fcoef, Gu, base);
            const double K2 = fma(fcoef, Gu, base);
            const uint32_t rowm = (uint32_t)wm3 * rsm;
            const uint32_t row0 = (uint32_t)wm2 * rsm;
            const uint32_t rowp = (uint32_t)wm1 * rsm;
            if (outl) {
                if constexpr (sizeof(ST) == 4) {
                    // FP32 storage: the moving populations in FP32 arithmetic,
                    // the rest population = rho - their stored sum (mass stays
                    // exact to FP64 rounding)
                    float g[8], t[8];
#pragma unroll
                    for (int m = 0; m < 8; ++m) g[m] = (float)gA.m[m];
                    const double msum = collide_moving_f32(A, B, C9, C3, K1, K2, omc, ux, uy, Fx,
                                                           Fy, Gx, Gy, g, t);
                    dst[0][row0 + xp] = t[0];
                    dst[2][row0 + xm] = t[2];
                    dst[1][rowp + xc] = t[1];
                    dst[3][rowm + xc] = t[3];
                    dst[4][rowp + xp] = t[4];
                    dst[6][rowm + xm] = t[6];
                    dst[5][rowp + xm] = t[5];
                    dst[7][rowm + xp] = t[7];
                    dstR[(uint32_t)wm2 * rsr + (uint32_t)xc] = rhm2 - msum;
                } else {
                    // the four opposite pairs, stored as they are formed; then
                    // the rest population
                    auto put = [&](gmptr<ST> p, uint32_t at, double v) { p[at] = (ST)v; };
                    double tp, tm;
                    collide_pair(A, B, C9, C3, K1, ux, Fx, Gx, tp, tm);
                    put(dst[0], row0 + xp, fma(omc, (double)gA.m[0], (1.0 / 9.0) * tp));
                    put(dst[2], row0 + xm, fma(omc, (double)gA.m[2], (1.0 / 9.0) * tm));
                    collide_pair(A, B, C9, C3, K1, uy, Fy, Gy, tp, tm);
                    put(dst[1], rowp + xc, fma(omc, (double)gA.m[1], (1.0 / 9.0) * tp));
                    put(dst[3], rowm + xc, fma(omc, (double)gA.m[3], (1.0 / 9.0) * tm));
                    collide_pair(A, B, C9, C3, K2, ux + uy, Fx + Fy, Gx + Gy, tp, tm);
                    put(dst[4], rowp + xp, fma(omc, (double)gA.m[4], (1.0 / 36.0) * tp));
                    put(dst[6], rowm + xm, fma(omc, (double)gA.m[6], (1.0 / 36.0) * tm));
                    collide_pair(A, B, C9, C3, K2, uy - ux, Fy - Fx, Gy - Gx, tp, tm);
                    put(dst[5], rowp + xm, fma(omc, (double)gA.m[5], (1.0 / 36.0) * tp));
                    put(dst[7], rowm + xp, fma(omc, (double)gA.m[7], (1.0 / 36.0) * tm));
                    dstR[(uint32_t)wm2 * rsr + (uint32_t)xc] =
                        fma(omc, gA.r, fma(4.0 / 9.0, fma(-2.0 * fcoef, Gu, base), orho));
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
    const char *bsrc = (const char *)(par ? sm->buf[1] : sm->buf[0]);
    char *bdst = (char *)(par ? sm->buf[0] : sm->buf[1]);
    const PopLayout<ST> P(NC, 9, f.nx, f.ny);
    f.rsr = (uint32_t)P.rest_row_stride();
    f.rsm = (uint32_t)P.move_row_stride();
    f.srcR = (gptr<double>)(const double *)(bsrc + P.rest(0, f.comp, 0));
    f.dstR = (gmptr<double>)(double *)(bdst + P.rest(0, f.comp, 0));
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        f.src[a - 1] = (gptr<ST>)(const ST *)(bsrc + P.move(0, f.comp, a, 0));
        f.dst[a - 1] = (gmptr<ST>)(ST *)(bdst + P.move(0, f.comp, a, 0));
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
    f.RT = C->RT;
    f.invRT = 1.0 / C->RT;
    f.omega = C->omega;
    f.fcoef = C->fcoef;
    f.bad = 0;
    const int rbeg = it.y0 - 2, rend = it.y0 + it.rows + 1;
    {
        int w = rbeg % f.ny;
        if (w < 0) w += f.ny;
        f.w0 = w;           // body() keeps w0 for its first row, then advances
        f.wm1 = f.wm2 = f.wm3 = 0;
    }

    PopRow<ST> g0, g1, g2, g3;
    g0.r = g1.r = g3.r = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) g0.m[a] = g1.m[a] = g3.m[a] = (ST)0;
    f.load_row(g2, f.w0);
    // register rings: g0..g3 = populations of rows r-2 .. r+1; h = rho_i of
    // rows r-3 .. r; p = psi_i of rows r-3 .. r-1; s = s of rows r-2 .. r;
    // q = Sraw_i of rows r-1, r.  (A rolled loop with ring moves keeps the
    // register pressure low enough for three waves per SIMD.)
    double h0 = 0.0, h1 = 0.0, h2 = 0.0, h3 = 0.0;
    double p1 = 0.0, p2 = 0.0, p3 = 0.0;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    double qn = 0.0, qo = 0.0;
    for (int r = rbeg; r <= rend; ++r) {
        f.body(r, rend, g0, g2, g3, h1, h2, h3, h0, p1, p2, p3, s1, s2, s0, qn, qo);
        {
            const double t = g0.r;
            g0.r = g1.r;
            g1.r = g2.r;
            g2.r = g3.r;
            g3.r = t;
        }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const ST t = g0.m[a];
            g0.m[a] = g1.m[a];
            g1.m[a] = g2.m[a];
            g2.m[a] = g3.m[a];
            g3.m[a] = t;
        }
        h1 = h2;
        h2 = h3;
        h3 = h0;
        p1 = p2;
        p2 = p3;
        s1 = s2;
        s2 = s0;
        qo = qn;
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

template <int NC>
int occ_nc(bool fp32) {
    int nb = 0;
    hipError_t e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, (const void *)k_fused_d2q9<NC, float>, 64 * NC, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, (const void *)k_fused_d2q9<NC, double>, 64 * NC, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

}  // namespace

int fused_blocks_per_cu(int ncomp, bool fp32) {
    switch (ncomp) {
        case 1: return occ_nc<1>(fp32);
        case 2: return occ_nc<2>(fp32);
        case 3: return occ_nc<3>(fp32);
        case 4: return occ_nc<4>(fp32);
        case 5: return occ_nc<5>(fp32);
        case 6: return occ_nc<6>(fp32);
        case 7: return occ_nc<7>(fp32);
        case 8: return occ_nc<8>(fp32);
        case 9: return occ_nc<9>(fp32);
        case 10: return occ_nc<10>(fp32);
        case 11: return occ_nc<11>(fp32);
        case 12: return occ_nc<12>(fp32);
        case 13: return occ_nc<13>(fp32);
        case 14: return occ_nc<14>(fp32);
        case 15: return occ_nc<15>(fp32);
        case 16: return occ_nc<16>(fp32);
        default: return 1;
    }
}

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
