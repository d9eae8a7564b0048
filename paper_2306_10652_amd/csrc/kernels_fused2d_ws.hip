// Fused one-pass D2Q9 step, store-wave variant (gfx950).
//
// Same work items, phases and arithmetic as the register-ring kernel
// (kernels_fused2d.hip): one wavefront per component, lane = column of a
// 64-column strip (60 output columns), marching up the rows of the item
// with two workgroup barriers per row.  What differs is the memory pipeline.
//
//  * Two extra store wavefronts per workgroup write the post-collision
//    populations to HBM.  The component waves put them in an LDS staging
//    block instead, so a component wave only ever has loads in flight.
//    Vector-memory loads and stores share one completion counter, and a
//    wave that has both in flight can only wait for all of them; with
//    loads alone the wait for a row stops at that row.
//  * Rows are requested three rows ahead.  A component wave keeps rows r
//    (being used), r+1 and r+2 (in flight) and row r-2 (input of this
//    row's collision) in registers; row r-1, which is only waiting, is
//    parked in a per-wave LDS stash.  The row loop is unrolled by three so
//    the registers of a row in flight are never copied (a copy would have
//    to wait for the load).
//
//  * The two store wavefronts also compute every per-site term that needs
//    all components (the helper work): the cubic-EOS mixture coefficients
//    of row r-1 (reciprocals and Z - 1 on store wave 0, the logarithmic
//    term on store wave 1) while the component waves collide and take
//    moments, and the sums over components of row r (b_m rt and rt; 1/rho
//    and j) after their stores.  The component waves then do the same work
//    between barriers, and the EOS chain is off their critical path.
//
// Per lead row r (output row y = r - 2):
//      (store waves) mixture coefficients of row r - 1
//   1  (component waves) moments of row r; G_i(y)
//   -- barrier --
//      (store waves) write the staged output row of lead row r - 1; sums
//      over components of row r
//   2  (component waves) s, psi_i(r-1), F_i(y), Sraw_i(r)
//   -- barrier --
//   3  (component waves) u(y), collision of row y -> LDS staging; row
//      r-1 stash -> registers, row r -> stash, request row r+3
// One extra pass of the loop flushes the last staged row.
#include "fused_common.h"

namespace {

using namespace fused;

constexpr int STORE_WAVES = 2;

template <int NC, typename ST>
struct WsLds {
    FusedLds<NC> f;
    double stR[NC][64];      // stash: rest population of row r-1
    ST stM[NC][8][64];       // stash: moving populations of row r-1
    double ogR[NC][64];      // staging: post-collision rest population of row y
    ST ogM[NC][8][64];       // staging: post-collision moving populations of row y
};

template <int NC, typename ST>
constexpr size_t ws_lds_bytes() {
    return sizeof(WsLds<NC, ST>);
}

template <int NC, typename ST>
struct Comp {
    WsLds<NC, ST> &W;
    FusedLds<NC> &L;
    cptr<SimConst> C;
    gptr<double> srcR;
    gptr<ST> src[8];
    uint32_t rsr, rsm;
    int comp, lane, xc, y0;
    double invM, bi, sqki, RT, omega, fcoef;
    uint32_t bad;

    // One row's nine loads, kept together and in program order (neither
    // the compiler's passes nor its scheduler may move loads across the
    // fences), so every wait on a row counts the rows requested after it.
    __device__ __forceinline__ void load_row(PopRow<ST> &g, int wrow) const {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
        g.r = srcR[(uint32_t)wrow * rsr + (uint32_t)xc];
        const uint32_t off = (uint32_t)wrow * rsm + (uint32_t)xc;
#pragma unroll
        for (int a = 0; a < 8; ++a) g.m[a] = src[a][off];
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
    }

    // ---- phase 1: moments of row r (gC); G_i of row y
    __device__ __forceinline__ void phase1(int r, const PopRow<ST> &gC, double rhm3, double rhm2,
                                           double rhm1, double &rh0, double &Gx, double &Gy) {
        const bool do_out = r >= y0 + 2;
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
        Gx = 0.0;
        Gy = 0.0;
        if (do_out) grad3(rhm3, rhm2, rhm1, Gx, Gy);
    }

    // ---- phase 2: s(r); psi_i(r-1); F_i(y); Sraw_i(r)
    __device__ __forceinline__ void phase2(int r, double rhm2, double rhm1, double rh0,
                                           double psm3, double psm2, double &psm1, double svm2,
                                           double svm1, double &sv0, double &sn, double so,
                                           double &Fx, double &Fy) {
        const bool do_s = r >= y0 - 1;
        const bool do_eos = r >= y0;
        const bool do_out = r >= y0 + 2;
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
        Fx = 0.0;
        Fy = 0.0;
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
    }

    // ---- phase 3: velocity and collision of row y = r - 2 into the staging
    // block (FP32 storage: moving populations in FP32 arithmetic, the rest
    // population = rho - their stored sum, so mass stays exact to FP64
    // rounding).
    __device__ __forceinline__ void phase3(int r, const PopRow<ST> &gA, double rhm2, double Fx,
                                           double Fy, double Gx, double Gy) {
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
        if constexpr (sizeof(ST) == 4) {
            float g[8], t[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) g[m] = (float)gA.m[m];
            const double msum = collide_moving_f32(A, B, C9, C3, K1, K2, omc, ux, uy, Fx, Fy, Gx,
                                                   Gy, g, t);
#pragma unroll
            for (int m = 0; m < 8; ++m) W.ogM[comp][m][lane] = (ST)t[m];
            W.ogR[comp][lane] = rhm2 - msum;
            return;
        }
        auto put = [&](int a, double v) { W.ogM[comp][a][lane] = (ST)v; };
        double tp, tm;
        collide_pair(A, B, C9, C3, K1, ux, Fx, Gx, tp, tm);
        put(0, fma(omc, (double)gA.m[0], (1.0 / 9.0) * tp));
        put(2, fma(omc, (double)gA.m[2], (1.0 / 9.0) * tm));
        collide_pair(A, B, C9, C3, K1, uy, Fy, Gy, tp, tm);
        put(1, fma(omc, (double)gA.m[1], (1.0 / 9.0) * tp));
        put(3, fma(omc, (double)gA.m[3], (1.0 / 9.0) * tm));
        collide_pair(A, B, C9, C3, K2, ux + uy, Fx + Fy, Gx + Gy, tp, tm);
        put(4, fma(omc, (double)gA.m[4], (1.0 / 36.0) * tp));
        put(6, fma(omc, (double)gA.m[6], (1.0 / 36.0) * tm));
        collide_pair(A, B, C9, C3, K2, uy - ux, Fy - Fx, Gy - Gx, tp, tm);
        put(5, fma(omc, (double)gA.m[5], (1.0 / 36.0) * tp));
        put(7, fma(omc, (double)gA.m[7], (1.0 / 36.0) * tm));
        W.ogR[comp][lane] = fma(omc, gA.r, fma(4.0 / 9.0, fma(-2.0 * fcoef, Gu, base), orho));
    }

    // Row r-1 from the stash into gA (it is row r-2 of the next lead row),
    // then row r (gC) into the stash.
    __device__ __forceinline__ void park(PopRow<ST> &gA, const PopRow<ST> &gC) {
        gA.r = W.stR[comp][lane];
#pragma unroll
        for (int a = 0; a < 8; ++a) gA.m[a] = W.stM[comp][a][lane];
        W.stR[comp][lane] = gC.r;
#pragma unroll
        for (int a = 0; a < 8; ++a) W.stM[comp][a][lane] = gC.m[a];
    }
};

// The store waves: wave sw writes the staged rows of components
// [sw CPW, (sw + 1) CPW), all nine directions; lane = column as in the
// component waves, the destination shifted by the direction's lattice
// vector (push streaming).  All values are read from LDS before the first
// store is issued: a store reads its data registers after issue, so
// reusing them for the next value would wait for the store to finish.
template <int NC, typename ST>
struct Store {
    static constexpr int CPW = (NC + STORE_WAVES - 1) / STORE_WAVES;
    WsLds<NC, ST> &W;
    FusedLds<NC> &L;
    cptr<SimConst> C;
    char *bdst;
    PopLayout<ST> P;
    uint32_t rsr, rsm;
    int sw, nx, ny, y0;
    int xsh[3];     // destination column for ex = -1, 0, +1
    bool outl;
    double RT, invRT;
    uint32_t bad;

    __device__ __forceinline__ void row(int yw) const {
        if (!outl) return;
        const int ym = yw == 0 ? ny - 1 : yw - 1;
        const int yp = yw + 1 == ny ? 0 : yw + 1;
        const int lane = threadIdx.x & 63;
        double vr[CPW];
        ST vm[CPW][8];
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int i = sw * CPW + j;
            if (i < NC) {
                vr[j] = W.ogR[i][lane];
#pragma unroll
                for (int m = 0; m < 8; ++m) vm[j][m] = W.ogM[i][m][lane];
            }
        }
#pragma unroll
        for (int j = 0; j < CPW; ++j) {
            const int i = sw * CPW + j;
            if (i < NC) {
                double *d = (double *)(bdst + P.rest(0, i, 0));
                d[(uint32_t)yw * rsr + (uint32_t)xsh[1]] = vr[j];
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int a = m + 1;
                    const int ex = D2Q9::ex(a), ey = D2Q9::ey(a);
                    const int yr = ey > 0 ? yp : (ey < 0 ? ym : yw);
                    ST *dm = (ST *)(bdst + P.move(0, i, a, 0));
                    dm[(uint32_t)yr * rsm + (uint32_t)xsh[ex + 1]] = vm[j][m];
                }
            }
        }
    }

    // Eq. (9)-(12), combined-log form, mixture coefficients of row r-1 (the
    // register-ring kernel computes the same terms on its helper
    // wavefronts): store wave 0 the reciprocals and Z - 1, store wave 1
    // the logarithmic term.  Status bits only for lead rows <= last (the
    // rows past it repeat the item's last loaded row).
    __device__ __forceinline__ void mixture(int r, int last) {
        if (r < y0) return;
        const int lane = threadIdx.x & 63;
        const double et1 = L.mx[(r - 1) & 1][1][lane];
        if (sw == 0) {
            const double rt1 = L.mx[(r - 1) & 1][0][lane];
            double xsum = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) xsum += L.xs[j][lane];
            const double inv_rt = frcp(rt1);
            const double am = xsum * inv_rt * inv_rt;
            const double ome = 1.0 - et1;
            if (!(ome > 0.0) && r <= last) bad |= FUG_ST_COVOLUME;
            const double inv_ome = frcp(ome);
            const double inv_bm = rt1 * frcp(et1);
            const double den = 1.0 + C->eu * et1 + C->ew * et1 * et1;
            const double zm1 = et1 * inv_ome - am * rt1 * invRT * frcp(den);
            L.eos[0][lane] = RT * inv_ome;
            L.eos[1][lane] = RT * zm1 * inv_bm;
            L.eos[2][lane] = am * inv_bm * inv_bm;
            L.eos[3][lane] = 2.0 * inv_bm * inv_rt;
        } else {
            L.eos[4][lane] = C->eos == 2
                                 ? et1
                                 : log((1.0 + C->d1 * et1) * frcp(1.0 + C->d2 * et1)) * C->dk;
        }
    }

    // Sums over components of row r: rt and b_m rt (store wave 0, for the
    // mixture coefficients of the next lead row), 1/rho and j (store wave 1,
    // for the velocity two rows later).
    __device__ __forceinline__ void sums(int r) {
        const int lane = threadIdx.x & 63;
        if (sw == 0) {
            if (r < y0 - 1) return;
            double rtt = 0.0, eta = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const double t = L.rt[j][lane];
                rtt += t;
                eta += C->b[j] * t;
            }
            L.mx[r & 1][0][lane] = rtt;
            L.mx[r & 1][1][lane] = eta;
        } else {
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
    }
};

template <int NC, typename ST>
__global__ __launch_bounds__(64 * (NC + STORE_WAVES)) void k_fused_d2q9_ws(
    const FusedItem *__restrict__ items_, const FusedSim *__restrict__ sims_, int flip) {
    __shared__ WsLds<NC, ST> lds;
    cptr<FusedItem> itp = (cptr<FusedItem>)items_ + blockIdx.x;
    const FusedItem it = {itp->sim, itp->x0, itp->y0, itp->rows};
    if (it.sim < 0) return;
    cptr<FusedSim> sm = (cptr<FusedSim>)sims_ + it.sim;
    const int par = (sm->parity ^ flip) & 1;
    cptr<SimConst> C = (cptr<SimConst>)sm->c;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nx = C->nx, ny = C->ny;
    const char *bsrc = (const char *)(par ? sm->buf[1] : sm->buf[0]);
    char *bdst = (char *)(par ? sm->buf[0] : sm->buf[1]);
    const PopLayout<ST> P(NC, 9, nx, ny);
    int xc = (it.x0 - 2 + lane) % nx;
    if (xc < 0) xc += nx;
    const int rbeg = it.y0 - 2, rend = it.y0 + it.rows + 1;
    auto wrap = [&](int v) {
        v %= ny;
        return v < 0 ? v + ny : v;
    };
    // Every wave runs the same loop (same barrier count); a pass of the
    // unrolled body handles lead rows r, r+1, r+2, up to rend + 1 (the flush).
    if (wave >= NC) {
        Store<NC, ST> s{lds, lds.f, C, bdst, P, (uint32_t)P.rest_row_stride(),
                        (uint32_t)P.move_row_stride(), wave - NC, nx, ny, it.y0, {0, 0, 0},
                        false, C->RT, 1.0 / C->RT, 0u};
        s.xsh[0] = xc == 0 ? nx - 1 : xc - 1;
        s.xsh[1] = xc;
        s.xsh[2] = xc == nx - 1 ? 0 : xc + 1;
        s.outl = lane >= 2 && lane < 62 && (it.x0 + lane - 2) < nx;
        // output row of lead row r - 1 is r - 3
        int yw = wrap(rbeg - 3);
        for (int r0 = rbeg; r0 <= rend + 1; r0 += 3) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int r = r0 + k;
                s.mixture(r, rend);
                __syncthreads();
                if (r - 1 >= it.y0 + 2 && r - 1 <= rend) s.row(yw);
                s.sums(r);
                yw = yw + 1 == ny ? 0 : yw + 1;
                __syncthreads();
            }
        }
        if (s.bad) atomicOr(sm->status, s.bad);
        return;
    }

    Comp<NC, ST> f{lds, lds.f, C};
    f.comp = wave;
    f.lane = lane;
    f.xc = xc;
    f.y0 = it.y0;
    f.rsr = (uint32_t)P.rest_row_stride();
    f.rsm = (uint32_t)P.move_row_stride();
    f.srcR = (gptr<double>)(const double *)(bsrc + P.rest(0, f.comp, 0));
#pragma unroll
    for (int a = 1; a < 9; ++a)
        f.src[a - 1] = (gptr<ST>)(const ST *)(bsrc + P.move(0, f.comp, a, 0));
    f.invM = C->invM[f.comp];
    f.bi = C->b[f.comp];
    f.sqki = C->sqk[f.comp];
    f.RT = C->RT;
    f.omega = C->omega;
    f.fcoef = C->fcoef;
    f.bad = 0;

    // rows in registers: gA = row r-2; X, Y, Z = rows r, r+1, r+2 in the
    // roles the unrolled body rotates.  Loads past rend repeat row rend.
    PopRow<ST> gA, X, Y, Z;
    gA.r = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) gA.m[a] = (ST)0;
    int lw = wrap(rbeg);     // wrapped index of the last row requested
    int ln = rbeg;           // its absolute index
    f.load_row(X, lw);
    ln++;
    lw = lw + 1 == ny ? 0 : lw + 1;
    f.load_row(Y, lw);
    ln++;
    lw = lw + 1 == ny ? 0 : lw + 1;
    f.load_row(Z, lw);
    double h0 = 0.0, h1 = 0.0, h2 = 0.0, h3 = 0.0;
    double p1 = 0.0, p2 = 0.0, p3 = 0.0;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    double qn = 0.0, qo = 0.0;

    // Phases 1 and 2, the ring moves and the next request run on every
    // pass, past rend too (on a repeat of row rend, with the status bits
    // masked): every path then has the same loads in flight, and each wait
    // stops at the row it needs.  Only the collision (phase 3) is limited
    // to the item's output rows.
    auto lead = [&](int r, PopRow<ST> &cur) {
        double Gx = 0.0, Gy = 0.0, Fx = 0.0, Fy = 0.0;
        const uint32_t bad0 = f.bad;
        f.phase1(r, cur, h1, h2, h3, h0, Gx, Gy);
        __syncthreads();
        f.phase2(r, h2, h3, h0, p1, p2, p3, s1, s2, s0, qn, qo, Fx, Fy);
        __syncthreads();
        if (r > rend) f.bad = bad0;
        if (r <= rend && r >= it.y0 + 2) f.phase3(r, gA, h2, Fx, Fy, Gx, Gy);
        f.park(gA, cur);
        if (ln < rend) {
            ln++;
            lw = lw + 1 == ny ? 0 : lw + 1;
        }
        f.load_row(cur, lw);
        h1 = h2;
        h2 = h3;
        h3 = h0;
        p1 = p2;
        p2 = p3;
        s1 = s2;
        s2 = s0;
        qo = qn;
    };
    for (int r0 = rbeg; r0 <= rend + 1; r0 += 3) {
        lead(r0, X);
        lead(r0 + 1, Y);
        lead(r0 + 2, Z);
    }
    if (f.bad) atomicOr(sm->status, f.bad);
}

template <int NC>
hipError_t launch_ws_nc(bool fp32, const FusedItem *items, int nitems, const FusedSim *sims,
                        int flip, hipStream_t st) {
    if (fp32)
        hipLaunchKernelGGL((k_fused_d2q9_ws<NC, float>), dim3(nitems),
                           dim3(64 * (NC + STORE_WAVES)), 0, st, items, sims, flip);
    else
        hipLaunchKernelGGL((k_fused_d2q9_ws<NC, double>), dim3(nitems),
                           dim3(64 * (NC + STORE_WAVES)), 0, st, items, sims, flip);
    return hipGetLastError();
}

template <int NC>
int occ_ws_nc(bool fp32) {
    int nb = 0;
    hipError_t e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, (const void *)k_fused_d2q9_ws<NC, float>,
                              64 * (NC + STORE_WAVES), 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                              &nb, (const void *)k_fused_d2q9_ws<NC, double>,
                              64 * (NC + STORE_WAVES), 0);
    return e == hipSuccess && nb > 0 ? nb : 0;
}

// LDS of the variant (must fit the 160 KiB of a gfx950 workgroup).
constexpr size_t WS_LDS_LIMIT = 160 * 1024;
template <int NC>
constexpr bool ws_fits_nc(bool fp32) {
    return (fp32 ? ws_lds_bytes<NC, float>() : ws_lds_bytes<NC, double>()) <= WS_LDS_LIMIT;
}

}  // namespace

// Component counts the store-wave variant is built for: up to 10
// components (12 waves; the LDS stash and staging of FP64 rows fit).
int fused_ws_max_comp() { return 10; }

bool fused_ws_fits(int ncomp, bool fp32) {
    switch (ncomp) {
        case 1: return ws_fits_nc<1>(fp32);
        case 2: return ws_fits_nc<2>(fp32);
        case 3: return ws_fits_nc<3>(fp32);
        case 4: return ws_fits_nc<4>(fp32);
        case 5: return ws_fits_nc<5>(fp32);
        case 6: return ws_fits_nc<6>(fp32);
        case 7: return ws_fits_nc<7>(fp32);
        case 8: return ws_fits_nc<8>(fp32);
        case 9: return ws_fits_nc<9>(fp32);
        case 10: return ws_fits_nc<10>(fp32);
        default: return false;
    }
}

int fused_ws_blocks_per_cu(int ncomp, bool fp32) {
    switch (ncomp) {
        case 1: return occ_ws_nc<1>(fp32);
        case 2: return occ_ws_nc<2>(fp32);
        case 3: return occ_ws_nc<3>(fp32);
        case 4: return occ_ws_nc<4>(fp32);
        case 5: return occ_ws_nc<5>(fp32);
        case 6: return occ_ws_nc<6>(fp32);
        case 7: return occ_ws_nc<7>(fp32);
        case 8: return occ_ws_nc<8>(fp32);
        case 9: return occ_ws_nc<9>(fp32);
        case 10: return occ_ws_nc<10>(fp32);
        default: return 0;
    }
}

hipError_t launch_fused_d2q9_ws(int ncomp, bool fp32, const FusedItem *items, int nitems,
                                const FusedSim *sims, int flip, hipStream_t st) {
    switch (ncomp) {
        case 1: return launch_ws_nc<1>(fp32, items, nitems, sims, flip, st);
        case 2: return launch_ws_nc<2>(fp32, items, nitems, sims, flip, st);
        case 3: return launch_ws_nc<3>(fp32, items, nitems, sims, flip, st);
        case 4: return launch_ws_nc<4>(fp32, items, nitems, sims, flip, st);
        case 5: return launch_ws_nc<5>(fp32, items, nitems, sims, flip, st);
        case 6: return launch_ws_nc<6>(fp32, items, nitems, sims, flip, st);
        case 7: return launch_ws_nc<7>(fp32, items, nitems, sims, flip, st);
        case 8: return launch_ws_nc<8>(fp32, items, nitems, sims, flip, st);
        case 9: return launch_ws_nc<9>(fp32, items, nitems, sims, flip, st);
        case 10: return launch_ws_nc<10>(fp32, items, nitems, sims, flip, st);
        default: return hipErrorInvalidValue;
    }
}
