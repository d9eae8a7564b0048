// Fused one-pass D2Q9 step (moments -> PR fugacity -> interface potential ->
// force -> collide -> push-stream) for gfx950.
//
// Work item = a 64-column strip (60 output columns plus a 2-column halo on
// each side) of one simulation, marching up `rows` output rows.  The
// workgroup has one wavefront per component (lane = column), so each lane
// keeps only its own component's 9 populations of the rows in flight in
// registers; quantities that mix components (total molar density, b_m rt,
// sum_j x_j (a alpha)_ij, s = sum_j sqrt(kappa_j) rt_j, momentum, total force)
// are exchanged through LDS, with two workgroup barriers per row.  The
// y-stencils use register rings, the x-stencils DPP lane shifts.
//
// Per lead row r (output row y = r - 2):
//   A  moments of row r (loaded one iteration earlier) -> LDS
//   B  row r-1: rt, b_m rt, S_i                        -> LDS (x_i S_i)
//   -- barrier --
//   C  row r-1: a_m, RT ln f_i; s(r); lap s(r-1); psi_i(r-1) = RT ln f_i - sqrt(k_i) lap s
//      totals of row r (rho, j)
//   D  row y: F_i = -rt_i grad psi_i, G_i = grad rho_i  -> LDS (F_i)
//   -- barrier --
//   E  row y: u = (j + F/2) / rho, collide the row-y populations, push-store
// Every population is read from HBM once per step; the 4 halo columns and
// the 4 warm-up rows of a work item are re-reads that neighbouring items
// issue at about the same time (the item order keeps them on one XCD).
#include "kernels.h"

namespace {

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

template <int NC, typename ST>
__global__ __launch_bounds__(64 * NC) void k_fused_d2q9(const FusedItem *__restrict__ items,
                                                        const FusedSim *__restrict__ sims,
                                                        int flip) {
    __shared__ double rt_l[2][NC][64];
    __shared__ double jx_l[NC][64];
    __shared__ double jy_l[NC][64];
    __shared__ double xs_l[NC][64];
    __shared__ double fx_l[NC][64];
    __shared__ double fy_l[NC][64];

    const FusedItem it = items[blockIdx.x];
    if (it.sim < 0) return;
    const FusedSim sm = sims[it.sim];
    const SimConst *__restrict__ C = sm.c;
    const int comp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int nx = C->nx, ny = C->ny;
    const int64_t ns = C->nsites;
    const int par = (sm.parity ^ flip) & 1;
    const ST *__restrict__ gsrc = (const ST *)sm.buf[par] + (int64_t)comp * 9 * ns;
    ST *__restrict__ gdst = (ST *)sm.buf[par ^ 1] + (int64_t)comp * 9 * ns;

    int xc = (it.x0 - 2 + lane) % nx;
    if (xc < 0) xc += nx;
    const int xm = xc == 0 ? nx - 1 : xc - 1;
    const int xp = xc == nx - 1 ? 0 : xc + 1;
    const bool outl = lane >= 2 && lane < 62 && (it.x0 + lane - 2) < nx;

    const double invM = C->invM[comp];
    const double bi = C->b[comp];
    const double sqki = C->sqk[comp];
    const double rb = C->rhobar[comp];
    const double RT = C->RT, omega = C->omega, fcoef = C->fcoef;
    const double *__restrict__ arow = C->aij + comp * FUG_MAXC;

    auto wrap_row = [ny](int r) {
        r %= ny;
        return r < 0 ? r + ny : r;
    };

    ST gp0[9], gp1[9], gp2[9], gp3[9];
    {
        const int64_t off = (int64_t)wrap_row(it.y0 - 2) * nx + xc;
#pragma unroll
        for (int a = 0; a < 9; ++a) gp2[a] = gsrc[a * ns + off];
#pragma unroll
        for (int a = 0; a < 9; ++a) gp0[a] = gp1[a] = gp3[a] = (ST)0;
    }
    double rho_r[4] = {0.0, 0.0, 0.0, 0.0};
    double psi_r[3] = {0.0, 0.0, 0.0};
    double s_r[3] = {0.0, 0.0, 0.0};
    double rt_r[3] = {1.0, 1.0, 1.0}, jx_r[3] = {0.0, 0.0, 0.0}, jy_r[3] = {0.0, 0.0, 0.0};
    uint32_t bad = 0;

    const int rbeg = it.y0 - 2, rend = it.y0 + it.rows + 1;
    for (int r = rbeg; r <= rend; ++r) {
        const int slot = r & 1;
        // prefetch row r + 1
        if (r < rend) {
            const int64_t off = (int64_t)wrap_row(r + 1) * nx + xc;
#pragma unroll
            for (int a = 0; a < 9; ++a) gp3[a] = gsrc[a * ns + off];
        }
        // ---- A: moments of row r
        {
            double v[9];
#pragma unroll
            for (int a = 0; a < 9; ++a) v[a] = (double)gp2[a];
            v[0] += rb;
            double rho = 0.0;
#pragma unroll
            for (int a = 0; a < 9; ++a) rho += v[a];
            const double jx = (v[1] - v[3]) + (v[5] - v[7]) + (v[8] - v[6]);
            const double jy = (v[2] - v[4]) + (v[5] - v[7]) + (v[6] - v[8]);
            rho_r[3] = rho;
            rt_l[slot][comp][lane] = rho * invM;
            jx_l[comp][lane] = jx;
            jy_l[comp][lane] = jy;
        }
        // ---- B: mixture sums of row r - 1
        const bool do_eos = r >= it.y0;
        double rtt = 1.0, eta = 0.0, Sraw = 0.0, rti = 1.0;
        if (do_eos) {
            rtt = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const double t = rt_l[slot ^ 1][j][lane];
                rtt += t;
                eta += C->b[j] * t;
                Sraw += arow[j] * t;
            }
            rti = rt_l[slot ^ 1][comp][lane];
            xs_l[comp][lane] = rti * Sraw / (rtt * rtt);
        }
        __syncthreads();
        // ---- C: totals of row r; fugacity and potential of row r - 1
        {
            double sv = 0.0, rtot = 0.0, jxt = 0.0, jyt = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const double t = rt_l[slot][j][lane];
                sv += C->sqk[j] * t;
                rtot += C->M[j] * t;
                jxt += jx_l[j][lane];
                jyt += jy_l[j][lane];
            }
            s_r[2] = sv;
            rt_r[2] = rtot;
            jx_r[2] = jxt;
            jy_r[2] = jyt;
        }
        if (do_eos) {
            double am = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) am += xs_l[j][lane];
            const MixSums m = pr_mixture(rtt, eta, am, RT);
            const double lnf = pr_RTlnf(m, RT, rti, bi, Sraw / rtt);
            const double L = lap3(s_r[0], s_r[1], s_r[2]);
            const double psi = lnf - sqki * L;
            psi_r[2] = psi;
            uint32_t b = m.bad;
            if (!(rti > 0.0)) b |= FUG_ST_NEGATIVE;
            if (!isfinite(psi)) b |= FUG_ST_NONFINITE;
            bad |= b;
        }
        // ---- D: forces of output row y = r - 2
        const bool do_out = r >= it.y0 + 2;
        double Fx = 0.0, Fy = 0.0, Gx = 0.0, Gy = 0.0;
        if (do_out) {
            double gx, gy;
            grad3(psi_r[0], psi_r[1], psi_r[2], gx, gy);
            const double rty = rho_r[1] * invM;
            Fx = -rty * gx;
            Fy = -rty * gy;
            grad3(rho_r[0], rho_r[1], rho_r[2], Gx, Gy);
            fx_l[comp][lane] = Fx;
            fy_l[comp][lane] = Fy;
        }
        __syncthreads();
        // ---- E: velocity, collision and push of row y
        if (do_out) {
            double Fsx = 0.0, Fsy = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                Fsx += fx_l[j][lane];
                Fsy += fy_l[j][lane];
            }
            const double ux = (jx_r[0] + 0.5 * Fsx) / rt_r[0];
            const double uy = (jy_r[0] + 0.5 * Fsy) / rt_r[0];
            const double uu = ux * ux + uy * uy;
            const double Fu = Fx * ux + Fy * uy;
            const double Gu = Gx * ux + Gy * uy;
            const double rho = rho_r[1];
            const int y = r - 2;
            const int yrow[3] = {wrap_row(y - 1), wrap_row(y), wrap_row(y + 1)};
            if (outl) {
#pragma unroll
                for (int a = 0; a < 9; ++a) {
                    double gv = (double)gp0[a];
                    if (a == 0) gv += rb;
                    double o = collide_one<D2Q9>(a, gv, rho, ux, uy, 0.0, Fx, Fy, 0.0, Gx, Gy, 0.0,
                                                 uu, Fu, Gu, omega, fcoef);
                    if (a == 0) o -= rb;
                    const int exa = D2Q9::ex(a), eya = D2Q9::ey(a);
                    const int xx = exa == 0 ? xc : (exa > 0 ? xp : xm);
                    const int64_t off = (int64_t)yrow[eya + 1] * nx + xx;
                    gdst[a * ns + off] = (ST)o;
                }
            }
        }
        // ---- rotate the rings
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            gp0[a] = gp1[a];
            gp1[a] = gp2[a];
            gp2[a] = gp3[a];
        }
        rho_r[0] = rho_r[1];
        rho_r[1] = rho_r[2];
        rho_r[2] = rho_r[3];
        psi_r[0] = psi_r[1];
        psi_r[1] = psi_r[2];
        s_r[0] = s_r[1];
        s_r[1] = s_r[2];
        rt_r[0] = rt_r[1];
        rt_r[1] = rt_r[2];
        jx_r[0] = jx_r[1];
        jx_r[1] = jx_r[2];
        jy_r[0] = jy_r[1];
        jy_r[1] = jy_r[2];
    }
    if (bad) atomicOr(sm.status, bad);
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
