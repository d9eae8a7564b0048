// Device helpers shared by the fused D2Q9 kernels (both variants): address
// space views, DPP lane shifts, the pairwise-difference stencils, helper
// wave placement, the factored D2Q9 collision, the LDS block and the
// population row type.
#pragma once

#include "kernels.h"

namespace fused {

// Address-space-qualified views: constant (scalar loads) and global.
template <class T> using cptr = const __attribute__((address_space(4))) T *;
template <class T> using gptr = const __attribute__((address_space(1))) T *;
template <class T> using gmptr = __attribute__((address_space(1))) T *;

// DPP wavefront shifts (GFX9 family): lane l receives lane l-1 (wave_shr:1)
// or lane l+1 (wave_shl:1).  Lanes 0 / 63 receive 0; only lanes 1..62 use
// shifted values.
__device__ __forceinline__ double from_left(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
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

// Wave that computes part p (0..3) of the per-site sums.  Waves of a
// workgroup are dealt to the 4 SIMDs of a CU in turn, so with NC % 4 != 0
// the SIMDs s >= NC % 4 hold one wave fewer; the parts go to their waves.
template <int NC>
__device__ constexpr int helper_wave(int p) {
    int light[16] = {0};
    int n = 0;
    for (int w = 0; w < NC; ++w)
        if (NC % 4 == 0 || w % 4 >= NC % 4) light[n++] = w;
    if (n == 0)
        for (int w = 0; w < NC; ++w) light[n++] = w;
    return light[p % n];
}

// D2Q9 collision of one component at one site, Eq. (1a)-(1c) with
// rho^c = 0 and cs^2 = 1/3, factored per opposite pair of directions:
//   g*_a = (1 - omega) g_a + w_a T_a,
//   T_a  = omega geq_a / w_a + c F_a / w_a
//        = eu (A + B eu + 9c eF + 3c eG) + 3c eF + K(|e_a|^2),
//   A = 3 omega rho, B = 4.5 omega rho, c = 1 - 1/(2 tau),
//   K(e2) = -1.5 omega rho u.u - 3c F.u + c (1.5 e2 - 2) G.u,
// and g*_0 = (1 - omega) g_0 + omega rho + w_0 K(0).  For the pair +e / -e
// with P = B eu + 9c eF + 3c eG:  T+ = eu (A + P) + 3c eF + K,
// T- = eu (P - A) - 3c eF + K.
__device__ __forceinline__ void collide_pair(double A, double B, double C9, double C3, double K,
                                             double eu, double eF, double eG, double &tp,
                                             double &tm) {
    const double P = fma(C3, eG, fma(C9, eF, B * eu));
    tp = fma(eu, A + P, fma(C3, eF, K));
    tm = fma(eu, P - A, fma(-C3, eF, K));
}

// The same collision for FP32 storage: the eight moving populations in
// FP32 arithmetic (they are stored in FP32; the per-site terms A, B, K, u,
// F, G come in FP64 and are rounded once).  The caller stores the rest
// population as rho - (the FP64 sum of the eight stored values, in
// direction order), so that Eq. (1a)-(1c), which conserve each
// component's mass, conserve it to FP64 rounding here too; the EOS, psi
// and the gradients stay FP64.  m: direction a = m + 1 of the D2Q9 order.
__device__ __forceinline__ double collide_moving_f32(double A, double B, double C9, double C3,
                                                     double K1, double K2, double omc, double ux,
                                                     double uy, double Fx, double Fy, double Gx,
                                                     double Gy, const float (&g)[8],
                                                     float (&t)[8]) {
    const float fA = (float)A, fB = (float)B, f9 = (float)C9, f3 = (float)C3;
    const float fomc = (float)omc;
    const float fux = (float)ux, fuy = (float)uy, fFx = (float)Fx, fFy = (float)Fy;
    const float fGx = (float)Gx, fGy = (float)Gy;
    auto pair = [&](float K, float eu, float eF, float eG, float w, int mp, int mm) {
        const float P = fmaf(f3, eG, fmaf(f9, eF, fB * eu));
        const float tp = fmaf(eu, fA + P, fmaf(f3, eF, K));
        const float tm = fmaf(eu, P - fA, fmaf(-f3, eF, K));
        t[mp] = fmaf(fomc, g[mp], w * tp);
        t[mm] = fmaf(fomc, g[mm], w * tm);
    };
    pair((float)K1, fux, fFx, fGx, 1.0f / 9.0f, 0, 2);
    pair((float)K1, fuy, fFy, fGy, 1.0f / 9.0f, 1, 3);
    pair((float)K2, fux + fuy, fFx + fFy, fGx + fGy, 1.0f / 36.0f, 4, 6);
    pair((float)K2, fuy - fux, fFy - fFx, fGy - fGx, 1.0f / 36.0f, 5, 7);
    double msum = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m) msum += (double)t[m];
    return msum;
}

template <int NC>
struct FusedLds {
    double rt[NC][64];      // molar densities of row r
    double jx[NC][64];      // per-component momentum of row r
    double jy[NC][64];
    double xs[NC][64];      // rt_i Sraw_i of row r
    double fx[NC][64];      // per-component force of row y
    double fy[NC][64];
    double tot[4][3][64];   // ring over rows (slot = row & 3): 1/rho, jx, jy
    double mx[2][2][64];    // ring over rows (slot = row & 1): rt, b_m rt
    double eos[5][64];      // row r-1: c1, c2a, c2b, c3b (helper A), lambda (helper B)
};

// 1/x to ~1 ulp: hardware reciprocal estimate and two Newton steps.
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Populations of one component at one site: the rest one in FP64, the
// moving ones (directions 1..8) in the storage type.
template <typename ST>
struct PopRow {
    double r;
    ST m[8];
};

}  // namespace fused
