// Second and third passes of the three-pass D3Q19 step, after the moments
// pass has written rho_i, RT ln f_i, s = sum sqrt(kappa_j) rt_j and j:
//   velocity    u = (j + F / 2) / rho, F = -sum_i rt_i grad psi_i
//               (Section II.A, Eq. (2)), with psi_i = RT ln f_i
//               - sqrt(kappa_i) lap s (Eq. (3)-(6)) formed in LDS: lap s at
//               the tile's one-site halo points from s staged with a
//               two-site halo, psi_i staged per component over the
//               one-site halo;
//   collision   every component of the tile in turn: psi_i (as above) and
//               rho_i staged over the one-site halo, F_i = -rt_i grad psi_i,
//               G_i = grad rho_i, collision (Eq. (1a)-(1c)) and push.
// psi is never written to memory (the four-pass path writes it and reads it
// back twice).  The collision keeps the stores streaming: while a
// component's populations are computed and stored, the next component's
// halo loads are in flight, and a workgroup holds no per-component
// registers.  Every site's arithmetic is the four-pass path's, term for
// term, so the two paths give the same bits.
#include "generic_tiles.h"

namespace {

using TG3 = TileGeom<D3Q19, TileC<D3Q19>>;
static_assert(2 * TG3::NH <= TG3::NH2, "the staging buffers reuse the s tile");

// lap s at the tile's one-site halo points into lL, from s staged with a
// two-site halo in ls2 (ls2 is free again once this returns).
__device__ __forceinline__ void lap_s(const SimConst *c, const TG3 &T, const double *s_f,
                                      double *ls2, double *lL) {
    T.stage2(c, s_f, ls2);
    __syncthreads();
    for (int k = threadIdx.x; k < TG3::NH; k += TPB) {
        const int k2 = TG3::halo2_index(k);
        const double sc = ls2[k2];
        double acc = 0.0;
#pragma unroll
        for (int a = 1; a < D3Q19::Q; ++a)
            acc = fma(D3Q19::w(a), ls2[k2 + TG3::lds2_off(a)] - sc, acc);
        lL[k] = 6.0 * acc;
    }
    __syncthreads();
}

// u = (j + F/2) / rho, F = -sum_i rt_i grad psi_i -> u_f
__global__ __launch_bounds__(TPB) void k_velocity_mu(const SimConst *__restrict__ c,
                                                     const double *__restrict__ rho_f,
                                                     const double *__restrict__ mu_f,
                                                     const double *__restrict__ s_f,
                                                     const double *__restrict__ j_f,
                                                     double *__restrict__ u_f) {
    __shared__ double lds[TG3::NH2 + TG3::NH];
    double *const lL = lds + TG3::NH2;
    const int unit = xcd_unit();
    // padding units leave as a whole workgroup, before any barrier
    if (unit >= TG3::count(c->nx, c->ny, c->nz)) return;
    const TG3 T(c, unit);
    const int64_t ns = c->nsites;
    const int N = c->N;
    const int64_t s = T.active ? (int64_t)T.x + (int64_t)c->nx * ((int64_t)T.y + (int64_t)c->ny * T.z) : 0;
    typename TG3::HaloRegs h;
    T.load_halo(c, mu_f, h);   // the first component's RT ln f, in flight meanwhile
    lap_s(c, T, s_f, lds, lL);
    // psi_i double-buffered (component i uses the buffer at (i & 1) * NH):
    // one barrier per component
    double Fx = 0.0, Fy = 0.0, Fz = 0.0, rhot = 0.0;
#pragma unroll 1
    for (int i = 0; i < N; ++i) {
        double *const b = lds + (i & 1) * TG3::NH;
        const double sq = c->sqk[i];
        T.put_halo(h, b, [&](int k, double v) { return fma(-sq, lL[k], v); });
        if (i + 1 < N) T.load_halo(c, mu_f + (int64_t)(i + 1) * ns, h);
        const double r = T.active ? rho_f[(int64_t)i * ns + s] : 0.0;
        __syncthreads();
        if (T.active) {
            double gx, gy, gz;
            T.grad(b, gx, gy, gz);
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
    u_f[2 * ns + s] = fma(0.5, Fz, j_f[2 * ns + s]) / rhot;
}

// Collision and push of every component of one tile; u from u_f.
// KEEP: tau != 1, the collision keeps (1 - omega) g of the old population.
template <typename ST, bool KEEP>
__global__ __launch_bounds__(TPB) void k_collide_mu(const SimConst *__restrict__ c,
                                                    const void *__restrict__ gs,
                                                    void *__restrict__ gd,
                                                    const double *__restrict__ rho_f,
                                                    const double *__restrict__ mu_f,
                                                    const double *__restrict__ s_f,
                                                    const double *__restrict__ u_f) {
    __shared__ double lds[TG3::NH2 + TG3::NH];
    double *const lp = lds;              // psi_i (one-site halo); with lr, reuses the s tile
    double *const lr = lds + TG3::NH;    // rho_i
    double *const lL = lds + TG3::NH2;
    const int unit = xcd_unit();
    if (unit >= TG3::count(c->nx, c->ny, c->nz)) return;
    const TG3 T(c, unit);
    const int64_t ns = c->nsites;
    const int N = c->N;
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const int64_t s = T.active ? (int64_t)T.x + (int64_t)nx * ((int64_t)T.y + (int64_t)ny * T.z) : 0;
    double ux = 0.0, uy = 0.0, uz = 0.0;
    if (T.active) {
        ux = u_f[s];
        uy = u_f[ns + s];
        uz = u_f[2 * ns + s];
    }
    typename TG3::HaloRegs hm, hr;
    T.load_halo(c, mu_f, hm);
    T.load_halo(c, rho_f, hr);
    lap_s(c, T, s_f, lds, lL);
    const PopLayout<ST> P(N, D3Q19::Q, nx, (int64_t)ny * nz);
    const char *const gsb = (const char *)gs;
    char *const gdb = (char *)gd;
    const double omega = c->omega, fcoef = c->fcoef;
#pragma unroll 1
    for (int i = 0; i < N; ++i) {
        const double sq = c->sqk[i];
        T.put_halo(hm, lp, [&](int k, double v) { return fma(-sq, lL[k], v); });
        T.put_halo(hr, lr, [](int, double v) { return v; });
        if (i + 1 < N) {
            T.load_halo(c, mu_f + (int64_t)(i + 1) * ns, hm);
            T.load_halo(c, rho_f + (int64_t)(i + 1) * ns, hr);
        }
        __syncthreads();
        if (T.active) {
            double gx, gy, gz, Gx, Gy, Gz;
            T.grad(lp, gx, gy, gz);
            T.grad(lr, Gx, Gy, Gz);
            const double r = lr[T.lc];
            const double rt = r * c->invM[i];
            const double Fx = -rt * gx, Fy = -rt * gy, Fz = -rt * gz;
            // the site is the same for every component: without this
            // (empty) register constraint the compiler keeps each
            // direction's destination address live across the component
            // loop (the collision takes u the same way, for its e_a.u terms)
            int px = T.x, py = T.y, pz = T.z;
            asm volatile("" : "+v"(px), "+v"(py), "+v"(pz));
            if constexpr (KEEP)
                collide_push_keep<D3Q19, ST>(P, gsb, gdb, i, px, py, pz, nx, ny, nz, r, ux, uy, uz,
                                             Fx, Fy, Fz, Gx, Gy, Gz, omega, fcoef);
            else
                collide_push_tau1<D3Q19, ST>(P, gdb, i, px, py, pz, nx, ny, nz, r, ux, uy, uz, Fx,
                                             Fy, Fz, Gx, Gy, Gz, omega, fcoef);
        }
        __syncthreads();   // lp and lr are rewritten for the next component
    }
}

}  // namespace

hipError_t launch_velocity_collide(bool fp32, const SimConst *c, int nx, int ny, int nz,
                                   const void *gs, void *gd, const double *rho_f,
                                   const double *mu_f, const double *s_f, const double *j_f,
                                   double *u_f, bool keep_old, hipStream_t st) {
    const unsigned nb = unit_blocks(TG3::count(nx, ny, nz));
    hipLaunchKernelGGL(k_velocity_mu, dim3(nb), dim3(TPB), 0, st, c, rho_f, mu_f, s_f, j_f, u_f);
    if (fp32) {
        if (keep_old)
            hipLaunchKernelGGL((k_collide_mu<float, true>), dim3(nb), dim3(TPB), 0, st, c, gs, gd,
                               rho_f, mu_f, s_f, u_f);
        else
            hipLaunchKernelGGL((k_collide_mu<float, false>), dim3(nb), dim3(TPB), 0, st, c, gs, gd,
                               rho_f, mu_f, s_f, u_f);
    } else {
        if (keep_old)
            hipLaunchKernelGGL((k_collide_mu<double, true>), dim3(nb), dim3(TPB), 0, st, c, gs, gd,
                               rho_f, mu_f, s_f, u_f);
        else
            hipLaunchKernelGGL((k_collide_mu<double, false>), dim3(nb), dim3(TPB), 0, st, c, gs, gd,
                               rho_f, mu_f, s_f, u_f);
    }
    return hipGetLastError();
}
