// Kernel launchers (C++ linkage, internal to the library).
#pragma once

#include "lbm_common.h"

// One work item of the fused D2Q9 kernel: a 60-column strip of a simulation
// starting at column x0, output rows [y0, y0 + rows).  sim < 0: padding.
struct FusedItem {
    int32_t sim, x0, y0, rows;
};

// Per-simulation pointers for the fused kernel.  The source buffer of a
// launch is buf[parity ^ flip], the destination the other one.
struct FusedSim {
    const SimConst *c;
    void *buf[2];
    uint32_t *status;
    int32_t parity;
    int32_t pad;
};

constexpr int FUSED_LANES = 64;
constexpr int FUSED_OUT = 60;  // output columns per strip (2-column halo each side)

hipError_t launch_init(int lattice, bool fp32, const SimConst *c, int64_t ns, const double *rho,
                       void *g, hipStream_t st);
// keep_old: tau != 1, the collision reads the old populations
hipError_t launch_step_generic(int lattice, bool fp32, const SimConst *c, int ncomp, int nx, int ny,
                               int nz, const void *gs, void *gd, double *rho_f, double *psi_f,
                               double *s_f, double *j_f, double *u_f, uint32_t *status,
                               bool keep_old, hipStream_t st);
// One member of a batched multi-pass step (fuglbm_step_many for simulations
// on the multi-pass kernels).  A launch reads buf[parity ^ flip] and writes
// the other buffer.  end[p]: work units of pass p through this member,
// cumulative over the table (p = 0: TPB-site blocks of the moments and
// interface passes, 1: velocity tiles, 2: collision (tile, component) units).
struct GenMember {
    const SimConst *c;
    void *buf[2];
    double *rho_f, *psi_f, *s_f, *j_f, *u_f;
    uint32_t *status;
    int64_t end[3];
    int32_t parity;
    int32_t pad;
};
// Work units of one simulation for the three kinds of GenMember::end.
void generic_units(int lattice, int ncomp, int nx, int ny, int nz, int64_t units[3]);
// One step of every member (same lattice, storage precision and keep_old);
// total[p] = members[nmembers - 1].end[p].
hipError_t launch_step_generic_batch(int lattice, bool fp32, bool keep_old,
                                     const GenMember *members, int nmembers,
                                     const int64_t total[3], int flip, hipStream_t st);
// Macroscopic fields of a state: rho_i, RT ln f_i -> psi_i, s, j and (u_f
// non-null) the force-corrected velocity.
hipError_t launch_fields(int lattice, bool fp32, const SimConst *c, int nx, int ny, int nz,
                         const void *g, double *rho_f, double *psi_f, double *s_f, double *j_f,
                         double *u_f, uint32_t *status, hipStream_t st);
// Diagnostic sums over the fields (rho_i, j, u): per-block partials in
// part[(ncomp + 1) * nblk * DIAG_QUANT], final sums in out[(ncomp + 1) * DIAG_QUANT]:
// out[i] = {mass_i, sum |rho_i - snap_i|, 0...} for i < ncomp (snap_i <- rho_i),
// out[ncomp] = {sum j (3), sum rho u (3)}.
constexpr int DIAG_QUANT = 6;
hipError_t launch_diag(int dim, int ncomp, int64_t ns, const double *rho_f, const double *j_f,
                       const double *u_f, double *snap, double *part, int nblk, double *out,
                       int use_snap, hipStream_t st);
int diag_blocks(int64_t ns);

// Fused one-pass D2Q9 step over a table of work items (any mix of
// simulations with the same component count and storage precision).
// Resident workgroups of the fused kernel per CU (occupancy query).
int fused_blocks_per_cu(int ncomp, bool fp32);

hipError_t launch_fused_d2q9(int ncomp, bool fp32, const FusedItem *items, int nitems,
                             const FusedSim *sims, int flip, hipStream_t st);

// Store-wave variant of the fused D2Q9 step (component waves only load;
// two extra waves per workgroup store; rows requested three ahead).  Same
// items, same results bit for bit.  Built for ncomp <= fused_ws_max_comp().
int fused_ws_max_comp();
bool fused_ws_fits(int ncomp, bool fp32);
int fused_ws_blocks_per_cu(int ncomp, bool fp32);
hipError_t launch_fused_d2q9_ws(int ncomp, bool fp32, const FusedItem *items, int nitems,
                                const FusedSim *sims, int flip, hipStream_t st);
