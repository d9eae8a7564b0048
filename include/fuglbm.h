/*
 * fuglbm.h -- C ABI of the MI355X (gfx950) fugacity-based multicomponent
 * lattice Boltzmann hot path.
 *
 * One step, for every lattice site r and component i (paper Section II):
 *   rho_i = sum_a g_{a,i};  rt_i = rho_i / M_i                (molar density)
 *   ln f_i from the Peng-Robinson EOS, Eq. (9)-(12), local in rt_1..rt_N
 *           (SRK or van der Waals in its place: fuglbm_mixture_desc.eos)
 *   psi_i = RT ln f_i - sqrt(kappa_i) lap(sum_j sqrt(kappa_j) rt_j)
 *           (Eq. (3)-(5) with the rank-one kappa_ij of Eq. (4), kappa_i of Eq. (6))
 *   F_i = -rt_i grad(psi_i);  u = (sum_i sum_a e_a g_{a,i} + F/2) / rho
 *   g_{a,i}(r + e_a, t+1) = g - (g - geq)/tau + (1 - 1/(2tau)) F_{a,i}
 *           (Eq. (1a); equilibrium Eq. (1b) with rho^c = 0; forcing Eq. (1c))
 * on a periodic D2Q9 or D3Q19 lattice, dt = dx = 1, cs^2 = 1/3.  grad and lap
 * are the isotropic lattice stencils
 *   grad phi = 3 sum_a w_a e_a (phi(r+e_a) - phi(r-e_a)) / 2,
 *   lap  phi = 6 sum_a w_a (phi(r+e_a) - phi(r)).
 *
 * Conventions
 *  - Every call returns fuglbm_status; nothing is thrown across the ABI.  On a
 *    non-OK status fuglbm_last_error() returns a message for the calling
 *    thread.
 *  - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *    device memory of the current device; hip_stream is a hipStream_t (NULL:
 *    the null stream).
 *  - Descriptors and host arrays are copied during the call; the library
 *    never keeps a caller's host pointer.
 *  - A mixture must outlive every simulation made from it.  Handles are not
 *    thread-safe: use one handle from one thread at a time.
 *  - Streams: fuglbm_step_n and fuglbm_step_many may be called on a
 *    simulation with a different hip_stream than its previous call; the
 *    new launches then wait, on the device, for the simulation's earlier
 *    work (an event the library records after each such call), with no host
 *    synchronisation.  The synchronising calls (read_moments, diagnostics,
 *    read/write_populations, set_tuning, destroy_sim) run on and wait for
 *    the stream of the simulation's last enqueuing call, which must still
 *    exist then.  fuglbm_step_many_noalloc does not order across streams
 *    (see there).
 *  - Device populations (two buffers swapped every step): with FP64
 *    storage they are blocked by lattice row (row = y + ny*z): row r holds
 *    the rest populations g_{0,i} of all components as [ncomp][pitch]
 *    doubles, then the moving ones g_{a,i}, a >= 1, as [ncomp][Q-1][pitch]
 *    doubles.  With FP32 storage every (component, direction) has one
 *    array over the whole grid: [ncomp][sites + pad] doubles (rest), then
 *    [ncomp][Q-1][sites + pad] floats (moving).  With FP32 storage the
 *    rest population is stored as rho_i minus the FP64 sum of the site's
 *    stored moving populations, so component masses are conserved to FP64
 *    rounding (Eq. (1a)-(1c) conserve each component's mass); the fused
 *    D2Q9 kernels and the multi-pass kernels at tau == 1 collide the
 *    moving populations in FP32 arithmetic (at tau != 1 the multi-pass
 *    collision runs in FP64 and folds the moving populations' rounding
 *    error into the rest population).  Moments, the EOS, psi_i and the gradients are
 *    FP64 in both precisions.  Host-side population arrays
 *    (read/write_populations) are [ncomp][Q][sites] FP64, site = x +
 *    nx*(y + ny*z).
 *  - Direction order a (lattice vector e_a):
 *    D2Q9   0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1); 5 (1,1);
 *           6 (-1,1); 7 (-1,-1); 8 (1,-1).
 *    D3Q19  0 (0,0,0); faces 1 (1,0,0); 2 (-1,0,0); 3 (0,1,0); 4 (0,-1,0);
 *           5 (0,0,1); 6 (0,0,-1); edges 7 (1,1,0); 8 (-1,-1,0);
 *           9 (1,-1,0); 10 (-1,1,0); 11 (1,0,1); 12 (-1,0,-1); 13 (1,0,-1);
 *           14 (-1,0,1); 15 (0,1,1); 16 (0,-1,-1); 17 (0,1,-1); 18 (0,-1,1).
 */
#ifndef FUGLBM_H
#define FUGLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FUGLBM_MAX_COMP 16

typedef enum {
    FUGLBM_OK = 0,
    FUGLBM_EINVAL = 1,        /* bad argument: null pointer, size, range, asymmetric kij, tau <= 1/2 */
    FUGLBM_ENOMEM = 2,        /* device or host allocation failed, or dev_buf too small */
    FUGLBM_EDEVICE = 3,       /* a HIP runtime call failed */
    FUGLBM_EUNPHYSICAL = 4,   /* input field with rho_i <= 0, non-finite, or b_m*rt >= 1 */
    FUGLBM_ENONFINITE = 5,    /* sticky: the device saw a non-finite or out-of-domain state */
    FUGLBM_ESTATE = 6         /* call not valid in the handle's state (mixed lattice in a batch, ...) */
} fuglbm_status;

/* The last enumerator of each input enum only widens it to 32 bits, so
 * that any int a C caller passes is a valid value of the type (the library
 * rejects values other than the named ones with EINVAL). */
typedef enum { FUGLBM_D2Q9 = 0, FUGLBM_D3Q19 = 1, FUGLBM_LATTICE_INT32_ = 0x7fffffff } fuglbm_lattice;
typedef enum { FUGLBM_FP64 = 0, FUGLBM_FP32_STORAGE = 1, FUGLBM_PRECISION_INT32_ = 0x7fffffff } fuglbm_precision;

/* Cubic equation of state p = RT/(v - b) - a alpha / ((v + d1 b)(v + d2 b)).
 * PR is the paper's (Section II.C, Eq. (9)-(12)): d1,2 = 1 +- sqrt2,
 * a = 0.457235529 R^2 Tc^2/pc, b = 0.077796074 R Tc/pc, alpha of Section II.C.
 * SRK: d1 = 1, d2 = 0, a = R^2 Tc^2 / (9 (2^(1/3) - 1) pc),
 * b = (2^(1/3) - 1) R Tc / (3 pc), Soave's alpha (m = 0.480 + 1.574 w - 0.176 w^2).
 * vdW: d1 = d2 = 0, a = 27 R^2 Tc^2 / (64 pc), b = R Tc / (8 pc), alpha = 1.
 * The method takes any of them unchanged (Section I); only ln f_i and the
 * pressure differ. */
typedef enum { FUGLBM_EOS_PR = 0, FUGLBM_EOS_SRK = 1, FUGLBM_EOS_VDW = 2 } fuglbm_eos;

/* Device status bits (fuglbm_diag.status). */
#define FUGLBM_ST_NONFINITE 1u   /* a non-finite ln f_i, density or population */
#define FUGLBM_ST_COVOLUME  2u   /* 1 - b_m rt <= 0 (outside the EOS domain) */
#define FUGLBM_ST_NEGATIVE  4u   /* some rt_i <= 0 */

typedef struct fuglbm_mixture fuglbm_mixture;
typedef struct fuglbm_sim fuglbm_sim;

/* Physical description of a mixture (paper Table I units).  Lattice units
 * are fixed by R, a and b of the reference component (paper Section III.A:
 * R = 1, a = 2/49, b = 2/21, M = 1 for C1); kappa_i = kappa_ref a_i / a_ref
 * (Eq. (6)-(8)). */
typedef struct {
    int32_t ncomp;                 /* 1..FUGLBM_MAX_COMP */
    const double *Tc_K;            /* [ncomp] critical temperature, K */
    const double *pc_bar;          /* [ncomp] critical pressure, bar */
    const double *omega;           /* [ncomp] acentric factor */
    const double *M_gmol;          /* [ncomp] molar mass, g/mol */
    const double *kij;             /* [ncomp*ncomp] row-major, symmetric, zero diagonal;
                                      NULL = all zero (delta_ij of Eq. (10)) */
    double T_K;                    /* temperature (isothermal), K */
    int32_t ref_comp;              /* anchor and kappa reference component */
    double a_ref_lu, b_ref_lu, R_lu; /* 0 = defaults 2/49, 2/21, 1 */
    double kappa_ref_lu;           /* kappa of the reference component, lattice units */
    double tau;                    /* BGK relaxation time, > 1/2 (paper: 1) */
    int32_t eos;                   /* fuglbm_eos; 0 (a zeroed descriptor) = PR */
} fuglbm_mixture_desc;

/* Diagnostics of the current state (paper Section II.A: Eq. (1a)-(1c)
 * conserve every component's mass, since sum_a F_a = 0, sum_a (geq - g) = 0
 * and streaming only moves populations).  FP64 sums in a fixed order over a
 * fixed site assignment (no float atomics): bitwise reproducible for a given
 * grid.  Unused momentum components (z in 2-D) are 0. */
typedef struct {
    int64_t step;                  /* steps taken since init */
    double mass[FUGLBM_MAX_COMP];  /* sum_r rho_i */
    double momentum[3];            /* sum_r (sum_i sum_a e_a g_{a,i} + F/2) = sum_r rho u,
                                      the force-corrected momentum, F = sum_i F_i */
    double momentum_pop[3];        /* sum_r sum_i sum_a e_a g_{a,i} (populations' own) */
    double residual;               /* max_i sum_r |rho_i(t) - rho_i(t-K)| / (K sum_r rho_i(t)),
                                      K = steps since the previous diagnostics call
                                      (0 on the first call) */
    uint32_t status;               /* OR of FUGLBM_ST_* bits seen since init */
} fuglbm_diag;

/* Build a mixture: unit conversion and every per-component constant in
 * FP64 (a_i, b_i, alpha_i(T), (a alpha)_ij, sqrt kappa_i, M_i).
 * The lattice-unit anchors a_ref_lu, b_ref_lu are those of the chosen EOS's
 * a and b (defaults 2/49, 2/21 for every EOS).
 * Errors: EINVAL for null/out-of-range fields, non-positive Tc/pc/M/T,
 * tau <= 1/2, asymmetric kij or a non-zero kij diagonal, an unknown eos;
 * ENOMEM. */
fuglbm_status fuglbm_init_mixture(const fuglbm_mixture_desc *desc, fuglbm_mixture **out);

/* Copy the lattice-unit constants into host array out[n]:
 * [RT, then for each component b_i, (a alpha)_i, sqrt(kappa_i), M_i, then the
 *  ncomp x ncomp matrix (a alpha)_ij row-major]; n must be >= 1 + 4N + N^2. */
fuglbm_status fuglbm_lattice_constants(const fuglbm_mixture *mix, double *out, size_t n);

void fuglbm_destroy_mixture(fuglbm_mixture *mix);

/* Bytes of device memory one simulation needs (both population buffers and
 * the library's workspace), i.e. the minimum size of a borrowed dev_buf. */
size_t fuglbm_fields_bytes(int32_t ncomp, fuglbm_lattice lattice, fuglbm_precision prec,
                           int32_t nx, int32_t ny, int32_t nz);

/* Create a simulation and set g = geq(rho_i, u = 0) (g_0 = rho_i, others 0).
 * rho: host [ncomp][nz][ny][nx] mass densities in lattice units.
 * dev_buf: NULL = the library allocates; else a device buffer of at least
 *   fuglbm_fields_bytes() bytes, 256-byte aligned, borrowed (the caller keeps
 *   it alive until fuglbm_destroy_sim).
 * Enqueued on hip_stream; rho is copied before return.
 * Errors: EINVAL (sizes < 1, nz != 1 for D2Q9), EUNPHYSICAL (rho_i <= 0,
 * non-finite, or b_m rt >= 1 somewhere), ENOMEM, EDEVICE. */
fuglbm_status fuglbm_init_fields(const fuglbm_mixture *mix, fuglbm_lattice lattice,
                                 fuglbm_precision prec, int32_t nx, int32_t ny, int32_t nz,
                                 const double *rho, void *dev_buf, void *hip_stream,
                                 fuglbm_sim **out);

/* Enqueue nsteps steps on hip_stream (asynchronous; no host sync).  Returns
 * the sticky ENONFINITE without launching if an earlier synchronising call
 * saw a device status bit. */
fuglbm_status fuglbm_step_n(fuglbm_sim *sim, int64_t nsteps, void *hip_stream);

/* Advance count simulations by nsteps each, batched: D2Q9 simulations on a
 * fused kernel that share ncomp and precision are packed into one tile
 * table (one launch per step); the others (D3Q19, and D2Q9 on the
 * multi-pass kernels) that share lattice, precision and tau == 1 or not
 * into one member table per group (each of the four multi-pass kernels
 * launched once per step for the whole group).  Results are bitwise those
 * of stepping each simulation alone.  Handles must be distinct.
 * Asynchronous on hip_stream. */
fuglbm_status fuglbm_step_many(fuglbm_sim *const *sims, int32_t count, int64_t nsteps,
                               void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * batched step as fuglbm_step_many, with bitwise the same results, that
 * allocates nothing.  Its work tables live in a fixed device array of the
 * library (1.06 MB per GPU, held until the process ends) and are written
 * by a small table kernel on hip_stream from the call's arguments; each
 * step is one plain launch of the fused kernel per (ncomp, precision)
 * class of members (no graph, no tuning: every member keeps its current
 * fused variant and rows per work item).
 * Limits: at most 256 simulations and 65536 fused work items per call
 * (EINVAL beyond); every member must be a D2Q9 simulation on a fused
 * kernel (EINVAL otherwise).  No stream ordering: a member's earlier work
 * on another stream must be complete or ordered before hip_stream by the
 * caller, and so must this call's launches before a later call on another
 * stream.  Members with a sticky device error are
 * skipped and ENONFINITE is returned after the others have been stepped.
 * Every call on one GPU shares the array: calls that overlap on one GPU
 * (other streams or threads before this call's launches have finished)
 * race and must not be made. */
fuglbm_status fuglbm_step_many_noalloc(fuglbm_sim *const *sims, int32_t count, int64_t nsteps,
                                       void *hip_stream);

/* Synchronise and read macroscopic fields: rho_out host [ncomp][sites] (or
 * NULL), u_out host [D][sites] force-corrected velocity (or NULL), diag (or
 * NULL; as fuglbm_diagnostics).  Returns ENONFINITE if a status bit is set
 * (the fields are still written). */
fuglbm_status fuglbm_read_moments(fuglbm_sim *sim, double *rho_out, double *u_out,
                                  fuglbm_diag *diag);

/* Synchronise and compute mass, momentum, residual and status (see
 * fuglbm_diag): one pass of the fields kernels over the current state, then
 * wavefront (DPP) reductions into per-block partials and one fixed-order
 * final sum per quantity.  Keeps rho_i(t) (FP64) as the snapshot for the
 * next residual.  Returns ENONFINITE if a status bit is set (diag is still
 * filled). */
fuglbm_status fuglbm_diagnostics(fuglbm_sim *sim, fuglbm_diag *diag);

/* Checkpoint / restore the raw populations, host [ncomp][Q][sites] FP64
 * (with FP32 storage the moving populations are widened / rounded to
 * nearest; the rest populations are FP64 either way). */
fuglbm_status fuglbm_read_populations(fuglbm_sim *sim, double *g_out);
fuglbm_status fuglbm_write_populations(fuglbm_sim *sim, const double *g_in, int64_t step);

/* Launch tuning: kernel 0 = automatic, 1 = four-pass generic kernels,
 * 2 = fused one-pass D2Q9 kernel (register ring), 3 = fused one-pass D2Q9
 * kernel with store wavefronts (ncomp <= 10; bit-identical results).
 * Automatic: the fused kernels for D2Q9 (1 beyond 2^32 buffer elements),
 * 1 for D3Q19;
 * rows = output rows per fused work item (>= 1, fixed), or 0 = autotuned:
 * the next fuglbm_step_n times a few trial launches per candidate (they
 * read the current state and write the spare buffer, so the state does
 * not move) and keeps the fastest; with kernel 0 both fused variants are
 * timed and the faster (variant, rows) is kept.  The choice is cached per
 * (nx, ny, ncomp, precision) for the process.  The state does not depend
 * on the variant or on rows.  fuglbm_step_many tunes one (variant, rows)
 * per batch shape the same way unless a member has fixed rows.
 * Autotuning is the default.  EINVAL for a kernel the simulation cannot
 * use, or rows < 0. */
fuglbm_status fuglbm_set_tuning(fuglbm_sim *sim, int32_t kernel, int32_t rows);

/* Query the launch tuning in use: kernel (1 generic, 2 or 3 fused) and
 * fused rows per work item (0 for the generic kernels; with autotuning,
 * the values chosen once a step has run). */
fuglbm_status fuglbm_get_tuning(const fuglbm_sim *sim, int32_t *kernel, int32_t *rows);

/* Query: Q, spatial dimension, sites, bytes moved per step by the
 * algorithm (every population read and written once: 2 N (8 + (Q-1) s)
 * per site, s = 8 for FP64 and 4 for FP32 storage), and the kernel in use. */
fuglbm_status fuglbm_sim_info(const fuglbm_sim *sim, int32_t *Q, int32_t *D, int64_t *sites,
                              int64_t *alg_bytes_per_step, int32_t *kernel);

/* Test hook: overwrite one population (component comp, direction a, site)
 * in the current buffer with value; synchronous. */
fuglbm_status fuglbm_poke_population(fuglbm_sim *sim, int32_t comp, int32_t a, int64_t site,
                                     double value);

void fuglbm_destroy_sim(fuglbm_sim *sim);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *fuglbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FUGLBM_H */
