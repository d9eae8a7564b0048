/*
 * Plain FP64 CPU oracle of the fugacity-based multicomponent lattice
 * Boltzmann step (paper Section II.A-II.C).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no source, header,
 * table or helper with the GPU library: the velocity sets, weights, stencils,
 * equation of state and collision are all written out again here.
 *
 * Every function follows the paper's notation:
 *   g[site][i][alpha]    populations, array-of-structures (this file's own
 *                        layout, deliberately unlike the GPU's);
 *   rho_i, rt_i          mass and molar density of component i (rt = rho~);
 *   lnf_i                ln of the fugacity of component i, Eq. (12) rewritten
 *                        so that it stays defined where p <= 0 (see below);
 *   psi_i = RT lnf_i - sum_j kappa_ij lap(rt_j)      (potential of Eq. (5));
 *   F_i = -rt_i grad(psi_i)                          (Eq. (3) and (5));
 *   u = (sum_i sum_a e_a g + F/2) / rho              (common velocity);
 *   g* = g - (g - geq)/tau + (1 - 1/(2 tau)) F_a     (Eq. (1a)), geq Eq. (1b)
 *                                                    with rho^c = 0, F_a Eq. (1c);
 *   push streaming with periodic wrap.
 * Discrete derivatives are the isotropic lattice stencils
 *   grad phi = cs^-2 sum_a w_a e_a (phi(r+e_a) - phi(r-e_a)) / 2,
 *   lap  phi = 2 cs^-2 sum_a w_a (phi(r+e_a) - phi(r)).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXC 16
#define OR_MAXQ 19

typedef struct {
    int lattice;            /* 0 = D2Q9, 1 = D3Q19 */
    int N;                  /* number of components */
    int nx, ny, nz;         /* nz = 1 for D2Q9 */
    double tau;
    double RT;
    double rho_c;           /* the rho^c constant of Eq. (1b); the paper sets 0 */
    double b[OR_MAXC];      /* co-volumes, lattice units */
    double M[OR_MAXC];      /* molar masses, lattice units */
    double sqk[OR_MAXC];    /* sqrt(kappa_i) */
    double aij[OR_MAXC * OR_MAXC]; /* (a alpha)_ij = sqrt(aa_i aa_j)(1 - k_ij) */
    int eos;                /* 0 = Peng-Robinson (the paper's), 1 = SRK, 2 = vdW */
    double d1, d2;          /* p = RT/(v-b) - a alpha/((v + d1 b)(v + d2 b)) */
} oracle_params;

/* ---- velocity sets ------------------------------------------------------ */
/* D2Q9: rest, 4 axis neighbours (w 1/9), 4 diagonals (w 1/36).               */
/* D3Q19: rest (1/3), 6 faces (1/18), 12 edges (1/36).                         */
static int lattice_set(int lattice, int e[][3], double *w) {
    if (lattice == 0) {
        static const int E[9][3] = {{0,0,0},{1,0,0},{0,1,0},{-1,0,0},{0,-1,0},
                                    {1,1,0},{-1,1,0},{-1,-1,0},{1,-1,0}};
        for (int a = 0; a < 9; ++a) {
            for (int d = 0; d < 3; ++d) e[a][d] = E[a][d];
            int n2 = E[a][0] * E[a][0] + E[a][1] * E[a][1];
            w[a] = n2 == 0 ? 4.0 / 9.0 : (n2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
        return 9;
    }
    int q = 0;
    for (int z = -1; z <= 1; ++z)
        for (int y = -1; y <= 1; ++y)
            for (int x = -1; x <= 1; ++x) {
                int n2 = x * x + y * y + z * z;
                if (n2 == 3) continue;
                e[q][0] = x; e[q][1] = y; e[q][2] = z;
                w[q] = n2 == 0 ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
                ++q;
            }
    /* move the rest direction to index 0 */
    for (int a = 0; a < q; ++a)
        if (e[a][0] == 0 && e[a][1] == 0 && e[a][2] == 0 && a != 0) {
            int t[3] = {e[0][0], e[0][1], e[0][2]};
            double tw = w[0];
            for (int d = 0; d < 3; ++d) { e[0][d] = e[a][d]; e[a][d] = t[d]; }
            w[0] = w[a]; w[a] = tw;
        }
    return q;
}

int oracle_velocity_set(int lattice, int *e_out, double *w_out) {
    int e[OR_MAXQ][3];
    double w[OR_MAXQ];
    int Q = lattice_set(lattice, e, w);
    for (int a = 0; a < Q; ++a) {
        for (int d = 0; d < 3; ++d) e_out[3 * a + d] = e[a][d];
        w_out[a] = w[a];
    }
    return Q;
}

static const double CS2 = 1.0 / 3.0;

/* ---- Eq. (1b): well-balanced equilibrium ------------------------------- */
void oracle_equilibrium(int lattice, double rho, double rho_c, const double *u,
                        double *geq) {
    int e[OR_MAXQ][3];
    double w[OR_MAXQ];
    int Q = lattice_set(lattice, e, w);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int a = 0; a < Q; ++a) {
        double eu = e[a][0] * u[0] + e[a][1] * u[1] + e[a][2] * u[2];
        double s = eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
        if (a == 0)
            geq[a] = rho - (1.0 - w[0]) * rho_c + w[0] * rho * s;
        else
            geq[a] = w[a] * rho_c + w[a] * rho * s;
    }
}

/* ---- Eq. (1c): forcing term; G = grad(rho_i), D = spatial dimension ----- */
void oracle_forcing(int lattice, const double *F, const double *G,
                    const double *u, double *Fa) {
    int e[OR_MAXQ][3];
    double w[OR_MAXQ];
    int Q = lattice_set(lattice, e, w);
    double D = lattice == 0 ? 2.0 : 3.0;
    for (int a = 0; a < Q; ++a) {
        double eu = e[a][0] * u[0] + e[a][1] * u[1] + e[a][2] * u[2];
        double e2 = (double)(e[a][0] * e[a][0] + e[a][1] * e[a][1] + e[a][2] * e[a][2]);
        double t1 = 0.0, t2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            double v1 = (e[a][d] - u[d]) / CS2 + eu * e[a][d] / (CS2 * CS2);
            double v2 = -u[d] + eu * e[a][d] / CS2 + 0.5 * (e2 / CS2 - D) * u[d];
            t1 += F[d] * v1;
            t2 += G[d] * v2;
        }
        Fa[a] = w[a] * t1 + w[a] * t2;
    }
}

/* ---- Eq. (9)-(12): cubic-EOS pressure and ln f_i ---------------------- */
/* Eq. (12) as printed contains ln(x_i p) and ln((v - b_m) p / RT), which are
 * undefined where p <= 0 (inside interfaces).  Their sum is
 * ln(rt_i RT / (1 - b_m rt)), so the oracle evaluates, for the cubic
 * p = RT/(v - b_m) - a_m / ((v + d1 b_m)(v + d2 b_m))  (PR: Eq. (9)),
 *   ln f_i = ln(rt_i RT/(1 - eta)) + (b_i/b_m)(Z - 1)
 *            - (a_m / (b_m RT)) (2 S_i / a_m - b_i / b_m) Lam,
 *   Lam = ln[(1 + d1 eta) / (1 + d2 eta)] / (d1 - d2)   (PR, SRK),
 *   Lam = eta                                           (vdW, d1 = d2 = 0:
 *         the limit, which gives b_i rt/(1 - eta) - 2 S_i rt / RT for the
 *         non-logarithmic terms, the textbook vdW expression),
 * eta = b_m rt, Z = p / (rt RT), S_i = sum_j x_j (a alpha)_ij.  For PR,
 * d1 - d2 = 2 sqrt2 and this is Eq. (12) term by term.
 * Returns status bits: 2 if 1 - eta <= 0, 4 if some rt_i <= 0.            */
int oracle_ln_fugacity(const oracle_params *P, const double *rt_i, double *lnf,
                       double *p_out) {
    const int N = P->N;
    int st = 0;
    double rt = 0.0;
    for (int i = 0; i < N; ++i) {
        rt += rt_i[i];
        if (!(rt_i[i] > 0.0)) st |= 4;
    }
    double x[OR_MAXC], S[OR_MAXC];
    for (int i = 0; i < N; ++i) x[i] = rt_i[i] / rt;
    double bm = 0.0;
    for (int i = 0; i < N; ++i) bm += x[i] * P->b[i];
    double am = 0.0;
    for (int i = 0; i < N; ++i) {
        S[i] = 0.0;
        for (int j = 0; j < N; ++j) S[i] += x[j] * P->aij[i * OR_MAXC + j];
        am += x[i] * S[i];
    }
    double eta = bm * rt;
    if (!(1.0 - eta > 0.0)) st |= 2;
    double p = rt * P->RT / (1.0 - eta)
             - am * rt * rt / ((1.0 + P->d1 * eta) * (1.0 + P->d2 * eta));
    double Z = p / (rt * P->RT);
    double Lam = P->eos == 2 ? eta
               : log((1.0 + P->d1 * eta) / (1.0 + P->d2 * eta)) / (P->d1 - P->d2);
    for (int i = 0; i < N; ++i) {
        lnf[i] = log(rt_i[i] * P->RT / (1.0 - eta)) + P->b[i] / bm * (Z - 1.0)
               - am / (bm * P->RT) * (2.0 * S[i] / am - P->b[i] / bm) * Lam;
    }
    if (p_out) *p_out = p;
    return st;
}

/* ---- grid helpers ------------------------------------------------------- */
static long nsites(const oracle_params *P) { return (long)P->nx * P->ny * P->nz; }

static long neighbour(const oracle_params *P, long s, const int *e) {
    long x = s % P->nx, y = (s / P->nx) % P->ny, z = s / ((long)P->nx * P->ny);
    x = (x + e[0] + P->nx) % P->nx;
    y = (y + e[1] + P->ny) % P->ny;
    z = (z + e[2] + P->nz) % P->nz;
    return x + (long)P->nx * (y + (long)P->ny * z);
}

/* grad phi at every site; out[d * sites + s] */
void oracle_gradient(const oracle_params *P, const double *phi, double *out) {
    int e[OR_MAXQ][3];
    double w[OR_MAXQ];
    int Q = lattice_set(P->lattice, e, w);
    long ns = nsites(P);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < ns; ++s) {
        double g[3] = {0.0, 0.0, 0.0};
        for (int a = 1; a < Q; ++a) {
            int me[3] = {-e[a][0], -e[a][1], -e[a][2]};
            double diff = phi[neighbour(P, s, e[a])] - phi[neighbour(P, s, me)];
            for (int d = 0; d < 3; ++d) g[d] += w[a] * e[a][d] * 0.5 * diff;
        }
        for (int d = 0; d < 3; ++d) out[d * ns + s] = g[d] / CS2;
    }
}

void oracle_laplacian(const oracle_params *P, const double *phi, double *out) {
    int e[OR_MAXQ][3];
    double w[OR_MAXQ];
    int Q = lattice_set(P->lattice, e, w);
    long ns = nsites(P);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < ns; ++s) {
        double acc = 0.0;
        for (int a = 1; a < Q; ++a) acc += w[a] * (phi[neighbour(P, s, e[a])] - phi[s]);
        out[s] = 2.0 * acc / CS2;
    }
}

/* ---- macroscopic fields of one state ------------------------------------ */
typedef struct {
    double *rho;   /* [N][sites] mass density */
    double *rt;    /* [N][sites] molar density */
    double *j;     /* [3][sites] sum_i sum_a e_a g */
    double *lnf;   /* [N][sites] */
    double *s;     /* [sites] sum_j sqrt(kappa_j) rt_j */
    double *L;     /* [sites] lap(s) */
    double *psi;   /* [N][sites] */
    double *F;     /* [N][3][sites] */
    double *G;     /* [N][3][sites] grad rho_i */
    double *u;     /* [3][sites] */
    double *rhot;  /* [sites] total mass density */
    double *tmp;   /* [3][sites] */
} fields;

static void fields_alloc(const oracle_params *P, fields *f) {
    long ns = nsites(P);
    int N = P->N;
    f->rho = calloc((size_t)N * ns, sizeof(double));
    f->rt = calloc((size_t)N * ns, sizeof(double));
    f->j = calloc((size_t)3 * ns, sizeof(double));
    f->lnf = calloc((size_t)N * ns, sizeof(double));
    f->s = calloc((size_t)ns, sizeof(double));
    f->L = calloc((size_t)ns, sizeof(double));
    f->psi = calloc((size_t)N * ns, sizeof(double));
    f->F = calloc((size_t)N * 3 * ns, sizeof(double));
    f->G = calloc((size_t)N * 3 * ns, sizeof(double));
    f->u = calloc((size_t)3 * ns, sizeof(double));
    f->rhot = calloc((size_t)ns, sizeof(double));
    f->tmp = calloc((size_t)3 * ns, sizeof(double));
}

static void fields_free(fields *f) {
    free(f->rho); free(f->rt); free(f->j); free(f->lnf); free(f->s); free(f->L);
    free(f->psi); free(f->F); free(f->G); free(f->u); free(f->rhot); free(f->tmp);
}

static int compute_fields(const oracle_params *P, const double *g, fields *f) {
    int e[OR_MAXQ][3];
    double w[OR_MAXQ];
    int Q = lattice_set(P->lattice, e, w);
    const int N = P->N;
    long ns = nsites(P);
    int status = 0;
    /* moments: rho_i = sum_a g, rt_i = rho_i / M_i, j = sum_i sum_a e_a g */
#pragma omp parallel for schedule(static)
    for (long s = 0; s < ns; ++s) {
        double j[3] = {0.0, 0.0, 0.0};
        double tot = 0.0;
        for (int i = 0; i < N; ++i) {
            double r = 0.0;
            for (int a = 0; a < Q; ++a) {
                double ga = g[((size_t)s * N + i) * Q + a];
                r += ga;
                for (int d = 0; d < 3; ++d) j[d] += e[a][d] * ga;
            }
            f->rho[(size_t)i * ns + s] = r;
            f->rt[(size_t)i * ns + s] = r / P->M[i];
            tot += r;
        }
        f->rhot[s] = tot;
        for (int d = 0; d < 3; ++d) f->j[(size_t)d * ns + s] = j[d];
    }
    /* local equation of state and s = sum_j sqrt(kappa_j) rt_j */
#pragma omp parallel for schedule(static) reduction(| : status)
    for (long s = 0; s < ns; ++s) {
        double rt[OR_MAXC], lnf[OR_MAXC];
        double sv = 0.0;
        for (int i = 0; i < N; ++i) {
            rt[i] = f->rt[(size_t)i * ns + s];
            sv += P->sqk[i] * rt[i];
        }
        status |= oracle_ln_fugacity(P, rt, lnf, NULL);
        for (int i = 0; i < N; ++i) {
            f->lnf[(size_t)i * ns + s] = lnf[i];
            if (!isfinite(lnf[i])) status |= 1;
        }
        f->s[s] = sv;
    }
    /* sum_j kappa_ij lap(rt_j) = sqrt(kappa_i) lap(s), Eq. (4)-(5) */
    oracle_laplacian(P, f->s, f->L);
    for (int i = 0; i < N; ++i)
        for (long s = 0; s < ns; ++s)
            f->psi[(size_t)i * ns + s] =
                P->RT * f->lnf[(size_t)i * ns + s] - P->sqk[i] * f->L[s];
    /* F_i = -rt_i grad(psi_i), G_i = grad(rho_i) */
    for (int i = 0; i < N; ++i) {
        oracle_gradient(P, f->psi + (size_t)i * ns, f->tmp);
        for (int d = 0; d < 3; ++d)
            for (long s = 0; s < ns; ++s)
                f->F[((size_t)i * 3 + d) * ns + s] =
                    -f->rt[(size_t)i * ns + s] * f->tmp[(size_t)d * ns + s];
        oracle_gradient(P, f->rho + (size_t)i * ns, f->G + (size_t)i * 3 * ns);
    }
    /* common velocity u = (j + F/2) / rho */
    for (long s = 0; s < ns; ++s)
        for (int d = 0; d < 3; ++d) {
            double Fs = 0.0;
            for (int i = 0; i < N; ++i) Fs += f->F[((size_t)i * 3 + d) * ns + s];
            f->u[(size_t)d * ns + s] = (f->j[(size_t)d * ns + s] + 0.5 * Fs) / f->rhot[s];
        }
    return status;
}

/* ---- initial populations: g = geq(rho_i, u = 0) ------------------------- */
void oracle_init(const oracle_params *P, const double *rho, double *g) {
    int e[OR_MAXQ][3];
    double w[OR_MAXQ];
    int Q = lattice_set(P->lattice, e, w);
    long ns = nsites(P);
    double u0[3] = {0.0, 0.0, 0.0};
    for (long s = 0; s < ns; ++s)
        for (int i = 0; i < P->N; ++i)
            oracle_equilibrium(P->lattice, rho[(size_t)i * ns + s], P->rho_c, u0,
                               g + ((size_t)s * P->N + i) * Q);
}

/* ---- one step: collide (Eq. 1a) and push-stream -------------------------- */
int oracle_step(const oracle_params *P, const double *g, double *gnew) {
    int e[OR_MAXQ][3];
    double w[OR_MAXQ];
    int Q = lattice_set(P->lattice, e, w);
    const int N = P->N;
    long ns = nsites(P);
    fields f;
    fields_alloc(P, &f);
    int status = compute_fields(P, g, &f);
    double tau = P->tau;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < ns; ++s) {
        double u[3], geq[OR_MAXQ], Fa[OR_MAXQ];
        for (int d = 0; d < 3; ++d) u[d] = f.u[(size_t)d * ns + s];
        for (int i = 0; i < N; ++i) {
            double Fi[3], Gi[3];
            for (int d = 0; d < 3; ++d) {
                Fi[d] = f.F[((size_t)i * 3 + d) * ns + s];
                Gi[d] = f.G[((size_t)i * 3 + d) * ns + s];
            }
            oracle_equilibrium(P->lattice, f.rho[(size_t)i * ns + s], P->rho_c, u, geq);
            oracle_forcing(P->lattice, Fi, Gi, u, Fa);
            for (int a = 0; a < Q; ++a) {
                double ga = g[((size_t)s * N + i) * Q + a];
                double gs = ga - (ga - geq[a]) / tau + (1.0 - 1.0 / (2.0 * tau)) * Fa[a];
                long t = neighbour(P, s, e[a]);
                gnew[((size_t)t * N + i) * Q + a] = gs;
            }
        }
    }
    fields_free(&f);
    return status;
}

/* n steps, ping-ponging between g and a scratch buffer; result left in g. */
int oracle_run(const oracle_params *P, double *g, long nsteps) {
    size_t n = (size_t)nsites(P) * P->N * (P->lattice == 0 ? 9 : 19);
    double *tmp = malloc(n * sizeof(double));
    int status = 0;
    for (long k = 0; k < nsteps; ++k) {
        status |= oracle_step(P, g, tmp);
        memcpy(g, tmp, n * sizeof(double));
    }
    free(tmp);
    return status;
}

/* Macroscopic readout: rho_i [N][sites], u [3][sites] (force-corrected),
 * optional psi [N][sites], lnf [N][sites], F [N][3][sites]. */
int oracle_fields(const oracle_params *P, const double *g, double *rho, double *u,
                  double *psi, double *lnf, double *F) {
    long ns = nsites(P);
    fields f;
    fields_alloc(P, &f);
    int status = compute_fields(P, g, &f);
    if (rho) memcpy(rho, f.rho, (size_t)P->N * ns * sizeof(double));
    if (u) memcpy(u, f.u, (size_t)3 * ns * sizeof(double));
    if (psi) memcpy(psi, f.psi, (size_t)P->N * ns * sizeof(double));
    if (lnf) memcpy(lnf, f.lnf, (size_t)P->N * ns * sizeof(double));
    if (F) memcpy(F, f.F, (size_t)P->N * 3 * ns * sizeof(double));
    fields_free(&f);
    return status;
}

/* ---- diagnostics of a state (mass, momentum, residual, status) ---------- */
/* For the state g (and, for the residual, the state g_prev taken K steps
 * earlier), summed site by site in site order:
 *   mass[i]     = sum_r rho_i(r)                       (per-component mass;
 *                 conserved by Eq. (1a)-(1c): sum_a F_a = 0 and
 *                 sum_a (geq - g) = 0, and streaming only moves populations);
 *   mom_pop[d]  = sum_r sum_i sum_a e_a g              (the populations' own
 *                 momentum);
 *   mom_u[d]    = sum_r (sum_i sum_a e_a g + F_d / 2)  (= sum_r rho u, the
 *                 force-corrected momentum of the common velocity u);
 *   residual    = max_i sum_r |rho_i(t) - rho_i(t-K)| / (K sum_r rho_i(t)),
 *                 0 when g_prev is NULL or K <= 0;
 * and returns the status bits of the state's fields (1 non-finite ln f_i,
 * 2 outside the EOS domain, 4 some rt_i <= 0).                              */
int oracle_diagnostics(const oracle_params *P, const double *g, const double *g_prev, long K,
                       double *mass, double *mom_pop, double *mom_u, double *residual) {
    const int N = P->N;
    long ns = nsites(P);
    fields f;
    fields_alloc(P, &f);
    int status = compute_fields(P, g, &f);
    for (int d = 0; d < 3; ++d) {
        mom_pop[d] = 0.0;
        mom_u[d] = 0.0;
    }
    for (int i = 0; i < N; ++i) mass[i] = 0.0;
    for (long s = 0; s < ns; ++s) {
        for (int i = 0; i < N; ++i) mass[i] += f.rho[(size_t)i * ns + s];
        for (int d = 0; d < 3; ++d) {
            double Fs = 0.0;
            for (int i = 0; i < N; ++i) Fs += f.F[((size_t)i * 3 + d) * ns + s];
            mom_pop[d] += f.j[(size_t)d * ns + s];
            mom_u[d] += f.j[(size_t)d * ns + s] + 0.5 * Fs;
        }
    }
    *residual = 0.0;
    if (g_prev && K > 0) {
        fields fp;
        fields_alloc(P, &fp);
        compute_fields(P, g_prev, &fp);
        for (int i = 0; i < N; ++i) {
            double num = 0.0;
            for (long s = 0; s < ns; ++s)
                num += fabs(f.rho[(size_t)i * ns + s] - fp.rho[(size_t)i * ns + s]);
            double r = num / ((double)K * mass[i]);
            if (r > *residual) *residual = r;
        }
        fields_free(&fp);
    }
    fields_free(&f);
    return status;
}

/* Thread count of the OpenMP loops (for timing the oracle at 1 thread and
 * at all cores); returns the count in effect before the call. */
int oracle_set_threads(int n) {
    int old = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return old;
}
