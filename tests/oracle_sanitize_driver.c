/* Test driver (test infrastructure only): runs the C oracle, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer, on a field read from
 * stdin, and prints the densities after the requested steps.
 *
 * stdin: lattice N nx ny nz eos tau RT d1 d2 steps, then b[N], M[N],
 * sqk[N], aij[N*N] (row-major), then rho[N*sites] (component-major).
 * stdout: rho after the steps, one value per line; exit status = the
 * oracle's status bits (0 = clean). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/lbm_oracle.c"

static double rd(void) {
    double v;
    if (scanf("%lf", &v) != 1) exit(90);
    return v;
}

int main(void) {
    oracle_params P;
    memset(&P, 0, sizeof(P));
    P.lattice = (int)rd();
    P.N = (int)rd();
    P.nx = (int)rd();
    P.ny = (int)rd();
    P.nz = (int)rd();
    P.eos = (int)rd();
    P.tau = rd();
    P.RT = rd();
    P.d1 = rd();
    P.d2 = rd();
    long steps = (long)rd();
    if (P.N < 1 || P.N > OR_MAXC) return 91;
    for (int i = 0; i < P.N; ++i) P.b[i] = rd();
    for (int i = 0; i < P.N; ++i) P.M[i] = rd();
    for (int i = 0; i < P.N; ++i) P.sqk[i] = rd();
    for (int i = 0; i < P.N; ++i)
        for (int j = 0; j < P.N; ++j) P.aij[i * OR_MAXC + j] = rd();
    const long ns = (long)P.nx * P.ny * P.nz;
    const int Q = P.lattice == 0 ? 9 : 19;
    double *rho = malloc(sizeof(double) * P.N * ns);
    double *g = malloc(sizeof(double) * P.N * ns * Q);
    double *out = malloc(sizeof(double) * P.N * ns);
    for (long k = 0; k < P.N * ns; ++k) rho[k] = rd();
    oracle_init(&P, rho, g);
    int st = oracle_run(&P, g, steps);
    oracle_fields(&P, g, out, NULL, NULL, NULL, NULL);
    for (long k = 0; k < P.N * ns; ++k) printf("%.17g\n", out[k]);
    free(rho);
    free(g);
    free(out);
    return st;
}
