/* A plain C user of the library (no Python): the Sec. 4.1 sine wave,
   rho = 1 + 0.2 sin(pi x), U = 1, p = 1 on [0, 2], periodic, 6th-order linear
   scheme, one period (t = 2).  The exact solution returns to the initial cell
   averages.  Also exercises the error path.  Exit status 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "gks.h"

int main(void)
{
    const int n = 80;
    const double pi = 3.14159265358979323846, g = 1.4, dx = 2.0 / n;
    double *W = malloc(sizeof(double) * 3 * n), *Wx = malloc(sizeof(double) * 3 * n);
    double *Wo = malloc(sizeof(double) * 3 * n), *Wxo = malloc(sizeof(double) * 3 * n);
    for (int i = 0; i < n; ++i) {
        const double a = i * dx, b = a + dx;
        const double rho = 1.0 + 0.2 * (cos(pi * a) - cos(pi * b)) / (pi * dx); /* exact average */
        const double drho = 0.2 * (sin(pi * b) - sin(pi * a)) / dx;             /* exact averaged slope */
        W[3 * i] = rho; W[3 * i + 1] = rho; W[3 * i + 2] = 1.0 / (g - 1.0) + 0.5 * rho;
        Wx[3 * i] = drho; Wx[3 * i + 1] = drho; Wx[3 * i + 2] = 0.5 * drho;
    }
    gks_problem p = {1, n, 1, 0.0, 2.0, 0.0, 1.0, g, 0.0, 0.3, 0.0, 2.0, 6, GKS_RECON_LINEAR, {0, 0, 0, 0}};
    const double* W0[1] = {W};
    const double* X0[1] = {Wx};
    gks_handle* h = NULL;

    /* error path: order 7 is rejected without a handle */
    p.order = 7;
    if (gks_init(&p, 1, GKS_PREC_FP64, W0, X0, NULL, NULL, &h) != GKS_EINVAL || h) {
        fprintf(stderr, "bad order accepted\n");
        return 1;
    }
    printf("rejected: %s\n", gks_last_error(NULL));
    p.order = 6;

    int st = gks_init(&p, 1, GKS_PREC_FP64, W0, X0, NULL, NULL, &h);
    if (st != GKS_OK) {
        fprintf(stderr, "gks_init: %s\n", gks_last_error(NULL));
        return 1;
    }
    int active = 1;
    while (active > 0) {
        st = gks_step(h, 1000, &active);
        if (st != GKS_OK) {
            fprintf(stderr, "gks_step: %s\n", gks_last_error(h));
            return 1;
        }
    }
    double t = 0.0;
    int64_t steps = 0;
    if (gks_state(h, 0, Wo, Wxo, NULL, &t, &steps) != GKS_OK) return 1;
    int status = -9;
    gks_problem_status(h, 0, &status);
    double l1 = 0.0, m0 = 0.0, m1 = 0.0;
    for (int i = 0; i < n; ++i) {
        l1 += fabs(Wo[3 * i] - W[3 * i]) / n;
        m0 += W[3 * i];
        m1 += Wo[3 * i];
    }
    gks_free(h);
    printf("t = %.15g after %lld steps, status %d, L1(rho) = %.3e, mass drift %.2e\n", t, (long long)steps, status, l1,
           fabs(m1 - m0) / m0);
    /* the 6th-order scheme at 80 cells: L1 ~ 1e-9 (Sec. 4.1); mass conserved to round-off */
    const int ok = t == 2.0 && status == 1 && l1 < 1e-8 && fabs(m1 - m0) / m0 < 1e-13;
    free(W); free(Wx); free(Wo); free(Wxo);
    return ok ? 0 : 1;
}
