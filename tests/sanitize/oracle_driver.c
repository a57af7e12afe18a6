/* Sanitizer driver of the oracle (direct_sum.c).  Reads one problem from
 * stdin:
 *   npatch x0 y0 h0 aspect ratio
 *   npatch lines: level n ox oy
 *   per patch: n*n sigma, n*n dsdx, n*n dsdy (row-major)
 *   ntarget, then ntarget lines: patch i j
 * and prints fx fy phi per target, then the generalized convolutions of one
 * fixed pair of sequences in the three modes (m = 2) and the cell integrals
 * of two cells. */
#include <stdio.h>
#include <stdlib.h>

int oracle_forces(int npatch, const int* level, const int* n, const int* ox, const int* oy,
                  double x0, double y0, double h0, double aspect, int ratio,
                  const double* const* sigma, const double* const* dsdx,
                  const double* const* dsdy, int ntarget, const int* tpatch, const int* ti,
                  const int* tj, double* fx, double* fy, int nthreads);
int oracle_potential(int npatch, const int* level, const int* n, const int* ox, const int* oy,
                     double x0, double y0, double h0, double aspect, int ratio,
                     const double* const* sigma, const double* const* dsdx,
                     const double* const* dsdy, int ntarget, const int* tpatch, const int* ti,
                     const int* tj, double* phi, int nthreads);
void oracle_genconv1d(int mode, int m, const double* b, int nb, const double* c, int nc,
                      double* a, int na);
void oracle_cell_integrals(double ua, double ub, double va, double vb, double out[6]);
void oracle_cell_potential(double ua, double ub, double va, double vb, double out[3]);

static double* read_field(int count)
{
    double* a = malloc(sizeof(double) * (size_t)count);
    for (int k = 0; k < count; ++k)
        if (scanf("%lf", &a[k]) != 1) exit(2);
    return a;
}

int main(void)
{
    int np, ratio;
    double x0, y0, h0, aspect;
    if (scanf("%d %lf %lf %lf %lf %d", &np, &x0, &y0, &h0, &aspect, &ratio) != 6 || np < 1 || np > 64)
        return 2;
    int *level = malloc(sizeof(int) * np), *n = malloc(sizeof(int) * np);
    int *ox = malloc(sizeof(int) * np), *oy = malloc(sizeof(int) * np);
    for (int k = 0; k < np; ++k)
        if (scanf("%d %d %d %d", &level[k], &n[k], &ox[k], &oy[k]) != 4) return 2;
    double **s = malloc(sizeof(double*) * np), **dx = malloc(sizeof(double*) * np);
    double** dy = malloc(sizeof(double*) * np);
    for (int k = 0; k < np; ++k) {
        s[k] = read_field(n[k] * n[k]);
        dx[k] = read_field(n[k] * n[k]);
        dy[k] = read_field(n[k] * n[k]);
    }
    int nt;
    if (scanf("%d", &nt) != 1 || nt < 1) return 2;
    int *tp = malloc(sizeof(int) * nt), *ti = malloc(sizeof(int) * nt), *tj = malloc(sizeof(int) * nt);
    for (int k = 0; k < nt; ++k)
        if (scanf("%d %d %d", &tp[k], &ti[k], &tj[k]) != 3) return 2;
    double *fx = malloc(sizeof(double) * nt), *fy = malloc(sizeof(double) * nt);
    double* phi = malloc(sizeof(double) * nt);
    if (oracle_forces(np, level, n, ox, oy, x0, y0, h0, aspect, ratio, (const double* const*)s,
                      (const double* const*)dx, (const double* const*)dy, nt, tp, ti, tj, fx, fy, 4))
        return 3;
    if (oracle_potential(np, level, n, ox, oy, x0, y0, h0, aspect, ratio, (const double* const*)s,
                         (const double* const*)dx, (const double* const*)dy, nt, tp, ti, tj, phi, 4))
        return 3;
    for (int k = 0; k < nt; ++k) printf("%.17g %.17g %.17g\n", fx[k], fy[k], phi[k]);
    const double b[8] = {1, 2, 3, 4, 5, 6, 7, 8}, c[4] = {1, -1, 2, -2};
    double a[12];
    for (int mode = 1; mode <= 3; ++mode) {
        oracle_genconv1d(mode, 2, b, 8, c, 4, a, 12);
        for (int k = 0; k < 12; ++k) printf("%.17g%c", a[k], k == 11 ? '\n' : ' ');
    }
    double ci[6], cp[3];
    oracle_cell_integrals(0.0, 1.0, 1.0, 2.0, ci);
    oracle_cell_potential(-3.0, -2.0, -0.5, 0.5, cp);
    printf("%.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g\n", ci[0], ci[1], ci[2], ci[3],
           ci[4], ci[5], cp[0], cp[1], cp[2]);
    for (int k = 0; k < np; ++k) {
        free(s[k]);
        free(dx[k]);
        free(dy[k]);
    }
    free(s); free(dx); free(dy); free(level); free(n); free(ox); free(oy);
    free(tp); free(ti); free(tj); free(fx); free(fy); free(phi);
    return 0;
}
