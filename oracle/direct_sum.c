/*
 * Thin-disk direct-sum force oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this file's library.  It shares no code with the HIP path.
 *
 * What it computes (Section 2.1 of the paper, "Approximation of second order
 * accuracy"): the mid-plane force of an infinitesimally thin disk,
 *
 *     F_x(t) = -d/dx Phi = sum over every active source cell c of
 *              integral_c (xbar - x_t) / rho^3 * sigma(xbar, ybar) dxbar dybar,
 *
 * with G = 1 and sigma reconstructed linearly in each cell about the SOURCE
 * cell centre (eq. eqnSigma):  sigma = s_c + dx_c (xbar - x_c) + dy_c (ybar - y_c).
 * The cell integrals are written as four-corner differences of closed-form
 * antiderivatives (eqs. eqnCalK, eqnbnot0, eqnbeq0) and summed directly,
 * O(cells^2): no FFT, no convolution structure, no blocking.
 *
 * Readings of the paper that this code takes (each justified in the design
 * notes):
 *   - expansion about the source-cell centre (eq. eqnSigma), not the target
 *     centre the following display shows;
 *   - slope antiderivatives G_xx(u,v) = v ln(u + r) and G_xy(u,v) = -r, each
 *     with the source-centre moment shift; the printed K^{x,x}, K^{x,y} do
 *     not differentiate back to the integrands they stand for;
 *   - sgn(0) = 0 in the u = 0 branch of K^{x,0} and epsilon = 0, with the
 *     cancellation-free rewrites below instead of the epsilon guard
 *     (eq. eqnCalKepsilon);
 *   - y-forces by exchanging the roles of x and y;
 *   - a level-l cell is active iff no level-(l+1) patch covers it; covered
 *     targets get force 0.
 *
 * The potential itself (eq. eqnPhixy0, Green's function -1/rho, G = 1) is
 * summed the same way:
 *
 *     Phi(t) = - sum over every active source cell c of
 *              integral_c sigma(xbar, ybar) / rho dxbar dybar,
 *
 * with the cell integrals of 1/rho, (xbar - x_c)/rho and (ybar - y_c)/rho
 * written as four-corner differences of their antiderivatives
 *     a(u, v)  = u ln(v + r) + v ln(u + r)        (d^2 a / du dv = 1 / r)
 *     bx(u, v) = v r / 2 + (u^2 / 2) ln(v + r)    (d^2 bx / du dv = u / r)
 *     by(u, v) = u r / 2 + (v^2 / 2) ln(u + r)    (d^2 by / du dv = v / r)
 * each term taken as 0 where its factor u, v (or u^2, v^2) is 0, its limit.
 *
 * Arithmetic: every antiderivative in x87 long double; per-target sums in
 * long double with Neumaier compensation; results rounded to double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;

/* The five antiderivatives at one corner (u, v) = (corner - target).
 *   g0   : d^2/dudv g0   = u / r^3   (K^{x,0}, eq. eqnCalK)
 *   g0s  : d^2/dudv g0s  = v / r^3   (x <-> y exchange of g0)
 *   gxx  : d^2/dudv gxx  = u^2 / r^3
 *   gyy  : d^2/dudv gyy  = v^2 / r^3 (x <-> y exchange of gxx)
 *   gxy  : d^2/dudv gxy  = u v / r^3 (symmetric in the exchange)          */
typedef struct { ld g0, g0s, gxx, gyy, gxy; } corner_t;

/* ln(b + sqrt(a^2 + b^2)) for a != 0, written without cancellation when
 * b < 0:  b + r = a^2 / (r - b).                                          */
static ld log_b_plus_r(ld a, ld b, ld r)
{
    if (b >= 0) return logl(b + r);
    return logl(a * a) - logl(r - b);
}

static corner_t corner_eval(ld u, ld v)
{
    corner_t c;
    ld r = sqrtl(u * u + v * v);
    /* g0 = -ln(v + r) for u != 0; for u = 0, -sgn(v) ln|v| (eq. eqnbeq0),
     * with sgn(0) = 0 so the value at the origin is 0.                    */
    if (u != 0) c.g0 = -log_b_plus_r(u, v, r);
    else if (v > 0) c.g0 = -logl(v);
    else if (v < 0) c.g0 = logl(-v);
    else c.g0 = 0;
    if (v != 0) c.g0s = -log_b_plus_r(v, u, r);
    else if (u > 0) c.g0s = -logl(u);
    else if (u < 0) c.g0s = logl(-u);
    else c.g0s = 0;
    /* gxx = v ln(u + r); zero on v = 0, where the integrand of the outer
     * u-integral, v/r, vanishes.                                          */
    c.gxx = (v != 0) ? v * log_b_plus_r(v, u, r) : 0;
    c.gyy = (u != 0) ? u * log_b_plus_r(u, v, r) : 0;
    c.gxy = -r;
    return c;
}

/* Cell integrals of one source cell [ua,ub] x [va,vb] (coordinates relative
 * to the target) with centre (uc, vc):
 *   out[0] I0  = int u / r^3                 out[3] J0  = int v / r^3
 *   out[1] Ixx = int (u - uc) u / r^3        out[4] Jyy = int (v - vc) v / r^3
 *   out[2] Ixy = int (v - vc) u / r^3        out[5] Jyx = int (u - uc) v / r^3
 * Each is the corner difference  F(ub,vb) - F(ua,vb) - F(ub,va) + F(ua,va).  */
static void cell_integrals_ld(ld ua, ld ub, ld va, ld vb, ld out[6])
{
    corner_t bb = corner_eval(ub, vb), ab = corner_eval(ua, vb);
    corner_t ba = corner_eval(ub, va), aa = corner_eval(ua, va);
    ld uc = (ua + ub) / 2, vc = (va + vb) / 2;
#define CORNER_DIFF(f) ((bb.f - ab.f) - (ba.f - aa.f))
    ld i0 = CORNER_DIFF(g0);
    ld j0 = CORNER_DIFF(g0s);
    out[0] = i0;
    out[1] = CORNER_DIFF(gxx) - uc * i0;
    out[2] = CORNER_DIFF(gxy) - vc * i0;
    out[3] = j0;
    out[4] = CORNER_DIFF(gyy) - vc * j0;
    out[5] = CORNER_DIFF(gxy) - uc * j0;
#undef CORNER_DIFF
}

/* Exported for the oracle's own pins. */
void oracle_cell_integrals(double ua, double ub, double va, double vb, double out[6])
{
    ld o[6];
    cell_integrals_ld(ua, ub, va, vb, o);
    for (int k = 0; k < 6; ++k) out[k] = (double)o[k];
}

/* Antiderivatives of the potential integrands at one corner (u, v). */
typedef struct { ld a, bx, by; } pcorner_t;

static pcorner_t pcorner_eval(ld u, ld v)
{
    pcorner_t c;
    ld r = sqrtl(u * u + v * v);
    ld lv = (u != 0) ? log_b_plus_r(u, v, r) : 0;   /* ln(v + r), used only times u */
    ld lu = (v != 0) ? log_b_plus_r(v, u, r) : 0;   /* ln(u + r), used only times v */
    c.a = u * lv + v * lu;
    c.bx = v * r / 2 + u * u / 2 * lv;
    c.by = u * r / 2 + v * v / 2 * lu;
    return c;
}

/* Potential cell integrals of [ua,ub] x [va,vb] relative to the target:
 *   out[0] P0 = int 1 / r,  out[1] Px = int (u - uc) / r,
 *   out[2] Py = int (v - vc) / r.                                         */
static void cell_potential_ld(ld ua, ld ub, ld va, ld vb, ld out[3])
{
    pcorner_t bb = pcorner_eval(ub, vb), ab = pcorner_eval(ua, vb);
    pcorner_t ba = pcorner_eval(ub, va), aa = pcorner_eval(ua, va);
    ld uc = (ua + ub) / 2, vc = (va + vb) / 2;
#define CORNER_DIFF(f) ((bb.f - ab.f) - (ba.f - aa.f))
    ld p0 = CORNER_DIFF(a);
    out[0] = p0;
    out[1] = CORNER_DIFF(bx) - uc * p0;
    out[2] = CORNER_DIFF(by) - vc * p0;
#undef CORNER_DIFF
}

void oracle_cell_potential(double ua, double ub, double va, double vb, double out[3])
{
    ld o[3];
    cell_potential_ld(ua, ub, va, vb, o);
    for (int k = 0; k < 3; ++k) out[k] = (double)o[k];
}

/* Neumaier-compensated long-double accumulator. */
typedef struct { ld s, c; } acc_t;
static void acc_add(acc_t* a, ld x)
{
    ld t = a->s + x;
    if (fabsl(a->s) >= fabsl(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/* Patch p covers level-l cell (i, j) of patch q iff p is on level l+1 and
 * the cell's footprint, scaled by the ratio, lies inside p.  All offsets are
 * integers in the patch's own cell units from the level-0 origin.          */
static int cell_covered(int npatch, const int* level, const int* n, const int* ox,
                        const int* oy, int ratio, int q, int i, int j)
{
    for (int p = 0; p < npatch; ++p) {
        if (level[p] != level[q] + 1) continue;
        long gx0 = (long)ratio * (ox[q] + i), gy0 = (long)ratio * (oy[q] + j);
        long gx1 = gx0 + ratio, gy1 = gy0 + ratio;
        if (gx0 >= ox[p] && gx1 <= (long)ox[p] + n[p] && gy0 >= oy[p] &&
            gy1 <= (long)oy[p] + n[p])
            return 1;
    }
    return 0;
}

/*
 * Direct sums at a list of targets: forces (what = 0: out0 = fx, out1 = fy)
 * or the potential (what = 1: out0 = phi, out1 unused, may be NULL).
 *   npatch patches; patch p is on level level[p], has n[p] x n[p] cells of
 *   width h = h0 / ratio^level[p] and height aspect * h, lower-left corner
 *   at (x0 + ox[p] h, y0 + oy[p] aspect h).
 *   sigma[p], dsdx[p], dsdy[p]: n[p]*n[p] doubles, row-major [j][i] (x
 *   fastest); dsdx / dsdy arrays may be NULL pointers (slope 0).
 *   Targets: (tpatch[k], ti[k], tj[k]) cell centres.  fx[k], fy[k] receive
 *   the force; a covered target receives 0.
 * Returns 0, or -1 on a malformed target index.
 */
static int direct_sum(int what, int npatch, const int* level, const int* n, const int* ox,
                      const int* oy, double x0, double y0, double h0, double aspect, int ratio,
                      const double* const* sigma, const double* const* dsdx,
                      const double* const* dsdy, int ntarget, const int* tpatch,
                      const int* ti, const int* tj, double* fx, double* fy, int nthreads)
{
    for (int k = 0; k < ntarget; ++k) {
        int q = tpatch[k];
        if (q < 0 || q >= npatch || ti[k] < 0 || ti[k] >= n[q] || tj[k] < 0 || tj[k] >= n[q])
            return -1;
    }
    /* Physical geometry of every patch. */
    ld* hp = (ld*)malloc(sizeof(ld) * (size_t)npatch);
    ld* xl = (ld*)malloc(sizeof(ld) * (size_t)npatch);
    ld* yl = (ld*)malloc(sizeof(ld) * (size_t)npatch);
    ld* hq = (ld*)malloc(sizeof(ld) * (size_t)npatch);
    for (int p = 0; p < npatch; ++p) {
        ld h = h0;
        for (int l = 0; l < level[p]; ++l) h /= ratio;
        hp[p] = h;
        hq[p] = h * (ld)aspect;
        xl[p] = (ld)x0 + ox[p] * h;
        yl[p] = (ld)y0 + oy[p] * hq[p];
    }
    /* Active flags of every source cell. */
    size_t total = 0;
    for (int p = 0; p < npatch; ++p) total += (size_t)n[p] * n[p];
    unsigned char* active = (unsigned char*)malloc(total ? total : 1);
    size_t* base = (size_t*)malloc(sizeof(size_t) * (size_t)npatch);
    {
        size_t b = 0;
        for (int p = 0; p < npatch; ++p) {
            base[p] = b;
            for (int j = 0; j < n[p]; ++j)
                for (int i = 0; i < n[p]; ++i)
                    active[b + (size_t)j * n[p] + i] =
                        !cell_covered(npatch, level, n, ox, oy, ratio, p, i, j);
            b += (size_t)n[p] * n[p];
        }
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int k = 0; k < ntarget; ++k) {
        int q = tpatch[k];
        if (!active[base[q] + (size_t)tj[k] * n[q] + ti[k]]) {
            fx[k] = 0;
            if (fy) fy[k] = 0;
            continue;
        }
        ld xt = xl[q] + (ti[k] + (ld)0.5) * hp[q];
        ld yt = yl[q] + (tj[k] + (ld)0.5) * hq[q];
        acc_t ax = {0, 0}, ay = {0, 0};
        for (int p = 0; p < npatch; ++p) {
            ld h = hp[p], hy = hq[p];
            const double* s = sigma[p];
            const double* sx = dsdx ? dsdx[p] : NULL;
            const double* sy = dsdy ? dsdy[p] : NULL;
            for (int j = 0; j < n[p]; ++j) {
                ld va = yl[p] + j * hy - yt, vb = yl[p] + (j + 1) * hy - yt;
                for (int i = 0; i < n[p]; ++i) {
                    size_t idx = (size_t)j * n[p] + i;
                    if (!active[base[p] + idx]) continue;
                    ld ua = xl[p] + i * h - xt, ub = xl[p] + (i + 1) * h - xt;
                    ld sg = s[idx];
                    ld gx = sx ? sx[idx] : 0, gy = sy ? sy[idx] : 0;
                    if (what == 0) {
                        ld c[6];
                        cell_integrals_ld(ua, ub, va, vb, c);
                        acc_add(&ax, sg * c[0]);
                        acc_add(&ax, gx * c[1]);
                        acc_add(&ax, gy * c[2]);
                        acc_add(&ay, sg * c[3]);
                        acc_add(&ay, gy * c[4]);
                        acc_add(&ay, gx * c[5]);
                    } else {
                        /* Phi = - sum sigma / rho: the Green's function -1/rho */
                        ld c[3];
                        cell_potential_ld(ua, ub, va, vb, c);
                        acc_add(&ax, -sg * c[0]);
                        acc_add(&ax, -gx * c[1]);
                        acc_add(&ax, -gy * c[2]);
                    }
                }
            }
        }
        fx[k] = (double)(ax.s + ax.c);
        if (fy) fy[k] = (double)(ay.s + ay.c);
    }
    free(hp);
    free(hq);
    free(xl);
    free(yl);
    free(active);
    free(base);
    return 0;
}

int oracle_forces(int npatch, const int* level, const int* n, const int* ox, const int* oy,
                  double x0, double y0, double h0, double aspect, int ratio,
                  const double* const* sigma, const double* const* dsdx,
                  const double* const* dsdy, int ntarget, const int* tpatch,
                  const int* ti, const int* tj, double* fx, double* fy, int nthreads)
{
    return direct_sum(0, npatch, level, n, ox, oy, x0, y0, h0, aspect, ratio, sigma, dsdx, dsdy,
                      ntarget, tpatch, ti, tj, fx, fy, nthreads);
}

int oracle_potential(int npatch, const int* level, const int* n, const int* ox,
                     const int* oy, double x0, double y0, double h0, double aspect, int ratio,
                     const double* const* sigma, const double* const* dsdx,
                     const double* const* dsdy, int ntarget, const int* tpatch,
                     const int* ti, const int* tj, double* phi, int nthreads)
{
    return direct_sum(1, npatch, level, n, ox, oy, x0, y0, h0, aspect, ratio, sigma, dsdx, dsdy,
                      ntarget, tpatch, ti, tj, phi, NULL, nthreads);
}

/*
 * The generalized convolutions of Section 2.2 written out as plain sums over
 * finite sequences (Cases 1', 2', 3'), 1-D:
 *   mode 1: a_n = sum_k b_{n-k} c_k            (ordinary convolution)
 *   mode 2: a_n = sum_k b_{m n - k} c_k        (eq. eqnbmnn)
 *   mode 3: a_n = sum_k b_{n - m k} c_k        (eq. eqnbnmn)
 * b has nb entries (indices 0..nb-1, zero elsewhere), c has nc entries.
 * a receives na entries, indices 0..na-1.                                   */
void oracle_genconv1d(int mode, int m, const double* b, int nb, const double* c, int nc,
                      double* a, int na)
{
    for (int nn = 0; nn < na; ++nn) {
        ld s = 0;
        for (int k = 0; k < nc; ++k) {
            long idx;
            if (mode == 1) idx = (long)nn - k;
            else if (mode == 2) idx = (long)m * nn - k;
            else idx = (long)nn - (long)m * k;
            if (idx >= 0 && idx < nb) s += (ld)b[idx] * c[k];
        }
        a[nn] = (double)s;
    }
}
