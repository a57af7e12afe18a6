// Device passes of the thin-disk force solver (gfx950).
//
// Kernel tables: the cell integrals of Section 2.1 for every lattice offset
// and polyphase phase, built in FP64 with cancellation-free forms.
// Convolution: zero-padded 2-D FFTs along rows (real <-> half-complex,
// written / read transposed so that every spectral column is contiguous) and
// along columns (fused with the kernel-spectrum products), Section 2.2.
#include <algorithm>
#include <mutex>

#include "td_fft.hpp"
#include "td_jobs.h"
#include "td_launch.h"

namespace td {

// ---------------------------------------------------------------------------
// Kernel tables (FP64)
// ---------------------------------------------------------------------------

// asinh(q/|w|) - asinh(p/|w|) at fixed w != 0 (p, q, w exact lattice
// values).  For p, q of one sign it is asinh(sinh(Q - P)) with
//   sinh(Q - P) = (q - p)(q + p) / w^2 / (a sqrt(1+b^2) + b sqrt(1+a^2)),
// a = |q|/|w|, b = |p|/|w|; forming (q - p)(q + p) from the exact values
// (rather than subtracting the rounded quotients) keeps the difference
// accurate to a few ulp however close p and q are relative to w.
__device__ double asinh_pair(double w, double p, double q)
{
    if (p == q) return 0.0;
    const double aw = fabs(w);
    if ((p >= 0 && q >= 0) || (p <= 0 && q <= 0)) {
        const double s = (p < 0 || q < 0) ? -1.0 : 1.0;
        const double a = fabs(q) / aw, b = fabs(p) / aw;
        const double num = (fabs(q) - fabs(p)) * (fabs(q) + fabs(p)) / (aw * aw);
        return s * asinh(num / (a * sqrt(1.0 + b * b) + b * sqrt(1.0 + a * a)));
    }
    return asinh(q / aw) - asinh(p / aw);
}

// Difference over the pair (p, q) at fixed w of the antiderivative branch:
//   w != 0: asinh(q/|w|) - asinh(p/|w|)  (= ln(q + r) - ln(p + r) at fixed w)
//   w == 0: sgn(q) ln|q| - sgn(p) ln|p| with sgn(0) = 0 (eq. eqnbeq0).
__device__ double branch_diff(double w, double p, double q)
{
    if (w != 0.0) return asinh_pair(w, p, q);
    // one sign: ln(q/p) for p, q > 0 and ln(p/q) for p, q < 0, as log1p of
    // an exact difference
    if (p > 0 && q > 0) return log1p((q - p) / p);
    if (p < 0 && q < 0) return log1p((p - q) / q);
    double lq = (q == 0) ? 0.0 : (q > 0 ? log(q) : -log(-q));
    double lp = (p == 0) ? 0.0 : (p > 0 ? log(p) : -log(-p));
    return lq - lp;
}

// Six cell integrals of [ua,ub] x [va,vb] (target at the origin):
// I0 = int u/r^3, Ixx = int (u-uc)u/r^3, Ixy = int (v-vc)u/r^3,
// J0 = int v/r^3, Jyy = int (v-vc)v/r^3, Jyx = int (u-uc)v/r^3.
// Corner differences are regrouped so that no step cancels more than the
// integral itself: A(u) = ln-difference over v at fixed u, B(v) over u at
// fixed v, and the r-difference in product form.
__device__ void cell_integrals(double ua, double ub, double va, double vb, double* out)
{
    double Aa = branch_diff(ua, va, vb), Ab = branch_diff(ub, va, vb);
    double Ba = branch_diff(va, ua, ub), Bb = branch_diff(vb, ua, ub);
    double i0 = Aa - Ab;
    double j0 = Ba - Bb;
    double gxx = (vb != 0 ? vb * Bb : 0.0) - (va != 0 ? va * Ba : 0.0);
    double gyy = (ub != 0 ? ub * Ab : 0.0) - (ua != 0 ? ua * Aa : 0.0);
    double raa = sqrt(ua * ua + va * va), rab = sqrt(ua * ua + vb * vb);
    double rba = sqrt(ub * ub + va * va), rbb = sqrt(ub * ub + vb * vb);
    // [r] = r(ub,vb) - r(ua,vb) - r(ub,va) + r(ua,va)
    double sa = rba + raa, sb = rbb + rab;
    double rr = (ub - ua) * (ub + ua) * (va - vb) * (va + vb) *
                (1.0 / (rba + rbb) + 1.0 / (raa + rab)) / (sa * sb);
    double uc = 0.5 * (ua + ub), vc = 0.5 * (va + vb);
    out[0] = i0;
    out[1] = gxx - uc * i0;
    out[2] = -rr - vc * i0;
    out[3] = j0;
    out[4] = gyy - vc * j0;
    out[5] = -rr - uc * j0;
}

// Potential cell integrals of [ua,ub] x [va,vb] (target at the origin):
// P0 = int 1/r, Px = int (u-uc)/r, Py = int (v-vc)/r, for the Green's
// function -1/rho of eq. eqnPhixy0 (the sign is applied with the scale).
// Antiderivatives u ln(v+r) + v ln(u+r), v r/2 + (u^2/2) ln(v+r) and their
// exchange, regrouped like the force integrals: the ln-differences at fixed
// u (A) and fixed v (B), and the r-differences at fixed v or u in product
// form.
__device__ void cell_potential(double ua, double ub, double va, double vb, double* out)
{
    double Aa = branch_diff(ua, va, vb), Ab = branch_diff(ub, va, vb);
    double Ba = branch_diff(va, ua, ub), Bb = branch_diff(vb, ua, ub);
    // [u ln(v+r)] and [v ln(u+r)]; a zero factor gives its limit 0
    double su = (ub != 0 ? ub * Ab : 0.0) - (ua != 0 ? ua * Aa : 0.0);
    double sv = (vb != 0 ? vb * Bb : 0.0) - (va != 0 ? va * Ba : 0.0);
    double p0 = su + sv;
    double raa = sqrt(ua * ua + va * va), rab = sqrt(ua * ua + vb * vb);
    double rba = sqrt(ub * ub + va * va), rbb = sqrt(ub * ub + vb * vb);
    // [v r] = vb (r_bb - r_ab) - va (r_ba - r_aa), r-differences at fixed v
    double dux = (ub - ua) * (ub + ua);
    double vr = dux * (vb / (rbb + rab) - va / (rba + raa));
    // [u r] = ub (r_bb - r_ba) - ua (r_ab - r_aa), at fixed u
    double dvy = (vb - va) * (vb + va);
    double ur = dvy * (ub / (rbb + rba) - ua / (rab + raa));
    // [u^2 ln(v+r)] and [v^2 ln(u+r)]
    double su2 = (ub != 0 ? ub * ub * Ab : 0.0) - (ua != 0 ? ua * ua * Aa : 0.0);
    double sv2 = (vb != 0 ? vb * vb * Bb : 0.0) - (va != 0 ? va * va * Ba : 0.0);
    double uc = 0.5 * (ua + ub), vc = 0.5 * (va + vb);
    out[0] = p0;
    out[1] = 0.5 * (vr + su2) - uc * p0;
    out[2] = 0.5 * (ur + sv2) - vc * p0;
}

// Entry (nx, ny) of the six M x M tables of one phase (family 1: the three
// potential tables, then three zero planes).  The lattice offset
// (output - input) is n = nx or nx - M; n = M/2 is never used and is 0.
//   kind 1 (same level):      cell [-n - 1/2, -n + 1/2]              (width 1)
//   kind 2 (finer source, m): cell [-m n + k - m/2, ... + 1]          (width 1)
//   kind 3 (coarser source):  cell [-m n - k - 1/2, ... + m]          (width m)
// all in units of the finer cell side (Section 2.1, Cases 1-3).
__global__ void k_table(TableJob J)
{
    const int M = J.M;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)M * M) return;
    const int nx = (int)(idx % M), ny = (int)(idx / M);
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (nx != M / 2 && ny != M / 2) {
        const double sx = (nx < M / 2) ? nx : nx - M;
        const double sy = (ny < M / 2) ? ny : ny - M;
        double ua, va, w;
        if (J.kind == 1) {
            ua = -sx - 0.5; va = -sy - 0.5; w = 1.0;
        } else if (J.kind == 2) {
            ua = -J.m * sx + J.kx - 0.5 * J.m;
            va = -J.m * sy + J.ky - 0.5 * J.m;
            w = 1.0;
        } else {
            ua = -J.m * sx - J.kx - 0.5;
            va = -J.m * sy - J.ky - 0.5;
            w = J.m;
        }
        // rectangular cells: y offsets and heights in units of the width
        const double a = J.aspect, wa = w * a;
        va *= a;
        if (J.family == 0) {
            cell_integrals(ua, ua + w, va, va + wa, v);
            if (J.kind == 3) {
                const double inv = 1.0 / J.m;
                v[1] *= inv; v[2] *= inv; v[4] *= inv; v[5] *= inv;
            }
        } else {
            // the potential carries one more length than the force: a
            // coarser source's inputs are scaled by its own cell side, m
            // times the table unit, hence 1/m (1/m^2 for the slopes)
            cell_potential(ua, ua + w, va, va + wa, v);
            if (J.kind == 3) {
                const double inv = 1.0 / J.m;
                v[0] *= inv; v[1] *= inv * inv; v[2] *= inv * inv;
            }
        }
    }
    const size_t plane = (size_t)M * M;
#pragma unroll
    for (int X = 0; X < 6; ++X) J.out[X * plane + idx] = v[X];
}


// Copy the twiddle table (M entries) into LDS; every pass of a workgroup's
// FFTs then reads it from there.  Ends with a workgroup barrier: the FFTs
// themselves may only order their own wavefront.
template <typename T, int M>
__device__ __forceinline__ void stage_twiddles(cpx<T>* dst, const cpx<T>* __restrict__ src)
{
    for (int i = threadIdx.x; i < M; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Job order of a column launch (see JobQueue): a direct launch runs job
// blockIdx.x; a persistent one pulls jobs from the work lists until all are
// drained.  Every thread of the workgroup takes part (the job is broadcast
// through LDS), so every wave reaches the same loop exit.
// ---------------------------------------------------------------------------

// Workgroup b takes the next job of the list of its own XCD (b mod TD_NXCD:
// workgroups are dispatched to the XCDs round-robin), then, once that list
// is drained, of the other lists in turn, skipping (by a plain read of its
// counter) a list already drained.  s[0] is the job handed to the
// workgroup, s[1] the list offset thread 0 has reached.
__device__ __forceinline__ int pull_job(const JobQueue& q, int* s)
{
    __syncthreads();  // the previous job's use of LDS is over
    if (threadIdx.x == 0) {
        int item = -1;
        for (int d = s[1]; d < TD_NXCD; ++d) {
            const int l = (blockIdx.x + d) % TD_NXCD;
            const int first = q.start[l], len = q.start[l + 1] - first;
            if (d > 0 && (int)__hip_atomic_load(q.counter + l, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT) >= len) {
                s[1] = d + 1;
                continue;
            }
            const int k = (int)atomicAdd(q.counter + l, 1u);
            if (k < len) {
                item = q.order[first + k];
                break;
            }
            s[1] = d + 1;
        }
        s[0] = item;
    }
    __syncthreads();
    return s[0];
}

__device__ __forceinline__ int first_job(const JobQueue& q, int* s)
{
    if (!q.order) return blockIdx.x;
    if (threadIdx.x == 0) s[1] = 0;
    return pull_job(q, s);
}

__device__ __forceinline__ int next_job(const JobQueue& q, int* s)
{
    return q.order ? pull_job(q, s) : -1;
}

// Zero n work-list counters (launched ahead of a solve's persistent
// launches; a kernel rather than a memset, so that it can be captured).
__global__ void __launch_bounds__(256) k_zero_counters(unsigned int* c, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) c[i] = 0;
}

// ---------------------------------------------------------------------------
// Pass 1: zero-padded real row FFTs, transposed write
// ---------------------------------------------------------------------------

__device__ __forceinline__ int floor_div(int a, int b)
{
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Workgroups are dispatched to the eight XCDs round-robin, and each XCD has
// its own L2.  Renumbering them so that runs of K consecutive jobs go to one
// XCD keeps neighbouring target rows -- which read the same cache lines of
// the transposed spectra (K rows of 8 bytes fill a 128-byte line) -- in one
// L2, while the runs still rotate over the XCDs for load balance.
__device__ __forceinline__ int xcd_block(int bid, int nblk)
{
    constexpr int NXCD = 8, K = 16;
    const int full = nblk - nblk % (NXCD * K);
    if (bid >= full) return bid;
    const int x = bid % NXCD, l = bid / NXCD;
    return (x + NXCD * (l / K)) * K + l % K;
}


// Patch tables are read through global-address-space pointers (uniform per
// job, so the loads are scalar).
typedef const __attribute__((address_space(1))) LevelPatches* gpatches;

// Is window cell (i, j) of a level covered by a patch of the next finer level?
__device__ __forceinline__ bool covered(gpatches L, int i, int j)
{
    bool c = false;
    for (int k = 0; k < L->nc; ++k)
        c |= i >= L->ci0[k] && i < L->ci0[k] + L->cn[k] && j >= L->cj0[k] && j < L->cj0[k] + L->cn[k];
    return c;
}

// C = blockDim/(M/8) complex sequences; sequence p carries stored rows
// row0 + 2p (real part) and row0 + 2p + 1 (imaginary part).
// Estimated slope of cell (i, j) of an n x n patch times the cell side,
// i.e. the slope in per-cell units that the slope fields carry after their
// scaling by the source level's h: half the centred difference of the
// neighbouring values along x (f == 1) or y (f == 2), the one-sided
// difference in the patch's first and last column / row, 0 when n == 1.
template <typename T>
__device__ __forceinline__ double cell_slope(const T* __restrict__ s, int n, int i, int j, int f)
{
    const int c = f == 1 ? i : j;
    const ptrdiff_t st = f == 1 ? 1 : (ptrdiff_t)n;
    const T* p = s + (ptrdiff_t)j * n + i;
    if (n == 1) return 0.0;
    if (c == 0) return (double)p[st] - (double)p[0];
    if (c == n - 1) return (double)p[0] - (double)p[-st];
    return 0.5 * ((double)p[st] - (double)p[-st]);
}

// ZP: zero-padded rows (the solve's inputs): lattice columns >= M/2 lie
// past the level's window (M >= 2 nx and the nesting, checked on the host),
// so only the lower half of each sequence is gathered and the first FFT
// pass skips the rest.  The kernel-table rows are full length (!ZP).
template <typename T, int M, bool ZP>
__global__ void __launch_bounds__(TD_MAX_THREADS) k_row_fwd(SegTable<RowFwdJob> segs,
                                                  const void* const* __restrict__ ptrs,
                                                  const FieldPtrs fp,
                                                  const cpx<T>* __restrict__ tw_g)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
    int slot_base;
    const void* aux;
    char* ws;
    // consecutive jobs (neighbouring stored rows, whose transposed outputs
    // share cache lines) run on one XCD, so their partial-line writes merge
    // in that XCD's L2
    const RowFwdJob J = segs.find(xcd_block(blockIdx.x, gridDim.x), &slot_base, &aux, &ws);
    const int C = blockDim.x / (M / 8);
    constexpr int SP = lds_stride<T>(M);
    cpx<T>* tw = buf + C * SP;
    stage_twiddles<T, M>(tw, tw_g);
    // source cells: window cell (m lc + col_off, m lr + row_off) of level
    // J.lvl, taken from the patch that holds it, zero where no patch does
    // or a finer patch covers it
    gpatches L = (gpatches)aux + J.lvl;
    const int np = L->np;
    const int rend = J.row0 + J.nrow;
    constexpr int NG = ZP ? M / 2 : M;  // columns gathered
    if (np == 1 && L->nc <= 1) {
        // one patch, at most one covered square (every level of a nested
        // hierarchy): the patch's and square's bounds are read once, into
        // scalar registers, instead of per element
        const uintptr_t raw = (uintptr_t)(fp.n ? fp.p[slot_base + L->pslot[0] + J.f]
                                               : ptrs[slot_base + L->pslot[0] + J.f]);
        const T* src = reinterpret_cast<const T*>(raw & ~(uintptr_t)1);
        const bool est = raw & 1;
        const int n = L->pn[0], pi0 = L->pi0[0], pj0 = L->pj0[0];
        const bool hc = L->nc == 1;
        const int ci0 = hc ? L->ci0[0] : 0, cj0 = hc ? L->cj0[0] : 0, cn = hc ? L->cn[0] : 0;
        // a given field's values are scaled in the plan's precision
        const T sc = (T)J.scale;
        // each thread walks its sequences p (rows 2p, 2p + 1 of the job) and
        // its columns; the row quantities are formed once per sequence
        const int LCS = min((int)blockDim.x, NG), RPI = blockDim.x / LCS;
        for (int p = threadIdx.x / LCS; p < C; p += RPI) {
            const int s0 = J.row0 + 2 * p;
            const int sr0 = J.m * (J.lr_first + s0) + J.row_off, sr1 = sr0 + J.m;
            const int j0 = sr0 - pj0, j1 = sr1 - pj0;
            const bool ok0 = src && s0 < rend && j0 >= 0 && j0 < n;
            const bool ok1 = src && s0 + 1 < rend && j1 >= 0 && j1 < n;
            // rows that cross the covered square
            const bool cy0 = sr0 >= cj0 && sr0 < cj0 + cn, cy1 = sr1 >= cj0 && sr1 < cj0 + cn;
            const T* row0 = src + (ptrdiff_t)(ok0 ? j0 : 0) * n;
            const T* row1 = src + (ptrdiff_t)(ok1 ? j1 : 0) * n;
            for (int lc = threadIdx.x % LCS; lc < NG; lc += LCS) {
                T a = 0, b = 0;
                const int scol = J.m * lc + J.col_off;
                const int i = scol - pi0;
                // lattice columns outside the source level's window, or
                // outside the patch, read nothing
                if (lc >= J.lc_lo && lc < J.lc_hi && i >= 0 && i < n) {
                    const bool cx = scol >= ci0 && scol < ci0 + cn;
                    if (ok0 && !(cx && cy0))
                        a = est ? (T)(J.est_scale * cell_slope(src, n, i, j0, J.f)) : sc * row0[i];
                    if (ok1 && !(cx && cy1))
                        b = est ? (T)(J.est_scale * cell_slope(src, n, i, j1, J.f)) : sc * row1[i];
                }
                buf[p * SP + lds_pos<T>(lc)] = cpx<T>{a, b};
            }
        }
    } else
    for (int idx = threadIdx.x; idx < C * NG; idx += blockDim.x) {
        const int p = idx / NG, lc = idx % NG;
        if (lc < J.lc_lo || lc >= J.lc_hi) {  // outside the source level's window
            buf[p * SP + lds_pos<T>(lc)] = cpx<T>{0, 0};
            continue;
        }
        const int s0 = J.row0 + 2 * p;
        const int scol = J.m * lc + J.col_off;
        const int sr0 = J.m * (J.lr_first + s0) + J.row_off, sr1 = sr0 + J.m;
        T a = 0, b = 0;
        for (int k = 0; k < np; ++k) {
            const int slot = slot_base + L->pslot[k] + J.f;
            // a slope slot tagged in bit 0 holds the patch's sigma: estimate
            // the slope from it (uniform over the workgroup)
            const uintptr_t raw = (uintptr_t)(fp.n ? fp.p[slot] : ptrs[slot]);
            const T* src = reinterpret_cast<const T*>(raw & ~(uintptr_t)1);
            const bool est = raw & 1;
            const int n = L->pn[k], i = scol - L->pi0[k];
            if (!src || i < 0 || i >= n) continue;
            const int j0 = sr0 - L->pj0[k], j1 = sr1 - L->pj0[k];
            if (s0 < rend && j0 >= 0 && j0 < n && !covered(L, scol, sr0))
                a = est ? (T)(J.est_scale * cell_slope(src, n, i, j0, J.f))
                        : (T)J.scale * src[(size_t)j0 * n + i];
            if (s0 + 1 < rend && j1 >= 0 && j1 < n && !covered(L, scol, sr1))
                b = est ? (T)(J.est_scale * cell_slope(src, n, i, j1, J.f))
                        : (T)J.scale * src[(size_t)j1 * n + i];
        }
        buf[p * SP + lds_pos<T>(lc)] = cpx<T>{a, b};
    }
    __syncthreads();
    fft_lds<T, M, false, ZP>(buf, tw);
    __syncthreads();  // the transposed write reads every sequence
    // each thread unpacks both rows of one sequence at one frequency (the
    // two real rows' spectra from z(kx) and conj z(M - kx)) and stores them
    // with one 16-byte store: the lanes of a frequency write its 2C rows
    // contiguously
    cpx<T>* out = reinterpret_cast<cpx<T>*>(ws + J.out);
    for (int idx = threadIdx.x; idx < (M / 2 + 1) * C; idx += blockDim.x) {
        const int p = idx % C, kx = idx / C;
        const int r = 2 * p;
        if (r >= J.nrow) continue;
        const cpx<T> z = buf[p * SP + lds_pos<T>(kx)];
        const cpx<T> zc = conj(buf[p * SP + lds_pos<T>((M - kx) & (M - 1))]);
        const cpx<T> X0{(T)0.5 * (z.re + zc.re), (T)0.5 * (z.im + zc.im)};
        const cpx<T> d = z - zc;  // (z - zc) / (2i)
        const cpx<T> X1{(T)0.5 * d.im, (T)-0.5 * d.re};
        cpx<T>* o = out + (size_t)kx * J.ld + J.row0 + r;
        if (r + 1 < J.nrow) {
            // o is only as aligned as one complex value (ld may be odd):
            // the type says so, and the compiler picks a store that allows it
            typedef T __attribute__((ext_vector_type(4), aligned(2 * sizeof(T)))) vec4a;
            *reinterpret_cast<vec4a*>(o) = vec4a{X0.re, X0.im, X1.re, X1.im};
        } else {
            o[0] = X0;
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel-spectrum lookup with the mirror symmetries of the phases
// ---------------------------------------------------------------------------

// Kernels X = 0..5: I0, Ixx, Ixy, J0, Jyy, Jyx.  Parity under x- and
// y-mirrors of the source cell about the target:
//   s_x = -1, 1, -1, 1, 1, -1 and s_y = 1, 1, -1, -1, 1, -1,
// written as bit masks of the negative entries.
__host__ __device__ constexpr int sign_x(int X) { return ((0x25 >> X) & 1) ? -1 : 1; }
__host__ __device__ constexpr int sign_y(int X) { return ((0x2C >> X) & 1) ? -1 : 1; }
// Potential family (flip bit 3): P0 even in both axes, Px odd in x, Py odd
// in y; the zero planes 3-5 take any sign.
__host__ __device__ constexpr int sign_x(int X, int fam) { return fam ? (X == 1 ? -1 : 1) : sign_x(X); }
__host__ __device__ constexpr int sign_y(int X, int fam) { return fam ? (X == 2 ? -1 : 1) : sign_y(X); }
// Kernel feeding output component c (0: Fx, 1: Fy) from field f (sigma,
// dsdx, dsdy): I0, Ixx, Ixy for Fx and J0, Jyx, Jyy for Fy.
__host__ __device__ constexpr int kern_of(int c, int f) { return c == 0 ? f : 3 + (3 - f) % 3; }

// Kernel spectra and workspace planes live in global memory; their
// addresses come from job descriptors, so the compiler cannot infer the
// address space by itself (and would emit flat loads, which also hold up
// every LDS wait).  Converted with C-style casts.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

// One complex value through a global pointer (a two-element vector load).
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ cpx<T> ldg(gptr<cpx<T>> p, ptrdiff_t i)
{
    const vec2<T> v = ((gptr<vec2<T>>)p)[i];
    return cpx<T>{v.x, v.y};
}

// The eight values this thread needs (frequencies ky = lane + q M/8) of
// stored kernel X at column kx.
//  flip bit 2: a same-level kernel, symmetric under both mirrors, stored as
//    one real R per frequency for ky in [0, M/2]: the spectrum is R when
//    s_x s_y = +1 and i R otherwise, and S(kx, ky) = s_y S(kx, M - ky);
//  otherwise a polyphase phase stored complex for all ky; bits 0 / 1 select
//    its x- / y-mirror image: S'(kx, ky) = s_x conj S(kx, -ky),
//    s_y S(kx, -ky), or s_x s_y conj S(kx, ky).
// kern_load issues the reads (the real layout fills only .re), so that they
// can be in flight across other work; kern_mac (below) forms the values and
// multiplies.
template <typename T, int M>
__device__ __forceinline__ void kern_load(cpx<T> (&z)[8], const void* Kv, int X, int kx, int flip,
                                          int lane)
{
    constexpr int TPS = M / 8, H = M / 2 + 1;
    if (flip & 4) {
        gptr<T> R = (gptr<T>)Kv + ((size_t)X * H + kx) * H;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int ky = lane + q * TPS;
            z[q].re = R[q < 4 ? ky : M - ky];  // ky >= M/2 from its mirror M - ky
        }
    } else {
        gptr<cpx<T>> K = (gptr<cpx<T>>)Kv + ((size_t)X * H + kx) * M;
        const int mir = flip & 3;
        if (mir == 1 || mir == 2) {
            // the mirror reads frequency -ky: (M - ky) mod M, i.e. M - lane
            // - q M/8 for q > 0 and (M - lane) mod M for q = 0
            gptr<cpx<T>> Kr = K + (M - lane);
            z[0] = ldg<T>(K, (M - lane) & (M - 1));
#pragma unroll
            for (int q = 1; q < 8; ++q) z[q] = ldg<T>(Kr, -(ptrdiff_t)(q * TPS));
        } else {
            gptr<cpx<T>> Kf = K + lane;
#pragma unroll
            for (int q = 0; q < 8; ++q) z[q] = ldg<T>(Kf, q * TPS);
        }
    }
}

// Index of a slot's current item, scalar when a slot is a whole wavefront
// (M/8 >= 64): its descriptor then loads into scalar registers and every
// branch on it is uniform.
template <int M>
__device__ __forceinline__ int slot_uniform(int i)
{
    if constexpr (M / 8 >= 64) return __builtin_amdgcn_readfirstlane(i);
    return i;
}

// A column-pass descriptor (ColIn / ColOut) at a slot's item index.  When a
// slot is a whole wavefront the index is uniform and the tables are
// read-only during the launch: a constant-address-space (scalar) load, so
// every branch on the descriptor's fields is uniform.
template <int M, typename D>
__device__ __forceinline__ D load_desc(const D* tab, int i)
{
    if constexpr (M / 8 >= 64) return load_const(tab, i);
    else return tab[i];
}

// acc += (S z.re + i S C z.im) * v over the thread's 8 frequencies, with the
// signs S, C = +-1 fixed at compile time (they become operand modifiers of
// the fused multiply-adds).
template <typename T, int S, int C>
__device__ __forceinline__ void mac_signed(cpx<T> (&acc)[8], const cpx<T> (&z)[8], const cpx<T> (&v)[8])
{
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        acc[q].re = fma((T)S * z[q].re, v[q].re, acc[q].re);
        acc[q].re = fma((T)(-S * C) * z[q].im, v[q].im, acc[q].re);
        acc[q].im = fma((T)S * z[q].re, v[q].im, acc[q].im);
        acc[q].im = fma((T)(S * C) * z[q].im, v[q].re, acc[q].im);
    }
}

// acc += K v, K the kernel X of a stored spectrum column z as kern_load
// read it (raw values), seen through the layout and mirror bits of `flip`
// as described above; flip and X uniform over the slot.  No per-value
// sign or select work: the sign pattern picks one of four products.
template <typename T, int M>
__device__ __forceinline__ void kern_mac(cpx<T> (&acc)[8], const cpx<T> (&z)[8], const cpx<T> (&v)[8],
                                         int X, int flip, int lane)
{
    const int fam = (flip >> 3) & 1;
    if (flip & 4) {
        // same-level kernel: one real R per frequency; the spectrum is R or
        // i R, and frequencies above M/2 (q > 4, and q = 4 but for lane 0,
        // ky = M/2, which is stored directly) carry the y-parity s_y
        const bool imag = sign_x(X, fam) * sign_y(X, fam) < 0;
        T r[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) r[q] = z[q].re;
        if (sign_y(X, fam) < 0) {
#pragma unroll
            for (int q = 5; q < 8; ++q) r[q] = -r[q];
            r[4] = lane > 0 ? -r[4] : r[4];
        }
        if (imag) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                acc[q].re = fma(-r[q], v[q].im, acc[q].re);
                acc[q].im = fma(r[q], v[q].re, acc[q].im);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                acc[q].re = fma(r[q], v[q].re, acc[q].re);
                acc[q].im = fma(r[q], v[q].im, acc[q].im);
            }
        }
    } else {
        // polyphase phase: mirror bits 0 / 1 give the sign s (x- and
        // y-parities) and x-mirrors conjugate
        const int mir = flip & 3;
        const int s = ((mir & 1) ? sign_x(X, fam) : 1) * ((mir & 2) ? sign_y(X, fam) : 1);
        const bool cj = mir & 1;
        if (s > 0) {
            if (cj) mac_signed<T, 1, -1>(acc, z, v);
            else mac_signed<T, 1, 1>(acc, z, v);
        } else {
            if (cj) mac_signed<T, -1, -1>(acc, z, v);
            else mac_signed<T, -1, 1>(acc, z, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 2: column FFTs fused with the kernel-spectrum products
// ---------------------------------------------------------------------------
// Slot (c, g) of a workgroup works on spectral column kx0 + c with its own
// LDS sequence.  Every loop below runs the same number of iterations in all
// slots of the workgroup (the FFTs synchronise the whole workgroup); slots
// without work transform zeros.  Each thread owns frequencies
// ky = lane + q M/8, q < 8, of its slot's sequence.

struct ColTables {
    const ColIn* ins;
    const ColOut* outs;
};

// Stored rows of input plane I, column kx, at the calling thread's
// elements lane + q M/8 of the column (q < 4; zero where no row is stored).
// Lattice rows >= M/2 hold no source cell (M >= 2 ny and the nesting,
// checked on the host): v[4..7] are not set, the forward transform skips
// them (ZIN).  (Unconditional loads from a clamped row -- row 0 of the
// workspace for a slot without an input -- then a select.)
template <typename T, int M>
__device__ __forceinline__ void load_column(cpx<T> (&v)[8], const char* ws, const ColIn& I, int kx,
                                            bool ok, int lane)
{
    constexpr int TPS = M / 8;
    gptr<cpx<T>> src = (gptr<cpx<T>>)(ws + (ok ? I.in + (int64_t)kx * I.ld * (int64_t)sizeof(cpx<T>) : 0));
    const int last = ok ? I.ld - 1 : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int sr = lane + q * TPS - I.lr_first;
        const cpx<T> x = ldg<T>(src, min(max(sr, 0), last));
        v[q] = (ok && sr >= 0 && sr <= last) ? x : cpx<T>{0, 0};
    }
}

// load_column split in two so that the loads can be issued one iteration
// ahead: the raw values (unconditional loads from a clamped row) and their
// validity, applied where the values are used.
template <typename T, int M, int N>
__device__ __forceinline__ void load_column_raw(cpx<T> (&x)[N], bool (&val)[N], const char* ws,
                                                const ColIn& I, int kx, bool ok, int lane)
{
    static_assert(N >= 4, "four values per thread");
    constexpr int TPS = M / 8;
    gptr<cpx<T>> src = (gptr<cpx<T>>)(ws + (ok ? I.in + (int64_t)kx * I.ld * (int64_t)sizeof(cpx<T>) : 0));
    const int last = ok ? I.ld - 1 : 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int sr = lane + q * TPS - I.lr_first;
        x[q] = ldg<T>(src, min(max(sr, 0), last));
        val[q] = ok && sr >= 0 && sr <= last;
    }
}

// exp(-2 pi i n / M), 0 <= n < M: the last radix-8 pass's twiddle
// exp(-2 pi i (n mod M/8) / M) (its r = 1 row), times the eighth root of
// unity exp(-i pi (n div M/8) / 4) by exact rotations and one product by
// 1/sqrt 2.
template <typename T, int M>
__device__ __forceinline__ cpx<T> unit_root(const cpx<T>* tw, int n)
{
    constexpr int E = M / 8;
    cpx<T> z = tw[tw_offset(M, E) + (n & (E - 1))];
    const int R = n / E;
    const T h = (T)0.70710678118654752440084436210484903928;
    if (R & 1) z = cpx<T>{h * (z.re + z.im), h * (z.im - z.re)};  // (1 - i) / sqrt 2
    if (R & 2) z = cpx<T>{z.im, -z.re};                              // -i
    if (R & 4) z = cpx<T>{-z.re, -z.im};                             // -1
    return z;
}

// Band-limited input plane I (all of its non-zero stored rows among the
// first I.rows <= D = M/S, S = band_span(M)): the raw values of the calling
// thread's inputs to the band transform's first pass (fft_regs_band).  Its
// element r is element c S + k of the span-S array, c = lane/S + r D/8,
// k = lane % S, which is the lattice row n = c (mod D) of the band
// [lr_first, lr_first + D), times a twiddle (band_inputs): stored row
// (c - lr_first) mod D, valid below I.rows.  (Unconditional loads from a
// clamped row, then a select, as in load_column_raw.)
template <typename T, int M>
__device__ __forceinline__ void load_band_raw(cpx<T> (&x)[8], bool (&val)[8], const char* ws,
                                              const ColIn& I, int kx, bool ok, int lane)
{
    constexpr int S = band_span(M), D = M / S;
    gptr<cpx<T>> src = (gptr<cpx<T>>)(ws + (ok ? I.in + (int64_t)kx * I.ld * (int64_t)sizeof(cpx<T>) : 0));
    const int last = ok ? I.rows - 1 : 0;
    const int c0 = lane / S - I.lr_first;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int sr = (c0 + r * (D / 8)) & (D - 1);
        x[r] = ldg<T>(src, min(sr, last));
        val[r] = ok && sr <= last;
    }
}

// The band transform's inputs from load_band_raw's values: the element of
// class c holds x[n] w_S^(k u), u = n div D, which is lr_first div D when
// c >= lr_first mod D and one more when the band wraps past a multiple of D
// before reaching c.
template <typename T, int M>
__device__ __forceinline__ void band_inputs(cpx<T> (&v)[8], const cpx<T> (&x)[8], const bool (&val)[8],
                                            int lr_first, const cpx<T>* tw, int lane)
{
    constexpr int S = band_span(M), D = M / S;
    const int k = lane % S, c = lane / S;
    const int t0 = lr_first / D, b = lr_first % D;
    // w_S^(k u) = exp(-2 pi i k u D / M)
    const cpx<T> g0 = unit_root<T, M>(tw, (t0 * k * D) & (M - 1));
    const cpx<T> g1 = unit_root<T, M>(tw, ((t0 + 1) * k * D) & (M - 1));
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const cpx<T> g = c + r * (D / 8) < b ? g1 : g0;
        v[r] = val[r] ? cmul(x[r], g) : cpx<T>{0, 0};
    }
}

// Rows [out_lr_first, out_lr_first + out_ld) of a transformed column from
// the calling thread's elements lane + r M/8; every stored row is below M/2
// (checked on the host), so r < 4, the half the inverse transforms form
// (ZOUT).
template <typename T, int M>
__device__ __forceinline__ void store_column(const cpx<T> (&w)[8], char* ws, const ColOut& O, int kx,
                                             int lane)
{
    constexpr int TPS = M / 8;
    cpx<T>* dst = reinterpret_cast<cpx<T>*>(ws + O.out) + (size_t)kx * O.out_ld;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int sr = lane + r * TPS - O.out_lr_first;
        if (sr >= 0 && sr < O.out_ld) dst[sr] = w[r];
    }
}

// One column job of the fused column pass (see ColJob).
template <typename T, int M>
__device__ __forceinline__ void col_job(const SegTable<ColJob>& segs, int item, cpx<T>* A,
                                        const cpx<T>* tw, int G, int tid, cpx<T>* A2)
{
    constexpr bool PP = col_pingpong<T, M>();
    constexpr int TPS = M / 8;
    constexpr int SP = lds_stride<T>(M);
    int slot_unused;
    const void* aux;
    char* ws;
    const ColJob J = segs.find(item, &slot_unused, &aux, &ws);
    const ColTables tabs = load_const(reinterpret_cast<const ColTables*>(aux), 0);
    const int slot = tid / TPS, lane_c = tid % TPS;
    const int lane = lane_c;
    // uniform over a wavefront when a slot is one (or more): the column,
    // its validity and every descriptor derived from them stay scalar
    const int c = slot_uniform<M>(slot / G), g = slot_uniform<M>(slot % G);
    const int kx = J.kx0 + c;
    const bool col_ok = c < J.ncol;
    cpx<T>* a = A + slot * SP;
    cpx<T>* col0 = A + c * G * SP;  // the column's first slot
    // Inside the loops the lane index is re-derived through an empty asm
    // barrier, so that the per-frequency addresses are recomputed in each
    // iteration instead of being hoisted and held in registers throughout.

    if (J.kind == 0) {
        // band-limited inputs (the job's last nband) in rounds r0 >= nb0:
        // the round's choice is uniform over the workgroup, so every slot
        // passes the same ordering points
        constexpr int BROWS = col_band_rows(M, (int)sizeof(cpx<T>));
        constexpr bool BAND = BROWS > 0;
        static_assert(!BAND || (band_ok(M) && BROWS == M / band_span(M)), "band bound");
        constexpr int NX = BAND ? 8 : 4;
        const int nb0 = J.nin - J.nband;
        cpx<T> ax[8], ay[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) ax[q] = ay[q] = cpx<T>{0, 0};
        // each input's column is loaded one iteration ahead, while the
        // previous input is transformed and multiplied
        ColIn In{};
        bool okn;
        cpx<T> xn[NX];
        bool vn[NX];
        auto prefetch = [&](int r, int lane_p) {
            const int i = slot_uniform<M>(r + g);
            okn = col_ok && i < J.nin;
            In = ColIn{};
            if (okn) In = load_desc<M>(tabs.ins, J.in0 + i);
            if constexpr (BAND) {
                if (r >= nb0) {
                    load_band_raw<T, M>(xn, vn, ws, In, kx, okn, lane_p);
                    return;
                }
            }
            load_column_raw<T, M>(xn, vn, ws, In, kx, okn, lane_p);
        };
        prefetch(0, lane_c);
        for (int r0 = 0; r0 < J.nin; r0 += G) {
            int lane = lane_c;
            asm volatile("" : "+v"(lane));
            const ColIn I = In;
            const bool ok = okn;
            const bool band = BAND && r0 >= nb0;
            cpx<T> v[8];
            if constexpr (BAND) {
                if (band) band_inputs<T, M>(v, xn, vn, I.lr_first, tw, lane);
            }
            if (!band) {
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = vn[q] ? xn[q] : cpx<T>{0, 0};
            }
            prefetch(r0 + G, lane);
            // FP32 with M >= 1024 reads the input's kernel columns before its
            // transform, so that the reads are in flight across it (32 VGPRs
            // held, still 3 waves per SIMD); FP64 and shorter M, whose
            // register budgets are tighter, read them after it
            constexpr bool KEARLY = sizeof(T) == 4 && M >= 1024;
            cpx<T> z0[8], z1[8];
            if (KEARLY && ok) {
                kern_load<T, M>(z0, I.kern, kern_of(0, I.f), kx, I.flip, lane);
                kern_load<T, M>(z1, I.kern, kern_of(1, I.f), kx, I.flip, lane);
            }
            // a slot without an input skips its transform when sequences
            // are ordered within their wavefront only (M/8 <= 64)
            if (M / 8 > 64 || ok) {
                if constexpr (BAND) {
                    if (band) fft_regs_band<T, M, PP>(v, A, tw, A2);
                    else fft_regs<T, M, false, true, false, PP>(v, A, tw, A2);
                } else {
                    fft_regs<T, M, false, true, false, PP>(v, A, tw, A2);
                }
            }
            if (ok) {
                if (!KEARLY) {
                    kern_load<T, M>(z0, I.kern, kern_of(0, I.f), kx, I.flip, lane);
                    kern_load<T, M>(z1, I.kern, kern_of(1, I.f), kx, I.flip, lane);
                }
                kern_mac<T, M>(ax, z0, v, kern_of(0, I.f), I.flip, lane);
                kern_mac<T, M>(ay, z1, v, kern_of(1, I.f), I.flip, lane);
            }
        }
        // reduce the slots' partial sums: Fx into slot 0, Fy into slot 1
        // (slot 0 as well when G == 1)
        const int gy = G > 1 ? 1 : 0;
        cpx<T> sx[8], sy[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) sx[q] = sy[q] = cpx<T>{0, 0};
#pragma unroll
        for (int q = 0; q < 8; ++q) a[lds_pos<T>(lane + q * TPS)] = ax[q];
        __syncthreads();
        if (g == 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int p = lds_pos<T>(lane + q * TPS);
                cpx<T> sum = col0[p];
                for (int h = 1; h < G; ++h) sum = sum + col0[h * SP + p];
                sx[q] = sum;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) a[lds_pos<T>(lane + q * TPS)] = ay[q];
        __syncthreads();
        if (g == gy) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int p = lds_pos<T>(lane + q * TPS);
                cpx<T> sum = col0[p];
                for (int h = 1; h < G; ++h) sum = sum + col0[h * SP + p];
                sy[q] = sum;
            }
        }
        __syncthreads();  // the sums are read: the slots' LDS is free again
        // inverse column transforms in registers (every slot transforms:
        // slot 0 Fx, slot gy Fy, the others zeros)
        cpx<T> w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = g == 0 ? sx[q] : (g == gy ? sy[q] : cpx<T>{0, 0});
        if (M / 8 > 64 || g == 0 || g == gy) fft_regs<T, M, true, false, true, PP>(w, A, tw, A2);
        if (col_ok && g == 0) store_column<T, M>(w, ws, load_desc<M>(tabs.outs, J.out0), kx, lane);
        if (col_ok && G > 1 && g == 1)
            store_column<T, M>(w, ws, load_desc<M>(tabs.outs, J.out0 + 1), kx, lane);
        if (G == 1) {
#pragma unroll
            for (int q = 0; q < 8; ++q) w[q] = sy[q];
            fft_regs<T, M, true, false, true, PP>(w, A, tw, A2);
            if (col_ok) store_column<T, M>(w, ws, load_desc<M>(tabs.outs, J.out0 + 1), kx, lane);
        }
        return;
    }

    // kind 1: transform the three inputs, keeping this thread's frequencies
    // of all three in registers
    cpx<T> vin[3][8];
    for (int r0 = 0; r0 < 3; r0 += G) {
        const int i = slot_uniform<M>(r0 + g);
        const bool ok = col_ok && i < 3;
        ColIn I{};
        if (ok) I = load_desc<M>(tabs.ins, J.in0 + i);
        cpx<T> v[8];
        load_column<T, M>(v, ws, I, kx, ok, lane);
        fft_regs<T, M, false, true, false, PP>(v, A, tw, A2);
#pragma unroll
        for (int q = 0; q < 8; ++q) a[lds_pos<T>(lane + q * TPS)] = v[q];
        __syncthreads();  // every slot reads the three transformed inputs
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            if (f >= r0 && f < r0 + G) {
#pragma unroll
                for (int q = 0; q < 8; ++q) vin[f][q] = col0[(f - r0) * SP + lds_pos<T>(lane + q * TPS)];
            }
        }
        __syncthreads();
    }
    for (int o0 = 0; o0 < J.nout; o0 += G) {
        int lane = lane_c;
        asm volatile("" : "+v"(lane));
        const int o = slot_uniform<M>(o0 + g);
        const bool ok = col_ok && o < J.nout;
        cpx<T> acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = cpx<T>{0, 0};
        ColOut O{0, nullptr, 0, 0, 0, 0};
        if (ok) {
            O = load_desc<M>(tabs.outs, J.out0 + o);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                cpx<T> z[8];
                kern_load<T, M>(z, O.kern, kern_of(O.comp, f), kx, O.flip, lane);
                kern_mac<T, M>(acc, z, vin[f], kern_of(O.comp, f), O.flip, lane);
            }
        }
        if (M / 8 > 64 || ok) fft_regs<T, M, true, false, true, PP>(acc, A, tw, A2);
        if (ok) store_column<T, M>(acc, ws, O, kx, lane);
    }
}

// PQ: a persistent launch (jobs pulled from the work lists of q); else one
// workgroup per job.  Separate instantiations: the job loop costs the direct
// launch registers and scalar uniformity.
//
// FP32 at M <= 512 is held to 128 VGPRs (4 waves per SIMD, a few registers
// spilled): its sequences fit one wavefront, so nothing waits at workgroup
// barriers and the extra waves hide memory latency (side by side: M = 512
// 17.6 -> 16.7 us on two-level 256^2; on the 64-disk batch M = 256 234 ->
// 196 us, M = 128 92 -> 70 us).  At M = 1024 the same cap cost 11%.
template <typename T, int M>
constexpr int col_waves_per_eu() { return sizeof(T) == 4 && M <= 512 ? 4 : 1; }

template <typename T, int M, bool PQ>
__global__ void __launch_bounds__(TD_MAX_THREADS) __attribute__((amdgpu_waves_per_eu(col_waves_per_eu<T, M>())))
k_col(SegTable<ColJob> segs,
                                                        const cpx<T>* __restrict__ tw_g, int G,
                                                        const JobQueue q)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TPS = M / 8;
    constexpr int SP = lds_stride<T>(M);
    const int S = blockDim.x / TPS;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    // the transforms' second buffers follow the first (ping-pong lengths)
    cpx<T>* A2 = A + S * SP;
    cpx<T>* tw = A + (col_pingpong<T, M>() ? 2 : 1) * S * SP;
    stage_twiddles<T, M>(tw, tw_g);
    if constexpr (PQ) {
        __shared__ int s_item[2];
        for (int item = first_job(q, s_item); item >= 0; item = next_job(q, s_item)) {
            // opaque thread index: nothing derived from it is hoisted out
            // of the job loop and held across jobs
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            col_job<T, M>(segs, item, A, tw, G, tid, A2);
        }
    } else {
        col_job<T, M>(segs, blockIdx.x, A, tw, G, threadIdx.x, A2);
    }
}

// ---------------------------------------------------------------------------
// Pass 4: complex-to-real row FFTs, window / phase extraction, accumulation
// ---------------------------------------------------------------------------

// a / m for a >= 0: a shift when m = 2^sh (sh >= 0), else a division.
__device__ __forceinline__ int ratio_div(int a, int m, int sh)
{
    return sh >= 0 ? a >> sh : a / m;
}

// A workgroup owns C target rows; each row's items -- (contribution, x-phase)
// pairs, one complex-to-real row transform each -- run G at a time in the
// row's G slots.  Spectra are read transposed ([kx][row]), rows fastest.
// The G M/8 threads of a row own its target columns x0 + t + k G M/8 and
// accumulate them in registers over all items.
// NQ: outputs per thread and row (nx <= NQ G M/8 for every job of the
// launch): 4 covers a level's own lattice (nx <= M/2), 16 any job (nx <= 2M).
template <typename T, int M, int NQ>
__global__ void __launch_bounds__(TD_MAX_THREADS) k_row_inv(SegTable<RowInvJob> segs,
                                                  void* const* __restrict__ ptrs,
                                                  const FieldPtrs fp,
                                                  const cpx<T>* __restrict__ tw_g, int G)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int TPS = M / 8;
    constexpr int H = M / 2 + 1;
    constexpr int SP = lds_stride<T>(M);
    const int S = blockDim.x / TPS;
    const int C = S / G;  // rows of this workgroup
    const int GT = G * TPS;
    cpx<T>* A = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* tw = A + S * SP;
    // per slot of a round (two rounds in flight: buffers 0 and 1):
    // contribution (-1: none), x-phase, the contribution's ratio shift and
    // origin column
    __shared__ int it_c[2][16], it_kxp[2][16], it_sh[2][16], it_oxs[2][16];
    stage_twiddles<T, M>(tw, tw_g);
    int slot_base;
    const void* aux;
    char* ws;
    const RowInvJob J = segs.find(blockIdx.x, &slot_base, &aux, &ws);
    const RowInvTables tabs = *reinterpret_cast<const RowInvTables*>(aux);
    const RowInvContrib* __restrict__ contribs = tabs.contribs + J.c0;
    gpatches L = (gpatches)tabs.levels + J.lvl;
    int nitems = 0;
    for (int k = 0; k < J.nc; ++k) nitems += contribs[k].m;
    const int crow = threadIdx.x / GT, t = threadIdx.x % GT;
    T accx[NQ], accy[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) { accx[q] = 0; accy[q] = 0; }
    // C and G are powers of two.  blockDim = S M/8, so the loads of thread
    // x always serve sequence sq = x mod S (slot gg, row cc), frequencies
    // kx0 + k M/8: the threads of one kx read consecutive stored rows.
    const int lgC = __builtin_ctz(C), lgS = __builtin_ctz(S);
    const int sq = threadIdx.x & (S - 1), gg_l = sq >> lgC, cc_l = sq & (C - 1);
    const int kx0 = threadIdx.x >> lgS;
    constexpr int NL = (H + TPS - 1) / TPS;  // frequencies per thread (5)
    // the slot table of the round starting at item r0, into buffer b
    auto tables = [&](int r0, int b) {
        if (threadIdx.x < G) {
            const int it = r0 + threadIdx.x;
            int c = -1, kxp = 0, sh = 0, oxs = 0;
            if (it < nitems) {
                int k = 0, rem = it;
                while (rem >= contribs[k].m) rem -= contribs[k].m, ++k;
                c = k;
                kxp = rem;
                sh = contribs[k].mshift >= 0 ? contribs[k].mshift : -contribs[k].m;
                oxs = contribs[k].ox_s;
            }
            it_c[b][threadIdx.x] = c;
            it_kxp[b][threadIdx.x] = kxp;
            it_sh[b][threadIdx.x] = sh;
            it_oxs[b][threadIdx.x] = oxs;
        }
    };
    // this thread's loads of the round in buffer b (the stored row of its
    // sequence: the target row's coarse-lattice row and y-phase, Case 3',
    // and the slot's x-phase), held in registers until stored to LDS
    cpx<T> px[NL], py[NL];
    auto issue = [&](int b) {
        const int ci = it_c[b][gg_l];
        gptr<cpx<T>> P = nullptr;
        int64_t ld = 0, cs = 0;
        if (ci >= 0 && cc_l < J.ny) {
            const RowInvContrib& Q = contribs[ci];
            const int gy = J.oy_t + J.y0 + cc_l;  // >= 0
            const int Jc = ratio_div(gy, Q.m, Q.mshift), kyp = gy - Jc * Q.m;
            const int sr = Jc - Q.oy_s - Q.lr_first;
            P = (gptr<cpx<T>>)(ws + Q.base) + ((int64_t)(kyp * Q.m + it_kxp[b][gg_l]) * Q.phase_stride + sr);
            ld = Q.ld;
            cs = Q.comp_stride;
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int kx = kx0 + k * TPS;
            px[k] = py[k] = cpx<T>{0, 0};
            if (P && kx < H) {
                px[k] = ldg<T>(P, (int64_t)kx * ld);
                py[k] = ldg<T>(P, (int64_t)kx * ld + cs);
            }
        }
    };
    tables(0, 0);
    __syncthreads();
    issue(0);
    int b = 0;
    for (int r0 = 0; r0 < nitems; r0 += G, b ^= 1) {
        // the round's values into LDS: sequence = x + i y of the row's two
        // components, Hermitian-extended
        cpx<T>* rowp = A + (cc_l * G + gg_l) * SP;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int kx = kx0 + k * TPS;
            if (kx >= H) break;
            cpx<T> X = px[k], Y = py[k];
            if (kx == 0 || kx == M / 2) { X.im = 0; Y.im = 0; }
            rowp[lds_pos<T>(kx)] = cpx<T>{X.re - Y.im, X.im + Y.re};
            if (kx > 0 && kx < M / 2) rowp[lds_pos<T>(M - kx)] = cpx<T>{X.re + Y.im, Y.re - X.im};
        }
        const bool more = r0 + G < nitems;
        if (more) tables(r0 + G, b ^ 1);
        __syncthreads();
        // the next round's loads are in flight during this round's
        // transform and gather
        if (more) issue(b ^ 1);
        // a slot without an item need not transform (its zeros are never
        // read); with M/8 <= 64 a sequence is ordered within its wavefront
        // only, so skipping it cannot unbalance a workgroup barrier
        if (M / 8 > 64 || it_c[b][(threadIdx.x / TPS) % G] >= 0) fft_lds<T, M, true, false, true>(A, tw);
        __syncthreads();  // outputs gather from every slot of their row
        for (int gg = 0; gg < G; ++gg) {
            if (it_c[b][gg] < 0) break;
            // it_sh: log2(m), or -m when m is not a power of two
            const int sh = it_sh[b][gg], kxp = it_kxp[b][gg], oxs = it_oxs[b][gg];
            const int mm = sh >= 0 ? 1 << sh : -sh;
            const cpx<T>* rowv = A + (crow * G + gg) * SP;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int ii = t + q * GT;
                if (ii >= J.nx) break;
                const int gx = J.ox_t + J.x0 + ii;  // >= 0
                const int Ic = ratio_div(gx, mm, sh >= 0 ? sh : -1);
                if (gx - Ic * mm != kxp) continue;
                const cpx<T> v = rowv[lds_pos<T>(Ic - oxs)];
                accx[q] += v.re;
                accy[q] += v.im;
            }
        }
        __syncthreads();
    }
    // outputs: window cell (ii, row) goes to the patch that holds it (none:
    // not part of the level); cells covered by a finer patch are written 0
    typedef __attribute__((address_space(1))) T* gout;
    const int row = J.y0 + crow;
    if (crow >= J.ny) return;
    for (int k = 0; k < L->np; ++k) {
        const int slot = slot_base + L->pslot[k] + 3;
        gout fx = (gout)(fp.n ? fp.p[slot] : ptrs[slot]);
        gout fy = (gout)(fp.n ? fp.p[slot + 1] : ptrs[slot + 1]);
        const int n = L->pn[k], j = row - L->pj0[k];
        if (j < 0 || j >= n) continue;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int ii0 = t + q * GT;
            if (ii0 >= J.nx) break;
            const int ii = J.x0 + ii0, i = ii - L->pi0[k];
            if (i < 0 || i >= n) continue;
            const bool cov = covered(L, ii, row);
            const size_t o = (size_t)j * n + i;
            if (!J.accumulate) {
                if (fx) fx[o] = cov ? (T)0 : accx[q];
                if (fy) fy[o] = cov ? (T)0 : accy[q];
            } else if (!cov) {
                if (fx) fx[o] += accx[q];
                if (fy) fy[o] += accy[q];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel-spectrum build: column FFT of the row-transformed FP64 tables,
// scaled by 1/M^2 (both inverse transforms are unnormalised) and stored in T.
// ---------------------------------------------------------------------------

template <typename TO, int M>
__global__ void __launch_bounds__(TD_MAX_THREADS) k_spec_col(const cpx<double>* __restrict__ rows,
                                                   void* __restrict__ out_v,
                                                   const cpx<double>* __restrict__ tw_g,
                                                   int quarter)  // bit 0: layout, bit 1: family
{
    cpx<TO>* out = reinterpret_cast<cpx<TO>*>(out_v);
    TO* outq = reinterpret_cast<TO*>(out_v);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<double>* buf = reinterpret_cast<cpx<double>*>(smem_raw);
    const int C = blockDim.x / (M / 8);
    constexpr int SP = lds_stride<double>(M);
    cpx<double>* tw = buf + C * SP;
    stage_twiddles<double, M>(tw, tw_g);
    constexpr int NCOL = M / 2 + 1;
    const int per_x = (NCOL + C - 1) / C;
    const int X = blockIdx.x / per_x;
    const int kx0 = (blockIdx.x % per_x) * C;
    for (int i = threadIdx.x; i < C * M; i += blockDim.x) {
        const int c = i / M, ky = i % M;
        cpx<double> v{0, 0};
        if (kx0 + c < NCOL) v = rows[((size_t)X * NCOL + kx0 + c) * M + ky];
        buf[c * SP + lds_pos<double>(ky)] = v;
    }
    __syncthreads();
    fft_lds<double, M, false>(buf, tw);
    __syncthreads();  // the output loop reads every sequence
    const double sc = 1.0 / ((double)M * (double)M);
    for (int i = threadIdx.x; i < C * M; i += blockDim.x) {
        const int c = i / M, ky = i % M;
        if (kx0 + c >= NCOL) continue;
        const cpx<double> v = buf[c * SP + lds_pos<double>(ky)];
        if (!(quarter & 1)) {
            out[((size_t)X * NCOL + kx0 + c) * M + ky] = cpx<TO>{(TO)(v.re * sc), (TO)(v.im * sc)};
        } else if (ky <= M / 2) {
            // same-level kernel: real (s_x s_y = +1) or imaginary spectrum
            const int fam = (quarter >> 1) & 1;
            const double r = (sign_x(X, fam) * sign_y(X, fam) > 0) ? v.re : v.im;
            outq[((size_t)X * NCOL + kx0 + c) * NCOL + ky] = (TO)(r * sc);
        }
    }
}

// ---------------------------------------------------------------------------
// Debug check: non-finite values of an output array, added to a counter
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256) k_count_nonfinite(const T* __restrict__ p, int64_t n,
                                                       unsigned long long* counter)
{
    unsigned int c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        c += isfinite(p[i]) ? 0u : 1u;
    // one atomic per wavefront that saw any
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(counter, (unsigned long long)c);
}

// ---------------------------------------------------------------------------
// Host-side launchers (dispatch on M)
// ---------------------------------------------------------------------------

#define TD_FOR_EACH_M(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

template <typename KF>
static hipError_t launch_common(KF kf, int blocks, int threads, size_t smem, hipStream_t st,
                                void** args)
{
    return hipLaunchKernel(reinterpret_cast<const void*>(kf), dim3(blocks), dim3(threads), args,
                           smem, st);
}

template <typename T>
hipError_t launch_row_fwd(int M, int C, int blocks, const SegTable<RowFwdJob>& segs,
                          const void* const* ptrs, const FieldPtrs& fp, const void* tw,
                          bool padded, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    const int threads = C * (M / 8);
    const size_t smem = lds_bytes(M, C, sizeof(cpx<T>));
    SegTable<RowFwdJob> s = segs;
    const void* const* p = ptrs;
    FieldPtrs f = fp;
    const cpx<T>* t = reinterpret_cast<const cpx<T>*>(tw);
    void* args[] = {&s, &p, &f, &t};
    switch (M) {
#define X(MM)                                                                            \
    case MM:                                                                             \
        if (padded) return launch_common(k_row_fwd<T, MM, true>, blocks, threads, smem, st, args); \
        if constexpr (sizeof(T) == 8)                                                    \
            return launch_common(k_row_fwd<T, MM, false>, blocks, threads, smem, st, args); \
        return hipErrorInvalidValue;
        TD_FOR_EACH_M(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_col(int M, int C, int G, int blocks, const SegTable<ColJob>& segs,
                      const void* tw, hipStream_t st, const JobQueue& queue)
{
    if (blocks <= 0) return hipSuccess;
    const int threads = C * G * (M / 8);
    const size_t smem = col_lds_bytes(M, C, sizeof(cpx<T>), G);
    SegTable<ColJob> s = segs;
    const cpx<T>* t = reinterpret_cast<const cpx<T>*>(tw);
    int g = G;
    JobQueue q = queue;
    void* args[] = {&s, &t, &g, &q};
    switch (M) {
#define X(MM)                                                                                      \
    case MM:                                                                                       \
        return q.order ? launch_common(k_col<T, MM, true>, blocks, threads, smem, st, args)       \
                       : launch_common(k_col<T, MM, false>, blocks, threads, smem, st, args);
        TD_FOR_EACH_M(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_row_inv(int M, int C, int G, int blocks, const SegTable<RowInvJob>& segs,
                          void* const* ptrs, const FieldPtrs& fp, const void* tw, hipStream_t st,
                          int nq)
{
    if (blocks <= 0) return hipSuccess;
    if (nq < 1 || nq > 16) return hipErrorInvalidValue;
    const int threads = C * G * (M / 8);
    const size_t smem = lds_bytes(M, C, sizeof(cpx<T>), G);
    SegTable<RowInvJob> s = segs;
    void* const* p = ptrs;
    FieldPtrs f = fp;
    const cpx<T>* t = reinterpret_cast<const cpx<T>*>(tw);
    int g = G;
    void* args[] = {&s, &p, &f, &t, &g};
    switch (M) {
#define X(MM)                                                                                   \
    case MM:                                                                                    \
        return nq <= 4 ? launch_common(k_row_inv<T, MM, 4>, blocks, threads, smem, st, args)    \
                       : launch_common(k_row_inv<T, MM, 16>, blocks, threads, smem, st, args);
        TD_FOR_EACH_M(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename TO>
hipError_t launch_spec_col(int M, int C, const void* rows, void* out, const void* tw64,
                           int quarter, hipStream_t st)
{
    const int threads = C * (M / 8);
    const int per_x = (M / 2 + 1 + C - 1) / C;
    const int blocks = 6 * per_x;
    const size_t smem = ((size_t)C * lds_stride<double>(M) + M) * sizeof(cpx<double>);
    const cpx<double>* r = reinterpret_cast<const cpx<double>*>(rows);
    void* o = out;
    const cpx<double>* t = reinterpret_cast<const cpx<double>*>(tw64);
    int q = quarter;
    void* args[] = {&r, &o, &t, &q};
    switch (M) {
#define X(MM) case MM: return launch_common(k_spec_col<TO, MM>, blocks, threads, smem, st, args);
        TD_FOR_EACH_M(X)
#undef X
    }
    return hipErrorInvalidValue;
}

// Workgroups of kernel kf (threads, dynamic LDS smem) one CU holds at once,
// from its register count and LDS: 4 SIMDs of 512 VGPRs per lane and at
// most 8 waves each, 160 KiB of LDS.
template <typename KF>
static int occupancy(KF kf, int threads, size_t smem)
{
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(kf)) != hipSuccess) return 1;
    const int waves = (threads + 63) / 64, per_simd = (waves + 3) / 4;
    const int vgpr = std::max(8, (a.numRegs + 7) & ~7);
    const int by_regs = std::min(8, 512 / vgpr) / per_simd;
    const int by_lds = (int)((160u * 1024u) / std::max<size_t>(1, smem + a.sharedSizeBytes));
    return std::max(1, std::min(by_regs, by_lds));
}

int col_resident_blocks(bool f64, int M, int C, int G)
{
    const int threads = C * G * (M / 8);
    const size_t es = f64 ? sizeof(cpx<double>) : sizeof(cpx<float>);
    const size_t smem = col_lds_bytes(M, C, es, G);
    switch (M) {
#define X(MM) \
    case MM: return f64 ? occupancy(k_col<double, MM, true>, threads, smem) : occupancy(k_col<float, MM, true>, threads, smem);
        TD_FOR_EACH_M(X)
#undef X
    }
    return 1;
}

hipError_t launch_zero_counters(unsigned int* c, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    void* args[] = {&c, &n};
    return launch_common(k_zero_counters, std::min(64, (n + 255) / 256), 256, 0, st, args);
}

hipError_t launch_count_nonfinite(bool f64, const void* p, int64_t n, unsigned long long* counter,
                                  hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    const int blocks = (int)std::min<int64_t>((n + threads - 1) / threads, 1024);
    int64_t nn = n;
    unsigned long long* c = counter;
    if (f64) {
        const double* pp = static_cast<const double*>(p);
        void* args[] = {&pp, &nn, &c};
        return launch_common(k_count_nonfinite<double>, blocks, threads, 0, st, args);
    }
    const float* pp = static_cast<const float*>(p);
    void* args[] = {&pp, &nn, &c};
    return launch_common(k_count_nonfinite<float>, blocks, threads, 0, st, args);
}

hipError_t launch_table(const TableJob& job, hipStream_t st)
{
    const long long n = (long long)job.M * job.M;
    const int threads = 256;
    const int blocks = (int)((n + threads - 1) / threads);
    TableJob j = job;
    void* args[] = {&j};
    // the launch's own status (not the thread's last error, which an
    // unrelated earlier call may have left behind)
    return launch_common(k_table, blocks, threads, 0, st, args);
}

template hipError_t launch_row_fwd<float>(int, int, int, const SegTable<RowFwdJob>&,
                                          const void* const*, const FieldPtrs&, const void*, bool,
                                          hipStream_t);
template hipError_t launch_row_fwd<double>(int, int, int, const SegTable<RowFwdJob>&,
                                           const void* const*, const FieldPtrs&, const void*, bool,
                                           hipStream_t);
template hipError_t launch_col<float>(int, int, int, int, const SegTable<ColJob>&, const void*,
                                      hipStream_t, const JobQueue&);
template hipError_t launch_col<double>(int, int, int, int, const SegTable<ColJob>&, const void*,
                                       hipStream_t, const JobQueue&);
template hipError_t launch_row_inv<float>(int, int, int, int, const SegTable<RowInvJob>&,
                                          void* const*, const FieldPtrs&, const void*, hipStream_t, int);
template hipError_t launch_row_inv<double>(int, int, int, int, const SegTable<RowInvJob>&,
                                           void* const*, const FieldPtrs&, const void*, hipStream_t, int);
template hipError_t launch_spec_col<float>(int, int, const void*, void*, const void*, int,
                                           hipStream_t);
template hipError_t launch_spec_col<double>(int, int, const void*, void*, const void*, int,
                                            hipStream_t);

// ---------------------------------------------------------------------------
// Workspace of the allocation-free solve (td_solve_noalloc): one file-scope
// device array per GPU, held until the process ends.  Host code never uses
// the array's name as an address: its device address is looked up once per
// device (hipGetSymbolAddress, that device current) and cached here.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[TD_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[TD_NOALLOC_MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= TD_NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes it current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

// Raise the dynamic-LDS limit of every instantiation to the CU's 160 KiB,
// less a margin for what a kernel declares statically.
hipError_t prepare_kernels()
{
    const int lim = (int)TD_MAX_DYN_LDS;
    hipError_t e = hipSuccess;
#define SETA(k) if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, lim);
#define X(MM) SETA((k_row_fwd<float, MM, true>)) SETA((k_row_fwd<double, MM, true>)) \
    SETA((k_row_fwd<double, MM, false>)) \
    SETA((k_col<float, MM, false>)) SETA((k_col<double, MM, false>)) \
    SETA((k_col<float, MM, true>)) SETA((k_col<double, MM, true>)) \
    SETA((k_row_inv<float, MM, 4>)) SETA((k_row_inv<double, MM, 4>)) \
    SETA((k_row_inv<float, MM, 16>)) SETA((k_row_inv<double, MM, 16>)) \
    SETA((k_spec_col<float, MM>)) SETA((k_spec_col<double, MM>))
    TD_FOR_EACH_M(X)
#undef X
#undef SETA
    return e;
}

}  // namespace td
