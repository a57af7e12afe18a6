// Device passes of the thin-disk force solver (gfx950).
//
// Kernel tables: the cell integrals of Section 2.1 for every lattice offset
// and polyphase phase, built in FP64 with cancellation-free forms.
// Convolution: zero-padded 2-D FFTs along rows (real <-> half-complex,
// written / read transposed so that every spectral column is contiguous) and
// along columns (fused with the kernel-spectrum products), Section 2.2.
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

// Entry (nx, ny) of the six M x M tables of one phase.  The lattice offset
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
        cell_integrals(ua, ua + w, va, va + w, v);
        if (J.kind == 3) {
            const double inv = 1.0 / J.m;
            v[1] *= inv; v[2] *= inv; v[4] *= inv; v[5] *= inv;
        }
    }
    const size_t plane = (size_t)M * M;
#pragma unroll
    for (int X = 0; X < 6; ++X) J.out[X * plane + idx] = v[X];
}

// ---------------------------------------------------------------------------
// Pass 1: zero-padded real row FFTs, transposed write
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T fetch_src(const T* __restrict__ src, const RowFwdJob& J, int lr,
                                       int lc)
{
    const int srow = J.m * lr + J.row_off;
    const int scol = J.m * lc + J.col_off;
    if (srow < 0 || srow >= J.n_src || scol < 0 || scol >= J.n_src) return (T)0;
    if (scol >= J.cov_i0 && scol < J.cov_i1 && srow >= J.cov_j0 && srow < J.cov_j1) return (T)0;
    return (T)(J.scale * (double)src[(size_t)srow * J.n_src + scol]);
}

// C = blockDim/(M/8) complex sequences; sequence p carries stored rows
// row0 + 2p (real part) and row0 + 2p + 1 (imaginary part).
template <typename T, int M>
__global__ void __launch_bounds__(1024) k_row_fwd(SegTable<RowFwdJob> segs,
                                                  const void* const* __restrict__ ptrs,
                                                  const cpx<T>* __restrict__ tw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
    int slot_base;
    const void* aux;
    char* ws;
    const RowFwdJob J = segs.find(blockIdx.x, &slot_base, &aux, &ws);
    const int C = blockDim.x / (M / 8);
    const T* src = reinterpret_cast<const T*>(ptrs[slot_base + J.src_slot]);
    const int rend = J.row0 + J.nrow;
    for (int idx = threadIdx.x; idx < C * M; idx += blockDim.x) {
        const int p = idx / M, lc = idx % M;
        const int s0 = J.row0 + 2 * p;
        T a = 0, b = 0;
        if (src) {
            if (s0 < rend) a = fetch_src(src, J, J.lr_first + s0, lc);
            if (s0 + 1 < rend) b = fetch_src(src, J, J.lr_first + s0 + 1, lc);
        }
        buf[idx] = cpx<T>{a, b};
    }
    __syncthreads();
    fft_lds<T, M, false>(buf, tw);
    cpx<T>* out = reinterpret_cast<cpx<T>*>(ws + J.out);
    const int R = 2 * C;
    for (int idx = threadIdx.x; idx < (M / 2 + 1) * R; idx += blockDim.x) {
        const int r = idx % R, kx = idx / R;
        if (r >= J.nrow) continue;
        const int p = r >> 1;
        const cpx<T> z = buf[p * M + kx];
        const cpx<T> zc = conj(buf[p * M + ((M - kx) & (M - 1))]);
        cpx<T> X;
        if ((r & 1) == 0) {
            X = cpx<T>{(T)0.5 * (z.re + zc.re), (T)0.5 * (z.im + zc.im)};
        } else {
            const cpx<T> d = z - zc;  // (z - zc) / (2i)
            X = cpx<T>{(T)0.5 * d.im, (T)-0.5 * d.re};
        }
        out[(size_t)kx * J.ld + J.row0 + r] = X;
    }
}

// ---------------------------------------------------------------------------
// Kernel-spectrum lookup with the mirror symmetries of the phases
// ---------------------------------------------------------------------------

// Kernels X = 0..5: I0, Ixx, Ixy, J0, Jyy, Jyx.  Parity under x- and
// y-mirrors of the source cell about the target.
__device__ __constant__ int kSignX[6] = {-1, 1, -1, 1, 1, -1};
__device__ __constant__ int kSignY[6] = {1, 1, -1, -1, 1, -1};
// Kernel feeding output component c (0: Fx, 1: Fy) from field f (sigma,
// dsdx, dsdy).
__device__ __constant__ int kKernOf[2][3] = {{0, 1, 2}, {3, 5, 4}};

template <typename T, int M>
__device__ __forceinline__ cpx<T> kern_at(const cpx<T>* __restrict__ K, int X, int kx, int ky,
                                          int flip)
{
    const int kyy = (flip == 1 || flip == 2) ? ((M - ky) & (M - 1)) : ky;
    cpx<T> s = K[((size_t)X * (M / 2 + 1) + kx) * M + kyy];
    if (flip & 1) s.im = -s.im;
    int sg = 1;
    if (flip & 1) sg *= kSignX[X];
    if (flip & 2) sg *= kSignY[X];
    if (sg < 0) s = cpx<T>{-s.re, -s.im};
    return s;
}

// ---------------------------------------------------------------------------
// Pass 2: column FFT, kernel products summed over inputs, inverse column FFT
// ---------------------------------------------------------------------------

template <typename T, int M>
__global__ void __launch_bounds__(1024) k_col_gather(SegTable<ColGatherJob> segs,
                                                     const cpx<T>* __restrict__ tw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int C = blockDim.x / (M / 8);
    cpx<T>* ax = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* ay = ax + C * M;
    cpx<T>* in = ay + C * M;
    int slot_unused;
    const void* aux;
    char* ws;
    const ColGatherJob J = segs.find(blockIdx.x, &slot_unused, &aux, &ws);
    const ColTerm* __restrict__ terms = reinterpret_cast<const ColTerm*>(aux);
    for (int i = threadIdx.x; i < C * M; i += blockDim.x) {
        ax[i] = cpx<T>{0, 0};
        ay[i] = cpx<T>{0, 0};
    }
    for (int t = 0; t < J.nterm; ++t) {
        const ColTerm Tm = terms[J.term0 + t];
        const cpx<T>* K = reinterpret_cast<const cpx<T>*>(Tm.kern);
        for (int f = 0; f < 3; ++f) {
            if (Tm.in[f] < 0) continue;
            const cpx<T>* src = reinterpret_cast<const cpx<T>*>(ws + Tm.in[f]);
            for (int i = threadIdx.x; i < C * M; i += blockDim.x) {
                const int c = i / M, ky = i % M;
                const int s = ky - Tm.in_lr_first;
                cpx<T> v{0, 0};
                if (c < J.ncol && s >= 0 && s < Tm.in_ld)
                    v = src[(size_t)(J.kx0 + c) * Tm.in_ld + s];
                in[i] = v;
            }
            __syncthreads();
            fft_lds<T, M, false>(in, tw);
            const int Xx = kKernOf[0][f], Xy = kKernOf[1][f];
            for (int i = threadIdx.x; i < C * M; i += blockDim.x) {
                const int c = i / M, ky = i % M;
                if (c >= J.ncol) continue;
                const int kx = J.kx0 + c;
                const cpx<T> b = in[i];
                ax[i] = ax[i] + cmul(kern_at<T, M>(K, Xx, kx, ky, Tm.flip), b);
                ay[i] = ay[i] + cmul(kern_at<T, M>(K, Xy, kx, ky, Tm.flip), b);
            }
            __syncthreads();
        }
    }
    fft_lds<T, M, true>(ax, tw);
    fft_lds<T, M, true>(ay, tw);
    cpx<T>* ox = reinterpret_cast<cpx<T>*>(ws + J.out_x);
    cpx<T>* oy = reinterpret_cast<cpx<T>*>(ws + J.out_y);
    for (int i = threadIdx.x; i < C * J.out_ld; i += blockDim.x) {
        const int c = i / J.out_ld, s = i % J.out_ld;
        if (c >= J.ncol) continue;
        const size_t o = (size_t)(J.kx0 + c) * J.out_ld + s;
        ox[o] = ax[c * M + J.out_lr_first + s];
        oy[o] = ay[c * M + J.out_lr_first + s];
    }
}

// ---------------------------------------------------------------------------
// Pass 3: one input, many polyphase outputs (coarser source, finer target)
// ---------------------------------------------------------------------------

template <typename T, int M>
__global__ void __launch_bounds__(1024) k_col_scatter(SegTable<ColScatterJob> segs,
                                                      const cpx<T>* __restrict__ tw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int C = blockDim.x / (M / 8);
    cpx<T>* in0 = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* acc = in0 + 3 * C * M;
    int slot_unused;
    const void* aux;
    char* ws;
    const ColScatterJob J = segs.find(blockIdx.x, &slot_unused, &aux, &ws);
    const ColScatterOut* __restrict__ outs = reinterpret_cast<const ColScatterOut*>(aux);
    bool present[3];
    for (int f = 0; f < 3; ++f) {
        present[f] = J.in[f] >= 0;
        cpx<T>* dst = in0 + f * C * M;
        const cpx<T>* src = present[f] ? reinterpret_cast<const cpx<T>*>(ws + J.in[f]) : nullptr;
        for (int i = threadIdx.x; i < C * M; i += blockDim.x) {
            const int c = i / M, ky = i % M;
            const int s = ky - J.in_lr_first;
            cpx<T> v{0, 0};
            if (src && c < J.ncol && s >= 0 && s < J.in_ld) v = src[(size_t)(J.kx0 + c) * J.in_ld + s];
            dst[i] = v;
        }
    }
    __syncthreads();
    for (int f = 0; f < 3; ++f)
        if (present[f]) fft_lds<T, M, false>(in0 + f * C * M, tw);
    for (int o = 0; o < J.nout; ++o) {
        const ColScatterOut O = outs[J.out0 + o];
        const cpx<T>* K = reinterpret_cast<const cpx<T>*>(O.kern);
        for (int comp = 0; comp < 2; ++comp) {
            for (int i = threadIdx.x; i < C * M; i += blockDim.x) {
                const int c = i / M, ky = i % M;
                cpx<T> a{0, 0};
                if (c < J.ncol) {
                    const int kx = J.kx0 + c;
                    for (int f = 0; f < 3; ++f)
                        if (present[f])
                            a = a + cmul(kern_at<T, M>(K, kKernOf[comp][f], kx, ky, O.flip),
                                         in0[f * C * M + i]);
                }
                acc[i] = a;
            }
            __syncthreads();
            fft_lds<T, M, true>(acc, tw);
            cpx<T>* dst = reinterpret_cast<cpx<T>*>(ws + (comp == 0 ? O.out_x : O.out_y));
            for (int i = threadIdx.x; i < C * O.out_ld; i += blockDim.x) {
                const int c = i / O.out_ld, s = i % O.out_ld;
                if (c >= J.ncol) continue;
                dst[(size_t)(J.kx0 + c) * O.out_ld + s] = acc[c * M + O.out_lr_first + s];
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 4: complex-to-real row FFTs, window / phase extraction, accumulation
// ---------------------------------------------------------------------------

__device__ __forceinline__ int floor_div(int a, int b)
{
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

template <typename T, int M>
__global__ void __launch_bounds__(1024) k_row_inv(SegTable<RowInvJob> segs,
                                                  void* const* __restrict__ ptrs,
                                                  const cpx<T>* __restrict__ tw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
    const int C = blockDim.x / (M / 8);  // rows of this job
    int slot_base;
    const void* aux;
    char* ws;
    const RowInvJob J = segs.find(blockIdx.x, &slot_base, &aux, &ws);
    const RowInvContrib* __restrict__ contribs = reinterpret_cast<const RowInvContrib*>(aux);
    constexpr int NQ = 16;  // up to C * 2M outputs over C * (M/8) threads (target n <= 2M)
    T accx[NQ], accy[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) { accx[q] = 0; accy[q] = 0; }
    const int nout = J.ny * J.nx;
    for (int k = 0; k < J.nc; ++k) {
        const RowInvContrib Q = contribs[J.c0 + k];
        const cpx<T>* base = reinterpret_cast<const cpx<T>*>(ws + Q.base);
        for (int kxp = 0; kxp < Q.m; ++kxp) {
            for (int i = threadIdx.x; i < C * (M / 2 + 1); i += blockDim.x) {
                const int r = i % C, kx = i / C;
                cpx<T> z{0, 0}, zr{0, 0};
                if (r < J.ny) {
                    const int g = J.oy_t + J.y0 + r;
                    const int Jc = floor_div(g, Q.m);
                    const int kyp = g - Jc * Q.m;
                    const int sr = Jc - Q.oy_s - Q.lr_first;
                    const cpx<T>* P = base + (size_t)(kyp * Q.m + kxp) * Q.phase_stride;
                    cpx<T> X = P[(size_t)kx * Q.ld + sr];
                    cpx<T> Y = P[Q.comp_stride + (size_t)kx * Q.ld + sr];
                    if (kx == 0 || kx == M / 2) { X.im = 0; Y.im = 0; }
                    z = cpx<T>{X.re - Y.im, X.im + Y.re};
                    zr = cpx<T>{X.re + Y.im, Y.re - X.im};
                }
                buf[r * M + kx] = z;
                if (kx > 0 && kx < M / 2) buf[r * M + M - kx] = zr;
            }
            __syncthreads();
            fft_lds<T, M, true>(buf, tw);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int idx = threadIdx.x + q * blockDim.x;
                if (idx >= nout) continue;
                const int r = idx / J.nx, ii = J.x0 + idx % J.nx;
                const int g = J.ox_t + ii;
                const int Ic = floor_div(g, Q.m);
                if (g - Ic * Q.m != kxp) continue;
                const cpx<T> v = buf[r * M + (Ic - Q.ox_s)];
                accx[q] += v.re;
                accy[q] += v.im;
            }
            __syncthreads();
        }
    }
    T* fx = reinterpret_cast<T*>(ptrs[slot_base + J.out_slot]);
    T* fy = reinterpret_cast<T*>(ptrs[slot_base + J.out_slot + 1]);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int idx = threadIdx.x + q * blockDim.x;
        if (idx >= nout) continue;
        const int r = idx / J.nx, ii = J.x0 + idx % J.nx;
        const int row = J.y0 + r;
        const bool cov = ii >= J.cov_i0 && ii < J.cov_i1 && row >= J.cov_j0 && row < J.cov_j1;
        const size_t o = (size_t)row * J.n_t + ii;
        if (!J.accumulate) {
            if (fx) fx[o] = cov ? (T)0 : accx[q];
            if (fy) fy[o] = cov ? (T)0 : accy[q];
        } else if (!cov) {
            if (fx) fx[o] += accx[q];
            if (fy) fy[o] += accy[q];
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel-spectrum build: column FFT of the row-transformed FP64 tables,
// scaled by 1/M^2 (both inverse transforms are unnormalised) and stored in T.
// ---------------------------------------------------------------------------

template <typename TO, int M>
__global__ void __launch_bounds__(1024) k_spec_col(const cpx<double>* __restrict__ rows,
                                                   cpx<TO>* __restrict__ out,
                                                   const cpx<double>* __restrict__ tw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<double>* buf = reinterpret_cast<cpx<double>*>(smem_raw);
    const int C = blockDim.x / (M / 8);
    constexpr int NCOL = M / 2 + 1;
    const int per_x = (NCOL + C - 1) / C;
    const int X = blockIdx.x / per_x;
    const int kx0 = (blockIdx.x % per_x) * C;
    for (int i = threadIdx.x; i < C * M; i += blockDim.x) {
        const int c = i / M, ky = i % M;
        cpx<double> v{0, 0};
        if (kx0 + c < NCOL) v = rows[((size_t)X * NCOL + kx0 + c) * M + ky];
        buf[i] = v;
    }
    __syncthreads();
    fft_lds<double, M, false>(buf, tw);
    const double sc = 1.0 / ((double)M * (double)M);
    for (int i = threadIdx.x; i < C * M; i += blockDim.x) {
        const int c = i / M, ky = i % M;
        if (kx0 + c >= NCOL) continue;
        const cpx<double> v = buf[i];
        out[((size_t)X * NCOL + kx0 + c) * M + ky] = cpx<TO>{(TO)(v.re * sc), (TO)(v.im * sc)};
    }
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
                          const void* const* ptrs, const void* tw, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    const int threads = C * (M / 8);
    const size_t smem = (size_t)C * M * sizeof(cpx<T>);
    SegTable<RowFwdJob> s = segs;
    const void* const* p = ptrs;
    const cpx<T>* t = reinterpret_cast<const cpx<T>*>(tw);
    void* args[] = {&s, &p, &t};
    switch (M) {
#define X(MM) case MM: return launch_common(k_row_fwd<T, MM>, blocks, threads, smem, st, args);
        TD_FOR_EACH_M(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_col_gather(int M, int C, int blocks, const SegTable<ColGatherJob>& segs,
                             const void* tw, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    const int threads = C * (M / 8);
    const size_t smem = (size_t)3 * C * M * sizeof(cpx<T>);
    SegTable<ColGatherJob> s = segs;
    const cpx<T>* t = reinterpret_cast<const cpx<T>*>(tw);
    void* args[] = {&s, &t};
    switch (M) {
#define X(MM) case MM: return launch_common(k_col_gather<T, MM>, blocks, threads, smem, st, args);
        TD_FOR_EACH_M(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_col_scatter(int M, int C, int blocks, const SegTable<ColScatterJob>& segs,
                              const void* tw, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    const int threads = C * (M / 8);
    const size_t smem = (size_t)4 * C * M * sizeof(cpx<T>);
    SegTable<ColScatterJob> s = segs;
    const cpx<T>* t = reinterpret_cast<const cpx<T>*>(tw);
    void* args[] = {&s, &t};
    switch (M) {
#define X(MM) case MM: return launch_common(k_col_scatter<T, MM>, blocks, threads, smem, st, args);
        TD_FOR_EACH_M(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_row_inv(int M, int C, int blocks, const SegTable<RowInvJob>& segs,
                          void* const* ptrs, const void* tw, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    const int threads = C * (M / 8);
    const size_t smem = (size_t)C * M * sizeof(cpx<T>);
    SegTable<RowInvJob> s = segs;
    void* const* p = ptrs;
    const cpx<T>* t = reinterpret_cast<const cpx<T>*>(tw);
    void* args[] = {&s, &p, &t};
    switch (M) {
#define X(MM) case MM: return launch_common(k_row_inv<T, MM>, blocks, threads, smem, st, args);
        TD_FOR_EACH_M(X)
#undef X
    }
    return hipErrorInvalidValue;
}

template <typename TO>
hipError_t launch_spec_col(int M, int C, const void* rows, void* out, const void* tw64,
                           hipStream_t st)
{
    const int threads = C * (M / 8);
    const int per_x = (M / 2 + 1 + C - 1) / C;
    const int blocks = 6 * per_x;
    const size_t smem = (size_t)C * M * sizeof(cpx<double>);
    const cpx<double>* r = reinterpret_cast<const cpx<double>*>(rows);
    cpx<TO>* o = reinterpret_cast<cpx<TO>*>(out);
    const cpx<double>* t = reinterpret_cast<const cpx<double>*>(tw64);
    void* args[] = {&r, &o, &t};
    switch (M) {
#define X(MM) case MM: return launch_common(k_spec_col<TO, MM>, blocks, threads, smem, st, args);
        TD_FOR_EACH_M(X)
#undef X
    }
    return hipErrorInvalidValue;
}

hipError_t launch_table(const TableJob& job, hipStream_t st)
{
    const long long n = (long long)job.M * job.M;
    const int threads = 256;
    const int blocks = (int)((n + threads - 1) / threads);
    hipLaunchKernelGGL(k_table, dim3(blocks), dim3(threads), 0, st, job);
    return hipGetLastError();
}

template hipError_t launch_row_fwd<float>(int, int, int, const SegTable<RowFwdJob>&,
                                          const void* const*, const void*, hipStream_t);
template hipError_t launch_row_fwd<double>(int, int, int, const SegTable<RowFwdJob>&,
                                           const void* const*, const void*, hipStream_t);
template hipError_t launch_col_gather<float>(int, int, int, const SegTable<ColGatherJob>&,
                                             const void*, hipStream_t);
template hipError_t launch_col_gather<double>(int, int, int, const SegTable<ColGatherJob>&,
                                              const void*, hipStream_t);
template hipError_t launch_col_scatter<float>(int, int, int, const SegTable<ColScatterJob>&,
                                              const void*, hipStream_t);
template hipError_t launch_col_scatter<double>(int, int, int, const SegTable<ColScatterJob>&,
                                               const void*, hipStream_t);
template hipError_t launch_row_inv<float>(int, int, int, const SegTable<RowInvJob>&,
                                          void* const*, const void*, hipStream_t);
template hipError_t launch_row_inv<double>(int, int, int, const SegTable<RowInvJob>&,
                                           void* const*, const void*, hipStream_t);
template hipError_t launch_spec_col<float>(int, int, const void*, void*, const void*,
                                           hipStream_t);
template hipError_t launch_spec_col<double>(int, int, const void*, void*, const void*,
                                            hipStream_t);

// Raise the dynamic-LDS limit of every instantiation to the CU's 160 KiB.
hipError_t prepare_kernels()
{
    const int lim = 160 * 1024;
    hipError_t e = hipSuccess;
#define SETA(k) if (e == hipSuccess) e = hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, lim);
#define X(MM) SETA((k_row_fwd<float, MM>)) SETA((k_row_fwd<double, MM>)) \
    SETA((k_col_gather<float, MM>)) SETA((k_col_gather<double, MM>)) \
    SETA((k_col_scatter<float, MM>)) SETA((k_col_scatter<double, MM>)) \
    SETA((k_row_inv<float, MM>)) SETA((k_row_inv<double, MM>)) \
    SETA((k_spec_col<float, MM>)) SETA((k_spec_col<double, MM>))
    TD_FOR_EACH_M(X)
#undef X
#undef SETA
    return e;
}

}  // namespace td
