// Batched LDS-resident Stockham FFTs for gfx950.
//
// A workgroup transforms C independent sequences of length M (a power of two,
// 16 <= M <= 4096) that sit in LDS lds_stride(M) elements apart.  The
// workgroup has exactly C*(M/8) threads; in every pass each thread holds
// eight complex values in registers: one radix-8 butterfly, two radix-4
// butterflies or four radix-2 butterflies.  Every pass reads its operands,
// synchronises, and writes them back permuted (Stockham autosort), so a
// single LDS buffer per sequence suffices and the result is in natural order.
// Zero-padded inputs (upper half zero) skip that half in the first pass, and
// transforms of which only the lower half is wanted skip it in the last.
//
// Forward: X[k] = sum_n x[n] exp(-2 pi i k n / M); inverse uses +i and is
// unnormalised.  Twiddles come from a table computed on the host in long
// double and staged in LDS, laid out per pass so that the lanes of a
// wavefront read consecutive entries (no bank conflicts): the radix-8 pass
// of span NS finds exp(-2 pi i r k / (8 NS)) at tw_offset(M, NS) +
// (r - 1) NS + k, r = 1..7, k < NS.  The table has fewer than M entries.
//
// Synchronisation: with M/8 <= 64 a sequence lives in one wavefront, whose
// LDS operations complete in order, so the passes only need a wave-level
// ordering point and the slots of a workgroup run independently; longer
// sequences span several wavefronts and use workgroup barriers.  fft_lds
// returns with the sequence ordered for its own wavefront(s) only: a caller
// that then reads another wavefront's sequence must __syncthreads() first.
//
// LDS layout: element i of a sequence is stored at lds_pos(i) = i + i/P,
// with one padding element per P = 16 (FP32) or 8 (FP64) elements;
// sequences are lds_stride(M) = M + M/8 elements apart.  The LDS serves an
// 8-byte access to 16 lanes per cycle (a 16-byte one to 8), so the lanes of
// a cycle are conflict-free when their elements differ modulo 16 (modulo 8).
// FP32 with P = 16 makes every read, and the stores of spans 1 and >= 16,
// conflict-free, but not the stores of spans 2-8: those passes store with
// P = 8 (and the next pass reads that layout), which needs the M/8 padding
// of the stride.  (Measured: P = 8 throughout cost FP32 about 3.6
// bank-conflict cycles per LDS instruction.)  FP64 uses P = 8 throughout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace td {

template <typename T>
__host__ __device__ constexpr int lds_pad() { return sizeof(T) == 4 ? 16 : 8; }
template <typename T>
__host__ __device__ constexpr int lds_stride(int M) { return M + M / 8; }
template <int P>
__device__ __forceinline__ int lds_pos_p(int i) { return i + i / P; }  // i >= 0
template <typename T>
__device__ __forceinline__ int lds_pos(int i) { return lds_pos_p<lds_pad<T>()>(i); }

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T r, T i) { return cpx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b)
{
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> rot_i(cpx<T> a)
{
    return INV ? cpx<T>{-a.im, a.re} : cpx<T>{a.im, -a.re};
}

// Butterflies.  ZIN: the upper half of the inputs, v[R/2 .. R-1], is zero
// (not read); ZOUT: only the lower half of the outputs, v[0 .. R/2-1], is
// wanted (the rest is left undefined).
template <typename T, bool INV, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void dft2(cpx<T>* v)
{
    if constexpr (ZIN) {
        v[1] = v[0];
    } else {
        cpx<T> a = v[0], b = v[1];
        v[0] = a + b;
        if constexpr (!ZOUT) v[1] = a - b;
    }
}

template <typename T, bool INV, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void dft4(cpx<T>* v)
{
    cpx<T> s02, d02, s13, d13;
    if constexpr (ZIN) {
        s02 = d02 = v[0];
        s13 = v[1];
        d13 = rot_i<T, INV>(v[1]);
    } else {
        s02 = v[0] + v[2];
        d02 = v[0] - v[2];
        s13 = v[1] + v[3];
        d13 = rot_i<T, INV>(v[1] - v[3]);
    }
    v[0] = s02 + s13;
    v[1] = d02 + d13;
    if constexpr (!ZOUT) {
        v[2] = s02 - s13;
        v[3] = d02 - d13;
    }
}

template <typename T, bool INV, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void dft8(cpx<T>* v)
{
    cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<T, INV, ZIN>(e);
    dft4<T, INV, ZIN>(o);
    const T h = (T)0.70710678118654752440084436210484903928;
    // o[k] *= w8^k,  w8 = exp(-+ i pi/4)
    o[1] = INV ? cpx<T>{h * (o[1].re - o[1].im), h * (o[1].re + o[1].im)}
               : cpx<T>{h * (o[1].re + o[1].im), h * (o[1].im - o[1].re)};
    o[2] = rot_i<T, INV>(o[2]);
    o[3] = INV ? cpx<T>{-h * (o[3].re + o[3].im), h * (o[3].re - o[3].im)}
               : cpx<T>{h * (o[3].im - o[3].re), -h * (o[3].re + o[3].im)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = e[k] + o[k];
        if constexpr (!ZOUT) v[k + 4] = e[k] - o[k];
    }
}

template <typename T, int R, bool INV, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void dftR(cpx<T>* v)
{
    if constexpr (R == 2) dft2<T, INV, ZIN, ZOUT>(v);
    else if constexpr (R == 4) dft4<T, INV, ZIN, ZOUT>(v);
    else dft8<T, INV, ZIN, ZOUT>(v);
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Span of the first radix-8 pass with twiddles: after a radix-2 / radix-4
// pass when log2(M) is not a multiple of 3, else after the first radix-8
// pass (span 1, no twiddles).
constexpr int tw_first_span(int M) { return ilog2(M) % 3 == 0 ? 8 : (1 << (ilog2(M) % 3)); }

// Offset of the radix-8 pass of span NS in the twiddle table.
constexpr int tw_offset(int M, int NS)
{
    int off = 0;
    for (int s = tw_first_span(M); s < NS; s *= 8) off += 7 * s;
    return off;
}

// Ordering point between the passes of one sequence (see above).
template <int M>
__device__ __forceinline__ void seq_sync()
{
    if constexpr (M / 8 <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// One Stockham pass of radix R at span NS on sequence x (length M), for the
// calling thread's `lane` in [0, M/8); it reads the layout of padding PR and
// writes that of padding PW.  In the first pass (NS == 1) a butterfly's
// inputs r >= R/2 are the elements >= M/2, so ZIN (those elements are zero)
// skips them; in the last (NS R == M) its outputs r >= R/2 land at >= M/2,
// so ZOUT (only elements < M/2 are wanted) does not form or store them.
//
// Register ends: the inputs of a thread's butterflies in the first pass,
// elements j + r M/R with j = lane + q M/8, are the elements lane + k M/8
// (k = q + r 8/R), and the outputs of its one radix-8 butterfly in the last
// pass are again lane + r M/8.  FROMR takes the first pass's inputs from
// vr[k] instead of LDS (or a later radix-8 pass's, elements lane + r M/8 of
// the array that pass reads: see fft_regs_band); TOR leaves the last pass's outputs in vr[r] instead
// of storing them (and ends without the closing ordering point: the one
// after its reads already orders them before any later write).
//
// Ping-pong (PP): the pass reads x and writes y, a second buffer of the
// sequence, so no thread can overwrite what another has yet to read and
// the ordering point after the reads is dropped -- except in a TOR pass,
// whose reads must complete before the next transform's first pass writes
// its buffer again.
template <typename T, int M, int R, int NS, bool INV, int PR, int PW, bool ZIN = false,
          bool ZOUT = false, bool FROMR = false, bool TOR = false, bool PP = false>
__device__ __forceinline__ void stockham_pass(cpx<T>* x, const cpx<T>* __restrict__ tw, int lane,
                                              cpx<T>* vr = nullptr, cpx<T>* y = nullptr)
{
    static_assert(!ZIN || NS == 1, "ZIN applies to the first pass");
    static_assert(!ZOUT || NS * R == M, "ZOUT applies to the last pass");
    static_assert(!FROMR || NS == 1 || R == 8, "FROMR applies to the first pass (or a radix-8 one)");
    static_assert(!TOR || (NS * R == M && R == 8), "TOR applies to the last (radix-8) pass");
    constexpr int B = 8 / R;          // butterflies per thread
    constexpr int STRIDE = M / R;     // distance between butterfly inputs
    constexpr int RIN = ZIN ? R / 2 : R, ROUT = ZOUT ? R / 2 : R;
    // For M >= 64 every read of a thread sits at a compile-time offset from
    // its first position, and every write of a butterfly at offset
    // r NS + (r NS)/PW from lds_pos(base): one address per thread and
    // butterfly, the rest immediate offsets.  (The offsets c are multiples of
    // PR, or of 8 with lane < 8 when M = 64, and base % PW + (r NS) % PW < PW
    // in every pass, so the padding splits over the sum.)
    constexpr bool LIN = M >= 64;
    cpx<T> v[B][R];
    if constexpr (FROMR) {
#pragma unroll
        for (int q = 0; q < B; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = r < RIN ? vr[q + r * B] : cpx<T>{0, 0};
    } else if constexpr (LIN) {
        const cpx<T>* rp = x + lds_pos_p<PR>(lane);
#pragma unroll
        for (int q = 0; q < B; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int c = q * (M / 8) + r * STRIDE;
                v[q][r] = r < RIN ? rp[c + c / PR] : cpx<T>{0, 0};
            }
    } else {
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const int j = lane + q * (M / 8);
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[q][r] = r < RIN ? x[lds_pos_p<PR>(j + r * STRIDE)] : cpx<T>{0, 0};
        }
    }
    if constexpr (!PP || TOR) seq_sync<M>();
    cpx<T>* const out = PP ? y : x;
#pragma unroll
    for (int q = 0; q < B; ++q) {
        const int j = lane + q * (M / 8);
        const int k = (NS == 1) ? 0 : (j % NS);
        if constexpr (NS > 1) {
            static_assert(R == 8, "only radix-8 passes carry twiddles");
            const cpx<T>* tp = tw + tw_offset(M, NS) + k;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cpx<T> w = tp[(r - 1) * NS];
                v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
            }
        }
        dftR<T, R, INV, ZIN, ZOUT>(v[q]);
        const int base = (j / NS) * NS * R + k;
        if constexpr (TOR) {
#pragma unroll
            for (int r = 0; r < ROUT; ++r) vr[r] = v[q][r];
        } else if constexpr (LIN) {
            cpx<T>* wp = out + lds_pos_p<PW>(base);
#pragma unroll
            for (int r = 0; r < ROUT; ++r) wp[r * NS + (r * NS) / PW] = v[q][r];
        } else {
#pragma unroll
            for (int r = 0; r < ROUT; ++r) out[lds_pos_p<PW>(base + r * NS)] = v[q][r];
        }
    }
    if constexpr (!TOR) seq_sync<M>();
}

// Padding of the layout a pass of span NS writes: FP32 stores of spans 2-8
// that another pass reads use 8, every other store the type's padding.
template <typename T, int M, int NS>
__host__ __device__ constexpr int pass_pad()
{
    return (sizeof(T) == 4 && NS >= 2 && NS <= 8 && NS * 8 < M) ? 8 : lds_pad<T>();
}

// The radix-8 passes from span NS on.  FROMR: the first of them takes its
// inputs from vr.  PP: each pass reads x and writes y; the next pass reads
// y and writes x.
template <typename T, int M, int NS, bool INV, int PR, bool ZIN, bool ZOUT, bool FROMR = false,
          bool TOR = false, bool PP = false>
__device__ __forceinline__ void radix8_passes(cpx<T>* x, const cpx<T>* __restrict__ tw, int lane,
                                              cpx<T>* vr = nullptr, cpx<T>* y = nullptr)
{
    if constexpr (NS < M) {
        constexpr int PW = pass_pad<T, M, NS>();
        stockham_pass<T, M, 8, NS, INV, PR, PW, ZIN && NS == 1, ZOUT && NS * 8 == M, FROMR,
                      TOR && NS * 8 == M, PP>(x, tw, lane, vr, y);
        if constexpr (PP)
            radix8_passes<T, M, NS * 8, INV, PW, ZIN, ZOUT, false, TOR, PP>(y, tw, lane, vr, x);
        else
            radix8_passes<T, M, NS * 8, INV, PW, ZIN, ZOUT, false, TOR>(x, tw, lane, vr);
    }
}

// Transform sequence `f = threadIdx.x / (M/8)` of the C sequences at buf
// (padded layout).  ZIN: elements M/2 .. M-1 of the input are zero and are
// not read (a zero-padded sequence); ZOUT: only elements 0 .. M/2-1 of the
// result are wanted, the others are left stale.
// Must be called by every thread of the workgroup (it synchronises).
//
// The thread index goes through an empty asm barrier: in a kernel that
// calls fft_lds inside a loop, every LDS address and twiddle of every pass
// is loop-invariant, and hoisting them all out of the loop would hold them
// in registers for its whole length (tens of VGPRs, halving occupancy).
template <typename T, int M, bool INV, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void fft_lds(cpx<T>* buf, const cpx<T>* __restrict__ tw)
{
    static_assert(M >= 16 && (M & (M - 1)) == 0, "M must be a power of two >= 16");
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int f = tid / (M / 8);
    const int lane = tid % (M / 8);
    cpx<T>* x = buf + (size_t)f * lds_stride<T>(M);
    constexpr int REM = ilog2(M) % 3;
    constexpr int P = lds_pad<T>();  // the layout in and out
    if constexpr (REM == 1) {
        stockham_pass<T, M, 2, 1, INV, P, P, ZIN>(x, tw, lane);
        radix8_passes<T, M, 2, INV, P, false, ZOUT>(x, tw, lane);
    } else if constexpr (REM == 2) {
        stockham_pass<T, M, 4, 1, INV, P, P, ZIN>(x, tw, lane);
        radix8_passes<T, M, 4, INV, P, false, ZOUT>(x, tw, lane);
    } else {
        radix8_passes<T, M, 1, INV, P, ZIN, ZOUT>(x, tw, lane);
    }
}

// fft_lds with register ends: the calling thread's elements lane + k M/8
// (k < 8) of its sequence (f = threadIdx.x / (M/8)) come in and go out in
// v[k]; only the middle passes use the sequence's LDS.  With ZIN, v[4..7]
// are not read; with ZOUT, only v[0..3] are formed.  Must be called by every
// thread of the workgroup; on return the sequence's LDS may be written
// again by any of its threads.
//
// buf2 != nullptr: ping-pong between the sequence's LDS buffer and a second
// one at the same offset from buf2 (one ordering point per pass instead of
// two; for sequences that span several wavefronts, where each ordering
// point is a workgroup barrier).
template <typename T, int M, bool INV, bool ZIN = false, bool ZOUT = false, bool PP = false>
__device__ __forceinline__ void fft_regs(cpx<T> (&v)[8], cpx<T>* buf, const cpx<T>* __restrict__ tw,
                                         cpx<T>* buf2 = nullptr)
{
    static_assert(M >= 16 && (M & (M - 1)) == 0, "M must be a power of two >= 16");
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int f = tid / (M / 8);
    const int lane = tid % (M / 8);
    cpx<T>* x = buf + (size_t)f * lds_stride<T>(M);
    cpx<T>* y = PP ? buf2 + (size_t)f * lds_stride<T>(M) : nullptr;
    constexpr int REM = ilog2(M) % 3;
    constexpr int P = lds_pad<T>();
    if constexpr (REM == 1) {
        stockham_pass<T, M, 2, 1, INV, P, P, ZIN, false, true, false, PP>(x, tw, lane, v, y);
        if constexpr (PP)
            radix8_passes<T, M, 2, INV, P, false, ZOUT, false, true, PP>(y, tw, lane, v, x);
        else radix8_passes<T, M, 2, INV, P, false, ZOUT, false, true>(x, tw, lane, v);
    } else if constexpr (REM == 2) {
        stockham_pass<T, M, 4, 1, INV, P, P, ZIN, false, true, false, PP>(x, tw, lane, v, y);
        if constexpr (PP)
            radix8_passes<T, M, 4, INV, P, false, ZOUT, false, true, PP>(y, tw, lane, v, x);
        else radix8_passes<T, M, 4, INV, P, false, ZOUT, false, true>(x, tw, lane, v);
    } else {
        radix8_passes<T, M, 1, INV, P, ZIN, ZOUT, true, true, PP>(x, tw, lane, v, y);
    }
}

// Band-limited forward transforms.  After the passes up to span S, element
// c S + k (c < D = M/S, k < S) of a sequence holds
//   sum_u x[c + u D] w_S^(u k),   u < S,  w_S = exp(-2 pi i / S),
// the length-S DFT of the elements congruent to c mod D.  When x is
// non-zero only on D cyclically consecutive elements, each class c holds
// at most one of them, x[n] with n = c (mod D), and the sum is that one
// term, x[n] w_S^(k (n div D)).  A transform of such an input can then
// start at span S from values formed directly from x: fft_regs_band starts
// at the span that the first radix-8 pass reaches, which saves that pass
// and the radix-2/4 one before it, with their LDS traffic and ordering
// points.  At least two passes must remain (the register-ended last one
// and one before it).
constexpr int band_span(int M) { return ilog2(M) % 3 == 0 ? 8 : 8 * tw_first_span(M); }
constexpr bool band_ok(int M) { return band_span(M) * 8 < M; }

// Forward transform with register ends (as fft_regs) of a band-limited
// sequence: v[r] comes in holding element lane + r M/8 of the span-S array
// above (S = band_span(M)), and goes out holding element lane + r M/8 of the
// transform.  Every thread of the workgroup must call it (or, with
// M/8 <= 64, every thread of the sequence's wavefront).  With ping-pong
// (buf2) the first remaining pass writes the second buffer, as the first
// pass of fft_regs does, so the two kinds of transform can follow each
// other on one sequence.
template <typename T, int M, bool PP = false>
__device__ __forceinline__ void fft_regs_band(cpx<T> (&v)[8], cpx<T>* buf, const cpx<T>* __restrict__ tw,
                                              cpx<T>* buf2 = nullptr)
{
    static_assert(band_ok(M), "band transforms need two passes after the band span");
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int f = tid / (M / 8);
    const int lane = tid % (M / 8);
    cpx<T>* x = buf + (size_t)f * lds_stride<T>(M);
    cpx<T>* y = PP ? buf2 + (size_t)f * lds_stride<T>(M) : nullptr;
    radix8_passes<T, M, band_span(M), false, lds_pad<T>(), false, false, true, true, PP>(x, tw, lane, v, y);
}

}  // namespace td
