// Launch interface between the host planner and the device passes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "td_jobs.h"

namespace td {

// A launch processes the concatenated job lists of up to TD_MAX_SEGS plans
// (one workgroup per job).  Each segment carries the pointer-table slot base
// of its solve and an auxiliary per-plan table (column inputs and outputs,
// or row contributions).  Passed by value as a kernel argument.
#define TD_MAX_SEGS 40

// Copy a read-only descriptor (tab[i]) through a constant-address-space
// pointer, dword by dword: with an index that is uniform over the
// wavefront the loads are scalar and the fields land in scalar registers.
template <typename D>
__device__ __forceinline__ D load_const(const D* tab, int i)
{
    static_assert(sizeof(D) % 4 == 0, "descriptor size");
    typedef const __attribute__((address_space(4))) uint32_t* cwords;
    cwords w = (cwords)(tab + i);
    uint32_t buf[sizeof(D) / 4];
#pragma unroll
    for (int k = 0; k < (int)(sizeof(D) / 4); ++k) buf[k] = w[k];
    D d;
    __builtin_memcpy(&d, buf, sizeof(D));
    return d;
}

template <typename Job>
struct SegTable {
    int32_t nseg;
    int32_t start[TD_MAX_SEGS + 1];  // first block of each segment; start[nseg] = total
    int32_t slot_base[TD_MAX_SEGS];
    const Job* jobs[TD_MAX_SEGS];
    const void* aux[TD_MAX_SEGS];
    char* ws[TD_MAX_SEGS];            // workspace base of the segment's solve

    __device__ __forceinline__ Job find(int block, int* slot, const void** aux_out,
                                        char** ws_out) const
    {
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= block) lo = mid;
            else hi = mid - 1;
        }
        *slot = slot_base[lo];
        *aux_out = aux[lo];
        *ws_out = ws[lo];
        // job tables are read-only while a launch runs and the index is the
        // same for the whole workgroup: a constant-address-space load, so
        // the descriptor lands in scalar registers
        return load_const(jobs[lo], block - start[lo]);
    }
};

// Field pointers of a launch: by value in the kernel arguments (n > 0, one
// solve of up to TD_MAX_PATCHES patches: 5 per patch -- sigma, dsdx, dsdy,
// fx, fy) or, for batches, in a device table (n == 0).  A slope slot whose
// bit 0 is set holds the patch's sigma pointer (bit cleared): the slope is
// estimated from sigma instead of read.
#define TD_KARG_PTRS 40
struct FieldPtrs {
    int32_t n;
    int32_t pad;
    void* p[TD_KARG_PTRS];
};

// Persistent column launches: the workgroups of a grid pull their jobs from
// per-XCD work lists instead of each running job blockIdx.x.  List l holds
// job indices of the launch's SegTable at order[start[l] .. start[l+1]);
// workgroup b serves list b % TD_NXCD first (workgroups are dispatched to
// the XCDs round-robin, so a list's jobs share one L2), then the others.
// counter[l] is list l's next position; the counters must be zero when the
// launch starts (launch_zero_counters).  order == nullptr: a direct launch.
#define TD_NXCD 8
struct JobQueue {
    const int32_t* order;
    const int32_t* start;   // [TD_NXCD + 1]
    unsigned int* counter;  // [TD_NXCD]
};

// Row inverse: nq = the most outputs per thread and row of any job of the
// launch, ceil(nx / (G M/8)) <= 16.
// padded: the solve's zero-padded rows (only lattice columns < M/2 can be
// non-zero); false: full-length rows (the kernel tables, FP64 only).
// blocks: the grid (direct launches: one workgroup per job).
template <typename T>
hipError_t launch_row_fwd(int M, int C, int blocks, const SegTable<RowFwdJob>& segs,
                          const void* const* ptrs, const FieldPtrs& fp, const void* tw,
                          bool padded, hipStream_t st);
template <typename T>
hipError_t launch_col(int M, int C, int G, int blocks, const SegTable<ColJob>& segs,
                      const void* tw, hipStream_t st, const JobQueue& queue = JobQueue{});
template <typename T>
hipError_t launch_row_inv(int M, int C, int G, int blocks, const SegTable<RowInvJob>& segs,
                          void* const* ptrs, const FieldPtrs& fp, const void* tw, hipStream_t st,
                          int nq);
// Column-pass workgroups of a launch shape that one CU holds at once, for
// sizing persistent grids.
int col_resident_blocks(bool f64, int M, int C, int G);
// Zero n work-list counters on stream st.
hipError_t launch_zero_counters(unsigned int* c, int n, hipStream_t st);
// quarter: bit 0 = quarter-real layout (same-level spectra), bit 1 = the
// potential kernel family (its parities decide real vs imaginary planes)
template <typename TO>
hipError_t launch_spec_col(int M, int C, const void* rows, void* out, const void* tw64,
                           int quarter, hipStream_t st);
hipError_t launch_table(const TableJob& job, hipStream_t st);
// Add the number of non-finite values of p[0 .. n) to *counter (debug mode).
hipError_t launch_count_nonfinite(bool f64, const void* p, int64_t n, unsigned long long* counter,
                                  hipStream_t st);

// Lift the dynamic-LDS cap of every pass instantiation (call once per device).
hipError_t prepare_kernels();

// The allocation-free solve's workspace: a device array of
// TD_NOALLOC_SCRATCH_BYTES per GPU (see td_solve_noalloc).  noalloc_scratch
// returns its device address on `device`, which must be the current device
// (looked up there once, then cached).
#ifndef TD_NOALLOC_SCRATCH_BYTES
#define TD_NOALLOC_SCRATCH_BYTES (32u << 20)
#endif
#define TD_NOALLOC_MAX_DEVICES 64
hipError_t noalloc_scratch(int device, void** ptr);

// Largest workgroup of any pass.  The launch bound lets the compiler give
// every thread up to 256 VGPRs (two waves per SIMD), so the per-thread
// FFT operands and partial sums stay in registers.
#define TD_MAX_THREADS 512

// Largest dynamic LDS a workgroup may request: 160 KiB less a margin for
// the kernels' static LDS (the row inverse's per-round tables, 2.4 KiB).
#define TD_MAX_DYN_LDS (160u * 1024u - 3072u)

// Dynamic LDS of one workgroup of each pass: C sequences (row_fwd) or C
// columns / rows x G slots, each padded to lds_stride(M), plus the twiddle
// table (M entries).
inline size_t lds_bytes(int M, int C, size_t elem, int G = 1)
{
    const size_t SP = (size_t)M + M / 8;
    return ((size_t)C * G * SP + M) * elem;
}

// Band-limited column inputs (fft_regs_band in td_fft.hpp): for FP32 and
// M >= 1024 a forward column transform whose input has at most M/S stored
// rows that can be non-zero (S the span after the first radix-8 pass: 16
// for M = 1024, 32 for 2048, 8 for 4096) starts at span S.  The bound M/S,
// or 0 where the column pass has no band path (FP64 would spill registers
// to hold the band's inputs).  elem: complex element bytes.
__host__ __device__ constexpr int col_band_rows(int M, int elem)
{
    return elem != 8 || M < 1024 ? 0 : M / (__builtin_ctz(M) % 3 == 0 ? 8 : 8 << (__builtin_ctz(M) % 3));
}

// The column pass's FP32 transforms of sequences longer than a wavefront
// (M/8 > 64) ping-pong between two LDS buffers per sequence: one workgroup
// barrier per FFT pass instead of two.  (FP64 would lose occupancy to the
// second buffer; shorter sequences synchronise within their wavefront.)
template <typename T, int M>
__host__ __device__ constexpr bool col_pingpong() { return sizeof(T) == 4 && M / 8 > 64; }
inline bool col_pingpong_rt(int M, size_t elem) { return elem == 8 && M / 8 > 64; }
inline size_t col_lds_bytes(int M, int C, size_t elem, int G = 1)
{
    const size_t SP = (size_t)M + M / 8;
    return lds_bytes(M, C, elem, G) + (col_pingpong_rt(M, elem) ? (size_t)C * G * SP * elem : 0);
}

}  // namespace td
