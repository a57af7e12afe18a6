// Launch interface between the host planner and the device passes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "td_jobs.h"

namespace td {

// A launch processes the concatenated job lists of up to TD_MAX_SEGS plans
// (one workgroup per job).  Each segment carries the pointer-table slot base
// of its solve and an auxiliary per-plan array (terms, scatter outputs or
// row contributions).  Passed by value as a kernel argument.
#define TD_MAX_SEGS 40

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
        return jobs[lo][block - start[lo]];
    }
};

template <typename T>
hipError_t launch_row_fwd(int M, int C, int blocks, const SegTable<RowFwdJob>& segs,
                          const void* const* ptrs, const void* tw, hipStream_t st);
template <typename T>
hipError_t launch_col_gather(int M, int C, int blocks, const SegTable<ColGatherJob>& segs,
                             const void* tw, hipStream_t st);
template <typename T>
hipError_t launch_col_scatter(int M, int C, int blocks, const SegTable<ColScatterJob>& segs,
                              const void* tw, hipStream_t st);
template <typename T>
hipError_t launch_row_inv(int M, int C, int blocks, const SegTable<RowInvJob>& segs,
                          void* const* ptrs, const void* tw, hipStream_t st);
template <typename TO>
hipError_t launch_spec_col(int M, int C, const void* rows, void* out, const void* tw64,
                           hipStream_t st);
hipError_t launch_table(const TableJob& job, hipStream_t st);

// Lift the dynamic-LDS cap of every pass instantiation (call once per device).
hipError_t prepare_kernels();

// Dynamic LDS of one workgroup of each pass (C sequences of length M).
inline size_t lds_bytes(int pass, int M, int C, size_t elem)
{
    // pass 0 row_fwd: 1 buffer; 1 gather: 3; 2 scatter: 4; 3 row_inv: 1
    static const int nbuf[4] = {1, 3, 4, 1};
    return (size_t)nbuf[pass] * C * M * elem;
}

}  // namespace td
