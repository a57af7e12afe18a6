// Host-only stand-ins for the device launchers, linked into the sanitizer
// build of the C-ABI's host logic.  The entry points that build exercises
// (hierarchy checks, snapping, host-only planning) never launch a kernel;
// any call to these reports an error instead.
#include <hip/hip_runtime_api.h>

#include "td_launch.h"

namespace td {

template <typename T>
hipError_t launch_row_fwd(int, int, int, const SegTable<RowFwdJob>&, const void* const*,
                          const FieldPtrs&, const void*, bool, hipStream_t)
{
    return hipErrorInvalidValue;
}
template <typename T>
hipError_t launch_col(int, int, int, int, const SegTable<ColJob>&, const void*, hipStream_t,
                      const JobQueue&)
{
    return hipErrorInvalidValue;
}
template <typename T>
hipError_t launch_row_inv(int, int, int, int, const SegTable<RowInvJob>&, void* const*,
                          const FieldPtrs&, const void*, hipStream_t, int)
{
    return hipErrorInvalidValue;
}
template <typename TO>
hipError_t launch_spec_col(int, int, const void*, void*, const void*, int, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_table(const TableJob&, hipStream_t) { return hipErrorInvalidValue; }
int col_resident_blocks(bool, int, int, int) { return 1; }
hipError_t launch_zero_counters(unsigned int*, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_count_nonfinite(bool, const void*, int64_t, unsigned long long*, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t prepare_kernels() { return hipErrorInvalidValue; }
hipError_t noalloc_scratch(int, void** p)
{
    *p = nullptr;
    return hipErrorInvalidValue;
}

template hipError_t launch_row_fwd<float>(int, int, int, const SegTable<RowFwdJob>&,
                                          const void* const*, const FieldPtrs&, const void*, bool,
                                          hipStream_t);
template hipError_t launch_row_fwd<double>(int, int, int, const SegTable<RowFwdJob>&,
                                           const void* const*, const FieldPtrs&, const void*,
                                           bool, hipStream_t);
template hipError_t launch_col<float>(int, int, int, int, const SegTable<ColJob>&, const void*,
                                      hipStream_t, const JobQueue&);
template hipError_t launch_col<double>(int, int, int, int, const SegTable<ColJob>&, const void*,
                                       hipStream_t, const JobQueue&);
template hipError_t launch_row_inv<float>(int, int, int, int, const SegTable<RowInvJob>&,
                                          void* const*, const FieldPtrs&, const void*,
                                          hipStream_t, int);
template hipError_t launch_row_inv<double>(int, int, int, int, const SegTable<RowInvJob>&,
                                           void* const*, const FieldPtrs&, const void*,
                                           hipStream_t, int);
template hipError_t launch_spec_col<float>(int, int, const void*, void*, const void*, int,
                                           hipStream_t);
template hipError_t launch_spec_col<double>(int, int, const void*, void*, const void*, int,
                                            hipStream_t);

}  // namespace td
