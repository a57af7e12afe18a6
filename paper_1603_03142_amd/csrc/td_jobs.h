// Work descriptors shared by the host planner and the device passes.
//
// A solve is four passes over lists of jobs (one workgroup per job):
//   1. row_fwd  zero-padded real-to-complex row FFTs of every source field
//               (own level and polyphase sub-grids of finer levels), written
//               transposed: spectrum column kx holds the rows.
//   2. col_fwd  forward FFT of every spectrum column, zero-padded to the
//               lattice length M: the full 2-D spectrum of every input.
//   3. col_mac  per spectral column and output: the sum over inputs of input
//               spectrum x kernel spectrum, then the inverse column FFT.
//               Outputs are a level's own force (same-level and finer-source
//               inputs, Case 2') and the polyphase outputs of a coarser
//               source onto a finer target (Case 3').
//   4. row_inv  complex-to-real row FFTs of the force spectra, window
//               extraction, phase interleave, sum over source levels,
//               covered-cell masking.
#pragma once
#include <stdint.h>

namespace td {

struct RowFwdJob {
    int32_t src_slot;   // pointer-table slot of the source field
    int32_t n_src;      // source array is n_src x n_src
    int32_t m;          // lattice -> source decimation
    int32_t row_off;    // source row = m * lattice_row + row_off
    int32_t col_off;    // source col = m * lattice_col + col_off
    int32_t lr_first;   // lattice row of stored row 0
    int32_t ld;         // stored rows per spectral column
    int32_t row0;       // first stored row of this job
    int32_t nrow;       // rows of this job
    int32_t cov_i0, cov_i1, cov_j0, cov_j1;  // covered source cells, half-open
    int32_t pad;
    double scale;       // multiplies every value (slope scaling)
    int64_t out;        // workspace byte offset: complex [M/2+1][ld]
};

// Forward column FFT of the C columns [kx0, kx0 + ncol) of one input plane.
struct ColFwdJob {
    int64_t in;          // workspace offset: complex [M/2+1][ld] (row pass output)
    int64_t out;         // workspace offset: complex [M/2+1][M] (2-D spectrum)
    int32_t ld;          // stored rows of the input plane
    int32_t lr_first;    // lattice row of stored row 0
    int32_t kx0, ncol;
};

// One product of an output: input spectrum x stored kernel spectrum X.
struct MacTerm {
    int64_t in;          // workspace offset: complex [M/2+1][M]
    const void* kern;    // stored kernel spectra (see kern_at)
    int32_t X;           // kernel index 0..5: I0, Ixx, Ixy, J0, Jyy, Jyx
    int32_t flip;        // mirror / layout bits of the stored spectrum
};

// One output column family: sum of its terms, inverse column FFT, rows
// [out_lr_first, out_lr_first + out_ld) written to [M/2+1][out_ld].
struct MacOut {
    int64_t out;         // workspace offset
    int32_t term0, nterm;
    int32_t out_ld, out_lr_first;
};

// Columns [kx0, kx0 + ncol) x outputs [out0, out0 + nout); each output's
// terms are split over `split` slots (nout * split <= slots per column),
// whose partial sums are reduced before the inverse FFT.
struct ColMacJob {
    int32_t kx0, ncol;
    int32_t out0, nout;
    int32_t split;
    int32_t pad;
};

struct RowInvContrib {
    int64_t base;          // workspace offset of phase (0,0), x component: complex [M/2+1][ld]
    int64_t phase_stride;  // complex elements between phases (phase = ky*m + kx)
    int64_t comp_stride;   // complex elements from x to y component
    int32_t m;             // 1: same lattice; else coarse-lattice ratio
    int32_t ld;
    int32_t lr_first;      // lattice row of stored row 0
    int32_t ox_s, oy_s;    // lattice origin: offsets of the lattice's level
    int32_t pad;
};

struct RowInvJob {
    int32_t n_t, ox_t, oy_t;    // target level size and offsets
    int32_t y0, ny;             // target rows of this job
    int32_t out_slot;           // fx slot; fy = out_slot + 1
    int32_t cov_i0, cov_i1, cov_j0, cov_j1;  // covered target cells
    int32_t c0, nc;             // contributions
    int32_t accumulate;         // 0: write (masking covered cells), 1: add
    int32_t x0, nx;             // target columns of this job (nx <= 2M)
    int32_t pad;
};

// Kernel-table request: one phase of one (M, case, m) key, written as six
// real M x M tables [X][ny][nx].
struct TableJob {
    int32_t M, kind, m, kx, ky;
    int32_t pad;
    double* out;
};

}  // namespace td
