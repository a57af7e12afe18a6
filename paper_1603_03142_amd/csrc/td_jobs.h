// Work descriptors shared by the host planner and the device passes.
//
// A solve is four passes over lists of jobs (one workgroup per job):
//   1. row_fwd     zero-padded real-to-complex row FFTs of every source field
//                  (own level and polyphase sub-grids of finer levels),
//                  written transposed: spectrum column kx holds the rows.
//   2. col_gather  per spectral column: column FFT of each input, multiply
//                  by the kernel spectra, sum, inverse column FFT -- the
//                  same-level and finer-source (Case 2') contributions to a
//                  level's own force.
//   3. col_scatter per spectral column: column FFT of a level's fields once,
//                  then one product and inverse column FFT per polyphase
//                  output of every finer target level (Case 3').
//   4. row_inv     complex-to-real row FFTs of the force spectra, window
//                  extraction, phase interleave, sum over source levels,
//                  covered-cell masking.
// Geometry is in "lattice" coordinates: the zero-padded M x M grid of one
// level's patch.  Intermediate spectra live in a workspace whose base comes
// with each launch segment: jobs hold byte offsets into it (so a plan can be
// bound to any workspace).  Kernel spectra are resident and addressed by
// absolute pointers; field pointers are looked up in a per-solve pointer
// table by slot.
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

struct ColTerm {
    int64_t in[3];      // workspace offsets: complex [M/2+1][in_ld] per field (sigma, dsdx, dsdy)
    const void* kern;   // stored kernel spectra of the phase: [6][M/2+1][M] complex
    int32_t in_ld;
    int32_t in_lr_first;
    int32_t flip;       // bit 0: x-mirror of the stored phase, bit 1: y-mirror
    int32_t pad;
};

struct ColGatherJob {
    int32_t kx0, ncol;   // spectral columns [kx0, kx0+ncol)
    int32_t term0, nterm;
    int64_t out_x;       // workspace offsets: complex [M/2+1][out_ld]
    int64_t out_y;
    int32_t out_ld;
    int32_t out_lr_first;
};

struct ColScatterOut {
    const void* kern;
    int64_t out_x;       // workspace offsets
    int64_t out_y;
    int32_t flip;
    int32_t out_ld;
    int32_t out_lr_first;
    int32_t pad;
};

struct ColScatterJob {
    int64_t in[3];       // workspace offsets
    int32_t in_ld, in_lr_first;
    int32_t kx0, ncol;
    int32_t out0, nout;
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
