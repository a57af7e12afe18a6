// Work descriptors shared by the host planner and the device passes.
//
// A solve is three passes over lists of jobs (one workgroup per job):
//   1. row_fwd  zero-padded real-to-complex row FFTs of every source field
//               (own level and polyphase sub-grids of finer levels), written
//               transposed: spectrum column kx holds the stored rows.
//   2. col      per spectral column: the forward column FFT of every input
//               plane, zero-padded to the lattice length M, multiplied by its
//               kernel spectra and summed per output, then the inverse column
//               FFT of every output.  Outputs are a level's own force
//               (same-level and finer-source inputs, Case 2') and the
//               polyphase outputs of a coarser source onto a finer target
//               (Case 3').  No 2-D input spectrum is ever stored.
//   3. row_inv  complex-to-real row FFTs of the force spectra, window
//               extraction, phase interleave, sum over source levels,
//               covered-cell masking.
#pragma once
#include <stdint.h>

namespace td {

#define TD_PATCHES_PER_LEVEL 8

// The patches of one level in its window coordinates (the window is the
// bounding rectangle of the level's patches; cells of the window outside
// every patch are not part of the level), and the squares covered by the
// next finer level's patches.  One per level and plan, in device memory.
struct LevelPatches {
    int32_t np, nc;
    int32_t pi0[TD_PATCHES_PER_LEVEL], pj0[TD_PATCHES_PER_LEVEL];  // patch origins
    int32_t pn[TD_PATCHES_PER_LEVEL];                             // patch sides
    int32_t pslot[TD_PATCHES_PER_LEVEL];   // pointer-table slot of the patch's field 0
    int32_t ci0[TD_PATCHES_PER_LEVEL], cj0[TD_PATCHES_PER_LEVEL];  // covered squares
    int32_t cn[TD_PATCHES_PER_LEVEL];
};

struct RowFwdJob {
    int32_t lvl;        // source level (index into the plan's LevelPatches)
    int32_t f;          // source field: pointer slot = pslot[patch] + f
    int32_t m;          // lattice -> source decimation
    int32_t row_off;    // source row = m * lattice_row + row_off (window coords)
    int32_t col_off;    // source col = m * lattice_col + col_off
    int32_t lr_first;   // lattice row of stored row 0
    int32_t ld;         // stored rows per spectral column
    int32_t row0;       // first stored row of this job
    int32_t nrow;       // rows of this job
    int32_t lc_lo, lc_hi;  // lattice columns that can hold a source cell (the
                           // others map outside the source level's window)
    int32_t pad;
    double scale;       // multiplies every value read (sigma, or a given slope)
    double est_scale;   // multiplies a slope estimated from sigma (per-cell units)
    int64_t out;        // workspace byte offset: complex [M/2+1][ld]
};

// One input plane of the column pass: a row-pass output [M/2+1][ld] whose
// stored rows sit at lattice rows [lr_first, lr_first + ld) (zero
// elsewhere), with the stored kernel spectra it is multiplied by.
struct ColIn {
    int64_t in;          // workspace offset: complex [M/2+1][ld]
    const void* kern;    // stored kernel spectra of the level pair (see kern_at)
    int32_t ld, lr_first;
    int32_t f;           // field: 0 sigma, 1 dsdx, 2 dsdy
    int32_t flip;        // bits 0/1: x/y mirror, 2: quarter-real layout,
                         // 3: potential kernel family (parities P0, Px, Py)
    int32_t rows;        // stored rows [0, rows) hold every source row (the
                         // rest of the ld are zeros)
    int32_t pad;
};

// One output plane of the column pass: the inverse column FFT of a sum of
// products, lattice rows [out_lr_first, out_lr_first + out_ld) written to
// [M/2+1][out_ld].
struct ColOut {
    int64_t out;         // workspace offset
    const void* kern;    // Case-3' outputs: the phase's stored kernel spectra
    int32_t out_ld, out_lr_first;
    int32_t comp;        // 0: Fx (or the potential), 1: Fy
    int32_t flip;        // Case-3' outputs: mirror bits of the phase (as ColIn)
};

// Columns [kx0, kx0 + ncol) of one job; a workgroup holds C columns x G
// slots.
//  kind 0 (a level's own force): inputs [in0, in0 + nin); slot g of a column
//    takes inputs g, g + G, ..., transforms each and accumulates it times its
//    kernels into Fx (output out0) and Fy (output out0 + 1); the slots'
//    partial sums are reduced before the two inverse transforms.  The last
//    nband inputs are band-limited (rows <= M / band_span(M)): a round of G
//    inputs that lies wholly among them uses the band transforms.
//  kind 1 (Case 3'): the three inputs [in0, in0 + 3) of the coarser level are
//    transformed once; outputs [out0, out0 + nout), one per (phase,
//    component), are formed from them G at a time and transformed back.
struct ColJob {
    int32_t kind;
    int32_t kx0, ncol;
    int32_t in0, nin;
    int32_t out0, nout;
    int32_t nband;
};

struct RowInvContrib {
    int64_t base;          // workspace offset of phase (0,0), x component: complex [M/2+1][ld]
    int64_t phase_stride;  // complex elements between phases (phase = ky*m + kx)
    int64_t comp_stride;   // complex elements from x to y component
    int32_t m;             // 1: same lattice; else coarse-lattice ratio
    int32_t ld;
    int32_t lr_first;      // lattice row of stored row 0
    int32_t ox_s, oy_s;    // lattice origin: offsets of the lattice's level
    int32_t mshift;        // log2(m), or -1 when m is not a power of two
};

struct RowInvJob {
    int32_t lvl;                // target level (index into the LevelPatches)
    int32_t nx_t, ny_t;         // target window size
    int32_t ox_t, oy_t;         // target window origin (level cells)
    int32_t y0, ny;             // target rows of this job
    int32_t c0, nc;             // contributions
    int32_t accumulate;         // 0: write (masking covered cells), 1: add
    int32_t x0, nx;             // target columns of this job (nx <= 2M)
};

// Auxiliary table of a row-inverse launch segment.
struct RowInvTables {
    const RowInvContrib* contribs;
    const LevelPatches* levels;
};

// Kernel-table request: one phase of one (M, case, m) key, written as six
// real M x M tables [X][ny][nx].
struct TableJob {
    int32_t M, kind, m, kx, ky;
    int32_t family;     // 0: force tables; 1: potential (P0, Px, Py, then zeros)
    double aspect;      // cell height / width (v coordinates in units of the width)
    double* out;
};

}  // namespace td
