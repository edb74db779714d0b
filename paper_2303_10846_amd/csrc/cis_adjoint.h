// Launchers of the adjoint solve's block preconditioner (FP64); the kernels are in cis_adjoint.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cis_internal.h"

namespace cis {

// Per-cell scratch of the block preconditioner, 24 doubles per cell: gW [nc][6], gq [nc][6], u [nc][6],
// r [nc][4] (face spectral radii of Eq. 41), D [nc][2] (macro diagonals).
constexpr int kBlockPrecondCellDoubles = 26;  // gW, gq, u (6 each), r_f (up to 6 slots), 2 diagonals

// out = P in over the full adjoint vector [G | R | W | q]: the W and q rows are eliminated exactly (their
// diagonal block is taken as the identity) and the phi Schur complement is approximated by the transpose of
// the linearised implicit step, micro_pairs transposed micro sweep pairs (0: the diagonal) followed by the
// transposed macro system with macro_pairs PR-SGS pairs.  tmp: a second full-length vector; cell: the scratch
// above.  in and out must not overlap tmp.
void launch_adj_block_precond(const Dev& d, const Bufs& b, const double* in, double* out, double* tmp, double* cell,
                              const int64_t* color_off, int64_t n_colors, int micro_pairs, int macro_pairs,
                              hipStream_t st);

}  // namespace cis
