// Launchers of the complex (reciprocal-space) kernels (zkernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace vbcsr {

// Per contribution c (a real block, listed by the block of O(k) it adds to):
// ph[2c], ph[2c+1] = cos, sin of -2 pi k . d_c with d_c = shifts[image[c]]
// (+ tau[col_idx[c]] - tau[blk_row[c]] when tau is given).
struct ZPhaseParams {
  const int32_t *image;
  const int32_t *blk_row;
  const int32_t *col_idx;
  const int32_t *shifts;  // [n_images * 3]
  const double *tau;      // [n * 3] or null
  double k[3];
  int64_t n;               // contributions
  double *ph;
};

// Block kb of O(k) is the sum over its contributions c in [cptr[kb],
// cptr[kb+1]) of ph_c * values[cgbase[c] ..] (row-major b_i x b_j), written
// column-major at fwd_pos[kb] of the forward pages and, conjugated and
// row-major, at tr_pos[kb] of the adjoint pages (complex elements of type T).
// One wave takes kSampleBlocks consecutive blocks; kvbase[kb] is
// cgbase[cptr[kb]], so a block's first contribution needs no further lookup.
constexpr int kSampleBlocks = 8;
struct ZSampleParams {
  int64_t nkb;
  const int32_t *kdim;    // per block: b_i | b_j << 16
  const int64_t *kbase;   // [nkb + 1] offset of each block's first value, graph order
  const int64_t *kvbase;  // per block
  const int64_t *cptr;    // [nkb + 1]
  const int64_t *cgbase;  // per contribution
  const double *values;
  const double *ph;       // per contribution: cos, sin
  const int64_t *fwd_pos, *tr_pos;
};

// Y = alpha * op(O) X + beta * Y over the panels of one direction (complex,
// interleaved re/im, leading dimensions in complex elements).
template <typename T>
struct ZSpmmParams {
  const RowDesc *rows;
  int32_t nrows;
  const int32_t *colx;
  const T *pages;
  const T *X;
  int64_t ldx;
  T *Y;
  int64_t ldy;
  int32_t nrhs;
  double ar, ai, br, bi;
  int64_t xrows;  // rows of X (columns of the operator)
};

hipError_t launch_zphase(const ZPhaseParams &p, hipStream_t s);
hipError_t launch_zsample(const ZSampleParams &p, void *fwd, void *tr, int elem_bytes,
                          hipStream_t s);
hipError_t launch_zspmm_f64(const ZSpmmParams<double> &p, hipStream_t s);
hipError_t launch_zspmm_f32(const ZSpmmParams<float> &p, hipStream_t s);
// forward pages (complex, column-major blocks) -> graph order row-major
hipError_t launch_zunpack(const void *fwd, int elem_bytes, const int64_t *pos,
                          const int32_t *krow, const int32_t *kcol, const int32_t *b,
                          const int64_t *kbase, int64_t nkb, void *dst, hipStream_t s);

}  // namespace vbcsr
