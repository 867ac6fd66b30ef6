// Launchers of the complex (reciprocal-space) kernels (zkernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace vbcsr {

// Per real block t: ph[2t], ph[2t+1] = cos, sin of -2 pi k . d_t with
// d_t = shifts[image[t]] (+ tau[col_t] - tau[row_t] when tau is given).
struct ZPhaseParams {
  const int32_t *image;
  const int32_t *blk_row;
  const int32_t *col_idx;
  const int32_t *shifts;  // [n_images * 3]
  const double *tau;      // [n * 3] or null
  double k[3];
  int64_t nnzb;
  double *ph;
};

// One wave per block kb of O(k): the sum over its real blocks
// t = cblk[cptr[kb] .. cptr[kb+1]) of ph_t * values[gbase[t] ..] (row-major
// b_i x b_j), written column-major at fwd_pos[kb] of the forward pages and,
// conjugated and row-major, at tr_pos[kb] of the adjoint pages (complex
// elements of type T).
struct ZSampleParams {
  const int32_t *b;
  const int32_t *krow, *kcol;
  const int64_t *cptr, *cblk;
  const int64_t *gbase;
  const double *values;
  const double *ph;
  const int64_t *fwd_pos, *tr_pos;
  int64_t nkb;
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
