// Launchers of the gfx950 kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>

#include "common.hpp"

namespace vbcsr {

// device allocation callback: the caller owns (and later frees) what it returns
using DevAlloc = std::function<hipError_t(void **, size_t)>;

// Arguments of one product launch over all panels of one direction.
//   Yout[r, c] = alpha * (A X)[r, c] + beta * Yin[r, c]   (Yin unread if beta == 0)
// With `mom` set, the kernel also adds R[r, c] * Yout[r, c] (in FP64) of its
// rows into mom[workgroup * nrhs + c].
template <typename T>
struct FwdParams {
  const RowDesc *rows;
  int32_t nrows;
  const int32_t *colx;
  const T *vals;        // FP64/FP32 pages (column-major panels)
  const uint16_t *hi;   // BF16 pages (8-column groups), BF16X3 only
  const uint16_t *lo;
  const int64_t *vbase16;
  const T *X;
  int64_t ldx;
  int64_t xrows;        // rows of X (columns of the operator)
  int32_t xrow16;       // set by the launcher: X rows start on 16-byte boundaries
  const T *Yin;
  int64_t ldyin;
  T *Yout;
  int64_t ldy;
  int32_t nrhs;
  double alpha, beta;
  const T *R;           // moment weights (Chebyshev), may be null
  int64_t ldr;
  double *mom;          // per-workgroup FP64 partial moments, may be null
};

// Kernel family and tiling chosen by the router.
enum class Kind { Vec, Mfma, Bf16x3 };

// Number of workgroups a product launch over `nrows` panels uses (the
// moment partials have this many rows).
int64_t product_workgroups(int64_t nrows);

hipError_t launch_spmm_f64(const FwdParams<double> &p, Kind kind, int tile, hipStream_t s);
hipError_t launch_spmm_f32(const FwdParams<float> &p, Kind kind, int tile, hipStream_t s);

// Graph-order values -> the pages of both directions, in one pass.
struct PackDir {
  const int64_t *pos;       // per graph block: page offset of its first value
  const int32_t *k0;        // per graph block: first panel column
  const int32_t *prow;      // per graph block: panel (processing order)
  const int64_t *vbase16;   // per panel: offset in the BF16 pages
  void *dst;                // double or float pages, or the BF16 hi pages
  uint16_t *dst_lo;         // BF16 lo pages (BF16X3 only)
};
struct PackParams {
  const int32_t *b;         // per atom
  const int32_t *blk_row;   // per graph block
  const int32_t *col_idx;   // per graph block
  const int64_t *gbase;     // per graph block: first value in graph order
  int64_t nnzb;
  int dst_kind;             // 0 = double pages, 1 = float pages, 2 = BF16 hi/lo pages
  PackDir dir[2];           // 0: forward panels (column-major blocks), 1: transposed
};
// src_dtype 0 / 1: graph-order double / float source, both page sets written.
hipError_t launch_pack(const PackParams &p, const void *src, int src_dtype, hipStream_t s);
// Map of one block at a transposed-page position: forward-page offset
// (column-major block) and transposed-page offset (row-major block) of its
// first value, and its shape.
struct PageRec {
  int64_t src, dst;
  int32_t bi, bj;
  int32_t pad[2];
};
static_assert(sizeof(PageRec) == 32, "PageRec layout");
// rec[u] for the graph block order[u] (u < nnzb), from the packing maps.
hipError_t launch_refresh_records(const PackParams &p, const int32_t *order, PageRec *rec,
                                  hipStream_t s);
// Transposed pages (dst) rebuilt from the forward pages (src), elem_bytes 8
// or 4, walking the transposed pages through rec.
hipError_t launch_refresh(const PageRec *rec, int64_t nnzb, int elem_bytes, const void *src,
                          void *dst, hipStream_t s);
// order[u] = graph block whose position pos[block] is the u-th smallest
// (page order of one direction; positions are distinct, below n_values).
hipError_t launch_page_order(const int64_t *pos, int64_t nnzb, int64_t n_values, int32_t *order,
                             const DevAlloc &alloc, hipStream_t s);

// dA (graph order) = block-sampled dY X^T, over the forward panels.
template <typename T>
struct SddmmParams {
  const RowDesc *rows;   // forward panels
  int32_t nrows;
  const int32_t *colx;   // per panel column: X row (4 entries of slack follow the table)
  const int64_t *colg;   // per panel column: (graph offset of block + q) << 7 | b_j
  const T *dY;
  int64_t lddy;
  const T *X;
  int64_t ldx;
  int32_t nrhs;
  T *dA;
  int64_t xrows;         // rows of X (columns of the operator)
  int32_t page_out;      // 1: dA in the forward pages' layout (colg unused)
};
hipError_t launch_sddmm_f64(const SddmmParams<double> &p, hipStream_t s);
hipError_t launch_sddmm_f32(const SddmmParams<float> &p, hipStream_t s);

// partial[w * nrhs + c] = sum over rows of chunk w of A[r, c] * B[r, c] (FP64).
hipError_t launch_coldot_f64(const double *A, int64_t lda, const double *B, int64_t ldb,
                             int64_t nrows, int32_t nrhs, double *partial, int64_t *nchunks,
                             hipStream_t s);
hipError_t launch_coldot_f32(const float *A, int64_t lda, const float *B, int64_t ldb,
                             int64_t nrows, int32_t nrhs, double *partial, int64_t *nchunks,
                             hipStream_t s);
int64_t coldot_chunks(int64_t nrows);
// out[c] = sum_{w < nparts} partial[w * nrhs + c], fixed order.
hipError_t launch_reduce_partials(const double *partial, int64_t nparts, int32_t nrhs, double *out,
                                  hipStream_t s);

// Numeric stage of the thresholded block product C = A B (one wave per
// output block).  Output block c (row atom oi[c], column atom oj[c]) is the
// sum over its products q in [pptr[c], pptr[c+1]) of A_ik B_kj, with A_ik at
// page offset pa[q] >> 8 of A's transposed pages (row-major b_i x b_k,
// b_k = pa[q] & 255) and B_kj at page offset pb[q] of B's forward pages
// (column-major b_k x b_j).  The block is written row-major at
// cvals + obase[c] and, when cnorm is set, its Frobenius norm to cnorm[c].
// A launch covers the blocks order[0 .. count) of one tile class.
struct SpgemmParams {
  const double *avals;
  const double *bvals;
  const int32_t *b;
  const int32_t *oi;
  const int32_t *oj;
  const int64_t *obase;
  const int64_t *pptr;
  const int64_t *pa;
  const int64_t *pb;
  const int32_t *order;
  int64_t count;
  double *cvals;          // C in graph order at obase (when fpages is null)
  double *cnorm;
  // C's own pages (when not null): block c at fpos[c] of the forward pages
  // (column-major) and at tpos[c] of the transposed pages (row-major)
  double *fpages, *tpages;
  const int64_t *fpos, *tpos;
};
// Tile class of a b_i x b_j block: 0 (1x1 tiles of 16), 1 (1x2), 2 (2x1),
// 3 (2x2), 4 (anything larger).
inline int spgemm_class(int bi, int bj) {
  const int ti = (bi + 15) / 16, tj = (bj + 15) / 16;
  return ti > 2 || tj > 2 ? 4 : (ti - 1) * 2 + (tj - 1);
}
hipError_t launch_spgemm_numeric(const SpgemmParams &p, int cls, int max_b, hipStream_t s);

// Symbolic stage of C = A B on the device (symbolic.hip).  Inputs are device
// arrays of the two handles: A's graph (row pointer arp, columns aci, row of
// every block arow), the page offset of every block of A in A's transposed
// pages (apos) and of B in B's forward pages (bpos), block sizes b, and the
// block norms an / bn (both null: every candidate is kept).  A candidate
// (i, j) is kept unless its bound sum_k ||A_ik|| ||B_kj||, summed over k in
// A's stored order, is below eps.  Outputs (device, allocated through
// `alloc`, which the caller frees): per kept block, in row order and with
// columns ascending, oi / oj / bound, obase and pptr (nC + 1 entries: value
// offsets in graph order, product ranges), C's row pointer crp (n + 1), the
// products pa (apos << 8 | b_k) / pb (bpos) in A's stored order of k, and
// the blocks grouped by tile class (order, stable; class k holds
// order[cls_begin[k] .. cls_begin[k+1])).
struct SymbolicIn {
  int32_t n;
  int64_t annzb;
  const int32_t *b;
  const int64_t *arp;
  const int32_t *aci, *arow;
  const int64_t *apos;
  const double *an;
  const int64_t *brp;
  const int32_t *bci;
  const int64_t *bpos;
  const double *bn;
  double eps;
};
struct SymbolicOut {
  int32_t *oi = nullptr, *oj = nullptr, *order = nullptr;
  int64_t *obase = nullptr, *pptr = nullptr, *pa = nullptr, *pb = nullptr, *crp = nullptr;
  double *bound = nullptr;
  int64_t nC = 0, nP = 0, nvals = 0, candidates = 0, products_all = 0;
  double flops = 0.0;
  int64_t cls_begin[6] = {0, 0, 0, 0, 0, 0};
};
// hipErrorInvalidValue when the product has 2^31 or more candidate products
hipError_t spgemm_symbolic_device(const SymbolicIn &in, SymbolicOut &out, const DevAlloc &alloc,
                                  hipStream_t s);

// Plan of an operator whose block graph is on the device (both directions,
// panels in the processing order `order`, a permutation of the n atoms):
// the per-block maps, panel descriptors, graph value offsets (gbase, nnzb + 1
// entries) and block rows that the host planner computes for the same order,
// and on the host the column-table and page sizes, the largest panel (values,
// before the alignment padding), the value count and
// the number of (b_i, b_j) shape classes.  Columns must be ascending within
// each row.  hipErrorInvalidValue for 2^31 or more blocks.
struct DevPlanIn {
  int32_t n;
  int64_t nnzb;
  const int32_t *b, *off;   // block sizes, first scalar rows (n entries)
  const int64_t *rp;        // row pointer (n + 1)
  const int32_t *ci;        // block columns (nnzb)
  const int32_t *order;     // processing order (n)
};
struct DevPlanDir {
  RowDesc *rows;            // n (device, written)
  int64_t *blk_pos;         // nnzb (device, written)
  int32_t *blk_k0, *blk_prow;
  int64_t n_values = 0, n_cols = 0, max_panel = 0;
};
struct DevPlanOut {
  int32_t *blk_row;         // nnzb (device, written)
  int64_t *gbase;           // nnzb + 1 (device, written)
  DevPlanDir dir[2];        // 0 = forward, 1 = transposed
  int64_t nnz = 0;
  int32_t n_shapes = 0;
};
hipError_t plan_device(const DevPlanIn &in, DevPlanOut &out, const DevAlloc &alloc, hipStream_t s);
// order[p] = the atom whose first scalar row is rows[p].yrow (off ascending,
// n entries): the processing order of an existing plan.
hipError_t launch_order_from_rows(const RowDesc *rows, int32_t np, const int32_t *off, int32_t n,
                                  int32_t *order, hipStream_t s);
hipError_t launch_iota(int32_t n, int32_t *order, hipStream_t s);

// Closing filter of the block product: block c of the pattern (row pointer
// rp, n + 1 entries; columns ci; graph value offsets obase, nC + 1 entries;
// values vals) is kept unless norm[c] < eps (a NaN norm keeps it); kept
// blocks keep their order.  The filtered row pointer, columns and values are
// carved out of one allocation made through `alloc` (left NULL when nothing
// is removed: the inputs stand); their counts are returned on the host.
struct FilterOut {
  int64_t *rp = nullptr;
  int32_t *ci = nullptr;
  double *vals = nullptr;
  int64_t nnzb = 0, nvals = 0;
};
hipError_t spgemm_filter_device(int32_t n, int64_t nC, const int64_t *rp, const int32_t *ci,
                                const int64_t *obase, const double *norm, double eps,
                                const double *vals, FilterOut &out, const DevAlloc &alloc,
                                hipStream_t s);
// out[k] = Frobenius norm of graph block k, read from forward pages at pos[k].
hipError_t launch_block_norms(const double *pages, const int64_t *pos, const int32_t *blk_row,
                              const int32_t *col_idx, const int32_t *b, int64_t nnzb, double *out,
                              hipStream_t s);
// Zero the gaps of FP64 / FP32 pages (elem_bytes 8 or 4) that packing does
// not write: after each of the np panels (rows in processing order) up to
// the next panel, and kPageSlack values after the last.
hipError_t launch_zero_gaps(const RowDesc *rows, int32_t np, int64_t n_values, int elem_bytes,
                            void *vals, hipStream_t s);
// dst[dbase[t] + e] = src[sbase[t] + e], e < size[t], t < nblk.
hipError_t launch_gather_blocks(const double *src, const int64_t *sbase, const int64_t *dbase,
                                const int32_t *size, int64_t nblk, double *dst, hipStream_t s);
// Forward pages (elem_bytes 8 or 4) -> graph-order row-major blocks at gbase.
hipError_t launch_unpack(const void *pages, int elem_bytes, const int64_t *pos,
                         const int32_t *blk_row, const int32_t *col_idx, const int32_t *b,
                         const int64_t *gbase, int64_t nnzb, void *dst, hipStream_t s);

// Kernel polynomial method: coef[k] = damped, doubled moments (damping 0 =
// none, 1 = Jackson), then rho[i] = density of states at x[i] (|x| < 1).
hipError_t launch_kpm_dos(const double *mu, int M, int damping, const double *x, int64_t np,
                          double *coef, double *rho, hipStream_t s);

// Column tables of one direction from the per-block maps: graph block k
// fills the b_c entries of its panel columns, starting at
// rows[prow[k]].cbase + k0[k], with colx = off[c] + q and (forward only,
// colg != null) colg = (gbase[k] + q) << 7 | b_c, where c = catom[k] is the
// atom indexing the block's panel columns (forward: its column, adjoint: its
// row).
struct ColumnParams {
  const RowDesc *rows;
  const int32_t *prow, *k0, *catom, *b, *off;
  const int64_t *gbase;
  int64_t nnzb;
  int32_t *colx;
  int64_t *colg;
};
hipError_t launch_columns(const ColumnParams &p, hipStream_t s);

// Halo buffers of a rank-local operator: buf[t] = X[rows[t]] (rows outside
// [0, xrows) skipped), and Y[red_rows[u]] += sum of buf[red_pos[e]] over
// e in [red_ptr[u], red_ptr[u+1]) in order (indices outside Y or the brows
// buffer rows skipped).  elem_bytes 8 (double) or 4 (float).
hipError_t launch_rows_pack(const void *X, int64_t xrows, int64_t ldx, const int32_t *rows,
                            int64_t nrows, int32_t nrhs, int elem_bytes, void *buf, int64_t ldb,
                            hipStream_t s);
hipError_t launch_rows_reduce(void *Y, int64_t yrows, int64_t ldy, const int32_t *red_rows,
                              const int64_t *red_ptr, const int64_t *red_pos, int64_t n_red,
                              int64_t brows, const void *buf, int64_t ldb, int32_t nrhs,
                              int elem_bytes, hipStream_t s);

// Scratch of the allocation-free entry points: a file-scope device array of
// kNoAllocScratchBytes per GPU.  *ptr receives its address on the current
// device (looked up with hipGetSymbolAddress on the first call per device).
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
hipError_t noalloc_scratch(void **ptr, size_t *bytes);

}  // namespace vbcsr
