// C ABI of the variable-block sparse library: handles, validation, routing
// and launches.  See include/vbcsr.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <system_error>

#include "../../include/vbcsr.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace vbcsr;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  try {
    g_last_error = msg;
  } catch (...) {
    g_last_error.clear();
  }
  return code;
}

}  // namespace

namespace vbcsr {
int set_error(int code, const std::string &msg) { return fail(code, msg); }

int api_exception(const char *where) {
  int code = VBCSR_EINVAL;
  auto note = [&](int c, const char *what) {
    code = c;
    try {
      g_last_error = std::string(where) + ": " + what;
    } catch (...) {
      g_last_error.clear();
    }
  };
  try {
    throw;
  } catch (const std::bad_alloc &) {
    note(VBCSR_ENOMEM, "host memory allocation failed");
  } catch (const std::length_error &) {
    note(VBCSR_ENOMEM, "host buffer size out of range");
  } catch (const std::system_error &e) {
    note(VBCSR_ENOMEM, e.what());
  } catch (const std::exception &e) {
    note(VBCSR_EINVAL, e.what());
  } catch (...) {
    note(VBCSR_EINVAL, "unknown exception");
  }
  return code;
}
}  // namespace vbcsr

namespace {

int hip_fail(hipError_t e, const char *where) {
  return fail(VBCSR_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, where)                         \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// Allocation counter for fault injection: VBCSR_FAIL_ALLOC_AFTER=n makes the
// (n+1)-th device allocation of the process fail with VBCSR_ENOMEM before any
// HIP call is made.
std::atomic<long> g_alloc_count{0};

int dev_alloc(void **p, size_t bytes) {
  *p = nullptr;
  const char *lim = std::getenv("VBCSR_FAIL_ALLOC_AFTER");
  const long n = g_alloc_count.fetch_add(1);
  if (lim && *lim && n >= std::atol(lim)) return fail(VBCSR_ENOMEM, "injected allocation failure");
  if (bytes == 0) return VBCSR_OK;
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return fail(VBCSR_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  return VBCSR_OK;
}

template <typename T>
int upload(T **dst, const T *src, size_t count, hipStream_t s) {
  int rc = dev_alloc(reinterpret_cast<void **>(dst), sizeof(T) * count);
  if (rc) return rc;
  if (count)
    HIP_TRY(hipMemcpyAsync(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice, s),
            "hipMemcpyAsync");
  return VBCSR_OK;
}

template <typename T, typename Alloc>
int upload(T **dst, const std::vector<T, Alloc> &src, hipStream_t s) {
  return upload(dst, src.data(), src.size(), s);
}

struct DevDir {
  RowDesc *rows = nullptr;
  int32_t *colx = nullptr;
  void *vals = nullptr;       // double or float pages (FP64/FP32)
  uint16_t *hi = nullptr;     // BF16 pages (BF16X3)
  uint16_t *lo = nullptr;
  int64_t *vbase16 = nullptr;
  int64_t *blk_pos = nullptr;
  int32_t *blk_k0 = nullptr;
  int32_t *blk_prow = nullptr;
  PageRec *page_recs = nullptr;  // transposed only: block maps in page order (built on
                                 // the first vbcsr_refresh_transposed)
  int64_t *colg = nullptr;    // forward direction only
  int64_t n_values = 0, n_values16 = 0;
  int32_t npanels = 0;        // forward: block rows; transposed: block columns
};

int env_path() {
  const char *e = std::getenv("VBCSR_PATH");
  if (!e) return VBCSR_PATH_AUTO;
  if (!std::strcmp(e, "vec")) return VBCSR_PATH_VEC;
  if (!std::strcmp(e, "mfma")) return VBCSR_PATH_MFMA;
  return VBCSR_PATH_AUTO;
}

}  // namespace

struct vbcsr_mat {
  int32_t n = 0;       // atoms: block columns (and block rows when square)
  int32_t n_rows = 0;  // block rows: n, or the owned atoms of a rank-local operator
  int64_t N = 0, N_rows = 0, nnzb = 0, nnz = 0;
  int32_t n_shapes = 0;
  vbcsr_prec prec = VBCSR_FP64;
  vbcsr_plan_opts opts{};
  // graph-order structure on the device
  int32_t *b = nullptr;
  int32_t *off = nullptr;
  int64_t *row_ptr = nullptr;
  int32_t *col_idx = nullptr;
  int32_t *blk_row = nullptr;
  int64_t *gbase = nullptr;
  DevDir dir[2];  // 0 = forward pages, 1 = transposed pages
  // forward values read from a caller's page buffer (vbcsr_use_pages):
  // own_fwd keeps the handle's own forward pages meanwhile
  void *own_fwd = nullptr;
  bool tr_stale = false;  // transposed pages not rebuilt since the forward source changed
  std::vector<void *> owned;
};

namespace {

size_t vec_elem(const vbcsr_mat *A) { return A->prec == VBCSR_FP64 ? 8 : 4; }

template <typename T>
int alloc_into(vbcsr_mat *A, T **p, size_t count) {
  int rc = dev_alloc(reinterpret_cast<void **>(p), sizeof(T) * count);
  if (rc == VBCSR_OK && *p) A->owned.push_back(*p);
  return rc;
}

template <typename T>
int upload_into(vbcsr_mat *A, T **p, const T *src, size_t count, hipStream_t s) {
  int rc = upload(p, src, count, s);
  if (rc == VBCSR_OK && *p) A->owned.push_back(*p);
  return rc;
}

template <typename T, typename Alloc>
int upload_into(vbcsr_mat *A, T **p, const std::vector<T, Alloc> &v, hipStream_t s) {
  return upload_into(A, p, v.data(), v.size(), s);
}

void free_all(vbcsr_mat *A) {
  if (!A) return;
  if (!A->owned.empty()) (void)hipDeviceSynchronize();
  for (void *p : A->owned) (void)hipFree(p);
  A->owned.clear();
}

// Pack graph-order values (device) into both directions' pages.
int pack_all(vbcsr_mat *A, const void *src, int src_dtype, hipStream_t s) {
  PackParams pp{};
  pp.b = A->b;
  pp.blk_row = A->blk_row;
  pp.col_idx = A->col_idx;
  pp.gbase = A->gbase;
  pp.nnzb = A->nnzb;
  pp.dst_kind = A->prec == VBCSR_BF16X3 ? 2 : A->prec == VBCSR_FP64 ? 0 : 1;
  for (int d = 0; d < 2; ++d) {
    const DevDir &D = A->dir[d];
    pp.dir[d].pos = D.blk_pos;
    pp.dir[d].k0 = D.blk_k0;
    pp.dir[d].prow = D.blk_prow;
    pp.dir[d].vbase16 = D.vbase16;
    pp.dir[d].dst = A->prec == VBCSR_BF16X3 ? static_cast<void *>(D.hi) : D.vals;
    pp.dir[d].dst_lo = D.lo;
  }
  hipError_t e = launch_pack(pp, src, src_dtype, s);
  if (e != hipSuccess) return hip_fail(e, "pack kernel launch");
  return VBCSR_OK;
}

bool ranges_overlap(const void *a, size_t abytes, const void *b, size_t bbytes) {
  const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
  return pa < pb + bbytes && pb < pa + abytes;
}

size_t span_bytes(int64_t rows, int64_t ld, int32_t nrhs, size_t elem) {
  if (rows <= 0) return 0;
  return ((size_t)(rows - 1) * (size_t)ld + (size_t)nrhs) * elem;
}

// X has xrows rows and Y yrows (N or N_rows, by direction); a vector with no
// rows may be NULL.
int check_vectors(const vbcsr_mat *A, const void *X, int64_t xrows, int64_t ldx, const void *Y,
                  int64_t yrows, int64_t ldy, int32_t nrhs, bool y_written) {
  if (!A) return fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (nrhs <= 0) return fail(VBCSR_EINVAL, "nrhs must be >= 1");
  if (ldx < nrhs || ldy < nrhs) return fail(VBCSR_EINVAL, "leading dimension smaller than nrhs");
  if ((xrows > 0 && !X) || (yrows > 0 && !Y)) return fail(VBCSR_EINVAL, "vector pointer is NULL");
  const size_t e = vec_elem(A);
  if (y_written && ranges_overlap(X, span_bytes(xrows, ldx, nrhs, e), Y, span_bytes(yrows, ldy, nrhs, e)))
    return fail(VBCSR_EINVAL, "input and output vectors overlap");
  return VBCSR_OK;
}

// Rows of the input and output vectors of direction d (0 forward, 1 adjoint).
int64_t in_rows(const vbcsr_mat *A, int d) { return d == 0 ? A->N : A->N_rows; }
int64_t out_rows(const vbcsr_mat *A, int d) { return d == 0 ? A->N_rows : A->N; }

int require_square(const vbcsr_mat *A, const char *where) {
  if (A && A->n_rows != A->n)
    return fail(VBCSR_EUNSUPPORTED,
                std::string(where) + ": needs a square operator (this one is rank-local)");
  return VBCSR_OK;
}

struct Route {
  Kind kind;
  int tile;
};

Route route(const vbcsr_mat *A, int32_t nrhs) {
  int path = env_path();
  if (path == VBCSR_PATH_AUTO) path = A->opts.path;
  if (A->prec == VBCSR_BF16X3) return {Kind::Bf16x3, nrhs <= 16 ? 1 : nrhs <= 32 ? 2 : 4};
  bool vec = path == VBCSR_PATH_VEC || (path == VBCSR_PATH_AUTO && nrhs <= 8);
  if (vec) {
    int t = A->opts.nrhs_tile;
    if (t != 1 && t != 2 && t != 4 && t != 8) t = nrhs <= 1 ? 1 : nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : 8;
    return {Kind::Vec, t};
  }
  return {Kind::Mfma, nrhs <= 16 ? 1 : nrhs <= 32 ? 2 : 4};
}

// One product over the panels of direction d.
int product(const vbcsr_mat *A, int d, const void *X, int64_t ldx, const void *Yin, int64_t ldyin,
            void *Yout, int64_t ldy, int32_t nrhs, double alpha, double beta, const void *R,
            int64_t ldr, double *mom, hipStream_t s) {
  if (d == 1 && A->tr_stale)
    return fail(VBCSR_EINVAL, "the transposed pages are stale: call vbcsr_refresh_transposed");
  const DevDir &D = A->dir[d];
  const Route rt = route(A, nrhs);
  hipError_t e;
  if (A->prec == VBCSR_FP64) {
    FwdParams<double> p{};
    p.rows = D.rows;
    p.nrows = D.npanels;
    p.colx = D.colx;
    p.vals = static_cast<const double *>(D.vals);
    p.X = static_cast<const double *>(X);
    p.ldx = ldx;
    p.xrows = in_rows(A, d);
    p.Yin = static_cast<const double *>(Yin);
    p.ldyin = ldyin;
    p.Yout = static_cast<double *>(Yout);
    p.ldy = ldy;
    p.nrhs = nrhs;
    p.alpha = alpha;
    p.beta = beta;
    p.R = static_cast<const double *>(R);
    p.ldr = ldr;
    p.mom = mom;
    e = launch_spmm_f64(p, rt.kind, rt.tile, s);
  } else {
    FwdParams<float> p{};
    p.rows = D.rows;
    p.nrows = D.npanels;
    p.colx = D.colx;
    p.vals = static_cast<const float *>(D.vals);
    p.hi = D.hi;
    p.lo = D.lo;
    p.vbase16 = D.vbase16;
    p.X = static_cast<const float *>(X);
    p.ldx = ldx;
    p.xrows = in_rows(A, d);
    p.Yin = static_cast<const float *>(Yin);
    p.ldyin = ldyin;
    p.Yout = static_cast<float *>(Yout);
    p.ldy = ldy;
    p.nrhs = nrhs;
    p.alpha = alpha;
    p.beta = beta;
    p.R = static_cast<const float *>(R);
    p.ldr = ldr;
    p.mom = mom;
    e = launch_spmm_f32(p, rt.kind, rt.tile, s);
  }
  if (e != hipSuccess) return hip_fail(e, "product kernel launch");
  return VBCSR_OK;
}

int plan_checked(int32_t n, const int32_t *b, const int64_t *row_ptr, const int32_t *col_idx,
                 int64_t n_values, const vbcsr_plan_opts *opts, HostPlan &plan,
                 bool with_columns, int32_t n_rows = -1) {
  std::string err;
  if (opts && (opts->row_order < VBCSR_ORDER_AUTO || opts->row_order > VBCSR_ORDER_CLUSTER))
    return fail(VBCSR_EINVAL, "row_order must be one of VBCSR_ORDER_*");
  int rc = validate_graph(n, b, row_ptr, col_idx, n_values, err);
  if (rc) return fail(rc, err);
  build_plan(n, b, row_ptr, col_idx, opts ? opts->row_order : VBCSR_ORDER_AUTO, plan,
             with_columns, n_rows);
  return VBCSR_OK;
}

// Column tables and zeroed value pages of direction d, once its panel
// descriptors, per-block maps (and BF16 panel bases) are on the device.
int finish_direction(vbcsr_mat *A, int d, int64_t n_cols, hipStream_t s) {
  DevDir &D = A->dir[d];
  int rc;
  // 4 entries of slack: a kernel may read a panel's indices in groups of
  // four (never using those past the panel)
  if ((rc = alloc_into(A, &D.colx, (size_t)n_cols + 4))) return rc;
  if (d == 0 && (rc = alloc_into(A, &D.colg, (size_t)n_cols))) return rc;
  {
    ColumnParams cp{};
    cp.rows = D.rows;
    cp.prow = D.blk_prow;
    cp.k0 = D.blk_k0;
    cp.catom = d == 0 ? A->col_idx : A->blk_row;
    cp.b = A->b;
    cp.off = A->off;
    cp.gbase = d == 0 ? A->gbase : nullptr;
    cp.nnzb = A->nnzb;
    cp.colx = D.colx;
    cp.colg = d == 0 ? D.colg : nullptr;
    hipError_t e = launch_columns(cp, s);
    if (e != hipSuccess) return hip_fail(e, "column table kernel launch");
  }
  if (A->prec == VBCSR_BF16X3) {
    if ((rc = alloc_into(A, &D.hi, (size_t)D.n_values16))) return rc;
    if ((rc = alloc_into(A, &D.lo, (size_t)D.n_values16))) return rc;
    if (D.n_values16) {
      hipError_t e = hipMemsetAsync(D.hi, 0, sizeof(uint16_t) * D.n_values16, s);
      if (e == hipSuccess) e = hipMemsetAsync(D.lo, 0, sizeof(uint16_t) * D.n_values16, s);
      if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    }
  } else {
    const size_t es = A->prec == VBCSR_FP64 ? 8 : 4;
    char *p = nullptr;
    // kPageSlack values after the pages: 16-byte reads that start on a
    // block's last value stay inside the allocation
    const size_t bytes = es * (size_t)(D.n_values + kPageSlack);
    if ((rc = alloc_into(A, &p, bytes))) return rc;
    // the padding after each panel must read as zero; every value position
    // is written by the packing that follows
    hipError_t e = launch_zero_gaps(D.rows, D.npanels, D.n_values, (int)es, p, s);
    if (e != hipSuccess) return hip_fail(e, "gap kernel launch");
    D.vals = p;
  }
  return VBCSR_OK;
}

// Shared by vbcsr_create (host values) and the block product (device values
// in graph order).
int create_impl(vbcsr_mat **out, int32_t n_atoms, const int32_t *block_sizes,
                const int64_t *row_ptr, const int32_t *col_idx, const void *values,
                bool values_on_device, int64_t n_values, vbcsr_prec prec,
                const vbcsr_plan_opts *opts, void *stream, int32_t n_rows = -1) {
  if (!out) return fail(VBCSR_EINVAL, "out is NULL");
  *out = nullptr;
  if (prec != VBCSR_FP64 && prec != VBCSR_FP32 && prec != VBCSR_BF16X3)
    return fail(VBCSR_EINVAL, "unknown precision");
  if (opts && (opts->rows_per_wg != 0 || opts->path < 0 || opts->path > VBCSR_PATH_MFMA))
    return fail(VBCSR_EINVAL, "invalid plan options");
  HostPlan plan;
  // column tables are built on the device from the per-block maps
  int rc = plan_checked(n_atoms, block_sizes, row_ptr, col_idx, n_values, opts, plan, false,
                        n_rows);
  if (rc) return rc;

  hipStream_t s = static_cast<hipStream_t>(stream);
  vbcsr_mat *A = new vbcsr_mat();
  // frees the partial handle on every early return and on an exception
  struct Guard {
    vbcsr_mat *&h;
    ~Guard() {
      if (h) {
        free_all(h);
        delete h;
      }
    }
  } guard{A};
  A->n = n_atoms;
  A->n_rows = plan.n_rows;
  A->N = plan.N;
  A->N_rows = plan.N_rows;
  A->nnzb = plan.nnzb;
  A->nnz = plan.nnz;
  A->n_shapes = (int32_t)plan.shapes.size();
  A->prec = prec;
  if (opts) A->opts = *opts;

  auto bail = [&](int code) { return code; };
  std::vector<int32_t> bvec(block_sizes, block_sizes + n_atoms);
  std::vector<int32_t> offv((size_t)n_atoms);
  for (int32_t i = 0; i < n_atoms; ++i) offv[i] = (int32_t)plan.off[i];
  if ((rc = upload_into(A, &A->b, bvec, s))) return bail(rc);
  if ((rc = upload_into(A, &A->off, offv, s))) return bail(rc);
  if ((rc = upload_into(A, &A->row_ptr, row_ptr, (size_t)n_atoms + 1, s))) return bail(rc);
  if ((rc = upload_into(A, &A->col_idx, col_idx, (size_t)plan.nnzb, s))) return bail(rc);
  if ((rc = upload_into(A, &A->blk_row, plan.blk_row, s))) return bail(rc);
  if ((rc = upload_into(A, &A->gbase, plan.gbase.data(), (size_t)plan.nnzb, s))) return bail(rc);
  for (int d = 0; d < 2; ++d) {
    const DirPlan &P = d == 0 ? plan.fwd : plan.tr;
    DevDir &D = A->dir[d];
    D.n_values = P.n_values;
    D.n_values16 = P.n_values16;
    D.npanels = (int32_t)P.rows.size();
    if ((rc = upload_into(A, &D.rows, P.rows, s))) return bail(rc);
    if ((rc = upload_into(A, &D.blk_pos, P.blk_pos, s))) return bail(rc);
    if ((rc = upload_into(A, &D.blk_k0, P.blk_k0, s))) return bail(rc);
    if ((rc = upload_into(A, &D.blk_prow, P.blk_prow, s))) return bail(rc);
    if (prec == VBCSR_BF16X3 && (rc = upload_into(A, &D.vbase16, P.vbase16, s))) return bail(rc);
    if ((rc = finish_direction(A, d, P.n_cols, s))) return bail(rc);
  }
  // initial values: host graph order -> device staging -> pages
  if (plan.nnz > 0 && values_on_device) {
    rc = pack_all(A, values, 0, s);
    hipError_t e = hipStreamSynchronize(s);
    if (rc) return bail(rc);
    if (e != hipSuccess) return bail(hip_fail(e, "create"));
  } else if (plan.nnz > 0) {
    double *stage = nullptr;
    if ((rc = dev_alloc(reinterpret_cast<void **>(&stage), sizeof(double) * plan.nnz))) return bail(rc);
    hipError_t e = values ? hipMemcpyAsync(stage, values, sizeof(double) * plan.nnz,
                                           hipMemcpyHostToDevice, s)
                          : hipMemsetAsync(stage, 0, sizeof(double) * plan.nnz, s);
    if (e == hipSuccess) {
      rc = pack_all(A, stage, 0, s);
      e = hipStreamSynchronize(s);
    }
    (void)hipFree(stage);
    if (rc) return bail(rc);
    if (e != hipSuccess) return bail(hip_fail(e, "create"));
  } else {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(hip_fail(e, "create"));
  }
  *out = A;
  A = nullptr;  // owned by the caller now
  return VBCSR_OK;
}

// An FP64 operator over A's atoms whose block graph is already on the device
// (row pointer d_rp, n + 1 entries; columns d_ci, ascending within each row)
// with graph-order values d_vals (n_values of them): planned on the device in
// the processing order d_order (a permutation of the atoms), so the pattern
// never passes through the host.  d_vals null: the pages are left for the
// caller to fill (their gaps are zero).
int create_planned_on_device(vbcsr_mat **out, const vbcsr_mat *A, int64_t nnzb, int64_t n_values,
                             const int64_t *d_rp, const int32_t *d_ci, const double *d_vals,
                             const int32_t *d_order, const vbcsr_plan_opts *opts,
                             const DevAlloc &tmp_alloc, hipStream_t s) {
  *out = nullptr;
  vbcsr_mat *C = new vbcsr_mat();
  struct Guard {
    vbcsr_mat *&h;
    ~Guard() {
      if (h) {
        free_all(h);
        delete h;
      }
    }
  } guard{C};
  const int32_t n = A->n;
  C->n = n;
  C->n_rows = n;
  C->N = A->N;
  C->N_rows = A->N;
  C->nnzb = nnzb;
  C->prec = VBCSR_FP64;
  if (opts) C->opts = *opts;
  int rc;
  if ((rc = alloc_into(C, &C->b, (size_t)n)) || (rc = alloc_into(C, &C->off, (size_t)n)) ||
      (rc = alloc_into(C, &C->row_ptr, (size_t)n + 1)) ||
      (rc = alloc_into(C, &C->col_idx, (size_t)nnzb)) ||
      (rc = alloc_into(C, &C->blk_row, (size_t)nnzb)) ||
      (rc = alloc_into(C, &C->gbase, (size_t)nnzb + 1)))
    return rc;
  HIP_TRY(hipMemcpyAsync(C->b, A->b, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
  HIP_TRY(hipMemcpyAsync(C->off, A->off, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s),
          "hipMemcpyAsync");
  HIP_TRY(hipMemcpyAsync(C->row_ptr, d_rp, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s),
          "hipMemcpyAsync");
  if (nnzb)
    HIP_TRY(hipMemcpyAsync(C->col_idx, d_ci, sizeof(int32_t) * nnzb, hipMemcpyDeviceToDevice, s),
            "hipMemcpyAsync");
  DevPlanIn pin{n, nnzb, C->b, C->off, C->row_ptr, C->col_idx, d_order};
  DevPlanOut po{};
  po.blk_row = C->blk_row;
  po.gbase = C->gbase;
  for (int d = 0; d < 2; ++d) {
    DevDir &D = C->dir[d];
    if ((rc = alloc_into(C, &D.rows, (size_t)n)) || (rc = alloc_into(C, &D.blk_pos, (size_t)nnzb)) ||
        (rc = alloc_into(C, &D.blk_k0, (size_t)nnzb)) ||
        (rc = alloc_into(C, &D.blk_prow, (size_t)nnzb)))
      return rc;
    po.dir[d].rows = D.rows;
    po.dir[d].blk_pos = D.blk_pos;
    po.dir[d].blk_k0 = D.blk_k0;
    po.dir[d].blk_prow = D.blk_prow;
  }
  {
    hipError_t e = plan_device(pin, po, tmp_alloc, s);
    if (e == hipErrorInvalidValue) return fail(VBCSR_EUNSUPPORTED, "the product has 2^31 or more blocks");
    if (e != hipSuccess) return hip_fail(e, "device plan");
  }
  if (po.nnz != n_values) return fail(VBCSR_ESHAPE, "product values do not match its pattern");
  // the same limit as validate_graph: one panel within 2^31 bytes in FP64
  constexpr int64_t kPanelMax = (int64_t(1) << 31) / 8;
  if (po.dir[0].max_panel >= kPanelMax)
    return fail(VBCSR_EUNSUPPORTED, "a block row of the product holds 2^28 or more values");
  if (po.dir[1].max_panel >= kPanelMax)
    return fail(VBCSR_EUNSUPPORTED, "a block column of the product holds 2^28 or more values");
  C->nnz = po.nnz;
  C->n_shapes = po.n_shapes;
  for (int d = 0; d < 2; ++d) {
    DevDir &D = C->dir[d];
    D.n_values = po.dir[d].n_values;
    D.n_values16 = 0;
    D.npanels = n;
    if ((rc = finish_direction(C, d, po.dir[d].n_cols, s))) return rc;
  }
  if (C->nnz > 0 && d_vals && (rc = pack_all(C, d_vals, 0, s))) return rc;
  HIP_TRY(hipStreamSynchronize(s), "spgemm");
  *out = C;
  C = nullptr;  // owned by the caller now
  return VBCSR_OK;
}


// Device allocations that live for one call; freed (after the stream has
// been synchronised by the caller) when the object goes out of scope.
struct TempAllocs {
  std::vector<void *> ptrs;
  template <typename T>
  int alloc(T **p, size_t count) {
    int rc = dev_alloc(reinterpret_cast<void **>(p), sizeof(T) * count);
    if (rc == VBCSR_OK && *p) ptrs.push_back(*p);
    return rc;
  }
  template <typename T, typename Alloc>
  int up(T **p, const std::vector<T, Alloc> &v, hipStream_t s) {
    int rc = upload(p, v, s);
    if (rc == VBCSR_OK && *p) ptrs.push_back(*p);
    return rc;
  }
  ~TempAllocs() {
    for (void *p : ptrs) (void)hipFree(p);
  }
};

template <typename T>
int d2h(std::vector<T> &dst, const T *src, size_t count, hipStream_t s) {
  dst.resize(count);
  if (count == 0) return VBCSR_OK;
  HIP_TRY(hipMemcpyAsync(dst.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost, s),
          "hipMemcpyAsync");
  return VBCSR_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

const char *vbcsr_last_error(void) { return g_last_error.c_str(); }

int vbcsr_plan_host(int32_t n_atoms, const int32_t *block_sizes, const int64_t *row_ptr,
                    const int32_t *col_idx, int64_t n_values, int32_t *n_shapes, int32_t *shapes,
                    int32_t max_shapes, int64_t *fwd_pos, int64_t *tr_pos, int64_t *page_values,
                    const vbcsr_plan_opts *opts) try {
  HostPlan plan;
  int rc = plan_checked(n_atoms, block_sizes, row_ptr, col_idx, n_values, opts, plan, false);
  if (rc) return rc;
  if (n_shapes) *n_shapes = (int32_t)plan.shapes.size();
  if (shapes)
    for (int32_t t = 0; t < std::min<int32_t>(max_shapes, (int32_t)plan.shapes.size()); ++t)
      for (int c = 0; c < 3; ++c) shapes[3 * t + c] = plan.shapes[t][c];
  if (fwd_pos) std::copy(plan.fwd.blk_pos.begin(), plan.fwd.blk_pos.end(), fwd_pos);
  if (tr_pos) std::copy(plan.tr.blk_pos.begin(), plan.tr.blk_pos.end(), tr_pos);
  if (page_values) *page_values = plan.fwd.n_values;
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_plan_host");
}

int vbcsr_create(vbcsr_mat **out, int32_t n_atoms, const int32_t *block_sizes,
                 const int64_t *row_ptr, const int32_t *col_idx, const double *values,
                 int64_t n_values, vbcsr_prec prec, const vbcsr_plan_opts *opts, void *stream) try {
  return create_impl(out, n_atoms, block_sizes, row_ptr, col_idx, values, false, n_values, prec,
                     opts, stream);
} catch (...) {
  return api_exception("vbcsr_create");
}

int vbcsr_create_local(vbcsr_mat **out, int32_t n_owned, int32_t n_ghost,
                       const int32_t *block_sizes, const int64_t *row_ptr, const int32_t *col_idx,
                       const double *values, int64_t n_values, vbcsr_prec prec,
                       const vbcsr_plan_opts *opts, void *stream) try {
  if (out) *out = nullptr;
  if (n_owned < 0 || n_ghost < 0) return fail(VBCSR_EINVAL, "n_owned and n_ghost must be >= 0");
  if ((int64_t)n_owned + n_ghost > INT32_MAX) return fail(VBCSR_EUNSUPPORTED, "more than 2^31-1 atoms");
  if (!row_ptr) return fail(VBCSR_EINVAL, "row_ptr is NULL");
  const int32_t n = n_owned + n_ghost;
  // the ghost atoms' rows are empty: the same graph as a square one over
  // owned + ghost atoms, with panels only for the owned rows
  std::vector<int64_t> rp((size_t)n + 1);
  std::copy(row_ptr, row_ptr + (size_t)n_owned + 1, rp.begin());
  std::fill(rp.begin() + n_owned + 1, rp.end(), row_ptr[n_owned]);
  return create_impl(out, n, block_sizes, rp.data(), col_idx, values, false, n_values, prec, opts,
                     stream, n_owned);
} catch (...) {
  return api_exception("vbcsr_create_local");
}

int vbcsr_shape(const vbcsr_mat *A, int32_t *n_row_atoms, int32_t *n_col_atoms, int64_t *n_rows,
                int64_t *n_cols) try {
  if (!A) return fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (n_row_atoms) *n_row_atoms = A->n_rows;
  if (n_col_atoms) *n_col_atoms = A->n;
  if (n_rows) *n_rows = A->N_rows;
  if (n_cols) *n_cols = A->N;
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_shape");
}

int vbcsr_set_values(vbcsr_mat *A, const void *values, int on_device, int dtype, void *stream) try {
  if (!A) return fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (dtype != 0 && dtype != 1) return fail(VBCSR_EINVAL, "dtype must be 0 (double) or 1 (float)");
  if (A->nnz == 0) return VBCSR_OK;
  if (!values) return fail(VBCSR_EINVAL, "values is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t es = dtype == 0 ? 8 : 4;
  // back to the handle's own forward pages; both page sets are rewritten
  if (A->own_fwd) {
    A->dir[0].vals = A->own_fwd;
    A->own_fwd = nullptr;
  }
  A->tr_stale = false;
  if (on_device) return pack_all(A, values, dtype, s);
  void *stage = nullptr;
  int rc = dev_alloc(&stage, es * A->nnz);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(stage, values, es * A->nnz, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    rc = pack_all(A, stage, dtype, s);
    e = hipStreamSynchronize(s);
  }
  (void)hipFree(stage);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "set_values");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_set_values");
}

int vbcsr_spmm(const vbcsr_mat *A, const void *X, int64_t ldx, void *Y, int64_t ldy, int32_t nrhs,
               double alpha, double beta, void *stream) try {
  int rc = A ? check_vectors(A, X, in_rows(A, 0), ldx, Y, out_rows(A, 0), ldy, nrhs, true)
             : fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (rc || out_rows(A, 0) == 0) return rc;
  return product(A, 0, X, ldx, Y, ldy, Y, ldy, nrhs, alpha, beta, nullptr, 0, nullptr,
                 static_cast<hipStream_t>(stream));
} catch (...) {
  return api_exception("vbcsr_spmm");
}

int vbcsr_spmm_t(const vbcsr_mat *A, const void *X, int64_t ldx, void *Y, int64_t ldy,
                 int32_t nrhs, double alpha, double beta, void *stream) try {
  int rc = A ? check_vectors(A, X, in_rows(A, 1), ldx, Y, out_rows(A, 1), ldy, nrhs, true)
             : fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (rc || out_rows(A, 1) == 0) return rc;
  return product(A, 1, X, ldx, Y, ldy, Y, ldy, nrhs, alpha, beta, nullptr, 0, nullptr,
                 static_cast<hipStream_t>(stream));
} catch (...) {
  return api_exception("vbcsr_spmm_t");
}

int vbcsr_sddmm(const vbcsr_mat *A, const void *dY, int64_t lddy, const void *X, int64_t ldx,
                int32_t nrhs, void *dA, void *stream) try {
  // dY is shaped like the forward output, X like the forward input
  int rc = A ? check_vectors(A, dY, A->N_rows, lddy, X, A->N, ldx, nrhs, false)
             : fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (rc) return rc;
  if (A->nnz == 0) return VBCSR_OK;
  if (!dA) return fail(VBCSR_EINVAL, "dA is NULL");
  const size_t e = vec_elem(A);
  const size_t abytes = e * (size_t)A->nnz;
  if (ranges_overlap(dA, abytes, dY, span_bytes(A->N_rows, lddy, nrhs, e)) ||
      ranges_overlap(dA, abytes, X, span_bytes(A->N, ldx, nrhs, e)))
    return fail(VBCSR_EINVAL, "dA overlaps an input");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t err;
  const DevDir &D = A->dir[0];
  if (A->prec == VBCSR_FP64) {
    SddmmParams<double> p{D.rows, D.npanels, D.colx, D.colg, static_cast<const double *>(dY), lddy,
                          static_cast<const double *>(X), ldx, nrhs, static_cast<double *>(dA),
                          A->N};
    err = launch_sddmm_f64(p, s);
  } else {
    SddmmParams<float> p{D.rows, D.npanels, D.colx, D.colg, static_cast<const float *>(dY), lddy,
                         static_cast<const float *>(X), ldx, nrhs, static_cast<float *>(dA),
                         A->N};
    err = launch_sddmm_f32(p, s);
  }
  if (err != hipSuccess) return hip_fail(err, "sddmm kernel launch");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_sddmm");
}

int vbcsr_page_size(const vbcsr_mat *A, int64_t *n_page_values) try {
  if (!A || !n_page_values) return fail(VBCSR_EINVAL, "NULL argument");
  if (A->prec == VBCSR_BF16X3)
    return fail(VBCSR_EUNSUPPORTED, "BF16X3 handles keep hi/lo pages: no page-layout values");
  *n_page_values = A->dir[0].n_values + kPageSlack;
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_page_size");
}

int vbcsr_get_pages(const vbcsr_mat *A, void *pages, void *stream) try {
  int64_t n = 0;
  if (int rc = vbcsr_page_size(A, &n)) return rc;
  if (!pages) return fail(VBCSR_EINVAL, "pages is NULL");
  HIP_TRY(hipMemcpyAsync(pages, A->dir[0].vals, vec_elem(A) * (size_t)n, hipMemcpyDeviceToDevice,
                         static_cast<hipStream_t>(stream)),
          "hipMemcpyAsync");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_get_pages");
}

int vbcsr_use_pages(vbcsr_mat *A, const void *pages) try {
  int64_t n = 0;
  if (int rc = vbcsr_page_size(A, &n)) return rc;
  if (pages) {
    if (!A->own_fwd) A->own_fwd = A->dir[0].vals;
    A->dir[0].vals = const_cast<void *>(pages);
  } else if (A->own_fwd) {
    A->dir[0].vals = A->own_fwd;
    A->own_fwd = nullptr;
  }
  A->tr_stale = true;
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_use_pages");
}

int vbcsr_refresh_transposed(vbcsr_mat *A, void *stream) try {
  int64_t n = 0;
  if (int rc = vbcsr_page_size(A, &n)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevDir &D = A->dir[1];
  const int es = A->prec == VBCSR_FP64 ? 8 : 4;
  if (A->nnz > 0 && !D.page_recs) {
    // first call: the blocks' maps in transposed-page order (the rebuild
    // walks the pages it writes)
    PageRec *recs = nullptr;
    int rc;
    if ((rc = dev_alloc(reinterpret_cast<void **>(&recs), sizeof(PageRec) * A->nnzb))) return rc;
    std::vector<void *> tmp;
    const DevAlloc alloc = [&](void **q, size_t bytes) -> hipError_t {
      if (dev_alloc(q, bytes) != VBCSR_OK) return hipErrorOutOfMemory;
      tmp.push_back(*q);
      return hipSuccess;
    };
    int32_t *order = nullptr;
    hipError_t e = alloc(reinterpret_cast<void **>(&order), sizeof(int32_t) * A->nnzb);
    if (e == hipSuccess) e = launch_page_order(D.blk_pos, A->nnzb, D.n_values, order, alloc, s);
    if (e == hipSuccess) {
      PackParams pp{};
      pp.b = A->b;
      pp.blk_row = A->blk_row;
      pp.col_idx = A->col_idx;
      pp.nnzb = A->nnzb;
      pp.dir[0].pos = A->dir[0].blk_pos;
      pp.dir[1].pos = D.blk_pos;
      e = launch_refresh_records(pp, order, recs, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (void *q : tmp) (void)hipFree(q);
    if (e != hipSuccess) {
      (void)hipFree(recs);
      return hip_fail(e, "page records");
    }
    A->owned.push_back(recs);
    D.page_recs = recs;
  }
  if (A->nnz > 0) {
    hipError_t e = launch_refresh(D.page_recs, A->nnzb, es, A->dir[0].vals, D.vals, s);
    if (e != hipSuccess) return hip_fail(e, "refresh kernel launch");
  }
  A->tr_stale = false;
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_refresh_transposed");
}

int vbcsr_sddmm_pages(const vbcsr_mat *A, const void *dY, int64_t lddy, const void *X,
                      int64_t ldx, int32_t nrhs, void *dA, void *stream) try {
  int64_t n = 0;
  if (int rc = vbcsr_page_size(A, &n)) return rc;
  if (int rc = check_vectors(A, dY, A->N_rows, lddy, X, A->N, ldx, nrhs, false)) return rc;
  if (!dA) return fail(VBCSR_EINVAL, "dA is NULL");
  const size_t e = vec_elem(A);
  const size_t abytes = e * (size_t)n;
  if (ranges_overlap(dA, abytes, dY, span_bytes(A->N_rows, lddy, nrhs, e)) ||
      ranges_overlap(dA, abytes, X, span_bytes(A->N, ldx, nrhs, e)))
    return fail(VBCSR_EINVAL, "dA overlaps an input");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevDir &D = A->dir[0];
  hipError_t err = hipSuccess;
  if (A->nnz > 0) {
    if (A->prec == VBCSR_FP64) {
      SddmmParams<double> p{D.rows, D.npanels, D.colx, D.colg, static_cast<const double *>(dY),
                            lddy, static_cast<const double *>(X), ldx, nrhs,
                            static_cast<double *>(dA), A->N, 1};
      err = launch_sddmm_f64(p, s);
    } else {
      SddmmParams<float> p{D.rows, D.npanels, D.colx, D.colg, static_cast<const float *>(dY),
                           lddy, static_cast<const float *>(X), ldx, nrhs,
                           static_cast<float *>(dA), A->N, 1};
      err = launch_sddmm_f32(p, s);
    }
    if (err != hipSuccess) return hip_fail(err, "sddmm kernel launch");
  }
  // the gaps between panels and the slack read as zero
  err = launch_zero_gaps(D.rows, D.npanels, D.n_values, (int)e, dA, s);
  if (err != hipSuccess) return hip_fail(err, "gap kernel launch");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_sddmm_pages");
}

int vbcsr_cheb_workspace_bytes(const vbcsr_mat *A, int32_t nrhs, int32_t degree, int64_t *bytes) try {
  if (!A || !bytes) return fail(VBCSR_EINVAL, "NULL argument");
  if (int rc = require_square(A, "vbcsr_cheb_workspace_bytes")) return rc;
  if (nrhs <= 0) return fail(VBCSR_EINVAL, "nrhs must be >= 1");
  if (degree < 0) return fail(VBCSR_EINVAL, "degree must be >= 0");
  const int64_t vec = ((int64_t)vec_elem(A) * A->N * nrhs + 255) / 256 * 256;
  const int64_t parts = std::max(product_workgroups(A->n), coldot_chunks(A->N));
  // two recurrence vectors, the per-workgroup partial moments, all moments
  *bytes = 2 * vec + 8 * parts * nrhs + 8 * (int64_t)(degree + 1) * nrhs;
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_cheb_workspace_bytes");
}

int vbcsr_cheb_moments(const vbcsr_mat *A, const void *R, int64_t ldr, int32_t nrhs,
                       int32_t degree, double *mu_host, void *workspace, int64_t ws_bytes,
                       void *stream) try {
  if (!A) return fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (int rc = require_square(A, "Chebyshev moments")) return rc;
  if (nrhs <= 0 || nrhs > 4096) return fail(VBCSR_EINVAL, "nrhs must be in [1, 4096]");
  if (ldr < nrhs) return fail(VBCSR_EINVAL, "ldr smaller than nrhs");
  if (degree < 0) return fail(VBCSR_EINVAL, "degree must be >= 0");
  if (!mu_host) return fail(VBCSR_EINVAL, "mu_host is NULL");
  if (A->N > 0 && !R) return fail(VBCSR_EINVAL, "R is NULL");
  int64_t need = 0;
  int rc = vbcsr_cheb_workspace_bytes(A, nrhs, degree, &need);
  if (rc) return rc;
  if (workspace && ws_bytes < need) return fail(VBCSR_EINVAL, "workspace too small");
  if (workspace && A->N > 0 &&
      ranges_overlap(workspace, (size_t)need, R, span_bytes(A->N, ldr, nrhs, vec_elem(A))))
    return fail(VBCSR_EINVAL, "R overlaps the workspace");
  if (A->N == 0) {
    std::fill(mu_host, mu_host + (size_t)(degree + 1) * nrhs, 0.0);
    return VBCSR_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  void *ws = workspace;
  if (!ws && (rc = dev_alloc(&ws, (size_t)need))) return rc;
  const int64_t vec = ((int64_t)vec_elem(A) * A->N * nrhs + 255) / 256 * 256;
  const int64_t nparts = std::max(product_workgroups(A->n), coldot_chunks(A->N));
  char *base = static_cast<char *>(ws);
  void *Ta = base;
  void *Tb = base + vec;
  double *parts = reinterpret_cast<double *>(base + 2 * vec);
  double *all_mu = parts + nparts * nrhs;
  std::vector<double> mu((size_t)(degree + 1) * nrhs);
  // mu_0 = <R, R>
  int64_t nch = 0;
  hipError_t e;
  if (A->prec == VBCSR_FP64)
    e = launch_coldot_f64(static_cast<const double *>(R), ldr, static_cast<const double *>(R), ldr,
                          A->N, nrhs, parts, &nch, s);
  else
    e = launch_coldot_f32(static_cast<const float *>(R), ldr, static_cast<const float *>(R), ldr,
                          A->N, nrhs, parts, &nch, s);
  if (e == hipSuccess) e = launch_reduce_partials(parts, nch, nrhs, all_mu, s);
  const int64_t npw = product_workgroups(A->n);
  // T_1 = A R; T_k = 2 A T_{k-1} - T_{k-2} written over the buffer of T_{k-2}
  // (each element is read once, by the thread that overwrites it), except at
  // k == 2 where T_0 is the caller's R.
  const void *prev = R;  // T_{k-2}
  int64_t ldprev = ldr;
  void *cur = Ta;        // T_{k-1}
  for (int32_t k = 1; k <= degree && e == hipSuccess && rc == VBCSR_OK; ++k) {
    if (k == 1) {
      rc = product(A, 0, R, ldr, Ta, nrhs, Ta, nrhs, nrhs, 1.0, 0.0, R, ldr, parts, s);
    } else {
      void *dst = (k == 2) ? Tb : const_cast<void *>(prev);
      rc = product(A, 0, cur, nrhs, prev, ldprev, dst, nrhs, nrhs, 2.0, -1.0, R, ldr, parts, s);
      prev = cur;
      ldprev = nrhs;
      cur = dst;
    }
    if (rc == VBCSR_OK) e = launch_reduce_partials(parts, npw, nrhs, all_mu + (size_t)k * nrhs, s);
  }
  if (e == hipSuccess && rc == VBCSR_OK)
    e = hipMemcpyAsync(mu.data(), all_mu, sizeof(double) * mu.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (!workspace) (void)hipFree(ws);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "cheb_moments");
  std::copy(mu.begin(), mu.end(), mu_host);
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_cheb_moments");
}

int vbcsr_cheb_moments_doubled(const vbcsr_mat *A, const void *R, int64_t ldr, int32_t nrhs,
                               int32_t degree, double *mu_host, void *workspace, int64_t ws_bytes,
                               void *stream) try {
  if (!A) return fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (int rc = require_square(A, "Chebyshev moments")) return rc;
  if (nrhs <= 0 || nrhs > 4096) return fail(VBCSR_EINVAL, "nrhs must be in [1, 4096]");
  if (ldr < nrhs) return fail(VBCSR_EINVAL, "ldr smaller than nrhs");
  if (degree < 0) return fail(VBCSR_EINVAL, "degree must be >= 0");
  if (!mu_host) return fail(VBCSR_EINVAL, "mu_host is NULL");
  if (A->N > 0 && !R) return fail(VBCSR_EINVAL, "R is NULL");
  int64_t need = 0;
  int rc = vbcsr_cheb_workspace_bytes(A, nrhs, degree, &need);
  if (rc) return rc;
  if (workspace && ws_bytes < need) return fail(VBCSR_EINVAL, "workspace too small");
  if (workspace && A->N > 0 &&
      ranges_overlap(workspace, (size_t)need, R, span_bytes(A->N, ldr, nrhs, vec_elem(A))))
    return fail(VBCSR_EINVAL, "R overlaps the workspace");
  if (A->N == 0) {
    std::fill(mu_host, mu_host + (size_t)(degree + 1) * nrhs, 0.0);
    return VBCSR_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  void *ws = workspace;
  if (!ws && (rc = dev_alloc(&ws, (size_t)need))) return rc;
  const int64_t vec = ((int64_t)vec_elem(A) * A->N * nrhs + 255) / 256 * 256;
  char *base = static_cast<char *>(ws);
  void *Ta = base;
  void *Tb = base + vec;
  double *parts = reinterpret_cast<double *>(base + 2 * vec);
  const int64_t nparts = std::max(product_workgroups(A->n), coldot_chunks(A->N));
  // raw[n]: <R,R> (n = 0), <T_{k-1},T_k> (n = 2k-1), <T_k,T_k> (n = 2k)
  double *raw = parts + nparts * nrhs;
  auto coldot = [&](const void *U, int64_t ldu, const void *V, int64_t ldv, double *out) {
    int64_t nch = 0;
    hipError_t e2 = A->prec == VBCSR_FP64
                        ? launch_coldot_f64(static_cast<const double *>(U), ldu,
                                            static_cast<const double *>(V), ldv, A->N, nrhs, parts,
                                            &nch, s)
                        : launch_coldot_f32(static_cast<const float *>(U), ldu,
                                            static_cast<const float *>(V), ldv, A->N, nrhs, parts,
                                            &nch, s);
    if (e2 == hipSuccess) e2 = launch_reduce_partials(parts, nch, nrhs, out, s);
    return e2;
  };
  hipError_t e = coldot(R, ldr, R, ldr, raw);
  const int64_t npw = product_workgroups(A->n);
  // T_k for k = 1 .. ceil(degree / 2), each written over T_{k-2} as in the
  // plain recurrence; the product's moment epilogue weights T_k by T_{k-1}
  const int32_t kmax = (degree + 1) / 2;
  const void *prev = R;  // T_{k-2}
  int64_t ldprev = ldr;
  const void *cur = R;   // T_{k-1}
  int64_t ldcur = ldr;
  for (int32_t k = 1; k <= kmax && e == hipSuccess && rc == VBCSR_OK; ++k) {
    void *dst;
    if (k == 1) {
      dst = Ta;
      rc = product(A, 0, R, ldr, Ta, nrhs, Ta, nrhs, nrhs, 1.0, 0.0, R, ldr, parts, s);
    } else {
      dst = (k == 2) ? Tb : const_cast<void *>(prev);
      rc = product(A, 0, cur, ldcur, prev, ldprev, dst, nrhs, nrhs, 2.0, -1.0, cur, ldcur, parts, s);
    }
    if (rc) break;
    e = launch_reduce_partials(parts, npw, nrhs, raw + (size_t)(2 * k - 1) * nrhs, s);
    if (e == hipSuccess && 2 * k <= degree) e = coldot(dst, nrhs, dst, nrhs, raw + (size_t)(2 * k) * nrhs);
    prev = cur;
    ldprev = ldcur;
    cur = dst;
    ldcur = nrhs;
  }
  std::vector<double> r((size_t)(degree + 1) * nrhs);
  if (e == hipSuccess && rc == VBCSR_OK)
    e = hipMemcpyAsync(r.data(), raw, sizeof(double) * r.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (!workspace) (void)hipFree(ws);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "cheb_moments_doubled");
  // mu_0 = <R,R>, mu_1 = <R,T_1>, mu_2k = 2<T_k,T_k> - mu_0, mu_2k+1 = 2<T_k,T_k+1> - mu_1
  for (int32_t c = 0; c < nrhs; ++c) {
    const double mu0 = r[c];
    const double mu1 = degree >= 1 ? r[(size_t)nrhs + c] : 0.0;
    for (int32_t n = 0; n <= degree; ++n) {
      const double v = r[(size_t)n * nrhs + c];
      mu_host[(size_t)n * nrhs + c] = n <= 1 ? v : 2.0 * v - ((n & 1) ? mu1 : mu0);
    }
  }
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_cheb_moments_doubled");
}

int vbcsr_cheb_step(const vbcsr_mat *A, const void *Tk, int64_t ldt, void *Tprev, int64_t ldp,
                    const void *R, int64_t ldr, int32_t nrhs, double *mu_dev, void *workspace,
                    int64_t ws_bytes, void *stream) try {
  if (int rc = require_square(A, "vbcsr_cheb_step")) return rc;
  int rc = A ? check_vectors(A, Tk, A->N, ldt, Tprev, A->N, ldp, nrhs, true)
             : fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (rc) return rc;
  if (nrhs > 4096) return fail(VBCSR_EINVAL, "nrhs must be <= 4096");
  if (ldr < nrhs) return fail(VBCSR_EINVAL, "ldr smaller than nrhs");
  if (!mu_dev) return fail(VBCSR_EINVAL, "mu_dev is NULL");
  if (A->N == 0) return VBCSR_OK;
  if (!R) return fail(VBCSR_EINVAL, "R is NULL");
  int64_t need = 0;
  if ((rc = vbcsr_cheb_workspace_bytes(A, nrhs, 0, &need))) return rc;
  if (!workspace || ws_bytes < need) return fail(VBCSR_EINVAL, "workspace missing or too small");
  // the product writes Tprev and then reads R at the same element; the
  // partial moments are written into the workspace, the moments into mu_dev
  {
    const size_t e = vec_elem(A);
    const size_t tb = span_bytes(A->N, ldp, nrhs, e), rb = span_bytes(A->N, ldr, nrhs, e),
                 kb = span_bytes(A->N, ldt, nrhs, e), mb = sizeof(double) * (size_t)nrhs;
    if (ranges_overlap(R, rb, Tprev, tb)) return fail(VBCSR_EINVAL, "R overlaps Tprev");
    if (ranges_overlap(workspace, (size_t)need, Tprev, tb) ||
        ranges_overlap(workspace, (size_t)need, Tk, kb) ||
        ranges_overlap(workspace, (size_t)need, R, rb) ||
        ranges_overlap(workspace, (size_t)need, mu_dev, mb))
      return fail(VBCSR_EINVAL, "workspace overlaps a vector or mu_dev");
    if (ranges_overlap(mu_dev, mb, Tprev, tb) || ranges_overlap(mu_dev, mb, Tk, kb) ||
        ranges_overlap(mu_dev, mb, R, rb))
      return fail(VBCSR_EINVAL, "mu_dev overlaps a vector");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t vec = ((int64_t)vec_elem(A) * A->N * nrhs + 255) / 256 * 256;
  double *parts = reinterpret_cast<double *>(static_cast<char *>(workspace) + 2 * vec);
  rc = product(A, 0, Tk, ldt, Tprev, ldp, Tprev, ldp, nrhs, 2.0, -1.0, R, ldr, parts, s);
  if (rc) return rc;
  hipError_t e = launch_reduce_partials(parts, product_workgroups(A->n), nrhs, mu_dev, s);
  if (e != hipSuccess) return hip_fail(e, "moment reduction launch");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_cheb_step");
}

int vbcsr_cheb_step_noalloc(const vbcsr_mat *A, const void *Tk, int64_t ldt, void *Tprev,
                            int64_t ldp, const void *R, int64_t ldr, int32_t nrhs, double *mu_dev,
                            void *stream) try {
  if (int rc = require_square(A, "vbcsr_cheb_step_noalloc")) return rc;
  int rc = A ? check_vectors(A, Tk, A->N, ldt, Tprev, A->N, ldp, nrhs, true)
             : fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (rc) return rc;
  if (nrhs > 4096) return fail(VBCSR_EINVAL, "nrhs must be <= 4096");
  if (ldr < nrhs) return fail(VBCSR_EINVAL, "ldr smaller than nrhs");
  if (!mu_dev) return fail(VBCSR_EINVAL, "mu_dev is NULL");
  if (A->N == 0) return VBCSR_OK;
  if (!R) return fail(VBCSR_EINVAL, "R is NULL");
  {
    const size_t e = vec_elem(A);
    const size_t tb = span_bytes(A->N, ldp, nrhs, e), rb = span_bytes(A->N, ldr, nrhs, e),
                 kb = span_bytes(A->N, ldt, nrhs, e), mb = sizeof(double) * (size_t)nrhs;
    if (ranges_overlap(R, rb, Tprev, tb)) return fail(VBCSR_EINVAL, "R overlaps Tprev");
    if (ranges_overlap(mu_dev, mb, Tprev, tb) || ranges_overlap(mu_dev, mb, Tk, kb) ||
        ranges_overlap(mu_dev, mb, R, rb))
      return fail(VBCSR_EINVAL, "mu_dev overlaps a vector");
  }
  // the per-workgroup partial moments live in the library's static scratch
  const int64_t npw = product_workgroups(A->n);
  const int64_t need = (int64_t)sizeof(double) * npw * nrhs;
  if (need > (int64_t)kNoAllocScratchBytes)
    return fail(VBCSR_EUNSUPPORTED,
                "vbcsr_cheb_step_noalloc: " + std::to_string(need) +
                    " bytes of partial moments (ceil(n_atoms / 4) * nrhs doubles) exceed the " +
                    std::to_string(kNoAllocScratchBytes) + "-byte scratch");
  void *ptr = nullptr;
  size_t bytes = 0;
  hipError_t e = noalloc_scratch(&ptr, &bytes);
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *parts = static_cast<double *>(ptr);
  // every workgroup of the product writes all nrhs of its partials, so the
  // scratch needs no clearing
  rc = product(A, 0, Tk, ldt, Tprev, ldp, Tprev, ldp, nrhs, 2.0, -1.0, R, ldr, parts, s);
  if (rc) return rc;
  e = launch_reduce_partials(parts, npw, nrhs, mu_dev, s);
  if (e != hipSuccess) return hip_fail(e, "moment reduction launch");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_cheb_step_noalloc");
}

int vbcsr_info(const vbcsr_mat *A, int64_t *n_rows, int64_t *nnzb, int64_t *n_values,
               int32_t *n_shapes) try {
  if (!A) return fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (n_rows) *n_rows = A->N_rows;
  if (nnzb) *nnzb = A->nnzb;
  if (n_values) *n_values = A->nnz;
  if (n_shapes) *n_shapes = A->n_shapes;
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_info");
}

void vbcsr_destroy(vbcsr_mat *A) {
  if (!A) return;
  free_all(A);
  delete A;
}

int vbcsr_get_structure(const vbcsr_mat *A, int32_t *block_sizes, int64_t *row_ptr,
                        int32_t *col_idx) try {
  if (!A) return fail(VBCSR_EINVAL, "matrix handle is NULL");
  if ((A->n && (!block_sizes || !row_ptr)) || (A->nnzb && !col_idx))
    return fail(VBCSR_EINVAL, "output pointer is NULL");
  if (A->n) {
    HIP_TRY(hipMemcpy(block_sizes, A->b, sizeof(int32_t) * A->n, hipMemcpyDeviceToHost),
            "hipMemcpy");
    HIP_TRY(hipMemcpy(row_ptr, A->row_ptr, sizeof(int64_t) * (A->n_rows + 1), hipMemcpyDeviceToHost),
            "hipMemcpy");
  } else if (row_ptr) {
    row_ptr[0] = 0;
  }
  if (A->nnzb)
    HIP_TRY(hipMemcpy(col_idx, A->col_idx, sizeof(int32_t) * A->nnzb, hipMemcpyDeviceToHost),
            "hipMemcpy");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_get_structure");
}

int vbcsr_get_values(const vbcsr_mat *A, void *values, int dtype, void *stream) try {
  if (!A) return fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (A->prec == VBCSR_BF16X3)
    return fail(VBCSR_EUNSUPPORTED, "BF16X3 handles keep only the split pages");
  const int want = A->prec == VBCSR_FP64 ? 0 : 1;
  if (dtype != want) return fail(VBCSR_EINVAL, "dtype must match the handle (0 FP64, 1 FP32)");
  if (A->nnz == 0) return VBCSR_OK;
  if (!values) return fail(VBCSR_EINVAL, "values is NULL");
  const DevDir &D = A->dir[0];
  hipError_t e = launch_unpack(D.vals, A->prec == VBCSR_FP64 ? 8 : 4, D.blk_pos, A->blk_row,
                               A->col_idx, A->b, A->gbase, A->nnzb, values,
                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "unpack kernel launch");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_get_values");
}

int vbcsr_spgemm(vbcsr_mat **out, const vbcsr_mat *A, const vbcsr_mat *B, double eps,
                 const vbcsr_plan_opts *opts, vbcsr_spgemm_stats *stats, void *stream) try {
  using clk = std::chrono::steady_clock;
  if (!out) return fail(VBCSR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!A || !B) return fail(VBCSR_EINVAL, "matrix handle is NULL");
  if (!(eps >= 0.0)) return fail(VBCSR_EINVAL, "eps must be >= 0");
  if (A->prec != VBCSR_FP64 || B->prec != VBCSR_FP64)
    return fail(VBCSR_EUNSUPPORTED, "the block product takes FP64 handles");
  if (int rc2 = require_square(A, "vbcsr_spgemm")) return rc2;
  if (int rc2 = require_square(B, "vbcsr_spgemm")) return rc2;
  if (A->n != B->n) return fail(VBCSR_EINVAL, "A and B must be over the same atoms");
  if (A->tr_stale)
    return fail(VBCSR_EINVAL, "A's transposed pages are stale: call vbcsr_refresh_transposed");
  if (opts && (opts->rows_per_wg != 0 || opts->path < 0 || opts->path > VBCSR_PATH_MFMA ||
               opts->row_order < VBCSR_ORDER_AUTO || opts->row_order > VBCSR_ORDER_CLUSTER))
    return fail(VBCSR_EINVAL, "invalid plan options");
  vbcsr_spgemm_stats st{};
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int32_t n = A->n;
  TempAllocs tmp;
  int rc;

  // block sizes back to the host (the handles must share them)
  auto t0 = clk::now();
  std::vector<int32_t> b, bb;
  if ((rc = d2h(b, A->b, n, s)) || (rc = d2h(bb, B->b, n, s))) return rc;
  // block norms, needed only to compare with a positive threshold
  double *dn = nullptr;
  if (eps > 0.0) {
    if ((rc = tmp.alloc(&dn, (size_t)(A->nnzb + B->nnzb)))) return rc;
    hipError_t e = launch_block_norms(static_cast<const double *>(A->dir[0].vals),
                                      A->dir[0].blk_pos, A->blk_row, A->col_idx, A->b, A->nnzb,
                                      dn, s);
    if (e == hipSuccess)
      e = launch_block_norms(static_cast<const double *>(B->dir[0].vals), B->dir[0].blk_pos,
                             B->blk_row, B->col_idx, B->b, B->nnzb, dn + A->nnzb, s);
    if (e != hipSuccess) return hip_fail(e, "block norm kernel launch");
  }
  HIP_TRY(hipStreamSynchronize(s), "spgemm");
  if (b != bb) return fail(VBCSR_EINVAL, "A and B must be over the same atoms (block sizes differ)");
  st.ms_norms = ms_since(t0);

  // symbolic stage on the device
  t0 = clk::now();
  SymbolicIn sin{};
  sin.n = n;
  sin.annzb = A->nnzb;
  sin.b = A->b;
  sin.arp = A->row_ptr;
  sin.aci = A->col_idx;
  sin.arow = A->blk_row;
  sin.apos = A->dir[1].blk_pos;
  sin.an = eps > 0.0 ? dn : nullptr;
  sin.brp = B->row_ptr;
  sin.bci = B->col_idx;
  sin.bpos = B->dir[0].blk_pos;
  sin.bn = eps > 0.0 ? dn + A->nnzb : nullptr;
  sin.eps = eps;
  SymbolicOut so;
  int alloc_rc = VBCSR_OK;
  const DevAlloc dalloc = [&](void **q, size_t bytes) -> hipError_t {
    char *c = nullptr;
    alloc_rc = tmp.alloc(&c, bytes);
    *q = c;
    return alloc_rc == VBCSR_OK ? hipSuccess : hipErrorOutOfMemory;
  };
  {
    hipError_t e = spgemm_symbolic_device(sin, so, dalloc, s);
    if (alloc_rc != VBCSR_OK) return alloc_rc;
    if (e == hipErrorInvalidValue)
      return fail(VBCSR_EUNSUPPORTED, "the block product has 2^31 or more block products");
    if (e != hipSuccess) return hip_fail(e, "symbolic stage");
  }
  const int64_t nC = so.nC;
  const int64_t nvals = so.nvals;
  st.candidates = so.candidates;
  st.kept_symbolic = nC;
  st.products = so.nP;
  st.flops = so.flops;
  const int64_t *cls_begin = so.cls_begin;
  SpgemmParams sp{};
  sp.avals = static_cast<const double *>(A->dir[1].vals);
  sp.bvals = static_cast<const double *>(B->dir[0].vals);
  sp.b = A->b;
  // C is laid out on the device in A's processing order (row order AUTO) or
  // in atom order; an RCM or cluster order of C's own graph comes from the
  // host planner, which takes the pattern back.  Without a final filter
  // (eps = 0) a device layout comes first and the numeric stage writes C's
  // two page sets directly.
  vbcsr_plan_opts copts{};
  if (opts) copts = *opts;
  const int32_t c_order = copts.row_order;
  const bool device_layout = c_order == VBCSR_ORDER_AUTO || c_order == VBCSR_ORDER_ATOM;
  const bool direct = device_layout && eps == 0.0;
  double *cvals = nullptr, *cnorm = nullptr;
  if ((!direct && (rc = tmp.alloc(&cvals, (size_t)nvals))) ||
      (eps > 0.0 && (rc = tmp.alloc(&cnorm, (size_t)nC))))
    return rc;
  st.ms_symbolic = ms_since(t0);
  auto processing_order = [&](int32_t **d_ord) -> int {
    int r;
    if ((r = tmp.alloc(d_ord, (size_t)std::max<int32_t>(n, 1)))) return r;
    hipError_t e2 = c_order == VBCSR_ORDER_ATOM
                        ? launch_iota(n, *d_ord, s)
                        : launch_order_from_rows(A->dir[0].rows, A->dir[0].npanels, A->off, n,
                                                 *d_ord, s);
    return e2 == hipSuccess ? VBCSR_OK : hip_fail(e2, "order kernel launch");
  };
  // C's handle until it is returned (freed on every failure after it exists)
  struct CGuard {
    vbcsr_mat **h;
    bool keep = false;
    ~CGuard() {
      if (!keep && *h) {
        free_all(*h);
        delete *h;
        *h = nullptr;
      }
    }
  } cguard{out};
  if (direct) {
    t0 = clk::now();
    int32_t *d_ord = nullptr;
    if ((rc = processing_order(&d_ord))) return rc;
    rc = create_planned_on_device(out, A, nC, nvals, so.crp, so.oj, nullptr, d_ord, &copts,
                                  dalloc, s);
    if (alloc_rc != VBCSR_OK) return alloc_rc;
    if (rc) return rc;
    st.ms_build = ms_since(t0);
    sp.fpages = static_cast<double *>((*out)->dir[0].vals);
    sp.tpages = static_cast<double *>((*out)->dir[1].vals);
    sp.fpos = (*out)->dir[0].blk_pos;
    sp.tpos = (*out)->dir[1].blk_pos;
  }
  sp.oi = so.oi;
  sp.oj = so.oj;
  sp.obase = so.obase;
  sp.pptr = so.pptr;
  sp.pa = so.pa;
  sp.pb = so.pb;
  sp.cvals = cvals;
  sp.cnorm = cnorm;
  const int32_t *d_order = so.order;

  // numeric stage, timed with events on the stream
  const int max_b = n ? *std::max_element(b.begin(), b.end()) : 1;
  hipEvent_t ev[2];
  HIP_TRY(hipEventCreate(&ev[0]), "hipEventCreate");
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(VBCSR_EHIP, "hipEventCreate");
  }
  hipError_t e = hipEventRecord(ev[0], s);
  for (int k = 0; k < 5 && e == hipSuccess && nC > 0; ++k) {
    SpgemmParams pk = sp;
    pk.order = d_order + cls_begin[k];
    pk.count = cls_begin[k + 1] - cls_begin[k];
    e = launch_spgemm_numeric(pk, k, max_b, s);
  }
  if (e == hipSuccess) e = hipEventRecord(ev[1], s);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (e != hipSuccess) return hip_fail(e, "numeric stage");
  st.ms_numeric = ms;
  if (direct) {   // C is complete
    st.nnzb = nC;
    cguard.keep = true;
    if (stats) *stats = st;
    return VBCSR_OK;
  }

  // closing norm filter on the device: drop computed blocks whose norm is
  // below eps (the pattern of C, its row pointer and values stay on the device)
  t0 = clk::now();
  const int64_t *c_rp = so.crp;
  const int32_t *c_ci = so.oj;
  const double *final_vals = cvals;
  int64_t c_nnzb = nC, final_nvals = nvals;
  if (eps > 0.0 && nC > 0) {
    FilterOut fo;
    e = spgemm_filter_device(n, nC, so.crp, so.oj, so.obase, cnorm, eps, cvals, fo, dalloc, s);
    if (alloc_rc != VBCSR_OK) return alloc_rc;
    if (e != hipSuccess) return hip_fail(e, "filter");
    if (fo.nnzb < nC) {
      c_rp = fo.rp;
      c_ci = fo.ci;
      final_vals = fo.vals;
      c_nnzb = fo.nnzb;
      final_nvals = fo.nvals;
    }
  }
  st.nnzb = c_nnzb;
  st.ms_filter = ms_since(t0);

  // C as an ordinary handle over the same atoms
  t0 = clk::now();
  if (device_layout) {
    int32_t *d_ord = nullptr;
    if ((rc = processing_order(&d_ord))) return rc;
    rc = create_planned_on_device(out, A, c_nnzb, final_nvals, c_rp, c_ci, final_vals, d_ord,
                                  &copts, dalloc, s);
    if (alloc_rc != VBCSR_OK) return alloc_rc;
  } else {
    std::vector<int64_t> hrp;
    std::vector<int32_t> hci;
    if ((rc = d2h(hrp, c_rp, (size_t)n + 1, s)) || (rc = d2h(hci, c_ci, (size_t)c_nnzb, s)))
      return rc;
    HIP_TRY(hipStreamSynchronize(s), "spgemm");
    rc = create_impl(out, n, b.data(), hrp.data(), c_nnzb ? hci.data() : nullptr, final_vals, true,
                     final_nvals, VBCSR_FP64, &copts, stream);
  }
  if (rc) return rc;
  st.ms_build = ms_since(t0);
  cguard.keep = true;
  if (stats) *stats = st;
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_spgemm");
}

int vbcsr_kpm_dos(const double *mu, int32_t n_moments, int32_t damping, const double *x,
                  int64_t npts, double *rho, double *work, void *stream) try {
  if (n_moments < 1) return fail(VBCSR_EINVAL, "n_moments must be >= 1");
  if (damping != VBCSR_KPM_NONE && damping != VBCSR_KPM_JACKSON)
    return fail(VBCSR_EINVAL, "damping must be VBCSR_KPM_NONE or VBCSR_KPM_JACKSON");
  if (npts < 0) return fail(VBCSR_EINVAL, "npts must be >= 0");
  if (!mu || (npts > 0 && (!x || !rho))) return fail(VBCSR_EINVAL, "array pointer is NULL");
  if (npts > 0 && ranges_overlap(x, sizeof(double) * npts, rho, sizeof(double) * npts))
    return fail(VBCSR_EINVAL, "x and rho overlap");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *coef = work;
  TempAllocs tmp;
  int rc;
  if (!coef && (rc = tmp.alloc(&coef, (size_t)n_moments))) return rc;
  hipError_t e = launch_kpm_dos(mu, n_moments, damping, x, npts, coef, rho, s);
  if (e != hipSuccess) return hip_fail(e, "kpm kernel launch");
  // a workspace allocated here is freed on return: finish with it first
  if (!work) HIP_TRY(hipStreamSynchronize(s), "kpm_dos");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_kpm_dos");
}

int vbcsr_kpm_threshold(int32_t n_moments, int64_t n_states, double fraction, double *threshold) try {
  if (n_moments < 1 || n_states < 1 || !(fraction > 0.0) || !threshold)
    return fail(VBCSR_EINVAL, "need n_moments >= 1, n_states >= 1, fraction > 0, threshold");
  const double sigma = M_PI / n_moments;
  *threshold = fraction / ((double)n_states * sigma * std::sqrt(2.0 * M_PI));
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_kpm_threshold");
}

int vbcsr_kpm_gap(const double *x, const double *rho, int64_t npts, double threshold, double *lo,
                  double *hi) try {
  if (!lo || !hi || (npts > 0 && (!x || !rho)) || npts < 0)
    return fail(VBCSR_EINVAL, "array pointer is NULL or npts < 0");
  for (int64_t i = 1; i < npts; ++i)
    if (!(x[i] > x[i - 1])) return fail(VBCSR_EINVAL, "x must be strictly ascending");
  *lo = *hi = std::nan("");
  int64_t prev = -1;  // last point at or above the threshold
  double best = -1.0;
  for (int64_t i = 0; i < npts; ++i) {
    if (!(rho[i] >= threshold)) continue;
    if (prev >= 0 && i - prev > 1 && x[i] - x[prev] > best) {
      best = x[i] - x[prev];
      *lo = x[prev];
      *hi = x[i];
    }
    prev = i;
  }
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_kpm_gap");
}

}  // extern "C"
