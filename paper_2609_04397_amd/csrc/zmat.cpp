// Reciprocal-space operators (paper, section 3.3, equation 4): a periodic
// real-space operator given as translation-resolved images, sampled at a
// k point into complex pages, and its complex products (forward, and the
// conjugate-transpose adjoint of equation 1).  See include/vbcsr.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/vbcsr.h"
#include "common.hpp"
#include "zkernels.hpp"

using namespace vbcsr;

struct vbcsr_zmat {
  int32_t n = 0, n_images = 0;
  int64_t N = 0, nnzb = 0, nnz = 0;   // real (image) blocks and values
  int64_t nkb = 0, nkv = 0;           // blocks and values of O(k)
  vbcsr_prec prec = VBCSR_FP64;
  bool has_tau = false;
  std::vector<int64_t> krp_host;
  std::vector<int32_t> kci_host;
  // device
  int32_t *b = nullptr, *image = nullptr, *blk_row = nullptr, *col_idx = nullptr;
  int32_t *shifts = nullptr, *krow = nullptr, *kcol = nullptr, *kdim = nullptr;
  double *tau = nullptr, *values = nullptr, *ph = nullptr;
  int64_t *cgbase = nullptr, *cptr = nullptr, *kbase = nullptr, *kvbase = nullptr;
  RowDesc *rows[2] = {nullptr, nullptr};
  int32_t *colx[2] = {nullptr, nullptr};
  int64_t *pos[2] = {nullptr, nullptr};
  void *pages[2] = {nullptr, nullptr};
  std::vector<void *> owned;
};

namespace {

int zfail(int code, const std::string &m) { return set_error(code, m); }

int zhip(hipError_t e, const char *where) {
  return set_error(VBCSR_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

template <typename T>
int zalloc(vbcsr_zmat *Z, T **p, size_t count) {
  *p = nullptr;
  if (count == 0) return VBCSR_OK;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * count);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return zfail(VBCSR_ENOMEM, "hipMalloc of " + std::to_string(sizeof(T) * count) + " bytes failed");
  }
  if (e != hipSuccess) return zhip(e, "hipMalloc");
  Z->owned.push_back(*p);
  return VBCSR_OK;
}

template <typename T>
int zup(vbcsr_zmat *Z, T **p, const T *src, size_t count, hipStream_t s) {
  int rc = zalloc(Z, p, count);
  if (rc || count == 0) return rc;
  hipError_t e = hipMemcpyAsync(*p, src, sizeof(T) * count, hipMemcpyHostToDevice, s);
  return e == hipSuccess ? VBCSR_OK : zhip(e, "hipMemcpyAsync");
}

void zfree(vbcsr_zmat *Z) {
  if (!Z->owned.empty()) (void)hipDeviceSynchronize();
  for (void *p : Z->owned) (void)hipFree(p);
  Z->owned.clear();
}

size_t celem(const vbcsr_zmat *Z) { return Z->prec == VBCSR_FP64 ? 8 : 4; }

}  // namespace

extern "C" {

int vbcsr_zmat_create(vbcsr_zmat **out, int32_t n_atoms, const int32_t *block_sizes,
                      const int64_t *row_ptr, const int32_t *col_idx, const int32_t *image,
                      int32_t n_images, const int32_t *shifts, const double *tau,
                      const double *values, int64_t n_values, vbcsr_prec prec,
                      const vbcsr_plan_opts *opts, void *stream) try {
  if (!out) return zfail(VBCSR_EINVAL, "out is NULL");
  *out = nullptr;
  if (prec == VBCSR_BF16X3) return zfail(VBCSR_EUNSUPPORTED, "complex operators are FP64 or FP32");
  if (prec != VBCSR_FP64 && prec != VBCSR_FP32) return zfail(VBCSR_EINVAL, "unknown precision");
  if (opts && (opts->rows_per_wg != 0 || opts->row_order < VBCSR_ORDER_AUTO ||
               opts->row_order > VBCSR_ORDER_CLUSTER))
    return zfail(VBCSR_EINVAL, "invalid plan options");
  if (n_images < 1 || !shifts) return zfail(VBCSR_EINVAL, "need n_images >= 1 and shifts");
  // the image graph: blocks (i, j, m); the same (i, j) may repeat under other images
  std::string err;
  if (n_atoms < 0 || !row_ptr) return zfail(VBCSR_EINVAL, "n_atoms < 0 or row_ptr NULL");
  const int64_t nnzb = n_atoms ? row_ptr[n_atoms] : 0;
  if (nnzb > 0 && !image) return zfail(VBCSR_EINVAL, "image is NULL");
  for (int64_t t = 0; t < nnzb; ++t)
    if (image[t] < 0 || image[t] >= n_images)
      return zfail(VBCSR_EINVAL, "image index out of range at block " + std::to_string(t));
  // k-space pattern: distinct (i, j) per row, ascending j
  std::vector<int64_t> krp((size_t)n_atoms + 1, 0);
  std::vector<int32_t> kci;
  std::vector<int64_t> kb_of(nnzb);
  {
    // validation of sizes, ranges and row_ptr by the ordinary planner check
    // on the k-space pattern happens below; here: row_ptr and column ranges
    if (row_ptr[0] != 0) return zfail(VBCSR_EINVAL, "row_ptr[0] must be 0");
    for (int32_t i = 0; i < n_atoms; ++i)
      if (row_ptr[i + 1] < row_ptr[i])
        return zfail(VBCSR_EINVAL, "row_ptr is decreasing at row " + std::to_string(i));
    if (nnzb > 0 && !col_idx) return zfail(VBCSR_EINVAL, "col_idx is NULL");
    std::vector<std::pair<int64_t, int64_t>> key;  // ((j, m), t)
    for (int32_t i = 0; i < n_atoms; ++i) {
      key.clear();
      for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
        if (col_idx[t] < 0 || col_idx[t] >= n_atoms)
          return zfail(VBCSR_EINVAL, "col_idx out of range in row " + std::to_string(i));
        key.push_back({(int64_t)col_idx[t] * n_images + image[t], t});
      }
      std::sort(key.begin(), key.end());
      for (size_t u = 0; u < key.size(); ++u) {
        if (u && key[u].first == key[u - 1].first)
          return zfail(VBCSR_EDUP, "duplicate block (" + std::to_string(i) + ", " +
                                       std::to_string(key[u].first / n_images) + ") in image " +
                                       std::to_string(key[u].first % n_images));
        const int32_t j = (int32_t)(key[u].first / n_images);
        if (kci.size() == (size_t)krp[i] || kci.back() != j) kci.push_back(j);
        kb_of[key[u].second] = (int64_t)kci.size() - 1;
      }
      krp[i + 1] = (int64_t)kci.size();
    }
  }
  // real values: same count check as the ordinary create
  int64_t nnz = 0;
  std::vector<int64_t> gbase(nnzb + 1, 0);
  std::vector<int32_t> brow(nnzb);
  for (int32_t i = 0; i < n_atoms; ++i) {
    if (!block_sizes || block_sizes[i] < 1 || block_sizes[i] > VBCSR_MAX_BLOCK)
      return zfail(block_sizes && block_sizes[i] > VBCSR_MAX_BLOCK ? VBCSR_EUNSUPPORTED
                                                                   : VBCSR_EINVAL,
                   "block size of atom " + std::to_string(i) + " out of range");
    for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
      brow[t] = i;
      gbase[t + 1] = gbase[t] + (int64_t)block_sizes[i] * block_sizes[col_idx[t]];
    }
  }
  nnz = gbase[nnzb];
  if (nnz != n_values)
    return zfail(VBCSR_ESHAPE, "n_values " + std::to_string(n_values) + " != " + std::to_string(nnz));
  const int64_t nkb = (int64_t)kci.size();
  int64_t nkv = 0;
  std::vector<int64_t> kbase(nkb + 1, 0);
  std::vector<int32_t> krow(nkb);
  for (int32_t i = 0; i < n_atoms; ++i)
    for (int64_t c = krp[i]; c < krp[i + 1]; ++c) {
      krow[c] = i;
      kbase[c + 1] = kbase[c] + (int64_t)block_sizes[i] * block_sizes[kci[c]];
    }
  nkv = kbase[nkb];
  int rc = validate_graph(n_atoms, block_sizes, krp.data(), kci.data(), nkv, err);
  if (rc) return zfail(rc, err);
  {
    // complex pages take 16 bytes per value: a block row or block column is
    // addressed with 32-bit byte offsets, so it must hold fewer than 2^27
    std::vector<int64_t> colv(n_atoms, 0);
    for (int32_t i = 0; i < n_atoms; ++i) {
      int64_t rv = 0;
      for (int64_t c = krp[i]; c < krp[i + 1]; ++c) {
        const int64_t v = (int64_t)block_sizes[i] * block_sizes[kci[c]];
        rv += v;
        colv[kci[c]] += v;
      }
      if (rv >= (int64_t(1) << 27))
        return zfail(VBCSR_EUNSUPPORTED, "block row " + std::to_string(i) + " of O(k) holds 2^27 or more values");
    }
    for (int32_t j = 0; j < n_atoms; ++j)
      if (colv[j] >= (int64_t(1) << 27))
        return zfail(VBCSR_EUNSUPPORTED, "block column " + std::to_string(j) + " of O(k) holds 2^27 or more values");
  }
  HostPlan plan;
  build_plan(n_atoms, block_sizes, krp.data(), kci.data(), opts ? opts->row_order : 0, plan);
  // contributions of every k-space block, in graph order
  std::vector<int64_t> cptr(nkb + 1, 0), cblk(nnzb);
  for (int64_t t = 0; t < nnzb; ++t) cptr[kb_of[t] + 1]++;
  for (int64_t c = 0; c < nkb; ++c) cptr[c + 1] += cptr[c];
  {
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t t = 0; t < nnzb; ++t) cblk[fill[kb_of[t]]++] = t;
  }
  // what the phase and sample kernels read per contribution
  std::vector<int32_t> cimage(nnzb), crow(nnzb), ccol(nnzb);
  std::vector<int64_t> cgbase(nnzb);
  for (int64_t c = 0; c < nnzb; ++c) {
    const int64_t t = cblk[c];
    cimage[c] = image[t];
    crow[c] = brow[t];
    ccol[c] = col_idx[t];
    cgbase[c] = gbase[t];
  }
  // per block of O(k): its sizes and where its first contribution's values start
  std::vector<int32_t> kdim(nkb);
  std::vector<int64_t> kvbase(nkb);
  for (int64_t c = 0; c < nkb; ++c) {
    kdim[c] = block_sizes[krow[c]] | block_sizes[kci[c]] << 16;
    kvbase[c] = cgbase[cptr[c]];
  }

  hipStream_t s = static_cast<hipStream_t>(stream);
  vbcsr_zmat *Z = new vbcsr_zmat();
  // frees the partial handle on every early return and on an exception
  struct Guard {
    vbcsr_zmat *&h;
    ~Guard() {
      if (h) {
        zfree(h);
        delete h;
      }
    }
  } guard{Z};
  Z->n = n_atoms;
  Z->n_images = n_images;
  Z->N = plan.N;
  Z->nnzb = nnzb;
  Z->nnz = nnz;
  Z->nkb = nkb;
  Z->nkv = nkv;
  Z->prec = prec;
  Z->has_tau = tau != nullptr;
  Z->krp_host = krp;
  Z->kci_host = kci;
  auto bail = [&](int code) { return code; };
  if ((rc = zup(Z, &Z->b, block_sizes, (size_t)n_atoms, s)) ||
      (rc = zup(Z, &Z->image, cimage.data(), (size_t)nnzb, s)) ||
      (rc = zup(Z, &Z->blk_row, crow.data(), (size_t)nnzb, s)) ||
      (rc = zup(Z, &Z->col_idx, ccol.data(), (size_t)nnzb, s)) ||
      (rc = zup(Z, &Z->shifts, shifts, (size_t)n_images * 3, s)) ||
      (tau && (rc = zup(Z, &Z->tau, tau, (size_t)n_atoms * 3, s))) ||
      (rc = zup(Z, &Z->cgbase, cgbase.data(), (size_t)nnzb, s)) ||
      (rc = zup(Z, &Z->cptr, cptr.data(), (size_t)nkb + 1, s)) ||
      (rc = zup(Z, &Z->kdim, kdim.data(), (size_t)nkb, s)) ||
      (rc = zup(Z, &Z->kvbase, kvbase.data(), (size_t)nkb, s)) ||
      (rc = zup(Z, &Z->krow, krow.data(), (size_t)nkb, s)) ||
      (rc = zup(Z, &Z->kcol, kci.data(), (size_t)nkb, s)) ||
      (rc = zup(Z, &Z->kbase, kbase.data(), (size_t)nkb + 1, s)) ||
      (rc = zalloc(Z, &Z->values, (size_t)nnz)) || (rc = zalloc(Z, &Z->ph, (size_t)nnzb * 2)))
    return bail(rc);
  if (nnz) {
    hipError_t e = values ? hipMemcpyAsync(Z->values, values, sizeof(double) * nnz,
                                           hipMemcpyHostToDevice, s)
                          : hipMemsetAsync(Z->values, 0, sizeof(double) * nnz, s);
    if (e != hipSuccess) return bail(zhip(e, "hipMemcpyAsync"));
  }
  for (int d = 0; d < 2; ++d) {
    const DirPlan &P = d == 0 ? plan.fwd : plan.tr;
    if ((rc = zup(Z, &Z->rows[d], P.rows.data(), P.rows.size(), s)) ||
        (rc = zup(Z, &Z->colx[d], P.colx.data(), P.colx.size(), s)) ||
        (rc = zup(Z, &Z->pos[d], P.blk_pos.data(), P.blk_pos.size(), s)))
      return bail(rc);
    // complex pages (two values per element); the panel padding reads zero
    const size_t bytes = 2 * celem(Z) * (size_t)(P.n_values + kPageSlack);
    char *pg = nullptr;
    if ((rc = zalloc(Z, &pg, bytes))) return bail(rc);
    hipError_t e = hipMemsetAsync(pg, 0, bytes, s);
    if (e != hipSuccess) return bail(zhip(e, "hipMemsetAsync"));
    Z->pages[d] = pg;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail(zhip(e, "zmat_create"));
  *out = Z;
  Z = nullptr;  // owned by the caller now
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_zmat_create");
}

int vbcsr_zmat_sample(vbcsr_zmat *Z, const double *k, int32_t convention, void *stream) try {
  if (!Z || !k) return zfail(VBCSR_EINVAL, "handle or k is NULL");
  if (!std::isfinite(k[0]) || !std::isfinite(k[1]) || !std::isfinite(k[2]))
    return zfail(VBCSR_EINVAL, "k must be finite");
  if (convention != VBCSR_PHASE_R && convention != VBCSR_PHASE_R_TAU)
    return zfail(VBCSR_EINVAL, "convention must be VBCSR_PHASE_R or VBCSR_PHASE_R_TAU");
  if (convention == VBCSR_PHASE_R_TAU && !Z->has_tau)
    return zfail(VBCSR_EINVAL, "the R+tau convention needs tau at create");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ZPhaseParams pp{};
  pp.image = Z->image;
  pp.blk_row = Z->blk_row;
  pp.col_idx = Z->col_idx;
  pp.shifts = Z->shifts;
  pp.tau = convention == VBCSR_PHASE_R_TAU ? Z->tau : nullptr;
  pp.k[0] = k[0];
  pp.k[1] = k[1];
  pp.k[2] = k[2];
  pp.n = Z->nnzb;
  pp.ph = Z->ph;
  hipError_t e = launch_zphase(pp, s);
  if (e != hipSuccess) return zhip(e, "phase kernel launch");
  ZSampleParams sp{};
  sp.nkb = Z->nkb;
  sp.kdim = Z->kdim;
  sp.kvbase = Z->kvbase;
  sp.kbase = Z->kbase;
  sp.cptr = Z->cptr;
  sp.cgbase = Z->cgbase;
  sp.values = Z->values;
  sp.ph = Z->ph;
  sp.fwd_pos = Z->pos[0];
  sp.tr_pos = Z->pos[1];
  e = launch_zsample(sp, Z->pages[0], Z->pages[1], (int)celem(Z), s);
  if (e != hipSuccess) return zhip(e, "sample kernel launch");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_zmat_sample");
}

int vbcsr_zmat_spmm(const vbcsr_zmat *Z, const void *X, int64_t ldx, void *Y, int64_t ldy,
                    int32_t nrhs, const double *alpha, const double *beta, int32_t adjoint,
                    void *stream) try {
  if (!Z || !alpha || !beta) return zfail(VBCSR_EINVAL, "handle, alpha or beta is NULL");
  if (nrhs <= 0) return zfail(VBCSR_EINVAL, "nrhs must be >= 1");
  if (ldx < nrhs || ldy < nrhs) return zfail(VBCSR_EINVAL, "leading dimension smaller than nrhs");
  if (Z->N == 0) return VBCSR_OK;
  if (!X || !Y) return zfail(VBCSR_EINVAL, "vector pointer is NULL");
  const size_t es = 2 * celem(Z);
  const char *xa = static_cast<const char *>(X), *ya = static_cast<const char *>(Y);
  const size_t xb = ((size_t)(Z->N - 1) * ldx + nrhs) * es, yb = ((size_t)(Z->N - 1) * ldy + nrhs) * es;
  if (xa < ya + yb && ya < xa + xb) return zfail(VBCSR_EINVAL, "input and output vectors overlap");
  const int d = adjoint ? 1 : 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (Z->prec == VBCSR_FP64) {
    ZSpmmParams<double> p{Z->rows[d], Z->n, Z->colx[d], static_cast<const double *>(Z->pages[d]),
                          static_cast<const double *>(X), ldx, static_cast<double *>(Y), ldy, nrhs,
                          alpha[0], alpha[1], beta[0], beta[1], Z->N};
    e = launch_zspmm_f64(p, s);
  } else {
    ZSpmmParams<float> p{Z->rows[d], Z->n, Z->colx[d], static_cast<const float *>(Z->pages[d]),
                         static_cast<const float *>(X), ldx, static_cast<float *>(Y), ldy, nrhs,
                         alpha[0], alpha[1], beta[0], beta[1], Z->N};
    e = launch_zspmm_f32(p, s);
  }
  if (e != hipSuccess) return zhip(e, "complex product kernel launch");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_zmat_spmm");
}

int vbcsr_zmat_info(const vbcsr_zmat *Z, int64_t *n_rows, int64_t *nnzb_k, int64_t *n_values_k) try {
  if (!Z) return zfail(VBCSR_EINVAL, "handle is NULL");
  if (n_rows) *n_rows = Z->N;
  if (nnzb_k) *nnzb_k = Z->nkb;
  if (n_values_k) *n_values_k = Z->nkv;
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_zmat_info");
}

int vbcsr_zmat_get_structure(const vbcsr_zmat *Z, int64_t *row_ptr, int32_t *col_idx) try {
  if (!Z || !row_ptr || (Z->nkb && !col_idx)) return zfail(VBCSR_EINVAL, "NULL argument");
  std::copy(Z->krp_host.begin(), Z->krp_host.end(), row_ptr);
  std::copy(Z->kci_host.begin(), Z->kci_host.end(), col_idx);
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_zmat_get_structure");
}

int vbcsr_zmat_get_values(const vbcsr_zmat *Z, void *values, void *stream) try {
  if (!Z) return zfail(VBCSR_EINVAL, "handle is NULL");
  if (Z->nkv == 0) return VBCSR_OK;
  if (!values) return zfail(VBCSR_EINVAL, "values is NULL");
  hipError_t e = launch_zunpack(Z->pages[0], (int)celem(Z), Z->pos[0], Z->krow, Z->kcol, Z->b,
                                Z->kbase, Z->nkb, values, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return zhip(e, "unpack kernel launch");
  return VBCSR_OK;
} catch (...) {
  return api_exception("vbcsr_zmat_get_values");
}

void vbcsr_zmat_destroy(vbcsr_zmat *Z) {
  if (!Z) return;
  zfree(Z);
  delete Z;
}

}  // extern "C"
