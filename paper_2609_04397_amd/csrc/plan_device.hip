// Layout of an operator whose block graph is already on the device (the
// product C of the block product, paper section 3.2): the per-block maps and
// panel descriptors that the host planner would build, computed by sorts and
// scans on the device so that the pattern never goes to the host.
//
// Forward panels are the block rows in a given processing order, each
// holding its blocks ordered by (b_j, j); transposed panels are the block
// columns in the same order, each holding its blocks ordered by (b_i, i).
// Both orders come from one stable radix sort of the blocks, in graph order,
// on the key (position of the panel's atom << 7 | b of the other atom): the
// graph order is ascending in (i, j), so ties keep j ascending within a
// block row and i ascending within a block column.  A scan of the member
// widths over the sorted blocks gives each block's column-table position;
// scans over the panels in processing order give each panel's first column
// and first value (panels start on kPanelAlign-value boundaries).  For the
// same processing order the result equals the host planner's.
#include <hipcub/hipcub.hpp>

#include "kernels.hpp"
#include "../../include/vbcsr.h"

namespace vbcsr {
namespace {

constexpr int kT = 256;
constexpr int kShapeSide = VBCSR_MAX_BLOCK + 1;

dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kT - 1) / kT)); }

int bits_for(int64_t v) {  // bits to hold 0 .. v
  int nb = 1;
  while (nb < 63 && (int64_t(1) << nb) <= v) ++nb;
  return nb;
}

// one wave per block row: its blocks' row and value counts
__global__ void __launch_bounds__(kT) k_pd_rows(int32_t n, const int64_t *rp, const int32_t *ci,
                                                const int32_t *b, int32_t *blk_row, int64_t *gsize,
                                                int64_t nnzb) {
  const int64_t i = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int64_t bi = b[i];
  for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += 64) {
    blk_row[k] = (int32_t)i;
    gsize[k] = bi * b[ci[k]];
  }
  if (i == 0 && lane == 0) gsize[nnzb] = 0;
}

// rank[order[p]] = p
__global__ void __launch_bounds__(kT) k_pd_rank(int32_t n, const int32_t *order, int32_t *rank) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p < n) rank[order[p]] = (int32_t)p;
}

// key of block k for direction d: panel atom r (d = 0: row, 1: column),
// member atom c; panel width accumulated per atom
__global__ void __launch_bounds__(kT) k_pd_keys(int64_t nnzb, int d, const int32_t *blk_row,
                                                const int32_t *ci, const int32_t *rank,
                                                const int32_t *b, uint64_t *key, int32_t *val,
                                                unsigned long long *width) {
  const int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (k >= nnzb) return;
  const int32_t r = d == 0 ? blk_row[k] : ci[k];
  const int32_t c = d == 0 ? ci[k] : blk_row[k];
  key[k] = (uint64_t)(uint32_t)rank[r] << 7 | (uint32_t)b[c];
  val[k] = (int32_t)k;
  atomicAdd(&width[r], (unsigned long long)b[c]);
}

// member widths in sorted order (entry nnzb = 0: the scan's total)
__global__ void __launch_bounds__(kT) k_pd_memberw(int64_t nnzb, int d, const int32_t *val,
                                                   const int32_t *blk_row, const int32_t *ci,
                                                   const int32_t *b, int64_t *w) {
  const int64_t u = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (u < nnzb) {
    const int32_t k = val[u];
    w[u] = b[d == 0 ? ci[k] : blk_row[k]];
  } else if (u == nnzb) {
    w[u] = 0;
  }
}

// per panel in processing order: width, value count and value count rounded
// up to kPanelAlign; entry n = 0
__global__ void __launch_bounds__(kT) k_pd_psize(int32_t np, const int32_t *order, const int32_t *b,
                                                 const unsigned long long *width, int64_t *pk,
                                                 int64_t *pv, int64_t *pu) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p < np) {
    const int32_t r = order[p];
    const int64_t K = (int64_t)width[r];
    pk[p] = K;
    pu[p] = (int64_t)b[r] * K;
    pv[p] = ((int64_t)b[r] * K + kPanelAlign - 1) / kPanelAlign * kPanelAlign;
  } else if (p == np) {
    pk[p] = 0;
    pv[p] = 0;
    pu[p] = 0;
  }
}

__global__ void __launch_bounds__(kT) k_pd_rowdesc(int32_t np, const int32_t *order,
                                                   const int32_t *b, const int32_t *off,
                                                   const unsigned long long *width,
                                                   const int64_t *cb, const int64_t *vb,
                                                   RowDesc *rows) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= np) return;
  const int32_t r = order[p];
  RowDesc rd;
  rd.vbase = vb[p];
  rd.cbase = cb[p];
  rd.K = (int32_t)width[r];   // below 2^28 once the panel limit is checked
  rd.yrow = off[r];
  rd.b = b[r];
  rd.pad = 0;
  rows[p] = rd;
}

__global__ void __launch_bounds__(kT) k_pd_blocks(int64_t nnzb, int d, const int32_t *val,
                                                  const int32_t *blk_row, const int32_t *ci,
                                                  const int32_t *b, const int32_t *rank,
                                                  const int64_t *cpos, const int64_t *cb,
                                                  const int64_t *vb, int64_t *blk_pos,
                                                  int32_t *blk_k0, int32_t *blk_prow) {
  const int64_t u = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (u >= nnzb) return;
  const int32_t k = val[u];
  const int32_t r = d == 0 ? blk_row[k] : ci[k];
  const int32_t p = rank[r];
  const int32_t k0 = (int32_t)(cpos[u] - cb[p]);
  blk_pos[k] = vb[p] + (int64_t)k0 * b[r];
  blk_k0[k] = k0;
  blk_prow[k] = p;
}

// shape classes (b_i, b_j): a histogram per workgroup in LDS, then one
// atomic per nonzero bin
__global__ void __launch_bounds__(kT) k_pd_shapes(int64_t nnzb, const int32_t *blk_row,
                                                  const int32_t *ci, const int32_t *b,
                                                  unsigned int *hist) {
  __shared__ unsigned int h[kShapeSide * kShapeSide];
  for (int t = threadIdx.x; t < kShapeSide * kShapeSide; t += kT) h[t] = 0;
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (k < nnzb) atomicAdd(&h[b[blk_row[k]] * kShapeSide + b[ci[k]]], 1u);
  __syncthreads();
  for (int t = threadIdx.x; t < kShapeSide * kShapeSide; t += kT)
    if (h[t]) atomicAdd(&hist[t], h[t]);
}

// order[p] = atom whose first scalar row is rows[p].yrow (off ascending)
__global__ void __launch_bounds__(kT) k_pd_order_of(int32_t np, const RowDesc *rows,
                                                    const int32_t *off, int32_t n,
                                                    int32_t *order) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= np) return;
  const int32_t y = rows[p].yrow;
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid] < y) lo = mid + 1;
    else hi = mid;
  }
  order[p] = lo;
}

__global__ void __launch_bounds__(kT) k_pd_iota(int32_t n, int32_t *order) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p < n) order[p] = (int32_t)p;
}

// closing filter: keep flags and value counts of the symbolic pattern's
// blocks (entry nC = 0)
__global__ void __launch_bounds__(kT) k_flt_flags(int64_t nC, const double *norm, double eps,
                                                  const int64_t *obase, int64_t *keep,
                                                  int64_t *vsz) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c < nC) {
    const bool kept = !(norm[c] < eps);
    keep[c] = kept ? 1 : 0;
    vsz[c] = kept ? obase[c + 1] - obase[c] : 0;
  } else if (c == nC) {
    keep[c] = 0;
    vsz[c] = 0;
  }
}

__global__ void __launch_bounds__(kT) k_flt_compact(int64_t nC, const int64_t *keep,
                                                    const int64_t *kidx, const int64_t *vpos,
                                                    const int32_t *ci, const int64_t *obase,
                                                    int32_t *ci_out, int64_t *sbase,
                                                    int64_t *dbase, int32_t *size) {
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c >= nC || !keep[c]) return;
  const int64_t t = kidx[c];
  ci_out[t] = ci[c];
  sbase[t] = obase[c];
  dbase[t] = vpos[c];
  size[t] = (int32_t)(obase[c + 1] - obase[c]);
}

__global__ void __launch_bounds__(kT) k_flt_rowptr(int32_t n, const int64_t *rp, const int64_t *kidx,
                                                   int64_t *rp_out) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i <= n) rp_out[i] = kidx[rp[i]];
}

}  // namespace

#define PD_TRY(x)                           \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

hipError_t launch_order_from_rows(const RowDesc *rows, int32_t np, const int32_t *off, int32_t n,
                                  int32_t *order, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pd_order_of, grid_for(np), dim3(kT), 0, s, np, rows, off, n, order);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t n, int32_t *order, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pd_iota, grid_for(n), dim3(kT), 0, s, n, order);
  return hipGetLastError();
}

hipError_t plan_device(const DevPlanIn &in, DevPlanOut &out, const DevAlloc &alloc,
                       hipStream_t s) {
  const int32_t n = in.n;
  const int64_t nnzb = in.nnzb;
  out.nnz = 0;
  out.n_shapes = 0;
  for (auto &d : out.dir) d.n_values = d.n_cols = d.max_panel = 0;
  if (nnzb >= (int64_t(1) << 31)) return hipErrorInvalidValue;  // 32-bit block indices below
  PD_TRY(hipGetLastError());

  // one allocation for every array (sizes are exact), one for hipCUB
  auto sz = [](size_t elem, size_t count) { return (elem * (count ? count : 1) + 255) / 256 * 256; };
  const size_t E = (size_t)nnzb, N1 = (size_t)n + 1;
  const size_t total = 2 * sz(8, E) + 2 * sz(4, E) + 3 * sz(8, E + 1) + sz(4, N1) +
                       6 * sz(8, N1) + sz(8, 2) + sz(4, kShapeSide * kShapeSide);
  char *base = nullptr;
  {
    void *q = nullptr;
    PD_TRY(alloc(&q, total));
    base = static_cast<char *>(q);
  }
  size_t used = 0;
  auto get = [&](auto **p, size_t count) {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
    *p = reinterpret_cast<T *>(base + used);
    used += sz(sizeof(T), count);
  };
  uint64_t *key = nullptr, *key_s = nullptr;
  int32_t *val = nullptr, *val_s = nullptr, *rank = nullptr;
  unsigned long long *width = nullptr;
  int64_t *gsize = nullptr, *w = nullptr, *cpos = nullptr, *pk = nullptr, *pv = nullptr,
          *pu = nullptr, *cb = nullptr, *vb = nullptr, *mx = nullptr;
  unsigned int *hist = nullptr;
  get(&key, E);
  get(&key_s, E);
  get(&val, E);
  get(&val_s, E);
  get(&gsize, E + 1);
  get(&w, E + 1);
  get(&cpos, E + 1);
  get(&rank, N1);
  get(&width, N1);
  get(&pk, N1);
  get(&pv, N1);
  get(&pu, N1);
  get(&cb, N1);
  get(&vb, N1);
  get(&mx, 2);
  get(&hist, kShapeSide * kShapeSide);
  void *cub_tmp = nullptr;
  size_t cub_bytes = 0;
  auto cub_run = [&](auto &&call) -> hipError_t {
    size_t need = 0;
    PD_TRY(call(nullptr, need));
    if (need > cub_bytes) {
      PD_TRY(alloc(&cub_tmp, need));
      cub_bytes = need;
    }
    return call(cub_tmp, need);
  };

  // block rows and graph value offsets
  if (nnzb > 0) {
    hipLaunchKernelGGL(k_pd_rows, grid_for((int64_t)n * 64), dim3(kT), 0, s, n, in.rp, in.ci, in.b,
                       out.blk_row, gsize, nnzb);
    PD_TRY(hipGetLastError());
  } else {
    PD_TRY(hipMemsetAsync(gsize, 0, sizeof(int64_t), s));
  }
  PD_TRY(cub_run([&](void *t, size_t &bytes) {
    return hipcub::DeviceScan::ExclusiveSum(t, bytes, gsize, out.gbase, (int)(E + 1), s);
  }));
  if (n > 0) {
    hipLaunchKernelGGL(k_pd_rank, grid_for(n), dim3(kT), 0, s, n, in.order, rank);
    PD_TRY(hipGetLastError());
  }
  const int end_bit = 7 + bits_for(n > 0 ? n - 1 : 0);
  int64_t host[3 * 2];
  for (int d = 0; d < 2; ++d) {
    DevPlanDir &D = out.dir[d];
    PD_TRY(hipMemsetAsync(width, 0, sizeof(unsigned long long) * N1, s));
    if (nnzb > 0) {
      hipLaunchKernelGGL(k_pd_keys, grid_for(nnzb), dim3(kT), 0, s, nnzb, d, out.blk_row, in.ci,
                         rank, in.b, key, val, width);
      PD_TRY(hipGetLastError());
      PD_TRY(cub_run([&](void *t, size_t &bytes) {
        return hipcub::DeviceRadixSort::SortPairs(t, bytes, key, key_s, val, val_s, (int)nnzb, 0,
                                                  end_bit, s);
      }));
    }
    hipLaunchKernelGGL(k_pd_memberw, grid_for(nnzb + 1), dim3(kT), 0, s, nnzb, d, val_s,
                       out.blk_row, in.ci, in.b, w);
    PD_TRY(hipGetLastError());
    PD_TRY(cub_run([&](void *t, size_t &bytes) {
      return hipcub::DeviceScan::ExclusiveSum(t, bytes, w, cpos, (int)(E + 1), s);
    }));
    hipLaunchKernelGGL(k_pd_psize, grid_for((int64_t)n + 1), dim3(kT), 0, s, n, in.order, in.b,
                       width, pk, pv, pu);
    PD_TRY(hipGetLastError());
    PD_TRY(cub_run([&](void *t, size_t &bytes) {
      return hipcub::DeviceReduce::Max(t, bytes, pu, mx + d, (int)N1, s);
    }));
    PD_TRY(hipMemcpyAsync(&host[3 * d + 2], mx + d, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PD_TRY(cub_run([&](void *t, size_t &bytes) {
      return hipcub::DeviceScan::ExclusiveSum(t, bytes, pk, cb, (int)N1, s);
    }));
    PD_TRY(cub_run([&](void *t, size_t &bytes) {
      return hipcub::DeviceScan::ExclusiveSum(t, bytes, pv, vb, (int)N1, s);
    }));
    PD_TRY(hipMemcpyAsync(&host[3 * d], cb + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PD_TRY(hipMemcpyAsync(&host[3 * d + 1], vb + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (n > 0) {
      hipLaunchKernelGGL(k_pd_rowdesc, grid_for(n), dim3(kT), 0, s, n, in.order, in.b, in.off,
                         width, cb, vb, D.rows);
      PD_TRY(hipGetLastError());
    }
    if (nnzb > 0) {
      hipLaunchKernelGGL(k_pd_blocks, grid_for(nnzb), dim3(kT), 0, s, nnzb, d, val_s, out.blk_row,
                         in.ci, in.b, rank, cpos, cb, vb, D.blk_pos, D.blk_k0, D.blk_prow);
      PD_TRY(hipGetLastError());
    }
    // the host copies above must land before the arrays are reused
    PD_TRY(hipStreamSynchronize(s));
    D.n_cols = host[3 * d];
    D.n_values = host[3 * d + 1];
    D.max_panel = host[3 * d + 2];
  }
  PD_TRY(hipMemsetAsync(hist, 0, sizeof(unsigned int) * kShapeSide * kShapeSide, s));
  if (nnzb > 0) {
    hipLaunchKernelGGL(k_pd_shapes, grid_for(nnzb), dim3(kT), 0, s, nnzb, out.blk_row, in.ci, in.b,
                       hist);
    PD_TRY(hipGetLastError());
  }
  std::vector<unsigned int> hh((size_t)kShapeSide * kShapeSide);
  PD_TRY(hipMemcpyAsync(hh.data(), hist, sizeof(unsigned int) * hh.size(), hipMemcpyDeviceToHost, s));
  PD_TRY(hipMemcpyAsync(&out.nnz, out.gbase + nnzb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PD_TRY(hipStreamSynchronize(s));
  for (unsigned int c : hh) out.n_shapes += c ? 1 : 0;
  return hipSuccess;
}

hipError_t spgemm_filter_device(int32_t n, int64_t nC, const int64_t *rp, const int32_t *ci,
                                const int64_t *obase, const double *norm, double eps,
                                const double *vals, FilterOut &out, const DevAlloc &alloc,
                                hipStream_t s) {
  out = FilterOut{};
  PD_TRY(hipGetLastError());
  auto sz = [](size_t elem, size_t count) { return (elem * (count ? count : 1) + 255) / 256 * 256; };
  const size_t C1 = (size_t)nC + 1;
  char *base = nullptr;
  {
    void *q = nullptr;
    PD_TRY(alloc(&q, 4 * sz(8, C1)));
    base = static_cast<char *>(q);
  }
  int64_t *keep = reinterpret_cast<int64_t *>(base);
  int64_t *vsz = reinterpret_cast<int64_t *>(base + sz(8, C1));
  int64_t *kidx = reinterpret_cast<int64_t *>(base + 2 * sz(8, C1));
  int64_t *vpos = reinterpret_cast<int64_t *>(base + 3 * sz(8, C1));
  void *cub_tmp = nullptr;
  size_t cub_bytes = 0;
  auto cub_run = [&](auto &&call) -> hipError_t {
    size_t need = 0;
    PD_TRY(call(nullptr, need));
    if (need > cub_bytes) {
      PD_TRY(alloc(&cub_tmp, need));
      cub_bytes = need;
    }
    return call(cub_tmp, need);
  };
  hipLaunchKernelGGL(k_flt_flags, grid_for(nC + 1), dim3(kT), 0, s, nC, norm, eps, obase, keep, vsz);
  PD_TRY(hipGetLastError());
  PD_TRY(cub_run([&](void *t, size_t &bytes) {
    return hipcub::DeviceScan::ExclusiveSum(t, bytes, keep, kidx, (int)C1, s);
  }));
  PD_TRY(cub_run([&](void *t, size_t &bytes) {
    return hipcub::DeviceScan::ExclusiveSum(t, bytes, vsz, vpos, (int)C1, s);
  }));
  int64_t counts[2];
  PD_TRY(hipMemcpyAsync(&counts[0], kidx + nC, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PD_TRY(hipMemcpyAsync(&counts[1], vpos + nC, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PD_TRY(hipStreamSynchronize(s));
  out.nnzb = counts[0];
  out.nvals = counts[1];
  if (out.nnzb == nC) return hipSuccess;   // nothing removed: the inputs stand
  const size_t K = (size_t)out.nnzb;
  {
    void *q = nullptr;
    PD_TRY(alloc(&q, sz(8, (size_t)n + 1) + sz(4, K) + 2 * sz(8, K) + sz(4, K) +
                         sz(8, (size_t)out.nvals)));
    char *p = static_cast<char *>(q);
    out.rp = reinterpret_cast<int64_t *>(p);
    p += sz(8, (size_t)n + 1);
    out.ci = reinterpret_cast<int32_t *>(p);
    p += sz(4, K);
    int64_t *sbase = reinterpret_cast<int64_t *>(p);
    p += sz(8, K);
    int64_t *dbase = reinterpret_cast<int64_t *>(p);
    p += sz(8, K);
    int32_t *size = reinterpret_cast<int32_t *>(p);
    p += sz(4, K);
    out.vals = reinterpret_cast<double *>(p);
    if (nC > 0) {
      hipLaunchKernelGGL(k_flt_compact, grid_for(nC), dim3(kT), 0, s, nC, keep, kidx, vpos, ci,
                         obase, out.ci, sbase, dbase, size);
      PD_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_flt_rowptr, grid_for((int64_t)n + 1), dim3(kT), 0, s, n, rp, kidx, out.rp);
    PD_TRY(hipGetLastError());
    PD_TRY(launch_gather_blocks(vals, sbase, dbase, size, out.nnzb, out.vals, s));
  }
  return hipSuccess;
}

hipError_t launch_page_order(const int64_t *pos, int64_t nnzb, int64_t n_values, int32_t *order,
                             const DevAlloc &alloc, hipStream_t s) {
  if (nnzb <= 0) return hipSuccess;
  if (nnzb >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  auto sz = [](size_t elem, size_t count) { return (elem * (count ? count : 1) + 255) / 256 * 256; };
  const size_t E = (size_t)nnzb;
  size_t cub_bytes = 0;
  PD_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, cub_bytes, pos, (int64_t *)nullptr,
                                            (const int32_t *)nullptr, order, (int)nnzb, 0,
                                            bits_for(n_values), s));
  void *q = nullptr;
  PD_TRY(alloc(&q, sz(8, E) + sz(4, E) + sz(1, cub_bytes)));
  char *base = static_cast<char *>(q);
  int64_t *pos_s = reinterpret_cast<int64_t *>(base);
  int32_t *iota = reinterpret_cast<int32_t *>(base + sz(8, E));
  void *cub_tmp = base + sz(8, E) + sz(4, E);
  hipLaunchKernelGGL(k_pd_iota, grid_for(nnzb), dim3(kT), 0, s, (int32_t)nnzb, iota);
  PD_TRY(hipGetLastError());
  return hipcub::DeviceRadixSort::SortPairs(cub_tmp, cub_bytes, pos, pos_s, iota, order, (int)nnzb,
                                            0, bits_for(n_values), s);
}

}  // namespace vbcsr
