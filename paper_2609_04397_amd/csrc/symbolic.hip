// Symbolic stage of the thresholded block product C = A B on the device
// (paper, section 3.2, equations 2 and 3): candidate blocks, the block-norm
// bound, the kept pattern and the per-block product lists the numeric stage
// consumes.
//
// Expand, sort, compress: every product A_ik B_kj of row i becomes one entry
// with key (j << 32 | position of A_ik in row i); a segmented radix sort per
// row orders the entries by candidate column j and, within a candidate, by
// A's stored order of k.  A candidate is a run of equal j; one thread sums its
// bound U_ij = sum_k ||A_ik|| ||B_kj|| over the run in that order (multiply
// and add rounded separately, as plain host arithmetic does), so every bound,
// and hence every keep or drop decision, is the one a sequential sweep over k
// in A's order computes.  Scans over the candidates give C's pattern
// (columns ascending per row), the value offsets of the kept blocks and
// their product ranges; the products of a kept block keep A's stored order.
#include <hipcub/hipcub.hpp>

#include "kernels.hpp"

namespace vbcsr {
namespace {

constexpr int kT = 256;

dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kT - 1) / kT)); }

// products of each stored block A_ik: the length of B's row k
__global__ void __launch_bounds__(kT) k_sym_count(const int32_t *aci, const int64_t *brp,
                                                  int64_t annzb, int64_t *cnt) {
  const int64_t ka = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (ka < annzb) {
    const int32_t k = aci[ka];
    cnt[ka] = brp[k + 1] - brp[k];
  } else if (ka == annzb) {
    cnt[ka] = 0;
  }
}

// seg[i] = first entry of row i (i <= n)
__global__ void __launch_bounds__(kT) k_sym_rowseg(const int64_t *arp, const int64_t *eoff,
                                                   int32_t n, int64_t *seg) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i <= n) seg[i] = eoff[arp[i]];
}

// one thread per stored block A_ik writes the entries of its products
__global__ void __launch_bounds__(kT) k_sym_expand(const int64_t *arp, const int32_t *aci,
                                                   const int32_t *arow, int64_t annzb,
                                                   const int64_t *brp, const int32_t *bci,
                                                   const int64_t *eoff, uint64_t *key,
                                                   int64_t *val) {
  const int64_t ka = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (ka >= annzb) return;
  const int32_t i = arow[ka];
  const uint32_t rel = (uint32_t)(ka - arp[i]);
  const int32_t k = aci[ka];
  const int64_t b0 = brp[k], b1 = brp[k + 1];
  const int64_t e0 = eoff[ka] - b0;
  for (int64_t kb = b0; kb < b1; ++kb) {
    key[e0 + kb] = ((uint64_t)(uint32_t)bci[kb] << 32) | rel;
    val[e0 + kb] = kb;
  }
}

// one wave per row: flag[e] = 1 where a candidate (a run of equal j) starts
__global__ void __launch_bounds__(kT) k_sym_flags(const int64_t *seg, int32_t n,
                                                  const uint64_t *key, int32_t *flag) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int lane = threadIdx.x & 63;
  const int64_t s0 = seg[row], s1 = seg[row + 1];
  for (int64_t e = s0 + lane; e < s1; e += 64)
    flag[e] = (e == s0 || (key[e] >> 32) != (key[e - 1] >> 32)) ? 1 : 0;
}

// candidate g: first entry and row (ginc = inclusive scan of the flags)
__global__ void __launch_bounds__(kT) k_sym_groups(const int64_t *seg, int32_t n,
                                                   const int32_t *flag, const int32_t *ginc,
                                                   int64_t *gstart, int32_t *grow) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int lane = threadIdx.x & 63;
  for (int64_t e = seg[row] + lane; e < seg[row + 1]; e += 64)
    if (flag[e]) {
      const int32_t g = ginc[e] - 1;
      gstart[g] = e;
      grow[g] = (int32_t)row;
    }
}

// one thread per candidate: bound (over the run, in A's order of k), product
// count, values and flops of the block if kept
__global__ void __launch_bounds__(kT) k_sym_reduce(
    int64_t nG, int64_t nE, const int64_t *gstart, const int32_t *grow, const uint64_t *key,
    const int64_t *val, const int64_t *arp, const int32_t *aci, const int32_t *b, const double *an,
    const double *bn, double eps, int64_t *gkeep, int64_t *gnp, int64_t *gvs, double *gfl,
    double *gbound, int32_t *gj) {
  const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (g >= nG) return;
  const int64_t e0 = gstart[g], e1 = g + 1 < nG ? gstart[g + 1] : nE;
  const int32_t i = grow[g];
  const int32_t j = (int32_t)(key[e0] >> 32);
  const int64_t a0 = arp[i];
  double u = 0.0;
  int64_t bks = 0;
  for (int64_t e = e0; e < e1; ++e) {
    const int64_t ka = a0 + (int64_t)(key[e] & 0xFFFFFFFFu);
    if (an) u = __dadd_rn(u, __dmul_rn(an[ka], bn[val[e]]));
    bks += b[aci[ka]];
  }
  const bool keep = an ? !(u < eps) : true;
  gkeep[g] = keep ? 1 : 0;
  gnp[g] = keep ? e1 - e0 : 0;
  gvs[g] = keep ? (int64_t)b[i] * b[j] : 0;
  gfl[g] = keep ? 2.0 * b[i] * (double)bks * b[j] : 0.0;
  gbound[g] = an ? u : 0.0;
  gj[g] = j;
}

// kept candidate g becomes block c = kidx[g] of C
__global__ void __launch_bounds__(kT) k_sym_emit(int64_t nG, const int64_t *gkeep,
                                                 const int64_t *kidx, const int32_t *grow,
                                                 const int32_t *gj, const double *gbound,
                                                 const int64_t *pptr_g, const int64_t *obase_g,
                                                 int32_t *oi, int32_t *oj, double *bound,
                                                 int64_t *pptr, int64_t *obase) {
  const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (g > nG) return;
  const int64_t c = kidx[g];
  if (g == nG) {  // closing offsets
    pptr[c] = pptr_g[g];
    obase[c] = obase_g[g];
    return;
  }
  if (!gkeep[g]) return;
  oi[c] = grow[g];
  oj[c] = gj[g];
  bound[c] = gbound[g];
  pptr[c] = pptr_g[g];
  obase[c] = obase_g[g];
}

// C's row pointer: kept candidates of the rows before i
__global__ void __launch_bounds__(kT) k_sym_rowptr(int32_t n, const int64_t *seg, int64_t nE,
                                                   int64_t nG, const int32_t *flag,
                                                   const int32_t *ginc, const int64_t *kidx,
                                                   int64_t *crp) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i > n) return;
  const int64_t e = seg[i];
  const int64_t gf = e < nE ? (int64_t)(ginc[e] - flag[e]) : nG;
  crp[i] = kidx[gf];
}

// one thread per entry of a kept candidate: its product
__global__ void __launch_bounds__(kT) k_sym_products(
    int64_t nE, const int32_t *ginc, const int64_t *gkeep, const int64_t *gstart,
    const int32_t *grow, const int64_t *pptr_g, const uint64_t *key, const int64_t *val,
    const int64_t *arp, const int32_t *aci, const int32_t *b, const int64_t *apos,
    const int64_t *bpos, int64_t *pa, int64_t *pb) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= nE) return;
  const int32_t g = ginc[e] - 1;
  if (!gkeep[g]) return;
  const int64_t pos = pptr_g[g] + (e - gstart[g]);
  const int64_t ka = arp[grow[g]] + (int64_t)(key[e] & 0xFFFFFFFFu);
  pa[pos] = (apos[ka] << 8) | (int64_t)b[aci[ka]];
  pb[pos] = bpos[val[e]];
}

__device__ __forceinline__ int sym_class(int bi, int bj) {
  const int ti = (bi + 15) / 16, tj = (bj + 15) / 16;
  return ti > 2 || tj > 2 ? 4 : (ti - 1) * 2 + (tj - 1);
}

// tile class of every block of C (keys of the stable class sort) and the
// class counts (per workgroup in LDS, then one global add per class)
__global__ void __launch_bounds__(kT) k_sym_class(int64_t nC, const int32_t *oi,
                                                  const int32_t *oj, const int32_t *b,
                                                  uint32_t *cls, int32_t *idx,
                                                  unsigned int *cnt) {
  __shared__ unsigned int lc[5];
  if (threadIdx.x < 5) lc[threadIdx.x] = 0;
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (c < nC) {
    const int k = sym_class(b[oi[c]], b[oj[c]]);
    cls[c] = (uint32_t)k;
    idx[c] = (int32_t)c;
    atomicAdd(&lc[k], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 5 && lc[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], lc[threadIdx.x]);
}

int bits_for(int64_t v) {  // bits to hold 0 .. v
  int nb = 1;
  while (nb < 63 && (int64_t(1) << nb) <= v) ++nb;
  return nb;
}

}  // namespace

#define SYM_TRY(x)                          \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

hipError_t spgemm_symbolic_device(const SymbolicIn &in, SymbolicOut &out, const DevAlloc &alloc,
                                  hipStream_t s) {
  out = SymbolicOut{};
  const int32_t n = in.n;
  const int64_t annzb = in.annzb;
  // arrays are carved out of a few large allocations (one per phase):
  // device allocations and frees cost about as much per call as per byte
  struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0;
  } arena;
  auto reserve = [&](size_t bytes) -> hipError_t {
    void *q = nullptr;
    hipError_t e = alloc(&q, bytes + 256);
    arena.base = static_cast<char *>(q);
    arena.size = bytes + 256;
    arena.used = 0;
    return e;
  };
  auto sz = [](size_t elem, size_t count) { return (elem * (count ? count : 1) + 255) / 256 * 256; };
  auto get = [&](auto **p, size_t count) -> hipError_t {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
    const size_t bytes = sz(sizeof(T), count);
    if (arena.used + bytes > arena.size) return hipErrorOutOfMemory;  // sizes below are exact
    *p = reinterpret_cast<T *>(arena.base + arena.used);
    arena.used += bytes;
    return hipSuccess;
  };
  auto fetch = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
    SYM_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    return hipStreamSynchronize(s);
  };
  // hipCUB temporary storage, reused across calls
  void *cub_tmp = nullptr;
  size_t cub_bytes = 0;
  auto cub_run = [&](auto &&call) -> hipError_t {
    size_t need = 0;
    SYM_TRY(call(nullptr, need));
    if (need > cub_bytes) {
      SYM_TRY(alloc(&cub_tmp, need));
      cub_bytes = need;
    }
    return call(cub_tmp, need);
  };

  // entries per stored block of A and their offsets
  int64_t *cnt = nullptr, *eoff = nullptr, *seg = nullptr;
  SYM_TRY(reserve(2 * sz(8, (size_t)annzb + 1) + sz(8, (size_t)n + 1)));
  SYM_TRY(get(&cnt, (size_t)annzb + 1));
  SYM_TRY(get(&eoff, (size_t)annzb + 1));
  SYM_TRY(get(&seg, (size_t)n + 1));
  hipLaunchKernelGGL(k_sym_count, grid_for(annzb + 1), dim3(kT), 0, s, in.aci, in.brp, annzb, cnt);
  SYM_TRY(hipGetLastError());
  SYM_TRY(cub_run([&](void *t, size_t &b) {
    return hipcub::DeviceScan::ExclusiveSum(t, b, cnt, eoff, (int)(annzb + 1), s);
  }));
  hipLaunchKernelGGL(k_sym_rowseg, grid_for((int64_t)n + 1), dim3(kT), 0, s, in.arp, eoff, n, seg);
  SYM_TRY(hipGetLastError());
  int64_t nE = 0;
  SYM_TRY(fetch(&nE, eoff + annzb, sizeof(int64_t)));
  if (nE >= (int64_t(1) << 31)) return hipErrorInvalidValue;  // beyond the 32-bit sort counts
  out.products_all = nE;
  if (nE == 0) {
    SYM_TRY(reserve(sz(8, (size_t)n + 1) + 2 * sz(8, 1)));
    SYM_TRY(get(&out.crp, (size_t)n + 1));
    SYM_TRY(hipMemsetAsync(out.crp, 0, sizeof(int64_t) * ((size_t)n + 1), s));
    SYM_TRY(get(&out.pptr, 1));
    SYM_TRY(get(&out.obase, 1));
    SYM_TRY(hipMemsetAsync(out.pptr, 0, sizeof(int64_t), s));
    SYM_TRY(hipMemsetAsync(out.obase, 0, sizeof(int64_t), s));
    return hipSuccess;
  }

  // expand and sort per row by (j, position of A_ik in the row)
  uint64_t *key = nullptr, *key_s = nullptr;
  int64_t *val = nullptr, *val_s = nullptr;
  int32_t *flag = nullptr, *ginc = nullptr;
  SYM_TRY(reserve(4 * sz(8, (size_t)nE) + 2 * sz(4, (size_t)nE)));
  SYM_TRY(get(&key, (size_t)nE));
  SYM_TRY(get(&key_s, (size_t)nE));
  SYM_TRY(get(&val, (size_t)nE));
  SYM_TRY(get(&val_s, (size_t)nE));
  hipLaunchKernelGGL(k_sym_expand, grid_for(annzb), dim3(kT), 0, s, in.arp, in.aci, in.arow, annzb,
                     in.brp, in.bci, eoff, key, val);
  SYM_TRY(hipGetLastError());
  const int end_bit = 32 + bits_for(n > 0 ? n - 1 : 0);
  SYM_TRY(cub_run([&](void *t, size_t &b) {
    return hipcub::DeviceSegmentedRadixSort::SortPairs(t, b, key, key_s, val, val_s, (int)nE, (int)n,
                                                       seg, seg + 1, 0, end_bit, s);
  }));

  // candidates: runs of equal j
  SYM_TRY(get(&flag, (size_t)nE));
  SYM_TRY(get(&ginc, (size_t)nE));
  const dim3 rows_grid((unsigned)((n + 3) / 4));
  hipLaunchKernelGGL(k_sym_flags, rows_grid, dim3(kT), 0, s, seg, n, key_s, flag);
  SYM_TRY(hipGetLastError());
  SYM_TRY(cub_run([&](void *t, size_t &b) {
    return hipcub::DeviceScan::InclusiveSum(t, b, flag, ginc, (int)nE, s);
  }));
  int32_t nG32 = 0;
  SYM_TRY(fetch(&nG32, ginc + (nE - 1), sizeof(int32_t)));
  const int64_t nG = nG32;
  out.candidates = nG;
  int64_t *gstart = nullptr;
  int32_t *grow = nullptr, *gj = nullptr;
  SYM_TRY(reserve(sz(8, (size_t)nG) + 2 * sz(4, (size_t)nG) + 6 * sz(8, (size_t)nG + 1) +
                  2 * sz(8, (size_t)nG) + sz(8, 1)));
  SYM_TRY(get(&gstart, (size_t)nG));
  SYM_TRY(get(&grow, (size_t)nG));
  SYM_TRY(get(&gj, (size_t)nG));
  hipLaunchKernelGGL(k_sym_groups, rows_grid, dim3(kT), 0, s, seg, n, flag, ginc, gstart, grow);
  SYM_TRY(hipGetLastError());

  // bounds, decisions and sizes per candidate; scans over the kept ones
  int64_t *gkeep = nullptr, *gnp = nullptr, *gvs = nullptr;
  int64_t *kidx = nullptr, *pptr_g = nullptr, *obase_g = nullptr;
  double *gfl = nullptr, *gbound = nullptr, *flops = nullptr;
  SYM_TRY(get(&gkeep, (size_t)nG + 1));
  SYM_TRY(get(&gnp, (size_t)nG + 1));
  SYM_TRY(get(&gvs, (size_t)nG + 1));
  SYM_TRY(get(&kidx, (size_t)nG + 1));
  SYM_TRY(get(&pptr_g, (size_t)nG + 1));
  SYM_TRY(get(&obase_g, (size_t)nG + 1));
  SYM_TRY(get(&gfl, (size_t)nG));
  SYM_TRY(get(&gbound, (size_t)nG));
  SYM_TRY(get(&flops, 1));
  SYM_TRY(hipMemsetAsync(gkeep + nG, 0, sizeof(int64_t), s));
  SYM_TRY(hipMemsetAsync(gnp + nG, 0, sizeof(int64_t), s));
  SYM_TRY(hipMemsetAsync(gvs + nG, 0, sizeof(int64_t), s));
  hipLaunchKernelGGL(k_sym_reduce, grid_for(nG), dim3(kT), 0, s, nG, nE, gstart, grow, key_s, val_s,
                     in.arp, in.aci, in.b, in.an, in.bn, in.eps, gkeep, gnp, gvs, gfl, gbound, gj);
  SYM_TRY(hipGetLastError());
  SYM_TRY(cub_run([&](void *t, size_t &b) {
    return hipcub::DeviceScan::ExclusiveSum(t, b, gkeep, kidx, (int)(nG + 1), s);
  }));
  SYM_TRY(cub_run([&](void *t, size_t &b) {
    return hipcub::DeviceScan::ExclusiveSum(t, b, gnp, pptr_g, (int)(nG + 1), s);
  }));
  SYM_TRY(cub_run([&](void *t, size_t &b) {
    return hipcub::DeviceScan::ExclusiveSum(t, b, gvs, obase_g, (int)(nG + 1), s);
  }));
  SYM_TRY(cub_run([&](void *t, size_t &b) {
    return hipcub::DeviceReduce::Sum(t, b, gfl, flops, (int)nG, s);
  }));
  int64_t tot[3];
  SYM_TRY(hipMemcpyAsync(&tot[0], kidx + nG, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SYM_TRY(hipMemcpyAsync(&tot[1], pptr_g + nG, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SYM_TRY(hipMemcpyAsync(&tot[2], obase_g + nG, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SYM_TRY(hipMemcpyAsync(&out.flops, flops, sizeof(double), hipMemcpyDeviceToHost, s));
  SYM_TRY(hipStreamSynchronize(s));
  const int64_t nC = tot[0];
  out.nC = nC;
  out.nP = tot[1];
  out.nvals = tot[2];

  // C's blocks, row pointer and product lists (and the class sort)
  SYM_TRY(reserve(2 * sz(4, (size_t)nC) + sz(8, (size_t)nC) + 2 * sz(8, (size_t)nC + 1) +
                  sz(8, (size_t)n + 1) + 2 * sz(8, (size_t)out.nP) + 2 * sz(4, (size_t)nC) +
                  2 * sz(4, (size_t)nC) + sz(4, 5)));
  SYM_TRY(get(&out.oi, (size_t)nC));
  SYM_TRY(get(&out.oj, (size_t)nC));
  SYM_TRY(get(&out.bound, (size_t)nC));
  SYM_TRY(get(&out.pptr, (size_t)nC + 1));
  SYM_TRY(get(&out.obase, (size_t)nC + 1));
  SYM_TRY(get(&out.crp, (size_t)n + 1));
  SYM_TRY(get(&out.pa, (size_t)out.nP));
  SYM_TRY(get(&out.pb, (size_t)out.nP));
  hipLaunchKernelGGL(k_sym_emit, grid_for(nG + 1), dim3(kT), 0, s, nG, gkeep, kidx, grow, gj,
                     gbound, pptr_g, obase_g, out.oi, out.oj, out.bound, out.pptr, out.obase);
  SYM_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_sym_rowptr, grid_for((int64_t)n + 1), dim3(kT), 0, s, n, seg, nE, nG, flag,
                     ginc, kidx, out.crp);
  SYM_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_sym_products, grid_for(nE), dim3(kT), 0, s, nE, ginc, gkeep, gstart, grow,
                     pptr_g, key_s, val_s, in.arp, in.aci, in.b, in.apos, in.bpos, out.pa, out.pb);
  SYM_TRY(hipGetLastError());

  // blocks grouped by tile class, stable
  if (nC > 0) {
    uint32_t *cls = nullptr, *cls_s = nullptr;
    int32_t *idx = nullptr;
    unsigned int *ccnt = nullptr;
    SYM_TRY(get(&cls, (size_t)nC));
    SYM_TRY(get(&cls_s, (size_t)nC));
    SYM_TRY(get(&idx, (size_t)nC));
    SYM_TRY(get(&out.order, (size_t)nC));
    SYM_TRY(get(&ccnt, 5));
    SYM_TRY(hipMemsetAsync(ccnt, 0, sizeof(unsigned int) * 5, s));
    hipLaunchKernelGGL(k_sym_class, grid_for(nC), dim3(kT), 0, s, nC, out.oi, out.oj, in.b, cls, idx,
                       ccnt);
    SYM_TRY(hipGetLastError());
    SYM_TRY(cub_run([&](void *t, size_t &b) {
      return hipcub::DeviceRadixSort::SortPairs(t, b, cls, cls_s, idx, out.order, (int)nC, 0, 3, s);
    }));
    unsigned int hc[5];
    SYM_TRY(fetch(hc, ccnt, sizeof(hc)));
    for (int k = 0; k < 5; ++k) out.cls_begin[k + 1] = out.cls_begin[k] + hc[k];
  }
  return hipSuccess;
}

}  // namespace vbcsr
