// gfx950 kernels of the reciprocal-space operator O(k) = sum_R e^{-2 pi i k.R} O(R)
// (paper, section 3.3, equation 4) and its complex products (section 3.2 and
// equation 1 with the conjugate transpose).
#include <hip/hip_runtime.h>

#include "zkernels.hpp"

namespace vbcsr {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

template <typename T> struct C2;
template <> struct C2<double> { using type = double2; };
template <> struct C2<float> { using type = float2; };

__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

__global__ void __launch_bounds__(kThreads) k_zphase(ZPhaseParams P) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= P.n) return;
  const int32_t *R = P.shifts + 3 * (int64_t)P.image[c];
  double d0 = R[0], d1 = R[1], d2 = R[2];
  if (P.tau) {
    const double *tj = P.tau + 3 * (int64_t)P.col_idx[c];
    const double *ti = P.tau + 3 * (int64_t)P.blk_row[c];
    d0 += tj[0] - ti[0];
    d1 += tj[1] - ti[1];
    d2 += tj[2] - ti[2];
  }
  const double th = -2.0 * M_PI * (P.k[0] * d0 + P.k[1] * d1 + P.k[2] * d2);
  double sn, cs;
  sincos(th, &sn, &cs);
  P.ph[2 * c] = cs;
  P.ph[2 * c + 1] = sn;
}

// Values in flight per lane in the sampling kernel.
constexpr int kSampleBatch = 8;

// The wave's blocks are kb0 .. kb0 + nb - 1, their values numbered 0 .. T-1
// in graph order; lane l takes values l, l + 64, ... in batches whose value
// and phase loads are all issued before the first use.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_zsample(ZSampleParams P, T *fwd, T *tr) {
  using V2 = typename C2<T>::type;
  const int64_t kb0 = ((int64_t)blockIdx.x * kWaves + wave_id()) * kSampleBlocks;
  if (kb0 >= P.nkb) return;
  const int lane = threadIdx.x & 63;
  const int nb = (int)min((int64_t)kSampleBlocks, P.nkb - kb0);
  // lane j < nb holds block kb0 + j; lane nb reads the end of the last block
  int d = 0, cnt = 0;
  int64_t base = 0, vb = 0, c0 = 0, fp = 0, tp = 0;
  if (lane <= nb) base = P.kbase[kb0 + lane];
  if (lane < nb) {
    const int64_t kb = kb0 + lane;
    d = P.kdim[kb];
    c0 = P.cptr[kb];
    cnt = (int)(P.cptr[kb + 1] - c0);
    vb = P.kvbase[kb];
    fp = P.fwd_pos[kb];
    tp = P.tr_pos[kb];
  }
  const int rel = (int)(base - __shfl(base, 0));  // value offset of lane j's block
  const int total = __builtin_amdgcn_readlane(rel, nb);
  int start[kSampleBlocks];
#pragma unroll
  for (int k = 0; k < kSampleBlocks; ++k)
    start[k] = k <= nb ? __builtin_amdgcn_readlane(rel, k) : total;
  const double2 *ph = reinterpret_cast<const double2 *>(P.ph);
  for (int v0 = 0; v0 < total; v0 += 64 * kSampleBatch) {
    double x[kSampleBatch];
    double2 w[kSampleBatch];
    int jv[kSampleBatch], ev[kSampleBatch];
#pragma unroll
    for (int u = 0; u < kSampleBatch; ++u) {
      const int v = v0 + 64 * u + lane;
      int j = 0;
#pragma unroll
      for (int k = 1; k < kSampleBlocks; ++k) j += start[k] <= v ? 1 : 0;
      jv[u] = j;
      ev[u] = v - __shfl(rel, j);
      const int64_t vbj = __shfl(vb, j), c0j = __shfl(c0, j);
      x[u] = 0.0;
      w[u] = make_double2(0.0, 0.0);
      if (v < total) {
        x[u] = P.values[vbj + ev[u]];
        w[u] = ph[c0j];
      }
    }
#pragma unroll
    for (int u = 0; u < kSampleBatch; ++u) {
      const int v = v0 + 64 * u + lane, j = jv[u], e = ev[u];
      const int dj = __shfl(d, j), cj = __shfl(cnt, j);
      const int64_t c0j = __shfl(c0, j), fj = __shfl(fp, j), tj = __shfl(tp, j);
      if (v >= total) continue;
      double re = x[u] * w[u].x, im = x[u] * w[u].y;
      for (int64_t c = c0j + 1; c < c0j + cj; ++c) {  // further images of the block
        const double y = P.values[P.cgbase[c] + e];
        const double2 z = ph[c];
        re = fma(y, z.x, re);
        im = fma(y, z.y, im);
      }
      const int bi = dj & 0xffff, bj = dj >> 16;
      const int p = e / bj, q = e - p * bj;
      V2 o;
      o.x = (T)re;
      o.y = (T)im;
      *reinterpret_cast<V2 *>(fwd + 2 * (fj + (int64_t)q * bi + p)) = o;  // column-major
      o.y = (T)(-im);
      *reinterpret_cast<V2 *>(tr + 2 * (tj + (int64_t)e)) = o;  // row-major (= A^H column-major)
    }
  }
}

// One wave per panel (block row of op(O)): lane (g, p) takes panel row p and
// the panel columns k = g, g + G, ... (G = floor(64 / b) groups), NR
// right-hand sides per pass; groups are reduced by shuffles.  Every complex
// product is four FMAs in T.
template <typename T, int NR>
__global__ void __launch_bounds__(kThreads) k_zspmm(ZSpmmParams<T> P) {
  using V = typename C2<T>::type;
  const int row = blockIdx.x * kWaves + wave_id();
  if (row >= P.nrows) return;
  const int lane = threadIdx.x & 63;
  const RowDesc rd = P.rows[row];
  const int b = rd.b, K = rd.K;
  const int G = 64 / b;
  const int g = lane / b, p = lane - g * b;
  const bool act = g < G;
  const V *__restrict__ A = reinterpret_cast<const V *>(P.pages) + rd.vbase;
  const int32_t *__restrict__ cx = P.colx + rd.cbase;
  const V *__restrict__ X = reinterpret_cast<const V *>(P.X);
  V *__restrict__ Y = reinterpret_cast<V *>(P.Y);
  for (int c0 = 0; c0 < P.nrhs; c0 += NR) {
    T re[NR], im[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) re[c] = im[c] = T(0);
    if (act && g < K) {
      // the operands of column k + G are in flight while column k
      // multiplies; the index is clamped to the last column (no branch
      // around the loads), the clamped copy is never multiplied
      const int nc = min(NR, P.nrhs - c0);
      V a = A[(int64_t)g * b + p];
      V x[NR];
      {
        const V *xr = X + (int64_t)cx[g] * P.ldx + c0;
#pragma unroll
        for (int c = 0; c < NR; ++c) x[c] = xr[min(c, nc - 1)];
      }
      for (int k = g; k < K; k += G) {
        const int kn = min(k + G, K - 1);
        const V an = A[(int64_t)kn * b + p];
        const V *xn = X + (int64_t)cx[kn] * P.ldx + c0;
        V xv[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) xv[c] = xn[min(c, nc - 1)];
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          re[c] = fma(a.x, x[c].x, re[c]);
          re[c] = fma(-a.y, x[c].y, re[c]);
          im[c] = fma(a.x, x[c].y, im[c]);
          im[c] = fma(a.y, x[c].x, im[c]);
        }
        a = an;
#pragma unroll
        for (int c = 0; c < NR; ++c) x[c] = xv[c];
      }
    }
    for (int st = 1; st < G; st <<= 1) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const T orr = __shfl_down(re[c], st * b, 64);
        const T oi = __shfl_down(im[c], st * b, 64);
        if (act && (g & (2 * st - 1)) == 0 && g + st < G) {
          re[c] += orr;
          im[c] += oi;
        }
      }
    }
    if (lane < b) {
      V *yr = Y + (int64_t)(rd.yrow + p) * P.ldy + c0;
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        if (c0 + c < P.nrhs) {
          const double sr = re[c], si = im[c];
          double yr_ = P.ar * sr - P.ai * si, yi_ = P.ar * si + P.ai * sr;
          if (P.br != 0.0 || P.bi != 0.0) {
            const V y = yr[c];
            yr_ += P.br * (double)y.x - P.bi * (double)y.y;
            yi_ += P.br * (double)y.y + P.bi * (double)y.x;
          }
          V o;
          o.x = (T)yr_;
          o.y = (T)yi_;
          yr[c] = o;
        }
      }
    }
  }
}

// Complex product on FP64 matrix cores, for 16 right-hand sides per tile:
// one wave per panel, M = panel rows in tiles of 16, K = panel columns in
// slices of 4, N = 16 right-hand sides per tile, NT tiles per pass.  Lane
// (m, kq) loads 16 bytes of A (row m, column 4s + kq: one complex value) and,
// per tile, 16 bytes of X (row colx[4s + kq], right-hand side m); four real
// products per complex tile accumulate Ar Xr, Ai Xi, Ar Xi, Ai Xr.  Rows past
// the panel, columns past K and right-hand sides past nrhs read zeros
// through the buffer bounds.  The next slice's operands are in flight while
// the current one multiplies.
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t zrsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ double2 zload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

template <int NT>
__global__ void __launch_bounds__(kThreads) k_zspmm_mfma(ZSpmmParams<double> P, uint32_t xbytes) {
  const int row = blockIdx.x * kWaves + wave_id();
  if (row >= P.nrows) return;
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, kq = lane >> 4;
  const RowDesc rd = P.rows[row];
  const int b = rd.b, K = rd.K;
  constexpr uint32_t kOut = 0x80000000u;
  const __amdgpu_buffer_rsrc_t ra = zrsrc(reinterpret_cast<const double2 *>(P.pages) + rd.vbase,
                                          (uint32_t)K * (uint32_t)b * 16u);
  const __amdgpu_buffer_rsrc_t rx = zrsrc(P.X, xbytes);
  const int32_t *__restrict__ cx = P.colx + rd.cbase;
  const int nsl = (K + 3) >> 2;
  double2 *__restrict__ Y = reinterpret_cast<double2 *>(P.Y);
  for (int mt = 0; mt * 16 < b; ++mt) {
    const int ar = mt * 16 + m;
    for (int c0 = 0; c0 < P.nrhs; c0 += 16 * NT) {
      v4d rr[NT], ii[NT], ri[NT], ir[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) rr[t] = ii[t] = ri[t] = ir[t] = v4d{0.0, 0.0, 0.0, 0.0};
      // three stages: the column index of slice s + 2, the values and X rows
      // of slice s + 1 (whose index arrived one slice earlier), the matrix
      // instructions of slice s; slices past the end repeat the last one
      auto ld_idx = [&](int s) {
        const int k = 4 * s + kq;
        return k < K ? cx[min(k, K - 1)] : -1;
      };
      auto ld = [&](int s, int xr, double2 &a, double2 (&x)[NT]) {
        const int k = 4 * s + kq;
        a = zload(ra, ar < b ? (uint32_t)(k * b + ar) * 16u : kOut);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int c = c0 + t * 16 + m;
          x[t] = zload(rx, xr >= 0 && c < P.nrhs
                                ? (uint32_t)(((int64_t)xr * P.ldx + c) * 16)
                                : kOut);
        }
      };
      if (nsl > 0) {
        double2 a, x[NT];
        int xi1 = ld_idx(min(1, nsl - 1));
        ld(0, ld_idx(0), a, x);
        for (int s = 0; s < nsl; ++s) {
          const int xi2 = ld_idx(min(s + 2, nsl - 1));
          double2 an, xn[NT];
          ld(min(s + 1, nsl - 1), xi1, an, xn);
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            rr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, x[t].x, rr[t], 0, 0, 0);
            ii[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, x[t].y, ii[t], 0, 0, 0);
            ri[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, x[t].y, ri[t], 0, 0, 0);
            ir[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, x[t].x, ir[t], 0, 0, 0);
          }
          a = an;
#pragma unroll
          for (int t = 0; t < NT; ++t) x[t] = xn[t];
          xi1 = xi2;
        }
      }
      // accumulator element e of quarter-wave kq: tile row kq + 4e, column m
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = c0 + t * 16 + m;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = mt * 16 + kq + 4 * e;
          if (r < b && c < P.nrhs) {
            const double sr = rr[t][e] - ii[t][e], si = ri[t][e] + ir[t][e];
            double2 *yp = Y + (int64_t)(rd.yrow + r) * P.ldy + c;
            double yr = P.ar * sr - P.ai * si, yi = P.ar * si + P.ai * sr;
            if (P.br != 0.0 || P.bi != 0.0) {
              const double2 y = *yp;
              yr += P.br * y.x - P.bi * y.y;
              yi += P.br * y.y + P.bi * y.x;
            }
            *yp = double2{yr, yi};
          }
        }
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_zunpack(const T *fwd, const int64_t *pos,
                                                      const int32_t *krow, const int32_t *kcol,
                                                      const int32_t *b, const int64_t *kbase,
                                                      int64_t nkb, T *dst) {
  const int64_t kb = (int64_t)blockIdx.x * kWaves + wave_id();
  if (kb >= nkb) return;
  const int lane = threadIdx.x & 63;
  const int bi = b[krow[kb]], bj = b[kcol[kb]];
  const T *f = fwd + 2 * pos[kb];
  T *d = dst + 2 * kbase[kb];
  for (int e = lane; e < bi * bj; e += 64) {
    const int p = e / bj, q = e - p * bj;
    d[2 * e] = f[2 * ((int64_t)q * bi + p)];
    d[2 * e + 1] = f[2 * ((int64_t)q * bi + p) + 1];
  }
}

template <typename T>
hipError_t launch_zspmm_t(const ZSpmmParams<T> &p, hipStream_t s) {
  if (p.nrows == 0) return hipSuccess;
  const dim3 grid((unsigned)((p.nrows + kWaves - 1) / kWaves));
  // right-hand sides per pass: every pass streams the pages once more
  if (p.nrhs == 1)
    hipLaunchKernelGGL((k_zspmm<T, 1>), grid, dim3(kThreads), 0, s, p);
  else if (p.nrhs == 2)
    hipLaunchKernelGGL((k_zspmm<T, 2>), grid, dim3(kThreads), 0, s, p);
  else if (p.nrhs <= 4)
    hipLaunchKernelGGL((k_zspmm<T, 4>), grid, dim3(kThreads), 0, s, p);
  else if (p.nrhs <= 8)
    hipLaunchKernelGGL((k_zspmm<T, 8>), grid, dim3(kThreads), 0, s, p);
  else
    hipLaunchKernelGGL((k_zspmm<T, 16>), grid, dim3(kThreads), 0, s, p);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zphase(const ZPhaseParams &p, hipStream_t s) {
  if (p.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zphase, dim3((unsigned)((p.n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_zsample(const ZSampleParams &p, void *fwd, void *tr, int elem_bytes,
                          hipStream_t s) {
  if (p.nkb == 0) return hipSuccess;
  const int64_t waves = (p.nkb + kSampleBlocks - 1) / kSampleBlocks;
  const dim3 grid((unsigned)((waves + kWaves - 1) / kWaves));
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_zsample<double>, grid, dim3(kThreads), 0, s, p,
                       static_cast<double *>(fwd), static_cast<double *>(tr));
  else
    hipLaunchKernelGGL(k_zsample<float>, grid, dim3(kThreads), 0, s, p,
                       static_cast<float *>(fwd), static_cast<float *>(tr));
  return hipGetLastError();
}

hipError_t launch_zspmm_f64(const ZSpmmParams<double> &p, hipStream_t s) {
  // 16 or more right-hand sides go to matrix cores when X spans less than
  // 2^31 bytes (one buffer descriptor with 32-bit offsets)
  const int64_t xspan = ((int64_t)p.xrows - 1) * p.ldx + p.nrhs;
  if (p.nrhs < 16 || p.nrows == 0 || xspan * 16 >= (int64_t(1) << 31)) return launch_zspmm_t(p, s);
  const dim3 grid((unsigned)((p.nrows + kWaves - 1) / kWaves));
  const uint32_t xb = (uint32_t)(xspan * 16);
  if (p.nrhs <= 16)
    hipLaunchKernelGGL(k_zspmm_mfma<1>, grid, dim3(kThreads), 0, s, p, xb);
  else if (p.nrhs <= 32)
    hipLaunchKernelGGL(k_zspmm_mfma<2>, grid, dim3(kThreads), 0, s, p, xb);
  else
    hipLaunchKernelGGL(k_zspmm_mfma<4>, grid, dim3(kThreads), 0, s, p, xb);
  return hipGetLastError();
}
hipError_t launch_zspmm_f32(const ZSpmmParams<float> &p, hipStream_t s) {
  return launch_zspmm_t(p, s);
}

hipError_t launch_zunpack(const void *fwd, int elem_bytes, const int64_t *pos,
                          const int32_t *krow, const int32_t *kcol, const int32_t *b,
                          const int64_t *kbase, int64_t nkb, void *dst, hipStream_t s) {
  if (nkb == 0) return hipSuccess;
  const dim3 grid((unsigned)((nkb + kWaves - 1) / kWaves));
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_zunpack<double>, grid, dim3(kThreads), 0, s,
                       static_cast<const double *>(fwd), pos, krow, kcol, b, kbase, nkb,
                       static_cast<double *>(dst));
  else
    hipLaunchKernelGGL(k_zunpack<float>, grid, dim3(kThreads), 0, s,
                       static_cast<const float *>(fwd), pos, krow, kcol, b, kbase, nkb,
                       static_cast<float *>(dst));
  return hipGetLastError();
}

}  // namespace vbcsr
