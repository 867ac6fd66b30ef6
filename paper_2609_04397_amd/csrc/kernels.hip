// gfx950 (CDNA4) kernels of the variable-block sparse library.
//
// Products run one 64-lane wave per panel (block row of A, or of A^T for the
// adjoint).  Panels are column-major b x K, so a run of consecutive panel
// values is a sequence of whole columns.  Two kernel families cover the
// forward product Y_i = sum_j A_ij X_j (paper, section 3.2):
//
//  * vector FMA (few right-hand sides): lane (g, p) owns panel row p of
//    column group g; with G = 64 / b groups, load step s reads the G*b
//    consecutive values [s*G*b, (s+1)*G*b) -- one contiguous wave access for
//    any block size -- and multiplies each by the X row of its column.
//    Partial sums of one panel row meet by a tree of cross-lane shuffles.
//  * matrix cores (many right-hand sides): the panel is the A operand of
//    16x16x4 FP64/FP32 MFMA (M = panel rows padded to 16 in registers only,
//    K = panel columns, N = 16 right-hand sides per tile); its 4-column slices
//    are again contiguous in memory.  The BF16x3 form uses 16x16x32 BF16 MFMA
//    on pages stored in 8-column groups (8 consecutive columns of one panel
//    row are 16 contiguous bytes, the per-lane A fragment).
//
// Every output element has exactly one writer (no atomics), so results are
// bitwise reproducible run to run.
#include <mutex>
#include <type_traits>

#include "kernels.hpp"

namespace vbcsr {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8u __attribute__((ext_vector_type(8)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
typedef unsigned int v2u32 __attribute__((ext_vector_type(2)));

// Index of the calling wave in its workgroup.  The shift is the same for all
// lanes of a wave, but the compiler cannot see that; reading it from the
// first lane puts it (and every row descriptor, address and buffer resource
// derived from it) in scalar registers.
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Give every XCD one contiguous range of logical workgroups so that
// panels that share input rows (spatial neighbours) share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int nx = 8;
  const int x = bid % nx, r = bid / nx;
  const int q = nblocks / nx, rem = nblocks % nx;
  return x * q + min(x, rem) + r;
}

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma_bf16(v8u a, v8u b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                 __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

template <typename T> struct Frag;
template <> struct Frag<double> { using type = v4d; };
template <> struct Frag<float> { using type = v4f; };

// Output row (within the 16x16 tile) of accumulator element i of the lanes
// in quarter-wave kq.  The FP32 and BF16 16x16 tiles give each quarter-wave
// four consecutive rows; the FP64 16x16x4 tile interleaves them with stride 4
// (lane layout measured on gfx950).
template <typename T> __device__ __forceinline__ int dst_row(int kq, int i);
template <> __device__ __forceinline__ int dst_row<double>(int kq, int i) { return kq + 4 * i; }
template <> __device__ __forceinline__ int dst_row<float>(int kq, int i) { return 4 * kq + i; }

// Round-to-nearest-even FP32 -> BF16 (finite inputs) and back.
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <bool MOM>
__device__ __forceinline__ void mom_init(double *s_mom, int nrhs) {
  if (MOM) {
    for (int c = threadIdx.x; c < kWaves * nrhs; c += kThreads) s_mom[c] = 0.0;
    __syncthreads();
  }
}

template <bool MOM>
__device__ __forceinline__ void mom_flush(const double *s_mom, int nrhs, int wg, double *out) {
  if (MOM) {
    __syncthreads();
    for (int c = threadIdx.x; c < nrhs; c += kThreads) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) t += s_mom[w * nrhs + c];
      out[(int64_t)wg * nrhs + c] = t;
    }
  }
}

// Wave-private LDS hand-off (LDS writes of a wave become visible to its
// own later LDS reads; no workgroup barrier needed).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Panel values are read exactly once per product: stream them past the
// caches (non-temporal) so the gathered X rows stay resident.
template <typename T>
__device__ __forceinline__ T stream_load(const T *p) {
  return __builtin_nontemporal_load(p);
}

// Raw buffer access to one panel: the descriptor (base, size in bytes) is
// wave-uniform and lives in scalar registers, each lane supplies a 32-bit
// byte offset, and offsets at or beyond the size read as zero.  Panel value
// streams use the non-temporal hint.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t panel_rsrc(const void *base, uint32_t bytes) {
  // 0x00020000: raw 32-bit buffer format of the gfx9 family
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           0x00020000);
}
template <typename T> __device__ __forceinline__ T buf_load_nt(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ double buf_load_nt<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 2));
}
template <> __device__ __forceinline__ float buf_load_nt<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 2));
}
template <typename T> __device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// 64 zeros, read in place of an X row where a lane has none (padding slices,
// columns past a staged chunk, right-hand sides past nrhs); any T of <= 8 bytes
__device__ __align__(16) double kZeroRow[64] = {};  // never written
template <typename T> __device__ __forceinline__ const T *zero_row() {
  return reinterpret_cast<const T *>(kZeroRow);
}

// Gather the X rows of panel columns [kc, kc + kn) into a wave-private LDS
// tile xs[col * NRP + c] (NRP >= nc values per row, zero-padded).  Each lane
// owns whole columns: the column indices of up to CPL columns per lane are
// loaded first, then every X load, then the LDS writes, so a chunk costs two
// memory round trips however many columns it holds.  The loads carry no
// branches: indices past the chunk read zero from the buffer and columns
// past the chunk (or right-hand sides past nc) read the row of zeros.
template <typename T, int NRP, int CPL>
__device__ __forceinline__ void stage_x(T *xs, const int32_t *__restrict__ cx, const T *__restrict__ X,
                                        int64_t ldx, int c0, int nc, int kc, int kn, int lane) {
  const __amdgpu_buffer_rsrc_t rc = panel_rsrc(cx + kc, (uint32_t)kn * 4);
  for (int k0 = 0; k0 < kn; k0 += 64 * CPL) {
    int32_t xr[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j)
      xr[j] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rc, (uint32_t)(k0 + j * 64 + lane) * 4, 0, 0);
    T v[CPL][NRP];
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int k = k0 + j * 64 + lane;
      const T *xp = k < kn ? X + (int64_t)xr[j] * ldx + c0 : zero_row<T>();
#pragma unroll
      for (int c = 0; c < NRP; ++c) v[j][c] = (c < nc ? xp : zero_row<T>())[c];
    }
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int k = k0 + j * 64 + lane;
      if (k < kn) {
#pragma unroll
        for (int c = 0; c < NRP; ++c) xs[k * NRP + c] = v[j][c];
      }
    }
  }
}

// Same tile from whole pieces of X rows, for full passes (nc = NRP) whose
// rows start on 16-byte boundaries: LPR lanes share a row and each loads up
// to 16 bytes of it, so one load instruction brings 64/LPR rows instead of
// one element of 64 rows.  A lane loads the indices of 64 columns, the
// others receive theirs through a lane permute, and CB blocks of 64 columns
// are in flight at a time.
template <int B> struct Bytes;
template <> struct Bytes<4> { using type = unsigned int; };
template <> struct Bytes<8> { using type = unsigned long long; };
template <> struct Bytes<16> { using type = v4u32; };

template <typename T, int NRP>
__device__ __forceinline__ void stage_x_rows(T *xs, const int32_t *__restrict__ cx,
                                             const T *__restrict__ X, int64_t ldx, int c0, int kc,
                                             int kn, int lane) {
  constexpr int RB = NRP * (int)sizeof(T);  // bytes of a staged row
  constexpr int LB = RB >= 16 ? 16 : RB;    // bytes per lane
  constexpr int LPR = RB / LB;              // lanes per row
  constexpr int RPI = 64 / LPR;             // rows per load instruction
  constexpr int EPL = LB / (int)sizeof(T);  // elements per lane
  constexpr int CB = LPR >= 4 ? 1 : 4 / LPR;
  using L = typename Bytes<LB>::type;
  const __amdgpu_buffer_rsrc_t rc = panel_rsrc(cx + kc, (uint32_t)kn * 4);
  const int sub = (lane % LPR) * EPL;
  for (int k0 = 0; k0 < kn; k0 += 64 * CB) {
    int32_t idx[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
      idx[cb] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rc, (uint32_t)(k0 + cb * 64 + lane) * 4, 0, 0);
    L v[CB][LPR];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int q = 0; q < LPR; ++q) {
        const int rl = q * RPI + lane / LPR;
        const int32_t r = __shfl(idx[cb], rl, 64);
        const int k = k0 + cb * 64 + rl;
        const T *xp = (k < kn ? X + (int64_t)r * ldx + c0 : zero_row<T>()) + sub;
        v[cb][q] = *reinterpret_cast<const L *>(xp);
      }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int q = 0; q < LPR; ++q) {
        const int k = k0 + cb * 64 + q * RPI + lane / LPR;
        if (k < kn) *reinterpret_cast<L *>(xs + k * NRP + sub) = v[cb][q];
      }
  }
}

// ---------------------------------------------------------------------------
// vector-FMA product, NR right-hand sides per pass
// ---------------------------------------------------------------------------
// The X rows of a chunk of panel columns are first gathered into a
// wave-private LDS buffer, so the value stream never waits on a dependent
// index -> X load chain.  The values of the next U steps are in flight while
// the current U steps are multiplied.
// Tuning of the two vector kernels, measured on the 32^3 lattice (b = 13),
// the zincblende particle and the three-species random operator: which pass
// widths use 16-byte value loads (the kernel after this one), the value
// loads in flight per lane (steps of look-ahead) and the LDS staging per
// wave in bytes.
template <typename T, int NR> constexpr bool use_vp() { return sizeof(T) == 8 ? NR <= 4 : NR == 1; }
template <typename T, int NR> constexpr int vec_depth() { return 8; }
template <typename T, int NR> constexpr int vec_xs_bytes() { return sizeof(T) == 8 && NR >= 4 ? 8192 : 4096; }
template <typename T, int NR> constexpr int vp_depth() { return sizeof(T) == 8 && NR >= 2 ? 8 : 4; }
template <typename T, int NR> constexpr int vp_xs_bytes() { return sizeof(T) == 8 && NR >= 2 ? 8192 : 4096; }

template <typename T, int NR, bool MOM>
__global__ void __launch_bounds__(kThreads) k_spmm_vec(FwdParams<T> P) {
  extern __shared__ double s_mom[];
  constexpr int XCAP = vec_xs_bytes<T, NR>() / sizeof(T);
  constexpr int U = vec_depth<T, NR>();
  __shared__ __align__(16) T xs_all[kWaves * XCAP];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const int row = wg * kWaves + w;
  T *xs = xs_all + w * XCAP;
  mom_init<MOM>(s_mom, P.nrhs);
  if (row < P.nrows) {
    const RowDesc rd = P.rows[row];
    const int b = rd.b, K = rd.K;
    // G column groups of b lanes; capped so that one staged chunk holds at
    // least G*U columns of NR values (otherwise ccap below would be 0 and the
    // chunk loop would not advance: b = 1 gives 64 groups)
    constexpr int GMAX = XCAP / (NR * U);
    static_assert(GMAX >= 1, "LDS staging buffer too small");
    const int G = min(64 / b, GMAX);
    const int g = lane / b;
    const int p = lane - g * b;
    const int GB = G * b;
    // panel columns per staged chunk: a positive multiple of G*U that fits
    const int ccap = (XCAP / NR) / (G * U) * (G * U);
    const int32_t *__restrict__ cxrow = P.colx + rd.cbase;
    for (int c0 = 0; c0 < P.nrhs; c0 += NR) {
      const int nc = min(NR, P.nrhs - c0);
      T acc[NR];
#pragma unroll
      for (int c = 0; c < NR; ++c) acc[c] = T(0);
      for (int kc = 0; kc < K; kc += ccap) {
        const int kn = min(ccap, K - kc);
        // steps over the chunk, rounded up to whole groups of U; values past
        // the chunk read as zero and meet zero-padded staged X rows
        const int ngrp = (kn + G * U - 1) / (G * U);
        const __amdgpu_buffer_rsrc_t vr =
            panel_rsrc(P.vals + rd.vbase + (int64_t)kc * b, (uint32_t)(kn * b * sizeof(T)));
        const uint32_t lo = (uint32_t)lane * sizeof(T);
        const uint32_t stepb = (uint32_t)GB * sizeof(T);
        T a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = buf_load_nt<T>(vr, lo + u * stepb);
        wave_lds_sync();  // previous chunk fully consumed
        if (NR > 1 && nc == NR && P.xrow16)
          stage_x_rows<T, NR>(xs, cxrow, P.X, P.ldx, c0, kc, kn, lane);
        else
          stage_x<T, NR, (NR <= 2 ? 4 : 2)>(xs, cxrow, P.X, P.ldx, c0, nc, kc, kn, lane);
        for (int e = kn * NR + lane; e < ngrp * G * U * NR; e += 64) xs[e] = T(0);
        wave_lds_sync();
        if (g < G) {
          for (int q = 0; q < ngrp; ++q) {
            const int s = q * U;
            T an[U];
#pragma unroll
            for (int u = 0; u < U; ++u) an[u] = buf_load_nt<T>(vr, lo + (s + U + u) * stepb);
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const T *xp = xs + ((s + u) * G + g) * NR;
#pragma unroll
              for (int c = 0; c < NR; ++c) acc[c] = fma(a[u], xp[c], acc[c]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] = an[u];
          }
        }
      }
      // groups g and g + st hold partial sums of the same panel row
      for (int st = 1; st < G; st <<= 1) {
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          const T o = __shfl_down(acc[c], st * b, 64);
          if ((g & (2 * st - 1)) == 0 && g + st < G) acc[c] += o;
        }
      }
      double mom[NR];
#pragma unroll
      for (int c = 0; c < NR; ++c) mom[c] = 0.0;
      if (lane < b) {
        const int64_t r = (int64_t)rd.yrow + p;
        T *yo = P.Yout + r * P.ldy + c0;
        const T *yi = P.Yin + r * P.ldyin + c0;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          if (c < nc) {
            T y = T(P.alpha) * acc[c];
            if (P.beta != 0.0) y = fma(T(P.beta), yi[c], y);
            yo[c] = y;
            if (MOM) mom[c] = (double)P.R[r * P.ldr + c0 + c] * (double)y;
          }
        }
      }
      if (MOM) {
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          const double t = wave_sum(mom[c]);
          if (lane == 0 && c < nc) s_mom[w * P.nrhs + c0 + c] += t;
        }
      }
    }
  }
  mom_flush<MOM>(s_mom, P.nrhs, wg, P.mom);
}

// ---------------------------------------------------------------------------
// vector-FMA product with 16-byte value loads
// ---------------------------------------------------------------------------
// A step covers C panel columns (C*b values, contiguous in the column-major
// panel); lane l loads the E = 16/sizeof(T) consecutive values E*l .. E*l+E-1
// of the step with one 16-byte load.  C is the largest multiple of E with
// C*b <= 64*E, so the step length is a multiple of b and every lane keeps
// the same E panel rows in every step; lanes l and l + b hold the same rows.
// X rows are staged in LDS as in the kernel above.
template <typename T, int NR, bool MOM>
__global__ void __launch_bounds__(kThreads) k_spmm_vp(FwdParams<T> P) {
  extern __shared__ double s_mom[];
  constexpr int E = 16 / (int)sizeof(T);
  constexpr int XCAP = vp_xs_bytes<T, NR>() / sizeof(T);
  constexpr int U = vp_depth<T, NR>();
  __shared__ __align__(16) T xs_all[kWaves * XCAP];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const int row = wg * kWaves + w;
  T *xs = xs_all + w * XCAP;
  mom_init<MOM>(s_mom, P.nrhs);
  if (row < P.nrows) {
    const RowDesc rd = P.rows[row];
    const int b = rd.b, K = rd.K;
    // columns per step (a multiple of E), capped so a staged chunk holds U steps
    constexpr int CMAX = XCAP / (NR * U) / E * E;
    static_assert(CMAX >= E, "LDS staging buffer too small");
    const int C = min((64 * E / b) / E * E, CMAX);
    const int NL = C * b / E;  // active lanes
    int cj[E], rj[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = E * lane + j;
      cj[j] = e / b;
      rj[j] = e - cj[j] * b;
    }
    const int ccap = (XCAP / NR) / (C * U) * (C * U);
    const int32_t *__restrict__ cxrow = P.colx + rd.cbase;
    for (int c0 = 0; c0 < P.nrhs; c0 += NR) {
      const int nc = min(NR, P.nrhs - c0);
      T acc[E][NR];
#pragma unroll
      for (int j = 0; j < E; ++j)
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[j][c] = T(0);
      for (int kc = 0; kc < K; kc += ccap) {
        const int kn = min(ccap, K - kc);
        const int ngrp = (kn + C * U - 1) / (C * U);
        // the chunk's values rounded up to whole 16-byte loads: the pages
        // pad every panel with zeros to a multiple of 4 values
        const __amdgpu_buffer_rsrc_t vr = panel_rsrc(P.vals + rd.vbase + (int64_t)kc * b,
                                                     (uint32_t)((kn * b + E - 1) / E * E * sizeof(T)));
        const uint32_t lo = (uint32_t)lane * 16;
        const uint32_t stepb = (uint32_t)(C * b) * sizeof(T);
        v4u32 a[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
          a[u] = __builtin_bit_cast(v4u32, __builtin_amdgcn_raw_buffer_load_b128(vr, lo + u * stepb, 0, 2));
        wave_lds_sync();
        if (NR > 1 && nc == NR && P.xrow16)
          stage_x_rows<T, NR>(xs, cxrow, P.X, P.ldx, c0, kc, kn, lane);
        else
          stage_x<T, NR, (NR <= 2 ? 4 : 2)>(xs, cxrow, P.X, P.ldx, c0, nc, kc, kn, lane);
        for (int e = kn * NR + lane; e < ngrp * C * U * NR; e += 64) xs[e] = T(0);
        wave_lds_sync();
        if (lane < NL) {
          for (int q = 0; q < ngrp; ++q) {
            const int s = q * U;
            v4u32 an[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
              an[u] = __builtin_bit_cast(
                  v4u32, __builtin_amdgcn_raw_buffer_load_b128(vr, lo + (s + U + u) * stepb, 0, 2));
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const T *av = reinterpret_cast<const T *>(&a[u]);
#pragma unroll
              for (int j = 0; j < E; ++j) {
                const T *xp = xs + ((s + u) * C + cj[j]) * NR;
#pragma unroll
                for (int c = 0; c < NR; ++c) acc[j][c] = fma(av[j], xp[c], acc[j][c]);
              }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] = an[u];
          }
        }
      }
      // lanes l and l + b hold the same rows: tree over the C/E groups
      const int ng = C / E;
      const int g = lane / b;
      for (int st = 1; st < ng; st <<= 1) {
#pragma unroll
        for (int j = 0; j < E; ++j)
#pragma unroll
          for (int c = 0; c < NR; ++c) {
            const T o = __shfl_down(acc[j][c], st * b, 64);
            if ((g & (2 * st - 1)) == 0 && g + st < ng) acc[j][c] += o;
          }
      }
      // lanes < b now hold values E*l + j of the first E*b; row p collects
      // values p + t*b, t < E (lane (p + t*b) / E, slot (p + t*b) % E)
      T ysum[NR];
#pragma unroll
      for (int c = 0; c < NR; ++c) ysum[c] = T(0);
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const int e = (lane < b ? lane : 0) + t * b;
        const int sl = e / E, sj = e - sl * E;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          T v = T(0);
#pragma unroll
          for (int j = 0; j < E; ++j) {
            const T o = __shfl(acc[j][c], sl, 64);
            v = sj == j ? o : v;
          }
          ysum[c] += v;
        }
      }
      double mom[NR];
#pragma unroll
      for (int c = 0; c < NR; ++c) mom[c] = 0.0;
      if (lane < b) {
        const int64_t r = (int64_t)rd.yrow + lane;
        T *yo = P.Yout + r * P.ldy + c0;
        const T *yi = P.Yin + r * P.ldyin + c0;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          if (c < nc) {
            T y = T(P.alpha) * ysum[c];
            if (P.beta != 0.0) y = fma(T(P.beta), yi[c], y);
            yo[c] = y;
            if (MOM) mom[c] = (double)P.R[r * P.ldr + c0 + c] * (double)y;
          }
        }
      }
      if (MOM) {
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          const double t = wave_sum(mom[c]);
          if (lane == 0 && c < nc) s_mom[w * P.nrhs + c0 + c] += t;
        }
      }
    }
  }
  mom_flush<MOM>(s_mom, P.nrhs, wg, P.mom);
}

// ---------------------------------------------------------------------------
// FP64 / FP32 matrix-core product
// ---------------------------------------------------------------------------
// A operand: the panel's 4-column slice (contiguous, 4*b values, panel row m
// in lane m, slice column kq in lane group kq); B operand: the X rows of
// those 4 columns.  Slices are taken in groups of U.  Two register sets
// alternate: while one group multiplies, the values and X rows of the next
// group and the column indices of the one after are in flight.  The loop
// has no data-dependent branch (a branch around a load makes the compiler
// wait for every load in flight): values and indices are buffer loads that
// read zero past the panel, and padding slices point at a row of zeros
// instead of a row of X.  Scheduling barriers keep each group's loads ahead
// of the previous group's matrix instructions.
//
// Fast path (VX = true): the N index of the 16x16 tiles is permuted so that
// lane m of tile t holds right-hand side c0 + l*16*VEC + VEC*m + e, with
// t = l*VEC + e and VEC elements per 16 bytes: one 16-byte load per lane and
// X row fetches VEC tiles, and outputs are written back 16 bytes at a time.
// It needs 16-byte aligned vectors, leading dimensions that are multiples of
// VEC and nrhs a multiple of 16*VEC*L.  The generic path (VX = false) loads
// one element per lane and tile and handles any nrhs and leading dimension.
template <typename T> struct Vec16;
template <> struct Vec16<double> { using type = double2; static constexpr int n = 2; };
template <> struct Vec16<float> { using type = float4; static constexpr int n = 4; };

template <typename T, int NT, bool MOM, bool VX, bool XB>
__global__ void __launch_bounds__(kThreads) k_spmm_mfma(FwdParams<T> P) {
  extern __shared__ double s_mom[];
  using V = typename Frag<T>::type;
  using L16 = typename Vec16<T>::type;
  constexpr int VEC = Vec16<T>::n;
  constexpr int NL = VX ? NT / VEC : 0;  // 16-byte loads per lane and X row
  constexpr int U = NT * sizeof(T) >= 32 ? 2 : 4;  // slices per group
  static_assert(!VX || NT % VEC == 0, "tile count must fill whole 16-byte loads");
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const int row = wg * kWaves + w;
  const int m = lane & 15;   // A: panel row in the tile; B and D: column in the tile
  const int kq = lane >> 4;  // A and B: column of the 4-column slice; D: row group
  mom_init<MOM>(s_mom, P.nrhs);
  if (row < P.nrows) {
    const RowDesc rd = P.rows[row];
    const int b = rd.b, K = rd.K;
    const int nsteps = (K + 3) >> 2;
    const T *__restrict__ vals = P.vals + rd.vbase;
    const int32_t *__restrict__ cx = P.colx + rd.cbase;
    // column of (tile t, lane m) relative to c0
    auto col = [&](int t) {
      return VX ? (t / VEC) * 16 * VEC + VEC * m + (t % VEC) : t * 16 + m;
    };
    for (int mt = 0; mt * 16 < b; ++mt) {
      const int p = mt * 16 + m;
      const bool prow = p < b;
      for (int c0 = 0; c0 < P.nrhs; c0 += 16 * NT) {
        V acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = V{};
        // panel sizes are below 2^31 bytes (checked at creation), so kOut is
        // past the end of every panel and reads zero
        constexpr uint32_t kOut = 0x80000000u;
        const __amdgpu_buffer_rsrc_t rv = panel_rsrc(vals, (uint32_t)((int64_t)K * b * sizeof(T)));
        const __amdgpu_buffer_rsrc_t rc = panel_rsrc(cx, (uint32_t)(K * 4));
        const uint32_t vlane = prow ? (uint32_t)(kq * b + p) * sizeof(T) : kOut;
        // XB: all of X lies within 2^31 bytes and is read through one buffer
        // descriptor (cheaper addressing); otherwise through 64-bit pointers
        const __amdgpu_buffer_rsrc_t rx =
            panel_rsrc(P.X, XB ? (uint32_t)(P.xrows * P.ldx * (int64_t)sizeof(T)) : 0u);
        const uint32_t xcol = (uint32_t)(c0 + (VX ? VEC * m : m)) * sizeof(T);
        auto ld_idx = [&](int g, int32_t(&xi)[U]) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int k = (g * U + u) * 4 + kq;
            const int32_t v = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rc, (uint32_t)k * 4, 0, 0);
            xi[u] = k < K ? v : -1;
          }
        };
        auto ld_val = [&](int g, T(&av)[U]) {
#pragma unroll
          for (int u = 0; u < U; ++u)
            av[u] = buf_load_nt<T>(rv, vlane + (uint32_t)((g * U + u) * 4 * b) * sizeof(T));
        };
        auto ld_x = [&](const int32_t(&xi)[U], T(&xv)[U][NT]) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if constexpr (XB) {
              // padding slices read past the descriptor: zeros
              const uint32_t ro =
                  xi[u] >= 0 ? (uint32_t)((int64_t)xi[u] * P.ldx * (int64_t)sizeof(T)) + xcol : kOut;
              if constexpr (VX) {
#pragma unroll
                for (int l = 0; l < (VX ? NL : 1); ++l) {
                  const L16 q = __builtin_bit_cast(
                      L16, __builtin_amdgcn_raw_buffer_load_b128(rx, ro + l * 16 * VEC * sizeof(T), 0, 0));
                  const T *qe = reinterpret_cast<const T *>(&q);
#pragma unroll
                  for (int e = 0; e < VEC; ++e) xv[u][l * VEC + e] = qe[e];
                }
              } else {
#pragma unroll
                for (int t = 0; t < NT; ++t)
                  xv[u][t] = buf_load<T>(rx, c0 + t * 16 + m < P.nrhs ? ro + t * 16 * sizeof(T) : kOut);
              }
            } else {
              // padding slices read a row of zeros instead of a row of X
              const T *xp = xi[u] >= 0 ? P.X + (int64_t)xi[u] * P.ldx + c0 : zero_row<T>();
              if constexpr (VX) {
#pragma unroll
                for (int l = 0; l < (VX ? NL : 1); ++l) {
                  const L16 q = *reinterpret_cast<const L16 *>(xp + l * 16 * VEC + VEC * m);
                  const T *qe = reinterpret_cast<const T *>(&q);
#pragma unroll
                  for (int e = 0; e < VEC; ++e) xv[u][l * VEC + e] = qe[e];
                }
              } else {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                  const int n = t * 16 + m;
                  xv[u][t] = (c0 + n < P.nrhs ? xp : zero_row<T>())[n];
                }
              }
            }
          }
        };
        auto mma = [&](const T(&av)[U], const T(&xv)[U][NT]) {
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = mfma(av[u], xv[u][t], acc[t]);
        };
        const int ngroups = (nsteps + U - 1) / U;
        T aA[U], aB[U], vA[U][NT], vB[U][NT];
        int32_t iA[U], iB[U];
        ld_idx(0, iA);
        ld_idx(1, iB);
        ld_x(iA, vA);
        ld_val(0, aA);
        for (int g = 0; g < ngroups; g += 2) {
          ld_idx(g + 2, iA);
          ld_x(iB, vB);
          ld_val(g + 1, aB);
          __builtin_amdgcn_sched_barrier(0);
          mma(aA, vA);
          __builtin_amdgcn_sched_barrier(0);
          if (g + 1 >= ngroups) break;
          ld_idx(g + 3, iB);
          ld_x(iA, vA);
          ld_val(g + 2, aA);
          __builtin_amdgcn_sched_barrier(0);
          mma(aB, vB);
          __builtin_amdgcn_sched_barrier(0);
        }
        // epilogue: row pr of the tile, columns col(t)
        double mmv[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) mmv[t] = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pr = mt * 16 + dst_row<T>(kq, i);
          if (pr < b) {
            const int64_t r = (int64_t)rd.yrow + pr;
            T y[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) y[t] = T(P.alpha) * acc[t][i];
            if constexpr (VX) {
#pragma unroll
              for (int l = 0; l < (VX ? NL : 1); ++l) {
                const int64_t cc = c0 + l * 16 * VEC + VEC * m;
                if (P.beta != 0.0) {
                  const L16 q = *reinterpret_cast<const L16 *>(P.Yin + r * P.ldyin + cc);
                  const T *qe = reinterpret_cast<const T *>(&q);
#pragma unroll
                  for (int e = 0; e < VEC; ++e) y[l * VEC + e] = fma(T(P.beta), qe[e], y[l * VEC + e]);
                }
                L16 o;
                T *oe = reinterpret_cast<T *>(&o);
#pragma unroll
                for (int e = 0; e < VEC; ++e) oe[e] = y[l * VEC + e];
                *reinterpret_cast<L16 *>(P.Yout + r * P.ldy + cc) = o;
                if (MOM) {
                  const L16 q = *reinterpret_cast<const L16 *>(P.R + r * P.ldr + cc);
                  const T *qe = reinterpret_cast<const T *>(&q);
#pragma unroll
                  for (int e = 0; e < VEC; ++e) mmv[l * VEC + e] += (double)qe[e] * (double)oe[e];
                }
              }
            } else {
#pragma unroll
              for (int t = 0; t < NT; ++t) {
                const int n = c0 + t * 16 + m;
                if (n < P.nrhs) {
                  if (P.beta != 0.0) y[t] = fma(T(P.beta), P.Yin[r * P.ldyin + n], y[t]);
                  P.Yout[r * P.ldy + n] = y[t];
                  if (MOM) mmv[t] += (double)P.R[r * P.ldr + n] * (double)y[t];
                }
              }
            }
          }
        }
        if (MOM) {
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            double mm = mmv[t];
            mm += __shfl_xor(mm, 16, 64);
            mm += __shfl_xor(mm, 32, 64);
            const int n = c0 + col(t);
            if (kq == 0 && n < P.nrhs) s_mom[w * P.nrhs + n] += mm;
          }
        }
      }
    }
  }
  mom_flush<MOM>(s_mom, P.nrhs, wg, P.mom);
}

// ---------------------------------------------------------------------------
// BF16x3 matrix-core product: a*x ~ ah*xh + ah*xl + al*xh, FP32 accumulation
// ---------------------------------------------------------------------------
// 32-column slices; lane (m, kg) owns 8 consecutive panel columns of row m
// (one 16-byte load per page) and, for the B operand, the same 8 columns of
// X in column m of the tile.  X is split into bf16 hi/lo on the fly.  Loads
// are branch-free and the next slice's values and indices are in flight
// while the current slice multiplies.
template <int NT, bool MOM>
__global__ void __launch_bounds__(kThreads) k_spmm_bf16x3(FwdParams<float> P) {
  extern __shared__ double s_mom[];
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const int row = wg * kWaves + w;
  const int m = lane & 15;
  const int kg = lane >> 4;  // 8-column group of the 32-column slice
  mom_init<MOM>(s_mom, P.nrhs);
  if (row < P.nrows) {
    const RowDesc rd = P.rows[row];
    const int b = rd.b, K = rd.K;
    const int ngroups = (K + 7) >> 3;
    const int nsteps = (K + 31) >> 5;
    const int64_t vb16 = P.vbase16[row];
    const int32_t *__restrict__ cx = P.colx + rd.cbase;
    for (int mt = 0; mt * 16 < b; ++mt) {
      const int p = mt * 16 + m;
      const bool prow = p < b;
      const int pc = prow ? p : b - 1;
      for (int c0 = 0; c0 < P.nrhs; c0 += 16 * NT) {
        int nn[NT];
        bool nok[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int n = c0 + t * 16 + m;
          nok[t] = n < P.nrhs;
          nn[t] = nok[t] ? n : P.nrhs - 1;
        }
        v4f acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = v4f{};
        auto fetch = [&](int s, v8u &h, v8u &l, int32_t *x) {
          const int grp = s * 4 + kg;
          const bool ok = prow && grp < ngroups;
          const int64_t a = vb16 + (int64_t)min(grp, max(ngroups - 1, 0)) * 8 * b + pc * 8;
          const v8u hv = stream_load(reinterpret_cast<const v8u *>(P.hi + a));
          const v8u lv = stream_load(reinterpret_cast<const v8u *>(P.lo + a));
          h = ok ? hv : v8u{};
          l = ok ? lv : v8u{};
#pragma unroll
          for (int u = 0; u < 8; ++u) x[u] = cx[min(grp * 8 + u, K - 1)];
        };
        v8u ah, al;
        int32_t xr[8];
        if (K > 0) fetch(0, ah, al, xr);
        for (int s = 0; s < nsteps; ++s) {
          float xv[NT][8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const bool kin = (s * 4 + kg) * 8 + u < K;
            const float *xp = P.X + (int64_t)xr[u] * P.ldx;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              const float v = xp[nn[t]];
              xv[t][u] = (kin && nok[t]) ? v : 0.0f;
            }
          }
          v8u nh, nl;
          int32_t xn[8];
          fetch(min(s + 1, nsteps - 1), nh, nl, xn);
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            v8u xh, xl;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const unsigned short h = bf16_rne(xv[t][u]);
              xh[u] = h;
              xl[u] = bf16_rne(xv[t][u] - bf16_to_f32(h));
            }
            acc[t] = mfma_bf16(ah, xh, acc[t]);
            acc[t] = mfma_bf16(ah, xl, acc[t]);
            acc[t] = mfma_bf16(al, xh, acc[t]);
          }
          ah = nh;
          al = nl;
#pragma unroll
          for (int u = 0; u < 8; ++u) xr[u] = xn[u];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int n = c0 + t * 16 + m;
          double mm = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int pr = mt * 16 + dst_row<float>(kg, i);
            if (pr < b && n < P.nrhs) {
              const int64_t r = (int64_t)rd.yrow + pr;
              float y = float(P.alpha) * acc[t][i];
              if (P.beta != 0.0) y = fmaf(float(P.beta), P.Yin[r * P.ldyin + n], y);
              P.Yout[r * P.ldy + n] = y;
              if (MOM) mm += (double)P.R[r * P.ldr + n] * (double)y;
            }
          }
          if (MOM) {
            mm += __shfl_xor(mm, 16, 64);
            mm += __shfl_xor(mm, 32, 64);
            if (kg == 0 && n < P.nrhs) s_mom[w * P.nrhs + n] += mm;
          }
        }
      }
    }
  }
  mom_flush<MOM>(s_mom, P.nrhs, wg, P.mom);
}

// BF16x3 fast path: 64 right-hand sides per pass, tile t of lane m holds
// column c0 + 4m + t, so the 8 X rows of a lane's 8-column group arrive as
// eight 16-byte loads; each row splits into hi/lo with the hardware
// round-to-nearest-even conversion (two values per instruction).  The loop
// is branch-free and double-buffered like the FP64/FP32 matrix-core kernel.
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned int pack_bf16(float a, float b) {
  return __builtin_bit_cast(unsigned int, v2bf{(__bf16)a, (__bf16)b});
}

template <bool MOM, bool XB>
__global__ void __launch_bounds__(kThreads) k_spmm_bf16x3_vx(FwdParams<float> P) {
  extern __shared__ double s_mom[];
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int w = wave_id();
  const int lane = threadIdx.x & 63;
  const int row = wg * kWaves + w;
  const int m = lane & 15;
  const int kg = lane >> 4;
  mom_init<MOM>(s_mom, P.nrhs);
  if (row < P.nrows) {
    const RowDesc rd = P.rows[row];
    const int b = rd.b, K = rd.K;
    const int ngroups = (K + 7) >> 3;
    const int nsteps = (K + 31) >> 5;
    const int64_t vb16 = P.vbase16[row];
    constexpr uint32_t kOut = 0x80000000u;
    // the row's BF16 pages, its column table and (XB) all of X, each read
    // through one buffer descriptor; offsets past the end read zero
    const uint32_t pbytes = (uint32_t)((int64_t)ngroups * 8 * b * sizeof(uint16_t));
    const __amdgpu_buffer_rsrc_t rh = panel_rsrc(P.hi + vb16, pbytes);
    const __amdgpu_buffer_rsrc_t rl = panel_rsrc(P.lo + vb16, pbytes);
    const __amdgpu_buffer_rsrc_t rc = panel_rsrc(P.colx + rd.cbase, (uint32_t)(K * 4));
    const __amdgpu_buffer_rsrc_t rx =
        panel_rsrc(P.X, XB ? (uint32_t)(P.xrows * P.ldx * (int64_t)sizeof(float)) : 0u);
    for (int mt = 0; mt * 16 < b; ++mt) {
      const int p = mt * 16 + m;
      const bool prow = p < b;
      const uint32_t vlane = prow ? (uint32_t)(kg * 8 * b + p * 8) * sizeof(uint16_t) : kOut;
      for (int c0 = 0; c0 < P.nrhs; c0 += 64) {
        v4f acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = v4f{};
        const uint32_t xcol = (uint32_t)(c0 + 4 * m) * sizeof(float);
        // step s covers panel columns [32 s, 32 s + 32); lane group kg holds
        // the 8 columns 32 s + 8 kg + u.  Two register sets alternate as in
        // the FP64/FP32 kernel: indices run two steps ahead, values and X
        // rows one step ahead.
        auto ld_idx = [&](int s, int32_t(&xi)[8]) {
          // the 8 column indices of the lane's group: two 16-byte loads
          // (past the panel's table the buffer reads zero; masked by k < K)
          const int k0 = (s * 4 + kg) * 8;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const v4u32 q = __builtin_bit_cast(
                v4u32, __builtin_amdgcn_raw_buffer_load_b128(rc, (uint32_t)(k0 + 4 * h) * 4, 0, 0));
#pragma unroll
            for (int u = 0; u < 4; ++u) xi[4 * h + u] = k0 + 4 * h + u < K ? (int32_t)q[u] : -1;
          }
        };
        auto ld_val = [&](int s, v8u &h, v8u &l) {
          const uint32_t off = vlane + (uint32_t)(s * 32 * b) * sizeof(uint16_t);
          h = __builtin_bit_cast(v8u, __builtin_amdgcn_raw_buffer_load_b128(rh, off, 0, 2));
          l = __builtin_bit_cast(v8u, __builtin_amdgcn_raw_buffer_load_b128(rl, off, 0, 2));
        };
        auto ld_x = [&](const int32_t(&xi)[8], float4(&xv)[8]) {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if constexpr (XB) {
              const uint32_t ro =
                  xi[u] >= 0 ? (uint32_t)((int64_t)xi[u] * P.ldx * (int64_t)sizeof(float)) + xcol : kOut;
              xv[u] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rx, ro, 0, 0));
            } else {
              const float *xp = xi[u] >= 0 ? P.X + (int64_t)xi[u] * P.ldx + c0 : zero_row<float>();
              xv[u] = *reinterpret_cast<const float4 *>(xp + 4 * m);
            }
          }
        };
        auto mma = [&](const v8u &ah, const v8u &al, const float4(&xv)[8]) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            v4u hi, lo;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float x0 = reinterpret_cast<const float *>(&xv[2 * q])[t];
              const float x1 = reinterpret_cast<const float *>(&xv[2 * q + 1])[t];
              const unsigned int h = pack_bf16(x0, x1);
              hi[q] = h;
              lo[q] = pack_bf16(x0 - __uint_as_float(h << 16), x1 - __uint_as_float(h & 0xFFFF0000u));
            }
            const v8u xh = __builtin_bit_cast(v8u, hi), xl = __builtin_bit_cast(v8u, lo);
            acc[t] = mfma_bf16(ah, xh, acc[t]);
            acc[t] = mfma_bf16(ah, xl, acc[t]);
            acc[t] = mfma_bf16(al, xh, acc[t]);
          }
        };
        v8u hA, lA, hB, lB;
        float4 xA[8], xB[8];
        int32_t iA[8], iB[8];
        ld_idx(0, iA);
        ld_idx(1, iB);
        ld_x(iA, xA);
        ld_val(0, hA, lA);
        for (int s = 0; s < nsteps; s += 2) {
          ld_idx(s + 2, iA);
          ld_x(iB, xB);
          ld_val(s + 1, hB, lB);
          __builtin_amdgcn_sched_barrier(0);
          mma(hA, lA, xA);
          __builtin_amdgcn_sched_barrier(0);
          if (s + 1 >= nsteps) break;
          ld_idx(s + 3, iB);
          ld_x(iA, xA);
          ld_val(s + 2, hA, lA);
          __builtin_amdgcn_sched_barrier(0);
          mma(hB, lB, xB);
          __builtin_amdgcn_sched_barrier(0);
        }
        double mmv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pr = mt * 16 + dst_row<float>(kg, i);
          if (pr < b) {
            const int64_t r = (int64_t)rd.yrow + pr;
            const int64_t cc = c0 + 4 * m;
            float4 y = {float(P.alpha) * acc[0][i], float(P.alpha) * acc[1][i],
                        float(P.alpha) * acc[2][i], float(P.alpha) * acc[3][i]};
            if (P.beta != 0.0) {
              const float4 q = *reinterpret_cast<const float4 *>(P.Yin + r * P.ldyin + cc);
              const float be = float(P.beta);
              y.x = fmaf(be, q.x, y.x);
              y.y = fmaf(be, q.y, y.y);
              y.z = fmaf(be, q.z, y.z);
              y.w = fmaf(be, q.w, y.w);
            }
            *reinterpret_cast<float4 *>(P.Yout + r * P.ldy + cc) = y;
            if (MOM) {
              const float4 q = *reinterpret_cast<const float4 *>(P.R + r * P.ldr + cc);
              mmv[0] += (double)q.x * (double)y.x;
              mmv[1] += (double)q.y * (double)y.y;
              mmv[2] += (double)q.z * (double)y.z;
              mmv[3] += (double)q.w * (double)y.w;
            }
          }
        }
        if (MOM) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            double mm = mmv[t];
            mm += __shfl_xor(mm, 16, 64);
            mm += __shfl_xor(mm, 32, 64);
            if (kg == 0) s_mom[w * P.nrhs + c0 + 4 * m + t] += mm;
          }
        }
      }
    }
  }
  mom_flush<MOM>(s_mom, P.nrhs, wg, P.mom);
}

// ---------------------------------------------------------------------------
// value packing: graph order (row-major blocks) -> pages
// ---------------------------------------------------------------------------
// One wave per run of kPackRun consecutive graph blocks (their values are
// contiguous in graph order): lane l takes elements l, l + 64, ... of the
// run, so every lane is busy whatever the block sizes and the loads of
// different elements are independent (the loop is unrolled four times to keep
// four in flight per lane).  A lane finds its block by comparing the element
// with the run's block starts (wave-uniform, in scalar registers) and reads
// the block's map from a wave-private LDS table.  For the FP64/FP32 pages one
// sweep in row-major order (the order of the source) writes the transposed
// pages as a contiguous copy and the forward pages (each block transposed)
// inside each block's own contiguous range.  BF16 pages (8-column groups)
// take one sweep per direction, each in the order in which its writes are
// contiguous.  Row and column of an element come from a reciprocal of the
// block width, corrected by one step (exact for offsets below 2^12 and
// widths up to 64).
constexpr int kPackRun = 8;
constexpr int kPackChunk = 4;

// Output map of panel column kk for the block-sampled product written in the
// forward pages' layout: column kk of the panel starts at vbase + kk * b and
// its rows are consecutive (stride 1).
__device__ __forceinline__ int64_t page_map(const RowDesc &rd, int kk) {
  return ((rd.vbase + (int64_t)kk * rd.b) << 7) | 1;
}

__device__ __forceinline__ void pack_store(const PackDir &D, int kind, int64_t pos, int k0,
                                           int64_t vb16, int h, int r, int c, double v) {
  if (kind == 2) {
    const int col = k0 + c;
    const int64_t a = vb16 + (int64_t)(col >> 3) * 8 * h + r * 8 + (col & 7);
    const float f = (float)v;
    const unsigned short hb = bf16_rne(f);
    static_cast<uint16_t *>(D.dst)[a] = hb;
    D.dst_lo[a] = bf16_rne(f - bf16_to_f32(hb));
  } else {
    const int64_t a = pos + (int64_t)c * h + r;
    if (kind == 0)
      static_cast<double *>(D.dst)[a] = v;
    else
      static_cast<float *>(D.dst)[a] = (float)v;
  }
}

struct PackRec {       // one block of a run, in LDS
  int32_t start;       // run-relative first value (graph order)
  int32_t bi, bj;
  int32_t kf, kt;      // BF16: first panel column, forward / transposed
  int32_t pad[3];
  int64_t pf, pt;      // page offset, forward / transposed
  int64_t vf, vt;      // BF16: panel base in the BF16 pages, forward / transposed
};
static_assert(sizeof(PackRec) == 64, "PackRec layout");

template <int SRC, int KIND>  // SRC 0/1: double/float source; KIND: dst_kind
__global__ void __launch_bounds__(kThreads) k_pack(PackParams P, const void *src) {
  __shared__ PackRec tab_all[kWaves * kPackRun];
  const int64_t k0 = ((int64_t)blockIdx.x * kWaves + wave_id()) * kPackRun;
  if (k0 >= P.nnzb) return;
  const int lane = threadIdx.x & 63;
  const int nb = (int)min((int64_t)kPackRun, P.nnzb - k0);
  PackRec *tab = tab_all + wave_id() * kPackRun;
  // lanes 0 .. nb-1 read one block's map each into the table
  int64_t g = 0;
  int n = 0;
  PackRec r{};
  if (lane < nb) {
    const int64_t k = k0 + lane;
    r.bi = P.b[P.blk_row[k]];
    r.bj = P.b[P.col_idx[k]];
    g = P.gbase[k];
    r.pf = P.dir[0].pos[k];
    r.pt = P.dir[1].pos[k];
    if (KIND == 2) {
      r.kf = P.dir[0].k0[k];
      r.kt = P.dir[1].k0[k];
      r.vf = P.dir[0].vbase16[P.dir[0].prow[k]];
      r.vt = P.dir[1].vbase16[P.dir[1].prow[k]];
    }
    n = r.bi * r.bj;
  }
  const int64_t g0 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(g >> 32), 0) << 32) |
                               (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)g, 0));
  const int start = (int)(g - g0);   // run-relative first value (lanes < nb)
  if (lane < nb) {
    r.start = start;
    tab[lane] = r;
  }
  wave_lds_sync();
  int st[kPackRun];   // block starts (wave-uniform; past nb: beyond the run)
  const int len = __builtin_amdgcn_readlane(start + n, nb - 1);
#pragma unroll
  for (int u = 0; u < kPackRun; ++u) st[u] = u < nb ? __builtin_amdgcn_readlane(start, u) : len;
  auto load = [&](int64_t at) {
    if constexpr (SRC == 0)
      return static_cast<const double *>(src)[at];
    else
      return (double)static_cast<const float *>(src)[at];
  };
  // sweep 0 in row-major order, sweep 1 (BF16 only) in column-major order.
  // Elements go in chunks of kPackChunk per lane: every load of a chunk is
  // issued before its first store, so a lane waits once per chunk (a lane
  // has only a few elements when blocks are small).
  for (int sweep = 0; sweep < (KIND == 2 ? 2 : 1); ++sweep) {
    for (int e0 = lane; e0 < len; e0 += 64 * kPackChunk) {
      double v[kPackChunk];
      int tt[kPackChunk], pp[kPackChunk], qq[kPackChunk];
#pragma unroll
      for (int c = 0; c < kPackChunk; ++c) {
        const int e = e0 + 64 * c;
        const int ec = e < len ? e : len - 1;
        int t = 0;
#pragma unroll
        for (int u = 1; u < kPackRun; ++u) t += ec >= st[u] ? 1 : 0;
        const PackRec &rt = tab[t];
        const int b1 = rt.bi, b2 = rt.bj;
        const int loc = ec - rt.start;
        int p, q;
        if (sweep == 0) {   // row-major: p = loc / b2
          p = (int)((float)loc * __builtin_amdgcn_rcpf((float)b2));
          q = loc - p * b2;
          if (q >= b2) { ++p; q -= b2; }
        } else {            // column-major: q = loc / b1
          q = (int)((float)loc * __builtin_amdgcn_rcpf((float)b1));
          p = loc - q * b1;
          if (p >= b1) { ++q; p -= b1; }
        }
        tt[c] = t;
        pp[c] = p;
        qq[c] = q;
        // row-major sweep: the source is read in its own order (the load
        // does not wait on the block lookup)
        v[c] = load(g0 + (sweep == 0 ? (int64_t)ec : (int64_t)rt.start + (int64_t)p * b2 + q));
      }
#pragma unroll
      for (int c = 0; c < kPackChunk; ++c) {
        if (e0 + 64 * c >= len) break;
        const PackRec &rt = tab[tt[c]];
        const int b1 = rt.bi, b2 = rt.bj, p = pp[c], q = qq[c];
        if (KIND != 2) {
          // transposed panel of atom j: height b_j, row q, column k0 + p
          pack_store(P.dir[1], KIND, rt.pt, 0, 0, b2, q, p, v[c]);
          // forward panel of atom i: height b_i, row p, column k0 + q
          pack_store(P.dir[0], KIND, rt.pf, 0, 0, b1, p, q, v[c]);
        } else if (sweep == 0) {
          pack_store(P.dir[0], KIND, rt.pf, rt.kf, rt.vf, b1, p, q, v[c]);
        } else {
          pack_store(P.dir[1], KIND, rt.pt, rt.kt, rt.vt, b2, q, p, v[c]);
        }
      }
    }
  }
}

// Rebuild of the transposed pages from the forward pages, walking the
// transposed pages: rec[u] describes the block at transposed-page position u
// (its forward-page and transposed-page offsets and its shape), so a wave
// reads its run's maps with one load per lane before its element loads.
__global__ void __launch_bounds__(kThreads) k_refresh_records(PackParams P, const int32_t *order,
                                                              PageRec *rec) {
  const int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (u >= P.nnzb) return;
  const int32_t k = order[u];
  PageRec r;
  r.src = P.dir[0].pos[k];
  r.dst = P.dir[1].pos[k];
  r.bi = P.b[P.blk_row[k]];
  r.bj = P.b[P.col_idx[k]];
  r.pad[0] = r.pad[1] = 0;
  rec[u] = r;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_refresh(const PageRec *rec, int64_t nnzb,
                                                      const T *src, T *dst) {
  __shared__ PageRec tab_all[kWaves * kPackRun];
  const int64_t u0 = ((int64_t)blockIdx.x * kWaves + wave_id()) * kPackRun;
  if (u0 >= nnzb) return;
  const int lane = threadIdx.x & 63;
  const int nb = (int)min((int64_t)kPackRun, nnzb - u0);
  PageRec *tab = tab_all + wave_id() * kPackRun;
  int n = 0;
  if (lane < nb) {
    const PageRec r = rec[u0 + lane];
    n = r.bi * r.bj;
    tab[lane] = r;
  }
  int incl = n;
#pragma unroll
  for (int o = 1; o < kPackRun; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  const int start = incl - n;
  wave_lds_sync();
  int st[kPackRun];
  const int len = __builtin_amdgcn_readlane(incl, nb - 1);
#pragma unroll
  for (int u = 0; u < kPackRun; ++u) st[u] = u < nb ? __builtin_amdgcn_readlane(start, u) : len;
  for (int e0 = lane; e0 < len; e0 += 64 * kPackChunk) {
    T v[kPackChunk];
    int64_t d[kPackChunk];
#pragma unroll
    for (int c = 0; c < kPackChunk; ++c) {
      const int e = min(e0 + 64 * c, len - 1);
      int t = 0, stt = 0;
#pragma unroll
      for (int u = 1; u < kPackRun; ++u)
        if (e >= st[u]) {
          t = u;
          stt = st[u];
        }
      const PageRec &r = tab[t];
      const int b1 = r.bi, b2 = r.bj, l = e - stt;
      // element (p, q): row-major at the destination, column-major at the source
      int p = (int)((float)l * __builtin_amdgcn_rcpf((float)b2));
      int q = l - p * b2;
      if (q >= b2) { ++p; q -= b2; }
      v[c] = src[r.src + (int64_t)q * b1 + p];
      d[c] = r.dst + l;
    }
#pragma unroll
    for (int c = 0; c < kPackChunk; ++c) {
      if (e0 + 64 * c >= len) break;
      dst[d[c]] = v[c];
    }
  }
}

// ---------------------------------------------------------------------------
// block-sampled dY X^T on matrix cores, one wave per forward panel
// ---------------------------------------------------------------------------
// For block row i the result is the b_i x K_i panel dY_i Xg_i^T, Xg_i the X
// rows of the panel's columns: a 16 x 16 output tile per MFMA chain with
// M = panel rows, N = 16 panel columns, K = right-hand sides.  Lane (m, kq)
// holds 8 of the right-hand sides of each 32-wide chunk, the same ones for
// both operands (the contraction order inside a chunk is permuted, the sum
// is the same).  Each output goes to graph order through colg = (graph
// offset of the column's block + q) << 7 | b_j.
template <typename T, int NCH>
__global__ void __launch_bounds__(kThreads) k_sddmm_mfma(SddmmParams<T> P) {
  using V = typename Frag<T>::type;
  const int row = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave_id();
  if (row >= P.nrows) return;
  const int lane = threadIdx.x & 63;
  const int m = lane & 15;
  const int kq = lane >> 4;
  const RowDesc rd = P.rows[row];
  const int b = rd.b, K = rd.K;
  if (K == 0) return;
  const int nch = (P.nrhs + 31) >> 5;
  const int ntiles = (K + 15) >> 4;
  const int32_t *__restrict__ cx = P.colx + rd.cbase;
  const int64_t *__restrict__ cg = P.colg + rd.cbase;
  for (int mt = 0; mt * 16 < b; ++mt) {
    const int p = mt * 16 + m;
    const T *dyrow = P.dY + ((int64_t)rd.yrow + (p < b ? p : b - 1)) * P.lddy;
    // lane group kq holds 8 right-hand sides of each 32-wide chunk, the same
    // ones for both operands: FP64 takes c = 32 ch + 8 l + 2 kq + e (l < 4,
    // e < 2), so the four lane groups of one 16-byte load read 64 contiguous
    // bytes of a row; FP32 takes c = 32 ch + 8 kq + s (two 16-byte loads)
    constexpr bool PAIR = sizeof(T) == 8;
    const int kofs = PAIR ? 2 * kq : 8 * kq;
    auto ldrun = [&](const T *src, int ch, bool ok, T *dst) {
      const int cb = ch * 32 + kofs;
      auto rhs = [&](int s) { return PAIR ? cb + 8 * (s >> 1) + (s & 1) : cb + s; };
      if (ch * 32 + 32 <= P.nrhs) {
#pragma unroll
        for (int s = 0; s < 8; ++s) dst[s] = src[rhs(s)];
#pragma unroll
        for (int s = 0; s < 8; ++s) dst[s] = ok ? dst[s] : T(0);
      } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int c = rhs(s);
          const T v = src[min(c, P.nrhs - 1)];
          dst[s] = (ok && c < P.nrhs) ? v : T(0);
        }
      }
    };
    // A fragments (dY rows) of the first NCH 32-wide chunks stay in registers
    T af[NCH][8];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) ldrun(dyrow, ch, p < b && ch < nch, af[ch]);
    // one 16-column tile: B fragments of chunk 0/1 and the output map
    struct Tile {
      T bv[NCH][8];
      const T *xrow;
      int64_t g;
      bool kin;
    };
    auto load_tile = [&](int j, Tile &tl) {
      const int kc = j * 16 + m;
      tl.kin = kc < K;
      const int kk = tl.kin ? kc : K - 1;
      tl.xrow = P.X + (int64_t)cx[kk] * P.ldx;
      tl.g = P.page_out ? page_map(rd, kk) : cg[kk];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) ldrun(tl.xrow, ch, tl.kin && ch < nch, tl.bv[ch]);
    };
    // one tile's products, split over two independent accumulator chains
    auto do_tile = [&](const Tile &tl) {
      V acc0 = V{}, acc1 = V{};
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
          acc0 = mfma(af[ch][s], tl.bv[ch][s], acc0);
          acc1 = mfma(af[ch][s + 1], tl.bv[ch][s + 1], acc1);
        }
      for (int ch = NCH; ch < nch; ++ch) {
        T av[8], bv[8];
        ldrun(dyrow, ch, p < b, av);
        ldrun(tl.xrow, ch, tl.kin, bv);
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
          acc0 = mfma(av[s], bv[s], acc0);
          acc1 = mfma(av[s + 1], bv[s + 1], acc1);
        }
      }
      if (tl.kin) {
        const int64_t base = tl.g >> 7;
        const int bj = (int)(tl.g & 127);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pr = mt * 16 + dst_row<T>(kq, i);
          if (pr < b) P.dA[base + (int64_t)pr * bj] = acc0[i] + acc1[i];
        }
      }
    };
    // one tile at a time: other waves hide the load latency (a prefetched
    // second tile raised register use enough to cost more than it hid)
    for (int j = 0; j < ntiles; ++j) {
      Tile t0;
      load_tile(j, t0);
      do_tile(t0);
    }
  }
}

// ---------------------------------------------------------------------------
// block-sampled dY X^T with the X rows of each tile staged in LDS
// ---------------------------------------------------------------------------
// Same products, accumulation order and output map as k_sddmm_mfma; only the
// way X reaches the B operand differs.  A tile's 16 X rows (CW right-hand
// sides each) are loaded with whole-row pieces -- 64 / (CW / EPL) rows per
// load instruction, EPL elements (16 bytes) per lane -- instead of 16 rows
// per instruction, written to a wave-private LDS tile (rows padded by EPL
// elements, so the fragment reads of the 16 rows hit distinct banks) and read
// back in the MFMA fragment order.  X is addressed through one buffer
// descriptor (all of X within 2^31 bytes): reads past its end return zero.
template <typename T, int CW>
__global__ void __launch_bounds__(kThreads) k_sddmm_lds(SddmmParams<T> P) {
  using V = typename Frag<T>::type;
  constexpr int NCH = CW / 32;                 // 32-wide chunks per pass
  constexpr int EPL = 16 / (int)sizeof(T);     // elements per 16-byte piece
  constexpr int LPR = CW / EPL;                // lanes per staged row
  constexpr int RPI = 64 / LPR;                // rows per staging load
  constexpr int RS = CW + EPL;                 // LDS row stride (elements)
  static_assert(CW == 32 || CW == 64, "pass width");
  __shared__ __align__(16) T xs_all[kWaves * 16 * RS];
  const int row = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave_id();
  if (row >= P.nrows) return;
  const int lane = threadIdx.x & 63;
  const int m = lane & 15;
  const int kq = lane >> 4;
  T *xs = xs_all + wave_id() * 16 * RS;
  const RowDesc rd = P.rows[row];
  const int b = rd.b, K = rd.K;
  if (K == 0) return;
  const int ntiles = (K + 15) >> 4;
  const int npass = (P.nrhs + CW - 1) / CW;
  const int32_t *__restrict__ cx = P.colx + rd.cbase;
  const int64_t *__restrict__ cg = P.colg + rd.cbase;
  const __amdgpu_buffer_rsrc_t rx =
      panel_rsrc(P.X, (uint32_t)(P.xrows * P.ldx * (int64_t)sizeof(T)));
  // contraction order inside a 32-wide chunk (the same for both operands):
  // FP64 c = 8 l + 2 kq + e (l < 4, e < 2), FP32 c = 8 kq + s
  constexpr bool PAIR = sizeof(T) == 8;
  const int kofs = PAIR ? 2 * kq : 8 * kq;
  auto rhs = [&](int ch, int s) { return ch * 32 + kofs + (PAIR ? 8 * (s >> 1) + (s & 1) : s); };
  const int sr = lane / LPR;            // staging: row within a load
  const int se = (lane % LPR) * EPL;    // staging: first element of the piece
  for (int mt = 0; mt * 16 < b; ++mt) {
    const int p = mt * 16 + m;
    const T *dyrow = P.dY + ((int64_t)rd.yrow + (p < b ? p : b - 1)) * P.lddy;
    T af[NCH][8];
    auto load_af = [&](int c0) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int c = c0 + rhs(ch, s);
          const T v = dyrow[min(c, P.nrhs - 1)];
          af[ch][s] = (p < b && c < P.nrhs) ? v : T(0);
        }
    };
    if (npass == 1) load_af(0);
    for (int j = 0; j < ntiles; ++j) {
      // lane r (and r + 16, r + 32, r + 48) holds tile column r
      const int kc = j * 16 + m;
      const int kk = kc < K ? kc : K - 1;
      const int32_t xr = cx[kk];
      const int64_t g = P.page_out ? page_map(rd, kk) : cg[kk];
      V acc0 = V{}, acc1 = V{};
      for (int pass = 0; pass < npass; ++pass) {
        const int c0 = pass * CW;
        if (npass > 1) load_af(c0);
        // stage the tile's 16 rows x CW right-hand sides
        typename Vec16<T>::type v[16 / RPI];
#pragma unroll
        for (int it = 0; it < 16 / RPI; ++it) {
          const int r = it * RPI + sr;
          const int32_t xrow = __shfl(xr, r, 64);
          const int c = c0 + se;
          const uint32_t off = (j * 16 + r < K && c < P.nrhs)
                                   ? (uint32_t)(((int64_t)xrow * P.ldx + c) * (int64_t)sizeof(T))
                                   : 0x80000000u;
          v[it] = __builtin_bit_cast(typename Vec16<T>::type,
                                     __builtin_amdgcn_raw_buffer_load_b128(rx, off, 0, 0));
        }
#pragma unroll
        for (int it = 0; it < 16 / RPI; ++it) {
          const int r = it * RPI + sr;
          const int c = c0 + se;
          T *e = reinterpret_cast<T *>(&v[it]);
#pragma unroll
          for (int q = 0; q < EPL; ++q) e[q] = c + q < P.nrhs ? e[q] : T(0);
          *reinterpret_cast<typename Vec16<T>::type *>(xs + r * RS + se) = v[it];
        }
        wave_lds_sync();
        T bv[NCH][8];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
          for (int s = 0; s < 8; ++s) bv[ch][s] = xs[m * RS + rhs(ch, s)];
        wave_lds_sync();  // every read done before the next staging
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
          for (int s = 0; s < 8; s += 2) {
            acc0 = mfma(af[ch][s], bv[ch][s], acc0);
            acc1 = mfma(af[ch][s + 1], bv[ch][s + 1], acc1);
          }
      }
      if (kc < K) {
        const int64_t base = g >> 7;
        const int bj = (int)(g & 127);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pr = mt * 16 + dst_row<T>(kq, i);
          if (pr < b) P.dA[base + (int64_t)pr * bj] = acc0[i] + acc1[i];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// block-sampled dY X^T in FP64 with the X rows loaded straight into LDS
// ---------------------------------------------------------------------------
// Same products, accumulation order and output map as k_sddmm_mfma, for
// nrhs = 32 NCH.  A step is one tile and one 32-wide chunk of right-hand
// sides.  Its 16 X row pieces (256 bytes each) go from memory to a 4 KiB
// wave-private LDS buffer by buffer-to-LDS loads, which hold no registers
// while in flight; the next step's loads are issued as soon as the current
// B fragments are in registers, so they overlap this step's matrix
// instructions.  A tile's outputs are stored during the first step of the
// next tile, from a second accumulator pair, after that step's loads are
// issued: the wait for the loads of a step never waits on stores issued
// after them.
//
// LDS layout: load instruction it (0..3) writes 64 lanes x 16 bytes to
// consecutive addresses; lane l (q = l >> 4) fetches row r = 4 q + it, piece
// (l & 15) ^ r, so row r sits at (r & 3) * 1 KiB + (r >> 2) * 256 bytes with
// its pieces permuted, and the fragment reads of 16 rows at one piece index
// hit 16 distinct bank groups.  Lane l reads the X row indices of its four
// rows with one 16-byte load (rows past the panel are not loaded).  Column indices and output maps are loaded two tiles ahead.
// Requires X within 2^31 bytes (one buffer descriptor).
// PAGE: outputs in the forward pages' layout (P.page_out), where a tile's
// outputs are one contiguous run and nothing is held back.
template <int NCH, bool PAGE>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) k_sddmm_dma(SddmmParams<double> P) {
  using LdsPtr = __attribute__((address_space(3))) void *;
  constexpr int CW = 32;
  __shared__ __align__(16) double xs_all[kWaves * 16 * CW];
  const int row = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave_id();
  if (row >= P.nrows) return;
  const int lane = threadIdx.x & 63;
  const int m = lane & 15;
  const int kq = lane >> 4;
  double *xs = xs_all + wave_id() * 16 * CW;
  const RowDesc rd = P.rows[row];
  const int b = rd.b, K = rd.K;
  if (K == 0) return;
  const int ntiles = (K + 15) >> 4;
  const int nsteps = ntiles * NCH;
  const int64_t *__restrict__ cg = P.colg + rd.cbase;
  const __amdgpu_buffer_rsrc_t rx =
      panel_rsrc(P.X, (uint32_t)(P.xrows * P.ldx * (int64_t)sizeof(double)));
  // the panel's indices rounded up to a group of four (the table has four
  // entries of slack), so a group is either wholly in range or wholly past it
  const __amdgpu_buffer_rsrc_t rc =
      panel_rsrc(P.colx + rd.cbase, (uint32_t)((K + 3) & ~3) * 4u);
  // X row indices of rows 4 kq .. 4 kq + 3 of tile j
  auto rows_of = [&](int j) {
    return __builtin_bit_cast(v4u32, __builtin_amdgcn_raw_buffer_load_b128(
                                         rc, (uint32_t)(j * 16 + 4 * kq) * 4u, 0, 0));
  };
  auto gmap_of = [&](int j) {
    const int kk = min(j * 16 + m, K - 1);
    return PAGE ? page_map(rd, kk) : cg[kk];
  };
  const int sslot = lane & 15;
  auto issue = [&](int s, v4u32 xr) {
    const int j = s / NCH, ch = s % NCH;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int r = 4 * kq + it;
      const int pc = sslot ^ r;
      const uint32_t off =
          j * 16 + r < K ? (uint32_t)(((int64_t)(int32_t)xr[it] * P.ldx + ch * CW + 2 * pc) *
                                      (int64_t)sizeof(double))
                         : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (LdsPtr)(xs + it * 4 * CW), 16, off, 0, 0, 0);
    }
  };
  const double *xm = xs + (m & 3) * 4 * CW + (m >> 2) * CW;   // row m in LDS
  for (int mt = 0; mt * 16 < b; ++mt) {
    const int p = mt * 16 + m;
    const double *dyrow = P.dY + ((int64_t)rd.yrow + (p < b ? p : b - 1)) * P.lddy;
    // A fragments: lane (m, kq) holds c = 32 ch + 8 l + 2 kq + e (l < 4, e < 2)
    double af[NCH][8];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const double v = dyrow[ch * CW + 2 * kq + 8 * (s >> 1) + (s & 1)];
        af[ch][s] = p < b ? v : 0.0;
      }
    // index registers: tiles j (cur), j + 1 (nxt), j + 2 (nn, loaded during
    // tile j); they move along at the start of a tile, after the step's wait,
    // so no copy waits on a load in flight
    v4u32 xr_cur = rows_of(0), xr_nxt = rows_of(1), xr_nn = xr_nxt;
    int64_t g_cur = gmap_of(0), g_nxt = gmap_of(1), g_nn = g_nxt, g_done = 0, g_carry = 0;
    issue(0, xr_cur);
    v4d acc0 = v4d{}, acc1 = v4d{};
    double done[4] = {0.0, 0.0, 0.0, 0.0}, carry[4] = {0.0, 0.0, 0.0, 0.0};
    int csplit = 16;   // lanes m >= csplit hold carried outputs of the tile before
    for (int j = 0; j < ntiles; ++j) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const int s = j * NCH + ch;
        double bv[8];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const double2 v = *reinterpret_cast<const double2 *>(xm + 2 * ((kq + 4 * l) ^ m));
          bv[2 * l] = v.x;
          bv[2 * l + 1] = v.y;
        }
        // the fragments are in registers before the buffer is refilled
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt, expcnt unchanged
        if (ch == 0 && j > 0) {
#pragma unroll
          for (int i = 0; i < 4; ++i) done[i] = acc0[i] + acc1[i];
          acc0 = v4d{};
          acc1 = v4d{};
          g_done = g_cur;
          xr_cur = xr_nxt;
          g_cur = g_nxt;
          xr_nxt = xr_nn;
          g_nxt = g_nn;
        }
        if (s + 1 < nsteps) issue(s + 1, ch == NCH - 1 ? xr_nxt : xr_cur);
        if (ch == 0) {
          xr_nn = rows_of(j + 2);
          g_nn = gmap_of(j + 2);
          if (j > 0) {
            // Outputs of tile j - 1 (a whole tile: j - 1 is not the last).
            // A block whose columns run on into tile j is held back and
            // stored with the rest of it after tile j, so that each block's
            // lines are written in one burst.  split = first column of that
            // block in tile j - 1 (16: none held back).
            const uint32_t u = (uint32_t)(g_done >> 7);
            const uint32_t up = __shfl(u, lane - 1, 64);
            const bool brk = m == 0 || u != up + 1u;
            const uint32_t u15 = __shfl(u, 15, 64);
            const uint32_t unext = (uint32_t)(__shfl(g_cur, 0, 64) >> 7);
            const uint32_t brks = (uint32_t)__ballot(brk) & 0xFFFFu;
            const int split = !PAGE && unext == u15 + 1u ? 31 - __builtin_clz(brks) : 16;
            if (m >= csplit) {
              const int64_t base = g_carry >> 7;
              const int bj = (int)(g_carry & 127);
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int pr = mt * 16 + dst_row<double>(kq, i);
                if (pr < b) P.dA[base + (int64_t)pr * bj] = carry[i];
              }
            }
            if (m < split) {
              const int64_t base = g_done >> 7;
              const int bj = (int)(g_done & 127);
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int pr = mt * 16 + dst_row<double>(kq, i);
                if (pr < b) P.dA[base + (int64_t)pr * bj] = done[i];
              }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) carry[i] = done[i];
            g_carry = g_done;
            csplit = split;
          }
        }
#pragma unroll
        for (int l = 0; l < 8; l += 2) {
          acc0 = mfma(af[ch][l], bv[l], acc0);
          acc1 = mfma(af[ch][l + 1], bv[l + 1], acc1);
        }
      }
    }
    // held-back outputs of the tile before the last, then the last tile
    if (m >= csplit) {
      const int64_t base = g_carry >> 7;
      const int bj = (int)(g_carry & 127);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pr = mt * 16 + dst_row<double>(kq, i);
        if (pr < b) P.dA[base + (int64_t)pr * bj] = carry[i];
      }
    }
    if ((ntiles - 1) * 16 + m < K) {
      const int64_t base = g_cur >> 7;
      const int bj = (int)(g_cur & 127);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pr = mt * 16 + dst_row<double>(kq, i);
        if (pr < b) P.dA[base + (int64_t)pr * bj] = acc0[i] + acc1[i];
      }
    }
  }
}

// The same in FP32 (nrhs = 32 NCH): a step is one tile and one 32-wide chunk
// of right-hand sides, whose 16 X row pieces (128 bytes each, 2 KiB) arrive
// by two buffer-to-LDS loads: lane l of load it fetches 16-byte piece
// (l & 7) ^ (r & 7) of row r = 8 it + (l >> 3), so row r sits at r * 128
// bytes with its pieces permuted and the fragment reads of 16 rows at one
// piece index spread over the banks.  Lane (m, kq) holds right-hand sides
// 8 kq .. 8 kq + 7 of each chunk for both operands (two pieces of its row;
// the contraction order inside a chunk is permuted, the sum is the same).
// A tile's outputs are stored during the first step of the next tile, after
// that step's loads are issued.  Requires X within 2^31 bytes, 16-byte
// aligned rows.
template <int NCH, bool PAGE>
__global__ void __launch_bounds__(kThreads) k_sddmm_dma32(SddmmParams<float> P) {
  using LdsPtr = __attribute__((address_space(3))) void *;
  constexpr int CW = 32;
  __shared__ __align__(16) float xs_all[kWaves * 16 * CW];
  const int row = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave_id();
  if (row >= P.nrows) return;
  const int lane = threadIdx.x & 63;
  const int m = lane & 15;
  const int kq = lane >> 4;
  float *xs = xs_all + wave_id() * 16 * CW;
  const RowDesc rd = P.rows[row];
  const int b = rd.b, K = rd.K;
  if (K == 0) return;
  const int ntiles = (K + 15) >> 4;
  const int nsteps = ntiles * NCH;
  const int64_t *__restrict__ cg = P.colg + rd.cbase;
  const __amdgpu_buffer_rsrc_t rx =
      panel_rsrc(P.X, (uint32_t)(P.xrows * P.ldx * (int64_t)sizeof(float)));
  // the panel's indices rounded up to a group of four (four entries of slack)
  const __amdgpu_buffer_rsrc_t rc =
      panel_rsrc(P.colx + rd.cbase, (uint32_t)((K + 3) & ~3) * 4u);
  const int lr = lane >> 3;   // this lane's rows of a step: lr and 8 + lr
  auto rows_of = [&](int j) {
    v2u32 r;
    r.x = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rc, (uint32_t)(j * 16 + lr) * 4u, 0, 0);
    r.y = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rc, (uint32_t)(j * 16 + 8 + lr) * 4u, 0,
                                                         0);
    return r;
  };
  auto gmap_of = [&](int j) {
    const int kk = min(j * 16 + m, K - 1);
    return PAGE ? page_map(rd, kk) : cg[kk];
  };
  auto issue = [&](int s, v2u32 xr) {
    const int j = s / NCH, ch = s % NCH;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int r = 8 * it + lr;
      const int pc = (lane & 7) ^ (r & 7);
      const uint32_t off =
          j * 16 + r < K ? (uint32_t)(((int64_t)(int32_t)xr[it] * P.ldx + ch * CW + 4 * pc) *
                                      (int64_t)sizeof(float))
                         : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (LdsPtr)(xs + it * 8 * CW), 16, off, 0, 0, 0);
    }
  };
  const float *xm = xs + m * CW;   // row m in LDS
  for (int mt = 0; mt * 16 < b; ++mt) {
    const int p = mt * 16 + m;
    const float *dyrow = P.dY + ((int64_t)rd.yrow + (p < b ? p : b - 1)) * P.lddy;
    // A fragments: lane (m, kq) holds c = 32 ch + 8 kq + t
    float af[NCH][8];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float v = dyrow[ch * CW + 8 * kq + t];
        af[ch][t] = p < b ? v : 0.0f;
      }
    v2u32 xr_cur = rows_of(0), xr_nxt = rows_of(1), xr_nn = xr_nxt;
    int64_t g_cur = gmap_of(0), g_nxt = gmap_of(1), g_nn = g_nxt, g_done = 0;
    issue(0, xr_cur);
    v4f acc0 = v4f{}, acc1 = v4f{};
    float done[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int j = 0; j < ntiles; ++j) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const int s = j * NCH + ch;
        float bv[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float4 v =
              *reinterpret_cast<const float4 *>(xm + 4 * ((2 * kq + h) ^ (m & 7)));
          bv[4 * h] = v.x;
          bv[4 * h + 1] = v.y;
          bv[4 * h + 2] = v.z;
          bv[4 * h + 3] = v.w;
        }
        // the fragments are in registers before the buffer is refilled
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt, expcnt unchanged
        if (ch == 0 && j > 0) {
#pragma unroll
          for (int i = 0; i < 4; ++i) done[i] = acc0[i] + acc1[i];
          acc0 = v4f{};
          acc1 = v4f{};
          g_done = g_cur;
          xr_cur = xr_nxt;
          g_cur = g_nxt;
          xr_nxt = xr_nn;
          g_nxt = g_nn;
        }
        if (s + 1 < nsteps) issue(s + 1, ch == NCH - 1 ? xr_nxt : xr_cur);
        if (ch == 0) {
          xr_nn = rows_of(j + 2);
          g_nn = gmap_of(j + 2);
          if (j > 0) {   // outputs of tile j - 1 (a whole tile)
            const int64_t base = g_done >> 7;
            const int bj = (int)(g_done & 127);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int pr = mt * 16 + dst_row<float>(kq, i);
              if (pr < b) P.dA[base + (int64_t)pr * bj] = done[i];
            }
          }
        }
#pragma unroll
        for (int t = 0; t < 8; t += 2) {
          acc0 = mfma(af[ch][t], bv[t], acc0);
          acc1 = mfma(af[ch][t + 1], bv[t + 1], acc1);
        }
      }
    }
    // outputs of the last tile
    if ((ntiles - 1) * 16 + m < K) {
      const int64_t base = g_cur >> 7;
      const int bj = (int)(g_cur & 127);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pr = mt * 16 + dst_row<float>(kq, i);
        if (pr < b) P.dA[base + (int64_t)pr * bj] = acc0[i] + acc1[i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// column dot products in FP64 and their fixed-order reduction
// ---------------------------------------------------------------------------
constexpr int kDotRows = 256;

template <typename T>
__global__ void __launch_bounds__(kThreads) k_coldot(const T *A, int64_t lda, const T *B, int64_t ldb,
                                                     int64_t nrows, int32_t nrhs, double *partial) {
  const int64_t r0 = (int64_t)blockIdx.x * kDotRows;
  const int64_t r1 = min(r0 + kDotRows, nrows);
  for (int c = threadIdx.x; c < nrhs; c += kThreads) {
    double t = 0.0;
    for (int64_t r = r0; r < r1; ++r) t += (double)A[r * lda + c] * (double)B[r * ldb + c];
    partial[(int64_t)blockIdx.x * nrhs + c] = t;
  }
}

__global__ void __launch_bounds__(kThreads) k_reduce(const double *partial, int64_t nparts,
                                                     int32_t nrhs, double *out) {
  __shared__ double s[kThreads];
  const int c = blockIdx.x;
  double t = 0.0;
  for (int64_t w = threadIdx.x; w < nparts; w += kThreads) t += partial[w * nrhs + c];
  s[threadIdx.x] = t;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = s[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int NR>
hipError_t launch_vec_nr(const FwdParams<T> &p0, hipStream_t s, dim3 grid, size_t shm) {
  FwdParams<T> p = p0;
  p.xrow16 = (reinterpret_cast<uintptr_t>(p.X) % 16 == 0 && (p.ldx * sizeof(T)) % 16 == 0) ? 1 : 0;
  if constexpr (use_vp<T, NR>()) {
    if (p.mom)
      hipLaunchKernelGGL((k_spmm_vp<T, NR, true>), grid, dim3(kThreads), shm, s, p);
    else
      hipLaunchKernelGGL((k_spmm_vp<T, NR, false>), grid, dim3(kThreads), 0, s, p);
  } else {
    if (p.mom)
      hipLaunchKernelGGL((k_spmm_vec<T, NR, true>), grid, dim3(kThreads), shm, s, p);
    else
      hipLaunchKernelGGL((k_spmm_vec<T, NR, false>), grid, dim3(kThreads), 0, s, p);
  }
  return hipGetLastError();
}

template <typename T, int NT, bool VX, bool XB>
hipError_t launch_mfma_xb(const FwdParams<T> &p, hipStream_t s, dim3 grid, size_t shm) {
  if (p.mom)
    hipLaunchKernelGGL((k_spmm_mfma<T, NT, true, VX, XB>), grid, dim3(kThreads), shm, s, p);
  else
    hipLaunchKernelGGL((k_spmm_mfma<T, NT, false, VX, XB>), grid, dim3(kThreads), 0, s, p);
  return hipGetLastError();
}

template <typename T, int NT, bool VX>
hipError_t launch_mfma_nt(const FwdParams<T> &p, hipStream_t s, dim3 grid, size_t shm) {
  // one buffer descriptor covers X when its rows span less than 2^31 bytes
  if (p.xrows * p.ldx * (int64_t)sizeof(T) < (int64_t(1) << 31))
    return launch_mfma_xb<T, NT, VX, true>(p, s, grid, shm);
  return launch_mfma_xb<T, NT, VX, false>(p, s, grid, shm);
}

// The vectorised fast path applies when every vector is 16-byte aligned,
// every leading dimension is a multiple of the 16-byte element count and the
// right-hand sides fill whole passes.
template <typename T>
bool vectorizable(const FwdParams<T> &p, int nt) {
  constexpr int VEC = 16 / sizeof(T);
  auto al = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  if (p.nrhs % (16 * nt) != 0) return false;
  if (!al(p.X) || !al(p.Yout) || (p.beta != 0.0 && !al(p.Yin)) || (p.mom && !al(p.R))) return false;
  if (p.ldx % VEC || p.ldy % VEC || (p.beta != 0.0 && p.ldyin % VEC) || (p.mom && p.ldr % VEC))
    return false;
  return true;
}

template <int NT>
hipError_t launch_bf16_nt(const FwdParams<float> &p, hipStream_t s, dim3 grid, size_t shm) {
  if (p.mom)
    hipLaunchKernelGGL((k_spmm_bf16x3<NT, true>), grid, dim3(kThreads), shm, s, p);
  else
    hipLaunchKernelGGL((k_spmm_bf16x3<NT, false>), grid, dim3(kThreads), 0, s, p);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spmm_t(const FwdParams<T> &p, Kind kind, int tile, hipStream_t s) {
  const int64_t nwg = product_workgroups(p.nrows);
  if (nwg == 0) return hipSuccess;
  const dim3 grid((unsigned)nwg);
  const size_t shm = p.mom ? sizeof(double) * kWaves * (size_t)p.nrhs : 0;
  if (kind == Kind::Vec) {
    switch (tile) {
      case 1: return launch_vec_nr<T, 1>(p, s, grid, shm);
      case 2: return launch_vec_nr<T, 2>(p, s, grid, shm);
      case 4: return launch_vec_nr<T, 4>(p, s, grid, shm);
      default: return launch_vec_nr<T, 8>(p, s, grid, shm);
    }
  }
  if constexpr (std::is_same<T, float>::value) {
    if (kind == Kind::Bf16x3) {
      if (vectorizable(p, 4)) {
        const bool xb = p.xrows * p.ldx * (int64_t)sizeof(float) < (int64_t(1) << 31);
        if (p.mom) {
          if (xb)
            hipLaunchKernelGGL((k_spmm_bf16x3_vx<true, true>), grid, dim3(kThreads), shm, s, p);
          else
            hipLaunchKernelGGL((k_spmm_bf16x3_vx<true, false>), grid, dim3(kThreads), shm, s, p);
        } else {
          if (xb)
            hipLaunchKernelGGL((k_spmm_bf16x3_vx<false, true>), grid, dim3(kThreads), 0, s, p);
          else
            hipLaunchKernelGGL((k_spmm_bf16x3_vx<false, false>), grid, dim3(kThreads), 0, s, p);
        }
        return hipGetLastError();
      }
      switch (tile) {
        case 1: return launch_bf16_nt<1>(p, s, grid, shm);
        case 2: return launch_bf16_nt<2>(p, s, grid, shm);
        default: return launch_bf16_nt<4>(p, s, grid, shm);
      }
    }
  }
  // matrix cores: tile = right-hand-side tiles of 16 per pass
  constexpr int VEC = 16 / sizeof(T);
  if (tile >= VEC && vectorizable(p, tile)) {
    if constexpr (VEC == 2) {
      if (tile == 2) return launch_mfma_nt<T, 2, true>(p, s, grid, shm);
    }
    return launch_mfma_nt<T, 4, true>(p, s, grid, shm);
  }
  switch (tile) {
    case 1: return launch_mfma_nt<T, 1, false>(p, s, grid, shm);
    case 2: return launch_mfma_nt<T, 2, false>(p, s, grid, shm);
    default: return launch_mfma_nt<T, 4, false>(p, s, grid, shm);
  }
}

// ---------------------------------------------------------------------------
// thresholded block product C = A B: numeric stage, block norms, unpacking
// ---------------------------------------------------------------------------
// One wave per output block C_ij (b_i x b_j, 16 x 16 output tiles): a
// matrix-core chain over all products A_ik B_kj of the block, every tile of
// the block accumulated in the same pass so that each operand load serves
// all tiles it belongs to.  The vector-memory instruction count bounds this
// kernel (as the products), so each lane loads 16 bytes: two consecutive
// inner indices k0 = 8t + 2kq and k0 + 1 of its row of A_ik (row-major, from
// A's transposed pages, which hold every block row-major) and of its column
// of B_kj (column-major, from B's forward pages).  Step pair t then feeds two
// matrix instructions, the first over k = 8t + {0, 2, 4, 6}, the second over
// 8t + {1, 3, 5, 7}; both operands use the same k per lane, so the sum is the
// same.  Lanes past the block (row, column or k0 >= b_k) read zeros through
// the buffer bounds; when k0 + 1 == b_k the second value belongs to the next
// row or column (or the slack after the pages) and is replaced by zero.
// Matrix instructions whose k are all past b_k are skipped.
__device__ __forceinline__ double2 pair_load(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                             bool second) {
  double2 v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  v.y = second ? v.y : 0.0;
  return v;
}

// Tiles [ti0, ti0 + TI) x [tj0, tj0 + TJ) of output block c.
template <int KS2, int TI, int TJ>
__device__ __forceinline__ void spgemm_tiles(const SpgemmParams &P, int64_t c, int bi, int bj,
                                             int ti0, int tj0, double &ss) {
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, kq = lane >> 4;
  const int64_t p0 = P.pptr[c];
  const int np = (int)(P.pptr[c + 1] - p0);
  const int64_t *__restrict__ pa = P.pa + p0;
  const int64_t *__restrict__ pb = P.pb + p0;
  constexpr uint32_t kOut = 0x80000000u;
  v4d acc[TI][TJ];
#pragma unroll
  for (int ti = 0; ti < TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int q = 0; q < np; ++q) {
    const int64_t ak = pa[q];
    const int bk = (int)(ak & 255);
    // one value of slack past each block: the pair load of k0 = b_k - 1 on
    // the last row reads it (and discards it)
    const __amdgpu_buffer_rsrc_t ra =
        panel_rsrc(P.avals + (ak >> 8), (uint32_t)(bi * bk + 1) * 8u);
    const __amdgpu_buffer_rsrc_t rb = panel_rsrc(P.bvals + pb[q], (uint32_t)(bk * bj + 1) * 8u);
    double2 av[TI][KS2], bv[TJ][KS2];
#pragma unroll
    for (int t = 0; t < KS2; ++t) {
      const int k0 = 8 * t + 2 * kq;
      const bool kin = k0 < bk, k2 = k0 + 1 < bk;
#pragma unroll
      for (int ti = 0; ti < TI; ++ti) {
        const int row = (ti0 + ti) * 16 + m;
        av[ti][t] = pair_load(ra, row < bi && kin ? (uint32_t)(row * bk + k0) * 8u : kOut, k2);
      }
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) {
        const int col = (tj0 + tj) * 16 + m;
        bv[tj][t] = pair_load(rb, col < bj && kin ? (uint32_t)(col * bk + k0) * 8u : kOut, k2);
      }
    }
#pragma unroll
    for (int t = 0; t < KS2; ++t) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (8 * t + h < bk) {
#pragma unroll
          for (int ti = 0; ti < TI; ++ti)
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj)
              acc[ti][tj] = mfma(h ? av[ti][t].y : av[ti][t].x, h ? bv[tj][t].y : bv[tj][t].x,
                                 acc[ti][tj]);
        }
      }
    }
  }
  if (P.fpages) {   // straight into C's pages: forward column-major, transposed row-major
    // the forward (column-major) stores go through a wave-private LDS copy
    // of the tile, so that 8 lanes write one whole column of 16 rows with
    // 16-byte stores (a lane's own values are rows 4 apart of one column)
    __shared__ __align__(16) double tl_all[kWaves * 16 * 18];
    double *tl = tl_all + wave_id() * 16 * 18;   // column-major, 18 per column
    double *ot = P.tpages + P.tpos[c];
    // the block's forward values: columns past b_j fall outside and are dropped
    const __amdgpu_buffer_rsrc_t rf =
        panel_rsrc(P.fpages + P.fpos[c], (uint32_t)(bi * bj) * 8u);
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = (ti0 + ti) * 16 + dst_row<double>(kq, e), col = (tj0 + tj) * 16 + m;
          if (r < bi && col < bj) {
            ot[(int64_t)r * bj + col] = acc[ti][tj][e];
            ss = fma(acc[ti][tj][e], acc[ti][tj][e], ss);
          }
          tl[m * 18 + dst_row<double>(kq, e)] = acc[ti][tj][e];
        }
        wave_lds_sync();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int cl = 8 * h + (lane >> 3), rl = 2 * (lane & 7);
          const int col = (tj0 + tj) * 16 + cl, r = (ti0 + ti) * 16 + rl;
          const double2 v = *reinterpret_cast<const double2 *>(tl + cl * 18 + rl);
          const uint32_t off = (uint32_t)(col * bi + r) * 8u;
          if (r + 1 < bi)
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u32, v), rf, off, 0, 0);
          else if (r < bi)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u32, v.x), rf, off, 0, 0);
        }
        wave_lds_sync();   // read before the next tile is written
      }
    return;
  }
  double *out = P.cvals + P.obase[c];
#pragma unroll
  for (int ti = 0; ti < TI; ++ti)
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = (ti0 + ti) * 16 + dst_row<double>(kq, e), col = (tj0 + tj) * 16 + m;
        if (r < bi && col < bj) {
          out[(int64_t)r * bj + col] = acc[ti][tj][e];
          ss = fma(acc[ti][tj][e], acc[ti][tj][e], ss);
        }
      }
}

// Output blocks P.order[0 .. P.count) of one tile class: TI x TJ tiles of
// 16 x 16, or (TI = TJ = 0) any size, one tile at a time.
template <int KS2, int TI, int TJ>
__global__ void __launch_bounds__(kThreads) k_spgemm(SpgemmParams P) {
  const int64_t w = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave_id();
  if (w >= P.count) return;
  const int64_t c = P.order[w];
  const int bi = P.b[P.oi[c]], bj = P.b[P.oj[c]];
  double ss = 0.0;
  if constexpr (TI > 0) {
    spgemm_tiles<KS2, TI, TJ>(P, c, bi, bj, 0, 0, ss);
  } else {
    for (int ti = 0; ti * 16 < bi; ++ti)
      for (int tj = 0; tj * 16 < bj; ++tj) spgemm_tiles<KS2, 1, 1>(P, c, bi, bj, ti, tj, ss);
  }
  if (P.cnorm) {
    ss = wave_sum(ss);
    if ((threadIdx.x & 63) == 0) P.cnorm[c] = sqrt(ss);
  }
}

// Frobenius norm of every stored block from the forward pages (a block is a
// contiguous run of b_i*b_j values there); one wave per block.
__global__ void __launch_bounds__(kThreads) k_block_norms(const double *pages, const int64_t *pos,
                                                          const int32_t *blk_row,
                                                          const int32_t *col_idx,
                                                          const int32_t *b, int64_t nnzb,
                                                          double *out) {
  const int64_t k = (int64_t)blockIdx.x * kWaves + wave_id();
  if (k >= nnzb) return;
  const int lane = threadIdx.x & 63;
  const int sz = b[blk_row[k]] * b[col_idx[k]];
  const double *v = pages + pos[k];
  double s = 0.0;
  for (int e = lane; e < sz; e += 64) s = fma(v[e], v[e], s);
  s = wave_sum(s);
  if (lane == 0) out[k] = sqrt(s);
}

// Zero the alignment gap after every panel and the slack after the last
// (the values themselves are written by the packing): one thread per panel.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_zero_gaps(const RowDesc *rows, int32_t np,
                                                        int64_t n_values, T *vals) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= np && !(p == 0 && np == 0)) return;
  const int64_t s = np ? rows[p].vbase + (int64_t)rows[p].b * rows[p].K : 0;
  const int64_t e = p + 1 < np ? rows[p + 1].vbase : n_values + kPageSlack;
  for (int64_t x = s; x < e; ++x) vals[x] = T(0);
}

// dst[dbase[t] + e] = src[sbase[t] + e] for e < size[t]; one wave per block.
__global__ void __launch_bounds__(kThreads) k_gather_blocks(const double *src,
                                                            const int64_t *sbase,
                                                            const int64_t *dbase,
                                                            const int32_t *size, int64_t nblk,
                                                            double *dst) {
  const int64_t t = (int64_t)blockIdx.x * kWaves + wave_id();
  if (t >= nblk) return;
  const int lane = threadIdx.x & 63;
  const double *sp = src + sbase[t];
  double *dp = dst + dbase[t];
  for (int e = lane; e < size[t]; e += 64) dp[e] = sp[e];
}

// Forward pages -> graph order (each block row-major at gbase); one wave per
// block.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_unpack(const T *pages, const int64_t *pos,
                                                     const int32_t *blk_row,
                                                     const int32_t *col_idx, const int32_t *b,
                                                     const int64_t *gbase, int64_t nnzb, T *dst) {
  const int64_t k = (int64_t)blockIdx.x * kWaves + wave_id();
  if (k >= nnzb) return;
  const int lane = threadIdx.x & 63;
  const int bi = b[blk_row[k]], bj = b[col_idx[k]];
  const T *sp = pages + pos[k];
  T *dp = dst + gbase[k];
  for (int e = lane; e < bi * bj; e += 64) {
    const int p = e / bj, q = e - p * bj;
    dp[e] = sp[(int64_t)q * bi + p];
  }
}

// ---------------------------------------------------------------------------
// kernel polynomial method: damped coefficients and the density of states
// ---------------------------------------------------------------------------
// c_0 = g_0 mu_0, c_k = 2 g_k mu_k (k >= 1): the coefficients of the series
// sum_k c_k T_k(x); g_k = 1 (no damping) or the Jackson factors
// [(M-k+1) cos(q k) + sin(q k) cot(q)] / (M+1), q = pi / (M+1).
__global__ void __launch_bounds__(kThreads) k_kpm_coef(const double *mu, int M, int damping,
                                                       double *c) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= M) return;
  double g = 1.0;
  if (damping == 1) {
    const double q = M_PI / (M + 1);
    g = ((double)(M - k + 1) * cos(q * k) + sin(q * k) * cos(q) / sin(q)) / (M + 1);
  }
  c[k] = (k == 0 ? 1.0 : 2.0) * g * mu[k];
}

// rho(x) = sum_k c_k T_k(x) / (pi sqrt(1 - x^2)) at every point, one lane per
// point, the series summed by Clenshaw's recurrence from the highest degree
// (b_k = c_k + 2x b_{k+1} - b_{k+2}; sum = c_0 + x b_1 - b_2).  All lanes read
// the same c_k: the coefficients come through the scalar cache, 16 per
// unrolled step.
__global__ void __launch_bounds__(kThreads) k_kpm_dos(const double *c, int M, const double *x,
                                                      int64_t np, double *rho) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const double xi = i < np ? x[i] : 0.0;
  const double tx = 2.0 * xi;
  double b1 = 0.0, b2 = 0.0;
  int k = M - 1;
  for (; k >= 16; k -= 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double b0 = fma(tx, b1, c[k - u] - b2);
      b2 = b1;
      b1 = b0;
    }
  }
  for (; k >= 1; --k) {
    const double b0 = fma(tx, b1, c[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  const double s = fma(xi, b1, c[0] - b2);
  if (i < np) rho[i] = s / (M_PI * sqrt(1.0 - xi * xi));
}

// One thread per graph block writes the column-table entries of its panel
// columns (set-up, once per structure).
__global__ void __launch_bounds__(kThreads) k_columns(ColumnParams P) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= P.nnzb) return;
  const int32_t c = P.catom[k];
  const int bc = P.b[c];
  const int64_t base = P.rows[P.prow[k]].cbase + P.k0[k];
  const int32_t o = P.off[c];
  for (int q = 0; q < bc; ++q) {
    P.colx[base + q] = o + q;
    if (P.colg) P.colg[base + q] = ((P.gbase[k] + q) << 7) | bc;
  }
}

}  // namespace

int64_t product_workgroups(int64_t nrows) { return (nrows + kWaves - 1) / kWaves; }

hipError_t launch_spmm_f64(const FwdParams<double> &p, Kind kind, int tile, hipStream_t s) {
  return launch_spmm_t<double>(p, kind == Kind::Bf16x3 ? Kind::Mfma : kind, tile, s);
}
hipError_t launch_spmm_f32(const FwdParams<float> &p, Kind kind, int tile, hipStream_t s) {
  return launch_spmm_t<float>(p, kind, tile, s);
}

hipError_t launch_pack(const PackParams &p, const void *src, int src_dtype, hipStream_t s) {
  if (p.nnzb == 0) return hipSuccess;
  const int64_t waves = (p.nnzb + kPackRun - 1) / kPackRun;
  const dim3 grid((unsigned)((waves + kWaves - 1) / kWaves));
  const int sel = src_dtype * 3 + p.dst_kind;
  switch (sel) {
    case 0: hipLaunchKernelGGL((k_pack<0, 0>), grid, dim3(kThreads), 0, s, p, src); break;
    case 1: hipLaunchKernelGGL((k_pack<0, 1>), grid, dim3(kThreads), 0, s, p, src); break;
    case 2: hipLaunchKernelGGL((k_pack<0, 2>), grid, dim3(kThreads), 0, s, p, src); break;
    case 3: hipLaunchKernelGGL((k_pack<1, 0>), grid, dim3(kThreads), 0, s, p, src); break;
    case 4: hipLaunchKernelGGL((k_pack<1, 1>), grid, dim3(kThreads), 0, s, p, src); break;
    case 5: hipLaunchKernelGGL((k_pack<1, 2>), grid, dim3(kThreads), 0, s, p, src); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sddmm_t(const SddmmParams<T> &p, hipStream_t s) {
  if (p.nrows == 0) return hipSuccess;
  const dim3 grid((unsigned)product_workgroups(p.nrows));
  // X rows staged through LDS when all of X fits one buffer descriptor
  if (p.xrows * p.ldx * (int64_t)sizeof(T) < (int64_t(1) << 31)) {
    if (std::is_same<T, double>::value && (p.nrhs == 32 || p.nrhs == 64)) {
      const auto &pd = reinterpret_cast<const SddmmParams<double> &>(p);
      if (p.nrhs == 32 && p.page_out)
        hipLaunchKernelGGL((k_sddmm_dma<1, true>), grid, dim3(kThreads), 0, s, pd);
      else if (p.nrhs == 32)
        hipLaunchKernelGGL((k_sddmm_dma<1, false>), grid, dim3(kThreads), 0, s, pd);
      else if (p.page_out)
        hipLaunchKernelGGL((k_sddmm_dma<2, true>), grid, dim3(kThreads), 0, s, pd);
      else
        hipLaunchKernelGGL((k_sddmm_dma<2, false>), grid, dim3(kThreads), 0, s, pd);
      return hipGetLastError();
    }
    if (std::is_same<T, float>::value && (p.nrhs == 32 || p.nrhs == 64) &&
        reinterpret_cast<uintptr_t>(p.X) % 16 == 0 && p.ldx % 4 == 0) {
      const auto &pf = reinterpret_cast<const SddmmParams<float> &>(p);
      if (p.nrhs == 32 && p.page_out)
        hipLaunchKernelGGL((k_sddmm_dma32<1, true>), grid, dim3(kThreads), 0, s, pf);
      else if (p.nrhs == 32)
        hipLaunchKernelGGL((k_sddmm_dma32<1, false>), grid, dim3(kThreads), 0, s, pf);
      else if (p.page_out)
        hipLaunchKernelGGL((k_sddmm_dma32<2, true>), grid, dim3(kThreads), 0, s, pf);
      else
        hipLaunchKernelGGL((k_sddmm_dma32<2, false>), grid, dim3(kThreads), 0, s, pf);
      return hipGetLastError();
    }
    if (p.nrhs <= 32)
      hipLaunchKernelGGL((k_sddmm_lds<T, 32>), grid, dim3(kThreads), 0, s, p);
    else
      hipLaunchKernelGGL((k_sddmm_lds<T, 64>), grid, dim3(kThreads), 0, s, p);
    return hipGetLastError();
  }
  // right-hand sides beyond the register-resident chunks are loaded per tile
  if (p.nrhs <= 32)
    hipLaunchKernelGGL((k_sddmm_mfma<T, 1>), grid, dim3(kThreads), 0, s, p);
  else
    hipLaunchKernelGGL((k_sddmm_mfma<T, 2>), grid, dim3(kThreads), 0, s, p);
  return hipGetLastError();
}
hipError_t launch_sddmm_f64(const SddmmParams<double> &p, hipStream_t s) {
  return launch_sddmm_t(p, s);
}
hipError_t launch_sddmm_f32(const SddmmParams<float> &p, hipStream_t s) {
  return launch_sddmm_t(p, s);
}

int64_t coldot_chunks(int64_t nrows) { return (nrows + kDotRows - 1) / kDotRows; }

hipError_t launch_coldot_f64(const double *A, int64_t lda, const double *B, int64_t ldb,
                             int64_t nrows, int32_t nrhs, double *partial, int64_t *nchunks,
                             hipStream_t s) {
  *nchunks = coldot_chunks(nrows);
  if (*nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_coldot<double>, dim3((unsigned)*nchunks), dim3(kThreads), 0, s, A, lda, B,
                     ldb, nrows, nrhs, partial);
  return hipGetLastError();
}
hipError_t launch_coldot_f32(const float *A, int64_t lda, const float *B, int64_t ldb,
                             int64_t nrows, int32_t nrhs, double *partial, int64_t *nchunks,
                             hipStream_t s) {
  *nchunks = coldot_chunks(nrows);
  if (*nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_coldot<float>, dim3((unsigned)*nchunks), dim3(kThreads), 0, s, A, lda, B,
                     ldb, nrows, nrhs, partial);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double *partial, int64_t nparts, int32_t nrhs, double *out,
                                  hipStream_t s) {
  if (nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)nrhs), dim3(kThreads), 0, s, partial, nparts, nrhs, out);
  return hipGetLastError();
}

template <int KS2>
hipError_t launch_spgemm_ks(const SpgemmParams &p, int cls, dim3 grid, hipStream_t s) {
  switch (cls) {
    case 0: hipLaunchKernelGGL((k_spgemm<KS2, 1, 1>), grid, dim3(kThreads), 0, s, p); break;
    case 1: hipLaunchKernelGGL((k_spgemm<KS2, 1, 2>), grid, dim3(kThreads), 0, s, p); break;
    case 2: hipLaunchKernelGGL((k_spgemm<KS2, 2, 1>), grid, dim3(kThreads), 0, s, p); break;
    case 3: hipLaunchKernelGGL((k_spgemm<KS2, 2, 2>), grid, dim3(kThreads), 0, s, p); break;
    default: hipLaunchKernelGGL((k_spgemm<KS2, 0, 0>), grid, dim3(kThreads), 0, s, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_spgemm_numeric(const SpgemmParams &p, int cls, int max_b, hipStream_t s) {
  if (p.count == 0) return hipSuccess;
  const dim3 grid((unsigned)((p.count + kWaves - 1) / kWaves));
  // pairs of inner indices held per product: ceil(max_b / 8)
  if (max_b <= 8) return launch_spgemm_ks<1>(p, cls, grid, s);
  if (max_b <= 16) return launch_spgemm_ks<2>(p, cls, grid, s);
  if (max_b <= 24) return launch_spgemm_ks<3>(p, cls, grid, s);
  if (max_b <= 32) return launch_spgemm_ks<4>(p, cls, grid, s);
  return launch_spgemm_ks<8>(p, cls, grid, s);
}

hipError_t launch_block_norms(const double *pages, const int64_t *pos, const int32_t *blk_row,
                              const int32_t *col_idx, const int32_t *b, int64_t nnzb, double *out,
                              hipStream_t s) {
  if (nnzb == 0) return hipSuccess;
  const dim3 grid((unsigned)((nnzb + kWaves - 1) / kWaves));
  hipLaunchKernelGGL(k_block_norms, grid, dim3(kThreads), 0, s, pages, pos, blk_row, col_idx, b,
                     nnzb, out);
  return hipGetLastError();
}

hipError_t launch_refresh_records(const PackParams &p, const int32_t *order, PageRec *rec,
                                  hipStream_t s) {
  if (p.nnzb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_refresh_records, dim3((unsigned)((p.nnzb + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, p, order, rec);
  return hipGetLastError();
}

hipError_t launch_refresh(const PageRec *rec, int64_t nnzb, int elem_bytes, const void *src,
                          void *dst, hipStream_t s) {
  if (nnzb == 0) return hipSuccess;
  const int64_t waves = (nnzb + kPackRun - 1) / kPackRun;
  const dim3 grid((unsigned)((waves + kWaves - 1) / kWaves));
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_refresh<double>, grid, dim3(kThreads), 0, s, rec, nnzb,
                       static_cast<const double *>(src), static_cast<double *>(dst));
  else
    hipLaunchKernelGGL(k_refresh<float>, grid, dim3(kThreads), 0, s, rec, nnzb,
                       static_cast<const float *>(src), static_cast<float *>(dst));
  return hipGetLastError();
}

hipError_t launch_zero_gaps(const RowDesc *rows, int32_t np, int64_t n_values, int elem_bytes,
                            void *vals, hipStream_t s) {
  const dim3 grid((unsigned)((std::max<int64_t>(np, 1) + kThreads - 1) / kThreads));
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_zero_gaps<double>, grid, dim3(kThreads), 0, s, rows, np, n_values,
                       static_cast<double *>(vals));
  else
    hipLaunchKernelGGL(k_zero_gaps<float>, grid, dim3(kThreads), 0, s, rows, np, n_values,
                       static_cast<float *>(vals));
  return hipGetLastError();
}

hipError_t launch_gather_blocks(const double *src, const int64_t *sbase, const int64_t *dbase,
                                const int32_t *size, int64_t nblk, double *dst, hipStream_t s) {
  if (nblk == 0) return hipSuccess;
  const dim3 grid((unsigned)((nblk + kWaves - 1) / kWaves));
  hipLaunchKernelGGL(k_gather_blocks, grid, dim3(kThreads), 0, s, src, sbase, dbase, size, nblk,
                     dst);
  return hipGetLastError();
}

hipError_t launch_unpack(const void *pages, int elem_bytes, const int64_t *pos,
                         const int32_t *blk_row, const int32_t *col_idx, const int32_t *b,
                         const int64_t *gbase, int64_t nnzb, void *dst, hipStream_t s) {
  if (nnzb == 0) return hipSuccess;
  const dim3 grid((unsigned)((nnzb + kWaves - 1) / kWaves));
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_unpack<double>, grid, dim3(kThreads), 0, s,
                       static_cast<const double *>(pages), pos, blk_row, col_idx, b, gbase, nnzb,
                       static_cast<double *>(dst));
  else
    hipLaunchKernelGGL(k_unpack<float>, grid, dim3(kThreads), 0, s,
                       static_cast<const float *>(pages), pos, blk_row, col_idx, b, gbase, nnzb,
                       static_cast<float *>(dst));
  return hipGetLastError();
}

hipError_t launch_kpm_dos(const double *mu, int M, int damping, const double *x, int64_t np,
                          double *coef, double *rho, hipStream_t s) {
  hipLaunchKernelGGL(k_kpm_coef, dim3((unsigned)((M + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     s, mu, M, damping, coef);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || np == 0) return e;
  hipLaunchKernelGGL(k_kpm_dos, dim3((unsigned)((np + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                     s, coef, M, x, np, rho);
  return hipGetLastError();
}

hipError_t launch_columns(const ColumnParams &p, hipStream_t s) {
  if (p.nnzb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_columns, dim3((unsigned)((p.nnzb + kThreads - 1) / kThreads)), dim3(kThreads),
                     0, s, p);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// halo exchange buffers of a rank-local operator
// ---------------------------------------------------------------------------
// buf[t, c] = X[rows[t], c]: one thread per element, consecutive threads
// along c (coalesced row pieces).  Rows outside [0, xrows) are skipped.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_rows_pack(const T *__restrict__ X, int64_t xrows,
                                                        int64_t ldx, const int32_t *__restrict__ rows,
                                                        int64_t nrows, int32_t nrhs,
                                                        T *__restrict__ buf, int64_t ldb) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= nrows * nrhs) return;
  const int64_t t = e / nrhs, c = e - t * nrhs;
  const int64_t r = rows[t];
  if (r < 0 || r >= xrows) return;
  buf[t * ldb + c] = X[r * ldx + c];
}

// Y[red_rows[u], c] += sum over e in [red_ptr[u], red_ptr[u+1]) of
// buf[red_pos[e], c], in e order: one thread per (u, c), so every output
// element has one writer.  Indices outside Y or the buffer are skipped.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_rows_reduce(T *__restrict__ Y, int64_t yrows,
                                                          int64_t ldy,
                                                          const int32_t *__restrict__ red_rows,
                                                          const int64_t *__restrict__ red_ptr,
                                                          const int64_t *__restrict__ red_pos,
                                                          int64_t n_red, int64_t brows,
                                                          const T *__restrict__ buf, int64_t ldb,
                                                          int32_t nrhs) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n_red * nrhs) return;
  const int64_t u = e / nrhs, c = e - u * nrhs;
  const int64_t r = red_rows[u];
  if (r < 0 || r >= yrows) return;
  T acc = Y[r * ldy + c];
  for (int64_t q = red_ptr[u]; q < red_ptr[u + 1]; ++q) {
    const int64_t s = red_pos[q];
    if (s >= 0 && s < brows) acc += buf[s * ldb + c];
  }
  Y[r * ldy + c] = acc;
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free entry points
// ---------------------------------------------------------------------------
// One copy per GPU, resident from the module's load to the end of the
// process.  In host code `scratch` names only the host-side stand-in of the
// array: its device address is looked up below, once per device, and only
// that address is ever passed to kernels.
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

hipError_t noalloc_scratch(void **ptr, size_t *bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kNoAllocScratchBytes;
  return hipSuccess;
}


hipError_t launch_rows_pack(const void *X, int64_t xrows, int64_t ldx, const int32_t *rows,
                            int64_t nrows, int32_t nrhs, int elem_bytes, void *buf, int64_t ldb,
                            hipStream_t s) {
  const int64_t n = nrows * nrhs;
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_rows_pack<double>, grid, dim3(kThreads), 0, s,
                       static_cast<const double *>(X), xrows, ldx, rows, nrows, nrhs,
                       static_cast<double *>(buf), ldb);
  else
    hipLaunchKernelGGL(k_rows_pack<float>, grid, dim3(kThreads), 0, s,
                       static_cast<const float *>(X), xrows, ldx, rows, nrows, nrhs,
                       static_cast<float *>(buf), ldb);
  return hipGetLastError();
}

hipError_t launch_rows_reduce(void *Y, int64_t yrows, int64_t ldy, const int32_t *red_rows,
                              const int64_t *red_ptr, const int64_t *red_pos, int64_t n_red,
                              int64_t brows, const void *buf, int64_t ldb, int32_t nrhs,
                              int elem_bytes, hipStream_t s) {
  const int64_t n = n_red * nrhs;
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads));
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_rows_reduce<double>, grid, dim3(kThreads), 0, s, static_cast<double *>(Y),
                       yrows, ldy, red_rows, red_ptr, red_pos, n_red, brows,
                       static_cast<const double *>(buf), ldb, nrhs);
  else
    hipLaunchKernelGGL(k_rows_reduce<float>, grid, dim3(kThreads), 0, s, static_cast<float *>(Y),
                       yrows, ldy, red_rows, red_ptr, red_pos, n_red, brows,
                       static_cast<const float *>(buf), ldb, nrhs);
  return hipGetLastError();
}

}  // namespace vbcsr
