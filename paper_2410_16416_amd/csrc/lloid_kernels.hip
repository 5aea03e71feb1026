// gfx950 kernels of the LLOID filtering path.
//
// Stages (the method's order, Sec. II.A): strain conversion, half-band
// decimation to every slice rate, the per-slice FIR bank as a sliding-window
// GEMM on MFMA, interpolation of the low-rate orthogonal SNR to the full
// rate, the mixing GEMM over the concatenated basis with a fused complex-SNR
// and per-window peak epilogue, and trigger compaction (Sec. II.B: only the
// triggers leave the device).  FP64 appears only in the sigma^2 sums.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "lloid_internal.h"

namespace lloid {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------- MFMA ops
// Operand type T: K per instruction (KS), elements per lane per operand (VEC).
// Lane l of a 32x32xKS instruction supplies row/column l % 32 and the VEC
// consecutive k values starting at (l / 32) * VEC; the 32x32 FP32 result puts
// rows 8 (r/4) + 4 (l/32) + r%4, r = 0..15, of column l % 32 in lane l.
template <typename T> struct Op;

template <> struct Op<_Float16> {
  static constexpr int KS = 16, VEC = 8;
  typedef half8 vec;
  static __device__ __forceinline__ f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ _Float16 cvt(float v) { return (_Float16)v; }
  static __device__ __forceinline__ float tof(_Float16 v) { return (float)v; }
};

template <> struct Op<__bf16> {
  static constexpr int KS = 16, VEC = 8;
  typedef bf16x8 vec;
  static __device__ __forceinline__ f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ __bf16 cvt(float v) { return (__bf16)v; }
  static __device__ __forceinline__ float tof(__bf16 v) { return (float)v; }
};

template <> struct Op<float> {
  static constexpr int KS = 2, VEC = 1;
  typedef float vec;
  static __device__ __forceinline__ f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ float cvt(float v) { return v; }
  static __device__ __forceinline__ float tof(float v) { return v; }
};

template <typename T> struct OutT { typedef T type; };

// ---------------------------------------------------------- small kernels

template <typename TI>
__global__ void k_convert(const TI *__restrict__ src, int64_t n, float *__restrict__ dst, int64_t dst_lo,
                          int64_t dst_len, float scale, int *__restrict__ bad) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= dst_len) return;
  int64_t a = dst_lo + t;
  float v = 0.f;
  if (a >= 0 && a < n) {
    double s = (double)src[a];
    if (!isfinite(s)) {
      atomicOr(bad, 1);
      s = 0.0;
    }
    v = (float)(s * (double)scale);
  }
  dst[t] = v;
}

// d[k] = sum_{|n| <= 32} g[n] u[2k - n]; g is zero at even n != 0 and 1/2 at 0,
// so the sum runs over the centre and symmetric odd pairs.
__global__ void k_decimate(const float *__restrict__ u, int64_t u_lo, int64_t u_len, float *__restrict__ d,
                           int64_t d_lo, int64_t d_len, const float *__restrict__ g) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d_len) return;
  int64_t c = 2 * (d_lo + t) - u_lo;  // buffer index of u[2k]
  auto at = [&](int64_t i) -> float { return (i >= 0 && i < u_len) ? u[i] : 0.f; };
  float acc = g[kHalfQ] * at(c);
  for (int n = 1; n <= kHalfQ; n += 2) acc += g[kHalfQ + n] * (at(c - n) + at(c + n));
  d[t] = acc;
}

template <typename TI, typename TO>
__global__ void k_interp(const TI *__restrict__ w, int64_t w_lo, int64_t w_len, int ldw, TO *__restrict__ v,
                         int64_t v_lo, int64_t v_len, int ldv, int col0, int channels,
                         const float *__restrict__ g) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t row = t / channels;
  int c = (int)(t - row * channels);
  if (row >= v_len) return;
  int64_t n = v_lo + row;
  float acc;
  if ((n & 1) == 0) {
    int64_t j = (n >> 1) - w_lo;
    acc = (j >= 0 && j < w_len) ? (float)w[j * ldw + c] : 0.f;
  } else {
    // odd n: v[n] = sum_j w[j] 2 g[n - 2j] over |n - 2j| <= 31
    acc = 0.f;
    int64_t jc = (n - 1) >> 1;  // n - 2 jc = 1
    for (int q = 0; q < kHalfQ / 2; ++q) {
      int64_t ja = jc - q - w_lo, jb = jc + 1 + q - w_lo;  // offsets n-2j = 1+2q and -(1+2q)
      float a = (ja >= 0 && ja < w_len) ? (float)w[ja * ldw + c] : 0.f;
      float b = (jb >= 0 && jb < w_len) ? (float)w[jb * ldw + c] : 0.f;
      acc += 2.f * g[kHalfQ + 1 + 2 * q] * (a + b);
    }
  }
  v[row * (int64_t)ldv + col0 + c] = (TO)acc;
}

template <typename T>
__global__ void k_cast_f64(const double *__restrict__ src, T *__restrict__ dst, int64_t n) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = (T)src[t];
}

__global__ void k_fill_u8(uint8_t *p, size_t bytes) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; t < bytes; t += stride) p[t] = 0;
}

__global__ void k_sigma2(const double *__restrict__ m, int n_templates, int lsum,
                         const double *__restrict__ inv_dec, double *__restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_templates) return;
  const double *rc = m + (int64_t)(2 * i) * lsum;
  const double *rs = rc + lsum;
  double acc = 0.0;
  for (int c = 0; c < lsum; ++c) acc += (rc[c] * rc[c] + rs[c] * rs[c]) * inv_dec[c];
  out[i] = acc;
}

// ------------------------------------------------------------ GEMM pieces

// Stage rows [r0, r0 + 32 MT) x k [k0, k0 + kBK) of a row-major [rows][ld]
// matrix into LDS (row pitch kBK + pad elements), zero past `rows`.
template <typename T, int BM, int PITCH>
__device__ __forceinline__ void stage_rows(const T *__restrict__ a, int64_t rows, int64_t ld, int64_t r0,
                                           int k0, T *lds) {
  constexpr int VPR = kBK * (int)sizeof(T) / 16;  // 16-byte vectors per row
  constexpr int NV = BM * VPR;
  for (int v = threadIdx.x; v < NV; v += kThreads) {
    int r = v / VPR, c = v % VPR;
    uint4 val = make_uint4(0, 0, 0, 0);
    if (r0 + r < rows) val = *(const uint4 *)(a + (r0 + r) * ld + k0 + c * (16 / (int)sizeof(T)));
    *(uint4 *)(lds + r * PITCH + c * (16 / (int)sizeof(T))) = val;
  }
}

template <typename T> struct Pitch {
  // +16 bytes per row keeps the 16-byte fragment reads of 32 lanes spread over banks
  static constexpr int value = kBK + 16 / (int)sizeof(T);
};

// ---------------------------------------------------------------- FIR
// o[l, k] = sum_m U[l, m] x[k - J/D - m] as D = A B with A = taps reversed
// (Ar[l, m'] = U[l, N-1-m']) and the Hankel operand B[m', k] = x[k + m' + base],
// base = -(J/D + N - 1).  The strain window of a K chunk sits in LDS as VEC
// copies shifted by 0..VEC-1 samples, so every lane's VEC consecutive samples
// are one aligned read whatever its column.
template <typename T, typename TO, int MT, int NT>
__global__ __launch_bounds__(kThreads) void k_fir(const T *__restrict__ a, int64_t rows, int np,
                                                  const float *__restrict__ x, int64_t x_lo, int64_t x_len,
                                                  int64_t base, int64_t k_lo, int64_t k_hi,
                                                  TO *__restrict__ out, int64_t out_lo, int ldo, int col0,
                                                  int col_limit) {
  typedef Op<T> O;
  constexpr int BM = 32 * MT, BN = kWaves * 32 * NT;
  constexpr int AP = Pitch<T>::value;
  constexpr int WC = BN + kBK + 8;  // copy length (multiple of 8)
  __shared__ __attribute__((aligned(16))) T As[BM * AP];
  __shared__ __attribute__((aligned(16))) T Bc[O::VEC * WC];
  __shared__ float raw[WC + 8];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.y * BM;
  const int64_t i0 = k_lo + (int64_t)blockIdx.x * BN;

  f32x16 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[mt][nt][e] = 0.f;

  for (int kc = 0; kc < np; kc += kBK) {
    __syncthreads();
    stage_rows<T, BM, AP>(a, rows, np, r0, kc, As);
    const int64_t w0 = i0 + kc + base - x_lo;  // buffer index of window sample 0
    for (int t = threadIdx.x; t < WC + 8; t += kThreads) {
      int64_t idx = w0 + t;
      raw[t] = (idx >= 0 && idx < x_len) ? x[idx] : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < O::VEC * WC; e += kThreads) {
      int r = e / WC, t = e - r * WC;
      Bc[e] = O::cvt(raw[t + r]);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kBK / O::KS; ++ks) {
      typename O::vec af[MT], bf[NT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        af[mt] = *(const typename O::vec *)(As + (mt * 32 + (lane & 31)) * AP + ks * O::KS + (lane >> 5) * O::VEC);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        int pos = wave * NT * 32 + nt * 32 + (lane & 31) + ks * O::KS + (lane >> 5) * O::VEC;
        int r = pos % O::VEC;
        bf[nt] = *(const typename O::vec *)(Bc + r * WC + (pos - r));
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = O::mfma(af[mt], bf[nt], acc[mt][nt]);
    }
  }

  // store: lane holds column i, rows rb..rb+3 for each group of four
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    int64_t col = i0 + wave * NT * 32 + nt * 32 + (lane & 31);
    if (col >= k_hi) continue;
    TO *orow = out + (col - out_lo) * (int64_t)ldo + col0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        int rb = (int)r0 + mt * 32 + 8 * g + 4 * (lane >> 5);
        if (rb + 4 <= col_limit) {
#pragma unroll
          for (int q = 0; q < 4; ++q) orow[rb + q] = (TO)acc[mt][nt][4 * g + q];
        }
      }
  }
}

// ------------------------------------------------------- mixing + peaks
// Y[c, n] = sum_k M[c, k] O[n, k] over the concatenated basis; rows 2i and
// 2i+1 (cos, sin) of template i land in the same lane, so |z|^2 and the
// running per-template peak stay in registers.  One workgroup owns whole
// trigger windows of one row tile: the peak of a window is reduced across
// lanes and waves without atomics (larger |z|^2 first, then lower sample).
struct Best {
  float v, re, im;
  int n;
};

__device__ __forceinline__ bool better(float va, int na, float vb, int nb) {
  return va > vb || (va == vb && na < nb);
}

template <typename T, int MT, int NT>
__global__ __launch_bounds__(kThreads) void k_mix_peak(const T *__restrict__ mix, int rows, int kcat,
                                                       int n_templates, const T *__restrict__ ocat,
                                                       int64_t n, float inv_scale, PeakArgs pa,
                                                       int n_rtiles, int64_t n_wgroups) {
  typedef Op<T> O;
  constexpr int BM = 32 * MT, BN = kWaves * 32 * NT;
  constexpr int P = Pitch<T>::value;
  __shared__ __attribute__((aligned(16))) T As[BM * P];
  __shared__ __attribute__((aligned(16))) T Bs[BN * P];
  __shared__ Best red[kWaves][BM / 2];

  // XCD-aware order: the 8 XCDs take workgroups round-robin, so give all row
  // tiles of one window the same XCD and neighbouring slots (shared O rows in L2).
  const int64_t b = blockIdx.x;
  const int xcd = (int)(b & 7);
  const int64_t slot = b >> 3;
  const int rt = (int)(slot % n_rtiles);
  const int64_t wgrp = slot / n_rtiles;
  const int64_t w = wgrp * 8 + xcd;
  if (w >= pa.n_windows) return;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)rt * BM;
  const int64_t ws = (w * pa.win_p) / pa.win_q;
  int64_t we = ((w + 1) * pa.win_p) / pa.win_q;
  if (we > n) we = n;

  Best best[MT][8];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int p = 0; p < 8; ++p) best[mt][p] = Best{-1.f, 0.f, 0.f, 0x7fffffff};

  for (int64_t n0 = ws; n0 < we; n0 += BN) {
    f32x16 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[mt][nt][e] = 0.f;

    for (int kc = 0; kc < kcat; kc += kBK) {
      __syncthreads();
      stage_rows<T, BM, P>(mix, rows, kcat, r0, kc, As);
      stage_rows<T, BN, P>(ocat + n0 * (int64_t)kcat, we - n0, kcat, 0, kc, Bs);
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < kBK / O::KS; ++ks) {
        typename O::vec af[MT], bf[NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          af[mt] = *(const typename O::vec *)(As + (mt * 32 + (lane & 31)) * P + ks * O::KS + (lane >> 5) * O::VEC);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          bf[nt] = *(const typename O::vec *)(Bs + (wave * NT * 32 + nt * 32 + (lane & 31)) * P + ks * O::KS +
                                             (lane >> 5) * O::VEC);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = O::mfma(af[mt], bf[nt], acc[mt][nt]);
      }
    }

    // epilogue: complex SNR of 8 templates per lane per row tile
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int64_t col = n0 + wave * NT * 32 + nt * 32 + (lane & 31);
      const bool ok = col < we;
      const int rel = (int)(col - ws);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          float re = acc[mt][nt][2 * p], im = acc[mt][nt][2 * p + 1];
          float v = re * re + im * im;
          if (ok && v > best[mt][p].v) best[mt][p] = Best{v, re, im, rel};
          if (pa.snr && ok) {
            int64_t i = (r0 + mt * 32 + 8 * (p >> 1) + 4 * (lane >> 5) + 2 * (p & 1)) >> 1;
            if (i < n_templates) {
              float2 z = make_float2(re * inv_scale, im * inv_scale);
              *(float2 *)(pa.snr + (i * n + col) * 2) = z;
            }
          }
        }
    }
  }

  // reduce the 32 columns of each half-wave, then the four waves
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      Best bb = best[mt][p];
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) {
        float ov = __shfl_xor(bb.v, off), ore = __shfl_xor(bb.re, off), oim = __shfl_xor(bb.im, off);
        int on = __shfl_xor(bb.n, off);
        if (better(ov, on, bb.v, bb.n)) bb = Best{ov, ore, oim, on};
      }
      if ((lane & 31) == 0) {
        int t = mt * 16 + 4 * (p >> 1) + 2 * (lane >> 5) + (p & 1);
        red[wave][t] = bb;
      }
    }
  __syncthreads();
  if (threadIdx.x < BM / 2) {
    int t = threadIdx.x;
    Best bb = red[0][t];
    for (int q = 1; q < kWaves; ++q)
      if (better(red[q][t].v, red[q][t].n, bb.v, bb.n)) bb = red[q][t];
    int64_t i = r0 / 2 + t;
    if (i < n_templates) {
      int64_t o = i * pa.n_windows + w;
      pa.peak_snr[o] = sqrtf(fmaxf(bb.v, 0.f)) * inv_scale;
      pa.peak_n[o] = ws + bb.n;
      pa.peak_phase[o] = atan2f(bb.im, bb.re);
    }
  }
}

// ---------------------------------------------------------- trigger compaction

__device__ __forceinline__ int64_t block_sum(int64_t v, int64_t *sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t tot = 0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) tot += sh[q];
  __syncthreads();
  return tot;
}

__global__ void k_trigger_count(const float *__restrict__ snr, int64_t n_windows, float thr,
                                int64_t *__restrict__ counts) {
  __shared__ int64_t sh[16];
  const float *row = snr + (int64_t)blockIdx.x * n_windows;
  int64_t c = 0;
  for (int64_t w = threadIdx.x; w < n_windows; w += blockDim.x) c += row[w] >= thr ? 1 : 0;
  c = block_sum(c, sh);
  if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

// exclusive prefix sum of counts[0..n) in place; total in *total (one block)
__global__ void k_trigger_scan(int64_t *counts, int n, int64_t *total) {
  __shared__ int64_t sh[1024];
  int64_t carry = 0;
  for (int base = 0; base < n; base += blockDim.x) {
    int i = base + threadIdx.x;
    int64_t v = i < n ? counts[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
      int64_t add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < n) counts[i] = carry + sh[threadIdx.x] - v;
    int64_t blk = sh[blockDim.x - 1];
    __syncthreads();
    carry += blk;
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_trigger_write(const float *__restrict__ snr, const int64_t *__restrict__ samp,
                                const float *__restrict__ phase, int64_t n_windows, float thr,
                                const int64_t *__restrict__ offsets, int64_t cap, int32_t bank_id,
                                int32_t detector, lloid_trigger *__restrict__ out) {
  __shared__ int sh[1024];
  const int64_t i = blockIdx.x;
  const float *row = snr + i * n_windows;
  int64_t run = offsets[i];
  for (int64_t base = 0; base < n_windows; base += blockDim.x) {
    int64_t w = base + threadIdx.x;
    int f = (w < n_windows && row[w] >= thr) ? 1 : 0;
    sh[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
      int add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    int64_t pos = run + sh[threadIdx.x] - f;
    if (f && pos < cap) {
      lloid_trigger t;
      t.bank = bank_id;
      t.detector = detector;
      t.template_id = (int32_t)i;
      t.reserved = 0;
      t.window = w;
      t.sample = samp[i * n_windows + w];
      t.snr = row[w];
      t.phase = phase[i * n_windows + w];
      out[pos] = t;
    }
    int blk = sh[blockDim.x - 1];
    __syncthreads();
    run += blk;
  }
}

// ------------------------------------------------------------ launchers

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_convert(const void *src, lloid_dtype dt, int64_t n, float *dst, int64_t dst_lo,
                          int64_t dst_len, float scale, int *bad, hipStream_t s) {
  if (dst_len <= 0) return hipSuccess;
  if (dt == LLOID_F64)
    k_convert<double><<<blocks_for(dst_len, 256), 256, 0, s>>>((const double *)src, n, dst, dst_lo, dst_len,
                                                                 scale, bad);
  else
    k_convert<float><<<blocks_for(dst_len, 256), 256, 0, s>>>((const float *)src, n, dst, dst_lo, dst_len,
                                                                scale, bad);
  return hipGetLastError();
}

hipError_t launch_decimate(const float *u, int64_t u_lo, int64_t u_len, float *d, int64_t d_lo,
                           int64_t d_len, const float *g, hipStream_t s) {
  if (d_len <= 0) return hipSuccess;
  k_decimate<<<blocks_for(d_len, 256), 256, 0, s>>>(u, u_lo, u_len, d, d_lo, d_len, g);
  return hipGetLastError();
}

template <typename T, typename TO>
static hipError_t fir_t(const SliceDev &sl, const float *x, int64_t x_lo, int64_t x_len, int64_t k_lo,
                        int64_t k_hi, void *out, int64_t out_lo, int ldo, int col0, int col_limit,
                        hipStream_t s) {
  constexpr int BM = 32 * kFirMT;
  const int64_t cols = k_hi - k_lo;
  if (cols <= 0) return hipSuccess;
  dim3 grid((unsigned)((cols + kFirBN - 1) / kFirBN), (unsigned)((sl.lrows + BM - 1) / BM));
  const int64_t base = -(sl.start_tap / sl.dec + sl.n_taps - 1);
  k_fir<T, TO, kFirMT, kFirNT><<<grid, kThreads, 0, s>>>((const T *)sl.basis, sl.lrows, sl.np, x, x_lo, x_len,
                                                          base, k_lo, k_hi, (TO *)out, out_lo, ldo, col0,
                                                          col_limit);
  return hipGetLastError();
}

hipError_t launch_fir(lloid_dtype t, const SliceDev &sl, const float *x, int64_t x_lo, int64_t x_len,
                      int64_t k_lo, int64_t k_hi, void *out, int64_t out_lo, int ldo, int col0, int col_limit,
                      hipStream_t s) {
  // level-0 slices write the compute type straight into the concatenated
  // operand; lower-rate slices keep FP32 for the interpolation cascade
  const bool to_f32 = sl.level > 0;
  switch (t) {
    case LLOID_F16:
      return to_f32 ? fir_t<_Float16, float>(sl, x, x_lo, x_len, k_lo, k_hi, out, out_lo, ldo, col0, col_limit, s)
                    : fir_t<_Float16, _Float16>(sl, x, x_lo, x_len, k_lo, k_hi, out, out_lo, ldo, col0, col_limit, s);
    case LLOID_BF16:
      return to_f32 ? fir_t<__bf16, float>(sl, x, x_lo, x_len, k_lo, k_hi, out, out_lo, ldo, col0, col_limit, s)
                    : fir_t<__bf16, __bf16>(sl, x, x_lo, x_len, k_lo, k_hi, out, out_lo, ldo, col0, col_limit, s);
    case LLOID_F32:
      return fir_t<float, float>(sl, x, x_lo, x_len, k_lo, k_hi, out, out_lo, ldo, col0, col_limit, s);
    default:
      return hipErrorInvalidValue;
  }
}

template <typename TI, typename TO>
static hipError_t interp_t(const void *w, int64_t w_lo, int64_t w_len, int ldw, void *v, int64_t v_lo,
                           int64_t v_len, int ldv, int col0, int channels, const float *g, hipStream_t s) {
  const int64_t total = v_len * channels;
  if (total <= 0) return hipSuccess;
  k_interp<TI, TO><<<blocks_for(total, 256), 256, 0, s>>>((const TI *)w, w_lo, w_len, ldw, (TO *)v, v_lo, v_len,
                                                          ldv, col0, channels, g);
  return hipGetLastError();
}

hipError_t launch_interp(lloid_dtype in_t, const void *w, int64_t w_lo, int64_t w_len, int ldw, lloid_dtype out_t,
                         void *v, int64_t v_lo, int64_t v_len, int ldv, int col0, int channels, const float *g,
                         hipStream_t s) {
  if (in_t != LLOID_F32) return hipErrorInvalidValue;
  switch (out_t) {
    case LLOID_F32: return interp_t<float, float>(w, w_lo, w_len, ldw, v, v_lo, v_len, ldv, col0, channels, g, s);
    case LLOID_F16: return interp_t<float, _Float16>(w, w_lo, w_len, ldw, v, v_lo, v_len, ldv, col0, channels, g, s);
    case LLOID_BF16: return interp_t<float, __bf16>(w, w_lo, w_len, ldw, v, v_lo, v_len, ldv, col0, channels, g, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t mix_t(const void *mix, int rows, int kcat, int n_templates, const void *ocat, int64_t n,
                        float inv_scale, const PeakArgs &pa, hipStream_t s) {
  constexpr int BM = 32 * kMixMT;
  const int n_rtiles = (rows + BM - 1) / BM;
  const int64_t n_wgroups = (pa.n_windows + 7) / 8;
  const int64_t blocks = n_wgroups * 8 * n_rtiles;
  if (blocks <= 0) return hipSuccess;
  k_mix_peak<T, kMixMT, kMixNT><<<(unsigned)blocks, kThreads, 0, s>>>((const T *)mix, rows, kcat, n_templates,
                                                                      (const T *)ocat, n, inv_scale, pa, n_rtiles,
                                                                      n_wgroups);
  return hipGetLastError();
}

hipError_t launch_mix_peak(lloid_dtype t, const void *mix, int rows, int kcat, int n_templates, const void *ocat,
                           int64_t n, float inv_scale, const PeakArgs &pa, hipStream_t s) {
  switch (t) {
    case LLOID_F16: return mix_t<_Float16>(mix, rows, kcat, n_templates, ocat, n, inv_scale, pa, s);
    case LLOID_BF16: return mix_t<__bf16>(mix, rows, kcat, n_templates, ocat, n, inv_scale, pa, s);
    case LLOID_F32: return mix_t<float>(mix, rows, kcat, n_templates, ocat, n, inv_scale, pa, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sigma2(const double *mix64, int n_templates, int lsum, const double *inv_dec_per_col,
                         double *out, hipStream_t s) {
  k_sigma2<<<blocks_for(n_templates, 128), 128, 0, s>>>(mix64, n_templates, lsum, inv_dec_per_col, out);
  return hipGetLastError();
}

hipError_t launch_cast_f64(const double *src, lloid_dtype t, void *dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (t) {
    case LLOID_F16: k_cast_f64<_Float16><<<blocks_for(n, 256), 256, 0, s>>>(src, (_Float16 *)dst, n); break;
    case LLOID_BF16: k_cast_f64<__bf16><<<blocks_for(n, 256), 256, 0, s>>>(src, (__bf16 *)dst, n); break;
    case LLOID_F32: k_cast_f64<float><<<blocks_for(n, 256), 256, 0, s>>>(src, (float *)dst, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_u8(void *p, size_t bytes, hipStream_t s) {
  if (!bytes) return hipSuccess;
  unsigned blocks = (unsigned)std::min<size_t>((bytes + 255) / 256, 65536);
  k_fill_u8<<<blocks, 256, 0, s>>>((uint8_t *)p, bytes);
  return hipGetLastError();
}

hipError_t launch_trigger_count(const float *peak_snr, int n_templates, int64_t n_windows, float thr,
                                int64_t *counts, hipStream_t s) {
  if (n_templates <= 0) return hipSuccess;
  k_trigger_count<<<n_templates, 256, 0, s>>>(peak_snr, n_windows, thr, counts);
  return hipGetLastError();
}

hipError_t launch_trigger_scan(int64_t *counts, int n_templates, int64_t *total, hipStream_t s) {
  k_trigger_scan<<<1, 1024, 0, s>>>(counts, n_templates, total);
  return hipGetLastError();
}

hipError_t launch_trigger_write(const float *peak_snr, const int64_t *peak_n, const float *peak_phase,
                                int n_templates, int64_t n_windows, float thr, const int64_t *offsets, int64_t cap,
                                int32_t bank_id, int32_t detector, lloid_trigger *out, hipStream_t s) {
  if (n_templates <= 0) return hipSuccess;
  k_trigger_write<<<n_templates, 1024, 0, s>>>(peak_snr, peak_n, peak_phase, n_windows, thr, offsets, cap, bank_id,
                                                detector, out);
  return hipGetLastError();
}

}  // namespace lloid
