// gfx950 kernels of the LLOID filtering path.
//
// Stages (the method's order, Sec. II.A): strain conversion, half-band
// decimation to every slice rate, the per-slice FIR bank as a sliding-window
// GEMM on MFMA, interpolation of the low-rate orthogonal SNR to the full
// rate, the mixing GEMM over the concatenated basis with a fused complex-SNR
// and per-window peak epilogue, and trigger compaction (Sec. II.B: only the
// triggers leave the device).  FP64 arithmetic appears only in the sigma^2 sums
// (FP64 inputs are converted once).
#include <hip/hip_runtime.h>
#include <type_traits>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <climits>
#include <cstdlib>

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

// Job owning flat work item `item`: the last job with item0 <= item.
template <typename J>
__device__ __forceinline__ int find_job(const J *__restrict__ jobs, int n_jobs, int64_t item) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].item0 <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------- small kernels

template <typename TI>
__global__ void k_convert(const TI *__restrict__ src, int64_t n, float *__restrict__ dst, int64_t dst_lo,
                          int64_t dst_len, float scale, int *__restrict__ bad) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= dst_len) return;
  int64_t a = dst_lo + t;
  float v = 0.f;
  if (a >= 0 && a < n) {
    // FP32 from here on: the scale is a power of two, so the product is the
    // scaled value rounded once; a sample that is not finite in FP32 is flagged
    v = (float)src[a] * scale;
    if (!isfinite(v)) {
      atomicOr(bad, 1);
      v = 0.f;
    }
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

template <typename T, int BK = kBK> struct Pitch {
  // row pitch of an LDS tile in elements: +16 bytes keeps the 16-byte fragment
  // reads of 8 consecutive rows on distinct banks; FP32 fragments are single
  // words, so one extra word per row does the same
  static constexpr int value = sizeof(T) == 4 ? BK + 1 : BK + 16 / (int)sizeof(T);
};

// Buffer resource over `bytes` bytes from `base`: loads past the end (or at
// negative offsets, which wrap to huge unsigned ones) return zero in hardware.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, int64_t bytes) {
  const int nb = bytes <= 0 ? 0 : (bytes > 0x7ffffff0 ? 0x7ffffff0 : (int)bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, nb, 0x00020000);
}

// Register-staged copy of a [ROWS][BK] chunk of a row-major matrix through a
// buffer resource: setup() fixes each thread's byte offsets, load(k0) issues
// the 16-byte global reads for columns [k0, k0 + BK) (rows past the resource
// read as zero), store() writes them to LDS.
template <typename T, int ROWS, int BK = kBK, int THREADS = kThreads> struct ChunkLoader {
  static constexpr int EPV = 16 / (int)sizeof(T);   // elements per 16-byte vector
  static constexpr int VPR = BK / EPV;               // vectors per row
  static constexpr int NV = ROWS * VPR;
  static constexpr int PER = (NV + THREADS - 1) / THREADS;
  uint4 r[PER];
  int voff[PER];

  __device__ __forceinline__ void setup(int ld) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int v = threadIdx.x + p * THREADS;
      voff[p] = v < NV ? ((v / VPR) * ld + (v % VPR) * EPV) * (int)sizeof(T) : 0x7ffffff0;
    }
  }
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, int soff_bytes) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff[p], soff_bytes, 0);
      r[p] = make_uint4(v[0], v[1], v[2], v[3]);
    }
  }
  __device__ __forceinline__ void store(T *lds) const {
    constexpr int P = Pitch<T, BK>::value;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int v = threadIdx.x + p * THREADS;
      if (NV % THREADS != 0 && v >= NV) break;
      const int row = v / VPR, c = v % VPR;
      if constexpr (sizeof(T) == 4) {
        float *d = (float *)lds + row * P + c * 4;
        d[0] = __uint_as_float(r[p].x);
        d[1] = __uint_as_float(r[p].y);
        d[2] = __uint_as_float(r[p].z);
        d[3] = __uint_as_float(r[p].w);
      } else {
        *(uint4 *)(lds + row * P + c * EPV) = r[p];
      }
    }
  }
};

// ---------------------------------------------------------------- FIR
// o[l, k] = sum_m U[l, m] x[k - J/D - m] as D = A B with A = taps reversed
// (Ar[l, m'] = U[l, N-1-m']) and the Hankel operand B[m', k] = x[k + m' + base],
// base = -(J/D + N - 1).  The four waves share the basis rows of the
// workgroup and split its columns.  The strain window of kFirKSup taps sits
// in LDS as VEC copies shifted by 0..VEC-1 samples, so every lane's VEC
// consecutive samples are one aligned read whatever its column; the basis
// streams through double-buffered LDS with the next chunk's global reads in
// flight during the current chunk's MFMAs.
// HR (16-bit operands): the Hankel operand repeats itself shifted, so the
// fragment of column block nt at k-step g is that of block 0 at k-step
// g + 2 nt (32 columns = 2 k-steps of 16 taps).  Each wave then keeps, per
// k-step parity, a window of NT fragments in registers and reads one new
// fragment from LDS per k-step instead of NT.
template <typename T, int MT, int NT, int NW, int BK, bool HR = false>
__global__ __launch_bounds__(64 * NW, NW == 4 ? 2 : 1) void k_fir(const FirJob *__restrict__ jobs, int n_jobs) {
  typedef Op<T> O;
  static_assert(!HR || O::KS == 16, "the fragment window needs 16 taps per k-step");
  constexpr int THREADS = 64 * NW;
  constexpr int BM = 32 * MT, BN = NW * 32 * NT;
  constexpr int P = Pitch<T, BK>::value;
  // strain window: BN columns + kFirKSup taps (+ the fragments the HR window
  // reads ahead past its last k-step).  With 16-bit operands the copies are
  // padded to WC = 32 mod 64 elements: the 16-byte fragment reads, each lane
  // in its own copy, then run without LDS bank conflicts (the bank-conflict
  // counter reads zero there; at 0, 16, 40 and 48 mod 64 it does not)
  constexpr int WC0 = BN + kFirKSup + 16 + (HR ? 2 * NT * 16 : 0);
  constexpr int WC = O::VEC == 8 ? (WC0 + 31) / 64 * 64 + 32 : WC0;
  __shared__ __attribute__((aligned(16))) T As[2][BM * P];
  __shared__ __attribute__((aligned(16))) T Bc[O::VEC * WC];

  const FirJob &jb = jobs[find_job(jobs, n_jobs, blockIdx.x)];
  const int64_t li = (int64_t)blockIdx.x - jb.item0;
  const int rows = jb.rows, np = jb.np;
  const T *a = (const T *)jb.basis;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (li % jb.n_rtiles) * BM;
  const int64_t i0 = jb.k_lo + (li / jb.n_rtiles) * BN;

  f32x16 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[mt][nt][e] = 0.f;

  // basis rows [r0, rows) of this workgroup; strain samples [0, x_len)
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(a + r0 * np, (rows - r0) * (int64_t)np * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(jb.x, jb.x_len * 4);
  const int64_t x_len = jb.x_len;
  ChunkLoader<T, BM, BK, THREADS> la;
  la.setup(np);
  la.load(ra, 0);
  // np is a multiple of kBK; with BK = 2 kBK the last chunk may hold one
  // valid half (the k-steps past np are skipped, whatever the loads brought)
  const int nchunks = (np + BK - 1) / BK;
  // lane's shifted copy: its column offset within a fragment is constant mod VEC
  const int lr = (lane & 31) % O::VEC;
  const T *bl = Bc + lr * WC + (wave * NT * 32 + (lane & 31) + (lane >> 5) * O::VEC - lr);
  // 32-column fragments of this wave that start before k_hi: a wave wholly
  // past the end of a ragged last tile skips its MFMAs (it still loads and
  // syncs); the HR window needs all NT fragments, so a partly live wave takes
  // the plain k-steps
  const int64_t wcol = i0 + wave * NT * 32;
  const int live = (int)(jb.k_hi <= wcol ? 0 : std::min<int64_t>(NT, (jb.k_hi - wcol + 31) / 32));
  int ksup = 0;
  typename O::vec hw[2][HR ? NT : 1];   // HR: fragment windows of the even and odd k-steps
  for (int c = 0; c < nchunks; ++c) {
    const int cur = c & 1, kc = c * BK;
    if (kc % kFirKSup == 0) {
      // new strain window for taps [kc, kc + kFirKSup); out-of-range samples read as zero
      if (c > 0) __syncthreads();
      ksup = kc;
      // copy r holds x[w0 + t + r] at t: a thread takes G consecutive
      // positions of every copy, issues the G + VEC - 1 sample reads it needs
      // back to back, and writes each copy's G values as one 16-byte store
      const int64_t w0 = i0 + kc + jb.base - jb.x_lo;
      constexpr int G = 16 / (int)sizeof(T);
      static_assert(WC % G == 0, "the strain window is whole 16-byte units");
      for (int t0 = threadIdx.x * G; t0 < WC; t0 += THREADS * G) {
        float v[G + O::VEC - 1];
#pragma unroll
        for (int u = 0; u < G + O::VEC - 1; ++u) {
          const int64_t idx = w0 + t0 + u;
          const int off = (idx >= 0 && idx < x_len) ? (int)idx * 4 : -4;
          v[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, off, 0, 0));
        }
#pragma unroll
        for (int r = 0; r < O::VEC; ++r) {
          T h[G];
#pragma unroll
          for (int g = 0; g < G; ++g) h[g] = O::cvt(v[r + g]);
          *(uint4 *)(Bc + r * WC + t0) = __builtin_bit_cast(uint4, h);
        }
      }
    }
    la.store(As[cur]);
    __syncthreads();
    if (c + 1 < nchunks) la.load(ra, (kc + BK) * (int)sizeof(T));
    auto ksteps = [&]() __attribute__((always_inline)) {
#pragma unroll
      for (int ks = 0; ks < BK / O::KS; ++ks) {
        if (BK > kBK && kc + ks * O::KS >= np) break;
        typename O::vec af[MT], bf[NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          af[mt] = *(const typename O::vec *)(As[cur] + (mt * 32 + (lane & 31)) * P + ks * O::KS + (lane >> 5) * O::VEC);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) bf[nt] = *(const typename O::vec *)(bl + (kc - ksup) + nt * 32 + ks * O::KS);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = O::mfma(af[mt], bf[nt], acc[mt][nt]);
      }
    };
    if constexpr (HR) {
      if (live == NT) {
        // F(j): block-0 fragment j k-steps into the strain window
        auto F = [&](int j) __attribute__((always_inline)) {
          return *(const typename O::vec *)(bl + j * O::KS);
        };
        const int g0 = (kc - ksup) / O::KS;
        if (kc == ksup) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            hw[0][nt] = F(2 * nt);
            hw[1][nt] = F(1 + 2 * nt);
          }
        }
#pragma unroll
        for (int ks = 0; ks < BK / O::KS; ++ks) {
          if (BK > kBK && kc + ks * O::KS >= np) break;
          typename O::vec af[MT];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            af[mt] = *(const typename O::vec *)(As[cur] + (mt * 32 + (lane & 31)) * P + ks * O::KS +
                                                 (lane >> 5) * O::VEC);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = O::mfma(af[mt], hw[ks & 1][nt], acc[mt][nt]);
          // this parity's next k-step (g + 2) needs blocks shifted by one
#pragma unroll
          for (int nt = 0; nt + 1 < NT; ++nt) hw[ks & 1][nt] = hw[ks & 1][nt + 1];
          hw[ks & 1][NT - 1] = F(g0 + ks + 2 * NT);
        }
      } else if (live > 0) {
        ksteps();
      }
    } else {
      if (live > 0) ksteps();
    }
  }

  // store: lane holds column i, rows rb..rb+3 for each group of four; level-0
  // slices write the time-major operand, lower-rate slices a channel-major
  // buffer for the interpolation (FP32 when the operand type is BF16)
  const int col_limit = jb.col_limit, ldo = jb.ldo;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int64_t col = i0 + wave * NT * 32 + nt * 32 + (lane & 31);
    if (col >= jb.k_hi) continue;
    const int64_t ro = (col - jb.out_lo) * (int64_t)ldo + jb.col0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int rb = (int)r0 + mt * 32 + 8 * g + 4 * (lane >> 5);
        if (rb + 4 <= col_limit) {
          if (jb.out_cm && jb.out_f32) {
            float *o = (float *)jb.out + (col - jb.out_lo);
#pragma unroll
            for (int q = 0; q < 4; ++q) o[(int64_t)(rb + q) * ldo] = acc[mt][nt][4 * g + q];
          } else if (jb.out_cm) {
            T *o = (T *)jb.out + (col - jb.out_lo);
#pragma unroll
            for (int q = 0; q < 4; ++q) o[(int64_t)(rb + q) * ldo] = O::cvt(acc[mt][nt][4 * g + q]);
          } else if (jb.out_f32) {
            float *o = (float *)jb.out + ro + rb;
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = acc[mt][nt][4 * g + q];
          } else {
            T *o = (T *)jb.out + ro + rb;
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = O::cvt(acc[mt][nt][4 * g + q]);
          }
        }
      }
  }
}

// ----------------------------------------------------- interpolation on MFMA
// One or two half-band x2 stages as one composite filter h_R (R = 2 or 4):
// out[c][n] = sum_u src[c][u] h_R[n - R u].  For a 32-sample output tile at n0
// (a multiple of 32) the taps that matter are u = U0 + kk, kk < 64, with
// U0 = n0 / R - (32 - 32 / R), and H[kk][t] = h_R[t - R kk + 32 R - 32] is the
// same matrix for every tile: it stays in registers as MFMA fragments while
// the channel-major source rows stream in.  A hop into a channel-major buffer
// computes D[c][t] (source rows as the A operand); the last hop, into the
// time-major mixing operand, computes D[t][c] with the operands swapped, so
// each store instruction writes 32 consecutive channels of two samples.
// TS: source and low-rate buffer type; TD: operand type of the last hop.
// The fragment of tile t at k-step ks is the VEC-sample block 2 ks + SB t
// past the lane's first one (the tiles' source windows start 32 / R = SB VEC
// samples apart), so a lane reads each block of its source window that the
// MFMAs use once, all reads issued before the MFMAs.  With SB even only the
// even blocks are used.
template <typename TS, bool TM, int SB>
__device__ __forceinline__ void upsample_blocks(__amdgpu_buffer_rsrc_t rs, int64_t base0,
                                                const typename Op<TS>::vec *hfr, f32x16 *acc) {
  typedef Op<TS> O;
  static_assert(O::KS == 2 * O::VEC, "two VEC blocks per k-step");
  constexpr int NKS = 64 / O::KS, CT = kUpCols / 32;
  constexpr int NB = 2 * (NKS - 1) + SB * (CT - 1) + 1;
  typename O::vec blk[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (SB % 2 == 0 && (j & 1)) continue;
    const int off = (int)((base0 + j * O::VEC) * (int64_t)sizeof(TS));
    if constexpr (O::VEC == 8)
      blk[j] = __builtin_bit_cast(typename O::vec, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    else
      blk[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
  }
  __builtin_amdgcn_sched_barrier(0);   // keep every read ahead of the MFMAs
#pragma unroll
  for (int t = 0; t < CT; ++t) {
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[t][e] = 0.f;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const typename O::vec a = blk[2 * ks + SB * t];
      acc[t] = TM ? O::mfma(hfr[ks], a, acc[t]) : O::mfma(a, hfr[ks], acc[t]);
    }
  }
}

// FP32 sources of the BF16 operand path: every source value x and filter
// tap h is split into a BF16 pair, x = x_hi + x_lo with x_hi = bf16(x) and
// x_lo = bf16(x - x_hi) (16 significant bits), and a product takes three
// BF16 MFMAs, x_hi h_hi + x_lo h_hi + x_hi h_lo (the dropped x_lo h_lo and
// the splits' remainders are of order 2^-16 relative), with FP32 sums: the
// 32x32x16 instruction in place of eight FP32 32x32x2 ones per k-step.
// Blocks are 8 source samples (two 16-byte reads), laid out as for 16-bit
// sources; hf holds the filter's hi fragments, then its lo fragments.
struct uint4x2 {
  __attribute__((ext_vector_type(4))) unsigned int a, b;
};

template <bool TM, int SB>
__device__ __forceinline__ void upsample_blocks_split(__amdgpu_buffer_rsrc_t rs, int64_t base0, const bf16x8 *hhi,
                                                      const bf16x8 *hlo, f32x16 *acc) {
  constexpr int NKS = 4, CT = kUpCols / 32;
  constexpr int NB = 2 * (NKS - 1) + SB * (CT - 1) + 1;
  typedef float f32x8 __attribute__((ext_vector_type(8)));
  f32x8 raw[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (SB % 2 == 0 && (j & 1)) continue;
    const int off = (int)((base0 + j * 8) * (int64_t)sizeof(float));
    const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    const auto v1 = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, 0, 0);
    raw[j] = __builtin_bit_cast(f32x8, (uint4x2{v0, v1}));
  }
  __builtin_amdgcn_sched_barrier(0);   // keep every read ahead of the MFMAs
  bf16x8 xhi[NB], xlo[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (SB % 2 == 0 && (j & 1)) continue;
    __bf16 h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      h[e] = (__bf16)raw[j][e];
      l[e] = (__bf16)(raw[j][e] - (float)h[e]);
    }
    xhi[j] = __builtin_bit_cast(bf16x8, h);
    xlo[j] = __builtin_bit_cast(bf16x8, l);
  }
#pragma unroll
  for (int t = 0; t < CT; ++t) {
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[t][e] = 0.f;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int j = 2 * ks + SB * t;
      if (TM) {
        acc[t] = Op<__bf16>::mfma(hlo[ks], xhi[j], acc[t]);
        acc[t] = Op<__bf16>::mfma(hhi[ks], xlo[j], acc[t]);
        acc[t] = Op<__bf16>::mfma(hhi[ks], xhi[j], acc[t]);
      } else {
        acc[t] = Op<__bf16>::mfma(xhi[j], hlo[ks], acc[t]);
        acc[t] = Op<__bf16>::mfma(xlo[j], hhi[ks], acc[t]);
        acc[t] = Op<__bf16>::mfma(xhi[j], hhi[ks], acc[t]);
      }
    }
  }
}

template <typename TS, typename TD, bool TM>
__device__ __forceinline__ void upsample_task(const UpJob &jb, int lane, int r0, int64_t n0) {
  typedef Op<TS> O;
  constexpr int NKS = 64 / O::KS;  // k-steps over the 64 composite taps
  constexpr int CT = kUpCols / 32; // 32-sample tiles per task
  const int R = jb.r;
  const int lgR = R == 4 ? 2 : 1;  // R is 2 or 4: shifts, not 64-bit divisions (their
                                   // branches would keep the tiles' reads apart)
  // FP32 sources feeding BF16 operands take the split-BF16 products
  constexpr bool SPLIT = std::is_same<TS, float>::value && std::is_same<TD, __bf16>::value;
  const int cR = 32 - 32 / R;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(jb.src, jb.src_bytes);
  const int64_t rowoff = (int64_t)(r0 + (lane & 31)) * jb.ld_src;
  f32x16 acc[CT];
  if constexpr (SPLIT) {
    const __bf16 *hf = (const __bf16 *)jb.hf;
    bf16x8 hhi[4], hlo[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      hhi[ks] = *(const bf16x8 *)(hf + (ks * 64 + lane) * 8);
      hlo[ks] = *(const bf16x8 *)(hf + kInterpFragEntries + (ks * 64 + lane) * 8);
    }
    const int64_t base0 = rowoff + (((n0 >> lgR) - cR) - jb.src_lo) + (lane >> 5) * 8;
    if (R == 4) upsample_blocks_split<TM, 1>(rs, base0, hhi, hlo, acc);
    else upsample_blocks_split<TM, 2>(rs, base0, hhi, hlo, acc);
  } else {
    const TS *hf = (const TS *)jb.hf;
    typename O::vec hfr[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) hfr[ks] = *(const typename O::vec *)(hf + (ks * 64 + lane) * O::VEC);
    const int64_t base0 = rowoff + (((n0 >> lgR) - cR) - jb.src_lo) + (lane >> 5) * O::VEC;
    constexpr int SB4 = 8 / O::VEC;   // 32 / R in VEC blocks for R = 4; twice that for R = 2
    if (R == 4) upsample_blocks<TS, TM, SB4>(rs, base0, hfr, acc);
    else upsample_blocks<TS, TM, 2 * SB4>(rs, base0, hfr, acc);
  }
  if constexpr (TM) {
    // lane holds channel r0 + lane % 32 at samples n0 + 32 t + 8 g + 4 (lane / 32) + q
    const int c = r0 + (lane & 31);
    if (c >= jb.channels) return;
    TD *d = (TD *)jb.dst + jb.col0 + c;
#pragma unroll
    for (int t = 0; t < CT; ++t)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t n = n0 + 32 * t + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        if (n >= jb.n_lo && n < jb.n_hi) d[(n - jb.dst_abs0) * jb.ld_dst] = Op<TD>::cvt(acc[t][e]);
      }
  } else {
    // lane holds sample n0 + 32 t + lane % 32 of channels r0 + 8 g + 4 (lane / 32) + q;
    // channels is a multiple of 16, so a lane's four channels are all in or all out
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int64_t n = n0 + 32 * t + (lane & 31);
      if (n < jb.n_lo || n >= jb.n_hi) continue;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int rb = r0 + 8 * g + 4 * (lane >> 5);
        if (rb >= jb.channels) continue;
        TS *d = (TS *)jb.dst + (int64_t)rb * jb.ld_dst + (n - jb.dst_abs0);
#pragma unroll
        for (int q = 0; q < 4; ++q) d[(int64_t)q * jb.ld_dst] = O::cvt(acc[t][4 * g + q]);
      }
    }
  }
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_upsample(const UpJob *__restrict__ jobs, int n_jobs) {
  const UpJob &jb = jobs[find_job(jobs, n_jobs, blockIdx.x)];
  // The 8 XCDs take workgroups round-robin and every job's items start at a
  // multiple of 8: give each XCD one contiguous run of the job's tasks, so
  // neighbouring column tiles (whose source windows overlap) share one L2.
  const int64_t n_tasks = (int64_t)jb.n_rtiles * jb.n_ctiles;
  const int64_t per_xcd = (n_tasks + 31) / 32;          // items per XCD, 4 tasks each
  const int64_t b = (int64_t)blockIdx.x - jb.item0;
  const int64_t li = (b & 7) * per_xcd + (b >> 3);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave task: 32 channels x kUpCols output samples
  const int64_t task = li * 4 + wave;
  if (task >= n_tasks) return;
  const int r0 = (int)(task % jb.n_rtiles) * 32;
  const int64_t n0 = jb.n_first + (task / jb.n_rtiles) * kUpCols;
  if (jb.dst_tm) upsample_task<TS, TD, true>(jb, lane, r0, n0);
  else upsample_task<TS, TD, false>(jb, lane, r0, n0);
}

// ------------------------------------------------------- mixing + peaks
// Y[c, n] = sum_k M[c, k] O[n, k] over the concatenated basis; rows 2i and
// 2i+1 (cos, sin) of template i land in the same lane, so |z|^2 and the
// running per-template peak (value, sample) stay in registers.  One
// workgroup owns whole trigger windows of one row tile: the peak of a
// window is reduced across lanes and waves without atomics (larger |z|^2
// first, then lower sample).  The phase at the peak is recomputed by
// k_peak_phase from the same operands.
__device__ __forceinline__ bool better(float va, int na, float vb, int nb) {
  return va > vb || (va == vb && na < nb);
}

struct VN {
  float v;
  int n;
};

template <typename T, int MT, int NT, int WM, int WN, int BK, bool SNR>
__global__ __launch_bounds__(64 * WM * WN) void k_mix_peak(const MixJob *__restrict__ jobs, int n_jobs) {
  typedef Op<T> O;
  constexpr int THREADS = 64 * WM * WN;
  constexpr int BM = 32 * MT * WM, BN = 32 * NT * WN;
  constexpr int P = Pitch<T, BK>::value;
  __shared__ __attribute__((aligned(16))) T As[2][BM * P];
  __shared__ __attribute__((aligned(16))) T Bs[2][BN * P];
  __shared__ VN red[WN][BM / 2];

  const MixJob &jb = jobs[find_job(jobs, n_jobs, blockIdx.x)];
  // XCD-aware order: the 8 XCDs take workgroups round-robin (every job's items
  // start at a multiple of 8), so give all row tiles of one window the same
  // XCD and neighbouring slots (shared operand rows in that XCD's L2).  A job
  // of fewer than 8 windows would leave XCDs idle that way: its items run
  // window-major over the row tiles instead, spread over all XCDs.
  const int64_t b = (int64_t)blockIdx.x - jb.item0;
  const int n_rtiles = jb.n_rtiles;
  int rt;
  int64_t wl;   // window within the job
  if (jb.nw >= 8) {
    const int64_t slot = b >> 3;
    rt = (int)(slot % n_rtiles);
    wl = (slot / n_rtiles) * 8 + (b & 7);
  } else {
    rt = (int)(b % n_rtiles);
    wl = b / n_rtiles;
  }
  if (wl >= jb.nw) return;
  const int64_t w = jb.w0 + wl;
  const T *mix = (const T *)jb.mix;
  const int rows = jb.rows, kcat = jb.kcat, kld = jb.kld, n_templates = jb.n_templates;
  const float inv_scale = jb.inv_scale;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t r0 = (int64_t)rt * BM;
  const int64_t ws = (w * jb.win_p) / jb.win_q;
  int64_t we = ((w + 1) * jb.win_p) / jb.win_q;
  if (we > jb.n_end) we = jb.n_end;
  const T *ocat = (const T *)jb.ocat + (ws - jb.ocat_abs0) * (int64_t)kld;   // row of sample ws
  VN best[MT][8];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int p = 0; p < 8; ++p) best[mt][p] = VN{-1.f, 0x7fffffff};

  // mixing rows [r0, rows) and operand rows [ws, we) of this workgroup; rows
  // past either end read as zero
  constexpr int ESZ = (int)sizeof(T);
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(mix + r0 * kld, (rows - r0) * (int64_t)kld * ESZ);
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(ocat, (we - ws) * (int64_t)kld * ESZ);
  // kcat is a multiple of 32; with BK = 64 the k-steps past kcat are skipped
  // (the rows' pitch kld is a multiple of 64: the chunks stay inside a row)
  const int nchunks = (kcat + BK - 1) / BK;
  ChunkLoader<T, BM, BK, THREADS> la;
  ChunkLoader<T, BN, BK, THREADS> lb;
  la.setup(kld);
  lb.setup(kld);
  la.load(ra, 0);
  lb.load(rb, 0);
  int it = 0;  // chunk counter across column steps: LDS buffer parity
  for (int64_t n0 = ws; n0 < we; n0 += BN) {
    const int brow = (int)(n0 - ws) * kld * ESZ;   // byte offset of this step's first operand row
    f32x16 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[mt][nt][e] = 0.f;

    for (int c = 0; c < nchunks; ++c, ++it) {
      const int cur = it & 1;
      la.store(As[cur]);
      lb.store(Bs[cur]);
      __syncthreads();
      if (c + 1 < nchunks) {
        la.load(ra, (c + 1) * BK * ESZ);
        lb.load(rb, brow + (c + 1) * BK * ESZ);
      } else if (n0 + BN < we) {
        la.load(ra, 0);
        lb.load(rb, brow + BN * kld * ESZ);
      }
#pragma unroll
      for (int ks = 0; ks < BK / O::KS; ++ks) {
        if (BK > 32 && c * BK + ks * O::KS >= kcat) break;
        typename O::vec af[MT], bf[NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          af[mt] = *(const typename O::vec *)(As[cur] + (wm * 32 * MT + mt * 32 + (lane & 31)) * P + ks * O::KS +
                                             (lane >> 5) * O::VEC);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          bf[nt] = *(const typename O::vec *)(Bs[cur] + (wn * 32 * NT + nt * 32 + (lane & 31)) * P + ks * O::KS +
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
      const int64_t col = n0 + wn * 32 * NT + nt * 32 + (lane & 31);
      const bool ok = col < we;
      const int rel = (int)(col - ws);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const float re = acc[mt][nt][2 * p], im = acc[mt][nt][2 * p + 1];
          const float v = re * re + im * im;
          if (ok && v > best[mt][p].v) best[mt][p] = VN{v, rel};
          if (SNR && ok) {
            const int64_t i = (r0 + wm * 32 * MT + mt * 32 + 8 * (p >> 1) + 4 * (lane >> 5) + 2 * (p & 1)) >> 1;
            if (i < n_templates) {
              // written once and not read here: a non-temporal store
              typedef float fv2 __attribute__((ext_vector_type(2)));
              __builtin_nontemporal_store(fv2{re * inv_scale, im * inv_scale},
                                          (fv2 *)(jb.snr + (i * jb.snr_ld + (col - jb.snr_abs0)) * 2));
            }
          }
        }
      }
    }
  }

  // reduce the 32 columns of each half-wave, then the waves that share rows
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      VN bb = best[mt][p];
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) {
        const float ov = __shfl_xor(bb.v, off);
        const int on = __shfl_xor(bb.n, off);
        if (better(ov, on, bb.v, bb.n)) bb = VN{ov, on};
      }
      if ((lane & 31) == 0) red[wn][wm * 16 * MT + mt * 16 + 4 * (p >> 1) + 2 * (lane >> 5) + (p & 1)] = bb;
    }
  __syncthreads();
  for (int t = threadIdx.x; t < BM / 2; t += THREADS) {
    VN bb = red[0][t];
#pragma unroll
    for (int q = 1; q < WN; ++q)
      if (better(red[q][t].v, red[q][t].n, bb.v, bb.n)) bb = red[q][t];
    const int64_t i = r0 / 2 + t;
    if (i < n_templates) {
      const int64_t o = i * jb.ld_peak + (w - jb.w_base);
      jb.peak_snr[o] = sqrtf(fmaxf(bb.v, 0.f)) * inv_scale;
      jb.peak_n[o] = ws + bb.n;
    }
  }
}

// 16-bit operands, direct-to-LDS form of the mixing kernel.  The operand
// chunks go from global memory straight into LDS (16-byte buffer loads with
// an LDS destination: no staging registers, no LDS store instructions), two
// buffers; rows past either matrix's end read as zero.  An LDS row holds BK
// elements in 16-byte chunks, chunk q of row r at position
// q ^ ((r / (16 / CPR)) % CPR) (CPR chunks per row), so the 16 rows that 16
// lanes read in one fragment load start on distinct banks.  Each output's K
// sum runs in the same order as in k_mix_peak, so the results are
// bit-identical.  The compiled shape: 256 x 256 tiles of eight 64 x 128
// waves, K chunks of 64 (128 KiB of LDS, one workgroup per CU).  Measured and
// not kept: four 128 x 128 waves (one wave per SIMD: its 256 accumulators
// leave the epilogue spilling, 7.6 against 4.0 ms per 1024-template
// detector-call) and two independent workgroups of 128 x 256 per CU with K
// chunks of 32 (4.9 ms).
template <int BK> struct DlRow {
  static constexpr int BYTES = 2 * BK, CPR = BYTES / 16, RPI = 1024 / BYTES;   // RPI: rows per load instruction
  static __device__ __forceinline__ int swz(int row, int q) { return q ^ ((row / (16 / CPR)) % CPR); }
};

typedef __attribute__((address_space(3))) void lds_void;

// Fragments of one k-step: MT A fragments (mixing rows wm*32*MT + mt*32 +
// lane%32) and NT B fragments (operand rows wn*32*NT + nt*32 + lane%32), 8
// consecutive k values from 16 ks + 8 (lane/32).
template <typename T, int BK, int MT, int NT>
__device__ __forceinline__ void dl_frags(const char *a, const char *b, int wm, int wn, int fr, int fh, int ks,
                                         typename Op<T>::vec (&af)[MT], typename Op<T>::vec (&bf)[NT]) {
  typedef DlRow<BK> R;
  const int qc = 2 * ks + fh;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int row = wm * 32 * MT + mt * 32 + fr;
    af[mt] = *(const typename Op<T>::vec *)(a + row * R::BYTES + R::swz(row, qc) * 16);
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int row = wn * 32 * NT + nt * 32 + fr;
    bf[nt] = *(const typename Op<T>::vec *)(b + row * R::BYTES + R::swz(row, qc) * 16);
  }
}

// FIRST: the first k-step of a column step, whose accumulators start at zero
// (the zero is the MFMA's constant operand, no register clearing)
template <typename T, int MT, int NT, bool FIRST = false>
__device__ __forceinline__ void dl_mfmas(const typename Op<T>::vec (&af)[MT], const typename Op<T>::vec (&bf)[NT],
                                         f32x16 (&acc)[MT][NT]) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      acc[mt][nt] = Op<T>::mfma(af[mt], bf[nt], FIRST ? f32x16{} : acc[mt][nt]);
}

// Schedule: the chunks of all column steps of the window form one sequence
// g = 0, 1, ...  (chunk c = g % nchunks of column step g / nchunks).  Within
// a chunk, the fragments of k-step ks + 1 are read while the MFMAs of ks
// run; before the MFMAs of the last k-step, every wave waits for the next
// chunk's loads and meets at the barrier, then reads the next chunk's first
// fragments and starts the loads of the chunk after it into the buffer just
// finished, and only then issues the last k-step's MFMAs.  With K chunks of
// 64 and kcat an odd multiple of 32, the last chunk of a column step holds 2
// k-steps: its upper 32 columns are loaded as out-of-range (zeros) for both
// operands, so the 4 k-steps always run and the extra products are exact
// zeros.  Waves: WM x WN, each 32 MT rows x 32 NT columns; WGS workgroups per
// CU.
template <typename T, int WM, int WN, int MT, int NT, int BK, int WGS, bool SNR>
__global__ __launch_bounds__(64 * WM * WN, WGS) void k_mix_dl(const MixJob *__restrict__ jobs, int n_jobs) {
  static_assert(sizeof(T) == 2, "16-bit operands only");
  typedef typename Op<T>::vec vec;
  typedef DlRow<BK> R;
  constexpr int NW = WM * WN, THREADS = 64 * NW;
  constexpr int BM = 32 * MT * WM, BN = 32 * NT * WN;
  constexpr int KS = BK / 16;                  // k-steps per chunk
  constexpr int JA = BM / R::RPI / NW, JB = BN / R::RPI / NW;   // load instructions per wave and chunk
  static_assert(JA * R::RPI * NW == BM && JB * R::RPI * NW == BN, "whole load instructions per wave");
  static_assert((R::RPI * NW) % 16 == 0, "one voffset per wave");
  static_assert(KS == 2 || KS == 4, "chunks of 32 or 64");
  __shared__ __attribute__((aligned(1024))) char As0[BM * R::BYTES];
  __shared__ __attribute__((aligned(1024))) char Bs0[BN * R::BYTES];
  __shared__ __attribute__((aligned(1024))) char As1[BM * R::BYTES];
  __shared__ __attribute__((aligned(1024))) char Bs1[BN * R::BYTES];
  __shared__ VN red[WN][BM / 2];

  const MixJob &jb = jobs[find_job(jobs, n_jobs, blockIdx.x)];
  const int64_t b = (int64_t)blockIdx.x - jb.item0;
  const int n_rtiles = jb.n_rtiles;
  int rt;
  int64_t wl;
  if (jb.nw >= 8) {
    const int64_t slot = b >> 3;
    rt = (int)(slot % n_rtiles);
    wl = (slot / n_rtiles) * 8 + (b & 7);
  } else {
    rt = (int)(b % n_rtiles);
    wl = b / n_rtiles;
  }
  if (wl >= jb.nw) return;
  const int64_t w = jb.w0 + wl;
  const T *mix = (const T *)jb.mix;
  const int rows = jb.rows, kcat = jb.kcat, kld = jb.kld, n_templates = jb.n_templates;
  const float inv_scale = jb.inv_scale;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const int64_t r0 = (int64_t)rt * BM;
  const int64_t ws = (w * jb.win_p) / jb.win_q;
  int64_t we = ((w + 1) * jb.win_p) / jb.win_q;
  if (we > jb.n_end) we = jb.n_end;
  const T *ocat = (const T *)jb.ocat + (ws - jb.ocat_abs0) * (int64_t)kld;
  VN best[MT][8];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int p = 0; p < 8; ++p) best[mt][p] = VN{-1.f, 0x7fffffff};

  constexpr int ESZ = 2;
  // rows of pitch kld (a multiple of 64 elements: every chunk row is one
  // 128-byte line of a line-aligned row)
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(mix + r0 * kld, (rows - r0) * (int64_t)kld * ESZ);
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(ocat, (we - ws) * (int64_t)kld * ESZ);
  const int nchunks = (kcat + BK - 1) / BK;
  const bool half_tail = (kcat % BK) != 0;   // K chunks of 64: the last one holds 32 columns
  const int nsteps = (int)((we - ws + BN - 1) / BN);
  const int G = nsteps * nchunks;
  // Load instruction j of this wave fills LDS rows RPI (NW j + wave) .. + RPI - 1
  // of a tile, lane i the 16-byte position i % CPR of row RPI (NW j + wave) +
  // i / CPR: logical chunk swz(row, i % CPR), the same for every j (the row
  // step is a multiple of 16 rows), so one voffset serves every instruction
  // and the row step goes into the scalar offset.
  const int vrow = R::RPI * wave + lane / R::CPR;
  const int lq = R::swz(vrow, lane % R::CPR);
  const int voffs = vrow * kld * ESZ + lq * 16;
  const int voffs_tail = lq < R::CPR / 2 ? voffs : 0x7ff00000;   // upper half of a half chunk: zeros
  const int jstep = R::RPI * NW * kld * ESZ;
  auto issue = [&](int g) {
    const int c = g % nchunks, st = g / nchunks;
    const int ka = c * BK * ESZ;
    const int kb = st * BN * kld * ESZ + ka;
    const int vo = (half_tail && c == nchunks - 1) ? voffs_tail : voffs;
    char *at = (g & 1) ? As1 : As0;
    char *bt = (g & 1) ? Bs1 : Bs0;
#pragma unroll
    for (int j = 0; j < JA; ++j)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_void *)(at + (NW * j + wave) * 1024), 16, vo,
                                               ka + j * jstep, 0, 0);
#pragma unroll
    for (int j = 0; j < JB; ++j)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_void *)(bt + (NW * j + wave) * 1024), 16, vo,
                                               kb + j * jstep, 0, 0);
  };
  const int fr = lane & 31, fh = lane >> 5;
  vec fa0[MT], fb0[NT], fa1[MT], fb1[NT];
  issue(0);
  __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
  __syncthreads();
  dl_frags<T, BK, MT, NT>(As0, Bs0, wm, wn, fr, fh, 0, fa0, fb0);
  if (G > 1) issue(1);
  int g = 0;
  for (int st = 0; st < nsteps; ++st) {
    f32x16 acc[MT][NT];
    // one chunk; FIRST: the column step's first (its first k-step starts the
    // sums); skip_hi: a half chunk (its k-steps 2 and 3 are zeros: no MFMAs)
    auto chunk = [&](auto first_c, bool skip_hi) {
      constexpr bool FIRST = decltype(first_c)::value;
      const char *a = (g & 1) ? As1 : As0;
      const char *bt = (g & 1) ? Bs1 : Bs0;
      // the phases stay in this order (the scheduler would otherwise hoist
      // the barrier above the MFMAs and group the reads)
      dl_frags<T, BK, MT, NT>(a, bt, wm, wn, fr, fh, 1, fa1, fb1);
      __builtin_amdgcn_sched_barrier(0);
      dl_mfmas<T, MT, NT, FIRST>(fa0, fb0, acc);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (KS == 4) {
        dl_frags<T, BK, MT, NT>(a, bt, wm, wn, fr, fh, 2, fa0, fb0);
        __builtin_amdgcn_sched_barrier(0);
        dl_mfmas<T, MT, NT>(fa1, fb1, acc);
        __builtin_amdgcn_sched_barrier(0);
        dl_frags<T, BK, MT, NT>(a, bt, wm, wn, fr, fh, 3, fa1, fb1);
        __builtin_amdgcn_sched_barrier(0);
        if (!skip_hi) dl_mfmas<T, MT, NT>(fa0, fb0, acc);
        __builtin_amdgcn_sched_barrier(0);
      }
      // the next chunk's loads (this wave's part) are done and this wave's
      // reads of the current buffer have returned; the barrier makes both
      // hold for every wave
      __builtin_amdgcn_s_waitcnt(0x0070);   // vmcnt(0) lgkmcnt(0)
      __syncthreads();
      if (g + 1 < G)
        dl_frags<T, BK, MT, NT>((g & 1) ? As0 : As1, (g & 1) ? Bs0 : Bs1, wm, wn, fr, fh, 0, fa0, fb0);
      if (g + 2 < G) issue(g + 2);
      __builtin_amdgcn_sched_barrier(0);
      if (KS == 2 || !skip_hi) dl_mfmas<T, MT, NT>(fa1, fb1, acc);
      __builtin_amdgcn_sched_barrier(0);
      ++g;
    };
    chunk(std::true_type{}, half_tail && nchunks == 1);
    for (int c = 1; c < nchunks; ++c) chunk(std::false_type{}, half_tail && c == nchunks - 1);
    // epilogue of the column step: complex SNR of 8 templates per lane per
    // row tile, running peaks
    const int64_t n0 = ws + (int64_t)st * BN;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int64_t col = n0 + wn * 32 * NT + nt * 32 + fr;
      const bool ok = col < we;
      const int rel = (int)(col - ws);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const float re = acc[mt][nt][2 * p], im = acc[mt][nt][2 * p + 1];
          const float v = re * re + im * im;
          if (ok && v > best[mt][p].v) best[mt][p] = VN{v, rel};
          if (SNR && ok) {
            const int64_t i = (r0 + wm * 32 * MT + mt * 32 + 8 * (p >> 1) + 4 * fh + 2 * (p & 1)) >> 1;
            if (i < n_templates) {
              // written once and not read here: a non-temporal store
              typedef float fv2 __attribute__((ext_vector_type(2)));
              __builtin_nontemporal_store(fv2{re * inv_scale, im * inv_scale},
                                          (fv2 *)(jb.snr + (i * jb.snr_ld + (col - jb.snr_abs0)) * 2));
            }
          }
        }
      }
    }
  }

  // reduce the 32 columns of each half-wave, then the waves that share rows
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      VN bb = best[mt][p];
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) {
        const float ov = __shfl_xor(bb.v, off);
        const int on = __shfl_xor(bb.n, off);
        if (better(ov, on, bb.v, bb.n)) bb = VN{ov, on};
      }
      if (fr == 0) red[wn][wm * 16 * MT + mt * 16 + 4 * (p >> 1) + 2 * fh + (p & 1)] = bb;
    }
  __syncthreads();
  for (int t = threadIdx.x; t < BM / 2; t += THREADS) {
    VN bb = red[0][t];
#pragma unroll
    for (int q = 1; q < WN; ++q)
      if (better(red[q][t].v, red[q][t].n, bb.v, bb.n)) bb = red[q][t];
    const int64_t i = r0 / 2 + t;
    if (i < n_templates) {
      const int64_t o = i * jb.ld_peak + (w - jb.w_base);
      jb.peak_snr[o] = sqrtf(fmaxf(bb.v, 0.f)) * inv_scale;
      jb.peak_n[o] = ws + bb.n;
    }
  }
}

// Phase and sub-sample refinement at each reported window peak: z_i at n* - 1,
// n*, n* + 1 recomputed as the dot products of mixing rows 2i, 2i+1 with those
// operand rows (FP32 accumulation; the operand holds one extra sample on each
// side of a chunk).  The refinement is the vertex of the parabola through the
// three |z| values (offset clipped to half a sample; none when the triple is
// not concave).  Peaks below `thr` get zeros (not reported).
// One thread per (template, window) entry tests the threshold and writes the
// zeros; then the whole wave takes its entries above it two at a time: lane k
// reads 16-byte vector k of each of the 5 rows of both (all 10 reads in
// flight at once) and the 12 partial sums are reduced over the wave.
template <typename T> struct Vec16 {
  T v[16 / sizeof(T)];
};

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_peak_phase(const MixJob *__restrict__ jobs, int n_jobs, int64_t entries,
                                                    float thr) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int job = 0;
  int64_t o = 0, row = 0;   // peak-table offset and template of this lane's entry
  bool hit = false;
  if (e < entries) {
    // job owning entry e: last job with e0 <= e
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].e0 <= e) lo = mid;
      else hi = mid - 1;
    }
    job = lo;
    const MixJob &jb = jobs[lo];
    const int64_t le = e - jb.e0;
    row = le / jb.nw;
    o = row * jb.ld_peak + (jb.w0 + le - row * jb.nw - jb.w_base);
    hit = jb.peak_snr[o] >= thr;
    if (!hit) {
      jb.peak_phase[o] = 0.f;
      jb.peak_dt[o] = 0.f;
      jb.peak_si[o] = 0.f;
    }
  }
  constexpr int EPV = 16 / (int)sizeof(T);
  uint64_t m = __ballot(hit);
  while (m) {
    // up to two entries of the wave; the second repeats the first when there is none
    const int s0 = __builtin_ctzll(m);
    m &= m - 1;
    const int s1 = m ? __builtin_ctzll(m) : s0;
    if (m) m &= m - 1;
    const int src[2] = {s0, s1};
    float acc[2][6];
    int jx[2];
    int64_t ox[2];
    const uint4 *mc[2], *ms[2], *o0[2];
    int nv[2], pv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      jx[t] = __builtin_amdgcn_readlane(job, src[t]);
      const MixJob &jb = jobs[jx[t]];
      const int64_t r = ((int64_t)__builtin_amdgcn_readlane((int)(row >> 32), src[t]) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)row, src[t]);
      ox[t] = ((int64_t)__builtin_amdgcn_readlane((int)(o >> 32), src[t]) << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)o, src[t]);
      // kcat and the row pitch kld are multiples of 32: whole 16-byte vectors
      nv[t] = jb.kcat / EPV;
      pv[t] = jb.kld / EPV;
      o0[t] = (const uint4 *)((const T *)jb.ocat + (jb.peak_n[ox[t]] - 1 - jb.ocat_abs0) * (int64_t)jb.kld);
      mc[t] = (const uint4 *)((const T *)jb.mix + (2 * r) * (int64_t)jb.kld);
      ms[t] = mc[t] + pv[t];
#pragma unroll
      for (int q = 0; q < 6; ++q) acc[t][q] = 0.f;
    }
    for (int k0 = 0; k0 < max(nv[0], nv[1]); k0 += 64) {
      const int k = k0 + lane;
      Vec16<T> c[2], d[2], a[2][3];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const bool ok = k < nv[t];
        const int kk = ok ? k : 0;
        c[t] = __builtin_bit_cast(Vec16<T>, mc[t][kk]);
        d[t] = __builtin_bit_cast(Vec16<T>, ms[t][kk]);
#pragma unroll
        for (int q = 0; q < 3; ++q) a[t][q] = __builtin_bit_cast(Vec16<T>, o0[t][q * pv[t] + kk]);
        if (!ok) c[t] = d[t] = Vec16<T>{};
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int j = 0; j < EPV; ++j) {
            // explicit FMAs: the same arithmetic in both slots (the compiler
            // would otherwise pair some products into dot-product
            // instructions that round differently)
            const float ov = Op<T>::tof(a[t][q].v[j]);
            acc[t][q] = __builtin_fmaf(Op<T>::tof(c[t].v[j]), ov, acc[t][q]);
            acc[t][3 + q] = __builtin_fmaf(Op<T>::tof(d[t].v[j]), ov, acc[t][3 + q]);
          }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int q = 0; q < 6; ++q) acc[t][q] = wave_sum(acc[t][q]);
    if (lane == 0) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        if (t == 1 && s1 == s0) break;
        const MixJob &jb = jobs[jx[t]];
        const float *re = acc[t], *im = acc[t] + 3;
        float amp[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) amp[q] = sqrtf(re[q] * re[q] + im[q] * im[q]) * jb.inv_scale;
        const float curv = amp[0] - 2.f * amp[1] + amp[2];
        float dt = 0.f, v = amp[1];
        if (curv < 0.f) {
          dt = fminf(0.5f, fmaxf(-0.5f, (amp[0] - amp[2]) / (2.f * curv)));
          v = amp[1] - 0.25f * (amp[0] - amp[2]) * dt;
        }
        jb.peak_phase[ox[t]] = atan2f(im[1], re[1]);
        jb.peak_dt[ox[t]] = dt;
        jb.peak_si[ox[t]] = v;
        if (jb.peak_z) jb.peak_z[ox[t]] = make_float2(re[1] * jb.inv_scale, im[1] * jb.inv_scale);
      }
    }
  }
}

// Signal-consistency value at each trigger peak (Sec. II.A computes phase and
// xi^2 for every trigger):
//   xi2 = sum_k |z[n* + k] - z[n*] R[k]|^2 / sum_k (2 - 2 |R[k]|^2)
// over the lags k = -K..K with 0 <= n* + k < n_end.  z is recomputed at the
// lags as MFMA tiles Z = M_rows * Ocat^T over groups of 16 triggers (32
// mixing rows: cos and sin of 16 templates) and 32 samples; the tile's
// epilogue adds each lane's lags to its eight triggers' sums, and z[n*] comes
// from the phase kernel.  Triggers are listed per window and sorted by peak
// sample, so that a group's lags lie close together: the samples a group
// covers are about its spread of peaks plus 2K (a chunk's operand holds K
// extra samples on each side).
//
// Two forms.  16-bit operands with kcat <= 512 (and autocorrelation tables
// of fewer than 2^31 entries) run two launches:
// k_xi2_list (one workgroup per (job, window)) stores the sorted keys and
// appends one unit per 64 of them to a list, and k_xi2_tiles (persistent
// workgroups taking units from that list) keeps each wave's A fragments in
// registers for the whole unit and stages every operand tile once in LDS for
// its four waves, with coalesced direct-to-LDS loads.  Otherwise k_xi2 does
// both in one workgroup per (job, window), reading fragments straight from
// memory.

constexpr int kXiThreads = 256;
constexpr int kXiList = 1024;   // triggers listed per pass over a window's templates
constexpr int kXiGroup = 16;    // triggers per MFMA row tile

// (job, window) item `item` of the signal-consistency launches: the last job
// with x0 <= item.
__device__ __forceinline__ int find_xi_job(const MixJob *__restrict__ jobs, int n_jobs, int64_t item) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].x0 <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One listing pass of window w (start ws) over templates [i0, F): the keys
// (n* - ws) << 32 | i of at most kXiList triggers in l_key, sorted by peak
// sample (template order among equal samples).  Returns how many; *i_next is
// the first template left for the next pass (F when none).  Every thread of
// the workgroup calls it.
__device__ int xi_list_pass(const MixJob &jb, int64_t w, int64_t ws, float thr, int i0, int64_t *l_key,
                            int *l_count, int *i_next_out) {
  const int F = jb.n_templates, lane = threadIdx.x & 63;
  if (threadIdx.x == 0) *l_count = 0;
  __syncthreads();
  int i_next = F;
  for (int ib = i0; ib < F; ib += kXiThreads) {
    const int i = ib + (int)threadIdx.x;
    const int64_t o = (int64_t)i * jb.ld_peak + (w - jb.w_base);
    const bool f = i < F && jb.peak_snr[o] >= thr;
    const uint64_t m = __ballot(f);
    int base = 0;
    if (lane == 0 && m) base = atomicAdd(l_count, (int)__popcll(m));
    base = __shfl(base, 0);
    if (f) {
      const int at = base + (int)__popcll(m & (lane ? (~0ull >> (64 - lane)) : 0ull));
      if (at < kXiList) l_key[at] = ((jb.peak_n[o] - ws) << 32) | (int64_t)i;
    }
    __syncthreads();
    const int cnt = *l_count;
    __syncthreads();
    if (cnt > kXiList) {   // full: this block's triggers wait for the next pass
      i_next = ib;
      break;
    }
  }
  int n_list = min(*l_count, kXiList);
  if (i_next < F) {
    // keep the triggers of templates below i_next (every one of them fits)
    __syncthreads();
    if (threadIdx.x == 0) {
      int k = 0;
      for (int t = 0; t < n_list; ++t)
        if ((int)(l_key[t] & 0xffffffff) < i_next) l_key[k++] = l_key[t];
      *l_count = k;
    }
    __syncthreads();
    n_list = *l_count;
  }
  // bitonic sort of the keys by peak sample (padding sorts last)
  int np2 = 1;
  while (np2 < n_list) np2 <<= 1;
  for (int t = n_list + (int)threadIdx.x; t < np2; t += kXiThreads) l_key[t] = INT64_MAX;
  __syncthreads();
  for (int size = 2; size <= np2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < np2 / 2; t += kXiThreads) {
        const int a = 2 * stride * (t / stride) + (t % stride), b2 = a + stride;
        const bool up = (a & size) == 0;
        const int64_t x = l_key[a], y = l_key[b2];
        if ((x > y) == up) {
          l_key[a] = y;
          l_key[b2] = x;
        }
      }
      __syncthreads();
    }
  *i_next_out = i_next;
  return n_list;
}

template <typename T>
__global__ __launch_bounds__(kXiThreads) void k_xi2(const MixJob *__restrict__ jobs, int n_jobs, float thr) {
  typedef Op<T> O;
  __shared__ int64_t l_key[kXiList];   // (n* - window start) << 32 | template
  __shared__ int l_count;

  // job and window of this workgroup
  const int64_t item = blockIdx.x;
  const MixJob &jb = jobs[find_xi_job(jobs, n_jobs, item)];
  const int64_t wl = item - jb.x0;
  if (!jb.acorr || wl >= jb.nw) return;   // uniform over the workgroup
  const int64_t w = jb.w0 + wl;
  const int64_t ws = (w * jb.win_p) / jb.win_q;
  const int K = jb.acorr_half, kcat = jb.kcat, F = jb.n_templates;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T *mix = (const T *)jb.mix;
  const T *ocat = (const T *)jb.ocat;
  const float2 *acorr = (const float2 *)jb.acorr;
  const float sc = jb.inv_scale;
  const int nks = kcat / O::KS;

  for (int i0 = 0; i0 < F;) {
    int i_next;
    const int n_list = xi_list_pass(jb, w, ws, thr, i0, l_key, &l_count, &i_next);

    // ---- groups of kXiGroup triggers, one wave each
    const int n_groups = (n_list + kXiGroup - 1) / kXiGroup;
    for (int g = wave; g < n_groups; g += kXiThreads / 64) {
      const int t0 = g * kXiGroup, nt = min(kXiGroup, n_list - t0);
      // A rows: lane row rr = lane % 32 is cos (even) or sin (odd) of trigger rr / 2
      const int tr = (lane & 31) >> 1;
      const int64_t ir = l_key[t0 + (tr < nt ? tr : 0)] & 0xffffffff;
      const T *arow = mix + (2 * ir + (lane & 1)) * (int64_t)jb.kld + (lane >> 5) * O::VEC;
      // the eight triggers of this lane's accumulator pairs: rows 8 (e/4) + 4 (lane/32) + e%4
      int64_t ns[8], ii[8];
      float2 zs[8];
      float num[8], den[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int tq = 4 * (p >> 1) + 2 * (lane >> 5) + (p & 1);
        const int64_t key = l_key[t0 + (tq < nt ? tq : 0)];
        ns[p] = tq < nt ? ws + (key >> 32) : INT64_MIN / 4;   // absent triggers reach no lag
        ii[p] = key & 0xffffffff;
        const float2 z = jb.peak_z[ii[p] * jb.ld_peak + (w - jb.w_base)];
        zs[p] = z;
        num[p] = 0.f;
        den[p] = 0.f;
      }
      // samples the group's lags reach, inside the data
      int64_t a0 = ws + (l_key[t0] >> 32) - K, a1 = ws + (l_key[t0 + nt - 1] >> 32) + K + 1;
      if (a0 < 0) a0 = 0;
      if (a1 > jb.n_end) a1 = jb.n_end;
      // blocks of U = 10 k-steps when that takes fewer blocks than U = 8 (30
      // k-steps: 3 instead of 4), else 8; more staging registers than 10 per
      // block would halve the occupancy
      auto tiles = [&](auto u_const) {
        constexpr int U = decltype(u_const)::value;
        for (int64_t s0 = a0; s0 < a1; s0 += 32) {
          const int64_t n = s0 + (lane & 31);
          const int64_t nb = n < a1 ? n : a1 - 1;
          const T *brow = ocat + (nb - jb.ocat_abs0) * (int64_t)jb.kld + (lane >> 5) * O::VEC;
          // two accumulators (even and odd k-steps) halve the MFMA dependency
          // chain.  Blocks of U k-steps issue all their reads before their MFMAs;
          // in the last block the k-steps past nks read k-step nks - 1 (in
          // range) and multiply a zero operand, so no k-step waits on its own
          // read alone and the block has no branches.
          f32x16 acc, acc2;
#pragma unroll
          for (int e = 0; e < 16; ++e) acc[e] = acc2[e] = 0.f;
          for (int ks = 0; ks < nks; ks += U) {
            typename O::vec af[U], bf[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int k = min(ks + u, nks - 1);
              af[u] = *(const typename O::vec *)(arow + k * O::KS);
              bf[u] = *(const typename O::vec *)(brow + k * O::KS);
              if (ks + u >= nks) bf[u] = typename O::vec{};
            }
            __builtin_amdgcn_sched_barrier(0);   // keep the block's reads ahead of its MFMAs
#pragma unroll
            for (int u = 0; u < U; u += 2) {
              acc = O::mfma(af[u], bf[u], acc);
              acc2 = O::mfma(af[u + 1], bf[u + 1], acc2);
            }
          }
#pragma unroll
          for (int e = 0; e < 16; ++e) acc[e] += acc2[e];
#pragma unroll
          for (int p = 0; p < 8; ++p) {
            const int64_t lag = n - ns[p];
            if (n < a1 && lag >= -K && lag <= K) {
              const float2 r = acorr[ii[p] * (2 * K + 1) + K + lag];
              const float dr = acc[2 * p] * sc - (zs[p].x * r.x - zs[p].y * r.y);
              const float di = acc[2 * p + 1] * sc - (zs[p].x * r.y + zs[p].y * r.x);
              num[p] += dr * dr + di * di;
              den[p] += 2.f - 2.f * (r.x * r.x + r.y * r.y);
            }
          }
        }
      };
      if ((nks + 9) / 10 < (nks + 7) / 8) tiles(std::integral_constant<int, 10>{});
      else tiles(std::integral_constant<int, 8>{});
      // sum each trigger's terms over the 32 lanes (samples) of its half-wave
#pragma unroll
      for (int p = 0; p < 8; ++p)
        for (int off = 1; off < 32; off <<= 1) {
          num[p] += __shfl_xor(num[p], off);
          den[p] += __shfl_xor(den[p], off);
        }
      if ((lane & 31) == 0) {
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const int tq = 4 * (p >> 1) + 2 * (lane >> 5) + (p & 1);
          if (tq < nt) jb.peak_xi[ii[p] * jb.ld_peak + (w - jb.w_base)] = den[p] > 0.f ? num[p] / den[p] : 0.f;
        }
      }
    }
    __syncthreads();
    i0 = i_next;
  }
}

// Listing launch of the two-launch form: keys of window w go to the job's
// listing slab at xi_key[(w - w_base) F + t], t = 0..count - 1 (one sorted
// run per listing pass), and units (item, 64 j, min(64, count - 64 j)) to
// units[counters[0]++ ...].  counters[0] starts at zero.
__global__ __launch_bounds__(kXiThreads) void k_xi2_list(const MixJob *__restrict__ jobs, int n_jobs, float thr,
                                                         XiUnit *__restrict__ units, int64_t cap,
                                                         int32_t *__restrict__ counters) {
  __shared__ int64_t l_key[kXiList];
  __shared__ int l_count, l_u0;
  const int64_t item = blockIdx.x;
  const MixJob &jb = jobs[find_xi_job(jobs, n_jobs, item)];
  const int64_t wl = item - jb.x0;
  if (!jb.acorr || wl >= jb.nw) return;   // uniform over the workgroup
  const int64_t w = jb.w0 + wl;
  const int64_t ws = (w * jb.win_p) / jb.win_q;
  const int F = jb.n_templates;
  int64_t *slab = jb.xi_key + (w - jb.w_base) * (int64_t)F;
  int count = 0;
  for (int i0 = 0; i0 < F;) {
    int i_next;
    const int n_list = xi_list_pass(jb, w, ws, thr, i0, l_key, &l_count, &i_next);
    for (int t = threadIdx.x; t < n_list; t += kXiThreads) slab[count + t] = l_key[t];
    count += n_list;
    __syncthreads();   // the next pass rewrites l_key
    i0 = i_next;
  }
  const int nu = (count + 63) / 64;
  if (nu == 0) return;
  if (threadIdx.x == 0) l_u0 = atomicAdd(&counters[0], nu);
  __syncthreads();
  for (int j = threadIdx.x; j < nu; j += kXiThreads) {
    const int64_t u = (int64_t)l_u0 + j;
    if (u < cap) units[u] = XiUnit{item, 64 * j, min(64, count - 64 * j)};
  }
}

// Staged operand tile: 32 rows (samples) of kcat 16-bit values, row pitch P =
// kcat / 8 + 1 16-byte chunks (odd, so 16 consecutive rows start on distinct
// banks): at most 33 loads of 64 chunks for kcat = 512.
constexpr int kXiTileBlocks = 33;
constexpr int kXiLoads = 9;   // loads per wave and tile: 4 waves x 9 >= kXiTileBlocks

// Tile launch of the two-launch form.  Workgroups take units from
// counters[1] until the list of counters[0] units is done.  Wave g of a unit
// owns its triggers 16 g .. 16 g + 15: the A fragments of every k-step stay in
// registers (NKS >= kcat / 16 k-steps; the ones past kcat are zeros) and its
// lag range [ga0, ga1) decides which tiles it multiplies.  The workgroup walks
// the union [ba0, ba1) of its waves' ranges in 32-sample tiles; each tile is
// loaded once into LDS, double-buffered.  Every wave issues exactly kXiLoads
// loads per tile (the ones past the tile land in a scratch block) and always
// issues the next tile (past the range: zeros), and the tile's
// autocorrelation reads go out before those loads: loads complete in issue
// order, so the epilogue then waits for its own reads only, not for the
// next tile.
template <typename T, int NKS>
__global__ __launch_bounds__(kXiThreads, 2) void k_xi2_tiles(const MixJob *__restrict__ jobs, int n_jobs,
                                                             const XiUnit *__restrict__ units, int64_t cap,
                                                             int32_t *__restrict__ counters) {
  static_assert(sizeof(T) == 2, "16-bit operands only");
  static_assert(NKS % 4 == 0 && NKS <= 32, "k-steps in blocks of 4, kcat <= 512");
  static_assert(4 * kXiLoads >= kXiTileBlocks, "whole tiles");
  typedef typename Op<T>::vec vec;
  __shared__ __attribute__((aligned(1024))) char Bt[2][kXiTileBlocks * 1024];
  __shared__ __attribute__((aligned(1024))) char Bx[1024];   // landing block of the loads past a tile
  __shared__ int64_t s_key[64];
  __shared__ float2 s_z[64];
  __shared__ int s_lo[64], s_ab[64];   // lag window start (relative to ws), autocorrelation row
  __shared__ int s_u;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int fr = lane & 31, fh = lane >> 5;
  const int64_t n_units = min((int64_t)counters[0], cap);
  for (;;) {
    if (threadIdx.x == 0) s_u = atomicAdd(&counters[1], 1);
    __syncthreads();
    const int u = __builtin_amdgcn_readfirstlane(s_u);   // the same in every lane: keep it scalar
    if (u >= n_units) break;                              // uniform over the workgroup
    const XiUnit un = units[u];
    const MixJob &jb = jobs[find_xi_job(jobs, n_jobs, un.item)];
    const int64_t w = jb.w0 + (un.item - jb.x0);
    const int64_t ws = (w * jb.win_p) / jb.win_q;
    const int64_t pcol = w - jb.w_base;
    const int K = jb.acorr_half, kcat = jb.kcat, nks = kcat / 16, nt_u = un.n;
    if (threadIdx.x < 64) {
      int64_t key = -1;
      float2 z = make_float2(0.f, 0.f);
      int lo = INT_MIN / 2, ab = 0;   // a missing trigger reaches no lag
      if (lane < nt_u) {
        key = jb.xi_key[pcol * jb.n_templates + un.first + lane];
        z = jb.peak_z[(key & 0xffffffff) * jb.ld_peak + pcol];
        lo = (int)(key >> 32) - K;
        ab = (int)(key & 0xffffffff) * (2 * K + 1);
      }
      s_key[lane] = key;
      s_z[lane] = z;
      s_lo[lane] = lo;
      s_ab[lane] = ab;
    }
    __syncthreads();

    // peak samples (relative to ws): range of this wave's group, then of the unit
    const int nr_l = (int)(s_key[lane] >> 32);
    int mn = lane < nt_u ? nr_l : INT_MAX, mx = lane < nt_u ? nr_l : INT_MIN;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      mn = min(mn, __shfl_xor(mn, off));
      mx = max(mx, __shfl_xor(mx, off));
    }
    const int gmn = __builtin_amdgcn_readfirstlane(__shfl(mn, 16 * wave));
    const int gmx = __builtin_amdgcn_readfirstlane(__shfl(mx, 16 * wave));
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      mn = min(mn, __shfl_xor(mn, off));
      mx = max(mx, __shfl_xor(mx, off));
    }
    mn = __builtin_amdgcn_readfirstlane(mn);
    mx = __builtin_amdgcn_readfirstlane(mx);
    const int64_t ba0 = max<int64_t>(0, ws + mn - K), ba1 = min<int64_t>(jb.n_end, ws + mx + K + 1);
    const bool has = 16 * wave < nt_u;
    const int64_t ga0 = has ? max<int64_t>(0, ws + gmn - K) : INT64_MAX;
    const int64_t ga1 = has ? min<int64_t>(jb.n_end, ws + gmx + K + 1) : INT64_MIN;

    // A fragments: lane row fr is cos (even) or sin (odd) of trigger 16 g + fr / 2
    // (a missing trigger repeats the unit's first; its rows are never used)
    vec af[NKS];
    {
      const int tr = 16 * wave + (fr >> 1);
      const int64_t i = s_key[tr < nt_u ? tr : 0] & 0xffffffff;
      const T *arow = (const T *)jb.mix + (2 * i + (lane & 1)) * (int64_t)jb.kld + fh * 8;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const vec v = *(const vec *)(arow + min(ks, nks - 1) * 16);
        af[ks] = ks < nks ? v : vec{};
      }
    }
    float num[8], den[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) num[p] = den[p] = 0.f;

    // tile loads: this wave's load i fills block 4 i + wave of the tile, lane
    // chunk c = 64 (4 i + wave) + lane = row c / P, position c % P (the pad
    // position reads the row's first chunk, rows past 31 read row 31).  The
    // resource ends at the unit's last sample: rows past it load zeros, and
    // so do the blocks past the tile's nblk (into Bx past kXiTileBlocks).
    const int cpr = kcat / 8, P = cpr + 1, nblk = (32 * P + 63) / 64;
    // the resource starts at the unit's first operand row (its extent is the
    // unit's lag range, not the whole operand)
    const int rowbytes = jb.kld * 2;   // operand row pitch
    const __amdgpu_buffer_rsrc_t rb =
        make_rsrc((const T *)jb.ocat + (ba0 - jb.ocat_abs0) * (int64_t)jb.kld, (ba1 - ba0) * (int64_t)rowbytes);
    const int dr = 256 / P, dq = 256 - dr * P;
    const int base0 = 0;
    auto issue = [&](int j) {
      // the chunk positions are recomputed per tile (a few ALU operations per
      // load) rather than held in registers across the loop
      int c0 = wave * 64 + lane;
      asm volatile("" : "+v"(c0));
      int r = c0 / P, q = c0 - r * P;
      const int tb = base0 + 32 * j * rowbytes;
      char *buf = Bt[j & 1];
#pragma unroll
      for (int i = 0; i < kXiLoads; ++i) {
        const int blk = 4 * i + wave;
        const int vo = blk < nblk ? tb + min(r, 31) * rowbytes + (q < cpr ? q : 0) * 16 : 0x7ffffff0;
        char *dst = blk < kXiTileBlocks ? buf + blk * 1024 : Bx;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_void *)dst, 16, vo, 0, 0, 0);
        q += dq;
        r += dr;
        if (q >= P) {
          q -= P;
          ++r;
        }
      }
    };
    const int ntl = (int)((ba1 - ba0 + 31) / 32);
    // a global (not generic) pointer: its reads count on the vector-memory
    // counter only, so the epilogue's wait leaves the next tile's loads in flight
    typedef float fv2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) const fv2 gfv2;
    gfv2 *acorr = (gfv2 *)jb.acorr;
    const float sc = jb.inv_scale;
    const int nrel0 = (int)(ba0 - ws) + fr, nrel_end = (int)(ba1 - ws);
    issue(0);
    for (int j = 0; j < ntl; ++j) {
      __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): this wave's loads of tile j
      __syncthreads();                      // every wave's; tile j - 1's buffer is free
      // the lane's eight triggers (accumulator rows 8 (e/4) + 4 fh + e%4):
      // autocorrelation at this lane's lag of each (a lag outside the window
      // reads entry 0 and adds nothing)
      const int nrel = nrel0 + 32 * j;   // this lane's sample, relative to ws
      fv2 r[8];
      bool in[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int t = 16 * wave + 4 * (p >> 1) + 2 * fh + (p & 1);
        const int d = nrel - s_lo[t];
        in[p] = nrel < nrel_end && (unsigned)d <= (unsigned)(2 * K);
        r[p] = acorr[in[p] ? s_ab[t] + d : 0];
      }
      issue(j + 1);   // past the range: zeros into the free buffer
      const int64_t s0 = ba0 + 32 * (int64_t)j;
      if (s0 < ga1 && s0 + 32 > ga0) {   // uniform over the wave
        const char *bb = Bt[j & 1] + (fr * P + fh) * 16;
        f32x16 acc;
#pragma unroll
        for (int kb = 0; kb < NKS; kb += 4) {
          vec bf[4];
#pragma unroll
          for (int u2 = 0; u2 < 4; ++u2) bf[u2] = *(const vec *)(bb + (kb + u2) * 32);
          __builtin_amdgcn_sched_barrier(0);   // the block's reads ahead of its MFMAs
#pragma unroll
          for (int u2 = 0; u2 < 4; ++u2) acc = Op<T>::mfma(af[kb + u2], bf[u2], kb + u2 == 0 ? f32x16{} : acc);
        }
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const float2 z = s_z[16 * wave + 4 * (p >> 1) + 2 * fh + (p & 1)];
          const float dre = acc[2 * p] * sc - (z.x * r[p].x - z.y * r[p].y);
          const float dim = acc[2 * p + 1] * sc - (z.x * r[p].y + z.y * r[p].x);
          if (in[p]) {
            num[p] += dre * dre + dim * dim;
            den[p] += 2.f - 2.f * (r[p].x * r[p].x + r[p].y * r[p].y);
          }
        }
      }
    }
    // sum each trigger's terms over the 32 lanes (samples) of its half-wave
#pragma unroll
    for (int p = 0; p < 8; ++p)
      for (int off = 1; off < 32; off <<= 1) {
        num[p] += __shfl_xor(num[p], off);
        den[p] += __shfl_xor(den[p], off);
      }
    if (fr == 0) {
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int t = 16 * wave + 4 * (p >> 1) + 2 * fh + (p & 1);
        if (t < nt_u)
          jb.peak_xi[(s_key[t] & 0xffffffff) * jb.ld_peak + pcol] = den[p] > 0.f ? num[p] / den[p] : 0.f;
      }
    }
    // the zeros issued past the range have landed and every wave is done
    // with the unit's keys and tiles before the next unit reuses them
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();
  }
}

// ---------------------------------------------------------- trigger compaction
// Stream compaction over the flat (job, template, window) order of every peak
// table: per-block flag counts, an exclusive scan of the block counts, then a
// rewrite of each block's flagged entries at its scanned offset.  A block
// covers kTrigPerBlock consecutive entries in kTrigPerBlock / 256 rounds of
// 256, so the cost follows the number of entries whatever the row shape.

constexpr int kTrigThreads = 256;

// Job owning flat entry e: the last job with elem0 <= e.
__device__ __forceinline__ int find_trig_job(const TrigJob *__restrict__ jobs, int n_jobs, int64_t e) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].elem0 <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = (int)(threadIdx.x & 63);
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

__global__ __launch_bounds__(kTrigThreads) void k_trigger_count(const TrigJob *__restrict__ jobs, int n_jobs,
                                                                int64_t n_elems, float thr,
                                                                int64_t *__restrict__ counts) {
  __shared__ int sh[kTrigThreads / 64];
  int c = 0;
  for (int k = 0; k < kTrigPerBlock / kTrigThreads; ++k) {
    const int64_t e = (int64_t)blockIdx.x * kTrigPerBlock + k * kTrigThreads + threadIdx.x;
    bool f = false;
    if (e < n_elems) {
      const TrigJob &jb = jobs[find_trig_job(jobs, n_jobs, e)];
      f = jb.snr[e - jb.elem0] >= thr;
    }
    c += __popcll(__ballot(f));
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int q = 0; q < kTrigThreads / 64; ++q) t += sh[q];
    counts[blockIdx.x] = t;
  }
}

// Exclusive prefix sum of counts[0..n) in place, total in *total; one block of
// 1024 threads, each taking 8 consecutive values per pass.
__global__ __launch_bounds__(1024) void k_trigger_scan(int64_t *counts, int64_t n, int64_t *total) {
  constexpr int V = 8, TPB = 1024;
  __shared__ int64_t wsum[TPB / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += (int64_t)TPB * V) {
    const int64_t i0 = base + (int64_t)threadIdx.x * V;
    int64_t v[V];
    int64_t own = 0;
#pragma unroll
    for (int q = 0; q < V; ++q) {
      v[q] = i0 + q < n ? counts[i0 + q] : 0;
      own += v[q];
    }
    // inclusive scan of the per-thread sums across the wave, then across waves
    int64_t inc = own;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t u = __shfl_up(inc, off);
      if (lane >= off) inc += u;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int64_t before = carry, pass = 0;
    for (int q = 0; q < TPB / 64; ++q) {
      if (q < wave) before += wsum[q];
      pass += wsum[q];
    }
    int64_t run = before + inc - own;
#pragma unroll
    for (int q = 0; q < V; ++q) {
      if (i0 + q < n) counts[i0 + q] = run;
      run += v[q];
    }
    carry += pass;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kTrigThreads) void k_trigger_write(const TrigJob *__restrict__ jobs, int n_jobs,
                                                                int64_t n_elems, float thr,
                                                                const int64_t *__restrict__ offsets, int64_t cap,
                                                                lloid_trigger *__restrict__ out) {
  __shared__ int sh[kTrigThreads / 64];
  const int wave = threadIdx.x >> 6;
  int64_t run = offsets[blockIdx.x];
  for (int k = 0; k < kTrigPerBlock / kTrigThreads; ++k) {
    const int64_t e = (int64_t)blockIdx.x * kTrigPerBlock + k * kTrigThreads + threadIdx.x;
    int j = 0;
    bool f = false;
    if (e < n_elems) {
      j = find_trig_job(jobs, n_jobs, e);
      f = jobs[j].snr[e - jobs[j].elem0] >= thr;
    }
    const uint64_t m = __ballot(f);
    if ((threadIdx.x & 63) == 0) sh[wave] = __popcll(m);
    __syncthreads();
    int64_t pos = run + __popcll(m & lanes_below());
    int blk = 0;
    for (int q = 0; q < kTrigThreads / 64; ++q) {
      if (q < wave) pos += sh[q];
      blk += sh[q];
    }
    if (f && pos < cap) {
      const TrigJob &jb = jobs[j];
      const int64_t o = e - jb.elem0;   // template o / nw, window o % nw of this table
      lloid_trigger t;
      t.bank = jb.bank_id;
      t.detector = jb.detector;
      t.template_id = (int32_t)(o / jb.nw);
      t.xi2 = jb.xi ? jb.xi[o] : 0.f;
      t.window = jb.w_base + o % jb.nw;
      t.sample = jb.peak_n[o];
      t.snr = jb.snr[o];
      t.phase = jb.phase[o];
      t.snr_interp = jb.si[o];
      t.dt = jb.dt[o];
      out[pos] = t;
    }
    run += blk;
    __syncthreads();
  }
}

// ---------------------------------------------------------- conditioning
// PSD, whitening and gating before the filter (Sec. II.A).  Each segment of L
// samples (hop L/2, periodic Hann window) is one workgroup: it loads the
// windowed samples into LDS and runs a radix-2 Stockham FFT there (two LDS
// buffers, one barrier per stage, output in natural order).  The PSD launch
// writes each segment's |X[f]|^2; their mean is taken per bin in FP64.  The
// whitening launch scales the spectrum by the gain, transforms back and
// writes the segment; the overlap-add sums the two segments over each sample.

// X = DFT(a) over n = 2^lg points with exponent sign * 2 pi i / n; a and b
// are LDS buffers of n values; returns the one that holds the result.
__device__ float2 *fft_lds(float2 *a, float2 *b, int n, int lg, float sign) {
  const int half = n >> 1;
  for (int st = 0; st < lg; ++st) {
    const int ns = 1 << st;
    for (int j = threadIdx.x; j < half; j += blockDim.x) {
      const int k = j & (ns - 1);
      const float2 a0 = a[j], a1 = a[j + half];
      float sn, cs;
      sincospif(sign * (float)k / (float)ns, &sn, &cs);   // angle sign * 2 pi k / (2 ns)
      const float tx = a1.x * cs - a1.y * sn, ty = a1.x * sn + a1.y * cs;
      const int idx = ((j >> st) << (st + 1)) + k;
      b[idx] = make_float2(a0.x + tx, a0.y + ty);
      b[idx + ns] = make_float2(a0.x - tx, a0.y - ty);
    }
    __syncthreads();
    float2 *t = a;
    a = b;
    b = t;
  }
  return a;
}

// One segment per workgroup: segment m = seg0 + blockIdx.x covers samples
// [m L/2, m L/2 + L) of x (zero outside [0, T)).  WHITEN = false: |X[f]|^2
// for f <= L/2 into parts; true: X scaled by gain[min(f, L - f)], inverse
// transform, real part / L into y.
template <bool WHITEN>
__global__ __launch_bounds__(256) void k_cond_segment(const float *__restrict__ x, int64_t T, int L, int lg,
                                                      int64_t seg0, const float *__restrict__ gain,
                                                      float *__restrict__ parts, float *__restrict__ y) {
  extern __shared__ float2 cbuf[];   // 2 L values
  float2 *a = cbuf, *b = cbuf + L;
  const int64_t lo = (seg0 + (int64_t)blockIdx.x) * (L / 2);
  for (int n = threadIdx.x; n < L; n += blockDim.x) {
    const int64_t t = lo + n;
    const float v = (t >= 0 && t < T) ? x[t] : 0.f;
    const float s = sinpif((float)n / (float)L);
    a[n] = make_float2(v * s * s, 0.f);
  }
  __syncthreads();
  float2 *X = fft_lds(a, b, L, lg, -1.f);
  if (!WHITEN) {
    const int nf = L / 2 + 1;
    for (int f = threadIdx.x; f < nf; f += blockDim.x)
      parts[(int64_t)blockIdx.x * nf + f] = X[f].x * X[f].x + X[f].y * X[f].y;
    return;
  }
  for (int f = threadIdx.x; f < L; f += blockDim.x) {
    const float g = gain[f <= L / 2 ? f : L - f];
    X[f] = make_float2(X[f].x * g, X[f].y * g);
  }
  __syncthreads();
  float2 *Y = fft_lds(X, X == a ? b : a, L, lg, 1.f);
  const float inv = 1.f / (float)L;
  for (int n = threadIdx.x; n < L; n += blockDim.x) y[(int64_t)blockIdx.x * L + n] = Y[n].x * inv;
}

// Per bin f <= L/2: the mean periodogram, c_f / (nseg f0 sum w^2) times the
// sum over segments (sum w^2 = 3 L / 8 for the periodic Hann window).  The
// sum over segments is compensated (Kahan): in FP32 its error stays at a few
// units of rounding whatever the number of segments.
__global__ void k_psd_mean(const float *__restrict__ parts, int64_t nseg, int L, float f0, float *__restrict__ psd) {
  const int nf = L / 2 + 1;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  float acc = 0.f, comp = 0.f;
  for (int64_t m = 0; m < nseg; ++m) {
    const float y = parts[m * nf + f] - comp;
    const float t = acc + y;
    comp = (t - acc) - y;
    acc = t;
  }
  const float c = (f == 0 || f == L / 2) ? 1.f : 2.f;
  psd[f] = c * acc / ((float)nseg * f0 * (0.375f * (float)L));
}

__global__ void k_psd_gain(const float *__restrict__ psd, int nf, float f0, float *__restrict__ gain) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const float s = psd[f];
  gain[f] = s > 0.f ? 1.f / sqrtf(s * f0 * 0.5f) : 0.f;
}

// xw[n] = the two segments' outputs over sample n (segment m starts at m L/2;
// y holds segments seg0, seg0 + 1, ...)
__global__ void k_overlap_add(const float *__restrict__ y, int64_t T, int L, int64_t seg0, float *__restrict__ xw) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= T) return;
  const int64_t h = L / 2;
  const int64_t mb = n / h, ma = mb - 1;
  xw[n] = y[(ma - seg0) * L + (n - ma * h)] + y[(mb - seg0) * L + (n - mb * h)];
}

// mask[k] = 1 for every k within half_width of a sample with |xw| > thr
__global__ void k_gate_mark(const float *__restrict__ xw, int64_t T, float thr, int half_width,
                            uint8_t *__restrict__ mask) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= T || !(fabsf(xw[n]) > thr)) return;
  const int64_t a = n - half_width < 0 ? 0 : n - half_width;
  const int64_t e = n + half_width + 1 > T ? T : n + half_width + 1;
  for (int64_t k = a; k < e; ++k) mask[k] = 1;
}

__global__ void k_gate_apply(const float *__restrict__ xw, const uint8_t *__restrict__ mask, int64_t T,
                             float *__restrict__ out, unsigned long long *__restrict__ count) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool g = n < T && mask[n];
  if (n < T) out[n] = g ? 0.f : xw[n];
  const uint64_t m = __ballot(g);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, (unsigned long long)__popcll(m));
}

// ---------------------------------------------------------- coincidence
// Pairs of triggers of two detectors with the same (bank, template) whose
// peak samples differ by at most max_dt (Sec. II.A, the coincidence
// generator).  Both lists are sorted by (bank, template, sample), so the
// partners of a[i] are one contiguous run of b, found by binary search; one
// thread per trigger of a counts its run, the counts are scanned, and the
// same threads write their pairs at the scanned offsets (a-major order).

__device__ __forceinline__ bool key_before(const lloid_trigger &x, int32_t bank, int32_t tmpl, int64_t sample) {
  if (x.bank != bank) return x.bank < bank;
  if (x.template_id != tmpl) return x.template_id < tmpl;
  return x.sample < sample;
}

__device__ __forceinline__ bool out_of_order(const lloid_trigger &x, const lloid_trigger &y) {
  return key_before(y, x.bank, x.template_id, x.sample);
}

// first j with b[j] not before (bank, tmpl, sample - max_dt)
__device__ __forceinline__ int64_t coinc_first(const lloid_trigger *__restrict__ b, int64_t nb,
                                               const lloid_trigger &t, int64_t max_dt) {
  int64_t lo = 0, hi = nb;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key_before(b[mid], t.bank, t.template_id, t.sample - max_dt)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ bool coinc_partner(const lloid_trigger &x, const lloid_trigger &t, int64_t max_dt) {
  return x.bank == t.bank && x.template_id == t.template_id && x.sample <= t.sample + max_dt;
}

__global__ void k_coinc_count(const lloid_trigger *__restrict__ a, int64_t na, const lloid_trigger *__restrict__ b,
                              int64_t nb, int64_t max_dt, int64_t *__restrict__ counts, uint8_t *__restrict__ bg_b,
                              int *__restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) {
    if (bg_b) bg_b[i] = 1;
    if (i + 1 < nb && out_of_order(b[i], b[i + 1])) *bad = 1;
  }
  if (i >= na) return;
  const lloid_trigger t = a[i];
  if (i + 1 < na && out_of_order(t, a[i + 1])) *bad = 1;
  int64_t c = 0;
  for (int64_t j = coinc_first(b, nb, t, max_dt); j < nb && coinc_partner(b[j], t, max_dt); ++j) ++c;
  counts[i] = c;
}

__global__ void k_coinc_write(const lloid_trigger *__restrict__ a, int64_t na, const lloid_trigger *__restrict__ b,
                              int64_t nb, int64_t max_dt, const int64_t *__restrict__ offsets, int64_t cap,
                              lloid_coinc *__restrict__ out, uint8_t *__restrict__ bg_a,
                              uint8_t *__restrict__ bg_b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= na) return;
  const lloid_trigger t = a[i];
  int64_t m = offsets[i];
  const int64_t m0 = m;
  for (int64_t j = coinc_first(b, nb, t, max_dt); j < nb && coinc_partner(b[j], t, max_dt); ++j, ++m) {
    const lloid_trigger u = b[j];
    if (bg_b) bg_b[j] = 0;
    if (m < cap) {
      lloid_coinc c;
      c.a = i;
      c.b = j;
      c.bank = t.bank;
      c.template_id = t.template_id;
      c.snr_net = sqrtf(t.snr * t.snr + u.snr * u.snr);
      c.dt = (float)(u.sample - t.sample) + (u.dt - t.dt);
      out[m] = c;
    }
  }
  if (bg_a) bg_a[i] = m == m0 ? 1 : 0;
}

// ---------------------------------------------------------- tuning input
// Counter-based hash (the 32-bit finaliser of MurmurHash3 applied to the
// sample index and seed) mapped to a uniform value of unit variance.
__global__ void k_noise(float *__restrict__ x, int64_t n, uint32_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t h = (uint32_t)i ^ (uint32_t)(i >> 32) * 0x9e3779b9u ^ seed;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  x[i] = ((float)h * (1.f / 4294967296.f) - 0.5f) * 3.4641016f;
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

hipError_t launch_noise(float *x, int64_t n, uint32_t seed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_noise<<<blocks_for(n, 256), 256, 0, s>>>(x, n, seed);
  return hipGetLastError();
}

hipError_t launch_decimate(const float *u, int64_t u_lo, int64_t u_len, float *d, int64_t d_lo,
                           int64_t d_len, const float *g, hipStream_t s) {
  if (d_len <= 0) return hipSuccess;
  k_decimate<<<blocks_for(d_len, 256), 256, 0, s>>>(u, u_lo, u_len, d, d_lo, d_len, g);
  return hipGetLastError();
}

template <typename T, int MT, int NT, int NW, int BK, bool HR = false>
static hipError_t fir_v(const FirJob *jobs, int n_jobs, int64_t n_items, hipStream_t s) {
  k_fir<T, MT, NT, NW, BK, HR><<<(unsigned)n_items, 64 * NW, 0, s>>>(jobs, n_jobs);
  return hipGetLastError();
}

template <typename T>
static hipError_t fir_t(int variant, const FirJob *jobs, int n_jobs, int64_t n_items, hipStream_t s) {
  switch (variant) {
    case 1: return fir_v<T, kFirMT, kFirNT, kFirWaves, kBK>(jobs, n_jobs, n_items, s);
    case 3:
    case 4:
      // 16-bit operands: the Hankel fragment window with basis chunks of 128
      // or 256 taps (a barrier per 8 or 16 k-steps instead of 4)
      if constexpr (sizeof(T) == 2) {
        if (variant == 3) return fir_v<T, 2, 4, kFirWaves, 4 * kBK, true>(jobs, n_jobs, n_items, s);
        return fir_v<T, 2, 4, kFirWaves, 8 * kBK, true>(jobs, n_jobs, n_items, s);
      } else {
        return fir_v<T, kFirMT, kFirNT, kFirWaves, kBK>(jobs, n_jobs, n_items, s);
      }
    case 5:
      // 16-bit operands: K chunks of 64 (twice the MFMAs per barrier)
      if constexpr (sizeof(T) == 2) return fir_v<T, kFirMT, kFirNT, kFirWaves, 2 * kBK>(jobs, n_jobs, n_items, s);
      else return fir_v<T, kFirMT, kFirNT, kFirWaves, kBK>(jobs, n_jobs, n_items, s);
    case 2:
      // 16-bit operands: 64 x 1024 tiles with the Hankel fragment window
      if constexpr (sizeof(T) == 2) return fir_v<T, 2, 4, kFirWaves, 2 * kBK, true>(jobs, n_jobs, n_items, s);
      else return fir_v<T, kFirMT, kFirNT, kFirWaves, kBK>(jobs, n_jobs, n_items, s);
    default:
      // 16-bit operands: the Hankel fragment window in four-wave 64 x 512
      // tiles, two workgroups per CU (one's strain-window fill and stores run
      // while the other's MFMAs do), basis chunks of 128 taps
      if constexpr (sizeof(T) == 2) return fir_v<T, 2, 4, 4, 4 * kBK, true>(jobs, n_jobs, n_items, s);
      else return fir_v<T, kFirMT, kFirNT, kFirWaves, kBK>(jobs, n_jobs, n_items, s);
  }
}

void fir_tile_shape(lloid_dtype t, int variant, int *bm, int *bn) {
  *bm = 32 * kFirMT;
  *bn = kFirWaves * 32 * kFirNT;
  if ((variant == 2 || variant == 3 || variant == 4) && t != LLOID_F32) *bm = 32 * 2, *bn = kFirWaves * 32 * 4;
  if (variant == 0 && t != LLOID_F32) *bm = 32 * 2, *bn = 4 * 32 * 4;
}

void mix_tile_shape(lloid_dtype, int variant, int *bm, int *bn) {
  switch (variant) {
    case 1: *bm = 32 * 4 * 2, *bn = 32 * 2 * 2; break;
    case 2: *bm = 32 * 2 * 4, *bn = 32 * 2 * 2; break;
    case 3: *bm = 32 * kMixMT * kMixWM, *bn = 32 * kMixNT * kMixWN; break;
    default: *bm = 32 * kMixMT * kMixWM, *bn = 32 * kMixNT * kMixWN; break;
  }
}

hipError_t launch_fir_jobs(lloid_dtype t, int variant, const FirJob *jobs, int n_jobs, int64_t n_items,
                           hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (t) {
    case LLOID_F16: return fir_t<_Float16>(variant, jobs, n_jobs, n_items, s);
    case LLOID_BF16: return fir_t<__bf16>(variant, jobs, n_jobs, n_items, s);
    case LLOID_F32: return fir_t<float>(variant, jobs, n_jobs, n_items, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_up_jobs(lloid_dtype t, const UpJob *jobs, int n_jobs, int64_t n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (t) {
    case LLOID_F32: k_upsample<float, float><<<(unsigned)n_items, 256, 0, s>>>(jobs, n_jobs); break;
    case LLOID_F16: k_upsample<_Float16, _Float16><<<(unsigned)n_items, 256, 0, s>>>(jobs, n_jobs); break;
    case LLOID_BF16: k_upsample<float, __bf16><<<(unsigned)n_items, 256, 0, s>>>(jobs, n_jobs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int MT, int NT, int WM, int WN, int BK>
static hipError_t mix_v(const MixJob *jobs, int n_jobs, int64_t n_items, bool with_snr, hipStream_t s) {
  if (with_snr)
    k_mix_peak<T, MT, NT, WM, WN, BK, true><<<(unsigned)n_items, 64 * WM * WN, 0, s>>>(jobs, n_jobs);
  else
    k_mix_peak<T, MT, NT, WM, WN, BK, false><<<(unsigned)n_items, 64 * WM * WN, 0, s>>>(jobs, n_jobs);
  return hipGetLastError();
}

template <typename T>
static hipError_t mix_t(int variant, const MixJob *jobs, int n_jobs, int64_t n_items, bool with_snr, hipStream_t s) {
  switch (variant) {
    case 1: return mix_v<T, 4, 2, 2, 2, 32>(jobs, n_jobs, n_items, with_snr, s);
    case 2: return mix_v<T, 2, 2, 4, 2, 32>(jobs, n_jobs, n_items, with_snr, s);
    case 3: return mix_v<T, kMixMT, kMixNT, kMixWM, kMixWN, 32>(jobs, n_jobs, n_items, with_snr, s);
    case 4:
      // 16-bit operands: register-staged K chunks of 64 (149.5 KB of LDS, one workgroup per CU)
      if constexpr (sizeof(T) == 2) return mix_v<T, kMixMT, kMixNT, kMixWM, kMixWN, 64>(jobs, n_jobs, n_items, with_snr, s);
      else return mix_v<T, kMixMT, kMixNT, kMixWM, kMixWN, 32>(jobs, n_jobs, n_items, with_snr, s);
    default:
      // 16-bit operands: direct-to-LDS K chunks of 64, eight 64 x 128 waves
      if constexpr (sizeof(T) == 2) {
        if (with_snr) k_mix_dl<T, 4, 2, 2, 4, 64, 1, true><<<(unsigned)n_items, 512, 0, s>>>(jobs, n_jobs);
        else k_mix_dl<T, 4, 2, 2, 4, 64, 1, false><<<(unsigned)n_items, 512, 0, s>>>(jobs, n_jobs);
        return hipGetLastError();
      } else {
        return mix_v<T, kMixMT, kMixNT, kMixWM, kMixWN, 32>(jobs, n_jobs, n_items, with_snr, s);
      }
  }
}

hipError_t launch_mix_jobs(lloid_dtype t, int variant, const MixJob *jobs, int n_jobs, int64_t n_items,
                           bool with_snr, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (t) {
    case LLOID_F16: return mix_t<_Float16>(variant, jobs, n_jobs, n_items, with_snr, s);
    case LLOID_BF16: return mix_t<__bf16>(variant, jobs, n_jobs, n_items, with_snr, s);
    case LLOID_F32: return mix_t<float>(variant, jobs, n_jobs, n_items, with_snr, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_peak_phase(lloid_dtype t, const MixJob *jobs, int n_jobs, int64_t n_entries, float phase_thr,
                             hipStream_t s) {
  if (n_entries <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n_entries + 255) / 256);   // one entry per thread
  switch (t) {
    case LLOID_F16: k_peak_phase<_Float16><<<blocks, 256, 0, s>>>(jobs, n_jobs, n_entries, phase_thr); break;
    case LLOID_BF16: k_peak_phase<__bf16><<<blocks, 256, 0, s>>>(jobs, n_jobs, n_entries, phase_thr); break;
    case LLOID_F32: k_peak_phase<float><<<blocks, 256, 0, s>>>(jobs, n_jobs, n_entries, phase_thr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_trigger_jobs(const TrigJob *jobs, int n_jobs, int64_t n_elems, float thr, int64_t *counts,
                               int64_t *total, int64_t cap, lloid_trigger *out, hipStream_t s) {
  const int64_t nblk = n_elems > 0 ? trig_blocks(n_elems) : 0;
  if (nblk > 0) k_trigger_count<<<(unsigned)nblk, kTrigThreads, 0, s>>>(jobs, n_jobs, n_elems, thr, counts);
  k_trigger_scan<<<1, 1024, 0, s>>>(counts, nblk, total);
  if (nblk > 0)
    k_trigger_write<<<(unsigned)nblk, kTrigThreads, 0, s>>>(jobs, n_jobs, n_elems, thr, counts, cap, out);
  return hipGetLastError();
}

hipError_t launch_xi2(lloid_dtype t, const MixJob *jobs, int n_jobs, int64_t n_windows, int kmax, int64_t acorr_max,
                      float thr, const XiWork &xw, int n_cu, hipStream_t s) {
  if (n_windows <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)n_windows;   // one workgroup per (job, window)
  const int nks = kmax / 16;
  // the tile launch indexes the autocorrelation tables with 32-bit offsets
  if (t != LLOID_F32 && nks <= 32 && acorr_max <= INT_MAX && xw.cap > 0) {
    hipError_t e = launch_fill_u8(xw.counters, 2 * sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    k_xi2_list<<<blocks, kXiThreads, 0, s>>>(jobs, n_jobs, thr, xw.units, xw.cap, xw.counters);
    // persistent: two workgroups per CU take units until the list is done
    const unsigned tb = (unsigned)std::min<int64_t>(xw.cap, 2 * (int64_t)std::max(n_cu, 1));
    const bool k16 = nks <= 16;
    if (t == LLOID_F16) {
      if (k16) k_xi2_tiles<_Float16, 16><<<tb, kXiThreads, 0, s>>>(jobs, n_jobs, xw.units, xw.cap, xw.counters);
      else k_xi2_tiles<_Float16, 32><<<tb, kXiThreads, 0, s>>>(jobs, n_jobs, xw.units, xw.cap, xw.counters);
    } else {
      if (k16) k_xi2_tiles<__bf16, 16><<<tb, kXiThreads, 0, s>>>(jobs, n_jobs, xw.units, xw.cap, xw.counters);
      else k_xi2_tiles<__bf16, 32><<<tb, kXiThreads, 0, s>>>(jobs, n_jobs, xw.units, xw.cap, xw.counters);
    }
    return hipGetLastError();
  }
  switch (t) {
    case LLOID_F16: k_xi2<_Float16><<<blocks, kXiThreads, 0, s>>>(jobs, n_jobs, thr); break;
    case LLOID_BF16: k_xi2<__bf16><<<blocks, kXiThreads, 0, s>>>(jobs, n_jobs, thr); break;
    case LLOID_F32: k_xi2<float><<<blocks, kXiThreads, 0, s>>>(jobs, n_jobs, thr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_condition(const float *x, int64_t T, int L, bool estimate, float f0, float *parts,
                            float *psd, float *gain, float *y, float *xw, float gate_thr, int gate_half,
                            uint8_t *mask, float *out, unsigned long long *count, hipStream_t s) {
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  const size_t lds = (size_t)2 * L * sizeof(float2);
  const int nf = L / 2 + 1;
  if (estimate) {
    const int64_t nseg = (T - L) / (L / 2) + 1;
    k_cond_segment<false><<<(unsigned)nseg, 256, lds, s>>>(x, T, L, lg, 0, nullptr, parts, nullptr);
    k_psd_mean<<<blocks_for(nf, 256), 256, 0, s>>>(parts, nseg, L, f0, psd);
  }
  k_psd_gain<<<blocks_for(nf, 256), 256, 0, s>>>(psd, nf, f0, gain);
  const int64_t nseg_w = (2 * (T - 1)) / L + 2;   // segments -1 .. floor(2 (T - 1) / L)
  k_cond_segment<true><<<(unsigned)nseg_w, 256, lds, s>>>(x, T, L, lg, -1, gain, nullptr, y);
  k_overlap_add<<<blocks_for(T, 256), 256, 0, s>>>(y, T, L, -1, gate_thr > 0.f ? xw : out);
  if (gate_thr > 0.f) {
    k_gate_mark<<<blocks_for(T, 256), 256, 0, s>>>(xw, T, gate_thr, gate_half, mask);
    k_gate_apply<<<blocks_for(T, 256), 256, 0, s>>>(xw, mask, T, out, count);
  }
  return hipGetLastError();
}

hipError_t launch_coincide(const lloid_trigger *a, int64_t na, const lloid_trigger *b, int64_t nb, int64_t max_dt,
                           int64_t *counts, int64_t *total, int *bad, int64_t cap, lloid_coinc *out, uint8_t *bg_a,
                           uint8_t *bg_b, hipStream_t s) {
  const int64_t nmax = std::max(na, nb);
  if (nmax > 0)
    k_coinc_count<<<blocks_for(nmax, 256), 256, 0, s>>>(a, na, b, nb, max_dt, counts, bg_b, bad);
  k_trigger_scan<<<1, 1024, 0, s>>>(counts, na, total);
  if (na > 0)
    k_coinc_write<<<blocks_for(na, 256), 256, 0, s>>>(a, na, b, nb, max_dt, counts, cap, out, bg_a, bg_b);
  return hipGetLastError();
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

}  // namespace lloid
