// MFMA GEMM kernels for gfx950.
//
// One workgroup (4 wavefronts, 2 x 2) owns a BM x BN tile of C; each
// wavefront owns a (BM/2) x (BN/2) sub-tile made of 16 x 16 MFMA blocks.
// The FP64/FP32 kernels are bounded to two resident waves per SIMD: with one
// wave (the 128 x 128 FP64 tile otherwise needs 384 registers per lane) the
// LDS and barrier latencies are exposed, with two the other wave fills them.
// Operand tiles are staged through LDS in k-major order, so that the lanes of
// one MFMA (row = lane % 16, k = lane / 16) read contiguous LDS words.  The
// next k-tile is fetched into registers while the current one is consumed.
//
// FP64 uses v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_16x16x4f32; split-BF16
// uses v_mfma_f32_16x16x32_bf16 three times per k-step (hi*hi + hi*lo + lo*hi)
// with FP32 accumulation.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace fno {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

template <typename T>
struct Acc;
template <>
struct Acc<double> {
  typedef d4_t type;
};
template <>
struct Acc<float> {
  typedef f4_t type;
};

__device__ __forceinline__ d4_t mfma4(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma4(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Tile of a workgroup.  The grid is one-dimensional over the MT x NT tiles
// (split-K slices in z).  Consecutive workgroup ids are spread round-robin
// over the 8 XCDs, each with its own L2: id L goes to XCD L % 8, so XCD x is
// given the contiguous tile range [x*q + min(x, r), ...) of its share, walked
// with M fastest (m_fast: consecutive tiles share a B column strip) or N
// fastest (consecutive tiles share an A row strip).  The operand whose strips
// are shared is then read from HBM about once instead of once per tile row.
__device__ __forceinline__ void tile_of(int64_t M, int64_t N, int BM, int BN, int m_fast, int64_t& m0, int64_t& n0,
                                        int64_t L) {
  const int64_t MT = (M + BM - 1) / BM, NT = (N + BN - 1) / BN, T = MT * NT;
  const int64_t q = T / 8, r = T % 8, x = L % 8, k = L / 8;
  const int64_t t = x * q + (x < r ? x : r) + k;
  const int64_t mt = m_fast ? t % MT : t / NT;
  const int64_t nt = m_fast ? t / MT : t % NT;
  m0 = mt * BM;
  n0 = nt * BN;
}

// ---------------------------------------------------------------------------
// 16x16x4 path (FP64 / FP32).  BK k values staged per tile (BK / 4 MFMA k-steps
// per pair of barriers): 16, or 32 for the FP32 tiles, whose MFMA steps take
// half as long, so the barriers and loads weigh twice as much per flop.
// (bx: the workgroup's linear tile index, bz: its split-K slice)
template <typename T, int BM, int BN, bool AK, bool BN_FAST, int BK, int VW>
__device__ __forceinline__ void gemm_k4_body(int64_t M, int64_t N, int64_t K, const T* __restrict__ A, int64_t lda,
                                             const T* __restrict__ B, int64_t ldb, T* __restrict__ C, int64_t ldc,
                                             T alpha, T beta, int64_t kchunk, int64_t cz, int m_fast, int64_t bx,
                                             int64_t bz) {
  {  // split-K: this z-slice owns K range [z*kchunk, z*kchunk + kchunk)
    const int64_t k0 = bz * kchunk;
    A += AK ? k0 : k0 * lda;
    B += BN_FAST ? k0 * ldb : k0;
    C += bz * cz;
    K = (K - k0 < kchunk) ? K - k0 : kchunk;
  }
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  // staged per thread: VW consecutive elements along the operand's fastest
  // index per global load (VW = 1: one element per load)
  constexpr int A_PER = BM * BK / VW / 256;
  constexpr int B_PER = BN * BK / VW / 256;
  static_assert(A_PER * VW * 256 == BM * BK && B_PER * VW * 256 == BN * BK, "tile shape");
  constexpr int AF = AK ? BK / VW : BM / VW;       // vectors along A's fast index
  constexpr int BF = BN_FAST ? BN / VW : BK / VW;  // vectors along B's fast index
  constexpr int PAD = (sizeof(T) == 8) ? 1 : 2;
  __shared__ T As[BK][BM + PAD];
  __shared__ T Bs[BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t m0, n0;
  tile_of(M, N, BM, BN, m_fast, m0, n0, bx);

  typename Acc<T>::type acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = (typename Acc<T>::type){0, 0, 0, 0};

  typedef T Vec __attribute__((ext_vector_type(VW)));  // 16 bytes when VW > 1: one dwordx4 load
  Vec ra[A_PER], rb[B_PER];
  // a run of VW elements from p: one 16-byte load when all are in range (the
  // host only selects VW > 1 when every run starts 16-byte aligned), else
  // one guarded load per element
  auto load_run = [&](const T* p, int64_t fast, int64_t fast_end, bool slow_ok) {
    Vec v;
    if constexpr (VW > 1) {
      if (slow_ok && fast + VW <= fast_end) {
        v = *(const Vec*)p;
        return v;
      }
    }
#pragma unroll
    for (int i = 0; i < VW; ++i) v[i] = (slow_ok && fast + i < fast_end) ? p[i] : (T)0;
    return v;
  };
  auto load_tiles = [&](int64_t k0) {
    if constexpr (VW == 1) {
#pragma unroll
      for (int p = 0; p < A_PER; ++p) {
        int e = tid + p * 256;
        int mm, kk;
        if (AK) {  // k fastest in memory: consecutive threads walk k
          kk = e % BK;
          mm = e / BK;
        } else {
          mm = e % BM;
          kk = e / BM;
        }
        int64_t gm = m0 + mm, gk = k0 + kk;
        T v = 0;
        if (gm < M && gk < K) v = AK ? A[gm * lda + gk] : A[gk * lda + gm];
        ra[p][0] = v;
      }
#pragma unroll
      for (int p = 0; p < B_PER; ++p) {
        int e = tid + p * 256;
        int nn, kk;
        if (BN_FAST) {
          nn = e % BN;
          kk = e / BN;
        } else {
          kk = e % BK;
          nn = e / BK;
        }
        int64_t gn = n0 + nn, gk = k0 + kk;
        T v = 0;
        if (gn < N && gk < K) v = BN_FAST ? B[gk * ldb + gn] : B[gn * ldb + gk];
        rb[p][0] = v;
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      const int e = tid + p * 256;
      const int f = (e % AF) * VW, sl = e / AF;  // fast and slow offsets in the tile
      if (AK) {  // k fastest in memory: consecutive threads walk k
        const int64_t gm = m0 + sl, gk = k0 + f;
        ra[p] = load_run(A + (gm < M ? gm : 0) * lda + gk, gk, K, gm < M);
      } else {
        const int64_t gm = m0 + f, gk = k0 + sl;
        ra[p] = load_run(A + (gk < K ? gk : 0) * lda + gm, gm, M, gk < K);
      }
    }
#pragma unroll
    for (int p = 0; p < B_PER; ++p) {
      const int e = tid + p * 256;
      const int f = (e % BF) * VW, sl = e / BF;
      if (BN_FAST) {
        const int64_t gn = n0 + f, gk = k0 + sl;
        rb[p] = load_run(B + (gk < K ? gk : 0) * ldb + gn, gn, N, gk < K);
      } else {
        const int64_t gn = n0 + sl, gk = k0 + f;
        rb[p] = load_run(B + (gn < N ? gn : 0) * ldb + gk, gk, K, gn < N);
      }
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      const int e = tid + p * 256;
      const int f = (e % AF) * VW, sl = e / AF;
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        if (AK)
          As[f + i][sl] = ra[p][i];
        else
          As[sl][f + i] = ra[p][i];
      }
    }
#pragma unroll
    for (int p = 0; p < B_PER; ++p) {
      const int e = tid + p * 256;
      const int f = (e % BF) * VW, sl = e / BF;
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        if (BN_FAST)
          Bs[sl][f + i] = rb[p][i];
        else
          Bs[f + i][sl] = rb[p][i];
      }
    }
  };

  // the MFMA steps of one staged k tile for the first `live` row blocks (a
  // compile-time count: each variant is a branch-free loop)
  auto mma_tile = [&](auto live) {
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      T af[TM], bfr[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = As[kr][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bfr[j] = Bs[kr][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        if (i < (int)live) {
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = mfma4(af[i], bfr[j], acc[i][j]);
        }
    }
  };

  const int64_t nk = (K + BK - 1) / BK;
  auto k_loop = [&](auto live) {
    if (nk > 0) load_tiles(0);
    for (int64_t kt = 0; kt < nk; ++kt) {
      __syncthreads();
      store_tiles();
      __syncthreads();
      if (kt + 1 < nk) load_tiles((kt + 1) * BK);
      mma_tile(live);
    }
  };
  if constexpr (VW > 1 && sizeof(T) == 8) {
    // In a partial last M tile a wavefront whose sub-tile holds at most one
    // 16-row block of C (the ring's 590 rows leave 78 in the last 128-row
    // tile) runs the one-block loop: a second copy of the loop, kept to the
    // FP64 vector tiles, where it costs no spills.  Other partial sub-tiles
    // run every block; their extra rows hold zeros and are not stored.
    const int wrow_first = __builtin_amdgcn_readfirstlane(wm * WM);  // uniform per wavefront
    const int64_t live_rows = M - (m0 + wrow_first);
    if (live_rows <= 16) {
      k_loop(std::integral_constant<int, 1>{});
    } else {
      k_loop(std::integral_constant<int, TM>{});
    }
  } else {
    // the same loop written out: built through the lambdas above, the FP32
    // 128 x 256 and 256 x 128 tiles get a different register allocation
    // with 24-44 spilled registers
    if (nk > 0) load_tiles(0);
    for (int64_t kt = 0; kt < nk; ++kt) {
      __syncthreads();
      store_tiles();
      __syncthreads();
      if (kt + 1 < nk) load_tiles((kt + 1) * BK);
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        const int kr = ks + (lane >> 4);
        T af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = As[kr][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < TN; ++j) bfr[j] = Bs[kr][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = mfma4(af[i], bfr[j], acc[i][j]);
      }
    }
  }

  // C/D layout of the 16x16 MFMA block: lane l holds column l % 16; the
  // FP32 instruction gives it rows 4 * (l / 16) + r, the FP64 instruction
  // rows l / 16 + 4 * r (r = 0..3).
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t col = n0 + wn * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (sizeof(T) == 8) ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int64_t row = m0 + wm * WM + i * 16 + rr;
        if (row < M && col < N) {
          T v = alpha * acc[i][j][r];
          if (beta != (T)0) v += beta * C[row * ldc + col];
          C[row * ldc + col] = v;
        }
      }
    }
}

// ---------------------------------------------------------------------------

template <typename T, int BM, int BN, bool AK, bool BN_FAST>
__global__ void __launch_bounds__(256, 2) gemm_k4_kernel(int64_t M, int64_t N, int64_t K, const T* __restrict__ A,
                                                      int64_t lda, const T* __restrict__ B, int64_t ldb,
                                                      T* __restrict__ C, int64_t ldc, T alpha, T beta,
                                                      int64_t kchunk, int64_t cz, int m_fast) {
  gemm_k4_body<T, BM, BN, AK, BN_FAST, 16, 1>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, kchunk, cz, m_fast, blockIdx.x,
                                                   blockIdx.z);
}

// Same tile with 16-byte global loads (4 floats or 2 doubles per load); the
// host launches it only when both operands' rows start 16-byte aligned.
template <typename T, int BM, int BN, bool AK, bool BN_FAST>
__global__ void __launch_bounds__(256, 2) gemm_k4v_kernel(int64_t M, int64_t N, int64_t K, const T* __restrict__ A,
                                                       int64_t lda, const T* __restrict__ B, int64_t ldb,
                                                       T* __restrict__ C, int64_t ldc, T alpha, T beta,
                                                       int64_t kchunk, int64_t cz, int m_fast) {
  gemm_k4_body<T, BM, BN, AK, BN_FAST, 16, 16 / sizeof(T)>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, kchunk, cz,
                                                           m_fast, blockIdx.x, blockIdx.z);
}

template <typename T, int BM, int BN, bool AK, bool BN_FAST>
__global__ void __launch_bounds__(256, 2) gemm_k32_kernel(int64_t M, int64_t N, int64_t K, const T* __restrict__ A,
                                                       int64_t lda, const T* __restrict__ B, int64_t ldb,
                                                       T* __restrict__ C, int64_t ldc, T alpha, T beta,
                                                       int64_t kchunk, int64_t cz, int m_fast) {
  gemm_k4_body<T, BM, BN, AK, BN_FAST, 32, 1>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, kchunk, cz, m_fast, blockIdx.x,
                                                   blockIdx.z);
}

template <typename T, int BM, int BN, bool AK, bool BN_FAST>
__global__ void __launch_bounds__(256, 2) gemm_k32v_kernel(int64_t M, int64_t N, int64_t K, const T* __restrict__ A,
                                                        int64_t lda, const T* __restrict__ B, int64_t ldb,
                                                        T* __restrict__ C, int64_t ldc, T alpha, T beta,
                                                        int64_t kchunk, int64_t cz, int m_fast) {
  gemm_k4_body<T, BM, BN, AK, BN_FAST, 32, 16 / sizeof(T)>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, kchunk, cz,
                                                           m_fast, blockIdx.x, blockIdx.z);
}

// Double-buffered 16x16x4 path (FP64 / FP32): two LDS stages, one barrier per
// k-tile.  While the MFMAs of stage s run, the next k-tile is already in
// flight from global memory into registers; it is written into the other LDS
// stage afterwards.  Same wave layout and C/D mapping as gemm_k4_kernel.
template <typename T, int BM, int BN, int BK, bool AK, bool BN_FAST>
__global__ void __launch_bounds__(256, 2) gemm_db_kernel(int64_t M, int64_t N, int64_t K, const T* __restrict__ A,
                                                      int64_t lda, const T* __restrict__ B, int64_t ldb,
                                                      T* __restrict__ C, int64_t ldc, T alpha, T beta,
                                                      int64_t kchunk, int64_t cz, int m_fast) {
  static_assert(BK % 4 == 0 && (BM * BK) % 256 == 0 && (BN * BK) % 256 == 0, "tile shape");
  {
    const int64_t k0 = (int64_t)blockIdx.z * kchunk;
    A += AK ? k0 : k0 * lda;
    B += BN_FAST ? k0 * ldb : k0;
    C += (int64_t)blockIdx.z * cz;
    K = (K - k0 < kchunk) ? K - k0 : kchunk;
  }
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int A_PER = BM * BK / 256;
  constexpr int B_PER = BN * BK / 256;
  constexpr int PAD = (sizeof(T) == 8) ? 1 : 2;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t m0, n0;
  tile_of(M, N, BM, BN, m_fast, m0, n0, blockIdx.x);

  typename Acc<T>::type acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = (typename Acc<T>::type){0, 0, 0, 0};

  T ra[A_PER], rb[B_PER];
  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      const int e = tid + p * 256;
      const int mm = AK ? e / BK : e % BM;
      const int kk = AK ? e % BK : e / BM;
      const int64_t gm = m0 + mm, gk = k0 + kk;
      ra[p] = (gm < M && gk < K) ? (AK ? A[gm * lda + gk] : A[gk * lda + gm]) : (T)0;
    }
#pragma unroll
    for (int p = 0; p < B_PER; ++p) {
      const int e = tid + p * 256;
      const int nn = BN_FAST ? e % BN : e / BK;
      const int kk = BN_FAST ? e / BN : e % BK;
      const int64_t gn = n0 + nn, gk = k0 + kk;
      rb[p] = (gn < N && gk < K) ? (BN_FAST ? B[gk * ldb + gn] : B[gn * ldb + gk]) : (T)0;
    }
  };
  auto store_tiles = [&](int s) {
#pragma unroll
    for (int p = 0; p < A_PER; ++p) {
      const int e = tid + p * 256;
      const int mm = AK ? e / BK : e % BM;
      const int kk = AK ? e % BK : e / BM;
      As[s][kk][mm] = ra[p];
    }
#pragma unroll
    for (int p = 0; p < B_PER; ++p) {
      const int e = tid + p * 256;
      const int nn = BN_FAST ? e % BN : e / BK;
      const int kk = BN_FAST ? e / BN : e % BK;
      Bs[s][kk][nn] = rb[p];
    }
  };

  const int64_t nk = (K + BK - 1) / BK;
  if (nk > 0) {
    load_tiles(0);
    store_tiles(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < nk;
    if (more) load_tiles((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      T af[TM], bfr[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = As[cur][kr][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bfr[j] = Bs[cur][kr][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mfma4(af[i], bfr[j], acc[i][j]);
    }
    if (more) store_tiles(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t col = n0 + wn * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (sizeof(T) == 8) ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int64_t row = m0 + wm * WM + i * 16 + rr;
        if (row < M && col < N) {
          T v = alpha * acc[i][j][r];
          if (beta != (T)0) v += beta * C[row * ldc + col];
          C[row * ldc + col] = v;
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 path: operands arrive as hi/lo BF16 pairs (x = hi + lo); three
// v_mfma_f32_16x16x32_bf16 per k step (lo*hi + hi*lo + hi*hi) with FP32
// accumulation.  The LDS tiles hold every operand row k-contiguous ([m][k]
// and [n][k], hi and lo apart), so the eight k values of one MFMA lane
// (row = lane % 16, k = 8 (lane / 16) + 0..7) are one 16-byte LDS read.
// BK = 32 is one MFMA k step; two LDS stages, one barrier per k tile, the
// next tile in flight from global memory while the MFMAs of this one run.
// Staging of an operand tile of R rows (R = 32, 64, 128) and 32 k values:
//   k fastest in memory: runs of 8 k values of one row, each one 16-byte
//     load and one 16-byte LDS write (R / 32 runs per thread);
//   rows fastest in memory: runs of 8 rows at KQ = R / 32 consecutive k
//     values per thread, transposed in registers into 8 LDS writes of KQ k
//     values; the lanes of a wavefront walk k first, so that each LDS write
//     instruction covers whole rows.
// VEC: every run starts 16-byte aligned (leading dimensions are multiples
// of 8); runs crossing an operand edge, and every run of VEC = false, load
// element by element.
typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));

constexpr int kB3K = 32;       // k values per staged tile
constexpr int kB3KP = 32 + 8;  // LDS row length (bf16): 80-byte rows, conflict-free 16-byte reads

template <bool VEC>
__device__ __forceinline__ bf8_t b3_run(const __bf16* p, int64_t fast, int64_t end, bool ok) {
  const __bf16 z = (__bf16)0.0f;
  bf8_t v = (bf8_t){z, z, z, z, z, z, z, z};
  if (!ok) return v;
  if (VEC && fast + 8 <= end) return *(const bf8_t*)p;
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (fast + i < end) v[i] = p[i];
  return v;
}

// one operand's staging: R rows of the tile, memory k-fast (KF) or rows-fast
template <int R, bool KF, bool VEC>
struct B3Op {
  static constexpr int KQ = R / 32;                // rows-fast: k values per thread
  static constexpr int NR = KF ? R / 32 : KQ;      // runs held per thread
  static constexpr int KQN = kB3K / KQ;            // rows-fast: k groups per row block
  bf8_t r[NR];

  __device__ __forceinline__ void load(const __bf16* hi, const __bf16* lo, int64_t ld, int64_t rows, int64_t K,
                                       int64_t r0, int64_t k0, int tid) {
    if constexpr (KF) {
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        const int u = tid + j * 256;
        const int arr = u / (4 * R), rem = u % (4 * R), row = rem >> 2, k8 = rem & 3;
        const int64_t gr = r0 + row, gk = k0 + 8 * k8;
        const __bf16* base = arr ? lo : hi;
        r[j] = b3_run<VEC>(base + (gr < rows ? gr : 0) * ld + gk, gk, K, gr < rows);
      }
    } else {
      const int arr = tid >> 7, u = tid & 127, kq = u % KQN, rb = u / KQN;
      const __bf16* base = arr ? lo : hi;
      const int64_t gr = r0 + 8 * rb;
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const int64_t gk = k0 + kq * KQ + q;
        r[q] = b3_run<VEC>(base + (gk < K ? gk : 0) * ld + gr, gr, rows, gk < K);
      }
    }
  }

  // S: this stage's [2 (hi, lo)][R][kB3KP]
  __device__ __forceinline__ void store(__bf16 (*S)[R][kB3KP], int tid) const {
    if constexpr (KF) {
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        const int u = tid + j * 256;
        const int arr = u / (4 * R), rem = u % (4 * R), row = rem >> 2, k8 = rem & 3;
        *(bf8_t*)&S[arr][row][8 * k8] = r[j];
      }
    } else {
      const int arr = tid >> 7, u = tid & 127, kq = u % KQN, rb = u / KQN;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        __bf16* d = &S[arr][8 * rb + i][kq * KQ];
        if constexpr (KQ == 4) {
          *(bf4_t*)d = (bf4_t){r[0][i], r[1][i], r[2][i], r[3][i]};
        } else if constexpr (KQ == 2) {
          *(bf2_t*)d = (bf2_t){r[0][i], r[1][i]};
        } else {
          *d = r[0][i];
        }
      }
    }
  }
};

template <int BM, int BN, bool AK, bool BN_FAST, bool VEC>
__global__ void __launch_bounds__(256, 2) gemm_bf16x3_kernel(int64_t M, int64_t N, int64_t K,
                                                             const __bf16* __restrict__ Ah,
                                                             const __bf16* __restrict__ Al, int64_t lda,
                                                             const __bf16* __restrict__ Bh,
                                                             const __bf16* __restrict__ Bl, int64_t ldb,
                                                             float* __restrict__ C, int64_t ldc, float alpha,
                                                             float beta, int64_t kchunk, int64_t cz, int m_fast) {
  {  // split-K: this z-slice owns K range [z*kchunk, z*kchunk + kchunk)
    const int64_t k0 = (int64_t)blockIdx.z * kchunk;
    const int64_t ao = AK ? k0 : k0 * lda, bo = BN_FAST ? k0 * ldb : k0;
    Ah += ao;
    Al += ao;
    Bh += bo;
    Bl += bo;
    C += (int64_t)blockIdx.z * cz;
    K = (K - k0 < kchunk) ? K - k0 : kchunk;
  }
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  __shared__ __attribute__((aligned(16))) __bf16 As[2][2][BM][kB3KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][2][BN][kB3KP];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t m0, n0;
  tile_of(M, N, BM, BN, m_fast, m0, n0, blockIdx.x);

  f4_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = (f4_t){0, 0, 0, 0};

  B3Op<BM, AK, VEC> sa;
  B3Op<BN, !BN_FAST, VEC> sb;
  const int64_t nk = (K + kB3K - 1) / kB3K;
  if (nk > 0) {
    sa.load(Ah, Al, lda, M, K, m0, 0, tid);
    sb.load(Bh, Bl, ldb, N, K, n0, 0, tid);
    sa.store(As[0], tid);
    sb.store(Bs[0], tid);
  }
  __syncthreads();
  const int kb = 8 * (lane >> 4);
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int cur = (int)(kt & 1);
    const bool more = kt + 1 < nk;
    if (more) {
      sa.load(Ah, Al, lda, M, K, m0, (kt + 1) * kB3K, tid);
      sb.load(Bh, Bl, ldb, N, K, n0, (kt + 1) * kB3K, tid);
    }
    bf8_t ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm * WM + i * 16 + (lane & 15);
      ah[i] = *(const bf8_t*)&As[cur][0][r][kb];
      al[i] = *(const bf8_t*)&As[cur][1][r][kb];
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int c = wn * WN + j * 16 + (lane & 15);
      bh[j] = *(const bf8_t*)&Bs[cur][0][c][kb];
      bl[j] = *(const bf8_t*)&Bs[cur][1][c][kb];
    }
    // the three products in three sweeps over the accumulators: consecutive
    // MFMAs never wait on each other's result
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
    if (more) {
      sa.store(As[cur ^ 1], tid);
      sb.store(Bs[cur ^ 1], tid);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t col = n0 + wn * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm * WM + i * 16 + 4 * (lane >> 4) + r;
        if (row < M && col < N) {
          float v = alpha * acc[i][j][r];
          if (beta != 0.0f) v += beta * C[row * ldc + col];
          C[row * ldc + col] = v;
        }
      }
    }
}
// ---------------------------------------------------------------------------
// Grouped GEMMs: one persistent launch computes the tiles of many GEMMs that
// share a kernel instantiation.  Each workgroup takes the next index of a
// device work queue (one counter per launch), finds the GEMM the index
// belongs to (each item holds its first index; its tiles follow), and runs
// that tile through the body of the single-GEMM kernel, so every tile gives
// the bits the single launch gives; workgroups leave when the queue is
// exhausted.
struct GroupItem {
  int64_t M, N, K, lda, ldb, ldc;
  const void* A;
  const void* B;
  void* C;
  double alpha, beta;
  int64_t first;           // first queue index; the item's tiles follow, split-K slice by slice
  int64_t nmn;             // output tiles per split-K slice
  int64_t kchunk, cz;      // split-K: k values per slice, partial-product stride (0: no split)
  int m_fast;
};

__global__ void grouped_reset_kernel(unsigned long long* __restrict__ q, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) q[i] = 0;
}

template <typename T, int BM, int BN, bool AK, bool BN_FAST, int VW>
__global__ void __launch_bounds__(256, 2) gemm_grouped_kernel(const GroupItem* __restrict__ items, int nitems,
                                                              int64_t total, unsigned long long* __restrict__ queue) {
  __shared__ int64_t w_s;
  for (;;) {
    if (threadIdx.x == 0) w_s = (int64_t)atomicAdd(queue, 1ull);
    __syncthreads();
    const int64_t w = w_s;
    if (w >= total) return;  // uniform over the workgroup
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (items[mid].first <= w)
        lo = mid;
      else
        hi = mid - 1;
    }
    const GroupItem& it = items[lo];
    const int64_t rem = w - it.first, z = rem / it.nmn;
    gemm_k4_body<T, BM, BN, AK, BN_FAST, 16, VW>(it.M, it.N, it.K, (const T*)it.A, it.lda, (const T*)it.B, it.ldb,
                                                 (T*)it.C, it.ldc, (T)it.alpha, (T)it.beta, it.kchunk, it.cz,
                                                 it.m_fast, rem - z * it.nmn, z);
    __syncthreads();  // the tile's LDS and w_s are reused by the next index
  }
}

// ---------------------------------------------------------------------------
// Tile table used by the planner and the autotuner.
struct TileCfg {
  int bm, bn;
  int bk;  // double-buffered k-tile depth (FP64 / FP32); 0 = single-buffered
  int kd;  // single-buffered k depth: 16 or 32
};
static const TileCfg kTiles[] = {{64, 64, 0, 16},   {128, 64, 0, 16},  {64, 128, 0, 16},  {128, 128, 0, 16},
                                 {32, 64, 0, 16},   {64, 32, 0, 16},   {128, 128, 16, 0}, {128, 128, 32, 0},
                                 {128, 64, 32, 0},  {64, 128, 32, 0},  {64, 64, 32, 0},   {256, 64, 0, 16},
                                 {64, 256, 0, 16},  {128, 128, 0, 32}, {128, 64, 0, 32},  {256, 128, 0, 16},
                                 {128, 256, 0, 16}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

// the last two tiles are FP32-only (the other precisions would run them as tile 3)
int gemm_num_tiles(Prec p) { return p == Prec::FP32 ? kNumTiles : kNumTiles - 2; }

static int default_tile(const GemmArgs& g) {
  // Prefer big tiles when the grid still fills the 256 CUs several times.
  auto blocks = [&](int bm, int bn) { return ((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn); };
  if (g.M >= 128 && g.N >= 128 && blocks(128, 128) >= 1024) return 3;
  if (g.M >= 128 && blocks(128, 64) >= 1024) return 1;
  if (g.N >= 128 && blocks(64, 128) >= 1024) return 2;
  if (g.M <= 32) return 4;
  if (g.N <= 32) return 5;
  return 0;
}

// Tile walk order: M fastest when B (K x N) is the larger operand, so that the
// workgroups of one XCD sharing a B column strip run back to back; N fastest
// otherwise.
static int m_fast_order(const GemmArgs& g) { return g.N > g.M ? 1 : 0; }

// reduction of split-K partials: C = alpha * sum_z P[z] + beta * C
template <typename T>
__global__ void __launch_bounds__(256) splitk_reduce_kernel(const T* __restrict__ P, int split, int64_t M, int64_t N,
                                                            T* __restrict__ C, int64_t ldc, T alpha, T beta) {
  const int64_t total = M * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    T s = 0;
    for (int z = 0; z < split; ++z) s += P[(int64_t)z * total + i];
    const int64_t r = i / N, c = i - r * N;
    T v = alpha * s;
    if (beta != (T)0) v += beta * C[r * ldc + c];
    C[r * ldc + c] = v;
  }
}

// Few outputs with many partials: one wavefront per output, each lane
// summing a fixed strided subset of the partials, then a fixed shuffle tree.
template <typename T>
__global__ void __launch_bounds__(256) splitk_reduce_wave_kernel(const T* __restrict__ P, int split, int64_t M,
                                                                 int64_t N, T* __restrict__ C, int64_t ldc, T alpha,
                                                                 T beta) {
  const int64_t total = M * N;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= total) return;  // uniform per wavefront
  T acc = 0;
  for (int z = lane; z < split; z += 64) acc += P[(int64_t)z * total + i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) {
    const int64_t r = i / N, c = i - r * N;
    T v = alpha * acc;
    if (beta != (T)0) v += beta * C[r * ldc + c];
    C[r * ldc + c] = v;
  }
}

// C = alpha * sum_z P[z] + beta * C over the split-K partials (deterministic:
// the order depends on the shape only)
template <typename T>
static void launch_splitk_reduce(const T* P, int split, int64_t M, int64_t N, T* C, int64_t ldc, T alpha, T beta,
                                 hipStream_t s) {
  const int64_t total = M * N;
  if (total < 16384 && split >= 64) {
    splitk_reduce_wave_kernel<T><<<dim3((unsigned)((total + 3) / 4)), 256, 0, s>>>(P, split, M, N, C, ldc, alpha,
                                                                                   beta);
  } else {
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    splitk_reduce_kernel<T><<<dim3((unsigned)blocks), 256, 0, s>>>(P, split, M, N, C, ldc, alpha, beta);
  }
}

// Tiles whose staged elements split into whole 16-byte vectors per thread.
template <typename T, int BM, int BN, int KD>
constexpr bool k4_vectorizable() {
  constexpr int vw = 16 / sizeof(T);
  return (BM * KD) % (vw * 256) == 0 && (BN * KD) % (vw * 256) == 0;
}

template <typename T, int BM, int BN, bool AK, bool BF, int KD>
static void k4_launch(dim3 grid, hipStream_t s, const GemmArgs& g, const T* A, const T* B, T* C, int64_t ldc, T al,
                      T be, int64_t kchunk, int64_t cz, int mf, bool vec) {
  if constexpr (k4_vectorizable<T, BM, BN, KD>()) {
    if (vec) {
      if constexpr (KD == 32)
        gemm_k32v_kernel<T, BM, BN, AK, BF><<<grid, 256, 0, s>>>(g.M, g.N, g.K, A, g.lda, B, g.ldb, C, ldc, al, be,
                                                                kchunk, cz, mf);
      else
        gemm_k4v_kernel<T, BM, BN, AK, BF><<<grid, 256, 0, s>>>(g.M, g.N, g.K, A, g.lda, B, g.ldb, C, ldc, al, be,
                                                               kchunk, cz, mf);
      return;
    }
  }
  if constexpr (KD == 32)
    gemm_k32_kernel<T, BM, BN, AK, BF><<<grid, 256, 0, s>>>(g.M, g.N, g.K, A, g.lda, B, g.ldb, C, ldc, al, be, kchunk,
                                                           cz, mf);
  else
    gemm_k4_kernel<T, BM, BN, AK, BF><<<grid, 256, 0, s>>>(g.M, g.N, g.K, A, g.lda, B, g.ldb, C, ldc, al, be, kchunk,
                                                          cz, mf);
}

// Both operands' rows (and split-K slices, cut at multiples of 16 k) start
// 16-byte aligned: the vector-load tiles apply.
static bool gemm_rows_aligned(const GemmArgs& g) {
  const int64_t vw = g.prec == Prec::FP64 ? 2 : 4;
  return g.prec != Prec::BF16X3 && ((uintptr_t)g.A % 16) == 0 && ((uintptr_t)g.B % 16) == 0 && g.lda % vw == 0 &&
         g.ldb % vw == 0;
}

template <typename T, int BM, int BN, int KD = 16>
static void launch_k4(const GemmArgs& g, hipStream_t s) {
  const int split = g.split > 1 ? g.split : 1;
  const int64_t kchunk = split > 1 ? (((g.K + split - 1) / split + KD - 1) / KD) * KD : (g.K > 0 ? g.K : 1);
  const int nz = split > 1 ? (int)((g.K + kchunk - 1) / kchunk) : 1;
  dim3 grid((unsigned)(((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM)), 1u, (unsigned)nz);
  const int mf = m_fast_order(g);
  const T* A = (const T*)g.A;
  const T* B = (const T*)g.B;
  T* C = split > 1 ? (T*)g.ws : (T*)g.C;
  const int64_t ldc = split > 1 ? g.N : g.ldc;
  const int64_t cz = split > 1 ? g.M * g.N : 0;
  T al = split > 1 ? (T)1 : (T)g.alpha, be = split > 1 ? (T)0 : (T)g.beta;
  const bool vec = gemm_rows_aligned(g);
  if (g.a_kfast && g.b_nfast)
    k4_launch<T, BM, BN, true, true, KD>(grid, s, g, A, B, C, ldc, al, be, kchunk, cz, mf, vec);
  else if (g.a_kfast)
    k4_launch<T, BM, BN, true, false, KD>(grid, s, g, A, B, C, ldc, al, be, kchunk, cz, mf, vec);
  else if (g.b_nfast)
    k4_launch<T, BM, BN, false, true, KD>(grid, s, g, A, B, C, ldc, al, be, kchunk, cz, mf, vec);
  else
    k4_launch<T, BM, BN, false, false, KD>(grid, s, g, A, B, C, ldc, al, be, kchunk, cz, mf, vec);
  if (split > 1) {
    launch_splitk_reduce<T>((const T*)g.ws, nz, g.M, g.N, (T*)g.C, g.ldc, (T)g.alpha, (T)g.beta, s);
  }
}

// Every operand row (and split-K slice, cut at multiples of 32 k) of both
// split-BF16 operands starts 16-byte aligned: the vector-load staging applies.
static bool b3_rows_aligned(const GemmArgs& g) {
  auto al = [](const void* p) { return ((uintptr_t)p % 16) == 0; };
  return al(g.A) && al(g.A_lo) && al(g.B) && al(g.B_lo) && g.lda % 8 == 0 && g.ldb % 8 == 0;
}

template <int BM, int BN, bool AK, bool BF>
static void b3_launch(dim3 grid, hipStream_t s, const GemmArgs& g, float* C, int64_t ldc, float al, float be,
                      int64_t kchunk, int64_t cz, int mf, bool vec) {
  const __bf16 *Ah = (const __bf16*)g.A, *Al = (const __bf16*)g.A_lo;
  const __bf16 *Bh = (const __bf16*)g.B, *Bl = (const __bf16*)g.B_lo;
  if (vec)
    gemm_bf16x3_kernel<BM, BN, AK, BF, true><<<grid, 256, 0, s>>>(g.M, g.N, g.K, Ah, Al, g.lda, Bh, Bl, g.ldb, C, ldc,
                                                                  al, be, kchunk, cz, mf);
  else
    gemm_bf16x3_kernel<BM, BN, AK, BF, false><<<grid, 256, 0, s>>>(g.M, g.N, g.K, Ah, Al, g.lda, Bh, Bl, g.ldb, C,
                                                                   ldc, al, be, kchunk, cz, mf);
}

template <int BM, int BN>
static void launch_b3(const GemmArgs& g, hipStream_t s) {
  const int split = g.split > 1 ? g.split : 1;
  const int64_t kchunk =
      split > 1 ? (((g.K + split - 1) / split + kB3K - 1) / kB3K) * kB3K : (g.K > 0 ? g.K : 1);
  const int nz = split > 1 ? (int)((g.K + kchunk - 1) / kchunk) : 1;
  dim3 grid((unsigned)(((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM)), 1u, (unsigned)nz);
  const int mf = m_fast_order(g);
  float* C = split > 1 ? (float*)g.ws : (float*)g.C;
  const int64_t ldc = split > 1 ? g.N : g.ldc;
  const int64_t cz = split > 1 ? g.M * g.N : 0;
  float al = split > 1 ? 1.0f : (float)g.alpha, be = split > 1 ? 0.0f : (float)g.beta;
  const bool vec = b3_rows_aligned(g);
  if (g.a_kfast && g.b_nfast)
    b3_launch<BM, BN, true, true>(grid, s, g, C, ldc, al, be, kchunk, cz, mf, vec);
  else if (g.a_kfast)
    b3_launch<BM, BN, true, false>(grid, s, g, C, ldc, al, be, kchunk, cz, mf, vec);
  else if (g.b_nfast)
    b3_launch<BM, BN, false, true>(grid, s, g, C, ldc, al, be, kchunk, cz, mf, vec);
  else
    b3_launch<BM, BN, false, false>(grid, s, g, C, ldc, al, be, kchunk, cz, mf, vec);
  if (split > 1) {
    launch_splitk_reduce<float>((const float*)g.ws, nz, g.M, g.N, (float*)g.C, g.ldc, (float)g.alpha,
                                (float)g.beta, s);
  }
}

template <int BM, int BN>
static void dispatch_tile(const GemmArgs& g, hipStream_t s) {
  if (g.prec == Prec::FP64)
    launch_k4<double, BM, BN>(g, s);
  else if (g.prec == Prec::FP32)
    launch_k4<float, BM, BN>(g, s);
  else
    launch_b3<BM, BN>(g, s);
}

// FP32-only tiles: a 128 x 64 (or 64 x 128) block per wavefront, the register
// budget of the FP64 128 x 128 tile; FP64 and split-BF16 run them as 128 x 128.
template <int BM, int BN>
static void dispatch_f32(const GemmArgs& g, hipStream_t s) {
  if (g.prec == Prec::FP32)
    launch_k4<float, BM, BN>(g, s);
  else if (g.prec == Prec::FP64)
    launch_k4<double, 128, 128>(g, s);
  else
    launch_b3<128, 128>(g, s);
}

// BK = 32 single-buffered tiles (FP64 / FP32); split-BF16 runs its own kernel.
template <int BM, int BN>
static void dispatch_k32(const GemmArgs& g, hipStream_t s) {
  if (g.prec == Prec::FP64)
    launch_k4<double, BM, BN, 32>(g, s);
  else if (g.prec == Prec::FP32)
    launch_k4<float, BM, BN, 32>(g, s);
  else
    launch_b3<BM, BN>(g, s);
}

// Tall and wide single-buffered tiles (one operand re-read fewer times when
// the other extent is small); split-BF16 runs them as 128 x 64.
template <int BM, int BN>
static void dispatch_tall(const GemmArgs& g, hipStream_t s) {
  if (g.prec == Prec::FP64)
    launch_k4<double, BM, BN>(g, s);
  else if (g.prec == Prec::FP32)
    launch_k4<float, BM, BN>(g, s);
  else
    launch_b3<128, 64>(g, s);
}

template <typename T, int BM, int BN, int BK>
static void launch_db(const GemmArgs& g, hipStream_t s) {
  const int split = g.split > 1 ? g.split : 1;
  const int64_t kchunk = split > 1 ? (((g.K + split - 1) / split + BK - 1) / BK) * BK : (g.K > 0 ? g.K : 1);
  const int nz = split > 1 ? (int)((g.K + kchunk - 1) / kchunk) : 1;
  dim3 grid((unsigned)(((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM)), 1u, (unsigned)nz);
  const int mf = m_fast_order(g);
  const T* A = (const T*)g.A;
  const T* B = (const T*)g.B;
  T* C = split > 1 ? (T*)g.ws : (T*)g.C;
  const int64_t ldc = split > 1 ? g.N : g.ldc;
  const int64_t cz = split > 1 ? g.M * g.N : 0;
  T al = split > 1 ? (T)1 : (T)g.alpha, be = split > 1 ? (T)0 : (T)g.beta;
  if (g.a_kfast && g.b_nfast)
    gemm_db_kernel<T, BM, BN, BK, true, true><<<grid, 256, 0, s>>>(g.M, g.N, g.K, A, g.lda, B, g.ldb, C, ldc, al,
                                                                   be, kchunk, cz, mf);
  else if (g.a_kfast)
    gemm_db_kernel<T, BM, BN, BK, true, false><<<grid, 256, 0, s>>>(g.M, g.N, g.K, A, g.lda, B, g.ldb, C, ldc, al,
                                                                    be, kchunk, cz, mf);
  else if (g.b_nfast)
    gemm_db_kernel<T, BM, BN, BK, false, true><<<grid, 256, 0, s>>>(g.M, g.N, g.K, A, g.lda, B, g.ldb, C, ldc, al,
                                                                    be, kchunk, cz, mf);
  else
    gemm_db_kernel<T, BM, BN, BK, false, false><<<grid, 256, 0, s>>>(g.M, g.N, g.K, A, g.lda, B, g.ldb, C, ldc,
                                                                     al, be, kchunk, cz, mf);
  if (split > 1) {
    launch_splitk_reduce<T>((const T*)g.ws, nz, g.M, g.N, (T*)g.C, g.ldc, (T)g.alpha, (T)g.beta, s);
  }
}

// double-buffered configurations: FP64/FP32 kernels; split-BF16 keeps its own kernel
template <int BM, int BN, int BK>
static void dispatch_db(const GemmArgs& g, hipStream_t s) {
  if (g.prec == Prec::FP64)
    launch_db<double, BM, BN, BK>(g, s);
  else if (g.prec == Prec::FP32)
    launch_db<float, BM, BN, BK>(g, s);
  else
    launch_b3<BM, BN>(g, s);
}

int gemm_split_factor(const GemmArgs& g) {
  // about 2048 workgroups (eight per CU) for small outputs with a long sum;
  // chunks of >= 128 k
  const int t = (g.tile >= 0 && g.tile < kNumTiles) ? g.tile : default_tile(g);
  const int64_t tiles = ((g.M + kTiles[t].bm - 1) / kTiles[t].bm) * ((g.N + kTiles[t].bn - 1) / kTiles[t].bn);
  if (tiles >= 512 || g.K < 512) return 1;
  int64_t s = (2048 + tiles - 1) / tiles;
  s = std::min<int64_t>(s, g.K / 128);
  s = std::min<int64_t>(s, kMaxSplit);
  return s < 2 ? 1 : (int)s;
}

size_t gemm_split_bytes(const GemmArgs& g, int split) {
  return (size_t)split * (size_t)(g.M * g.N) * (g.prec == Prec::FP64 ? 8 : 4);
}

int gemm_default_tile(const GemmArgs& g) { return default_tile(g); }

int64_t gemm_tiles(const GemmArgs& g) {
  const int t = (g.tile >= 0 && g.tile < kNumTiles) ? g.tile : default_tile(g);
  return ((g.M + kTiles[t].bm - 1) / kTiles[t].bm) * ((g.N + kTiles[t].bn - 1) / kTiles[t].bn) *
         (g.split > 1 ? g.split : 1);
}

std::string gemm_label(const GemmArgs& g) {
  int t = (g.tile >= 0 && g.tile < kNumTiles) ? g.tile : default_tile(g);
  if (t >= 15 && g.prec != Prec::FP32) t = 3;  // FP32-only tiles run as 128 x 128
  std::string bm = std::to_string(kTiles[t].bm), bn = std::to_string(kTiles[t].bn);
  std::string lay = std::string(g.a_kfast ? "true" : "false") + ", " + (g.b_nfast ? "true" : "false");
  if (g.prec == Prec::BF16X3) {
    if (kTiles[t].bm == 256 || kTiles[t].bn == 256) bm = "128", bn = "64";
    return "fno::gemm_bf16x3_kernel<" + bm + ", " + bn + ", " + lay + ", " + (b3_rows_aligned(g) ? "true" : "false") +
           ">";
  }
  if (kTiles[t].bk > 0)
    return std::string("fno::gemm_db_kernel<") + (g.prec == Prec::FP64 ? "double" : "float") + ", " + bm + ", " +
           bn + ", " + std::to_string(kTiles[t].bk) + ", " + lay + ">";
  const int vw = g.prec == Prec::FP64 ? 2 : 4, kd = kTiles[t].kd;
  const bool vec = gemm_rows_aligned(g) && (kTiles[t].bm * kd) % (vw * 256) == 0 && (kTiles[t].bn * kd) % (vw * 256) == 0;
  const char* name = kd == 32 ? (vec ? "fno::gemm_k32v_kernel<" : "fno::gemm_k32_kernel<")
                              : (vec ? "fno::gemm_k4v_kernel<" : "fno::gemm_k4_kernel<");
  return std::string(name) + (g.prec == Prec::FP64 ? "double" : "float") + ", " + bm + ", " + bn + ", " + lay + ">";
}

void launch_gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M == 0 || g.N == 0) return;
  int t = (g.tile >= 0 && g.tile < kNumTiles) ? g.tile : default_tile(g);
  switch (t) {
    case 0: dispatch_tile<64, 64>(g, s); break;
    case 1: dispatch_tile<128, 64>(g, s); break;
    case 2: dispatch_tile<64, 128>(g, s); break;
    case 3: dispatch_tile<128, 128>(g, s); break;
    case 4: dispatch_tile<32, 64>(g, s); break;
    case 5: dispatch_tile<64, 32>(g, s); break;
    case 6: dispatch_db<128, 128, 16>(g, s); break;
    case 7: dispatch_db<128, 128, 32>(g, s); break;
    case 8: dispatch_db<128, 64, 32>(g, s); break;
    case 9: dispatch_db<64, 128, 32>(g, s); break;
    case 10: dispatch_db<64, 64, 32>(g, s); break;
    case 11: dispatch_tall<256, 64>(g, s); break;
    case 12: dispatch_tall<64, 256>(g, s); break;
    case 13: dispatch_k32<128, 128>(g, s); break;
    case 14: dispatch_k32<128, 64>(g, s); break;
    case 15: dispatch_f32<256, 128>(g, s); break;
    default: dispatch_f32<128, 256>(g, s); break;
  }
  FNO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Grouped launches (host side)
size_t gemm_group_item_bytes() { return sizeof(GroupItem); }

namespace {
constexpr int kGroupTiles = 6;  // the single-buffered 16-deep tiles (the defaults)
constexpr int kGroupKeys = 2 * kGroupTiles * 8;  // precision x tile x (A layout, B layout, vector loads)

template <typename T, int BM, int BN>
void grouped_launch_tile(int key_lay, const GroupItem* dev, int n, int64_t total, unsigned long long* q,
                         hipStream_t s) {
  const unsigned grid = (unsigned)std::min<int64_t>(total, 1024);
  const bool ak = key_lay & 1, bf = key_lay & 2, vec = key_lay & 4;
  constexpr int V = 16 / sizeof(T);
  if constexpr (k4_vectorizable<T, BM, BN, 16>()) {
    if (vec) {
      if (ak && bf)
        gemm_grouped_kernel<T, BM, BN, true, true, V><<<grid, 256, 0, s>>>(dev, n, total, q);
      else if (ak)
        gemm_grouped_kernel<T, BM, BN, true, false, V><<<grid, 256, 0, s>>>(dev, n, total, q);
      else if (bf)
        gemm_grouped_kernel<T, BM, BN, false, true, V><<<grid, 256, 0, s>>>(dev, n, total, q);
      else
        gemm_grouped_kernel<T, BM, BN, false, false, V><<<grid, 256, 0, s>>>(dev, n, total, q);
      return;
    }
  }
  if (ak && bf)
    gemm_grouped_kernel<T, BM, BN, true, true, 1><<<grid, 256, 0, s>>>(dev, n, total, q);
  else if (ak)
    gemm_grouped_kernel<T, BM, BN, true, false, 1><<<grid, 256, 0, s>>>(dev, n, total, q);
  else if (bf)
    gemm_grouped_kernel<T, BM, BN, false, true, 1><<<grid, 256, 0, s>>>(dev, n, total, q);
  else
    gemm_grouped_kernel<T, BM, BN, false, false, 1><<<grid, 256, 0, s>>>(dev, n, total, q);
}

template <typename T>
void grouped_launch(int tile, int key_lay, const GroupItem* dev, int n, int64_t total, unsigned long long* q,
                    hipStream_t s) {
  switch (tile) {
    case 0: grouped_launch_tile<T, 64, 64>(key_lay, dev, n, total, q, s); break;
    case 1: grouped_launch_tile<T, 128, 64>(key_lay, dev, n, total, q, s); break;
    case 2: grouped_launch_tile<T, 64, 128>(key_lay, dev, n, total, q, s); break;
    case 3: grouped_launch_tile<T, 128, 128>(key_lay, dev, n, total, q, s); break;
    case 4: grouped_launch_tile<T, 32, 64>(key_lay, dev, n, total, q, s); break;
    default: grouped_launch_tile<T, 64, 32>(key_lay, dev, n, total, q, s); break;
  }
}
}  // namespace

int gemm_group_max_launches() { return kGroupKeys; }

void launch_gemm_grouped(const std::vector<GemmArgs>& gs, void* pin, void* dev, void* queue, hipStream_t s) {
  // bucket the GEMMs by kernel instantiation; the others run one by one
  std::vector<std::vector<int>> bucket(kGroupKeys);
  for (int i = 0; i < (int)gs.size(); ++i) {
    GemmArgs g = gs[i];
    g.tile = -1;
    if (g.M == 0 || g.N == 0) continue;
    const int t = default_tile(g);
    if (g.prec == Prec::BF16X3 || t >= kGroupTiles || (g.split > 1 && !g.ws)) {
      g.tile = t;
      if (!g.ws) g.split = 1;
      launch_gemm(g, s);
      continue;
    }
    const bool vec = gemm_rows_aligned(g);
    const int lay = (g.a_kfast ? 1 : 0) | (g.b_nfast ? 2 : 0) | (vec ? 4 : 0);
    bucket[((g.prec == Prec::FP64 ? 0 : 1) * kGroupTiles + t) * 8 + lay].push_back(i);
  }
  GroupItem* hp = (GroupItem*)pin;
  int used = 0;
  std::vector<std::pair<int, int>> reduce;  // (GEMM, slices) of the split-K items
  struct Launch {
    int key, off, n;
    int64_t total;
  };
  std::vector<Launch> launches;
  for (int key = 0; key < kGroupKeys; ++key) {
    if (bucket[key].empty()) continue;
    const int tile = (key / 8) % kGroupTiles;
    Launch L{key, used, 0, 0};
    for (int i : bucket[key]) {
      const GemmArgs& g = gs[i];
      GroupItem it{};
      it.M = g.M;
      it.N = g.N;
      it.K = g.K;
      it.lda = g.lda;
      it.ldb = g.ldb;
      it.A = g.A;
      it.B = g.B;
      it.first = L.total;
      it.nmn = ((g.M + kTiles[tile].bm - 1) / kTiles[tile].bm) * ((g.N + kTiles[tile].bn - 1) / kTiles[tile].bn);
      it.m_fast = m_fast_order(g);
      int64_t nz = 1;
      if (g.split > 1) {  // partial products of the K slices into g.ws, summed after the launch
        it.kchunk = (((g.K + g.split - 1) / g.split + 15) / 16) * 16;
        nz = (g.K + it.kchunk - 1) / it.kchunk;
        it.C = g.ws;
        it.ldc = g.N;
        it.cz = g.M * g.N;
        it.alpha = 1.0;
        it.beta = 0.0;
        reduce.push_back({i, (int)nz});
      } else {
        it.kchunk = g.K > 0 ? g.K : 1;
        it.cz = 0;
        it.C = g.C;
        it.ldc = g.ldc;
        it.alpha = g.alpha;
        it.beta = g.beta;
      }
      L.total += it.nmn * nz;
      hp[used++] = it;
      ++L.n;
    }
    launches.push_back(L);
  }
  if (launches.empty()) return;
  FNO_HIP(hipMemcpyAsync(dev, hp, sizeof(GroupItem) * (size_t)used, hipMemcpyHostToDevice, s));
  unsigned long long* q = (unsigned long long*)queue;
  grouped_reset_kernel<<<1, 128, 0, s>>>(q, (int)launches.size());
  for (size_t j = 0; j < launches.size(); ++j) {
    const Launch& L = launches[j];
    const int tile = (L.key / 8) % kGroupTiles, lay = L.key % 8;
    const GroupItem* d = (const GroupItem*)dev + L.off;
    if (L.key / (8 * kGroupTiles) == 0)
      grouped_launch<double>(tile, lay, d, L.n, L.total, q + j, s);
    else
      grouped_launch<float>(tile, lay, d, L.n, L.total, q + j, s);
  }
  for (auto& r : reduce) {
    const GemmArgs& g = gs[r.first];
    if (g.prec == Prec::FP64)
      launch_splitk_reduce<double>((const double*)g.ws, r.second, g.M, g.N, (double*)g.C, g.ldc, g.alpha, g.beta, s);
    else
      launch_splitk_reduce<float>((const float*)g.ws, r.second, g.M, g.N, (float*)g.C, g.ldc, (float)g.alpha,
                                  (float)g.beta, s);
  }
  FNO_HIP(hipGetLastError());
}

}  // namespace fno
