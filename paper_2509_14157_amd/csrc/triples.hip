// Fused triples residual (see triples.hpp for the algebra).
//
// GEMM per occupied triple t: Y_t (v x C(v,2)) = A_t (v x K) B_t (K x C(v,2)),
// K = the K segments
//   0        pp-ladder   K = C(v,2)      A: T3 row t gathered, B: W3_vvvv^T
//   1        one-body    K = v           A: F3_vv,            B: T3 row t gathered
//   2..4     ring p      K = (o-2) v     A: W3_ovvo of x_p,   B: T3 rows (m, pair_p) gathered
//   5..7     driver p    K = v           A: T2 of pair_p,     B: W3_vvvo rows of x_p
//   8..10    driver p    K = o           A: W3_ovoo of pair_p, B: T2 rows (x_p, m)
// One workgroup (4 wavefronts, 2 x 2) computes a 64 x 128 tile of Y_t (the
// 64 rows cover every a < v <= 64 of the triple); the k tiles of all segments
// form one software pipeline: two LDS stages, one barrier per k tile, the
// next tile's gathers in flight while the MFMAs of the current one run.
#include "triples.hpp"

#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace fno {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct AccT;
template <>
struct AccT<double> {
  typedef d4_t type;
};
template <>
struct AccT<float> {
  typedef f4_t type;
};

__device__ __forceinline__ d4_t mma(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mma(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int cb2(int n) { return n * (n - 1) / 2; }
__device__ __forceinline__ int cb3(int n) { return n * (n - 1) * (n - 2) / 6; }

// colex rank of the sorted triple {x, p, q} (p < q) and the sign of the
// permutation that sorts (x, p, q); sign 0 when x equals p or q
__device__ __forceinline__ int tri_rank(int x, int p, int q, int& s) {
  if (x < p) {
    s = 1;
    return x + cb2(p) + cb3(q);
  }
  if (x < q) {
    s = (x == p) ? 0 : -1;
    return p + cb2(x) + cb3(q);
  }
  s = (x == q) ? 0 : 1;
  return p + cb2(q) + cb3(x);
}

constexpr int kBM = 64, kBN = 128, kBK = 16, kThreads = 256;
constexpr int kSegs = 11;
constexpr int kPanel = 16;  // triples per panel of the tile order

struct Params {
  R3FusedArgs a;
  IndexTables tb;
  int nv2, nv3, no2, nt, ntn;  // C(v,2), C(v,3), C(o,2), C(o,3), N tiles per triple
  int kt_begin[kSegs + 1];     // first k tile of each segment
  int seg_k[kSegs];            // K of each segment
  int ep;                      // padded e range of the ring segments (multiple of 16)
  int panel;                   // triples per panel of the tile order
};

// LDS tiles of one k tile: one stage for FP64 (24.4 KB, so that four
// workgroups fit a CU), two for FP32.  FP64 / FP32: k-major tiles, one
// element per lane per v_mfma_*_16x16x4 step.  Split-BF16: the staged FP32
// values split into hi + lo BF16 halves (x = hi + lo to about 16 bits),
// stored with k contiguous per row, so that the four k values of a lane of
// v_mfma_f32_16x16x16_bf16 (row = lane % 16, k = 4 (lane / 16) + 0..3) are
// one 8-byte LDS read; rows padded to 40 bytes.
constexpr int kB3Row = kBK + 4;
template <typename T, bool B3>
struct FusedTiles {
  static constexpr int kStages = sizeof(T) == 8 ? 1 : 2;
  T As[kStages][kBK][kBM + 1];
  __attribute__((aligned(16))) T Bs[kStages][kBK][kBN + ((sizeof(T) == 8) ? 2 : 4)];  // B rows 16-byte aligned
};
template <>
struct FusedTiles<float, true> {
  __attribute__((aligned(16))) unsigned short Ah[2][2][kBM][kB3Row];  // [stage][hi, lo][row a][k]
  __attribute__((aligned(16))) unsigned short Bh[2][2][kBN][kB3Row];  // [stage][hi, lo][column bc][k]
};

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef unsigned short u4_t __attribute__((ext_vector_type(4)));

// x = hi + lo, both rounded to nearest even BF16 (hi from x, lo from x - hi)
__device__ __forceinline__ void split_bf16(float x, unsigned short& h, unsigned short& l) {
  const __bf16 hb = (__bf16)x;
  const __bf16 lb = (__bf16)(x - (float)hb);
  h = __builtin_bit_cast(unsigned short, hb);
  l = __builtin_bit_cast(unsigned short, lb);
}

// Element mappings of the staged tiles (uniform per k tile):
//   A: 0 = rows of 16-byte vectors along k (pp-ladder, rows of T3v),
//      1 = one element per lane with k fastest, 2 = one element per lane with
//      the row fastest (k uniform per wavefront)
//   B: 0 = rows of 16-byte vectors along the columns (k uniform per vector
//      row: W3_vvvv^T, T3v), 1 = one element per lane, column fastest
// (B3: split-BF16 products from FP32 operands, T = float)
// (FP64: four waves per SIMD, i.e. at most 128 registers per lane)
template <typename T, bool B3 = false>
__global__ void __launch_bounds__(kThreads, sizeof(T) == 8 ? 4 : 2) r3_fused_kernel(Params P) {
  constexpr int VW = 16 / sizeof(T);          // elements per 16-byte vector
  constexpr int AV = kBM * kBK / VW / kThreads;  // A vectors per thread
  constexpr int BV = kBK * kBN / VW / kThreads;  // B vectors per thread
  typedef T Vec __attribute__((ext_vector_type(VW)));
  static_assert(AV * VW == 4 && BV * VW == 8, "slot counts");
  static_assert(!B3 || sizeof(T) == 4, "split-BF16 stages FP32 values");
  __shared__ FusedTiles<T, B3> L;
  const R3FusedArgs& g = P.a;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // tiles: each XCD takes a contiguous range of the tile order; the order
  // walks panels of `panel` triples, column tile by column tile, so the
  // tiles running together on an XCD share column strips of W3_vvvv^T and
  // of the ring's T3v rows, and the panel's own T3v rows, through its L2
  int t, n0;
  {
    const int64_t n = gridDim.x, b = blockIdx.x, q = n / 8, r = n % 8, x = b % 8, k = b / 8;
    const int64_t L = x * q + (x < r ? x : r) + k;
    const int64_t per = (int64_t)P.panel * P.ntn;
    const int pn = (int)(L / per);
    const int rem = (int)(L - pn * per);
    const int pe = min(P.panel, P.nt - pn * P.panel);
    t = pn * P.panel + rem % pe;
    n0 = (rem / pe) * kBN;
  }
  const int v = g.v, o = g.o, nv2 = P.nv2;
  const int64_t ldy = g.ldy;
  const uint8_t* d3 = P.tb.dec[3] + 3 * t;
  const int tt[3] = {d3[0], d3[1], d3[2]};
  const T* T3v = (const T*)g.T3v;
  const T* T3vt = T3v + (int64_t)t * v * ldy;
  const T* WT = (const T*)g.WT;

  typename AccT<T>::type acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (typename AccT<T>::type){0, 0, 0, 0};

  // a staged k tile in registers and the element mappings it was loaded with
  struct Regs {
    T a[4], b[8];
    int amode, bmode;
  };

  // placement p of the triple: x = t_p, pair (q0 < q1) = the other two
  auto placement = [&](int p, int& x, int& q0, int& q1) {
    x = tt[p];
    q0 = tt[p == 0 ? 1 : 0];
    q1 = tt[p == 2 ? 1 : 2];
  };
  // Unguarded row loads for the hot segments: every buffer they read is
  // padded so that rows a >= v, rows e >= v, columns >= C(v,2) and k beyond
  // the segment stay inside the allocation.  Those elements meet zeros in
  // the other operand (k) or land in accumulator rows / columns that are
  // never stored (a, bc).
  // A[a][kk] = scale * abase[a * lda + kk] (16 values per row)
  auto load_a_rows = [&](Regs& R, const auto* abase, int64_t lda, T scale) {
    typedef std::remove_cv_t<std::remove_pointer_t<decltype(abase)>> S;
    constexpr int SW = 16 / sizeof(S);
    typedef S SVec __attribute__((ext_vector_type(SW)));
    R.amode = 0;
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int q = tid + kThreads * i;
      const int a = q / (kBK / VW), kv = (q % (kBK / VW)) * VW;
      const SVec* src = (const SVec*)(abase + a * lda + kv);
#pragma unroll
      for (int h = 0; h < VW / SW; ++h) {
        const SVec y = src[h];
#pragma unroll
        for (int j = 0; j < SW; ++j) R.a[i * VW + h * SW + j] = scale * (T)y[j];
      }
    }
  };
  // k of the i-th B element a thread stages in the element-wise modes:
  // split-BF16 gives each thread 8 consecutive k of one column (stored as
  // k-contiguous LDS runs), the other precisions k = tid / 128 + 2 i
  auto bk = [&](int i) { return B3 ? 8 * (tid >> 7) + i : (tid >> 7) + 2 * i; };
  // B[kk][n] = scale * bbase[kk * ldb + n]  (bbase already at column n0)
  auto load_b_rows = [&](Regs& R, const T* bbase, int64_t ldb, T scale) {
    R.bmode = 0;
    if constexpr (B3) {
#pragma unroll
      for (int i = 0; i < 8; ++i) R.b[i] = scale * bbase[(int64_t)bk(i) * ldb + (tid & (kBN - 1))];
      return;
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int q = tid + kThreads * i;
      const int kk = q / (kBN / VW), nv = (q % (kBN / VW)) * VW;
      const Vec y = *(const Vec*)(bbase + kk * ldb + nv);
#pragma unroll
      for (int j = 0; j < VW; ++j) R.b[i * VW + j] = scale * y[j];
    }
  };

  auto load_tile = [&](int kt, Regs& R) {
    int s = 0;
#pragma unroll
    for (int q = 1; q < kSegs; ++q) s += (kt >= P.kt_begin[q]) ? 1 : 0;
    const int k0 = (kt - P.kt_begin[s]) * kBK;
    const int K = P.seg_k[s];
    if (s == 0) {
      // pp-ladder: A[a, ef] = T3v[t][a][ef], B[ef, bc] = W3_vvvv^T[ef][bc]
      load_a_rows(R, T3vt + k0, ldy, (T)1);
      load_b_rows(R, WT + (int64_t)k0 * ldy + n0, ldy, (T)1);
    } else if (s == 1) {
      // one-body: A[a, e] = F3_vv[a][e] (rows padded to ep), B[e, bc] = T3v[t][e][bc]
      load_a_rows(R, g.Fvvp + k0, P.ep, (T)1);
      load_b_rows(R, T3vt + (int64_t)k0 * ldy + n0, ldy, (T)1);
    } else if (s <= 4) {
      // ring, placement p: the k tiles walk m' (the o - 2 occupied m outside
      // the pair) and, for each, e in steps of 16 over the padded range ep;
      // A[a, e] = (-1)^p W3_ovvo[m][a][e][x], B[e, bc] = +-T3[m pair, e b c]
      const int p = s - 2;
      int x, q0, q1;
      placement(p, x, q0, q1);
      const int ltile = kt - P.kt_begin[s], per_m = P.ep / kBK;
      int m = ltile / per_m;
      const int e0 = (ltile - m * per_m) * kBK;
      m += (m >= q0) ? 1 : 0;
      m += (m >= q1) ? 1 : 0;
      int so;
      const int ro = tri_rank(m, q0, q1, so);
      const T sg = (T)(((p & 1) ? -1 : 1) * so);
      load_a_rows(R, g.Aring + ((int64_t)x * v * o + m) * P.ep + e0, (int64_t)o * P.ep, sg);
      load_b_rows(R, T3v + ((int64_t)ro * v + e0) * ldy + n0, ldy, (T)1);
      (void)K;
    } else if (s <= 7) {
      // driver: A[a, e] = (-1)^p T2[pair, a e], B[e, bc] = W3_vvvo[x][e][bc]
      const int p = s - 5;
      int x, q0, q1;
      placement(p, x, q0, q1);
      const double sp = (p & 1) ? -1.0 : 1.0;
      const double* t2row = g.T2 + (int64_t)(q0 + cb2(q1)) * nv2;
      R.amode = 2;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kk = wave + 4 * i, a = lane, k = k0 + kk;
        double val = 0;
        if (k < K && a < v && a != k) val = a < k ? sp * t2row[a + cb2(k)] : -sp * t2row[k + cb2(a)];
        R.a[i] = (T)val;
      }
      R.bmode = 1;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + bk(i), c = n0 + (tid & (kBN - 1));
        R.b[i] = (T)((k < K && c < nv2) ? g.Wvvvo[((int64_t)x * v + k) * nv2 + c] : 0.0);
      }
    } else {
      // driver: A[a, m] = -(-1)^p W3_ovoo[m][a][pair], B[m, bc] = T2[x m, bc]
      const int p = s - 8;
      int x, q0, q1;
      placement(p, x, q0, q1);
      const double sp = (p & 1) ? 1.0 : -1.0;
      const int pr = q0 + cb2(q1);
      R.amode = 2;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kk = wave + 4 * i, a = lane, k = k0 + kk;
        R.a[i] = (T)((k < K && a < v) ? sp * g.Wovoo[((int64_t)k * v + a) * P.no2 + pr] : 0.0);
      }
      R.bmode = 1;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + bk(i), c = n0 + (tid & (kBN - 1));
        double val = 0;
        if (k < K && c < nv2 && k != x) {
          const int lo = k < x ? k : x, hi = k < x ? x : k;
          const double sg = k < x ? -1.0 : 1.0;  // (x, m) sorted
          val = sg * g.T2[(int64_t)(lo + cb2(hi)) * nv2 + c];
        }
        R.b[i] = (T)val;
      }
    }
  };

  auto store_tile = [&](int st, const Regs& R) {
    if constexpr (B3) {
      // A rows: 4 consecutive k of row a per vector (mode 0) or single
      // elements; B: 8 consecutive k of one column per thread
      unsigned short h, l;
      if (R.amode == 0) {
        const int a = tid / (kBK / VW), kv = (tid % (kBK / VW)) * VW;
        u4_t vh, vl;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          split_bf16(R.a[j], h, l);
          vh[j] = h;
          vl[j] = l;
        }
        *(u4_t*)&L.Ah[st][0][a][kv] = vh;
        *(u4_t*)&L.Ah[st][1][a][kv] = vl;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = R.amode == 1 ? (tid & 15) : wave + 4 * i;
          const int a = R.amode == 1 ? (tid >> 4) + 16 * i : lane;
          split_bf16(R.a[i], h, l);
          L.Ah[st][0][a][k] = h;
          L.Ah[st][1][a][k] = l;
        }
      }
      {  // both B modes: 8 consecutive k of column c, two 8-byte runs per half
        const int c = tid & (kBN - 1), k8 = bk(0);
        u4_t vh[2], vl[2];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          split_bf16(R.b[i], h, l);
          vh[i >> 2][i & 3] = h;
          vl[i >> 2][i & 3] = l;
        }
        *(u4_t*)&L.Bh[st][0][c][k8] = vh[0];
        *(u4_t*)&L.Bh[st][0][c][k8 + 4] = vh[1];
        *(u4_t*)&L.Bh[st][1][c][k8] = vl[0];
        *(u4_t*)&L.Bh[st][1][c][k8 + 4] = vl[1];
      }
      return;
    } else {
    if (R.amode == 0) {
#pragma unroll
      for (int i = 0; i < AV; ++i) {
        const int q = tid + kThreads * i;
        const int a = q / (kBK / VW), kv = (q % (kBK / VW)) * VW;
#pragma unroll
        for (int j = 0; j < VW; ++j) L.As[st][kv + j][a] = R.a[i * VW + j];
      }
    } else if (R.amode == 1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) L.As[st][tid & 15][(tid >> 4) + 16 * i] = R.a[i];
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) L.As[st][wave + 4 * i][lane] = R.a[i];
    }
    if (R.bmode == 0) {
#pragma unroll
      for (int i = 0; i < BV; ++i) {
        const int q = tid + kThreads * i;
        const int kk = q / (kBN / VW), nv = (q % (kBN / VW)) * VW;
        Vec x;
#pragma unroll
        for (int j = 0; j < VW; ++j) x[j] = R.b[i * VW + j];
        *(Vec*)&L.Bs[st][kk][nv] = x;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) L.Bs[st][(tid >> 7) + 2 * i][tid & (kBN - 1)] = R.b[i];
    }
    }
  };

  const int nk = P.kt_begin[kSegs];
  // MFMAs of one LDS stage: the operands of k step s + 1 are read into the
  // other register set while the MFMAs of step s issue (the scheduler is asked
  // to interleave the LDS reads with the MFMAs), so a step's LDS latency is
  // covered by the previous step's matrix work
  auto mma_stage = [&](int cur) {
    if constexpr (B3) {
      // one 16 x 16 x 16 step per tile and block: lo*hi, hi*lo, then hi*hi,
      // each a sweep over the 8 accumulators
      const int kb = 4 * (lane >> 4);
      __builtin_amdgcn_s_setprio(1);
      s4_t ah[2], al[2], bh[4], bl[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = wm * 32 + i * 16 + (lane & 15);
        ah[i] = *(const s4_t*)&L.Ah[cur][0][r][kb];
        al[i] = *(const s4_t*)&L.Ah[cur][1][r][kb];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = wn * 64 + j * 16 + (lane & 15);
        bh[j] = *(const s4_t*)&L.Bh[cur][0][c][kb];
        bl[j] = *(const s4_t*)&L.Bh[cur][1][c][kb];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bh[j], acc[i][j], 0, 0, 0);
      __builtin_amdgcn_s_setprio(0);
      return;
    } else {
    T af[2][2], bf[2][4];
    auto read = [&](int ks, int r) {
      const int kr = ks + (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) af[r][i] = L.As[cur][kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[r][j] = L.Bs[cur][kr][wn * 64 + j * 16 + (lane & 15)];
    };
    __builtin_amdgcn_iglp_opt(0);
    if constexpr (sizeof(T) == 8) {
      // FP64 (four waves per SIMD): one operand register set, each k step's
      // operands read right before its MFMAs; the other waves cover the wait
#pragma unroll
      for (int st = 0; st < kBK / 4; ++st) {
        read(4 * st, 0);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = mma(af[0][i], bf[0][j], acc[i][j]);
      }
      return;
    }
    // FP32: the wave raises its priority while it issues its MFMAs, so that
    // the SIMD's other waves' staging work does not delay them (FP64 MFMAs
    // are long enough that this only slows the staging)
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(1);
    read(0, 0);
#pragma unroll
    for (int st = 0; st < kBK / 4; ++st) {
      const int r = st & 1;
      if (st + 1 < kBK / 4) read(4 * (st + 1), r ^ 1);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mma(af[r][i], bf[r][j], acc[i][j]);
    }
    if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(0);
    }
  };
  if constexpr (sizeof(T) == 4 && !B3) {
    // FP32: two k tiles in flight (the MFMA work of one tile is too short to
    // cover a global load): the loads of tile kt + 2 are issued before the
    // MFMAs of tile kt, while tile kt + 1, loaded one step earlier, is stored
    // to the other LDS stage after them.  (Split-BF16 keeps one tile in
    // flight: the second register set costs it a wave per SIMD, which loses
    // more than the deeper prefetch gains.)
    Regs R0, R1;
    load_tile(0, R0);
    store_tile(0, R0);
    if (nk > 1) load_tile(1, R1);
    __syncthreads();
    auto step = [&](int kt, Regs& Rfree, Regs& Rnext) {
      const int cur = kt & 1;
      if (kt + 2 < nk) load_tile(kt + 2, Rfree);
      mma_stage(cur);
      if (kt + 1 < nk) store_tile(cur ^ 1, Rnext);
      __syncthreads();
    };
    int kt = 0;
    for (; kt + 1 < nk; kt += 2) {
      step(kt, R0, R1);
      step(kt + 1, R1, R0);
    }
    if (kt < nk) step(kt, R0, R1);
  } else if constexpr (sizeof(T) == 8) {
    // FP64, one LDS stage: the loads of tile kt + 1 are issued before the
    // MFMAs of tile kt and stored into the stage once every wave has read it
    // (two barriers per k tile; four workgroups per CU keep the matrix pipes
    // fed across them)
    Regs R;
    load_tile(0, R);
    store_tile(0, R);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const bool more = kt + 1 < nk;
      if (more) load_tile(kt + 1, R);
      mma_stage(0);
      __syncthreads();
      if (more) {
        store_tile(0, R);
        __syncthreads();
      }
    }
  } else {
    // one k tile in flight: the loads of tile kt + 1 are issued before the
    // MFMAs of tile kt and stored to the other LDS stage after them
    Regs R;
    load_tile(0, R);
    store_tile(0, R);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      const bool more = kt + 1 < nk;
      if (more) load_tile(kt + 1, R);
      mma_stage(cur);
      if (more) store_tile(cur ^ 1, R);
      __syncthreads();
    }
  }

  // C/D layout of the 16x16 block: lane l holds column l % 16; FP64 rows
  // l / 16 + 4 r, FP32 rows 4 (l / 16) + r
  T* Y = (T*)g.Y + (int64_t)t * v * ldy;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (sizeof(T) == 8) ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int a = wm * 32 + i * 16 + rr;
        if (a < v && c < nv2) Y[(int64_t)a * ldy + c] = acc[i][j][r];
      }
    }
}

// T3v[t][x][p] = T3[t, x, p0, p1] (p = pair p0 < p1; zero for x in the pair
// and for p >= C(v,2)), one workgroup per occupied triple t and largest
// letter c.  The colex block T3[t, (a < b < c)] (C(c,2) values, contiguous)
// is read once, coalesced, and staged in LDS; it supplies
//   row c, pairs p < C(c,2):            T3v[t][c][a + C(b,2)] = T3[t, abc]
//   rows x <= c, pairs (p0, c):         T3v[t][x][p0 + C(c,2)] = -T3[t, p0 x c] (p0 < x)
//                                                               +T3[t, x p0 c] (p0 > x)
//                                                               0              (p0 == x or x == c)
// and the padding pairs p >= C(v,2) of row c.  Every element of T3v is
// written by exactly one workgroup; the workgroups after the last triple
// write the padding rows.
constexpr int kT3vMaxV = 64;

template <typename T>
__global__ void __launch_bounds__(256) r3_t3v_kernel(int v, int nv2, int nv3, int64_t ldy, int64_t rows,
                                                     const double* __restrict__ T3, T* __restrict__ T3v) {
  __shared__ double blk[kT3vMaxV * (kT3vMaxV - 1) / 2];
  const int64_t nblk = rows;  // one per (t, c)
  const int tid = threadIdx.x;
  if ((int64_t)blockIdx.x >= nblk) {  // padding row
    T* dst = T3v + (rows + ((int64_t)blockIdx.x - nblk)) * ldy;
    for (int64_t i = tid; i < ldy; i += 256) dst[i] = (T)0;
    return;
  }
  const int t = (int)(blockIdx.x / v), c = (int)(blockIdx.x % v);
  const int nc = cb2(c);
  const double* src = T3 + (int64_t)t * nv3 + cb3(c);
  T* rowc = T3v + ((int64_t)t * v + c) * ldy;
  for (int i = tid; i < nc; i += 256) {
    const double x = src[i];
    blk[i] = x;
    rowc[i] = (T)x;
  }
  for (int i = nc + tid; i < nc + c; i += 256) rowc[i] = (T)0;
  for (int64_t i = nv2 + tid; i < ldy; i += 256) rowc[i] = (T)0;
  __syncthreads();
  T* band = T3v + (int64_t)t * v * ldy + nc;
  for (int e = tid; e < c * c; e += 256) {
    const int x = e / c, p0 = e - x * c;
    const double val = p0 < x ? -blk[p0 + cb2(x)] : (p0 > x ? blk[x + cb2(p0)] : 0.0);
    band[(int64_t)x * ldy + p0] = (T)val;
  }
}

// WT[ef][bc] = W[bc][ef] (square C(v,2) matrix, rows of WT padded to ldy with
// zeros), through 32 x 32 LDS tiles
template <typename T>
__global__ void __launch_bounds__(256) r3_wt_kernel(int n, int64_t ldy, int64_t rows_all, const double* __restrict__ W,
                                                    T* __restrict__ WT) {
  __shared__ double tile[32][33];
  const int tiles = (int)((ldy + 31) / 32);
  const int bi = blockIdx.x / tiles, bj = blockIdx.x % tiles;  // WT rows bi (ef), columns bj (bc)
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int bc = bj * 32 + r, ef = bi * 32 + tx;
    tile[r][tx] = (bc < n && ef < n) ? W[(int64_t)bc * n + ef] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t ef = bi * 32 + r, bc = bj * 32 + tx;
    if (ef < rows_all && bc < ldy) WT[ef * ldy + bc] = (T)tile[tx][r];
  }
}

// R3[t, abc] += Y_t[a, bc] - Y_t[b, ac] + Y_t[c, ab]; a thread per output,
// blocks over one triple's contiguous range of outputs (the triple's Y block
// is then read by neighbouring blocks of one XCD)
template <typename T>
__global__ void __launch_bounds__(256) r3_fold_kernel(IndexTables tb, int v, int nv3, int nblk, const T* __restrict__ Y,
                                                      int64_t ldy, double* __restrict__ R3) {
  int64_t L;
  {
    const int64_t n = gridDim.x, b = blockIdx.x, q = n / 8, r = n % 8, x = b % 8, k = b / 8;
    L = x * q + (x < r ? x : r) + k;
  }
  const int t = (int)(L / nblk);
  const int u = (int)(L % nblk) * 256 + threadIdx.x;
  if (u >= nv3) return;
  const int a = tb.dec[3][3 * u], b = tb.dec[3][3 * u + 1], c = tb.dec[3][3 * u + 2];
  const T* Yt = Y + (int64_t)t * v * ldy;
  const double z = (double)Yt[(int64_t)a * ldy + b + cb2(c)] - (double)Yt[(int64_t)b * ldy + a + cb2(c)] +
                   (double)Yt[(int64_t)c * ldy + a + cb2(b)];
  R3[(int64_t)t * nv3 + u] += z;
}

__global__ void __launch_bounds__(256) r3_ring_operand_kernel(const double* __restrict__ W, int o, int v, int ep,
                                                              double* __restrict__ A) {
  // A[x][a][m][e] = W[m][a][e][x] (e < v; zero for v <= e < ep): a block
  // per (x, a), a thread per (m, e)
  const int x = blockIdx.x / v, a = blockIdx.x % v;
  double* dst = A + ((int64_t)x * v + a) * o * ep;
  for (int q = threadIdx.x; q < o * ep; q += blockDim.x) {
    const int m = q / ep, e = q % ep;
    dst[q] = e < v ? W[(((int64_t)m * v + a) * v + e) * o + x] : 0.0;
  }
}

// Fvvp[a][e] = F3_vv[a][e] for a, e < v, zero elsewhere (kBM rows of ep)
__global__ void r3_fvv_pad_kernel(const double* __restrict__ F, int v, int ep, double* __restrict__ Fp) {
  const int a = blockIdx.x;
  for (int e = threadIdx.x; e < ep; e += blockDim.x) Fp[a * ep + e] = (a < v && e < v) ? F[a * v + e] : 0.0;
}

// C[t][t'] = sum_p (-1)^p [ W3_oooo[(t' \ x_p)][pair_p] s1 - F3_oo[t' \ pair_p][x_p] s2 ]
// where the first term needs x_p in t', the second pair_p inside t', and
// s1, s2 are the signs that sort (m, n, x_p) and (pair_p, m) into t'.
__global__ void __launch_bounds__(256) r3_occ_operator_kernel(IndexTables tb, int o, int nt, int no2,
                                                              const double* __restrict__ Woooo,
                                                              const double* __restrict__ Foo, double* __restrict__ C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nt * nt) return;
  const int t = (int)(i / nt), u = (int)(i % nt);
  const int tt[3] = {tb.dec[3][3 * t], tb.dec[3][3 * t + 1], tb.dec[3][3 * t + 2]};
  const int uu[3] = {tb.dec[3][3 * u], tb.dec[3][3 * u + 1], tb.dec[3][3 * u + 2]};
  double acc = 0;
  for (int p = 0; p < 3; ++p) {
    const int x = tt[p];
    const int q0 = tt[p == 0 ? 1 : 0], q1 = tt[p == 2 ? 1 : 2];
    const double sp = (p & 1) ? -1.0 : 1.0;
    // hh-ladder: t' = sorted(m, n, x) with m < n
    for (int w = 0; w < 3; ++w)
      if (uu[w] == x) {
        const int m = uu[w == 0 ? 1 : 0], n = uu[w == 2 ? 1 : 2];
        // (m, n, x) -> sorted: x moves past 2 - w letters
        const double s1 = ((2 - w) & 1) ? -1.0 : 1.0;
        acc += sp * s1 * Woooo[(int64_t)(m + cb2(n)) * no2 + q0 + cb2(q1)];
      }
    // F_oo: t' = sorted(q0, q1, m)
    int w = -1, hits = 0;
    for (int z = 0; z < 3; ++z) {
      if (uu[z] == q0 || uu[z] == q1)
        ++hits;
      else
        w = z;
    }
    if (hits == 2) {
      const int m = uu[w];
      const double s2 = ((2 - w) & 1) ? -1.0 : 1.0;
      acc -= sp * s2 * Foo[(int64_t)m * o + x];
    }
  }
  C[i] = acc;
}

int ceil_div(int a, int b) { return (a + b - 1) / b; }

Params make_params(const IndexTables& tb, const R3FusedArgs& a) {
  Params P{};
  P.a = a;
  P.tb = tb;
  const int o = a.o, v = a.v;
  P.nv2 = (int)binom_host(v, 2);
  P.nv3 = (int)binom_host(v, 3);
  P.no2 = (int)binom_host(o, 2);
  P.nt = (int)binom_host(o, 3);
  P.ntn = ceil_div(P.nv2, kBN);
  P.ep = (v + kBK - 1) / kBK * kBK;
  P.panel = std::min(P.nt, kPanel);
  const int ks[kSegs] = {P.nv2, v, (o - 2) * P.ep, (o - 2) * P.ep, (o - 2) * P.ep, v, v, v, o, o, o};
  int kt = 0;
  for (int s = 0; s < kSegs; ++s) {
    P.seg_k[s] = ks[s];
    P.kt_begin[s] = kt;
    kt += ceil_div(ks[s], kBK);
  }
  P.kt_begin[kSegs] = kt;
  return P;
}

}  // namespace

int64_t r3_fused_ldy(int v) {
  const int64_t nv2 = (int64_t)binom_host(v, 2);
  return (nv2 + kBK - 1) / kBK * kBK;
}

// the fused kernel reads past the last triple's rows (rows a or e up to 63)
// and past the last row's end (columns up to the last 128-column tile):
// whole padding rows after the data, all written (zeros) by the operand
// kernels in the compute type, so that they hold finite values whatever
// precision last used the buffer
static int64_t pad_rows(int v) { return kBM + (2 * kBN + r3_fused_ldy(v) - 1) / r3_fused_ldy(v); }

int64_t r3_fused_t3v_elems(int o, int v) { return r3_fused_y_elems(o, v) + pad_rows(v) * r3_fused_ldy(v); }

int64_t r3_fused_y_elems(int o, int v) { return (int64_t)binom_host(o, 3) * v * r3_fused_ldy(v); }

int64_t r3_fused_wt_elems(int v) { return (r3_fused_ldy(v) + pad_rows(v)) * r3_fused_ldy(v); }

int64_t r3_fvv_padded_elems(int v) { return (int64_t)kBM * ((v + kBK - 1) / kBK * kBK); }

double r3_fused_executed_flops(int o, int v) {
  IndexTables tb{};
  R3FusedArgs a;
  a.o = o;
  a.v = v;
  const Params P = make_params(tb, a);
  return 2.0 * kBM * kBN * kBK * (double)P.kt_begin[kSegs] * P.ntn * P.nt;
}

void launch_r3_fused(const IndexTables& tb, const R3FusedArgs& a, Prec prec, hipStream_t s) {
  FNO_REQUIRE(a.o >= 3 && a.v >= 3 && a.v <= kBM, kEINVAL, "fused triples residual needs 3 <= o, 3 <= v <= 64");
  FNO_REQUIRE(a.o <= tb.dec_max_n[3] && a.v <= tb.dec_max_n[3] && a.v <= tb.dec_max_n[2], kEINVAL,
              "index tables too small for the fused triples residual");
  FNO_REQUIRE(a.ldy == r3_fused_ldy(a.v), kEINVAL, "bad Y leading dimension");
  FNO_REQUIRE(a.T3v && a.WT && a.Y, kEINVAL, "fused triples residual: missing buffers");
  const Params P = make_params(tb, a);
  const int64_t tiles = (int64_t)P.nt * P.ntn;
  FNO_REQUIRE(tiles < (1ll << 31), kEINVAL, "too many tiles");
  if (prec == Prec::FP64)
    r3_fused_kernel<double><<<dim3((unsigned)tiles), kThreads, 0, s>>>(P);
  else if (prec == Prec::FP32)
    r3_fused_kernel<float><<<dim3((unsigned)tiles), kThreads, 0, s>>>(P);
  else
    r3_fused_kernel<float, true><<<dim3((unsigned)tiles), kThreads, 0, s>>>(P);
  FNO_HIP(hipGetLastError());
}

void launch_r3_fold(const IndexTables& tb, int o, int v, const void* Y, int64_t ldy, Prec prec, double* R3,
                    hipStream_t s) {
  const int nt = (int)binom_host(o, 3), nv3 = (int)binom_host(v, 3);
  const int nblk = ceil_div(nv3, 256);
  const int64_t blocks = (int64_t)nt * nblk;
  if (blocks == 0) return;
  if (prec == Prec::FP64)
    r3_fold_kernel<double><<<dim3((unsigned)blocks), 256, 0, s>>>(tb, v, nv3, nblk, (const double*)Y, ldy, R3);
  else
    r3_fold_kernel<float><<<dim3((unsigned)blocks), 256, 0, s>>>(tb, v, nv3, nblk, (const float*)Y, ldy, R3);
  FNO_HIP(hipGetLastError());
}

int64_t r3_ring_operand_elems(int o, int v) {
  const int64_t ep = (v + kBK - 1) / kBK * kBK;
  return ((int64_t)o * v + kBM) * o * ep;
}

void launch_r3_ring_operand(const double* Wovvo, const double* Fvv, int o, int v, double* Aring, double* Fvvp,
                            hipStream_t s) {
  const int ep = (v + kBK - 1) / kBK * kBK;
  r3_ring_operand_kernel<<<dim3((unsigned)(o * v)), 256, 0, s>>>(Wovvo, o, v, ep, Aring);
  r3_fvv_pad_kernel<<<dim3(kBM), 64, 0, s>>>(Fvv, v, ep, Fvvp);
  FNO_HIP(hipGetLastError());
}

void launch_r3_t3v(const IndexTables& tb, int o, int v, const double* T3, void* T3v, Prec prec, hipStream_t s) {
  const int nv2 = (int)binom_host(v, 2), nv3 = (int)binom_host(v, 3);
  const int64_t ldy = r3_fused_ldy(v), rows = (int64_t)binom_host(o, 3) * v;
  const int64_t rows_all = r3_fused_t3v_elems(o, v) / ldy;
  FNO_REQUIRE(v <= kT3vMaxV, kEINVAL, "T3v: more than 64 virtual orbitals");
  const int64_t blocks = rows_all;  // rows (t, c) first, then the padding rows
  if (prec == Prec::FP64)
    r3_t3v_kernel<double><<<dim3((unsigned)blocks), 256, 0, s>>>(v, nv2, nv3, ldy, rows, T3, (double*)T3v);
  else
    r3_t3v_kernel<float><<<dim3((unsigned)blocks), 256, 0, s>>>(v, nv2, nv3, ldy, rows, T3, (float*)T3v);
  FNO_HIP(hipGetLastError());
}

void launch_r3_wt(int v, const double* Wvvvv, void* WT, Prec prec, hipStream_t s) {
  const int nv2 = (int)binom_host(v, 2);
  const int64_t ldy = r3_fused_ldy(v), wrows_all = r3_fused_wt_elems(v) / ldy;
  const int64_t tiles = (ldy + 31) / 32, wblocks = ((wrows_all + 31) / 32) * tiles;
  if (prec == Prec::FP64)
    r3_wt_kernel<double><<<dim3((unsigned)wblocks), 256, 0, s>>>(nv2, ldy, wrows_all, Wvvvv, (double*)WT);
  else
    r3_wt_kernel<float><<<dim3((unsigned)wblocks), 256, 0, s>>>(nv2, ldy, wrows_all, Wvvvv, (float*)WT);
  FNO_HIP(hipGetLastError());
}

void launch_r3_operands(const IndexTables& tb, int o, int v, const double* T3, const double* Wvvvv, void* T3v,
                        void* WT, Prec prec, hipStream_t s) {
  launch_r3_t3v(tb, o, v, T3, T3v, prec, s);
  launch_r3_wt(v, Wvvvv, WT, prec, s);
}

void launch_r3_occ_operator(const IndexTables& tb, int o, const double* Woooo, const double* Foo, double* C,
                            hipStream_t s) {
  const int nt = (int)binom_host(o, 3), no2 = (int)binom_host(o, 2);
  const int64_t n = (int64_t)nt * nt;
  r3_occ_operator_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(tb, o, nt, no2, Woooo, Foo, C);
  FNO_HIP(hipGetLastError());
}

}  // namespace fno
