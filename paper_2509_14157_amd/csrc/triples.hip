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

struct Params {
  R3FusedArgs a;
  IndexTables tb;
  int nv2, nv3, no2, nt, ntn;  // C(v,2), C(v,3), C(o,2), C(o,3), N tiles per triple
  int kt_begin[kSegs + 1];     // first k tile of each segment
  int seg_k[kSegs];            // K of each segment
};

template <typename T>
__global__ void __launch_bounds__(kThreads, 2) r3_fused_kernel(Params P) {
  constexpr int PAD = (sizeof(T) == 8) ? 1 : 2;
  __shared__ T As[2][kBK][kBM + PAD];
  __shared__ T Bs[2][kBK][kBN + PAD];
  const R3FusedArgs& g = P.a;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // tiles: triple fast within an XCD's contiguous range, so consecutive
  // tiles of one XCD share the column strip of W3_vvvv in its L2
  int64_t L;
  {
    const int64_t n = gridDim.x, b = blockIdx.x, q = n / 8, r = n % 8, x = b % 8, k = b / 8;
    L = x * q + (x < r ? x : r) + k;
  }
  const int t = (int)(L % P.nt);
  const int n0 = (int)(L / P.nt) * kBN;
  const int v = g.v, o = g.o, nv2 = P.nv2, nv3 = P.nv3;
  const uint8_t* d3 = P.tb.dec[3] + 3 * t;
  const int tt[3] = {d3[0], d3[1], d3[2]};
  const double* T3t = g.T3 + (int64_t)t * nv3;

  // this thread's column for the column-fast B tiles: its (b, c) stay in registers
  const int ncol = tid & (kBN - 1);
  const int col = n0 + ncol;
  const bool col_ok = col < nv2;
  int cb = 0, cc = 1;
  if (col_ok) {
    cb = P.tb.dec[2][2 * col];
    cc = P.tb.dec[2][2 * col + 1];
  }

  typename AccT<T>::type acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (typename AccT<T>::type){0, 0, 0, 0};

  T ra[4], rb[8];
  bool a_kfast = false, b_kfast = false;  // element mapping of the tile in registers

  // placement p of the triple: x = t_p, pair (q0 < q1) = the other two
  auto placement = [&](int p, int& x, int& q0, int& q1) {
    x = tt[p];
    q0 = tt[p == 0 ? 1 : 0];
    q1 = tt[p == 2 ? 1 : 2];
  };

  auto load_tile = [&](int kt) {
    int s = 0;
#pragma unroll
    for (int q = 1; q < kSegs; ++q) s += (kt >= P.kt_begin[q]) ? 1 : 0;
    const int k0 = (kt - P.kt_begin[s]) * kBK;
    const int K = P.seg_k[s];
    if (s == 0) {
      // pp-ladder: A[a, ef] = T3[t, a e f], lanes over a, k uniform per wave
      a_kfast = false;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kk = wave + 4 * i, a = lane, k = k0 + kk;
        double val = 0;
        if (k < K && a < v) {
          const int e = P.tb.dec[2][2 * k], f = P.tb.dec[2][2 * k + 1];
          int sg;
          const int r = tri_rank(a, e, f, sg);
          if (sg) val = sg * T3t[r];
        }
        ra[i] = (T)val;
      }
      // B[ef, bc] = W3_vvvv[bc][ef]: k fastest in memory, 16-element runs
      b_kfast = true;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int kk = tid & 15, nn = (tid >> 4) + 16 * i, k = k0 + kk, c = n0 + nn;
        rb[i] = (T)((k < K && c < nv2) ? g.Wvvvv[(int64_t)c * nv2 + k] : 0.0);
      }
    } else if (s == 1) {
      // one-body: A[a, e] = F3_vv[a][e], B[e, bc] = T3[t, e b c]
      a_kfast = true;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kk = tid & 15, a = (tid >> 4) + 16 * i, k = k0 + kk;
        ra[i] = (T)((k < K && a < v) ? g.Fvv[a * v + k] : 0.0);
      }
      b_kfast = false;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + (tid >> 7) + 2 * i;
        double val = 0;
        if (k < K && col_ok) {
          int sg;
          const int r = tri_rank(k, cb, cc, sg);
          if (sg) val = sg * T3t[r];
        }
        rb[i] = (T)val;
      }
    } else if (s <= 4) {
      // ring, placement p: k = m' v + e over the o - 2 occupied m outside the pair
      const int p = s - 2;
      int x, q0, q1;
      placement(p, x, q0, q1);
      const double sp = (p & 1) ? -1.0 : 1.0;
      a_kfast = true;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kk = tid & 15, a = (tid >> 4) + 16 * i, k = k0 + kk;
        double val = 0;
        if (k < K && a < v) {
          int m = k / v;
          const int e = k - m * v;
          m += (m >= q0) ? 1 : 0;
          m += (m >= q1) ? 1 : 0;
          val = sp * g.Aring[(((int64_t)x * v + a) * o + m) * v + e];
        }
        ra[i] = (T)val;
      }
      b_kfast = false;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + (tid >> 7) + 2 * i;  // uniform per wavefront
        double val = 0;
        if (k < K && col_ok) {
          int m = k / v;
          const int e = k - m * v;
          m += (m >= q0) ? 1 : 0;
          m += (m >= q1) ? 1 : 0;
          int so, sv;
          const int ro = tri_rank(m, q0, q1, so);
          const int rv = tri_rank(e, cb, cc, sv);
          if (sv) val = (so * sv) * g.T3[(int64_t)ro * nv3 + rv];
        }
        rb[i] = (T)val;
      }
    } else if (s <= 7) {
      // driver: A[a, e] = (-1)^p T2[pair, a e], B[e, bc] = W3_vvvo[x][e][bc]
      const int p = s - 5;
      int x, q0, q1;
      placement(p, x, q0, q1);
      const double sp = (p & 1) ? -1.0 : 1.0;
      const double* t2row = g.T2 + (int64_t)(q0 + cb2(q1)) * nv2;
      a_kfast = false;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kk = wave + 4 * i, a = lane, k = k0 + kk;
        double val = 0;
        if (k < K && a < v && a != k) {
          val = a < k ? sp * t2row[a + cb2(k)] : -sp * t2row[k + cb2(a)];
        }
        ra[i] = (T)val;
      }
      b_kfast = false;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + (tid >> 7) + 2 * i;
        rb[i] = (T)((k < K && col_ok) ? g.Wvvvo[((int64_t)x * v + k) * nv2 + col] : 0.0);
      }
    } else {
      // driver: A[a, m] = -(-1)^p W3_ovoo[m][a][pair], B[m, bc] = T2[x m, bc]
      const int p = s - 8;
      int x, q0, q1;
      placement(p, x, q0, q1);
      const double sp = (p & 1) ? 1.0 : -1.0;
      const int pr = q0 + cb2(q1);
      a_kfast = false;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kk = wave + 4 * i, a = lane, k = k0 + kk;
        ra[i] = (T)((k < K && a < v) ? sp * g.Wovoo[((int64_t)k * v + a) * P.no2 + pr] : 0.0);
      }
      b_kfast = false;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + (tid >> 7) + 2 * i;
        double val = 0;
        if (k < K && col_ok && k != x) {
          const int lo = k < x ? k : x, hi = k < x ? x : k;
          const double sg = k < x ? -1.0 : 1.0;  // (x, m) sorted
          val = sg * g.T2[(int64_t)(lo + cb2(hi)) * nv2 + col];
        }
        rb[i] = (T)val;
      }
    }
  };

  auto store_tile = [&](int st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (a_kfast)
        As[st][tid & 15][(tid >> 4) + 16 * i] = ra[i];
      else
        As[st][wave + 4 * i][lane] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (b_kfast)
        Bs[st][tid & 15][(tid >> 4) + 16 * i] = rb[i];
      else
        Bs[st][(tid >> 7) + 2 * i][tid & (kBN - 1)] = rb[i];
    }
  };

  const int nk = P.kt_begin[kSegs];
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) load_tile(kt + 1);
#pragma unroll
    for (int ks = 0; ks < kBK; ks += 4) {
      const int kr = ks + (lane >> 4);
      T af[2], bf[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[cur][kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[cur][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mma(af[i], bf[j], acc[i][j]);
    }
    if (more) store_tile(cur ^ 1);
    __syncthreads();
  }

  // C/D layout of the 16x16 block: lane l holds column l % 16; FP64 rows
  // l / 16 + 4 r, FP32 rows 4 (l / 16) + r
  T* Y = (T*)g.Y + (int64_t)t * v * g.ldy;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (sizeof(T) == 8) ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int a = wm * 32 + i * 16 + rr;
        if (a < v && c < nv2) Y[(int64_t)a * g.ldy + c] = acc[i][j][r];
      }
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

__global__ void __launch_bounds__(256) r3_ring_operand_kernel(const double* __restrict__ W, int o, int v,
                                                              double* __restrict__ A) {
  // A[x][a][m][e] = W[m][a][e][x]; a thread per element of A
  const int64_t n = (int64_t)o * v * o * v;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(i % v);
    int64_t r = i / v;
    const int m = (int)(r % o);
    r /= o;
    const int a = (int)(r % v);
    const int x = (int)(r / v);
    A[i] = W[(((int64_t)m * v + a) * v + e) * o + x];
  }
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
  const int ks[kSegs] = {P.nv2, v, (o - 2) * v, (o - 2) * v, (o - 2) * v, v, v, v, o, o, o};
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
  return (nv2 + 3) / 4 * 4;
}

int64_t r3_fused_y_elems(int o, int v) { return (int64_t)binom_host(o, 3) * v * r3_fused_ldy(v); }

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
  FNO_REQUIRE(a.ldy >= (int64_t)binom_host(a.v, 2), kEINVAL, "bad Y leading dimension");
  const Params P = make_params(tb, a);
  const int64_t tiles = (int64_t)P.nt * P.ntn;
  FNO_REQUIRE(tiles < (1ll << 31), kEINVAL, "too many tiles");
  if (prec == Prec::FP64)
    r3_fused_kernel<double><<<dim3((unsigned)tiles), kThreads, 0, s>>>(P);
  else
    r3_fused_kernel<float><<<dim3((unsigned)tiles), kThreads, 0, s>>>(P);
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

void launch_r3_ring_operand(const double* Wovvo, int o, int v, double* Aring, hipStream_t s) {
  const int64_t n = (int64_t)o * v * o * v;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  r3_ring_operand_kernel<<<dim3((unsigned)blocks), 256, 0, s>>>(Wovvo, o, v, Aring);
  FNO_HIP(hipGetLastError());
}

void launch_r3_occ_operator(const IndexTables& tb, int o, const double* Woooo, const double* Foo, double* C,
                            hipStream_t s) {
  const int nt = (int)binom_host(o, 3), no2 = (int)binom_host(o, 2);
  const int64_t n = (int64_t)nt * nt;
  r3_occ_operator_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(tb, o, nt, no2, Woooo, Foo, C);
  FNO_HIP(hipGetLastError());
}

}  // namespace fno
