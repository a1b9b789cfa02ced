// T3 terms outside the triples residual from T3v (see triples_side.hpp).
//
// Kernels, in launch order:
//   side_slab_kernel      integral rows of the products, 16-byte aligned and
//   side_a2_kernel        zero padded (GoP, GvP, Gx; A2 below)
//   side_nt_kernel        S_t = A T3v[t]^T per triple: 64 x 64 tiles, both
//                         operands read along the pair index ef
//   side_nn_kernel<0>     W3_vvvo partial sums: per k, the pairs mn outside k
//                         in nsplit groups, A = <mn||fe> rows, B = T3v rows
//   side_nn_kernel<1>     per triple, A = <pair_p||j e> and F[t_p][e] rows
//   side_w3_kernel        W3_vvvo += the partial sums, W3_ovoo -= gathers of S
//   side_r12_kernel       R1 and R2 += gathers of S and of the NN products
#include "triples_side.hpp"

#include "kernels.hpp"
#include "triples.hpp"

namespace fno {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ d4_t mma(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int cb2(int n) { return n * (n - 1) / 2; }
__device__ __forceinline__ int cb3(int n) { return n * (n - 1) * (n - 2) / 6; }

// colex rank of the sorted triple {x, p, q} (p < q) and (-1)^(position of x
// in it), the sign of the permutation that sorts (x, p, q); 0 when x is p or q
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
__device__ __forceinline__ int position(int x, int p, int q) { return x < p ? 0 : (x < q ? 1 : 2); }

// blocks are handed to the 8 XCDs in turn; this gives each XCD a contiguous
// range of logical tiles, so the tiles that share operand rows share an L2
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t n) {
  const int64_t q = n / 8, r = n % 8, x = b % 8, k = b / 8;
  return x * q + (x < r ? x : r) + k;
}

struct OpArgs {
  IndexTables tb;
  const double* Gd;
  const double* Fd;
  double* buf;
  SideShape sh;
  int64_t n_goP, n_gvP, n_gx, n_a2;
};

// GoP[q][ef]     = <mn||ef>        q = (m < n) < C(o,2), rows up to nto*64
// GvP[m][b][ef]  = <bm||ef>        b < 64 rows per m
// Gx[q][e][f]    = <mn||fe>        e < 64, f < ep
// (ef a pair e < f, columns padded to ldy; every other element zero), one
// workgroup per row of GoP (with the Gx block of the same q) or of GvP.  The
// two fixed indices select the v x v slab Gd[p][q][o + r][o + s], which is
// read along s (contiguous in Gd), staged in LDS and written out in pair
// order and, for Gx, transposed.
__global__ void __launch_bounds__(256) side_slab_kernel(OpArgs P) {
  __shared__ double sl[64][65];
  const SideShape& sh = P.sh;
  const int o = sh.o, v = sh.v, n = sh.n;
  const uint8_t* d2 = P.tb.dec[2];
  const int tid = threadIdx.x;
  const int64_t ngo = (int64_t)sh.nto * 64, row = blockIdx.x;
  int p = 0, q = 0;
  bool live;
  double* dst;
  if (row < ngo) {
    live = row < sh.no2;
    if (live) {
      p = d2[2 * row];
      q = d2[2 * row + 1];
    }
    dst = P.buf + sh.goP + row * sh.ldy;
  } else {
    const int64_t r2 = row - ngo;
    const int m = (int)(r2 / 64), b = (int)(r2 % 64);
    live = b < v;
    p = o + b;
    q = m;
    dst = P.buf + sh.gvP + r2 * sh.ldy;
  }
  if (live) {  // uniform per workgroup
    const double* g = P.Gd + (((int64_t)p * n + q) * n + o) * n + o;
    for (int e = tid; e < v * v; e += 256) {
      const int r = e / v, c = e - r * v;
      sl[r][c] = g[(int64_t)r * n + c];
    }
  }
  __syncthreads();
  for (int64_t c = tid; c < sh.ldy; c += 256) dst[c] = (live && c < sh.nv2) ? sl[d2[2 * c]][d2[2 * c + 1]] : 0.0;
  if (row < sh.no2) {
    double* gx = P.buf + sh.gx + row * 64 * sh.ep;
    for (int e = tid; e < 64 * sh.ep; e += 256) {
      const int r = e / sh.ep, f = e - r * sh.ep;
      gx[e] = (r < v && f < v) ? sl[f][r] : 0.0;
    }
  }
}

// A2[t][r][e]    = <pair_p||j e>   r = p (o + 1) + j, j < o
//                = F[t_p][e]       r = p (o + 1) + o
// (e < ep; every other element zero), a thread per element (rows of Gd and
// Fd read along e)
__global__ void __launch_bounds__(256) side_a2_kernel(OpArgs P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n_a2) return;
  const SideShape& sh = P.sh;
  const int o = sh.o, v = sh.v, n = sh.n;
  const int64_t per = (int64_t)sh.mt2 * 64 * sh.ep;
  const int t = (int)(i / per);
  const int rem = (int)(i % per), r = rem / sh.ep, e = rem % sh.ep;
  const int p = r / (o + 1), j = r % (o + 1);
  double val = 0;
  if (p < 3 && e < v) {
    const uint8_t* d3 = P.tb.dec[3] + 3 * t;
    const int x = d3[p], q0 = d3[p == 0 ? 1 : 0], q1 = d3[p == 2 ? 1 : 2];
    val = j < o ? P.Gd[(((int64_t)q0 * n + q1) * n + j) * n + o + e] : P.Fd[(int64_t)x * n + o + e];
  }
  P.buf[sh.a2 + i] = val;
}

struct NTArgs {
  IndexTables tb;
  const double* T3v;
  const double* GoP;
  const double* GvP;
  double* S;
  int v, nto, mts;
  int64_t ldy;
};

// S[t][mt*64 + r][c] = sum_{k < ldy} A[r][k] T3v[t][c][k]: A = GoP rows
// (mt < nto) or GvP rows of m = t_p (mt = nto + p).  64 x 64 tile, 4
// wavefronts of 32 x 32, k tiles of 16 through two LDS stages.  Rows c >= v
// of T3v[t] belong to the next triple or to the buffer's padding; their
// columns of S are never read.
__global__ void __launch_bounds__(256, 2) side_nt_kernel(NTArgs P) {
  __shared__ double As[2][16][65];
  __shared__ double Bs[2][16][65];
  const int64_t L = xcd_order(blockIdx.x, gridDim.x);
  const int t = (int)(L / P.mts), mt = (int)(L % P.mts);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  const int64_t ldy = P.ldy;
  const double* A = mt < P.nto ? P.GoP + (int64_t)mt * 64 * ldy
                               : P.GvP + (int64_t)P.tb.dec[3][3 * t + (mt - P.nto)] * 64 * ldy;
  const double* B = P.T3v + (int64_t)t * P.v * ldy;
  d4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (d4_t){0, 0, 0, 0};
  d2_t ra[2], rb[2];
  auto load = [&](int kt) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int q = tid + 256 * i, row = q >> 3, kv = (q & 7) * 2;
      ra[i] = *(const d2_t*)(A + row * ldy + kt * 16 + kv);
      rb[i] = *(const d2_t*)(B + row * ldy + kt * 16 + kv);
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int q = tid + 256 * i, row = q >> 3, kv = (q & 7) * 2;
      As[st][kv][row] = ra[i][0];
      As[st][kv + 1][row] = ra[i][1];
      Bs[st][kv][row] = rb[i][0];
      Bs[st][kv + 1][row] = rb[i][1];
    }
  };
  const int nk = (int)(ldy / 16);
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) load(kt + 1);
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[cur][kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = Bs[cur][kr][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mma(af[i], bf[j], acc[i][j]);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
  }
  // C/D layout of the FP64 16x16 block: lane l holds column l % 16, rows
  // l / 16 + 4 r
  double* S = P.S + ((int64_t)t * P.mts + mt) * 64 * 64;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm * 32 + i * 16 + (lane >> 4) + 4 * r, col = wn * 32 + j * 16 + (lane & 15);
        S[row * 64 + col] = acc[i][j][r];
      }
}

struct NNArgs {
  IndexTables tb;
  const double* A;  // Gx (mode 0) or A2 (mode 1)
  const double* T3v;
  double* out;      // W3_vvvo partial sums (mode 0) or per-triple products (mode 1)
  SideShape sh;
};

// Mode 0: out[s][k][e][bc] = -sum_{pairs mn of group s, k outside mn}
//   (-1)^p(k) sum_f Gx[mn][e][f] T3v[t(k m n)][f][bc]
// Mode 1: out[t][r][bc] = sum_e A2[t][r][e] T3v[t][e][bc], r < 3 (o + 1)
// 64 x 128 tiles (rows e or r, columns bc), k tiles of 16 over f or e (the
// padded range ep; A is zero beyond v, so the T3v rows of the next triple or
// of the padding that those k meet add nothing).
template <int MODE>
__global__ void __launch_bounds__(256, 2) side_nn_kernel(NNArgs P) {
  __shared__ double As[2][16][65];
  __shared__ __attribute__((aligned(16))) double Bs[2][16][130];
  const SideShape& sh = P.sh;
  const int64_t L = xcd_order(blockIdx.x, gridDim.x);
  const int n0 = (int)(L % sh.ntn) * 128;
  const int job = (int)(L / sh.ntn);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  const int64_t ldy = sh.ldy;
  const int per = sh.ep / 16, v = sh.v;
  int k = 0, grp = 0, c0 = 0, t = 0, mtile = 0, nk;
  if (MODE == 0) {
    k = job / sh.nsplit;
    grp = job % sh.nsplit;
    c0 = (int)((int64_t)grp * sh.nchunk / sh.nsplit);
    const int c1 = (int)((int64_t)(grp + 1) * sh.nchunk / sh.nsplit);
    nk = (c1 - c0) * per;
  } else {
    t = job / sh.mt2;
    mtile = job % sh.mt2;
    nk = per;
  }
  d4_t acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (d4_t){0, 0, 0, 0};
  d2_t ra[2], rb[4];
  auto load = [&](int kt) {
    const double* abase;
    const double* bbase;
    double scale = 1.0;
    const int e0 = (kt % per) * 16;
    if (MODE == 0) {
      // the (kt / per)-th pair (m' < n') of the o - 1 letters other than k
      const int c = c0 + kt / per;
      int m = P.tb.dec[2][2 * c], n = P.tb.dec[2][2 * c + 1];
      m += (m >= k) ? 1 : 0;
      n += (n >= k) ? 1 : 0;
      int s;
      const int rank = tri_rank(k, m, n, s);
      scale = -(double)s;
      abase = P.A + (int64_t)(m + cb2(n)) * 64 * sh.ep + e0;
      bbase = P.T3v + ((int64_t)rank * v + e0) * ldy + n0;
    } else {
      abase = P.A + (int64_t)(t * sh.mt2 + mtile) * 64 * sh.ep + e0;
      bbase = P.T3v + ((int64_t)t * v + e0) * ldy + n0;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int q = tid + 256 * i, row = q >> 3, kv = (q & 7) * 2;
      ra[i] = scale * *(const d2_t*)(abase + row * sh.ep + kv);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = tid + 256 * i, kk = q >> 6, nv = (q & 63) * 2;
      rb[i] = *(const d2_t*)(bbase + kk * ldy + nv);
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int q = tid + 256 * i, row = q >> 3, kv = (q & 7) * 2;
      As[st][kv][row] = ra[i][0];
      As[st][kv + 1][row] = ra[i][1];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = tid + 256 * i, kk = q >> 6, nv = (q & 63) * 2;
      *(d2_t*)&Bs[st][kk][nv] = rb[i];
    }
  };
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) load(kt + 1);
#pragma unroll
    for (int ks = 0; ks < 16; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[2], bf[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[cur][kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[cur][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mma(af[i], bf[j], acc[i][j]);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = n0 + wn * 64 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm * 32 + i * 16 + (lane >> 4) + 4 * r;
        if (c >= sh.nv2) continue;
        if (MODE == 0) {
          if (row < v) P.out[((int64_t)(grp * sh.o + k) * v + row) * ldy + c] = acc[i][j][r];
        } else {
          const int rr = mtile * 64 + row;
          if (rr < sh.rows2) P.out[((int64_t)t * sh.rows2 + rr) * ldy + c] = acc[i][j][r];
        }
      }
    }
}

// W3_vvvo[k][e][bc] += sum_s Wp[s][k][e][bc]
// W3_ovoo[m][c][jk] -= sum_{n outside jk, n != m} (-1)^p(n) sgn(m, n) S[t(jkn)][{m,n}][c]
__global__ void __launch_bounds__(256) side_w3_kernel(IndexTables tb, SideShape sh, const double* __restrict__ buf,
                                                      double* __restrict__ W3vvvo, double* __restrict__ W3ovoo) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int o = sh.o, v = sh.v;
  const int64_t n1 = (int64_t)o * v * sh.nv2;
  if (i < n1) {
    const int64_t ke = i / sh.nv2, bc = i % sh.nv2;
    double acc = 0;
    for (int s = 0; s < sh.nsplit; ++s) acc += buf[sh.wp + ((int64_t)s * o * v + ke) * sh.ldy + bc];
    W3vvvo[i] += acc;
    return;
  }
  i -= n1;
  if (i >= (int64_t)o * v * sh.no2) return;
  const int jk = (int)(i % sh.no2);
  const int mc = (int)(i / sh.no2), m = mc / v, c = mc % v;
  const int j = tb.dec[2][2 * jk], k = tb.dec[2][2 * jk + 1];
  const double* S = buf + sh.s;
  double acc = 0;
  for (int n = 0; n < o; ++n) {
    if (n == j || n == k || n == m) continue;
    int s;
    const int rank = tri_rank(n, j, k, s);
    const int lo = m < n ? m : n, hi = m < n ? n : m;
    const double sg = (m < n) ? (double)s : -(double)s;
    acc += sg * S[((int64_t)rank * sh.mts * 64 + lo + cb2(hi)) * 64 + c];
  }
  W3ovoo[i] -= acc;
}

// R1[i][a] += sum_{m<n outside i} (-1)^p(i) S[t(imn)][mn][a]
// R2[ij][ab] += sum_{m outside ij} (-1)^p(m) ( O2[t][p(m)(o+1) + o][ab]
//                 + S[t][nto*64 + 64 p(m) + b][a] - S[t][nto*64 + 64 p(m) + a][b] )
//             - sum_{m<n outside i} (-1)^p(i) O2[t(imn)][p(i)(o+1) + j][ab]
//             + sum_{m<n outside j} (-1)^p(j) O2[t(jmn)][p(j)(o+1) + i][ab]
// A block owns 64 consecutive outputs (R1 first, then R2); its four
// wavefronts take every fourth m and every fourth pair mn, and the four
// partial sums are added in a fixed order.
__global__ void __launch_bounds__(256) side_r12_kernel(IndexTables tb, SideShape sh, const double* __restrict__ buf,
                                                       double* __restrict__ R1, double* __restrict__ R2) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
  const int o = sh.o, v = sh.v;
  const double* S = buf + sh.s;
  const double* O2 = buf + sh.o2;
  const uint8_t* d2 = tb.dec[2];
  const int64_t n1 = (int64_t)o * v, n2 = (int64_t)sh.no2 * sh.nv2;
  double acc = 0;
  if (idx < n1) {
    const int i = (int)(idx / v), a = (int)(idx % v);
    for (int q = w; q < sh.no2; q += 4) {
      const int m = d2[2 * q], n = d2[2 * q + 1];
      if (m == i || n == i) continue;
      int s;
      const int rank = tri_rank(i, m, n, s);
      acc += s * S[((int64_t)rank * sh.mts * 64 + q) * 64 + a];
    }
  } else if (idx < n1 + n2) {
    const int64_t r2 = idx - n1;
    const int ij = (int)(r2 / sh.nv2), ab = (int)(r2 % sh.nv2);
    const int i = d2[2 * ij], j = d2[2 * ij + 1], a = d2[2 * ab], b = d2[2 * ab + 1];
    const int64_t ldy = sh.ldy;
    for (int m = w; m < o; m += 4) {
      if (m == i || m == j) continue;
      int s;
      const int rank = tri_rank(m, i, j, s);
      const int p = position(m, i, j);
      const double* St = S + ((int64_t)rank * sh.mts * 64 + sh.nto * 64 + 64 * p) * 64;
      acc += s * (O2[((int64_t)rank * sh.rows2 + p * (o + 1) + o) * ldy + ab] + St[b * 64 + a] - St[a * 64 + b]);
    }
    for (int q = w; q < sh.no2; q += 4) {
      const int m = d2[2 * q], n = d2[2 * q + 1];
      if (m != i && n != i) {
        int s;
        const int rank = tri_rank(i, m, n, s);
        acc -= s * O2[((int64_t)rank * sh.rows2 + position(i, m, n) * (o + 1) + j) * ldy + ab];
      }
      if (m != j && n != j) {
        int s;
        const int rank = tri_rank(j, m, n, s);
        acc += s * O2[((int64_t)rank * sh.rows2 + position(j, m, n) * (o + 1) + i) * ldy + ab];
      }
    }
  }
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && idx < n1 + n2) {
    const double sum = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    if (idx < n1)
      R1[idx] += sum;
    else
      R2[idx - n1] += sum;
  }
}

int64_t up32(int64_t x) { return (x + 31) / 32 * 32; }
unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

SideShape side_shape(int o, int v) {
  SideShape sh;
  sh.o = o;
  sh.v = v;
  sh.n = o + v;
  sh.no2 = (int)binom_host(o, 2);
  sh.nt = (int)binom_host(o, 3);
  sh.nv2 = (int)binom_host(v, 2);
  sh.ldy = r3_fused_ldy(v);
  sh.ep = (v + 15) / 16 * 16;
  sh.nto = (sh.no2 + 63) / 64;
  sh.mts = sh.nto + 3;
  sh.rows2 = 3 * (o + 1);
  sh.mt2 = (sh.rows2 + 63) / 64;
  sh.nchunk = (int)binom_host(o - 1, 2);
  sh.ntn = (sh.nv2 + 127) / 128;
  sh.nsplit = std::max(1, std::min(sh.nchunk, (512 + o * sh.ntn - 1) / (o * sh.ntn)));
  int64_t off = 0;
  sh.goP = off;
  off += up32((int64_t)sh.nto * 64 * sh.ldy);
  sh.gvP = off;
  off += up32((int64_t)o * 64 * sh.ldy);
  sh.gx = off;
  off += up32((int64_t)sh.no2 * 64 * sh.ep);
  sh.a2 = off;
  off += up32((int64_t)sh.nt * sh.mt2 * 64 * sh.ep);
  sh.s = off;
  off += up32((int64_t)sh.nt * sh.mts * 64 * 64);
  sh.o2 = off;
  off += up32((int64_t)sh.nt * sh.rows2 * sh.ldy);
  sh.wp = off;
  off += up32((int64_t)sh.nsplit * o * v * sh.ldy);
  sh.total = off;
  return sh;
}

double side_executed_flops(const SideShape& sh) {
  const double nt_fl = 2.0 * sh.nt * sh.mts * 64.0 * 64.0 * sh.ldy;
  const double w3_fl = 2.0 * sh.o * sh.ntn * 64.0 * 128.0 * sh.nchunk * sh.ep;
  const double r2_fl = 2.0 * sh.nt * sh.mt2 * sh.ntn * 64.0 * 128.0 * sh.ep;
  return nt_fl + w3_fl + r2_fl;
}

void launch_side_operands(const IndexTables& tb, const SideShape& sh, const double* Gd, const double* Fd,
                          double* buf, hipStream_t s) {
  FNO_REQUIRE(sh.o >= 3 && sh.v >= 3 && sh.v <= 64, kEINVAL, "side T3 terms need 3 <= o, 3 <= v <= 64");
  FNO_REQUIRE(sh.o <= tb.dec_max_n[3] && sh.o <= tb.dec_max_n[2] && sh.v <= tb.dec_max_n[2], kEINVAL,
              "index tables too small for the side T3 terms");
  OpArgs P{};
  P.tb = tb;
  P.Gd = Gd;
  P.Fd = Fd;
  P.buf = buf;
  P.sh = sh;
  P.n_goP = (int64_t)sh.nto * 64 * sh.ldy;
  P.n_gvP = (int64_t)sh.o * 64 * sh.ldy;
  P.n_gx = (int64_t)sh.no2 * 64 * sh.ep;
  P.n_a2 = (int64_t)sh.nt * sh.mt2 * 64 * sh.ep;
  side_slab_kernel<<<dim3((unsigned)((int64_t)(sh.nto + sh.o) * 64)), 256, 0, s>>>(P);
  side_a2_kernel<<<blocks_for(P.n_a2), 256, 0, s>>>(P);
  FNO_HIP(hipGetLastError());
}

void launch_side_products(const IndexTables& tb, const SideShape& sh, const double* T3v, double* buf,
                          hipStream_t s) {
  NTArgs a{};
  a.tb = tb;
  a.T3v = T3v;
  a.GoP = buf + sh.goP;
  a.GvP = buf + sh.gvP;
  a.S = buf + sh.s;
  a.v = sh.v;
  a.nto = sh.nto;
  a.mts = sh.mts;
  a.ldy = sh.ldy;
  side_nt_kernel<<<dim3((unsigned)(sh.nt * sh.mts)), 256, 0, s>>>(a);
  NNArgs b{};
  b.tb = tb;
  b.T3v = T3v;
  b.sh = sh;
  b.A = buf + sh.gx;
  b.out = buf + sh.wp;
  side_nn_kernel<0><<<dim3((unsigned)(sh.o * sh.nsplit * sh.ntn)), 256, 0, s>>>(b);
  b.A = buf + sh.a2;
  b.out = buf + sh.o2;
  side_nn_kernel<1><<<dim3((unsigned)(sh.nt * sh.mt2 * sh.ntn)), 256, 0, s>>>(b);
  FNO_HIP(hipGetLastError());
}

void launch_side_w3(const IndexTables& tb, const SideShape& sh, const double* buf, double* W3vvvo, double* W3ovoo,
                    hipStream_t s) {
  const int64_t n = (int64_t)sh.o * sh.v * (sh.nv2 + sh.no2);
  side_w3_kernel<<<blocks_for(n), 256, 0, s>>>(tb, sh, buf, W3vvvo, W3ovoo);
  FNO_HIP(hipGetLastError());
}

void launch_side_r12(const IndexTables& tb, const SideShape& sh, const double* buf, double* R1, double* R2,
                     hipStream_t s) {
  const int64_t n = (int64_t)sh.o * sh.v + (int64_t)sh.no2 * sh.nv2;
  side_r12_kernel<<<dim3((unsigned)((n + 63) / 64)), 256, 0, s>>>(tb, sh, buf, R1, R2);
  FNO_HIP(hipGetLastError());
}

}  // namespace fno
