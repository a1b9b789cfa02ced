// Streaming kernels: operand expansion, antisymmetrizing fold, Jacobi update,
// reductions.  All of them are HBM bound; threads walk the output linearly so
// stores coalesce, and the packed sources they gather from are small enough
// to stay in L2 / the MALL.
#include <hip/hip_bf16.h>
#include <cstdio>
#include <cstdlib>

#include "kernels.hpp"

namespace fno {

// Workgroup b of a launch runs on XCD b % 8.  xcd_chunk maps b to a logical
// block so that each XCD walks one contiguous range of the n blocks:
// neighbouring blocks, which share source rows and cache lines, then meet in
// the same L2.  A bijection on [0, n).
__device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t n) {
  const int64_t q = n / 8, r = n % 8, x = b % 8, k = b / 8;
  return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------- expand
// dst[r, c] (rows x cols, row-major when col_fast, else column-major) =
//   sign * src[operand(r, c)], converted to the GEMM operand precision.
template <typename Out>
__device__ __forceinline__ void store_val(Out* dst, int64_t i, double v) {
  dst[i] = (Out)v;
}

template <typename Out>
__global__ void __launch_bounds__(256) expand_kernel(IndexTables tb, OperandDesc op, MatDim rows, MatDim cols,
                                                     const double* __restrict__ src, Out* __restrict__ dst,
                                                     int col_fast, int64_t total) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < total; i += stride) {
    int64_t r, c;
    if (col_fast) {
      r = i / cols.size;
      c = i - r * cols.size;
    } else {
      c = i / rows.size;
      r = i - c * rows.size;
    }
    int val[kMaxLetters];
    decode_dim(tb, rows, r, val);
    decode_dim(tb, cols, c, val);
    int sign;
    int64_t off = operand_offset(tb, op, val, &sign);
    double v = sign ? sign * src[off] : 0.0;
    store_val<Out>(dst, i, v);
  }
}

// Split-BF16: hi = RNE_bf16(x), lo = RNE_bf16(x - hi), interleaved per element.
__global__ void __launch_bounds__(256) expand_bf16x2_kernel(IndexTables tb, OperandDesc op, MatDim rows,
                                                            MatDim cols, const double* __restrict__ src,
                                                            __hip_bfloat16* __restrict__ hi,
                                                            __hip_bfloat16* __restrict__ lo, int col_fast,
                                                            int64_t total) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < total; i += stride) {
    int64_t r, c;
    if (col_fast) {
      r = i / cols.size;
      c = i - r * cols.size;
    } else {
      c = i / rows.size;
      r = i - c * rows.size;
    }
    int val[kMaxLetters];
    decode_dim(tb, rows, r, val);
    decode_dim(tb, cols, c, val);
    int sign;
    int64_t off = operand_offset(tb, op, val, &sign);
    float x = sign ? (float)(sign * src[off]) : 0.0f;
    __hip_bfloat16 h = __float2bfloat16(x);
    float rem = x - __bfloat162float(h);
    hi[i] = h;
    lo[i] = __float2bfloat16(rem);
  }
}

void launch_expand(const IndexTables& tb, const OperandDesc& op, const MatDim& rows, const MatDim& cols,
                   const double* src, void* dst, void* dst_lo, Prec prec, bool col_fast, hipStream_t s) {
  int64_t total = rows.size * cols.size;
  if (total == 0) return;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (prec == Prec::FP64)
    expand_kernel<double><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(tb, op, rows, cols, src, (double*)dst,
                                                                       col_fast ? 1 : 0, total);
  else if (prec == Prec::FP32)
    expand_kernel<float><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(tb, op, rows, cols, src, (float*)dst,
                                                                      col_fast ? 1 : 0, total);
  else
    expand_bf16x2_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(
        tb, op, rows, cols, src, (__hip_bfloat16*)dst, (__hip_bfloat16*)dst_lo, col_fast ? 1 : 0, total);
  FNO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- fold
// out[e] += alpha * sum_c sign_c * X[row(c), col(c)] for every packed output
// element e; the coset representatives c come from the host planner.
template <typename XT>
__global__ void __launch_bounds__(256) fold_kernel(IndexTables tb, OperandDesc outd, MatDim outdims,
                                                   MatDim xrows, MatDim xcols, FoldCombos fc,
                                                   const XT* __restrict__ X, double* __restrict__ out,
                                                   double alpha, int64_t total) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < total; i += stride) {
    int val[kMaxLetters];
    decode_dim(tb, outdims, i, val);
    double acc = 0.0;
    for (int c = 0; c < fc.ncombo; ++c) {
      int pv[kMaxLetters];
      for (int l = 0; l < fc.nletters; ++l) pv[l] = val[fc.src[c][l]];
      int64_t r = 0;
      for (int q = 0; q < xrows.ngroups; ++q) {
        const DimGroup& G = xrows.grp[q];
        int x[kMaxGroup];
        for (int s = 0; s < G.g; ++s) x[s] = pv[G.letter[s]];
        r = r * G.count + colex_encode(tb, x, G.g);
      }
      int64_t col = 0;
      for (int q = 0; q < xcols.ngroups; ++q) {
        const DimGroup& G = xcols.grp[q];
        int x[kMaxGroup];
        for (int s = 0; s < G.g; ++s) x[s] = pv[G.letter[s]];
        col = col * G.count + colex_encode(tb, x, G.g);
      }
      acc += fc.sign[c] * (double)X[r * xcols.size + col];
    }
    int sgn;
    int64_t off = operand_offset(tb, outd, val, &sgn);
    out[off] += alpha * acc;
  }
}

void launch_fold(const IndexTables& tb, const OperandDesc& outd, const MatDim& outdims, const MatDim& xrows,
                 const MatDim& xcols, const FoldCombos& fc, const void* X, Prec xprec, double* out, double alpha,
                 hipStream_t s) {
  int64_t total = outdims.size;
  if (total == 0) return;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (xprec == Prec::FP64)
    fold_kernel<double><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(tb, outd, outdims, xrows, xcols, fc,
                                                                     (const double*)X, out, alpha, total);
  else
    fold_kernel<float><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(tb, outd, outdims, xrows, xcols, fc,
                                                                    (const float*)X, out, alpha, total);
  FNO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- elementwise
__global__ void __launch_bounds__(256) fill_kernel(double* __restrict__ x, double v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) x[i] = v;
}

void launch_fill(double* x, double v, int64_t n, hipStream_t s) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  fill_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(x, v, n);
  FNO_HIP(hipGetLastError());
}

// Several arrays cleared by one launch: blockIdx.y picks the array.
constexpr int kZeroMax = 16;
struct ZeroList {
  double* p[kZeroMax];
  int64_t n[kZeroMax];
};
__global__ void __launch_bounds__(256) zero_many_kernel(ZeroList z) {
  double* p = z.p[blockIdx.y];
  const int64_t n = z.n[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

void launch_zero_many(double* const* ptrs, const int64_t* ns, int count, hipStream_t s) {
  int i = 0;
  while (i < count) {
    ZeroList z{};
    int k = 0;
    int64_t nmax = 0;
    for (; i < count && k < kZeroMax; ++i) {
      if (ns[i] <= 0) continue;
      z.p[k] = ptrs[i];
      z.n[k] = ns[i];
      nmax = std::max(nmax, ns[i]);
      ++k;
    }
    if (k == 0) continue;
    const int64_t blocks = std::min<int64_t>((nmax + 255) / 256, 4096);
    zero_many_kernel<<<dim3((unsigned)blocks, (unsigned)k), dim3(256), 0, s>>>(z);
    FNO_HIP(hipGetLastError());
  }
}

__global__ void __launch_bounds__(256) axpby_kernel(double* __restrict__ y, const double* __restrict__ x, double a,
                                                    double b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) y[i] = a * x[i] + b * y[i];
}

void launch_axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t s) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  axpby_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(y, x, a, b, n);
  FNO_HIP(hipGetLastError());
}

// y_j = a * x_j for j < count and y_j = 0 for count <= j < rows, each of n
// elements (y_j = y + j * ldy, x_j = x + j * ldx): a block of vectors in one launch
__global__ void __launch_bounds__(256) scale_rows_kernel(double* __restrict__ y, int64_t ldy,
                                                         const double* __restrict__ x, int64_t ldx, double a,
                                                         int64_t n, int count) {
  const int j = blockIdx.y;
  double* yj = y + (int64_t)j * ldy;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
  if (j < count) {  // uniform per block: rows past count are never read
    const double* xj = x + (int64_t)j * ldx;
    for (int64_t i = i0; i < n; i += step) yj[i] = a * xj[i];
  } else {
    for (int64_t i = i0; i < n; i += step) yj[i] = 0.0;
  }
}

void launch_scale_rows(double* y, int64_t ldy, const double* x, int64_t ldx, double a, int64_t n, int count, int rows,
                       hipStream_t s) {
  if (n == 0 || rows == 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  scale_rows_kernel<<<dim3((unsigned)blocks, (unsigned)rows), dim3(256), 0, s>>>(y, ldy, x, ldx, a, n, count);
  FNO_HIP(hipGetLastError());
}

// Zeroth-order denominators of a packed block: D = sum_holes e_h - sum_particles e_p
// scaled by hole_sign / particle_sign (both +1 for amplitudes; the EOM diagonal
// uses D = sum_p e_p - sum_h e_h).  out = D (shift applied: out = shift - D when
// shift_mode).
__global__ void __launch_bounds__(256) denom_kernel(IndexTables tb, MatDim dims, int nh, const double* __restrict__ eo,
                                                    const double* __restrict__ ev, double* __restrict__ out,
                                                    int64_t total) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < total; i += stride) {
    int val[kMaxLetters];
    decode_dim(tb, dims, i, val);
    double d = 0.0;
    int nl = 0;
    for (int q = 0; q < dims.ngroups; ++q) nl += dims.grp[q].g;
    for (int l = 0; l < nl; ++l) d += (l < nh) ? eo[val[l]] : -ev[val[l]];
    out[i] = d;
  }
}

void launch_denominators(const IndexTables& tb, const MatDim& dims, int nh, const double* eo, const double* ev,
                         double* out, hipStream_t s) {
  int64_t total = dims.size;
  if (total == 0) return;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  denom_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(tb, dims, nh, eo, ev, out, total);
  FNO_HIP(hipGetLastError());
}

// t += r / d  (Jacobi step); also writes the step into `step` when non-null.
__global__ void __launch_bounds__(256) jacobi_kernel(double* __restrict__ t, const double* __restrict__ r,
                                                     const double* __restrict__ d, double* __restrict__ step,
                                                     int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    double s = r[i] / d[i];
    t[i] += s;
    if (step) step[i] = s;
  }
}

void launch_jacobi(double* t, const double* r, const double* d, double* step, int64_t n, hipStream_t s) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  jacobi_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(t, r, d, step, n);
  FNO_HIP(hipGetLastError());
}

// y = x / (shift - d) elementwise with a floor on |shift - d| (Davidson preconditioner).
__global__ void __launch_bounds__(256) precond_kernel(double* __restrict__ y, const double* __restrict__ x,
                                                      const double* __restrict__ d, double shift, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    double den = shift - d[i];
    if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
    y[i] = x[i] / den;
  }
}

void launch_precond(double* y, const double* x, const double* d, double shift, int64_t n, hipStream_t s) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  precond_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(y, x, d, shift, n);
  FNO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- reductions
// Batched dot products: out[j] = sum_i x_j[i] * y[i] for j < nvec, with
// x_j = xs + j * ldx.  Deterministic: fixed block partition, wavefront
// shuffles, then a second pass over the per-block partials in fixed order.
constexpr int kDotBlocks = 512;

__global__ void __launch_bounds__(256) dot_partial_kernel(const double* __restrict__ xs, int64_t ldx,
                                                          const double* __restrict__ y, int64_t n,
                                                          double* __restrict__ partial) {
  const int j = blockIdx.y;
  const double* x = xs + (int64_t)j * ldx;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc += x[i] * y[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double wsum[4];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wsum[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ void __launch_bounds__(256) dot_final_kernel(const double* __restrict__ partial, int nblk,
                                                        double* __restrict__ out) {
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partial[(int64_t)j * nblk + i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double wsum[4];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wsum[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[j] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ void __launch_bounds__(256) dot_final_acc_kernel(const double* __restrict__ partial, int nblk,
                                                            double* __restrict__ out, double alpha, double beta) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partial[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double wsum[4];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wsum[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double d = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    out[0] = beta != 0.0 ? alpha * d + beta * out[0] : alpha * d;
  }
}

int dot_partial_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > kDotBlocks) b = kDotBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_dots(const double* xs, int64_t ldx, int nvec, const double* y, int64_t n, double* partial, double* out,
                 hipStream_t s) {
  if (nvec == 0) return;
  int nb = dot_partial_blocks(n);
  dot_partial_kernel<<<dim3(nb, nvec), dim3(256), 0, s>>>(xs, ldx, y, n, partial);
  FNO_HIP(hipGetLastError());
  dot_final_kernel<<<dim3(nvec), dim3(256), 0, s>>>(partial, nb, out);
  FNO_HIP(hipGetLastError());
}

void launch_dot_acc(const double* x, const double* y, int64_t n, double* partial, double* out, double alpha,
                    double beta, hipStream_t s) {
  int nb = dot_partial_blocks(n);
  dot_partial_kernel<<<dim3(nb, 1), dim3(256), 0, s>>>(x, n, y, n, partial);
  FNO_HIP(hipGetLastError());
  dot_final_acc_kernel<<<dim3(1), dim3(256), 0, s>>>(partial, nb, out, alpha, beta);
  FNO_HIP(hipGetLastError());
}

// One pass of a Jacobi step with its DIIS bookkeeping:
//   e = r / d,  t_next = t + e,  e_slot = e,  |r|^2,  <e_k | e> for k < nk
// (e_k = es + k * ld; slot k == slot is the new e itself).  Reads t, r, d and
// the nk history error vectors once (the slot's old vector too, so that every
// load is unconditional); per-block partials (row 0: |r|^2, row 1 + k:
// <e_k|e>) are summed in a fixed order by diis_final_kernel.
constexpr int kDiisBlocks = 2048;
constexpr int kDiisMaxVec = 16;

template <int NK>
__global__ void __launch_bounds__(256) diis_step_kernel(const double* __restrict__ t, const double* __restrict__ r,
                                                        const double* __restrict__ d, double* __restrict__ t_next,
                                                        double* __restrict__ es, int64_t ld, int slot, int64_t n,
                                                        double* __restrict__ partial) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  double acc[NK + 1];
#pragma unroll
  for (int k = 0; k <= NK; ++k) acc[k] = 0.0;
  double* e_new = es + (int64_t)slot * ld;
  // pairs of elements with 16-byte loads (every array starts 16-byte aligned
  // and the history stride ld is even); the odd last element, if any, below
  const int64_t np = n / 2;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = 2 * p;
    // every load of the pair first (the slot's old value is read and
    // replaced by the new error), then the arithmetic
    d2 h[NK > 0 ? NK : 1];
#pragma unroll
    for (int k = 0; k < NK; ++k) h[k] = *(const d2*)(es + (int64_t)k * ld + i);
    const d2 ri = *(const d2*)(r + i);
    const d2 di = *(const d2*)(d + i);
    const d2 ti = *(const d2*)(t + i);
    d2 e;
    e.x = ri.x / di.x;
    e.y = ri.y / di.y;
    *(d2*)(t_next + i) = ti + e;
    *(d2*)(e_new + i) = e;
    acc[0] += ri.x * ri.x + ri.y * ri.y;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const d2 hk = k == slot ? e : h[k];
      acc[1 + k] += hk.x * e.x + hk.y * e.y;
    }
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t i = n - 1;
    const double ri = r[i], e = ri / d[i];
    double hk[NK > 0 ? NK : 1];
#pragma unroll
    for (int k = 0; k < NK; ++k) hk[k] = es[(int64_t)k * ld + i];
    t_next[i] = t[i] + e;
    e_new[i] = e;
    acc[0] += ri * ri;
#pragma unroll
    for (int k = 0; k < NK; ++k) acc[1 + k] += (k == slot ? e : hk[k]) * e;
  }
  __shared__ double wsum[4][NK + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k <= NK; ++k) {
    double a = acc[k];
    for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
    if (lane == 0) wsum[w][k] = a;
  }
  __syncthreads();
  if (threadIdx.x <= NK)
    partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] =
        wsum[0][threadIdx.x] + wsum[1][threadIdx.x] + wsum[2][threadIdx.x] + wsum[3][threadIdx.x];
}

// out_rr = row 0 of the partials, out_ov[k] = row 1 + k
__global__ void __launch_bounds__(256) diis_final_kernel(const double* __restrict__ partial, int nblk,
                                                         double* __restrict__ out_rr, double* __restrict__ out_ov) {
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partial[(int64_t)j * nblk + i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double wsum[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wsum[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double v = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (j == 0)
      out_rr[0] = v;
    else
      out_ov[j - 1] = v;
  }
}

int diis_step_partials(int nk) { return (nk + 1) * kDiisBlocks; }

void launch_diis_step(const double* t, const double* r, const double* d, double* t_next, double* es, int64_t ld,
                      int slot, int nk, int64_t n, double* partial, double* out_rr, double* out_ov, hipStream_t s) {
  FNO_REQUIRE(nk >= 0 && nk <= kDiisMaxVec && (nk == 0 || (slot >= 0 && slot < nk)), kEINVAL,
              "DIIS step: history of " + std::to_string(nk) + " vectors, slot " + std::to_string(slot));
  FNO_REQUIRE(ld >= n && ld % 2 == 0, kEINVAL, "DIIS step: history stride must be even and cover n");
  for (const void* p : {(const void*)t, (const void*)r, (const void*)d, (const void*)t_next, (const void*)es})
    FNO_REQUIRE(((uintptr_t)p & 15) == 0, kEINVAL, "DIIS step: arrays must be 16-byte aligned");
  if (n == 0) return;
  int64_t blocks = (n / 2 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > kDiisBlocks) blocks = kDiisBlocks;
  const dim3 grid((unsigned)blocks), blk(256);
  switch (nk) {
#define FNO_DIIS_CASE(K) \
  case K:                \
    diis_step_kernel<K><<<grid, blk, 0, s>>>(t, r, d, t_next, es, ld, slot, n, partial); \
    break;
    FNO_DIIS_CASE(0) FNO_DIIS_CASE(1) FNO_DIIS_CASE(2) FNO_DIIS_CASE(3) FNO_DIIS_CASE(4) FNO_DIIS_CASE(5)
    FNO_DIIS_CASE(6) FNO_DIIS_CASE(7) FNO_DIIS_CASE(8) FNO_DIIS_CASE(9) FNO_DIIS_CASE(10) FNO_DIIS_CASE(11)
    FNO_DIIS_CASE(12) FNO_DIIS_CASE(13) FNO_DIIS_CASE(14) FNO_DIIS_CASE(15) FNO_DIIS_CASE(16)
#undef FNO_DIIS_CASE
  }
  FNO_HIP(hipGetLastError());
  diis_final_kernel<<<dim3(nk + 1), dim3(256), 0, s>>>(partial, (int)blocks, out_rr, out_ov);
  FNO_HIP(hipGetLastError());
}

// CC correlation energy (eq 7) in closed form over unique index pairs:
//   E = sum_ia f_ia t_ia + sum_{i<j, a<b} <ij||ab> (t_ij^ab + t_ia t_jb - t_ib t_ja)
// (the quarter-weighted sum over all ijab of <ij||ab> t_ij^ab and the half-
// weighted one of <ij||ab> t_ia t_jb, folded onto i < j, a < b with the
// antisymmetry of the integrals).  f: n x n, g: n^4 (both row-major, occupied
// orbitals first), t1: o x v, t2: packed [i<j][a<b] (colex pairs).  Per-block
// partials in a fixed partition, summed in a fixed order by dot_final_acc.
constexpr int kEnergyBlocks = 256;

__device__ __forceinline__ void unpair(int64_t p, int& x0, int& x1) {
  // x0 < x1 with p = x0 + x1 (x1 - 1) / 2
  int h = (int)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
  while ((int64_t)h * (h - 1) / 2 > p) --h;
  while ((int64_t)(h + 1) * h / 2 <= p) ++h;
  x1 = h;
  x0 = (int)(p - (int64_t)h * (h - 1) / 2);
}

__global__ void __launch_bounds__(256) cc_energy_kernel(const double* __restrict__ f, const double* __restrict__ g,
                                                        const double* __restrict__ t1, const double* __restrict__ t2,
                                                        int o, int v, double* __restrict__ partial) {
  const int64_t n = o + v;
  const int64_t nv2 = (int64_t)v * (v - 1) / 2, no2 = (int64_t)o * (o - 1) / 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < no2 * nv2; q += stride) {
    int i, j, a, b;
    unpair(q / nv2, i, j);
    unpair(q % nv2, a, b);
    const double gv = g[((i * n + j) * n + o + a) * n + o + b];
    acc += gv * (t2[q] + t1[i * v + a] * t1[j * v + b] - t1[i * v + b] * t1[j * v + a]);
  }
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < (int64_t)o * v; q += stride) {
    const int64_t i = q / v, a = q - i * v;
    acc += f[i * n + o + a] * t1[q];
  }
  for (int s = 32; s > 0; s >>= 1) acc += __shfl_down(acc, s, 64);
  __shared__ double wsum[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wsum[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

void launch_cc_energy(const double* f, const double* g, const double* t1, const double* t2, int o, int v,
                      double* partial, double* out, hipStream_t s) {
  cc_energy_kernel<<<dim3(kEnergyBlocks), dim3(256), 0, s>>>(f, g, t1, t2, o, v, partial);
  FNO_HIP(hipGetLastError());
  dot_final_acc_kernel<<<dim3(1), dim3(256), 0, s>>>(partial, kEnergyBlocks, out, 1.0, 0.0);
  FNO_HIP(hipGetLastError());
}

// y -= sum_j c[j] * x_j   (Gram-Schmidt projection / Ritz combination)
__global__ void __launch_bounds__(256) gemv_acc_kernel(double* __restrict__ y, const double* __restrict__ xs,
                                                       int64_t ldx, const double* __restrict__ c, int nvec,
                                                       double alpha, double beta, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    double acc = 0.0;
    for (int j = 0; j < nvec; ++j) acc += c[j] * xs[(int64_t)j * ldx + i];
    y[i] = beta * y[i] + alpha * acc;
  }
}

// The same on element pairs (16-byte loads and stores; every element gets the
// same operations in the same order as in gemv_acc_kernel), for 16-byte
// aligned y and x_j with an even stride; the odd last element separately.
__global__ void __launch_bounds__(256) gemv_acc2_kernel(double* __restrict__ y, const double* __restrict__ xs,
                                                        int64_t ldx, const double* __restrict__ c, int nvec,
                                                        double alpha, double beta, int64_t n) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int64_t np = n / 2;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = 2 * p;
    double a0 = 0.0, a1 = 0.0;
    for (int j = 0; j < nvec; ++j) {
      const d2 x = *(const d2*)(xs + (int64_t)j * ldx + i);
      a0 += c[j] * x.x;
      a1 += c[j] * x.y;
    }
    const d2 yv = *(const d2*)(y + i);
    d2 out;
    out.x = beta * yv.x + alpha * a0;
    out.y = beta * yv.y + alpha * a1;
    *(d2*)(y + i) = out;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t i = n - 1;
    double acc = 0.0;
    for (int j = 0; j < nvec; ++j) acc += c[j] * xs[(int64_t)j * ldx + i];
    y[i] = beta * y[i] + alpha * acc;
  }
}

// DIIS step on the device (one workgroup): store the overlaps of the newest
// error vector (history slot `slot`) with the vectors of the slots in use
// into the overlap matrix B (16 x 16, by slot), and, when extrapolating, solve
//   [ B/s  -1 ] [c]   [ 0]
//   [ -1    0 ] [l] = [-1]     (s = the largest diagonal element)
// over those slots by Gaussian elimination with partial pivoting, the
// system in LDS and each elimination step's row updates spread over the
// threads (every element is updated by the same operations as in a serial
// elimination).  coef gets the coefficients by slot, or the unit vector of
// `slot` when the system is singular (a pivot below 1e-300) or no
// extrapolation is asked for.
__global__ void __launch_bounds__(256) diis_kernel(double* __restrict__ B, const double* __restrict__ ov, int slot,
                                                   DiisSlots ord, int extrap, int nc, double* __restrict__ coef) {
  __shared__ double A[17][18], b[17], f[17];
  __shared__ int fail, piv;
  const int tid = threadIdx.x, k = ord.k, n = k + 1;
  // B entries of the new slot come from ov; the others were stored before
  auto bval = [&](int qa, int qb) {
    return qa == slot ? ov[qb] : (qb == slot ? ov[qa] : B[qa * 16 + qb]);
  };
  if (extrap && k >= 1) {
    double scale = 0;
    for (int a = 0; a < k; ++a) scale = fmax(scale, fabs(bval(ord.slot[a], ord.slot[a])));
    if (scale == 0) scale = 1;
    for (int e = tid; e < n * n; e += blockDim.x) {
      const int r = e / n, c = e % n;
      A[r][c] = (r < k && c < k) ? bval(ord.slot[r], ord.slot[c]) / scale : ((r == k && c == k) ? 0.0 : -1.0);
    }
    for (int r = tid; r < n; r += blockDim.x) b[r] = (r == k) ? -1.0 : 0.0;
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int c = 0; c < n; ++c) {
      if (tid == 0) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
          if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
        if (fabs(A[p][c]) < 1e-300) fail = 1;
        piv = p;
      }
      __syncthreads();
      if (fail) break;
      const int p = piv;
      if (p != c) {
        for (int q = tid; q < n; q += blockDim.x) {
          const double t = A[p][q];
          A[p][q] = A[c][q];
          A[c][q] = t;
        }
        if (tid == 0) {
          const double t = b[p];
          b[p] = b[c];
          b[c] = t;
        }
      }
      __syncthreads();
      for (int r = c + 1 + tid; r < n; r += blockDim.x) f[r] = A[r][c] / A[c][c];
      __syncthreads();
      const int w = n - c;
      for (int e = tid; e < (n - c - 1) * w; e += blockDim.x) {
        const int r = c + 1 + e / w, q = c + e % w;
        if (f[r] != 0) A[r][q] -= f[r] * A[c][q];
      }
      for (int r = c + 1 + tid; r < n; r += blockDim.x)
        if (f[r] != 0) b[r] -= f[r] * b[c];
      __syncthreads();
    }
    if (!fail && tid == 0) {
      for (int r = n - 1; r >= 0; --r) {
        double acc = b[r];
        for (int q = r + 1; q < n; ++q) acc -= A[r][q] * b[q];
        b[r] = acc / A[r][r];
      }
    }
    __syncthreads();
  }
  const bool solved = extrap && k >= 1 && !fail;
  for (int c = tid; c < nc; c += blockDim.x) coef[c] = solved ? 0.0 : (c == slot ? 1.0 : 0.0);
  __syncthreads();
  if (solved)
    for (int a = tid; a < k; a += blockDim.x) coef[ord.slot[a]] = b[a];
  for (int a = tid; a < k; a += blockDim.x) {
    const int q = ord.slot[a];
    B[slot * 16 + q] = ov[q];
    B[q * 16 + slot] = ov[q];
  }
}

void launch_diis(double* B, const double* ov, int slot, const DiisSlots& ord, bool extrap, int nc, double* coef,
                 hipStream_t s) {
  diis_kernel<<<1, 256, 0, s>>>(B, ov, slot, ord, extrap ? 1 : 0, nc, coef);
  FNO_HIP(hipGetLastError());
}

void launch_combine(double* y, const double* xs, int64_t ldx, const double* c, int nvec, double alpha, double beta,
                    int64_t n, hipStream_t s) {
  if (n == 0) return;
  if (n >= 2 && ldx % 2 == 0 && (((uintptr_t)y | (uintptr_t)xs) & 15) == 0) {
    int64_t blocks = (n / 2 + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    gemv_acc2_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(y, xs, ldx, c, nvec, alpha, beta, n);
    FNO_HIP(hipGetLastError());
    return;
  }
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  gemv_acc_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(y, xs, ldx, c, nvec, alpha, beta, n);
  FNO_HIP(hipGetLastError());
}

}  // namespace fno

namespace fno {

// ---------------------------------------------------------------- plan tables
__global__ void __launch_bounds__(256) dim_table_kernel(IndexTables tb, OperandDesc op, MatDim dims, unsigned mask,
                                                        int64_t* __restrict__ off, int8_t* __restrict__ sign) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dims.size;
       i += (int64_t)gridDim.x * blockDim.x) {
    int val[kMaxLetters];
    decode_dim(tb, dims, i, val);
    int64_t o = op.base;
    int sg = 1;
    for (int q = 0; q < op.ngroups; ++q) {
      if (!((mask >> q) & 1u)) continue;
      const GroupDesc& G = op.grp[q];
      if (G.g == 1) {
        o += (int64_t)(val[G.letter[0]] + G.off) * G.stride;
        continue;
      }
      int x[kMaxGroup];
      for (int s = 0; s < G.g; ++s) x[s] = val[G.letter[s]];
      for (int a = 1; a < G.g; ++a) {
        int v = x[a], b = a - 1;
        while (b >= 0 && x[b] > v) {
          x[b + 1] = x[b];
          --b;
          sg = -sg;
        }
        x[b + 1] = v;
      }
      bool rep = false;
      for (int a = 1; a < G.g; ++a) rep |= (x[a] == x[a - 1]);
      if (rep) {
        sg = 0;
        continue;
      }
      o += colex_encode(tb, x, G.g) * G.stride;
    }
    off[i] = o;
    sign[i] = (int8_t)sg;
  }
}

void launch_dim_table(const IndexTables& tb, const OperandDesc& op, const MatDim& dims, unsigned group_mask,
                      int64_t* off, int8_t* sign, hipStream_t s) {
  if (dims.size == 0) return;
  int64_t blocks = std::min<int64_t>((dims.size + 255) / 256, 16384);
  dim_table_kernel<<<dim3((unsigned)blocks), 256, 0, s>>>(tb, op, dims, group_mask, off, sign);
  FNO_HIP(hipGetLastError());
}

__global__ void __launch_bounds__(256) sub_index_kernel(MatDim dims, unsigned dg_mask, int32_t* __restrict__ sub) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dims.size;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t idx = i, r = 0, mult = 1;
    for (int q = dims.ngroups - 1; q >= 0; --q) {
      int64_t t = idx % dims.grp[q].count;
      idx /= dims.grp[q].count;
      if ((dg_mask >> q) & 1u) {
        r += t * mult;
        mult *= dims.grp[q].count;
      }
    }
    sub[i] = (int32_t)r;
  }
}

void launch_sub_index(const IndexTables&, const MatDim& dims, unsigned dg_mask, int32_t* sub, hipStream_t s) {
  if (dims.size == 0) return;
  int64_t blocks = std::min<int64_t>((dims.size + 255) / 256, 16384);
  sub_index_kernel<<<dim3((unsigned)blocks), 256, 0, s>>>(dims, dg_mask, sub);
  FNO_HIP(hipGetLastError());
}

__global__ void __launch_bounds__(256) mixed_table_kernel(IndexTables tb, OperandDesc op, int grp, MatDim pr,
                                                          MatDim pc, int64_t* __restrict__ off,
                                                          int8_t* __restrict__ sign) {
  const int64_t total = pr.size * pc.size;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    int val[kMaxLetters];
    decode_dim(tb, pr, i / pc.size, val);
    decode_dim(tb, pc, i % pc.size, val);
    const GroupDesc& G = op.grp[grp];
    int x[kMaxGroup];
    int sg = 1;
    for (int s = 0; s < G.g; ++s) x[s] = val[G.letter[s]];
    for (int a = 1; a < G.g; ++a) {
      int v = x[a], b = a - 1;
      while (b >= 0 && x[b] > v) {
        x[b + 1] = x[b];
        --b;
        sg = -sg;
      }
      x[b + 1] = v;
    }
    bool rep = false;
    for (int a = 1; a < G.g; ++a) rep |= (x[a] == x[a - 1]);
    off[i] = rep ? 0 : colex_encode(tb, x, G.g) * G.stride;
    sign[i] = rep ? 0 : (int8_t)sg;
  }
}

void launch_mixed_table(const IndexTables& tb, const OperandDesc& op, int grp, const MatDim& part_r,
                        const MatDim& part_c, int64_t* off, int8_t* sign, hipStream_t s) {
  int64_t total = part_r.size * part_c.size;
  if (total == 0) return;
  int64_t blocks = std::min<int64_t>((total + 255) / 256, 16384);
  mixed_table_kernel<<<dim3((unsigned)blocks), 256, 0, s>>>(tb, op, grp, part_r, part_c, off, sign);
  FNO_HIP(hipGetLastError());
}

struct ShufSrc {
  int8_t src[kMaxCombos][kMaxLetters];
};

__global__ void __launch_bounds__(256) fold_table_kernel(IndexTables tb, DimGroup og, int nshuf, ShufSrc sh,
                                                         int nletters, MatDim xr, MatDim xc, unsigned xr_mask,
                                                         unsigned xc_mask, int64_t* __restrict__ rowc,
                                                         int64_t* __restrict__ colc) {
  const int64_t total = og.count * nshuf;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(i / og.count);
    const int64_t u = i % og.count;
    int val[kMaxLetters];
    for (int l = 0; l < kMaxLetters; ++l) val[l] = 0;
    int x[kMaxGroup];
    colex_decode(tb, u, og.g, x);
    for (int t = 0; t < og.g; ++t) val[og.letter[t]] = x[t];
    int pv[kMaxLetters];
    for (int l = 0; l < nletters; ++l) pv[l] = val[sh.src[s][l]];
    // strides of the X row / column DimGroups
    int64_t r = 0, mult = 1;
    for (int q = xr.ngroups - 1; q >= 0; --q) {
      const DimGroup& G = xr.grp[q];
      if ((xr_mask >> q) & 1u) {
        int y[kMaxGroup];
        for (int t = 0; t < G.g; ++t) y[t] = pv[G.letter[t]];
        r += colex_encode(tb, y, G.g) * mult;
      }
      mult *= G.count;
    }
    int64_t c = 0;
    mult = 1;
    for (int q = xc.ngroups - 1; q >= 0; --q) {
      const DimGroup& G = xc.grp[q];
      if ((xc_mask >> q) & 1u) {
        int y[kMaxGroup];
        for (int t = 0; t < G.g; ++t) y[t] = pv[G.letter[t]];
        c += colex_encode(tb, y, G.g) * mult;
      }
      mult *= G.count;
    }
    rowc[i] = r;
    colc[i] = c;
  }
}

void launch_fold_table(const IndexTables& tb, const DimGroup& og, int nshuf, const int8_t* shuf_src, int nletters,
                       const MatDim& xrows, const MatDim& xcols, unsigned xr_mask, unsigned xc_mask, int64_t* rowc,
                       int64_t* colc, hipStream_t s) {
  ShufSrc sh{};
  for (int k = 0; k < nshuf; ++k)
    for (int l = 0; l < kMaxLetters; ++l) sh.src[k][l] = shuf_src[k * kMaxLetters + l];
  int64_t total = og.count * nshuf;
  if (total == 0) return;
  int64_t blocks = std::min<int64_t>((total + 255) / 256, 16384);
  fold_table_kernel<<<dim3((unsigned)blocks), 256, 0, s>>>(tb, og, nshuf, sh, nletters, xrows, xcols, xr_mask,
                                                           xc_mask, rowc, colc);
  FNO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- hot paths
// Each thread owns one column c (its table entries stay in registers) and
// walks a contiguous range of rows, kRowStep rows per step.  The row entries
// are uniform per step (scalar loads); within a step every table gather of
// the rows is issued before the first is used, then every source gather, so a
// wavefront keeps kRowStep independent chains in flight instead of one.
constexpr int kRowStep = 4;
__device__ const double kExpandZero = 0.0;

template <int MODE>  // 0 = FP64, 1 = FP32, 2 = split-BF16 (hi, lo)
__device__ __forceinline__ void expand_store(void* dst, void* dst_lo, int64_t i, double v) {
  if constexpr (MODE == 0) {
    ((double*)dst)[i] = v;
  } else if constexpr (MODE == 1) {
    ((float*)dst)[i] = (float)v;
  } else {
    const float x = (float)v;
    const __hip_bfloat16 h = __float2bfloat16(x);
    ((__hip_bfloat16*)dst)[i] = h;
    ((__hip_bfloat16*)dst_lo)[i] = __float2bfloat16(x - __bfloat162float(h));
  }
}

template <int MODE, int NM, int R>
__device__ __forceinline__ void expand_rows(const ExpandTab& t, const double* __restrict__ src, void* dst,
                                            void* dst_lo, int64_t r, int64_t c, int64_t co, int cs,
                                            const int32_t (&csub)[kMaxMixed]) {
  int64_t o[R];
  int sg[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    o[q] = t.row_off[r + q] + co;
    sg[q] = t.row_sign[r + q] * cs;
  }
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    int64_t to[R];
    int ts[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t k = (int64_t)t.row_sub[m][r + q] * t.ncsub[m] + csub[m];
      to[q] = t.tab_off[m][k];
      ts[q] = t.tab_sign[m][k];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      o[q] += to[q];
      sg[q] *= ts[q];
    }
  }
  // lanes with a repeated index read a zero from a fixed address: the loads
  // stay unconditional (no branch, so no wait) and never touch an empty source
  double v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) v[q] = *(sg[q] ? src + o[q] : &kExpandZero);
#pragma unroll
  for (int q = 0; q < R; ++q) expand_store<MODE>(dst, dst_lo, (r + q) * t.ld + c, sg[q] * v[q]);
}

template <int MODE, int NM>
__global__ void __launch_bounds__(256) expand_tab_kernel(ExpandTab t, const double* __restrict__ src, void* dst,
                                                         void* dst_lo) {
  const int64_t L = xcd_chunk((int64_t)blockIdx.y * gridDim.x + blockIdx.x, (int64_t)gridDim.x * gridDim.y);
  const int64_t bx = L % gridDim.x, by = L / gridDim.x;
  const int64_t c = bx * blockDim.x + threadIdx.x;
  if (c >= t.cols) return;
  const int64_t co = t.col_off[c];
  const int cs = t.col_sign[c];
  int32_t csub[kMaxMixed] = {0, 0};
#pragma unroll
  for (int m = 0; m < NM; ++m) csub[m] = t.col_sub[m][c];
  // a contiguous range of rows per block: neighbouring rows gather from
  // neighbouring source elements, so the cache lines are reused
  const int64_t per = (t.rows + gridDim.y - 1) / gridDim.y;
  const int64_t r_end = (by + 1) * per < t.rows ? (by + 1) * per : t.rows;
  int64_t r = by * per;
  for (; r + kRowStep <= r_end; r += kRowStep) expand_rows<MODE, NM, kRowStep>(t, src, dst, dst_lo, r, c, co, cs, csub);
  for (; r < r_end; ++r) expand_rows<MODE, NM, 1>(t, src, dst, dst_lo, r, c, co, cs, csub);
}

// Narrow matrices (few columns): one thread per element over the flat index.
template <int MODE>  // 0 = FP64, 1 = FP32, 2 = split-BF16
__global__ void __launch_bounds__(256) expand_tab_flat_kernel(ExpandTab t, const double* __restrict__ src, void* dst,
                                                              void* dst_lo) {
  const int64_t total = t.rows * t.cols;
  const int64_t first = xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  for (int64_t i = first; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t.cols == 1 ? i : i / t.cols;
    const int64_t c = i - r * t.cols;
    int64_t o = t.row_off[r] + t.col_off[c];
    int s = t.row_sign[r] * t.col_sign[c];
    for (int m = 0; m < t.nmixed; ++m) {
      const int64_t k = (int64_t)t.row_sub[m][r] * t.ncsub[m] + t.col_sub[m][c];
      o += t.tab_off[m][k];
      s *= t.tab_sign[m][k];
    }
    const double v = s ? s * src[o] : 0.0;
    const int64_t d = r * t.ld + c;  // rows may be padded (t.ld >= t.cols)
    if (MODE == 0) {
      ((double*)dst)[d] = v;
    } else if (MODE == 1) {
      ((float*)dst)[d] = (float)v;
    } else {
      const float x = (float)v;
      const __hip_bfloat16 h = __float2bfloat16(x);
      ((__hip_bfloat16*)dst)[d] = h;
      ((__hip_bfloat16*)dst_lo)[d] = __float2bfloat16(x - __bfloat162float(h));
    }
  }
}

// out[i] += alpha * (gathered element i), the expansion as an M x 1 matrix
__global__ void __launch_bounds__(256) expand_tab_acc_kernel(ExpandTab t, const double* __restrict__ src,
                                                             double* __restrict__ out, double alpha) {
  const int64_t total = t.rows * t.cols;
  const int64_t first = xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  for (int64_t i = first; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t.cols == 1 ? i : i / t.cols;
    const int64_t c = i - r * t.cols;
    int64_t o = t.row_off[r] + t.col_off[c];
    int s = t.row_sign[r] * t.col_sign[c];
    for (int m = 0; m < t.nmixed; ++m) {
      const int64_t k = (int64_t)t.row_sub[m][r] * t.ncsub[m] + t.col_sub[m][c];
      o += t.tab_off[m][k];
      s *= t.tab_sign[m][k];
    }
    if (s) out[i] += alpha * (s * src[o]);
  }
}

void launch_expand_tab_acc(const ExpandTab& t, const double* src, double* out, double alpha, hipStream_t s) {
  const int64_t total = t.rows * t.cols;
  if (total == 0) return;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  expand_tab_acc_kernel<<<dim3((unsigned)blocks), 256, 0, s>>>(t, src, out, alpha);
  FNO_HIP(hipGetLastError());
}

template <int MODE>
static void launch_expand_rows_m(int nm, dim3 grid, const ExpandTab& t, const double* src, void* dst, void* dst_lo,
                                 hipStream_t s) {
  if (nm == 0)
    expand_tab_kernel<MODE, 0><<<grid, 256, 0, s>>>(t, src, dst, dst_lo);
  else if (nm == 1)
    expand_tab_kernel<MODE, 1><<<grid, 256, 0, s>>>(t, src, dst, dst_lo);
  else
    expand_tab_kernel<MODE, 2><<<grid, 256, 0, s>>>(t, src, dst, dst_lo);
}

static void launch_expand_rows(int mode, int nm, dim3 grid, const ExpandTab& t, const double* src, void* dst,
                               void* dst_lo, hipStream_t s) {
  FNO_REQUIRE(nm >= 0 && nm <= kMaxMixed, kEINVAL, "expansion table with too many straddling groups");
  if (mode == 0)
    launch_expand_rows_m<0>(nm, grid, t, src, dst, dst_lo, s);
  else if (mode == 1)
    launch_expand_rows_m<1>(nm, grid, t, src, dst, dst_lo, s);
  else
    launch_expand_rows_m<2>(nm, grid, t, src, dst, dst_lo, s);
}

void launch_expand_tab(const ExpandTab& t, const double* src, void* dst, void* dst_lo, Prec prec, hipStream_t s) {
  if (t.rows == 0 || t.cols == 0) return;
  FNO_REQUIRE(t.ld >= t.cols, kEINVAL, "expansion row stride shorter than its rows");
  if (t.cols < 128) {
    const int64_t total = t.rows * t.cols;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    if (prec == Prec::FP64)
      expand_tab_flat_kernel<0><<<dim3((unsigned)blocks), 256, 0, s>>>(t, src, dst, dst_lo);
    else if (prec == Prec::FP32)
      expand_tab_flat_kernel<1><<<dim3((unsigned)blocks), 256, 0, s>>>(t, src, dst, dst_lo);
    else
      expand_tab_flat_kernel<2><<<dim3((unsigned)blocks), 256, 0, s>>>(t, src, dst, dst_lo);
    FNO_HIP(hipGetLastError());
    return;
  }
  const unsigned gx = (unsigned)((t.cols + 255) / 256);
  // enough blocks in y to have ~8K blocks in flight
  int64_t gy = std::max<int64_t>(1, std::min<int64_t>(t.rows, (8192 + gx - 1) / gx));
  gy = std::min<int64_t>(gy, 65535);
  dim3 grid(gx, (unsigned)gy);
  const int mode = prec == Prec::FP64 ? 0 : prec == Prec::FP32 ? 1 : 2;
  launch_expand_rows(mode, t.nmixed, grid, t, src, dst, dst_lo, s);
  FNO_HIP(hipGetLastError());
}

template <typename XT>
__global__ void __launch_bounds__(256) fold_tab_kernel(FoldTab t, const XT* __restrict__ X, double* __restrict__ out,
                                                       double alpha, int64_t total) {
  const int64_t first = xcd_chunk(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  for (int64_t e = first; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t u[kMaxOutGroups];
    int64_t idx = e;
    for (int k = t.ngroups - 1; k >= 0; --k) {
      u[k] = idx % t.count[k];
      idx /= t.count[k];
    }
    double acc = 0.0;
    for (int c = 0; c < t.ncombo; ++c) {
      int64_t r = 0, col = 0;
      for (int k = 0; k < t.ngroups; ++k) {
        const int64_t j = (int64_t)t.combo[c][k] * t.count[k] + u[k];
        r += t.rowc[k][j];
        col += t.colc[k][j];
      }
      acc += t.csign[c] * (double)X[r * t.xcols + col];
    }
    out[e] += alpha * acc;
  }
}

// Same fold with the group and combo counts fixed at compile time: the loops
// unroll, so every table entry and every X element of one output is requested
// before the first is used (two memory round trips per output instead of a
// chain of dependent ones).  Summation order as in fold_tab_kernel.
//
// SH (every group has at most kShufMax shuffles): each group's row and column
// parts are read once per shuffle and shared by the combos that pick it (a
// two-group fold with 3 x 3 combos reads 12 table entries instead of 36).
constexpr int kShufMax = 3;
template <typename XT, int NG, int NC, bool SH>
__global__ void __launch_bounds__(256) fold_tab_fixed_kernel(FoldTab t, const XT* __restrict__ X,
                                                             double* __restrict__ out, double alpha, int64_t total,
                                                             int64_t chunk) {
  // each block walks `chunk` consecutive outputs: the matrix lines read by one
  // 256-output step (for the shuffles whose fastest output index runs along
  // the rows of X) are read again by the next steps, from this CU's cache
  const int64_t begin = xcd_chunk(blockIdx.x, gridDim.x) * chunk;
  const int64_t end = begin + chunk < total ? begin + chunk : total;
  for (int64_t e = begin + threadIdx.x; e < end; e += blockDim.x) {
    int64_t u[NG];
    int64_t idx = e;
#pragma unroll
    for (int k = NG - 1; k >= 0; --k) {
      u[k] = idx % t.count[k];
      idx /= t.count[k];
    }
    int64_t addr[NC];
    if constexpr (SH) {
      int64_t rr[NG][kShufMax], cc[NG][kShufMax];
#pragma unroll
      for (int k = 0; k < NG; ++k)
#pragma unroll
        for (int q = 0; q < kShufMax; ++q) {
          rr[k][q] = 0;
          cc[k][q] = 0;
          if (q < t.nshuf[k]) {
            const int64_t j = (int64_t)q * t.count[k] + u[k];
            rr[k][q] = t.rowc[k][j];
            cc[k][q] = t.colc[k][j];
          }
        }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        int64_t r = 0, col = 0;
#pragma unroll
        for (int k = 0; k < NG; ++k) {
          const int q = t.combo[c][k];
          r += q == 0 ? rr[k][0] : (q == 1 ? rr[k][1] : rr[k][2]);
          col += q == 0 ? cc[k][0] : (q == 1 ? cc[k][1] : cc[k][2]);
        }
        addr[c] = r * t.xcols + col;
      }
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        int64_t r = 0, col = 0;
#pragma unroll
        for (int k = 0; k < NG; ++k) {
          const int64_t j = (int64_t)t.combo[c][k] * t.count[k] + u[k];
          r += t.rowc[k][j];
          col += t.colc[k][j];
        }
        addr[c] = r * t.xcols + col;
      }
    }
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = (double)X[addr[c]];
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) acc += t.csign[c] * v[c];
    out[e] += alpha * acc;
  }
}

// Three output groups whose first has a single shuffle (the root or instance
// index), the shuffle counts NS1 and NS2 of the other two fixed at compile
// time.  The host builds the combos as a mixed-radix product, so combo
// c = p1 + NS1 * p2 takes shuffle p1 of group 1 and p2 of group 2: every table
// entry of an output is read once and addressed at compile time, and the sum
// runs over c in the same order as the other fold kernels.
template <typename XT, int NS1, int NS2>
__global__ void __launch_bounds__(256) fold_tab_prod3_kernel(FoldTab t, const XT* __restrict__ X,
                                                             double* __restrict__ out, double alpha, int64_t total,
                                                             int64_t chunk) {
  constexpr int NC = NS1 * NS2;
  const int64_t begin = xcd_chunk(blockIdx.x, gridDim.x) * chunk;
  const int64_t end = begin + chunk < total ? begin + chunk : total;
  for (int64_t e = begin + threadIdx.x; e < end; e += blockDim.x) {
    int64_t idx = e;
    const int64_t u2 = idx % t.count[2];
    idx /= t.count[2];
    const int64_t u1 = idx % t.count[1];
    idx /= t.count[1];
    const int64_t u0 = idx % t.count[0];
    const int64_t r0 = t.rowc[0][u0], c0 = t.colc[0][u0];
    int64_t r1[NS1], c1[NS1], r2[NS2], c2[NS2];
#pragma unroll
    for (int q = 0; q < NS1; ++q) {
      r1[q] = t.rowc[1][(int64_t)q * t.count[1] + u1];
      c1[q] = t.colc[1][(int64_t)q * t.count[1] + u1];
    }
#pragma unroll
    for (int q = 0; q < NS2; ++q) {
      r2[q] = t.rowc[2][(int64_t)q * t.count[2] + u2];
      c2[q] = t.colc[2][(int64_t)q * t.count[2] + u2];
    }
    double v[NC];
#pragma unroll
    for (int p2 = 0; p2 < NS2; ++p2)
#pragma unroll
      for (int p1 = 0; p1 < NS1; ++p1)
        v[p1 + NS1 * p2] = (double)X[(r0 + r1[p1] + r2[p2]) * t.xcols + c0 + c1[p1] + c2[p2]];
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) acc += t.csign[c] * v[c];
    out[e] += alpha * acc;
  }
}

// True when the combo table is the mixed-radix product the product kernels assume.
static bool fold_is_product(const FoldTab& t) {
  if (t.nshuf[1] * t.nshuf[2] != t.ncombo || t.ncombo > kMaxCombos) return false;
  int c = 0;
  for (int p2 = 0; p2 < t.nshuf[2]; ++p2)
    for (int p1 = 0; p1 < t.nshuf[1]; ++p1, ++c)
      if (t.combo[c][0] != 0 || t.combo[c][1] != p1 || t.combo[c][2] != p2) return false;
  return c == t.ncombo;
}

template <typename XT>
static void fold_launch(const FoldTab& t, const XT* X, double* out, double alpha, int64_t total, hipStream_t s) {
  const dim3 grid((unsigned)std::min<int64_t>((total + 255) / 256, 65536));
  // chunks of 8 steps for the largest outputs (the 4p2h / 4h2p sigma blocks)
  const int64_t chunk = total >= ((int64_t)16 << 20) ? 2048 : 256;
  const dim3 cgrid((unsigned)((total + chunk - 1) / chunk));
  if (t.ngroups == 3 && t.nshuf[0] == 1 && fold_is_product(t)) {
#define FNO_FOLD_PROD(A, B)                                                                    \
  if (t.nshuf[1] == A && t.nshuf[2] == B) {                                                    \
    fold_tab_prod3_kernel<XT, A, B><<<cgrid, 256, 0, s>>>(t, X, out, alpha, total, chunk);     \
    return;                                                                                    \
  }
    // every pair the EOM tables produce: hole and particle groups of up to four
    // letters, whose antisymmetrizers have 1, 2, 3, 4, 6 or 12 shuffles
    FNO_FOLD_PROD(1, 1) FNO_FOLD_PROD(1, 2) FNO_FOLD_PROD(2, 1) FNO_FOLD_PROD(2, 2)
    FNO_FOLD_PROD(1, 3) FNO_FOLD_PROD(3, 1) FNO_FOLD_PROD(2, 3) FNO_FOLD_PROD(3, 2) FNO_FOLD_PROD(3, 3)
    FNO_FOLD_PROD(1, 4) FNO_FOLD_PROD(4, 1) FNO_FOLD_PROD(2, 4) FNO_FOLD_PROD(4, 2)
    FNO_FOLD_PROD(1, 6) FNO_FOLD_PROD(6, 1) FNO_FOLD_PROD(2, 6) FNO_FOLD_PROD(6, 2)
    FNO_FOLD_PROD(1, 12) FNO_FOLD_PROD(12, 1) FNO_FOLD_PROD(2, 12) FNO_FOLD_PROD(12, 2)
#undef FNO_FOLD_PROD
  }
  bool sh = true;
  for (int k = 0; k < t.ngroups; ++k) sh = sh && t.nshuf[k] <= kShufMax;
  static const bool trace_shapes = std::getenv("FNO_TRACE") != nullptr;
  if (trace_shapes) {
    std::fprintf(stderr, "[fno] fold shape: %d groups, %d combos, shuffles", t.ngroups, t.ncombo);
    for (int k = 0; k < t.ngroups; ++k) std::fprintf(stderr, " %d", t.nshuf[k]);
    std::fprintf(stderr, ", %lld outputs\n", (long long)total);
  }
#define FNO_FOLD_CASE(NG, NC)                                                                        \
  if (t.ngroups == NG && t.ncombo == NC) {                                                           \
    if (sh)                                                                                          \
      fold_tab_fixed_kernel<XT, NG, NC, true><<<cgrid, 256, 0, s>>>(t, X, out, alpha, total, chunk);  \
    else                                                                                             \
      fold_tab_fixed_kernel<XT, NG, NC, false><<<cgrid, 256, 0, s>>>(t, X, out, alpha, total, chunk); \
    return;                                                                                          \
  }
  // every (groups, combos) pair the ground-state and EOM tables produce:
  // up to three output groups (batch index, hole group, particle group) and
  // products of the per-group shuffle counts 1, 2, 3, 4, 6
  FNO_FOLD_CASE(1, 1) FNO_FOLD_CASE(1, 2) FNO_FOLD_CASE(1, 3) FNO_FOLD_CASE(1, 4) FNO_FOLD_CASE(1, 6)
  FNO_FOLD_CASE(2, 1) FNO_FOLD_CASE(2, 2) FNO_FOLD_CASE(2, 3) FNO_FOLD_CASE(2, 4) FNO_FOLD_CASE(2, 6)
  FNO_FOLD_CASE(2, 8) FNO_FOLD_CASE(2, 9) FNO_FOLD_CASE(2, 12) FNO_FOLD_CASE(2, 16) FNO_FOLD_CASE(2, 18)
  FNO_FOLD_CASE(2, 24) FNO_FOLD_CASE(2, 36)
  FNO_FOLD_CASE(3, 1) FNO_FOLD_CASE(3, 2) FNO_FOLD_CASE(3, 3) FNO_FOLD_CASE(3, 4) FNO_FOLD_CASE(3, 6)
  FNO_FOLD_CASE(3, 8) FNO_FOLD_CASE(3, 9) FNO_FOLD_CASE(3, 12) FNO_FOLD_CASE(3, 16) FNO_FOLD_CASE(3, 18)
  FNO_FOLD_CASE(3, 24) FNO_FOLD_CASE(3, 36)
  FNO_FOLD_CASE(4, 1) FNO_FOLD_CASE(4, 2) FNO_FOLD_CASE(4, 3) FNO_FOLD_CASE(4, 4) FNO_FOLD_CASE(4, 6)
#undef FNO_FOLD_CASE
  static bool trace = std::getenv("FNO_TRACE") != nullptr;
  if (trace) std::fprintf(stderr, "[fno] generic fold: %d groups, %d combos\n", t.ngroups, t.ncombo);
  fold_tab_kernel<XT><<<grid, 256, 0, s>>>(t, X, out, alpha, total);
}

void launch_fold_tab(const FoldTab& t, const void* X, Prec xprec, double* out, double alpha, int64_t total,
                     hipStream_t s) {
  if (total == 0) return;
  if (xprec == Prec::FP64)
    fold_launch<double>(t, (const double*)X, out, alpha, total, s);
  else
    fold_launch<float>(t, (const float*)X, out, alpha, total, s);
  FNO_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- T1 dressing
// One index of the dressed integrals g^ = (X x X) g (Y x Y), X = 1 - t1 on the
// creation indices, Y = 1 + t1 on the annihilation indices (t1[i][a] couples
// occupied i with virtual a only).  In place on g (n^4, row-major), slot
// `pos` (stride n^(3-pos)):
//   creation:     g[.., a, ..] -= sum_i t1[i][a] g[.., i, ..]   (virtual slice from the occupied one)
//   annihilation: g[.., i, ..] += sum_a t1[i][a] g[.., a, ..]   (occupied slice from the virtual one)
// Each pass reads only the slice it does not write.
__global__ void __launch_bounds__(256) dress_pass_kernel(double* __restrict__ g, const double* __restrict__ t1,
                                                         int nocc, int nvir, int64_t inner, int creation,
                                                         int64_t total) {
  const int n = nocc + nvir;
  const int ntarget = creation ? nvir : nocc;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t in = e % inner;
    const int64_t rest = e / inner;
    const int tp = (int)(rest % ntarget);
    const int64_t outer = rest / ntarget;
    const int64_t base = outer * n * inner + in;
    double acc = 0.0;
    if (creation) {
      for (int i = 0; i < nocc; ++i) acc -= t1[(int64_t)i * nvir + tp] * g[base + (int64_t)i * inner];
      g[base + (int64_t)(nocc + tp) * inner] += acc;
    } else {
      for (int a = 0; a < nvir; ++a) acc += t1[(int64_t)tp * nvir + a] * g[base + (int64_t)(nocc + a) * inner];
      g[base + (int64_t)tp * inner] += acc;
    }
  }
}

// Same update, one thread per position of the other three slots: the thread
// reads its source slice once and produces every target of the slot (the
// occupied side, at most kDressMaxOcc values, lives in registers).
constexpr int kDressMaxOcc = 32;
template <int MAXO>
__global__ void __launch_bounds__(256) dress_slice_kernel(double* __restrict__ g, const double* __restrict__ t1,
                                                          int nocc, int nvir, int64_t inner, int creation,
                                                          int64_t total) {
  const int n = nocc + nvir;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t in = e % inner;
    const int64_t outer = e / inner;
    double* base = g + outer * n * inner + in;
    double occ[MAXO];
    if (creation) {
      // g[a] -= sum_i t1[i][a] g[i]
#pragma unroll
      for (int i = 0; i < MAXO; ++i) occ[i] = i < nocc ? base[(int64_t)i * inner] : 0.0;
      // 8 virtual rows at a time: their loads are issued before any store
      for (int a0 = 0; a0 < nvir; a0 += 8) {
        double gv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) gv[u] = a0 + u < nvir ? base[(int64_t)(nocc + a0 + u) * inner] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (a0 + u >= nvir) break;
          double acc = 0.0;
#pragma unroll
          for (int i = 0; i < MAXO; ++i)
            if (i < nocc) acc += t1[(int64_t)i * nvir + a0 + u] * occ[i];
          base[(int64_t)(nocc + a0 + u) * inner] = gv[u] - acc;
        }
      }
    } else {
      // g[i] += sum_a t1[i][a] g[a]
#pragma unroll
      for (int i = 0; i < MAXO; ++i) occ[i] = 0.0;
      for (int a0 = 0; a0 < nvir; a0 += 8) {
        double gv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) gv[u] = a0 + u < nvir ? base[(int64_t)(nocc + a0 + u) * inner] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (a0 + u >= nvir) break;
#pragma unroll
          for (int i = 0; i < MAXO; ++i)
            if (i < nocc) occ[i] += t1[(int64_t)i * nvir + a0 + u] * gv[u];
        }
      }
#pragma unroll
      for (int i = 0; i < MAXO; ++i)
        if (i < nocc) base[(int64_t)i * inner] += occ[i];
    }
  }
}

// First creation slot of the dressing fused with the copy from the undressed
// integrals: Gd[i, :] = G[i, :], Gd[a, :] = G[a, :] - sum_i t1[i][a] G[i, :]
// over the first index (rows of n^3 elements), one thread per column with
// the o occupied values in registers.
template <int MAXO>
__global__ void __launch_bounds__(256) dress_first_slot_kernel(const double* __restrict__ G, double* __restrict__ Gd,
                                                               const double* __restrict__ t1, int nocc, int nvir,
                                                               int64_t n3) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n3; c += (int64_t)gridDim.x * blockDim.x) {
    double occ[MAXO];
#pragma unroll
    for (int i = 0; i < MAXO; ++i)
      if (i < nocc) {
        occ[i] = G[(int64_t)i * n3 + c];
        Gd[(int64_t)i * n3 + c] = occ[i];
      }
    for (int a = 0; a < nvir; ++a) {
      double acc = G[(int64_t)(nocc + a) * n3 + c];
#pragma unroll
      for (int i = 0; i < MAXO; ++i)
        if (i < nocc) acc -= t1[(int64_t)i * nvir + a] * occ[i];
      Gd[(int64_t)(nocc + a) * n3 + c] = acc;
    }
  }
}


bool launch_dress_first_slot(const double* G, double* Gd, const double* t1, int nocc, int nvir, hipStream_t s) {
  if (nocc > kDressMaxOcc || nocc == 0 || nvir == 0) return false;
  const int64_t n = nocc + nvir, n3 = n * n * n;
  const unsigned blocks = (unsigned)std::min<int64_t>((n3 + 255) / 256, 65536);
  if (nocc <= 8)
    dress_first_slot_kernel<8><<<blocks, 256, 0, s>>>(G, Gd, t1, nocc, nvir, n3);
  else if (nocc <= 16)
    dress_first_slot_kernel<16><<<blocks, 256, 0, s>>>(G, Gd, t1, nocc, nvir, n3);
  else
    dress_first_slot_kernel<kDressMaxOcc><<<blocks, 256, 0, s>>>(G, Gd, t1, nocc, nvir, n3);
  FNO_HIP(hipGetLastError());
  return true;
}

void launch_dress_pass(double* g, const double* t1, int nocc, int nvir, int pos, bool creation, hipStream_t s) {
  if (nocc <= kDressMaxOcc) {
    const int64_t n = nocc + nvir;
    int64_t inner = 1, outer = 1;
    for (int q = pos + 1; q < 4; ++q) inner *= n;
    for (int q = 0; q < pos; ++q) outer *= n;
    const int64_t total = outer * inner;
    if (total == 0 || nvir == 0 || nocc == 0) return;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    const int cr = creation ? 1 : 0;
    if (nocc <= 8)
      dress_slice_kernel<8><<<dim3((unsigned)blocks), 256, 0, s>>>(g, t1, nocc, nvir, inner, cr, total);
    else if (nocc <= 16)
      dress_slice_kernel<16><<<dim3((unsigned)blocks), 256, 0, s>>>(g, t1, nocc, nvir, inner, cr, total);
    else
      dress_slice_kernel<kDressMaxOcc><<<dim3((unsigned)blocks), 256, 0, s>>>(g, t1, nocc, nvir, inner, cr, total);
    FNO_HIP(hipGetLastError());
    return;
  }
  const int64_t n = nocc + nvir;
  int64_t inner = 1;
  for (int q = pos + 1; q < 4; ++q) inner *= n;
  int64_t outer = 1;
  for (int q = 0; q < pos; ++q) outer *= n;
  const int64_t total = outer * (creation ? nvir : nocc) * inner;
  if (total == 0) return;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  dress_pass_kernel<<<dim3((unsigned)blocks), 256, 0, s>>>(g, t1, nocc, nvir, inner, creation ? 1 : 0, total);
  FNO_HIP(hipGetLastError());
}

}  // namespace fno

// ---------------------------------------------------------------- learned guess (MLP)
namespace fno {
namespace mlp {

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }

// Z[r][c] += b[c]; A = silu(Z) (act != 0) or A = Z
__global__ void __launch_bounds__(256) bias_act_kernel(float* __restrict__ Z, const float* __restrict__ b,
                                                       float* __restrict__ A, int64_t rows, int cols, int act) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const float z = Z[e] + b[e % cols];
    Z[e] = z;
    A[e] = act ? z * sigm(z) : z;
  }
}

// dZ = dA * silu'(Z)
__global__ void __launch_bounds__(256) act_grad_kernel(const float* __restrict__ Z, const float* __restrict__ dA,
                                                       float* __restrict__ dZ, int64_t total) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const float s = sigm(Z[e]);
    dZ[e] = dA[e] * s * (1.0f + Z[e] * (1.0f - s));
  }
}

// column sums of a rows x cols matrix (bias gradients); one thread per column
__global__ void __launch_bounds__(256) colsum_kernel(const float* __restrict__ X, float* __restrict__ out, int64_t rows,
                                                     int cols) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int64_t r = 0; r < rows; ++r) s += X[r * cols + c];
  out[c] = s;
}

// weighted MSE: loss_part[block] partial sums of sum_o w_o (Y - T)^2 / rows, dY = 2 w (Y - T) / rows
__global__ void __launch_bounds__(256) mse_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                  const float* __restrict__ w, float* __restrict__ dY,
                                                  float* __restrict__ part, int64_t rows, int cols) {
  __shared__ float red[256];
  const int64_t total = rows * cols;
  float acc = 0.0f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[e] - T[e];
    const float wo = w[e % cols];
    acc += wo * d * d;
    dY[e] = 2.0f * wo * d / (float)rows;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] / (float)rows;
}

// Adam (bias-corrected) on a flat parameter vector
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// FP32 -> BF16 (round to nearest even), lo part zero: single-BF16 operands for
// the BF16 MFMA path
__global__ void __launch_bounds__(256) to_bf16_kernel(const float* __restrict__ x, __hip_bfloat16* __restrict__ hi,
                                                      __hip_bfloat16* __restrict__ lo, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    hi[e] = __float2bfloat16(x[e]);
    lo[e] = __float2bfloat16(0.0f);
  }
}

static int64_t nblocks(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

void bias_act(float* Z, const float* b, float* A, int64_t rows, int cols, bool act, hipStream_t s) {
  if (rows * cols == 0) return;
  bias_act_kernel<<<dim3((unsigned)nblocks(rows * cols)), 256, 0, s>>>(Z, b, A, rows, cols, act ? 1 : 0);
  FNO_HIP(hipGetLastError());
}
void act_grad(const float* Z, const float* dA, float* dZ, int64_t n, hipStream_t s) {
  if (n == 0) return;
  act_grad_kernel<<<dim3((unsigned)nblocks(n)), 256, 0, s>>>(Z, dA, dZ, n);
  FNO_HIP(hipGetLastError());
}
void colsum(const float* X, float* out, int64_t rows, int cols, hipStream_t s) {
  colsum_kernel<<<dim3((unsigned)((cols + 255) / 256)), 256, 0, s>>>(X, out, rows, cols);
  FNO_HIP(hipGetLastError());
}
int mse_blocks(int64_t n) { return (int)std::min<int64_t>(nblocks(n), 1024); }
void mse(const float* Y, const float* T, const float* w, float* dY, float* part, int64_t rows, int cols,
         hipStream_t s) {
  mse_kernel<<<dim3((unsigned)mse_blocks(rows * cols)), 256, 0, s>>>(Y, T, w, dY, part, rows, cols);
  FNO_HIP(hipGetLastError());
}
void adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps, int step,
          hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  adam_kernel<<<dim3((unsigned)nblocks(n)), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  FNO_HIP(hipGetLastError());
}
void to_bf16(const float* x, void* hi, void* lo, int64_t n, hipStream_t s) {
  if (n == 0) return;
  to_bf16_kernel<<<dim3((unsigned)nblocks(n)), 256, 0, s>>>(x, (__hip_bfloat16*)hi, (__hip_bfloat16*)lo, n);
  FNO_HIP(hipGetLastError());
}

}  // namespace mlp
}  // namespace fno

namespace fno {
namespace mlp {

// Features of T3 elements for the learned guess (one row of kFeat per element):
//   x / sx, |x| / sx, D / 10, e_i, e_j, e_k, e_a, e_b, e_c
// x the MP-style guess (two Jacobi steps from zero), D the denominator
// sum e_holes - sum e_particles, e the orbital energies (occupied then
// virtual).  With t3c the targets are (t3c - x) / sx and the dressed-diagonal
// shift (sum fo_holes - sum fv_particles) - D.  idx selects elements (null:
// row r of the output is element e0 + r of T3).
__global__ void __launch_bounds__(256) features_kernel(IndexTables tb, int nocc, int nvir, const double* __restrict__ x,
                                                       const double* __restrict__ den, const double* __restrict__ eps,
                                                       double inv_sx, const int64_t* __restrict__ idx, int64_t e0,
                                                       int64_t ns,
                                                       float* __restrict__ feat, const double* __restrict__ t3c,
                                                       const double* __restrict__ fdiag, float* __restrict__ targ) {
  const int64_t cv3 = (int64_t)nvir * (nvir - 1) * (nvir - 2) / 6;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ns; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx ? idx[r] : e0 + r;
    const int64_t h = e / cv3, p = e - h * cv3;
    const uint8_t* hh = tb.dec[3] + h * 3;
    const uint8_t* pp = tb.dec[3] + p * 3;
    const double xv = x[e], dv = den[e];
    float* f = feat + r * kFeat;
    f[0] = (float)(xv * inv_sx);
    f[1] = (float)(fabs(xv) * inv_sx);
    f[2] = (float)(dv * 0.1);
    for (int t = 0; t < 3; ++t) {
      f[3 + t] = (float)eps[hh[t]];
      f[6 + t] = (float)eps[nocc + pp[t]];
    }
    if (targ) {
      double dd = 0.0;
      for (int t = 0; t < 3; ++t) dd += fdiag[hh[t]] - fdiag[nocc + pp[t]];
      targ[r * 2 + 0] = (float)((t3c[e] - xv) * inv_sx);
      targ[r * 2 + 1] = (float)(dd - dv);
    }
  }
}

// Apply the network outputs Y (n x 2, FP32) to the guess: t3 = x + sx y0, and
// the T3 Jacobi denominator D' = D + y1 kept within [2 D, D / 2] (D < 0).
__global__ void __launch_bounds__(256) apply_guess_kernel(double* __restrict__ t3, const double* __restrict__ x,
                                                          double* __restrict__ den, const float* __restrict__ Y,
                                                          double sx, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    t3[e] = x[e] + sx * (double)Y[e * 2 + 0];
    const double d = den[e];
    const double s = d + (double)Y[e * 2 + 1];
    den[e] = fmin(fmax(s, 2.0 * d), 0.5 * d);
  }
}

// rows of X gathered by a counter-based hash of (seed, row): minibatch sampling
__global__ void __launch_bounds__(256) gather_kernel(const float* __restrict__ X, const float* __restrict__ T,
                                                     float* __restrict__ Xb, float* __restrict__ Tb, int64_t n,
                                                     int64_t rows, uint64_t seed) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + (uint64_t)r * 0xBF58476D1CE4E5B9ull + 0x94D049BB133111EBull;
    z ^= z >> 31;
    z *= 0xD6E8FEB86659FD93ull;
    z ^= z >> 29;
    const int64_t src = (int64_t)(z % (uint64_t)n);
    for (int c = 0; c < kFeat; ++c) Xb[r * kFeat + c] = X[src * kFeat + c];
    Tb[r * 2 + 0] = T[src * 2 + 0];
    Tb[r * 2 + 1] = T[src * 2 + 1];
  }
}

void features(const IndexTables& tb, int nocc, int nvir, const double* x, const double* den, const double* eps,
              double sx, const int64_t* idx, int64_t e0, int64_t ns, float* feat, const double* t3c,
              const double* fdiag, float* targ, hipStream_t s) {
  if (ns == 0) return;
  features_kernel<<<dim3((unsigned)nblocks(ns)), 256, 0, s>>>(tb, nocc, nvir, x, den, eps, 1.0 / sx, idx, e0, ns,
                                                              feat, t3c, fdiag, targ);
  FNO_HIP(hipGetLastError());
}
void apply_guess(double* t3, const double* x, double* den, const float* Y, double sx, int64_t n, hipStream_t s) {
  if (n == 0) return;
  apply_guess_kernel<<<dim3((unsigned)nblocks(n)), 256, 0, s>>>(t3, x, den, Y, sx, n);
  FNO_HIP(hipGetLastError());
}
void gather(const float* X, const float* T, float* Xb, float* Tb, int64_t n, int64_t rows, uint64_t seed,
            hipStream_t s) {
  gather_kernel<<<dim3((unsigned)nblocks(rows)), 256, 0, s>>>(X, T, Xb, Tb, n, rows, seed);
  FNO_HIP(hipGetLastError());
}

}  // namespace mlp
}  // namespace fno
