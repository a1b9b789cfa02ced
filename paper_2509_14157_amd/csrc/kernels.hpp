// Host-side launchers of the device kernels.
#pragma once

#include <string>

#include "layout.hpp"

namespace fno {

void launch_expand(const IndexTables& tb, const OperandDesc& op, const MatDim& rows, const MatDim& cols,
                   const double* src, void* dst, void* dst_lo, Prec prec, bool col_fast, hipStream_t s);
void launch_fold(const IndexTables& tb, const OperandDesc& outd, const MatDim& outdims, const MatDim& xrows,
                 const MatDim& xcols, const FoldCombos& fc, const void* X, Prec xprec, double* out, double alpha,
                 hipStream_t s);
void launch_fill(double* x, double v, int64_t n, hipStream_t s);
// ptrs[i][0 .. ns[i]) = 0 for every i, in as few launches as possible
void launch_zero_many(double* const* ptrs, const int64_t* ns, int count, hipStream_t s);

// table construction (run once per plan)
// off[i], sign[i] for i < dims.size: contribution of the operand groups set in
// group_mask, for letter values decoded from index i of `dims`.
void launch_dim_table(const IndexTables& tb, const OperandDesc& op, const MatDim& dims, unsigned group_mask,
                      int64_t* off, int8_t* sign, hipStream_t s);
// sub[i] = mixed-radix index of the DimGroups of `dims` selected by dg_mask.
void launch_sub_index(const IndexTables& tb, const MatDim& dims, unsigned dg_mask, int32_t* sub, hipStream_t s);
// tab[rs * part_c.size + cs]: contribution of operand group `grp` for the
// letters of row part rs and column part cs.
void launch_mixed_table(const IndexTables& tb, const OperandDesc& op, int grp, const MatDim& part_r,
                        const MatDim& part_c, int64_t* off, int8_t* sign, hipStream_t s);
// fold tables of one output group: for each shuffle (src letters) and tuple u.
void launch_fold_table(const IndexTables& tb, const DimGroup& og, int nshuf, const int8_t* shuf_src, int nletters,
                       const MatDim& xrows, const MatDim& xcols, unsigned xr_mask, unsigned xc_mask,
                       int64_t* rowc, int64_t* colc, hipStream_t s);

// out[i] += alpha * element i of the expansion (an M x 1 gather), FP64
void launch_expand_tab_acc(const ExpandTab& t, const double* src, double* out, double alpha, hipStream_t s);
void launch_expand_tab(const ExpandTab& t, const double* src, void* dst, void* dst_lo, Prec prec, hipStream_t s);
void launch_fold_tab(const FoldTab& t, const void* X, Prec xprec, double* out, double alpha, int64_t total,
                     hipStream_t s);
// One slot of the T1 similarity transform of the integrals, in place (see kernels.hip).
void launch_dress_pass(double* g, const double* t1, int nocc, int nvir, int pos, bool creation, hipStream_t s);
// Gd = G with the first creation slot dressed (one streaming pass); false
// (nothing launched) for more than 32 occupied orbitals
bool launch_dress_first_slot(const double* G, double* Gd, const double* t1, int nocc, int nvir, hipStream_t s);
// y_j = a * x_j for j < count, y_j = 0 for count <= j < rows (n elements each; y_j = y + j*ldy, x_j = x + j*ldx)
void launch_scale_rows(double* y, int64_t ldy, const double* x, int64_t ldx, double a, int64_t n, int count, int rows,
                       hipStream_t s);
void launch_axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t s);
void launch_denominators(const IndexTables& tb, const MatDim& dims, int nh, const double* eo, const double* ev,
                         double* out, hipStream_t s);
void launch_jacobi(double* t, const double* r, const double* d, double* step, int64_t n, hipStream_t s);
void launch_precond(double* y, const double* x, const double* d, double shift, int64_t n, hipStream_t s);
int dot_partial_blocks(int64_t n);
// out[0] = alpha * (x . y) + beta * out[0] over n contiguous elements
// (partial needs dot_partial_blocks(n) doubles); deterministic.
void launch_dot_acc(const double* x, const double* y, int64_t n, double* partial, double* out, double alpha,
                    double beta, hipStream_t s);
void launch_dots(const double* xs, int64_t ldx, int nvec, const double* y, int64_t n, double* partial, double* out,
                 hipStream_t s);
// A Jacobi step with its DIIS bookkeeping in one pass over n elements:
// e = r / d, t_next = t + e, es[slot] = e, *out_rr = |r|^2 and
// out_ov[k] = <es[k] | e> for k < nk (es[k] = es + k * ld with ld even and
// >= n, nk <= 16; nk = 0: no history).  Every array 16-byte aligned.
// partial needs diis_step_partials(nk) doubles; deterministic.
int diis_step_partials(int nk);
void launch_diis_step(const double* t, const double* r, const double* d, double* t_next, double* es, int64_t ld,
                      int slot, int nk, int64_t n, double* partial, double* out_rr, double* out_ov, hipStream_t s);
// *out = CC correlation energy from f (n x n), g (n^4), t1 (o x v) and packed
// t2 (see kernels.hip); partial needs 256 doubles
void launch_cc_energy(const double* f, const double* g, const double* t1, const double* t2, int o, int v,
                      double* partial, double* out, hipStream_t s);
// History slots of a DIIS step, oldest first.
struct DiisSlots {
  int k = 0;
  int slot[16] = {};
};
// The DIIS overlap update and coefficient solve on the device (kernels.hip).
void launch_diis(double* B, const double* ov, int slot, const DiisSlots& ord, bool extrap, int nc, double* coef,
                 hipStream_t s);
void launch_combine(double* y, const double* xs, int64_t ldx, const double* c, int nvec, double alpha, double beta,
                    int64_t n, hipStream_t s);

// C[M x N] (row-major, ldc) = alpha * A * B + beta * C.
//   a_kfast: A element (m, k) at A[m * lda + k]  (else A[k * lda + m])
//   b_nfast: B element (k, n) at B[k * ldb + n]  (else B[n * ldb + k])
// FP64 and FP32 operands use the 16x16x4 MFMA of their type; BF16X3 takes
// hi/lo operand pairs and accumulates hi*hi + hi*lo + lo*hi in FP32.
struct GemmArgs {
  Prec prec;
  int64_t M, N, K;
  const void* A;
  const void* A_lo;
  int64_t lda;
  bool a_kfast;
  const void* B;
  const void* B_lo;
  int64_t ldb;
  bool b_nfast;
  void* C;
  int64_t ldc;
  double alpha, beta;
  int tile;   // tile configuration index (autotuner), -1 = default
  // split-K: the K range is cut into `split` chunks whose partial products go
  // to `ws` (split * M * N elements of the accumulator type) and are summed
  // in a fixed order by a second kernel (deterministic)
  int split = 1;
  void* ws = nullptr;
};
// Number of K chunks worth using for this shape (1 = no split, at most
// kMaxSplit) and the workspace bytes it needs.
constexpr int kMaxSplit = 1024;
int gemm_split_factor(const GemmArgs& g);
size_t gemm_split_bytes(const GemmArgs& g, int split);
void launch_gemm(const GemmArgs& g, hipStream_t s);
// Name of the kernel instantiation launch_gemm would use (as tools demangle it).
std::string gemm_label(const GemmArgs& g);
int gemm_num_tiles(Prec p);
int gemm_default_tile(const GemmArgs& g);  // the tile launch_gemm uses for tile = -1
int64_t gemm_tiles(const GemmArgs& g);      // workgroups launch_gemm runs for g (split-K slices included)
// Grouped GEMMs: the GEMMs of `gs` (independent: no output read by another)
// in one persistent launch per kernel instantiation, each workgroup taking
// tiles of any of them from a device work queue.  Every GEMM runs with its
// default tile, split into g.split K slices when g.split > 1 and g.ws holds
// their partial products (summed afterwards in a fixed order), and gives the
// bits launch_gemm gives with those settings (split-BF16 and the non-default
// tiles run one by one).
// pin: pinned host table and dev: device table of gs.size() items of
// gemm_group_item_bytes() each (the host table must stay unchanged until the
// stream has passed the launch); queue: gemm_group_max_launches() 8-byte
// counters.
size_t gemm_group_item_bytes();
int gemm_group_max_launches();
void launch_gemm_grouped(const std::vector<GemmArgs>& gs, void* pin, void* dev, void* queue, hipStream_t s);


// ---- learned guess: MLP building blocks (FP32) and T3 feature / guess kernels
namespace mlp {
constexpr int kFeat = 9;  // features per T3 element
void bias_act(float* Z, const float* b, float* A, int64_t rows, int cols, bool act, hipStream_t s);
void act_grad(const float* Z, const float* dA, float* dZ, int64_t n, hipStream_t s);
void colsum(const float* X, float* out, int64_t rows, int cols, hipStream_t s);
int mse_blocks(int64_t n);
void mse(const float* Y, const float* T, const float* w, float* dY, float* part, int64_t rows, int cols,
         hipStream_t s);
void adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps, int step,
          hipStream_t s);
void to_bf16(const float* x, void* hi, void* lo, int64_t n, hipStream_t s);
void features(const IndexTables& tb, int nocc, int nvir, const double* x, const double* den, const double* eps,
              double sx, const int64_t* idx, int64_t e0, int64_t ns, float* feat, const double* t3c,
              const double* fdiag, float* targ, hipStream_t s);
void apply_guess(double* t3, const double* x, double* den, const float* Y, double sx, int64_t n, hipStream_t s);
void gather(const float* X, const float* T, float* Xb, float* Tb, int64_t n, int64_t rows, uint64_t seed,
            hipStream_t s);
}  // namespace mlp

}  // namespace fno
