// Fused triples residual of the CCSDT amplitude equations (eq 5 projected
// on the triples, the connected form used in cc.cpp), one occupied triple at
// a time.
//
// For a sorted occupied triple t = (t0 < t1 < t2) every R3 term of the
// T1-dressed CCSDT equations is either
//   * an occupied-only operator on packed T3 rows (hh-ladder, F_oo term):
//       R3[t, :] += sum_t' C[t, t'] T3[t', :]       (C: C(o,3) x C(o,3)), or
//   * antisymmetric in the three virtual letters through P(a/bc) of a
//     product Y_t[a, bc] (b < c) in which the occupied antisymmetrizer is a
//     sum over the three placements x = t_p, pair = t \ {t_p}, sign (-1)^p:
//       Y_t[a, bc] =  sum_{e<f} T3[t, aef] W3_vvvv[bc, ef]                 (pp-ladder)
//                   + sum_e F3_vv[a, e] T3[t, ebc]                          (one-body)
//                   + sum_p (-1)^p sum_{m,e} W3_ovvo[m a e x] T3[m pair, e b c]  (ring)
//                   + sum_p (-1)^p sum_e T2[pair, a e] W3_vvvo[x e, bc]     (driver)
//                   - sum_p (-1)^p sum_m W3_ovoo[m a, pair] T2[x m, bc]     (driver)
//     and   R3[t, abc] += Y_t[a, bc] - Y_t[b, ac] + Y_t[c, ab].
// The second form is one MFMA GEMM per triple, A (v x K) times B (K x C(v,2))
// with K the concatenation of the five sums (the occupied placements enter as
// K segments, so rows with the summed occupied letter inside the pair are
// skipped instead of computed and discarded).  T3 and T2 are gathered from
// packed storage straight into the GEMM's LDS tiles; no expanded operand and
// no per-term product is written.
#pragma once

#include "layout.hpp"

namespace fno {

struct R3FusedArgs {
  int o = 0, v = 0;
  const double* T3 = nullptr;     // [C(o,3)][C(v,3)] packed, colex
  // T3 with its first virtual letter unpacked, [C(o,3)][v (x)][ldy (pair p<q)]
  // = T3[t, x p q] (zero where x is in the pair and in the row padding), and
  // W3_vvvv transposed, [C(v,2) (ef)][ldy (bc)]; both in the compute type
  void* T3v = nullptr;
  void* WT = nullptr;
  const double* T2 = nullptr;     // [C(o,2)][C(v,2)]
  const double* Wvvvv = nullptr;  // W3_vvvv [C(v,2) (bc)][C(v,2) (ef)]
  const double* Fvvp = nullptr;   // F3_vv [64 (a)][ep (e)], zero outside a, e < v
  const double* Aring = nullptr;  // W3_ovvo rearranged: [x][a][m][e < ep] = W3_ovvo[m][a][e][x], ep = v rounded up to 16
  const double* Wvvvo = nullptr;  // W3_vvvo [o (k)][v (e)][C(v,2) (bc)]
  const double* Wovoo = nullptr;  // W3_ovoo [o (m)][v (c)][C(o,2) (jk)]
  void* Y = nullptr;              // [C(o,3)][v][ldy] in the accumulator type of the precision
  int64_t ldy = 0;
};

// Elements of the accumulator Y and of T3v (per element: 8 bytes FP64, 4
// bytes FP32 / split-BF16), of WT, and the padded row length of all three.
int64_t r3_fused_y_elems(int o, int v);
int64_t r3_fused_t3v_elems(int o, int v);  // with the padding the fused kernel reads
int64_t r3_fused_wt_elems(int v);
int64_t r3_fused_ldy(int v);
int64_t r3_fvv_padded_elems(int v);
// T3v and WT (above) from T3 and W3_vvvv, in the compute type of prec,
// together or one at a time
void launch_r3_t3v(const IndexTables& tb, int o, int v, const double* T3, void* T3v, Prec prec, hipStream_t s);
void launch_r3_wt(int v, const double* Wvvvv, void* WT, Prec prec, hipStream_t s);
void launch_r3_operands(const IndexTables& tb, int o, int v, const double* T3, const double* Wvvvv, void* T3v,
                        void* WT, Prec prec, hipStream_t s);
// Y = the products above for every triple (all of Y is written).
void launch_r3_fused(const IndexTables& tb, const R3FusedArgs& a, Prec prec, hipStream_t s);
// R3[t, abc] += Y_t[a, bc] - Y_t[b, ac] + Y_t[c, ab]
void launch_r3_fold(const IndexTables& tb, int o, int v, const void* Y, int64_t ldy, Prec prec, double* R3,
                    hipStream_t s);
// Aring[x][a][m][e] = W3_ovvo[m][a][e][x] (zero rows pad e to a multiple of
// 16; zero rows a >= v after the last x) and Fvvp from F3_vv
int64_t r3_ring_operand_elems(int o, int v);
void launch_r3_ring_operand(const double* Wovvo, const double* Fvv, int o, int v, double* Aring, double* Fvvp,
                            hipStream_t s);
// C[t][t'] of the occupied-only terms from W3_oooo [C(o,2) (mn)][C(o,2) (ij)] and F3_oo [o (m)][o (i)]
void launch_r3_occ_operator(const IndexTables& tb, int o, const double* Woooo, const double* Foo, double* C,
                            hipStream_t s);
// Flops the fused GEMM executes per call (MFMA work on its padded tiles).
double r3_fused_executed_flops(int o, int v);

}  // namespace fno
