// The T3 terms of the CCSDT equations (eq 5) outside the triples residual,
// computed from T3v, the triples residual's operand (T3 with its first
// virtual letter unpacked, triples.hpp), instead of from expanded copies of
// T3.  With T1-dressed integrals <pq||rs> (the views of Gd) and F = F_ov:
//   W3_vvvo[k][e][bc] -= sum_{m<n} sum_f T3[m n k, f b c] <mn||fe>
//   W3_ovoo[m][c][jk] -= sum_n sum_{e<f} <mn||ef> T3[j k n, c e f]
//   R1[i][a]          += sum_{m<n} sum_{e<f} <mn||ef> T3[i m n, a e f]
//   R2[ij][ab]        += sum_m sum_e F[m][e] T3[i j m, a b e]
//                      + P(ab) sum_m sum_{e<f} T3[i j m, a e f] <bm||ef>
//                      - P(ij) sum_{m<n} sum_e <mn||je> T3[i m n, a b e]
// For a sorted occupied triple t and the placement p of one of its letters
// (x = t_p, pair = the other two), T3 with x moved to the front of its
// occupied slots is (-1)^p T3[t], so each term is a sum over triples and
// placements of products of T3v rows T3v[t][x][:] with integral rows:
//   NT products  S_t[r][c] = sum_{e<f} A_r[ef] T3v[t][c][ef] with the rows
//     A_r = <mn||ef> (every pair mn) and <b t_p||ef> (b < v, each placement)
//     (R1, W3_ovoo and the P(ab) term of R2);
//   NN products  sum_e A[r][e] T3v[t][e][bc]: per k summed over the triples
//     that hold k (A = <mn||fe>, W3_vvvo), and per triple with the rows
//     <pair_p||j e> and F[t_p][e] of each placement (the F and P(ij) terms
//     of R2).
// Every product is an FP64 MFMA GEMM on 16-byte row loads; the sums over
// triples and placements are gathers, one output element per thread.
#pragma once

#include "layout.hpp"

namespace fno {

struct SideShape {
  int o = 0, v = 0, n = 0;
  int no2 = 0, nt = 0, nv2 = 0;
  int64_t ldy = 0;  // padded row length of T3v
  int ep = 0;       // v rounded up to 16
  int nto = 0;      // 64-row tiles of the <mn||ef> rows
  int mts = 0;      // 64-row tiles of the NT products per triple (nto + 3)
  int rows2 = 0;    // rows of the per-triple NN products, 3 (o + 1)
  int mt2 = 0;      // their 64-row tiles
  int nchunk = 0;   // pairs mn outside one k, C(o-1, 2)
  int nsplit = 0;   // groups of those pairs (W3_vvvo partial sums)
  int ntn = 0;      // 128-column tiles of a T3v row
  // element offsets (doubles) in one buffer, each 32-element aligned
  int64_t goP = 0, gvP = 0, gx = 0, a2 = 0, s = 0, o2 = 0, wp = 0, total = 0;
};

// Shapes and buffer layout for o occupied and v virtual spin-orbitals;
// valid for 3 <= o, 3 <= v <= 64 and 3 (o + 1) <= 64 * 8.
SideShape side_shape(int o, int v);

// Integral rows of the products, from the dressed integrals Gd [n][n][n][n]
// and Fock matrix Fd [n][n] (n = o + v, occupied first).
void launch_side_operands(const IndexTables& tb, const SideShape& sh, const double* Gd, const double* Fd,
                          double* buf, hipStream_t s);
// The NT and NN products from the FP64 T3v.
void launch_side_products(const IndexTables& tb, const SideShape& sh, const double* T3v, double* buf,
                          hipStream_t s);
// W3_vvvo ("o,v,vv") and W3_ovoo ("o,v,oo") T3 pieces from the products.
void launch_side_w3(const IndexTables& tb, const SideShape& sh, const double* buf, double* W3vvvo, double* W3ovoo,
                    hipStream_t s);
// R1 ("o,v") and R2 ("oo,vv") T3 terms from the products.
void launch_side_r12(const IndexTables& tb, const SideShape& sh, const double* buf, double* R1, double* R2,
                     hipStream_t s);
// Flops the product kernels execute per call (MFMA work on their padded tiles).
double side_executed_flops(const SideShape& sh);

}  // namespace fno
