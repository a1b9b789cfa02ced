// Packed antisymmetric tensor layouts and the kernel-side descriptors.
//
// Every tensor is a sequence of index groups stored row-major (last group
// fastest).  A group of g > 1 slots holds strictly increasing index tuples
// (the tensor is antisymmetric in those slots) in colexicographic order:
// tuple x0 < x1 < ... < x{g-1} sits at sum_t C(x_t, t+1).  Colex order is
// prefix-stable, so one decode table per g serves every range size.
// A group of one slot may be a view [off, off+n) of a larger dimension.
#pragma once

#include "common.hpp"

namespace fno {

// ---- device constant tables ----------------------------------------------
struct IndexTables {
  const uint32_t* binom;   // binom[n * (kMaxGroup + 1) + k], n < kBinomN
  const uint8_t* dec[kMaxGroup + 1];  // dec[g][idx * g + t]: colex tuples of size g
  int dec_max_n[kMaxGroup + 1];       // largest n the table covers
};

// One storage group of an operand seen through the letters of a term.
struct GroupDesc {
  int g;                       // slots in the group
  int off;                     // index offset (single-slot views)
  int64_t stride;              // element stride of the group
  int8_t letter[kMaxGroup];    // term letter of each slot, storage order
};

struct OperandDesc {
  int ngroups;
  int64_t base;                // element offset of the view origin
  GroupDesc grp[kMaxGroups];
};

// One packed group of a GEMM matrix dimension (rows or columns).
struct DimGroup {
  int g;
  int n;
  int64_t count;               // C(n, g) (or n when g == 1)
  int8_t letter[kMaxGroup];    // letters in ascending-value order
};

struct MatDim {
  int ngroups;
  int64_t size;
  DimGroup grp[kMaxGroups];
};

constexpr int kMaxLetters = 16;
constexpr int kMaxCombos = 48;

// Antisymmetrizer of a fold: for each coset representative, the letter whose
// output value each letter takes, and its sign.
struct FoldCombos {
  int ncombo;
  int nletters;
  int8_t src[kMaxCombos][kMaxLetters];
  int8_t sign[kMaxCombos];
};

// Table-driven operand expansion: offset(r, c) = row_off[r] + col_off[c]
// + sum_m tab_m[row_sub_m[r] * ncsub_m + col_sub_m[c]], and the product of
// the matching signs (0 marks a repeated index of an antisymmetric group).
constexpr int kMaxMixed = 2;
struct ExpandTab {
  int64_t rows, cols;
  int64_t ld;  // destination row stride (elements, >= cols) of the row kernel
  const int64_t* row_off;
  const int8_t* row_sign;
  const int64_t* col_off;
  const int8_t* col_sign;
  int nmixed;
  int64_t ncsub[kMaxMixed];
  const int32_t* row_sub[kMaxMixed];
  const int32_t* col_sub[kMaxMixed];
  const int64_t* tab_off[kMaxMixed];
  const int8_t* tab_sign[kMaxMixed];
};

// Table-driven fold over a whole packed output: element e = mixed-radix
// tuple indices u_k of the output groups; each coset representative c picks
// one shuffle s_k per group; X row/col = sum_k rowc_k[s_k][u_k] / colc_k.
constexpr int kMaxOutGroups = 4;
struct FoldTab {
  int ngroups;
  int64_t count[kMaxOutGroups];     // tuples per output group
  int nshuf[kMaxOutGroups];
  const int64_t* rowc[kMaxOutGroups];   // [s * count + u]
  const int64_t* colc[kMaxOutGroups];
  int ncombo;
  int8_t combo[kMaxCombos][kMaxOutGroups];  // shuffle index per group
  int8_t csign[kMaxCombos];                 // sign of the coset representative
  int64_t xcols;
};

#ifdef __HIPCC__
__device__ __forceinline__ int64_t colex_encode(const IndexTables& tb, const int* x, int g) {
  int64_t r = 0;
  for (int t = 0; t < g; ++t) r += tb.binom[x[t] * (kMaxGroup + 1) + (t + 1)];
  return r;
}

__device__ __forceinline__ void colex_decode(const IndexTables& tb, int64_t idx, int g, int* x) {
  if (g == 1) {
    x[0] = (int)idx;
    return;
  }
  const uint8_t* p = tb.dec[g] + idx * g;
  for (int t = 0; t < g; ++t) x[t] = p[t];
}

// Decode a row/column index of a matrix dimension into letter values.
__device__ __forceinline__ void decode_dim(const IndexTables& tb, const MatDim& d, int64_t idx, int* val) {
  for (int q = d.ngroups - 1; q >= 0; --q) {
    const DimGroup& G = d.grp[q];
    int64_t t = idx % G.count;
    idx /= G.count;
    int x[kMaxGroup];
    colex_decode(tb, t, G.g, x);
    for (int s = 0; s < G.g; ++s) val[G.letter[s]] = x[s];
  }
}

// Element offset and sign of an operand entry for the given letter values;
// sign 0 when two antisymmetric slots coincide.
__device__ __forceinline__ int64_t operand_offset(const IndexTables& tb, const OperandDesc& op, const int* val,
                                                  int* sign_out) {
  int64_t off = op.base;
  int sign = 1;
  for (int q = 0; q < op.ngroups; ++q) {
    const GroupDesc& G = op.grp[q];
    if (G.g == 1) {
      off += (int64_t)(val[G.letter[0]] + G.off) * G.stride;
      continue;
    }
    int x[kMaxGroup];
    for (int s = 0; s < G.g; ++s) x[s] = val[G.letter[s]];
    // insertion sort with parity
    for (int a = 1; a < G.g; ++a) {
      int v = x[a];
      int b = a - 1;
      while (b >= 0 && x[b] > v) {
        x[b + 1] = x[b];
        --b;
        sign = -sign;
      }
      x[b + 1] = v;
    }
    for (int a = 1; a < G.g; ++a)
      if (x[a] == x[a - 1]) sign = 0;
    off += colex_encode(tb, x, G.g) * G.stride;
  }
  *sign_out = sign;
  return off;
}
#endif

}  // namespace fno
