// State of one EOM variant: R-space layout, tensors of the sigma terms, Davidson storage.
#pragma once
#include <cmath>
#include <string>
#include <vector>

#include "context.hpp"

namespace fno {

struct EomTables {
  const char* const* decl;
  int ndecl;
  const char* const* views;
  int nviews;
  const int (*blocks)[2];
  const int* sign;
  const char* const* in;
  const char* const* out;
  int nblocks;
  const char* const* zero;
  int nzero;
  const char* const* terms;
  int nterms;
  const char* const* prim_decl;  // T-only intermediates (DIP, DEA): built once per amplitudes
  int nprim_decl;
  const char* const* prep;
  int nprep;
};

// Graph state of one sigma program (right- or left-hand).
struct SigmaGraph {
  Program prog;
  bool stable = false;
  uint64_t stable_epoch = 0;
  int stable_prec = -1;
  bool stable_profiled = false;
  std::string stable_filter;
};

struct Context::EomSpace {
  int kind = 0;
  EomTables tab{};
  EomTables ltab{};            // the left-hand (transposed) program; shares views and T-only intermediates
  bool left_made = false;      // its adjoint tensors exist
  std::vector<Block> blocks;   // (nh, np), packed sizes and offsets in the R vector
  int64_t dim = 0;
  int nb = 1;                  // vectors per sigma evaluation (batch slot of every R-derived tensor)
  double* diag = nullptr;      // zeroth-order diagonal sum e_particles - sum e_holes
  std::vector<std::string> created;  // engine tensors owned by this variant
  bool ready = false;
  // the sigma sweeps (zeroing + terms) replayed from hipGraphs once a
  // host-launched sweep allocated nothing (same rules as the CC residual)
  SigmaGraph rg, lg;
  double sweep_tri = 0, sweep_all = 0;  // algorithmic flops of one sweep
};

// State of one resumable Davidson solve (eom.cpp).
struct Context::Davidson {
  int kind = 0;
  EOMOptions opt;
  int64_t dim = 0;
  int nroots = 0, max_sub = 0;
  // V: orthonormal basis, S: its sigma vectors, X: Ritz vectors, T: residuals
  // and staging (2 * nroots vectors); small device matrices: gres (products
  // of vector blocks), cm (combination coefficients), gws (split-K partials)
  double *V = nullptr, *S = nullptr, *X = nullptr, *T = nullptr, *gres = nullptr, *cm = nullptr, *gws = nullptr;
  size_t gws_bytes = 0;
  int nv = 0, ns = 0, it = 0, status = kENOCONV;
  int gn = 0;  // G = V^T S is valid for the first gn basis vectors
  bool done = false, trace = false;
  std::vector<double> G, theta, theta_imag, theta_old, rn;
  std::vector<std::vector<double>> yold;  // previous iteration's Ritz coefficients
};

}  // namespace fno
