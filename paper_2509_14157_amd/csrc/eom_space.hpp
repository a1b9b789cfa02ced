// State of one EOM variant: R-space layout, tensors of the sigma terms, Davidson storage.
#pragma once
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

struct Context::EomSpace {
  int kind = 0;
  EomTables tab{};
  std::vector<Block> blocks;   // (nh, np), packed sizes and offsets in the R vector
  int64_t dim = 0;
  double* diag = nullptr;      // zeroth-order diagonal sum e_particles - sum e_holes
  std::vector<std::string> created;  // engine tensors owned by this variant
  bool ready = false;
};

}  // namespace fno
