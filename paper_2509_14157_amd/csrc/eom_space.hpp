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
};

struct Context::EomSpace {
  int kind = 0;
  EomTables tab{};
  std::vector<Block> blocks;   // (nh, np), packed sizes and offsets in the R vector
  int64_t dim = 0;
  double* diag = nullptr;      // zeroth-order diagonal sum e_particles - sum e_holes
  bool ready = false;
};

}  // namespace fno
