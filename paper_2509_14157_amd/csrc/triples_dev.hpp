// Host helpers shared by the context-free fused triples entry points.
#pragma once

#include <string>

#include "../../include/fnocc.h"
#include "triples.hpp"

namespace fno {

constexpr int kDevMaxDevices = 64;

// byte offsets of the working buffers (T3v, W3_vvvv^T, Y, ring operand,
// padded F3_vv, occupied operator) in one scratch block, 256-byte aligned
struct Layout {
  size_t t3v, wt, y, aring, fvvp, occ, total;
};
Layout layout(int o, int v, Prec p);

struct Inputs {
  const double *T3, *T2, *Wvvvv, *Fvv, *Wovvo, *Wvvvo, *Wovoo, *Woooo, *Foo;
};

// argument checks shared by the entry points; returns the product precision
Prec check_args(int device, int o, int v, fno_prec prec, const Inputs& in, const double* R3);
// the device's decode tables (static device arrays, filled at the first call
// on that device, with that device current)
IndexTables dev_tables(int device);
// R3 += the fused triples terms, with the working buffers in `base`
void run_pass(const IndexTables& tb, int o, int v, Prec prec, const Inputs& in, double* R3, unsigned char* base,
              hipStream_t s);

extern thread_local std::string g_dev_err;

template <typename F>
int dev_guard(F&& f) {
  try {
    g_dev_err.clear();
    return f();
  } catch (const Error& e) {
    g_dev_err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_dev_err = e.what();
    return kEDEVICE;
  }
}

}  // namespace fno
