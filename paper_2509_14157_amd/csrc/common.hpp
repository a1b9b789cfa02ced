// Shared definitions of the FNO-EOM-CCSDT GPU library (gfx950 / MI355X).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace fno {

// Library error carrying one of the public status codes.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

enum Status {
  kOK = 0,
  kEINVAL = -1,
  kENOMEM = -2,
  kEDEVICE = -3,
  kENOCONV = -4,
  kENONFINITE = -5,
  kESTATE = -6,
};

#define FNO_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::fno::Error(e_ == hipErrorOutOfMemory ? ::fno::kENOMEM : ::fno::kEDEVICE, \
                         std::string(#call) + ": " + hipGetErrorString(e_));           \
    } while (0)

#define FNO_REQUIRE(cond, code, msg)                                  \
  do {                                                                \
    if (!(cond)) throw ::fno::Error((code), std::string(msg));        \
  } while (0)

// Largest supported ranks of one antisymmetric index group, and of a tensor.
constexpr int kMaxGroup = 4;
constexpr int kMaxSlots = 8;
constexpr int kMaxGroups = 8;
constexpr int kBinomN = 257;   // binomial table covers C(n, k) for n < kBinomN, k <= kMaxGroup

// Host binomial coefficient (exact in 64 bits for the sizes used here).
inline uint64_t binom_host(int n, int k) {
  if (k < 0 || n < k) return 0;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}

enum class Prec : int { FP64 = 0, FP32 = 1, BF16X3 = 2 };

}  // namespace fno
