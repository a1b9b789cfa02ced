// EOM-CCSDT sigma vectors and block Davidson (IP, DIP, EA, DEA).
#include "eom_space.hpp"

namespace fno {


size_t Context::eom_size(int) { throw Error(kEINVAL, "EOM not available in this build"); }
void Context::eom_sigma(int, Prec, const double*, double*, size_t) {
  throw Error(kEINVAL, "EOM not available in this build");
}
int Context::eom(int, const EOMOptions&, EOMResult&) { throw Error(kEINVAL, "EOM not available in this build"); }
void Context::setup_eom(int) {}

}  // namespace fno
