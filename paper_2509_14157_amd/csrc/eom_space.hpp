// State of one EOM variant (R-space layout, Davidson storage).
#pragma once
#include "context.hpp"

namespace fno {
struct Context::EomSpace {
  int kind = 0;
};
}  // namespace fno
