// Persistent schedule: placeholder until the cooperative kernel lands.
#pragma once

#include "msl_passes.hpp"

namespace msl {

inline bool persistent_preferred(const Ctx&, int) { return false; }

inline hipError_t launch_persistent(const Ctx&, const PhaseSpec&, int, unsigned*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace msl
