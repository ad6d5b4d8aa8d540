// Launch interface of the proposal-network kernels.
#pragma once

#include "ibmc_internal.h"

namespace ibmc {
}  // namespace ibmc
