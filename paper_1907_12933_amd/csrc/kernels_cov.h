// Launch interface of the coverage kernels.
#pragma once

#include "ibmc_internal.h"

namespace ibmc {
}  // namespace ibmc
