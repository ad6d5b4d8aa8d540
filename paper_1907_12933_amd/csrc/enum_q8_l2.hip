// Enumeration kernel instances: two weight layers (one hidden layer).
#include "enum_q8_impl.h"

namespace ibmc {

static const EnumVariant kL2[] = {
    IBMC_VAR_LDS(2, 1, 0, 1), IBMC_VAR_LDS(2, 1, 0, 2), IBMC_VAR_LDS(2, 1, 0, 4),
    IBMC_VAR_LDS(2, 2, 0, 1), IBMC_VAR_LDS(2, 2, 0, 2), IBMC_VAR_LDS(2, 2, 0, 4),
    IBMC_VAR_LDS(2, 4, 0, 1), IBMC_VAR_LDS(2, 4, 0, 2), IBMC_VAR_LDS(2, 4, 0, 4),
    IBMC_VAR_LDS(2, 8, 0, 1), IBMC_VAR_LDS(2, 8, 0, 2),
    IBMC_VAR_L2(2, 16, 0, 1),
};

const EnumVariant *enum_variants_l2(int *count) {
    *count = (int)(sizeof(kL2) / sizeof(kL2[0]));
    return kL2;
}

}  // namespace ibmc
