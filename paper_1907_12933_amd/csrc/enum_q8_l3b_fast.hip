// Enumeration kernel instances: three weight layers, wide hidden layers.
#include "enum_q8_impl.h"

namespace ibmc {

static const EnumVariant kL3bF[] = {
    IBMC_VAR_LDS_F(3, 4, 4, 1), IBMC_VAR_LDS_F(3, 4, 4, 2), IBMC_VAR_LDS_F(3, 4, 4, 4),
    IBMC_VAR_L2_F(3, 4, 4, 1), IBMC_VAR_L2_F(3, 4, 4, 2),
    IBMC_VAR_L2_F(3, 8, 4, 1), IBMC_VAR_L2_F(3, 4, 8, 1), IBMC_VAR_L2_F(3, 8, 8, 1), IBMC_VAR_L2_F(3, 8, 8, 2),
    IBMC_VAR_L2_F(3, 1, 8, 1), IBMC_VAR_L2_F(3, 2, 8, 1), IBMC_VAR_L2_F(3, 8, 1, 1), IBMC_VAR_L2_F(3, 8, 2, 1),
};

const EnumVariant *enum_variants_l3b_fast(int *count) {
    *count = (int)(sizeof(kL3bF) / sizeof(kL3bF[0]));
    return kL3bF;
}

}  // namespace ibmc
