// Enumeration kernel instances for networks with more than 16 classes: the
// output layer loops over its M-tiles and every point takes the full argmax.
#include "enum_q8_impl.h"

namespace ibmc {

static const EnumVariant kGeneral[] = {
    IBMC_VAR_LDS_G(2, 1, 0, 1, 0), IBMC_VAR_LDS_G(2, 2, 0, 1, 0), IBMC_VAR_LDS_G(2, 4, 0, 1, 0),
    IBMC_VAR_L2_G(2, 8, 0, 1, 0), IBMC_VAR_L2_G(2, 16, 0, 1, 0),
    IBMC_VAR_L2_G(3, 1, 1, 1, 0), IBMC_VAR_L2_G(3, 1, 2, 1, 0), IBMC_VAR_L2_G(3, 1, 4, 1, 0), IBMC_VAR_L2_G(3, 1, 8, 1, 0),
    IBMC_VAR_L2_G(3, 2, 1, 1, 0), IBMC_VAR_L2_G(3, 2, 2, 1, 0), IBMC_VAR_L2_G(3, 2, 4, 1, 0), IBMC_VAR_L2_G(3, 2, 8, 1, 0),
    IBMC_VAR_L2_G(3, 4, 1, 1, 0), IBMC_VAR_L2_G(3, 4, 2, 1, 0), IBMC_VAR_L2_G(3, 4, 4, 1, 0), IBMC_VAR_L2_G(3, 4, 8, 1, 0),
    IBMC_VAR_L2_G(3, 8, 1, 1, 0), IBMC_VAR_L2_G(3, 8, 2, 1, 0), IBMC_VAR_L2_G(3, 8, 4, 1, 0), IBMC_VAR_L2_G(3, 8, 8, 1, 0),
    IBMC_VAR_L2_G(3, 1, 1, 1, 1), IBMC_VAR_L2_G(3, 1, 2, 1, 1), IBMC_VAR_L2_G(3, 1, 4, 1, 1), IBMC_VAR_L2_G(3, 1, 8, 1, 1),
    IBMC_VAR_L2_G(3, 2, 1, 1, 1), IBMC_VAR_L2_G(3, 2, 2, 1, 1), IBMC_VAR_L2_G(3, 2, 4, 1, 1), IBMC_VAR_L2_G(3, 2, 8, 1, 1),
    IBMC_VAR_L2_G(3, 4, 1, 1, 1), IBMC_VAR_L2_G(3, 4, 2, 1, 1), IBMC_VAR_L2_G(3, 4, 4, 1, 1), IBMC_VAR_L2_G(3, 4, 8, 1, 1),
    IBMC_VAR_L2_G(3, 8, 1, 1, 1), IBMC_VAR_L2_G(3, 8, 2, 1, 1), IBMC_VAR_L2_G(3, 8, 4, 1, 1), IBMC_VAR_L2_G(3, 8, 8, 1, 1),
};

const EnumVariant *enum_variants_general(int *count) {
    *count = (int)(sizeof(kGeneral) / sizeof(kGeneral[0]));
    return kGeneral;
}

}  // namespace ibmc
