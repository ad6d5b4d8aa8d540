// Enumeration kernel instances: three weight layers, narrow first hidden layer, fast hidden epilogue.
#include "enum_q8_impl.h"

namespace ibmc {

static const EnumVariant kL3aF[] = {
    IBMC_VAR_LDS_F(3, 1, 1, 1), IBMC_VAR_LDS_F(3, 1, 1, 2), IBMC_VAR_LDS_F(3, 1, 1, 4),
    IBMC_VAR_LDS_F(3, 1, 2, 1), IBMC_VAR_LDS_F(3, 1, 2, 2),
    IBMC_VAR_LDS_F(3, 2, 1, 1), IBMC_VAR_LDS_F(3, 2, 1, 2), IBMC_VAR_LDS_F(3, 2, 1, 4),
    IBMC_VAR_LDS_F(3, 2, 2, 1), IBMC_VAR_LDS_F(3, 2, 2, 2), IBMC_VAR_LDS_F(3, 2, 2, 4),
    IBMC_VAR_LDS_F(3, 1, 4, 1), IBMC_VAR_LDS_F(3, 2, 4, 1), IBMC_VAR_LDS_F(3, 2, 4, 2),
    IBMC_VAR_LDS_F(3, 4, 1, 1), IBMC_VAR_LDS_F(3, 4, 1, 2), IBMC_VAR_LDS_F(3, 4, 2, 1), IBMC_VAR_LDS_F(3, 4, 2, 2),
};

const EnumVariant *enum_variants_l3a_fast(int *count) {
    *count = (int)(sizeof(kL3aF) / sizeof(kL3aF[0]));
    return kL3aF;
}

}  // namespace ibmc
