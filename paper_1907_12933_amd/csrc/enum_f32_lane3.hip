// Float enumeration instances, one point per lane: three weight layers
// (first hidden width padded to 16 .. 128, second to 16 .. 64, classes to
// 8 / 16).
#include "f32_impl.h"

namespace ibmc {

static const F32LaneVariant kLaneL3[] = {
    IBMC_F32_LANE(16, 16, 8),   IBMC_F32_LANE(16, 16, 16),  IBMC_F32_LANE(32, 16, 8),  IBMC_F32_LANE(32, 16, 16),
    IBMC_F32_LANE(32, 32, 8),   IBMC_F32_LANE(32, 32, 16),  IBMC_F32_LANE(64, 16, 8),  IBMC_F32_LANE(64, 16, 16),
    IBMC_F32_LANE(64, 32, 8),   IBMC_F32_LANE(64, 32, 16),  IBMC_F32_LANE(64, 64, 8),  IBMC_F32_LANE(64, 64, 16),
    IBMC_F32_LANE(128, 16, 8),  IBMC_F32_LANE(128, 16, 16), IBMC_F32_LANE(128, 32, 8), IBMC_F32_LANE(128, 32, 16),
    IBMC_F32_LANE(128, 64, 8),  IBMC_F32_LANE(128, 64, 16),
};

const F32LaneVariant *f32_lane_variants_l3(int *n) {
    *n = (int)(sizeof(kLaneL3) / sizeof(kLaneL3[0]));
    return kLaneL3;
}

}  // namespace ibmc
