// Float enumeration instances, one point per lane: two weight layers
// (hidden width padded to 16 / 32 / 64 / 128, classes to 8 / 16).
#include "f32_impl.h"

namespace ibmc {

static const F32LaneVariant kLaneL2[] = {
    IBMC_F32_LANE(16, 0, 8),  IBMC_F32_LANE(16, 0, 16),  IBMC_F32_LANE(32, 0, 8),  IBMC_F32_LANE(32, 0, 16),
    IBMC_F32_LANE(64, 0, 8),  IBMC_F32_LANE(64, 0, 16),  IBMC_F32_LANE(128, 0, 8), IBMC_F32_LANE(128, 0, 16),
};

const F32LaneVariant *f32_lane_variants_l2(int *n) {
    *n = (int)(sizeof(kLaneL2) / sizeof(kLaneL2[0]));
    return kLaneL2;
}

}  // namespace ibmc
