// Level translations of order 12, one per lane (screened Coulomb, local-to-local, transposed).
#include "fmm_lane_level.hpp"

DDLPB_LEVEL_LANE_INSTANCE(yl2lT, 2, true)
