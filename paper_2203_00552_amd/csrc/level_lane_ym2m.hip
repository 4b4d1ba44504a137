// Level translations of order 12, one per lane (screened Coulomb, multipole-to-multipole).
#include "fmm_lane_level.hpp"

DDLPB_LEVEL_LANE_INSTANCE(ym2m, 0, false)
