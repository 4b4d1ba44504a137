// Level translations of order 12, one per lane (screened Coulomb, multipole-to-multipole, transposed).
#include "fmm_lane_level.hpp"

DDLPB_LEVEL_LANE_INSTANCE(ym2mT, 0, true)
