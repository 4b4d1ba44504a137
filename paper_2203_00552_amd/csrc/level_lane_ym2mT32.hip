// Level translations of order 12, one per lane, FP32 vector (screened Coulomb, multipole to multipole, transposed).
#include "fmm_lane_level32.hpp"

DDLPB_LEVEL_LANE32_INSTANCE(ym2mT32, 0, true)
