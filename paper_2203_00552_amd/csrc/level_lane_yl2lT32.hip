// Level translations of order 12, one per lane, FP32 vector (screened Coulomb, local to local, transposed).
#include "fmm_lane_level32.hpp"

DDLPB_LEVEL_LANE32_INSTANCE(yl2lT32, 2, true)
