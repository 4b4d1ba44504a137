// Level translations of order 12, one per lane, FP32 vector (screened Coulomb, local to local).
#include "fmm_lane_level32.hpp"

DDLPB_LEVEL_LANE32_INSTANCE(yl2l32, 2, false)
