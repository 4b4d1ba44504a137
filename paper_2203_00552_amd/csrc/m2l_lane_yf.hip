// Multipole-to-local translations of order 12, one per lane (screened Coulomb, forward).
#include "fmm_lane.hpp"

DDLPB_M2L_LANE_INSTANCE(yf, true, false)
