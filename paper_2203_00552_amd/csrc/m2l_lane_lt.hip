// Multipole-to-local translations of order 12, one per lane (Coulomb, transposed).
#include "fmm_lane.hpp"

DDLPB_M2L_LANE_INSTANCE(lt, false, true)
