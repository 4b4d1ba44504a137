// Multipole-to-local translations of order 12, one per lane, FP32 vector (screened Coulomb).
#include "fmm_lane32.hpp"

DDLPB_M2L_LANE32_INSTANCE(yf32, false)
