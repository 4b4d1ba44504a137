// Host-visible part of the one-translation-per-lane multipole-to-local kernels of
// order 12 (fmm_lane.hpp): the sparsity pattern of the fixed rotation J, the layout
// of the tables, and the entry points of the four instances (screened Coulomb or
// Coulomb, forward or transposed), each compiled in a translation unit of its own.
#pragma once
#include <hip/hip_runtime.h>

namespace ddlpb {
struct FmmDev;
namespace lane12 {

constexpr int kP = 12, kP1 = 13, kPP = 169;
constexpr int kGroup = 16;                      // lanes per fixed node
constexpr int kOwn = (kPP + kGroup - 1) / kGroup;  // sums per lane after the reduce-scatter

constexpr int iabs(int a) { return a < 0 ? -a : a; }
constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int xpar(int m) { return m >= 0 ? (m & 1) : ((1 - m) & 1); }
// J_l[ma][mb] may be nonzero (see the header comment)
constexpr bool jnz(int l, int ma, int mb) {
  return ((mb >= 0) == (((l + iabs(ma)) & 1) == 0)) && xpar(ma) == xpar(mb);
}
// pattern of J (tr = false) or J^T (tr = true), row a and column b counted from -l
constexpr bool pat(bool tr, int l, int a, int b) { return tr ? jnz(l, b - l, a - l) : jnz(l, a - l, b - l); }
constexpr int row_count(bool tr, int l, int a) {
  int c = 0;
  for (int b = 0; b <= 2 * l; ++b) c += pat(tr, l, a, b) ? 1 : 0;
  return c;
}
// position of entry (l, a, b) in the table of J (or J^T): rows in order of (l, a), the
// pattern entries of a row in order of b
constexpr int entry_offset(bool tr, int l, int a, int b) {
  int o = 0;
  for (int l2 = 0; l2 < l; ++l2)
    for (int a2 = 0; a2 <= 2 * l2; ++a2) o += row_count(tr, l2, a2);
  for (int a2 = 0; a2 < a; ++a2) o += row_count(tr, l, a2);
  for (int b2 = 0; b2 < b; ++b2) o += pat(tr, l, a, b2) ? 1 : 0;
  return o;
}
constexpr int jtab_size(bool tr) { return entry_offset(tr, kP + 1, 0, 0); }

// z-translation tables of the generic kernels (host fmm::Tables::Z): for every output
// degree lo and order am <= lo, for every input degree li >= am, the Yukawa table has
// min(lo, li) - am + 1 coefficients (summed against k_n(z) z^n), the Laplace table one
constexpr int nks(int lo, int li, int am) { return imin(lo, li) - am + 1; }
constexpr int zoff(bool yuk, int lo, int am, int li) {
  int o = 0;
  for (int lo2 = 0; lo2 <= kP; ++lo2)
    for (int am2 = 0; am2 <= lo2; ++am2)
      for (int li2 = am2; li2 <= kP; ++li2) {
        if (lo2 == lo && am2 == am && li2 == li) return o;
        o += yuk ? nks(lo2, li2, am2) : 1;
      }
  return o;
}

constexpr int kZYn = zoff(true, kP + 1, 0, 0);   // Yukawa z-translation coefficients
constexpr int kZLn = zoff(false, kP + 1, 0, 0);  // Coulomb z-translation coefficients

constexpr int kJn = jtab_size(false), kJTn = jtab_size(true);
constexpr int kLaneWaves = 4;  // wavefronts per block: they share the z-translation table in LDS

struct LaneTab {
  const double* Z;   // z-translation coefficients of the kernel type and direction (generic table order)
  const int* order;  // nodes by decreasing list length
  int* counter;      // work counter, zero at launch
};

// instances: yf (screened Coulomb), yt (its transpose), lf (Coulomb), lt (its transpose)
#define DDLPB_M2L_LANE_DECL(NAME)                                                                        \
  hipError_t upload_##NAME(const double* J, const double* JT);                                          \
  hipError_t launch_##NAME(const FmmDev& f, const LaneTab& t, int nn, const int* lptr, const int* lidx, \
                           const double* in, double* out, int blocks, hipStream_t s);                   \
  hipError_t occupancy_##NAME(int* blocks_per_cu);
DDLPB_M2L_LANE_DECL(yf)
DDLPB_M2L_LANE_DECL(yt)
DDLPB_M2L_LANE_DECL(lf)
DDLPB_M2L_LANE_DECL(lt)
// FP32-vector instances of the screened Coulomb kernel (fmm_lane32.hpp): yf32, yt32
DDLPB_M2L_LANE_DECL(yf32)
DDLPB_M2L_LANE_DECL(yt32)
#undef DDLPB_M2L_LANE_DECL

// Level translations of the screened Coulomb expansions (fmm_lane_level.hpp), one node
// of the level per lane: ym2m (upward pass), yl2l (downward pass) and their transposes
// ym2mT (transposed downward pass), yl2lT (transposed upward pass).  Z is the
// z-translation table of the level kinds in the direction of the instance.
#define DDLPB_LEVEL_LANE_DECL(NAME)                                                                      \
  hipError_t upload_##NAME(const double* J, const double* JT);                                          \
  hipError_t launch_##NAME(const FmmDev& f, const double* Z, int count, const int* nodes, const int* child, \
                           const int* parent, double* E, hipStream_t s);
DDLPB_LEVEL_LANE_DECL(ym2m)
DDLPB_LEVEL_LANE_DECL(yl2l)
DDLPB_LEVEL_LANE_DECL(ym2mT)
DDLPB_LEVEL_LANE_DECL(yl2lT)
// FP32-vector instances (fmm_lane_level32.hpp)
DDLPB_LEVEL_LANE_DECL(ym2m32)
DDLPB_LEVEL_LANE_DECL(yl2l32)
DDLPB_LEVEL_LANE_DECL(ym2mT32)
DDLPB_LEVEL_LANE_DECL(yl2lT32)
#undef DDLPB_LEVEL_LANE_DECL

}  // namespace lane12
}  // namespace ddlpb
