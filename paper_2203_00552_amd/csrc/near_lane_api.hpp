// Host-visible part of the near-field A/B kernels with one neighbour cap per lane
// (near_lane.hip): argument block, incore cache layout and entry points.
//
// Both directions walk the reverse cap list of a sphere j: the grid points x_i^n of
// other spheres that lie inside sphere j, with their weights omega_ij(x_i^n).  On every
// such point the regular solid harmonics of sphere j, S_lm((x_i^n - x_j) / r_j) (the
// A basis, Sec. 2.2), and the ratios i_l(kappa |x_i^n - x_j|) / i_l(kappa r_j) divided by
// (|x_i^n - x_j| / r_j)^l (which turn S into the B basis) are needed:
//  * transposed pass (A^T, B^T): the coefficients of sphere j collect, over its
//    reverse caps, the point values of the adjoint iterate times these functions;
//  * forward pass (A, B): every reverse cap gets the value of the expansion of sphere
//    j at its point; the per-point sums over the caps of a grid point are taken by
//    the caller in the fixed order of the forward lists.
// A group of 16 lanes owns one sphere j and takes 16 of its caps at a time; the group's
// 16 partial sums are combined by a reduce-scatter over DPP row permutations, so every
// result is a fixed-order sum (bitwise reproducible, no atomics).
#pragma once
#include <hip/hip_runtime.h>

namespace ddlpb {
namespace nearlane {

constexpr int kMaxLm = 8;       // largest degree with a lane kernel
constexpr int kGroup = 16;      // lanes per sphere

// values per cap in the incore cache: the (LM+1)^2 harmonics and LM+1 radial ratios
__host__ __device__ constexpr int cache_stride(int lm) { return (lm + 1) * (lm + 1) + lm + 1; }

struct NearArgs {
  int M, N, LUR, nterms;
  double kappa;
  const double* leb;   // [N][4]: direction and weight
  const double* xyz;   // [M][3]
  const double* rad;   // [M]
  const int* rptr;     // [M+1] reverse cap ranges
  const int* rci;      // reverse caps: sphere i of the grid point
  const int* rcn;      // reverse caps: point index n
  const double* rcw;   // reverse caps: omega_ij(x_i^n)
  const double* isgr;  // [M][LUR]: 1 / sigma_l(kappa^2 r_j^2)
  const int* jord;     // [M]: spheres by decreasing number of reverse caps (work order:
                       // the four spheres of a wavefront carry similar work)
  // incore cache (nullptr: everything on the fly).  Sphere j's caps start at cap
  // position coff[j] (a multiple of 16); the block of caps 16 b .. 16 b + 15 holds value
  // t of cap 16 b + q at cache[(16 b) * T + 16 t + q], T = cache_stride(lmax).
  const double* cache;
  const long* coff;
};

// recurrence constants of the normalised Legendre functions (same definition as the
// main library's tables: P_m^m = pmm[m], P_l^m = ra z P_{l-1}^m - rb r^2 P_{l-2}^m,
// indexed by l (l + 1) / 2 + m), once per device
hipError_t upload_tables(const double* pmm, const double* ra, const double* rb);

// out = c0 base + c1 (near part of L_AB^T) Z, with zr / ze the point values of Z
// (Syn of each sphere's coefficients, [M][N] each); prec 1 computes in FP32.
// base may alias out.
hipError_t launch_ltz(int lmax, int prec, const NearArgs& a, const double* base, double c0, const double* zr,
                      const double* ze, double c1, double* out, hipStream_t s);
// capv[2 c], capv[2 c + 1] = omega (A, B expansion of sphere j at the point of reverse
// cap c) for the coefficients X ([2M][L]); prec 1 computes in FP32
hipError_t launch_lx(int lmax, int prec, const NearArgs& a, const double* X, double* capv, hipStream_t s);
// fills the incore cache (a.cache) for every reverse cap
hipError_t launch_fill(int lmax, const NearArgs& a, double* cache, hipStream_t s);

}  // namespace nearlane
}  // namespace ddlpb
