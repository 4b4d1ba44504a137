// ddLPB kernels for gfx950: grid switching fields, per-sphere harmonic
// transforms, the sparse neighbour-sphere A/B operators (and transposes), the
// single-layer (screened Coulomb) field by direct summation and its adjoint,
// the vacuum Coulomb field, Krylov helpers and the force assembly.
//
// Layouts (all FP64, row-major):
//   centres xyz [M][3], radii [M], charges [M]
//   Lebedev rule leb [N][4] = (s_x, s_y, s_z, w)
//   Y table [N][LY]  (Y_lm(s_n), index l*l+l+m)
//   grid functions [M][N]; harmonic vectors [M][L] and solution vectors [2][M][L]
//   per-sphere radial tables [M][LUR] (LUR = lmax+2)
//   active points: the grid points with chi^eta > 0, listed sphere by sphere
//   (act_sph[k], act_n[k]), act_ptr[M+1].
#pragma once
#include <type_traits>

#include "device_math.hpp"

namespace ddlpb {

constexpr int kMaxN = 974;

__device__ __forceinline__ int deg_of(int lm) {
  int l = (int)sqrt((double)lm);
  while ((l + 1) * (l + 1) <= lm) ++l;
  while (l * l > lm) --l;
  return l;
}

// ------------------------------------------------------------- grid fields
// f^i(x_i^n) = sum_{j in N_i} chi_eta(|x_i^n - x_j| / r_j),  U = 1 - min(f, 1)   (Sec. 3.1)
__global__ void k_grid_fields(int M, int N, const double* __restrict__ xyz, const double* __restrict__ rad,
                              const double* __restrict__ leb, const int* __restrict__ nptr,
                              const int* __restrict__ nidx, double eta, double* __restrict__ f,
                              double* __restrict__ U) {
  long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (g >= (long)M * N) return;
  int i = (int)(g / N), n = (int)(g - (long)i * N);
  const double px = xyz[3 * i] + rad[i] * leb[4 * n];
  const double py = xyz[3 * i + 1] + rad[i] * leb[4 * n + 1];
  const double pz = xyz[3 * i + 2] + rad[i] * leb[4 * n + 2];
  double fs = 0.0;
  for (int a = nptr[i]; a < nptr[i + 1]; ++a) {
    int j = nidx[a];
    double dx = px - xyz[3 * j], dy = py - xyz[3 * j + 1], dz = pz - xyz[3 * j + 2];
    fs += chi_eta(sqrt(dx * dx + dy * dy + dz * dz) / rad[j], eta);
  }
  f[g] = fs;
  U[g] = fs < 1.0 ? 1.0 - fs : 0.0;
}

// number of active points (U > 0) and cap pairs (omega > 0) per sphere
__global__ void k_active_count(int M, int N, const double* __restrict__ U, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  int c = 0;
  for (int n = 0; n < N; ++n) c += U[(long)i * N + n] > 0.0;
  cnt[i] = c;
}
__global__ void k_active_fill(int M, int N, const double* __restrict__ U, const int* __restrict__ ptr,
                              int* __restrict__ act_sph, int* __restrict__ act_n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  int k = ptr[i];
  for (int n = 0; n < N; ++n)
    if (U[(long)i * N + n] > 0.0) { act_sph[k] = i; act_n[k] = n; ++k; }
}

// cap pairs (i, n, j) with |x_i^n - x_j| < r_j, i.e. omega_ij(x_i^n) > 0, per sphere
__global__ void k_cap_count(int M, int N, const double* __restrict__ xyz, const double* __restrict__ rad,
                            const double* __restrict__ leb, const int* __restrict__ nptr,
                            const int* __restrict__ nidx, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  int c = 0;
  for (int n = 0; n < N; ++n) {
    const double px = xyz[3 * i] + rad[i] * leb[4 * n], py = xyz[3 * i + 1] + rad[i] * leb[4 * n + 1],
                 pz = xyz[3 * i + 2] + rad[i] * leb[4 * n + 2];
    for (int a = nptr[i]; a < nptr[i + 1]; ++a) {
      const int j = nidx[a];
      const double dx = px - xyz[3 * j], dy = py - xyz[3 * j + 1], dz = pz - xyz[3 * j + 2];
      c += (dx * dx + dy * dy + dz * dz < rad[j] * rad[j]);
    }
  }
  cnt[i] = c;
}

__global__ void k_fill(long n, double v, double* __restrict__ a) {
  long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (g < n) a[g] = v;
}

// ----------------------------------------------------- single-layer moments
// m_j = C^j (.) An_j(U_j (.) (e_j + Syn(y_j))), y_j = ycr_l X_r,j + yce_l X_e,j  (Sec. 2.2, Q and P chi)
// Optionally stores h = e + Syn(y) on the grid.
template <int LM>
__global__ __launch_bounds__(256) void k_moments(int M, int N, int LY, const double* __restrict__ Y,
                                                  const double* __restrict__ leb, const double* __restrict__ U,
                                                  const double* __restrict__ X, const double* __restrict__ ycr,
                                                  const double* __restrict__ yce, int LUR,
                                                  const double* __restrict__ egrid, const double* __restrict__ Cl,
                                                  double* __restrict__ h_out, double* __restrict__ m_out) {
  constexpr int L = (LM + 1) * (LM + 1);
  __shared__ double y[L];
  __shared__ double hu[kMaxN];
  const int j = blockIdx.x;
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    double v = 0.0;
    if (X) {
      int l = deg_of(t);
      v = ycr[j * LUR + l] * X[(long)j * L + t] + yce[j * LUR + l] * X[(long)(M + j) * L + t];
    }
    y[t] = v;
  }
  __syncthreads();
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    double h = egrid ? egrid[(long)j * N + n] : 0.0;
    if (X) {
      const double* Yn = Y + (long)n * LY;
#pragma unroll 9
      for (int t = 0; t < L; ++t) h += Yn[t] * y[t];
    }
    if (h_out) h_out[(long)j * N + n] = h;
    hu[n] = U[(long)j * N + n] * h;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    double acc = 0.0;
    for (int n = 0; n < N; ++n) acc += leb[4 * n + 3] * Y[(long)n * LY + t] * hu[n];
    m_out[(long)j * L + t] = Cl[j * LUR + deg_of(t)] * acc;
  }
}

// ------------------------------------------------ single-layer field (direct)
// Phi(x) = sum_j sum_lm m_jlm k_l(kappa|x-x_j|)/k_l(kappa r_j) Y_lm((x-x_j)/|x-x_j|)
// at every active point, or its gradient with respect to x (GRAD).  One thread
// per active point, source spheres staged through LDS in chunks.
template <int LM, bool GRAD>
__global__ __launch_bounds__(256) void k_sl_field_direct(int M, int N, int nact, const int* __restrict__ act_sph,
                                                          const int* __restrict__ act_n,
                                                          const double* __restrict__ xyz,
                                                          const double* __restrict__ rad,
                                                          const double* __restrict__ leb,
                                                          const double* __restrict__ m,
                                                          const double* __restrict__ ur, int LUR, double kappa,
                                                          int exclude_self, double* __restrict__ out) {
  constexpr int L = (LM + 1) * (LM + 1);
  constexpr int CH = 16;
  __shared__ double sm[CH * L];
  __shared__ double sx[CH * 4];
  __shared__ double sur[CH * (LM + 1)];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = k < nact;
  const int i = active ? act_sph[k] : -1;
  const int n = active ? act_n[k] : 0;
  double p[3] = {0, 0, 0};
  if (active)
    for (int a = 0; a < 3; ++a) p[a] = xyz[3 * i + a] + rad[i] * leb[4 * n + a];
  using T = typename std::conditional<GRAD, Dual<double>, double>::type;
  T acc(0.0);
  for (int j0 = 0; j0 < M; j0 += CH) {
    const int nc = min(CH, M - j0);
    __syncthreads();
    for (int t = threadIdx.x; t < nc * L; t += blockDim.x) sm[t] = m[(long)j0 * L + t];
    for (int t = threadIdx.x; t < nc; t += blockDim.x) {
      const int j = j0 + t;
      sx[4 * t] = xyz[3 * j]; sx[4 * t + 1] = xyz[3 * j + 1]; sx[4 * t + 2] = xyz[3 * j + 2]; sx[4 * t + 3] = rad[j];
      for (int l = 0; l <= LM; ++l) sur[t * (LM + 1) + l] = 1.0 / ur[j * LUR + l];
    }
    __syncthreads();
    if (!active) continue;
    for (int c = 0; c < nc; ++c) {
      if (exclude_self && j0 + c == i) continue;
      const double rj = sx[4 * c + 3], irj = 1.0 / rj;
      T v[3];
      for (int a = 0; a < 3; ++a) {
        v[a] = T(p[a]);
        if constexpr (GRAD) v[a].g[a] = 1.0;
        v[a] = (v[a] - T(sx[4 * c + a])) * irj;  // scaled relative position
      }
      T rho = dsqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) * rj;
      T u[LM + 1];
      k_weights<LM, T>(rho, kappa, u);
      const double* mc = sm + c * L;
      const double* iu = sur + c * (LM + 1);
      T part[LM + 1];
#pragma unroll
      for (int l = 0; l <= LM; ++l) part[l] = T(0.0);
      for_each_solid_harmonic<LM, T>(v[0], v[1], v[2], [&](int l, int idx, const T& S) { part[l] = part[l] + mc[idx] * S; });
#pragma unroll
      for (int l = 0; l <= LM; ++l) acc = acc + (iu[l] * u[l]) * part[l];
    }
  }
  if (!active) return;
  if constexpr (GRAD) {
    for (int a = 0; a < 3; ++a) out[3L * k + a] = acc.g[a];
  } else {
    out[(long)i * N + n] = acc;
  }
}

// -------------------------------------------- single-layer adjoint (direct)
// lambda_jlm = sum_{(i,n) active} c_in k_l(kappa|x_i^n-x_j|)/k_l(kappa r_j) Y_lm(...), l <= LMO.
// One block per target sphere j, threads over all active source points,
// register accumulation and a deterministic block reduction.
template <int LMO>
__global__ __launch_bounds__(256) void k_sl_adjoint_direct(int M, int N, int nact, const int* __restrict__ act_sph,
                                                            const int* __restrict__ act_n,
                                                            const double* __restrict__ xyz,
                                                            const double* __restrict__ rad,
                                                            const double* __restrict__ leb,
                                                            const double* __restrict__ cgrid,
                                                            const double* __restrict__ ur, int LUR, double kappa,
                                                            int exclude_self, double* __restrict__ lam) {
  constexpr int LO = (LMO + 1) * (LMO + 1);
  __shared__ double red[4 * LO];
  const int j = blockIdx.x;
  const double xj = xyz[3 * j], yj = xyz[3 * j + 1], zj = xyz[3 * j + 2], rj = rad[j], irj = 1.0 / rj;
  double iu[LMO + 1];
#pragma unroll
  for (int l = 0; l <= LMO; ++l) iu[l] = 1.0 / ur[j * LUR + l];
  double acc[LO];
#pragma unroll
  for (int t = 0; t < LO; ++t) acc[t] = 0.0;
  for (int k = threadIdx.x; k < nact; k += blockDim.x) {
    const int i = act_sph[k], n = act_n[k];
    if (exclude_self && i == j) continue;
    const double c = cgrid[(long)i * N + n];
    if (c == 0.0) continue;
    const double vx = (xyz[3 * i] + rad[i] * leb[4 * n] - xj) * irj;
    const double vy = (xyz[3 * i + 1] + rad[i] * leb[4 * n + 1] - yj) * irj;
    const double vz = (xyz[3 * i + 2] + rad[i] * leb[4 * n + 2] - zj) * irj;
    const double rho = sqrt(vx * vx + vy * vy + vz * vz) * rj;
    double u[LMO + 1];
    k_weights<LMO, double>(rho, kappa, u);
#pragma unroll
    for (int l = 0; l <= LMO; ++l) u[l] *= c * iu[l];
    for_each_solid_harmonic<LMO, double>(vx, vy, vz, [&](int l, int idx, double S) { acc[idx] += u[l] * S; });
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < LO; ++t) {
    double v = wave_sum(acc[t]);
    if (lane == 0) red[wid * LO + t] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < LO; t += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w * LO + t];
    lam[(long)j * LO + t] = s;
  }
}

// ------------------------------------------- single-layer field (listed pairs)
// Same field as k_sl_field_direct, restricted to the source spheres listed for the
// target point's own sphere (CSR lptr/lidx): the near part of a split evaluation.
// R is the compute type of one (point, sphere) interaction: double, or float on the
// mixed path, where the offset x - x_j is formed in FP64 and rounded once, the weights
// and harmonics of the pair run in FP32 and the sum over the listed spheres is FP64.
// iur = 1 / u_l(r_j) [M][LUR].
template <class R>
__device__ __forceinline__ R recip(double x) {
  if constexpr (sizeof(R) == 8) return 1.0 / x;
  else return __builtin_amdgcn_rcpf((float)x);
}
__device__ __forceinline__ double widen(float x) { return (double)x; }
__device__ __forceinline__ Dual<double> widen(const Dual<float>& x) {
  Dual<double> r;
  r.v = x.v;
  for (int a = 0; a < 3; ++a) r.g[a] = x.g[a];
  return r;
}
template <int LM, bool GRAD, class R = double>
__global__ __launch_bounds__(256) void k_sl_field_list(int M, int N, int nact, const int* __restrict__ act_sph,
                                                        const int* __restrict__ act_n, const double* __restrict__ xyz,
                                                        const double* __restrict__ rad, const double* __restrict__ leb,
                                                        const int* __restrict__ lptr, const int* __restrict__ lidx,
                                                        const double* __restrict__ m, const double* __restrict__ iur,
                                                        int LUR, double kappa, int exclude_self, int accumulate,
                                                        double* __restrict__ out) {
  constexpr int L = (LM + 1) * (LM + 1);
  constexpr bool f64 = sizeof(R) == 8;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nact) return;
  const int i = act_sph[k], n = act_n[k];
  double p[3];
  for (int a = 0; a < 3; ++a) p[a] = xyz[3 * i + a] + rad[i] * leb[4 * n + a];
  using T = typename std::conditional<GRAD, Dual<R>, R>::type;
  using A = typename std::conditional<GRAD, Dual<double>, double>::type;
  A acc(0.0);
  for (int q = lptr[i]; q < lptr[i + 1]; ++q) {
    const int j = lidx[q];
    if (exclude_self && j == i) continue;
    const double rj = rad[j];
    const R irj = recip<R>(rj);
    T v[3];
    for (int a = 0; a < 3; ++a) {
      v[a] = T(R(p[a] - xyz[3 * j + a]));
      if constexpr (GRAD) v[a].g[a] = R(1);
      v[a] = v[a] * irj;
    }
    T rho = dsqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) * R(rj);
    T u[LM + 1];
    k_weights<LM, T>(rho, kappa, u);
    const double* mc = m + (long)j * L;
    T part[LM + 1];
#pragma unroll
    for (int l = 0; l <= LM; ++l) part[l] = T(R(0));
    for_each_solid_harmonic<LM, T>(v[0], v[1], v[2],
                                   [&](int l, int idx, const T& S) { part[l] = part[l] + R(mc[idx]) * S; });
    if constexpr (f64) {
#pragma unroll
      for (int l = 0; l <= LM; ++l) acc = acc + (u[l] * iur[j * LUR + l]) * part[l];
    } else {
      T sj(R(0));
#pragma unroll
      for (int l = 0; l <= LM; ++l) sj = sj + (u[l] * R(iur[j * LUR + l])) * part[l];
      acc = acc + widen(sj);
    }
  }
  if constexpr (GRAD) {
    for (int a = 0; a < 3; ++a) out[3L * k + a] = (accumulate ? out[3L * k + a] : 0.0) + acc.g[a];
  } else {
    const long in = (long)i * N + n;
    out[in] = (accumulate ? out[in] : 0.0) + acc;
  }
}

// Active grid points packed for the adjoint single layer: pt[k] = (x_i^n, c_in) of active
// point k (sphere act_sph[k], point act_n[k]), c the grid charge of this call.
__global__ void k_pack_points(int nact, int N, const int* __restrict__ act_sph, const int* __restrict__ act_n,
                              const double* __restrict__ xyz, const double* __restrict__ rad,
                              const double* __restrict__ leb, const double* __restrict__ cgrid,
                              double4* __restrict__ pt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nact) return;
  const int i = act_sph[k], n = act_n[k];
  const double r = rad[i];
  pt[k] = make_double4(xyz[3 * i] + r * leb[4 * n], xyz[3 * i + 1] + r * leb[4 * n + 1],
                       xyz[3 * i + 2] + r * leb[4 * n + 2], cgrid[(long)i * N + n]);
}

// Adjoint of k_sl_field_list: lambda_j = sum over the active points of the spheres listed
// for j of c_p k_l(kappa|x_p-x_j|)/k_l(kappa r_j) Y_lm (the lists are symmetric), with the
// active points packed by k_pack_points (consecutive points of a sphere are consecutive
// 32-byte records, and a point costs one load).
// R = float (mixed path): each thread's running sums over its points are FP32, the
// sums across threads FP64.
template <int LMO, class R = double>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_sl_adjoint_list(
    int M, const int* __restrict__ act_ptr, const double4* __restrict__ pt, const double* __restrict__ xyz,
    const double* __restrict__ rad, const int* __restrict__ lptr, const int* __restrict__ lidx,
    const double* __restrict__ iur, int LUR, double kappa, int exclude_self, int accumulate, int LDL,
    double* __restrict__ lam) {
  constexpr int LO = (LMO + 1) * (LMO + 1);
  __shared__ double red[4 * LO];
  const int j = blockIdx.x;
  const double xj = xyz[3 * j], yj = xyz[3 * j + 1], zj = xyz[3 * j + 2], rj = rad[j];
  const R irj = recip<R>(rj);
  // 1 / u_l(r_j) in LDS (registers go to the LO accumulators)
  __shared__ R iu[LMO + 1];
  if (threadIdx.x <= LMO) iu[threadIdx.x] = R(iur[j * LUR + threadIdx.x]);
  R acc[LO];
#pragma unroll
  for (int t = 0; t < LO; ++t) acc[t] = R(0);
  // the active points of up to kSlaSeg listed spheres are numbered consecutively
  // (prefix sums in LDS) so that every thread of the block has points to take
  constexpr int kSlaSeg = 128;
  __shared__ int seg_base[kSlaSeg], seg_pre[kSlaSeg + 1];
  for (int q0 = lptr[j]; q0 < lptr[j + 1]; q0 += kSlaSeg) {
    const int ns = min(kSlaSeg, lptr[j + 1] - q0);
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc_n = 0;
      for (int u = 0; u < ns; ++u) {
        const int i = lidx[q0 + u];
        seg_base[u] = act_ptr[i];
        seg_pre[u] = acc_n;
        acc_n += (exclude_self && i == j) ? 0 : act_ptr[i + 1] - act_ptr[i];
      }
      seg_pre[ns] = acc_n;
    }
    __syncthreads();
    const int total = seg_pre[ns];
    // record of point f (position, grid charge): binary search for its sphere in LDS
    auto fetch = [&](int f) {
      int lo = 0, hi = ns - 1;  // last u with seg_pre[u] <= f
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_pre[mid] <= f) lo = mid; else hi = mid - 1;
      }
      return pt[seg_base[lo] + (f - seg_pre[lo])];
    };
    // the next point's record is loaded before the current point is evaluated
    double4 pn = make_double4(0.0, 0.0, 0.0, 0.0);
    if ((int)threadIdx.x < total) pn = fetch(threadIdx.x);
    for (int f = threadIdx.x; f < total; f += blockDim.x) {
      const double4 p = pn;
      if (f + (int)blockDim.x < total) pn = fetch(f + blockDim.x);
      if (p.w == 0.0) continue;
      const R vx = R(p.x - xj) * irj;
      const R vy = R(p.y - yj) * irj;
      const R vz = R(p.z - zj) * irj;
      const R rho = dsqrt(vx * vx + vy * vy + vz * vz) * R(rj);
      R u[LMO + 1];
      k_weights<LMO, R>(rho, kappa, u);
#pragma unroll
      for (int l = 0; l <= LMO; ++l) u[l] *= R(p.w) * iu[l];
      for_each_solid_harmonic<LMO, R>(vx, vy, vz, [&](int l, int idx, R S) { acc[idx] += u[l] * S; });
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < LO; ++t) {
    double v = wave_sum((double)acc[t]);
    if (lane == 0) red[wid * LO + t] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < LO; t += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w * LO + t];
    lam[(long)j * LDL + t] = (accumulate ? lam[(long)j * LDL + t] : 0.0) + s;
  }
}

// --------------------------------------------------- vacuum field (direct)
// psi_0(x) = sum_k q_k/(eps1 |x - x_k|) and e = (eps1/eps2) d_n psi_0 at active points (Sec. 2.2, G0, F0).
__global__ __launch_bounds__(256) void k_laplace_field_direct(int M, int N, int nact, const int* __restrict__ act_sph,
                                                              const int* __restrict__ act_n,
                                                              const double* __restrict__ xyz,
                                                              const double* __restrict__ rad,
                                                              const double* __restrict__ leb,
                                                              const double* __restrict__ q, double eps1,
                                                              double eps2, double* __restrict__ psi_out,
                                                              double* __restrict__ e_out) {
  __shared__ double sq[256 * 4];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = k < nact;
  const int i = active ? act_sph[k] : 0, n = active ? act_n[k] : 0;
  double p[3], s[3];
  for (int a = 0; a < 3; ++a) { s[a] = leb[4 * n + a]; p[a] = xyz[3 * i + a] + rad[i] * s[a]; }
  double psi = 0.0, dn = 0.0;
  for (int k0 = 0; k0 < M; k0 += 256) {
    const int nc = min(256, M - k0);
    __syncthreads();
    if ((int)threadIdx.x < nc) {
      const int kk = k0 + threadIdx.x;
      sq[4 * threadIdx.x] = xyz[3 * kk]; sq[4 * threadIdx.x + 1] = xyz[3 * kk + 1];
      sq[4 * threadIdx.x + 2] = xyz[3 * kk + 2]; sq[4 * threadIdx.x + 3] = q[kk];
    }
    __syncthreads();
    if (!active) continue;
    for (int c = 0; c < nc; ++c) {
      double vx = p[0] - sq[4 * c], vy = p[1] - sq[4 * c + 1], vz = p[2] - sq[4 * c + 2];
      double id = 1.0 / sqrt(vx * vx + vy * vy + vz * vz);
      double qi = sq[4 * c + 3] * id;
      psi += qi;
      dn -= qi * id * id * (vx * s[0] + vy * s[1] + vz * s[2]);
    }
  }
  if (!active) return;
  psi_out[(long)i * N + n] = psi / eps1;
  e_out[(long)i * N + n] = dn / eps2;
}

// ------------------------------------------------------ apply L (near part)
// out_r = c0 base_r + c1 An(sum_j omega_ij vA_j) + cg An(U (gr1 + gr2))
// out_e = c0 base_e + c1 An(sum_j omega_ij vB_j) + cg An(U ge)
// with vA_j(x) = sum_lm X_r,jlm (|x-x_j|/r_j)^l Y_lm, vB_j the same with
// i_l(kappa|x-x_j|)/i_l(kappa r_j) (Sec. 2.2, A and B).  One block per sphere.
template <int LM>
__global__ __launch_bounds__(256) void k_apply_LX(int M, int N, int LY, const double* __restrict__ Y,
                                                   const double* __restrict__ leb, const double* __restrict__ xyz,
                                                   const double* __restrict__ rad, const int* __restrict__ nptr,
                                                   const int* __restrict__ nidx, const double* __restrict__ f,
                                                   const double* __restrict__ U, const double* __restrict__ sgr,
                                                   int LUR, double kappa, double eta, int nterms,
                                                   const double* __restrict__ base, double c0,
                                                   const double* __restrict__ nearX, double c1,
                                                   const double* __restrict__ gr1, const double* __restrict__ gr2,
                                                   const double* __restrict__ ge, double cg,
                                                   double* __restrict__ out) {
  constexpr int L = (LM + 1) * (LM + 1);
  __shared__ double vA[kMaxN], vB[kMaxN], gR[kMaxN], gE[kMaxN];
  const int i = blockIdx.x;
  const double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2], ri = rad[i];
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    double a = 0.0, b = 0.0;
    if (nearX) {
      const double px = xi + ri * leb[4 * n], py = yi + ri * leb[4 * n + 1], pz = zi + ri * leb[4 * n + 2];
      const double fv = f[(long)i * N + n];
      const double dfac = fv > 1.0 ? 1.0 / fv : 1.0;
      for (int q = nptr[i]; q < nptr[i + 1]; ++q) {
        const int j = nidx[q];
        const double irj = 1.0 / rad[j];
        const double vx = (px - xyz[3 * j]) * irj, vy = (py - xyz[3 * j + 1]) * irj, vz = (pz - xyz[3 * j + 2]) * irj;
        const double t2 = vx * vx + vy * vy + vz * vz;
        if (t2 >= 1.0) continue;
        const double om = dfac * chi_eta(sqrt(t2), eta);
        if (om == 0.0) continue;
        double sg[LM + 1];
        sigma_weights<LM, double>(kappa * kappa * rad[j] * rad[j] * t2, nterms, sg);
#pragma unroll
        for (int l = 0; l <= LM; ++l) sg[l] /= sgr[j * LUR + l];
        const double* Xr = nearX + (long)j * L;
        const double* Xe = nearX + (long)(M + j) * L;
        double sa = 0.0, pb[LM + 1];
#pragma unroll
        for (int l = 0; l <= LM; ++l) pb[l] = 0.0;
        for_each_solid_harmonic<LM, double>(vx, vy, vz, [&](int l, int idx, double S) {
          sa += Xr[idx] * S;
          pb[l] += Xe[idx] * S;
        });
        double sb = 0.0;
#pragma unroll
        for (int l = 0; l <= LM; ++l) sb += sg[l] * pb[l];
        a += om * sa;
        b += om * sb;
      }
    }
    vA[n] = a;
    vB[n] = b;
    const double u = U[(long)i * N + n];
    gR[n] = gr1 ? u * (gr1[(long)i * N + n] + (gr2 ? gr2[(long)i * N + n] : 0.0)) : 0.0;
    gE[n] = ge ? u * ge[(long)i * N + n] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    double sa = 0.0, sb = 0.0, sr = 0.0, se = 0.0;
    for (int n = 0; n < N; ++n) {
      const double wy = leb[4 * n + 3] * Y[(long)n * LY + t];
      sa += wy * vA[n];
      sb += wy * vB[n];
      sr += wy * gR[n];
      se += wy * gE[n];
    }
    const long ir = (long)i * L + t, ie = (long)(M + i) * L + t;
    double orr = c1 * sa + cg * sr, oe = c1 * sb + cg * se;
    if (base) { orr += c0 * base[ir]; oe += c0 * base[ie]; }
    out[ir] = orr;
    out[ie] = oe;
  }
}

// ---------------------------------------------- syntheses on the grid
// mode 0: zr = Syn(Z_r), ze = Syn(Z_e);  mode 1: c = w U Syn(Z_r + Z_e) (adjoint charges)
// YT: harmonic table transposed, [LY][N] (consecutive threads read consecutive points)
template <int LM>
__global__ __launch_bounds__(512) void k_syn2(int M, int N, int LY, const double* __restrict__ YT,
                                              const double* __restrict__ leb, const double* __restrict__ U,
                                              const double* __restrict__ Z, int mode, double* __restrict__ o1,
                                              double* __restrict__ o2) {
  constexpr int L = (LM + 1) * (LM + 1);
  __shared__ double zr[L], ze[L];
  const int i = blockIdx.x;
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    zr[t] = Z[(long)i * L + t];
    ze[t] = Z[(long)(M + i) * L + t];
  }
  __syncthreads();
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    double a = 0.0, b = 0.0;
#pragma unroll 9
    for (int t = 0; t < L; ++t) {
      const double y = YT[(long)t * N + n];
      a += y * zr[t];
      b += y * ze[t];
    }
    if (mode == 0) {
      o1[(long)i * N + n] = a;
      o2[(long)i * N + n] = b;
    } else {
      o1[(long)i * N + n] = leb[4 * n + 3] * U[(long)i * N + n] * (a + b);
    }
  }
}

// ------------------------------------------------------- apply L^T
// out_r = c0 base_r + c1 sum_{i in N_j} sum_n w_n omega_ij^n zr_in basisA_j(x_i^n) + ycr (.) mu_j
// out_e = c0 base_e + c1 (same with ze and basisB) + yce (.) mu_j,
// mu_j = An_j(U_j Syn(C^j (.) lambda_j)) (transpose of the C-part).  One block per sphere j.
template <int LM>
__global__ __launch_bounds__(256) void k_apply_LTZ(int M, int N, int LY, const double* __restrict__ Y,
                                                    const double* __restrict__ leb, const double* __restrict__ xyz,
                                                    const double* __restrict__ rad, const int* __restrict__ nptr,
                                                    const int* __restrict__ nidx, const double* __restrict__ f,
                                                    const double* __restrict__ U, const double* __restrict__ sgr,
                                                    const double* __restrict__ ycr, const double* __restrict__ yce,
                                                    const double* __restrict__ Cl, int LUR, double kappa, double eta,
                                                    int nterms, const double* __restrict__ base, double c0,
                                                    const double* __restrict__ zr, const double* __restrict__ ze,
                                                    double c1, const double* __restrict__ lam, int LLAM,
                                                    double* __restrict__ out) {
  constexpr int L = (LM + 1) * (LM + 1);
  __shared__ double gg[kMaxN];
  __shared__ double cl[L], mu[L];
  __shared__ double red[8 * L];
  const int j = blockIdx.x;
  if (lam) {
    for (int t = threadIdx.x; t < L; t += blockDim.x) cl[t] = Cl[j * LUR + deg_of(t)] * lam[(long)j * LLAM + t];
    __syncthreads();
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
      const double* Yn = Y + (long)n * LY;
      double a = 0.0;
#pragma unroll 9
      for (int t = 0; t < L; ++t) a += Yn[t] * cl[t];
      gg[n] = U[(long)j * N + n] * a;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
      double a = 0.0;
      for (int n = 0; n < N; ++n) a += leb[4 * n + 3] * Y[(long)n * LY + t] * gg[n];
      mu[t] = a;
    }
  } else {
    for (int t = threadIdx.x; t < L; t += blockDim.x) mu[t] = 0.0;
  }
  double accA[L], accB[L];
#pragma unroll
  for (int t = 0; t < L; ++t) { accA[t] = 0.0; accB[t] = 0.0; }
  if (zr) {
    const double xj = xyz[3 * j], yj = xyz[3 * j + 1], zj = xyz[3 * j + 2], rj = rad[j], irj = 1.0 / rj;
    double isg[LM + 1];
#pragma unroll
    for (int l = 0; l <= LM; ++l) isg[l] = 1.0 / sgr[j * LUR + l];
    const int q0 = nptr[j], nq = nptr[j + 1] - q0;
    for (int pidx = threadIdx.x; pidx < nq * N; pidx += blockDim.x) {
      const int a = pidx / N, n = pidx - a * N;
      const int i = nidx[q0 + a];
      const double vx = (xyz[3 * i] + rad[i] * leb[4 * n] - xj) * irj;
      const double vy = (xyz[3 * i + 1] + rad[i] * leb[4 * n + 1] - yj) * irj;
      const double vz = (xyz[3 * i + 2] + rad[i] * leb[4 * n + 2] - zj) * irj;
      const double t2 = vx * vx + vy * vy + vz * vz;
      if (t2 >= 1.0) continue;
      const double fv = f[(long)i * N + n];
      const double om = (fv > 1.0 ? 1.0 / fv : 1.0) * chi_eta(sqrt(t2), eta);
      if (om == 0.0) continue;
      const double wom = leb[4 * n + 3] * om;
      const double cA = wom * zr[(long)i * N + n], cB = wom * ze[(long)i * N + n];
      double sg[LM + 1];
      sigma_weights<LM, double>(kappa * kappa * rj * rj * t2, nterms, sg);
#pragma unroll
      for (int l = 0; l <= LM; ++l) sg[l] *= cB * isg[l];
      for_each_solid_harmonic<LM, double>(vx, vy, vz, [&](int l, int idx, double S) {
        accA[idx] += cA * S;
        accB[idx] += sg[l] * S;
      });
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
#pragma unroll
  for (int t = 0; t < L; ++t) {
    double a = wave_sum(accA[t]);
    double b = wave_sum(accB[t]);
    if (lane == 0) { red[wid * 2 * L + t] = a; red[wid * 2 * L + L + t] = b; }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < nw; ++w) { a += red[w * 2 * L + t]; b += red[w * 2 * L + L + t]; }
    const int l = deg_of(t);
    const long ir = (long)j * L + t, ie = (long)(M + j) * L + t;
    double orr = c1 * a + ycr[j * LUR + l] * mu[t];
    double oe = c1 * b + yce[j * LUR + l] * mu[t];
    if (base) { orr += c0 * base[ir]; oe += c0 * base[ie]; }
    out[ir] = orr;
    out[ie] = oe;
  }
}

// ---------------------------------------------------------- Krylov helpers
// part[v * nb + b] = sum over block b's range of V[v][k] * w[k]
// Partial dot products of kDotV vectors V[v0 .. v0+kDotV) (stride ldv) with w over one
// chunk of D per block: w is read once for kDotV vectors.  part[v * gridDim.x + block].
constexpr int kDotV = 8;
__global__ __launch_bounds__(256) void k_mdot_part(long D, int nv, const double* __restrict__ V, long ldv,
                                                    const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double sh[kDotV][4];
  const int v0 = blockIdx.y * kDotV, nvb = min(kDotV, nv - v0);
  const long chunk = (D + gridDim.x - 1) / gridDim.x;
  const long k0 = blockIdx.x * chunk, k1 = min(D, k0 + chunk);
  double s[kDotV];
#pragma unroll
  for (int u = 0; u < kDotV; ++u) s[u] = 0.0;
  const double* Vv = V + (long)v0 * ldv;
  for (long k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const double wk = w[k];
#pragma unroll
    for (int u = 0; u < kDotV; ++u)
      if (u < nvb) s[u] += Vv[u * ldv + k] * wk;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;  // blockDim.x == 256
#pragma unroll
  for (int u = 0; u < kDotV; ++u) {
    const double t = wave_sum(s[u]);
    if (lane == 0) sh[u][wid] = t;
  }
  __syncthreads();
  if (threadIdx.x < nvb)
    part[(long)(v0 + threadIdx.x) * gridDim.x + blockIdx.x] =
        ((sh[threadIdx.x][0] + sh[threadIdx.x][1]) + sh[threadIdx.x][2]) + sh[threadIdx.x][3];
}
__global__ __launch_bounds__(256) void k_mdot_final(int nb, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[16];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[(long)v * nb + b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[v] = s;
}
// w -= sum_v V[v] h[v]
__global__ void k_mupdate(long D, int nv, const double* __restrict__ V, long ldv, const double* __restrict__ h,
                          double* __restrict__ w) {
  long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= D) return;
  double s = w[k];
  for (int v = 0; v < nv; ++v) s -= V[v * ldv + k] * h[v];
  w[k] = s;
}
// per-degree scaling of coefficient rows: out[j][t] = a[j][l] A[j][t] (+ b[j][l] B[j][t]),
// l the degree of t; A (and B) with row stride lda, out with stride L
__global__ void k_deg_scale(int M, int L, int LUR, const double* __restrict__ a, const double* __restrict__ A,
                            const double* __restrict__ b, const double* __restrict__ B, int lda,
                            double* __restrict__ out) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= (long)M * L) return;
  const int j = (int)(k / L), t = (int)(k - (long)j * L), l = deg_of(t);
  double v = a[j * LUR + l] * A[(long)j * lda + t];
  if (b) v += b[j * LUR + l] * B[(long)j * lda + t];
  out[k] = v;
}
// g *= U on the grid
__global__ void k_mul_grid(long MN, const double* __restrict__ U, double* __restrict__ g) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k < MN) g[k] *= U[k];
}
// out_r[j][t] += ycr[j][l] mu[j][t], out_e[j][t] += yce[j][l] mu[j][t]
__global__ void k_lam_out(int M, int L, int LUR, const double* __restrict__ ycr, const double* __restrict__ yce,
                          const double* __restrict__ mu, double* __restrict__ out) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= (long)M * L) return;
  const int j = (int)(k / L), t = (int)(k - (long)j * L), l = deg_of(t);
  out[k] += ycr[j * LUR + l] * mu[k];
  out[(long)M * L + k] += yce[j * LUR + l] * mu[k];
}
// adjoint grid charges from the two syntheses: c_in = w_n U_in (zr_in + ze_in)
__global__ void k_charges_from_syn(long MN, int N, const double* __restrict__ leb, const double* __restrict__ U,
                                   const double* __restrict__ zr, const double* __restrict__ ze,
                                   double* __restrict__ c) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= MN) return;
  const int n = (int)(k % N);
  c[k] = leb[4 * n + 3] * U[k] * (zr[k] + ze[k]);
}
// out += t at the active points (U > 0); inactive points keep their value
__global__ void k_add_active(long MN, const double* __restrict__ U, const double* __restrict__ t,
                             double* __restrict__ out) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= MN) return;
  if (U[k] > 0.0) out[k] += t[k];
}
// y = a x + b y
__global__ void k_axpby(long D, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k < D) y[k] = a * x[k] + b * y[k];
}
// out = (g_r - g_e, 0) [mode 0] or (g_e, g_e) [mode 1] for g = (g_r, g_e), ML entries per half
__global__ void k_rhs_parts(long ML, int mode, const double* __restrict__ g, double* __restrict__ out) {
  long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= ML) return;
  if (mode == 0) {
    out[k] = g[k] - g[ML + k];
    out[ML + k] = 0.0;
  } else {
    out[k] = g[ML + k];
    out[ML + k] = g[ML + k];
  }
}
// y = sum_v V[v] c[v]
// Per-block maxima of |a - b| (b may be null: |a|) and |s + a| (s may be null: |a|):
// part[2 block], part[2 block + 1]; grid-stride, 256 threads.
__global__ __launch_bounds__(256) void k_amax2(long D, const double* __restrict__ a, const double* __restrict__ b,
                                               const double* __restrict__ s, double* __restrict__ part) {
  __shared__ double sh[2][256];
  double m1 = 0.0, m2 = 0.0;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < D; k += 256L * gridDim.x) {
    const double av = a[k];
    m1 = fmax(m1, fabs(b ? av - b[k] : av));
    m2 = fmax(m2, fabs(s ? s[k] + av : av));
  }
  sh[0][threadIdx.x] = m1;
  sh[1][threadIdx.x] = m2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + w]);
      sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0];
    part[2 * blockIdx.x + 1] = sh[1][0];
  }
}

__global__ void k_mcomb(long D, int nv, const double* __restrict__ V, long ldv, const double* __restrict__ c,
                        double* __restrict__ y) {
  long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= D) return;
  double s = 0.0;
  for (int v = 0; v < nv; ++v) s += V[v * ldv + k] * c[v];
  y[k] = s;
}

// E = sum_j q_j X_r,j00 / (2 sqrt(4 pi))   (Sec. 3 energy equation, psi_r(x_j) = X_r,j00 Y_00)
__global__ __launch_bounds__(1024) void k_energy(int M, int L, const double* __restrict__ X, const double* __restrict__ q,
                                                 double* __restrict__ out) {
  __shared__ double sh[32];
  Comp acc;  // compensated: M terms of both signs
  for (int j = threadIdx.x; j < M; j += blockDim.x) acc.add(q[j] * X[(long)j * L]);
  const double s = block_sum_comp(acc, sh);
  if (threadIdx.x == 0) out[0] = s * 0.14104739588693907;  // 1/(2 sqrt(4 pi))
}

}  // namespace ddlpb

namespace ddlpb {

// ------------------------------------------------------------ cap lists
// Caps: (i, n, j) with |x_i^n - x_j| < r_j, stored per sphere i sorted by (n, j):
// cap_n, cap_slot (position of j in N_i), cap_w (omega_ij(x_i^n)); per-point ranges pcp[i*(N+1)+n].
// Reverse caps per sphere j: (i, n, omega) with j in N_i, sorted by (i, n).
__global__ void k_caps_fill(int M, int N, const double* __restrict__ xyz, const double* __restrict__ rad,
                            const double* __restrict__ leb, const int* __restrict__ nptr, const int* __restrict__ nidx,
                            const double* __restrict__ f, double eta, const int* __restrict__ cptr,
                            int* __restrict__ cap_n, int* __restrict__ cap_slot, double* __restrict__ cap_w,
                            int* __restrict__ pcp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  int c = cptr[i];
  for (int n = 0; n < N; ++n) {
    pcp[(long)i * (N + 1) + n] = c;
    const double px = xyz[3 * i] + rad[i] * leb[4 * n], py = xyz[3 * i + 1] + rad[i] * leb[4 * n + 1],
                 pz = xyz[3 * i + 2] + rad[i] * leb[4 * n + 2];
    const double fv = f[(long)i * N + n];
    const double dfac = fv > 1.0 ? 1.0 / fv : 1.0;
    for (int a = nptr[i]; a < nptr[i + 1]; ++a) {
      const int j = nidx[a];
      const double dx = px - xyz[3 * j], dy = py - xyz[3 * j + 1], dz = pz - xyz[3 * j + 2];
      const double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 < rad[j] * rad[j]) {
        cap_n[c] = n;
        cap_slot[c] = a - nptr[i];
        cap_w[c] = dfac * chi_eta(sqrt(d2) / rad[j], eta);
        ++c;
      }
    }
  }
  pcp[(long)i * (N + 1) + N] = c;
}
// reverse caps: count per j then fill (deterministic order: i ascending in N_j, then n)
__global__ void k_rcaps_count(int M, int N, const double* __restrict__ xyz, const double* __restrict__ rad,
                              const double* __restrict__ leb, const int* __restrict__ nptr,
                              const int* __restrict__ nidx, int* __restrict__ cnt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int c = 0;
  for (int a = nptr[j]; a < nptr[j + 1]; ++a) {
    const int i = nidx[a];
    for (int n = 0; n < N; ++n) {
      const double dx = xyz[3 * i] + rad[i] * leb[4 * n] - xyz[3 * j], dy = xyz[3 * i + 1] + rad[i] * leb[4 * n + 1] - xyz[3 * j + 1],
                   dz = xyz[3 * i + 2] + rad[i] * leb[4 * n + 2] - xyz[3 * j + 2];
      c += (dx * dx + dy * dy + dz * dz < rad[j] * rad[j]);
    }
  }
  cnt[j] = c;
}
__global__ void k_rcaps_fill(int M, int N, const double* __restrict__ xyz, const double* __restrict__ rad,
                             const double* __restrict__ leb, const int* __restrict__ nptr, const int* __restrict__ nidx,
                             const double* __restrict__ f, double eta, const int* __restrict__ rptr,
                             int* __restrict__ rc_i, int* __restrict__ rc_n, double* __restrict__ rc_w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int c = rptr[j];
  for (int a = nptr[j]; a < nptr[j + 1]; ++a) {
    const int i = nidx[a];
    for (int n = 0; n < N; ++n) {
      const double dx = xyz[3 * i] + rad[i] * leb[4 * n] - xyz[3 * j], dy = xyz[3 * i + 1] + rad[i] * leb[4 * n + 1] - xyz[3 * j + 1],
                   dz = xyz[3 * i + 2] + rad[i] * leb[4 * n + 2] - xyz[3 * j + 2];
      const double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 < rad[j] * rad[j]) {
        const double fv = f[(long)i * N + n];
        rc_i[c] = i;
        rc_n[c] = n;
        rc_w[c] = (fv > 1.0 ? 1.0 / fv : 1.0) * chi_eta(sqrt(d2) / rad[j], eta);
        ++c;
      }
    }
  }
}

// Position in the reverse lists of every forward cap: the reverse cap (j; i, n) is the
// forward cap of point (i, n) whose neighbour slot names j.  found counts the matches
// (the host checks that every cap was matched).
__global__ void k_cap_perm(int M, int N, const int* __restrict__ nptr, const int* __restrict__ nidx,
                           const int* __restrict__ rptr, const int* __restrict__ rc_i, const int* __restrict__ rc_n,
                           const int* __restrict__ pcp, const int* __restrict__ cap_slot, int* __restrict__ f2r,
                           int* __restrict__ found) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int cnt = 0;
  for (int r = rptr[j]; r < rptr[j + 1]; ++r) {
    const int i = rc_i[r], n = rc_n[r];
    const long pp = (long)i * (N + 1) + n;
    for (int f = pcp[pp]; f < pcp[pp + 1]; ++f)
      if (nidx[nptr[i] + cap_slot[f]] == j) {
        f2r[f] = r;
        ++cnt;
        break;
      }
  }
  atomicAdd(found, cnt);
}

// Point values of the near part from the per-cap values of the lane kernel: for every
// grid point, the sum over its caps in forward-list order, plus the grid terms
// (U (gr1 + gr2) and U ge, scaled by cg); Vpt [2M][N] is the input of the An GEMM.
__global__ void k_point_sums(int M, int N, const int* __restrict__ pcp, const int* __restrict__ f2r,
                             const double* __restrict__ capv, double c1, const double* __restrict__ U,
                             const double* __restrict__ gr1, const double* __restrict__ gr2,
                             const double* __restrict__ ge, double cg, double* __restrict__ Vpt) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long MN = (long)M * N;
  if (idx >= MN) return;
  const int i = (int)(idx / N), n = (int)(idx - (long)i * N);
  double a = 0.0, b = 0.0;
  if (capv) {
    const long pp = (long)i * (N + 1) + n;
    for (int f = pcp[pp]; f < pcp[pp + 1]; ++f) {
      const double2 v = *reinterpret_cast<const double2*>(capv + 2L * f2r[f]);
      a += v.x;
      b += v.y;
    }
  }
  const double u = U[idx];
  const double gR = gr1 ? u * (gr1[idx] + (gr2 ? gr2[idx] : 0.0)) : 0.0;
  const double gE = ge ? u * ge[idx] : 0.0;
  Vpt[idx] = c1 * a + cg * gR;
  Vpt[MN + idx] = c1 * b + cg * gE;
}


// ------------------------------------------- apply L (near part) from cap lists
// Same result as k_apply_LX: one block per sphere i.  Each cap is evaluated by four
// lanes (the harmonic columns m = q mod 4 of lane q, see solid_harmonic_quad) and
// reduced across them; the coefficients of up to kNbrLds neighbours and the
// recurrence constants are staged in LDS; per-point sums are taken in cap order
// (deterministic), then the An transforms.  Dynamic LDS: k_apply_LX_caps_lds().
constexpr int kCapChunk = 512;
constexpr int kNbrLds = 16;
// LDS entries (of the compute type) of k_apply_LX_caps
template <int LM>
__host__ __device__ constexpr size_t k_apply_LX_caps_lds_entries(int N) {
  return 4 * (size_t)N + 2 * kCapChunk + (size_t)kNbrLds * 2 * (LM + 1) * (LM + 1) + (LM + 1) + (LM + 1) * (LM + 2);
}
// R: compute type (double, or float on the mixed path); inputs and outputs are FP64
template <int LM, class R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_apply_LX_caps(int M, int N, int LY, const double* __restrict__ Y,
                                                        const double* __restrict__ leb, const double* __restrict__ xyz,
                                                        const double* __restrict__ rad, const int* __restrict__ nptr,
                                                        const int* __restrict__ nidx, const int* __restrict__ cptr,
                                                        const int* __restrict__ cap_n, const int* __restrict__ cap_slot,
                                                        const double* __restrict__ cap_w, const int* __restrict__ pcp,
                                                        const double* __restrict__ U, const double* __restrict__ isgr,
                                                        int LUR, double kappa, int nterms,
                                                        const double* __restrict__ base, double c0,
                                                        const double* __restrict__ nearX, double c1,
                                                        const double* __restrict__ gr1, const double* __restrict__ gr2,
                                                        const double* __restrict__ ge, double cg,
                                                        double* __restrict__ out, double* __restrict__ Vpt) {
  constexpr int L = (LM + 1) * (LM + 1);
  constexpr int NT = (LM + 1) * (LM + 2) / 2;
  extern __shared__ double sh_raw[];
  R* vA = reinterpret_cast<R*>(sh_raw);
  R* vB = vA + N;
  R* gR = vB + N;
  R* gE = gR + N;
  R* capA = gE + N;
  R* capB = capA + kCapChunk;
  R* sX = capB + kCapChunk;
  R* spmm = sX + kNbrLds * 2 * L;
  R* sra = spmm + (LM + 1);
  R* srb = sra + NT;
  const int i = blockIdx.x;
  const double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2], ri = rad[i];
  const int q0 = nptr[i], K = nptr[i + 1] - q0;
  const bool lds_x = K <= kNbrLds;
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    vA[n] = R(0);
    vB[n] = R(0);
    const double u = U[(long)i * N + n];
    gR[n] = R(gr1 ? u * (gr1[(long)i * N + n] + (gr2 ? gr2[(long)i * N + n] : 0.0)) : 0.0);
    gE[n] = R(ge ? u * ge[(long)i * N + n] : 0.0);
  }
  for (int t = threadIdx.x; t < NT; t += blockDim.x) {
    sra[t] = R(c_ra[t]);
    srb[t] = R(c_rb[t]);
    if (t <= LM) spmm[t] = R(c_pmm[t]);
  }
  if (nearX && lds_x) {
    for (int t = threadIdx.x; t < K * 2 * L; t += blockDim.x) {
      const int a = t / (2 * L), r = t - a * 2 * L;
      const int j = nidx[q0 + a];
      sX[t] = R(r < L ? nearX[(long)j * L + r] : nearX[(long)(M + j) * L + r - L]);
    }
  }
  __syncthreads();
  if (nearX) {
    const int qd = threadIdx.x & 3, nq = blockDim.x >> 2;
    const int c0i = cptr[i], c1i = cptr[i + 1];
    for (int cb = c0i; cb < c1i; cb += kCapChunk) {
      const int ce = min(c1i, cb + kCapChunk);
      for (int c = cb + (threadIdx.x >> 2); c < ce; c += nq) {  // the four lanes of a quad share c
        const int n = cap_n[c], a = cap_slot[c];
        const int j = nidx[q0 + a];
        const double irj = 1.0 / rad[j];
        const R vx = R((xi + ri * leb[4 * n] - xyz[3 * j]) * irj), vy = R((yi + ri * leb[4 * n + 1] - xyz[3 * j + 1]) * irj),
                vz = R((zi + ri * leb[4 * n + 2] - xyz[3 * j + 2]) * irj);
        const R t2 = vx * vx + vy * vy + vz * vz;
        R sg[LM + 1];
        sigma_weights<LM, R>(R(kappa * kappa * rad[j] * rad[j]) * t2, nterms, sg);
        R sa = R(0), sb = R(0), pb[LM + 1];
#pragma unroll
        for (int l = 0; l <= LM; ++l) pb[l] = R(0);
        if (lds_x) {
          const R* Xr = sX + a * 2 * L;
          const R* Xe = Xr + L;
          solid_harmonic_quad<LM, R>(vx, vy, vz, qd, spmm, sra, srb, [&](int l, int idx, R S) {
            sa += Xr[idx] * S;
            pb[l] += Xe[idx] * S;
          });
        } else {
          const double* Xr = nearX + (long)j * L;
          const double* Xe = nearX + (long)(M + j) * L;
          solid_harmonic_quad<LM, R>(vx, vy, vz, qd, spmm, sra, srb, [&](int l, int idx, R S) {
            sa += R(Xr[idx]) * S;
            pb[l] += R(Xe[idx]) * S;
          });
        }
#pragma unroll
        for (int l = 0; l <= LM; ++l) sb += pb[l] * sg[l] * R(isgr[j * LUR + l]);
        sa += __shfl_xor(sa, 1);
        sb += __shfl_xor(sb, 1);
        sa += __shfl_xor(sa, 2);
        sb += __shfl_xor(sb, 2);
        if (qd == 0) {
          const R w = R(cap_w[c]);
          capA[c - cb] = w * sa;
          capB[c - cb] = w * sb;
        }
      }
      __syncthreads();
      for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const int p0 = max(pcp[(long)i * (N + 1) + n], cb), p1 = min(pcp[(long)i * (N + 1) + n + 1], ce);
        R a = R(0), b = R(0);
        for (int c = p0; c < p1; ++c) { a += capA[c - cb]; b += capB[c - cb]; }
        vA[n] += a;
        vB[n] += b;
      }
      __syncthreads();
    }
  }
  if (Vpt) {
    // point values only: the An transforms of all spheres are one GEMM on the host side
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
      Vpt[(long)i * N + n] = c1 * (double)vA[n] + cg * (double)gR[n];
      Vpt[(long)(M + i) * N + n] = c1 * (double)vB[n] + cg * (double)gE[n];
    }
    return;
  }
  // An transforms: the point sum of every coefficient is split over kAnParts thread
  // groups (all threads busy), partial sums combined in LDS (reusing the cap buffers)
  constexpr int kAnParts = 3;
  const bool grid_terms = gr1 != nullptr || ge != nullptr;  // uniform: the single-layer part
  const int nper = (N + kAnParts - 1) / kAnParts;
  R* part = capA;  // [kAnParts][4][L], over capA, capB and sX (no longer used)
  static_assert(kAnParts * 4 * L <= 2 * kCapChunk + kNbrLds * 2 * L, "An partial sums exceed the cap buffers");
  for (int u = threadIdx.x; u < kAnParts * L; u += blockDim.x) {
    const int t = u % L, g = u / L;
    const int n0 = g * nper, n1 = min(N, n0 + nper);
    R sa = R(0), sb = R(0), sr = R(0), se = R(0);
    if (grid_terms) {
      for (int n = n0; n < n1; ++n) {
        const R wy = R(leb[4 * n + 3] * Y[(long)n * LY + t]);
        sa += wy * vA[n];
        sb += wy * vB[n];
        sr += wy * gR[n];
        se += wy * gE[n];
      }
    } else {
      for (int n = n0; n < n1; ++n) {
        const R wy = R(leb[4 * n + 3] * Y[(long)n * LY + t]);
        sa += wy * vA[n];
        sb += wy * vB[n];
      }
    }
    part[(g * 4 + 0) * L + t] = sa;
    part[(g * 4 + 1) * L + t] = sb;
    part[(g * 4 + 2) * L + t] = sr;
    part[(g * 4 + 3) * L + t] = se;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    R sa = R(0), sb = R(0), sr = R(0), se = R(0);
#pragma unroll
    for (int g = 0; g < kAnParts; ++g) {
      sa += part[(g * 4 + 0) * L + t];
      sb += part[(g * 4 + 1) * L + t];
      sr += part[(g * 4 + 2) * L + t];
      se += part[(g * 4 + 3) * L + t];
    }
    const long ir = (long)i * L + t, ie = (long)(M + i) * L + t;
    double orr = c1 * (double)sa + cg * (double)sr, oe = c1 * (double)sb + cg * (double)se;
    if (base) { orr += c0 * base[ir]; oe += c0 * base[ie]; }
    out[ir] = orr;
    out[ie] = oe;
  }
}

// Transposed near part from reverse cap lists (same result as the near part of
// k_apply_LTZ).  One block of 128 threads per sphere j; caps are taken kLtzChunk at a
// time: the four lanes of each cap write its harmonics (columns m = q mod 4) and
// weights to LDS, then one thread per coefficient accumulates over the chunk.
constexpr int kLtzChunk = 32;
template <int LM>
__host__ __device__ constexpr size_t k_apply_LTZ_caps_lds_entries(int N) {
  return (size_t)(N > kLtzChunk * (LM + 1) * (LM + 1) ? N : kLtzChunk * (LM + 1) * (LM + 1)) + 2 * (LM + 1) * (LM + 1) +
         kLtzChunk * (LM + 2) + (LM + 1) + (LM + 1) * (LM + 2);
}
template <int LM, class R>
__global__ __launch_bounds__(128) void k_apply_LTZ_caps(int M, int N, int LY, const double* __restrict__ Y,
                                                         const double* __restrict__ YT,
                                                         const double* __restrict__ leb, const double* __restrict__ xyz,
                                                         const double* __restrict__ rad, const int* __restrict__ rptr,
                                                         const int* __restrict__ rc_i, const int* __restrict__ rc_n,
                                                         const double* __restrict__ rc_w, const double* __restrict__ U,
                                                         const double* __restrict__ isgr, const double* __restrict__ ycr,
                                                         const double* __restrict__ yce, const double* __restrict__ Cl,
                                                         int LUR, double kappa, int nterms,
                                                         const double* __restrict__ base, double c0,
                                                         const double* __restrict__ zr, const double* __restrict__ ze,
                                                         double c1, const double* __restrict__ lam, int LLAM,
                                                         double* __restrict__ out) {
  constexpr int L = (LM + 1) * (LM + 1);
  constexpr int NT = (LM + 1) * (LM + 2) / 2;
  extern __shared__ double sh_raw[];
  R* sh = reinterpret_cast<R*>(sh_raw);
  // the harmonics buffer doubles as the point buffer of the single-layer part
  R* Sb = sh;                                                      // [kLtzChunk][L]
  R* gg = sh;                                                      // [N]
  R* cl = sh + (N > kLtzChunk * L ? N : kLtzChunk * L);            // [L]
  R* mu = cl + L;                                                  // [L]
  R* fA = mu + L;                                                  // [kLtzChunk]
  R* fB = fA + kLtzChunk;                                          // [kLtzChunk][LM+1]
  R* spmm = fB + kLtzChunk * (LM + 1);
  R* sra = spmm + (LM + 1);
  R* srb = sra + NT;
  const int j = blockIdx.x;  // blockDim.x == 128
  for (int t = threadIdx.x; t < NT; t += blockDim.x) {
    sra[t] = R(c_ra[t]);
    srb[t] = R(c_rb[t]);
    if (t <= LM) spmm[t] = R(c_pmm[t]);
  }
  if (lam) {
    for (int t = threadIdx.x; t < L; t += blockDim.x) cl[t] = R(Cl[j * LUR + deg_of(t)] * lam[(long)j * LLAM + t]);
    __syncthreads();
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
      R a = R(0);
      for (int t = 0; t < L; ++t) a += R(YT[(long)t * N + n]) * cl[t];
      gg[n] = R(U[(long)j * N + n]) * a;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
      R a = R(0);
      for (int n = 0; n < N; ++n) a += R(leb[4 * n + 3] * Y[(long)n * LY + t]) * gg[n];
      mu[t] = a;
    }
  } else {
    for (int t = threadIdx.x; t < L; t += blockDim.x) mu[t] = R(0);
  }
  __syncthreads();  // gg is reused as the harmonics buffer
  constexpr int NA = (L + 127) / 128;  // coefficients per thread: threadIdx.x + 128 r
  R accA[NA], accB[NA];
#pragma unroll
  for (int r = 0; r < NA; ++r) { accA[r] = R(0); accB[r] = R(0); }
  if (zr) {
    const double xj = xyz[3 * j], yj = xyz[3 * j + 1], zj = xyz[3 * j + 2], rj = rad[j], irj = 1.0 / rj;
    const int qd = threadIdx.x & 3, cl4 = threadIdx.x >> 2;  // cap of the quad in the chunk
    const int r0 = rptr[j], r1 = rptr[j + 1];
    for (int cb = r0; cb < r1; cb += kLtzChunk) {
      const int cnt = min(kLtzChunk, r1 - cb);
      if (cl4 < cnt) {
        const int c = cb + cl4;
        const int i = rc_i[c], n = rc_n[c];
        const R vx = R((xyz[3 * i] + rad[i] * leb[4 * n] - xj) * irj);
        const R vy = R((xyz[3 * i + 1] + rad[i] * leb[4 * n + 1] - yj) * irj);
        const R vz = R((xyz[3 * i + 2] + rad[i] * leb[4 * n + 2] - zj) * irj);
        if (qd == 0) {
          const R t2 = vx * vx + vy * vy + vz * vz;
          const double wom = leb[4 * n + 3] * rc_w[c];
          const R cB = R(wom * ze[(long)i * N + n]);
          R sg[LM + 1];
          sigma_weights<LM, R>(R(kappa * kappa * rj * rj) * t2, nterms, sg);
          fA[cl4] = R(wom * zr[(long)i * N + n]);
#pragma unroll
          for (int l = 0; l <= LM; ++l) fB[cl4 * (LM + 1) + l] = sg[l] * cB * R(isgr[j * LUR + l]);
        }
        R* Sr = Sb + cl4 * L;
        solid_harmonic_quad<LM, R>(vx, vy, vz, qd, spmm, sra, srb, [&](int, int idx, R S) { Sr[idx] = S; });
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < NA; ++r) {
        const int t = threadIdx.x + 128 * r;
        if (t < L) {
          const int tdeg = deg_of(t);
          for (int c = 0; c < cnt; ++c) {
            const R S = Sb[c * L + t];
            accA[r] += fA[c] * S;
            accB[r] += fB[c * (LM + 1) + tdeg] * S;
          }
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int r = 0; r < NA; ++r) {
    const int t = threadIdx.x + 128 * r;
    if (t >= L) continue;
    const int l = deg_of(t);
    const long ir = (long)j * L + t, ie = (long)(M + j) * L + t;
    double orr = c1 * (double)accA[r] + ycr[j * LUR + l] * (double)mu[t];
    double oe = c1 * (double)accB[r] + yce[j * LUR + l] * (double)mu[t];
    if (base) { orr += c0 * base[ir]; oe += c0 * base[ie]; }
    out[ir] = orr;
    out[ie] = oe;
  }
}

}  // namespace ddlpb
