// Device-side special functions for the ddLPB kernels (gfx950).
//
//  * Regular solid harmonics S_lm(v) = |v|^l Y_lm(v/|v|) of the real orthonormal
//    spherical harmonics (Y_{l,m} ~ cos(m phi) for m > 0, ~ sin(|m| phi) for m < 0,
//    no Condon-Shortley sign, index l*l+l+m), evaluated by a recurrence in
//    Cartesian form so that no direction has to be normalised (a grid point
//    close to another sphere's centre is harmless).
//  * Radial weights of the modified spherical Bessel functions:
//      k-weights  u_l(rho) = k_l(kappa rho) / rho^l   (upward recurrence, stable)
//      i-weights  sigma_l(z^2) = i_l(z) / z^l        (series at the top, downward
//                                                      recurrence, stable)
//  * A forward-mode dual number (value + gradient) for gradients with respect to
//    an evaluation point.
#pragma once
#include <hip/hip_runtime.h>

namespace ddlpb {

constexpr int kLmaxDev = 24;                          // largest degree of the constant tables
constexpr int kTri = (kLmaxDev + 1) * (kLmaxDev + 2) / 2;
__host__ __device__ constexpr int tri(int l, int m) { return l * (l + 1) / 2 + m; }
__host__ __device__ constexpr int lmi(int l, int m) { return l * l + l + m; }

// Normalised Legendre recurrence constants (filled by the host once per device):
//   P_m^m = c_pmm[m],  P_{m+1}^m = c_ra[tri(m+1,m)] z P_m^m,
//   P_l^m = c_ra[tri(l,m)] z P_{l-1}^m - c_rb[tri(l,m)] r^2 P_{l-2}^m
// where P_l^m already carries the normalisation of Y_lm.
__constant__ double c_pmm[kLmaxDev + 1];
__constant__ double c_ra[kTri];
__constant__ double c_rb[kTri];
// the same constants rounded to FP32, for the single-precision kernels of the mixed path
__constant__ float c_pmm_f[kLmaxDev + 1];
__constant__ float c_ra_f[kTri];
__constant__ float c_rb_f[kTri];
// Coefficients of the sigma_l series: c_sinv[l * kSigTerms + k] = 1 / (2 (k+1) (2l+2k+3)).
constexpr int kSigTerms = 64;
__constant__ double c_sinv[(kLmaxDev + 2) * kSigTerms];

// ------------------------------------------------------------------ dual
template <class R>
struct Dual {
  R v, g[3];
  __device__ Dual() {}
  __device__ Dual(R a) : v(a) { g[0] = g[1] = g[2] = R(0); }
};
template <class R> __device__ __forceinline__ Dual<R> operator+(const Dual<R>& a, const Dual<R>& b) { Dual<R> r; r.v = a.v + b.v; for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] + b.g[k]; return r; }
template <class R> __device__ __forceinline__ Dual<R> operator-(const Dual<R>& a, const Dual<R>& b) { Dual<R> r; r.v = a.v - b.v; for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] - b.g[k]; return r; }
template <class R> __device__ __forceinline__ Dual<R> operator*(const Dual<R>& a, const Dual<R>& b) { Dual<R> r; r.v = a.v * b.v; for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k]; return r; }
template <class R> __device__ __forceinline__ Dual<R> operator*(R s, const Dual<R>& a) { Dual<R> r; r.v = s * a.v; for (int k = 0; k < 3; ++k) r.g[k] = s * a.g[k]; return r; }
template <class R> __device__ __forceinline__ Dual<R> operator*(const Dual<R>& a, R s) { return s * a; }
template <class R> __device__ __forceinline__ Dual<R> operator/(const Dual<R>& a, const Dual<R>& b) {
  Dual<R> r; R ib = R(1) / b.v; r.v = a.v * ib;
  for (int k = 0; k < 3; ++k) r.g[k] = (a.g[k] - r.v * b.g[k]) * ib;
  return r;
}
template <class R> __device__ __forceinline__ Dual<R> dsqrt(const Dual<R>& a) {
  Dual<R> r; r.v = sqrt(a.v); R h = R(0.5) / r.v;
  for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] * h;
  return r;
}
template <class R> __device__ __forceinline__ Dual<R> dexp(const Dual<R>& a) {
  Dual<R> r; r.v = exp(a.v);
  for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] * r.v;
  return r;
}
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float dsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double dexp(double a) { return exp(a); }
__device__ __forceinline__ float dexp(float a) { return expf(a); }

template <class T> struct ScalarOf { using type = T; };
template <class R> struct ScalarOf<Dual<R>> { using type = R; };

// ---------------------------------------------------- solid harmonics
// Calls f(l, m_index, S_lm) for every (l,m), l <= LM, in the order m = 0..LM, l = m..LM.
// T may be a scalar or a Dual (then S carries its gradient w.r.t. (x,y,z)).
template <int LM, class T, class F>
__device__ __forceinline__ void for_each_solid_harmonic(const T& x, const T& y, const T& z, F&& f) {
  using R = typename ScalarOf<T>::type;
  const T r2 = x * x + y * y + z * z;
  T cm(R(1)), sm(R(0));
#pragma unroll
  for (int m = 0; m <= LM; ++m) {
    if (m > 0) {
      T c2 = x * cm - y * sm;
      sm = x * sm + y * cm;
      cm = c2;
    }
    T p2(R(0)), p1(R(0));
#pragma unroll
    for (int l = m; l <= LM; ++l) {
      constexpr bool f32 = sizeof(R) == 4;
      const R pmm = f32 ? R(c_pmm_f[m]) : R(c_pmm[m]);
      const R ra = f32 ? R(c_ra_f[tri(l, m)]) : R(c_ra[tri(l, m)]);
      const R rb = f32 ? R(c_rb_f[tri(l, m)]) : R(c_rb[tri(l, m)]);
      T p;
      if (l == m) p = T(pmm);
      else if (l == m + 1) p = ra * (z * p1);
      else p = ra * (z * p1) - rb * (r2 * p2);
      if (m == 0) {
        f(l, lmi(l, 0), p);
      } else {
        f(l, lmi(l, m), p * cm);
        f(l, lmi(l, -m), p * sm);
      }
      p2 = p1;
      p1 = p;
    }
  }
}

// The same harmonics split over four lanes: the lane with q = 0..3 produces the
// columns m = q, q+4, q+8, ... (both signs), in increasing l; pmm/ra/rb are the
// recurrence constants (copies of c_pmm/c_ra/c_rb, e.g. in LDS).
template <int LM, class R, class F>
__device__ __forceinline__ void solid_harmonic_quad(R x, R y, R z, int q, const R* pmm, const R* ra, const R* rb,
                                                    F&& f) {
  constexpr int NC = LM / 4 + 1;
  const R r2 = x * x + y * y + z * z;
  R cq = R(1), sq = R(0);  // (x + i y)^q
  for (int k = 0; k < q; ++k) {
    const R c2 = x * cq - y * sq;
    sq = x * sq + y * cq;
    cq = c2;
  }
  const R c2 = x * x - y * y, s2 = R(2) * x * y;
  const R c4 = c2 * c2 - s2 * s2, s4 = R(2) * c2 * s2;
  R cm[NC], sm[NC], p1[NC], p2[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (k == 0) { cm[0] = cq; sm[0] = sq; }
    else { cm[k] = cm[k - 1] * c4 - sm[k - 1] * s4; sm[k] = cm[k - 1] * s4 + sm[k - 1] * c4; }
    p1[k] = R(0);
    p2[k] = R(0);
  }
#pragma unroll
  for (int l = 0; l <= LM; ++l) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int m = q + 4 * k;
      if (m > l) continue;
      R p;
      if (m == l) p = pmm[m];
      else if (m == l - 1) p = ra[tri(l, m)] * (z * p1[k]);
      else p = ra[tri(l, m)] * (z * p1[k]) - rb[tri(l, m)] * (r2 * p2[k]);
      p2[k] = p1[k];
      p1[k] = p;
      if (m == 0) {
        f(l, l * l + l, p);
      } else {
        f(l, l * l + l + m, p * cm[k]);
        f(l, l * l + l - m, p * sm[k]);
      }
    }
  }
}

// ------------------------------------------------------ Bessel weights
// u_l = k_l(kappa rho) / rho^l for l = 0..LM (k_l = sqrt(pi/(2z)) K_{l+1/2}(z)).
// One division per call: with ir = 1/rho, u_0 = (pi/2) e^{-z} ir / kappa and
// u_1 = (pi/2) e^{-z} (z + 1) ir^3 / kappa^2 (z = kappa rho).
template <int LM, class T>
__device__ __forceinline__ void k_weights(const T& rho, double kappa, T* u) {
  using R = typename ScalarOf<T>::type;
  const R halfpi = R(1.5707963267948966);
  const R ik = R(1.0 / kappa);
  const T ir = T(R(1)) / rho;
  T z = R(kappa) * rho;
  T e = dexp(T(R(0)) - z);
  const T eh = halfpi * (e * ir);
  u[0] = ik * eh;
  T ir2 = ir * ir;
  if (LM >= 1) u[1] = (ik * ik) * ((eh * (z + T(R(1)))) * ir2);
#pragma unroll
  for (int l = 1; l < LM; ++l) u[l + 1] = (u[l - 1] + R((2.0 * l + 1.0) / kappa) * u[l]) * ir2;
}
template <class R> __device__ __forceinline__ Dual<R> operator+(const Dual<R>& a, R s) { Dual<R> r = a; r.v += s; return r; }

// sigma_l(z2) = i_l(z)/z^l, l = 0..LM: series for LM+1 and LM, then
// sigma_{l-1} = z2 sigma_{l+1} + (2l+1) sigma_l.
template <int LM, class T>
__device__ __forceinline__ void sigma_weights(const T& z2, int nterms, T* sg) {
  using R = typename ScalarOf<T>::type;
  T top[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int l = LM + 1 - q;
    double df = 1.0;
    for (int k = 2 * l + 1; k > 1; k -= 2) df *= k;
    T term = T(R(1.0 / df));
    T sum = term;
    for (int k = 0; k < nterms; ++k) {
      const double ck = (l <= kLmaxDev + 1 && k < kSigTerms) ? c_sinv[l * kSigTerms + k]
                                                             : 0.5 / ((k + 1.0) * (2.0 * l + 2.0 * k + 3.0));
      term = (term * z2) * R(ck);
      sum = sum + term;
    }
    top[q] = sum;
  }
  T sp1 = top[0];
  sg[LM] = top[1];
#pragma unroll
  for (int l = LM; l >= 1; --l) {
    T s = z2 * sp1 + R(2.0 * l + 1.0) * sg[l];
    sp1 = sg[l];
    sg[l - 1] = s;
  }
}

// ------------------------------------------------------------ switching
// chi_eta(t): 1 for t <= 1-eta, 0 for t >= 1, C^2 quintic in between; and its derivative.
__device__ __forceinline__ double chi_eta(double t, double eta) {
  if (t <= 1.0 - eta) return 1.0;
  if (t >= 1.0) return 0.0;
  double u = (1.0 - t) / eta;
  return u * u * u * (u * (6.0 * u - 15.0) + 10.0);
}
__device__ __forceinline__ double chi_eta_d(double t, double eta) {
  if (t <= 1.0 - eta || t >= 1.0) return 0.0;
  double u = (1.0 - t) / eta;
  return -30.0 * u * u * (u - 1.0) * (u - 1.0) / eta;
}

// -------------------------------------------------------- reductions
template <class R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// Deterministic block sum (blockDim.x multiple of 64, <= 1024); result valid in all threads.
template <class R>
__device__ __forceinline__ R block_sum(R v, R* sh /* >= 16 entries */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  R t = R(0);
  for (int k = 0; k < nw; ++k) t += sh[k];
  return t;
}

// Compensated FP64 summation (Neumaier): the running sum and, separately, the sum of
// the rounding errors of every addition (each recovered exactly by TwoSum).
struct Comp {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  __device__ __forceinline__ double value() const { return s + c; }
};
// a + b for compensated pairs: TwoSum of the sums, the errors added (commutative, so
// both lanes of a butterfly get the same bits)
__device__ __forceinline__ Comp comp_merge(const Comp& a, const Comp& b) {
  Comp r;
  r.s = a.s + b.s;
  const double bp = r.s - a.s;
  r.c = (a.c + b.c) + ((a.s - (r.s - bp)) + (b.s - bp));
  return r;
}
// Deterministic compensated block sum (blockDim.x multiple of 64, <= 1024); the value
// is valid in all threads.
__device__ __forceinline__ double block_sum_comp(Comp v, double* sh /* >= 32 entries */) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    Comp o;
    o.s = __shfl_xor(v.s, off, 64);
    o.c = __shfl_xor(v.c, off, 64);
    v = comp_merge(v, o);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) { sh[2 * wid] = v.s; sh[2 * wid + 1] = v.c; }
  __syncthreads();
  Comp t;
  for (int k = 0; k < nw; ++k) {
    Comp o;
    o.s = sh[2 * k];
    o.c = sh[2 * k + 1];
    t = comp_merge(t, o);
  }
  return t.value();
}

}  // namespace ddlpb
