// Host-side tables of the ddLPB library: Legendre recurrence constants,
// modified spherical Bessel functions, per-sphere scalars and the gradient
// coupling tables of the single-layer basis.  Everything here is FP64 and runs
// once per context (or once per process for the constant tables).
#pragma once
#include <cmath>
#include <vector>

#include "lebedev_data.h"

namespace ddlpb {
namespace host {

constexpr double kPi = 3.14159265358979323846;

inline int tri(int l, int m) { return l * (l + 1) / 2 + m; }
inline int lmi(int l, int m) { return l * l + l + m; }

// Normalisation of Y_lm: sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) * sqrt(2 if m>0).
inline double ynorm(int l, int m) {
  double lr = 0.0;  // log((l-m)!/(l+m)!)
  for (int k = l - m + 1; k <= l + m; ++k) lr -= std::log((double)k);
  double v = std::log((2.0 * l + 1.0) / (4.0 * kPi)) + lr;
  if (m > 0) v += std::log(2.0);
  return std::exp(0.5 * v);
}

// Constants of the normalised Legendre recurrence used by the device code.
inline void legendre_tables(int lmax, std::vector<double>& pmm, std::vector<double>& ra, std::vector<double>& rb) {
  pmm.assign(lmax + 1, 0.0);
  ra.assign((lmax + 1) * (lmax + 2) / 2, 0.0);
  rb.assign((lmax + 1) * (lmax + 2) / 2, 0.0);
  for (int m = 0; m <= lmax; ++m) {
    double df = 1.0;
    for (int k = 2 * m - 1; k > 1; k -= 2) df *= k;
    pmm[m] = ynorm(m, m) * df;
    for (int l = m + 1; l <= lmax; ++l) {
      ra[tri(l, m)] = (2.0 * l - 1.0) / (l - m) * ynorm(l, m) / ynorm(l - 1, m);
      if (l >= m + 2) rb[tri(l, m)] = (l + m - 1.0) / (l - m) * ynorm(l, m) / ynorm(l - 2, m);
    }
  }
}

// ------------------------------------------------------------ host dual
struct HD {
  double v, g[3];
  HD(double a = 0.0) : v(a), g{0, 0, 0} {}
};
inline HD operator+(HD a, const HD& b) { a.v += b.v; for (int k = 0; k < 3; ++k) a.g[k] += b.g[k]; return a; }
inline HD operator-(HD a, const HD& b) { a.v -= b.v; for (int k = 0; k < 3; ++k) a.g[k] -= b.g[k]; return a; }
inline HD operator*(const HD& a, const HD& b) { HD r; r.v = a.v * b.v; for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k]; return r; }
inline HD operator/(const HD& a, const HD& b) { HD r; r.v = a.v / b.v; for (int k = 0; k < 3; ++k) r.g[k] = (a.g[k] - r.v * b.g[k]) / b.v; return r; }
inline HD hsqrt(const HD& a) { HD r; r.v = std::sqrt(a.v); for (int k = 0; k < 3; ++k) r.g[k] = 0.5 * a.g[k] / r.v; return r; }
inline HD hexp(const HD& a) { HD r; r.v = std::exp(a.v); for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] * r.v; return r; }
inline double hsqrt(double a) { return std::sqrt(a); }
inline double hexp(double a) { return std::exp(a); }

// Solid harmonics S_lm(v) = |v|^l Y_lm(v/|v|) (same convention as the device code).
template <class T>
void solid_harmonics(int lmax, const T& x, const T& y, const T& z, T* S) {
  std::vector<double> pmm, ra, rb;
  legendre_tables(lmax, pmm, ra, rb);
  T r2 = x * x + y * y + z * z;
  T cm(1.0), sm(0.0);
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) { T c2 = x * cm - y * sm; sm = x * sm + y * cm; cm = c2; }
    T p2(0.0), p1(0.0);
    for (int l = m; l <= lmax; ++l) {
      T p;
      if (l == m) p = T(pmm[m]);
      else if (l == m + 1) p = T(ra[tri(l, m)]) * z * p1;
      else p = T(ra[tri(l, m)]) * z * p1 - T(rb[tri(l, m)]) * r2 * p2;
      if (m == 0) S[lmi(l, 0)] = p;
      else { S[lmi(l, m)] = p * cm; S[lmi(l, -m)] = p * sm; }
      p2 = p1; p1 = p;
    }
  }
}

// k_l(z) = sqrt(pi/(2z)) K_{l+1/2}(z) for l = 0..lmax (upward recurrence).
template <class T>
void bessel_k(int lmax, const T& z, T* k) {
  T e = hexp(T(0.0) - z);
  k[0] = T(kPi / 2) * e / z;
  if (lmax >= 1) k[1] = T(kPi / 2) * e * (z + T(1.0)) / (z * z);
  for (int l = 1; l < lmax; ++l) k[l + 1] = k[l - 1] + T(2.0 * l + 1.0) / z * k[l];
}

// sigma_l(z^2) = i_l(z)/z^l for l = 0..lmax: series at degrees lmax+1 and lmax, then
// the downward recurrence sigma_{l-1} = z^2 sigma_{l+1} + (2l+1) sigma_l.
inline void bessel_sigma(int lmax, double z2, double* sg) {
  double top[2];
  for (int q = 0; q < 2; ++q) {
    int l = lmax + 1 - q;
    double df = 1.0;
    for (int k = 2 * l + 1; k > 1; k -= 2) df *= k;
    double term = 1.0 / df, sum = term;
    for (int k = 0; k < 500; ++k) {
      term *= z2 * 0.5 / ((k + 1.0) * (2.0 * l + 2.0 * k + 3.0));
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    top[q] = sum;
  }
  double sp1 = top[0];
  sg[lmax] = top[1];
  for (int l = lmax; l >= 1; --l) {
    double s = z2 * sp1 + (2.0 * l + 1.0) * sg[l];
    sp1 = sg[l];
    sg[l - 1] = s;
  }
}
// number of series terms needed on the device for z^2 <= z2max (relative 1e-17)
inline int sigma_terms(int lmax, double z2max) {
  int l = lmax;
  double df = 1.0;
  for (int k = 2 * l + 1; k > 1; k -= 2) df *= k;
  double term = 1.0 / df, sum = term;
  int k = 0;
  for (; k < 500; ++k) {
    term *= z2max * 0.5 / ((k + 1.0) * (2.0 * l + 2.0 * k + 3.0));
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return k + 2;
}

inline const ddlpb_tables::LebedevRule* lebedev_rule(int npts) {
  for (int k = 0; k < ddlpb_tables::kNumLebedevRules; ++k)
    if (ddlpb_tables::kLebedevRules[k].n == npts) return &ddlpb_tables::kLebedevRules[k];
  return nullptr;
}
inline const ddlpb_tables::LebedevRule* lebedev_rule_min_degree(int deg) {
  for (int k = 0; k < ddlpb_tables::kNumLebedevRules; ++k)
    if (ddlpb_tables::kLebedevRules[k].degree >= deg) return &ddlpb_tables::kLebedevRules[k];
  return nullptr;
}

// Gradient coupling of the decaying basis F_lm(v) = k_l(kappa|v|) Y_lm(v/|v|):
//   d/dv_a F_lm = kappa * sum_{l'm'} d[a][lm][l'm'] F_l'm'   (l' = l +- 1),
// obtained exactly by projecting the gradient (forward-mode dual numbers) on a
// sphere |v| = rho0 onto Y_l'm' with a Lebedev rule of degree >= 2 lmax + 2.
// Output d[3][L][Lp], L = (lmax+1)^2, Lp = (lmax+2)^2.
inline bool gradient_coupling(int lmax, std::vector<double>& d) {
  const int L = (lmax + 1) * (lmax + 1), Lp = (lmax + 2) * (lmax + 2);
  const auto* rule = lebedev_rule_min_degree(2 * lmax + 2);
  if (!rule) return false;
  const double z0 = 1.0;  // kappa rho0; the coefficients do not depend on it
  std::vector<double> kk(lmax + 3);
  bessel_k<double>(lmax + 2, z0, kk.data());
  d.assign((size_t)3 * L * Lp, 0.0);
  std::vector<HD> S(L);
  std::vector<double> Yp(Lp);
  std::vector<HD> kd(lmax + 2);
  for (int n = 0; n < rule->n; ++n) {
    const double* sw = rule->xyzw + 4 * n;
    HD v[3];
    for (int a = 0; a < 3; ++a) { v[a] = HD(z0 * sw[a]); v[a].g[a] = 1.0; }  // kappa = 1 units
    solid_harmonics<HD>(lmax, v[0], v[1], v[2], S.data());
    HD rho = hsqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    bessel_k<HD>(lmax + 1, rho, kd.data());
    solid_harmonics<double>(lmax + 1, sw[0], sw[1], sw[2], Yp.data());
    HD rl(1.0);
    for (int l = 0; l <= lmax; ++l) {
      HD rad = kd[l] / rl;  // k_l(rho)/rho^l
      for (int m = -l; m <= l; ++m) {
        HD F = rad * S[lmi(l, m)];
        for (int a = 0; a < 3; ++a)
          for (int lp = (l > 0 ? l - 1 : 1); lp <= l + 1; lp += 2)
            for (int mp = -lp; mp <= lp; ++mp)
              d[((size_t)a * L + lmi(l, m)) * Lp + lmi(lp, mp)] += sw[3] * F.g[a] * Yp[lmi(lp, mp)] / kk[lp];
      }
      rl = rl * rho;
    }
  }
  for (auto& v : d) if (std::fabs(v) < 1e-13) v = 0.0;
  return true;
}

}  // namespace host
}  // namespace ddlpb
