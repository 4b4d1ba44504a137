// ddLPB oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously-correct FP64 CPU implementation of the discrete
// ddLPB solvation energy, its adjoint solve and its analytical forces
// (Jha, Nottoli, Mikhalev, Quan, Stamm, "Linear scaling computation of forces
// for the domain-decomposition linear Poisson--Boltzmann method").
//
// Only the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark may load this library.  The product path never links it.  It shares
// no code with the HIP implementation: spherical harmonics, Bessel functions,
// switching functions, operators and solvers are all written out here again.
//
// Everything is direct O(M^2) summation; there is no fast multipole method.
// The scalar type is a template parameter so that the same code evaluated in
// std::complex<double> gives complex-step derivatives of the energy, and in a
// small forward-mode dual number type gives gradients of basis functions.
//
// Readings of the paper taken here (each is listed again in the design notes):
//  * Bessel arguments carry kappa: i_l(kappa*|x-x_j|), k_l(kappa*r_j); a prime
//    is d/dr and therefore includes a factor kappa (Sec. 2.2, eqs. for B, C1,
//    C2, Q and the Bessel ratios).
//  * The energy pairs X_r with q_j / sqrt(4 pi) in the (l,m)=(0,0) slot, i.e.
//    E = 1/2 sum_j q_j psi_r(x_j) (Sec. 3, energy equation).
//  * The constant term of the switching polynomial p_eta is 10 eta^2-15 eta+6
//    (Sec. 3.1), which makes chi_eta the C^2 quintic smoothstep.
//  * Lebedev weights sum to 4 pi.
//  * d^i = 1 where f <= 1 (this also covers f = 0 and |N_i| = 0).
//  * Real spherical harmonics: orthonormal, Y_{l,m} ~ cos(m phi) for m > 0,
//    ~ sin(|m| phi) for m < 0, no Condon-Shortley sign (Y_{1,1} ~ +x).
//    Index l*l + l + m.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <vector>
#include <algorithm>

namespace {

using cplx = std::complex<double>;

// ------------------------------------------------------------ scalar helpers
inline double re(double x) { return x; }
inline double re(const cplx& x) { return x.real(); }

// Forward-mode dual number with a 3-vector of derivatives (used for gradients
// of basis functions with respect to the evaluation point).
struct D3 {
  double v, d[3];
  D3() : v(0), d{0, 0, 0} {}
  D3(double a) : v(a), d{0, 0, 0} {}
};
inline double re(const D3& x) { return x.v; }
inline D3 operator+(const D3& a, const D3& b) { D3 r; r.v = a.v + b.v; for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
inline D3 operator-(const D3& a, const D3& b) { D3 r; r.v = a.v - b.v; for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
inline D3 operator-(const D3& a) { D3 r; r.v = -a.v; for (int k = 0; k < 3; ++k) r.d[k] = -a.d[k]; return r; }
inline D3 operator*(const D3& a, const D3& b) { D3 r; r.v = a.v * b.v; for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
inline D3 operator/(const D3& a, const D3& b) { D3 r; r.v = a.v / b.v; for (int k = 0; k < 3; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v); return r; }
inline D3& operator+=(D3& a, const D3& b) { a = a + b; return a; }
inline D3& operator-=(D3& a, const D3& b) { a = a - b; return a; }
inline D3& operator*=(D3& a, const D3& b) { a = a * b; return a; }
inline D3 operator*(double s, const D3& a) { D3 r; r.v = s * a.v; for (int k = 0; k < 3; ++k) r.d[k] = s * a.d[k]; return r; }
inline D3 operator*(const D3& a, double s) { return s * a; }
inline D3 operator/(const D3& a, double s) { return (1.0 / s) * a; }
inline D3 operator/(double s, const D3& a) { return D3(s) / a; }
inline D3 operator+(const D3& a, double s) { D3 r = a; r.v += s; return r; }
inline D3 operator-(double s, const D3& a) { D3 r = -a; r.v += s; return r; }
inline D3 sqrt(const D3& a) { D3 r; r.v = std::sqrt(a.v); for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] / (2.0 * r.v); return r; }
inline D3 exp(const D3& a) { D3 r; r.v = std::exp(a.v); for (int k = 0; k < 3; ++k) r.d[k] = a.d[k] * r.v; return r; }
using std::sqrt;
using std::exp;

inline double absre(double x) { return std::fabs(x); }
inline double absre(const cplx& x) { return std::abs(x); }
inline double absre(const D3& x) { return std::fabs(x.v); }

const double PI = 3.14159265358979323846;

inline int lm_index(int l, int m) { return l * l + l + m; }
const int LMAX_ORACLE = 30;  // largest degree the fixed-size work arrays allow

// ------------------------------------------------ real spherical harmonics
// Regular solid harmonics S_lm(v) = |v|^l Y_lm(v/|v|), a polynomial in (x,y,z):
//   S_lm = N_lm * Pi_l^|m|(z, r^2) * {Re (x+iy)^m | Im (x+iy)^|m| | 1}
// with Pi_l^m = r^{l-m} d^m P_l/dmu^m (mu = z/r), obtained from the Legendre
// recurrence (l-m) Pi_l^m = (2l-1) z Pi_{l-1}^m - (l+m-1) r^2 Pi_{l-2}^m,
// Pi_m^m = (2m-1)!!, and N_lm = sqrt((2l+1)/(4pi) * 2 (l-m)!/(l+m)!) for m > 0,
// sqrt((2l+1)/(4pi)) for m = 0.
double norm_lm(int l, int m) {
  double f = 1.0;  // (l-m)!/(l+m)!
  for (int k = l - m + 1; k <= l + m; ++k) f /= k;
  double n = (2.0 * l + 1.0) / (4.0 * PI) * f;
  if (m > 0) n *= 2.0;
  return std::sqrt(n);
}

template <class T>
void solid_harmonics(int lmax, const T& x, const T& y, const T& z, T* S) {
  T r2 = x * x + y * y + z * z;
  T Cm[LMAX_ORACLE + 2], Sm[LMAX_ORACLE + 2], Pi[LMAX_ORACLE + 2];
  Cm[0] = T(1.0);
  Sm[0] = T(0.0);
  for (int m = 1; m <= lmax; ++m) {
    Cm[m] = x * Cm[m - 1] - y * Sm[m - 1];
    Sm[m] = x * Sm[m - 1] + y * Cm[m - 1];
  }
  for (int m = 0; m <= lmax; ++m) {
    double dfact = 1.0;  // (2m-1)!!
    for (int k = 2 * m - 1; k > 1; k -= 2) dfact *= k;
    Pi[m] = T(dfact);
    if (m + 1 <= lmax) Pi[m + 1] = (2.0 * m + 1.0) * z * Pi[m];
    for (int l = m + 2; l <= lmax; ++l)
      Pi[l] = ((2.0 * l - 1.0) * z * Pi[l - 1] - (l + m - 1.0) * r2 * Pi[l - 2]) / double(l - m);
    for (int l = m; l <= lmax; ++l) {
      double nlm = norm_lm(l, m);
      if (m == 0) {
        S[lm_index(l, 0)] = nlm * Pi[l];
      } else {
        S[lm_index(l, m)] = nlm * Pi[l] * Cm[m];
        S[lm_index(l, -m)] = nlm * Pi[l] * Sm[m];
      }
    }
  }
}

// Y_lm(v/|v|) for a unit (or any non-zero) vector.
void sph_harm_unit(int lmax, const double* v, double* Y) {
  double r = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  solid_harmonics<double>(lmax, v[0] / r, v[1] / r, v[2] / r, Y);
}

// ------------------------------------------------------ Bessel functions
// sigma_l(z^2) = i_l(z) / z^l = sum_k (z^2/2)^k / (k! (2l+2k+1)!!)   (power series
// of the modified spherical Bessel function of the first kind).
template <class T>
T sigma_l(int l, const T& z2) {
  double df = 1.0;
  for (int k = 2 * l + 1; k > 1; k -= 2) df *= k;
  T term = T(1.0 / df);
  T sum = term;
  for (int k = 0; k < 400; ++k) {
    term = term * z2 * (0.5 / ((k + 1.0) * (2.0 * l + 2.0 * k + 3.0)));
    sum = sum + term;
    if (absre(term) <= 1e-18 * absre(sum)) break;
  }
  return sum;
}

// i_l(z) for z > 0 (real, or complex with a tiny imaginary part for complex steps).
template <class T>
T sph_i(int l, const T& z) { return std::pow(z, l) * sigma_l<T>(l, z * z); }

// k_l(z) = sqrt(pi/(2z)) K_{l+1/2}(z), l = 0..lmax, by the stable upward
// recurrence k_{l+1} = k_{l-1} + (2l+1)/z k_l.
template <class T>
void sph_k_all(int lmax, const T& z, T* k) {
  T e = exp(T(0.0) - z);
  k[0] = (PI / 2.0) * e / z;
  if (lmax >= 1) k[1] = (PI / 2.0) * e * (z + 1.0) / (z * z);
  for (int l = 1; l + 1 <= lmax; ++l) k[l + 1] = k[l - 1] + (2.0 * l + 1.0) / z * k[l];
}
template <class T>
T sph_k(int l, const T& z) {
  std::vector<T> k(l + 2);
  sph_k_all<T>(l + 1, z, k.data());
  return k[l];
}
// Derivatives (d/dz):  i_l' = i_{l+1} + (l/z) i_l,   k_l' = -k_{l+1} + (l/z) k_l.
template <class T>
T sph_i_prime(int l, const T& z) { return sph_i(l + 1, z) + double(l) / z * sph_i(l, z); }
template <class T>
T sph_k_prime(int l, const T& z) { return T(0.0) - sph_k(l + 1, z) + double(l) / z * sph_k(l, z); }

// ------------------------------------------------------ switching function
// p_eta(t) = eta^-5 (1-t)^3 (6 t^2 + (15 eta - 12) t + 10 eta^2 - 15 eta + 6)
template <class T>
T chi_eta(const T& t, double eta) {
  if (re(t) <= 1.0 - eta) return T(1.0);
  if (re(t) >= 1.0) return T(0.0);
  T a = 1.0 - t;
  return std::pow(eta, -5.0) * a * a * a * (6.0 * t * t + (15.0 * eta - 12.0) * t + (10.0 * eta * eta - 15.0 * eta + 6.0));
}
// d chi_eta / dt
double chi_eta_prime(double t, double eta) {
  if (t <= 1.0 - eta || t >= 1.0) return 0.0;
  double a = 1.0 - t;
  double poly = 6.0 * t * t + (15.0 * eta - 12.0) * t + (10.0 * eta * eta - 15.0 * eta + 6.0);
  double dpoly = 12.0 * t + 15.0 * eta - 12.0;
  return std::pow(eta, -5.0) * (-3.0 * a * a * poly + a * a * a * dpoly);
}

// ---------------------------------------------------------------- problem
template <class T>
struct Problem {
  int M, lmax, L, N;
  std::vector<T> x;             // [M][3] centres
  std::vector<T> r;             // radii (complex for complex-step derivatives in r)
  std::vector<double> q;        // charges
  double eps1, eps2, kappa, eta;
  std::vector<double> s, w;     // Lebedev points [N][3], weights [N]
  std::vector<double> Y;        // Y_lm(s_n)  [N][L]
  std::vector<T> Cl, Dl;        // C_l^j, i_l'(r_j)/i_l(r_j)  [M][lmax+1]
  std::vector<T> sig_r;         // sigma_l(kappa^2 r_j^2)     [M][lmax+1]
  std::vector<T> k_r;           // k_l(kappa r_j)             [M][lmax+1]
  std::vector<std::vector<int>> nbr;  // N_i
  // grid fields
  std::vector<T> xg;            // grid points x_i^n [M][N][3]
  std::vector<T> f, U;          // f^i(x_i^n), chi^eta_i(x_i^n) [M][N]

  void init(int M_, const double* x_, const double* r_, const double* q_, double e1, double e2,
            double kap, double et, int lmax_, int N_, const double* s_, const double* w_) {
    M = M_; lmax = lmax_; L = (lmax + 1) * (lmax + 1); N = N_;
    x.resize(3 * M);
    for (int k = 0; k < 3 * M; ++k) x[k] = T(x_[k]);
    r.resize(M);
    for (int k = 0; k < M; ++k) r[k] = T(r_[k]);
    q.assign(q_, q_ + M);
    eps1 = e1; eps2 = e2; kappa = kap; eta = et;
    s.assign(s_, s_ + 3 * N);
    w.assign(w_, w_ + N);
    Y.resize((size_t)N * L);
    for (int n = 0; n < N; ++n) sph_harm_unit(lmax, &s[3 * n], &Y[(size_t)n * L]);
    radial_constants();
  }
  // per-sphere constants of the radii (Sec. 2.2): C_l^j, i_l'/i_l, sigma_l and k_l at r_j
  void radial_constants() {
    Cl.resize((size_t)M * (lmax + 1));
    Dl.resize((size_t)M * (lmax + 1));
    sig_r.resize((size_t)M * (lmax + 1));
    k_r.resize((size_t)M * (lmax + 1));
    for (int j = 0; j < M; ++j) {
      T z = kappa * r[j];
      for (int l = 0; l <= lmax; ++l) {
        T di = kappa * sph_i_prime(l, z) / sph_i(l, z);   // i_l'(r_j)/i_l(r_j), d/dr
        T dk = kappa * sph_k_prime(l, z) / sph_k(l, z);   // k_l'(r_j)/k_l(r_j), d/dr
        Cl[j * (lmax + 1) + l] = 1.0 / (di - dk);
        Dl[j * (lmax + 1) + l] = di;
        sig_r[j * (lmax + 1) + l] = sigma_l<T>(l, z * z);
        k_r[j * (lmax + 1) + l] = sph_k(l, z);
      }
    }
  }

  // Neighbour sets: spheres whose balls intersect (decided on real parts).
  void build_neighbours() {
    nbr.assign(M, {});
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        if (i == j) continue;
        double d2 = 0;
        for (int a = 0; a < 3; ++a) { double dd = re(x[3 * i + a]) - re(x[3 * j + a]); d2 += dd * dd; }
        if (std::sqrt(d2) < re(r[i]) + re(r[j])) nbr[i].push_back(j);
      }
  }

  // t = r_1^j(x) = |x - x_j| / r_j
  T tval(const T* p, int j) const {
    T dx = p[0] - x[3 * j], dy = p[1] - x[3 * j + 1], dz = p[2] - x[3 * j + 2];
    return sqrt(dx * dx + dy * dy + dz * dz) / r[j];
  }

  // Grid points and the regularised switching fields (Sec. 3.1).
  void build_grid() {
    xg.resize((size_t)M * N * 3);
    f.assign((size_t)M * N, T(0.0));
    U.assign((size_t)M * N, T(0.0));
    for (int i = 0; i < M; ++i)
      for (int n = 0; n < N; ++n) {
        T* p = &xg[((size_t)i * N + n) * 3];
        for (int a = 0; a < 3; ++a) p[a] = x[3 * i + a] + r[i] * s[3 * n + a];
        T fs = T(0.0);
        for (int j : nbr[i]) fs = fs + chi_eta(tval(p, j), eta);
        f[(size_t)i * N + n] = fs;
        U[(size_t)i * N + n] = (re(fs) < 1.0) ? T(1.0) - fs : T(0.0);  // 1 - min(f,1)
      }
  }
  // d^i = min(f,1)/f
  T dfac(size_t in) const { return (re(f[in]) > 1.0) ? T(1.0) / f[in] : T(1.0); }
  T omega(int i, int n, int j) const {
    const T* p = &xg[((size_t)i * N + n) * 3];
    return dfac((size_t)i * N + n) * chi_eta(tval(p, j), eta);
  }

  // --- basis functions of sphere j evaluated at a point p (Sec. 2.2):
  // A basis: r_l^j(p) Y_lm^j(p) = S_lm(p - x_j) / r_j^l
  template <class S_>
  void basisA(int j, const S_* p, S_* out) const {
    S_ v[3];
    for (int a = 0; a < 3; ++a) v[a] = p[a] - S_(re_or(x[3 * j + a]));
    solid_harmonics<S_>(lmax, v[0], v[1], v[2], out);
    for (int l = 0; l <= lmax; ++l) {
      T sc = std::pow(r[j], -l);
      for (int m = -l; m <= l; ++m) out[lm_index(l, m)] = out[lm_index(l, m)] * sc;
    }
  }
  // B basis: i_l(kappa d)/i_l(kappa r_j) Y_lm^j(p) = S_lm(v)/r_j^l * sigma_l(kappa^2 d^2)/sigma_l(kappa^2 r_j^2)
  template <class S_>
  void basisB(int j, const S_* p, S_* out) const {
    S_ v[3];
    for (int a = 0; a < 3; ++a) v[a] = p[a] - S_(re_or(x[3 * j + a]));
    solid_harmonics<S_>(lmax, v[0], v[1], v[2], out);
    S_ d2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    for (int l = 0; l <= lmax; ++l) {
      S_ sc = std::pow(r[j], -l) * sigma_l<S_>(l, kappa * kappa * d2) / sig_r[j * (lmax + 1) + l];
      for (int m = -l; m <= l; ++m) out[lm_index(l, m)] = out[lm_index(l, m)] * sc;
    }
  }
  // single-layer basis: k_l(kappa rho)/k_l(kappa r_j) Y_lm^j(p) = k_l(kappa rho)/rho^l S_lm(v)/k_l(kappa r_j)
  template <class S_>
  void basisK(int j, const S_* p, S_* out) const {
    S_ v[3];
    for (int a = 0; a < 3; ++a) v[a] = p[a] - S_(re_or(x[3 * j + a]));
    solid_harmonics<S_>(lmax, v[0], v[1], v[2], out);
    S_ rho = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    S_ k[LMAX_ORACLE + 2];
    sph_k_all<S_>(lmax, kappa * rho, k);
    S_ rl = S_(1.0);
    for (int l = 0; l <= lmax; ++l) {
      S_ sc = k[l] / (rl * k_r[j * (lmax + 1) + l]);
      for (int m = -l; m <= l; ++m) out[lm_index(l, m)] = out[lm_index(l, m)] * sc;
      rl = rl * rho;
    }
  }
  // The basis functions above are templated on the evaluation type S_ which is
  // either T itself or D3 (then the centre is taken as a constant).
  static double re_or(const double& a) { return a; }
  static cplx re_or(const cplx& a) { return a; }

  // An_i(v)_lm = sum_n w_n Y_lm(s_n) v_n ;  Syn(c)_n = sum_lm Y_lm(s_n) c_lm
  void An(const T* v, T* c) const {
    for (int lm = 0; lm < L; ++lm) {
      T acc = T(0.0);
      for (int n = 0; n < N; ++n) acc = acc + w[n] * Y[(size_t)n * L + lm] * v[n];
      c[lm] = acc;
    }
  }
  void Syn(const T* c, T* v) const {
    for (int n = 0; n < N; ++n) {
      T acc = T(0.0);
      for (int lm = 0; lm < L; ++lm) acc = acc + Y[(size_t)n * L + lm] * c[lm];
      v[n] = acc;
    }
  }
  int lof(int lm) const { int l = 0; while ((l + 1) * (l + 1) <= lm) ++l; return l; }

  // Vacuum potential psi_0 and its normal derivative at grid point (i,n):
  // psi_0(x) = sum_k q_k / (eps1 |x - x_k|)
  void psi0_at(int i, int n, T& psi, T& dn) const {
    const T* p = &xg[((size_t)i * N + n) * 3];
    psi = T(0.0); dn = T(0.0);
    for (int k = 0; k < M; ++k) {
      T v[3];
      for (int a = 0; a < 3; ++a) v[a] = p[a] - x[3 * k + a];
      T d = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      psi = psi + q[k] / (eps1 * d);
      T vs = v[0] * s[3 * n] + v[1] * s[3 * n + 1] + v[2] * s[3 * n + 2];
      dn = dn - q[k] * vs / (eps1 * d * d * d);
    }
  }

  // Phi[m](x_i^n) = sum_j sum_lm m_jlm k_l^j(x) Y_lm^j(x), evaluated where U > 0.
  void single_layer_field(const std::vector<T>& m, std::vector<T>& Phi) const {
    Phi.assign((size_t)M * N, T(0.0));
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < M; ++i) {
      std::vector<T> b(L);
      for (int n = 0; n < N; ++n) {
        size_t in = (size_t)i * N + n;
        if (!(re(U[in]) > 0.0)) continue;
        T acc = T(0.0);
        for (int j = 0; j < M; ++j) {
          basisK<T>(j, &xg[in * 3], b.data());
          for (int lm = 0; lm < L; ++lm) acc = acc + m[(size_t)j * L + lm] * b[lm];
        }
        Phi[in] = acc;
      }
    }
  }
  // lambda_jlm = sum_{i,n} c_in k_l^j(x_i^n) Y_lm^j(x_i^n)  (transpose of the above)
  void single_layer_adjoint(const std::vector<T>& c, std::vector<T>& lam) const {
    lam.assign((size_t)M * L, T(0.0));
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < M; ++j) {
      std::vector<T> b(L);
      for (int i = 0; i < M; ++i)
        for (int n = 0; n < N; ++n) {
          size_t in = (size_t)i * N + n;
          if (!(re(U[in]) > 0.0)) continue;
          basisK<T>(j, &xg[in * 3], b.data());
          for (int lm = 0; lm < L; ++lm) lam[(size_t)j * L + lm] = lam[(size_t)j * L + lm] + c[in] * b[lm];
        }
    }
  }
  // m_j = C^j (.) An_j(U_j (.) h_j)   for a grid function h
  void single_layer_moments(const std::vector<T>& h, std::vector<T>& m) const {
    m.assign((size_t)M * L, T(0.0));
    std::vector<T> v(N);
    for (int j = 0; j < M; ++j) {
      for (int n = 0; n < N; ++n) v[n] = U[(size_t)j * N + n] * h[(size_t)j * N + n];
      An(v.data(), &m[(size_t)j * L]);
      for (int lm = 0; lm < L; ++lm) m[(size_t)j * L + lm] = m[(size_t)j * L + lm] * Cl[j * (lmax + 1) + lof(lm)];
    }
  }

  // ---------------------------------------------------------- right-hand side
  // g = (G0 + F0, F0) with G0_i = -An_i(U psi0),
  // F0_i = -(eps1/eps2) An_i(U sum_j S_ji) = -An_i(U Phi[C (.) An(U e)]), e = (eps1/eps2) d_n psi0.
  void rhs(std::vector<T>& g, std::vector<T>* e_out = nullptr) const {
    std::vector<T> psi((size_t)M * N, T(0.0)), e((size_t)M * N, T(0.0));
    for (int i = 0; i < M; ++i)
      for (int n = 0; n < N; ++n) {
        size_t in = (size_t)i * N + n;
        if (!(re(U[in]) > 0.0)) continue;
        T p0, dn;
        psi0_at(i, n, p0, dn);
        psi[in] = p0;
        e[in] = (eps1 / eps2) * dn;
      }
    std::vector<T> m0, Phi;
    single_layer_moments(e, m0);
    single_layer_field(m0, Phi);
    g.assign((size_t)2 * M * L, T(0.0));
    std::vector<T> v(N), c(L);
    for (int i = 0; i < M; ++i) {
      for (int n = 0; n < N; ++n) v[n] = -U[(size_t)i * N + n] * psi[(size_t)i * N + n];
      An(v.data(), c.data());  // G0
      for (int lm = 0; lm < L; ++lm) g[(size_t)i * L + lm] = c[lm];
      for (int n = 0; n < N; ++n) v[n] = -U[(size_t)i * N + n] * Phi[(size_t)i * N + n];
      An(v.data(), c.data());  // F0
      for (int lm = 0; lm < L; ++lm) {
        g[(size_t)i * L + lm] = g[(size_t)i * L + lm] + c[lm];
        g[(size_t)(M + i) * L + lm] = c[lm];
      }
    }
    if (e_out) *e_out = e;
  }

  // ------------------------------------------------- matrix-free operator L
  // y_j = (eps1/eps2)(l/r_j) X_r,j - (i_l'(r_j)/i_l(r_j)) X_e,j ; the C-part of L X is
  // CX_i = An_i(U_i Phi[m]) with m_j = C^j (.) An_j(U_j Syn(y_j)).
  // part: 0 = L, 1 = L_AB = [A 0; 0 B] only, 2 = L_C = [C1 C2; C1 C2] only (Sec. 4 splitting)
  void apply(const T* X, T* Yo, int part = 0) const {
    const T* Xr = X;
    const T* Xe = X + (size_t)M * L;
    std::vector<T> h((size_t)M * N), yv(L), m, Phi;
    for (int j = 0; j < M; ++j) {
      for (int lm = 0; lm < L; ++lm) {
        int l = lof(lm);
        yv[lm] = (eps1 / eps2) * (double(l) / r[j]) * Xr[(size_t)j * L + lm] - Dl[j * (lmax + 1) + l] * Xe[(size_t)j * L + lm];
      }
      Syn(yv.data(), &h[(size_t)j * N]);
    }
    if (part != 1) {
      single_layer_moments(h, m);
      single_layer_field(m, Phi);
    } else {
      Phi.assign((size_t)M * N, T(0.0));
    }
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < M; ++i) {
      std::vector<T> vA(N, T(0.0)), vB(N, T(0.0)), vC(N), b(L), c(L);
      for (int n = 0; n < N; ++n) {
        const T* p = &xg[((size_t)i * N + n) * 3];
        for (int j : nbr[i]) {
          T om = omega(i, n, j);
          if (re(om) == 0.0) continue;
          basisA<T>(j, p, b.data());
          T a = T(0.0);
          for (int lm = 0; lm < L; ++lm) a = a + Xr[(size_t)j * L + lm] * b[lm];
          basisB<T>(j, p, b.data());
          T bb = T(0.0);
          for (int lm = 0; lm < L; ++lm) bb = bb + Xe[(size_t)j * L + lm] * b[lm];
          vA[n] = vA[n] + om * a;
          vB[n] = vB[n] + om * bb;
        }
        vC[n] = U[(size_t)i * N + n] * Phi[(size_t)i * N + n];
      }
      std::vector<T> cA(L), cB(L), cC(L);
      An(vA.data(), cA.data());
      An(vB.data(), cB.data());
      An(vC.data(), cC.data());
      const double sAB = part == 2 ? 0.0 : 1.0;
      for (int lm = 0; lm < L; ++lm) {
        Yo[(size_t)i * L + lm] = sAB * (Xr[(size_t)i * L + lm] - cA[lm]) + cC[lm];
        Yo[(size_t)(M + i) * L + lm] = sAB * (Xe[(size_t)i * L + lm] - cB[lm]) + cC[lm];
      }
    }
  }

  // Transposed operator L^T = [A^T 0; 0 B^T] + [C1^T C1^T; C2^T C2^T].
  void apply_T(const T* Z, T* W, int part = 0) const {
    const T* Zr = Z;
    const T* Ze = Z + (size_t)M * L;
    // C-part: zeta = Z_r + Z_e;  c_in = w_n U_in Syn(zeta_i)_n ; lambda = K^T c;
    // mu_j = An_j(U_j Syn(C^j (.) lambda_j)) ; C1^T zeta = a (.) mu, C2^T zeta = b (.) mu
    std::vector<T> c((size_t)M * N), zeta(L), lam;
    for (int i = 0; i < M; ++i) {
      for (int lm = 0; lm < L; ++lm) zeta[lm] = Zr[(size_t)i * L + lm] + Ze[(size_t)i * L + lm];
      Syn(zeta.data(), &c[(size_t)i * N]);
      for (int n = 0; n < N; ++n) c[(size_t)i * N + n] = w[n] * U[(size_t)i * N + n] * c[(size_t)i * N + n];
    }
    if (part != 1) single_layer_adjoint(c, lam); else lam.assign((size_t)M * L, T(0.0));
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < M; ++j) {
      std::vector<T> cl(L), g(N), mu(L), b(L), accA(L, T(0.0)), accB(L, T(0.0)), zi(N), ze(N);
      for (int lm = 0; lm < L; ++lm) cl[lm] = Cl[j * (lmax + 1) + lof(lm)] * lam[(size_t)j * L + lm];
      Syn(cl.data(), g.data());
      for (int n = 0; n < N; ++n) g[n] = U[(size_t)j * N + n] * g[n];
      An(g.data(), mu.data());
      // A^T and B^T: gather from the spheres i that have j as a neighbour
      for (int i : nbr[j]) {
        Syn(&Zr[(size_t)i * L], zi.data());
        Syn(&Ze[(size_t)i * L], ze.data());
        for (int n = 0; n < N; ++n) {
          T om = omega(i, n, j);
          if (re(om) == 0.0) continue;
          const T* p = &xg[((size_t)i * N + n) * 3];
          basisA<T>(j, p, b.data());
          for (int lm = 0; lm < L; ++lm) accA[lm] = accA[lm] + w[n] * om * zi[n] * b[lm];
          basisB<T>(j, p, b.data());
          for (int lm = 0; lm < L; ++lm) accB[lm] = accB[lm] + w[n] * om * ze[n] * b[lm];
        }
      }
      for (int lm = 0; lm < L; ++lm) {
        int l = lof(lm);
        T a = (eps1 / eps2) * (double(l) / r[j]);
        T bb = T(0.0) - Dl[j * (lmax + 1) + l];
        const double sAB = part == 2 ? 0.0 : 1.0;
        W[(size_t)j * L + lm] = sAB * (Zr[(size_t)j * L + lm] - accA[lm]) + a * mu[lm];
        W[(size_t)(M + j) * L + lm] = sAB * (Ze[(size_t)j * L + lm] - accB[lm]) + bb * mu[lm];
      }
    }
  }

  // ------------------------------------- literal dense assembly (small M only)
  // Builds L and g entry by entry from the matrix definitions of Sec. 2.2
  // (A, B, C1, C2 through Q and P chi, G0, F0 through S and c0).
  void assemble_dense(std::vector<T>& Lm, std::vector<T>& g) const {
    const size_t ML = (size_t)M * L, D = 2 * ML;
    Lm.assign(D * D, T(0.0));
    for (size_t a = 0; a < D; ++a) Lm[a * D + a] = T(1.0);
    std::vector<T> b(L);
    // A_ij, B_ij (i != j)
    for (int i = 0; i < M; ++i)
      for (int j : nbr[i])
        for (int n = 0; n < N; ++n) {
          T om = omega(i, n, j);
          if (re(om) == 0.0) continue;
          const T* p = &xg[((size_t)i * N + n) * 3];
          std::vector<T> bA(L), bB(L);
          basisA<T>(j, p, bA.data());
          basisB<T>(j, p, bB.data());
          for (int lm = 0; lm < L; ++lm)
            for (int lp = 0; lp < L; ++lp) {
              T wy = w[n] * om * Y[(size_t)n * L + lm];
              Lm[((size_t)i * L + lm) * D + (size_t)j * L + lp] -= wy * bA[lp];
              Lm[(ML + (size_t)i * L + lm) * D + ML + (size_t)j * L + lp] -= wy * bB[lp];
            }
        }
    // P chi_j, then Q [M L][M N]
    std::vector<T> P((size_t)M * L * L, T(0.0));
    for (int j = 0; j < M; ++j)
      for (int a = 0; a < L; ++a)
        for (int c = 0; c < L; ++c) {
          T acc = T(0.0);
          for (int n = 0; n < N; ++n) acc = acc + w[n] * U[(size_t)j * N + n] * Y[(size_t)n * L + a] * Y[(size_t)n * L + c];
          P[((size_t)j * L + a) * L + c] = acc;
        }
    std::vector<T> Q((size_t)M * L * M * N, T(0.0));
    for (int j = 0; j < M; ++j)
      for (int i = 0; i < M; ++i)
        for (int n = 0; n < N; ++n) {
          size_t in = (size_t)i * N + n;
          if (!(re(U[in]) > 0.0)) continue;  // Q only enters multiplied by chi^e_i(x_i^n)
          basisK<T>(j, &xg[in * 3], b.data());
          for (int lp = 0; lp < L; ++lp) {
            T acc = T(0.0);
            for (int l0 = 0; l0 < L; ++l0)
              acc = acc + Cl[j * (lmax + 1) + lof(l0)] * P[((size_t)j * L + l0) * L + lp] * b[l0];
            Q[((size_t)j * L + lp) * (M * N) + in] = acc;
          }
        }
    // C1, C2
    for (int i = 0; i < M; ++i)
      for (int lm = 0; lm < L; ++lm)
        for (int j = 0; j < M; ++j)
          for (int lp = 0; lp < L; ++lp) {
            T acc = T(0.0);
            for (int n = 0; n < N; ++n) {
              size_t in = (size_t)i * N + n;
              acc = acc + w[n] * U[in] * Y[(size_t)n * L + lm] * Q[((size_t)j * L + lp) * (M * N) + in];
            }
            int l = lof(lp);
            T c1 = (eps1 / eps2) * acc * (double(l) / r[j]);
            T c2 = -acc * Dl[j * (lmax + 1) + l];
            size_t row_r = (size_t)i * L + lm, row_e = ML + row_r;
            size_t col_r = (size_t)j * L + lp, col_e = ML + col_r;
            Lm[row_r * D + col_r] += c1;
            Lm[row_r * D + col_e] += c2;
            Lm[row_e * D + col_r] += c1;
            Lm[row_e * D + col_e] += c2;
          }
    // right-hand side: G0, c0, S, F0
    std::vector<T> psi((size_t)M * N, T(0.0)), dn((size_t)M * N, T(0.0));
    for (int i = 0; i < M; ++i)
      for (int n = 0; n < N; ++n) {
        size_t in = (size_t)i * N + n;
        if (!(re(U[in]) > 0.0)) continue;
        psi0_at(i, n, psi[in], dn[in]);
      }
    std::vector<T> c0((size_t)M * L, T(0.0));
    for (int j = 0; j < M; ++j)
      for (int a = 0; a < L; ++a) {
        T acc = T(0.0);
        for (int n = 0; n < N; ++n) acc = acc + w[n] * U[(size_t)j * N + n] * dn[(size_t)j * N + n] * Y[(size_t)n * L + a];
        c0[(size_t)j * L + a] = acc;
      }
    std::vector<T> Ssum((size_t)M * N, T(0.0));
    for (int i = 0; i < M; ++i)
      for (int n = 0; n < N; ++n) {
        size_t in = (size_t)i * N + n;
        if (!(re(U[in]) > 0.0)) continue;
        T acc = T(0.0);
        for (int j = 0; j < M; ++j) {
          basisK<T>(j, &xg[in * 3], b.data());
          for (int a = 0; a < L; ++a) acc = acc + Cl[j * (lmax + 1) + lof(a)] * c0[(size_t)j * L + a] * b[a];
        }
        Ssum[in] = acc;
      }
    g.assign(D, T(0.0));
    for (int i = 0; i < M; ++i)
      for (int lm = 0; lm < L; ++lm) {
        T G0 = T(0.0), F0 = T(0.0);
        for (int n = 0; n < N; ++n) {
          size_t in = (size_t)i * N + n;
          G0 = G0 - w[n] * U[in] * psi[in] * Y[(size_t)n * L + lm];
          F0 = F0 + w[n] * U[in] * Y[(size_t)n * L + lm] * Ssum[in];
        }
        F0 = -(eps1 / eps2) * F0;
        g[(size_t)i * L + lm] = G0 + F0;
        g[ML + (size_t)i * L + lm] = F0;
      }
  }
};

// ------------------------------------------------------------ linear algebra
// Dense LU with partial pivoting, solves A x = b in place (A is n x n row-major).
template <class T>
int lu_solve(int n, std::vector<T> A, std::vector<T>& b) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = absre(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = absre(A[(size_t)i * n + k]);
      if (v > best) { best = v; p = i; }
    }
    if (best == 0.0) return -1;
    if (p != k) {
      for (int c = 0; c < n; ++c) std::swap(A[(size_t)k * n + c], A[(size_t)p * n + c]);
      std::swap(b[k], b[p]);
    }
    T piv = A[(size_t)k * n + k];
#pragma omp parallel for
    for (int i = k + 1; i < n; ++i) {
      T fct = A[(size_t)i * n + k] / piv;
      if (absre(fct) == 0.0) continue;
      for (int c = k + 1; c < n; ++c) A[(size_t)i * n + c] -= fct * A[(size_t)k * n + c];
      b[i] -= fct * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    T acc = b[k];
    for (int c = k + 1; c < n; ++c) acc -= A[(size_t)k * n + c] * b[c];
    b[k] = acc / A[(size_t)k * n + k];
  }
  return 0;
}

// Restarted GMRES(m) with modified Gram-Schmidt, no preconditioner, stops when
// ||b - A x|| <= tol ||b||.  x holds the initial guess on entry.
template <class Op>
int gmres(size_t n, const Op& op, const std::vector<double>& b, std::vector<double>& x, double tol,
          int restart, int maxit, int* iters) {
  double bn = 0;
  for (double v : b) bn += v * v;
  bn = std::sqrt(bn);
  if (bn == 0.0) { std::fill(x.begin(), x.end(), 0.0); if (iters) *iters = 0; return 0; }
  std::vector<double> r(n), Ax(n);
  int total = 0;
  while (total < maxit) {
    op(x.data(), Ax.data());
    for (size_t k = 0; k < n; ++k) r[k] = b[k] - Ax[k];
    double beta = 0;
    for (double v : r) beta += v * v;
    beta = std::sqrt(beta);
    if (beta <= tol * bn) break;
    std::vector<std::vector<double>> V(1, std::vector<double>(n));
    for (size_t k = 0; k < n; ++k) V[0][k] = r[k] / beta;
    std::vector<std::vector<double>> H(restart + 1, std::vector<double>(restart, 0.0));
    std::vector<double> cs(restart), sn(restart), gvec(restart + 1, 0.0);
    gvec[0] = beta;
    int j = 0;
    for (; j < restart && total < maxit; ++j, ++total) {
      std::vector<double> wv(n);
      op(V[j].data(), wv.data());
      for (int i = 0; i <= j; ++i) {
        double h = 0;
        for (size_t k = 0; k < n; ++k) h += wv[k] * V[i][k];
        H[i][j] = h;
        for (size_t k = 0; k < n; ++k) wv[k] -= h * V[i][k];
      }
      double hn = 0;
      for (double v : wv) hn += v * v;
      hn = std::sqrt(hn);
      H[j + 1][j] = hn;
      V.emplace_back(n);
      if (hn > 0) for (size_t k = 0; k < n; ++k) V[j + 1][k] = wv[k] / hn;
      for (int i = 0; i < j; ++i) {
        double t = cs[i] * H[i][j] + sn[i] * H[i + 1][j];
        H[i + 1][j] = -sn[i] * H[i][j] + cs[i] * H[i + 1][j];
        H[i][j] = t;
      }
      double den = std::sqrt(H[j][j] * H[j][j] + H[j + 1][j] * H[j + 1][j]);
      cs[j] = H[j][j] / den;
      sn[j] = H[j + 1][j] / den;
      H[j][j] = den;
      H[j + 1][j] = 0;
      gvec[j + 1] = -sn[j] * gvec[j];
      gvec[j] = cs[j] * gvec[j];
      if (std::fabs(gvec[j + 1]) <= tol * bn) { ++j; ++total; break; }
    }
    std::vector<double> yv(j);
    for (int i = j - 1; i >= 0; --i) {
      double acc = gvec[i];
      for (int c = i + 1; c < j; ++c) acc -= H[i][c] * yv[c];
      yv[i] = acc / H[i][i];
    }
    for (int i = 0; i < j; ++i)
      for (size_t k = 0; k < n; ++k) x[k] += yv[i] * V[i][k];
  }
  // final residual check
  op(x.data(), Ax.data());
  double rn = 0;
  for (size_t k = 0; k < n; ++k) rn += (b[k] - Ax[k]) * (b[k] - Ax[k]);
  if (iters) *iters = total;
  return std::sqrt(rn) <= tol * bn * 1.0001 ? 0 : 1;
}

// Flexible GMRES(m) (right preconditioned, the preconditioned directions stored)
// with modified Gram-Schmidt; stops when ||b - A x|| <= tol ||b||.  The
// preconditioner is any approximate inverse, here an inner solve of the sparse
// part L_AB = [A 0; 0 B], the paper's preconditioner for the coupled system
// (Sec. 4, opening: L_AB approximates L and is cheap to invert).  It changes the
// iteration count only; the iterate still satisfies the same residual test.
template <class Op, class Prec>
int fgmres(size_t n, const Op& op, const Prec& prec, const std::vector<double>& b, std::vector<double>& x,
           double tol, int restart, int maxit, int* iters) {
  double bn = 0;
  for (double v : b) bn += v * v;
  bn = std::sqrt(bn);
  if (bn == 0.0) { std::fill(x.begin(), x.end(), 0.0); if (iters) *iters = 0; return 0; }
  std::vector<double> r(n), Ax(n);
  int total = 0;
  while (total < maxit) {
    op(x.data(), Ax.data());
    for (size_t k = 0; k < n; ++k) r[k] = b[k] - Ax[k];
    double beta = 0;
    for (double v : r) beta += v * v;
    beta = std::sqrt(beta);
    if (beta <= tol * bn) break;
    std::vector<std::vector<double>> V(1, std::vector<double>(n)), Z;
    for (size_t k = 0; k < n; ++k) V[0][k] = r[k] / beta;
    std::vector<std::vector<double>> H(restart + 1, std::vector<double>(restart, 0.0));
    std::vector<double> cs(restart), sn(restart), gvec(restart + 1, 0.0);
    gvec[0] = beta;
    int j = 0;
    for (; j < restart && total < maxit; ++j, ++total) {
      Z.emplace_back(n);
      prec(V[j].data(), Z[j].data());
      std::vector<double> wv(n);
      op(Z[j].data(), wv.data());
      for (int i = 0; i <= j; ++i) {
        double h = 0;
        for (size_t k = 0; k < n; ++k) h += wv[k] * V[i][k];
        H[i][j] = h;
        for (size_t k = 0; k < n; ++k) wv[k] -= h * V[i][k];
      }
      double hn = 0;
      for (double v : wv) hn += v * v;
      hn = std::sqrt(hn);
      H[j + 1][j] = hn;
      V.emplace_back(n);
      if (hn > 0) for (size_t k = 0; k < n; ++k) V[j + 1][k] = wv[k] / hn;
      for (int i = 0; i < j; ++i) {
        double t = cs[i] * H[i][j] + sn[i] * H[i + 1][j];
        H[i + 1][j] = -sn[i] * H[i][j] + cs[i] * H[i + 1][j];
        H[i][j] = t;
      }
      double den = std::sqrt(H[j][j] * H[j][j] + H[j + 1][j] * H[j + 1][j]);
      cs[j] = H[j][j] / den;
      sn[j] = H[j + 1][j] / den;
      H[j][j] = den;
      H[j + 1][j] = 0;
      gvec[j + 1] = -sn[j] * gvec[j];
      gvec[j] = cs[j] * gvec[j];
      if (std::fabs(gvec[j + 1]) <= tol * bn) { ++j; ++total; break; }
    }
    std::vector<double> yv(j);
    for (int i = j - 1; i >= 0; --i) {
      double acc = gvec[i];
      for (int c = i + 1; c < j; ++c) acc -= H[i][c] * yv[c];
      yv[i] = acc / H[i][i];
    }
    for (int i = 0; i < j; ++i)
      for (size_t k = 0; k < n; ++k) x[k] += yv[i] * Z[i][k];
  }
  op(x.data(), Ax.data());
  double rn = 0;
  for (size_t k = 0; k < n; ++k) rn += (b[k] - Ax[k]) * (b[k] - Ax[k]);
  if (iters) *iters = total;
  return std::sqrt(rn) <= tol * bn * 1.0001 ? 0 : 1;
}

// ------------------------------------------------------------------ forces
// Gradient of the energy via the adjoint method (Sec. 3, force equation):
// dE = 1/2 < dg - dL X , X_adj >.  With X and X_adj frozen this is the gradient
// of
//   E_f = 1/2 sum_i sum_n w_n [ xi_r sum_j omega_ij vA_j + xi_e sum_j omega_ij vB_j
//                               - U (xi_r psi0 + xi_s Phi[m(e, y)]) ]
// (xi = Syn(X_adj), xi_s = xi_r + xi_e, m(e,y)_j = C^j (.) An_j(U_j (e_j + Syn y_j))),
// which collects the terms of Sec. 3.1: derivatives of omega (three cases), of
// the A/B basis (radial, Bessel and angular parts), of chi^eta (C-part and RHS),
// of Q through k_l, Y_lm and P chi, of psi_0 and of d_n psi_0.
void forces(const Problem<double>& P, const std::vector<double>& X, const std::vector<double>& Xa,
            std::vector<double>& grad_out) {
  const int M = P.M, N = P.N, L = P.L, lmax = P.lmax;
  const double eta = P.eta;
  std::vector<double> xr((size_t)M * N), xe((size_t)M * N), xs((size_t)M * N);
  for (int i = 0; i < M; ++i) {
    P.Syn(&Xa[(size_t)i * L], &xr[(size_t)i * N]);
    P.Syn(&Xa[(size_t)(M + i) * L], &xe[(size_t)i * N]);
    for (int n = 0; n < N; ++n) xs[(size_t)i * N + n] = xr[(size_t)i * N + n] + xe[(size_t)i * N + n];
  }
  // psi0, grad psi0 at U>0 points ; e = (eps1/eps2) d_n psi0 ; h = e + Syn(y)
  std::vector<double> psi((size_t)M * N, 0.0), e((size_t)M * N, 0.0), h((size_t)M * N, 0.0);
  for (int i = 0; i < M; ++i)
    for (int n = 0; n < N; ++n) {
      size_t in = (size_t)i * N + n;
      if (!(P.U[in] > 0.0)) continue;
      double p0, dn;
      P.psi0_at(i, n, p0, dn);
      psi[in] = p0;
      e[in] = (P.eps1 / P.eps2) * dn;
    }
  std::vector<double> yv(L);
  for (int j = 0; j < M; ++j) {
    for (int lm = 0; lm < L; ++lm) {
      int l = P.lof(lm);
      yv[lm] = (P.eps1 / P.eps2) * (double(l) / P.r[j]) * X[(size_t)j * L + lm] - P.Dl[j * (lmax + 1) + l] * X[(size_t)(M + j) * L + lm];
    }
    P.Syn(yv.data(), &h[(size_t)j * N]);
    for (int n = 0; n < N; ++n) h[(size_t)j * N + n] += e[(size_t)j * N + n];
  }
  std::vector<double> m, Phi, lam, c((size_t)M * N, 0.0);
  P.single_layer_moments(h, m);
  P.single_layer_field(m, Phi);
  for (size_t in = 0; in < (size_t)M * N; ++in) c[in] = P.w[in % N] * P.U[in] * xs[in];
  P.single_layer_adjoint(c, lam);
  std::vector<double> eta_g((size_t)M * N), cl(L);
  for (int j = 0; j < M; ++j) {
    for (int lm = 0; lm < L; ++lm) cl[lm] = P.Cl[j * (lmax + 1) + P.lof(lm)] * lam[(size_t)j * L + lm];
    P.Syn(cl.data(), &eta_g[(size_t)j * N]);
  }

  std::vector<double> grad((size_t)M * 3, 0.0);
#pragma omp parallel
  {
    std::vector<double> gl((size_t)M * 3, 0.0);
    std::vector<double> bA(L), bB(L);
    std::vector<D3> dA(L), dB(L), dK(L);
#pragma omp for schedule(dynamic)
    for (int i = 0; i < M; ++i) {
      for (int n = 0; n < N; ++n) {
        const size_t in = (size_t)i * N + n;
        const double* p = &P.xg[in * 3];
        const double wn = P.w[n];
        const double fv = P.f[in], Uv = P.U[in], dv = P.dfac(in);
        const double dd = (fv > 1.0) ? -1.0 / (fv * fv) : 0.0;  // d'(f)
        const auto& nb = P.nbr[i];
        const int K = (int)nb.size();
        std::vector<double> tk(K), ch(K), chp(K), V(K, 0.0), ek(3 * K);
        double S1 = 0.0;
        for (int a = 0; a < K; ++a) {
          int k = nb[a];
          double v[3], d2 = 0;
          for (int q = 0; q < 3; ++q) { v[q] = p[q] - P.x[3 * k + q]; d2 += v[q] * v[q]; }
          double d = std::sqrt(d2);
          for (int q = 0; q < 3; ++q) ek[3 * a + q] = v[q] / d;  // e^k(x_i^n)
          tk[a] = d / P.r[k];
          ch[a] = chi_eta(tk[a], eta);
          chp[a] = chi_eta_prime(tk[a], eta);
          if (ch[a] != 0.0 || chp[a] != 0.0) {
            P.basisA<double>(k, p, bA.data());
            P.basisB<double>(k, p, bB.data());
            double va = 0, vb = 0;
            for (int lm = 0; lm < L; ++lm) { va += X[(size_t)k * L + lm] * bA[lm]; vb += X[(size_t)(M + k) * L + lm] * bB[lm]; }
            V[a] = xr[in] * va + xe[in] * vb;
          }
          S1 += ch[a] * V[a];
        }
        const double W = (Uv > 0.0) ? psi[in] * xr[in] + Phi[in] * xs[in] : 0.0;
        for (int a = 0; a < K; ++a) {
          if (chp[a] == 0.0) continue;
          int k = nb[a];
          // omega_ij = d chi_j : d omega_ij/dt_k = d'(f) chi_k' chi_j + d chi_j' delta_jk
          double dT = 0.5 * wn * (dd * chp[a] * S1 + dv * chp[a] * V[a]);
          // U = 1 - min(f,1): dU/dt_k = -chi_k' where f < 1
          if (Uv > 0.0) dT += 0.5 * wn * (W + h[in] * eta_g[in]) * chp[a];
          for (int q = 0; q < 3; ++q) {
            double gq = dT * ek[3 * a + q] / P.r[k];  // dt_k/dx_i^n = e^k/r_k
            gl[3 * i + q] += gq;
            gl[3 * k + q] -= gq;
          }
        }
        // near-field basis derivatives (radial, Bessel, angular): omega grad v
        for (int a = 0; a < K; ++a) {
          if (ch[a] == 0.0) continue;
          int k = nb[a];
          double om = dv * ch[a];
          D3 pd[3];
          for (int q = 0; q < 3; ++q) { pd[q] = D3(p[q]); pd[q].d[q] = 1.0; }
          P.basisA<D3>(k, pd, dA.data());
          P.basisB<D3>(k, pd, dB.data());
          for (int q = 0; q < 3; ++q) {
            double gv = 0;
            for (int lm = 0; lm < L; ++lm) gv += xr[in] * X[(size_t)k * L + lm] * dA[lm].d[q] + xe[in] * X[(size_t)(M + k) * L + lm] * dB[lm].d[q];
            double gq = 0.5 * wn * om * gv;
            gl[3 * i + q] += gq;
            gl[3 * k + q] -= gq;
          }
        }
        if (!(Uv > 0.0)) continue;
        // psi_0 and d_n psi_0 as functions of the point and the charge positions
        for (int k = 0; k < M; ++k) {
          if (k == i) continue;  // x_i^n - x_i = r_i s_n does not move
          double v[3], d2 = 0;
          for (int q = 0; q < 3; ++q) { v[q] = p[q] - P.x[3 * k + q]; d2 += v[q] * v[q]; }
          double d = std::sqrt(d2), d3 = d2 * d, d5 = d3 * d2;
          const double* sn = &P.s[3 * n];
          double vs = v[0] * sn[0] + v[1] * sn[1] + v[2] * sn[2];
          for (int q = 0; q < 3; ++q) {
            double gpsi = -P.q[k] * v[q] / (P.eps1 * d3);                                  // grad psi0 from k
            double hess = P.q[k] / P.eps2 * (3.0 * v[q] * vs / d5 - sn[q] / d3);           // grad (eps1/eps2) d_n psi0 from k
            double gq = -0.5 * wn * Uv * (xr[in] * gpsi + eta_g[in] * hess);
            gl[3 * i + q] += gq;
            gl[3 * k + q] -= gq;
          }
        }
        // single-layer field at fixed moments: x_i^n - x_j for j != i
        D3 pd[3];
        for (int q = 0; q < 3; ++q) { pd[q] = D3(p[q]); pd[q].d[q] = 1.0; }
        for (int j = 0; j < M; ++j) {
          if (j == i) continue;
          P.basisK<D3>(j, pd, dK.data());
          for (int q = 0; q < 3; ++q) {
            double gv = 0;
            for (int lm = 0; lm < L; ++lm) gv += m[(size_t)j * L + lm] * dK[lm].d[q];
            double gq = -0.5 * wn * Uv * xs[in] * gv;
            gl[3 * i + q] += gq;
            gl[3 * j + q] -= gq;
          }
        }
      }
    }
#pragma omp critical
    for (size_t k = 0; k < gl.size(); ++k) grad[k] += gl[k];
  }
  grad_out = grad;
}

template <class T>
Problem<T> make_problem(int M, const double* x, const double* r, const double* q, double e1, double e2,
                        double kap, double eta, int lmax, int N, const double* s, const double* w) {
  Problem<T> P;
  P.init(M, x, r, q, e1, e2, kap, eta, lmax, N, s, w);
  P.build_neighbours();
  P.build_grid();
  return P;
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

// Real orthonormal spherical harmonics Y_lm(v/|v|) for n vectors; out [n][(lmax+1)^2].
void oracle_sph_harm(int lmax, int n, const double* v, double* out) {
  int L = (lmax + 1) * (lmax + 1);
  for (int k = 0; k < n; ++k) sph_harm_unit(lmax, v + 3 * k, out + (size_t)k * L);
}
// i_l(z), k_l(z), i_l'(z), k_l'(z) for l = 0..lmax; out [4][lmax+1].
void oracle_bessel(int lmax, double z, double* out) {
  for (int l = 0; l <= lmax; ++l) {
    out[l] = sph_i(l, z);
    out[(lmax + 1) + l] = sph_k(l, z);
    out[2 * (lmax + 1) + l] = sph_i_prime(l, z);
    out[3 * (lmax + 1) + l] = sph_k_prime(l, z);
  }
}
// chi_eta(t), chi_eta'(t) for n values of t; out [2][n].
void oracle_switch(double eta, int n, const double* t, double* out) {
  for (int k = 0; k < n; ++k) {
    out[k] = chi_eta<double>(t[k], eta);
    out[n + k] = chi_eta_prime(t[k], eta);
  }
}

#define ORACLE_ARGS int M, const double *x, const double *r, const double *q, double eps1, double eps2, \
    double kappa, double eta, int lmax, int N, const double *s, const double *w
#define ORACLE_PASS M, x, r, q, eps1, eps2, kappa, eta, lmax, N, s, w

// Per-sphere constants C_l^j and i_l'(r_j)/i_l(r_j); out [2][M][lmax+1].
void oracle_sphere_constants(ORACLE_ARGS, double* out) {
  auto P = make_problem<double>(ORACLE_PASS);
  size_t K = (size_t)M * (lmax + 1);
  for (size_t k = 0; k < K; ++k) { out[k] = P.Cl[k]; out[K + k] = P.Dl[k]; }
}

// Grid fields f^i(x_i^n) and chi^eta_i(x_i^n); out [2][M][N].  Also neighbour counts [M].
void oracle_grid_fields(ORACLE_ARGS, double* fout, double* Uout, int* nnbr) {
  auto P = make_problem<double>(ORACLE_PASS);
  for (size_t k = 0; k < (size_t)M * N; ++k) { fout[k] = P.f[k]; Uout[k] = P.U[k]; }
  for (int i = 0; i < M; ++i) nnbr[i] = (int)P.nbr[i].size();
}

// Right-hand side g [2][M][L].
void oracle_rhs(ORACLE_ARGS, double* g) {
  auto P = make_problem<double>(ORACLE_PASS);
  std::vector<double> gv;
  P.rhs(gv);
  std::copy(gv.begin(), gv.end(), g);
}

// Y = L X (transpose = 0) or Y = L^T X (transpose = 1), matrix-free.
// part 0: the whole operator; 1: the sparse part L_AB only; 2: the single-layer part L_C only.
void oracle_apply(ORACLE_ARGS, int transpose, int part, const double* X, double* Yo) {
  auto P = make_problem<double>(ORACLE_PASS);
  if (transpose) P.apply_T(X, Yo, part); else P.apply(X, Yo, part);
}

// Literal dense assembly of L [(2ML)^2] and g [2ML].
void oracle_dense(ORACLE_ARGS, double* Lout, double* gout) {
  auto P = make_problem<double>(ORACLE_PASS);
  std::vector<double> Lm, g;
  P.assemble_dense(Lm, g);
  std::copy(Lm.begin(), Lm.end(), Lout);
  std::copy(g.begin(), g.end(), gout);
}

// Full energy + adjoint + forces.
//   method 0: dense LU of the literal matrix;  method 1: GMRES on the matrix-free operator;
//   method 2: flexible GMRES on it, preconditioned by inner GMRES solves of L_AB.
//   Outputs (any may be NULL): energy, X [2ML], Xadj [2ML], forces [M][3] (F = -grad E).
//   info[0..1] = GMRES iterations (primal, adjoint).  Returns 0 on success.
int oracle_solve(ORACLE_ARGS, int method, double tol, int restart, int maxit, double* energy, double* Xout,
                 double* Xaout, double* forces_out, int* info) {
  auto P = make_problem<double>(ORACLE_PASS);
  const int L = P.L;
  const size_t D = (size_t)2 * M * L;
  std::vector<double> X(D, 0.0), Xa(D, 0.0), Qv(D, 0.0), g;
  for (int j = 0; j < M; ++j) Qv[(size_t)j * L] = q[j] / std::sqrt(4.0 * PI);
  int rc = 0, it1 = 0, it2 = 0;
  if (method == 0) {
    std::vector<double> Lm;
    P.assemble_dense(Lm, g);
    X = g;
    rc |= lu_solve<double>((int)D, Lm, X);
    std::vector<double> LT(D * D);
    for (size_t a = 0; a < D; ++a)
      for (size_t b = 0; b < D; ++b) LT[b * D + a] = Lm[a * D + b];
    Xa = Qv;
    rc |= lu_solve<double>((int)D, LT, Xa);
  } else if (method == 1) {
    P.rhs(g);
    auto opL = [&](const double* in, double* out) { P.apply(in, out); };
    auto opLT = [&](const double* in, double* out) { P.apply_T(in, out); };
    rc |= gmres(D, opL, g, X, tol, restart, maxit, &it1);
    rc |= 2 * gmres(D, opLT, Qv, Xa, tol, restart, maxit, &it2);
  } else {
    // flexible GMRES preconditioned by an inner GMRES solve of L_AB (or L_AB^T) to
    // relative residual 1e-4 (at most 60 steps), from zero
    P.rhs(g);
    auto opL = [&](const double* in, double* out) { P.apply(in, out); };
    auto opLT = [&](const double* in, double* out) { P.apply_T(in, out); };
    auto opAB = [&](const double* in, double* out) { P.apply(in, out, 1); };
    auto opABT = [&](const double* in, double* out) { P.apply_T(in, out, 1); };
    auto precAB = [&](const double* in, double* out) {
      std::vector<double> rhs(in, in + D), z(D, 0.0);
      gmres(D, opAB, rhs, z, 1e-4, 60, 60, nullptr);
      std::copy(z.begin(), z.end(), out);
    };
    auto precABT = [&](const double* in, double* out) {
      std::vector<double> rhs(in, in + D), z(D, 0.0);
      gmres(D, opABT, rhs, z, 1e-4, 60, 60, nullptr);
      std::copy(z.begin(), z.end(), out);
    };
    rc |= fgmres(D, opL, precAB, g, X, tol, restart, maxit, &it1);
    rc |= 2 * fgmres(D, opLT, precABT, Qv, Xa, tol, restart, maxit, &it2);
  }
  double E = 0.0;
  for (int j = 0; j < M; ++j) E += 0.5 * q[j] * X[(size_t)j * L] / std::sqrt(4.0 * PI);
  if (energy) *energy = E;
  if (Xout) std::copy(X.begin(), X.end(), Xout);
  if (Xaout) std::copy(Xa.begin(), Xa.end(), Xaout);
  if (info) { info[0] = it1; info[1] = it2; }
  if (forces_out) {
    std::vector<double> grad;
    forces(P, X, Xa, grad);
    for (size_t k = 0; k < grad.size(); ++k) forces_out[k] = -grad[k];
  }
  return rc;
}

// Single-layer field Phi[m](x_i^n) = sum_j sum_lm m_jlm k_l(kappa|x - x_j|)/k_l(kappa r_j)
// Y_lm(x - x_j) at the grid points with chi^eta_i > 0 (zero elsewhere), for given
// per-sphere coefficients m [M][L]; out [M][N].
void oracle_single_layer_field(ORACLE_ARGS, const double* m, double* Phi) {
  auto P = make_problem<double>(ORACLE_PASS);
  std::vector<double> mv(m, m + (size_t)M * P.L), out;
  P.single_layer_field(mv, out);
  std::copy(out.begin(), out.end(), Phi);
}

// Forces for given X and X_adj (e.g. produced elsewhere); forces [M][3] = -grad E.
void oracle_forces_from(ORACLE_ARGS, const double* X, const double* Xa, double* forces_out) {
  auto P = make_problem<double>(ORACLE_PASS);
  size_t D = (size_t)2 * M * P.L;
  std::vector<double> Xv(X, X + D), Xav(Xa, Xa + D), grad;
  forces(P, Xv, Xav, grad);
  for (size_t k = 0; k < grad.size(); ++k) forces_out[k] = -grad[k];
}

// Complex-step derivative dE/dx_{atom,coord} = Im E(x + i h e) / h, dense LU path.
int oracle_energy_cs(ORACLE_ARGS, int atom, int coord, double h, double* dE) {
  Problem<cplx> P;
  P.init(M, x, r, q, eps1, eps2, kappa, eta, lmax, N, s, w);
  if (coord < 3) {
    P.x[3 * atom + coord] += cplx(0.0, h);
  } else {  // coord 3: the radius r_atom (every radial constant follows it)
    P.r[atom] += cplx(0.0, h);
    P.radial_constants();
  }
  P.build_neighbours();
  P.build_grid();
  std::vector<cplx> Lm, g;
  P.assemble_dense(Lm, g);
  std::vector<cplx> X = g;
  int rc = lu_solve<cplx>((int)g.size(), Lm, X);
  cplx E = 0.0;
  for (int j = 0; j < M; ++j) E += 0.5 * q[j] * X[(size_t)j * P.L] / std::sqrt(4.0 * PI);
  *dE = E.imag() / h;
  return rc;
}

}  // extern "C"
