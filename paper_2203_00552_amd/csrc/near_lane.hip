// Near-field A/B couplings with one neighbour cap per lane (interface and layout in
// near_lane_api.hpp).
//
// Sec. 2.2 defines the off-diagonal blocks A_ij and B_ij as Lebedev sums over the grid
// points of sphere i that lie inside sphere j, of omega_ij times the A (or B) basis
// function of sphere j times Y_lm(s_n).  The basis functions of sphere j on such a
// point are S_l'm'(v) with v = (x_i^n - x_j) / r_j (regular solid harmonics: r^l Y_lm,
// a polynomial in v, so a point close to x_j needs no normalised direction) and, for
// B, S_l'm'(v) times sigma_l'(kappa^2 r_j^2 |v|^2) / sigma_l'(kappa^2 r_j^2) with
// sigma_l(z^2) = i_l(z) / z^l, which equals i_l'(kappa rho) / i_l'(kappa r_j) Y_l'm'.
//
// Every lane takes one cap (point, sphere j) at a time and runs the harmonic
// recurrence for all (l', m') in registers; all loops are unrolled at compile time, so
// every index is a constant.  The transposed kernel keeps the 2 (lmax+1)^2 running
// sums of its sphere's coefficients in registers; the forward kernel keeps its sphere's
// coefficients in registers and writes one (A, B) value pair per cap.
#include <utility>

#include <hip/hip_runtime.h>

#include "near_lane_api.hpp"

namespace ddlpb {
namespace nearlane {

// Recurrence constants in the order the harmonics use them: for every order m, P_m^m,
// then for l = m+1..kRecLm the pair (ra(l, m), rb(l, m)).
constexpr int kRecLm = kMaxLm;
__host__ __device__ constexpr int rec_col(int m) {
  int o = 0;
  for (int k = 0; k < m; ++k) o += 1 + 2 * (kRecLm - k);
  return o;
}
__host__ __device__ constexpr int rec_off(int l, int m) { return l == m ? rec_col(m) : rec_col(m) + 1 + 2 * (l - m - 1); }
constexpr int kRecN = rec_col(kRecLm + 1);

// Harmonics of the columns M0 <= |m| < M1 (degree <= lm), and the position of column m
// in that range's generation order.
__host__ __device__ constexpr int col_count(int lm, int m0, int m1) {
  int c = 0;
  for (int m = m0; m < m1 && m <= lm; ++m) c += (lm - m + 1) * (m == 0 ? 1 : 2);
  return c;
}
__host__ __device__ constexpr int col_slot(int lm, int m0, int m) { return col_count(lm, m0, m); }
// index l*l+l+m of slot s of the range starting at column m0
__host__ __device__ constexpr int slot_index(int lm, int m0, int s) {
  for (int m = m0; m <= lm; ++m) {
    const int n = (lm - m + 1) * (m == 0 ? 1 : 2);
    if (s < n) {
      const int l = m == 0 ? s : m + s / 2;
      return l * l + l + (m == 0 ? 0 : (s % 2 == 0 ? m : -m));
    }
    s -= n;
  }
  return -1;
}
// Running sums per lane are limited to about 150 registers: with more, the kernel walks
// its caps twice, each time over one of two column ranges split at col_split(lm).
template <class R>
__host__ __device__ constexpr int n_passes(int lm) {
  return 2 * (lm + 1) * (lm + 1) * (int)(sizeof(R) / 4) > 150 ? 2 : 1;
}
__host__ __device__ constexpr int col_split(int lm) {
  int best = 1, bv = 1 << 30;
  for (int ms = 1; ms <= lm; ++ms) {
    const int a = col_count(lm, 0, ms), b = col_count(lm, ms, lm + 1);
    const int v = a > b ? a : b;
    if (v < bv) { bv = v; best = ms; }
  }
  return best;
}

static __constant__ double t_rec_d[kRecN];
static __constant__ float t_rec_f[kRecN];

typedef const __attribute__((address_space(4))) double cdbl;
typedef const __attribute__((address_space(4))) float cflt;
template <class R> struct CTab;
template <> struct CTab<double> { typedef cdbl type; };
template <> struct CTab<float> { typedef cflt type; };

// The table pointer passed through an empty asm statement that also reads `dep`: loads
// through the result come after `dep` is computed, so the compiler neither hoists the
// (loop-invariant) constants out of the cap loop nor keeps them all alive at once.
template <class P, class D>
__device__ __forceinline__ P* pin(P* p, D dep) {
  asm volatile("" : "+s"(p) : "v"(dep));
  return p;
}
template <class R>
__device__ __forceinline__ typename CTab<R>::type* rec_table() {
  if constexpr (sizeof(R) == 8) return (cdbl*)t_rec_d;
  else return (cflt*)t_rec_f;
}

template <class F, int... I>
__device__ __forceinline__ void sfor_(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// f(integral_constant<int, i>) for i = 0..N-1, unrolled at compile time
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (N > 0) sfor_(f, std::make_integer_sequence<int, N>{});
}

// f(l, slot, index l*l+l+m, S_lm(x, y, z)) for every (l, m) with l <= LM and M0 <= |m| < M1,
// in the order |m| = M0..M1-1, l = |m|..LM, +|m| before -|m| (l, the running slot and
// the index as integral constants).  The columns are independent recurrences, so a
// range of them costs only its own harmonics (and M0 steps of (x + i y)^m).
template <int LM, int M0, int M1, class R, class F>
__device__ __forceinline__ void harmonics(R x, R y, R z, F&& f) {
  const R r2 = x * x + y * y + z * z;
  R cm = R(1), sm = R(0);  // (x + i y)^m
  sfor<M1>([&](auto M_) {
    constexpr int m = decltype(M_)::value;
    if constexpr (m > 0) {
      const R c2 = x * cm - y * sm;
      sm = x * sm + y * cm;
      cm = c2;
    }
    if constexpr (m >= M0) {
      auto* tab = pin(rec_table<R>(), cm);
      R p1 = R(0), p2 = R(0);
      sfor<LM + 1 - m>([&](auto K_) {
        constexpr int l = m + decltype(K_)::value;
        constexpr int slot = col_slot(LM, M0, m) + (m == 0 ? l : 2 * (l - m));
        R p;
        if constexpr (l == m) p = tab[rec_off(m, m)];
        else if constexpr (l == m + 1) p = tab[rec_off(l, m)] * (z * p1);
        else p = tab[rec_off(l, m)] * (z * p1) - tab[rec_off(l, m) + 1] * (r2 * p2);
        if constexpr (m == 0) {
          f(std::integral_constant<int, l>{}, std::integral_constant<int, slot>{},
            std::integral_constant<int, l * l + l>{}, p);
        } else {
          f(std::integral_constant<int, l>{}, std::integral_constant<int, slot>{},
            std::integral_constant<int, l * l + l + m>{}, p * cm);
          f(std::integral_constant<int, l>{}, std::integral_constant<int, slot + 1>{},
            std::integral_constant<int, l * l + l - m>{}, p * sm);
        }
        p2 = p1;
        p1 = p;
      });
    }
  });
}

__host__ __device__ constexpr double inv_dfact(int l) {  // 1 / (2l+1)!!
  double d = 1.0;
  for (int k = 2 * l + 1; k > 1; k -= 2) d *= k;
  return 1.0 / d;
}
// Coefficient k of the series sigma_l(z2) = sum_k z2^k / (2^k k! (2l+2k+1)!!).
__host__ __device__ constexpr double sig_coef(int l, int k) {
  double c = inv_dfact(l);
  for (int j = 0; j < k; ++j) c *= 0.5 / ((j + 1.0) * (2.0 * l + 2.0 * j + 3.0));
  return c;
}
constexpr int kSigFixed = 8;  // terms of the unrolled series (used when they suffice)
// sig_coef(l, k) for l <= kMaxLm + 1, k <= kSigFixed, read through a pinned pointer
// (kept out of the registers between caps)
constexpr int kSigN = (kMaxLm + 2) * (kSigFixed + 1);
static __constant__ double t_sig_d[kSigN];
static __constant__ float t_sig_f[kSigN];
template <class R>
__device__ __forceinline__ typename CTab<R>::type* sig_table() {
  if constexpr (sizeof(R) == 8) return (cdbl*)t_sig_d;
  else return (cflt*)t_sig_f;
}
// sigma_l(z2) = i_l(z) / z^l for l = 0..LM: the series for LM+1 and LM (nterms terms;
// with nterms <= kSigFixed the first kSigFixed terms in Horner form), then the
// downward recurrence sigma_{l-1} = z2 sigma_{l+1} + (2l+1) sigma_l
template <int LM, class R>
__device__ __forceinline__ void sigma(R z2, int nterms, R (&sg)[LM + 1]) {
  R sa, sb;
  if (nterms <= kSigFixed) {  // uniform branch
    auto* tab = pin(sig_table<R>(), z2);
    constexpr int oa = (LM + 1) * (kSigFixed + 1), ob = LM * (kSigFixed + 1);
    sa = tab[oa + kSigFixed];
    sb = tab[ob + kSigFixed];
    sfor<kSigFixed>([&](auto K_) {
      constexpr int k = kSigFixed - 1 - decltype(K_)::value;
      sa = sa * z2 + tab[oa + k];
      sb = sb * z2 + tab[ob + k];
    });
  } else {
    R ta = R(inv_dfact(LM + 1)), tb = R(inv_dfact(LM));
    sa = ta;
    sb = tb;
    for (int k = 0; k < nterms; ++k) {
      ta = ta * z2 * R(0.5 / ((k + 1.0) * (2.0 * LM + 2.0 * k + 5.0)));
      tb = tb * z2 * R(0.5 / ((k + 1.0) * (2.0 * LM + 2.0 * k + 3.0)));
      sa += ta;
      sb += tb;
    }
  }
  R sp1 = sa;
  sg[LM] = sb;
  sfor<LM>([&](auto K_) {
    constexpr int l = LM - decltype(K_)::value;
    const R s = z2 * sp1 + R(2 * l + 1) * sg[l];
    sp1 = sg[l];
    sg[l - 1] = s;
  });
}

// ---------------------------------------------------------------- reduce-scatter
template <int CTRL>
__device__ __forceinline__ double dpp_mv(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mv(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
// one step over a 16-lane row: the partner (DPP pattern CTRL) holds the same index
// set; this lane keeps the odd or the even entries (bit) and adds the partner's copies
template <int N, int CTRL, class R>
__device__ __forceinline__ void rs_step(const R (&in)[N], R (&out)[(N + 1) / 2], bool bit) {
  sfor<(N + 1) / 2>([&](auto I_) {
    constexpr int i = decltype(I_)::value;
    const R x0 = in[2 * i];
    R x1 = R(0);
    if constexpr (2 * i + 1 < N) x1 = in[2 * i + 1];
    const R keep = bit ? x1 : x0, send = bit ? x0 : x1;
    out[i] = keep + dpp_mv<CTRL>(send);
  });
}
constexpr int half(int n) { return (n + 1) / 2; }
__host__ __device__ constexpr int deg(int t) {
  int l = 0;
  while ((l + 1) * (l + 1) <= t) ++l;
  return l;
}

// ---------------------------------------------------------------- kernels
// Geometry of one reverse cap of sphere j: v = (x_i^n - x_j) / r_j, omega, the Lebedev
// weight times omega, and the point's flat index i N + n.
struct Cap {
  double vx, vy, vz, w, wom;
  long pt;
};
__device__ __forceinline__ Cap cap_geom(const NearArgs& a, int i, int n, double w, double xj, double yj, double zj,
                                        double irj) {
  Cap g;
  g.w = w;
  const double* lp = a.leb + 4 * n;
  const double ri = a.rad[i];
  g.vx = (a.xyz[3 * i] + ri * lp[0] - xj) * irj;
  g.vy = (a.xyz[3 * i + 1] + ri * lp[1] - yj) * irj;
  g.vz = (a.xyz[3 * i + 2] + ri * lp[2] - zj) * irj;
  g.wom = lp[3] * g.w;
  g.pt = (long)i * a.N + n;
  return g;
}
// The index triple (i, n, omega) of reverse cap c, fetched one cap ahead of its use so
// that the dependent loads of the next cap do not wait for it.
struct CapIdx {
  int i = 0, n = 0;
  double w = 0.0;
  __device__ __forceinline__ void fetch(const NearArgs& a, int c, int r1) {
    if (c < r1) {
      i = a.rci[c];
      n = a.rcn[c];
      w = a.rcw[c];
    }
  }
};
// column range of pass P of NP
template <int LM, int NP, int P>
struct Cols {
  static constexpr int m0 = NP == 1 ? 0 : (P == 0 ? 0 : col_split(LM));
  static constexpr int m1 = NP == 1 ? LM + 1 : (P == 0 ? col_split(LM) : LM + 1);
  static constexpr int n = col_count(LM, m0, m1);
};

// out = c0 base + c1 (sum over the reverse caps of sphere j of the A / B basis times the
// point values), per coefficient of sphere j
template <int LM, class R, bool INC>
__global__ __launch_bounds__(256) void k_ltz(NearArgs a, const double* __restrict__ base, double c0,
                                             const double* __restrict__ zr, const double* __restrict__ ze,
                                             double c1, double* __restrict__ out) {
  constexpr int L = (LM + 1) * (LM + 1), T = cache_stride(LM), NP = n_passes<R>(LM);
  const int g = threadIdx.x & 15;
  const int jq = (int)(((long)blockIdx.x * blockDim.x + threadIdx.x) >> 4);
  const bool valid = jq < a.M;
  const int j = valid ? a.jord[jq] : 0;  // idle groups still take part in the reductions
  const int r0 = a.rptr[j], r1 = (valid && zr != nullptr) ? a.rptr[j + 1] : r0;
  const double xj = a.xyz[3 * j], yj = a.xyz[3 * j + 1], zj = a.xyz[3 * j + 2], rj = a.rad[j], irj = 1.0 / rj;
  const R kr2 = R(a.kappa * a.kappa * rj * rj);
  const long cb = INC ? a.coff[j] : 0;
  const bool b3 = (g >> 3) & 1, b2 = (g >> 2) & 1, b1 = (g >> 1) & 1, b0 = g & 1;
  const int gr = ((g & 1) << 3) | ((g & 2) << 1) | ((g & 4) >> 1) | ((g & 8) >> 3);
  sfor<NP>([&](auto P_) {
    using C = Cols<LM, NP, decltype(P_)::value>;
    constexpr int V = 2 * C::n;  // A sums of the range's harmonics, then the B sums
    R acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = R(0);
    CapIdx nx;
    nx.fetch(a, r0 + g, r1);
    for (int c = r0 + g, k = 0; c < r1; c += kGroup, ++k) {
      const CapIdx cur = nx;
      nx.fetch(a, c + kGroup, r1);
      R fA, fB[LM + 1];
      if constexpr (INC) {
        const int i = cur.i, n = cur.n;
        const long pt = (long)i * a.N + n;
        const double wom = a.leb[4 * n + 3] * cur.w;
        fA = R(wom * zr[pt]);
        const R cB = R(wom * ze[pt]);
        const double* cp = a.cache + (cb + (long)kGroup * k) * T + g;
#pragma unroll
        for (int l = 0; l <= LM; ++l) fB[l] = cB * R(cp[kGroup * (L + l)]);
        sfor<C::n>([&](auto S_) {
          constexpr int s = decltype(S_)::value, t = slot_index(LM, C::m0, s), l = deg(t);
          const R S = R(cp[kGroup * t]);
          acc[s] = fA * S + acc[s];
          acc[C::n + s] = fB[l] * S + acc[C::n + s];
        });
      } else {
        const Cap q = cap_geom(a, cur.i, cur.n, cur.w, xj, yj, zj, irj);
        fA = R(q.wom * zr[q.pt]);
        const R cB = R(q.wom * ze[q.pt]);
        const R vx = R(q.vx), vy = R(q.vy), vz = R(q.vz);
        R sg[LM + 1];
        sigma<LM, R>(kr2 * (vx * vx + vy * vy + vz * vz), a.nterms, sg);
#pragma unroll
        for (int l = 0; l <= LM; ++l) fB[l] = cB * sg[l] * R(a.isgr[(long)j * a.LUR + l]);
        harmonics<LM, C::m0, C::m1, R>(vx, vy, vz, [&](auto L_, auto S_, auto, R S) {
          constexpr int l = decltype(L_)::value, s = decltype(S_)::value;
          acc[s] = fA * S + acc[s];
          acc[C::n + s] = fB[l] * S + acc[C::n + s];
        });
      }
    }
    // the group's 16 partial sums: afterwards this lane holds slots 16 e + rev4(g)
    R s1[half(V)], s2[half(half(V))], s3[half(half(half(V)))], s4[half(half(half(half(V))))];
    rs_step<V, 0x140>(acc, s1, b3);               // row mirror: partner 15 - g
    rs_step<half(V), 0x141>(s1, s2, b2);          // row half mirror: partner 7 - g in eight lanes
    rs_step<half(half(V)), 0x4E>(s2, s3, b1);     // quad permutation (2, 3, 0, 1)
    rs_step<half(half(half(V))), 0xB1>(s3, s4, b0);  // quad permutation (1, 0, 3, 2)
    if (valid) {
#pragma unroll
      for (int e = 0; e < half(half(half(half(V)))); ++e) {
        const int v = kGroup * e + gr;
        if (v >= V) continue;
        const int part = v >= C::n, t = slot_index(LM, C::m0, v - part * C::n);
        const long o = (long)(part * a.M + j) * L + t;
        double r = c1 * (double)s4[e];
        if (base) r += c0 * base[o];
        out[o] = r;
      }
    }
  });
}

// capv[2c], capv[2c+1] = omega times the A and B expansions of sphere j (coefficients X)
// at the point of reverse cap c.  The coefficients are the same for the 16 lanes of a
// group: they sit in LDS (broadcast reads, fetched per cap through a pinned pointer so
// that they are not hoisted into registers), which leaves the registers to one pass
// over all harmonics.
typedef __attribute__((address_space(3))) double ldbl;
typedef __attribute__((address_space(3))) float lflt;
template <class R> struct LTab;
template <> struct LTab<double> { typedef ldbl type; };
template <> struct LTab<float> { typedef lflt type; };
template <class P, class D>
__device__ __forceinline__ P* pin_lds(P* p, D dep) {
  asm volatile("" : "+v"(p) : "v"(dep));
  return p;
}
template <int LM, class R, bool INC>
__global__ __launch_bounds__(256) void k_lx(NearArgs a, const double* __restrict__ X, double* __restrict__ capv) {
  constexpr int L = (LM + 1) * (LM + 1), T = cache_stride(LM);
  __shared__ R sx[256 / kGroup][2 * L];
  const int g = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int jq = (int)(((long)blockIdx.x * blockDim.x + threadIdx.x) >> 4);
  const int j = jq < a.M ? a.jord[jq] : -1;
  if (j >= 0)
    for (int t = g; t < 2 * L; t += kGroup) sx[grp][t] = R(X[(long)(t < L ? j : a.M + j) * L + (t < L ? t : t - L)]);
  __syncthreads();
  if (j < 0) return;
  const int r0 = a.rptr[j], r1 = a.rptr[j + 1];
  const double xj = a.xyz[3 * j], yj = a.xyz[3 * j + 1], zj = a.xyz[3 * j + 2], rj = a.rad[j], irj = 1.0 / rj;
  const R kr2 = R(a.kappa * a.kappa * rj * rj);
  const long cb = INC ? a.coff[j] : 0;
  typedef typename LTab<R>::type LT;
  LT* xs = (LT*)&sx[grp][0];
  CapIdx nx;
  nx.fetch(a, r0 + g, r1);
  for (int c = r0 + g, k = 0; c < r1; c += kGroup, ++k) {
    const CapIdx cur = nx;
    nx.fetch(a, c + kGroup, r1);
    R pa[LM + 1], pb[LM + 1], sgw[LM + 1];
#pragma unroll
    for (int l = 0; l <= LM; ++l) { pa[l] = R(0); pb[l] = R(0); }
    double w;
    if constexpr (INC) {
      w = cur.w;
      const double* cp = a.cache + (cb + (long)kGroup * k) * T + g;
      LT* xp = pin_lds(xs, cp[0]);
      sfor<L>([&](auto T_) {
        constexpr int t = decltype(T_)::value, l = deg(t);
        const R S = R(cp[kGroup * t]);
        pa[l] = xp[t] * S + pa[l];
        pb[l] = xp[L + t] * S + pb[l];
      });
#pragma unroll
      for (int l = 0; l <= LM; ++l) sgw[l] = R(cp[kGroup * (L + l)]);
    } else {
      const Cap q = cap_geom(a, cur.i, cur.n, cur.w, xj, yj, zj, irj);
      w = q.w;
      const R vx = R(q.vx), vy = R(q.vy), vz = R(q.vz);
      R sg[LM + 1];
      sigma<LM, R>(kr2 * (vx * vx + vy * vy + vz * vz), a.nterms, sg);
#pragma unroll
      for (int l = 0; l <= LM; ++l) sgw[l] = sg[l] * R(a.isgr[(long)j * a.LUR + l]);
      LT* xp = pin_lds(xs, vx);
      harmonics<LM, 0, LM + 1, R>(vx, vy, vz, [&](auto L_, auto, auto I_, R S) {
        constexpr int l = decltype(L_)::value, t = decltype(I_)::value;
        pa[l] = xp[t] * S + pa[l];
        pb[l] = xp[L + t] * S + pb[l];
      });
    }
    R sa = R(0), sb = R(0);
#pragma unroll
    for (int l = 0; l <= LM; ++l) {
      sa += pa[l];
      sb = pb[l] * sgw[l] + sb;
    }
    double2 o;
    o.x = w * (double)sa;
    o.y = w * (double)sb;
    *reinterpret_cast<double2*>(capv + 2L * c) = o;
  }
}

// the incore cache: harmonics and radial ratios of every reverse cap, in FP64
template <int LM>
__global__ __launch_bounds__(256) void k_fill(NearArgs a, double* __restrict__ cache) {
  constexpr int L = (LM + 1) * (LM + 1), T = cache_stride(LM);
  const int g = threadIdx.x & 15;
  const int jq = (int)(((long)blockIdx.x * blockDim.x + threadIdx.x) >> 4);
  if (jq >= a.M) return;
  const int j = a.jord[jq];
  const int r0 = a.rptr[j], r1 = a.rptr[j + 1];
  const double xj = a.xyz[3 * j], yj = a.xyz[3 * j + 1], zj = a.xyz[3 * j + 2], rj = a.rad[j], irj = 1.0 / rj;
  const double kr2 = a.kappa * a.kappa * rj * rj;
  const long cb = a.coff[j];
  for (int c = r0 + g, k = 0; c < r1; c += kGroup, ++k) {
    const Cap q = cap_geom(a, a.rci[c], a.rcn[c], a.rcw[c], xj, yj, zj, irj);
    double* cp = cache + (cb + (long)kGroup * k) * T + g;
    double sg[LM + 1];
    sigma<LM, double>(kr2 * (q.vx * q.vx + q.vy * q.vy + q.vz * q.vz), a.nterms, sg);
#pragma unroll
    for (int l = 0; l <= LM; ++l) cp[kGroup * (L + l)] = sg[l] * a.isgr[(long)j * a.LUR + l];
    harmonics<LM, 0, LM + 1, double>(q.vx, q.vy, q.vz,
                                     [&](auto, auto, auto I_, double S) { cp[kGroup * decltype(I_)::value] = S; });
  }
}

// ---------------------------------------------------------------- host side
hipError_t upload_tables(const double* pmm, const double* ra, const double* rb) {
  double rec[kRecN];
  float recf[kRecN];
  for (int m = 0; m <= kRecLm; ++m) {
    rec[rec_off(m, m)] = pmm[m];
    for (int l = m + 1; l <= kRecLm; ++l) {
      const int t = l * (l + 1) / 2 + m;
      rec[rec_off(l, m)] = ra[t];
      rec[rec_off(l, m) + 1] = rb[t];
    }
  }
  for (int k = 0; k < kRecN; ++k) recf[k] = (float)rec[k];
  double sig[kSigN];
  float sigf[kSigN];
  for (int l = 0; l <= kMaxLm + 1; ++l)
    for (int k = 0; k <= kSigFixed; ++k) {
      sig[l * (kSigFixed + 1) + k] = sig_coef(l, k);
      sigf[l * (kSigFixed + 1) + k] = (float)sig_coef(l, k);
    }
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(t_rec_d), rec, sizeof(rec));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(t_rec_f), recf, sizeof(recf));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(t_sig_d), sig, sizeof(sig));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(t_sig_f), sigf, sizeof(sigf));
  return e;
}

namespace {
inline int blocks_for(int M) { return (int)(((long)M * kGroup + 255) / 256); }
#define NL_DISPATCH(LMV, BODY)                        \
  switch (LMV) {                                      \
    case 0: { constexpr int LMc = 0; BODY; } break;   \
    case 1: { constexpr int LMc = 1; BODY; } break;   \
    case 2: { constexpr int LMc = 2; BODY; } break;   \
    case 3: { constexpr int LMc = 3; BODY; } break;   \
    case 4: { constexpr int LMc = 4; BODY; } break;   \
    case 5: { constexpr int LMc = 5; BODY; } break;   \
    case 6: { constexpr int LMc = 6; BODY; } break;   \
    case 7: { constexpr int LMc = 7; BODY; } break;   \
    case 8: { constexpr int LMc = 8; BODY; } break;   \
    default: return hipErrorInvalidValue;             \
  }
}  // namespace

hipError_t launch_ltz(int lmax, int prec, const NearArgs& a, const double* base, double c0, const double* zr,
                      const double* ze, double c1, double* out, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  const bool inc = a.cache != nullptr;
  NL_DISPATCH(lmax, {
    if (prec == 1) {
      if (inc) hipLaunchKernelGGL((k_ltz<LMc, float, true>), dim3(blocks_for(a.M)), dim3(256), 0, s, a, base, c0, zr, ze, c1, out);
      else hipLaunchKernelGGL((k_ltz<LMc, float, false>), dim3(blocks_for(a.M)), dim3(256), 0, s, a, base, c0, zr, ze, c1, out);
    } else {
      if (inc) hipLaunchKernelGGL((k_ltz<LMc, double, true>), dim3(blocks_for(a.M)), dim3(256), 0, s, a, base, c0, zr, ze, c1, out);
      else hipLaunchKernelGGL((k_ltz<LMc, double, false>), dim3(blocks_for(a.M)), dim3(256), 0, s, a, base, c0, zr, ze, c1, out);
    }
  });
  return hipGetLastError();
}

hipError_t launch_lx(int lmax, int prec, const NearArgs& a, const double* X, double* capv, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  const bool inc = a.cache != nullptr;
  NL_DISPATCH(lmax, {
    if (prec == 1) {
      if (inc) hipLaunchKernelGGL((k_lx<LMc, float, true>), dim3(blocks_for(a.M)), dim3(256), 0, s, a, X, capv);
      else hipLaunchKernelGGL((k_lx<LMc, float, false>), dim3(blocks_for(a.M)), dim3(256), 0, s, a, X, capv);
    } else {
      if (inc) hipLaunchKernelGGL((k_lx<LMc, double, true>), dim3(blocks_for(a.M)), dim3(256), 0, s, a, X, capv);
      else hipLaunchKernelGGL((k_lx<LMc, double, false>), dim3(blocks_for(a.M)), dim3(256), 0, s, a, X, capv);
    }
  });
  return hipGetLastError();
}

hipError_t launch_fill(int lmax, const NearArgs& a, double* cache, hipStream_t s) {
  if (a.M <= 0) return hipSuccess;
  NL_DISPATCH(lmax, hipLaunchKernelGGL((k_fill<LMc>), dim3(blocks_for(a.M)), dim3(256), 0, s, a, cache));
  return hipGetLastError();
}

}  // namespace nearlane
}  // namespace ddlpb
