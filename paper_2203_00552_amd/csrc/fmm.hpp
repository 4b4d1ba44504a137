// Fast multipole method on the device (Appendix): translations of the screened
// Coulomb (Yukawa) and Coulomb (Laplace) expansions between tree nodes.
//
// Scaled bases about a centre c with scale R (the node radius):
//   Yukawa   multipole  k_l(kappa|v|)/k_l(kappa R) Y_lm(v/|v|),   local  i_l(kappa|v|)/i_l(kappa R) Y_lm
//   Laplace  multipole  (R/|v|)^(l+1) Y_lm(v/|v|),               local  (|v|/R)^l Y_lm
// A leaf is one sphere (centre x_j, scale r_j), so the sphere's own expansions are
// the leaf expansions.  Every translation rotates the frame so that the target
// centre lies on the negative z axis of the source centre (three z-rotations and
// two applications of the fixed 90-degree rotation J), applies the translation
// along z (Appendix formulas for Yukawa; their kappa -> 0 limits for Laplace)
// and rotates back.  The adjoint passes apply exact transposes.
//
// One 64-lane wavefront (one block) performs one translation at a time with its
// vectors in LDS.
#pragma once
#include "device_math.hpp"
#include "fmm_types.hpp"

namespace ddlpb {

constexpr int kPmaxFmm = 20;
constexpr int kPFmm = (kPmaxFmm + 1) * (kPmaxFmm + 1);


// The same scratch as pointers into dynamic LDS, sized for the tree's order p
struct TransView {
  double *b0, *b1, *bes, *pw1, *pw2, *radS, *radT, *cph, *sph, *cth, *sth;
};
__host__ __device__ constexpr int trans_view_doubles(int p) {
  return 3 * (p + 1) * (p + 1) + 3 * (2 * p + 4) + 2 * (p + 2) + 4 * (p + 1);  // incl. the accumulator
}
// carve the view (and the accumulator, returned) from `base`
__device__ __forceinline__ double* carve_trans_view(double* base, int p, TransView& v) {
  const int P = (p + 1) * (p + 1);
  v.b0 = base;
  v.b1 = v.b0 + P;
  v.bes = v.b1 + P;
  v.pw1 = v.bes + (2 * p + 4);
  v.pw2 = v.pw1 + (2 * p + 4);
  v.radS = v.pw2 + (2 * p + 4);
  v.radT = v.radS + (p + 2);
  v.cph = v.radT + (p + 2);
  v.sph = v.cph + (p + 1);
  v.cth = v.sph + (p + 1);
  v.sth = v.cth + (p + 1);
  return v.sth + (p + 1);  // accumulator, P entries
}

struct TransScratch {
  double b0[kPFmm], b1[kPFmm];
  double bes[2 * kPmaxFmm + 4];
  double pw1[2 * kPmaxFmm + 4], pw2[2 * kPmaxFmm + 4];
  double radS[kPmaxFmm + 2], radT[kPmaxFmm + 2];
  double cph[kPmaxFmm + 1], sph[kPmaxFmm + 1], cth[kPmaxFmm + 1], sth[kPmaxFmm + 1];
};

// Synchronisation of the lanes cooperating on one translation: the whole block, or
// only the wavefront when every wavefront of the block works on its own translation.
template <bool WAVE>
__device__ __forceinline__ void tsync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}
template <bool WAVE> __device__ __forceinline__ int tlane() { return WAVE ? (int)(threadIdx.x & 63) : (int)threadIdx.x; }
template <bool WAVE> __device__ __forceinline__ int tstride() { return WAVE ? 64 : (int)blockDim.x; }

__device__ __forceinline__ double ipow_d(double b, int e) {
  double r = 1.0;
  while (e) {
    if (e & 1) r *= b;
    b *= b;
    e >>= 1;
  }
  return r;
}
__device__ __forceinline__ void cpow_d(double c, double s, int e, double& rc, double& rs) {
  double xc = 1.0, xs = 0.0;
  while (e) {
    if (e & 1) { const double t = xc * c - xs * s; xs = xc * s + xs * c; xc = t; }
    const double t = c * c - s * s;
    s = 2.0 * c * s;
    c = t;
    e >>= 1;
  }
  rc = xc;
  rs = xs;
}

// J or J^T on the degrees of a vector with Pdeg = (pdeg+1)^2 entries (row table of P entries)
__device__ __forceinline__ void japply_sparse_deg(const double* __restrict__ jv, const int* __restrict__ jr, int mat,
                                                  int P, int Pdeg, const double* src, double* dst, int lane) {
  for (int t = lane; t < Pdeg; t += 64) {
    const int off = jr[2 * (mat * P + t)], d = jr[2 * (mat * P + t) + 1];
    const int cnt = (d >> 12) & 255, st = d >> 20;
    const double* x = src + (d & 4095);
    const double* v = jv + off;
    double s = 0.0;
    for (int k = 0; k < cnt; ++k) s += v[k] * x[st * k];
    dst[t] = s;
  }
}
// sigma_n(z2) = i_n(z)/z^n for n = 0..nmax (series at the top, downward recurrence)
__device__ __forceinline__ void sigma_all(double z2, int nmax, double* sg) {
  double top[2];
  for (int q = 0; q < 2; ++q) {
    const int l = nmax + 1 - q;
    double df = 1.0;
    for (int k = 2 * l + 1; k > 1; k -= 2) df *= k;
    double term = 1.0 / df, sum = term;
    for (int k = 0; k < 200; ++k) {
      term *= z2 * 0.5 / ((k + 1.0) * (2.0 * l + 2.0 * k + 3.0));
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    top[q] = sum;
  }
  double sp1 = top[0];
  sg[nmax] = top[1];
  for (int l = nmax; l >= 1; --l) {
    const double s = z2 * sp1 + (2.0 * l + 1.0) * sg[l];
    sp1 = sg[l];
    sg[l - 1] = s;
  }
}
// k_n(z) for n = 0..nmax (upward recurrence)
__device__ __forceinline__ void kbes_all(double z, int nmax, double* k) {
  const double e = exp(-z);
  k[0] = 1.5707963267948966 * e / z;
  if (nmax >= 1) k[1] = 1.5707963267948966 * e * (z + 1.0) / (z * z);
  for (int l = 1; l < nmax; ++l) k[l + 1] = k[l - 1] + (2.0 * l + 1.0) / z * k[l];
}

// rotation of the pairs (l, +-m) about z by the angle with cos(m a) = co[m] (sign sg
// (-1)^m when alt), sin(m a) = ss sg si[m]; 64 lanes
__device__ __forceinline__ void zrot_table(double* c, int pdeg, const double* co_t, const double* si_t, bool alt,
                                           double ss, int lane) {
  const int npairs = pdeg * (pdeg + 1) / 2;  // (l, m>0) pairs
  for (int t = lane; t < npairs; t += 64) {
    int l = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f) + 1;
    while (l * (l - 1) / 2 > t) --l;
    while ((l + 1) * l / 2 <= t) ++l;
    const int m = t - l * (l - 1) / 2 + 1;
    const double sg = (alt && (m & 1)) ? -1.0 : 1.0;
    const double co = sg * co_t[m], si = ss * sg * si_t[m];
    const double a = c[lmi(l, m)], b = c[lmi(l, -m)];
    c[lmi(l, m)] = a * co - b * si;
    c[lmi(l, -m)] = a * si + b * co;
  }
}

// Translation (kind 0 M2M, 1 M2L, 2 L2L) from node S to node T of the expansion in
// sc.b0 (degree ps; degree pt when transposed); the result is added to acc
// (degree pt; ps when transposed).  One 64-lane block (WAVE: one wavefront of a
// larger block) calls it with all lanes.  The per-translation tables (Bessel
// values, powers, node scales, cos/sin of m*phi and m*theta as powers of the unit
// complex numbers of the centre offset) are computed one entry per lane.
template <bool WAVE, class SC>
__device__ void translate(const FmmDev& f, const double* __restrict__ Atab, const int* __restrict__ Aoff, int kind,
                          int S, int T, int ps, int pt, int transposed, SC& sc, double* acc) {
  const int lane = tlane<WAVE>();
  const int P1 = f.p + 1;
  const int nmax = ps + pt;
  double d0 = f.center[3 * T] - f.center[3 * S], d1 = f.center[3 * T + 1] - f.center[3 * S + 1],
         d2 = f.center[3 * T + 2] - f.center[3 * S + 2];
  const double rxy = sqrt(d0 * d0 + d1 * d1);
  double rho = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  double ct = 1.0, st = 0.0, cp = 1.0, sp = 0.0;
  if (rho > 1e-12) {
    ct = d2 / rho;
    st = rxy / rho;
    if (rxy > 0.0) { cp = d0 / rxy; sp = d1 / rxy; }
  } else {
    rho = 1e-12;
  }
  if (lane <= f.p) {
    cpow_d(cp, sp, lane, sc.cph[lane], sc.sph[lane]);
    cpow_d(ct, st, lane, sc.cth[lane], sc.sth[lane]);
  }
  const double RS = f.radius[S], RT = f.radius[T];
  if (f.kernel == 0) {
    const double z = f.kappa * rho;
    if (lane <= nmax) {
      const int n = lane;
      if (kind == 1) {
        // k_n(z) by the upward recurrence k_{j+1} = k_{j-1} + (2j+1)/z k_j
        const double iz = 1.0 / z;
        double km = 1.5707963267948966 * exp(-z) * iz, kc = km * (1.0 + iz);
        for (int j = 1; j < n; ++j) {
          const double kn = km + (2.0 * j + 1.0) * iz * kc;
          km = kc;
          kc = kn;
        }
        sc.bes[n] = n == 0 ? km : kc;
        sc.pw1[n] = ipow_d(-iz, n);  // (-z)^-n
      } else {
        // sigma_n(z^2) = i_n(z)/z^n = sum_k (z^2/2)^k / (k! (2n+2k+1)!!)
        const double z2 = z * z;
        double df = 1.0;
        for (int k = 3; k <= 2 * n + 1; k += 2) df *= k;
        double term = 1.0 / df, sum = term;
        for (int k = 0; k < 400; ++k) {
          const double ck = (n <= kLmaxDev + 1 && k < kSigTerms) ? c_sinv[n * kSigTerms + k]
                                                                 : 0.5 / ((k + 1.0) * (2.0 * n + 2.0 * k + 3.0));
          term *= z2 * ck;
          sum += term;
          if (term < 1e-18 * sum) break;
        }
        sc.bes[n] = sum;
        sc.pw1[n] = ipow_d(z, n);
      }
    }
    if (lane <= ps) sc.radS[lane] = (kind == 2) ? 1.0 / f.iR[S * P1 + lane] : f.kRi[S * P1 + lane];
    if (lane <= pt) sc.radT[lane] = (kind == 0) ? f.kR[T * P1 + lane] : f.iR[T * P1 + lane];
  } else if (lane <= nmax + 1) {
    // powers of the ratios of the Laplace translations
    double a1, a2;
    if (kind == 0) { a1 = RS / RT; a2 = rho / RT; }        // (RS/RT)^(l+1) (rho/RT)^(l'-l)
    else if (kind == 1) { a1 = RT / rho; a2 = RS / rho; }  // (RT/rho)^l' (RS/rho)^(l+1)
    else { a1 = RT / RS; a2 = rho / RS; }                  // (RT/RS)^l' (rho/RS)^(l-l')
    sc.pw1[lane] = ipow_d(a1, lane);
    sc.pw2[lane] = ipow_d(a2, lane);
  }
  tsync<WAVE>();
  const int pin = transposed ? pt : ps, pout = transposed ? ps : pt;
  const int Pin = (pin + 1) * (pin + 1), Pout = (pout + 1) * (pout + 1);
  // rotate the input to the frame where the target sits on the -z axis:
  // z-rotation by -phi, J, z-rotation by pi - theta, J^T
  zrot_table(sc.b0, pin, sc.cph, sc.sph, false, -1.0, lane);
  tsync<WAVE>();
  japply_sparse_deg(f.jval, f.jrow, 0, P1 * P1, Pin, sc.b0, sc.b1, lane);
  tsync<WAVE>();
  zrot_table(sc.b1, pin, sc.cth, sc.sth, true, -1.0, lane);
  tsync<WAVE>();
  japply_sparse_deg(f.jval, f.jrow, 1, P1 * P1, Pin, sc.b1, sc.b0, lane);
  tsync<WAVE>();
  // translation along z
  const int nout = (pout + 1) * (pout + 1);
  for (int t = tlane<WAVE>(); t < nout; t += tstride<WAVE>()) {
    const int lo = (int)sqrt((double)t + 0.5);
    const int m = t - lo * lo - lo, am = abs(m);
    double s = 0.0;
    for (int li = am; li <= pin; ++li) {
      const int l = transposed ? lo : li;   // source degree
      const int lp = transposed ? li : lo;  // target degree
      double e;
      if (f.kernel == 0) {
        const double* Ar = Atab + Aoff[((size_t)l * P1 + lp) * P1 + am] - am;
        double sk = 0.0;
        const int kmax = min(l, lp);
        if (kind == 1) {
          for (int k = am; k <= kmax; ++k) sk += Ar[k] * sc.bes[l + lp - k] * sc.pw1[k];
          e = sk * sc.radT[lp] * sc.radS[l] * ((l & 1) ? -1.0 : 1.0);
        } else {
          for (int k = am; k <= kmax; ++k) sk += Ar[k] * sc.bes[l + lp - k] * sc.pw1[l + lp - 2 * k];
          e = sk * sc.radT[lp] * sc.radS[l] * ((kind == 2 && ((l + lp) & 1)) ? -1.0 : 1.0);
        }
      } else {
        const double a = Atab[((size_t)l * P1 + lp) * P1 + am];
        if (a == 0.0) continue;
        if (kind == 0) e = a * sc.pw1[l + 1] * sc.pw2[lp - l];
        else if (kind == 1) e = a * sc.pw1[lp] * sc.pw2[l + 1];
        else e = a * sc.pw1[lp] * sc.pw2[l - lp];
      }
      s += e * sc.b0[lmi(li, m)];
    }
    sc.b1[t] = s;
  }
  tsync<WAVE>();
  // rotate back: J, z-rotation by theta - pi, J^T, z-rotation by phi
  japply_sparse_deg(f.jval, f.jrow, 0, P1 * P1, Pout, sc.b1, sc.b0, lane);
  tsync<WAVE>();
  zrot_table(sc.b0, pout, sc.cth, sc.sth, true, 1.0, lane);
  tsync<WAVE>();
  japply_sparse_deg(f.jval, f.jrow, 1, P1 * P1, Pout, sc.b0, sc.b1, lane);
  tsync<WAVE>();
  zrot_table(sc.b1, pout, sc.cph, sc.sph, false, 1.0, lane);
  tsync<WAVE>();
  for (int t = tlane<WAVE>(); t < nout; t += tstride<WAVE>()) acc[t] += sc.b1[t];
  tsync<WAVE>();
}

// coefficient table of a kernel type and translation kind, in global memory
__device__ __forceinline__ const double* coef_table(const FmmDev& f, int kind) {
  const int P1 = f.p + 1;
  return f.kernel == 0 ? f.A : f.AL + (size_t)kind * P1 * P1 * P1;
}

// per-node Bessel scales k_l(kappa R), i_l(kappa R), l = 0..p
__global__ void k_fmm_node_radial(int nn, int p, double kappa, const double* __restrict__ radius, double* __restrict__ kR,
                                  double* __restrict__ kRi, double* __restrict__ iR) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const double z = kappa * radius[n];
  double sg[kPmaxFmm + 2], kk[kPmaxFmm + 2];
  sigma_all(z * z, p, sg);
  kbes_all(z, p, kk);
  double zl = 1.0;
  for (int l = 0; l <= p; ++l) {
    kR[n * (p + 1) + l] = kk[l];
    kRi[n * (p + 1) + l] = 1.0 / kk[l];
    iR[n * (p + 1) + l] = sg[l] * zl;
    zl *= z;
  }
}

// leaf expansions from per-sphere coefficients (degree ps, row stride lds), zero padded to degree p
__global__ void k_fmm_leaf_set(int M, int p, int ps, int lds, const int* __restrict__ sphere_leaf,
                               const double* __restrict__ src, double* __restrict__ E) {
  const int j = blockIdx.x;
  const int P = (p + 1) * (p + 1), Ps = (ps + 1) * (ps + 1);
  double* e = E + (long)sphere_leaf[j] * P;
  for (int t = threadIdx.x; t < P; t += blockDim.x) e[t] = t < Ps ? src[(long)j * lds + t] : 0.0;
}
// per-sphere coefficients (degree pd, row stride ldd) from leaf expansions; accumulate or overwrite
__global__ void k_fmm_leaf_get(int M, int p, int pd, int ldd, const int* __restrict__ sphere_leaf,
                               const double* __restrict__ E, int accumulate, double* __restrict__ dst) {
  const int j = blockIdx.x;
  const int P = (p + 1) * (p + 1), Pd = (pd + 1) * (pd + 1);
  const double* e = E + (long)sphere_leaf[j] * P;
  for (int t = threadIdx.x; t < Pd; t += blockDim.x) {
    const double v = t < P ? e[t] : 0.0;
    dst[(long)j * ldd + t] = accumulate ? dst[(long)j * ldd + t] + v : v;
  }
}

// Level passes: kLevelWaves wavefronts per block, each translating one node at a
// time (grid-stride over the level's nodes); the block stages the coefficient table
// of its translation kind (and, for Yukawa, the offsets of the packed table) in LDS
// once.  Dynamic LDS: level_lds_bytes().
constexpr int kLevelWaves = 8;
__host__ __device__ inline size_t level_table_doubles(int kernel, int p, int nA) {
  const size_t P1 = p + 1, P3 = P1 * P1 * P1;
  return kernel == 0 ? (size_t)nA + (P3 + 1) / 2 : P3;  // Yukawa: table, then the int offsets
}
__host__ __device__ inline size_t level_lds_bytes(int kernel, int p, int nA, int stage) {
  return ((stage ? level_table_doubles(kernel, p, nA) : 0) + (size_t)kLevelWaves * trans_view_doubles(p)) *
         sizeof(double);
}
__device__ __forceinline__ void stage_level_table(const FmmDev& f, int kind, int stage, double* tab, const double*& At,
                                                  const int*& Ao) {
  const int P1 = f.p + 1, P3 = P1 * P1 * P1;
  if (!stage) {  // table too large for LDS: read it from global memory
    At = coef_table(f, kind);
    Ao = f.Aoff;
    return;
  }
  if (f.kernel == 0) {
    int* off = (int*)(tab + f.nA);
    for (int t = threadIdx.x; t < f.nA; t += blockDim.x) tab[t] = f.A[t];
    for (int t = threadIdx.x; t < P3; t += blockDim.x) off[t] = f.Aoff[t];
    Ao = off;
  } else {
    const double* src = f.AL + (size_t)kind * P3;
    for (int t = threadIdx.x; t < P3; t += blockDim.x) tab[t] = src[t];
    Ao = f.Aoff;  // unused by the Laplace translations
  }
  At = tab;
  __syncthreads();
}

// upward pass of one level: M[n] = sum_children M2M(child -> n) M[child]  (internal nodes only)
__global__ __launch_bounds__(64 * kLevelWaves) void k_fmm_upward(FmmDev f, const int* __restrict__ nodes, int count,
                                                                 const int* __restrict__ child, int stage,
                                                                 double* __restrict__ E) {
  extern __shared__ double lvl_tab[];
  const double* At;
  const int* Ao;
  stage_level_table(f, 0, stage, lvl_tab, At, Ao);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  TransView sc;
  double* acc = carve_trans_view(
      lvl_tab + (stage ? level_table_doubles(f.kernel, f.p, f.nA) : 0) + (size_t)w * trans_view_doubles(f.p), f.p, sc);
  const int P = (f.p + 1) * (f.p + 1);
  for (int b = blockIdx.x * kLevelWaves + w; b < count; b += gridDim.x * kLevelWaves) {
    const int n = nodes[b];
    if (child[2 * n] < 0) continue;  // leaf: already set (uniform for the wavefront)
    for (int t = lane; t < P; t += 64) acc[t] = 0.0;
    for (int c = 0; c < 2; ++c) {
      const int ch = child[2 * n + c];
      tsync<true>();
      for (int t = lane; t < P; t += 64) sc.b0[t] = E[(long)ch * P + t];
      tsync<true>();
      translate<true>(f, At, Ao, 0, ch, n, f.p, f.p, 0, sc, acc);
    }
    for (int t = lane; t < P; t += 64) E[(long)n * P + t] = acc[t];
    tsync<true>();
  }
}

// multipole-to-local: L[T] = sum_{S in list(T)} M2L(S -> T) M[S]  (every node, lists by target)
// transposed: Mu[S] = sum_{T in list^T(S)} M2L(S -> T)^T Lambda[T]  (lists by source)
__global__ __launch_bounds__(64) void k_fmm_m2l(FmmDev f, int nn, const int* __restrict__ lptr,
                                                const int* __restrict__ lidx, int transposed,
                                                const double* __restrict__ Ein, double* __restrict__ Eout) {
  __shared__ TransScratch sc;
  __shared__ double acc[kPFmm];
  const int P = (f.p + 1) * (f.p + 1);
  for (int n = blockIdx.x; n < nn; n += gridDim.x) {
    for (int t = threadIdx.x; t < P; t += blockDim.x) acc[t] = 0.0;
    for (int q = lptr[n]; q < lptr[n + 1]; ++q) {
      const int o = lidx[q];
      __syncthreads();
      for (int t = threadIdx.x; t < P; t += blockDim.x) sc.b0[t] = Ein[(long)o * P + t];
      __syncthreads();
      if (!transposed) translate<false>(f, coef_table(f, 1), f.Aoff, 1, o, n, f.p, f.p, 0, sc, acc);
      else translate<false>(f, coef_table(f, 1), f.Aoff, 1, n, o, f.p, f.p, 1, sc, acc);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < P; t += blockDim.x) Eout[(long)n * P + t] = acc[t];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Multipole-to-local, one wavefront per translation, tables in LDS.
//
// Same operator as translate(kind 1) with the work laid out for a wavefront:
//   * the rotation angles enter only through cos/sin of m*phi and m*theta, taken as
//     integer powers of the unit complex numbers built from the centre offset
//     (no trigonometric calls);
//   * J and J^T are applied through their sparse rows (a quarter of the entries);
//   * the z translation is computed once per (l_out, |m|) pair and applied to +m and
//     -m, with each lane reading its coefficients contiguously and the pairs dealt
//     to lanes by longest-first balancing;
//   * the first rotation is fused with the load of the input expansion and the last
//     one with the accumulation, which stays in registers; the next source of the
//     list is fetched into registers while the current one is translated;
//   * wavefronts take target nodes from a counter in the order given by `order`
//     (longest lists first).
// LDS: the tables (shared by the block) followed by one scratch area per wavefront.
__host__ __device__ constexpr int m2l_fast_wave_doubles(int p) { return 2 * (p + 1) * (p + 1) + 8 * (p + 1); }

// order m of the lane's item i, packed 6 bits per item (offset 32)
__device__ __forceinline__ int item_m(int mpack, int i) { return ((mpack >> (6 * i)) & 63) - 32; }
__device__ __forceinline__ int item_l(int lpack, int i) { return (lpack >> (6 * i)) & 63; }

// in-place rotation about z by the angle with cos/sin of m*angle = ((-1)^m c[m], ss (-1)^m s[m])
// (pairs (l, +-m) handled by the lane of the +m entry)
template <int NI>
__device__ __forceinline__ void zrot_alt(double* b, int P, const double* c, const double* s, double ss, int lane,
                                         int mpack) {
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int t = lane + 64 * i, m = item_m(mpack, i);
    if (t < P && m > 0) {
      const double sg = (m & 1) ? -1.0 : 1.0;
      const double a = b[t], bb = b[t - 2 * m], co = sg * c[m], si = ss * sg * s[m];
      b[t] = a * co - bb * si;
      b[t - 2 * m] = a * si + bb * co;
    }
  }
}

// z-translation table of one M2L launch (kernel type and direction)
struct M2LTab {
  const double* Z;     // entries, see the host tables
  const int* slot;     // [nslot][2]: lo << 8 | |m| (or -1), offset
  const int* order;    // target node order (longest lists first)
  int* counter;        // work counter, zero at launch
  const double* jpad;  // rows of J and J^T padded per group of 64, [mat][g][k][lane]
  int nZ, nslot, njpad;
  int kpack;           // padded row length of group g in bits 4g..4g+3 (even)
};

// J or J^T (one matrix of the padded table, already offset by the lane) applied to
// src: lane row t = lane + 64 i sums K_i products with a step of 2 along src; the
// padding has zero values (its src reads stay inside the wavefront's scratch, which
// holds finite values only).  The trip counts are uniform over the wavefront.
template <int NI>
__device__ __forceinline__ void japply_pad(const double* v, const int* xb, int shift, int kpack,
                                           const double* src, double* dst, int lane, int P) {
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int K = (kpack >> (4 * i)) & 15;
    const double* x = src + ((xb[64 * i] >> shift) & 0xffff);
    double s = 0.0;
    for (int k = 0; k < K; k += 2) {
      s = fma(v[0], x[0], s);
      s = fma(v[64], x[2], s);
      v += 128;
      x += 4;
    }
    if (lane + 64 * i < P) dst[lane + 64 * i] = s;
  }
}

template <int NI, bool ALDS, bool YUK>
__global__ __launch_bounds__(1024) void k_fmm_m2l_fast(FmmDev f, M2LTab zt, int nn, const int* __restrict__ lptr,
                                                       const int* __restrict__ lidx, int transposed,
                                                       const double* __restrict__ Ein, double* __restrict__ Eout) {
  extern __shared__ double smem[];
  const int p = f.p, P1 = p + 1, P = P1 * P1;
  const int nw = blockDim.x >> 6;
  const int wd = m2l_fast_wave_doubles(p);
  // block-shared tables
  double* jv = smem;
  double* zl = jv + zt.njpad;
  double* wsb = zl + (ALDS ? zt.nZ : 0);
  int* zs = (int*)(wsb + nw * wd);
  int* xbl = zs + 2 * zt.nslot;  // [NI][64]: first column of row t of J (low 16 bits) and of J^T (high 16 bits)
  for (int t = threadIdx.x; t < zt.njpad; t += blockDim.x) jv[t] = zt.jpad[t];
  for (int t = threadIdx.x; t < 2 * zt.nslot; t += blockDim.x) zs[t] = zt.slot[t];
  for (int t = threadIdx.x; t < 64 * NI; t += blockDim.x)
    xbl[t] = t < P ? ((f.jrow[2 * t + 1] & 4095) | ((f.jrow[2 * (P + t) + 1] & 4095) << 16)) : 0;
  if constexpr (ALDS) {
    for (int t = threadIdx.x; t < zt.nZ; t += blockDim.x) zl[t] = zt.Z[t];
  }
  // the padded J reads may run past a vector into the scratch behind it: start finite
  for (int t = threadIdx.x; t < nw * wd; t += blockDim.x) wsb[t] = 0.0;
  __syncthreads();
  const double* Z;
  if constexpr (ALDS) Z = zl; else Z = zt.Z;

  // the wavefront index is uniform: keep it (and every scratch address) in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  double* b0 = wsb + w * wd;
  double* b1 = b0 + P;
  double* kt = b1 + P;         // k_n(z) z^n, n = 0..2p (2p+2)
  double* sIn = kt + 2 * P1;   // degree scale of the input
  double* sOut = sIn + P1;     // degree scale of the output
  double* cph = sOut + P1;
  double* sph = cph + P1;
  double* cth = sph + P1;
  double* sth = cth + P1;
  const int nj = zt.njpad / 2;

  // lane items t = lane + 64 i: degree and order, 6 bits each; first column of the J rows
  int mpack = 0, lpack = 0;
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int t = lane + 64 * i;
    const int l = (int)sqrtf((float)t + 0.5f);
    mpack |= ((t - l * l - l + 32) & 63) << (6 * i);
    lpack |= (l & 63) << (6 * i);
  }

  for (;;) {
    int k = 0;
    if (lane == 0) k = atomicAdd(zt.counter, 1);
    k = __builtin_amdgcn_readfirstlane(__shfl(k, 0));
    if (k >= nn) break;
    const int n = zt.order[k];
    const int q0 = lptr[n], q1 = lptr[n + 1];
    double acc[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) acc[i] = 0.0;
    // data of the fixed node n (target, or source when transposed): i_l(kappa R) or 1/k_l(kappa R)
    const double cnx = f.center[3 * n], cny = f.center[3 * n + 1], cnz = f.center[3 * n + 2];
    double rfix = 0.0;
    if (YUK && lane <= p) rfix = transposed ? f.kRi[n * P1 + lane] : f.iR[n * P1 + lane];
    // first source, fetched ahead
    double va[NI], vb[NI], vc = 0.0, vr = 0.0;
    auto fetch = [&](int o) {
      const double* src = Ein + (long)o * P;
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int t = lane + 64 * i;
        va[i] = t < P ? src[t] : 0.0;
        vb[i] = t < P ? src[t - 2 * item_m(mpack, i)] : 0.0;
      }
      vc = lane < 3 ? f.center[3 * o + lane] : 0.0;
      vr = 0.0;
      if (YUK && lane <= p) vr = transposed ? f.iR[o * P1 + lane] : f.kRi[o * P1 + lane];
    };
    if (q0 < q1) fetch(lidx[q0]);
    for (int q = q0; q < q1; ++q) {
      const double cox = __shfl(vc, 0), coy = __shfl(vc, 1), coz = __shfl(vc, 2);
      const double rvar = vr;
      const int o = lidx[q];
      const double dx = transposed ? cox - cnx : cnx - cox, dy = transposed ? coy - cny : cny - coy,
                   dz = transposed ? coz - cnz : cnz - coz;
      const double rxy = sqrt(dx * dx + dy * dy), rho = sqrt(dx * dx + dy * dy + dz * dz);
      const double irho = 1.0 / rho;
      tsync<true>();  // the previous translation is done with the per-translation tables
      if (lane <= p) {
        double c1 = 1.0, s1 = 0.0;
        if (rxy > 0.0) { const double ir = 1.0 / rxy; c1 = dx * ir; s1 = dy * ir; }
        cpow_d(c1, s1, lane, cph[lane], sph[lane]);
        cpow_d(dz * irho, rxy * irho, lane, cth[lane], sth[lane]);
        double u, v;  // source-degree and target-degree scales
        if constexpr (YUK) {
          // k-sum against k_n(z) z^n; z^-(l+l') (-1)^l and the node scales go to the degrees
          const double zi = irho * f.kinv;
          const double zl = ipow_d(zi, lane);
          const double rs = transposed ? rfix : rvar, rt = transposed ? rvar : rfix;
          u = rs * zl * ((lane & 1) ? -1.0 : 1.0);
          v = rt * zl;
        } else {
          const double RT = f.radius[transposed ? o : n], RS = f.radius[transposed ? n : o];
          u = ipow_d(RS * irho, lane + 1);
          v = ipow_d(RT * irho, lane);
        }
        sIn[lane] = transposed ? v : u;
        sOut[lane] = transposed ? u : v;
      }
      if (YUK && lane <= 2 * p) {
        // k_n(z) z^n by the upward recurrence kt_{n+1} = z^2 kt_{n-1} + (2n+1) kt_n
        const double z = f.kappa * rho, z2 = z * z;
        double km = 1.5707963267948966 * exp(-z) * irho * f.kinv;
        double kc = km * (z + 1.0), c = 3.0;  // km = kt_{j-1}, kc = kt_j, c = 2j + 1
        int j = 1;
        for (; j + 1 < lane; j += 2) {
          km = z2 * km + c * kc;
          kc = z2 * kc + (c + 2.0) * km;
          c += 4.0;
        }
        if (j < lane) {
          const double kn = z2 * km + c * kc;
          km = kc;
          kc = kn;
        }
        kt[lane] = lane == 0 ? km : kc;
      }
      tsync<true>();
      // input scaled by degree and rotated by -phi about z; then the next source is
      // fetched into the same registers
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        if (lane + 64 * i >= P) continue;
        const int m = item_m(mpack, i), am = m < 0 ? -m : m;
        double v = va[i];
        if (m > 0) v = va[i] * cph[am] + vb[i] * sph[am];
        else if (m < 0) v = va[i] * cph[am] - vb[i] * sph[am];
        b0[lane + 64 * i] = v * sIn[item_l(lpack, i)];
      }
      if (q + 1 < q1) fetch(lidx[q + 1]);
      tsync<true>();
      japply_pad<NI>(jv + lane, xbl + lane, 0, zt.kpack, b0, b1, lane, P);
      tsync<true>();
      zrot_alt<NI>(b1, P, cth, sth, -1.0, lane, mpack);  // pi - theta
      tsync<true>();
      japply_pad<NI>(jv + nj + lane, xbl + lane, 16, zt.kpack, b1, b0, lane, P);
      tsync<true>();
      // translation along z
      for (int s = lane; s < zt.nslot; s += 64) {
        const int code = zs[2 * s];
        if (code < 0) continue;
        const int lo = code >> 8, am = code & 255;
        const double* zp = Z + zs[2 * s + 1];
        double sp = 0.0, sm = 0.0;
        // running quantities at degree li: ib = li^2 + li, kp = kt + lo + li - am,
        // nk = min(lo, li) - am + 1 terms of the k-sum
        int ib = am * am + am, di = 2 * am + 2, nk = 1;
        const double* kp = kt + lo;
        for (int li = am; li <= p; ++li) {
          double e;
          if constexpr (YUK) {
            e = 0.0;
            for (int kk = 0; kk < nk; ++kk) e = fma(zp[kk], kp[-kk], e);
            zp += nk;
          } else {
            e = *zp++;
          }
          sp = fma(e, b0[ib + am], sp);
          sm = fma(e, b0[ib - am], sm);
          ib += di;
          di += 2;
          ++kp;
          nk += li < lo ? 1 : 0;
        }
        b1[lo * lo + lo + am] = sp;
        if (am) b1[lo * lo + lo - am] = sm;
      }
      tsync<true>();
      japply_pad<NI>(jv + lane, xbl + lane, 0, zt.kpack, b1, b0, lane, P);
      tsync<true>();
      zrot_alt<NI>(b0, P, cth, sth, 1.0, lane, mpack);  // theta - pi
      tsync<true>();
      japply_pad<NI>(jv + nj + lane, xbl + lane, 16, zt.kpack, b0, b1, lane, P);
      tsync<true>();
      // rotation by phi, scaled by degree, accumulated in registers
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        if (lane + 64 * i >= P) continue;
        const int m = item_m(mpack, i), am = m < 0 ? -m : m;
        const double a = b1[lane + 64 * i];
        double r = a;
        if (m != 0) {
          const double bm = b1[lane + 64 * i - 2 * m];
          r = m > 0 ? a * cph[am] - bm * sph[am] : bm * sph[am] + a * cph[am];
        }
        acc[i] += r * sOut[item_l(lpack, i)];
      }
    }
#pragma unroll
    for (int i = 0; i < NI; ++i)
      if (lane + 64 * i < P) Eout[(long)n * P + lane + 64 * i] = acc[i];
  }
}

// LDS bytes of k_fmm_m2l_fast for nw wavefronts per block
inline size_t m2l_fast_lds_bytes(int p, int nZ, int njpad, int nslot, int nw, bool alds) {
  const size_t d = (size_t)njpad + (alds ? (size_t)nZ : 0) + (size_t)nw * m2l_fast_wave_doubles(p);
  const size_t NI = ((size_t)(p + 1) * (p + 1) + 63) / 64;
  return d * sizeof(double) + (2 * (size_t)nslot + 64 * NI) * sizeof(int);
}

// downward pass of one level: L[n] += L2L(parent -> n) L[parent]
// transposed downward (adjoint of the upward pass): Mu[n] += M2M(n -> parent)^T Mu[parent]
__global__ __launch_bounds__(64 * kLevelWaves) void k_fmm_downward(FmmDev f, const int* __restrict__ nodes, int count,
                                                                   const int* __restrict__ parent, int transposed,
                                                                   int stage, double* __restrict__ E) {
  extern __shared__ double lvl_tab[];
  const double* At;
  const int* Ao;
  stage_level_table(f, transposed ? 0 : 2, stage, lvl_tab, At, Ao);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  TransView sc;
  double* acc = carve_trans_view(
      lvl_tab + (stage ? level_table_doubles(f.kernel, f.p, f.nA) : 0) + (size_t)w * trans_view_doubles(f.p), f.p, sc);
  const int P = (f.p + 1) * (f.p + 1);
  for (int b = blockIdx.x * kLevelWaves + w; b < count; b += gridDim.x * kLevelWaves) {
    const int n = nodes[b];
    const int par = parent[n];
    if (par < 0) continue;
    for (int t = lane; t < P; t += 64) { acc[t] = 0.0; sc.b0[t] = E[(long)par * P + t]; }
    tsync<true>();
    if (!transposed) translate<true>(f, At, Ao, 2, par, n, f.p, f.p, 0, sc, acc);
    else translate<true>(f, At, Ao, 0, n, par, f.p, f.p, 1, sc, acc);
    for (int t = lane; t < P; t += 64) E[(long)n * P + t] += acc[t];
    tsync<true>();
  }
}

// transposed upward pass of one level (adjoint of the downward pass):
// Lambda[n] += sum_children L2L(n -> child)^T Lambda[child]
__global__ __launch_bounds__(64 * kLevelWaves) void k_fmm_upward_T(FmmDev f, const int* __restrict__ nodes, int count,
                                                                   const int* __restrict__ child, int stage,
                                                                   double* __restrict__ E) {
  extern __shared__ double lvl_tab[];
  const double* At;
  const int* Ao;
  stage_level_table(f, 2, stage, lvl_tab, At, Ao);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  TransView sc;
  double* acc = carve_trans_view(
      lvl_tab + (stage ? level_table_doubles(f.kernel, f.p, f.nA) : 0) + (size_t)w * trans_view_doubles(f.p), f.p, sc);
  const int P = (f.p + 1) * (f.p + 1);
  for (int b = blockIdx.x * kLevelWaves + w; b < count; b += gridDim.x * kLevelWaves) {
    const int n = nodes[b];
    if (child[2 * n] < 0) continue;
    for (int t = lane; t < P; t += 64) acc[t] = 0.0;
    for (int c = 0; c < 2; ++c) {
      const int ch = child[2 * n + c];
      tsync<true>();
      for (int t = lane; t < P; t += 64) sc.b0[t] = E[(long)ch * P + t];
      tsync<true>();
      translate<true>(f, At, Ao, 2, n, ch, f.p, f.p, 1, sc, acc);
    }
    for (int t = lane; t < P; t += 64) E[(long)n * P + t] += acc[t];
    tsync<true>();
  }
}

}  // namespace ddlpb

namespace ddlpb {

// ---------------------------------------------------- sphere <-> grid glue
// Far field at the active points from the sphere locals SL [M][P] (scale r_i: a local
// evaluated on its own sphere has radial factor 1):
//   mode 0 (Yukawa):  out1 += sum SL Y(s_n)
//   mode 1 (Laplace): out1 += sum SL Y(s_n),  out2 += c2 sum (l / r_i) SL Y(s_n)  (normal derivative)
__global__ __launch_bounds__(256) void k_l2p(int nact, int N, int P, int LY, const int* __restrict__ act_sph,
                                             const int* __restrict__ act_n, const double* __restrict__ rad,
                                             const double* __restrict__ YT, const double* __restrict__ SL, int mode,
                                             double c2, double* __restrict__ out1, double* __restrict__ out2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nact) return;
  const int i = act_sph[k], n = act_n[k];
  const double* s = SL + (long)i * P;
  double v = 0.0, dn = 0.0;
  int l = 0;
  for (int t = 0; t < P; ++t) {
    if ((l + 1) * (l + 1) <= t) ++l;
    const double a = YT[(long)t * N + n] * s[t];
    v += a;
    dn += l * a;
  }
  const long in = (long)i * N + n;
  out1[in] += v;
  if (mode == 1) out2[in] += c2 * dn / rad[i];
}

// Dual of the grid evaluation: Lam_i,lm = sum_n (g1_in + (l/r_i) g2_in) Y_lm(s_n), l <= p
__global__ __launch_bounds__(256) void k_p2l_dual(int M, int N, int P, int LY, const double* __restrict__ rad,
                                                  const double* __restrict__ Y, const double* __restrict__ g1,
                                                  const double* __restrict__ g2, double* __restrict__ Lam) {
  __shared__ double a[kMaxN], b[kMaxN];
  const int i = blockIdx.x;
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    a[n] = g1[(long)i * N + n];
    b[n] = g2 ? g2[(long)i * N + n] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < P; t += blockDim.x) {
    const int l = (int)sqrt((double)t + 0.5);
    const double sl = l / rad[i];
    double s = 0.0;
    for (int n = 0; n < N; ++n) s += (a[n] + sl * b[n]) * Y[(long)n * LY + t];
    Lam[(long)i * P + t] = s;
  }
}

// Vacuum field by listed pairs (near part): psi += sum q_k/(eps1 d), e += (1/eps2) sum d_n(q_k / d)
__global__ __launch_bounds__(256) void k_laplace_field_list(int N, int nact, const int* __restrict__ act_sph,
                                                            const int* __restrict__ act_n, const double* __restrict__ xyz,
                                                            const double* __restrict__ rad, const double* __restrict__ leb,
                                                            const double* __restrict__ q, const int* __restrict__ lptr,
                                                            const int* __restrict__ lidx, double eps1, double eps2,
                                                            double* __restrict__ psi_out, double* __restrict__ e_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nact) return;
  const int i = act_sph[k], n = act_n[k];
  double p[3], s[3];
  for (int a = 0; a < 3; ++a) { s[a] = leb[4 * n + a]; p[a] = xyz[3 * i + a] + rad[i] * s[a]; }
  double psi = 0.0, dn = 0.0;
  for (int t = lptr[i]; t < lptr[i + 1]; ++t) {
    const int j = lidx[t];
    const double vx = p[0] - xyz[3 * j], vy = p[1] - xyz[3 * j + 1], vz = p[2] - xyz[3 * j + 2];
    const double id = 1.0 / sqrt(vx * vx + vy * vy + vz * vz);
    const double qi = q[j] * id;
    psi += qi;
    dn -= qi * id * id * (vx * s[0] + vy * s[1] + vz * s[2]);
  }
  const long in = (long)i * N + n;
  psi_out[in] += psi / eps1;
  e_out[in] += dn / eps2;
}

// Gradient (w.r.t. the point) of the far single-layer field from the Yukawa sphere local
// sum_lm SL_ilm i_l(kappa|v|)/i_l(kappa r_i) Y_lm(v), v = x - x_i, at every active point;
// added to gphi [nact][3].
template <int PD>
__global__ __launch_bounds__(128) void k_local_grad_yuk(int nact, const int* __restrict__ act_sph,
                                                        const int* __restrict__ act_n, const double* __restrict__ rad,
                                                        const double* __restrict__ leb, const double* __restrict__ iR_s,
                                                        int ldi, double kappa, int nterms,
                                                        const double* __restrict__ SL, double* __restrict__ gphi) {
  constexpr int P = (PD + 1) * (PD + 1);
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nact) return;
  const int i = act_sph[k], n = act_n[k];
  using D = Dual<double>;
  const double ri = rad[i], iri = 1.0 / ri;
  D v[3];
  for (int a = 0; a < 3; ++a) { v[a] = D(leb[4 * n + a]); v[a].g[a] = iri; }  // v = (x - x_i)/r_i, dv/dx = 1/r_i
  D z2 = (kappa * kappa * ri * ri) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  D sg[PD + 1];
  sigma_weights<PD, D>(z2, nterms, sg);
  const double* s = SL + (long)i * P;
  D part[PD + 1];
#pragma unroll
  for (int l = 0; l <= PD; ++l) part[l] = D(0.0);
  for_each_solid_harmonic<PD, D>(v[0], v[1], v[2], [&](int l, int idx, const D& S) { part[l] = part[l] + s[idx] * S; });
  D acc(0.0);
#pragma unroll
  for (int l = 0; l <= PD; ++l) acc = acc + (1.0 / iR_s[(long)i * ldi + l]) * (sg[l] * part[l]);
  for (int a = 0; a < 3; ++a) gphi[3L * k + a] += acc.g[a];
}

// Laplace far-field target terms at every active point from the sphere local of the
// vacuum field (value scale r_i): out[k] += c (xi_r grad psi + eta (eps1/eps2) grad (s . grad psi)),
// c = -1/2 w U; uses nested dual numbers for the Hessian.
template <int PD>
__global__ __launch_bounds__(128) void k_local_force_lap(int N, int nact, const int* __restrict__ act_sph,
                                                         const int* __restrict__ act_n, const double* __restrict__ rad,
                                                         const double* __restrict__ leb, const double* __restrict__ U,
                                                         const double* __restrict__ xr, const double* __restrict__ etag,
                                                         double eps1, double eps2, const double* __restrict__ SL,
                                                         double* __restrict__ fpt) {
  constexpr int P = (PD + 1) * (PD + 1);
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nact) return;
  const int i = act_sph[k], n = act_n[k];
  const long in = (long)i * N + n;
  using D = Dual<double>;
  using DD = Dual<D>;
  const double ri = rad[i], iri = 1.0 / ri;
  const double s[3] = {leb[4 * n], leb[4 * n + 1], leb[4 * n + 2]};
  DD v[3];
  for (int a = 0; a < 3; ++a) {
    D inner(s[a]);
    inner.g[a] = iri;  // inner derivative: gradient
    v[a] = DD(inner);
    D og(0.0);
    og.v = iri;        // outer derivative along axis a, value part
    for (int b = 0; b < 3; ++b) v[a].g[b] = D(0.0);
    v[a].g[a] = og;
  }
  const double* sl = SL + (long)i * P;
  DD acc(D(0.0));
  for_each_solid_harmonic<PD, DD>(v[0], v[1], v[2], [&](int l, int idx, const DD& S) { acc = acc + D(sl[idx]) * S; });
  // acc.g[a].v = d psi / dx_a ; acc.g[a].g[b] = d2 psi / dx_a dx_b
  const double c = -0.5 * leb[4 * n + 3] * U[in];
  const double ce = c * etag[in] * (eps1 / eps2);
  for (int a = 0; a < 3; ++a) {
    double hs = 0.0;
    for (int b = 0; b < 3; ++b) hs += acc.g[a].g[b] * s[b];
    fpt[3L * k + a] += c * xr[in] * acc.g[a].v + ce * hs;
  }
}

// Laplace source terms by listed pairs (near part): the charge k moves, the points of the
// listed spheres other than k do not.
__global__ __launch_bounds__(256) void k_force_laplace_source_list(int N, const int* __restrict__ act_ptr,
                                                                   const int* __restrict__ act_n,
                                                                   const double* __restrict__ xyz,
                                                                   const double* __restrict__ rad,
                                                                   const double* __restrict__ leb,
                                                                   const double* __restrict__ q, double eps1,
                                                                   double eps2, const double* __restrict__ U,
                                                                   const double* __restrict__ xr,
                                                                   const double* __restrict__ etag,
                                                                   const int* __restrict__ lptr,
                                                                   const int* __restrict__ lidx,
                                                                   double* __restrict__ out) {
  __shared__ double sh[32];
  const int kq = blockIdx.x;
  const double xk = xyz[3 * kq], yk = xyz[3 * kq + 1], zk = xyz[3 * kq + 2], qk = q[kq];
  Comp acc[3];
  for (int t = lptr[kq]; t < lptr[kq + 1]; ++t) {
    const int i = lidx[t];
    if (i == kq) continue;
    for (int kk = act_ptr[i] + threadIdx.x; kk < act_ptr[i + 1]; kk += blockDim.x) {
      const int n = act_n[kk];
      const long in = (long)i * N + n;
      const double c = -0.5 * leb[4 * n + 3] * U[in];
      const double a1 = c * xr[in] / eps1, a2 = c * etag[in] / eps2;
      const double s[3] = {leb[4 * n], leb[4 * n + 1], leb[4 * n + 2]};
      const double v3[3] = {xyz[3 * i] + rad[i] * s[0] - xk, xyz[3 * i + 1] + rad[i] * s[1] - yk,
                            xyz[3 * i + 2] + rad[i] * s[2] - zk};
      const double d2 = v3[0] * v3[0] + v3[1] * v3[1] + v3[2] * v3[2], id = 1.0 / sqrt(d2), id2 = id * id,
                   id3 = id2 * id;
      const double vs = v3[0] * s[0] + v3[1] * s[1] + v3[2] * s[2];
      for (int a = 0; a < 3; ++a)
        acc[a].add(-qk * (a1 * (-v3[a] * id3) + a2 * (3.0 * v3[a] * vs * id3 * id2 - s[a] * id3)));
    }
  }
  for (int c = 0; c < 3; ++c) {
    double s = block_sum_comp(acc[c], sh);
    if (threadIdx.x == 0) out[3L * kq + c] += s;
  }
}

// Laplace target terms by listed pairs (near part), charges k != i of the listed spheres
__global__ __launch_bounds__(256) void k_force_points_lap_list(int N, int nact, const int* __restrict__ act_sph,
                                                               const int* __restrict__ act_n,
                                                               const double* __restrict__ xyz,
                                                               const double* __restrict__ rad,
                                                               const double* __restrict__ leb,
                                                               const double* __restrict__ q, double eps1, double eps2,
                                                               const double* __restrict__ U,
                                                               const double* __restrict__ xr,
                                                               const double* __restrict__ etag,
                                                               const int* __restrict__ lptr,
                                                               const int* __restrict__ lidx,
                                                               double* __restrict__ fpt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nact) return;
  const int i = act_sph[k], n = act_n[k];
  const long in = (long)i * N + n;
  double p[3], s[3];
  for (int a = 0; a < 3; ++a) { s[a] = leb[4 * n + a]; p[a] = xyz[3 * i + a] + rad[i] * s[a]; }
  const double c = -0.5 * leb[4 * n + 3] * U[in];
  const double a1 = c * xr[in] / eps1, a2 = c * etag[in] / eps2;
  double acc[3] = {0, 0, 0};
  for (int t = lptr[i]; t < lptr[i + 1]; ++t) {
    const int j = lidx[t];
    if (j == i) continue;
    const double vx = p[0] - xyz[3 * j], vy = p[1] - xyz[3 * j + 1], vz = p[2] - xyz[3 * j + 2];
    const double d2 = vx * vx + vy * vy + vz * vz, id = 1.0 / sqrt(d2), id2 = id * id, id3 = id2 * id;
    const double qk = q[j];
    const double vs = vx * s[0] + vy * s[1] + vz * s[2];
    const double v3[3] = {vx, vy, vz};
    for (int a = 0; a < 3; ++a) acc[a] += qk * (a1 * (-v3[a] * id3) + a2 * (3.0 * v3[a] * vs * id3 * id2 - s[a] * id3));
  }
  for (int a = 0; a < 3; ++a) fpt[3L * k + a] += acc[a];
}

// grids of the source-side Laplace functional: g1 = c xi_r / eps1, g2 = c eta / eps2, c = -1/2 w U
__global__ void k_lap_src_grids(int M, int N, const double* __restrict__ leb, const double* __restrict__ U,
                                const double* __restrict__ xr, const double* __restrict__ etag, double eps1,
                                double eps2, double* __restrict__ g1, double* __restrict__ g2) {
  const long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (g >= (long)M * N) return;
  const int n = (int)(g % N);
  const double c = -0.5 * leb[4 * n + 3] * U[g];
  g1[g] = c * xr[g] / eps1;
  g2[g] = c * etag[g] / eps2;
}

// Near part of the charge derivative S_k (see k_dq_laplace_source): active points of the
// spheres in the near list of k (symmetric lists, k itself included).
__global__ __launch_bounds__(256) void k_dq_laplace_source_list(int N, const int* __restrict__ act_ptr,
                                                                const int* __restrict__ act_n,
                                                                const double* __restrict__ xyz,
                                                                const double* __restrict__ rad,
                                                                const double* __restrict__ leb, double eps1,
                                                                double eps2, const double* __restrict__ U,
                                                                const double* __restrict__ xr,
                                                                const double* __restrict__ etag,
                                                                const int* __restrict__ lptr,
                                                                const int* __restrict__ lidx, double* __restrict__ out) {
  __shared__ double sh[16];
  const int kq = blockIdx.x;
  const double xk = xyz[3 * kq], yk = xyz[3 * kq + 1], zk = xyz[3 * kq + 2];
  double acc = 0.0;
  for (int t = lptr[kq]; t < lptr[kq + 1]; ++t) {
    const int i = lidx[t];
    for (int kk = act_ptr[i] + threadIdx.x; kk < act_ptr[i + 1]; kk += blockDim.x) {
      const int n = act_n[kk];
      const long in = (long)i * N + n;
      const double c = -0.5 * leb[4 * n + 3] * U[in];
      const double a1 = c * xr[in] / eps1, a2 = c * etag[in] / eps2;
      const double s0 = leb[4 * n], s1 = leb[4 * n + 1], s2 = leb[4 * n + 2];
      const double v0 = xyz[3 * i] + rad[i] * s0 - xk, v1 = xyz[3 * i + 1] + rad[i] * s1 - yk,
                   v2 = xyz[3 * i + 2] + rad[i] * s2 - zk;
      const double id = 1.0 / sqrt(v0 * v0 + v1 * v1 + v2 * v2);
      acc += a1 * id - a2 * (v0 * s0 + v1 * s1 + v2 * s2) * id * id * id;
    }
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[kq] = s;
}
// dE/dq_k = 1/2 X_r,k00 / sqrt(4 pi) + S_k (near) + far part: the transposed Laplace FMM
// of the weights gives the dual of each charge's degree-0 source coefficient
// q sqrt(4 pi) / r_k (Mu_k[0]); Mu = nullptr in direct mode.
__global__ void k_dq_final(int M, int L, const double* __restrict__ X, const double* __restrict__ rad,
                           const double* __restrict__ Mu, int ldm, double* __restrict__ dq) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  double v = dq[k] + 0.5 * X[(long)k * L] * 0.28209479177387814;  // 1/sqrt(4 pi)
  if (Mu) v += Mu[(long)k * ldm] * 3.5449077018110318 / rad[k];  // sqrt(4 pi)
  dq[k] = v;
}

// Far Laplace source terms from the adjoint multipoles at the charges (degree >= 1):
// grad_{x_k} += q_k sqrt(4 pi/3)/r_k^2 (Mu_k[1,1], Mu_k[1,-1], Mu_k[1,0])
__global__ void k_force_lap_far_source(int M, int ldm, const double* __restrict__ q, const double* __restrict__ rad,
                                       const double* __restrict__ Mu, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const double f = q[k] * 2.0466534158929770 / (rad[k] * rad[k]);  // sqrt(4 pi / 3)
  out[3L * k + 0] += f * Mu[(long)k * ldm + 3];
  out[3L * k + 1] += f * Mu[(long)k * ldm + 1];
  out[3L * k + 2] += f * Mu[(long)k * ldm + 2];
}

}  // namespace ddlpb
