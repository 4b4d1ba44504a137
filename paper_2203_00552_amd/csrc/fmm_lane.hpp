// Multipole-to-local translations of order p = 12 with one translation per lane.
//
// The operator is the one of k_fmm_m2l_fast (rotation-based translation of the
// Appendix: z-rotation by the azimuth, the fixed 90-degree rotation J, z-rotation
// by the polar angle, J^T, the translation along z, and the inverse rotations),
// written for a different mapping onto the wavefront: every lane carries one whole
// translation, with its 169-coefficient vector in registers, and the program is
// unrolled at compile time, so every index (degree, order, table position) is a
// constant and every instruction works for 64 translations at once.
//
// Work layout: a wavefront is four groups of 16 lanes; a group takes one fixed node
// n (the target; the source of the transposed pass) and walks its interaction list
// 16 entries at a time, one list entry per lane.  The 16 translated vectors of a
// chunk are summed across the group by a reduce-scatter over DPP row permutations
// (after which each lane owns 11 of the 169 sums) and accumulated in registers, so
// the result is a fixed-order sum: bitwise reproducible, no atomics.
//
// Sparsity of J (rotation by +90 degrees about x, real harmonics without the
// Condon-Shortley phase): J commutes with the reflection x -> -x, so rows and
// columns have equal parity under it (order m >= 0: m mod 2; m < 0: (|m| + 1) mod
// 2), and it maps the reflection y -> -y onto z -> -z, so a row of z-parity
// (-1)^(l + |m|) = +1 only meets columns of cosine type (m >= 0) and the others
// only sine-type columns.  The host checks the numerical J against this pattern
// before the kernel is used.
#pragma once
#include <utility>

#include <hip/hip_runtime.h>

#include "fmm_types.hpp"
#include "fmm_lane_api.hpp"

namespace ddlpb {
namespace lane12 {

constexpr int kRowMax = kP + 1;  // longest row of J or J^T
// z-translation coefficients of one (lo, li, |m|) entry: at most p + 1
constexpr int kZMax = kP + 1;

// J and J^T in their pattern orders (rows contiguous), shared by every context on a
// device (uploaded once; they depend on p only).  Constant address space: uniform
// reads are scalar loads through the scalar cache, which holds both (12 KB).
static __constant__ double c_lane_j[kJn];
static __constant__ double c_lane_jt[kJTn];

// Table pointers in the constant (4) and LDS (3) address spaces.  pin() passes a
// pointer through an empty asm statement that also reads `dep`: the loads through the
// result stay after the value `dep` is computed and are neither hoisted out of the
// loops nor merged with equal loads elsewhere, which bounds how long the loaded
// constants live (all the table reads are otherwise loop invariant).
typedef const __attribute__((address_space(4))) double cdbl;
typedef const __attribute__((address_space(3))) double ldbl;
__device__ __forceinline__ cdbl* pin(cdbl* p, double dep) {
  asm volatile("" : "+s"(p) : "v"(dep));
  return p;
}
__device__ __forceinline__ ldbl* pin(ldbl* p, double dep) {
  asm volatile("" : "+v"(p) : "v"(dep));
  return p;
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

// value of lane (this lane's DPP partner) for a double: both halves moved
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One step of the reduce-scatter over a 16-lane row: the partner (DPP pattern CTRL)
// holds the same index set; this lane keeps the odd or the even entries (bit) and
// receives the partner's copies of them.
template <int N, int CTRL>
__device__ __forceinline__ void rs_step(const double (&in)[N], double (&out)[(N + 1) / 2], bool bit) {
  sfor<(N + 1) / 2>([&](auto I_) {
    constexpr int i = decltype(I_)::value;
    const double x0 = in[2 * i];
    double x1 = 0.0;
    if constexpr (2 * i + 1 < N) x1 = in[2 * i + 1];
    const double keep = bit ? x1 : x0, send = bit ? x0 : x1;
    out[i] = keep + dpp_d<CTRL>(send);
  });
}

// cos(m a), sin(m a) for m = 0..p of the two rotation angles, by the recurrence of
// (cos a + i sin a)^m
__device__ __forceinline__ void trig_tables(double c1, double s1, double ct, double st, double (&cph)[kP1],
                                            double (&sph)[kP1], double (&cth)[kP1], double (&sth)[kP1]) {
  cph[0] = 1.0; sph[0] = 0.0; cth[0] = 1.0; sth[0] = 0.0;
  sfor<kP>([&](auto M_) {
    constexpr int m = decltype(M_)::value + 1;
    cph[m] = cph[m - 1] * c1 - sph[m - 1] * s1;
    sph[m] = sph[m - 1] * c1 + cph[m - 1] * s1;
    cth[m] = cth[m - 1] * ct - sth[m - 1] * st;
    sth[m] = sth[m - 1] * ct + cth[m - 1] * st;
  });
}


// the pattern entries of row a of J (TRJ false) or J^T (TRJ true), degree l, into r
// (loaded after dep is known)
template <int l, bool TRJ, int a>
__device__ __forceinline__ void jrow_load(double (&r)[kRowMax], double dep) {
  if constexpr (a <= 2 * l) {
    constexpr int off = entry_offset(TRJ, l, a, 0), cnt = row_count(TRJ, l, a);
    cdbl* p = pin(TRJ ? (cdbl*)c_lane_jt : (cdbl*)c_lane_j, dep);
    sfor<cnt>([&](auto I_) {
      constexpr int i = decltype(I_)::value;
      r[i] = p[off + i];
    });
  }
}
// J or J^T on the degree-l block b (2l+1 entries) -> c; the constants of row a + 1
// are fetched while row a is applied (after row a - 1 is done)
template <int l, bool TRJ>
__device__ __forceinline__ void japply(const double (&b)[2 * l + 1], double (&c)[2 * l + 1]) {
  double cur[kRowMax], nxt[kRowMax];
  double dep = b[0];
  jrow_load<l, TRJ, 0>(cur, dep);
  sfor<2 * l + 1>([&](auto A_) {
    constexpr int a = decltype(A_)::value;
    jrow_load<l, TRJ, a + 1>(nxt, dep);
    double s = 0.0;
    sfor<2 * l + 1>([&](auto B_) {
      constexpr int bb = decltype(B_)::value;
      if constexpr (pat(TRJ, l, a, bb)) {
        constexpr int k = [] {
          int c = 0;
          for (int x = 0; x < bb; ++x) c += pat(TRJ, l, a, x) ? 1 : 0;
          return c;
        }();
        s = fma(cur[k], b[bb], s);
      }
    });
    c[a] = s;
    dep = s;
#pragma unroll
    for (int x = 0; x < kRowMax; ++x) cur[x] = nxt[x];
  });
}

// the coefficients of one (lo, li, |m|) entry of the z translation from the table in
// LDS into r (loaded after dep is known)
template <bool YUK, int lo, int am, int li>
__device__ __forceinline__ void zrow_load(ldbl* zs, double (&r)[kZMax], double dep) {
  if constexpr (lo <= kP && li <= kP) {
    constexpr int off = zoff(YUK, lo, am, li), cnt = YUK ? nks(lo, li, am) : 1;
    ldbl* p = pin(zs, dep);
    sfor<cnt>([&](auto I_) {
      constexpr int i = decltype(I_)::value;
      r[i] = p[off + i];
    });
  }
}

// YUK: screened Coulomb (else Coulomb) expansions; TR: transposed pass (lists by
// source, Mu[S] = sum_T M2L(S -> T)^T Lambda[T]).  Every node in t.order is written.
template <bool YUK, bool TR>
__global__ __launch_bounds__(64 * kLaneWaves) void k_fmm_m2l_lane(FmmDev f, LaneTab t, int nn,
                                                                const int* __restrict__ lptr,
                                                                const int* __restrict__ lidx,
                                                                const double* __restrict__ Ein,
                                                                double* __restrict__ Eout) {
  __shared__ double zsm[kZYn];
  for (int i = threadIdx.x; i < (YUK ? kZYn : kZLn); i += blockDim.x) zsm[i] = t.Z[i];
  __syncthreads();  // the only barrier: afterwards every wavefront takes work on its own
  ldbl* zl = (ldbl*)zsm;
  const int lane = threadIdx.x & 63, j = lane & 15;
  // this lane's sums after the reduce-scatter: entries 16 i + rev4(j)
  const int jr = ((j & 1) << 3) | ((j & 2) << 1) | ((j & 4) >> 1) | ((j & 8) >> 3);
  const bool b3 = (j >> 3) & 1, b2 = (j >> 2) & 1, b1 = (j >> 1) & 1, b0 = j & 1;
  for (;;) {
    int k0 = 0;
    if (lane == 0) k0 = atomicAdd(t.counter, 64 / kGroup);
    k0 = __builtin_amdgcn_readfirstlane(__shfl(k0, 0));
    if (k0 >= nn) break;
    const int kk = k0 + (lane >> 4);
    const int n = kk < nn ? t.order[kk] : -1;
    const int q0 = n >= 0 ? lptr[n] : 0, q1 = n >= 0 ? lptr[n + 1] : 0;
    int mx = q1 - q0;
    mx = max(mx, __shfl_xor(mx, 16));
    mx = max(mx, __shfl_xor(mx, 32));
    mx = __builtin_amdgcn_readfirstlane(mx);
    const int nf = n >= 0 ? n : 0;
    const double cnx = f.center[3 * nf], cny = f.center[3 * nf + 1], cnz = f.center[3 * nf + 2];
    double acc[kOwn];
#pragma unroll
    for (int i = 0; i < kOwn; ++i) acc[i] = 0.0;
    for (int c = 0; c < mx; c += kGroup) {
      const int q = q0 + c + j;
      const bool act = q < q1;
      const int o = act ? lidx[q] : 0;
      // offset from the source centre to the target centre
      double dx = 0.0, dy = 0.0, dz = 1.0;
      if (act) {
        const double ox = f.center[3 * o], oy = f.center[3 * o + 1], oz = f.center[3 * o + 2];
        dx = TR ? ox - cnx : cnx - ox;
        dy = TR ? oy - cny : cny - oy;
        dz = TR ? oz - cnz : cnz - oz;
      }
      const double rxy = sqrt(dx * dx + dy * dy), rho = sqrt(dx * dx + dy * dy + dz * dz);
      const double irho = 1.0 / rho;
      double c1 = 1.0, s1 = 0.0;
      if (rxy > 0.0) {
        const double ir = 1.0 / rxy;
        c1 = dx * ir;
        s1 = dy * ir;
      }
      const double ct = dz * irho, st = rxy * irho;
      // cos / sin of m phi and m theta (recomputed for the second rotation so that the
      // tables are not held across the z translation)
      double cph[kP1], sph[kP1], cth[kP1], sth[kP1];
      trig_tables(c1, s1, ct, st, cph, sph, cth, sth);
      // degree scales of the input (list member o) and of the output (fixed node n)
      double sin_[kP1], sout[kP1];
      if constexpr (YUK) {
        const double zi = irho * f.kinv;
        double zl = 1.0;
        sfor<kP1>([&](auto L_) {
          constexpr int l = decltype(L_)::value;
          const double sg = (l & 1) ? -1.0 : 1.0;
          // forward: source o (1/k_l(kappa R_o), (-1)^l), target n (i_l(kappa R_n));
          // transposed: the roles of the two scales are exchanged
          const double ri = TR ? f.iR[o * kP1 + l] : sg * f.kRi[o * kP1 + l];
          const double ro = TR ? sg * f.kRi[nf * kP1 + l] : f.iR[nf * kP1 + l];
          sin_[l] = act ? ri * zl : 0.0;
          sout[l] = ro * zl;
          zl *= zi;
        });
      } else {
        const double Ro = f.radius[o] * irho, Rn = f.radius[nf] * irho;
        // forward: (R_S/rho)^(l+1) in, (R_T/rho)^l out; transposed: (R_T/rho)^l in, (R_S/rho)^(l+1) out
        double pi = TR ? 1.0 : Ro, po = TR ? Rn : 1.0;
        sfor<kP1>([&](auto L_) {
          constexpr int l = decltype(L_)::value;
          sin_[l] = act ? pi : 0.0;
          sout[l] = po;
          pi *= Ro;
          po *= Rn;
        });
      }
      // k_n(z) z^n, n = 0..2p, by the upward recurrence kt_{n+1} = z^2 kt_{n-1} + (2n+1) kt_n
      double kt[2 * kP + 1];
      if constexpr (YUK) {
        const double z = f.kappa * rho, z2 = z * z;
        kt[0] = 1.5707963267948966 * exp(-z) * irho * f.kinv;
        kt[1] = kt[0] * (z + 1.0);
        sfor<2 * kP - 1>([&](auto N_) {
          constexpr int nn1 = decltype(N_)::value + 1;
          kt[nn1 + 1] = z2 * kt[nn1 - 1] + (2.0 * nn1 + 1.0) * kt[nn1];
        });
      }
      // the list member's expansion
      double v[kPP];
      {
        const double* __restrict__ src = Ein + (long)o * kPP;
#pragma unroll
        for (int k = 0; k < kPP; ++k) v[k] = src[k];
      }
      // rotation into the frame whose z axis points from source to target, per degree:
      // z-rotation by phi with the input scale, J, z-rotation by pi - theta, J^T
      sfor<kP1>([&](auto L_) {
        constexpr int l = decltype(L_)::value, w = 2 * l + 1;
        double b[w], cc[w];
        b[l] = v[l * l + l] * sin_[l];
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          const double a = v[l * l + l + m], bb = v[l * l + l - m];
          b[l + m] = (a * cph[m] + bb * sph[m]) * sin_[l];
          b[l - m] = (bb * cph[m] - a * sph[m]) * sin_[l];
        });
        japply<l, false>(b, cc);
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          const double sg = (m & 1) ? -1.0 : 1.0;
          const double co = sg * cth[m], si = -sg * sth[m];
          const double a = cc[l + m], bb = cc[l - m];
          cc[l + m] = a * co - bb * si;
          cc[l - m] = a * si + bb * co;
        });
        japply<l, true>(cc, b);
#pragma unroll
        for (int a = 0; a < w; ++a) v[l * l + a] = b[a];
      });
      // translation along z, per order |m| (the same matrix for +m and -m); the
      // coefficients of the next (lo, li) entry are fetched while one is applied
      sfor<kP1>([&](auto AM_) {
        constexpr int am = decltype(AM_)::value, nb = kP1 - am;
        double op[nb], om[nb];
#pragma unroll
        for (int x = 0; x < nb; ++x) { op[x] = 0.0; om[x] = 0.0; }
        double zc[kZMax], zn[kZMax];
        double dep = v[am * am + am];
        zrow_load<YUK, am, am, am>(zl, zc, dep);
        sfor<nb * nb>([&](auto G_) {
          constexpr int g = decltype(G_)::value, lo = am + g / nb, li = am + g % nb;
          constexpr int g2 = g + 1, lo2 = am + g2 / nb, li2 = am + g2 % nb;
          if constexpr (g2 < nb * nb) zrow_load<YUK, lo2, am, li2>(zl, zn, dep);
          double e;
          if constexpr (YUK) {
            e = 0.0;
            sfor<nks(lo, li, am)>([&](auto K_) {
              constexpr int q2 = decltype(K_)::value;
              e = fma(zc[q2], kt[lo + li - am - q2], e);
            });
          } else {
            e = zc[0];
          }
          op[lo - am] = fma(e, v[li * li + li + am], op[lo - am]);
          if constexpr (am > 0) om[lo - am] = fma(e, v[li * li + li - am], om[lo - am]);
          dep = e;
#pragma unroll
          for (int x = 0; x < kZMax; ++x) zc[x] = zn[x];
        });
        sfor<nb>([&](auto LO_) {
          constexpr int lo = am + decltype(LO_)::value;
          v[lo * lo + lo + am] = op[lo - am];
          if constexpr (am > 0) v[lo * lo + lo - am] = om[lo - am];
        });
      });
      // back to the original frame: J, z-rotation by theta - pi, J^T, z-rotation by
      // phi with the output scale
      {
        double c1b = c1, s1b = s1, ctb = ct, stb = st;
        asm volatile("" : "+v"(c1b), "+v"(s1b), "+v"(ctb), "+v"(stb));  // a fresh evaluation, not a reuse
        trig_tables(c1b, s1b, ctb, stb, cph, sph, cth, sth);
      }
      sfor<kP1>([&](auto L_) {
        constexpr int l = decltype(L_)::value, w = 2 * l + 1;
        double b[w], cc[w];
#pragma unroll
        for (int a = 0; a < w; ++a) b[a] = v[l * l + a];
        japply<l, false>(b, cc);
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          const double sg = (m & 1) ? -1.0 : 1.0;
          const double co = sg * cth[m], si = sg * sth[m];
          const double a = cc[l + m], bb = cc[l - m];
          cc[l + m] = a * co - bb * si;
          cc[l - m] = a * si + bb * co;
        });
        japply<l, true>(cc, b);
        v[l * l + l] = b[l] * sout[l];
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          const double a = b[l + m], bm = b[l - m];
          v[l * l + l + m] = (a * cph[m] - bm * sph[m]) * sout[l];
          v[l * l + l - m] = (a * sph[m] + bm * cph[m]) * sout[l];
        });
      });
      // sum of the group's 16 vectors, scattered: afterwards this lane holds the sums of
      // entries 16 i + rev4(j)
      double r1[85], r2[43], r3[22], r4[11];
      rs_step<kPP, 0x140>(v, r1, b3);   // row mirror: partner 15 - j
      rs_step<85, 0x141>(r1, r2, b2);   // row half mirror: partner 7 - j within eight lanes
      rs_step<43, 0x4E>(r2, r3, b1);    // quad permutation (2, 3, 0, 1)
      rs_step<22, 0xB1>(r3, r4, b0);    // quad permutation (1, 0, 3, 2)
#pragma unroll
      for (int i = 0; i < kOwn; ++i) acc[i] += r4[i];
    }
    if (n >= 0) {
#pragma unroll
      for (int i = 0; i < kOwn; ++i) {
        const int k = kGroup * i + jr;
        if (k < kPP) Eout[(long)n * kPP + k] = acc[i];
      }
    }
  }
}

}  // namespace lane12
}  // namespace ddlpb

// Host side of one instance, defined in the translation unit that instantiates it
// (m2l_lane_*.hip): the tables of that unit's copy of the constant arrays, and the
// launch.
#define DDLPB_M2L_LANE_INSTANCE(NAME, YUK, TR)                                                              \
  namespace ddlpb {                                                                                       \
  namespace lane12 {                                                                                      \
  hipError_t upload_##NAME(const double* J, const double* JT) {                                           \
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_lane_j), J, sizeof(double) * kJn);                      \
    if (e != hipSuccess) return e;                                                                        \
    return hipMemcpyToSymbol(HIP_SYMBOL(c_lane_jt), JT, sizeof(double) * kJTn);                           \
  }                                                                                                       \
  hipError_t launch_##NAME(const FmmDev& f, const LaneTab& t, int nn, const int* lptr, const int* lidx,   \
                           const double* in, double* out, int blocks, hipStream_t s) {                    \
    hipLaunchKernelGGL((k_fmm_m2l_lane<YUK, TR>), dim3(blocks), dim3(64 * kLaneWaves), 0, s, f, t, nn, lptr, \
                       lidx, in, out);                                                                    \
    return hipGetLastError();                                                                             \
  }                                                                                                       \
  hipError_t occupancy_##NAME(int* blocks_per_cu) {                                                       \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                  \
        blocks_per_cu, reinterpret_cast<const void*>(&k_fmm_m2l_lane<YUK, TR>), 64 * kLaneWaves, 0);       \
  }                                                                                                       \
  }                                                                                                       \
  }
