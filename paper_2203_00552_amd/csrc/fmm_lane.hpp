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

// (c, s) <- (c, s) * (c1, s1): the next power of the unit complex number c1 + i s1
// (cos and sin of the next multiple of the angle)
__device__ __forceinline__ void cmul_step(double& c, double& s, double c1, double s1) {
  const double t = c * c1 - s * s1;
  s = s * c1 + c * s1;
  c = t;
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

// The z translation of order |m| = am walks its coefficients as a flat sequence of
// terms (lo, li, k): output degree lo, input degree li and, for the screened Coulomb
// kernel, the k-th coefficient of the sum against k_n(z) z^n (n of them for the
// pair).  The table holds each (lo, am) row contiguously.
struct ZTerm {
  int lo, li, k, n, off;
};
constexpr int zterm_count(bool yuk, int am) {
  int c = 0;
  for (int lo = am; lo <= kP; ++lo)
    for (int li = am; li <= kP; ++li) c += yuk ? nks(lo, li, am) : 1;
  return c;
}
constexpr ZTerm zterm(bool yuk, int am, int t) {
  for (int lo = am; lo <= kP; ++lo)
    for (int li = am; li <= kP; ++li) {
      const int n = yuk ? nks(lo, li, am) : 1;
      if (t < n) return ZTerm{lo, li, t, n, zoff(yuk, lo, am, li) + t};
      t -= n;
    }
  return ZTerm{-1, -1, -1, 0, 0};
}
constexpr int kZChunk = 4;  // coefficients fetched per step, one step ahead

// the coefficients of chunk c of the terms of order am, from the table in LDS, into r
// (loaded after dep is known)
template <bool YUK, int am, int c>
__device__ __forceinline__ void zchunk_load(ldbl* zs, double (&r)[kZChunk], double dep) {
  constexpr int nt = zterm_count(YUK, am);
  if constexpr (c * kZChunk < nt) {
    ldbl* p = pin(zs, dep);
    sfor<kZChunk>([&](auto I_) {
      constexpr int t = c * kZChunk + decltype(I_)::value;
      if constexpr (t < nt) r[decltype(I_)::value] = p[zterm(YUK, am, t).off];
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
  __shared__ double accs[kOwn][64 * kLaneWaves];  // each lane's 11 running sums (own column)
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
#pragma unroll
    for (int i = 0; i < kOwn; ++i) accs[i][threadIdx.x] = 0.0;
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
      // cos / sin of m phi and m theta come from the recurrence of (cos a + i sin a)^m,
      // run again inside every degree (holding the tables would cost 104 registers)
      // degree scales of the input (the list member o): screened Coulomb forward
      // 1/k_l(kappa R_o) (-1)^l, transposed i_l(kappa R_o), times (kappa rho)^-l;
      // Coulomb forward (R_o/rho)^(l+1), transposed (R_o/rho)^l
      double sin_[kP1];
      if constexpr (YUK) {
        const double zi = irho * f.kinv;
        double zl = 1.0;
        sfor<kP1>([&](auto L_) {
          constexpr int l = decltype(L_)::value;
          const double sg = (l & 1) ? -1.0 : 1.0;
          const double ri = TR ? f.iR[o * kP1 + l] : sg * f.kRi[o * kP1 + l];
          sin_[l] = act ? ri * zl : 0.0;
          zl *= zi;
        });
      } else {
        const double Ro = f.radius[o] * irho;
        double pi = TR ? 1.0 : Ro;
        sfor<kP1>([&](auto L_) {
          constexpr int l = decltype(L_)::value;
          sin_[l] = act ? pi : 0.0;
          pi *= Ro;
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
        double cm = 1.0, sm = 0.0;
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          cmul_step(cm, sm, c1, s1);
          const double a = v[l * l + l + m], bb = v[l * l + l - m];
          b[l + m] = (a * cm + bb * sm) * sin_[l];
          b[l - m] = (bb * cm - a * sm) * sin_[l];
        });
        japply<l, false>(b, cc);
        cm = 1.0;
        sm = 0.0;
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          cmul_step(cm, sm, ct, st);
          const double sg = (m & 1) ? -1.0 : 1.0;
          const double co = sg * cm, si = -sg * sm;
          const double a = cc[l + m], bb = cc[l - m];
          cc[l + m] = a * co - bb * si;
          cc[l - m] = a * si + bb * co;
        });
        japply<l, true>(cc, b);
#pragma unroll
        for (int a = 0; a < w; ++a) v[l * l + a] = b[a];
      });
      // k_n(z) z^n, n = 0..2p, by the upward recurrence kt_{n+1} = z^2 kt_{n-1} + (2n+1) kt_n
      double kt[2 * kP + 1];
      if constexpr (YUK) {
        double rz = rho;
        asm volatile("" : "+v"(rz) : "v"(v[0]));  // computed here, after the first rotation
        const double z = f.kappa * rz, z2 = z * z;
        kt[0] = 1.5707963267948966 * exp(-z) / z;
        kt[1] = kt[0] * (z + 1.0);
        sfor<2 * kP - 1>([&](auto N_) {
          constexpr int nn1 = decltype(N_)::value + 1;
          kt[nn1 + 1] = z2 * kt[nn1 - 1] + (2.0 * nn1 + 1.0) * kt[nn1];
        });
      }
      // translation along z, per order |m| (the same matrix for +m and -m); the
      // coefficients are fetched a chunk ahead
      sfor<kP1>([&](auto AM_) {
        constexpr int am = decltype(AM_)::value, nb = kP1 - am, nt = zterm_count(YUK, am);
        double op[nb], om[nb];
#pragma unroll
        for (int x = 0; x < nb; ++x) { op[x] = 0.0; om[x] = 0.0; }
        double cur[kZChunk], nxt[kZChunk];
        double dep = v[am * am + am], e = 0.0;
        zchunk_load<YUK, am, 0>(zl, cur, dep);
        sfor<nt>([&](auto T_) {
          constexpr int t = decltype(T_)::value, pos = t % kZChunk;
          constexpr ZTerm z = zterm(YUK, am, t);
          if constexpr (pos == 0) zchunk_load<YUK, am, t / kZChunk + 1>(zl, nxt, dep);
          if constexpr (YUK) {
            e = z.k == 0 ? cur[pos] * kt[z.lo + z.li - am] : fma(cur[pos], kt[z.lo + z.li - am - z.k], e);
          } else {
            e = cur[pos];
          }
          if constexpr (z.k == z.n - 1) {
            op[z.lo - am] = fma(e, v[z.li * z.li + z.li + am], op[z.lo - am]);
            if constexpr (am > 0) om[z.lo - am] = fma(e, v[z.li * z.li + z.li - am], om[z.lo - am]);
            dep = e;
          }
          if constexpr (pos == kZChunk - 1) {
#pragma unroll
            for (int x = 0; x < kZChunk; ++x) cur[x] = nxt[x];
          }
        });
        sfor<nb>([&](auto LO_) {
          constexpr int lo = am + decltype(LO_)::value;
          v[lo * lo + lo + am] = op[lo - am];
          if constexpr (am > 0) v[lo * lo + lo - am] = om[lo - am];
        });
      });
      // degree scales of the output (the fixed node n): screened Coulomb forward
      // i_l(kappa R_n), transposed 1/k_l(kappa R_n) (-1)^l, times (kappa rho)^-l;
      // Coulomb forward (R_n/rho)^l, transposed (R_n/rho)^(l+1); read after the
      // translation so that they are not held across it
      double sout[kP1];
      {
        int nfp = nf;
        double irp = irho;
        asm volatile("" : "+v"(nfp), "+v"(irp) : "v"(v[0]));
        if constexpr (YUK) {
          const double zi = irp * f.kinv;
          double zl = 1.0;
          sfor<kP1>([&](auto L_) {
            constexpr int l = decltype(L_)::value;
            const double sg = (l & 1) ? -1.0 : 1.0;
            sout[l] = (TR ? sg * f.kRi[nfp * kP1 + l] : f.iR[nfp * kP1 + l]) * zl;
            zl *= zi;
          });
        } else {
          const double Rn = f.radius[nfp] * irp;
          double po = TR ? Rn : 1.0;
          sfor<kP1>([&](auto L_) {
            constexpr int l = decltype(L_)::value;
            sout[l] = po;
            po *= Rn;
          });
        }
      }
      // back to the original frame: J, z-rotation by theta - pi, J^T, z-rotation by
      // phi with the output scale
      sfor<kP1>([&](auto L_) {
        constexpr int l = decltype(L_)::value, w = 2 * l + 1;
        double b[w], cc[w];
#pragma unroll
        for (int a = 0; a < w; ++a) b[a] = v[l * l + a];
        japply<l, false>(b, cc);
        double cm = 1.0, sm = 0.0;
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          cmul_step(cm, sm, ct, st);
          const double sg = (m & 1) ? -1.0 : 1.0;
          const double co = sg * cm, si = sg * sm;
          const double a = cc[l + m], bb = cc[l - m];
          cc[l + m] = a * co - bb * si;
          cc[l - m] = a * si + bb * co;
        });
        japply<l, true>(cc, b);
        v[l * l + l] = b[l] * sout[l];
        cm = 1.0;
        sm = 0.0;
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          cmul_step(cm, sm, c1, s1);
          const double a = b[l + m], bm = b[l - m];
          v[l * l + l + m] = (a * cm - bm * sm) * sout[l];
          v[l * l + l - m] = (a * sm + bm * cm) * sout[l];
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
      for (int i = 0; i < kOwn; ++i) accs[i][threadIdx.x] += r4[i];
    }
    if (n >= 0) {
#pragma unroll
      for (int i = 0; i < kOwn; ++i) {
        const int k = kGroup * i + jr;
        if (k < kPP) Eout[(long)n * kPP + k] = accs[i][threadIdx.x];
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
