// Screened Coulomb multipole-to-local translations of order 12, one per lane, with the
// coefficient vector in FP32 (the mixed path): the operator of k_fmm_m2l_lane (same work
// layout, same rotations, same z-translation table), with
//   * the source expansion scaled per degree in FP64 and rounded once to FP32;
//   * the rotations (z-rotations, J, J^T) and the reduce-scatter over the 16 lanes of a
//     group in FP32 (J and J^T as FP32 constants);
//   * the translation along z in FP64: k_n(z) z^n, the coefficient sums and the output
//     scale per degree stay FP64 (their terms reach 1e44 at p = 12, beyond FP32), and the
//     translated vector is rounded to FP32 after the output scale, where its entries are
//     of the order of the result;
//   * the sums over the list chunks in FP64 (LDS).
// The vector takes 169 registers instead of 338, so a translation fits the register
// file without the scratch spills of the FP64 kernel.
#pragma once
#include "fmm_lane.hpp"

namespace ddlpb {
namespace lane12 {

static __constant__ float c_lane_jf[kJn];
static __constant__ float c_lane_jtf[kJTn];

typedef const __attribute__((address_space(4))) float cflt;
__device__ __forceinline__ cflt* pin(cflt* p, float dep) {
  asm volatile("" : "+s"(p) : "v"(dep));
  return p;
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int N, int CTRL>
__device__ __forceinline__ void rs_step_f(const float (&in)[N], float (&out)[(N + 1) / 2], bool bit) {
  sfor<(N + 1) / 2>([&](auto I_) {
    constexpr int i = decltype(I_)::value;
    const float x0 = in[2 * i];
    float x1 = 0.0f;
    if constexpr (2 * i + 1 < N) x1 = in[2 * i + 1];
    const float keep = bit ? x1 : x0, send = bit ? x0 : x1;
    out[i] = keep + dpp_f<CTRL>(send);
  });
}
__device__ __forceinline__ void cmul_step_f(float& c, float& s, float c1, float s1) {
  const float t = c * c1 - s * s1;
  s = s * c1 + c * s1;
  c = t;
}
template <int l, bool TRJ, int a>
__device__ __forceinline__ void jrow_load_f(float (&r)[kRowMax], float dep) {
  if constexpr (a <= 2 * l) {
    constexpr int off = entry_offset(TRJ, l, a, 0), cnt = row_count(TRJ, l, a);
    cflt* p = pin(TRJ ? (cflt*)c_lane_jtf : (cflt*)c_lane_jf, dep);
    sfor<cnt>([&](auto I_) {
      constexpr int i = decltype(I_)::value;
      r[i] = p[off + i];
    });
  }
}
template <int l, bool TRJ>
__device__ __forceinline__ void japply_f(const float (&b)[2 * l + 1], float (&c)[2 * l + 1]) {
  float cur[kRowMax], nxt[kRowMax];
  float dep = b[0];
  jrow_load_f<l, TRJ, 0>(cur, dep);
  sfor<2 * l + 1>([&](auto A_) {
    constexpr int a = decltype(A_)::value;
    jrow_load_f<l, TRJ, a + 1>(nxt, dep);
    float s = 0.0f;
    sfor<2 * l + 1>([&](auto B_) {
      constexpr int bb = decltype(B_)::value;
      if constexpr (pat(TRJ, l, a, bb)) {
        constexpr int k = [] {
          int c = 0;
          for (int x = 0; x < bb; ++x) c += pat(TRJ, l, a, x) ? 1 : 0;
          return c;
        }();
        s = fmaf(cur[k], b[bb], s);
      }
    });
    c[a] = s;
    dep = s;
#pragma unroll
    for (int x = 0; x < kRowMax; ++x) cur[x] = nxt[x];
  });
}

// TR: transposed pass (lists by source).  Every node in t.order is written.
template <bool TR>
__global__ __launch_bounds__(64 * kLaneWaves) void k_fmm_m2l_lane32(FmmDev f, LaneTab t, int nn,
                                                                  const int* __restrict__ lptr,
                                                                  const int* __restrict__ lidx,
                                                                  const double* __restrict__ Ein,
                                                                  double* __restrict__ Eout) {
  __shared__ double zsm[kZYn];
  __shared__ double accs[kOwn][64 * kLaneWaves];  // each lane's 11 running sums (FP64)
  for (int i = threadIdx.x; i < kZYn; i += blockDim.x) zsm[i] = t.Z[i];
  __syncthreads();  // the only barrier: afterwards every wavefront takes work on its own
  ldbl* zl = (ldbl*)zsm;
  const int lane = threadIdx.x & 63, j = lane & 15;
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
      double dx = 0.0, dy = 0.0, dz = 1.0;
      if (act) {
        const double ox = f.center[3 * o], oy = f.center[3 * o + 1], oz = f.center[3 * o + 2];
        dx = TR ? ox - cnx : cnx - ox;
        dy = TR ? oy - cny : cny - oy;
        dz = TR ? oz - cnz : cnz - oz;
      }
      const double rxy = sqrt(dx * dx + dy * dy), rho = sqrt(dx * dx + dy * dy + dz * dz);
      const double irho = 1.0 / rho;
      double c1d = 1.0, s1d = 0.0;
      if (rxy > 0.0) {
        const double ir = 1.0 / rxy;
        c1d = dx * ir;
        s1d = dy * ir;
      }
      const float c1 = (float)c1d, s1 = (float)s1d;
      const float ct = (float)(dz * irho), st = (float)(rxy * irho);
      // the list member's expansion times the input degree scales (screened Coulomb:
      // forward 1/k_l(kappa R_o) (-1)^l, transposed i_l(kappa R_o), times (kappa rho)^-l),
      // formed in FP64 and rounded once
      float v[kPP];
      {
        const double zi = irho * f.kinv;
        double zp = 1.0;
        const double* __restrict__ src = Ein + (long)o * kPP;
        sfor<kP1>([&](auto L_) {
          constexpr int l = decltype(L_)::value;
          const double sg = (l & 1) ? -1.0 : 1.0;
          const double ri = TR ? f.iR[o * kP1 + l] : sg * f.kRi[o * kP1 + l];
          const double sc = act ? ri * zp : 0.0;
#pragma unroll
          for (int a = 0; a < 2 * l + 1; ++a) v[l * l + a] = (float)(src[l * l + a] * sc);
          zp *= zi;
        });
      }
      // rotation into the frame whose z axis points from source to target, per degree
      sfor<kP1>([&](auto L_) {
        constexpr int l = decltype(L_)::value, w = 2 * l + 1;
        float b[w], cc[w];
        b[l] = v[l * l + l];
        float cm = 1.0f, sm = 0.0f;
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          cmul_step_f(cm, sm, c1, s1);
          const float a = v[l * l + l + m], bb = v[l * l + l - m];
          b[l + m] = a * cm + bb * sm;
          b[l - m] = bb * cm - a * sm;
        });
        japply_f<l, false>(b, cc);
        cm = 1.0f;
        sm = 0.0f;
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          cmul_step_f(cm, sm, ct, st);
          const float sg = (m & 1) ? -1.0f : 1.0f;
          const float co = sg * cm, si = -sg * sm;
          const float a = cc[l + m], bb = cc[l - m];
          cc[l + m] = a * co - bb * si;
          cc[l - m] = a * si + bb * co;
        });
        japply_f<l, true>(cc, b);
#pragma unroll
        for (int a = 0; a < w; ++a) v[l * l + a] = b[a];
      });
      // k_n(z) z^n, n = 0..2p (FP64)
      double kt[2 * kP + 1];
      {
        double rz = rho;
        asm volatile("" : "+v"(rz) : "v"(v[0]));
        const double z = f.kappa * rz, z2 = z * z;
        kt[0] = 1.5707963267948966 * exp(-z) / z;
        kt[1] = kt[0] * (z + 1.0);
        sfor<2 * kP - 1>([&](auto N_) {
          constexpr int nn1 = decltype(N_)::value + 1;
          kt[nn1 + 1] = z2 * kt[nn1 - 1] + (2.0 * nn1 + 1.0) * kt[nn1];
        });
      }
      // output degree scales (the fixed node n): forward i_l(kappa R_n), transposed
      // 1/k_l(kappa R_n) (-1)^l, times (kappa rho)^-l, applied in FP64 before rounding
      double sout[kP1];
      {
        const double zi = irho * f.kinv;
        double zp = 1.0;
        sfor<kP1>([&](auto L_) {
          constexpr int l = decltype(L_)::value;
          const double sg = (l & 1) ? -1.0 : 1.0;
          sout[l] = (TR ? sg * f.kRi[nf * kP1 + l] : f.iR[nf * kP1 + l]) * zp;
          zp *= zi;
        });
      }
      // translation along z per order |m| in FP64
      sfor<kP1>([&](auto AM_) {
        constexpr int am = decltype(AM_)::value, nb = kP1 - am, nt = zterm_count(true, am);
        double op[nb], om[nb];
#pragma unroll
        for (int x = 0; x < nb; ++x) { op[x] = 0.0; om[x] = 0.0; }
        double cur[kZChunk], nxt[kZChunk];
        double dep = (double)v[am * am + am], e = 0.0;
        zchunk_load<true, am, 0>(zl, cur, dep);
        sfor<nt>([&](auto T_) {
          constexpr int tt = decltype(T_)::value, pos = tt % kZChunk;
          constexpr ZTerm z = zterm(true, am, tt);
          if constexpr (pos == 0) zchunk_load<true, am, tt / kZChunk + 1>(zl, nxt, dep);
          e = z.k == 0 ? cur[pos] * kt[z.lo + z.li - am] : fma(cur[pos], kt[z.lo + z.li - am - z.k], e);
          if constexpr (z.k == z.n - 1) {
            op[z.lo - am] = fma(e, (double)v[z.li * z.li + z.li + am], op[z.lo - am]);
            if constexpr (am > 0) om[z.lo - am] = fma(e, (double)v[z.li * z.li + z.li - am], om[z.lo - am]);
            dep = e;
          }
          if constexpr (pos == kZChunk - 1) {
#pragma unroll
            for (int x = 0; x < kZChunk; ++x) cur[x] = nxt[x];
          }
        });
        sfor<nb>([&](auto LO_) {
          constexpr int lo = am + decltype(LO_)::value;
          v[lo * lo + lo + am] = (float)(op[lo - am] * sout[lo]);
          if constexpr (am > 0) v[lo * lo + lo - am] = (float)(om[lo - am] * sout[lo]);
        });
      });
      // back to the original frame: J, z-rotation by theta - pi, J^T, z-rotation by phi
      sfor<kP1>([&](auto L_) {
        constexpr int l = decltype(L_)::value, w = 2 * l + 1;
        float b[w], cc[w];
#pragma unroll
        for (int a = 0; a < w; ++a) b[a] = v[l * l + a];
        japply_f<l, false>(b, cc);
        float cm = 1.0f, sm = 0.0f;
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          cmul_step_f(cm, sm, ct, st);
          const float sg = (m & 1) ? -1.0f : 1.0f;
          const float co = sg * cm, si = sg * sm;
          const float a = cc[l + m], bb = cc[l - m];
          cc[l + m] = a * co - bb * si;
          cc[l - m] = a * si + bb * co;
        });
        japply_f<l, true>(cc, b);
        v[l * l + l] = b[l];
        cm = 1.0f;
        sm = 0.0f;
        sfor<l>([&](auto M_) {
          constexpr int m = decltype(M_)::value + 1;
          cmul_step_f(cm, sm, c1, s1);
          const float a = b[l + m], bm = b[l - m];
          v[l * l + l + m] = a * cm - bm * sm;
          v[l * l + l - m] = a * sm + bm * cm;
        });
      });
      // sum of the group's 16 vectors, scattered (FP32), then FP64 running sums
      float r1[85], r2[43], r3[22], r4[11];
      rs_step_f<kPP, 0x140>(v, r1, b3);
      rs_step_f<85, 0x141>(r1, r2, b2);
      rs_step_f<43, 0x4E>(r2, r3, b1);
      rs_step_f<22, 0xB1>(r3, r4, b0);
#pragma unroll
      for (int i = 0; i < kOwn; ++i) accs[i][threadIdx.x] += (double)r4[i];
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

// Host side of one FP32 instance (forward or transposed), in its own translation unit.
#define DDLPB_M2L_LANE32_INSTANCE(NAME, TR)                                                                 \
  namespace ddlpb {                                                                                       \
  namespace lane12 {                                                                                      \
  hipError_t upload_##NAME(const double* J, const double* JT) {                                           \
    float jf[kJn], jtf[kJTn];                                                                             \
    for (int i = 0; i < kJn; ++i) jf[i] = (float)J[i];                                                    \
    for (int i = 0; i < kJTn; ++i) jtf[i] = (float)JT[i];                                                 \
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_lane_jf), jf, sizeof(float) * kJn);                     \
    if (e != hipSuccess) return e;                                                                        \
    return hipMemcpyToSymbol(HIP_SYMBOL(c_lane_jtf), jtf, sizeof(float) * kJTn);                          \
  }                                                                                                       \
  hipError_t launch_##NAME(const FmmDev& f, const LaneTab& t, int nn, const int* lptr, const int* lidx,   \
                           const double* in, double* out, int blocks, hipStream_t s) {                    \
    hipLaunchKernelGGL((k_fmm_m2l_lane32<TR>), dim3(blocks), dim3(64 * kLaneWaves), 0, s, f, t, nn, lptr,  \
                       lidx, in, out);                                                                    \
    return hipGetLastError();                                                                             \
  }                                                                                                       \
  hipError_t occupancy_##NAME(int* blocks_per_cu) {                                                       \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                  \
        blocks_per_cu, reinterpret_cast<const void*>(&k_fmm_m2l_lane32<TR>), 64 * kLaneWaves, 0);          \
  }                                                                                                       \
  }                                                                                                       \
  }
