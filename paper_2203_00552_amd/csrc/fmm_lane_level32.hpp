// Screened Coulomb multipole-to-multipole and local-to-local translations of order 12,
// one per lane, with the coefficient vector in FP32 (the mixed path): the operator of
// k_fmm_level_lane with the split of k_fmm_m2l_lane32 -- the input times its degree
// scales formed in FP64 and rounded once, the rotations in FP32, the translation along z
// (sigma_n(z^2), the coefficient sums) and the output degree scales in FP64, the result
// rounded after the output scale and accumulated into the FP64 node rows.
#pragma once
#include "fmm_lane32.hpp"

namespace ddlpb {
namespace lane12 {

template <int KIND, bool TR>
__global__ __launch_bounds__(64 * kLaneWaves) void k_fmm_level_lane32(FmmDev f, const double* __restrict__ Ztab,
                                                                  int count, const int* __restrict__ nodes,
                                                                  const int* __restrict__ child,
                                                                  const int* __restrict__ parent,
                                                                  double* __restrict__ E) {
  constexpr bool kUp = (KIND == 0) != TR;  // sources: the children (else the parent)
  __shared__ double zsm[kZYn];
  for (int i = threadIdx.x; i < kZYn; i += blockDim.x) zsm[i] = Ztab[i];
  __syncthreads();  // the only barrier: afterwards every lane works on its own node
  ldbl* zl = (ldbl*)zsm;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  const int n = nodes[b];
  int src[2];
  int ns;
  if constexpr (kUp) {
    src[0] = child[2 * n];
    src[1] = child[2 * n + 1];
    if (src[0] < 0) return;  // a leaf has no children
    ns = 2;
  } else {
    src[0] = parent[n];
    src[1] = -1;
    if (src[0] < 0) return;  // the root has no parent
    ns = 1;
  }
  const double cnx = f.center[3 * n], cny = f.center[3 * n + 1], cnz = f.center[3 * n + 2];
#pragma unroll 1
  for (int s = 0; s < ns; ++s) {
    const int o = src[s];
    // offset from the source centre to the target centre (the fixed node is the target of
    // the forward translations, the source of the transposed ones)
    const double ox = f.center[3 * o], oy = f.center[3 * o + 1], oz = f.center[3 * o + 2];
    const double dx = TR ? ox - cnx : cnx - ox, dy = TR ? oy - cny : cny - oy, dz = TR ? oz - cnz : cnz - oz;
    const double rxy = sqrt(dx * dx + dy * dy), rho = sqrt(dx * dx + dy * dy + dz * dz);
    double c1 = 1.0, s1 = 0.0, ct = 1.0, st = 0.0;
    if (rxy > 0.0) {
      const double ir = 1.0 / rxy;
      c1 = dx * ir;
      s1 = dy * ir;
    }
    if (rho > 0.0) {
      const double irho = 1.0 / rho;
      ct = dz * irho;
      st = rxy * irho;
    }
    // input scales (input node o): M2M 1/k_l(kappa R_o), L2L (-1)^l / i_l(kappa R_o);
    // transposed M2M k_l(kappa R_o), transposed L2L (-1)^l i_l(kappa R_o)
    double sin_[kP1];
    sfor<kP1>([&](auto L_) {
      constexpr int l = decltype(L_)::value;
      const double sg = (KIND == 2 && (l & 1)) ? -1.0 : 1.0;
      double sc;
      if constexpr (KIND == 0) sc = TR ? f.kR[o * kP1 + l] : f.kRi[o * kP1 + l];
      else sc = TR ? f.iR[o * kP1 + l] : 1.0 / f.iR[o * kP1 + l];
      sin_[l] = sg * sc;
    });
    // the input times its degree scales, formed in FP64 and rounded once
    float v[kPP];
    {
      const double* __restrict__ srcv = E + (long)o * kPP;
      sfor<kP1>([&](auto L_) {
        constexpr int l = decltype(L_)::value;
#pragma unroll
        for (int a = 0; a < 2 * l + 1; ++a) v[l * l + a] = (float)(srcv[l * l + a] * sin_[l]);
      });
    }
    const float c1f = (float)c1, s1f = (float)s1, ctf = (float)ct, stf = (float)st;
    // rotation into the frame whose z axis points from source to target, per degree
    sfor<kP1>([&](auto L_) {
      constexpr int l = decltype(L_)::value, w = 2 * l + 1;
      float bb[w], cc[w];
      bb[l] = v[l * l + l];
      float cm = 1.0f, sm = 0.0f;
      sfor<l>([&](auto M_) {
        constexpr int m = decltype(M_)::value + 1;
        cmul_step_f(cm, sm, c1f, s1f);
        const float a = v[l * l + l + m], b2 = v[l * l + l - m];
        bb[l + m] = a * cm + b2 * sm;
        bb[l - m] = b2 * cm - a * sm;
      });
      japply_f<l, false>(bb, cc);
      cm = 1.0f;
      sm = 0.0f;
      sfor<l>([&](auto M_) {
        constexpr int m = decltype(M_)::value + 1;
        cmul_step_f(cm, sm, ctf, stf);
        const float sg = (m & 1) ? -1.0f : 1.0f;
        const float co = sg * cm, si = -sg * sm;
        const float a = cc[l + m], b2 = cc[l - m];
        cc[l + m] = a * co - b2 * si;
        cc[l - m] = a * si + b2 * co;
      });
      japply_f<l, true>(cc, bb);
#pragma unroll
      for (int a = 0; a < w; ++a) v[l * l + a] = bb[a];
    });
    // sigma_n(z^2), n = 0..2p: the series for 2p and 2p-1, then the downward recurrence
    // sigma_{n-1} = z^2 sigma_{n+1} + (2n+1) sigma_n; z^j, j = 0..p; and z^2
    double sg[2 * kP + 1], zp[kP1], z2h;
    {
      double rz = rho;
      asm volatile("" : "+v"(rz) : "v"(v[0]));  // computed here, after the first rotation
      const double z = f.kappa * rz, z2 = z * z;
      double ta = 1.0, tb = 1.0;  // 1 / (4p+1)!!, 1 / (4p-1)!!
      for (int k = 3; k <= 4 * kP + 1; k += 2) {
        ta /= k;
        if (k <= 4 * kP - 1) tb /= k;
      }
      double sa = ta, sb = tb;
      for (int k = 0; k < 400; ++k) {
        ta *= z2 * (0.5 / ((k + 1.0) * (4.0 * kP + 2.0 * k + 3.0)));
        tb *= z2 * (0.5 / ((k + 1.0) * (4.0 * kP + 2.0 * k + 1.0)));
        sa += ta;
        sb += tb;
        if (ta <= 1e-18 * sa && tb <= 1e-18 * sb) break;
      }
      sg[2 * kP] = sa;
      sg[2 * kP - 1] = sb;
      double sp1 = sa;
      sfor<2 * kP - 1>([&](auto K_) {
        constexpr int nn = 2 * kP - 1 - decltype(K_)::value;
        sg[nn - 1] = z2 * sp1 + (2.0 * nn + 1.0) * sg[nn];
        sp1 = sg[nn];
      });
      zp[0] = 1.0;
      sfor<kP>([&](auto J_) {
        constexpr int j = decltype(J_)::value + 1;
        zp[j] = zp[j - 1] * z;
      });
      z2h = z2;
    }
    // output scales (the fixed node n): M2M k_l(kappa R_n), L2L (-1)^l i_l(kappa R_n);
    // transposed M2M 1/k_l(kappa R_n), transposed L2L (-1)^l / i_l(kappa R_n)
    double sout[kP1];
    {
      const int nfp = n;
      sfor<kP1>([&](auto L_) {
        constexpr int l = decltype(L_)::value;
        const double sgn = (KIND == 2 && (l & 1)) ? -1.0 : 1.0;
        double sc;
        if constexpr (KIND == 0) sc = TR ? f.kRi[nfp * kP1 + l] : f.kR[nfp * kP1 + l];
        else sc = TR ? 1.0 / f.iR[nfp * kP1 + l] : f.iR[nfp * kP1 + l];
        sout[l] = sgn * sc;
      });
    }
    // translation along z, per order |m| (FP64), the output scale applied before rounding
    sfor<kP1>([&](auto AM_) {
      constexpr int am = decltype(AM_)::value, nb = kP1 - am, nt = zterm_count(true, am);
      double op[nb], om[nb];
#pragma unroll
      for (int x = 0; x < nb; ++x) { op[x] = 0.0; om[x] = 0.0; }
      double cur[kZChunk], nxt[kZChunk];
      double dep = (double)v[am * am + am], e = 0.0;
      zchunk_load<true, am, 0>(zl, cur, dep);
      sfor<nt>([&](auto T_) {
        constexpr int t = decltype(T_)::value, pos = t % kZChunk;
        constexpr ZTerm z = zterm(true, am, t);
        constexpr int k = am + z.k;               // the sum index
        constexpr int nidx = z.lo + z.li - k;     // sigma_{l+l'-k}
        constexpr int dl = z.lo > z.li ? z.lo - z.li : z.li - z.lo;
        if constexpr (pos == 0) zchunk_load<true, am, t / kZChunk + 1>(zl, nxt, dep);
        const double term = cur[pos] * sg[nidx];
        e = z.k == 0 ? term : fma(e, z2h, term);
        if constexpr (z.k == z.n - 1) {
          e *= zp[dl];
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
      float bb[w], cc[w];
#pragma unroll
      for (int a = 0; a < w; ++a) bb[a] = v[l * l + a];
      japply_f<l, false>(bb, cc);
      float cm = 1.0f, sm = 0.0f;
      sfor<l>([&](auto M_) {
        constexpr int m = decltype(M_)::value + 1;
        cmul_step_f(cm, sm, ctf, stf);
        const float sgm = (m & 1) ? -1.0f : 1.0f;
        const float co = sgm * cm, si = sgm * sm;
        const float a = cc[l + m], b2 = cc[l - m];
        cc[l + m] = a * co - b2 * si;
        cc[l - m] = a * si + b2 * co;
      });
      japply_f<l, true>(cc, bb);
      v[l * l + l] = bb[l];
      cm = 1.0f;
      sm = 0.0f;
      sfor<l>([&](auto M_) {
        constexpr int m = decltype(M_)::value + 1;
        cmul_step_f(cm, sm, c1f, s1f);
        const float a = bb[l + m], bm = bb[l - m];
        v[l * l + l + m] = a * cm - bm * sm;
        v[l * l + l - m] = a * sm + bm * cm;
      });
    });
    // accumulate into the fixed node's row (the forward upward pass overwrites it with
    // its first child's contribution)
    double* __restrict__ dst = E + (long)n * kPP;
    if (kUp && !TR && s == 0) {
#pragma unroll
      for (int k = 0; k < kPP; ++k) dst[k] = (double)v[k];
    } else {
#pragma unroll
      for (int k = 0; k < kPP; ++k) dst[k] += (double)v[k];
    }
  }
}

}  // namespace lane12
}  // namespace ddlpb

#define DDLPB_LEVEL_LANE32_INSTANCE(NAME, KIND, TR)                                                          \
  namespace ddlpb {                                                                                        \
  namespace lane12 {                                                                                       \
  hipError_t upload_##NAME(const double* J, const double* JT) {                                            \
    float jf[kJn], jtf[kJTn];                                                                              \
    for (int i = 0; i < kJn; ++i) jf[i] = (float)J[i];                                                     \
    for (int i = 0; i < kJTn; ++i) jtf[i] = (float)JT[i];                                                  \
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_lane_jf), jf, sizeof(float) * kJn);                      \
    if (e != hipSuccess) return e;                                                                         \
    return hipMemcpyToSymbol(HIP_SYMBOL(c_lane_jtf), jtf, sizeof(float) * kJTn);                           \
  }                                                                                                        \
  hipError_t launch_##NAME(const FmmDev& f, const double* Z, int count, const int* nodes, const int* child, \
                           const int* parent, double* E, hipStream_t s) {                                  \
    if (count <= 0) return hipSuccess;                                                                     \
    const int threads = 64 * kLaneWaves;                                                                   \
    hipLaunchKernelGGL((k_fmm_level_lane32<KIND, TR>), dim3((count + threads - 1) / threads), dim3(threads), 0, \
                       s, f, Z, count, nodes, child, parent, E);                                           \
    return hipGetLastError();                                                                              \
  }                                                                                                        \
  }                                                                                                        \
  }
