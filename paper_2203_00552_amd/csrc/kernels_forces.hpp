// Force assembly kernels (Sec. 3.1 and the Sec. 3 force equation).
//
// With X and X_adj fixed, grad_{x_k} E equals the gradient of
//   E_f = 1/2 sum_i sum_n w_n [ xi_r sum_j omega_ij vA_j + xi_e sum_j omega_ij vB_j
//                               - U (xi_r psi0 + xi_s Phi[m(e, y)]) ]
// (xi = Syn(X_adj), xi_s = xi_r + xi_e, m(e,y)_j = C^j (.) An_j(U_j (e_j + Syn y_j)),
// e = (eps1/eps2) d_n psi0).  The kernels below evaluate the pieces of that
// gradient: derivatives of omega_ij and chi^eta_i through chi_eta (three
// geometric cases), derivatives of the A/B basis (radial, Bessel, angular), of
// psi_0 and d_n psi_0 at grid points and at the charges, and of the
// single-layer field with respect to the evaluation point and the source
// centre.  Every per-atom sum is a fixed-order reduction (no float atomics),
// so results are bitwise reproducible.
#pragma once
#include "kernels_direct.hpp"

namespace ddlpb {

// Switching-function and near-field terms.  One block per sphere i, threads over
// grid points; a block reduction per neighbour slot writes fnb[nptr[i]+a] (the
// contribution that acts on x_i with + and on the neighbour with -), and fself[i].
template <int LM>
__global__ __launch_bounds__(256) void k_force_switch(int M, int N, const double* __restrict__ leb,
                                                       const double* __restrict__ xyz,
                                                       const double* __restrict__ rad,
                                                       const int* __restrict__ nptr, const int* __restrict__ nidx,
                                                       const double* __restrict__ f, const double* __restrict__ U,
                                                       const double* __restrict__ sgr, int LUR, double kappa,
                                                       double eta, int nterms, const double* __restrict__ X,
                                                       const double* __restrict__ xr, const double* __restrict__ xe,
                                                       const double* __restrict__ psi, const double* __restrict__ Phi,
                                                       const double* __restrict__ hg, const double* __restrict__ etag,
                                                       double* __restrict__ fnb, double* __restrict__ fself) {
  constexpr int L = (LM + 1) * (LM + 1);
  __shared__ double s1[kMaxN];
  __shared__ double sh[16];
  const int i = blockIdx.x;
  const double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2], ri = rad[i];
  const int q0 = nptr[i], K = nptr[i + 1] - q0;
  // S1(x_i^n) = sum_j chi_j (xi_r vA_j + xi_e vB_j), needed where f > 1 (d'(f) != 0)
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    const long in = (long)i * N + n;
    double acc = 0.0;
    if (f[in] > 1.0) {
      const double px = xi + ri * leb[4 * n], py = yi + ri * leb[4 * n + 1], pz = zi + ri * leb[4 * n + 2];
      for (int a = 0; a < K; ++a) {
        const int j = nidx[q0 + a];
        const double irj = 1.0 / rad[j];
        const double vx = (px - xyz[3 * j]) * irj, vy = (py - xyz[3 * j + 1]) * irj, vz = (pz - xyz[3 * j + 2]) * irj;
        const double t2 = vx * vx + vy * vy + vz * vz;
        if (t2 >= 1.0) continue;
        const double ch = chi_eta(sqrt(t2), eta);
        if (ch == 0.0) continue;
        double sg[LM + 1];
        sigma_weights<LM, double>(kappa * kappa * rad[j] * rad[j] * t2, nterms, sg);
        const double* Xr = X + (long)j * L;
        const double* Xe = X + (long)(M + j) * L;
        double sa = 0.0, pb[LM + 1];
#pragma unroll
        for (int l = 0; l <= LM; ++l) pb[l] = 0.0;
        for_each_solid_harmonic<LM, double>(vx, vy, vz, [&](int l, int idx, double S) { sa += Xr[idx] * S; pb[l] += Xe[idx] * S; });
        double sb = 0.0;
#pragma unroll
        for (int l = 0; l <= LM; ++l) sb += pb[l] * sg[l] / sgr[j * LUR + l];
        acc += ch * (xr[in] * sa + xe[in] * sb);
      }
    }
    s1[n] = acc;
  }
  __syncthreads();
  double own[3] = {0, 0, 0};
  for (int a = 0; a < K; ++a) {
    const int j = nidx[q0 + a];
    const double rj = rad[j], irj = 1.0 / rj;
    double g[3] = {0, 0, 0};
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
      const long in = (long)i * N + n;
      const double px = xi + ri * leb[4 * n], py = yi + ri * leb[4 * n + 1], pz = zi + ri * leb[4 * n + 2];
      const double dx = (px - xyz[3 * j]) * irj, dy = (py - xyz[3 * j + 1]) * irj, dz = (pz - xyz[3 * j + 2]) * irj;
      const double t2 = dx * dx + dy * dy + dz * dz;
      if (t2 >= 1.0) continue;
      const double t = sqrt(t2);
      const double ch = chi_eta(t, eta), chp = chi_eta_d(t, eta);
      if (ch == 0.0) continue;
      const double wn = leb[4 * n + 3];
      const double fv = f[in], Uv = U[in];
      const double dv = fv > 1.0 ? 1.0 / fv : 1.0;
      const double dd = fv > 1.0 ? -1.0 / (fv * fv) : 0.0;
      // basis values and gradients with respect to the grid point (dual numbers)
      using D = Dual<double>;
      D v[3];
      v[0] = D(px); v[0].g[0] = 1.0; v[0] = (v[0] - D(xyz[3 * j])) * irj;
      v[1] = D(py); v[1].g[1] = 1.0; v[1] = (v[1] - D(xyz[3 * j + 1])) * irj;
      v[2] = D(pz); v[2].g[2] = 1.0; v[2] = (v[2] - D(xyz[3 * j + 2])) * irj;
      D z2 = (kappa * kappa * rj * rj) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      D sg[LM + 1];
      sigma_weights<LM, D>(z2, nterms, sg);
      const double* Xr = X + (long)j * L;
      const double* Xe = X + (long)(M + j) * L;
      D sa(0.0), pb[LM + 1];
#pragma unroll
      for (int l = 0; l <= LM; ++l) pb[l] = D(0.0);
      for_each_solid_harmonic<LM, D>(v[0], v[1], v[2], [&](int l, int idx, const D& S) {
        sa = sa + Xr[idx] * S;
        pb[l] = pb[l] + Xe[idx] * S;
      });
      D sb(0.0);
#pragma unroll
      for (int l = 0; l <= LM; ++l) sb = sb + (1.0 / sgr[j * LUR + l]) * (pb[l] * sg[l]);
      const double xrv = xr[in], xev = xe[in];
      const double V = xrv * sa.v + xev * sb.v;
      double dT = 0.5 * wn * (dd * chp * s1[n] + dv * chp * V);
      if (Uv > 0.0) {
        const double W = psi[in] * xrv + Phi[in] * (xrv + xev);
        dT += 0.5 * wn * (W + hg[in] * etag[in]) * chp;
      }
      const double et = irj / t;  // e^j / r_j = (scaled v) / (t r_j)
      const double dxyz[3] = {dx, dy, dz};
      for (int c = 0; c < 3; ++c)
        g[c] += dT * dxyz[c] * et + 0.5 * wn * dv * ch * (xrv * sa.g[c] + xev * sb.g[c]);
    }
    for (int c = 0; c < 3; ++c) {
      double s = block_sum(g[c], sh);
      own[c] += s;
      if (threadIdx.x == 0) fnb[3L * (q0 + a) + c] = s;
    }
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) fself[3L * i + c] = own[c];
}

// Target-side terms at every active point (x_i^n moves with x_i):
//   Laplace:  -1/2 w U (xi_r grad psi0_k + eta (eps1/eps2) grad d_n psi0_k) for charges k != i
//   Yukawa:   -1/2 w U xi_s grad Phi'  (Phi' without the sphere's own term)
__global__ __launch_bounds__(256) void k_force_points(int M, int N, int nact, const int* __restrict__ act_sph,
                                                      const int* __restrict__ act_n, const double* __restrict__ xyz,
                                                      const double* __restrict__ rad, const double* __restrict__ leb,
                                                      const double* __restrict__ q, double eps1, double eps2,
                                                      const double* __restrict__ U, const double* __restrict__ xr,
                                                      const double* __restrict__ xe, const double* __restrict__ etag,
                                                      const double* __restrict__ gradPhi, int laplace_direct,
                                                      double* __restrict__ fpt) {
  __shared__ double sq[256 * 4];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = k < nact;
  const int i = active ? act_sph[k] : 0, n = active ? act_n[k] : 0;
  double p[3], s[3];
  for (int a = 0; a < 3; ++a) { s[a] = leb[4 * n + a]; p[a] = xyz[3 * i + a] + rad[i] * s[a]; }
  const long in = (long)i * N + n;
  const double c = active ? -0.5 * leb[4 * n + 3] * U[in] : 0.0;
  const double a1 = active ? c * xr[in] / eps1 : 0.0;       // multiplies q_k grad(1/d)
  const double a2 = active ? c * etag[in] / eps2 : 0.0;     // multiplies q_k grad(s . grad(1/d))
  double acc[3] = {0, 0, 0};
  if (laplace_direct) {
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
      for (int cc = 0; cc < nc; ++cc) {
        if (k0 + cc == i) continue;
        const double vx = p[0] - sq[4 * cc], vy = p[1] - sq[4 * cc + 1], vz = p[2] - sq[4 * cc + 2];
        const double d2 = vx * vx + vy * vy + vz * vz, id = 1.0 / sqrt(d2), id2 = id * id, id3 = id2 * id;
        const double qk = sq[4 * cc + 3];
        const double vs = vx * s[0] + vy * s[1] + vz * s[2];
        const double v3[3] = {vx, vy, vz};
        for (int a = 0; a < 3; ++a)
          acc[a] += qk * (a1 * (-v3[a] * id3) + a2 * (3.0 * v3[a] * vs * id3 * id2 - s[a] * id3));
      }
    }
  }
  if (!active) return;
  const double cs = c * (xr[in] + xe[in]);
  for (int a = 0; a < 3; ++a) fpt[3L * k + a] = acc[a] + cs * gradPhi[3L * k + a];
}

// sum of the per-point vectors of each sphere (fixed order)
__global__ __launch_bounds__(256) void k_sum_points(int M, const int* __restrict__ act_ptr, const double* __restrict__ fpt,
                                                    double* __restrict__ out) {
  __shared__ double sh[32];
  const int i = blockIdx.x;
  Comp a[3];
  for (int k = act_ptr[i] + threadIdx.x; k < act_ptr[i + 1]; k += blockDim.x)
    for (int c = 0; c < 3; ++c) a[c].add(fpt[3L * k + c]);
  for (int c = 0; c < 3; ++c) {
    double s = block_sum_comp(a[c], sh);
    if (threadIdx.x == 0) out[3L * i + c] = s;
  }
}

// Source-side Laplace terms: the charge k moves, the grid point (i,n), i != k, does not.
__global__ __launch_bounds__(256) void k_force_laplace_source(int M, int N, int nact, const int* __restrict__ act_sph,
                                                              const int* __restrict__ act_n,
                                                              const double* __restrict__ xyz,
                                                              const double* __restrict__ rad,
                                                              const double* __restrict__ leb,
                                                              const double* __restrict__ q, double eps1, double eps2,
                                                              const double* __restrict__ U,
                                                              const double* __restrict__ xr,
                                                              const double* __restrict__ etag,
                                                              double* __restrict__ out) {
  __shared__ double sh[32];
  const int kq = blockIdx.x;
  const double xk = xyz[3 * kq], yk = xyz[3 * kq + 1], zk = xyz[3 * kq + 2], qk = q[kq];
  Comp acc[3];  // every active point of the other spheres: compensated
  for (int k = threadIdx.x; k < nact; k += blockDim.x) {
    const int i = act_sph[k], n = act_n[k];
    if (i == kq) continue;
    const long in = (long)i * N + n;
    const double c = -0.5 * leb[4 * n + 3] * U[in];
    const double a1 = c * xr[in] / eps1, a2 = c * etag[in] / eps2;
    const double s[3] = {leb[4 * n], leb[4 * n + 1], leb[4 * n + 2]};
    const double v3[3] = {xyz[3 * i] + rad[i] * s[0] - xk, xyz[3 * i + 1] + rad[i] * s[1] - yk,
                          xyz[3 * i + 2] + rad[i] * s[2] - zk};
    const double d2 = v3[0] * v3[0] + v3[1] * v3[1] + v3[2] * v3[2], id = 1.0 / sqrt(d2), id2 = id * id, id3 = id2 * id;
    const double vs = v3[0] * s[0] + v3[1] * s[1] + v3[2] * s[2];
    for (int a = 0; a < 3; ++a)
      acc[a].add(-qk * (a1 * (-v3[a] * id3) + a2 * (3.0 * v3[a] * vs * id3 * id2 - s[a] * id3)));
  }
  for (int c = 0; c < 3; ++c) {
    double s = block_sum_comp(acc[c], sh);
    if (threadIdx.x == 0) out[3L * kq + c] = s;
  }
}

// Charge derivative of 1/2 <X_adj, g> (Sec. 3: the adjoint solution differentiates the
// energy with respect to any parameter of the right-hand side): g depends on q_k through
// psi_0 and d_n psi_0 at the grid points, so
//   S_k = sum_p a1_p / |p - x_k| - a2_p ((p - x_k) . s_p) / |p - x_k|^3,
//   a1 = -1/2 w U xi_r / eps1,  a2 = -1/2 w U eta / eps2,
// over every active point p (the sphere of k included).  Direct sums, one block per atom.
__global__ __launch_bounds__(256) void k_dq_laplace_source(int M, int N, int nact, const int* __restrict__ act_sph,
                                                           const int* __restrict__ act_n,
                                                           const double* __restrict__ xyz,
                                                           const double* __restrict__ rad,
                                                           const double* __restrict__ leb, double eps1, double eps2,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ xr,
                                                           const double* __restrict__ etag, double* __restrict__ out) {
  __shared__ double sh[16];
  const int kq = blockIdx.x;
  const double xk = xyz[3 * kq], yk = xyz[3 * kq + 1], zk = xyz[3 * kq + 2];
  double acc = 0.0;
  for (int k = threadIdx.x; k < nact; k += blockDim.x) {
    const int i = act_sph[k], n = act_n[k];
    const long in = (long)i * N + n;
    const double c = -0.5 * leb[4 * n + 3] * U[in];
    const double a1 = c * xr[in] / eps1, a2 = c * etag[in] / eps2;
    const double s0 = leb[4 * n], s1 = leb[4 * n + 1], s2 = leb[4 * n + 2];
    const double v0 = xyz[3 * i] + rad[i] * s0 - xk, v1 = xyz[3 * i + 1] + rad[i] * s1 - yk,
                 v2 = xyz[3 * i + 2] + rad[i] * s2 - zk;
    const double id = 1.0 / sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    acc += a1 * id - a2 * (v0 * s0 + v1 * s1 + v2 * s2) * id * id * id;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[kq] = s;
}

// Source-side single-layer term: 1/2 sum_lm m_jlm sum_l'm' kappa d[a][lm][l'm'] k_l'(kappa r_j)/k_l(kappa r_j) lambda'_jl'm'
// with lambda' the adjoint field of the grid charges c = w U xi_s on the other spheres, degree lmax+1.
template <int LM>
__global__ __launch_bounds__(128) void k_force_yukawa_source(int M, const double* __restrict__ m,
                                                              const double* __restrict__ lamp,
                                                              const double* __restrict__ dtab,
                                                              const double* __restrict__ kr, int LUR, double kappa,
                                                              double* __restrict__ out) {
  constexpr int L = (LM + 1) * (LM + 1), LP = (LM + 2) * (LM + 2);
  __shared__ double sh[16];
  const int j = blockIdx.x;
  double acc[3] = {0, 0, 0};
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    const int l = deg_of(t);
    const double mj = m[(long)j * L + t];
    if (mj == 0.0) continue;
    for (int a = 0; a < 3; ++a) {
      const double* dr = dtab + ((long)a * L + t) * LP;
      double s = 0.0;
      for (int tp = (l > 0 ? (l - 1) * (l - 1) : 1); tp < (l + 2) * (l + 2); ++tp) {
        if (dr[tp] == 0.0) continue;
        const int lp = deg_of(tp);
        s += dr[tp] * kr[j * LUR + lp] * lamp[(long)j * LP + tp];
      }
      acc[a] += 0.5 * kappa * mj * s / kr[j * LUR + l];
    }
  }
  for (int c = 0; c < 3; ++c) {
    double s = block_sum(acc[c], sh);
    if (threadIdx.x == 0) out[3L * j + c] = s;
  }
}

// eta_j = Syn(C^j (.) lambda_j) with lambda_j = lambda'_j + sum_n c_jn Y_lm(s_n) (own sphere added back)
template <int LM>
__global__ __launch_bounds__(256) void k_eta(int M, int N, int LY, const double* __restrict__ Y,
                                              const double* __restrict__ cgrid, const double* __restrict__ lamp,
                                              int LLAM, const double* __restrict__ Cl, int LUR,
                                              double* __restrict__ etag) {
  constexpr int L = (LM + 1) * (LM + 1);
  __shared__ double cl[L];
  __shared__ double cg[kMaxN];
  const int j = blockIdx.x;
  for (int n = threadIdx.x; n < N; n += blockDim.x) cg[n] = cgrid[(long)j * N + n];
  __syncthreads();
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    double s = lamp[(long)j * LLAM + t];
    for (int n = 0; n < N; ++n) s += cg[n] * Y[(long)n * LY + t];
    cl[t] = Cl[j * LUR + deg_of(t)] * s;
  }
  __syncthreads();
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    const double* Yn = Y + (long)n * LY;
    double a = 0.0;
    for (int t = 0; t < L; ++t) a += Yn[t] * cl[t];
    etag[(long)j * N + n] = a;
  }
}

// F_k = -(grad contributions), gathered in a fixed order.
__global__ void k_force_final(int M, const int* __restrict__ nptr, const int* __restrict__ nidx,
                              const int* __restrict__ nrev, const double* __restrict__ fnb,
                              const double* __restrict__ fself, const double* __restrict__ fpts,
                              const double* __restrict__ flsrc, const double* __restrict__ fysrc,
                              double* __restrict__ F) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  for (int c = 0; c < 3; ++c) {
    Comp g;  // compensated per-atom sum of the force terms
    g.add(fself[3L * k + c]);
    g.add(fpts[3L * k + c]);
    g.add(flsrc[3L * k + c]);
    g.add(fysrc[3L * k + c]);
    for (int b = nptr[k]; b < nptr[k + 1]; ++b) {
      const int i = nidx[b];
      g.add(-fnb[3L * (nptr[i] + nrev[b]) + c]);
    }
    F[3L * k + c] = -g.value();
  }
}

// ------------------------------------------- potentials at arbitrary points
// Ball of a point: the sphere i with the smallest |x - x_i| / r_i (so a point of the
// cavity gets a ball that contains it).  One thread per point, all spheres scanned.
__global__ __launch_bounds__(256) void k_nearest_ball(int n, const double* __restrict__ pts, int M,
                                                      const double* __restrict__ xyz, const double* __restrict__ rad,
                                                      int* __restrict__ ball) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double px = pts[3 * k], py = pts[3 * k + 1], pz = pts[3 * k + 2];
  double best = 1e300;
  int bi = 0;
  for (int i = 0; i < M; ++i) {
    const double dx = px - xyz[3 * i], dy = py - xyz[3 * i + 1], dz = pz - xyz[3 * i + 2];
    const double s = (dx * dx + dy * dy + dz * dz) / (rad[i] * rad[i]);
    if (s < best) { best = s; bi = i; }
  }
  ball[k] = bi;
}

// Reaction and extended potentials from the expansions of ball i = ball[k] (Sec. 2):
//   psi_r(x) = sum_lm X_r,ilm (|x - x_i| / r_i)^l Y_lm,
//   psi_e(x) = sum_lm X_e,ilm i_l(kappa |x - x_i|) / i_l(kappa r_i) Y_lm,
// and their gradients (dual numbers in x).  out[k][8] = psi_r, psi_e, grad psi_r,
// grad psi_e.  With v = (x - x_i)/r_i the first basis is the solid harmonic S_lm(v)
// and the second sigma_l(kappa^2 r_i^2 |v|^2) / sigma_l(kappa^2 r_i^2) S_lm(v).
template <int LM>
__global__ __launch_bounds__(256) void k_eval_points(int n, const double* __restrict__ pts, const int* __restrict__ ball,
                                                     int M, int L, int LUR, const double* __restrict__ X,
                                                     const double* __restrict__ xyz, const double* __restrict__ rad,
                                                     const double* __restrict__ isgr, double kappa, int nterms,
                                                     double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = ball[k];
  const double ri = rad[i], iri = 1.0 / ri;
  using D = Dual<double>;
  D v[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    v[c] = D(pts[3 * k + c]);
    v[c].g[c] = 1.0;
    v[c] = (v[c] - D(xyz[3 * i + c])) * iri;
  }
  D z2 = (kappa * kappa * ri * ri) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  D sg[LM + 1];
  sigma_weights<LM, D>(z2, nterms, sg);
  const double* Xr = X + (long)i * L;
  const double* Xe = X + (long)(M + i) * L;
  D sa(0.0), pb[LM + 1];
#pragma unroll
  for (int l = 0; l <= LM; ++l) pb[l] = D(0.0);
  for_each_solid_harmonic<LM, D>(v[0], v[1], v[2], [&](int l, int idx, const D& S) {
    sa = sa + Xr[idx] * S;
    pb[l] = pb[l] + Xe[idx] * S;
  });
  D sb(0.0);
#pragma unroll
  for (int l = 0; l <= LM; ++l) sb = sb + isgr[(long)i * LUR + l] * (pb[l] * sg[l]);
  double* o = out + 8L * k;
  o[0] = sa.v;
  o[1] = sb.v;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o[2 + c] = sa.g[c];
    o[5 + c] = sb.g[c];
  }
}

}  // namespace ddlpb

namespace ddlpb {

// ---------------------------------------------------------------- radius gradient
// dE/dr_k for every sphere from the same frozen functional E_f as the forces (Sec. 3:
// the adjoint solution differentiates E with respect to any parameter).  The radius
// r_k enters E_f (i) through the grid points x_k^n = x_k + r_k s_n, which move
// radially: the derivative is s_n . (gradient with respect to the point), (ii) through
// t = |x - x_k| / r_k in chi_eta (omega, f, U), and (iii) through the per-degree
// normalisers of sphere k's bases and constants (Sec. 2.2):
//   A basis  r_k^-l                        -> -l / r_k
//   B basis  1 / i_l(kappa r_k)            -> -D_l,  D_l = kappa i_l'/i_l (kappa r_k)
//   single layer 1 / k_l(kappa r_k)        -> -dk_l, dk_l = kappa k_l'/k_l (kappa r_k)
//   C_l = (2/pi) kappa r^2 i_l k_l         -> C_l'/C_l = 2/r + D_l + dk_l
//   y_r = (eps1/eps2) l/r X_r, y_e = -D_l X_e -> -(eps1/eps2) l/r^2 X_r, -D_l' X_e
// with D_l' = kappa^2 + l(l+1)/r^2 - 2 D_l / r - D_l^2 (modified spherical Bessel
// equation).  Every per-sphere sum is a fixed-order reduction.

// Switching and A/B basis terms.  Block i (the sphere of the grid points), one
// neighbour j at a time: rnb[nptr[i] + a] = dE_f/dr_j of the terms evaluated on sphere
// i's points; rself[i] = the radial motion of those points.  Same quantities as
// k_force_switch (dT = dE_f/dt_j at the point, V = xi_r vA_j + xi_e vB_j).
template <int LM>
__global__ __launch_bounds__(256) void k_rgrad_switch(int M, int N, const double* __restrict__ leb,
                                                       const double* __restrict__ xyz,
                                                       const double* __restrict__ rad,
                                                       const int* __restrict__ nptr, const int* __restrict__ nidx,
                                                       const double* __restrict__ f, const double* __restrict__ U,
                                                       const double* __restrict__ sgr, const double* __restrict__ yce,
                                                       int LUR, double kappa, double eta, int nterms,
                                                       const double* __restrict__ X, const double* __restrict__ xr,
                                                       const double* __restrict__ xe, const double* __restrict__ psi,
                                                       const double* __restrict__ Phi, const double* __restrict__ hg,
                                                       const double* __restrict__ etag, double* __restrict__ rnb,
                                                       double* __restrict__ rself) {
  constexpr int L = (LM + 1) * (LM + 1);
  __shared__ double s1[kMaxN];
  __shared__ double sh[16];
  const int i = blockIdx.x;
  const double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2], ri = rad[i];
  const int q0 = nptr[i], K = nptr[i + 1] - q0;
  // S1(x_i^n) = sum_j chi_j V_j where f > 1 (the derivative of d(f) = 1/f)
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    const long in = (long)i * N + n;
    double acc = 0.0;
    if (f[in] > 1.0) {
      const double px = xi + ri * leb[4 * n], py = yi + ri * leb[4 * n + 1], pz = zi + ri * leb[4 * n + 2];
      for (int a = 0; a < K; ++a) {
        const int j = nidx[q0 + a];
        const double irj = 1.0 / rad[j];
        const double vx = (px - xyz[3 * j]) * irj, vy = (py - xyz[3 * j + 1]) * irj, vz = (pz - xyz[3 * j + 2]) * irj;
        const double t2 = vx * vx + vy * vy + vz * vz;
        if (t2 >= 1.0) continue;
        const double ch = chi_eta(sqrt(t2), eta);
        if (ch == 0.0) continue;
        double sg[LM + 1];
        sigma_weights<LM, double>(kappa * kappa * rad[j] * rad[j] * t2, nterms, sg);
        const double* Xr = X + (long)j * L;
        const double* Xe = X + (long)(M + j) * L;
        double sa = 0.0, pb[LM + 1];
#pragma unroll
        for (int l = 0; l <= LM; ++l) pb[l] = 0.0;
        for_each_solid_harmonic<LM, double>(vx, vy, vz, [&](int l, int idx, double S) { sa += Xr[idx] * S; pb[l] += Xe[idx] * S; });
        double sb = 0.0;
#pragma unroll
        for (int l = 0; l <= LM; ++l) sb += pb[l] * sg[l] / sgr[j * LUR + l];
        acc += ch * (xr[in] * sa + xe[in] * sb);
      }
    }
    s1[n] = acc;
  }
  __syncthreads();
  double own = 0.0;
  for (int a = 0; a < K; ++a) {
    const int j = nidx[q0 + a];
    const double rj = rad[j], irj = 1.0 / rj;
    double gj = 0.0;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
      const long in = (long)i * N + n;
      const double sx = leb[4 * n], sy = leb[4 * n + 1], sz = leb[4 * n + 2];
      const double px = xi + ri * sx, py = yi + ri * sy, pz = zi + ri * sz;
      const double dx = (px - xyz[3 * j]) * irj, dy = (py - xyz[3 * j + 1]) * irj, dz = (pz - xyz[3 * j + 2]) * irj;
      const double t2 = dx * dx + dy * dy + dz * dz;
      if (t2 >= 1.0) continue;
      const double t = sqrt(t2);
      const double ch = chi_eta(t, eta), chp = chi_eta_d(t, eta);
      if (ch == 0.0) continue;
      const double wn = leb[4 * n + 3];
      const double fv = f[in], Uv = U[in];
      const double dv = fv > 1.0 ? 1.0 / fv : 1.0;
      const double dd = fv > 1.0 ? -1.0 / (fv * fv) : 0.0;
      using D = Dual<double>;
      D v[3];
      v[0] = D(px); v[0].g[0] = 1.0; v[0] = (v[0] - D(xyz[3 * j])) * irj;
      v[1] = D(py); v[1].g[1] = 1.0; v[1] = (v[1] - D(xyz[3 * j + 1])) * irj;
      v[2] = D(pz); v[2].g[2] = 1.0; v[2] = (v[2] - D(xyz[3 * j + 2])) * irj;
      D z2 = (kappa * kappa * rj * rj) * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      D sg[LM + 1];
      sigma_weights<LM, D>(z2, nterms, sg);
      const double* Xr = X + (long)j * L;
      const double* Xe = X + (long)(M + j) * L;
      D sa(0.0), pb[LM + 1];
      double sal = 0.0;  // sum_l l (A part of degree l): d vA / d r_j = -sal / r_j
#pragma unroll
      for (int l = 0; l <= LM; ++l) pb[l] = D(0.0);
      for_each_solid_harmonic<LM, D>(v[0], v[1], v[2], [&](int l, int idx, const D& S) {
        sa = sa + Xr[idx] * S;
        sal += (double)l * Xr[idx] * S.v;
        pb[l] = pb[l] + Xe[idx] * S;
      });
      D sb(0.0);
      double dsb = 0.0;  // d vB / d r_j = -sum_l D_l (B part of degree l); yce = -D_l
#pragma unroll
      for (int l = 0; l <= LM; ++l) {
        const D bl = (1.0 / sgr[j * LUR + l]) * (pb[l] * sg[l]);
        sb = sb + bl;
        dsb += yce[j * LUR + l] * bl.v;
      }
      const double xrv = xr[in], xev = xe[in];
      const double V = xrv * sa.v + xev * sb.v;
      double dT = 0.5 * wn * (dd * chp * s1[n] + dv * chp * V);
      if (Uv > 0.0) {
        const double W = psi[in] * xrv + Phi[in] * (xrv + xev);
        dT += 0.5 * wn * (W + hg[in] * etag[in]) * chp;
      }
      const double om = 0.5 * wn * dv * ch;
      // radial motion of the point: s . d/dp
      const double et = irj / t;
      own += dT * (dx * sx + dy * sy + dz * sz) * et +
             om * (xrv * (sa.g[0] * sx + sa.g[1] * sy + sa.g[2] * sz) + xev * (sb.g[0] * sx + sb.g[1] * sy + sb.g[2] * sz));
      // r_j: dt/dr_j = -t / r_j, and the normalisers of the A and B bases
      gj += dT * (-t * irj) + om * (xrv * (-sal * irj) + xev * dsb);
    }
    const double s = block_sum(gj, sh);
    if (threadIdx.x == 0) rnb[q0 + a] = s;
  }
  const double s = block_sum(own, sh);
  if (threadIdx.x == 0) rself[i] = s;
}

// Radial motion of the active points of sphere i against the target-side point
// gradients fpt (psi_0, d_n psi_0 and the single-layer field of the other spheres and
// charges), plus sphere i's own charge, which stays at x_i while the points move:
// d/dr (1/r) = -1/r^2, d/dr (s . grad 1/|x - x_i|) = 2/r^3.
__global__ __launch_bounds__(256) void k_rgrad_points(int N, const int* __restrict__ act_ptr,
                                                      const int* __restrict__ act_n, const double* __restrict__ rad,
                                                      const double* __restrict__ leb, const double* __restrict__ q,
                                                      double eps1, double eps2, const double* __restrict__ U,
                                                      const double* __restrict__ xr, const double* __restrict__ etag,
                                                      const double* __restrict__ fpt, double* __restrict__ out) {
  __shared__ double sh[32];
  const int i = blockIdx.x;
  const double ri = rad[i], qi = q[i];
  const double o1 = -qi / (ri * ri), o2 = 2.0 * qi / (ri * ri * ri);
  Comp acc;
  for (int k = act_ptr[i] + threadIdx.x; k < act_ptr[i + 1]; k += blockDim.x) {
    const int n = act_n[k];
    const long in = (long)i * N + n;
    const double c = -0.5 * leb[4 * n + 3] * U[in];
    const double a1 = c * xr[in] / eps1, a2 = c * etag[in] / eps2;
    acc.add(fpt[3L * k] * leb[4 * n] + fpt[3L * k + 1] * leb[4 * n + 1] + fpt[3L * k + 2] * leb[4 * n + 2]);
    acc.add(a1 * o1 + a2 * o2);
  }
  const double s = block_sum_comp(acc, sh);
  if (threadIdx.x == 0) out[i] = s;
}

// Normaliser terms of sphere j's single layer (block j):
//   1/2 sum_lm dk_l m_jlm lambda'_jlm - 1/2 sum_lm (C_l'/C_l) m_jlm lambda_jlm
//   + 1/2 sum_lm ((eps1/eps2) l/r^2 X_r,jlm + D_l' X_e,jlm) mu_jlm
// with lambda = lambda' + An_j(c_j) (own sphere added back, c = w U xi_s) and
// mu = sum_n w_n U_j eta_j Y_lm(s_n).  rtab [4][M][LUR]: dk_l, C_l'/C_l,
// (eps1/eps2) l/r^2, D_l'.
template <int LM>
__global__ __launch_bounds__(256) void k_rgrad_source(int M, int N, int LY, const double* __restrict__ Y,
                                                      const double* __restrict__ leb, const double* __restrict__ U,
                                                      const double* __restrict__ cgrid,
                                                      const double* __restrict__ etag,
                                                      const double* __restrict__ lamp, int LLAM,
                                                      const double* __restrict__ m, const double* __restrict__ X,
                                                      const double* __restrict__ rtab, int LUR,
                                                      double* __restrict__ out) {
  constexpr int L = (LM + 1) * (LM + 1);
  __shared__ double cg[kMaxN], ue[kMaxN];
  __shared__ double sh[16];
  const int j = blockIdx.x;
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    const long jn = (long)j * N + n;
    cg[n] = cgrid[jn];
    ue[n] = leb[4 * n + 3] * U[jn] * etag[jn];
  }
  __syncthreads();
  const long MU = (long)M * LUR;
  double acc = 0.0;
  for (int t = threadIdx.x; t < L; t += blockDim.x) {
    const int l = deg_of(t);
    double own = 0.0, mu = 0.0;
    for (int n = 0; n < N; ++n) {
      const double y = Y[(long)n * LY + t];
      own += cg[n] * y;
      mu += ue[n] * y;
    }
    const long jl = (long)j * LUR + l;
    const double lp = lamp[(long)j * LLAM + t], mj = m[(long)j * L + t];
    acc += 0.5 * rtab[jl] * mj * lp - 0.5 * rtab[MU + jl] * mj * (lp + own) +
           0.5 * (rtab[2 * MU + jl] * X[(long)j * L + t] + rtab[3 * MU + jl] * X[(long)(M + j) * L + t]) * mu;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[j] = s;
}

// dE/dr_k = rself + rpts + rsrc + the switching terms of the spheres that have k as a
// neighbour, gathered in a fixed order
__global__ void k_rgrad_final(int M, const int* __restrict__ nptr, const int* __restrict__ nidx,
                              const int* __restrict__ nrev, const double* __restrict__ rnb,
                              const double* __restrict__ rself, const double* __restrict__ rpts,
                              const double* __restrict__ rsrc, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  Comp g;
  g.add(rself[k]);
  g.add(rpts[k]);
  g.add(rsrc[k]);
  for (int b = nptr[k]; b < nptr[k + 1]; ++b) g.add(rnb[nptr[nidx[b]] + nrev[b]]);
  out[k] = g.value();
}

}  // namespace ddlpb
