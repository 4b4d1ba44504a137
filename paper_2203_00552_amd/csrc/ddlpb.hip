// ddLPB library for MI355X (gfx950): context, device workspace, solvers and the C ABI.
//
// Call order (Sec. 3.1, final summary of the force computation): ddlpb_setup ->
// ddlpb_solve (primal L X = g) -> ddlpb_adjoint (L^T X_adj = Q) -> ddlpb_forces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ddlpb.h"
#include "host_math.hpp"
#include "kernels_forces.hpp"

using namespace ddlpb;

namespace {

constexpr int kMaxLmax = 10;

struct HipError {
  hipError_t e;
};
#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t err__ = (x);                        \
    if (err__ != hipSuccess) throw HipError{err__}; \
  } while (0)

// One-time upload of the Legendre recurrence constants per device.
std::mutex g_const_mu;
std::map<int, bool> g_const_done;
void ensure_constants() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_const_mu);
  if (g_const_done[dev]) return;
  std::vector<double> pmm, ra, rb;
  host::legendre_tables(kLmaxDev, pmm, ra, rb);
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_pmm), pmm.data(), pmm.size() * sizeof(double)));
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_ra), ra.data(), ra.size() * sizeof(double)));
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_rb), rb.data(), rb.size() * sizeof(double)));
  g_const_done[dev] = true;
}

}  // namespace

struct ddlpb_ctx {
  // ---- problem
  int M = 0, lmax = 0, L = 0, LP = 0, LY = 0, LUR = 0, N = 0, fmm_order = 0;
  double eps1 = 1, eps2 = 78.54, kappa = 0.1, eta = 0.1;
  std::vector<double> x, r, q;
  const ddlpb_tables::LebedevRule* rule = nullptr;
  // ---- options
  int precision = 0, restart = 40, sweeps = 8, maxit = 500, leaf = 32;
  double theta = 0.5;
  // ---- host analysis
  std::vector<int> nptr, nidx, nrev;
  int nterms = 8;
  // ---- device
  hipStream_t stream = nullptr;
  bool ws_bound = false, ws_owned = false, dev_ready = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // device pointers
  double *d_xyz = nullptr, *d_rad = nullptr, *d_q = nullptr, *d_leb = nullptr, *d_Y = nullptr;
  int *d_nptr = nullptr, *d_nidx = nullptr, *d_nrev = nullptr;
  double *d_f = nullptr, *d_U = nullptr;
  int *d_actcnt = nullptr, *d_actptr = nullptr, *d_actsph = nullptr, *d_actn = nullptr;
  double *d_ycr = nullptr, *d_yce = nullptr, *d_Cl = nullptr, *d_sgr = nullptr, *d_ur = nullptr, *d_kr = nullptr;
  double *d_dtab = nullptr;
  double *d_m = nullptr, *d_lam = nullptr;
  double *d_psi = nullptr, *d_e = nullptr, *d_Phi = nullptr, *d_h = nullptr, *d_zr = nullptr, *d_ze = nullptr,
         *d_cg = nullptr, *d_eta = nullptr, *d_xr = nullptr, *d_xe = nullptr;
  double *d_g = nullptr, *d_X = nullptr, *d_Xa = nullptr, *d_Q = nullptr, *d_w = nullptr, *d_t1 = nullptr,
         *d_t2 = nullptr, *d_t3 = nullptr, *d_V = nullptr;
  double *d_part = nullptr, *d_hv = nullptr, *d_scal = nullptr;
  double *d_fnb = nullptr, *d_fself = nullptr, *d_fpt = nullptr, *d_fpts = nullptr, *d_flsrc = nullptr,
         *d_fysrc = nullptr, *d_gphi = nullptr, *d_F = nullptr;
  int nact = 0;
  int nb_dot = 256;
  // ---- state
  int state = 0;  // 0 = set up, 1 = primal solved, 2 = adjoint solved
  bool rhs_ready = false;
  double energy = 0.0;
  ddlpb_stats stats{};
};

namespace {

const char* kErr[] = {"ok", "invalid argument", "coincident sphere centres", "out of memory",
                      "device (HIP) error", "solver did not converge", "call order violated"};

int check_inputs(int32_t M, const double* x, const double* r, const double* q, double e1, double e2, double kap,
                 int lmax, int nleb, int p) {
  if (M < 1 || !x || !r || !q) return DDLPB_EINVAL;
  if (!(e1 > 0) || !(e2 > 0) || !(kap > 0) || !std::isfinite(e1) || !std::isfinite(e2) || !std::isfinite(kap))
    return DDLPB_EINVAL;
  if (lmax < 0 || lmax > kMaxLmax || p < 0 || p > 20) return DDLPB_EINVAL;
  const auto* rule = host::lebedev_rule(nleb);
  if (!rule || rule->degree < 2 * lmax) return DDLPB_EINVAL;
  if (nleb > kMaxN) return DDLPB_EINVAL;
  for (int i = 0; i < M; ++i) {
    if (!std::isfinite(x[3 * i]) || !std::isfinite(x[3 * i + 1]) || !std::isfinite(x[3 * i + 2])) return DDLPB_EINVAL;
    if (!(r[i] > 0) || !std::isfinite(r[i]) || !std::isfinite(q[i])) return DDLPB_EINVAL;
  }
  return DDLPB_OK;
}

// Neighbour lists N_i = {j != i : |x_i - x_j| < r_i + r_j} by a uniform cell list, sorted by j.
int build_neighbours(ddlpb_ctx* c) {
  const int M = c->M;
  double rmax = 0;
  for (double v : c->r) rmax = std::max(rmax, v);
  const double cell = 2.0 * rmax;
  double lo[3] = {1e300, 1e300, 1e300};
  for (int i = 0; i < M; ++i)
    for (int a = 0; a < 3; ++a) lo[a] = std::min(lo[a], c->x[3 * i + a]);
  auto key = [&](long ix, long iy, long iz) { return (ix * 1000003L + iy) * 1000033L + iz; };
  std::unordered_map<long, std::vector<int>> cells;
  cells.reserve(M);
  std::vector<long> ci(3L * M);
  for (int i = 0; i < M; ++i) {
    for (int a = 0; a < 3; ++a) ci[3L * i + a] = (long)std::floor((c->x[3 * i + a] - lo[a]) / cell);
    cells[key(ci[3L * i], ci[3L * i + 1], ci[3L * i + 2])].push_back(i);
  }
  std::vector<std::vector<int>> nb(M);
  for (int i = 0; i < M; ++i) {
    for (long dx = -1; dx <= 1; ++dx)
      for (long dy = -1; dy <= 1; ++dy)
        for (long dz = -1; dz <= 1; ++dz) {
          auto it = cells.find(key(ci[3L * i] + dx, ci[3L * i + 1] + dy, ci[3L * i + 2] + dz));
          if (it == cells.end()) continue;
          for (int j : it->second) {
            if (j == i) continue;
            double d2 = 0;
            for (int a = 0; a < 3; ++a) { double t = c->x[3 * i + a] - c->x[3 * j + a]; d2 += t * t; }
            double d = std::sqrt(d2);
            if (d < 1e-12) return DDLPB_EGEOM;
            if (d < c->r[i] + c->r[j]) nb[i].push_back(j);
          }
        }
    std::sort(nb[i].begin(), nb[i].end());
  }
  c->nptr.assign(M + 1, 0);
  for (int i = 0; i < M; ++i) c->nptr[i + 1] = c->nptr[i] + (int)nb[i].size();
  c->nidx.resize(c->nptr[M]);
  c->nrev.resize(c->nptr[M]);
  for (int i = 0; i < M; ++i) std::copy(nb[i].begin(), nb[i].end(), c->nidx.begin() + c->nptr[i]);
  for (int i = 0; i < M; ++i)
    for (int a = c->nptr[i]; a < c->nptr[i + 1]; ++a) {
      int j = c->nidx[a];
      auto b = std::lower_bound(nb[j].begin(), nb[j].end(), i);
      c->nrev[a] = (int)(b - nb[j].begin());
    }
  return DDLPB_OK;
}

// ------------------------------------------------------------ workspace
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

void carve(ddlpb_ctx* c, char* base, size_t* total) {
  Carver cv{base};
  const size_t M = c->M, N = c->N, MN = M * N, D = 2 * M * c->L, nnz = c->nidx.size();
  c->d_xyz = cv.take<double>(3 * M);
  c->d_rad = cv.take<double>(M);
  c->d_q = cv.take<double>(M);
  c->d_leb = cv.take<double>(4 * N);
  c->d_Y = cv.take<double>(N * c->LY);
  c->d_nptr = cv.take<int>(M + 1);
  c->d_nidx = cv.take<int>(std::max<size_t>(nnz, 1));
  c->d_nrev = cv.take<int>(std::max<size_t>(nnz, 1));
  c->d_f = cv.take<double>(MN);
  c->d_U = cv.take<double>(MN);
  c->d_actcnt = cv.take<int>(M);
  c->d_actptr = cv.take<int>(M + 1);
  c->d_actsph = cv.take<int>(MN);
  c->d_actn = cv.take<int>(MN);
  c->d_ycr = cv.take<double>(M * c->LUR);
  c->d_yce = cv.take<double>(M * c->LUR);
  c->d_Cl = cv.take<double>(M * c->LUR);
  c->d_sgr = cv.take<double>(M * c->LUR);
  c->d_ur = cv.take<double>(M * c->LUR);
  c->d_kr = cv.take<double>(M * c->LUR);
  c->d_dtab = cv.take<double>(3 * (size_t)c->L * c->LP);
  c->d_m = cv.take<double>(M * c->L);
  c->d_lam = cv.take<double>(M * c->LP);
  c->d_psi = cv.take<double>(MN);
  c->d_e = cv.take<double>(MN);
  c->d_Phi = cv.take<double>(MN);
  c->d_h = cv.take<double>(MN);
  c->d_zr = cv.take<double>(MN);
  c->d_ze = cv.take<double>(MN);
  c->d_cg = cv.take<double>(MN);
  c->d_eta = cv.take<double>(MN);
  c->d_xr = cv.take<double>(MN);
  c->d_xe = cv.take<double>(MN);
  c->d_g = cv.take<double>(D);
  c->d_X = cv.take<double>(D);
  c->d_Xa = cv.take<double>(D);
  c->d_Q = cv.take<double>(D);
  c->d_w = cv.take<double>(D);
  c->d_t1 = cv.take<double>(D);
  c->d_t2 = cv.take<double>(D);
  c->d_t3 = cv.take<double>(D);
  c->d_V = cv.take<double>((size_t)(c->restart + 1) * D);
  c->d_part = cv.take<double>((size_t)(c->restart + 2) * c->nb_dot);
  c->d_hv = cv.take<double>(c->restart + 2);
  c->d_scal = cv.take<double>(16);
  c->d_fnb = cv.take<double>(3 * std::max<size_t>(nnz, 1));
  c->d_fself = cv.take<double>(3 * M);
  c->d_fpt = cv.take<double>(3 * MN);
  c->d_fpts = cv.take<double>(3 * M);
  c->d_flsrc = cv.take<double>(3 * M);
  c->d_fysrc = cv.take<double>(3 * M);
  c->d_gphi = cv.take<double>(3 * MN);
  c->d_F = cv.take<double>(3 * M);
  *total = cv.off + 256;
}

size_t workspace_size(ddlpb_ctx* c) {
  size_t t = 0;
  carve(c, nullptr, &t);
  return t;
}

// ------------------------------------------------------------ launchers
#define LM_DISPATCH(LMV, BODY)                 \
  switch (LMV) {                               \
    case 0: { constexpr int LMc = 0; BODY; } break;  \
    case 1: { constexpr int LMc = 1; BODY; } break;  \
    case 2: { constexpr int LMc = 2; BODY; } break;  \
    case 3: { constexpr int LMc = 3; BODY; } break;  \
    case 4: { constexpr int LMc = 4; BODY; } break;  \
    case 5: { constexpr int LMc = 5; BODY; } break;  \
    case 6: { constexpr int LMc = 6; BODY; } break;  \
    case 7: { constexpr int LMc = 7; BODY; } break;  \
    case 8: { constexpr int LMc = 8; BODY; } break;  \
    case 9: { constexpr int LMc = 9; BODY; } break;  \
    case 10: { constexpr int LMc = 10; BODY; } break; \
    case 11: { constexpr int LMc = 11; BODY; } break; \
    default: throw HipError{hipErrorInvalidValue};   \
  }

inline unsigned nblk(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void fill(ddlpb_ctx* c, double* p, long n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, c->stream, n, v, p);
  HIPCHK(hipGetLastError());
}

// m = C (.) An(U (.) (e + Syn(y(X))))
void moments(ddlpb_ctx* c, const double* X, const double* egrid, double* h_out, double* m_out) {
  LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_moments<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M, c->N, c->LY,
                                          c->d_Y, c->d_leb, c->d_U, X, c->d_ycr, c->d_yce, c->LUR, egrid, c->d_Cl,
                                          h_out, m_out));
  HIPCHK(hipGetLastError());
}

// Phi (value on the grid, zero on inactive points) or grad Phi' at active points
void sl_field(ddlpb_ctx* c, const double* m, bool grad, int exclude_self, double* out) {
  if (c->nact == 0) return;
  if (!grad) fill(c, out, (long)c->M * c->N, 0.0);
  if (grad) {
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_sl_field_direct<LMc, true>), dim3(nblk(c->nact, 256)), dim3(256), 0,
                                            c->stream, c->M, c->N, c->nact, c->d_actsph, c->d_actn, c->d_xyz,
                                            c->d_rad, c->d_leb, m, c->d_ur, c->LUR, c->kappa, exclude_self, out));
  } else {
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_sl_field_direct<LMc, false>), dim3(nblk(c->nact, 256)), dim3(256), 0,
                                            c->stream, c->M, c->N, c->nact, c->d_actsph, c->d_actn, c->d_xyz,
                                            c->d_rad, c->d_leb, m, c->d_ur, c->LUR, c->kappa, exclude_self, out));
  }
  HIPCHK(hipGetLastError());
}

// lambda (stride (lo+1)^2) from grid charges
void sl_adjoint(ddlpb_ctx* c, const double* cgrid, int lo, int exclude_self, double* lam) {
  if (c->nact == 0) { fill(c, lam, (long)c->M * (lo + 1) * (lo + 1), 0.0); return; }
  LM_DISPATCH(lo, hipLaunchKernelGGL((k_sl_adjoint_direct<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M, c->N,
                                     c->nact, c->d_actsph, c->d_actn, c->d_xyz, c->d_rad, c->d_leb, cgrid, c->d_ur,
                                     c->LUR, c->kappa, exclude_self, lam));
  HIPCHK(hipGetLastError());
}

void apply_LX(ddlpb_ctx* c, const double* base, double c0, const double* nearX, double c1, const double* gr1,
              const double* gr2, const double* ge, double cg, double* out) {
  LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_apply_LX<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M, c->N, c->LY,
                                          c->d_Y, c->d_leb, c->d_xyz, c->d_rad, c->d_nptr, c->d_nidx, c->d_f, c->d_U,
                                          c->d_sgr, c->LUR, c->kappa, c->eta, c->nterms, base, c0, nearX, c1, gr1,
                                          gr2, ge, cg, out));
  HIPCHK(hipGetLastError());
}

void syn2(ddlpb_ctx* c, const double* Z, int mode, double* o1, double* o2) {
  LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_syn2<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M, c->N, c->LY,
                                          c->d_Y, c->d_leb, c->d_U, Z, mode, o1, o2));
  HIPCHK(hipGetLastError());
}

void apply_LTZ(ddlpb_ctx* c, const double* base, double c0, const double* zr, const double* ze, double c1,
               const double* lam, int llam, double* out) {
  LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_apply_LTZ<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M, c->N, c->LY,
                                          c->d_Y, c->d_leb, c->d_xyz, c->d_rad, c->d_nptr, c->d_nidx, c->d_f, c->d_U,
                                          c->d_sgr, c->d_ycr, c->d_yce, c->d_Cl, c->LUR, c->kappa, c->eta, c->nterms,
                                          base, c0, zr, ze, c1, lam, llam, out));
  HIPCHK(hipGetLastError());
}

// ---- operators
// y = L x
void op_L(ddlpb_ctx* c, const double* x, double* y) {
  moments(c, x, nullptr, nullptr, c->d_m);
  sl_field(c, c->d_m, false, 0, c->d_Phi);
  apply_LX(c, x, 1.0, x, -1.0, c->d_Phi, nullptr, c->d_Phi, 1.0, y);
}
// y = L^T x
void op_LT(ddlpb_ctx* c, const double* x, double* y) {
  syn2(c, x, 1, c->d_cg, nullptr);
  sl_adjoint(c, c->d_cg, c->lmax, 0, c->d_lam);
  syn2(c, x, 0, c->d_zr, c->d_ze);
  apply_LTZ(c, x, 1.0, c->d_zr, c->d_ze, -1.0, c->d_lam, c->L, y);
}
// z = P^-1 v: k Jacobi sweeps z <- v + (I - L_AB) z from z = v (or the transposed sweeps)
void precond(ddlpb_ctx* c, bool transpose, const double* v, double* z) {
  const long D = 2L * c->M * c->L;
  HIPCHK(hipMemcpyAsync(z, v, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  for (int s = 0; s < c->sweeps; ++s) {
    if (!transpose) {
      apply_LX(c, v, 1.0, z, 1.0, nullptr, nullptr, nullptr, 0.0, c->d_t3);
    } else {
      syn2(c, z, 0, c->d_zr, c->d_ze);
      apply_LTZ(c, v, 1.0, c->d_zr, c->d_ze, 1.0, nullptr, 0, c->d_t3);
    }
    HIPCHK(hipMemcpyAsync(z, c->d_t3, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  }
}

// ---- BLAS-1 on the device (deterministic reductions)
void mdot(ddlpb_ctx* c, int nv, const double* V, long ldv, const double* w, double* h_host) {
  const long D = 2L * c->M * c->L;
  hipLaunchKernelGGL(k_mdot_part, dim3(c->nb_dot, nv), dim3(256), 0, c->stream, D, nv, V, ldv, w, c->d_part);
  hipLaunchKernelGGL(k_mdot_final, dim3(nv), dim3(256), 0, c->stream, c->nb_dot, c->d_part, c->d_hv);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h_host, c->d_hv, nv * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}
double norm2(ddlpb_ctx* c, const double* w) {
  double h;
  mdot(c, 1, w, 0, w, &h);
  return std::sqrt(h);
}
void mupdate(ddlpb_ctx* c, int nv, const double* V, long ldv, const double* h_host, double* w) {
  const long D = 2L * c->M * c->L;
  HIPCHK(hipMemcpyAsync(c->d_hv, h_host, nv * sizeof(double), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_mupdate, dim3(nblk(D, 256)), dim3(256), 0, c->stream, D, nv, V, ldv, c->d_hv, w);
  HIPCHK(hipGetLastError());
}
void axpby(ddlpb_ctx* c, double a, const double* x, double b, double* y) {
  const long D = 2L * c->M * c->L;
  hipLaunchKernelGGL(k_axpby, dim3(nblk(D, 256)), dim3(256), 0, c->stream, D, a, x, b, y);
  HIPCHK(hipGetLastError());
}

// Right-preconditioned restarted GMRES with classical Gram-Schmidt and one
// re-orthogonalisation; stops at ||b - A x|| <= tol ||b||.
int gmres(ddlpb_ctx* c, bool transpose, const double* b, double* x, double tol, int* iters, double* relres) {
  const long D = 2L * c->M * c->L;
  const int m = c->restart;
  auto op = [&](const double* in, double* out) { if (transpose) op_LT(c, in, out); else op_L(c, in, out); };
  const double bn = norm2(c, b);
  *iters = 0;
  *relres = 0.0;
  if (bn == 0.0) { fill(c, x, D, 0.0); return DDLPB_OK; }
  int total = 0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), h(m + 1), h2(m + 1), y(m);
  double rel = 0.0;
  bool conv = false;
  while (true) {
    op(x, c->d_w);
    HIPCHK(hipMemcpyAsync(c->d_V, b, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    axpby(c, -1.0, c->d_w, 1.0, c->d_V);  // V0 = b - A x
    const double beta = norm2(c, c->d_V);
    rel = beta / bn;
    if (rel <= tol) { conv = true; break; }
    if (total >= c->maxit) break;
    axpby(c, 0.0, c->d_w, 1.0 / beta, c->d_V);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int j = 0;
    for (; j < m && total < c->maxit; ++j) {
      precond(c, transpose, c->d_V + (long)j * D, c->d_t1);
      double* w = c->d_V + (long)(j + 1) * D;
      op(c->d_t1, w);
      mdot(c, j + 1, c->d_V, D, w, h.data());
      mupdate(c, j + 1, c->d_V, D, h.data(), w);
      mdot(c, j + 1, c->d_V, D, w, h2.data());
      mupdate(c, j + 1, c->d_V, D, h2.data(), w);
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i] + h2[i];
      const double hn = norm2(c, w);
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0) axpby(c, 0.0, c->d_w, 1.0 / hn, w);
      for (int i = 0; i < j; ++i) {
        double t = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = t;
      }
      const double den = std::hypot(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j]);
      cs[j] = H[(size_t)j * m + j] / den;
      sn[j] = H[(size_t)(j + 1) * m + j] / den;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++total;
      if (std::fabs(gv[j + 1]) <= 0.5 * tol * bn || hn == 0.0) { ++j; break; }
    }
    for (int i = j - 1; i >= 0; --i) {
      double a = gv[i];
      for (int k = i + 1; k < j; ++k) a -= H[(size_t)i * m + k] * y[k];
      y[i] = a / H[(size_t)i * m + i];
    }
    HIPCHK(hipMemcpyAsync(c->d_hv, y.data(), j * sizeof(double), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_mcomb, dim3(nblk(D, 256)), dim3(256), 0, c->stream, D, j, c->d_V, D, c->d_hv, c->d_t2);
    HIPCHK(hipGetLastError());
    precond(c, transpose, c->d_t2, c->d_t1);
    axpby(c, 1.0, c->d_t1, 1.0, x);
  }
  *iters = total;
  *relres = rel;
  return conv ? DDLPB_OK : DDLPB_ENOCONV;
}

// ------------------------------------------------------------ device setup
void upload_and_init(ddlpb_ctx* c) {
  ensure_constants();
  const int M = c->M, N = c->N, LUR = c->LUR;
  // per-sphere radial tables (FP64, host)
  std::vector<double> ycr((size_t)M * LUR), yce((size_t)M * LUR), Cl((size_t)M * LUR), sgr((size_t)M * LUR),
      ur((size_t)M * LUR), kr((size_t)M * LUR);
  std::vector<double> sg(LUR + 1), kk(LUR + 1);
  double rmax = 0;
  for (int j = 0; j < M; ++j) {
    const double rj = c->r[j], z = c->kappa * rj;
    rmax = std::max(rmax, rj);
    host::bessel_sigma(LUR, z * z, sg.data());
    host::bessel_k<double>(LUR, z, kk.data());
    for (int l = 0; l < LUR; ++l) {
      ycr[(size_t)j * LUR + l] = (c->eps1 / c->eps2) * l / rj;
      // i_l'(kappa r)/i_l(kappa r) * kappa = kappa^2 r sigma_{l+1}/sigma_l + l/r
      yce[(size_t)j * LUR + l] = -(c->kappa * c->kappa * rj * sg[l + 1] / sg[l] + l / rj);
      // C_l = (2/pi) kappa r^2 i_l(kappa r) k_l(kappa r)  (Wronskian form of (i'/i - k'/k)^-1)
      Cl[(size_t)j * LUR + l] = 2.0 / host::kPi * c->kappa * rj * rj * std::pow(z, l) * sg[l] * kk[l];
      sgr[(size_t)j * LUR + l] = sg[l];
      ur[(size_t)j * LUR + l] = kk[l] / std::pow(rj, l);
      kr[(size_t)j * LUR + l] = kk[l];
    }
  }
  c->nterms = host::sigma_terms(c->lmax, c->kappa * c->kappa * rmax * rmax);
  // Y table up to degree lmax+1
  std::vector<double> Y((size_t)N * c->LY);
  for (int n = 0; n < N; ++n) {
    const double* s = c->rule->xyzw + 4 * n;
    host::solid_harmonics<double>(c->lmax + 1, s[0], s[1], s[2], &Y[(size_t)n * c->LY]);
  }
  std::vector<double> dtab;
  host::gradient_coupling(c->lmax, dtab);
  auto up = [&](void* d, const void* h, size_t bytes) {
    if (bytes) HIPCHK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c->stream));
  };
  up(c->d_xyz, c->x.data(), 3 * M * sizeof(double));
  up(c->d_rad, c->r.data(), M * sizeof(double));
  up(c->d_q, c->q.data(), M * sizeof(double));
  up(c->d_leb, c->rule->xyzw, 4 * N * sizeof(double));
  up(c->d_Y, Y.data(), Y.size() * sizeof(double));
  up(c->d_nptr, c->nptr.data(), (M + 1) * sizeof(int));
  up(c->d_nidx, c->nidx.data(), c->nidx.size() * sizeof(int));
  up(c->d_nrev, c->nrev.data(), c->nrev.size() * sizeof(int));
  up(c->d_ycr, ycr.data(), ycr.size() * sizeof(double));
  up(c->d_yce, yce.data(), yce.size() * sizeof(double));
  up(c->d_Cl, Cl.data(), Cl.size() * sizeof(double));
  up(c->d_sgr, sgr.data(), sgr.size() * sizeof(double));
  up(c->d_ur, ur.data(), ur.size() * sizeof(double));
  up(c->d_kr, kr.data(), kr.size() * sizeof(double));
  up(c->d_dtab, dtab.data(), dtab.size() * sizeof(double));
  // Q: Q_r,j00 = q_j / sqrt(4 pi)
  std::vector<double> Qv((size_t)2 * M * c->L, 0.0);
  for (int j = 0; j < M; ++j) Qv[(size_t)j * c->L] = c->q[j] / std::sqrt(4.0 * host::kPi);
  up(c->d_Q, Qv.data(), Qv.size() * sizeof(double));
  const long D = 2L * M * c->L;
  fill(c, c->d_X, D, 0.0);
  fill(c, c->d_Xa, D, 0.0);
  c->dev_ready = true;
}

// grid fields and active point lists (depend on the centres)
void geometry_on_device(ddlpb_ctx* c) {
  const int M = c->M, N = c->N;
  HIPCHK(hipMemcpyAsync(c->d_xyz, c->x.data(), 3 * M * sizeof(double), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_grid_fields, dim3(nblk((long)M * N, 256)), dim3(256), 0, c->stream, M, N, c->d_xyz, c->d_rad,
                     c->d_leb, c->d_nptr, c->d_nidx, c->eta, c->d_f, c->d_U);
  hipLaunchKernelGGL(k_active_count, dim3(nblk(M, 128)), dim3(128), 0, c->stream, M, N, c->d_U, c->d_actcnt);
  HIPCHK(hipGetLastError());
  std::vector<int> cnt(M), ptr(M + 1, 0);
  HIPCHK(hipMemcpyAsync(cnt.data(), c->d_actcnt, M * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int i = 0; i < M; ++i) ptr[i + 1] = ptr[i] + cnt[i];
  c->nact = ptr[M];
  HIPCHK(hipMemcpyAsync(c->d_actptr, ptr.data(), (M + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_active_fill, dim3(nblk(M, 128)), dim3(128), 0, c->stream, M, N, c->d_U, c->d_actptr,
                     c->d_actsph, c->d_actn);
  HIPCHK(hipGetLastError());
  c->stats.n_active_points = c->nact;
  c->stats.n_near_pairs = (int64_t)M * M;
  c->rhs_ready = false;
}

int ensure_device(ddlpb_ctx* c) {
  if (c->dev_ready) return DDLPB_OK;
  size_t need = workspace_size(c);
  if (!c->ws_bound) {
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) return DDLPB_ENOMEM;
    c->ws = (char*)p;
    c->ws_bytes = need;
    c->ws_owned = true;
  }
  size_t t;
  carve(c, c->ws, &t);
  auto t0 = std::chrono::steady_clock::now();
  upload_and_init(c);
  geometry_on_device(c);
  HIPCHK(hipStreamSynchronize(c->stream));
  c->stats.ms_setup = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return DDLPB_OK;
}

void compute_rhs(ddlpb_ctx* c) {
  const long MN = (long)c->M * c->N;
  fill(c, c->d_psi, MN, 0.0);
  fill(c, c->d_e, MN, 0.0);
  if (c->nact > 0) {
    hipLaunchKernelGGL(k_laplace_field_direct, dim3(nblk(c->nact, 256)), dim3(256), 0, c->stream, c->M, c->N, c->nact,
                       c->d_actsph, c->d_actn, c->d_xyz, c->d_rad, c->d_leb, c->d_q, c->eps1, c->eps2, c->d_psi,
                       c->d_e);
    HIPCHK(hipGetLastError());
  }
  moments(c, nullptr, c->d_e, nullptr, c->d_m);
  sl_field(c, c->d_m, false, 0, c->d_Phi);
  apply_LX(c, nullptr, 0.0, nullptr, 0.0, c->d_psi, c->d_Phi, c->d_Phi, -1.0, c->d_g);
  c->rhs_ready = true;
}

double elapsed_ms(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const HipError&) {
    return DDLPB_EDEVICE;
  } catch (const std::bad_alloc&) {
    return DDLPB_ENOMEM;
  }
}

}  // namespace

// ======================================================================== ABI
extern "C" {

int ddlpb_setup(int32_t n_atoms, const double* centers, const double* radii, const double* charges, double eps_in,
                double eps_out, double kappa, int32_t lmax, int32_t n_lebedev, int32_t fmm_order, ddlpb_ctx** out) {
  if (!out) return DDLPB_EINVAL;
  int rc = check_inputs(n_atoms, centers, radii, charges, eps_in, eps_out, kappa, lmax, n_lebedev, fmm_order);
  if (rc) return rc;
  return guarded([&]() -> int {
    auto* c = new ddlpb_ctx();
    c->M = n_atoms;
    c->lmax = lmax;
    c->L = (lmax + 1) * (lmax + 1);
    c->LP = (lmax + 2) * (lmax + 2);
    c->LY = c->LP;
    c->LUR = lmax + 2;
    c->N = n_lebedev;
    c->rule = host::lebedev_rule(n_lebedev);
    c->fmm_order = fmm_order;
    c->eps1 = eps_in; c->eps2 = eps_out; c->kappa = kappa;
    c->x.assign(centers, centers + 3L * n_atoms);
    c->r.assign(radii, radii + n_atoms);
    c->q.assign(charges, charges + n_atoms);
    int r2 = build_neighbours(c);
    if (r2) { delete c; return r2; }
    c->stats.fmm_order = fmm_order;
    c->stats.fmm_order_below_lmax = (fmm_order > 0 && fmm_order < lmax) ? 1 : 0;
    *out = c;
    return DDLPB_OK;
  });
}

int ddlpb_solve(ddlpb_ctx* c, double tol, double* energy_out) {
  if (!c || !(tol > 0)) return DDLPB_EINVAL;
  return guarded([&]() -> int {
    int rc = ensure_device(c);
    if (rc) return rc;
    auto t0 = std::chrono::steady_clock::now();
    if (!c->rhs_ready) compute_rhs(c);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->stats.ms_rhs = elapsed_ms(t0);
    t0 = std::chrono::steady_clock::now();
    int it = 0;
    double rel = 0;
    rc = gmres(c, false, c->d_g, c->d_X, tol, &it, &rel);
    c->stats.iters_primal = it;
    c->stats.resid_primal = rel;
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(1024), 0, c->stream, c->M, c->L, c->d_X, c->d_q, c->d_scal);
    HIPCHK(hipGetLastError());
    double E = 0;
    HIPCHK(hipMemcpyAsync(&E, c->d_scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->stats.ms_primal = elapsed_ms(t0);
    c->energy = E;
    if (energy_out) *energy_out = E;
    c->state = 1;
    return rc;
  });
}

int ddlpb_adjoint(ddlpb_ctx* c, double tol) {
  if (!c || !(tol > 0)) return DDLPB_EINVAL;
  if (c->state < 1) return DDLPB_ESTATE;
  return guarded([&]() -> int {
    auto t0 = std::chrono::steady_clock::now();
    int it = 0;
    double rel = 0;
    int rc = gmres(c, true, c->d_Q, c->d_Xa, tol, &it, &rel);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->stats.iters_adjoint = it;
    c->stats.resid_adjoint = rel;
    c->stats.ms_adjoint = elapsed_ms(t0);
    c->state = 2;
    return rc;
  });
}

int ddlpb_forces(ddlpb_ctx* c, double* forces_out) {
  if (!c || !forces_out) return DDLPB_EINVAL;
  if (c->state < 2) return DDLPB_ESTATE;
  return guarded([&]() -> int {
    auto t0 = std::chrono::steady_clock::now();
    const int M = c->M, N = c->N;
    const long MN = (long)M * N;
    // xi_r, xi_e on the grid; grid charges c = w U xi_s
    syn2(c, c->d_Xa, 0, c->d_xr, c->d_xe);
    syn2(c, c->d_Xa, 1, c->d_cg, nullptr);
    // h = e + Syn(y(X)), m = C (.) An(U h), Phi = Phi[m] (full)
    moments(c, c->d_X, c->d_e, c->d_h, c->d_m);
    sl_field(c, c->d_m, false, 0, c->d_Phi);
    // lambda' (other spheres only, degree lmax+1) and eta = Syn(C (.) lambda)
    sl_adjoint(c, c->d_cg, c->lmax + 1, 1, c->d_lam);
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_eta<LMc>), dim3(M), dim3(256), 0, c->stream, M, N, c->LY, c->d_Y,
                                            c->d_cg, c->d_lam, c->LP, c->d_Cl, c->LUR, c->d_eta));
    HIPCHK(hipGetLastError());
    // grad Phi' at active points
    if (c->nact > 0) sl_field(c, c->d_m, true, 1, c->d_gphi);
    // switching / near-field terms
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_force_switch<LMc>), dim3(M), dim3(256), 0, c->stream, M, N, c->d_leb,
                                            c->d_xyz, c->d_rad, c->d_nptr, c->d_nidx, c->d_f, c->d_U, c->d_sgr,
                                            c->LUR, c->kappa, c->eta, c->nterms, c->d_X, c->d_xr, c->d_xe, c->d_psi,
                                            c->d_Phi, c->d_h, c->d_eta, c->d_fnb, c->d_fself));
    HIPCHK(hipGetLastError());
    // target-side point terms, summed per sphere
    fill(c, c->d_fpts, 3L * M, 0.0);
    if (c->nact > 0) {
      hipLaunchKernelGGL(k_force_points, dim3(nblk(c->nact, 256)), dim3(256), 0, c->stream, M, N, c->nact,
                         c->d_actsph, c->d_actn, c->d_xyz, c->d_rad, c->d_leb, c->d_q, c->eps1, c->eps2, c->d_U,
                         c->d_xr, c->d_xe, c->d_eta, c->d_gphi, 1, c->d_fpt);
      hipLaunchKernelGGL(k_sum_points, dim3(M), dim3(256), 0, c->stream, M, c->d_actptr, c->d_fpt, c->d_fpts);
      HIPCHK(hipGetLastError());
    }
    // source-side terms
    hipLaunchKernelGGL(k_force_laplace_source, dim3(M), dim3(256), 0, c->stream, M, N, c->nact, c->d_actsph,
                       c->d_actn, c->d_xyz, c->d_rad, c->d_leb, c->d_q, c->eps1, c->eps2, c->d_U, c->d_xr, c->d_eta,
                       c->d_flsrc);
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_force_yukawa_source<LMc>), dim3(M), dim3(128), 0, c->stream, M,
                                            c->d_m, c->d_lam, c->d_dtab, c->d_kr, c->LUR, c->kappa, c->d_fysrc));
    hipLaunchKernelGGL(k_force_final, dim3(nblk(M, 256)), dim3(256), 0, c->stream, M, c->d_nptr, c->d_nidx,
                       c->d_nrev, c->d_fnb, c->d_fself, c->d_fpts, c->d_flsrc, c->d_fysrc, c->d_F);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(forces_out, c->d_F, 3L * M * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    (void)MN;
    c->stats.ms_forces = elapsed_ms(t0);
    return DDLPB_OK;
  });
}

void ddlpb_free(ddlpb_ctx* c) {
  if (!c) return;
  if (c->ws_owned && c->ws) (void)hipFree(c->ws);
  delete c;
}

int ddlpb_set_option(ddlpb_ctx* c, const char* key, double v) {
  if (!c || !key) return DDLPB_EINVAL;
  std::string k(key);
  const bool fixed = c->dev_ready;
  if (k == "eta") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v > 0 && v <= 1)) return DDLPB_EINVAL;
    c->eta = v;
  } else if (k == "precision") {
    if (fixed) return DDLPB_ESTATE;
    if (v != 0 && v != 1) return DDLPB_EINVAL;
    c->precision = (int)v;
    c->stats.precision = (int)v;
  } else if (k == "gmres_restart") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v >= 1 && v <= 200)) return DDLPB_EINVAL;
    c->restart = (int)v;
  } else if (k == "inner_sweeps") {
    if (!(v >= 0 && v <= 64)) return DDLPB_EINVAL;
    c->sweeps = (int)v;
  } else if (k == "max_iter") {
    if (!(v >= 1 && v <= 1e6)) return DDLPB_EINVAL;
    c->maxit = (int)v;
  } else if (k == "leaf_size") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v >= 1 && v <= 4096)) return DDLPB_EINVAL;
    c->leaf = (int)v;
  } else if (k == "theta") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v > 0 && v < 1)) return DDLPB_EINVAL;
    c->theta = v;
  } else {
    return DDLPB_EINVAL;
  }
  return DDLPB_OK;
}

int ddlpb_update_centers(ddlpb_ctx* c, const double* centers) {
  if (!c || !centers) return DDLPB_EINVAL;
  for (int i = 0; i < 3 * c->M; ++i)
    if (!std::isfinite(centers[i])) return DDLPB_EINVAL;
  return guarded([&]() -> int {
    std::vector<double> old = c->x;
    std::vector<int> onptr = c->nptr, onidx = c->nidx, onrev = c->nrev;
    c->x.assign(centers, centers + 3L * c->M);
    int rc = build_neighbours(c);
    if (rc) { c->x = old; c->nptr = onptr; c->nidx = onidx; c->nrev = onrev; return rc; }
    if (c->dev_ready) {
      if (c->nidx.size() != onidx.size()) {
        // neighbour count changed: the workspace layout changes, rebuild the device state
        std::vector<double> X(2L * c->M * c->L), Xa(2L * c->M * c->L);
        HIPCHK(hipMemcpyAsync(X.data(), c->d_X, X.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(Xa.data(), c->d_Xa, Xa.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        size_t need = workspace_size(c);
        if (c->ws_bound && need > c->ws_bytes) return DDLPB_ENOMEM;
        if (c->ws_owned && need > c->ws_bytes) {
          (void)hipFree(c->ws);
          void* p = nullptr;
          if (hipMalloc(&p, need) != hipSuccess) { c->ws = nullptr; c->dev_ready = false; return DDLPB_ENOMEM; }
          c->ws = (char*)p;
          c->ws_bytes = need;
        }
        size_t t;
        carve(c, c->ws, &t);
        upload_and_init(c);
        HIPCHK(hipMemcpyAsync(c->d_X, X.data(), X.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->d_Xa, Xa.data(), Xa.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
      } else {
        HIPCHK(hipMemcpyAsync(c->d_nidx, c->nidx.data(), c->nidx.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->d_nrev, c->nrev.data(), c->nrev.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->d_nptr, c->nptr.data(), (c->M + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
      }
      geometry_on_device(c);
      HIPCHK(hipStreamSynchronize(c->stream));
    }
    c->state = 0;
    c->rhs_ready = false;
    return DDLPB_OK;
  });
}

size_t ddlpb_workspace_bytes(const ddlpb_ctx* c) {
  if (!c) return 0;
  return workspace_size(const_cast<ddlpb_ctx*>(c));
}

int ddlpb_bind_workspace(ddlpb_ctx* c, void* dev, size_t bytes) {
  if (!c || !dev) return DDLPB_EINVAL;
  if (((uintptr_t)dev & 255) != 0) return DDLPB_EINVAL;
  if (bytes < workspace_size(c)) return DDLPB_ENOMEM;
  if (c->dev_ready) return DDLPB_ESTATE;
  if (c->ws_owned && c->ws) (void)hipFree(c->ws);
  c->ws_owned = false;
  c->ws_bound = true;
  c->ws = (char*)dev;
  c->ws_bytes = bytes;
  return DDLPB_OK;
}

int ddlpb_set_stream(ddlpb_ctx* c, void* s) {
  if (!c) return DDLPB_EINVAL;
  c->stream = (hipStream_t)s;
  return DDLPB_OK;
}

int ddlpb_get_stats(const ddlpb_ctx* c, ddlpb_stats* out) {
  if (!c || !out) return DDLPB_EINVAL;
  *out = c->stats;
  return DDLPB_OK;
}

const char* ddlpb_strerror(int code) {
  int k = -code;
  if (k < 0 || k > 6) return "unknown error";
  return kErr[k];
}

int ddlpb_get_grid(ddlpb_ctx* c, double* f_out, double* u_out) {
  if (!c) return DDLPB_EINVAL;
  return guarded([&]() -> int {
    int rc = ensure_device(c);
    if (rc) return rc;
    const size_t MN = (size_t)c->M * c->N;
    if (f_out) HIPCHK(hipMemcpyAsync(f_out, c->d_f, MN * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (u_out) HIPCHK(hipMemcpyAsync(u_out, c->d_U, MN * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DDLPB_OK;
  });
}

int ddlpb_get_solution(ddlpb_ctx* c, double* x_out, double* xadj_out) {
  if (!c) return DDLPB_EINVAL;
  if (c->state < 1 && x_out) return DDLPB_ESTATE;
  if (c->state < 2 && xadj_out) return DDLPB_ESTATE;
  return guarded([&]() -> int {
    const size_t D = 2L * c->M * c->L;
    if (x_out) HIPCHK(hipMemcpyAsync(x_out, c->d_X, D * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (xadj_out) HIPCHK(hipMemcpyAsync(xadj_out, c->d_Xa, D * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DDLPB_OK;
  });
}

int ddlpb_get_rhs(ddlpb_ctx* c, double* g_out) {
  if (!c || !g_out) return DDLPB_EINVAL;
  return guarded([&]() -> int {
    int rc = ensure_device(c);
    if (rc) return rc;
    if (!c->rhs_ready) compute_rhs(c);
    const size_t D = 2L * c->M * c->L;
    HIPCHK(hipMemcpyAsync(g_out, c->d_g, D * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DDLPB_OK;
  });
}

int ddlpb_apply(ddlpb_ctx* c, int32_t transpose, const double* x_in, double* y_out) {
  if (!c || !x_in || !y_out) return DDLPB_EINVAL;
  return guarded([&]() -> int {
    int rc = ensure_device(c);
    if (rc) return rc;
    const size_t D = 2L * c->M * c->L;
    HIPCHK(hipMemcpyAsync(c->d_t2, x_in, D * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (transpose) op_LT(c, c->d_t2, c->d_w); else op_L(c, c->d_t2, c->d_w);
    HIPCHK(hipMemcpyAsync(y_out, c->d_w, D * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DDLPB_OK;
  });
}

}  // extern "C"
