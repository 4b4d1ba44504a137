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
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/ddlpb.h"
#include "host_math.hpp"
#include "kernels_forces.hpp"
#include "fmm.hpp"
#include "fmm_host.hpp"
#include "gemm_mfma.hpp"
#include "fmm_lane_api.hpp"
#include "near_lane_api.hpp"

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
  {
    std::vector<float> pf(pmm.begin(), pmm.end()), af(ra.begin(), ra.end()), bf(rb.begin(), rb.end());
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_pmm_f), pf.data(), pf.size() * sizeof(float)));
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_ra_f), af.data(), af.size() * sizeof(float)));
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_rb_f), bf.data(), bf.size() * sizeof(float)));
  }
  std::vector<double> sinv((kLmaxDev + 2) * kSigTerms);
  for (int l = 0; l <= kLmaxDev + 1; ++l)
    for (int k = 0; k < kSigTerms; ++k) sinv[l * kSigTerms + k] = 0.5 / ((k + 1.0) * (2.0 * l + 2.0 * k + 3.0));
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_sinv), sinv.data(), sinv.size() * sizeof(double)));
  HIPCHK(nearlane::upload_tables(pmm.data(), ra.data(), rb.data()));
  g_const_done[dev] = true;
}

// Internal order of the Lebedev points: the leaves of a recursive bisection (split at
// the median of the coordinate with the largest spread), so that the points of a
// spherical cap -- the grid points of a sphere inside a neighbour -- have few runs of
// consecutive indices and reads of per-point data by cap are coalesced.  Every sum
// over the points is independent of the order up to rounding.
void order_points(const double* xyzw, int N, std::vector<int>& ord) {
  ord.resize(N);
  for (int n = 0; n < N; ++n) ord[n] = n;
  std::function<void(int, int)> split = [&](int lo, int hi) {
    if (hi - lo <= 2) return;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int k = lo; k < hi; ++k)
      for (int a = 0; a < 3; ++a) {
        mn[a] = std::min(mn[a], xyzw[4 * ord[k] + a]);
        mx[a] = std::max(mx[a], xyzw[4 * ord[k] + a]);
      }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (mx[a] - mn[a] > mx[ax] - mn[ax]) ax = a;
    std::sort(ord.begin() + lo, ord.begin() + hi, [&](int p, int q) {
      const double a = xyzw[4 * p + ax], b = xyzw[4 * q + ax];
      return a < b || (a == b && p < q);
    });
    const int mid = (lo + hi) / 2;
    split(lo, mid);
    split(mid, hi);
  };
  split(0, N);
}

}  // namespace

struct ddlpb_ctx {
  // ---- problem
  int M = 0, lmax = 0, L = 0, LP = 0, LY = 0, LUR = 0, N = 0, fmm_order = 0;
  double eps1 = 1, eps2 = 78.54, kappa = 0.1, eta = 0.05;
  std::vector<double> x, r, q;
  const ddlpb_tables::LebedevRule* rule = nullptr;
  // the rule's points and weights in the library's internal order (spatially coherent,
  // see order_points) and the rule's index of every internal point
  std::vector<double> leb;
  std::vector<int> leb_orig;
  // ---- options
  int precision = 0, restart = 100, sweeps = 1, maxit = 400;
  int cur_prec = 0;           // compute type of the operator kernels now: 0 FP64, 1 FP32 (inner mixed solves)
  bool sl32 = false;          // near single layer of the operator in FP32 (outer iterations of precision 1)
  int fp64_iters = 0;         // FP64 outer iterations after the FP32 ones in the last solve (precision 1)
  bool mixed_sl = false;
  bool inner_reorth = false;  // option inner_reorth: second Gram-Schmidt pass in the inner Krylov steps
  bool m2l32 = false;         // screened Coulomb M2L with the FP32 vector (precision 1; level passes too with mixed_lvl)
  bool mixed_lvl = false;     // option mixed_levels: the order-12 level translations of the FP32 passes in FP32 too
  bool mixed_m2l = true;      // precision 1: outer iterations with the FP32-vector M2L (option mixed_m2l)
  bool mixed_forces = true;   // precision 1: single-layer force terms with FP32 pairs and M2L (option mixed_forces)      // precision 1: outer iterations with the FP32 near single layer (option mixed_near_sl)
  double *d_rr = nullptr, *d_dd = nullptr;
  double* d_YT = nullptr;
  double* d_WY = nullptr;     // w_n Y_lm(s_n), [N][L] (column-major L x N): the An projection as a GEMM
  double* d_Vpt = nullptr;    // point values of the A/B sums, [2M][N], input of the An GEMM
  int apply_fp32 = 0;         // ddlpb_apply: 1 FP32 near-field A/B kernels, 2 FP32 near single layer, 3 FP32-vector M2L (diagnostic)
  int pkrylov = 6;            // > 0: preconditioner = this many GMRES steps on L_AB (flexible outer)
  int solver = 0;             // 0: GMRES, 1: Jacobi-DIIS (the paper's macro/micro iterations)
  int diis_max = 8;           // DIIS history length
  int inner_iters = 12;       // GMRES steps on the near operator P per outer iteration
  double pdelta = -1.0;       // P keeps the single-layer blocks of spheres with |x_i-x_j| < r_i+r_j+pdelta
  bool warm_start = true;
  double theta = 0.6;
  int leaf_size = 1;          // FMM leaf groups: nodes of at most this many spheres interact directly
  int m2l_waves = 0;          // wavefronts per block of the LDS-resident M2L kernel (0: automatic, -1: block kernel)
  int m2l_lane = 1;           // order 12: the one-translation-per-lane M2L kernels (when m2l_waves is 0)
  int level_lane = 1024;      // order 12, screened Coulomb: levels of at least this many nodes take the
                              // one-translation-per-lane M2M / L2L kernels (0: never)
  int near_lane = 1;          // lmax <= 8: the near-field A/B kernels with one cap per lane
  int near_incore = 0;        // with near_lane: harmonics of every reverse cap kept in device memory
  bool use_lane = false;      // lane kernels set up for the current geometry
  int* d_f2r = nullptr;       // forward cap -> its position in the reverse lists
  double* d_capv = nullptr;   // (A, B) value pair of every reverse cap, [2 cap_cap]
  long* d_coff = nullptr;     // incore cache: first (padded) cap position of every sphere
  int* d_jord = nullptr;      // spheres by decreasing number of reverse caps
  double* d_cache = nullptr;  // incore cache (owned by the context, outside the workspace)
  size_t cache_bytes = 0;
  int m2l_layout = 0;         // last M2L layout: wavefronts per block, negative with tables in global memory
  struct M2LCfg { bool valid = false, alds = false; int nw = 0, per_cu = 0; size_t bytes = 0; } m2l_cfg[2];
  // ---- host analysis
  std::vector<int> nptr, nidx, nrev;
  std::vector<int> pptr, pidx;  // sphere pairs of the near preconditioner (self included)
  size_t nnz_cap = 0, pnz_cap = 0;  // capacities of the device copies of nidx / pidx
  size_t cap_est = 0, cap_cap = 0;  // estimated cap pairs and the capacity of the cap lists
  bool use_caps = false;            // cap lists built for the current geometry
  bool cap_lists = true;            // option cap_lists: 0 forces the kernels without cap lists
  int nterms = 8, nterms_p = 8;
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
  double* d_pt4 = nullptr;
  double *d_mu1 = nullptr, *d_mu2 = nullptr;
  double *d_ycr = nullptr, *d_yce = nullptr, *d_Cl = nullptr, *d_sgr = nullptr, *d_isgr = nullptr, *d_ur = nullptr, *d_iur = nullptr, *d_kr = nullptr;
  double *d_dtab = nullptr;
  double *d_rtab = nullptr;  // radius derivatives of the radial constants [4][M][LUR]
  double *d_m = nullptr, *d_lam = nullptr;
  double *d_psi = nullptr, *d_e = nullptr, *d_Phi = nullptr, *d_h = nullptr, *d_zr = nullptr, *d_ze = nullptr,
         *d_cg = nullptr, *d_eta = nullptr, *d_xr = nullptr, *d_xe = nullptr;
  double *d_g = nullptr, *d_X = nullptr, *d_Xa = nullptr, *d_Q = nullptr, *d_w = nullptr, *d_t1 = nullptr,
         *d_t2 = nullptr, *d_t3 = nullptr, *d_V = nullptr;
  double *d_part = nullptr, *d_hv = nullptr, *d_scal = nullptr;
  int *d_pptr = nullptr, *d_pidx = nullptr;
  int *d_cptr = nullptr, *d_capn = nullptr, *d_capslot = nullptr, *d_pcp = nullptr, *d_rptr = nullptr,
      *d_rci = nullptr, *d_rcn = nullptr;
  double *d_capw = nullptr, *d_rcw = nullptr;
  double *d_Z = nullptr, *d_Vin = nullptr, *d_t4 = nullptr, *d_t5 = nullptr;
  double *d_fnb = nullptr, *d_fself = nullptr, *d_fpt = nullptr, *d_fpts = nullptr, *d_flsrc = nullptr,
         *d_fysrc = nullptr, *d_gphi = nullptr, *d_F = nullptr;
  int nact = 0;
  long ncap = 0;  // cap pairs (i, n, j) with omega > 0, counted on the host
  double near_pairs_pts = 0.0;  // (active point, listed source sphere) pairs of the near list
  int nb_dot = 1024;
  int mk = 0;  // vectors the dot-product scratch holds (d_part, d_hv)
  // ---- fast multipole method (fmm_order > 0)
  fmm::Tree tree;
  fmm::Tables tables;
  size_t m2l_cap = 0, near_cap = 0;
  double *d_fcen = nullptr, *d_frad = nullptr, *d_fkR = nullptr, *d_fkRi = nullptr, *d_fiR = nullptr, *d_fA = nullptr, *d_fAL = nullptr,
         *d_fJ = nullptr, *d_Mn = nullptr, *d_Ln = nullptr, *d_SL = nullptr, *d_Lam = nullptr, *d_sgp = nullptr,
         *d_qsrc = nullptr, *d_tmp4 = nullptr;
  double* d_fjval = nullptr;
  int* d_fjrow = nullptr;
  double* d_fjpad = nullptr;
  double* d_fZ[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [kernel][direction]
  int* d_fZslot[2] = {nullptr, nullptr};
  double* d_fZl[2] = {nullptr, nullptr};  // level z-translation table [direction]
  int *d_fm2lord = nullptr, *d_fctr = nullptr;
  int *d_fJoff = nullptr, *d_fAoff = nullptr, *d_fchild = nullptr, *d_fparent = nullptr, *d_flevn = nullptr, *d_fm2lp = nullptr,
      *d_fm2ls = nullptr, *d_fnp = nullptr, *d_fni = nullptr,
      *d_sleaf = nullptr;
  double near_pts_fmm = 0.0;  // (active point, near source sphere) pairs of the FMM near list
  // ---- per-kernel device timing (option "kernel_timing")
  struct KTimer {
    std::string name;
    double ms = 0.0, work = 0.0;
    long launches = 0;
  };
  bool ktiming = false;
  std::vector<KTimer> ktimers;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  // ---- state
  int state = 0;  // 0 = set up, 1 = primal solved, 2 = adjoint solved
  bool rhs_ready = false;
  long inner_total = 0;
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
  if (lmax < 0 || lmax > kMaxLmax || p < 0 || p > 16) return DDLPB_EINVAL;
  // the grid must resolve the products of two degree-lmax harmonics with a margin of
  // two degrees: An_i(U_i Syn(c)) projects through the switching function, and with
  // less (lmax 8 on 110 points, degree 17) the operator's condition number grows
  // fivefold and the solves stagnate
  const auto* rule = host::lebedev_rule(nleb);
  if (!rule || rule->degree < 2 * lmax + 2) return DDLPB_EINVAL;
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
  std::atomic<bool> coincident{false};
  // sphere by sphere on the host threads (each list is sorted, so the result does not
  // depend on the schedule)
  fmm::parallel_for(M, 512, [&](long i) {
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
            if (d < 1e-12) coincident.store(true, std::memory_order_relaxed);
            if (d < c->r[i] + c->r[j]) nb[i].push_back(j);
          }
        }
    std::sort(nb[i].begin(), nb[i].end());
  });
  if (coincident.load()) return DDLPB_EGEOM;
  c->nptr.assign(M + 1, 0);
  for (int i = 0; i < M; ++i) c->nptr[i + 1] = c->nptr[i] + (int)nb[i].size();
  // cap pairs: the fraction of sphere i's surface inside ball j is (1 - c0)/2 with
  // c0 = (r_i^2 + d^2 - r_j^2) / (2 r_i d); Lebedev points are close to uniform.
  double est = 0.0;
  for (int i = 0; i < M; ++i)
    for (int j : nb[i]) {
      double d2 = 0;
      for (int a = 0; a < 3; ++a) { double t = c->x[3 * i + a] - c->x[3 * j + a]; d2 += t * t; }
      const double d = std::sqrt(d2);
      double c0 = (c->r[i] * c->r[i] + d2 - c->r[j] * c->r[j]) / (2.0 * c->r[i] * d);
      c0 = std::min(1.0, std::max(-1.0, c0));
      est += std::ceil(1.25 * c->N * 0.5 * (1.0 - c0) + 8.0);
    }
  c->cap_est = (size_t)est;
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

// Sphere pairs (i, j) with |x_i - x_j| < r_i + r_j + delta, i itself included, sorted by j.
void build_pairs(const ddlpb_ctx* c, double delta, std::vector<int>& ptr, std::vector<int>& idx) {
  const int M = c->M;
  if (delta < 0.0) {  // no two-level preconditioner: no pairs
    ptr.assign(M + 1, 0);
    idx.clear();
    return;
  }
  double rmax = 0;
  for (double v : c->r) rmax = std::max(rmax, v);
  const double cell = 2.0 * rmax + std::max(delta, 0.0);
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
  ptr.assign(M + 1, 0);
  idx.clear();
  std::vector<int> row;
  for (int i = 0; i < M; ++i) {
    row.clear();
    for (long dx = -1; dx <= 1; ++dx)
      for (long dy = -1; dy <= 1; ++dy)
        for (long dz = -1; dz <= 1; ++dz) {
          auto it = cells.find(key(ci[3L * i] + dx, ci[3L * i + 1] + dy, ci[3L * i + 2] + dz));
          if (it == cells.end()) continue;
          for (int j : it->second) {
            double d2 = 0;
            for (int a = 0; a < 3; ++a) { double t = c->x[3 * i + a] - c->x[3 * j + a]; d2 += t * t; }
            if (j == i || std::sqrt(d2) < c->r[i] + c->r[j] + delta) row.push_back(j);
          }
        }
    std::sort(row.begin(), row.end());
    idx.insert(idx.end(), row.begin(), row.end());
    ptr[i + 1] = (int)idx.size();
  }
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
  const size_t M = c->M, N = c->N, MN = M * N, D = 2 * M * c->L;
  c->nnz_cap = std::max(c->nnz_cap, c->nidx.size());
  c->pnz_cap = std::max(c->pnz_cap, c->pidx.size());
  const size_t nnz = c->nnz_cap;
  c->d_xyz = cv.take<double>(3 * M);
  c->d_rad = cv.take<double>(M);
  c->d_q = cv.take<double>(M);
  c->d_leb = cv.take<double>(4 * N);
  c->d_Y = cv.take<double>(N * c->LY);
  c->d_YT = cv.take<double>(N * c->LY);  // transposed [LY][N]: coalesced over points
  c->d_WY = cv.take<double>((size_t)N * c->L);
  c->d_Vpt = cv.take<double>(2 * MN);
  c->d_nptr = cv.take<int>(M + 1);
  c->d_nidx = cv.take<int>(std::max<size_t>(nnz, 1));
  c->d_nrev = cv.take<int>(std::max<size_t>(nnz, 1));
  c->d_f = cv.take<double>(MN);
  c->d_U = cv.take<double>(MN);
  c->d_actcnt = cv.take<int>(M);
  c->d_actptr = cv.take<int>(M + 1);
  c->d_actsph = cv.take<int>(MN);
  c->d_actn = cv.take<int>(MN);
  c->d_pt4 = cv.take<double>(4 * MN);  // active points and grid charges, packed [nact][4]
  c->d_ycr = cv.take<double>(M * c->LUR);
  c->d_yce = cv.take<double>(M * c->LUR);
  c->d_Cl = cv.take<double>(M * c->LUR);
  c->d_sgr = cv.take<double>(M * c->LUR);
  c->d_isgr = cv.take<double>(M * c->LUR);
  c->d_ur = cv.take<double>(M * c->LUR);
  c->d_iur = cv.take<double>(M * c->LUR);  // 1 / ur
  c->d_kr = cv.take<double>(M * c->LUR);
  c->d_dtab = cv.take<double>(3 * (size_t)c->L * c->LP);
  c->d_rtab = cv.take<double>(4 * (size_t)M * c->LUR);
  c->d_m = cv.take<double>(M * c->L);
  c->d_mu1 = cv.take<double>(M * c->L);  // coefficient rows of the two-product stages
  c->d_mu2 = cv.take<double>(M * c->L);
  c->d_lam = cv.take<double>(M * c->LP);
  c->d_psi = cv.take<double>(MN);
  c->d_e = cv.take<double>(MN);
  c->d_Phi = cv.take<double>(MN);
  c->d_h = cv.take<double>(MN);
  c->d_zr = cv.take<double>(2 * MN);  // zr and ze adjacent: [2M][N], output of the Syn GEMM
  c->d_ze = c->d_zr + MN;
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
  const bool two_level = c->pdelta >= 0.0;
  // flexible directions: two-level or Krylov preconditioner, or the FP32 sweeps of precision 1
  c->d_Z = (two_level || c->pkrylov > 0 || c->precision == 1) ? cv.take<double>((size_t)c->restart * D) : nullptr;
  c->d_Vin = (two_level || c->pkrylov > 0)
                 ? cv.take<double>((size_t)(std::max(c->inner_iters, c->pkrylov) + 1) * D)
                 : nullptr;
  c->d_t4 = cv.take<double>(D);
  c->d_t5 = cv.take<double>(D);
  c->d_rr = c->precision == 2 ? cv.take<double>(D) : nullptr;  // residual and correction of the refinement
  c->d_dd = c->precision == 2 ? cv.take<double>(D) : nullptr;
  c->d_pptr = cv.take<int>(M + 1);
  c->cap_cap = std::max(c->cap_cap, c->cap_est);
  c->d_cptr = cv.take<int>(M + 1);
  c->d_rptr = cv.take<int>(M + 1);
  c->d_pcp = cv.take<int>(M * (N + 1));
  c->d_capn = cv.take<int>(std::max<size_t>(c->cap_cap, 1));
  c->d_capslot = cv.take<int>(std::max<size_t>(c->cap_cap, 1));
  c->d_capw = cv.take<double>(std::max<size_t>(c->cap_cap, 1));
  c->d_rci = cv.take<int>(std::max<size_t>(c->cap_cap, 1));
  c->d_rcn = cv.take<int>(std::max<size_t>(c->cap_cap, 1));
  c->d_rcw = cv.take<double>(std::max<size_t>(c->cap_cap, 1));
  c->d_f2r = cv.take<int>(std::max<size_t>(c->cap_cap, 1));
  c->d_capv = cv.take<double>(2 * std::max<size_t>(c->cap_cap, 1));
  c->d_coff = cv.take<long>(M);
  c->d_jord = cv.take<int>(M);
  c->d_pidx = cv.take<int>(std::max<size_t>(c->pnz_cap, 1));
  // dot-product scratch: the outer basis, the inner GMRES of either preconditioner and
  // the DIIS histories all call mdot with at most this many vectors
  const int mk = std::max(std::max(c->restart, c->inner_iters), std::max(c->pkrylov, c->diis_max)) + 2;
  c->mk = mk;
  c->d_part = cv.take<double>((size_t)mk * c->nb_dot);
  c->d_hv = cv.take<double>(mk);
  c->d_scal = cv.take<double>(16);
  c->d_fnb = cv.take<double>(3 * std::max<size_t>(nnz, 1));
  c->d_fself = cv.take<double>(3 * M);
  c->d_fpt = cv.take<double>(3 * MN);
  c->d_fpts = cv.take<double>(3 * M);
  c->d_flsrc = cv.take<double>(3 * M);
  c->d_fysrc = cv.take<double>(3 * M);
  c->d_gphi = cv.take<double>(3 * MN);
  c->d_F = cv.take<double>(3 * M);
  if (c->fmm_order > 0) {
    const size_t nn = c->tree.nnodes, p1 = c->fmm_order + 1, P = p1 * p1;
    c->m2l_cap = std::max(c->m2l_cap, c->tree.m2l_src.size());
    c->near_cap = std::max(c->near_cap, c->tree.near_idx.size());
    c->d_fcen = cv.take<double>(3 * nn);
    c->d_frad = cv.take<double>(nn);
    c->d_fkR = cv.take<double>(nn * p1);
    c->d_fkRi = cv.take<double>(nn * p1);
    c->d_fiR = cv.take<double>(nn * p1);
    c->d_fchild = cv.take<int>(2 * nn);
    c->d_fparent = cv.take<int>(nn);
    c->d_flevn = cv.take<int>(nn);
    c->d_sleaf = cv.take<int>(M);
    c->d_fm2lp = cv.take<int>(nn + 1);
    c->d_fm2ls = cv.take<int>(std::max<size_t>(c->m2l_cap, 1));
    c->d_fnp = cv.take<int>(M + 1);
    c->d_fni = cv.take<int>(std::max<size_t>(c->near_cap, 1));
    c->d_fA = cv.take<double>(std::max<size_t>(c->tables.Ap.size(), 1));
    c->d_fAoff = cv.take<int>(p1 * p1 * p1);
    c->d_fAL = cv.take<double>(3 * p1 * p1 * p1);
    c->d_fJ = cv.take<double>(std::max<size_t>(c->tables.J.size(), 1));
    c->d_fJoff = cv.take<int>(p1 + 1);
    c->d_fjval = cv.take<double>(std::max<size_t>(c->tables.Jval.size(), 1));
    c->d_fjrow = cv.take<int>(std::max<size_t>(c->tables.Jrow.size(), 1));
    c->d_fjpad = cv.take<double>(std::max<size_t>(c->tables.Jpad.size(), 1));
    for (int k = 0; k < 2; ++k) {
      for (int d = 0; d < 2; ++d) c->d_fZ[k][d] = cv.take<double>(std::max<size_t>(c->tables.Z[k][d].size(), 1));
      c->d_fZslot[k] = cv.take<int>(std::max<size_t>(c->tables.Zslot[k].size(), 1));
    }
    for (int d = 0; d < 2; ++d) c->d_fZl[d] = cv.take<double>(std::max<size_t>(c->tables.Zlvl[d].size(), 1));
    c->d_fm2lord = cv.take<int>(nn);
    c->d_fctr = cv.take<int>(64);
    c->d_Mn = cv.take<double>(nn * P);
    c->d_Ln = cv.take<double>(nn * P);
    c->d_SL = cv.take<double>(M * P);
    c->d_Lam = cv.take<double>(M * P);
    c->d_sgp = cv.take<double>(M * (p1 + 1));
    c->d_qsrc = cv.take<double>(M);
    c->d_tmp4 = cv.take<double>(4 * M);
  }
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

#define P_DISPATCH(PV, BODY)                        \
  switch (PV) {                                     \
    case 2: { constexpr int PDc = 2; BODY; } break;   \
    case 3: { constexpr int PDc = 3; BODY; } break;   \
    case 4: { constexpr int PDc = 4; BODY; } break;   \
    case 5: { constexpr int PDc = 5; BODY; } break;   \
    case 6: { constexpr int PDc = 6; BODY; } break;   \
    case 7: { constexpr int PDc = 7; BODY; } break;   \
    case 8: { constexpr int PDc = 8; BODY; } break;   \
    case 9: { constexpr int PDc = 9; BODY; } break;   \
    case 10: { constexpr int PDc = 10; BODY; } break; \
    case 11: { constexpr int PDc = 11; BODY; } break; \
    case 12: { constexpr int PDc = 12; BODY; } break; \
    case 13: { constexpr int PDc = 13; BODY; } break; \
    case 14: { constexpr int PDc = 14; BODY; } break; \
    case 15: { constexpr int PDc = 15; BODY; } break; \
    case 16: { constexpr int PDc = 16; BODY; } break; \
    default: throw HipError{hipErrorInvalidValue};    \
  }

inline unsigned nblk(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Per-kernel device time: events recorded on the context's stream around a launch.
struct KScope {
  ddlpb_ctx* c;
  int idx = -1;
  hipEvent_t e0{}, e1{};
  KScope(ddlpb_ctx* c_, const char* name, double work) : c(c_) {
    if (!c->ktiming) return;
    for (size_t k = 0; k < c->ktimers.size(); ++k)
      if (c->ktimers[k].name == name) idx = (int)k;
    if (idx < 0) { c->ktimers.push_back({name}); idx = (int)c->ktimers.size() - 1; }
    c->ktimers[idx].work += work;
    c->ktimers[idx].launches += 1;
    e0 = take(); e1 = take();
    HIPCHK(hipEventRecord(e0, c->stream));
  }
  hipEvent_t take() {
    if (c->ev_pool.empty()) { hipEvent_t e; HIPCHK(hipEventCreate(&e)); return e; }
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  ~KScope() noexcept(false) {
    if (idx < 0) return;
    HIPCHK(hipEventRecord(e1, c->stream));
    c->ev_pending.push_back({idx, {e0, e1}});
  }
};
void ktimer_flush(ddlpb_ctx* c) {
  if (c->ev_pending.empty()) return;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (auto& p : c->ev_pending) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
    c->ktimers[p.first].ms += ms;
    c->ev_pool.push_back(p.second.first);
    c->ev_pool.push_back(p.second.second);
  }
  c->ev_pending.clear();
}
// algorithmic flops of one (point, sphere) single-layer interaction at degree lm:
// 2L for the contraction with the coefficients, ~3L for the harmonic recurrence,
// 3 per degree for the Bessel weights, ~25 for distance, exp and the first two weights
inline double flops_sl_pair(int lm) { double L = (lm + 1.0) * (lm + 1.0); return 5.0 * L + 3.0 * (lm + 1) + 25.0; }
// one neighbour-cap interaction of the A/B operators: harmonic recurrence, two contractions,
// the i_l weights (two series of nterms terms and the downward recurrence)
inline double flops_cap_pair(int lm, int nterms) { double L = (lm + 1.0) * (lm + 1.0); return 7.0 * L + 6.0 * nterms + 8.0 * (lm + 1) + 30.0; }

// out (R x C, ldo) = A (R x K, lda) B (K x C, ldb) + c0 base (base null: no term), FP64
// matrix cores: k_gemm_f64_kc for a deep contraction into few columns (depth chunked),
// else k_gemm_f64 with 16 S rows of A per block in LDS, S = 4, 2 or 1, the largest whose
// chunk fits 80 KB (two blocks per compute unit)
void gemm_f64(ddlpb_ctx* c, int R, int C, int K, const double* A, int lda, const double* B, int ldb,
              const double* base, double c0, double* out, int ldo) {
  if (R <= 0 || C <= 0) return;
  if (C <= 16 * kGemmWaves && K > 128) {
    // deep contraction into at most eight column tiles (the projection An): depth in
    // chunks of 52, four strips per block (27 KB of LDS)
    constexpr int S = 4, KC = 52;
    const size_t lds = (size_t)16 * S * (KC + 1) * sizeof(double);
    const dim3 grid((unsigned)((R + 16 * S - 1) / (16 * S))), block(64 * ((C + 15) / 16));
    hipLaunchKernelGGL(k_gemm_f64_kc<S>, grid, block, lds, c->stream, R, C, K, KC, A, lda, B, ldb, base, c0, out,
                       ldo);
    HIPCHK(hipGetLastError());
    return;
  }
  int S = 4;
  while (S > 1 && gemm_f64_lds(S, K) > 80 * 1024) S /= 2;
  const size_t lds = gemm_f64_lds(S, K);
  if (lds > 160 * 1024) throw HipError{hipErrorInvalidValue};
  const int nw = std::min(kGemmWaves, (C + 15) / 16);
  const dim3 grid((unsigned)((R + 16 * S - 1) / (16 * S))), block(64 * nw);
  auto go = [&](auto kern) {
    if (lds > 65536)
      HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
    hipLaunchKernelGGL(kern, grid, block, lds, c->stream, R, C, K, A, lda, B, ldb, base, c0, out, ldo);
  };
  if (S == 4) go(k_gemm_f64<4>);
  else if (S == 2) go(k_gemm_f64<2>);
  else go(k_gemm_f64<1>);
  HIPCHK(hipGetLastError());
}
void fill(ddlpb_ctx* c, double* p, long n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, c->stream, n, v, p);
  HIPCHK(hipGetLastError());
}

void gemm_f64(ddlpb_ctx* c, int R, int C, int K, const double* A, int lda, const double* B, int ldb,
              const double* base, double c0, double* out, int ldo);
// mu2 = An(U (.) Syn(mu1)) for every sphere: two matrix-core products through the
// point-value scratch d_Vpt (free between the operator stages that use it)
void syn_u_an(ddlpb_ctx* c) {
  const long MN = (long)c->M * c->N;
  gemm_f64(c, c->M, c->N, c->L, c->d_mu1, c->L, c->d_YT, c->N, nullptr, 0.0, c->d_Vpt, c->N);
  hipLaunchKernelGGL(k_mul_grid, dim3(nblk(MN, 256)), dim3(256), 0, c->stream, MN, c->d_U, c->d_Vpt);
  HIPCHK(hipGetLastError());
  gemm_f64(c, c->M, c->L, c->N, c->d_Vpt, c->N, c->d_WY, c->L, nullptr, 0.0, c->d_mu2, c->L);
}
// m = C (.) An(U (.) (e + Syn(y(X))))
void moments(ddlpb_ctx* c, const double* X, const double* egrid, double* h_out, double* m_out) {
  if (X && !egrid && !h_out) {
    // y(X) per degree, then the two products, then the C_l scaling
    const long ML = (long)c->M * c->L;
    hipLaunchKernelGGL(k_deg_scale, dim3(nblk(ML, 256)), dim3(256), 0, c->stream, c->M, c->L, c->LUR, c->d_ycr, X,
                       c->d_yce, X + ML, c->L, c->d_mu1);
    HIPCHK(hipGetLastError());
    syn_u_an(c);
    hipLaunchKernelGGL(k_deg_scale, dim3(nblk(ML, 256)), dim3(256), 0, c->stream, c->M, c->L, c->LUR, c->d_Cl,
                       c->d_mu2, nullptr, nullptr, c->L, m_out);
    HIPCHK(hipGetLastError());
    return;
  }
  LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_moments<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M, c->N, c->LY,
                                          c->d_Y, c->d_leb, c->d_U, X, c->d_ycr, c->d_yce, c->LUR, egrid, c->d_Cl,
                                          h_out, m_out));
  HIPCHK(hipGetLastError());
}

// Phi (value on the grid, zero on inactive points) or grad Phi' at active points
void sl_field(ddlpb_ctx* c, const double* m, bool grad, int exclude_self, double* out) {
  if (c->nact == 0) return;
  if (!grad) fill(c, out, (long)c->M * c->N, 0.0);
  KScope ks(c, grad ? "sl_field_grad" : "sl_field", (grad ? 4.0 : 1.0) * flops_sl_pair(c->lmax) * (double)c->nact * c->M);
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
  KScope ks(c, "sl_adjoint", flops_sl_pair(lo) * (double)c->nact * c->M);
  LM_DISPATCH(lo, hipLaunchKernelGGL((k_sl_adjoint_direct<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M, c->N,
                                     c->nact, c->d_actsph, c->d_actn, c->d_xyz, c->d_rad, c->d_leb, cgrid, c->d_ur,
                                     c->LUR, c->kappa, exclude_self, lam));
  HIPCHK(hipGetLastError());
}

void an_gemm(ddlpb_ctx* c, const double* base, double c0, double* out);
nearlane::NearArgs near_args(ddlpb_ctx* c);
// near-field A/B kernels over the cap lists in compute type R (float on the mixed path)
template <class R>
void launch_LX_caps(ddlpb_ctx* c, const double* base, double c0, const double* nearX, double c1, const double* gr1,
                    const double* gr2, const double* ge, double cg, double* out) {
  const bool gemm = std::is_same<R, double>::value;  // FP64: An transforms as one GEMM
  LM_DISPATCH(c->lmax, {
    const size_t lds = k_apply_LX_caps_lds_entries<LMc>(c->N) * sizeof(R);
    if (lds > 65536)
      HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_apply_LX_caps<LMc, R>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((k_apply_LX_caps<LMc, R>), dim3(c->M), dim3(256), lds, c->stream, c->M, c->N, c->LY, c->d_Y,
                       c->d_leb, c->d_xyz, c->d_rad, c->d_nptr, c->d_nidx, c->d_cptr, c->d_capn, c->d_capslot,
                       c->d_capw, c->d_pcp, c->d_U, c->d_isgr, c->LUR, c->kappa, c->nterms, base, c0, nearX, c1, gr1,
                       gr2, ge, cg, out, gemm ? c->d_Vpt : nullptr);
  });
  HIPCHK(hipGetLastError());
  if (gemm) an_gemm(c, base, c0, out);
}
// out = c0 base + An(point values in d_Vpt): [2M][L] = Vpt [2M][N] x WY [N][L]
void an_gemm(ddlpb_ctx* c, const double* base, double c0, double* out) {
  gemm_f64(c, 2 * c->M, c->L, c->N, c->d_Vpt, c->N, c->d_WY, c->L, base, c0, out, c->L);
}
template <class R>
void launch_LTZ_caps(ddlpb_ctx* c, const double* base, double c0, const double* zr, const double* ze, double c1,
                     const double* lam, int llam, double* out) {
  LM_DISPATCH(c->lmax, {
    const size_t lds = k_apply_LTZ_caps_lds_entries<LMc>(c->N) * sizeof(R);
    if (lds > 65536)
      HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_apply_LTZ_caps<LMc, R>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((k_apply_LTZ_caps<LMc, R>), dim3(c->M), dim3(128), lds, c->stream, c->M, c->N, c->LY, c->d_Y,
                       c->d_YT, c->d_leb, c->d_xyz, c->d_rad, c->d_rptr, c->d_rci, c->d_rcn, c->d_rcw, c->d_U, c->d_isgr,
                       c->d_ycr, c->d_yce, c->d_Cl, c->LUR, c->kappa, c->nterms, base, c0, zr, ze, c1, lam, llam, out);
  });
  HIPCHK(hipGetLastError());
}

void apply_LX(ddlpb_ctx* c, const double* base, double c0, const double* nearX, double c1, const double* gr1,
              const double* gr2, const double* ge, double cg, double* out) {
  if (c->use_lane) {
    // per-cap values by the sphere that owns the harmonics, per-point sums in forward
    // order, then the An transforms of all spheres as one GEMM
    if (nearX) {
      KScope ks(c, c->cur_prec == 1 ? "near_lx_f32" : "near_lx", flops_cap_pair(c->lmax, c->nterms) * (double)c->ncap);
      HIPCHK(nearlane::launch_lx(c->lmax, c->cur_prec, near_args(c), nearX, c->d_capv, c->stream));
    }
    {
      KScope ks(c, "near_point_sums", 0.0);
      const long MN = (long)c->M * c->N;
      hipLaunchKernelGGL(k_point_sums, dim3(nblk(MN, 256)), dim3(256), 0, c->stream, c->M, c->N, c->d_pcp, c->d_f2r,
                         nearX ? c->d_capv : nullptr, c1, c->d_U, gr1, gr2, ge, cg, c->d_Vpt);
      HIPCHK(hipGetLastError());
    }
    KScope ks(c, "an_gemm", 2.0 * c->N * c->L * 2.0 * c->M);
    an_gemm(c, base, c0, out);
    return;
  }
  KScope ks(c, "apply_LX", nearX ? flops_cap_pair(c->lmax, c->nterms) * (double)c->ncap : 0.0);
  if (c->use_caps) {
    if (c->cur_prec == 1) launch_LX_caps<float>(c, base, c0, nearX, c1, gr1, gr2, ge, cg, out);
    else launch_LX_caps<double>(c, base, c0, nearX, c1, gr1, gr2, ge, cg, out);
    return;
  }
  LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_apply_LX<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M, c->N, c->LY,
                                          c->d_Y, c->d_leb, c->d_xyz, c->d_rad, c->d_nptr, c->d_nidx, c->d_f, c->d_U,
                                          c->d_sgr, c->LUR, c->kappa, c->eta, c->nterms, base, c0, nearX, c1, gr1,
                                          gr2, ge, cg, out));
  HIPCHK(hipGetLastError());
}

void syn2(ddlpb_ctx* c, const double* Z, int mode, double* o1, double* o2) {
  if (mode == 0 && o1 == c->d_zr && o2 == c->d_ze) {
    // Syn of every sphere at once: [2M][N] = Z [2M][L] x Y^T, with Y^T = YT [LY][N]
    KScope ks(c, "syn_gemm", 2.0 * c->N * c->L * 2.0 * c->M);
    gemm_f64(c, 2 * c->M, c->N, c->L, Z, c->L, c->d_YT, c->N, nullptr, 0.0, c->d_zr, c->N);
    return;
  }
  const int nt = std::min(512, (c->N + 63) / 64 * 64);
  LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_syn2<LMc>), dim3(c->M), dim3(nt), 0, c->stream, c->M, c->N, c->LY,
                                          c->d_YT, c->d_leb, c->d_U, Z, mode, o1, o2));
  HIPCHK(hipGetLastError());
}

void apply_LTZ(ddlpb_ctx* c, const double* base, double c0, const double* zr, const double* ze, double c1,
               const double* lam, int llam, double* out) {
  if (c->use_lane) {
    {
      KScope ks(c, c->cur_prec == 1 ? "near_ltz_f32" : "near_ltz",
                zr ? flops_cap_pair(c->lmax, c->nterms) * (double)c->ncap : 0.0);
      HIPCHK(nearlane::launch_ltz(c->lmax, c->cur_prec, near_args(c), base, c0, zr, ze, c1, out, c->stream));
    }
    if (lam) {
      KScope ks(c, "sl_adjoint_part", 4.0 * c->N * c->L * (double)c->M);
      // mu = An(U Syn(C_l lam)) by the two matrix-core products, then out += (ycr, yce) mu
      const long ML = (long)c->M * c->L;
      hipLaunchKernelGGL(k_deg_scale, dim3(nblk(ML, 256)), dim3(256), 0, c->stream, c->M, c->L, c->LUR, c->d_Cl, lam,
                         nullptr, nullptr, llam, c->d_mu1);
      HIPCHK(hipGetLastError());
      syn_u_an(c);
      hipLaunchKernelGGL(k_lam_out, dim3(nblk(ML, 256)), dim3(256), 0, c->stream, c->M, c->L, c->LUR, c->d_ycr,
                         c->d_yce, c->d_mu2, out);
      HIPCHK(hipGetLastError());
    }
    return;
  }
  KScope ks(c, "apply_LTZ", zr ? flops_cap_pair(c->lmax, c->nterms) * (double)c->ncap : 0.0);
  if (c->use_caps) {
    if (c->cur_prec == 1) launch_LTZ_caps<float>(c, base, c0, zr, ze, c1, lam, llam, out);
    else launch_LTZ_caps<double>(c, base, c0, zr, ze, c1, lam, llam, out);
    return;
  }
  LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_apply_LTZ<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M, c->N, c->LY,
                                          c->d_Y, c->d_leb, c->d_xyz, c->d_rad, c->d_nptr, c->d_nidx, c->d_f, c->d_U,
                                          c->d_sgr, c->d_ycr, c->d_yce, c->d_Cl, c->LUR, c->kappa, c->eta, c->nterms,
                                          base, c0, zr, ze, c1, lam, llam, out));
  HIPCHK(hipGetLastError());
}

void sl_field_list(ddlpb_ctx* c, const int* lptr, const int* lidx, const double* m, bool grad, int exclude_self,
                   int accumulate, double* out) {
  if (c->nact == 0) return;
  KScope ks(c, grad ? "sl_near_grad" : "sl_near", (grad ? 4.0 : 1.0) * flops_sl_pair(c->lmax) * c->near_pairs_pts);
  if (grad) {
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_sl_field_list<LMc, true>), dim3(nblk(c->nact, 256)), dim3(256), 0,
                                            c->stream, c->M, c->N, c->nact, c->d_actsph, c->d_actn, c->d_xyz,
                                            c->d_rad, c->d_leb, lptr, lidx, m, c->d_iur, c->LUR, c->kappa,
                                            exclude_self, accumulate, out));
  } else {
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_sl_field_list<LMc, false>), dim3(nblk(c->nact, 256)), dim3(256), 0,
                                            c->stream, c->M, c->N, c->nact, c->d_actsph, c->d_actn, c->d_xyz,
                                            c->d_rad, c->d_leb, lptr, lidx, m, c->d_iur, c->LUR, c->kappa,
                                            exclude_self, accumulate, out));
  }
  HIPCHK(hipGetLastError());
}
// active points with this call's grid charges, packed for k_sl_adjoint_list
const double4* pack_points(ddlpb_ctx* c, const double* cgrid) {
  double4* pt = reinterpret_cast<double4*>(c->d_pt4);
  if (c->nact > 0) {
    hipLaunchKernelGGL(k_pack_points, dim3(nblk(c->nact, 256)), dim3(256), 0, c->stream, c->nact, c->N, c->d_actsph,
                       c->d_actn, c->d_xyz, c->d_rad, c->d_leb, cgrid, pt);
    HIPCHK(hipGetLastError());
  }
  return pt;
}
void sl_adjoint_list(ddlpb_ctx* c, const int* lptr, const int* lidx, const double* cgrid, int lo, int exclude_self,
                     int accumulate, int ldl, double* lam) {
  KScope ks(c, "sl_near_adjoint", flops_sl_pair(lo) * c->near_pairs_pts);
  const double4* pt = pack_points(c, cgrid);
  LM_DISPATCH(lo, hipLaunchKernelGGL((k_sl_adjoint_list<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M, c->d_actptr,
                                     pt, c->d_xyz, c->d_rad, lptr, lidx, c->d_iur, c->LUR, c->kappa, exclude_self,
                                     accumulate, ldl, lam));
  HIPCHK(hipGetLastError());
}

// ---- fast multipole passes
FmmDev fmm_dev(ddlpb_ctx* c, int kernel) {
  FmmDev f;
  f.kernel = kernel;
  f.p = c->fmm_order;
  f.kappa = c->kappa;
  f.A = c->d_fA; f.Aoff = c->d_fAoff; f.nA = (int)c->tables.Ap.size();
  f.AL = c->d_fAL; f.J = c->d_fJ; f.Joff = c->d_fJoff;
  f.jval = c->d_fjval; f.jrow = c->d_fjrow; f.njval = (int)c->tables.Jval.size();
  f.center = c->d_fcen; f.radius = c->d_frad; f.kR = c->d_fkR; f.kRi = c->d_fkRi; f.iR = c->d_fiR;
  f.kinv = c->kappa > 0 ? 1.0 / c->kappa : 0.0;
  return f;
}
// flops of one translation at order p: four rotations by J, the z-translation sum
inline double flops_translation(int p) {
  double rot = 0.0, oz = 0.0;
  for (int l = 0; l <= p; ++l) rot += (2.0 * l + 1.0) * (2.0 * l + 1.0);
  for (int l = 0; l <= p; ++l)
    for (int lp = 0; lp <= p; ++lp)
      for (int m = -std::min(l, lp); m <= std::min(l, lp); ++m) oz += 2.0 * (std::min(l, lp) - std::abs(m) + 1) + 4.0;
  return 8.0 * rot + oz;
}
// flops of one multipole-to-local translation as k_fmm_m2l_fast performs it: four sparse
// rotations by J, four z-rotations, the degree scalings of input and output and the z
// translation per (l_out, |m|, l_in)
inline double flops_m2l_fast(int kernel, int p, size_t njval) {
  double oz = 0.0;
  for (int lo = 0; lo <= p; ++lo)
    for (int am = 0; am <= lo; ++am)
      for (int li = am; li <= p; ++li) {
        const int nk = std::min(lo, li) - am + 1;
        oz += (kernel == 0 ? 2.0 * nk : 0.0) + (am ? 4.0 : 2.0);
      }
  const double P = (p + 1.0) * (p + 1.0);
  return 2.0 * 2.0 * (double)njval + 4.0 * 6.0 * p * (p + 1) / 2.0 + 2.0 * P + oz;
}
template <int NI, bool YUK>
const void* m2l_fast_fn(bool alds) {
  return alds ? reinterpret_cast<const void*>(&k_fmm_m2l_fast<NI, true, YUK>)
              : reinterpret_cast<const void*>(&k_fmm_m2l_fast<NI, false, YUK>);
}
template <int NI>
const void* m2l_fast_fn(int kernel, bool alds) {
  return kernel == 0 ? m2l_fast_fn<NI, true>(alds) : m2l_fast_fn<NI, false>(alds);
}
const void* m2l_fast_fn(int NI, int kernel, bool alds) {
  switch (NI) {
    case 1: return m2l_fast_fn<1>(kernel, alds);
    case 2: return m2l_fast_fn<2>(kernel, alds);
    case 3: return m2l_fast_fn<3>(kernel, alds);
    case 4: return m2l_fast_fn<4>(kernel, alds);
    default: return m2l_fast_fn<5>(kernel, alds);
  }
}
// Block layout of k_fmm_m2l_fast: the most resident wavefronts per compute unit as
// reported by the occupancy calculator (registers and LDS); ties go to the tables in
// LDS, then to larger blocks.  nw = 0: no layout fits.
void m2l_config(ddlpb_ctx* c, int kernel, int& nw, bool& alds, size_t& bytes, int& blocks_per_cu) {
  auto& cc = c->m2l_cfg[kernel];
  if (cc.valid) {
    nw = cc.nw; alds = cc.alds; bytes = cc.bytes; blocks_per_cu = cc.per_cu;
    return;
  }
  int dev = 0, maxlds = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const int p = c->fmm_order, P = (p + 1) * (p + 1), NI = (P + 63) / 64;
  const auto& tb = c->tables;
  const int nZ = (int)tb.Z[kernel][0].size(), nj = (int)tb.Jpad.size();
  nw = 0;
  alds = false;
  bytes = 0;
  blocks_per_cu = 0;
  if (NI > 5 || c->m2l_waves < 0 || !tb.jpad_ok) return;
  int best = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const bool a = pass == 0;
    const void* fn = m2l_fast_fn(NI, kernel, a);
    hipFuncAttributes fa;
    HIPCHK(hipFuncGetAttributes(&fa, fn));
    for (int w : {16, 8, 4, 2, 1}) {
      if (c->m2l_waves > 0 && w != c->m2l_waves) continue;
      if (64 * w > fa.maxThreadsPerBlock) continue;  // beyond the kernel's launch bound
      const size_t b = m2l_fast_lds_bytes(p, nZ, nj, tb.nslot, w, a);
      if (b > (size_t)maxlds) continue;
      if (b > 65536) HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b));
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64 * w, b) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      const int waves = w * nb;
      if (waves > best) { best = waves; nw = w; alds = a; bytes = b; blocks_per_cu = nb; }
    }
  }
  cc.valid = true; cc.nw = nw; cc.alds = alds; cc.bytes = bytes; cc.per_cu = blocks_per_cu;
}
template <int NI>
void launch_m2l_fast(ddlpb_ctx* c, const FmmDev& f, const M2LTab& zt, int nw, bool alds, size_t bytes, int blocks,
                     const int* lptr, const int* lidx, int transposed, const double* in, double* out) {
  const void* fn = m2l_fast_fn(NI, f.kernel, alds);
  void* args[] = {(void*)&f, (void*)&zt, (void*)&c->tree.nnodes, (void*)&lptr, (void*)&lidx, (void*)&transposed,
                  (void*)&in, (void*)&out};
  HIPCHK(hipLaunchKernel(fn, dim3(blocks), dim3(64 * nw), args, bytes, c->stream));
}
__global__ void k_zero_ints(int* p, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) p[t] = 0;
}

// Tables of the order-12 lane kernels, per device: J and J^T in the pattern order of
// fmm_lane_api.hpp, uploaded once into each instance's constant arrays after checking
// that every nonzero of the numerical J lies inside the pattern.  State per device:
// 1 ready, -1 unusable (pattern mismatch).
std::mutex g_lane_mu;
std::map<int, int> g_lane_state;
int lane_tables_ready(const fmm::Tables& tb) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_lane_mu);
  auto it = g_lane_state.find(dev);
  if (it != g_lane_state.end()) return it->second;
  int state = 1;
  if (tb.pmax != lane12::kP) state = -1;
  std::vector<double> J, JT;
  for (int l = 0; state > 0 && l <= lane12::kP; ++l) {
    const int w = 2 * l + 1;
    auto val = [&](int a, int b) { return tb.J[tb.Joff[l] + a * w + b]; };
    for (int a = 0; a < w; ++a)
      for (int b = 0; b < w; ++b) {
        if (lane12::pat(false, l, a, b)) J.push_back(val(a, b));
        else if (val(a, b) != 0.0) state = -1;
        if (lane12::pat(true, l, a, b)) JT.push_back(val(b, a));
      }
  }
  if (state > 0 && ((int)J.size() != lane12::kJn || (int)JT.size() != lane12::kJTn)) state = -1;
  if (state > 0) {
    HIPCHK(lane12::upload_yf(J.data(), JT.data()));
    HIPCHK(lane12::upload_yt(J.data(), JT.data()));
    HIPCHK(lane12::upload_lf(J.data(), JT.data()));
    HIPCHK(lane12::upload_lt(J.data(), JT.data()));
    HIPCHK(lane12::upload_yf32(J.data(), JT.data()));
    HIPCHK(lane12::upload_yt32(J.data(), JT.data()));
    HIPCHK(lane12::upload_ym2m(J.data(), JT.data()));
    HIPCHK(lane12::upload_yl2l(J.data(), JT.data()));
    HIPCHK(lane12::upload_ym2mT(J.data(), JT.data()));
    HIPCHK(lane12::upload_yl2lT(J.data(), JT.data()));
    HIPCHK(lane12::upload_ym2m32(J.data(), JT.data()));
    HIPCHK(lane12::upload_yl2l32(J.data(), JT.data()));
    HIPCHK(lane12::upload_ym2mT32(J.data(), JT.data()));
    HIPCHK(lane12::upload_yl2lT32(J.data(), JT.data()));
  }
  g_lane_state[dev] = state;
  return state;
}
// launch of the lane kernel of the pass; false when it does not apply
bool launch_m2l_lane(ddlpb_ctx* c, const FmmDev& f, const int* lptr, const int* lidx, int transposed, const double* in,
                     double* out) {
  if (f.p != lane12::kP || !c->m2l_lane || c->m2l_waves != 0) return false;
  if (lane_tables_ready(c->tables) < 0) return false;
  // 4, 5: the FP32-vector screened Coulomb instances (mixed outer iterations)
  const int which = (c->m2l32 && f.kernel == 0) ? 4 + (transposed ? 1 : 0)
                                                : (f.kernel == 0 ? 0 : 2) + (transposed ? 1 : 0);
  int per_cu = 0, dev = 0, ncu = 0;
  hipError_t (*occ[6])(int*) = {lane12::occupancy_yf, lane12::occupancy_yt, lane12::occupancy_lf,
                                lane12::occupancy_lt, lane12::occupancy_yf32, lane12::occupancy_yt32};
  HIPCHK(occ[which](&per_cu));
  if (per_cu < 1) return false;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int groups = (c->tree.nnodes + 64 / lane12::kGroup - 1) / (64 / lane12::kGroup);
  const int blocks = std::max(1, std::min(ncu * per_cu, (groups + lane12::kLaneWaves - 1) / lane12::kLaneWaves));
  lane12::LaneTab t;
  t.Z = c->d_fZ[f.kernel][transposed ? 1 : 0];
  t.order = c->d_fm2lord;
  t.counter = c->d_fctr;
  c->m2l_layout = 100 + which;
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, c->stream, c->d_fctr, 1);
  HIPCHK(hipGetLastError());
  hipError_t (*fn[6])(const FmmDev&, const lane12::LaneTab&, int, const int*, const int*, const double*, double*, int,
                      hipStream_t) = {lane12::launch_yf,   lane12::launch_yt,   lane12::launch_lf,
                                      lane12::launch_lt,   lane12::launch_yf32, lane12::launch_yt32};
  HIPCHK(fn[which](f, t, c->tree.nnodes, lptr, lidx, in, out, blocks, c->stream));
  return true;
}
void launch_m2l(ddlpb_ctx* c, const FmmDev& f, const int* lptr, const int* lidx, int transposed, const double* in,
                double* out) {
  const auto& t = c->tree;
  const auto& tb = c->tables;
  const bool f32 = c->m2l32 && f.kernel == 0 && f.p == lane12::kP && c->m2l_lane && c->m2l_waves == 0;
  KScope ks(c, f.kernel == 0 ? (transposed ? (f32 ? "m2l_yukawa_T_f32" : "m2l_yukawa_T") : (f32 ? "m2l_yukawa_f32" : "m2l_yukawa"))
                             : (transposed ? "m2l_laplace_T" : "m2l_laplace"),
            flops_m2l_fast(f.kernel, f.p, tb.Jval.size()) * (double)t.m2l_src.size());
  if (launch_m2l_lane(c, f, lptr, lidx, transposed, in, out)) return;
  int nw, per_cu;
  bool alds;
  size_t bytes;
  m2l_config(c, f.kernel, nw, alds, bytes, per_cu);
  const int P = (f.p + 1) * (f.p + 1), NI = (P + 63) / 64;
  if (nw > 0) {
    int dev = 0, ncu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    c->m2l_layout = nw * (alds ? 1 : -1);
    const int blocks = std::max(1, std::min((t.nnodes + nw - 1) / nw, ncu * std::max(per_cu, 1)));
    M2LTab zt;
    zt.Z = c->d_fZ[f.kernel][transposed ? 1 : 0];
    zt.slot = c->d_fZslot[f.kernel];
    zt.order = c->d_fm2lord;
    zt.counter = c->d_fctr;
    zt.nZ = (int)tb.Z[f.kernel][0].size();
    zt.nslot = tb.nslot;
    zt.jpad = c->d_fjpad;
    zt.njpad = (int)tb.Jpad.size();
    zt.kpack = tb.jpad_kpack;
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, c->stream, c->d_fctr, 1);
    switch (NI) {
      case 1: launch_m2l_fast<1>(c, f, zt, nw, alds, bytes, blocks, lptr, lidx, transposed, in, out); break;
      case 2: launch_m2l_fast<2>(c, f, zt, nw, alds, bytes, blocks, lptr, lidx, transposed, in, out); break;
      case 3: launch_m2l_fast<3>(c, f, zt, nw, alds, bytes, blocks, lptr, lidx, transposed, in, out); break;
      case 4: launch_m2l_fast<4>(c, f, zt, nw, alds, bytes, blocks, lptr, lidx, transposed, in, out); break;
      default: launch_m2l_fast<5>(c, f, zt, nw, alds, bytes, blocks, lptr, lidx, transposed, in, out); break;
    }
  } else {
    hipLaunchKernelGGL(k_fmm_m2l, dim3(std::min(t.nnodes, 8192)), dim3(64), 0, c->stream, f, t.nnodes, lptr, lidx,
                       transposed, in, out);
  }
  HIPCHK(hipGetLastError());
}
// blocks of a level pass: one wavefront per node, at most 8 blocks per compute unit
inline int level_blocks(int cnt) { return std::max(1, std::min((cnt + kLevelWaves - 1) / kLevelWaves, 2048)); }
// LDS layout of the level passes: the coefficient table is staged when table and
// scratch fit in 150 KB; the kernels are allowed the dynamic size they need
void level_lds(ddlpb_ctx* c, const FmmDev& f, int& stage, size_t& bytes) {
  stage = level_lds_bytes(f.kernel, f.p, f.nA, 1) <= 150 * 1024 ? 1 : 0;
  bytes = level_lds_bytes(f.kernel, f.p, f.nA, stage);
  if (bytes > 65536) {
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fmm_upward), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes));
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fmm_downward),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fmm_upward_T),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  }
  (void)c;
}
// One level pass: which 0 M2M (upward), 1 L2L (downward), 2 transposed M2M (downward),
// 3 transposed L2L (upward).  Order 12 with the screened Coulomb kernel takes the
// one-node-per-lane kernels on levels of at least level_lane nodes; otherwise the
// wavefront-per-node kernels run.
void run_level(ddlpb_ctx* c, const FmmDev& f, int which, int lev, int stage, size_t lb, double* E) {
  const auto& t = c->tree;
  const int cnt = t.level_ptr[lev + 1] - t.level_ptr[lev];
  const bool up = which == 0 || which == 3;
  // translations: one per child of the level's nodes (upward), one per node (downward)
  const double ntr = up ? (double)(t.level_ptr[lev + 2] - t.level_ptr[lev + 1]) : (double)cnt;
  const int* nodes = c->d_flevn + t.level_ptr[lev];
  if (f.kernel == 0 && f.p == lane12::kP && c->level_lane > 0 && cnt >= c->level_lane &&
      (int)c->tables.Zlvl[0].size() == lane12::kZYn && lane_tables_ready(c->tables) > 0) {
    const bool f32 = c->m2l32 && c->mixed_lvl;
    KScope ks(c, f32 ? "level_lane_f32" : "level_lane", flops_translation(f.p) * ntr);
    hipError_t (*fn[8])(const FmmDev&, const double*, int, const int*, const int*, const int*, double*,
                        hipStream_t) = {lane12::launch_ym2m,   lane12::launch_yl2l,   lane12::launch_ym2mT,
                                        lane12::launch_yl2lT,  lane12::launch_ym2m32, lane12::launch_yl2l32,
                                        lane12::launch_ym2mT32, lane12::launch_yl2lT32};
    // 4..7: the FP32-vector instances (outer iterations of the mixed path)
    HIPCHK(fn[which + (f32 ? 4 : 0)](f, c->d_fZl[which >= 2 ? 1 : 0], cnt, nodes, c->d_fchild, c->d_fparent,
                                          E, c->stream));
    return;
  }
  KScope ks(c, "level_generic", flops_translation(f.p) * ntr);
  if (which == 0)
    hipLaunchKernelGGL(k_fmm_upward, dim3(level_blocks(cnt)), dim3(64 * kLevelWaves), lb, c->stream, f, nodes, cnt,
                       c->d_fchild, stage, E);
  else if (which == 3)
    hipLaunchKernelGGL(k_fmm_upward_T, dim3(level_blocks(cnt)), dim3(64 * kLevelWaves), lb, c->stream, f, nodes, cnt,
                       c->d_fchild, stage, E);
  else
    hipLaunchKernelGGL(k_fmm_downward, dim3(level_blocks(cnt)), dim3(64 * kLevelWaves), lb, c->stream, f, nodes, cnt,
                       c->d_fparent, which == 2 ? 1 : 0, stage, E);
  HIPCHK(hipGetLastError());
}
// sphere locals SL [M][P] of the far field of per-sphere sources src (degree ps, stride lds)
void fmm_forward(ddlpb_ctx* c, int kernel, const double* src, int ps, int lds, double* SL) {
  const auto& t = c->tree;
  const int p = c->fmm_order, P = (p + 1) * (p + 1);
  FmmDev f = fmm_dev(c, kernel);
  int stage = 0;
  size_t lb = 0;
  level_lds(c, f, stage, lb);
  KScope ks(c, kernel == 0 ? "pass_fmm_yukawa" : "pass_fmm_laplace",
            flops_translation(p) * (double)(t.m2l_src.size() + 2.0 * (t.nnodes - 1)));
  hipLaunchKernelGGL(k_fmm_leaf_set, dim3(c->M), dim3(64), 0, c->stream, c->M, p, ps, lds, c->d_sleaf, src, c->d_Mn);
  for (int lev = t.nlevels - 2; lev >= 0; --lev) run_level(c, f, 0, lev, stage, lb, c->d_Mn);
  launch_m2l(c, f, c->d_fm2lp, c->d_fm2ls, 0, c->d_Mn, c->d_Ln);
  for (int lev = 1; lev < t.nlevels; ++lev) run_level(c, f, 1, lev, stage, lb, c->d_Ln);
  hipLaunchKernelGGL(k_fmm_leaf_get, dim3(c->M), dim3(64), 0, c->stream, c->M, p, p, P, c->d_sleaf, c->d_Ln, 0, SL);
  HIPCHK(hipGetLastError());
}
// transpose of fmm_forward: per-sphere dual sources (degree pd, stride ldd) from the dual sphere locals Lam [M][P]
void fmm_transpose(ddlpb_ctx* c, int kernel, const double* Lam, int pd, int ldd, int accumulate, double* out) {
  const auto& t = c->tree;
  const int p = c->fmm_order, P = (p + 1) * (p + 1);
  FmmDev f = fmm_dev(c, kernel);
  int stage = 0;
  size_t lb = 0;
  level_lds(c, f, stage, lb);
  KScope ks(c, kernel == 0 ? "pass_fmm_yukawa_T" : "pass_fmm_laplace_T",
            flops_translation(p) * (double)(t.m2l_src.size() + 2.0 * (t.nnodes - 1)));
  fill(c, c->d_Ln, (long)t.nnodes * P, 0.0);
  hipLaunchKernelGGL(k_fmm_leaf_set, dim3(c->M), dim3(64), 0, c->stream, c->M, p, p, P, c->d_sleaf, Lam, c->d_Ln);
  for (int lev = t.nlevels - 2; lev >= 0; --lev) run_level(c, f, 3, lev, stage, lb, c->d_Ln);
  launch_m2l(c, f, c->d_fm2lp, c->d_fm2ls, 1, c->d_Ln, c->d_Mn);  // symmetric lists: by source
  for (int lev = 1; lev < t.nlevels; ++lev) run_level(c, f, 2, lev, stage, lb, c->d_Mn);
  hipLaunchKernelGGL(k_fmm_leaf_get, dim3(c->M), dim3(64), 0, c->stream, c->M, p, pd, ldd, c->d_sleaf, c->d_Mn,
                     accumulate, out);
  HIPCHK(hipGetLastError());
}
void l2p(ddlpb_ctx* c, int mode, double c2, double* out1, double* out2) {
  if (c->nact == 0) return;
  const int P = (c->fmm_order + 1) * (c->fmm_order + 1);
  if (mode == 0) {
    // the sphere locals at every grid point, [M][N] = SL [M][P] x YT [P][N], on the matrix
    // cores into the point-value scratch, then added at the active points
    const long MN = (long)c->M * c->N;
    gemm_f64(c, c->M, c->N, P, c->d_SL, P, c->d_YT, c->N, nullptr, 0.0, c->d_Vpt, c->N);
    hipLaunchKernelGGL(k_add_active, dim3(nblk(MN, 256)), dim3(256), 0, c->stream, MN, c->d_U, c->d_Vpt, out1);
    HIPCHK(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL(k_l2p, dim3(nblk(c->nact, 256)), dim3(256), 0, c->stream, c->nact, c->N, P, c->LY, c->d_actsph,
                     c->d_actn, c->d_rad, c->d_YT, c->d_SL, mode, c2, out1, out2);
  HIPCHK(hipGetLastError());
}
void p2l_dual(ddlpb_ctx* c, const double* g1, const double* g2, double* Lam) {
  const int P = (c->fmm_order + 1) * (c->fmm_order + 1);
  if (!g2) {
    // Lam [M][P] = g1 [M][N] x Y [N][P]: a dense product against the harmonic table,
    // on the FP64 matrix cores
    gemm_f64(c, c->M, P, c->N, g1, c->N, c->d_Y, c->LY, nullptr, 0.0, Lam, P);
    return;
  }
  hipLaunchKernelGGL(k_p2l_dual, dim3(c->M), dim3(256), 0, c->stream, c->M, c->N, P, c->LY, c->d_rad, c->d_Y, g1, g2,
                     Lam);
  HIPCHK(hipGetLastError());
}
// Phi[m] on the grid (zero at inactive points): direct, or FMM near list + far field
void sl_field_full(ddlpb_ctx* c, const double* m, double* Phi) {
  if (c->fmm_order == 0) { sl_field(c, m, false, 0, Phi); return; }
  fill(c, Phi, (long)c->M * c->N, 0.0);
  if (c->nact == 0) return;
  if (c->sl32) {
    KScope ks(c, "sl_near_f32", flops_sl_pair(c->lmax) * c->near_pts_fmm);
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_sl_field_list<LMc, false, float>), dim3(nblk(c->nact, 256)),
                                            dim3(256), 0, c->stream, c->M, c->N, c->nact, c->d_actsph, c->d_actn,
                                            c->d_xyz, c->d_rad, c->d_leb, c->d_fnp, c->d_fni, m, c->d_iur, c->LUR,
                                            c->kappa, 0, 1, Phi));
  } else {
    KScope ks(c, "sl_near", flops_sl_pair(c->lmax) * c->near_pts_fmm);
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_sl_field_list<LMc, false>), dim3(nblk(c->nact, 256)), dim3(256), 0,
                                            c->stream, c->M, c->N, c->nact, c->d_actsph, c->d_actn, c->d_xyz,
                                            c->d_rad, c->d_leb, c->d_fnp, c->d_fni, m, c->d_iur, c->LUR, c->kappa, 0, 1,
                                            Phi));
  }
  fmm_forward(c, 0, m, c->lmax, c->L, c->d_SL);
  l2p(c, 0, 0.0, Phi, nullptr);
}
// lambda (degree lo, stride ldl) from grid charges: direct, or FMM near list + far field
void sl_adjoint_full(ddlpb_ctx* c, const double* cgrid, int lo, int exclude_self, int ldl, double* lam) {
  if (c->fmm_order == 0) { sl_adjoint(c, cgrid, lo, exclude_self, lam); return; }
  if (c->sl32) {
    KScope ks(c, "sl_near_adjoint_f32", flops_sl_pair(lo) * c->near_pts_fmm);
    const double4* pt = pack_points(c, cgrid);
    LM_DISPATCH(lo, hipLaunchKernelGGL((k_sl_adjoint_list<LMc, float>), dim3(c->M), dim3(256), 0, c->stream, c->M,
                                       c->d_actptr, pt, c->d_xyz, c->d_rad, c->d_fnp, c->d_fni, c->d_iur, c->LUR,
                                       c->kappa, exclude_self, 0, ldl, lam));
    HIPCHK(hipGetLastError());
  } else {
    KScope ks(c, "sl_near_adjoint", flops_sl_pair(lo) * c->near_pts_fmm);
    const double4* pt = pack_points(c, cgrid);
    LM_DISPATCH(lo, hipLaunchKernelGGL((k_sl_adjoint_list<LMc>), dim3(c->M), dim3(256), 0, c->stream, c->M,
                                       c->d_actptr, pt, c->d_xyz, c->d_rad, c->d_fnp, c->d_fni, c->d_iur, c->LUR,
                                       c->kappa, exclude_self, 0, ldl, lam));
    HIPCHK(hipGetLastError());
  }
  p2l_dual(c, cgrid, nullptr, c->d_Lam);
  fmm_transpose(c, 0, c->d_Lam, lo, ldl, 1, lam);
}

// ---- operators
// y = P x with P = L_AB + the single-layer blocks of near sphere pairs (two-level preconditioner)
void op_P(ddlpb_ctx* c, const double* x, double* y) {
  moments(c, x, nullptr, nullptr, c->d_m);
  fill(c, c->d_Phi, (long)c->M * c->N, 0.0);
  sl_field_list(c, c->d_pptr, c->d_pidx, c->d_m, false, 0, 0, c->d_Phi);
  apply_LX(c, x, 1.0, x, -1.0, c->d_Phi, nullptr, c->d_Phi, 1.0, y);
}
void op_PT(ddlpb_ctx* c, const double* x, double* y) {
  syn2(c, x, 1, c->d_cg, nullptr);
  sl_adjoint_list(c, c->d_pptr, c->d_pidx, c->d_cg, c->lmax, 0, 0, c->L, c->d_lam);
  syn2(c, x, 0, c->d_zr, c->d_ze);
  apply_LTZ(c, x, 1.0, c->d_zr, c->d_ze, -1.0, c->d_lam, c->L, y);
}
// y = L x
void op_L(ddlpb_ctx* c, const double* x, double* y) {
  moments(c, x, nullptr, nullptr, c->d_m);
  sl_field_full(c, c->d_m, c->d_Phi);
  apply_LX(c, x, 1.0, x, -1.0, c->d_Phi, nullptr, c->d_Phi, 1.0, y);
}
// y = L^T x
void op_LT(ddlpb_ctx* c, const double* x, double* y) {
  // one synthesis of x serves both the grid charges of the single layer and the A/B part
  syn2(c, x, 0, c->d_zr, c->d_ze);
  const long MN = (long)c->M * c->N;
  hipLaunchKernelGGL(k_charges_from_syn, dim3(nblk(MN, 256)), dim3(256), 0, c->stream, MN, c->N, c->d_leb, c->d_U,
                     c->d_zr, c->d_ze, c->d_cg);
  HIPCHK(hipGetLastError());
  sl_adjoint_full(c, c->d_cg, c->lmax, 0, c->L, c->d_lam);
  apply_LTZ(c, x, 1.0, c->d_zr, c->d_ze, -1.0, c->d_lam, c->L, y);
}
// z = P^-1 v: k Jacobi sweeps z <- v + (I - L_AB) z from z = v (or the transposed sweeps)
// The sweeps alternate between z and the scratch vector d_t3 so that the last one
// lands in z; the first reads v itself (z = v before it), so no copies are made.
void precond(ddlpb_ctx* c, bool transpose, const double* v, double* z) {
  const long D = 2L * c->M * c->L;
  const int k = c->sweeps;
  if (k == 0) {
    HIPCHK(hipMemcpyAsync(z, v, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return;
  }
  const double* in = v;
  for (int s = 0; s < k; ++s) {
    double* out = ((k - 1 - s) % 2 == 0) ? z : c->d_t3;
    if (!transpose) {
      apply_LX(c, v, 1.0, in, 1.0, nullptr, nullptr, nullptr, 0.0, out);
    } else {
      syn2(c, in, 0, c->d_zr, c->d_ze);
      apply_LTZ(c, v, 1.0, c->d_zr, c->d_ze, 1.0, nullptr, 0, out);
    }
    in = out;
  }
}

// ---- BLAS-1 on the device (deterministic reductions)
void mdot(ddlpb_ctx* c, int nv, const double* V, long ldv, const double* w, double* h_host) {
  const long D = 2L * c->M * c->L;
  if (nv < 1 || nv > c->mk) throw HipError{hipErrorInvalidValue};  // scratch holds mk vectors
  hipLaunchKernelGGL(k_mdot_part, dim3(c->nb_dot, (nv + kDotV - 1) / kDotV), dim3(256), 0, c->stream, D, nv, V, ldv, w,
                     c->d_part);
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
  if (nv < 1 || nv > c->mk) throw HipError{hipErrorInvalidValue};
  HIPCHK(hipMemcpyAsync(c->d_hv, h_host, nv * sizeof(double), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_mupdate, dim3(nblk(D, 256)), dim3(256), 0, c->stream, D, nv, V, ldv, c->d_hv, w);
  HIPCHK(hipGetLastError());
}
void axpby(ddlpb_ctx* c, double a, const double* x, double b, double* y) {
  const long D = 2L * c->M * c->L;
  hipLaunchKernelGGL(k_axpby, dim3(nblk(D, 256)), dim3(256), 0, c->stream, D, a, x, b, y);
  HIPCHK(hipGetLastError());
}

using VecOp = std::function<void(const double*, double*)>;

// Restarted right-preconditioned GMRES with classical Gram-Schmidt and one
// re-orthogonalisation (reorth; the short inner solves of the preconditioner may go
// without it).  Flexible (FGMRES) when Z is given: the preconditioned
// directions are stored, so the preconditioner may change between iterations.
// Stops at ||b - A x|| <= tol ||b|| (or after maxit iterations / max_cycles cycles).
int gmres_core(ddlpb_ctx* c, const VecOp& op, const VecOp& prec, const double* b, double* x, double tol, int m,
               int maxit, int max_cycles, bool x_zero, double* V, double* Z, double* tw, double* tz, double* tc,
               int* iters, double* relres, bool reorth = true) {
  const long D = 2L * c->M * c->L;
  const double bn = norm2(c, b);
  *iters = 0;
  *relres = 0.0;
  if (bn == 0.0) { fill(c, x, D, 0.0); return DDLPB_OK; }
  int total = 0, cycles = 0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), h(m + 1), h2(m + 1), y(m);
  double rel = 1.0;
  bool conv = false;
  while (true) {
    if (x_zero && cycles == 0) {
      HIPCHK(hipMemcpyAsync(V, b, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    } else {
      op(x, tw);
      HIPCHK(hipMemcpyAsync(V, b, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      axpby(c, -1.0, tw, 1.0, V);
    }
    const double beta = norm2(c, V);
    const double rel_prev = rel;
    rel = beta / bn;
    if (rel <= tol) { conv = true; break; }
    if (total >= maxit || cycles >= max_cycles) break;
    // stagnation: a whole restart cycle that reduced the residual by less than 10 %
    if (cycles >= 1 && m >= 20 && rel > 0.9 * rel_prev) break;
    axpby(c, 0.0, V, 1.0 / beta, V);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int j = 0;
    for (; j < m && total < maxit; ++j) {
      double* zj = Z ? Z + (long)j * D : tz;
      prec(V + (long)j * D, zj);
      double* w = V + (long)(j + 1) * D;
      op(zj, w);
      mdot(c, j + 1, V, D, w, h.data());
      mupdate(c, j + 1, V, D, h.data(), w);
      if (reorth) {
        mdot(c, j + 1, V, D, w, h2.data());
        mupdate(c, j + 1, V, D, h2.data(), w);
      } else {
        std::fill(h2.begin(), h2.end(), 0.0);
      }
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i] + h2[i];
      const double hn = norm2(c, w);
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0) axpby(c, 0.0, w, 1.0 / hn, w);
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
    if (j > c->mk) throw HipError{hipErrorInvalidValue};
    HIPCHK(hipMemcpyAsync(c->d_hv, y.data(), j * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (Z) {
      hipLaunchKernelGGL(k_mcomb, dim3(nblk(D, 256)), dim3(256), 0, c->stream, D, j, Z, D, c->d_hv, tc);
      HIPCHK(hipGetLastError());
    } else {
      hipLaunchKernelGGL(k_mcomb, dim3(nblk(D, 256)), dim3(256), 0, c->stream, D, j, V, D, c->d_hv, tw);
      HIPCHK(hipGetLastError());
      prec(tw, tc);
    }
    if (x_zero && cycles == 0) HIPCHK(hipMemcpyAsync(x, tc, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    else axpby(c, 1.0, tc, 1.0, x);
    ++cycles;
    if (max_cycles == 1) { rel = std::fabs(gv[j]) / bn; break; }
  }
  *iters = total;
  *relres = rel;
  return conv ? DDLPB_OK : DDLPB_ENOCONV;
}

// Outer solve of L X = b (or L^T X = b).  Two-level preconditioner: a few GMRES
// steps on P = L_AB + near single-layer blocks, themselves preconditioned by
// Jacobi sweeps on L_AB; the outer method is then flexible GMRES.
int gmres(ddlpb_ctx* c, bool transpose, const double* b, double* x, double tol, int* iters, double* relres) {
  VecOp opL = [&](const double* in, double* out) { if (transpose) op_LT(c, in, out); else op_L(c, in, out); };
  VecOp jac = [&](const double* in, double* out) { precond(c, transpose, in, out); };
  if (c->pkrylov > 0 && c->pdelta < 0.0) {
    // Krylov preconditioner: pkrylov GMRES steps on L_AB (each preconditioned by the
    // Jacobi sweeps) in place of the sweeps alone; the outer method is flexible GMRES
    VecOp opAB = [&](const double* in, double* out) {
      if (!transpose) {
        apply_LX(c, in, 1.0, in, -1.0, nullptr, nullptr, nullptr, 0.0, out);
      } else {
        syn2(c, in, 0, c->d_zr, c->d_ze);
        apply_LTZ(c, in, 1.0, c->d_zr, c->d_ze, -1.0, nullptr, 0, out);
      }
    };
    const bool fp32 = c->precision == 1 && c->use_caps;
    VecOp jacp = [&](const double* in, double* out) {
      const int keep = c->cur_prec;
      if (fp32) c->cur_prec = 1;
      precond(c, transpose, in, out);
      c->cur_prec = keep;
    };
    // on the mixed path the whole inner solve (its L_AB products and sweeps) runs the
    // near-field kernels in FP32; its vectors, dots and norms stay FP64
    VecOp inner = [&](const double* in, double* out) {
      int it = 0;
      double rr = 0;
      const int keep = c->cur_prec;
      if (fp32) c->cur_prec = 1;
      (void)gmres_core(c, opAB, jacp, in, out, 1e-30, c->pkrylov, c->pkrylov, 1, true, c->d_Vin, nullptr, c->d_t4,
                       c->d_t1, c->d_t5, &it, &rr, c->inner_reorth);
      c->cur_prec = keep;
      c->inner_total += it;
    };
    if (!fp32 || c->fmm_order == 0 || !(c->mixed_sl || c->mixed_m2l))
      return gmres_core(c, opL, inner, b, x, tol, c->restart, c->maxit, 1 << 30, false, c->d_V, c->d_Z, c->d_w,
                        c->d_t1, c->d_t2, iters, relres);
    // mixed path with the FMM: the outer iterations apply the operator with its near
    // single layer in FP32; then the FP64 operator's residual b - L x decides, and
    // flexible GMRES continues from x on the FP64 operator until it meets tol (the
    // FP64 outer refinement; usually the check alone)
    struct Sl32 {
      ddlpb_ctx* c;
      explicit Sl32(ddlpb_ctx* cc) : c(cc) {
        c->sl32 = c->mixed_sl;
        c->m2l32 = c->mixed_m2l;
      }
      ~Sl32() {
        c->sl32 = false;
        c->m2l32 = false;
      }
    };
    VecOp opLm = [&](const double* in, double* out) {
      Sl32 g(c);
      opL(in, out);
    };
    int it1 = 0;
    double rr1 = 0.0;
    (void)gmres_core(c, opLm, inner, b, x, tol, c->restart, c->maxit, 1 << 30, false, c->d_V, c->d_Z, c->d_w,
                     c->d_t1, c->d_t2, &it1, &rr1);
    int it2 = 0;
    const int rc = gmres_core(c, opL, inner, b, x, tol, c->restart, std::max(0, c->maxit - it1), 1 << 30, false,
                              c->d_V, c->d_Z, c->d_w, c->d_t1, c->d_t2, &it2, relres);
    *iters = it1 + it2;
    c->fp64_iters += it2;
    return rc;
  }
  if (c->precision == 1 && c->use_caps && c->pdelta < 0.0) {
    // FP32 Jacobi sweeps as the preconditioner of flexible GMRES on the FP64 operator:
    // the sweeps are linear only up to single-precision rounding, so the
    // preconditioned directions are stored (FGMRES) and the FP64 residual is minimised
    VecOp jac32 = [&](const double* in, double* out) {
      const int keep = c->cur_prec;
      c->cur_prec = 1;
      precond(c, transpose, in, out);
      c->cur_prec = keep;
    };
    return gmres_core(c, opL, jac32, b, x, tol, c->restart, c->maxit, 1 << 30, false, c->d_V, c->d_Z, c->d_w,
                      c->d_t1, c->d_t2, iters, relres);
  }
  if (c->pdelta < 0.0)
    return gmres_core(c, opL, jac, b, x, tol, c->restart, c->maxit, 1 << 30, false, c->d_V, nullptr, c->d_w,
                      c->d_t1, c->d_t2, iters, relres);
  VecOp opP = [&](const double* in, double* out) { if (transpose) op_PT(c, in, out); else op_P(c, in, out); };
  VecOp inner = [&](const double* in, double* out) {
    int it = 0;
    double rr = 0;
    (void)gmres_core(c, opP, jac, in, out, 1e-3, c->inner_iters, c->inner_iters, 1, true, c->d_Vin, nullptr,
                     c->d_t4, c->d_t1, c->d_t5, &it, &rr);
    c->inner_total += it;
  };
  return gmres_core(c, opL, inner, b, x, tol, c->restart, c->maxit, 1 << 30, false, c->d_V, c->d_Z, c->d_w,
                    c->d_t1, c->d_t2, iters, relres);
}

// L x = b (or L^T x = b).  Precision 0 and 1: GMRES (1: FP32 preconditioner, see
// gmres).  Precision 2: FP64 iterative refinement around
// GMRES solves of the correction equation with the FP32 near-field kernels (FP64
// Krylov vectors, orthogonalisation and norms); each correction is solved to the
// relative tolerance that would meet tol, but not below kInnerFloor, and the FP64
// residual decides when to stop.
// The FP32 operator is linear only up to single-precision rounding, so an inner
// solve cannot go much below cond(L) * 1e-7; corrections are solved to at most
// 1e-4 relative and at most one Krylov cycle each, and the refinement contracts.
constexpr int kMaxRefine = 10;
constexpr double kInnerFloor = 1e-4;
int diis_solve(ddlpb_ctx* c, bool transpose, const double* b, double* x, double tol, int* iters, double* relres);
int solve_system(ddlpb_ctx* c, bool transpose, const double* b, double* x, double tol, int* iters, double* relres) {
  c->cur_prec = 0;
  if (c->solver == 1) {  // Jacobi-DIIS, FP64
    c->stats.refinements = 0;
    return diis_solve(c, transpose, b, x, tol, iters, relres);
  }
  if (c->precision != 2 || !c->use_caps || !c->d_rr) {
    c->fp64_iters = 0;
    const int rc = gmres(c, transpose, b, x, tol, iters, relres);
    c->stats.refinements = c->fp64_iters;
    return rc;
  }
  const long D = 2L * c->M * c->L;
  const double bn = norm2(c, b);
  if (bn == 0.0) {
    fill(c, x, D, 0.0);
    *iters = 0;
    *relres = 0.0;
    c->stats.refinements = 0;
    return DDLPB_OK;
  }
  const int maxit = c->maxit;
  int total = 0, refs = 0;
  double rel = 0.0;
  for (;;) {
    if (transpose) op_LT(c, x, c->d_rr);
    else op_L(c, x, c->d_rr);
    axpby(c, 1.0, b, -1.0, c->d_rr);  // r = b - L x (FP64 operator)
    rel = norm2(c, c->d_rr) / bn;
    if (rel <= tol || refs >= kMaxRefine || total >= maxit) break;
    const double tin = std::min(0.5, std::max(0.5 * tol / rel, kInnerFloor));
    fill(c, c->d_dd, D, 0.0);
    int it = 0;
    double rr = 0.0;
    c->cur_prec = 1;
    c->maxit = std::min(maxit - total, c->restart);
    (void)gmres(c, transpose, c->d_rr, c->d_dd, tin, &it, &rr);
    c->maxit = maxit;
    c->cur_prec = 0;
    axpby(c, 1.0, c->d_dd, 1.0, x);  // x += d
    total += it;
    ++refs;
  }
  c->stats.refinements = refs;
  *iters = total;
  *relres = rel;
  return rel <= tol ? DDLPB_OK : DDLPB_ENOCONV;
}

// ------------------------------------------------------ Jacobi-DIIS solver
// max |a - b| and max |s + a| over the 2ML entries (null b or s: that term is |a|)
void amax2(ddlpb_ctx* c, const double* a, const double* b, const double* s, double* m1, double* m2) {
  const long D = 2L * c->M * c->L;
  hipLaunchKernelGGL(k_amax2, dim3(c->nb_dot), dim3(256), 0, c->stream, D, a, b, s, c->d_part);
  HIPCHK(hipGetLastError());
  std::vector<double> h(2 * (size_t)c->nb_dot);
  HIPCHK(hipMemcpyAsync(h.data(), c->d_part, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  *m1 = *m2 = 0.0;
  for (int k = 0; k < c->nb_dot; ++k) {
    *m1 = std::max(*m1, h[2 * k]);
    *m2 = std::max(*m2, h[2 * k + 1]);
  }
}

// DIIS (Pulay) extrapolation for a fixed point x = F(x): keeps the last m values
// f_i = F(x_i) and errors e_i = f_i - x_i on the device (slots F[i], E[i], stride D),
// their Gram matrix on the host, and returns sum_i c_i f_i with sum_i c_i = 1
// minimising |sum_i c_i e_i| (Pulay 1980).
struct Diis {
  ddlpb_ctx* c;
  double *F, *E;
  int m, count = 0, head = 0;
  std::vector<double> B;  // [m][m] Gram matrix of the error slots
  Diis(ddlpb_ctx* c_, double* F_, double* E_, int m_) : c(c_), F(F_), E(E_), m(m_), B((size_t)m_ * m_, 0.0) {}
  void reset() { count = head = 0; }
  // slot for the next pair (the caller writes f and e there), then push() records it
  double* fslot() { return F + (long)head * 2L * c->M * c->L; }
  double* eslot() { return E + (long)head * 2L * c->M * c->L; }
  void push() {
    const long D = 2L * c->M * c->L;
    const int n = std::min(count + 1, m);
    std::vector<double> h(n);
    mdot(c, n, E, D, eslot(), h.data());
    for (int i = 0; i < n; ++i) B[(size_t)head * m + i] = B[(size_t)i * m + head] = h[i];
    count = n;
    head = (head + 1) % m;
  }
  // x = sum c_i f_i; false when the bordered system is singular (x untouched)
  bool extrapolate(double* x) {
    const int n = count, A = n + 1;
    double scale = 0.0;
    for (int i = 0; i < n; ++i) scale = std::max(scale, B[(size_t)i * m + i]);
    if (!(scale > 0.0)) return false;
    std::vector<double> G((size_t)A * A, 0.0), r(A, 0.0);
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < n; ++j) G[(size_t)i * A + j] = B[(size_t)i * m + j] / scale;
      G[(size_t)i * A + n] = G[(size_t)n * A + i] = 1.0;
    }
    r[n] = 1.0;
    for (int k = 0; k < A; ++k) {  // Gaussian elimination, partial pivoting
      int piv = k;
      for (int i = k + 1; i < A; ++i)
        if (std::fabs(G[(size_t)i * A + k]) > std::fabs(G[(size_t)piv * A + k])) piv = i;
      if (std::fabs(G[(size_t)piv * A + k]) < 1e-14) return false;
      if (piv != k) {
        for (int j = 0; j < A; ++j) std::swap(G[(size_t)k * A + j], G[(size_t)piv * A + j]);
        std::swap(r[k], r[piv]);
      }
      for (int i = k + 1; i < A; ++i) {
        const double f = G[(size_t)i * A + k] / G[(size_t)k * A + k];
        for (int j = k; j < A; ++j) G[(size_t)i * A + j] -= f * G[(size_t)k * A + j];
        r[i] -= f * r[k];
      }
    }
    std::vector<double> cf(A);
    for (int i = A - 1; i >= 0; --i) {
      double v = r[i];
      for (int j = i + 1; j < A; ++j) v -= G[(size_t)i * A + j] * cf[j];
      cf[i] = v / G[(size_t)i * A + i];
    }
    const long D = 2L * c->M * c->L;
    if (n > c->mk) throw HipError{hipErrorInvalidValue};
    HIPCHK(hipMemcpyAsync(c->d_hv, cf.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_mcomb, dim3(nblk(D, 256)), dim3(256), 0, c->stream, D, n, F, D, c->d_hv, x);
    HIPCHK(hipGetLastError());
    return true;
  }
};

// The paper's solver (Sec. 4, opening): macro-iterations X <- L_AB^{-1}(g - L_C X)
// accelerated by DIIS, L_AB being the preconditioner; each L_AB solve by
// micro-iterations (Jacobi sweeps X <- b + (I - L_AB) X, the diagonal blocks being
// the identity, also accelerated by DIIS) started from the previous macro iterate,
// i.e. the correction d of L_AB d = g - L X starts from zero.  Both stop on the
// relative infinity-norm increment: tol for the macro, tol / 100 for the micro
// iterations.  relres reports the final ||g - L X|| / ||g||.
int diis_solve(ddlpb_ctx* c, bool transpose, const double* b, double* x, double tol, int* iters, double* relres) {
  const long D = 2L * c->M * c->L;
  const int m = std::min(c->diis_max, (c->restart + 1 - 4) / 4);
  *iters = 0;
  *relres = 0.0;
  if (m < 2) return DDLPB_EINVAL;
  const double bn = norm2(c, b);
  if (bn == 0.0) { fill(c, x, D, 0.0); return DDLPB_OK; }
  double* V = c->d_V;
  Diis mac(c, V, V + (long)m * D, m), mic(c, V + 2L * m * D, V + 3L * m * D, m);
  double* r = V + 4L * m * D;  // g - L X
  double* d = r + D;           // micro iterate (correction)
  double* dn = d + D;          // Jacobi image of d
  auto op = [&](const double* in, double* out) { if (transpose) op_LT(c, in, out); else op_L(c, in, out); };
  auto sweep = [&](const double* rhs, const double* z, double* out) {  // rhs + (I - L_AB) z
    if (!transpose) {
      apply_LX(c, rhs, 1.0, z, 1.0, nullptr, nullptr, nullptr, 0.0, out);
    } else {
      syn2(c, z, 0, c->d_zr, c->d_ze);
      apply_LTZ(c, rhs, 1.0, c->d_zr, c->d_ze, 1.0, nullptr, 0, out);
    }
  };
  const double tin = tol / 100.0;
  bool conv = false;
  int it = 0;
  for (; it < c->maxit && !conv; ++it) {
    op(x, c->d_w);
    HIPCHK(hipMemcpyAsync(r, b, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    axpby(c, -1.0, c->d_w, 1.0, r);
    // micro-iterations on L_AB d = r from d = 0 (first Jacobi image: d = r)
    mic.reset();
    HIPCHK(hipMemcpyAsync(d, r, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    for (int mi = 0; mi < 200; ++mi) {
      sweep(r, d, dn);
      c->inner_total += 1;
      double inc, nrm;
      amax2(c, dn, d, x, &inc, &nrm);
      if (inc <= tin * nrm) {
        HIPCHK(hipMemcpyAsync(d, dn, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        break;
      }
      HIPCHK(hipMemcpyAsync(mic.fslot(), dn, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipMemcpyAsync(mic.eslot(), dn, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      axpby(c, -1.0, d, 1.0, mic.eslot());
      mic.push();
      if (!mic.extrapolate(d)) HIPCHK(hipMemcpyAsync(d, dn, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    }
    // macro fixed point: F(X) = X + d
    double inc, nrm;
    amax2(c, d, nullptr, x, &inc, &nrm);
    if (inc <= tol * nrm) conv = true;
    HIPCHK(hipMemcpyAsync(mac.fslot(), x, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    axpby(c, 1.0, d, 1.0, mac.fslot());
    HIPCHK(hipMemcpyAsync(mac.eslot(), d, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (conv) {
      HIPCHK(hipMemcpyAsync(x, mac.fslot(), D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      break;
    }
    mac.push();
    if (!mac.extrapolate(x)) axpby(c, 1.0, d, 1.0, x);
  }
  op(x, c->d_w);
  HIPCHK(hipMemcpyAsync(r, b, D * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  axpby(c, -1.0, c->d_w, 1.0, r);
  *relres = norm2(c, r) / bn;
  *iters = conv ? it + 1 : it;
  return conv ? DDLPB_OK : DDLPB_ENOCONV;
}

// ------------------------------------------------------------ device setup
void upload_and_init(ddlpb_ctx* c) {
  ensure_constants();
  const int M = c->M, N = c->N, LUR = c->LUR;
  // per-sphere radial tables (FP64, host)
  std::vector<double> ycr((size_t)M * LUR), yce((size_t)M * LUR), Cl((size_t)M * LUR), sgr((size_t)M * LUR),
      ur((size_t)M * LUR), kr((size_t)M * LUR), rtab(4 * (size_t)M * LUR, 0.0);
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
      if (l + 1 < LUR) {
        // radius derivatives (dE/dr_j): dk_l = kappa k_l'/k_l, C_l'/C_l = 2/r + D_l + dk_l,
        // (eps1/eps2) l/r^2, D_l' = kappa^2 + l(l+1)/r^2 - 2 D_l/r - D_l^2 (Bessel equation)
        const double Dl = c->kappa * c->kappa * rj * sg[l + 1] / sg[l] + l / rj;
        const double dk = -c->kappa * kk[l + 1] / kk[l] + l / rj;
        const size_t jl = (size_t)j * LUR + l, MU = (size_t)M * LUR;
        rtab[jl] = dk;
        rtab[MU + jl] = 2.0 / rj + Dl + dk;
        rtab[2 * MU + jl] = (c->eps1 / c->eps2) * l / (rj * rj);
        rtab[3 * MU + jl] = c->kappa * c->kappa + l * (l + 1.0) / (rj * rj) - 2.0 * Dl / rj - Dl * Dl;
      }
    }
  }
  c->nterms = host::sigma_terms(c->lmax, c->kappa * c->kappa * rmax * rmax);
  // Y table up to degree max(lmax + 1, p): the local expansions of degree p are
  // evaluated on the sphere grids in full
  std::vector<double> Y((size_t)N * c->LY);
  const int ydeg = (int)std::lround(std::sqrt((double)c->LY)) - 1;
  for (int n = 0; n < N; ++n) {
    const double* s = c->leb.data() + 4 * n;
    host::solid_harmonics<double>(ydeg, s[0], s[1], s[2], &Y[(size_t)n * c->LY]);
  }
  std::vector<double> dtab;
  host::gradient_coupling(c->lmax, dtab);
  auto up = [&](void* d, const void* h, size_t bytes) {
    if (bytes) HIPCHK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c->stream));
  };
  up(c->d_xyz, c->x.data(), 3 * M * sizeof(double));
  up(c->d_rad, c->r.data(), M * sizeof(double));
  up(c->d_q, c->q.data(), M * sizeof(double));
  up(c->d_leb, c->leb.data(), 4 * N * sizeof(double));
  up(c->d_Y, Y.data(), Y.size() * sizeof(double));
  std::vector<double> YT(Y.size());
  for (int n = 0; n < N; ++n)
    for (int t = 0; t < c->LY; ++t) YT[(size_t)t * N + n] = Y[(size_t)n * c->LY + t];
  up(c->d_YT, YT.data(), YT.size() * sizeof(double));
  std::vector<double> WY((size_t)N * c->L);
  for (int n = 0; n < N; ++n)
    for (int t = 0; t < c->L; ++t) WY[(size_t)n * c->L + t] = c->leb[4 * n + 3] * Y[(size_t)n * c->LY + t];
  up(c->d_WY, WY.data(), WY.size() * sizeof(double));
  up(c->d_nptr, c->nptr.data(), (M + 1) * sizeof(int));
  up(c->d_nidx, c->nidx.data(), c->nidx.size() * sizeof(int));
  up(c->d_nrev, c->nrev.data(), c->nrev.size() * sizeof(int));
  up(c->d_pptr, c->pptr.data(), (M + 1) * sizeof(int));
  up(c->d_pidx, c->pidx.data(), c->pidx.size() * sizeof(int));
  up(c->d_ycr, ycr.data(), ycr.size() * sizeof(double));
  up(c->d_yce, yce.data(), yce.size() * sizeof(double));
  up(c->d_Cl, Cl.data(), Cl.size() * sizeof(double));
  up(c->d_sgr, sgr.data(), sgr.size() * sizeof(double));
  up(c->d_rtab, rtab.data(), rtab.size() * sizeof(double));
  std::vector<double> isgr(sgr.size());
  for (size_t k = 0; k < sgr.size(); ++k) isgr[k] = sgr[k] != 0.0 ? 1.0 / sgr[k] : 0.0;
  up(c->d_isgr, isgr.data(), isgr.size() * sizeof(double));
  up(c->d_ur, ur.data(), ur.size() * sizeof(double));
  std::vector<double> iur(ur.size());
  for (size_t k = 0; k < ur.size(); ++k) iur[k] = ur[k] != 0.0 ? 1.0 / ur[k] : 0.0;
  up(c->d_iur, iur.data(), iur.size() * sizeof(double));
  up(c->d_kr, kr.data(), kr.size() * sizeof(double));
  up(c->d_dtab, dtab.data(), dtab.size() * sizeof(double));
  if (c->fmm_order > 0) {
    const int p1 = c->fmm_order + 1;
    up(c->d_fA, c->tables.Ap.data(), c->tables.Ap.size() * sizeof(double));
    up(c->d_fAoff, c->tables.Aoff.data(), c->tables.Aoff.size() * sizeof(int));
    up(c->d_fAL, c->tables.AL.data(), c->tables.AL.size() * sizeof(double));
    up(c->d_fJ, c->tables.J.data(), c->tables.J.size() * sizeof(double));
    up(c->d_fJoff, c->tables.Joff.data(), c->tables.Joff.size() * sizeof(int));
    up(c->d_fjval, c->tables.Jval.data(), c->tables.Jval.size() * sizeof(double));
    up(c->d_fjrow, c->tables.Jrow.data(), c->tables.Jrow.size() * sizeof(int));
    up(c->d_fjpad, c->tables.Jpad.data(), c->tables.Jpad.size() * sizeof(double));
    for (int k = 0; k < 2; ++k) {
      for (int d = 0; d < 2; ++d) up(c->d_fZ[k][d], c->tables.Z[k][d].data(), c->tables.Z[k][d].size() * sizeof(double));
      up(c->d_fZslot[k], c->tables.Zslot[k].data(), c->tables.Zslot[k].size() * sizeof(int));
    }
    for (int d = 0; d < 2; ++d) up(c->d_fZl[d], c->tables.Zlvl[d].data(), c->tables.Zlvl[d].size() * sizeof(double));
    // sigma_l(kappa^2 r_i^2) up to degree p (normalisation of the sphere locals)
    std::vector<double> sgp((size_t)M * (p1 + 1)), sgt(p1 + 2), qs(M);
    for (int j = 0; j < M; ++j) {
      host::bessel_sigma(p1, c->kappa * c->kappa * c->r[j] * c->r[j], sgt.data());
      for (int l = 0; l <= p1; ++l) sgp[(size_t)j * (p1 + 1) + l] = sgt[l];
      qs[j] = c->q[j] * std::sqrt(4.0 * host::kPi) / (c->eps1 * c->r[j]);  // charge as a degree-0 multipole at scale r_j
    }
    up(c->d_sgp, sgp.data(), sgp.size() * sizeof(double));
    up(c->d_qsrc, qs.data(), qs.size() * sizeof(double));
    c->nterms_p = host::sigma_terms(c->fmm_order, c->kappa * c->kappa * rmax * rmax);
  }
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
void upload_tree(ddlpb_ctx* c) {
  const auto& t = c->tree;
  auto up = [&](void* d, const void* h, size_t bytes) {
    if (bytes) HIPCHK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c->stream));
  };
  up(c->d_fcen, t.center.data(), t.center.size() * sizeof(double));
  up(c->d_frad, t.radius.data(), t.radius.size() * sizeof(double));
  up(c->d_fchild, t.child.data(), t.child.size() * sizeof(int));
  up(c->d_fparent, t.parent.data(), t.parent.size() * sizeof(int));
  up(c->d_flevn, t.level_nodes.data(), t.level_nodes.size() * sizeof(int));
  up(c->d_sleaf, t.sphere_leaf.data(), t.sphere_leaf.size() * sizeof(int));
  up(c->d_fm2lp, t.m2l_ptr.data(), t.m2l_ptr.size() * sizeof(int));
  up(c->d_fm2ls, t.m2l_src.data(), t.m2l_src.size() * sizeof(int));
  up(c->d_fm2lord, t.m2l_order.data(), t.m2l_order.size() * sizeof(int));
  up(c->d_fnp, t.near_ptr.data(), t.near_ptr.size() * sizeof(int));
  up(c->d_fni, t.near_idx.data(), t.near_idx.size() * sizeof(int));
  hipLaunchKernelGGL(k_fmm_node_radial, dim3(nblk(t.nnodes, 128)), dim3(128), 0, c->stream, t.nnodes, c->fmm_order,
                     c->kappa, c->d_frad, c->d_fkR, c->d_fkRi, c->d_fiR);
  HIPCHK(hipGetLastError());
  c->stats.n_m2l = (int64_t)t.m2l_src.size();
  c->stats.n_near_pairs = (int64_t)t.near_idx.size();
}

nearlane::NearArgs near_args(ddlpb_ctx* c) {
  nearlane::NearArgs a;
  a.M = c->M;
  a.N = c->N;
  a.LUR = c->LUR;
  a.nterms = c->nterms;
  a.kappa = c->kappa;
  a.leb = c->d_leb;
  a.xyz = c->d_xyz;
  a.rad = c->d_rad;
  a.rptr = c->d_rptr;
  a.rci = c->d_rci;
  a.rcn = c->d_rcn;
  a.rcw = c->d_rcw;
  a.isgr = c->d_isgr;
  a.cache = c->near_incore ? c->d_cache : nullptr;
  a.coff = c->d_coff;
  a.jord = c->d_jord;
  return a;
}

// The lane kernels need every forward cap's position in the reverse lists (for the
// per-point sums of the forward pass) and, with near_incore, the cache of harmonics.
// rcnt: reverse caps per sphere; nrev: their total.
void setup_lane(ddlpb_ctx* c, const std::vector<int>& rcnt, long nrev) {
  const int M = c->M, N = c->N;
  c->use_lane = false;
  if (!c->near_lane || c->lmax > nearlane::kMaxLm || nrev != c->ncap) return;
  HIPCHK(hipMemsetAsync(c->d_actcnt, 0, sizeof(int), c->stream));
  hipLaunchKernelGGL(k_cap_perm, dim3(nblk(M, 64)), dim3(64), 0, c->stream, M, N, c->d_nptr, c->d_nidx, c->d_rptr,
                     c->d_rci, c->d_rcn, c->d_pcp, c->d_capslot, c->d_f2r, c->d_actcnt);
  HIPCHK(hipGetLastError());
  int found = 0;
  HIPCHK(hipMemcpyAsync(&found, c->d_actcnt, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (found != c->ncap) return;  // forward and reverse lists disagree: keep the cap kernels
  {
    std::vector<int> ord(M);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int p, int q) { return rcnt[p] > rcnt[q]; });
    HIPCHK(hipMemcpyAsync(c->d_jord, ord.data(), M * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));  // ord is freed at the end of this block
  }
  c->use_lane = true;
  if (!c->near_incore) return;
  // incore: sphere j's caps at padded position coff[j] (a multiple of 16)
  std::vector<long> coff(M);
  long tot = 0;
  for (int j = 0; j < M; ++j) {
    coff[j] = tot;
    tot += (rcnt[j] + nearlane::kGroup - 1) / nearlane::kGroup * nearlane::kGroup;
  }
  const size_t need = std::max<size_t>((size_t)tot * nearlane::cache_stride(c->lmax) * sizeof(double), 256);
  if (need > c->cache_bytes) {
    if (c->d_cache) HIPCHK(hipFree(c->d_cache));
    c->d_cache = nullptr;
    c->cache_bytes = 0;
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) throw std::bad_alloc();
    c->d_cache = (double*)p;
    c->cache_bytes = need;
  }
  HIPCHK(hipMemcpyAsync(c->d_coff, coff.data(), M * sizeof(long), hipMemcpyHostToDevice, c->stream));
  HIPCHK(nearlane::launch_fill(c->lmax, near_args(c), c->d_cache, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

void geometry_on_device(ddlpb_ctx* c) {
  const int M = c->M, N = c->N;
  HIPCHK(hipMemcpyAsync(c->d_xyz, c->x.data(), 3 * M * sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (c->fmm_order > 0) upload_tree(c);
  hipLaunchKernelGGL(k_grid_fields, dim3(nblk((long)M * N, 256)), dim3(256), 0, c->stream, M, N, c->d_xyz, c->d_rad,
                     c->d_leb, c->d_nptr, c->d_nidx, c->eta, c->d_f, c->d_U);
  hipLaunchKernelGGL(k_active_count, dim3(nblk(M, 128)), dim3(128), 0, c->stream, M, N, c->d_U, c->d_actcnt);
  HIPCHK(hipGetLastError());
  std::vector<int> cnt(M), ptr(M + 1, 0);
  HIPCHK(hipMemcpyAsync(cnt.data(), c->d_actcnt, M * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int i = 0; i < M; ++i) ptr[i + 1] = ptr[i] + cnt[i];
  c->nact = ptr[M];
  c->near_pairs_pts = 0.0;
  for (int i = 0; i < M; ++i) c->near_pairs_pts += (double)cnt[i] * (c->pptr[i + 1] - c->pptr[i]);
  HIPCHK(hipMemcpyAsync(c->d_actptr, ptr.data(), (M + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_cap_count, dim3(nblk(M, 128)), dim3(128), 0, c->stream, M, N, c->d_xyz, c->d_rad, c->d_leb,
                     c->d_nptr, c->d_nidx, c->d_actcnt);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(cnt.data(), c->d_actcnt, M * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->ncap = 0;
  for (int i = 0; i < M; ++i) c->ncap += cnt[i];
  c->stats.n_cap_pairs = c->ncap;
  {
    int dev = 0, maxlds = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    size_t need = 0;
    LM_DISPATCH(c->lmax, need = std::max(k_apply_LX_caps_lds_entries<LMc>(N), k_apply_LTZ_caps_lds_entries<LMc>(N)) *
                                sizeof(double));
    c->use_caps = c->cap_lists && (size_t)c->ncap <= c->cap_cap && need <= (size_t)maxlds;
  }
  if (c->use_caps) {
    std::vector<int> cp(M + 1, 0);
    for (int i = 0; i < M; ++i) cp[i + 1] = cp[i] + cnt[i];
    HIPCHK(hipMemcpyAsync(c->d_cptr, cp.data(), (M + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_caps_fill, dim3(nblk(M, 64)), dim3(64), 0, c->stream, M, N, c->d_xyz, c->d_rad, c->d_leb,
                       c->d_nptr, c->d_nidx, c->d_f, c->eta, c->d_cptr, c->d_capn, c->d_capslot, c->d_capw, c->d_pcp);
    hipLaunchKernelGGL(k_rcaps_count, dim3(nblk(M, 64)), dim3(64), 0, c->stream, M, N, c->d_xyz, c->d_rad, c->d_leb,
                       c->d_nptr, c->d_nidx, c->d_actcnt);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(cnt.data(), c->d_actcnt, M * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < M; ++i) cp[i + 1] = cp[i] + cnt[i];
    HIPCHK(hipMemcpyAsync(c->d_rptr, cp.data(), (M + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_rcaps_fill, dim3(nblk(M, 64)), dim3(64), 0, c->stream, M, N, c->d_xyz, c->d_rad, c->d_leb,
                       c->d_nptr, c->d_nidx, c->d_f, c->eta, c->d_rptr, c->d_rci, c->d_rcn, c->d_rcw);
    HIPCHK(hipGetLastError());
    setup_lane(c, cnt, cp[M]);
  } else {
    c->use_lane = false;
  }
  hipLaunchKernelGGL(k_active_fill, dim3(nblk(M, 128)), dim3(128), 0, c->stream, M, N, c->d_U, c->d_actptr,
                     c->d_actsph, c->d_actn);
  HIPCHK(hipGetLastError());
  c->stats.n_active_points = c->nact;
  if (c->fmm_order == 0) c->stats.n_near_pairs = (int64_t)M * M;
  c->near_pts_fmm = 0.0;
  if (c->fmm_order > 0)
    for (int i = 0; i < M; ++i) c->near_pts_fmm += (double)(ptr[i + 1] - ptr[i]) * (c->tree.near_ptr[i + 1] - c->tree.near_ptr[i]);
  c->rhs_ready = false;
}

int ensure_device(ddlpb_ctx* c) {
  if (c->dev_ready) return DDLPB_OK;
  size_t need = workspace_size(c);
  // options set after ddlpb_bind_workspace may have enlarged the layout
  if (c->ws_bound && need > c->ws_bytes) return DDLPB_ENOMEM;
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
  if (c->nact > 0 && c->fmm_order == 0) {
    KScope ks(c, "laplace_field", 16.0 * (double)c->nact * c->M);
    hipLaunchKernelGGL(k_laplace_field_direct, dim3(nblk(c->nact, 256)), dim3(256), 0, c->stream, c->M, c->N, c->nact,
                       c->d_actsph, c->d_actn, c->d_xyz, c->d_rad, c->d_leb, c->d_q, c->eps1, c->eps2, c->d_psi,
                       c->d_e);
    HIPCHK(hipGetLastError());
  } else if (c->nact > 0) {
    {
      KScope ks(c, "laplace_near", 16.0 * c->near_pts_fmm);
      hipLaunchKernelGGL(k_laplace_field_list, dim3(nblk(c->nact, 256)), dim3(256), 0, c->stream, c->N, c->nact,
                         c->d_actsph, c->d_actn, c->d_xyz, c->d_rad, c->d_leb, c->d_q, c->d_fnp, c->d_fni, c->eps1,
                         c->eps2, c->d_psi, c->d_e);
      HIPCHK(hipGetLastError());
    }
    fmm_forward(c, 1, c->d_qsrc, 0, 1, c->d_SL);
    l2p(c, 1, c->eps1 / c->eps2, c->d_psi, c->d_e);
  }
  moments(c, nullptr, c->d_e, nullptr, c->d_m);
  sl_field_full(c, c->d_m, c->d_Phi);
  apply_LX(c, nullptr, 0.0, nullptr, 0.0, c->d_psi, c->d_Phi, c->d_Phi, -1.0, c->d_g);
  c->rhs_ready = true;
}

// Fields of the frozen functional E_f shared by the forces and the radius gradient
// (Sec. 3): xi = Syn(X_adj) on the grids, grid charges c = w U xi_s, h = e + Syn(y(X)),
// m = C (.) An(U h), Phi = Phi[m], lambda' (other spheres, degree lmax+1), eta =
// Syn(C (.) lambda), the gradient of Phi' at the active points and the target-side point
// gradients fpt (psi_0, d_n psi_0 of the other charges and the single-layer field of
// the other spheres).
void adjoint_fields(ddlpb_ctx* c) {
  const int M = c->M, N = c->N;
  syn2(c, c->d_Xa, 0, c->d_xr, c->d_xe);
  syn2(c, c->d_Xa, 1, c->d_cg, nullptr);
  moments(c, c->d_X, c->d_e, c->d_h, c->d_m);
  sl_field_full(c, c->d_m, c->d_Phi);
  sl_adjoint_full(c, c->d_cg, c->lmax + 1, 1, c->LP, c->d_lam);
  LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_eta<LMc>), dim3(M), dim3(256), 0, c->stream, M, N, c->LY, c->d_Y,
                                          c->d_cg, c->d_lam, c->LP, c->d_Cl, c->LUR, c->d_eta));
  HIPCHK(hipGetLastError());
  if (c->nact == 0) return;
  const bool fmmode = c->fmm_order > 0;
  // grad Phi' at active points (near part by pairs, far part from the sphere locals)
  if (!fmmode) {
    sl_field(c, c->d_m, true, 1, c->d_gphi);
  } else if (c->sl32) {
    KScope ks(c, "sl_near_grad_f32", 4.0 * flops_sl_pair(c->lmax) * c->near_pts_fmm);
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_sl_field_list<LMc, true, float>), dim3(nblk(c->nact, 256)),
                                            dim3(256), 0, c->stream, c->M, c->N, c->nact, c->d_actsph, c->d_actn,
                                            c->d_xyz, c->d_rad, c->d_leb, c->d_fnp, c->d_fni, c->d_m, c->d_iur,
                                            c->LUR, c->kappa, 1, 0, c->d_gphi));
    HIPCHK(hipGetLastError());
  } else {
    KScope ks(c, "sl_near_grad", 4.0 * flops_sl_pair(c->lmax) * c->near_pts_fmm);
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_sl_field_list<LMc, true>), dim3(nblk(c->nact, 256)), dim3(256), 0,
                                            c->stream, c->M, c->N, c->nact, c->d_actsph, c->d_actn, c->d_xyz,
                                            c->d_rad, c->d_leb, c->d_fnp, c->d_fni, c->d_m, c->d_iur, c->LUR,
                                            c->kappa, 1, 0, c->d_gphi));
    HIPCHK(hipGetLastError());
  }
  if (fmmode) {
    fmm_forward(c, 0, c->d_m, c->lmax, c->L, c->d_SL);
    P_DISPATCH(c->fmm_order, hipLaunchKernelGGL((k_local_grad_yuk<PDc>), dim3(nblk(c->nact, 128)), dim3(128), 0,
                                                c->stream, c->nact, c->d_actsph, c->d_actn, c->d_rad, c->d_leb,
                                                c->d_sgp, c->fmm_order + 2, c->kappa, c->nterms_p, c->d_SL,
                                                c->d_gphi));
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_force_points, dim3(nblk(c->nact, 256)), dim3(256), 0, c->stream, M, N, c->nact, c->d_actsph,
                     c->d_actn, c->d_xyz, c->d_rad, c->d_leb, c->d_q, c->eps1, c->eps2, c->d_U, c->d_xr, c->d_xe,
                     c->d_eta, c->d_gphi, fmmode ? 0 : 1, c->d_fpt);
  HIPCHK(hipGetLastError());
  if (fmmode) {
    hipLaunchKernelGGL(k_force_points_lap_list, dim3(nblk(c->nact, 256)), dim3(256), 0, c->stream, N, c->nact,
                       c->d_actsph, c->d_actn, c->d_xyz, c->d_rad, c->d_leb, c->d_q, c->eps1, c->eps2, c->d_U,
                       c->d_xr, c->d_eta, c->d_fnp, c->d_fni, c->d_fpt);
    fmm_forward(c, 1, c->d_qsrc, 0, 1, c->d_SL);
    P_DISPATCH(c->fmm_order, hipLaunchKernelGGL((k_local_force_lap<PDc>), dim3(nblk(c->nact, 128)), dim3(128), 0,
                                                c->stream, N, c->nact, c->d_actsph, c->d_actn, c->d_rad, c->d_leb,
                                                c->d_U, c->d_xr, c->d_eta, c->eps1, c->eps2, c->d_SL, c->d_fpt));
    HIPCHK(hipGetLastError());
  }
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
    c->LY = std::max(c->LP, (fmm_order + 1) * (fmm_order + 1));
    c->LUR = lmax + 2;
    c->N = n_lebedev;
    c->rule = host::lebedev_rule(n_lebedev);
    order_points(c->rule->xyzw, n_lebedev, c->leb_orig);
    c->leb.resize(4 * (size_t)n_lebedev);
    for (int n = 0; n < n_lebedev; ++n)
      for (int k = 0; k < 4; ++k) c->leb[4 * (size_t)n + k] = c->rule->xyzw[4 * (size_t)c->leb_orig[n] + k];
    c->fmm_order = fmm_order;
    c->eps1 = eps_in; c->eps2 = eps_out; c->kappa = kappa;
    c->x.assign(centers, centers + 3L * n_atoms);
    c->r.assign(radii, radii + n_atoms);
    c->q.assign(charges, charges + n_atoms);
    int r2 = build_neighbours(c);
    if (r2) { delete c; return r2; }
    build_pairs(c, c->pdelta, c->pptr, c->pidx);
    if (fmm_order > 0) {
      if (fmm_order < lmax + 1) { delete c; return DDLPB_EINVAL; }
      fmm::build_tables(fmm_order, c->tables);
      fmm::build_tree(c->M, c->x.data(), c->r.data(), c->tree);
      fmm::build_lists(c->M, c->r.data(), c->theta, c->tree, c->leaf_size);
      c->stats.n_m2l = (int64_t)c->tree.m2l_src.size();
      c->stats.n_near_pairs = (int64_t)c->tree.near_idx.size();
    }
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
    if (!c->warm_start) fill(c, c->d_X, 2L * c->M * c->L, 0.0);
    rc = solve_system(c, false, c->d_g, c->d_X, tol, &it, &rel);
    c->stats.iters_primal = it;
    c->stats.resid_primal = rel;
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(1024), 0, c->stream, c->M, c->L, c->d_X, c->d_q, c->d_scal);
    HIPCHK(hipGetLastError());
    double E = 0;
    HIPCHK(hipMemcpyAsync(&E, c->d_scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    ktimer_flush(c);
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
    if (!c->warm_start) fill(c, c->d_Xa, 2L * c->M * c->L, 0.0);
    int rc = solve_system(c, true, c->d_Q, c->d_Xa, tol, &it, &rel);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->stats.iters_adjoint = it;
    c->stats.resid_adjoint = rel;
    ktimer_flush(c);
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
    {
      // mixed path with the FMM: the single-layer terms of the force fields with FP32
      // pairs (FP64 sums) and the FP32-vector M2L (option mixed_forces)
      const bool f32 = c->precision == 1 && c->fmm_order > 0 && c->mixed_forces;
      struct Flags {
        ddlpb_ctx* c;
        ~Flags() { c->sl32 = c->m2l32 = false; }
      } restore{c};
      c->sl32 = f32;
      c->m2l32 = f32;
      adjoint_fields(c);
    }
    const bool fmmode = c->fmm_order > 0;
    // switching / near-field terms
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_force_switch<LMc>), dim3(M), dim3(256), 0, c->stream, M, N, c->d_leb,
                                            c->d_xyz, c->d_rad, c->d_nptr, c->d_nidx, c->d_f, c->d_U, c->d_sgr,
                                            c->LUR, c->kappa, c->eta, c->nterms, c->d_X, c->d_xr, c->d_xe, c->d_psi,
                                            c->d_Phi, c->d_h, c->d_eta, c->d_fnb, c->d_fself));
    HIPCHK(hipGetLastError());
    // target-side point terms, summed per sphere
    fill(c, c->d_fpts, 3L * M, 0.0);
    if (c->nact > 0) {
      hipLaunchKernelGGL(k_sum_points, dim3(M), dim3(256), 0, c->stream, M, c->d_actptr, c->d_fpt, c->d_fpts);
      HIPCHK(hipGetLastError());
    }
    // source-side terms
    if (!fmmode) {
      hipLaunchKernelGGL(k_force_laplace_source, dim3(M), dim3(256), 0, c->stream, M, N, c->nact, c->d_actsph,
                         c->d_actn, c->d_xyz, c->d_rad, c->d_leb, c->d_q, c->eps1, c->eps2, c->d_U, c->d_xr, c->d_eta,
                         c->d_flsrc);
    } else {
      fill(c, c->d_flsrc, 3L * M, 0.0);
      hipLaunchKernelGGL(k_force_laplace_source_list, dim3(M), dim3(256), 0, c->stream, N, c->d_actptr, c->d_actn,
                         c->d_xyz, c->d_rad, c->d_leb, c->d_q, c->eps1, c->eps2, c->d_U, c->d_xr, c->d_eta, c->d_fnp,
                         c->d_fni, c->d_flsrc);
      hipLaunchKernelGGL(k_lap_src_grids, dim3(nblk((long)M * N, 256)), dim3(256), 0, c->stream, M, N, c->d_leb,
                         c->d_U, c->d_xr, c->d_eta, c->eps1, c->eps2, c->d_zr, c->d_ze);
      HIPCHK(hipGetLastError());
      p2l_dual(c, c->d_zr, c->d_ze, c->d_Lam);
      fmm_transpose(c, 1, c->d_Lam, 1, 4, 0, c->d_tmp4);
      hipLaunchKernelGGL(k_force_lap_far_source, dim3(nblk(M, 256)), dim3(256), 0, c->stream, M, 4, c->d_q, c->d_rad,
                         c->d_tmp4, c->d_flsrc);
      HIPCHK(hipGetLastError());
    }
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_force_yukawa_source<LMc>), dim3(M), dim3(128), 0, c->stream, M,
                                            c->d_m, c->d_lam, c->d_dtab, c->d_kr, c->LUR, c->kappa, c->d_fysrc));
    hipLaunchKernelGGL(k_force_final, dim3(nblk(M, 256)), dim3(256), 0, c->stream, M, c->d_nptr, c->d_nidx,
                       c->d_nrev, c->d_fnb, c->d_fself, c->d_fpts, c->d_flsrc, c->d_fysrc, c->d_F);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(forces_out, c->d_F, 3L * M * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    ktimer_flush(c);
    c->stats.ms_forces = elapsed_ms(t0);
    return DDLPB_OK;
  });
}

int ddlpb_radius_gradient(ddlpb_ctx* c, double* dedr_out) {
  if (!c || !dedr_out) return DDLPB_EINVAL;
  if (c->state < 2) return DDLPB_ESTATE;
  return guarded([&]() -> int {
    const int M = c->M, N = c->N;
    adjoint_fields(c);
    // buffers of the force terms hold the scalar radius terms: fnb (per neighbour
    // slot), fself, fpts, fysrc (per sphere); the result goes to F
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_rgrad_switch<LMc>), dim3(M), dim3(256), 0, c->stream, M, N, c->d_leb,
                                            c->d_xyz, c->d_rad, c->d_nptr, c->d_nidx, c->d_f, c->d_U, c->d_sgr,
                                            c->d_yce, c->LUR, c->kappa, c->eta, c->nterms, c->d_X, c->d_xr, c->d_xe,
                                            c->d_psi, c->d_Phi, c->d_h, c->d_eta, c->d_fnb, c->d_fself));
    HIPCHK(hipGetLastError());
    fill(c, c->d_fpts, M, 0.0);
    if (c->nact > 0) {
      hipLaunchKernelGGL(k_rgrad_points, dim3(M), dim3(256), 0, c->stream, N, c->d_actptr, c->d_actn, c->d_rad,
                         c->d_leb, c->d_q, c->eps1, c->eps2, c->d_U, c->d_xr, c->d_eta, c->d_fpt, c->d_fpts);
      HIPCHK(hipGetLastError());
    }
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_rgrad_source<LMc>), dim3(M), dim3(256), 0, c->stream, M, N, c->LY,
                                            c->d_Y, c->d_leb, c->d_U, c->d_cg, c->d_eta, c->d_lam, c->LP, c->d_m,
                                            c->d_X, c->d_rtab, c->LUR, c->d_fysrc));
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_rgrad_final, dim3(nblk(M, 256)), dim3(256), 0, c->stream, M, c->d_nptr, c->d_nidx,
                       c->d_nrev, c->d_fnb, c->d_fself, c->d_fpts, c->d_fysrc, c->d_F);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(dedr_out, c->d_F, (size_t)M * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    ktimer_flush(c);
    return DDLPB_OK;
  });
}

namespace {
int check_eval_args(const ddlpb_ctx* c, int32_t n_points, const double* points, const int32_t* spheres,
                    const double* out) {
  if (!c || n_points < 0 || (n_points > 0 && (!points || !out))) return DDLPB_EINVAL;
  if (c->state < 1) return DDLPB_ESTATE;
  for (long k = 0; k < 3L * n_points; ++k)
    if (!std::isfinite(points[k])) return DDLPB_EINVAL;
  if (spheres)
    for (int k = 0; k < n_points; ++k)
      if (spheres[k] < 0 || spheres[k] >= c->M) return DDLPB_EINVAL;
  return DDLPB_OK;
}
// bytes of device staging per evaluation point: the point, its ball and 8 results
constexpr size_t kEvalBytesPerPoint = 3 * sizeof(double) + 8 * sizeof(double) + sizeof(int);
// staging layout inside a block of n points: points [n][3], results [n][8], balls [n]
void eval_staged(ddlpb_ctx* c, int32_t n_points, const double* points, const int32_t* spheres, double* out,
                 char* blk) {
  const size_t bp = 3L * n_points * sizeof(double), bo = 8L * n_points * sizeof(double);
  double* dp = (double*)blk;
  double* dout = (double*)(blk + bp);
  int* dball = (int*)(blk + bp + bo);
  HIPCHK(hipMemcpyAsync(dp, points, bp, hipMemcpyHostToDevice, c->stream));
  if (spheres) {
    HIPCHK(hipMemcpyAsync(dball, spheres, (size_t)n_points * sizeof(int), hipMemcpyHostToDevice, c->stream));
  } else {
    hipLaunchKernelGGL(k_nearest_ball, dim3(nblk(n_points, 256)), dim3(256), 0, c->stream, n_points, dp, c->M,
                       c->d_xyz, c->d_rad, dball);
    HIPCHK(hipGetLastError());
  }
  LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_eval_points<LMc>), dim3(nblk(n_points, 256)), dim3(256), 0, c->stream,
                                          n_points, dp, dball, c->M, c->L, c->LUR, c->d_X, c->d_xyz, c->d_rad,
                                          c->d_isgr, c->kappa, c->nterms, dout));
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(out, dout, bo, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

// Staging of ddlpb_eval_potentials_noalloc: one fixed array per GPU, held from the
// first call on that GPU until the process ends.  In host code `scratch` names a
// host-side stand-in; its device address on each GPU comes from hipGetSymbolAddress
// (kept per device in g_scratch_dev) and only that address is used.
constexpr size_t kNoallocMaxPoints = DDLPB_NOALLOC_MAX_POINTS;
constexpr size_t kScratchBytes = kNoallocMaxPoints * kEvalBytesPerPoint;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_dev;
char* scratch_on_current_device() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_dev.find(dev);
  if (it != g_scratch_dev.end()) return it->second;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p || ((uintptr_t)p & 255) != 0) throw HipError{hipErrorInvalidSymbol};
  g_scratch_dev[dev] = (char*)p;
  return (char*)p;
}
}  // namespace

int ddlpb_eval_potentials(ddlpb_ctx* c, int32_t n_points, const double* points, const int32_t* spheres,
                          double* out) {
  int rc = check_eval_args(c, n_points, points, spheres, out);
  if (rc || n_points == 0) return rc;
  return guarded([&]() -> int {
    // points, balls and results in one temporary device block (freed before return)
    char* blk = nullptr;
    if (hipMalloc((void**)&blk, (size_t)n_points * kEvalBytesPerPoint) != hipSuccess) {
      (void)hipGetLastError();
      return DDLPB_ENOMEM;
    }
    try {
      eval_staged(c, n_points, points, spheres, out, blk);
    } catch (...) {
      (void)hipStreamSynchronize(c->stream);
      (void)hipFree(blk);
      throw;
    }
    HIPCHK(hipFree(blk));
    return DDLPB_OK;
  });
}

int ddlpb_eval_potentials_noalloc(ddlpb_ctx* c, int32_t n_points, const double* points, const int32_t* spheres,
                                  double* out) {
  int rc = check_eval_args(c, n_points, points, spheres, out);
  if (rc) return rc;
  if ((size_t)n_points > kNoallocMaxPoints) return DDLPB_EINVAL;
  if (n_points == 0) return DDLPB_OK;
  return guarded([&]() -> int {
    // every staged entry is written before it is read (copies, ball search, kernel):
    // nothing of the previous call's contents is used
    eval_staged(c, n_points, points, spheres, out, scratch_on_current_device());
    return DDLPB_OK;
  });
}

int ddlpb_charge_gradient(ddlpb_ctx* c, double* dedq_out) {
  if (!c || !dedq_out) return DDLPB_EINVAL;
  if (c->state < 2) return DDLPB_ESTATE;
  return guarded([&]() -> int {
    const int M = c->M, N = c->N;
    // xi_r, grid charges, lambda' and eta: the adjoint fields of the force assembly
    syn2(c, c->d_Xa, 0, c->d_xr, c->d_xe);
    syn2(c, c->d_Xa, 1, c->d_cg, nullptr);
    sl_adjoint_full(c, c->d_cg, c->lmax + 1, 1, c->LP, c->d_lam);
    LM_DISPATCH(c->lmax, hipLaunchKernelGGL((k_eta<LMc>), dim3(M), dim3(256), 0, c->stream, M, N, c->LY, c->d_Y,
                                            c->d_cg, c->d_lam, c->LP, c->d_Cl, c->LUR, c->d_eta));
    HIPCHK(hipGetLastError());
    double* dq = c->d_tmp4 ? c->d_tmp4 : c->d_F;  // [M] (forces buffer when no FMM scratch)
    const double* Mu = nullptr;
    if (c->fmm_order == 0) {
      if (c->nact > 0)
        hipLaunchKernelGGL(k_dq_laplace_source, dim3(M), dim3(256), 0, c->stream, M, N, c->nact, c->d_actsph,
                           c->d_actn, c->d_xyz, c->d_rad, c->d_leb, c->eps1, c->eps2, c->d_U, c->d_xr, c->d_eta, dq);
      else
        fill(c, dq, M, 0.0);
    } else {
      hipLaunchKernelGGL(k_dq_laplace_source_list, dim3(M), dim3(256), 0, c->stream, N, c->d_actptr, c->d_actn,
                         c->d_xyz, c->d_rad, c->d_leb, c->eps1, c->eps2, c->d_U, c->d_xr, c->d_eta, c->d_fnp, c->d_fni,
                         dq);
      hipLaunchKernelGGL(k_lap_src_grids, dim3(nblk((long)M * N, 256)), dim3(256), 0, c->stream, M, N, c->d_leb,
                         c->d_U, c->d_xr, c->d_eta, c->eps1, c->eps2, c->d_zr, c->d_ze);
      HIPCHK(hipGetLastError());
      p2l_dual(c, c->d_zr, c->d_ze, c->d_Lam);
      fmm_transpose(c, 1, c->d_Lam, 0, 1, 0, c->d_F);  // Mu_k[0] in the forces buffer
      Mu = c->d_F;
    }
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_dq_final, dim3(nblk(M, 256)), dim3(256), 0, c->stream, M, c->L, c->d_X, c->d_rad, Mu, 1, dq);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(dedq_out, dq, (size_t)M * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    ktimer_flush(c);
    return DDLPB_OK;
  });
}

int ddlpb_dielectric_gradient(ddlpb_ctx* c, double* dedeps_out) {
  if (!c || !dedeps_out) return DDLPB_EINVAL;
  if (c->state < 2) return DDLPB_ESTATE;
  return guarded([&]() -> int {
    const long ML = (long)c->M * c->L, D = 2 * ML;
    // C1 X_r in both rows: the single-layer part of L applied to (X_r, 0)
    HIPCHK(hipMemcpyAsync(c->d_t1, c->d_X, ML * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    fill(c, c->d_t1 + ML, ML, 0.0);
    moments(c, c->d_t1, nullptr, nullptr, c->d_m);
    sl_field_full(c, c->d_m, c->d_Phi);
    apply_LX(c, nullptr, 0.0, nullptr, 0.0, c->d_Phi, nullptr, c->d_Phi, 1.0, c->d_t2);
    double a = 0.0, b = 0.0, f0 = 0.0;
    mdot(c, 1, c->d_Xa, 0, c->d_t2, &a);  // <X_adj,r + X_adj,e, C1 X_r>
    hipLaunchKernelGGL(k_rhs_parts, dim3(nblk(ML, 256)), dim3(256), 0, c->stream, ML, 0, c->d_g, c->d_t3);
    HIPCHK(hipGetLastError());
    mdot(c, 1, c->d_Xa, 0, c->d_t3, &b);  // <X_adj,r, G0>, G0 = g_r - g_e
    hipLaunchKernelGGL(k_rhs_parts, dim3(nblk(ML, 256)), dim3(256), 0, c->stream, ML, 1, c->d_g, c->d_t3);
    HIPCHK(hipGetLastError());
    mdot(c, 1, c->d_Xa, 0, c->d_t3, &f0);  // <X_adj,r + X_adj,e, F0>, F0 = g_e
    (void)D;
    // dE/d lambda = 1/2 <X_adj, dg/d lambda - (dL/d lambda) X> (Sec. 3): G0 ~ 1/eps_in,
    // F0 ~ 1/eps_out, C1 ~ eps_in/eps_out, A, B, C2 independent of both
    dedeps_out[0] = -(b + a) / (2.0 * c->eps1);
    dedeps_out[1] = (a - f0) / (2.0 * c->eps2);
    ktimer_flush(c);
    return DDLPB_OK;
  });
}

void ddlpb_free(ddlpb_ctx* c) {
  if (!c) return;
  if (c->ws_owned && c->ws) (void)hipFree(c->ws);
  if (c->d_cache) (void)hipFree(c->d_cache);
  for (auto& p : c->ev_pending) { (void)hipEventDestroy(p.second.first); (void)hipEventDestroy(p.second.second); }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
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
    if (v != 0 && v != 1 && v != 2) return DDLPB_EINVAL;
    c->precision = (int)v;
    c->stats.precision = (int)v;
  } else if (k == "gmres_restart") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v >= 1 && v <= 200)) return DDLPB_EINVAL;
    c->restart = (int)v;
  } else if (k == "inner_sweeps") {
    if (!(v >= 0 && v <= 64)) return DDLPB_EINVAL;
    c->sweeps = (int)v;
  } else if (k == "precond_delta") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v < 0 || v <= 20.0)) return DDLPB_EINVAL;
    c->pdelta = v;
    build_pairs(c, c->pdelta, c->pptr, c->pidx);
  } else if (k == "inner_iters") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v >= 1 && v <= 200)) return DDLPB_EINVAL;
    c->inner_iters = (int)v;
  } else if (k == "kernel_timing") {
    c->ktiming = v != 0;
  } else if (k == "warm_start") {
    c->warm_start = v != 0;
  } else if (k == "max_iter") {
    if (!(v >= 1 && v <= 1e6)) return DDLPB_EINVAL;
    c->maxit = (int)v;
  } else if (k == "precond_krylov") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v >= 0 && v <= 64)) return DDLPB_EINVAL;
    c->pkrylov = (int)v;
  } else if (k == "cap_lists") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v == 0 || v == 1)) return DDLPB_EINVAL;
    c->cap_lists = v != 0;
  } else if (k == "mixed_forces") {
    if (!(v == 0 || v == 1)) return DDLPB_EINVAL;
    c->mixed_forces = v != 0;
  } else if (k == "inner_reorth") {
    if (!(v == 0 || v == 1)) return DDLPB_EINVAL;
    c->inner_reorth = v != 0;
  } else if (k == "mixed_levels") {
    if (!(v == 0 || v == 1)) return DDLPB_EINVAL;
    c->mixed_lvl = v != 0;
  } else if (k == "mixed_m2l") {
    if (!(v == 0 || v == 1)) return DDLPB_EINVAL;
    c->mixed_m2l = v != 0;
  } else if (k == "mixed_near_sl") {
    if (!(v == 0 || v == 1)) return DDLPB_EINVAL;
    c->mixed_sl = v != 0;
  } else if (k == "apply_fp32") {
    if (!(v >= 0 && v <= 3)) return DDLPB_EINVAL;
    c->apply_fp32 = (int)v;
  } else if (k == "m2l_waves") {
    if (!(v == -1 || v == 0 || v == 1 || v == 2 || v == 4 || v == 8 || v == 16)) return DDLPB_EINVAL;
    c->m2l_waves = (int)v;
    c->m2l_cfg[0].valid = c->m2l_cfg[1].valid = false;
  } else if (k == "m2l_lane") {
    if (!(v == 0 || v == 1)) return DDLPB_EINVAL;
    c->m2l_lane = (int)v;
  } else if (k == "level_lane") {
    if (v < 0 || v > 1e9 || v != (double)(long)v) return DDLPB_EINVAL;
    c->level_lane = (int)v;
  } else if (k == "near_lane" || k == "near_incore") {
    // cap structures depend on both: set before the first device call
    if (fixed) return DDLPB_ESTATE;
    if (!(v == 0 || v == 1)) return DDLPB_EINVAL;
    (k == "near_lane" ? c->near_lane : c->near_incore) = (int)v;
  } else if (k == "solver") {
    if (!(v == 0 || v == 1)) return DDLPB_EINVAL;
    c->solver = (int)v;
  } else if (k == "diis_max") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v >= 2 && v <= 32)) return DDLPB_EINVAL;
    c->diis_max = (int)v;
  } else if (k == "leaf_size") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v >= 1 && v <= 64 && v == (int)v)) return DDLPB_EINVAL;
    c->leaf_size = (int)v;
    if (c->fmm_order > 0) {
      fmm::build_lists(c->M, c->r.data(), c->theta, c->tree, c->leaf_size);
      c->stats.n_m2l = (int64_t)c->tree.m2l_src.size();
      c->stats.n_near_pairs = (int64_t)c->tree.near_idx.size();
    }
  } else if (k == "theta") {
    if (fixed) return DDLPB_ESTATE;
    if (!(v > 0 && v < 1)) return DDLPB_EINVAL;
    c->theta = v;
    if (c->fmm_order > 0) {
      fmm::build_lists(c->M, c->r.data(), c->theta, c->tree, c->leaf_size);
      c->stats.n_m2l = (int64_t)c->tree.m2l_src.size();
      c->stats.n_near_pairs = (int64_t)c->tree.near_idx.size();
    }
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
    // previous geometry, restored when the new one cannot be set up (EGEOM, ENOMEM)
    const std::vector<double> old = c->x;
    const std::vector<int> onptr = c->nptr, onidx = c->nidx, onrev = c->nrev, opptr = c->pptr, opidx = c->pidx;
    // the old tree is moved aside (not copied) when a new one is built
    fmm::Tree otree;
    if (c->fmm_order > 0) otree = std::move(c->tree);
    const size_t ocap_est = c->cap_est, onnz = c->nnz_cap, opnz = c->pnz_cap, ocap = c->cap_cap, om2l = c->m2l_cap,
                 onear = c->near_cap;
    auto restore = [&]() {
      c->x = old; c->nptr = onptr; c->nidx = onidx; c->nrev = onrev; c->pptr = opptr; c->pidx = opidx;
      if (c->fmm_order > 0) c->tree = std::move(otree);
      c->cap_est = ocap_est; c->nnz_cap = onnz; c->pnz_cap = opnz; c->cap_cap = ocap;
      c->m2l_cap = om2l; c->near_cap = onear;
    };
    c->x.assign(centers, centers + 3L * c->M);
    int rc = build_neighbours(c);
    if (rc) { restore(); return rc; }
    build_pairs(c, c->pdelta, c->pptr, c->pidx);
    if (c->fmm_order > 0) {
      // the leaves sit at the sphere centres: the tree and its lists follow the atoms
      fmm::build_tree(c->M, c->x.data(), c->r.data(), c->tree);
      fmm::build_lists(c->M, c->r.data(), c->theta, c->tree, c->leaf_size);
    }
    if (c->dev_ready) {
      const bool relayout = c->nidx.size() > c->nnz_cap || c->pidx.size() > c->pnz_cap || c->cap_est > c->cap_cap ||
                            (c->fmm_order > 0 && (c->tree.m2l_src.size() > c->m2l_cap ||
                                                  c->tree.near_idx.size() > c->near_cap));
      if (relayout) {
        // list capacities exceeded: the workspace layout changes; keep X and X_adj
        std::vector<double> X(2L * c->M * c->L), Xa(2L * c->M * c->L);
        HIPCHK(hipMemcpyAsync(X.data(), c->d_X, X.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(Xa.data(), c->d_Xa, Xa.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        c->nnz_cap = c->nidx.size() + c->nidx.size() / 4 + 64;
        c->pnz_cap = c->pidx.size() + c->pidx.size() / 4 + 64;
        c->cap_cap = c->cap_est + c->cap_est / 4 + 64;
        if (c->fmm_order > 0) {
          c->m2l_cap = c->tree.m2l_src.size() + c->tree.m2l_src.size() / 4 + 64;
          c->near_cap = c->tree.near_idx.size() + c->tree.near_idx.size() / 4 + 64;
        }
        size_t need = workspace_size(c);
        if (c->ws_bound && need > c->ws_bytes) {
          restore();
          size_t t;
          carve(c, c->ws, &t);  // device pointers of the previous layout
          return DDLPB_ENOMEM;
        }
        if (c->ws_owned && need > c->ws_bytes) {
          // the new block first: when it cannot be had, the old one and its state stay
          void* p = nullptr;
          if (hipMalloc(&p, need) != hipSuccess) {
            (void)hipGetLastError();
            restore();
            size_t t;
            carve(c, c->ws, &t);
            return DDLPB_ENOMEM;
          }
          HIPCHK(hipStreamSynchronize(c->stream));
          (void)hipFree(c->ws);
          c->ws = (char*)p;
          c->ws_bytes = need;
        }
        size_t t;
        carve(c, c->ws, &t);
        upload_and_init(c);
        HIPCHK(hipMemcpyAsync(c->d_X, X.data(), X.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->d_Xa, Xa.data(), Xa.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
      } else {
        auto up = [&](void* d, const void* h, size_t bytes) {
          if (bytes) HIPCHK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c->stream));
        };
        up(c->d_nidx, c->nidx.data(), c->nidx.size() * sizeof(int));
        up(c->d_nrev, c->nrev.data(), c->nrev.size() * sizeof(int));
        up(c->d_nptr, c->nptr.data(), (c->M + 1) * sizeof(int));
        up(c->d_pidx, c->pidx.data(), c->pidx.size() * sizeof(int));
        up(c->d_pptr, c->pptr.data(), (c->M + 1) * sizeof(int));
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

int ddlpb_kernel_times(ddlpb_ctx* c, int32_t idx, char* name_out, double* ms, int64_t* launches, double* work) {
  if (!c || idx < 0) return DDLPB_EINVAL;
  if (idx >= (int)c->ktimers.size()) return DDLPB_EINVAL;
  const auto& t = c->ktimers[idx];
  if (name_out) { std::strncpy(name_out, t.name.c_str(), 63); name_out[63] = 0; }
  if (ms) *ms = t.ms;
  if (launches) *launches = t.launches;
  if (work) *work = t.work;
  return DDLPB_OK;
}

int ddlpb_kernel_times_reset(ddlpb_ctx* c) {
  if (!c) return DDLPB_EINVAL;
  return guarded([&]() -> int {
    ktimer_flush(c);
    for (auto& t : c->ktimers) { t.ms = 0; t.work = 0; t.launches = 0; }
    return DDLPB_OK;
  });
}

int ddlpb_get_grid(ddlpb_ctx* c, double* f_out, double* u_out) {
  if (!c) return DDLPB_EINVAL;
  return guarded([&]() -> int {
    int rc = ensure_device(c);
    if (rc) return rc;
    const int M = c->M, N = c->N;
    const size_t MN = (size_t)M * N;
    std::vector<double> tmp(MN);
    for (int k = 0; k < 2; ++k) {  // back to the rule's point order
      double* dst = k == 0 ? f_out : u_out;
      if (!dst) continue;
      HIPCHK(hipMemcpyAsync(tmp.data(), k == 0 ? c->d_f : c->d_U, MN * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      for (int i = 0; i < M; ++i)
        for (int n = 0; n < N; ++n) dst[(size_t)i * N + c->leb_orig[n]] = tmp[(size_t)i * N + n];
    }
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
    c->cur_prec = c->apply_fp32 == 1 ? 1 : 0;
    c->sl32 = c->apply_fp32 == 2;
    c->m2l32 = c->apply_fp32 == 3;
    try {
      if (transpose) op_LT(c, c->d_t2, c->d_w); else op_L(c, c->d_t2, c->d_w);
    } catch (...) {
      c->cur_prec = 0;
      c->sl32 = c->m2l32 = false;
      throw;
    }
    c->cur_prec = 0;
    c->sl32 = c->m2l32 = false;
    HIPCHK(hipMemcpyAsync(y_out, c->d_w, D * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DDLPB_OK;
  });
}

}  // extern "C"
