// Host side of the fast multipole method (Appendix): tree, interaction lists
// and translation coefficient tables.
//
// Tree: binary, built by recursive median splits of the sphere centres along the
// widest axis; every leaf is one sphere (so a leaf expansion is the sphere's own
// expansion, centred at x_j with scale r_j).  Node radius R encloses every grid
// point of the node's spheres (max |x_j - c| + r_j).
// Lists: symmetric dual traversal with the acceptance test R_T + R_S < theta |c_T - c_S|;
// accepted pairs are multipole-to-local translations, rejected leaf pairs are
// evaluated directly (near list, sphere pairs).
#pragma once
#include <algorithm>
#include <atomic>
#include <cmath>
#include <functional>
#include <numeric>
#include <thread>
#include <utility>
#include <vector>

#include "host_math.hpp"

namespace ddlpb {
namespace fmm {

struct Tree {
  int nnodes = 0, nlevels = 0;
  std::vector<double> center;     // [nnodes][3]
  std::vector<double> radius;     // [nnodes]
  std::vector<int> child;         // [nnodes][2], -1 for leaves
  std::vector<int> parent;        // [nnodes]
  std::vector<int> level;         // [nnodes]
  std::vector<int> leaf_sphere;   // [nnodes], sphere index of a leaf or -1
  std::vector<int> sphere_leaf;   // [M], node index of the sphere's leaf
  std::vector<int> sph;           // [M], spheres in tree order: node n holds sph[lo[n] .. hi[n])
  std::vector<int> lo, hi;        // [nnodes]
  std::vector<int> level_ptr, level_nodes;  // nodes grouped by level (CSR)
  // interaction lists
  // per target node, source nodes (sorted); the lists are symmetric, so the list of a
  // node is also the list of targets it is a source for (the transposed lists)
  std::vector<int> m2l_ptr, m2l_src;
  std::vector<int> near_ptr, near_idx;  // per target sphere, source spheres (self included)
  std::vector<int> m2l_order;  // nodes by decreasing list length (work order)
};

inline void build_tree(int M, const double* x, const double* r, Tree& t) {
  std::vector<int> idx(M);
  std::iota(idx.begin(), idx.end(), 0);
  t.center.clear(); t.radius.clear(); t.child.clear(); t.parent.clear(); t.level.clear(); t.leaf_sphere.clear();
  t.lo.clear(); t.hi.clear();
  t.sphere_leaf.assign(M, -1);
  std::function<int(int, int, int, int)> rec = [&](int lo, int hi, int par, int lev) -> int {
    const int id = (int)t.radius.size();
    t.center.resize(3 * (id + 1));
    t.radius.push_back(0.0);
    t.child.push_back(-1); t.child.push_back(-1);
    t.parent.push_back(par);
    t.level.push_back(lev);
    t.leaf_sphere.push_back(-1);
    t.lo.push_back(lo);
    t.hi.push_back(hi);
    double bmin[3] = {1e300, 1e300, 1e300}, bmax[3] = {-1e300, -1e300, -1e300};
    for (int k = lo; k < hi; ++k)
      for (int a = 0; a < 3; ++a) {
        bmin[a] = std::min(bmin[a], x[3 * idx[k] + a]);
        bmax[a] = std::max(bmax[a], x[3 * idx[k] + a]);
      }
    double c[3];
    for (int a = 0; a < 3; ++a) c[a] = 0.5 * (bmin[a] + bmax[a]);
    if (hi - lo == 1) for (int a = 0; a < 3; ++a) c[a] = x[3 * idx[lo] + a];
    double R = 0.0;
    for (int k = lo; k < hi; ++k) {
      const int j = idx[k];
      double d2 = 0;
      for (int a = 0; a < 3; ++a) { double v = x[3 * j + a] - c[a]; d2 += v * v; }
      R = std::max(R, std::sqrt(d2) + r[j]);
    }
    for (int a = 0; a < 3; ++a) t.center[3 * id + a] = c[a];
    t.radius[id] = R;
    if (hi - lo == 1) {
      t.leaf_sphere[id] = idx[lo];
      t.sphere_leaf[idx[lo]] = id;
      return id;
    }
    int ax = 0;
    for (int a = 1; a < 3; ++a) if (bmax[a] - bmin[a] > bmax[ax] - bmin[ax]) ax = a;
    const int mid = (lo + hi) / 2;
    std::nth_element(idx.begin() + lo, idx.begin() + mid, idx.begin() + hi, [&](int p, int q) {
      if (x[3 * p + ax] != x[3 * q + ax]) return x[3 * p + ax] < x[3 * q + ax];
      return p < q;
    });
    const int c0 = rec(lo, mid, id, lev + 1);
    const int c1 = rec(mid, hi, id, lev + 1);
    t.child[2 * id] = c0;
    t.child[2 * id + 1] = c1;
    return id;
  };
  rec(0, M, -1, 0);
  t.sph = idx;
  t.nnodes = (int)t.radius.size();
  t.nlevels = *std::max_element(t.level.begin(), t.level.end()) + 1;
  t.level_ptr.assign(t.nlevels + 1, 0);
  for (int v : t.level) t.level_ptr[v + 1]++;
  for (int l = 0; l < t.nlevels; ++l) t.level_ptr[l + 1] += t.level_ptr[l];
  t.level_nodes.assign(t.nnodes, 0);
  std::vector<int> fillp(t.level_ptr.begin(), t.level_ptr.end() - 1);
  for (int n = 0; n < t.nnodes; ++n) t.level_nodes[fillp[t.level[n]]++] = n;
}

// Runs body(i) for i in [0, n) on up to 16 host threads (dynamic chunks of `chunk`).
template <class F>
inline void parallel_for(long n, long chunk, F body) {
  const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::atomic<long> next{0};
  auto work = [&]() {
    for (;;) {
      const long i0 = next.fetch_add(chunk);
      if (i0 >= n) return;
      for (long i = i0; i < std::min(n, i0 + chunk); ++i) body(i);
    }
  };
  if (nt == 1 || n <= chunk) { work(); return; }
  std::vector<std::thread> th;
  for (int k = 1; k < nt; ++k) th.emplace_back(work);
  work();
  for (auto& x : th) x.join();
}

// CSR of the pairs (key, value) grouped by key (nkeys keys), values of a key sorted
// increasingly; pairs come in per-task vectors.
inline void pairs_to_csr(const std::vector<std::vector<std::pair<int, int>>>& parts, int nkeys,
                         std::vector<int>& ptr, std::vector<int>& idx) {
  std::vector<std::atomic<int>> cnt(nkeys + 1);
  for (auto& c : cnt) c.store(0, std::memory_order_relaxed);
  parallel_for((long)parts.size(), 1, [&](long k) {
    for (const auto& pr : parts[k]) cnt[pr.first].fetch_add(1, std::memory_order_relaxed);
  });
  ptr.assign(nkeys + 1, 0);
  for (int n = 0; n < nkeys; ++n) ptr[n + 1] = ptr[n] + cnt[n].load(std::memory_order_relaxed);
  idx.assign(ptr[nkeys], 0);
  for (int n = 0; n < nkeys; ++n) cnt[n].store(ptr[n], std::memory_order_relaxed);
  parallel_for((long)parts.size(), 1, [&](long k) {
    for (const auto& pr : parts[k]) idx[cnt[pr.first].fetch_add(1, std::memory_order_relaxed)] = pr.second;
  });
  parallel_for(nkeys, 1024, [&](long n) { std::sort(idx.begin() + ptr[n], idx.begin() + ptr[n + 1]); });
}

// Interaction lists by a symmetric dual traversal: self(A) = self(A1) + self(A2) +
// mutual(A1, A2); mutual(A, B) is accepted as the two translations A -> B and B -> A
// when R_A + R_B < theta |c_A - c_B|, is a near pair (both ways) when both are
// leaf groups -- nodes of at most leaf_size spheres, whose spheres then interact
// directly pair by pair -- and otherwise splits the larger node (ties by index).
// With leaf_size 1 the leaf groups are the single-sphere leaves.  The list of every
// node is therefore also its transposed list.  The traversal is expanded
// breadth-first into a frontier of pending tasks that host threads finish
// depth-first; the lists are assembled by counting sorts with each list sorted, so
// the result does not depend on the thread schedule.
inline void build_lists(int M, const double* r, double theta, Tree& t, int leaf_size = 1) {
  auto is_leaf = [&](int n) { return t.hi[n] - t.lo[n] <= leaf_size; };
  // every sphere of A with every sphere of B (both orders when A != B)
  auto all_pairs = [&](int A, int B, std::vector<std::pair<int, int>>& on) {
    for (int a = t.lo[A]; a < t.hi[A]; ++a)
      for (int b = t.lo[B]; b < t.hi[B]; ++b) {
        on.push_back({t.sph[a], t.sph[b]});
        if (A != B) on.push_back({t.sph[b], t.sph[a]});
      }
  };
  using Pairs = std::vector<std::pair<int, int>>;
  // one task (A == B: self, else mutual): emits pairs, appends subtasks to `sub`
  auto visit = [&](int A, int B, Pairs& om, Pairs& on, Pairs& sub) {
    if (A == B) {
      if (is_leaf(A)) { all_pairs(A, A, on); return; }
      const int c1 = t.child[2 * A], c2 = t.child[2 * A + 1];
      sub.push_back({c1, c2});
      sub.push_back({c2, c2});
      sub.push_back({c1, c1});
      return;
    }
    double d2 = 0;
    for (int a = 0; a < 3; ++a) { double v = t.center[3 * A + a] - t.center[3 * B + a]; d2 += v * v; }
    if (t.radius[A] + t.radius[B] < theta * std::sqrt(d2)) {
      om.push_back({A, B});
      om.push_back({B, A});
      return;
    }
    const bool la = is_leaf(A), lb = is_leaf(B);
    if (la && lb) {
      all_pairs(A, B, on);
      return;
    }
    const bool split_a = lb || (!la && (t.radius[A] > t.radius[B] || (t.radius[A] == t.radius[B] && A < B)));
    if (split_a) {
      sub.push_back({t.child[2 * A + 1], B});
      sub.push_back({t.child[2 * A], B});
    } else {
      sub.push_back({A, t.child[2 * B + 1]});
      sub.push_back({A, t.child[2 * B]});
    }
  };
  Pairs frontier{{0, 0}}, nextf;
  std::vector<Pairs> m2l(1), near(1);
  while (!frontier.empty() && frontier.size() < 32768) {
    nextf.clear();
    for (auto [A, B] : frontier) visit(A, B, m2l[0], near[0], nextf);
    frontier.swap(nextf);
  }
  const long nf = (long)frontier.size();
  const long per = 8;
  const long nparts = (nf + per - 1) / per;
  m2l.resize(1 + nparts);
  near.resize(1 + nparts);
  parallel_for(nparts, 1, [&](long k) {
    Pairs stack;
    for (long f = k * per; f < std::min(nf, (k + 1) * per); ++f) {
      stack.push_back(frontier[f]);
      while (!stack.empty()) {
        const auto [A, B] = stack.back();
        stack.pop_back();
        visit(A, B, m2l[1 + k], near[1 + k], stack);
      }
    }
  });
  pairs_to_csr(m2l, t.nnodes, t.m2l_ptr, t.m2l_src);
  pairs_to_csr(near, M, t.near_ptr, t.near_idx);
  t.m2l_order.resize(t.nnodes);
  std::iota(t.m2l_order.begin(), t.m2l_order.end(), 0);
  std::stable_sort(t.m2l_order.begin(), t.m2l_order.end(), [&](int a, int b) {
    return t.m2l_ptr[a + 1] - t.m2l_ptr[a] > t.m2l_ptr[b + 1] - t.m2l_ptr[b];
  });
  (void)r;
}

// ------------------------------------------------------ coefficient tables
inline double lfact(int n) { return std::lgamma(n + 1.0); }
inline double dfact(int n) { double v = 1.0; for (int k = n; k > 1; k -= 2) v *= k; return v; }
// normalisation of the real harmonics with the sign (-1)^m for m != 0
inline double ntil(int l, int m) {
  const int am = std::abs(m);
  if (am == 0) return std::sqrt((2.0 * l + 1.0) / (4.0 * host::kPi));
  const double s = (am % 2) ? -1.0 : 1.0;
  return s * std::sqrt(2.0 * (2.0 * l + 1.0) / (4.0 * host::kPi) * std::exp(lfact(l - am) - lfact(l + am)));
}
// C_N(l, m, l') = N(l,m) (2l'+1) (l'-|m|)! (l+|m|)! / N(l',m)
inline double cn(int l, int m, int lp) {
  const int am = std::abs(m);
  return ntil(l, m) / ntil(lp, m) * (2.0 * lp + 1.0) * std::exp(lfact(lp - am) + lfact(l + am));
}
// C_{l m k}^{l'} = (2k)! / (2^k (k+m)! k! (k-m)! (l'-k)! (l-k)!)
inline double clmk(int l, int m, int k, int lp) {
  return std::exp(lfact(2 * k) - k * std::log(2.0) - lfact(k + m) - lfact(k) - lfact(k - m) - lfact(lp - k) - lfact(l - k));
}

struct Tables {
  int pmax = 0;
  // Yukawa: A[((l*(P1) + l')*(P1) + |m|)*(P1) + k] = C_N C_{lmk}^{l'}
  std::vector<double> A;
  // Laplace: per kind (0 m2m, 1 m2l, 2 l2l): AL[kind][(l*(P1) + l')*(P1) + |m|]
  std::vector<double> AL;
  // packed Yukawa coefficients: Ap[Aoff[(l*P1 + l')*P1 + |m|] + (k - |m|)], k = |m|..min(l, l')
  std::vector<double> Ap;
  std::vector<int> Aoff;
  // rotation by +90 degrees about x: packed blocks J_l [(2l+1)^2], row m'+l, column m+l
  std::vector<double> J;
  std::vector<int> Joff;
  // Sparse rows of J (mat 0) and J^T (mat 1).  Every row of a block has its nonzeros
  // on every second column of one run (the blocks split by the parity classes of m):
  // Jrow[2 * (mat * L + t)] = offset into Jval, Jrow[2 * (mat * L + t) + 1] = index
  // l^2 + (first m + l) of the first column | count << 12 | column step << 20, for
  // the row t = l^2 + l + m'.
  std::vector<double> Jval;
  std::vector<int> Jrow;
  // The same rows for the wavefront M2L kernel: row t = 64 g + lane of group g, padded
  // with zeros to K_g entries (the largest count of the group, rounded up to even),
  // laid out [mat][g][k][lane]; K_g in 4-bit fields of jpad_kpack.  Needs every row to
  // be one run of step 2 (jpad_ok).
  std::vector<double> Jpad;
  int jpad_kpack = 0;
  bool jpad_ok = false;
  // z-translation coefficients of the M2L kernel laid out per output pair (lo, |m|):
  // Z[kern][dir] holds for every pair the entries of l_in = |m|..p in order (Yukawa:
  // k = |m|..min(lo, l_in); Laplace: one value); dir 0 is the forward translation
  // (lo = target degree), dir 1 its transpose (lo = source degree).  Pairs are dealt
  // to the 64 lanes by longest-first balancing: Zslot[kern][2 s] = lo << 8 | |m| of
  // the pair in slot s (lane s mod 64; -1 when empty), Zslot[kern][2 s + 1] = offset.
  std::vector<double> Z[2][2];
  // Yukawa z-translation coefficients without the (-1)^k sign, same layout as Z[0][dir],
  // for the level passes (M2M, L2L), whose offsets are not sign-flipped
  std::vector<double> Zlvl[2];
  std::vector<int> Zslot[2];
  int nslot = 0;
};

inline void build_tables(int pmax, Tables& tb) {
  const int P1 = pmax + 1;
  tb.pmax = pmax;
  tb.A.assign((size_t)P1 * P1 * P1 * P1, 0.0);
  tb.AL.assign((size_t)3 * P1 * P1 * P1, 0.0);
  for (int l = 0; l <= pmax; ++l)
    for (int lp = 0; lp <= pmax; ++lp)
      for (int am = 0; am <= std::min(l, lp); ++am) {
        const double c = cn(l, am, lp);
        for (int k = am; k <= std::min(l, lp); ++k)
          tb.A[(((size_t)l * P1 + lp) * P1 + am) * P1 + k] = c * clmk(l, am, k, lp);
        // Laplace limits of the scaled Yukawa translations
        const size_t o = ((size_t)l * P1 + lp) * P1 + am;
        if (lp >= l)  // M2M keeps k = l
          tb.AL[0 * (size_t)P1 * P1 * P1 + o] = c * clmk(l, am, l, lp) * dfact(2 * lp - 1) / (dfact(2 * l - 1) * dfact(2 * lp + 1));
        double s = 0.0;  // M2L keeps every k
        for (int k = am; k <= std::min(l, lp); ++k)
          s += clmk(l, am, k, lp) * dfact(2 * l + 2 * lp - 2 * k - 1) * ((k % 2) ? -1.0 : 1.0);
        tb.AL[1 * (size_t)P1 * P1 * P1 + o] = c * ((l % 2) ? -1.0 : 1.0) * s / (dfact(2 * lp + 1) * dfact(2 * l - 1));
        if (l >= lp)  // L2L keeps k = l'
          tb.AL[2 * (size_t)P1 * P1 * P1 + o] = c * clmk(l, am, lp, lp) * (((l + lp) % 2) ? -1.0 : 1.0) * dfact(2 * l + 1) /
                                                 (dfact(2 * lp + 1) * dfact(2 * l + 1));
      }
  tb.Aoff.assign((size_t)P1 * P1 * P1, 0);
  tb.Ap.clear();
  for (int l = 0; l <= pmax; ++l)
    for (int lp = 0; lp <= pmax; ++lp)
      for (int am = 0; am <= std::min(l, lp); ++am) {
        tb.Aoff[((size_t)l * P1 + lp) * P1 + am] = (int)tb.Ap.size();
        for (int k = am; k <= std::min(l, lp); ++k) tb.Ap.push_back(tb.A[(((size_t)l * P1 + lp) * P1 + am) * P1 + k]);
      }
  {
    const int npair = P1 * (P1 + 1) / 2;
    tb.nslot = 64 * ((npair + 63) / 64);
    const int R = tb.nslot / 64;
    for (int kern = 0; kern < 2; ++kern) {
      std::vector<int> off(npair);
      std::vector<double> work(npair);
      for (int d = 0; d < 2; ++d) tb.Z[kern][d].clear();
      if (kern == 0)
        for (int d = 0; d < 2; ++d) tb.Zlvl[d].clear();
      for (int lo = 0; lo <= pmax; ++lo)
        for (int am = 0; am <= lo; ++am) {
          const int u = lo * (lo + 1) / 2 + am;
          off[u] = (int)tb.Z[kern][0].size();
          work[u] = 0.0;
          for (int li = am; li <= pmax; ++li) {
            const int kmax = std::min(lo, li);
            for (int d = 0; d < 2; ++d) {
              const int l = d ? lo : li, lp = d ? li : lo;
              if (kern == 0) {  // (-1)^k folded in: the kernel sums against k_n(z) z^n
                for (int k = am; k <= kmax; ++k) {
                  tb.Z[kern][d].push_back(tb.A[(((size_t)l * P1 + lp) * P1 + am) * P1 + k] * ((k & 1) ? -1.0 : 1.0));
                  tb.Zlvl[d].push_back(tb.A[(((size_t)l * P1 + lp) * P1 + am) * P1 + k]);
                }
              } else {
                tb.Z[kern][d].push_back(tb.AL[1 * (size_t)P1 * P1 * P1 + ((size_t)l * P1 + lp) * P1 + am]);
              }
            }
            work[u] += kern == 0 ? 3.0 * (kmax - am + 1) + 7.0 : 7.0;
          }
        }
      std::vector<int> order(npair);
      std::iota(order.begin(), order.end(), 0);
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
      std::vector<double> load(64, 0.0);
      std::vector<int> used(64, 0);
      tb.Zslot[kern].assign(2 * (size_t)tb.nslot, -1);
      for (int u : order) {
        int best = -1;
        for (int ln = 0; ln < 64; ++ln)
          if (used[ln] < R && (best < 0 || load[ln] < load[best])) best = ln;
        const int slot = best + 64 * used[best]++;
        load[best] += work[u];
        int lo = 0;
        while ((lo + 1) * (lo + 2) / 2 <= u) ++lo;
        tb.Zslot[kern][2 * slot] = (lo << 8) | (u - lo * (lo + 1) / 2);
        tb.Zslot[kern][2 * slot + 1] = off[u];
      }
    }
  }
  // J_l[m', m] = sum_n w_n Y_lm'(s_n) Y_lm(Q^T s_n), Q = rotation by +90 degrees about x,
  // exact for a Lebedev rule of degree >= 2 pmax.
  const auto* rule = host::lebedev_rule_min_degree(2 * pmax);
  const int L = P1 * P1;
  tb.Joff.assign(P1 + 1, 0);
  for (int l = 0; l <= pmax; ++l) tb.Joff[l + 1] = tb.Joff[l] + (2 * l + 1) * (2 * l + 1);
  tb.J.assign(tb.Joff[P1], 0.0);
  std::vector<double> Y(L), YQ(L);
  for (int n = 0; n < rule->n; ++n) {
    const double* s = rule->xyzw + 4 * n;
    host::solid_harmonics<double>(pmax, s[0], s[1], s[2], Y.data());
    // Q^T s for Q = Rx(90): Q = [[1,0,0],[0,0,-1],[0,1,0]], Q^T s = (s_x, s_z, -s_y)
    host::solid_harmonics<double>(pmax, s[0], s[2], -s[1], YQ.data());
    for (int l = 0; l <= pmax; ++l)
      for (int a = -l; a <= l; ++a)
        for (int b = -l; b <= l; ++b)
          tb.J[tb.Joff[l] + (a + l) * (2 * l + 1) + (b + l)] += s[3] * Y[host::lmi(l, a)] * YQ[host::lmi(l, b)];
  }
  // entries that vanish by symmetry come out of the quadrature at rounding level
  for (double& v : tb.J)
    if (std::fabs(v) < 1e-12) v = 0.0;
  tb.Jval.clear();
  tb.Jrow.assign((size_t)4 * L, 0);
  for (int mat = 0; mat < 2; ++mat)
    for (int l = 0; l <= pmax; ++l) {
      const int w = 2 * l + 1;
      for (int a = 0; a < w; ++a) {
        std::vector<int> cols;
        for (int b = 0; b < w; ++b) {
          const double v = mat == 0 ? tb.J[tb.Joff[l] + a * w + b] : tb.J[tb.Joff[l] + b * w + a];
          if (v != 0.0) cols.push_back(b);
        }
        if (cols.empty()) cols.push_back(0);
        // one run of step 2 when every nonzero has the parity of the first (accidental
        // zeros inside the run are stored), else the dense row
        int step = 2;
        for (int b : cols)
          if ((b - cols[0]) % 2) step = 1;
        const int first = step == 2 ? cols.front() : 0, last = step == 2 ? cols.back() : w - 1;
        cols.clear();
        for (int b = first; b <= last; b += step) cols.push_back(b);
        const size_t t = (size_t)l * l + a;
        tb.Jrow[2 * (mat * L + t)] = (int)tb.Jval.size();
        tb.Jrow[2 * (mat * L + t) + 1] = (l * l + cols[0]) | ((int)cols.size() << 12) | (step << 20);
        for (int b : cols) tb.Jval.push_back(mat == 0 ? tb.J[tb.Joff[l] + a * w + b] : tb.J[tb.Joff[l] + b * w + a]);
      }
    }
  const int G = (L + 63) / 64;
  std::vector<int> K(G, 0);
  tb.jpad_ok = G <= 7;
  for (int mat = 0; mat < 2; ++mat)
    for (int t = 0; t < L; ++t) {
      const int d = tb.Jrow[2 * (mat * L + t) + 1], cnt = (d >> 12) & 255, st = d >> 20;
      if (cnt > 1 && st != 2) tb.jpad_ok = false;
      K[t / 64] = std::max(K[t / 64], cnt);
    }
  tb.jpad_kpack = 0;
  tb.Jpad.clear();
  if (tb.jpad_ok) {
    for (int g = 0; g < G; ++g) {
      K[g] += K[g] & 1;
      if (K[g] > 14) tb.jpad_ok = false;
      tb.jpad_kpack |= K[g] << (4 * g);
    }
    for (int mat = 0; mat < 2; ++mat)
      for (int g = 0; g < G; ++g)
        for (int k = 0; k < K[g]; ++k)
          for (int lane = 0; lane < 64; ++lane) {
            const int t = 64 * g + lane;
            double v = 0.0;
            if (t < L) {
              const int off = tb.Jrow[2 * (mat * L + t)], cnt = (tb.Jrow[2 * (mat * L + t) + 1] >> 12) & 255;
              if (k < cnt) v = tb.Jval[off + k];
            }
            tb.Jpad.push_back(v);
          }
  }
}

}  // namespace fmm
}  // namespace ddlpb
