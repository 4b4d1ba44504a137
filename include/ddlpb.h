/*
 * ddlpb.h -- C ABI of the MI355X (gfx950) ddLPB library.
 *
 * The library computes the discrete ddLPB electrostatic solvation energy of a
 * union of atomic spheres, its adjoint solution and the analytical solvation
 * forces (Jha, Nottoli, Mikhalev, Quan, Stamm: "Linear scaling computation of
 * forces for the domain-decomposition linear Poisson--Boltzmann method").
 * Every numerical step runs in HIP kernels on the current GPU.
 *
 * Problem statement (Sec. 1 and Sec. 2.1): point charges q_j at the centres
 * x_j of balls of radius r_j; permittivity eps_in inside the union of balls,
 * eps_out and Debye--Hueckel screening constant kappa outside.  Discretisation
 * (Sec. 2.2): real spherical harmonics up to degree lmax on every sphere and
 * a Lebedev rule with n_lebedev points.  Units: Angstrom, elementary charge;
 * energies in e^2/Angstrom, forces in e^2/Angstrom^2 (Coulomb constant 1).
 *
 * Conventions common to every call:
 *   - Return value 0 = success, a negative DDLPB_E* code on error.  No C++
 *     exception crosses the boundary.  On error, outputs are left unwritten.
 *   - Pointers named *_host are host memory owned by the caller; the library
 *     copies what it needs before returning.  Results are on the host when a
 *     call returns.
 *   - A context is used by one host thread at a time; different contexts are
 *     independent (no global mutable state besides per-device constant tables).
 */
#ifndef DDLPB_H
#define DDLPB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define DDLPB_OK 0
#define DDLPB_EINVAL (-1)   /* invalid argument (sizes, non-finite values, unsupported grid) */
#define DDLPB_EGEOM (-2)    /* coincident sphere centres (distance < 1e-12 A) */
#define DDLPB_ENOMEM (-3)   /* device or host allocation failed / workspace too small */
#define DDLPB_EDEVICE (-4)  /* a HIP call failed */
#define DDLPB_ENOCONV (-5)  /* iterative solver did not reach the tolerance in max_iter, or
                               stagnated (a restart cycle reduced the residual < 10 %) */
#define DDLPB_ESTATE (-6)   /* call order violated (e.g. forces before adjoint) */

typedef struct ddlpb_ctx ddlpb_ctx;

/* Per-solve statistics (ddlpb_get_stats). */
typedef struct {
  int32_t iters_primal;      /* GMRES iterations of the last primal solve */
  int32_t iters_adjoint;     /* GMRES iterations of the last adjoint solve */
  double resid_primal;       /* final relative residual ||g - L X|| / ||g|| */
  double resid_adjoint;      /* final relative residual ||Q - L^T X_adj|| / ||Q|| */
  double ms_setup;           /* device setup (grid fields, tables, tree) */
  double ms_rhs;             /* right-hand side g */
  double ms_primal;          /* primal solve */
  double ms_adjoint;         /* adjoint solve */
  double ms_forces;          /* force assembly */
  int64_t n_cap_pairs;       /* (i, n, j) triples with omega_ij(x_i^n) > 0 */
  int64_t n_active_points;   /* grid points with chi^eta_i(x_i^n) > 0 */
  int64_t n_near_pairs;      /* sphere pairs evaluated directly in the single layer */
  int64_t n_m2l;             /* multipole-to-local translations per field evaluation */
  int32_t fmm_order;         /* 0 = direct summation */
  int32_t precision;         /* 0 = FP64, 1 = mixed */
  int32_t refinements;       /* mixed paths: FP64 iterations (precision 1) or refinement steps (2) */
  int32_t fmm_order_below_lmax; /* 1 if 0 < fmm_order < lmax (forces inaccurate, Sec. 4.1.2) */
} ddlpb_stats;

/*
 * ddlpb_setup -- validate inputs, copy them and analyse the geometry.
 *   n_atoms     M >= 1
 *   centers     [M][3] row-major, host, Angstrom
 *   radii       [M] host, Angstrom, > 0
 *   charges     [M] host, e
 *   eps_in, eps_out > 0; kappa > 0 (1/Angstrom)
 *   lmax        0..10, maximal harmonic degree on every sphere (Sec. 2.2)
 *   n_lebedev   one of 6, 14, 26, 38, 50, 74, 86, 110, 146, 170, 194, 230, 266, 302,
 *               350, 434, 590, 770, 974 and of quadrature degree >= 2*lmax + 2 (the
 *               projection through the switching function needs the margin: lmax 8
 *               on 110 points, degree 17, is rejected)
 *   fmm_order   0 = direct O(M^2) single layer and vacuum field;
 *               p = lmax+1..16: fast multipole method of order p (Appendix) for
 *               the single layer (screened Coulomb) and the vacuum (Coulomb)
 *               field; p must exceed lmax because the force terms need the
 *               adjoint field at degree lmax+1
 *   out         receives the new context
 * Defaults (change with ddlpb_set_option before the first solve): eta = 0.05,
 * FP64, restart 100, preconditioner = 6 GMRES steps on L_AB each preconditioned
 * by 1 Jacobi sweep (flexible outer GMRES), precond_delta -1 (off), max_iter 400,
 * theta 0.6.
 * Errors: EINVAL, EGEOM, ENOMEM.  Device memory is allocated lazily at the
 * first solve unless a workspace is bound.
 */
int ddlpb_setup(int32_t n_atoms, const double* centers, const double* radii, const double* charges,
                double eps_in, double eps_out, double kappa, int32_t lmax, int32_t n_lebedev,
                int32_t fmm_order, ddlpb_ctx** out);

/*
 * ddlpb_solve -- primal solve L X = g (Sec. 2.2 block system) to relative
 * residual tol, then the energy E_s = 1/2 sum_j q_j psi_r(x_j) (Sec. 3 energy
 * equation), written to *energy_out (host, e^2/Angstrom).
 * Errors: ENOCONV (best iterate kept, energy written), EDEVICE, ENOMEM.
 */
int ddlpb_solve(ddlpb_ctx* ctx, double tol, double* energy_out);

/*
 * ddlpb_adjoint -- adjoint solve L^T X_adj = Q (Sec. 3 adjoint system) to
 * relative residual tol.  Requires a prior ddlpb_solve (else ESTATE).
 */
int ddlpb_adjoint(ddlpb_ctx* ctx, double tol);

/*
 * ddlpb_forces -- analytical forces F = -grad_{x_k} E_s (Sec. 3.1, contracted
 * with X_adj as in the Sec. 3 force equation), written to forces_out [M][3]
 * (host, e^2/Angstrom^2).  Requires a prior ddlpb_adjoint (else ESTATE).
 */
int ddlpb_forces(ddlpb_ctx* ctx, double* forces_out);

/*
 * ddlpb_eval_potentials -- the reaction and extended potentials at arbitrary
 * points from the solved expansions (Sec. 2: psi_r(x) = sum_lm X_r,ilm
 * (|x - x_i|/r_i)^l Y_lm and psi_e(x) = sum_lm X_e,ilm i_l(kappa|x - x_i|) /
 * i_l(kappa r_i) Y_lm for x in the ball i), with their gradients; -grad psi_r is
 * the reaction field, e.g. for coupling to QM or polarisable models.
 *   points  [n][3] host, Angstrom
 *   spheres [n] host: the ball whose expansion each point uses (0..M-1), or NULL
 *           for the ball with the smallest |x - x_i| / r_i (a ball containing
 *           the point when there is one; found by scanning all M spheres)
 *   out     [n][8] host, caller-owned: psi_r, psi_e, d psi_r / dx,y,z,
 *           d psi_e / dx,y,z (e / Angstrom, e / Angstrom^2)
 * Requires a prior ddlpb_solve.  Allocates a temporary device block of 92 bytes
 * per point.  Errors: EINVAL (n < 0, null pointers, non-finite points, ball index
 * out of range), ESTATE, ENOMEM.
 */
int ddlpb_eval_potentials(ddlpb_ctx* ctx, int32_t n_points, const double* points, const int32_t* spheres,
                          double* out);

/*
 * ddlpb_eval_potentials_noalloc -- ddlpb_eval_potentials for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * hosts that forbid hipMalloc).  Same arguments, results and errors, and the same
 * kernels; the points, balls and results are staged in a fixed array of the
 * library's device memory instead of a temporary block, so a call allocates
 * nothing.  At most DDLPB_NOALLOC_MAX_POINTS points per call (EINVAL beyond).
 * The array is per GPU (92 bytes per point, 6 MB) and is held from the first call
 * on a GPU until the process ends; every call on that GPU shares it, so calls that
 * overlap on one GPU (other threads, other streams) race and must be serialised
 * by the caller.  No entry needs to start at zero: each call writes every staged
 * value before reading it.
 */
#define DDLPB_NOALLOC_MAX_POINTS 65536
int ddlpb_eval_potentials_noalloc(ddlpb_ctx* ctx, int32_t n_points, const double* points,
                                  const int32_t* spheres, double* out);

/*
 * ddlpb_charge_gradient -- dE_s/dq_k for every atom, written to dedq_out [M]
 * (host, e/Angstrom).  The adjoint solution gives the derivative with respect to
 * any parameter of the system at no further solve (Sec. 3, adjoint method):
 * dE/dq_k = 1/2 X_r,k00 / sqrt(4 pi) + 1/2 <X_adj, dg/dq_k>, where g depends on
 * q_k through psi_0 and d_n psi_0 at the grid points.  Since E is quadratic in q,
 * sum_k q_k dE/dq_k = 2 E.  Requires a prior ddlpb_adjoint (else ESTATE).
 * Errors: EINVAL, ESTATE, EDEVICE.
 */
int ddlpb_charge_gradient(ddlpb_ctx* ctx, double* dedq_out);

/*
 * ddlpb_dielectric_gradient -- dE_s/d eps_in and dE_s/d eps_out, written to
 * dedeps_out [2] (host, e^2/Angstrom per unit of permittivity), from the same adjoint
 * solution (Sec. 3: dE/d lambda = 1/2 <X_adj, dg/d lambda - (dL/d lambda) X> for any
 * parameter lambda).  The permittivities enter the right-hand side through psi_0
 * (~ 1/eps_in) and the normal-derivative term (~ 1/eps_out), and the operator only
 * through eps_in/eps_out in C1, so one extra single-layer product (C1 X_r) and three
 * dot products suffice; eps_in dE/d eps_in + eps_out dE/d eps_out = -E.
 * Requires a prior ddlpb_adjoint (else ESTATE).  Errors: EINVAL, ESTATE, EDEVICE.
 */
int ddlpb_dielectric_gradient(ddlpb_ctx* ctx, double* dedeps_out);

/*
 * ddlpb_radius_gradient -- dE_s/dr_j for every atom, written to dedr_out [M] (host,
 * e^2/Angstrom^2), from the same adjoint solution (Sec. 3: dE/d lambda =
 * 1/2 <X_adj, dg/d lambda - (dL/d lambda) X> for any parameter lambda).  The radius
 * moves the sphere's grid points radially (x_j^n = x_j + r_j s_n), enters the
 * switching function through |x - x_j| / r_j (Sec. 3.1) and every per-degree
 * normaliser of the sphere's bases and constants (Sec. 2.2: r_j^-l, i_l(kappa r_j),
 * k_l(kappa r_j), C_l^j and the y terms of C1 and C2).  The force intermediates are
 * recomputed (one more far-field pass of each kind with the FMM).  Requires a prior
 * ddlpb_adjoint (else ESTATE).  Errors: EINVAL, ESTATE, EDEVICE.
 */
int ddlpb_radius_gradient(ddlpb_ctx* ctx, double* dedr_out);

/* ddlpb_free -- release the context and any device memory it allocated. NULL is a no-op. */
void ddlpb_free(ddlpb_ctx* ctx);

/*
 * ddlpb_set_option -- set a tuning option before the first solve (else ESTATE
 * for options that change the discrete problem: eta, precision, fmm_order).
 *   "eta"            switching width of chi_eta (Sec. 3.1), 0 < eta <= 1
 *   "precision"      0 = FP64 everywhere.
 *                    1 = mixed: the preconditioner (the Krylov steps on L_AB and
 *                    their Jacobi sweeps) runs the near-field A/B kernels in FP32;
 *                    flexible GMRES (FP64 residual, vectors, orthogonalisation,
 *                    norms) restores the tolerance.  With the FMM at order 12 the
 *                    outer iterations run the multipole-to-local translations
 *                    with an FP32 coefficient vector (option mixed_m2l), and with
 *                    option mixed_near_sl = 1 the near single layer (the directly
 *                    summed sphere pairs of the C part) in FP32 (FP32 per pair,
 *                    FP64 sums); then the FP64 operator's residual b - L x
 *                    decides: flexible GMRES continues on the FP64 operator from x
 *                    until it meets tol (stats.refinements counts those FP64
 *                    iterations of the last solve).
 *                    2 = mixed with FP32 operator: FP64 iterative refinement (FP64
 *                    residual b - L x) around GMRES solves of the correction
 *                    equation in which the near-field kernels (operator and
 *                    sweeps) compute in FP32 (stats.refinements counts the steps).
 *                    In both, Bessel ratios, the FMM translations, the energy and
 *                    the forces stay FP64.  Both need the cap lists (else FP64 is
 *                    used).
 *   "gmres_restart"  outer Krylov subspace size (1..200)
 *   "inner_sweeps"   Jacobi sweeps on L_AB = [A 0; 0 B] used as the innermost
 *                    preconditioner (0..64; Sec. 4 uses L_AB as preconditioner)
 *   "precond_krylov" k > 0: the preconditioner is k GMRES steps on L_AB, each
 *                    preconditioned by the inner_sweeps Jacobi sweeps, and the
 *                    outer method is flexible GMRES (0..64, default 6);
 *                    0: the sweeps alone (then 24 sweeps is a good choice)
 *   "precond_delta"  two-level preconditioner: each outer (flexible) GMRES step
 *                    is preconditioned by inner GMRES steps on P = L_AB + the
 *                    single-layer blocks of sphere pairs with |x_i - x_j| <
 *                    r_i + r_j + delta (Angstrom); < 0 (default) disables it
 *   "inner_iters"    inner GMRES steps on P per outer step (1..200, default 12)
 *   "max_iter"       maximal GMRES iterations per solve
 *   "theta"          FMM acceptance parameter (0 < theta < 1)
 *   "leaf_size"      FMM leaf groups (1..64, default 1): a rejected pair of tree
 *                    nodes of at most this many spheres each interacts sphere by
 *                    sphere in the near field instead of being split further, which
 *                    trades multipole-to-local translations for direct pairs; the
 *                    expansions still start and end at the single spheres.  Set
 *                    before the first solve (else ESTATE).
 *   "solver"         0 (default): GMRES as above; 1: the Jacobi-DIIS scheme of
 *                    Sec. 4, opening (macro-iterations X <- X + L_AB^-1 (g - L X) with DIIS,
 *                    L_AB^-1 by DIIS-accelerated Jacobi micro-iterations, both
 *                    stopping on the relative infinity-norm increment, tol and
 *                    tol/100; FP64; stats report the final relative residual)
 *   "diis_max"       DIIS history length (2..32, default 8; at most
 *                    (gmres_restart - 3) / 4, the histories use the GMRES basis)
 *   "warm_start"     1 (default): solves start from the previous X / X_adj;
 *                    0: every solve starts from zero
 *   "mixed_near_sl"  1: precision 1 with the FMM applies the near single layer
 *                    of the outer iterations in FP32 (see "precision"); 0 (default)
 *   "mixed_m2l"      1 (default): precision 1 with the FMM at order 12 runs the
 *                    screened Coulomb multipole-to-local translations of the outer
 *                    iterations with an FP32 coefficient vector (rotations and
 *                    reduction FP32; translation along z, degree scales and sums
 *                    FP64), followed by the same FP64 residual check; 0: FP64
 *   "cap_lists"      1 (default): the A/B couplings walk per-sphere cap lists (the
 *                    neighbour points inside each sphere) when they fit the
 *                    workspace estimate; 0: always the kernels that find the caps
 *                    on the fly from the neighbour lists (the fallback; FP64 only)
 *   "inner_reorth"   1: the inner Krylov steps of the preconditioner (precond_krylov)
 *                    re-orthogonalise their basis like the outer GMRES; 0 (default):
 *                    one classical Gram-Schmidt pass (the outer flexible GMRES, which
 *                    re-orthogonalises, absorbs the inexact preconditioner)
 *   "mixed_levels"   1: where the FP32-vector M2L runs (mixed_m2l, mixed_forces),
 *                    the order-12 screened Coulomb M2M/L2L level translations run
 *                    with the FP32 vector as well; 0 (default: they cost the mixed
 *                    adjoint more iterations than they save)
 *   "mixed_forces"   1 (default): precision 1 with the FMM computes the single-layer
 *                    terms of ddlpb_forces (near pairs of the field, its gradient
 *                    and the transposed sums) with FP32 pairs and FP64 sums, and
 *                    its order-12 screened Coulomb translations with the FP32
 *                    vector; 0: FP64
 *   "apply_fp32"     1: ddlpb_apply uses the FP32 near-field A/B kernels of the
 *                    mixed preconditioner; 2: the FP32 near single layer of the
 *                    mixed outer iterations (FMM only); 3: the FP32-vector
 *                    multipole-to-local translations (FMM order 12); 0: FP64
 *                    (diagnostic: operator error of the mixed path)
 *   "m2l_waves"      wavefronts per block of the wavefront multipole-to-local
 *                    kernel (0 = chosen from the occupancy calculator; 1, 2, 4,
 *                    8, 16; -1 = the one-node-per-block kernel built on the
 *                    generic translation, a reference for the fast kernels); a
 *                    value other than 0 also turns the lane kernel off
 *   "m2l_lane"       1 (default): at FMM order 12 the multipole-to-local
 *                    translations run one per lane (Appendix translation, unrolled
 *                    for order 12); 0: the wavefront kernel
 *   "level_lane"     at FMM order 12 with the screened Coulomb kernel, the tree
 *                    levels of at least this many nodes (default 1024) run their
 *                    multipole-to-multipole and local-to-local translations one
 *                    node per lane (same Appendix translation); smaller levels, and
 *                    0, take the wavefront-per-node kernels
 *   "near_lane"      1 (default): for lmax <= 8 the near-field A/B couplings
 *                    (Sec. 2.2, A_ij and B_ij) run one neighbour cap per lane,
 *                    grouped by the sphere whose basis functions are evaluated;
 *                    0: the cap-list kernels (always used for lmax > 8).  Set
 *                    before the first solve (else ESTATE).
 *   "near_incore"    1: with near_lane, the harmonics and radial ratios of every
 *                    cap are computed once per geometry and kept in device memory
 *                    ((lmax+1)^2 + lmax + 1 doubles per cap, allocated by the
 *                    library outside the workspace; ENOMEM if it does not fit)
 *                    instead of being recomputed in every application (the
 *                    paper's "incore" variant of the sparse products, Sec. 4).
 *                    Set before the first solve (else ESTATE).
 *   "kernel_timing"  1: record the device time of every kernel launch with HIP
 *                    events on the context's stream (see ddlpb_kernel_times)
 * Errors: EINVAL (unknown key or value out of range), ESTATE.
 */
int ddlpb_set_option(ddlpb_ctx* ctx, const char* key, double value);

/*
 * ddlpb_update_centers -- new conformation of the same molecule (same radii,
 * charges and parameters); [M][3] host.  Neighbour lists, caps and (with the
 * FMM) the tree and its interaction lists are rebuilt for the new centres; X
 * and X_adj are kept as initial guesses of the next solves.  Errors: EINVAL,
 * EGEOM, ENOMEM (a bound workspace too small for the new lists).
 */
int ddlpb_update_centers(ddlpb_ctx* ctx, const double* centers);

/*
 * Device memory and stream binding (lets a framework such as PyTorch own them).
 * ddlpb_workspace_bytes: bytes of device memory the context needs for its
 *   current geometry and options (also the HBM footprint used for admission).
 * ddlpb_bind_workspace: use [dev, dev+bytes) (device pointer, 256-byte aligned)
 *   instead of allocating; the caller keeps it alive until ddlpb_free or the
 *   next bind.  ENOMEM if bytes < ddlpb_workspace_bytes.
 * ddlpb_set_stream: enqueue all work on this hipStream_t (NULL = default stream).
 */
size_t ddlpb_workspace_bytes(const ddlpb_ctx* ctx);
int ddlpb_bind_workspace(ddlpb_ctx* ctx, void* dev, size_t bytes);
int ddlpb_set_stream(ddlpb_ctx* ctx, void* hip_stream);

/*
 * Per-kernel device time (when the option "kernel_timing" is 1), accumulated
 * since the context was created or since ddlpb_kernel_times_reset.
 * ddlpb_kernel_times: entry idx (0-based) -> name (>= 64 bytes), total ms,
 *   number of launches and the algorithmic work (flops) those launches did;
 *   EINVAL when idx is past the last kernel.
 */
int ddlpb_kernel_times(ddlpb_ctx* ctx, int32_t idx, char* name_out, double* ms, int64_t* launches, double* work);
int ddlpb_kernel_times_reset(ddlpb_ctx* ctx);

/* ddlpb_get_stats -- copy the statistics of the last calls. */
int ddlpb_get_stats(const ddlpb_ctx* ctx, ddlpb_stats* out);

/* ddlpb_strerror -- static description of an error code. */
const char* ddlpb_strerror(int code);

/*
 * Inspection entry points (tests and diagnostics).  All buffers are host memory.
 * ddlpb_get_grid:     f^i(x_i^n) and chi^eta_i(x_i^n) (Sec. 3.1), each [M][N].
 * ddlpb_get_solution: X and X_adj (Sec. 2.2 and Sec. 3), each [2][M][L],
 *                     L = (lmax+1)^2, index l*l+l+m; either may be NULL.
 * ddlpb_get_rhs:      g = (G0 + F0, F0) (Sec. 2.2), [2][M][L].
 * ddlpb_apply:        Y = L X (transpose 0) or L^T X (transpose 1) with the
 *                     context's operators (FMM if fmm_order > 0), [2][M][L].
 */
int ddlpb_get_grid(ddlpb_ctx* ctx, double* f_out, double* u_out);
int ddlpb_get_solution(ddlpb_ctx* ctx, double* x_out, double* xadj_out);
int ddlpb_get_rhs(ddlpb_ctx* ctx, double* g_out);
int ddlpb_apply(ddlpb_ctx* ctx, int32_t transpose, const double* x_in, double* y_out);

#ifdef __cplusplus
}
#endif
#endif /* DDLPB_H */
