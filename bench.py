"""Benchmark: ddLPB energy + forces throughput (atoms/s) on one MI355X.

One step = one complete energy + forces evaluation of a synthetic protein-like
cluster already resident on the device: new conformation (grid switching
fields and right-hand side), primal solve, adjoint solve and force assembly,
every solve started from zero.  Prints one JSON line.

Default workload: 100,000-atom jittered-lattice cluster (radii {1.2,1.5,1.7,1.8} A,
charges N(0, 0.3) neutralised), lmax 8, 302 Lebedev points, tolerance 1e-6.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (= matrix) peak
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (= matrix) peak
PRECISION = {"fp64": 0, "mixed": 1, "mixed-refine": 2}


def measured_traffic(kernel, atoms):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summaries
    (profiles/*.md lines "traffic_bytes_per_launch: <label> atoms=<n> src=<file>
    sha1=<12 hex> bytes=<B>"), used only if they were taken on this workload with the
    current source of that kernel."""
    import glob
    import hashlib
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if not line.startswith("traffic_bytes_per_launch:"):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[2:])
            if line.split()[1] != kernel or int(kv.get("atoms", -1)) != atoms or "src" not in kv:
                continue
            src = os.path.join(ROOT, kv["src"])
            if os.path.exists(src) and hashlib.sha1(open(src, "rb").read()).hexdigest()[:12] == kv["sha1"]:
                return float(kv["bytes"])
    return None


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--atoms", type=int, default=None)
    p.add_argument("--lmax", type=int, default=8)
    p.add_argument("--nleb", type=int, default=302)
    p.add_argument("--fmm-order", type=int, default=None)
    p.add_argument("--precision", choices=["fp64", "mixed", "mixed-refine"], default="fp64",
                   help="mixed: FP32 preconditioner sweeps in FGMRES on the FP64 operator; "
                        "mixed-refine: FP32 operator inside FP64 iterative refinement")
    p.add_argument("--tol", type=float, default=1e-6)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--probe-radius", type=float, default=0.0,
                   help="add this to every radius (1.4: solvent-accessible radii, many more caps)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--serve-requests", type=int, default=512,
                   help="requests of the serving run (0: skip); the serving workload has 512")
    p.add_argument("--mixed-steps", type=int, default=1,
                   help="timed steps of the mixed-precision leg (0: skip)")
    p.add_argument("--serve-slots", type=int, default=8)
    p.add_argument("--serve-precision", choices=["fp64", "mixed", "mixed-refine"], default="mixed",
                   help="precision of the serving requests (the serving workload is specified in mixed precision)")
    p.add_argument("--option", action="append", default=[], metavar="KEY=VALUE",
                   help="extra context option (ddlpb_set_option), repeatable")
    p.add_argument("--accuracy", action="store_true",
                   help="only measure the FMM error of the workload against direct sums: one application "
                        "of L and L^T at --atoms (default 100k), energy and forces at --accuracy-atoms")
    p.add_argument("--accuracy-atoms", type=int, default=10000)
    p.add_argument("--copy-probe", type=int, default=0, metavar="GIB",
                   help="only copy GIB GiB device to device three times and exit: the calibration run "
                        "of the HBM traffic counters")
    return p.parse_args()


def physical_cores():
    """Physical cores of the host (lscpu), or None."""
    import subprocess
    try:
        out = subprocess.run(["lscpu", "-p=CORE,SOCKET"], capture_output=True, text=True, timeout=10).stdout
        return len({ln for ln in out.splitlines() if ln and not ln.startswith("#")}) or None
    except Exception:
        return None


def cpu_baseline(args, n_c, n_ab, atoms):
    """The oracle (plain FP64 C++/OpenMP, direct sums, no FMM) on a bounded sample of the
    same workload, scaled to the timed workload: one application of its single-layer
    part (cost ~ M^2: active points x source spheres) and of its sparse A/B part (~ M)
    on a 1,000-atom cluster of the same generator, multiplied by the operator
    applications of one GPU step (n_c single-layer, n_ab A/B products, from the GPU's
    iteration counts) and scaled to `atoms`; plus the full energy + forces of the
    12-atom configuration (dense LU) as a directly measured run."""
    import numpy as np
    import oracle
    from paper_2203_00552_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    x, r, q = inputs.small_cluster(0)
    t0 = time.perf_counter()
    oracle.Problem(x, r, q, lmax=6, n_lebedev=110).solve("dense", tol=1e-8)
    t_small = time.perf_counter() - t0
    n = 1000
    x, r, q = inputs.lattice_cluster(n, seed=args.seed)
    P = oracle.Problem(x, r, q, lmax=args.lmax, n_lebedev=args.nleb)
    X = np.random.default_rng(1).normal(size=(2, n, P.L))
    t0 = time.perf_counter()
    P.apply(X, part="C")
    t_c = time.perf_counter() - t0
    t0 = time.perf_counter()
    P.apply(X, part="AB")
    t_ab = time.perf_counter() - t0
    scale = atoms / n
    seconds = n_c * t_c * scale * scale + n_ab * t_ab * scale
    # the same two applications on one core, at 300 atoms (a child process, so that its
    # OpenMP runtime starts with one thread; it does not touch the GPU)
    n1 = 300
    code = ("import time, numpy as np, oracle\n"
            "from paper_2203_00552_amd import inputs\n"
            f"x, r, q = inputs.lattice_cluster({n1}, seed={args.seed})\n"
            f"P = oracle.Problem(x, r, q, lmax={args.lmax}, n_lebedev={args.nleb})\n"
            f"X = np.random.default_rng(1).normal(size=(2, {n1}, P.L))\n"
            "t0 = time.perf_counter(); P.apply(X, part='C'); t1 = time.perf_counter(); P.apply(X, part='AB')\n"
            "print(t1 - t0, time.perf_counter() - t1)\n")
    one = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=dict(os.environ, OMP_NUM_THREADS="1"),
                         capture_output=True, text=True, timeout=600)
    t1c, t1ab = (float(v) for v in one.stdout.split()[-2:])
    s1 = atoms / n1
    seconds_1 = n_c * t1c * s1 * s1 + n_ab * t1ab * s1
    return {"value": atoms / seconds, "unit": "atoms/s", "cores": threads, "physical_cores": physical_cores(),
            "one_core": {"value": atoms / seconds_1, "unit": "atoms/s", "cores": 1,
                         "sample": f"single-layer apply {t1c:.2f} s and A/B apply {t1ab:.3f} s at {n1} atoms, "
                                   f"scaled the same way: {seconds_1 / 3600:.3g} h per step"},
            "kind": "oracle", "extrapolated": True,
            "sample": f"oracle single-layer apply {t_c:.1f} s and A/B apply {t_ab:.2f} s at 1,000 atoms (same "
                      f"generator, lmax {args.lmax}, {args.nleb} points), scaled to {atoms} atoms by M^2 and M and "
                      f"multiplied by {n_c} single-layer and {n_ab} A/B applications (one GPU step): "
                      f"{seconds / 3600:.3g} h per step; 12-atom energy + forces (dense) {t_small:.2f} s",
            "seconds_per_step": seconds}


def serving(args):
    """Continuous-batching run: Poisson arrivals (mean 200/s), atom counts log-uniform in
    [50, 20000], lmax in {6, 8}, 110 or 302 points, tol 1e-6, energy + forces."""
    from paper_2203_00552_amd import inputs
    from paper_2203_00552_amd.serve import Request, Server, latency_summary, run_arrivals
    spec = inputs.serving_requests(args.serve_requests, rate=200.0, seed=args.seed)
    reqs, times = [], []
    for k, sp in enumerate(spec):
        x, r, q = inputs.lattice_cluster(sp["n"], seed=sp["seed"])
        reqs.append(Request(x, r, q, lmax=sp["lmax"], n_lebedev=sp["n_lebedev"], tol=1e-6,
                            precision=PRECISION[args.serve_precision], rid=k))
        times.append(sp["t"])
    server = Server(slots=args.serve_slots)
    res, span = run_arrivals(server, reqs, times)
    server.close()
    out = latency_summary(res, span, offered_atoms=sum(sp["n"] for sp in spec), arrival_span=times[-1])
    out.update({"slots": args.serve_slots, "max_in_flight": server.max_in_flight, "rate_per_s": 200.0,
                "precision": args.serve_precision, "sizes": "log-uniform [50, 20000] atoms"})
    return out


def accuracy(args):
    """FMM (order p, theta 0.6) against direct sums on the timed workload: relative
    errors (max norm over the largest entry) of L X and L^T X for a seeded X with
    coefficients decaying like the solutions' (exp(-0.4 l)) at --atoms, and of the energy
    and the forces (normwise) of full solves (tol 1e-10) at --accuracy-atoms."""
    import numpy as np
    from paper_2203_00552_amd import Context, inputs
    fmm = args.fmm_order if args.fmm_order is not None else 12
    out = {"fmm_order": fmm, "lmax": args.lmax, "n_lebedev": args.nleb}
    atoms = args.atoms if args.atoms is not None else 100000
    x, r, q = inputs.lattice_cluster(atoms, seed=args.seed)
    L = (args.lmax + 1) ** 2
    decay = np.exp(-0.4 * np.repeat(np.arange(args.lmax + 1), 2 * np.arange(args.lmax + 1) + 1))
    X = np.random.default_rng(5).normal(size=(2, atoms, L)) * decay
    res = {}
    for p in (0, fmm):
        c = Context(x, r, q, lmax=args.lmax, n_lebedev=args.nleb, fmm_order=p)
        t0 = time.perf_counter()
        res[p] = (c.apply(X), c.apply(X, transpose=True), time.perf_counter() - t0)
        c.close()
        log(f"apply at {atoms} atoms, fmm_order {p}: {res[p][2]:.1f} s")
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
    out["operator"] = {"atoms": atoms, "L_rel_err": rel(res[fmm][0], res[0][0]),
                       "LT_rel_err": rel(res[fmm][1], res[0][1]), "seconds_direct": res[0][2]}
    n = args.accuracy_atoms
    x, r, q = inputs.lattice_cluster(n, seed=args.seed)
    ef = {}
    for p in (0, fmm):
        c = Context(x, r, q, lmax=args.lmax, n_lebedev=args.nleb, fmm_order=p)
        E = c.solve(1e-10)
        c.adjoint(1e-10)
        ef[p] = (E, c.forces())
        c.close()
        log(f"energy and forces at {n} atoms, fmm_order {p}: E = {E:.12g}")
    out["energy_forces"] = {"atoms": n, "tol": 1e-10, "energy_direct": ef[0][0], "energy_fmm": ef[fmm][0],
                            "energy_rel_err": abs(ef[fmm][0] / ef[0][0] - 1),
                            "force_rel_err": rel(ef[fmm][1], ef[0][1])}
    print(json.dumps({"accuracy": out}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; runs on more than one GPU are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_probe > 0:
        a = torch.ones(args.copy_probe << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_gib": args.copy_probe, "copies": 3}))
        return
    if args.accuracy:
        accuracy(args)
        return
    from paper_2203_00552_amd import Context, inputs

    fmm = args.fmm_order if args.fmm_order is not None else 12
    atoms = args.atoms if args.atoms is not None else 100000
    x, r, q = inputs.lattice_cluster(atoms, seed=args.seed)
    r = r + args.probe_radius
    log(f"generated {atoms} atoms")
    torch.cuda.init()
    extra = {kv.split("=")[0]: float(kv.split("=")[1]) for kv in args.option}

    def make(precision):
        return Context(x, r, q, eps_in=1.0, eps_out=78.54, kappa=0.104, lmax=args.lmax, n_lebedev=args.nleb,
                       fmm_order=fmm, options=dict({"warm_start": 0, "kernel_timing": 1, "precision": precision},
                                                   **extra), torch_workspace=True)

    def step(ctx):
        # a timed solve that does not reach the tolerance raises (DDLPB_ENOCONV): no
        # unconverged step is ever counted
        ctx.update_centers(x)
        E = ctx.solve(args.tol)
        ctx.adjoint(args.tol)
        return E, ctx.forces()

    def timed(ctx, steps, warmup, label):
        for i in range(warmup):
            E, _ = step(ctx)
            log(f"{label} warmup step {i} done, E = {E:.10g}")
        ctx.kernel_times_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            E, F = step(ctx)
            log(f"{label} timed step {i} done")
        torch.cuda.synchronize()
        return E, F, time.perf_counter() - t0

    ctx = make(PRECISION[args.precision])
    log("context set up")
    E, F, dt = timed(ctx, args.steps, args.warmup, args.precision)
    st = ctx.stats()
    kt = ctx.kernel_times()
    ctx.close()
    # roofline of the three kernels with the most device time (labels pass_* time whole FMM
    # passes, not one kernel); work = the library's count of algorithmic flops per launch
    # (the flops of one translation, cap or pair times the units of the launch), time =
    # HIP events on the context's stream
    fp32_labels = ("apply_LX", "apply_LTZ")  # cap-list kernels: one label for both precisions
    tops = sorted(((k, v) for k, v in kt.items() if not k.startswith("pass_")), key=lambda kv: -kv[1][0])[:3]

    def roof(name, ms, nl, work):
        fp32 = name.endswith("_f32") or (args.precision != "fp64" and name in fp32_labels)
        peak = PEAK_FP32_TFLOPS if fp32 else PEAK_FP64_TFLOPS
        achieved = work / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        return {"bound": "alu", "kernel": name, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": measured_traffic(name, atoms) if args.precision == "fp64" else None,
                "launches_per_step": nl / args.steps, "ms_per_launch": ms / nl if nl else 0.0,
                "flops_per_launch": work / nl if nl else 0.0}

    def roof_mfma(name):
        # the dense table products on the FP64 matrix cores: algorithmic 2 N L flops per
        # row and table (unpadded), against the FP64 matrix peak
        ms, nl, work = kt[name]
        achieved = work / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        return {"bound": "mfma", "kernel": name, "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": measured_traffic(name, atoms) if args.precision == "fp64" else None,
                "launches_per_step": nl / args.steps,
                "ms_per_launch": ms / nl if nl else 0.0, "flops_per_launch": work / nl if nl else 0.0}

    name, (ms, nl, work) = tops[0]
    out = {
        "metric": "energy+forces atoms/sec at 100k atoms, tol 1e-6; served p50/p99 latency",
        "value": atoms * args.steps / dt,
        "unit": "atoms/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"jittered-lattice cluster, {atoms} atoms, lmax {args.lmax}, {args.nleb} Lebedev "
                               f"points, tol {args.tol:g}, " + (f"FMM p={fmm}" if fmm else "direct sums")
                               + (f", radii +{args.probe_radius:g} A" if args.probe_radius else ""),
                   "atoms": atoms, "lmax": args.lmax, "n_lebedev": args.nleb, "fmm_order": fmm,
                   "precision": args.precision, "tol": args.tol, "options": extra},
        "roofline": roof(name, ms, nl, work),
        "roofline_top3": [roof(k, *v) for k, v in tops],
        "roofline_mfma": [roof_mfma(k) for k in ("syn_gemm", "an_gemm") if k in kt],
        "energy": E, "iters": [st["iters_primal"], st["iters_adjoint"]], "cap_pairs": st["n_cap_pairs"],
        "residuals": [st["resid_primal"], st["resid_adjoint"]],
        "phase_ms": {k: st[k] for k in ("ms_rhs", "ms_primal", "ms_adjoint", "ms_forces")},
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in sorted(kt.items(), key=lambda kv: -kv[1][0])},
    }
    if args.mixed_steps > 0 and args.precision == "fp64":
        # the same step in mixed precision (FP32 near-field sweeps in the preconditioner,
        # FP64 outer solver), its speed and its distance from the FP64 results
        mctx = make(PRECISION["mixed"])
        Em, Fm, dtm = timed(mctx, args.mixed_steps, 0, "mixed")
        mst = mctx.stats()
        mkt = mctx.kernel_times()
        mctx.close()
        out["mixed"] = {"value": atoms * args.mixed_steps / dtm, "unit": "atoms/s",
                        "ms_per_step": dtm * 1e3 / args.mixed_steps,
                        "speedup_vs_fp64": (dt / args.steps) / (dtm / args.mixed_steps),
                        "energy_rel_err_vs_fp64": abs(Em - E) / abs(E),
                        "force_rel_err_vs_fp64": float(np.abs(Fm - F).max() / np.abs(F).max()),
                        "iters": [mst["iters_primal"], mst["iters_adjoint"]],
                        "fp64_iters_after_fp32_adjoint": mst["refinements"],
                        "residuals": [mst["resid_primal"], mst["resid_adjoint"]],
                        "kernels_ms_per_step": {k: v[0] / args.mixed_steps
                                                for k, v in sorted(mkt.items(), key=lambda kv: -kv[1][0])[:12]}}
        log("mixed leg done")
    if args.serve_requests > 0:
        log(f"serving run: {args.serve_requests} requests")
        out["serving"] = serving(args)
        log("serving run done")
    if not args.no_cpu_baseline:
        log("oracle sample on the host")
        per = lambda *labels: sum(kt[k][1] for k in labels if k in kt) / args.steps
        n_c = per("sl_near", "sl_near_adjoint", "sl_field", "sl_adjoint")
        n_ab = per("apply_LX", "apply_LTZ", "near_lx", "near_ltz", "near_lx_f32", "near_ltz_f32")
        out["cpu_baseline"] = cpu_baseline(args, n_c, n_ab, atoms)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
