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
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (= matrix) peak
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (= matrix) peak
PRECISION = {"fp64": 0, "mixed": 1, "mixed-refine": 2}


def measured_traffic(kernel, atoms):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (profiles/), if it was taken on this workload with the current kernel source."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2203_00552_amd", "csrc", "fmm.hpp")
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()[:12]
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if not line.startswith("traffic_bytes_per_launch:"):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[2:])
            if (line.split()[1] == kernel and int(kv["atoms"]) == atoms and kv["fmm_hpp_sha1"] == sha):
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
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-atoms", type=int, default=100)
    p.add_argument("--serve-requests", type=int, default=64,
                   help="requests of the serving run (0: skip); the full workload has 512")
    p.add_argument("--serve-slots", type=int, default=8)
    p.add_argument("--serve-precision", choices=["fp64", "mixed", "mixed-refine"], default="mixed",
                   help="precision of the serving requests (the serving workload is specified in mixed precision)")
    p.add_argument("--option", action="append", default=[], metavar="KEY=VALUE",
                   help="extra context option (ddlpb_set_option), repeatable")
    p.add_argument("--copy-probe", type=int, default=0, metavar="GIB",
                   help="only copy GIB GiB device to device three times and exit: the calibration run "
                        "of the HBM traffic counters")
    return p.parse_args()


def cpu_baseline(args):
    """The oracle (plain FP64 C++/OpenMP, direct sums) on a bounded sample of the same
    generator: full energy + forces of a small cluster, reported as atoms/s."""
    import oracle
    from paper_2203_00552_amd import inputs
    n = args.cpu_sample_atoms
    x, r, q = inputs.lattice_cluster(n, seed=args.seed)
    P = oracle.Problem(x, r, q, lmax=args.lmax, n_lebedev=args.nleb)
    t0 = time.perf_counter()
    P.solve("gmres", tol=args.tol)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n / dt, "unit": "atoms/s", "cores": cores, "kind": "oracle",
            "sample": f"{n}-atom cluster of the same generator, lmax {args.lmax}, {args.nleb} points, "
                      f"tol {args.tol:g}, full energy+forces in {dt:.1f} s (direct O(M^2) sums: the "
                      f"oracle's cost per atom grows linearly with M)"}


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
    out = latency_summary(res, span)
    out.update({"slots": args.serve_slots, "max_in_flight": server.max_in_flight, "rate_per_s": 200.0,
                "precision": args.serve_precision, "sizes": "log-uniform [50, 20000] atoms"})
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not supported",
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
    from paper_2203_00552_amd import Context, inputs

    fmm = args.fmm_order if args.fmm_order is not None else 12
    atoms = args.atoms if args.atoms is not None else 100000
    x, r, q = inputs.lattice_cluster(atoms, seed=args.seed)
    log(f"generated {atoms} atoms")
    torch.cuda.init()
    ctx = Context(x, r, q, eps_in=1.0, eps_out=78.54, kappa=0.104, lmax=args.lmax, n_lebedev=args.nleb,
                  fmm_order=fmm, options=dict({"warm_start": 0, "kernel_timing": 1,
                                               "precision": PRECISION[args.precision]},
                                              **{kv.split("=")[0]: float(kv.split("=")[1]) for kv in args.option}),
                  torch_workspace=True)
    log("context set up")

    def step():
        ctx.update_centers(x)
        E = ctx.solve(args.tol, allow_noconv=True)
        ctx.adjoint(args.tol, allow_noconv=True)
        F = ctx.forces()
        return E, F

    for i in range(args.warmup):
        E, _ = step()
        log(f"warmup step {i} done, E = {E:.10g}")
    ctx.kernel_times_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        E, F = step()
        log(f"timed step {i} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.stats()
    kt = ctx.kernel_times()
    # dominant kernel (entries named pass_* time whole FMM passes, not one kernel)
    name, (ms, nl, work) = max(((k, v) for k, v in kt.items() if not k.startswith("pass_")),
                               key=lambda kv: kv[1][0])
    # only the near-field A/B kernels have FP32 instances (mixed modes); the FMM is FP64
    fp32_kernel = args.precision != "fp64" and name in ("apply_LX", "apply_LTZ")
    peak = PEAK_FP32_TFLOPS if fp32_kernel else PEAK_FP64_TFLOPS
    achieved = work / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
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
                               f"points, tol {args.tol:g}, " + (f"FMM p={fmm}" if fmm else "direct sums"),
                   "atoms": atoms, "lmax": args.lmax, "n_lebedev": args.nleb, "fmm_order": fmm,
                   "precision": args.precision, "tol": args.tol,
                   "options": {kv.split("=")[0]: float(kv.split("=")[1]) for kv in args.option}},
        "roofline": {"bound": "alu", "kernel": name, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(name, atoms) if args.precision == "fp64" else None,
                     "launches_per_step": nl / args.steps,
                     "kernel_ms_per_step": ms / args.steps},
        "energy": E, "iters": [st["iters_primal"], st["iters_adjoint"]],
        "phase_ms": {k: st[k] for k in ("ms_rhs", "ms_primal", "ms_adjoint", "ms_forces")},
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in sorted(kt.items(), key=lambda kv: -kv[1][0])},
    }
    ctx.close()
    if args.serve_requests > 0:
        log(f"serving run: {args.serve_requests} requests")
        out["serving"] = serving(args)
        log("serving run done")
    if not args.no_cpu_baseline:
        log("oracle sample on the host")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
