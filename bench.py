"""Benchmark: unknowns/s solved to 1e-10 relative residual by tweed multigrid on
the 4097^2 wall-clustered grid (tanh clustering, g = 3, V(2,2), FP64), plus the
smoother half-sweep's achieved HBM bandwidth against the MI355X roofline.

One step = one mg_solve from u = 0 to ||f - L u||_inf / ||f||_inf < 1e-10 on
inputs already resident in HBM.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-refinement] [--extras]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_CELLS = 4096                 # 4097^2 nodes, 4095^2 unknowns
STRETCH = ("tanh_wall", 3.0)
SEED = 1001
TOL = 1e-10
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# algorithmic bytes of one block-relaxation half-sweep per interior unknown
# (FP64): f read at the relaxed colour (8 B x 1/2), u read at the other colour
# (8 B x 1/2), u written at the relaxed colour (8 B x 1/2)
HALF_SWEEP_BYTES_PER_UNKNOWN = 12.0
PMC_FILE = os.path.join(ROOT, "profiles", "tweed_halfsweep_4097_pmc.json")
# the sources of that kernel: the counter summary is valid for them only
PMC_SOURCES = ["paper_2110_08389_amd/csrc/kernels.hip", "paper_2110_08389_amd/csrc/sweep_core.h",
               "paper_2110_08389_amd/csrc/twmg_internal.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    """CPU model and the cores this process may use (the oracle's host)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "cpus_online": os.cpu_count(), "cpus_usable": usable}


def cpu_baseline(f, cycles_gpu):
    """The FP64 oracle on this host: a whole solve of the timed workload (from
    u = 0 until the relative defect is below 1e-10, every cycle and defect
    norm), first on one thread, then on every usable core (its parallel loops
    give the same bits; the cycle counts are checked equal)."""
    import numpy as np

    import oracle as O

    x = O.coords(*STRETCH, N_CELLS)
    H = O.Hierarchy([x, x], "tweed")
    unknowns = (N_CELLS - 1) ** 2
    info = host_info()
    old = O.get_threads()
    legs = {}
    try:
        for nt in (1, info["cpus_usable"] or 1):
            O.set_threads(nt)
            t0 = time.perf_counter()
            _, k, hist, sto = H.solve(np.zeros_like(f), f, tol=TOL)
            dt = time.perf_counter() - t0
            legs[nt] = (dt, k, sto, float(hist[-1]) if k else 0.0)
            log(f"oracle solve on {nt} thread(s): {k} cycles, {dt:.1f} s")
    finally:
        O.set_threads(old)
    dt1, k1, st1, rel1 = legs[1]
    nall = max(legs)
    dtn, kn, _, _ = legs[nall]
    if kn != k1:
        log(f"oracle: {k1} cycles on one thread but {kn} on {nall}")
    return {"value": unknowns / dt1, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"one whole oracle solve of the 4097^2 workload from u=0 to 1e-10 ({k1} V(2,2) cycles, "
                      f"status {st1}, rel residual {rel1:.2e}; the GPU solve takes {cycles_gpu}): {dt1:.1f} s "
                      f"on one thread",
            "all_cores": {"value": unknowns / dtn, "cores": nall, "seconds": dtn, "cycles": kn,
                          "same_cycles_as_one_thread": kn == k1},
            "host": info}


def refinement_record(pkg, inputs, torch, dev, reps=3):
    """The centre-clustered 2049^2 workload (sinh, b = 4), wireframe W(2,2) to
    1e-10: plain FP64 against FP32 cycles inside FP64 refinement on the same
    GPU, with the refined solution's error against the FP64 one (whose
    iterates match the FP64 oracle's to 1e-12 in the parity tests)."""
    n = 2048
    f = torch.tensor(inputs.normal((n + 1, n + 1), 1002), device=dev)
    rec = {"workload": "2D Poisson 2049^2 nodes, sinh centre clustering b=4 both axes, wireframe W(2,2), "
                       "f ~ N(0,1) seed 1002, tol 1e-10"}
    sol = {}
    for prec in ("fp64", "fp32_ir"):
        s = pkg.Solver([n, n], stretch=("sinh_centre", 4.0), smoother="wireframe", gamma=2, precision=prec,
                       max_cycles=60, device=dev)
        ms, st, u = timed_solve(s, f, torch, reps=reps, keep=True)
        sol[prec] = u
        rec[prec] = {"ms": ms, "cycles": st["cycles"], "status": st["status"], "rel_res": st["rel_res"],
                     "unknowns_per_s": (n - 1) ** 2 / (ms * 1e-3)}
        del s
    a, b = sol["fp64"], sol["fp32_ir"]
    rec["fp32_ir"]["rel_error_vs_fp64"] = float((b - a).abs().max() / a.abs().max())
    rec["fp32_ir_speedup"] = rec["fp64"]["ms"] / rec["fp32_ir"]["ms"]
    return rec


# the other workloads, for profiling runs: (cells per axis, stretching,
# smoother, gamma, batch, seed, distribution, tol)
WORKLOADS = {
    "wireframe2049": ([2048, 2048], ("sinh_centre", 4.0), "wireframe", 2, 1, 1002, "normal", 1e-10),
    "tweed3d257": ([256, 256, 256], ("tanh_wall", 2.5), "tweed", 1, 1, 1003, "uniform", 1e-9),
    "batch1025": ([1024, 1024], ("tanh_wall", 2.5), "tweed", 1, 16, 1004, "normal", 1e-10),
    "adz4097": ([4096, 4096], ("tanh_wall", 3.0), "adz", 1, 1, 1001, "uniform", 1e-10),
}


def profile_workload(pkg, inputs, torch, dev, args):
    """K solves of one of the other workloads from u = 0 (after W warm-up
    solves), timed on the host; prints one JSON line with the time per solve."""
    n, stretch, sm, gamma, B, seed, dist, tol = WORKLOADS[args.workload]
    s = pkg.Solver(n, stretch=stretch, smoother=sm, gamma=gamma, batch=B, precision=args.precision,
                   max_cycles=400, device=dev)
    shape = s.shape(0)
    f = torch.tensor(inputs.uniform(shape, seed) if dist == "uniform" else inputs.normal(shape, seed), device=dev)
    u = s.zeros()
    for _ in range(args.warmup):
        s.solve(f, tol=tol, u=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = s.solve(f, tol=tol, u=u)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / max(args.steps, 1)
    unknowns = B
    for k in n:
        unknowns *= k - 1
    print(json.dumps({"workload": args.workload, "precision": args.precision, "ms_per_solve": ms,
                      "cycles": st["cycles"], "status": st["status"], "rel_res": st["rel_res"],
                      "unknowns_per_s": unknowns / (ms * 1e-3)}), flush=True)


def source_sha(paths):
    import hashlib

    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", action="store_true", help="also time the other workloads")
    ap.add_argument("--sweep-reps", type=int, default=20)
    ap.add_argument("--no-refinement", action="store_true",
                    help="skip the FP64 vs FP32-refinement record of the 2049^2 wireframe workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default=None,
                    help="only time K solves of another workload (for profiling runs; no benchmark line)")
    ap.add_argument("--precision", choices=["fp64", "fp32_ir"], default="fp64")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the solver has no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        # a plain copy of known size: FETCH_SIZE and WRITE_SIZE of its kernel
        # should each read 512 MiB; their ratio to that is the counter scale
        # an elementwise kernel (reads a, writes b once each), not the runtime's
        # copy path; the views start 8 bytes into their buffers, which rules
        # out torch's 32-byte vector accesses, so each lane moves 8 bytes as
        # the solver's kernels do (the counters' scale depends on that)
        n = 64 * 1024 * 1024
        a = torch.ones(n + 1, dtype=torch.float64, device="cuda")[1:]
        b = torch.empty(n + 1, dtype=torch.float64, device="cuda")[1:]
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8}))
        return

    import paper_2110_08389_amd as pkg
    from paper_2110_08389_amd import inputs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.workload:
        profile_workload(pkg, inputs, torch, dev, args)
        return
    t0 = time.perf_counter()
    s = pkg.Solver([N_CELLS, N_CELLS], stretch=STRETCH, smoother="tweed", nu1=2, nu2=2, gamma=1,
                   precision="fp64", max_cycles=100, device=dev)
    setup_s = time.perf_counter() - t0
    log(f"setup {setup_s:.2f} s")
    f_np = inputs.uniform((N_CELLS + 1, N_CELLS + 1), SEED)
    f = torch.tensor(f_np, device=dev)
    u = s.zeros()
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        s.solve(f, tol=TOL, u=u)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = s.solve(f, tol=TOL, u=u)
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / args.steps
    log(f"timed {args.steps} solves: {ms:.3f} ms/solve")
    unknowns = (N_CELLS - 1) ** 2
    st = stats[-1]
    if st["status"] != 0:
        log("solve did not converge:", st)

    # dominant kernel: the finest-level red half-sweep (one launch of
    # k_block_sweep<double,2,256>) on arrays in the solver's device layout,
    # timed with events on the stream the library launches on (the handle's
    # stream = torch's current stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ud, fd = s.to_layout(torch.zeros_like(u)), s.to_layout(f)
    s.half_sweep(ud, fd, 0)
    ev0.record(stream)
    for _ in range(args.sweep_reps):
        s.half_sweep(ud, fd, 0)
    ev1.record(stream)
    torch.cuda.synchronize()
    half_ms = ev0.elapsed_time(ev1) / args.sweep_reps
    alg_bytes = HALF_SWEEP_BYTES_PER_UNKNOWN * unknowns
    achieved = alg_bytes / (half_ms * 1e-3) / 1e9
    # HBM traffic of that kernel from the committed rocprofv3 counter summary,
    # valid only for the kernel sources it was taken with
    traffic = None
    if os.path.exists(PMC_FILE):
        try:
            pmc = json.load(open(PMC_FILE))
            if pmc.get("source_sha") == source_sha(PMC_SOURCES):
                traffic = pmc.get("bytes_per_launch")
            else:
                log("roofline.traffic: the counter summary predates the current kernel sources; reported as null")
        except Exception:  # a malformed profile summary leaves traffic unknown
            traffic = None
    # per-cycle convergence factor of the solve, beside the paper's two-grid
    # figure for tweed with nu = 4 on the tanh c = 3 grid (Table 3)
    hist = st["history"]
    factor = hist[-1] ** (1.0 / len(hist)) if hist else None
    ratios = [hist[0]] + [hist[k] / hist[k - 1] for k in range(1, len(hist))] if hist else []
    refine = None
    if not args.no_refinement:
        log("refinement record (2049^2 wireframe W(2,2)) ...")
        refine = refinement_record(pkg, inputs, torch, dev)

    out = {
        "metric": "unknowns/s solved to 1e-10 rel. residual (tweed MG, 4097^2); sweep HBM GB/s",
        "value": unknowns / (ms * 1e-3),
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: f i.i.d. uniform[-1,1], seed 1001 (numpy PCG64), zero Dirichlet data",
        "config": {"workload": "2D Poisson 4097^2 nodes, tanh wall clustering g=3 both axes, tweed V(2,2), "
                               "full weighting, bilinear prolongation, coarsest 3x3, FP64, tol 1e-10",
                   "cycles": st["cycles"], "rel_res": st["rel_res"], "setup_s": round(setup_s, 3),
                   "half_sweep_ms": half_ms,
                   "convergence": {"mean_factor_per_cycle": factor, "per_cycle": ratios,
                                   "paper_two_grid_rho_tweed_tanh3_nu4": 0.0204,
                                   "note": "paper Table 3 (two-grid, 65^2); the V-cycle factor on 4097^2 is "
                                           "measured on the defect max-norm"}},
        **({"fp32_refinement": refine} if refine else {}),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_block_sweep<double,2,256> (finest-level tweed red half-sweep)",
                     "alg_bytes_per_launch": alg_bytes},
    }
    if args.extras:
        log("extras ...")
        out["extras"] = extras(pkg, inputs, torch, dev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(f_np, st["cycles"])
    print(json.dumps(out), flush=True)


def timed_solve(s, f, torch, reps=3, bc=None, tol=TOL, keep=False):
    u = s.zeros()
    s.solve(f, bc, tol=tol, u=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, st = s.solve(f, bc, tol=tol, u=u)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    return (ms, st, u) if keep else (ms, st)


def extras(pkg, inputs, torch, dev):
    """The other workloads: same GPU, stated final residuals."""
    res = {}
    # the headline grid with the comparison smoothers (checkerboard does not
    # converge on this stretching; it is stopped after 40 cycles)
    f = torch.tensor(inputs.uniform((N_CELLS + 1, N_CELLS + 1), SEED), device=dev)
    for sm, cap in (("checkerboard", 40), ("adz", 60)):
        s = pkg.Solver([N_CELLS, N_CELLS], stretch=STRETCH, smoother=sm, max_cycles=cap, device=dev)
        ms, st = timed_solve(s, f, torch, reps=1)
        log("extras:", sm, st["cycles"], st["status"], f"{ms:.2f} ms")
        res[f"{sm}_4097_V22_fp64"] = {"ms": ms, "cycles": st["cycles"], "status": st["status"],
                                      "rel_res": st["rel_res"], "unknowns_per_s": (N_CELLS - 1) ** 2 / (ms * 1e-3)}
        del s
    n = 2048
    f = torch.tensor(inputs.normal((n + 1, n + 1), 1002), device=dev)
    for prec in ("fp64", "fp32_ir"):
        for gamma in (1, 2):
            s = pkg.Solver([n, n], stretch=("sinh_centre", 4.0), smoother="wireframe", gamma=gamma,
                           precision=prec, max_cycles=60, device=dev)
            ms, st = timed_solve(s, f, torch)
            log("extras:", prec, gamma, st["cycles"], f"{ms:.2f} ms")
            res[f"wireframe_2049_{'V' if gamma == 1 else 'W'}22_{prec}"] = {
                "ms": ms, "cycles": st["cycles"], "status": st["status"], "rel_res": st["rel_res"],
                "unknowns_per_s": (n - 1) ** 2 / (ms * 1e-3)}
            del s
    n = 256
    f = torch.tensor(inputs.uniform((n + 1,) * 3, 1003), device=dev)
    for prec in ("fp64", "fp32_ir"):
        s = pkg.Solver([n, n, n], stretch=("tanh_wall", 2.5), smoother="tweed", precision=prec, max_cycles=400,
                       device=dev)
        ms, st = timed_solve(s, f, torch, reps=1, tol=1e-9)
        log("extras: 3d", prec, st["cycles"], f"{ms:.2f} ms")
        res[f"tweed3d_257_V22_{prec}"] = {"ms": ms, "cycles": st["cycles"], "status": st["status"],
                                          "rel_res": st["rel_res"], "unknowns_per_s": (n - 1) ** 3 / (ms * 1e-3)}
        del s
    n, B = 1024, 16
    f, bc, w = inputs.normal_triplet((B, n + 1, n + 1), 1004)
    s = pkg.Solver([n, n], stretch=("tanh_wall", 2.5), smoother="tweed", batch=B, device=dev)
    ft, bt, wt = (torch.tensor(a, device=dev) for a in (f, bc, w))
    ms, st = timed_solve(s, ft, torch, reps=1, bc=bt)
    lam = s.zeros()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, sta = s.solve_adjoint(wt, tol=TOL, lam=lam)
    s.bc_grad(lam, wt)
    torch.cuda.synchronize()
    msa = 1e3 * (time.perf_counter() - t0)
    res["batch16_1025_forward"] = {"ms": ms, "cycles": st["cycles"], "status": st["status"],
                                   "unknowns_per_s": B * (n - 1) ** 2 / (ms * 1e-3)}
    res["batch16_1025_adjoint_plus_bcgrad"] = {"ms": msa, "cycles": sta["cycles"], "status": sta["status"]}
    return res


if __name__ == "__main__":
    main()
