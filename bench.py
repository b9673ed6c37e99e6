"""Benchmark: unknowns/s solved to 1e-10 relative residual by tweed multigrid on
the 4097^2 wall-clustered grid (tanh clustering, g = 3, V(2,2), FP64), plus the
smoother half-sweep's achieved HBM bandwidth against the MI355X roofline.

One step = one mg_solve from u = 0 to ||f - L u||_inf / ||f||_inf < 1e-10 on
inputs already resident in HBM.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--extras]
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(f, cycles_gpu):
    """The FP64 oracle on this host, single-threaded: the first three V(2,2)
    cycles at full size from u = 0 (a bounded sample of about 15 s), their
    mean time per cycle scaled to the cycle count the GPU solve needs."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O

    x = O.coords(*STRETCH, N_CELLS)
    H = O.Hierarchy([x, x], "tweed")
    ncyc = 3
    u = np.zeros_like(f)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(ncyc):
            u = H.cycle(u, f, 2, 2)
        dt = (time.perf_counter() - t0) / ncyc
    unknowns = (N_CELLS - 1) ** 2
    return {"value": unknowns / (dt * cycles_gpu), "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {ncyc} V(2,2) tweed cycles at 4097^2 from u=0 ({ncyc * dt:.1f} s on one thread, "
                      f"{dt:.2f} s per cycle), scaled to the {cycles_gpu} cycles the solve takes"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", action="store_true", help="also time the other workloads")
    ap.add_argument("--sweep-reps", type=int, default=20)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy (counter calibration)")
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
    traffic = None
    if os.path.exists(PMC_FILE):
        try:
            traffic = json.load(open(PMC_FILE)).get("bytes_per_launch")
        except Exception:  # a malformed profile summary leaves traffic unknown
            traffic = None

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
                   "half_sweep_ms": half_ms},
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


def timed_solve(s, f, torch, reps=3, bc=None, tol=TOL):
    u = s.zeros()
    s.solve(f, bc, tol=tol, u=u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, st = s.solve(f, bc, tol=tol, u=u)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps, st


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
