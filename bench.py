"""Benchmark: converged 6-DoF SCP solves per second on one MI355X.

Workload: the throughput Monte Carlo (65,536 instances, K = 30 nodes, FP32, fixed 15 SCP
iterations x 1,000 PIPG iterations, seeded dispersions including inertia and thrust lever
arm), inputs resident in HBM before timing.  A step is one complete batched solve (initial
guess, every discretization, power iteration, PIPG and reference update).  Beside the FP32
headline the same workload is solved by the FP64 path (fewer steps) and reported in the same
line.  Prints one JSON line.

Roofline: the dominant kernel is the subproblem kernel (PIPG).  Its achieved rate is the
algorithmic FP32 work of the PIPG iterations it ran divided by its launch durations,
measured with HIP events recorded on the stream the library launches on.  The CPU baseline
is the FP64 oracle on a bounded, evenly spaced sample of the same workload, run on the host
cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak (packed issue)
NX = 15                           # state entries per node
WORKLOAD = "C4"
WORKLOAD_NAMES = {
    "C1": "Monte Carlo 1,024 x K=20, 15 SCP x 1,000 PIPG iterations, seeded dispersions (seed 1)",
    "C2": "uneven Monte Carlo 16,384 x K in {10,20,30}, early exit (SCP 1e-4, PIPG 1e-5), "
          "widened dispersions (seed 2)",
    "C4": "throughput 65,536 x K=30, 15 SCP x 1,000 PIPG iterations, J and r_T dispersed (seed 4)",
    "F1": "paper's Monte Carlo: 256 runs, r0 ~ U(6,9) x U(3,6) x U(1,2), K=30, at most 25 SCP x "
          "2,500 PIPG iterations, SCP early exit (seed 5)",
    "F1S": "paper's Monte Carlo with the speed bound ||v|| <= 2.5: 256 runs, r0 ~ U(6,9) x "
           "U(3,6) x U(1,2), K=30, at most 25 SCP x 2,500 PIPG iterations, SCP early exit (seed 5)",
    "F2": "paper's Monte Carlo with the reaction-control torque (n_u = 7): 256 runs, r0 ~ "
          "U(6,9) x U(3,6) x U(1,2), K=30, at most 25 SCP x 2,500 PIPG iterations, SCP early "
          "exit (seed 5)",
}
SWEEP_SIZES = (1, 4, 16, 64, 256, 1024, 4096, 16384, 65536)


def pipg_flops_per_iter(K, n_u=4):
    """Algorithmic flops of one PIPG_custom iteration of one instance with K nodes and n_u
    controls per node: the block products A^-_k, B^-_k, B^+_k and their transposes (A^-_k has
    196 free entries: its mass row and y column are fixed; B^-_k and B^+_k 15 n_u each), 2
    flops per multiply-add, plus the vector updates of the primal/dual steps and the
    extrapolation (428 flops per interval, 9 per state or control entry of a node)."""
    M = K - 1
    return M * (4 * (196 + 30 * n_u) + 428) + 9 * (NX + n_u) * K


KERNEL_SOURCES = ("paper_2404_18034_amd/csrc/scp_kernels.hip",
                  "paper_2404_18034_amd/csrc/scp_common.hpp",
                  "paper_2404_18034_amd/csrc/scp_dpp.hpp",
                  "paper_2404_18034_amd/csrc/lander_model.hpp")
# hardware-counter summaries of the subproblem kernel's HBM traffic, per workload
TRAFFIC_FILES = {"C1": os.path.join(ROOT, "profiles", "subproblem_kernel_traffic_mc1024.txt"),
                 "C4": os.path.join(ROOT, "profiles", "subproblem_kernel_traffic_c4.txt")}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per subproblem launch from the committed hardware-counter summary of this
    workload, or None when there is no summary or when the kernel sources changed since the
    counters were taken."""
    path = TRAFFIC_FILES.get(workload)
    if path is None or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(cfg, inst, n_sample, threads, kmax):
    """The FP64 oracle on the host cores: `n_sample` evenly spaced instances of the batch
    (ids stride * i) on `threads` threads, plus a serial run on a sixteenth of them (the
    paper's CPU reference solves one instance at a time)."""
    import oracle
    oracle.build()
    B = inst["K"].shape[0]
    stride = max(1, B // n_sample)
    out = {}
    for n, th in ((n_sample, threads), (max(1, n_sample // 16), 1)):
        ids = np.arange(n) * stride
        sub = {k: v[ids] for k, v in inst.items()}
        t = time.perf_counter()
        r = oracle.solve(cfg, sub["x0"], sub["xf"], sub["params"], sub["K"], kmax=kmax,
                         nthreads=th)
        out[th] = (n, time.perf_counter() - t, int(np.sum(r["status"] == 0)))
    n, dt, conv = out[threads]
    n1, dt1, conv1 = out[1]
    return dict(value=round(conv / dt, 3), unit="converged solves/s", cores=threads,
                kind="oracle",
                sample="instances %d*i, i < %d, of the %d (same settings), %d threads, %.1f s "
                       "wall, %d converged; the rate is that of the sample" % (
                           stride, n, B, threads, dt, conv),
                single_thread=dict(value=round(conv1 / dt1, 3), instances=n1,
                                   wall_s=round(dt1, 2), converged=conv1))


def fp64_leg(cfg, inst, steps, K):
    """The same workload on the FP64 path (graph replay, the compiler's register budget): one
    untimed solve, then `steps` timed solves."""
    import torch
    from paper_2404_18034_amd import api
    B = inst["K"].shape[0]
    solver = api.BatchSolver(dict(cfg, mode=1, occupancy=0), dtype="f64", k_max=K, max_batch=B,
                             device=0)
    try:
        prob = solver.to_device(inst)
        sol = solver.alloc_solution(B)
        solver.solve_into(prob, sol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            solver.solve_into(prob, sol)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        conv = int(np.sum(sol["status"].cpu().numpy() == 0))
    finally:
        solver.close()
    return dict(value=round(conv / (ms * 1e-3), 2), unit="converged solves/s", dtype="f64",
                steps=steps, ms_per_step=round(ms, 3), converged=conv,
                solves_per_s_all=round(B / (ms * 1e-3), 2))


def sweep(args):
    """Batch-size sweep on the paper's Monte Carlo distribution (the analog of its CPU/GPU
    solve-time comparison): GPU time of one batched solve of B runs (ids 0..B-1), against the
    oracle on the host cores, measured on a few runs and extrapolated linearly in B (a serial
    solver's time is linear in the number of runs).  One JSON line per batch size."""
    import torch
    import oracle
    from paper_2404_18034_amd import api
    from paper_2404_18034_amd import instances as I

    cfg = I.solver_settings("F1")
    cfg["mode"], cfg["occupancy"] = 1, 5
    probe = I.make_instances("F1", ids=range(64))
    oracle.build()
    cpu = {}
    for th, n in ((1, 4), (16, 64)):
        sub = {k: v[:n] for k, v in probe.items()}
        t = time.perf_counter()
        oracle.solve(cfg, sub["x0"], sub["xf"], sub["params"], sub["K"], kmax=30, nthreads=th)
        cpu[th] = (time.perf_counter() - t) / n
    print(json.dumps({"sweep": "oracle", "s_per_run_1_thread": round(cpu[1], 4),
                      "s_per_run_16_threads": round(cpu[16], 5)}), flush=True)
    bmax = max(SWEEP_SIZES)
    solver = api.BatchSolver(cfg, dtype="f32", k_max=30, max_batch=bmax, device=0)
    sol = solver.alloc_solution(bmax)
    crossover = None
    for B in SWEEP_SIZES:
        inst = I.make_instances("F1", ids=range(B))
        prob = solver.to_device(inst)
        solver.solve_into(prob, sol)  # warm-up (graph capture for this argument set)
        torch.cuda.synchronize()
        reps = 3 if B <= 4096 else 1
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            solver.solve_into(prob, sol)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        gpu = sorted(ts)[len(ts) // 2]
        conv = int(np.sum(sol["status"][:B].cpu().numpy() == 0))
        if crossover is None and gpu < B * cpu[1]:
            crossover = B
        print(json.dumps({"sweep": "F1", "batch": B, "gpu_s": round(gpu, 5),
                          "oracle_1_thread_s": round(B * cpu[1], 4),
                          "oracle_16_threads_s": round(B * cpu[16], 4),
                          "converged": conv, "gpu_runs_per_s": round(B / gpu, 1)}), flush=True)
    print(json.dumps({"sweep": "summary", "first_batch_where_gpu_beats_serial_oracle": crossover,
                      "mode": [1, 5]}), flush=True)
    solver.close()


def multistart(args):
    """Multi-start on the paper's Monte Carlo at K = 20 with the node-wise convex sets (256
    problems; starts with the initial dilation guess s_init in {4, 5, 6, 7}, all 1,024 solves
    in one batch, then the choice of the converged start of lowest cost): converged problems
    and time, against the single start s_init = 5.  One JSON line."""
    import torch
    from paper_2404_18034_amd import api
    from paper_2404_18034_amd import instances as I

    cfg = I.solver_settings("F1", node_projections=31)
    cfg["mode"], cfg["occupancy"] = 1, 6
    inst = I.make_instances("F1")
    inst["K"] = np.full(256, 20, np.int32)
    s_init = (4.0, 5.0, 6.0, 7.0)
    rep = I.multistart(inst, s_init)
    solver = api.BatchSolver(cfg, dtype="f32", k_max=20, max_batch=len(rep["K"]), device=0)
    res = {}
    for name, data, starts in (("single", inst, 1), ("multi", rep, len(s_init))):
        prob = solver.to_device(data)
        sol = solver.alloc_solution(len(data["K"]))
        best = torch.empty(256, dtype=torch.int32, device="cuda:0")
        out = solver.alloc_solution(256)
        for _ in range(1 + args.steps):
            if _ == 1:
                torch.cuda.synchronize()
                t = time.perf_counter()
            solver.solve_into(prob, sol)
            solver.select_best_into(sol, 256, starts, best, out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / args.steps
        res[name] = dict(ms=round(ms, 3), converged=int(np.sum(best.cpu().numpy() >= 0)))
    solver.close()
    print(json.dumps({"multistart": "paper's Monte Carlo, 256 problems, K=20, FP32",
                      "s_init": s_init, "single_start_s_init_5": res["single"],
                      "four_starts": res["multi"]}), flush=True)


def grad(args):
    """Gradients (the vector-Jacobian product of the last SCP iteration, scp_batch_grad) on the
    differentiation workload: 4,096 x K = 20 in FP32, the forward solve recorded (untimed),
    then `steps` batched products timed (200 differentiated PIPG steps, checkpoints every 20).
    The oracle's gradient is central differences of its truncated map (2 x 18 evaluations),
    timed on a few instances.  One JSON line."""
    import torch
    import oracle
    from paper_2404_18034_amd import api
    from paper_2404_18034_amd import instances as I

    cfg = I.solver_settings("C3")
    inst = I.make_instances("C3")
    B = len(inst["K"])
    out = {"grad": "vector-Jacobian product of the last SCP iteration, 4,096 x K=20, FP32, "
                   "200 differentiated PIPG steps (checkpoints every 20)"}
    grads = []
    # the RK4 share by the reverse sweep (general form) and by forward tangents (two
    # parameters reach the discretization)
    for name, tangent in (("reverse_rk4", 0), ("tangent_rk4", 1)):
        solver = api.BatchSolver(dict(cfg, grad_rk4_tangent=tangent), dtype="f32", k_max=20,
                                 max_batch=B, device=0)
        prob = solver.to_device(inst)
        sol, last = solver.solve_record_into(prob, solver.alloc_solution(B),
                                             solver.alloc_lastiter(B))
        cot = torch.ones((B, 2), dtype=torch.float32, device="cuda:0")
        g = torch.empty((B, 18), dtype=torch.float32, device="cuda:0")
        solver.grad_into(prob, last, cot, g)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            solver.grad_into(prob, last, cot, g)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / args.steps
        grads.append(g.cpu().numpy())
        out[name] = {"ms_per_batch": round(ms, 3), "gradients_per_s": round(B / (ms * 1e-3), 1),
                     "finite": bool(np.all(np.isfinite(grads[-1])))}
        solver.close()
    out["forms_max_rel_diff"] = float(np.max(np.abs(grads[0] - grads[1])) /
                                      max(np.max(np.abs(grads[0])), 1e-30))
    if not args.no_cpu:
        n = 4
        t = time.perf_counter()
        for b in range(n):
            K = int(inst["K"][b])
            L = oracle.lastiter_state(cfg, inst["x0"][b], inst["xf"][b], inst["params"][b], K)
            theta = oracle.theta_of(inst["x0"][b], inst["params"][b])
            for i in range(theta.size):
                for sgn in (1.0, -1.0):
                    th = theta.copy()
                    th[i] += sgn * 1e-6
                    oracle.truncated_map(cfg, inst["x0"][b], inst["xf"][b], inst["params"][b], K,
                                         th, L, cfg["grad_pipg_steps"])
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(n / dt, 3), "unit": "gradients/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "%d instances, central differences (36 map "
                                         "evaluations each, after the recorded solve), %.1f s"
                                         % (n, dt)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", default=WORKLOAD, choices=["C1", "C2", "C4", "F1", "F1S", "F2"],
                    help="C4 (default): the 65,536 x K=30 throughput Monte Carlo, the largest "
                         "single-GPU configuration of the metric's 1k-64k range; C1 (1,024 x "
                         "K=20), C2 (16,384 uneven K, early exit), F1 (the paper's 256-run "
                         "Monte Carlo), F1S (with the speed bound) and F2 (with the torque control) for "
                         "reference")
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="timed solves of the same workload on the FP64 path (0: skip)")
    ap.add_argument("--grad", action="store_true",
                    help="time the batched gradient (scp_batch_grad) on the differentiation "
                         "workload (4,096 x K=20)")
    ap.add_argument("--multistart", action="store_true",
                    help="multi-start on the paper's Monte Carlo at K=20 (four s_init guesses)")
    ap.add_argument("--sweep", action="store_true",
                    help="batch-size sweep 1..65,536 on the paper's Monte Carlo distribution "
                         "against the oracle on the host (one JSON line per size)")
    ap.add_argument("--mode", type=int, default=None,
                    help="dispatch mode (0 launches, 1 graph, 2 ordered, 3 persistent, 4 K-bucketed); "
                         "default: autotuned on the workload")
    ap.add_argument("--occupancy", type=int, default=None, choices=[0, 4, 5, 6],
                    help="subproblem register-budget variant with --mode (default 0)")
    ap.add_argument("--scalar-dilation", action="store_true",
                    help="one dilation value over the horizon instead of one per node")
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a reference "
                         "kernel of known traffic for hardware-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (instances are independent; a multi-GPU run would "
              "shard the batch with no exchange). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        sweep(args)
        return
    if args.multistart:
        multistart(args)
        return
    if args.grad:
        grad(args)
        return

    import torch
    from paper_2404_18034_amd import api
    from paper_2404_18034_amd import instances as I

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    wl = args.workload
    cfgd = I.CONFIGS[wl]
    cfg = I.solver_settings(wl, scalar_dilation=int(args.scalar_dilation))
    if args.mode is not None:
        cfg["mode"] = args.mode
        if args.occupancy is not None:
            cfg["occupancy"] = args.occupancy
    inst = I.make_instances(wl)
    B, K = cfgd["B"], max(cfgd["K"])
    solver = api.BatchSolver(cfg, dtype=args.dtype, k_max=K, max_batch=B, device=0)
    prob = solver.to_device(inst)
    sol = solver.alloc_solution(B)
    torch.cuda.synchronize()
    tuned = None
    if args.mode is None:
        tuned = solver.autotune(prob, sol)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        solver.solve_into(prob, sol)
    torch.cuda.synchronize()

    # timed region: exactly `steps` solves, no profiling events inside
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.solve_into(prob, sol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    status = sol["status"].cpu().numpy()
    pipg_iters = sol["pipg_iters"].cpu().numpy()
    converged = int(np.sum(status == 0))
    ms_per_step = dt * 1e3 / args.steps

    # per-kernel launch durations (HIP events on the library's stream), separate solves
    solver.profile(True)
    per = {"discretize": [0.0, 0], "prepare": [0.0, 0], "subproblem": [0.0, 0], "init": [0.0, 0]}
    nprof = max(1, min(args.steps, 5))
    for _ in range(nprof):
        solver.solve_into(prob, sol)
        for k, (ms, n) in solver.profile_read().items():
            per[k][0] += ms
            per[k][1] += n
    solver.profile(False)
    sub_ms = per["subproblem"][0] / nprof            # per solve
    sub_launches = per["subproblem"][1] / nprof
    Ks = inst["K"].astype(np.int64)
    flops_per_solve = float(np.sum(pipg_iters.astype(np.float64) *
                                   np.array([pipg_flops_per_iter(k, solver.n_u) for k in Ks])))
    achieved = flops_per_solve / (sub_ms * 1e-3) / 1e12
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=FP32_VECTOR_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                    traffic=None if args.scalar_dilation else measured_traffic(wl),
                    kernel="subproblem_kernel",
                    avg_launch_ms=round(sub_ms / max(sub_launches, 1), 4),
                    kernel_ms_per_step={k: round(v[0] / nprof, 3) for k, v in per.items()})

    out = {
        "metric": "converged 6-DoF SCP solves/sec, 1k-64k-run Monte Carlo, FP32 vs FP64 plain",
        "value": round(converged / (ms_per_step * 1e-3), 2),
        "unit": "converged solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[wl] + (", one dilation value over the horizon"
                                                     if args.scalar_dilation else ""),
                   "batch": B, "K": sorted(set(int(k) for k in cfgd["K"])),
                   "scp_iters": cfg["scp_iters_max"], "pipg_iters": cfg["pipg_iters_max"],
                   "early_exit": bool(cfg["early_exit"]), "node_projections": cfg["node_projections"],
                   "scalar_dilation": bool(args.scalar_dilation),
                   "power_iteration": "f32" if cfg.get("power_fp32", 0) else "f64",
                   "n_u": solver.n_u,
                   "mode": solver.mode(), "parallelism": "single GPU"},
        "converged": converged, "solves_per_s_all": round(B / (ms_per_step * 1e-3), 2),
        "roofline": roofline,
    }
    if tuned is not None:
        out["autotune_ms"] = {str(m): round(v, 3) for m, v in tuned[1].items()}
    solver.close()
    if args.dtype == "f32" and args.fp64_steps > 0:
        out["fp64"] = fp64_leg(cfg, inst, args.fp64_steps, K)
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(cfg, inst, args.cpu_sample, threads, K)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
