"""Throughput benchmark: SSP-RK3 steps of the IDP Q1 Euler scheme on one GPU.

Default workload: 3D Q1 hex grid 257^3 nodes (16,974,593 nodes), interior
nodes jittered by up to 0.2 h, Morton node order, uniform Mach 3 flow
(rho 1.4, p 1, u 3 e_x) with a seeded density blob field of amplitude 0.2,
boundary held, FP64.  A step is three forward-Euler stages (every sweep of
the method); the metric is node updates per second per stage.

Prints one JSON line (stdout); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP64_PEAK_TFS = 78.6         # MI355X vector FP64, TFLOP/s
# FP64 operations per unordered pair of the viscosity sweep at 257^3 (one
# wave-speed bound for the mirror-image pairs, two for the 0.7% on boundary
# faces, with their x^y series, divisions and square roots, the psi terms of
# the two states once; FMA = 2): every operation of the formula runs exactly
# once, so the count rocprofv3 measures for it
# (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64) is its algorithmic count.
VISCOSITY_FLOP_PER_PAIR = 438
KERNEL_SOURCES = ["paper_2007_00094_amd/csrc/idp_kernels.hip",
                  "paper_2007_00094_amd/csrc/idp_device.h",
                  "paper_2007_00094_amd/csrc/kernels.h",
                  "paper_2007_00094_amd/csrc/sweep_common.h"]
COUNTERS = os.path.join(ROOT, "profiles", "counters_mach3_257_morton.md")
FP64_VECTOR_PEAK = 78.6e12   # MI355X FP64 vector, flop/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(dim, n, nnz, marked):
    """Compulsory bytes of each kernel per SSP-RK3 step: every array a
    launch reads or writes counted once (neighbour gathers and transposed
    reads assumed cached), from the data layout of the library, summed over
    the step's launches.  marked: off-diagonal entries with s1 < 1 (their
    pairs are the pass-2 limiter's work list and the entries pass 2
    visits)."""
    nc = dim + 2
    packa = 8 * (nc + 3)       # pack A as the forward reads it: U, p, c, eta/rho
    packl = 8 * (nc + 3)       # pack L: U, p, phi, alpha
    packb = 8 * (2 * nc + 2)   # pack B: U, R, alpha, m
    coef = 8                   # pack B's tau/(lambda_i m_i)
    rowb = 8 * (nc + 3)        # U^L, bounds
    cb = 8 * dim
    npairs = (nnz - n) // 2
    slow = marked // 2
    touched = min(n, marked)   # rows with a marked entry (at most)
    return {
        # U read; pack A and pack L written (pack L's alpha by the indicator)
        "node_pack": 3 * n * (8 * nc + packa + packl - 8),
        # per pair: 4 ids, c_ij and c_ji, d written twice; U, p, c of the
        # nodes; the indicator: c_ij and a 16-bit halo position per entry,
        # eta/rho per node, alpha written twice
        "pair_viscosity": 3 * (npairs * (16 + 2 * cb + 16) + n * 8 * (nc + 2) +
                               nnz * (cb + 2) + n * (8 + 16)),
        # stage 1 only: d per entry; m_i, the diagonal's position read,
        # d_ii and tau_i written
        "row_diagonal": nnz * 8 + n * (8 + 4 + 16),
        # per entry: column, c_ij, d_ij; per node: alpha_i, m_i, lambda_i
        # read, pack B and the row record written; stages 2 and 3 also
        # d_ii and tau_i
        "row_low_order": 3 * (nnz * (4 + cb + 8) + n * (packl + 3 * 8 + packb + coef + rowb)) +
                         2 * n * (4 + 16),
        # per pair: 4 ids, d, m_ij, s written twice and once in pair order
        "pair_limiter1": 3 * (npairs * (16 + 8 + 8 + 16 + 8) + n * (packb + coef + rowb)),
        # per entry: column, s1, d, m_ij and the entry's mask bit; per node:
        # lambda_i, U^L read, the pass-1 state and l2self written; the list
        "row_pass1": 3 * (nnz * (4 + 8 + 8 + 8) + nnz // 8 +
                          n * (packb + 8 + 8 * nc + 8 * nc + 8) + slow * 4),
        # per listed pair: its entry, the transposed position and the two
        # columns, d, m_ij, s1, s2 written twice; the two rows' pack B and
        # pass-1 records
        "pair_limiter2": 3 * (slow * (4 + 4 + 8 + 8 + 8 + 8 + 16) +
                              touched * (packb + coef + 64)),
        # per node: the pass-1 state, U0 and the hold flag read, the output
        # written, the mask bits; per marked entry: column, s1, s2, d,
        # m_ij, the neighbour's pack B; its row's pack B and lambda
        "row_pass2": 3 * (n * (8 * nc + 8 * nc + 8 * nc + 1) + nnz // 8 +
                          marked * (4 + 8 + 8 + 8 + 8 + packb) +
                          touched * (packb + coef + 8)),
    }


# FP64 operations per stencil entry of the indicator phase of the viscosity
# sweep (fluxes, their difference dotted with c_ij, v = m/rho, the a_i and
# b_i sums): the diagonal sweep's measured count with the indicator.
INDICATOR_FLOP_PER_ENTRY = 133


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed counter summary
    (scaled FETCH_SIZE + WRITE_SIZE), or None if the kernel sources changed
    since the counters were taken."""
    import hashlib
    if not os.path.exists(COUNTERS):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    text = open(COUNTERS).read().split()
    try:
        if text[text.index("source_hash:") + 1] != h.hexdigest()[:16]:
            return None
    except ValueError:
        return None
    for i, w in enumerate(text):
        if w == "traffic_bytes_per_launch:" and text[i + 1] == kernel:
            return float(text[i + 2])
    return None


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(mesh, U0, radius, steps, single_steps):
    """The oracle, as it stands, on a patch of the same mesh and state:
    nodes within graph distance ``radius`` of the mesh centre; ``steps``
    steps with every host thread, then ``single_steps`` on one thread."""
    import oracle
    from paper_2007_00094_amd import inputs
    centre = int(np.argmin(np.sum((mesh.coords - 0.5) ** 2, axis=1)))
    sub, nodes, _ = inputs.extract_patch(mesh, [centre], radius)
    threads = oracle.set_threads(0)
    o = oracle.Oracle(sub, dirichlet=sub.boundary)
    U = U0[nodes].copy()
    dt = o.max_dt(U)
    t0 = time.perf_counter()
    for _ in range(steps):
        U, _, _ = o.step(U, dt=dt)
    t = time.perf_counter() - t0
    single = None
    if single_steps > 0:
        oracle.set_threads(1)
        t1 = time.perf_counter()
        for _ in range(single_steps):
            U, _, _ = o.step(U, dt=dt)
        t1 = time.perf_counter() - t1
        oracle.set_threads(threads)
        single = sub.n_nodes * 3 * single_steps / t1
    return {"value": sub.n_nodes * 3 * steps / t, "unit": "node-updates/s",
            "cores": threads, "kind": "oracle",
            "single_thread_value": single, "cpu_model": cpu_model(),
            "host_threads": os.cpu_count(),
            "sample": f"{steps} SSP-RK3 step(s) on a {sub.n_nodes}-node patch "
                      f"(graph radius {radius} around the centre) of the same mesh "
                      f"and state, fixed dt, {threads} OpenMP threads, {t:.1f} s; "
                      f"then {single_steps} step(s) on 1 thread"}


def hbm_copy_bandwidth(gib=4.0, reps=3):
    """Achievable HBM bandwidth: the best of ``reps`` timed device copies of
    ``gib`` GiB (bytes read + written), triads a = b + s c (2 read, 1
    written) and sums (read only: the sweeps read far more than they
    write), in GB/s."""
    import torch
    n = int(gib * 2**30 // 8)
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    z = torch.full_like(x, 2.0)
    best_copy = best_triad = best_read = 0.0
    acc = torch.zeros((), dtype=torch.float64, device="cuda")
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        best_copy = max(best_copy, 16.0 * n / (a.elapsed_time(b) * 1e-3) / 1e9)
        a.record()
        torch.add(x, z, alpha=0.5, out=y)
        b.record()
        b.synchronize()
        best_triad = max(best_triad, 24.0 * n / (a.elapsed_time(b) * 1e-3) / 1e9)
        a.record()
        torch.sum(y, dim=0, out=acc)
        b.record()
        b.synchronize()
        best_read = max(best_read, 8.0 * n / (a.elapsed_time(b) * 1e-3) / 1e9)
    del x, y, z, acc
    torch.cuda.empty_cache()
    return {"copy_GB_per_s": round(best_copy, 1), "triad_GB_per_s": round(best_triad, 1),
            "read_GB_per_s": round(best_read, 1), "bytes_per_array": 8 * n}


def batched_bench(steps, schedule=None, tile=0, loop=True):
    """64 independent 2D four-quadrant meshes of uneven sizes: the tuned
    batched schedule (or the given one) against one context per instance
    stepped in a loop."""
    import torch
    from paper_2007_00094_amd import inputs
    from paper_2007_00094_amd.solver import BatchSolver, Solver
    batch = inputs.batch_workload()
    U0 = np.concatenate([u for _, u in batch])
    bs = BatchSolver([m for m, _ in batch])
    if schedule is None:
        best, tuner_ms = bs.tune(torch.tensor(U0, device="cuda"), 2)
        sched = None
    else:
        sched = BatchSolver.schedule(schedule, tile)
        best, tuner_ms = sched, {}
    U = torch.tensor(U0, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs.steps(U, steps, schedule=sched)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    if not loop:
        n = int(bs.n)
        bs.close()
        return {"schedule": {"kind": schedule, "tile": tile}, "nodes": n, "steps": steps,
                "batched_ms_per_step": t_batch / steps * 1e3}
    sols = [Solver(m, asynchronous=True) for m, _ in batch]
    Us = [torch.tensor(u, device="cuda") for _, u in batch]
    for so, u in zip(sols, Us):
        so.step(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for so, u in zip(sols, Us):
            so.step(u)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    assert all(so.status() == 0 for so in sols), "a batch instance's step failed or warned"
    for so in sols:
        so.close()
    n = int(bs.n)
    kind = {1: "launches", 2: "persistent"}[best.kind]
    bs.close()
    return {"workload": "64 2D four-quadrant Q1 meshes, sides log-uniform in [33, 513] "
                        "(seeds 100-163), per-instance CFL dt",
            "instances": len(batch), "nodes": n, "steps": steps,
            "schedule": {"kind": kind, "tile": int(best.tile)},
            "tuner_ms_per_2_steps": {k: round(v, 2) for k, v in tuner_ms.items()},
            "batched_node_updates_per_s": n * 3 * steps / t_batch,
            "loop_node_updates_per_s": n * 3 * steps / t_loop,
            "batched_ms_per_step": t_batch / steps * 1e3,
            "loop_ms_per_step": t_loop / steps * 1e3,
            "speedup_vs_loop": t_loop / t_batch}


def adjoint_bench(steps, every):
    """Checkpointed adjoint of the 65^3 smooth-blob run: forward with
    checkpoints every `every` steps, then the backward (recomputation
    included) of the gradient of the kinetic energy in [0.4, 0.6]^3 at the
    final time; dt frozen from a base run.  One warm pair, one timed pair."""
    import torch
    from paper_2007_00094_amd import inputs
    from paper_2007_00094_amd.solver import Solver
    mesh, U0 = inputs.workload("adjoint_3d", n=65)
    s = Solver(mesh)
    U = torch.tensor(U0, device="cuda")
    dts = []
    for _ in range(steps):
        dt, st = s.step(U)
        assert st == 0, f"base run failed or warned: {st}"
        dts.append(dt)
    # cotangent of J = sum_{x_i in box} m_i |m_i|^2 / (2 rho_i) at the final state
    box = torch.tensor(np.all((mesh.coords >= 0.4) & (mesh.coords <= 0.6), axis=1), device="cuda")
    mi = torch.tensor(s.matrices()["m_i"], device="cuda")
    Uf = U.clone().requires_grad_(True)
    mom = Uf[:, 1:4]
    J = (mi * box * (mom * mom).sum(1) / (2 * Uf[:, 0])).sum()
    J.backward()
    W = Uf.grad.detach().clone()
    res = []
    for _ in range(2):
        U = torch.tensor(U0, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.forward_checkpoints(U, dts, every)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        g = s.adjoint_checkpoints(dts, every, W)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        res.append((tf, tb))
    tf, tb = res[-1]
    assert torch.isfinite(g).all()
    # the stage VJP alone: in the checkpointed backward the recomputation of
    # the next segment runs beside the VJPs on a second stream, so event
    # times taken there would include the contention
    U = torch.tensor(U0, device="cuda")
    s.set_timing(True)
    for _ in range(10):
        s.euler_stage_vjp(U, dts[0], W)
    torch.cuda.synchronize()
    kt = s.kernel_times()
    s.set_timing(False)
    vjp_ms, vjp_n = kt["stage_vjp"]
    fwd_ms = sum(ms for k, (ms, c) in kt.items() if k != "stage_vjp")
    fwd_n = kt["pair_viscosity"][1]
    s.close()
    return {"workload": "adjoint_3d_65^3_morton: isothermal Gaussian density blobs (p = rho), "
                        "at rest; gradient of the kinetic energy in [0.4, 0.6]^3 at the final "
                        "time w.r.t. U0",
            "nodes": mesh.n_nodes, "steps": steps, "checkpoint_every": every,
            "forward_ms": tf * 1e3, "adjoint_ms": tb * 1e3,
            "adjoint_over_forward": tb / tf,
            "stage_vjp_ms": vjp_ms / vjp_n, "recorded_stage_ms": fwd_ms / fwd_n,
            "recompute_overlapped": True,
            "forward_ms_per_step": tf / steps * 1e3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=257, help="nodes per side")
    ap.add_argument("--order", default="morton", choices=["morton", "random", "lex"])
    ap.add_argument("--renumber", action="store_true",
                    help="the library renumbers the nodes along a Morton curve")
    ap.add_argument("--split-p", action="store_true",
                    help="the paper's variant 3: the low-order sweep stores the viscous "
                         "part of P_ij for the limiter sweeps and passes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-mesh batched measurement")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--batch-schedule", choices=["launches", "persistent"], default=None,
                    help="with --only batch: run this schedule (no tuner, no loop)")
    ap.add_argument("--batch-tile", type=int, default=64,
                    help="persistent: units per item, or -n: n items per instance sweep")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint measurement")
    ap.add_argument("--only", choices=["batch", "adjoint"], default=None,
                    help="run only that measurement and print its object (for profiling)")
    ap.add_argument("--no-staging", action="store_true",
                    help="row sweeps gather from memory instead of staging in LDS")
    ap.add_argument("--sell-sigma", type=int, default=64,
                    help="SELL-C-sigma sorting window in rows (multiple of 64; 0: all rows)")
    ap.add_argument("--adjoint-steps", type=int, default=200)
    ap.add_argument("--cpu-radius", type=int, default=24)
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--cpu-single-steps", type=int, default=2,
                    help="steps of the oracle on one thread (0: skip)")
    ap.add_argument("--newton-max", type=int, default=2,
                    help="Newton iterations of the limiter (the method's default is 2)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device copy of GIB GiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch
        n = int(args.copy_calibration * 2**30 // 8)
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding design notes); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2007_00094_amd import capi, inputs
    from paper_2007_00094_amd.solver import Solver

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.only == "batch":
        if args.batch_schedule:
            out = batched_bench(args.batch_steps, args.batch_schedule, args.batch_tile,
                                loop=False)
        else:
            out = batched_bench(args.batch_steps)
        print(json.dumps(out), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(adjoint_bench(args.adjoint_steps, 20)), flush=True)
        return
    t = time.perf_counter()
    mesh, U0 = inputs.workload("mach3_3d", n=args.n, order=args.order)
    log(f"mesh {mesh.n_nodes} nodes, {mesh.n_cells} cells in {time.perf_counter() - t:.1f} s")
    t = time.perf_counter()
    s = Solver(mesh, asynchronous=True, newton_max=args.newton_max,
               staging=not args.no_staging, sell_sigma=args.sell_sigma, renumber=args.renumber,
               split_p=args.split_p)
    torch.cuda.synchronize()
    log(f"solver created: nnz {s.nnz}, {s.device_bytes / 2**30:.1f} GiB device, "
        f"{time.perf_counter() - t:.1f} s")
    U = torch.tensor(U0, device="cuda")
    for _ in range(args.warmup):
        s.step(U)
    torch.cuda.synchronize()
    assert s.status() in (0, 1), "warm-up steps failed"
    if s.status() == 1:
        log("WARNING: a warm-up step exceeded a stage-2/3 CFL bound")
    log(f"{args.warmup} warm-up steps done")

    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.step(U)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = s.status()
    assert st in (0, 1), f"timed steps failed: {st}"
    if st == 1:
        log("WARNING: a timed step exceeded a stage-2/3 CFL bound (invariant domain not "
            "guaranteed for it)")
    times = s.kernel_times()
    s.set_timing(False)
    log(f"{args.steps} timed steps in {elapsed:.3f} s")
    for k, (ms, cnt) in times.items():
        if cnt:
            log(f"  {k:18s} {ms / cnt:9.3f} ms/launch x {cnt}")

    stages = 3 * args.steps
    value = mesh.n_nodes * stages / elapsed
    # the entries with s1 < 1 of the last stage (pass 2's work)
    s1 = s.debug(capi.IDP_DBG_L1)
    marked = int(np.count_nonzero(s1 != 1.0))
    del s1
    log(f"entries with s1 < 1 in the last stage: {marked} of {s.nnz - mesh.n_nodes}")
    algo = algorithmic_bytes(mesh.dim, mesh.n_nodes, s.nnz, marked)
    per_step = {k: times[k][0] / args.steps for k in algo}
    dom = max(algo, key=lambda k: per_step[k])
    kernels = {k: {"ms_per_step": round(per_step[k], 4),
                   "launches_per_step": times[k][1] // args.steps,
                   "GB_per_s": round(algo[k] / (per_step[k] / 1e3) / 1e9, 1)}
               for k in algo if times[k][1]}
    traffic = measured_traffic(dom) if (args.n == 257 and args.order == "morton" and
                                        not args.split_p and not args.renumber) else None
    launches = times[dom][1] // args.steps
    avg_s = per_step[dom] / launches / 1e3
    bytes_launch = algo[dom] // launches
    achieved = bytes_launch / avg_s / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": bytes_launch,
                "launch_ms": round(avg_s * 1e3, 4)}
    if dom == "pair_viscosity":
        # its FP64 work beside: the wave-speed bounds per pair, the indicator
        # per entry, against the vector FP64 peak
        flops = (VISCOSITY_FLOP_PER_PAIR * (s.nnz - mesh.n_nodes) / 2 +
                 INDICATOR_FLOP_PER_ENTRY * s.nnz)
        roofline["fp64_TFLOP_per_s"] = round(flops / avg_s / 1e12, 2)
        roofline["fp64_frac"] = round(flops / avg_s / 1e12 / FP64_PEAK_TFS, 4)

    s.close()
    log("achievable HBM bandwidth: 4 GiB copy and triad")
    roofline["measured_hbm"] = hbm_copy_bandwidth()
    roofline["frac_of_measured_copy"] = round(
        roofline["achieved"] / roofline["measured_hbm"]["copy_GB_per_s"], 4) \
        if roofline["unit"] == "GB/s" else None
    batched = None
    if not args.no_batch:
        log("batched: 64 meshes, tuned schedule vs per-instance loop")
        batched = batched_bench(args.batch_steps)
        log(f"  batched {batched['batched_ms_per_step']:.2f} ms/step, loop "
            f"{batched['loop_ms_per_step']:.2f} ms/step, {batched['speedup_vs_loop']:.2f}x")
    adjoint = None
    if not args.no_adjoint:
        log(f"adjoint: 65^3, {args.adjoint_steps} steps, checkpoints every 20")
        adjoint = adjoint_bench(args.adjoint_steps, 20)
        log(f"  forward {adjoint['forward_ms']:.1f} ms, adjoint {adjoint['adjoint_ms']:.1f} ms, "
            f"ratio {adjoint['adjoint_over_forward']:.2f}, stage VJP {adjoint['stage_vjp_ms']:.3f} ms")
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a patch)")
        cpu = cpu_baseline(mesh, U0, args.cpu_radius, args.cpu_steps, args.cpu_single_steps)
    out = {
        "metric": "Q1 node-updates/s per RK stage FP64; HBM GB/s; adjoint/forward time ratio",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"mach3_3d_{args.n}^3_{args.order}",
                   "newton_max_iter": args.newton_max, "lds_staging": not args.no_staging,
                   "sell_sigma": args.sell_sigma, "renumbered": args.renumber,
                   "split_p_variant3": args.split_p,
                   "nodes": mesh.n_nodes, "nnz": s.nnz, "stages": stages,
                   "parallelism": "single GPU"},
        "cfl_warning": st == 1,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "batched": batched,
        "adjoint": adjoint,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
