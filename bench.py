"""Benchmark: push-relabel epsilon-approximate assignment on one MI355X.

Workload (default): two sets of n = 10,000 points drawn uniformly in the unit
square (float32, seed 0), squared Euclidean cost scaled to max 1, eps = 0.01,
int16 rounded costs. One step = one whole solve: cost build, phase loop,
completion, cost and statistics (in device memory), with X and Y already in
HBM; the timed steps are enqueued back to back, and
`ms_per_solve_reading_stats` gives the rate of solves that each read their
statistics back to the host.

Prints one JSON line. `roofline` is taken for the dominant kernel; its
achieved rate uses algorithmic bytes (entries examined x 2 B for the phase
loop, the n x n int16 write for the cost build) over the kernel's average
device time over the timed steps, from HIP events that the loop launches
carry on the library's stream.
`cpu_baseline` times the CPU oracle on the same instance.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "n=10k ε=.01 solve ms + phase-scan HBM GB/s; batched solves/s vs plain loop"


TRAFFIC_FILES = {(10000, 2, "auto"): "traffic_points_n10000_d2_eps0.01.json",
                 (50000, 3, "auto"): "traffic_points_n50000_d3_eps0.005.json",
                 (50000, 3, "matrix"): "traffic_points_n50000_d3_eps0.005_matrix.json"}


def measured_traffic(n, d, kernel, storage="auto"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload, or None when there is none or the kernel
    sources have changed since the counters were taken."""
    import hashlib
    name = TRAFFIC_FILES.get((n, d, storage))
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec["source_sha256"] or kernel not in rec["kernels"]:
        return None
    k = rec["kernels"][kernel]
    return round(k["fetch_bytes"] + k["write_bytes"], 1)


def host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0)), os.cpu_count()


def cpu_baseline(X, Y, eps, reps):
    """The single-threaded C oracle on the same instance, pinned to one host
    core (the last one this process may use) while it runs."""
    import oracle
    n = X.shape[0]
    model, allowed, total = host_cpu()
    before = os.sched_getaffinity(0)
    core = max(before)
    os.sched_setaffinity(0, {core})
    try:
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            k, _ = oracle.round_points_f32(X, Y, eps)
            oracle.solve_rounded(k, oracle.threshold(eps, n))
            times.append(time.perf_counter() - t0)
        # the clustered transport of the transport_clustered leg at eps = 0.01
        from paper_2203_03732_amd import synth
        C, nu, mu = synth.transport_clouds(1000, 1000, seed=11, shift=1.0)
        t0 = time.perf_counter()
        oracle.ot_solve_clustered(C, nu, mu, 0.01)
        ot_ms = 1e3 * (time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, before)
    ms = 1e3 * sum(times) / len(times)
    return {"value": round(ms, 3), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": f"{reps} whole solve(s) of the same instance (binary32 cost build "
                      f"+ phase loop + completion), single-threaded C pinned to core {core}",
            "host_cpu": model, "host_cores_allowed": allowed, "host_cores_total": total,
            "transport_clustered_eps_0.01": {
                "value": round(ot_ms, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                "sample": "one whole solve of the transport_clustered leg's eps = 0.01 "
                          "workload (scaling, rounding, clustered phases, plan and repair)"}}


def bench_batched(prot, synth, torch, reps=10):
    """512 independent instances (n uniform in [64, 1024], standard normal
    points in R^16, eps = 0.05): one graph replay of the batched solve vs a
    host loop of single-instance solves on the same stream."""
    import numpy as np
    ns, Xs, Ys = synth.gaussian_batch(512, 64, 1024, 16, seed=0)
    X = torch.from_numpy(np.concatenate(Xs)).cuda()
    Y = torch.from_numpy(np.concatenate(Ys)).cuda()
    ctx = prot.Context(0)

    def replay_ms_of(plan):
        plan.run(X, Y)
        plan.capture(X, Y)
        plan.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.replay()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    default_plan = ctx.batch(ns, 16, 0.05)
    default_ms = replay_ms_of(default_plan)
    default_plan.close()
    # the autotuner times every configuration on these inputs (untimed here)
    cfg, tuned_ms, tried = ctx.autotune_batch(ns, 16, 0.05, X, Y, reps=3)
    plan = ctx.batch(ns, 16, 0.05, config=cfg)
    replay_ms = replay_ms_of(plan)
    Xl = [torch.from_numpy(x).cuda() for x in Xs]
    Yl = [torch.from_numpy(y).cuda() for y in Ys]
    ctx.reserve(max(ns), with_matrix=True)
    for x, y in zip(Xl[:8], Yl[:8]):
        ctx.solve_points(x, y, 0.05)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for x, y in zip(Xl, Yl):
        ctx.solve_points(x, y, 0.05)
    torch.cuda.synchronize()
    loop_ms = 1e3 * (time.perf_counter() - t0)
    # the same loop enqueuing only (no statistics, no synchronisation per
    # solve), one synchronisation at the end
    t0 = time.perf_counter()
    for x, y in zip(Xl, Yl):
        ctx.solve_points(x, y, 0.05, stats=False)
    torch.cuda.synchronize()
    enq_ms = 1e3 * (time.perf_counter() - t0)
    st = plan.stats()
    plan.close()
    ctx.close()
    return {"workload": "512 instances, n~U[64,1024], N(0,I) in R^16, eps=0.05",
            "graph_replay_ms": round(replay_ms, 4),
            "solves_per_s": round(512 / (replay_ms * 1e-3), 1),
            "plain_loop_ms": round(loop_ms, 3),
            "plain_loop_solves_per_s": round(512 / (loop_ms * 1e-3), 1),
            "ratio_vs_plain_loop": round(loop_ms / replay_ms, 2),
            "plain_loop_enqueue_only_ms": round(enq_ms, 3),
            "ratio_vs_plain_loop_enqueue_only": round(enq_ms / replay_ms, 2),
            "autotuned_config": cfg, "configs_timed": tried,
            "default_config_replay_ms": round(default_ms, 4),
            "mean_phases": round(float(np.mean([s["phases"] for s in st])), 2)}


def bench_large(prot, synth, torch, reps=5):
    """Two sets of 50,000 uniform points in the unit cube, eps = 0.005: whole
    solves as the library chooses to run them (the 5 GB int16 matrix exceeds
    the Infinity Cache, so the greedy step recomputes costs from the points)."""
    X, Y = synth.uniform_points(50000, 3, seed=0)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    ctx = prot.Context(0)
    ctx.solve_points(Xd, Yd, 0.005)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = ctx.solve_points(Xd, Yd, 0.005)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    st = r.stats
    ctx.close()
    return {"workload": "n=50000 points U[0,1]^3 squared-Euclidean eps=0.005 seed=0",
            "ms_per_solve": round(ms, 4), "ms_build": round(st["ms_build"], 4),
            "ms_loop": round(st["ms_loop_kernel"], 4), "phases": st["phases"],
            "scanned": st["scanned"], "cost": st["cost"]}


def bench_large_matrix(prot, synth, torch, reps=5):
    """The same 50,000-point instance with its 5.06 GB int16 rounded-cost
    matrix built and resident in HBM (far beyond the 256 MB Infinity Cache):
    whole solves, and the phase loop's useful scan rate (2 B per entry
    examined over the loop kernel's device time) against 8 TB/s."""
    X, Y = synth.uniform_points(50000, 3, seed=0)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    ctx = prot.Context(0)
    ctx.reserve(50000, with_matrix=True)
    ctx.solve_points(Xd, Yd, 0.005, storage="matrix")
    torch.cuda.synchronize()
    loop_ms, build_ms = [], []
    t0 = time.perf_counter()
    for _ in range(reps):
        r = ctx.solve_points(Xd, Yd, 0.005, storage="matrix")
        loop_ms.append(r.stats["ms_loop_kernel"])
        build_ms.append(r.stats["ms_build"])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    st = r.stats
    ctx.close()
    lm, bm = sum(loop_ms) / reps, sum(build_ms) / reps
    scan_gbs = 2.0 * st["scanned"] / (lm * 1e-3) / 1e9
    write_gbs = 2.0 * 50000 * prot.pitch(50000) / (bm * 1e-3) / 1e9
    return {"workload": "n=50000 points U[0,1]^3 squared-Euclidean eps=0.005 seed=0, "
                        "int16 matrix (5.06 GB) resident in HBM",
            "ms_per_solve": round(ms, 4), "ms_build": round(bm, 4), "ms_loop": round(lm, 4),
            "phases": st["phases"], "rounds": st["rounds"], "scanned": st["scanned"],
            "loop_scan_GBps": round(scan_gbs, 1), "loop_frac_of_hbm_peak": round(scan_gbs / HBM_PEAK_GBS, 4),
            # HBM bytes per loop launch from the committed counters (null if
            # the kernel sources changed since), against 2 B per entry examined
            "loop_traffic_bytes": measured_traffic(
                50000, 3, "phase_loop_kernel<false, 0, false, false, false>", "matrix"),
            "loop_algorithmic_bytes": 2 * st["scanned"],
            "build_write_GBps": round(write_gbs, 1), "cost": st["cost"]}


def bench_uniform_costs(prot, synth, torch, reps=20):
    """1000 x 1000 costs i.i.d. uniform in [0, 1), eps = 0.1: whole solves
    of the cost-matrix entry point (rounding by eq. (1), phase loop,
    completion), C resident in HBM."""
    C = synth.uniform_costs(1000, seed=0)
    Cd = torch.from_numpy(C).cuda()
    ctx = prot.Context(0)
    ctx.solve_cost(Cd, 0.1)
    torch.cuda.synchronize()
    loop_ms = []
    t0 = time.perf_counter()
    for _ in range(reps):
        r = ctx.solve_cost(Cd, 0.1)
        loop_ms.append(r.stats["ms_loop_kernel"])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    st = r.stats
    ctx.close()
    return {"workload": "assignment 1000 x 1000 costs U[0,1) eps=0.1 seed=0",
            "ms_per_solve": round(ms, 4), "ms_round": round(st["ms_build"], 4),
            "ms_loop": round(sum(loop_ms) / reps, 4), "phases": st["phases"],
            "rounds": st["rounds"], "scanned": st["scanned"], "cost": st["cost"]}


def bench_unbalanced(prot, synth, torch, reps=5):
    """The unbalanced case: 20,000 supply points uniform in [0, 0.5]^2 over
    30,000 demand points uniform in the unit square, eps = 0.01 (T = 200):
    whole solves as the library chooses to run them."""
    X, Y = synth.uniform_points(20000, 2, seed=3, n_a=30000)
    X = (X * 0.5).astype(X.dtype)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    ctx = prot.Context(0)

    def timed(storage):
        ctx.solve_points(Xd, Yd, 0.01, storage=storage)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = ctx.solve_points(Xd, Yd, 0.01, storage=storage)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps, r.stats

    ms, st = timed("auto")
    # the same solve with the 1.2 GB int16 matrix built and stored from the
    # start (the library's own choice starts recomputing the costs, as the
    # matrix exceeds the Infinity Cache, and hands over to the matrix once
    # the loop has run long enough to pay for it)
    ms_m, st_m = timed("matrix")
    ctx.close()
    return {"workload": "n_b=20000 points U[0,0.5]^2 over n_a=30000 points U[0,1]^2 "
                        "squared-Euclidean eps=0.01 seed=3",
            "ms_per_solve": round(ms, 4), "ms_build": round(st["ms_build"], 4),
            "ms_loop": round(st["ms_loop_kernel"], 4), "phases": st["phases"],
            "scanned": st["scanned"],
            "entries_per_s_loop": round(st["scanned"] / (st["ms_loop_kernel"] * 1e-3), 1),
            "cost": st["cost"],
            "stored_matrix": {"ms_per_solve": round(ms_m, 4), "ms_build": round(st_m["ms_build"], 4),
                              "ms_loop": round(st_m["ms_loop_kernel"], 4),
                              "same_cost": st_m["cost"] == st["cost"]}}


def bench_transport(prot, synth, torch, reps=5):
    """Optimal transport (Section 4) between two 1,000-point clouds in the
    plane, the demand cloud shifted by 1, random masses, eps = 0.1: whole
    solves (scaling, copies, phase loop, plan and repair) with C, nu and mu
    resident in HBM."""
    C, nu, mu = synth.transport_clouds(1000, 1000, seed=11, shift=1.0)
    Cd, nud, mud = (torch.from_numpy(x).cuda() for x in (C, nu, mu))
    ctx = prot.Context(0)
    r = ctx.ot_solve(Cd, nud, mud, 0.1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = ctx.ot_solve(Cd, nud, mud, 0.1, plan=r.plan)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    st = r.stats
    ctx.close()
    return {"workload": "optimal transport, 1000 x 1000 points U[0,1]^2 vs U[1,2]x[0,1], "
                        "random masses, squared-Euclidean, eps=0.1 seed=11",
            "ms_per_solve": round(ms, 4), "ms_prepare": round(st["ms_build"], 4),
            "ms_loop": round(st["ms_loop_kernel"], 4), "copies_b": st["copies_b"],
            "copies_a": st["copies_a"], "phases": st["phases"], "rounds": st["rounds"],
            "scanned": st["scanned"], "cost": st["cost"],
            "repaired_mass": st["repaired_mass"]}


CLUSTER_EPS = (0.1, 0.01)  # --cluster-eps narrows it (one workload per kernel trace)


def bench_transport_clustered(prot, synth, torch, reps=5):
    """Optimal transport with each point's copies kept as two dual clusters
    (Section 4, Lemma 4.1) on the clouds of the transport leg: eps = 0.1
    (beside the explicit copies) and eps = 0.01 (theta = 400,000 copies a
    side, past what explicit copies allow). Whole solves, inputs in HBM."""
    C, nu, mu = synth.transport_clouds(1000, 1000, seed=11, shift=1.0)
    Cd, nud, mud = (torch.from_numpy(x).cuda() for x in (C, nu, mu))
    ctx = prot.Context(0)
    out = {}
    for eps in CLUSTER_EPS:
        r = ctx.ot_solve(Cd, nud, mud, eps, clustered=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = ctx.ot_solve(Cd, nud, mud, eps, plan=r.plan, clustered=True)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        st = r.stats
        out[f"eps_{eps}"] = {
            "workload": "optimal transport, 1000 x 1000 points U[0,1]^2 vs U[1,2]x[0,1], "
                        f"random masses, squared-Euclidean, eps={eps} seed=11, copies as "
                        "two dual clusters per point",
            "ms_per_solve": round(ms, 4), "ms_prepare": round(st["ms_build"], 4),
            "ms_loop": round(st["ms_loop_kernel"], 4), "copies_b": st["copies_b"],
            "copies_a": st["copies_a"], "phases": st["phases"], "rounds": st["rounds"],
            "us_per_phase": round(1e3 * st["ms_loop_kernel"] / max(1, st["phases"]), 2),
            "scanned": st["scanned"], "cost": st["cost"],
            # the loop reads each scanned position's int16 cost once: its rate
            # against the HBM peak (the loop is bound by hand-over and barrier
            # latency, not by bytes)
            "scan_GBps": round(2.0 * st["scanned"] / (st["ms_loop_kernel"] * 1e-3) / 1e9, 2),
            "scan_frac_of_hbm_peak": round(2.0 * st["scanned"] / (st["ms_loop_kernel"] * 1e-3)
                                           / 1e9 / HBM_PEAK_GBS, 6),
            "repaired_mass": st["repaired_mass"]}
    ctx.close()
    return out


def bench_cost_variants(prot, synth, torch, reps=5):
    """Section 5's two workloads with their own costs: n = 10,000 uniform
    points in the unit square with the plain Euclidean cost (eps = 0.01),
    and n = 10,000 stroke images of 784 pixels with half the L1 distance of
    the normalised images (eps = 0.1). Whole solves, inputs in HBM."""
    out = {}
    cases = [("euclidean", synth.uniform_points(10000, 2, seed=0), 0.01,
              "n=10000 points U[0,1]^2 Euclidean eps=0.01 seed=0"),
             ("l1_normalized", (synth.digit_images(10000, seed=31),
                                synth.digit_images(10000, seed=32)), 0.1,
              "n=10000 28x28 stroke images, L1 of normalised images / 2, eps=0.1")]
    for metric, (X, Y), eps, name in cases:
        Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
        ctx = prot.Context(0)
        ctx.set_cost_metric(metric)
        r = ctx.solve_points(Xd, Yd, eps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = ctx.solve_points(Xd, Yd, eps)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        st = r.stats
        ctx.close()
        out[metric] = {"workload": name, "ms_per_solve": round(ms, 4),
                       "ms_build": round(st["ms_build"], 4),
                       "ms_loop": round(st["ms_loop_kernel"], 4), "phases": st["phases"],
                       "rounds": st["rounds"], "scanned": st["scanned"], "cost": st["cost"]}
    return out


def bench_ot_loss(prot, synth, torch, reps=5):
    """64 instances, n = 2048, X ~ N(0, I_64), Y ~ N(0.5, I_64), eps = 0.01:
    forward (batched solve + loss) and hand-written backward."""
    X, Y = synth.shifted_gaussian_batch(64, 2048, 64, 0.5, seed=0)
    Xd = torch.from_numpy(X).cuda().requires_grad_(True)
    Yd = torch.from_numpy(Y).cuda().requires_grad_(True)
    prot.ot_match_loss(Xd, Yd, 0.01).sum().backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        Xd.grad = None
        Yd.grad = None
        prot.ot_match_loss(Xd, Yd, 0.01).sum().backward()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    # the batched solve alone (the plan the loss reuses), and what it did
    import numpy as np
    plan = prot.context(0).cached_batch([2048] * 64, 64, 0.01)
    Xp, Yp = Xd.detach().view(64 * 2048, 64), Yd.detach().view(64 * 2048, 64)
    plan.run(Xp, Yp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.run(Xp, Yp, check=False)
    torch.cuda.synchronize()
    solve_ms = 1e3 * (time.perf_counter() - t0) / reps
    st = plan.stats()
    return {"workload": "64 x n=2048, R^64, X~N(0,I), Y~N(0.5,I), eps=0.01",
            "fwd_bwd_ms": round(ms, 3), "batched_solve_ms": round(solve_ms, 3),
            "mean_phases": round(float(np.mean([x["phases"] for x in st])), 2),
            "mean_rounds": round(float(np.mean([x["rounds"] for x in st])), 2),
            "scanned_total": int(sum(x["scanned"] for x in st))}


def phase_report(prot, synth, torch, n, d, eps, seed, storage="auto", rounds_of=None):
    """Per-phase evidence for the phase loop: |B'|, proposal rounds, entries
    examined, |M'|, the phase's device time from the per-round timestamps
    (PROT_DEBUG_ROUND_TIMES; the timestamps add a little time of their own)
    and the useful scan rate (2 B per entry examined / time)."""
    import numpy as np
    os.environ["PROT_DEBUG_ROUND_TIMES"] = "1"
    X, Y = synth.uniform_points(n, d, seed=seed)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    ctx = prot.Context(0)
    if storage == "matrix":
        ctx.reserve(n, with_matrix=True)
    for _ in range(3):
        res = ctx.solve_points(Xd, Yd, eps, storage=storage)
    torch.cuda.synchronize()
    tr = ctx.trace()
    rt = ctx.round_times()
    ctx.close()
    loop_us = 1e3 * res.stats["ms_loop_kernel"]
    # last exit (100 MHz ticks) of every phase's rounds
    ends = {}
    for arr, ex, ph in rt:
        ends[int(ph)] = max(ends.get(int(ph), 0), int(ex))
    phases = len(tr)
    dur = np.zeros(phases)
    for p in range(1, phases):
        if p in ends and p - 1 in ends:
            dur[p] = (ends[p] - ends[p - 1]) / 100.0
    dur[0] = max(loop_us - dur[1:].sum(), 0.0)  # phase 0 also holds the launch
    print(f"# per-phase report: n={n} d={d} eps={eps} seed={seed} storage={storage}; "
          f"loop {loop_us:.1f} us with round timestamps on", flush=True)
    print(f"{'phase':>5s} {'|B_i|':>7s} {'rounds':>6s} {'entries':>11s} {'|M_i|':>6s} "
          f"{'us':>8s} {'GB/s':>8s}")
    for p in range(phases):
        gbs = 2.0 * tr[p, 2] / (dur[p] * 1e-6) / 1e9 if dur[p] > 0 else 0.0
        print(f"{p:5d} {tr[p, 0]:7d} {tr[p, 1]:6d} {tr[p, 2]:11d} {tr[p, 3]:6d} {dur[p]:8.1f} "
              f"{gbs:8.1f}")
    if rounds_of is not None:
        # round r's exit minus the previous round's exit (the first round of
        # the phase: minus the previous phase's last exit)
        prev = None
        print(f"# rounds of phase {rounds_of}: exit-to-exit us, latest arrival to exit us")
        for i, (arr, ex, ph) in enumerate(rt):
            if int(ph) == rounds_of and ex > 0 and prev is not None:
                print(f"round {i:4d}  {(ex - prev) / 100.0:8.2f}  {(ex - arr) / 100.0:8.2f}")
            if ex > 0:
                prev = int(ex)
    tot = 2.0 * tr[:, 2].sum()
    print(f"total: {tr[:, 2].sum()} entries, {tot / 1e6:.1f} MB useful in {loop_us:.1f} us = "
          f"{tot / (loop_us * 1e-6) / 1e9:.1f} GB/s (bytes-weighted over the phases)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--d", type=int, default=2)
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-reps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and OT-loss measurements")
    ap.add_argument("--phase-report", action="store_true",
                    help="print a per-phase table of the phase loop instead of the bench line")
    ap.add_argument("--storage", default="auto", choices=["auto", "matrix", "on_the_fly"],
                    help="rounded costs of the timed solves (and of --phase-report): as the "
                         "library chooses, the stored matrix, or recomputed in the scan")
    ap.add_argument("--only", default=None,
                    choices=["batched", "ot_loss", "uniform_costs", "large", "large_matrix",
                             "unbalanced", "transport", "transport_clustered",
                             "cost_variants"],
                    help="run only this extra measurement and print its JSON (for profiling)")
    ap.add_argument("--cluster-eps", type=float, default=None,
                    help="run the clustered-transport leg at this eps only")
    ap.add_argument("--rounds-of", type=int, default=None,
                    help="with --phase-report: also list the rounds of this phase")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after the bench, run 5 plain device copies of this many MiB "
                         "(reference kernel for scaling memory counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for {args.gpus}); "
              "the solver has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2203_03732_amd as prot
    from paper_2203_03732_amd import synth

    torch.cuda.set_device(0)
    if args.cluster_eps is not None:
        global CLUSTER_EPS
        CLUSTER_EPS = (args.cluster_eps,)
    n, d, eps = args.n, args.d, args.eps
    if args.phase_report:
        phase_report(prot, synth, torch, n, d, eps, args.seed, args.storage, args.rounds_of)
        return
    legs = {"batched": bench_batched, "ot_loss": bench_ot_loss,
            "uniform_costs": bench_uniform_costs, "large": bench_large,
            "large_matrix": bench_large_matrix, "unbalanced": bench_unbalanced,
            "transport": bench_transport, "transport_clustered": bench_transport_clustered,
            "cost_variants": bench_cost_variants}
    if args.only:
        print(json.dumps({args.only: legs[args.only](prot, synth, torch)}), flush=True)
        return
    X, Y = synth.uniform_points(n, d, seed=args.seed)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    ctx = prot.Context(0)
    ctx.reserve(n, with_matrix=True)

    storage = args.storage
    for _ in range(args.warmup):
        ctx.solve_points(Xd, Yd, eps, storage=storage)
    torch.cuda.synchronize()

    # The timed steps are enqueued back to back (stats=False: each solve's
    # statistics stay in device memory, nothing synchronises between steps);
    # the loop kernel's device time of every timed step comes from the
    # events its launch carries, read after the timed region.
    timing = "enqueued back to back"
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.solve_points(Xd, Yd, eps, storage=storage, stats=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    try:
        ok = ctx.status() == "ok"
    except prot.ProtError as e:
        print(f"bench: a solve enqueued without statistics failed ({e}); timing solves that "
              "read their statistics back instead", file=sys.stderr)
        ok = False
    if not ok:
        # (a solve that reads its statistics back retries a launch the GPU
        # could not hold whole, which an enqueued one cannot)
        timing = "one synchronised solve at a time"
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.solve_points(Xd, Yd, eps, storage=storage)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    # (the context keeps the events of the last 1,024 launches)
    loop_ms = list(ctx.loop_times(min(args.steps, 1024)))
    assert len(loop_ms) == min(args.steps, 1024)
    # statistics of the same solve (deterministic), and the rate of solves
    # that read their statistics back one by one
    n_sync = max(1, min(args.steps, 50))
    build_ms, scanned = [], []
    t0 = time.perf_counter()
    for _ in range(n_sync):
        res = ctx.solve_points(Xd, Yd, eps, storage=storage)
        build_ms.append(res.stats["ms_build"])
        scanned.append(res.stats["scanned"])
    torch.cuda.synchronize()
    ms_per_solve_sync = 1e3 * (time.perf_counter() - t0) / n_sync
    st = res.stats

    # algorithmic bytes per launch
    loop_bytes = 2.0 * float(np.mean(scanned))
    build_bytes = 2.0 * n * prot.pitch(n) + 2 * 2 * n * d * 4
    mean_loop, mean_build = float(np.mean(loop_ms)), float(np.mean(build_ms))
    # names as the kernel trace shows them (the library recomputes the costs
    # in the scan, for d = 2, 3, when asked or when the int16 matrix would
    # exceed 256 MiB)
    on_the_fly = storage == "on_the_fly" or (
        storage == "auto" and d in (2, 3) and 2 * n * prot.pitch(n) > (256 << 20))
    loop_name = f"phase_loop_kernel<false, {d if on_the_fly else 0}, false, false, false>"
    if on_the_fly:
        build_bytes = 2 * 2 * n * d * 4  # the points only
    kernels = {
        loop_name: {"bound": "hbm", "ms": mean_loop, "bytes": loop_bytes},
        "cost_build": {"bound": "hbm", "ms": mean_build, "bytes": build_bytes},
    }
    dom_name = max(kernels, key=lambda k: kernels[k]["ms"])
    dom = kernels[dom_name]
    achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    roofline = {"bound": dom["bound"], "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic(n, d, dom_name, storage), "kernel": dom_name,
                "algorithmic_bytes": round(dom["bytes"], 1)}

    out = {
        "metric": METRIC,
        "value": round(ms_per_step, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16",
        "data": "synthetic",
        "config": {"workload": f"assignment n={n} points U[0,1]^{d} squared-Euclidean "
                               f"eps={eps} seed={args.seed}",
                   "n": n, "d": d, "eps": eps, "storage": storage, "parallelism": "single-gpu"},
        "solves_per_s": round(1e3 / ms_per_step, 3),
        # steps enqueued back to back; a solve that also reads its
        # statistics back (one host synchronisation per solve) takes this
        "ms_per_solve_reading_stats": round(ms_per_solve_sync, 4),
        "timed_steps": timing,
        "phase_scan_GBps": round(loop_bytes / (mean_loop * 1e-3) / 1e9, 2),
        "kernels_ms": {k: round(v["ms"], 5) for k, v in kernels.items()},
        "solve": {s: st[s] for s in ("phases", "rounds", "max_rounds", "scanned", "sum_free",
                                     "completed_pairs", "sum_k")} | {"cost": st["cost"]},
        "roofline": roofline,
    }
    ctx.close()
    if not args.no_extras:
        for name, leg in legs.items():
            out[name] = leg(prot, synth, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, Y, eps, args.cpu_reps)
    print(json.dumps(out), flush=True)
    if args.copy_calibration_mb:
        nbytes = args.copy_calibration_mb << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes}), flush=True)


if __name__ == "__main__":
    main()
