"""Throughput benchmark: all-pairs shortest paths by blocked Floyd-Warshall on one MI355X.

Metric (arXiv:1902.04446, Sec. 5.4): cell updates per second, n^3 / t, for one
APSP solve.  Workload: k-nearest-neighbour graph (k = 10, union-symmetrised)
over 16384 seeded Swiss-roll points with N(0, 0.05^2) noise, fp32 Euclidean
edge weights, dense 16384 x 16384 fp32 matrix (1 GiB), +inf for non-edges.

One step = restore the input matrix from a pristine device copy, then one full
solve (input normalisation + all 128 rounds of phases 1-3).  The matrix is in
HBM before timing starts.  The timed region is exactly ``--steps`` steps,
bracketed by device synchronisation.

Besides the headline line, the JSON carries
  roofline     the phase-3 kernel (min-plus tile update, ~98% of the work):
               algorithmic cell updates / its event-timed duration, as fp32
               operations (an add and a min per update) against MI355X's
               published fp32 vector peak (see ``FP32_PEAK_FLOPS``), with the
               instruction set's and the measured instruction mix's ceilings;
  cpu_baseline the host oracle (plain Floyd-Warshall in fp64, all host cores)
               timed on a bounded sample of the same workload: the first
               pivots of the n = 16384 problem, scaled by n / pivots (every
               pivot step costs the same, the loop being data-independent).
Progress goes to stderr; the one JSON line goes to stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peak of the VALU for this arithmetic, from MI355X's unit counts and clock:
# 256 CUs x 2.4 GHz x 128 fp32 lanes per clock x 2 flops (a fused multiply-add)
# = 157.3 TFLOP/s, the published fp32 vector figure.  A min-plus cell update is
# two fp32 operations, an add and a min (no multiply-add: it cannot fuse), so
# against that figure an update counts 2 ops and the peak is 78.6 T updates/s.
# Two ceilings below it bound what this instruction set can reach:
#   ISA_FRAC    updates take 1.5 lane-instructions (c = min3(c, a0+b0, a1+b1)
#               folds two updates into 2 adds + 1 min3), 4 ops per 3 lane-slots
#               against the 2 ops per lane-slot of an FMA: 2/3 of the peak;
#   the measured register-only update mix (VALU probe, reported live): about
#               0.58 of the peak, since the 3-operand min3 issues at half the
#               add's lane rate.
CUS, CLOCK_HZ = 256, 2.4e9
FP32_LANES_PER_CLK = 128
FP32_PEAK_FLOPS = CUS * CLOCK_HZ * FP32_LANES_PER_CLK * 2   # 157.3e12
OPS_PER_UPDATE = 2                                          # one add, one min
PEAK_UPD = FP32_PEAK_FLOPS / OPS_PER_UPDATE                 # 78.6e12 updates/s
ISA_FRAC = (4 / 3) / 2                                      # 0.667 of the peak

PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "traffic_phase3_swiss16384_f32.txt")
# the phase-3 kernel and the schedule that launches it (the traffic figures
# hold while these sources are unchanged)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1902_04446_amd", "csrc", f)
                  for f in ("apsp_plain.hip", "apsp_pair.hip", "apsp_tile.h", "apsp_tilemap.h",
                            "apsp_runtime.hip")]


def cell_updates_per_s(n: int, seconds: float) -> float:
    """Throughput of one APSP solve: n^3 cell updates over the wall time (Sec. 5.4)."""
    return float(n) ** 3 / seconds


def log(msg: str) -> None:
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def phase3_rest_updates(n: int, b: int) -> tuple[int, int]:
    """Algorithmic cell updates of the phase-3 "rest" launches of one solve
    (every round r but the last: the entries outside block rows/columns r and
    r+1, each with |K_r| candidates) and the number of such launches."""
    q = -(-n // b)
    total = 0
    for r in range(q - 1):
        kw = min(b, n - r * b)
        kw1 = min(b, n - (r + 1) * b)
        total += (n - kw - kw1) ** 2 * kw
    return total, q - 1


def phase3_pair_updates(n: int, b: int) -> tuple[int, int]:
    """The same for the round-pair schedule: one rest launch group per pair of
    rounds (r, r+1), over the entries outside block rows/columns r .. r+3, each
    with |K_r| + |K_r+1| candidates, plus round r-1's deferred update of the
    previous pair's block row/column r-2 that those launches apply; and the
    number of pairs.  With an odd round count the last round runs alone."""
    q = -(-n // b)

    def w(x):
        return min(b, n - x * b) if 0 <= x < q else 0

    total, pairs = 0, 0
    r = 0
    while r + 1 < q:
        excl = sum(w(x) for x in range(r, min(r + 4, q)))
        out = n - excl
        total += out * out * (w(r) + w(r + 1))
        if r >= 2:
            p = r - 2
            side = out - w(p + 1)
            total += (2 * w(p) * side - w(p) * w(p)) * w(p + 1)
        pairs += 1
        r += 2
    return total, pairs


def valu_probe() -> dict | None:
    """Measured lane-instruction rates of the update's instructions on this GPU."""
    import ctypes

    path = os.path.join(ROOT, "paper_1902_04446_amd", "libapsp_probe.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    rates = (ctypes.c_double * 4)()
    if lib.apsp_probe_valu_rates(rates) != 0:
        return None
    add_f32, add_u32, min3_i32, min3_u32 = (float(x) for x in rates)
    ceiling = 1.0 / (1.0 / add_f32 + 0.5 / min3_i32)
    mix = ctypes.c_double(0.0)
    mix_t = mix.value / 1e12 if lib.apsp_probe_update_mix(ctypes.byref(mix)) == 0 else None
    return {"unit": "T lane-instr/s", "v_add_f32": round(add_f32 / 1e12, 2),
            "v_add_u32": round(add_u32 / 1e12, 2), "v_min3_i32": round(min3_i32 / 1e12, 2),
            "v_min3_u32": round(min3_u32 / 1e12, 2),
            "standalone_rates_in_sequence_T": round(ceiling / 1e12, 2),
            "update_mix_T_updates_per_s": round(mix.value / 1e12, 2) if mix_t else None}


def phase3_traffic() -> float | None:
    """HBM bytes per phase-3 launch from the committed rocprofv3 counter runs,
    or None when the kernel source changed since those counters were taken."""
    import hashlib

    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    src = h.hexdigest()
    if kv.get("kernel_source_sha256") != src:
        return None
    return float(kv["bytes_per_launch"])


def cpu_model() -> str | None:
    """The host CPU's model name (as lscpu prints it, from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(n: int, u, v, w, target_s: float) -> dict:
    """Time the host oracle on pivots of the same workload, on all host threads
    (``target_s`` of work) and on one thread (a quarter of it).

    Every pivot step of the plain Floyd-Warshall loop does the same n^2 updates
    whatever the data (it is branch-free), so the rate over k pivots is the
    rate of the whole solve, which is projected as n / k times the sample."""
    import numpy as np

    import graphgen as gg
    import oracle

    threads = oracle.max_threads()
    W = gg.dense_from_edges(n, u, v, w, np.float32)
    D = oracle.prepare(W)
    del W

    def sample(k0: int, budget: float, nthreads: int):
        t0 = time.perf_counter()
        oracle.fw_steps(D, k0, k0 + 2, threads=nthreads)
        per = (time.perf_counter() - t0) / 2
        k = int(max(2, min(n - k0 - 2, budget / max(per, 1e-9))))
        t0 = time.perf_counter()
        oracle.fw_steps(D, k0 + 2, k0 + 2 + k, threads=nthreads)
        dt = time.perf_counter() - t0
        return k0 + 2, k, dt, k * float(n) ** 2 / dt

    k0, k, dt, rate = sample(0, target_s, threads)
    log(f"cpu baseline: {k} pivots on {threads} threads in {dt:.1f} s")
    k1_0, k1, dt1, rate1 = sample(k0 + k, target_s / 4, 1)
    log(f"cpu baseline: {k1} pivots on 1 thread in {dt1:.1f} s")
    return {"value": rate / 1e9, "unit": "G cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"pivots {k0}..{k0 + k - 1} of the n={n} fp64 Floyd-Warshall loop on "
                      f"{threads} threads ({k} of {n} pivots, {dt:.1f} s); every pivot step "
                      f"costs the same, so the full solve projects to {n / k * dt:.0f} s",
            "single_thread": {"value": rate1 / 1e9, "unit": "G cell-updates/s", "cores": 1,
                              "sample": f"pivots {k1_0}..{k1_0 + k1 - 1} ({k1} pivots, "
                                        f"{dt1:.1f} s); full solve projects to "
                                        f"{n / k1 * dt1:.0f} s"},
            "cpu_model": cpu_model(), "host_threads": os.cpu_count()}


def bench_batched(apsp, torch, dev, count: int, reps: int, loop_too: bool = True,
                  profile_only: bool = False) -> dict:
    """Many small graphs: one batched launch vs a loop of single-graph solves.

    4096 ER graphs, n log-uniform in [32, 512], p = 8/n, int32 U{1..1000}.
    The metric is sum(n_i^3) / t over the whole batch.  ``profile_only``:
    exactly one run of a width-128 plan (for a profiler to see one run's
    launches), timed, nothing else.
    """
    import graphgen as gg

    log(f"batched: generating {count} graphs")
    Ws = gg.batched_graphs(count, item=0)
    sum_n3 = float(sum(int(W.shape[0]) ** 3 for W in Ws))
    pristine = [torch.from_numpy(W).to(dev) for W in Ws]
    # each graph in its own buffer with the row length rounded up to 4
    # elements (16-byte rows), the layout the vector loads need
    work = []
    for p_ in pristine:
        n_ = p_.shape[0]
        work.append(torch.empty((n_, (n_ + 3) // 4 * 4), dtype=p_.dtype, device=dev)[:, :n_])

    def reset():
        for w_, p_ in zip(work, pristine):
            w_.copy_(p_)

    def timed(fn):
        best = float("inf")
        for _ in range(reps):
            reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    def same_as(ref):
        return all(torch.equal(a, b) for a, b in zip(ref, work))

    if profile_only:
        reset()
        p_ = apsp.BatchPlan(work, tile=128)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p_.run()
        torch.cuda.synchronize()
        t_one = time.perf_counter() - t0
        info = p_.info()
        p_.close()
        log(f"batched: one width-128 plan run {t_one * 1e3:.2f} ms ({info['launches']} launches)")
        return {"workload": f"{count} ER graphs, n log-uniform [32,512], p=8/n, int32 U{{1..1000}}",
                "profile_only": True, "one_run_ms": round(t_one * 1e3, 3), "plan": info}

    # fixed widths first, then the autotuned table (which plans created after
    # the tuning pick up)
    fixed = {}
    ref = None
    same = True
    for tile in (128, 64):
        p_ = apsp.BatchPlan(work, tile=tile)
        fixed[tile] = (timed(p_.run), p_.info())
        p_.close()
        if ref is None:
            ref = [w_.clone() for w_ in work]
        else:
            same = same and same_as(ref)
    reset()  # the tuner solves copies of the batch as it is now: the inputs
    t0 = time.perf_counter()
    tune = apsp.batched_autotune_batch(work)
    t_tune = time.perf_counter() - t0
    log(f"batched: autotuned widths {tune['widths']} in {t_tune:.2f} s "
        f"(all-128 {tune['ms_all_128']:.3f} ms, tuned {tune['ms_tuned']:.3f} ms)")
    plan = apsp.BatchPlan(work)
    t_batched = timed(plan.run)
    same = same and same_as(ref)
    # the same plan captured once in a HIP graph (its run only launches
    # kernels) and replayed: one submission for all of its launches
    reset()
    torch.cuda.synchronize()
    t_graph = None
    try:
        hip_graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(hip_graph):
            plan.run()
    except RuntimeError as exc:  # reported, not fatal: the eager figures stand
        log(f"batched: HIP graph capture failed: {exc}")
    else:
        t_graph = timed(hip_graph.replay)
        same = same and same_as(ref)
        del hip_graph
    # the same graphs in contiguous n x n buffers (rows off 16 bytes when n %
    # 4 != 0): the plan gives those graphs working copies
    contig = [torch.empty_like(p_) for p_ in pristine]

    def reset_contig():
        for c_, p_ in zip(contig, pristine):
            c_.copy_(p_)

    plan_c = apsp.BatchPlan(contig)
    t_contig = float("inf")
    for _ in range(reps):
        reset_contig()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan_c.run()
        torch.cuda.synchronize()
        t_contig = min(t_contig, time.perf_counter() - t0)
    plan_c.close()
    same = same and all(torch.equal(a, b) for a, b in zip(ref, contig))
    del contig
    t0 = time.perf_counter()
    args = apsp.BatchArgs(work)  # the list marshalled once (Python work, ~1 us per matrix)
    t_marshal = time.perf_counter() - t0
    t_oneshot = timed(lambda: apsp.solve_batched(args))
    same = same and same_as(ref)
    t_noalloc = timed(lambda: apsp.solve_batched_noalloc(args))
    same = same and same_as(ref)
    info = plan.info()
    plan.close()

    def loop():
        for w_ in work:
            apsp.solve(w_)

    t_loop = float("nan")
    if loop_too:
        t_loop = timed(loop)
        same = same and same_as(ref)
    log(f"batched: tuned plan run {t_batched * 1e3:.2f} ms ({info['launches']} launches), "
        f"replayed from a HIP graph {t_graph * 1e3 if t_graph is not None else float('nan'):.2f} ms, "
        f"on contiguous rows (working copies) {t_contig * 1e3:.2f} ms; "
        f"width 128 only {fixed[128][0] * 1e3:.2f} ms, width 64 only {fixed[64][0] * 1e3:.2f} ms; "
        f"one-shot call {t_oneshot * 1e3:.2f} ms, allocation-free call {t_noalloc * 1e3:.2f} ms "
        f"(marshalling the list {t_marshal * 1e3:.2f} ms), per-graph loop {t_loop * 1e3:.2f} ms, "
        f"identical={same}")
    return {"workload": f"{count} ER graphs, n log-uniform [32,512], p=8/n, int32 U{{1..1000}}; "
                        "row length rounded up to 4 elements",
            "sum_n3": sum_n3, "batched_ms": round(t_batched * 1e3, 3),
            "plan": info, "tuned_widths": tune["widths"],
            "autotune_ms_all128_tuned": [round(tune["ms_all_128"], 4), round(tune["ms_tuned"], 4)],
            "autotune_s": round(t_tune, 3),
            "width128_only_ms": round(fixed[128][0] * 1e3, 3),
            "width64_only_ms": round(fixed[64][0] * 1e3, 3),
            "graph_replay_ms": round(t_graph * 1e3, 3) if t_graph is not None else None,
            "contiguous_rows_ms": round(t_contig * 1e3, 3),
            "oneshot_call_ms": round(t_oneshot * 1e3, 3),
            "noalloc_call_ms": round(t_noalloc * 1e3, 3),
            "python_marshal_ms": round(t_marshal * 1e3, 3),
            "plain_loop_ms": round(t_loop * 1e3, 3) if loop_too else None,
            "batched_T_cell_updates_per_s": round(sum_n3 / t_batched / 1e12, 3),
            "plain_loop_T_cell_updates_per_s":
                round(sum_n3 / t_loop / 1e12, 3) if loop_too else None,
            "speedup": round(t_loop / t_batched, 2) if loop_too else None,
            "bit_identical": bool(same)}


# the host policy measured best for p99 at 0.8 C (2000 requests per run):
# first come first served, n = 8192 requests one at a time beside the rest
# (p99 70.9 ms; round-robin 73.5, SRPT 74.1, one request >= 4096 at a time
# 110-141 ms)
SERVING_POLICY = {"slots": 4, "slice_rounds": 8, "inflight": 2, "policy": "fifo",
                  "max_running": None, "large_n": 8192, "max_large": 1}


def bench_serving(apsp, torch, dev, count: int, loads=(0.5, 0.8, 1.2), policy=None,
                  warmup_frac: float = 0.1, capacity=None) -> dict:
    """Poisson stream of APSP requests, n in {256, 1024, 4096, 8192} with
    probabilities {.4, .3, .2, .1}, each a seeded Swiss-roll kNN graph (k=10,
    fp32).  Capacity C = requests per second of back-to-back plain solves of
    the same kind of requests on one stream; the server then runs `count`
    requests at each given fraction of C, the first `warmup_frac` of them
    left out of the latency figures, and reports p50 / p99 latency (overall
    and per size) and cell updates per second.  The lone solve time of each
    size is measured beside it.
    """
    import numpy as np

    import graphgen as gg
    from paper_1902_04446_amd.serving import ApspServer, GpuBackend, Request

    pol = dict(SERVING_POLICY, **(policy or {}))
    per_size = 3
    log("serving: generating the request pool")
    pool = {n: [gg.swiss_roll_knn(n, gg.CFG_SERVING, 10 * n + k) for k in range(per_size)]
            for n in gg.SERVING_SIZES}

    def make(qps, item, cnt=count):
        arr, ns = gg.serving_requests(cnt, qps, item=item)
        return [Request(rid=i, n=int(n), arrival=float(a), payload=pool[int(n)][i % per_size])
                for i, (a, n) in enumerate(zip(arr, ns))]

    # lone solve time of each size (matrix resident, one plain solve)
    lone = {}
    for n in gg.SERVING_SIZES:
        u, v, w = pool[n][0]
        P = gg.device_dense_from_edges(n, u, v, w, np.float32, dev)
        X = torch.empty_like(P)
        ts = []
        for _ in range(6):
            X.copy_(P)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            apsp.solve(X)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        lone[str(n)] = round(sorted(ts[1:])[2] * 1e3, 3)
        del P, X
    log(f"serving: lone solve ms {lone}")

    # capacity: the same kind of requests, one after another, plain solves on
    # one stream; the median of three timed passes after an untimed one over
    # 300 of them
    probe = make(1.0, 0, min(count, 500))
    backend = GpuBackend(dev, slots=1, keep_results=False)

    def plain(reqs):
        for r in reqs:
            D = backend.alloc(r, 0)
            backend.load(D, r, 0)
            apsp.solve(D, stream=backend.streams[0])

    plain(probe[:300])
    passes = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain(probe)
        torch.cuda.synchronize()
        passes.append(time.perf_counter() - t0)
    backend.close()
    t_plain = sorted(passes)[1]
    cap = len(probe) / t_plain
    work = float(sum(float(r.n) ** 3 for r in probe))
    log(f"serving: plain back-to-back {len(probe)} requests in {t_plain:.3f} s "
        f"-> capacity {cap:.1f} req/s, {work / t_plain / 1e12:.2f} T cell-updates/s")
    if capacity is not None:  # a capacity measured earlier (policy sweeps)
        cap = float(capacity)
    runs = []
    warm = int(round(warmup_frac * count))
    for k, f in enumerate(loads):
        qps = f * cap
        reqs = make(qps, k + 1)
        backend = GpuBackend(dev, slots=pol["slots"], keep_results=False)
        srv = ApspServer(backend, hbm_budget=8 << 30, slots=pol["slots"],
                         slice_rounds=pol["slice_rounds"], inflight=pol["inflight"],
                         policy=pol["policy"], max_running=pol["max_running"],
                         large_n=pol["large_n"], max_large=pol["max_large"], warmup=warm)
        st = srv.run(reqs, realtime=True)
        backend.close()
        st["load"] = f
        st["qps"] = round(qps, 2)
        for key in ("p50_ms", "p99_ms", "mean_ms"):
            st[key] = round(st[key], 3) if st[key] is not None else None
        for v in st["per_size"].values():
            for key in ("p50_ms", "p99_ms", "max_ms"):
                v[key] = round(v[key], 3)
        st["p99_over_lone_8192"] = round(st["p99_ms"] / lone["8192"], 3) if st["p99_ms"] else None
        st["T_cell_updates_per_s"] = round(st.pop("cell_updates_per_s") / 1e12, 3)
        st["makespan_s"] = round(st["makespan_s"], 3)
        log(f"serving: load {f:.1f}C ({qps:.0f} req/s): p50 {st['p50_ms']} ms, "
            f"p99 {st['p99_ms']} ms ({st['p99_over_lone_8192']} x lone 8192), "
            f"{st['T_cell_updates_per_s']} T cell-updates/s; per size "
            + ", ".join(f"{n}: {v['p50_ms']}/{v['p99_ms']}" for n, v in st["per_size"].items()))
        runs.append(st)
    return {"workload": "Poisson arrivals, n in {256,1024,4096,8192} w.p. {.4,.3,.2,.1}, "
                        "Swiss-roll kNN fp32", "requests_per_run": count,
            "warmup_excluded": warm, "lone_solve_ms": lone,
            "plain_capacity_req_per_s": round(cap, 2), "capacity_probe_requests": len(probe),
            "capacity_probe_passes_s": [round(x, 3) for x in passes],
            "plain_T_cell_updates_per_s": round(work / t_plain / 1e12, 3),
            "policy": pol, "hbm_budget_GiB": 8, "runs": runs}


def bench_variants(apsp, torch, dev, pristine, work, n: int, b: int) -> dict:
    """The other solvers on the same device, measured beside the headline:
    the symmetric (upper-triangle) variant on the same n = 16384 input, a
    standalone 8192^3 min-plus product, repeated squaring vs the blocked
    method on a 4096-vertex Swiss-roll graph, and an int32 solve at n."""
    import numpy as np

    import graphgen as gg

    def timed(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    out = {}
    # symmetric variant: executed updates = upper panel and upper phase-3 blocks
    def sym():
        work.copy_(pristine)
        apsp.solve_symmetric(work)

    def full():
        work.copy_(pristine)
        apsp.solve(work)

    t_sym, t_full = timed(sym), timed(full)
    sym()
    ref = work.clone()
    full()
    q = -(-n // b)
    executed = sum(((q - 1) + (q - 1) * q // 2) * b ** 3 for _ in range(q)) + q * b ** 3
    out["symmetric"] = {"n": n, "ms": round(t_sym * 1e3, 3), "full_ms": round(t_full * 1e3, 3),
                        "T_cell_updates_per_s_n3": round(float(n) ** 3 / t_sym / 1e12, 3),
                        "executed_updates": executed,
                        "T_executed_updates_per_s": round(executed / t_sym / 1e12, 3),
                        "identical_to_full": bool(torch.equal(ref, work))}
    log(f"variants: symmetric {t_sym * 1e3:.1f} ms vs full {t_full * 1e3:.1f} ms")
    del ref
    # min-plus product
    m = 8192
    g = torch.Generator(device=dev)
    g.manual_seed(1902)
    A = torch.rand((m, m), device=dev, generator=g) * 10
    B = torch.rand((m, m), device=dev, generator=g) * 10
    C = torch.empty((m, m), device=dev)
    t_mp = timed(lambda: apsp.minplus(C, A, B))
    out["minplus"] = {"m": m, "n": m, "k": m, "dtype": "f32", "ms": round(t_mp * 1e3, 3),
                      "T_cell_updates_per_s": round(float(m) ** 3 / t_mp / 1e12, 3)}
    log(f"variants: min-plus {m}^3 in {t_mp * 1e3:.1f} ms")
    del A, B, C
    # repeated squaring vs blocked
    ns = 4096
    u, v, w = gg.swiss_roll_knn(ns, gg.CFG_TEST, 4096)
    P = gg.device_dense_from_edges(ns, u, v, w, np.float32, dev)
    X = torch.empty_like(P)
    Y = torch.empty_like(P)

    def squaring():
        X.copy_(P)
        apsp.solve_squaring(X, Y)

    def blocked():
        X.copy_(P)
        apsp.solve(X)

    t_sq, t_bl = timed(squaring), timed(blocked)
    out["squaring"] = {"n": ns, "squarings": apsp.squarings(ns), "ms": round(t_sq * 1e3, 3),
                       "blocked_ms": round(t_bl * 1e3, 3),
                       "T_product_updates_per_s": round(
                           apsp.squarings(ns) * float(ns) ** 3 / t_sq / 1e12, 3)}
    log(f"variants: squaring n={ns} {t_sq * 1e3:.1f} ms vs blocked {t_bl * 1e3:.1f} ms")
    del P, X, Y
    # int32 at the headline size: random weights U{1..100} on every pair, so
    # 2 (n-1) wmax < 2^24 and the tiles run on the fp32 pipe (exactly)
    g2 = torch.Generator(device=dev)
    g2.manual_seed(1902)
    Pi = torch.randint(1, 101, (n, n), dtype=torch.int32, device=dev, generator=g2)
    Xi = torch.empty_like(Pi)

    def int_solve():
        Xi.copy_(Pi)
        apsp.solve(Xi)

    t_int = timed(int_solve)
    out["int32_solve"] = {"n": n, "weights": "U{1..100} dense", "ms": round(t_int * 1e3, 3),
                          "T_cell_updates_per_s": round(float(n) ** 3 / t_int / 1e12, 3)}
    log(f"variants: int32 solve n={n} {t_int * 1e3:.1f} ms")
    # The same fp32 kernels on other data: the GPU is power-limited and the
    # power depends on how many bits the operands toggle.
    Pf = Pi.float()
    del Pi, Xi
    Xf = torch.empty_like(Pf)

    def f32_solve():
        Xf.copy_(Pf)
        apsp.solve(Xf)

    t_fint = timed(f32_solve)
    Pf.uniform_(0.5, 1.5, generator=g2)
    t_frand = timed(f32_solve)
    out["data_sensitivity"] = {
        "n": n, "swiss_roll_ms": round(t_full * 1e3, 3),
        "f32_integer_valued_U1_100_ms": round(t_fint * 1e3, 3),
        "f32_uniform_0.5_1.5_ms": round(t_frand * 1e3, 3)}
    log(f"variants: fp32 solve n={n}: integer-valued weights {t_fint * 1e3:.1f} ms, "
        f"uniform [0.5, 1.5) {t_frand * 1e3:.1f} ms, Swiss roll {t_full * 1e3:.1f} ms")
    del Pf, Xf
    return out


def bench_stretch(apsp, torch, dev, rounds: int) -> dict:
    """n = 262144 (a 256 GiB fp32 matrix, the paper's largest problem) on one GPU.

    A full solve takes minutes, so a few rounds are timed and the solve time
    is projected as rounds x the time of one: every round does the same work
    (2(q-1) panel tiles and (q-1)^2 update tiles, n being a multiple of 128)
    and the kernels do not branch on the data.  Their power draw does,
    though: adds on +inf (no edge yet) toggle few bits, and the first rounds
    of a kNN graph this size see almost nothing else, so they run at a
    higher clock than the bulk of a solve.  The graph therefore gets hub
    edges (a star over vertices 0..383 and an edge from every other vertex
    to one of them), which make every entry finite after 3 rounds, and the
    timed rounds come after those 3.  An even count of timed rounds runs as
    whole pairs of rounds, as a full solve does.
    """
    import numpy as np

    import graphgen as gg

    n = 262144
    need = n * n * 4
    free, _ = torch.cuda.mem_get_info()
    if free < need + (4 << 30):
        log(f"stretch: skipped, {free / 2**30:.0f} GiB free < {need / 2**30:.0f} GiB + 4 GiB")
        return {"n": n, "skipped": f"{free / 2**30:.0f} GiB of device memory free"}
    b = apsp.round_width(n, apsp.APSP_F32)
    q = -(-n // b)
    fill_rounds = 3
    log(f"stretch: building Swiss-roll kNN graph n={n} with hub edges (256 GiB matrix)")
    u, v, w = gg.swiss_roll_knn(n, gg.CFG_SWISS_256K, 0)
    u, v, w = gg.with_hub_edges(n, u, v, w, fill_rounds * b, gg.rng_for(gg.CFG_SWISS_256K, 1))
    D = gg.device_dense_from_edges(n, u, v, w, np.float32, dev)
    del u, v, w
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    apsp.solve_rounds(D, 0, fill_rounds)  # normalisation + rounds that fill every entry
    torch.cuda.synchronize()
    t_fill = time.perf_counter() - t0
    t0 = time.perf_counter()
    apsp.solve_rounds(D, fill_rounds, fill_rounds + rounds)
    torch.cuda.synchronize()
    t_rounds = time.perf_counter() - t0
    del D
    torch.cuda.empty_cache()
    per_round = t_rounds / rounds
    projected = per_round * q
    log(f"stretch: rounds 0..{fill_rounds - 1} {t_fill / fill_rounds * 1e3:.1f} ms each, rounds "
        f"{fill_rounds}..{fill_rounds + rounds - 1} {per_round * 1e3:.1f} ms each; projected "
        f"solve {projected:.0f} s")
    return {"n": n, "matrix_GiB": need / 2**30, "round_width": b, "rounds": q,
            "workload": "Swiss-roll kNN (k=10, union) plus hub edges, fp32",
            "rounds_timed": rounds, "first_timed_round": fill_rounds,
            "ms_per_round": round(per_round * 1e3, 2),
            "fill_rounds_ms_each": round(t_fill / fill_rounds * 1e3, 2),
            "projected_solve_s": round(projected, 1),
            "projected_T_cell_updates_per_s": round(float(n) ** 3 / projected / 1e12, 3)}


def rest_roofline(phases: dict, K: int, n: int, b: int) -> dict:
    """Roofline entry of the dominant phase-3 kernel from K profiled solves
    (summed phase times in ms)."""
    q = -(-n // b)
    rest_upd, rest_launches = phase3_rest_updates(n, b)
    pair_upd, pair_launches = phase3_pair_updates(n, b)
    launches = phases["phase3_rest_launches"] / K
    if q >= 3 and launches == pair_launches:
        kernel = ("k_pair_rest_direct, kRest2 (phase 3 of a pair of rounds in one pass, k "
                  "over two blocks, outside block rows/columns r .. r+3; 128x128 tiles, "
                  "operands staged straight into LDS; two concurrent launches per pair, one "
                  "per band of block rows; per-launch figures are per pair of rounds)")
        launch_s = phases["phase3_rest"] / K / 1e3 / pair_launches
        per_launch = pair_upd / pair_launches
    elif q >= 3 and launches == rest_launches:
        kernel = ("k_tiles<kRest> (phase 3 minus block row/column r+1, 128x128 tiles; two "
                  "concurrent launches per round, one per band of block rows; per-launch "
                  "figures are per round)")
        launch_s = phases["phase3_rest"] / K / 1e3 / rest_launches
        per_launch = rest_upd / rest_launches
    else:  # no lookahead split at this size: whole phase 3 in one launch per round
        kernel = "k_tiles<kAll> (phase 3, 128x128 tiles)"
        launch_s = phases["phase3"] / K / 1e3 / q
        per_launch = sum((n - min(b, n - r * b)) ** 2 * min(b, n - r * b) for r in range(q)) / q
    achieved = per_launch / launch_s
    return {
        "bound": "alu",
        "kernel": kernel,
        "achieved": round(achieved * OPS_PER_UPDATE / 1e12, 3),
        "peak": round(FP32_PEAK_FLOPS / 1e12, 2),
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_UPD, 4),
        "traffic": None,
        "ops_per_update": OPS_PER_UPDATE,
        "achieved_T_cell_updates_per_s": round(achieved / 1e12, 3),
        "ceiling_isa_frac": round(ISA_FRAC, 4),
        "per_launch_updates": round(per_launch),
        "avg_launch_ms": round(launch_s * 1e3, 4),
    }


def bench_small(apsp, torch, dev, sizes=(256, 1024, 2048, 4096), reps: int = 20) -> dict:
    """Single solves of small Swiss-roll kNN graphs (fp32, matrix resident):
    median solve time at the library's round width (64 up to n = 5120) and,
    for comparison, with rounds of 128."""
    import numpy as np

    import graphgen as gg

    out = {}
    for n in sizes:
        u, v, w = gg.swiss_roll_knn(n, gg.CFG_SERVING, 10 * n)
        P = gg.device_dense_from_edges(n, u, v, w, np.float32, dev)
        X = torch.empty_like(P)
        res = {"round_width": apsp.round_width(n, apsp.APSP_F32)}
        for label, lim in (("ms", None), ("width128_ms", 0)):
            prev = apsp.set_width64_max_n(lim) if lim is not None else None
            try:
                ts = []
                for i in range(reps + 2):
                    X.copy_(P)
                    a = torch.cuda.Event(enable_timing=True)
                    e = torch.cuda.Event(enable_timing=True)
                    a.record()
                    apsp.solve(X)
                    e.record()
                    torch.cuda.synchronize()
                    if i >= 2:
                        ts.append(a.elapsed_time(e))
            finally:
                if prev is not None:
                    apsp.set_width64_max_n(prev)
            res[label] = round(sorted(ts)[len(ts) // 2], 4)
        res["T_cell_updates_per_s"] = round(float(n) ** 3 / (res["ms"] * 1e-3) / 1e12, 3)
        out[str(n)] = res
        log(f"small: n={n} {res['ms']} ms at width {res['round_width']} "
            f"({res['width128_ms']} ms at 128)")
        del P, X
    return {"workload": "Swiss-roll kNN (k=10, union), fp32; median of "
                        f"{reps} solves, HIP events around apsp_solve", "sizes": out}


def bench_long(apsp, torch, dev, n: int = 65536) -> dict:
    """One full solve of the n = 65536 Swiss-roll kNN workload (16 GiB fp32
    matrix, 512 rounds): whole-solve throughput and per-phase times."""
    import numpy as np

    import graphgen as gg

    need = n * n * 4
    free, _ = torch.cuda.mem_get_info()
    if free < need + (2 << 30):
        return {"n": n, "skipped": f"{free / 2**30:.0f} GiB of device memory free"}
    log(f"long run: building Swiss-roll kNN graph n={n} (16 GiB matrix)")
    u, v, w = gg.swiss_roll_knn(n, gg.CFG_SWISS_64K, 0)
    D = gg.device_dense_from_edges(n, u, v, w, np.float32, dev)
    del u, v, w
    torch.cuda.synchronize()
    b = apsp.round_width(n, apsp.APSP_F32)
    t0 = time.perf_counter()
    t = apsp.solve_profiled(D)
    wall = time.perf_counter() - t0
    del D
    torch.cuda.empty_cache()
    log(f"long run: n={n} solve {t['total']:.0f} ms ({wall:.2f} s wall)")
    return {"n": n, "matrix_GiB": need / 2**30, "round_width": b, "rounds": -(-n // b),
            "workload": "Swiss-roll kNN (k=10, union), fp32",
            "solve_ms": round(t["total"], 1), "wall_s": round(wall, 3),
            "T_cell_updates_per_s": round(float(n) ** 3 / (t["total"] * 1e-3) / 1e12, 3),
            "phase_ms": {k: round(vv, 3) for k, vv in t.items()},
            "roofline": rest_roofline(t, 1, n, b)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--batched", type=int, default=4096,
                    help="graphs in the batched-vs-plain comparison (0 disables it)")
    ap.add_argument("--variants", type=int, default=1,
                    help="measure the symmetric, product and squaring solvers (0 disables)")
    ap.add_argument("--serving", type=int, default=2000,
                    help="requests per serving load level (0 disables the serving section)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU time budget of the oracle baseline sample (0 disables it)")
    ap.add_argument("--batched-loop", type=int, default=1,
                    help="also time the batch as a loop of single-graph solves (0 skips it)")
    ap.add_argument("--batched-profile", type=int, default=0,
                    help="1: the batched section is exactly one width-128 plan run (for profilers)")
    ap.add_argument("--long-run", type=int, default=1,
                    help="one full n=65536 solve with per-phase times (0 disables it)")
    ap.add_argument("--stretch-rounds", type=int, default=4,
                    help="timed rounds of the n=262144 solve (0 disables it)")
    ap.add_argument("--small", type=int, default=1,
                    help="single solves of n = 256 .. 4096 (0 disables them)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the whole matrix lives in one MI355X's HBM and the "
              "library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import graphgen as gg
    import paper_1902_04446_amd as apsp

    n = args.n
    dev = torch.device("cuda:0")
    log(f"building Swiss-roll kNN graph n={n}")
    cfg = {16384: gg.CFG_SWISS_16K, 65536: gg.CFG_SWISS_64K}.get(n, gg.CFG_TEST)
    u, v, w = gg.swiss_roll_knn(n, cfg, 0)
    pristine = gg.device_dense_from_edges(n, u, v, w, np.float32, dev)
    work = torch.empty_like(pristine)
    # a plain elementwise read+write of the matrix: the calibration kernel for
    # the FETCH_SIZE / WRITE_SIZE counter runs (outside the timed region)
    torch.neg(pristine, out=work)
    torch.cuda.synchronize()
    probe = valu_probe()
    if probe:
        log(f"VALU probe: {probe}")
    b = apsp.round_width(n, apsp.APSP_F32)

    def step():
        work.copy_(pristine)
        return apsp.solve_profiled(work)

    for i in range(args.warmup):
        t = step()
        log(f"warmup {i}: {t['total']:.1f} ms")
    torch.cuda.synchronize()
    phases = {"prologue": 0.0, "phase1": 0.0, "phase2": 0.0, "phase3": 0.0, "total": 0.0,
              "phase3_rest": 0.0, "phase3_rest_launches": 0.0, "phase3_other": 0.0}
    t0 = time.perf_counter()
    step_ms = []
    for i in range(args.steps):
        ts = time.perf_counter()
        t = step()  # the profiled solve waits for its own completion
        step_ms.append((time.perf_counter() - ts) * 1e3)
        for key in phases:
            phases[key] += t[key]
        log(f"step {i}: solve {t['total']:.1f} ms (phase3 {t['phase3']:.1f} ms)")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    K = args.steps
    value = K * float(n) ** 3 / elapsed
    phase_ms = {k: round(vv / K, 3) for k, vv in phases.items()}

    q = -(-n // b)
    roofline = rest_roofline(phases, K, n, b)
    roofline["traffic"] = phase3_traffic() if n == 16384 else None
    roofline["solve_frac"] = round(value / PEAK_UPD, 4)
    if probe and probe.get("update_mix_T_updates_per_s"):
        mix = probe["update_mix_T_updates_per_s"] * 1e12
        roofline["ceiling_mix_frac"] = round(mix / PEAK_UPD, 4)
        roofline["frac_of_mix_ceiling"] = round(
            roofline["achieved_T_cell_updates_per_s"] * 1e12 / mix, 4)

    variants = None
    if args.variants:
        variants = bench_variants(apsp, torch, dev, pristine, work, n, b)

    small = bench_small(apsp, torch, dev) if args.small else None

    batched = None
    if args.batched > 0:
        batched = bench_batched(apsp, torch, dev, args.batched, reps=3,
                                loop_too=bool(args.batched_loop),
                                profile_only=bool(args.batched_profile))

    serving = None
    if args.serving > 0:
        serving = bench_serving(apsp, torch, dev, args.serving)

    long_run = None
    if args.long_run > 0 and n != 65536:
        del pristine, work
        torch.cuda.empty_cache()
        pristine = work = None
        long_run = bench_long(apsp, torch, dev)

    stretch = None
    if args.stretch_rounds > 0:
        del pristine, work
        torch.cuda.empty_cache()
        stretch = bench_stretch(apsp, torch, dev, args.stretch_rounds)

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(n, u, v, w, args.cpu_seconds)

    out = {
        "metric": f"APSP cell-updates/s (n^3/t), n={n} FP32",
        "value": round(value / 1e12, 4),
        "unit": "T cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / K * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"blocked Floyd-Warshall, Swiss-roll kNN (k=10, union) n={n}, "
                               "fp32 dense matrix, +inf non-edges",
                   "n": n, "round_width": b, "rounds": q},
        "phase_ms": phase_ms,
        "step_ms": {"min": round(min(step_ms), 3),
                    "median": round(sorted(step_ms)[len(step_ms) // 2], 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "valu_probe": probe,
        "variants": variants,
        "small_solves": small,
        "batched": batched,
        "serving": serving,
        "long_run": long_run,
        "stretch": stretch,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
