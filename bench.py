"""Benchmark of the blip orbital-evaluation hot path on one MI355X.

Workload: the TiO2-supercell-shaped table (18x18x12 bohr cell, 72x72x48
grid, 768 real orbitals, FP32 coefficients N(0,1)/sqrt(S)) evaluated at
quasi-simultaneous move blocks of 1,536 positions (Gaussian sigma = 0.5 bohr
displacements of uniform electron sites, unwrapped).  One step is one
blip_eval of a whole block: FP64 wrap and split, weights, the 64-row
gather-accumulate of value, gradient and Laplacian, and the stores.
Timed steps rotate through 16 independent blocks (different walkers).

Prints ONE JSON line with the metric, the roofline of the evaluation kernel
(algorithmic bytes per launch / average launch time from HIP events on the
launch stream), the plain single-block kernel on the same blocks, and the
FP64 oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "orbital evals/s (val+grad+lap, 768 orbs) & HBM GB/s vs plain; p50/p99 served"
UNIT = "orbital evals/s"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector (and matrix) peak
NROT = 16
COUNTERS = os.path.join(ROOT, "profiles", "tiled_kernel_tio2_block1536_counters.json")
KERNEL_SOURCES = ["paper_1204_1121_amd/csrc/blip_device.hpp",
                  "paper_1204_1121_amd/csrc/blip_launch.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def distinct_rows(lattice, n, pos) -> int:
    """Exact number of distinct coefficient rows a block touches (the U of
    the algorithmic byte count): every site of every position's 4x4x4
    stencil, de-duplicated.  Measurement only."""
    G = np.linalg.inv(np.asarray(lattice, dtype=np.float64))
    u = pos @ G
    u = u - np.floor(u)
    u[u >= 1.0] = 0.0
    nn = np.asarray(n, dtype=np.int64)
    t = u * nn
    i0 = np.floor(t).astype(np.int64)
    i0[i0 >= nn] = 0
    m = np.arange(-1, 3)
    i1 = (i0[:, 0, None] + m) % nn[0]
    i2 = (i0[:, 1, None] + m) % nn[1]
    i3 = (i0[:, 2, None] + m) % nn[2]
    rows = ((i1[:, :, None, None] * nn[1] + i2[:, None, :, None]) * nn[2]
            + i3[:, None, None, :])
    return int(np.unique(rows.reshape(-1)).size)


ELEM_FLOOR = 1e-3


def error_figures(got: dict, ref: dict) -> dict:
    """Per component group (val, grad, lap): the normwise error
    max|y - y*| / max|y*| over the group, and the 99th percentile and maximum
    of the elementwise error |y - y*| / (|y*| + 1e-3 max|y*|) (the floor keeps
    elements next to a node of an orbital from dividing by ~0)."""
    out = {}
    for k, r in ref.items():
        g = got.get(k)
        if g is None or r is None:
            continue
        r = np.asarray(r)
        d = np.abs(np.asarray(g) - r)
        mx = float(np.max(np.abs(r))) if r.size else 0.0
        den = np.abs(r) + ELEM_FLOOR * mx
        e = d / np.where(den > 0, den, 1.0)
        out[k] = {"norm": float(np.max(d)) / mx if mx > 0 else float(np.max(d, initial=0.0)),
                  "elem_p99": float(np.percentile(e, 99)) if e.size else 0.0,
                  "elem_max": float(np.max(e)) if e.size else 0.0}
    return out


def merge_errors(reps) -> dict:
    """Worst case over several error_figures reports."""
    out = {}
    for rep in reps:
        for k, v in rep.items():
            cur = out.setdefault(k, {"norm": 0.0, "elem_p99": 0.0, "elem_max": 0.0})
            for f in cur:
                cur[f] = max(cur[f], v[f])
    return out


def time_region(fn, blocks, steps, warmup, stream):
    """The timed region: warmup untimed steps, then exactly `steps` steps
    bracketed by synchronisation, with one HIP event pair on the launch
    stream around them.  Returns (wall seconds, mean GPU seconds per step
    from the events)."""
    import torch
    for i in range(warmup):
        fn(blocks[i % len(blocks)])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(steps):
        fn(blocks[(warmup + i) % len(blocks)])
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) * 1e-3 / steps


def time_launches(fn, blocks, steps, warmup, stream, pre=None):
    """Run fn(block) warmup+steps times; returns (wall seconds for the timed
    steps, per-launch durations in seconds from an event pair around each
    launch).  ``pre`` (optional) runs before each launch, outside its pair."""
    import torch
    for i in range(warmup):
        fn(blocks[i % len(blocks)])
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        if pre is not None:
            pre()
        ev[i][0].record(stream)
        fn(blocks[(warmup + i) % len(blocks)])
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    durs = [a.elapsed_time(b) * 1e-3 for a, b in ev]
    return wall, durs


def cpu_description() -> str:
    """The host CPU as lscpu names it: model name, family/model/stepping,
    sockets x cores x threads (a virtual machine may report a generic model
    name; the family and model numbers still identify the part)."""
    import subprocess
    f = {}
    try:
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for line in r.stdout.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                f[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if not f.get("Model name"):
        try:
            with open("/proc/cpuinfo") as fh:
                for line in fh:
                    if line.startswith("model name"):
                        f["Model name"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    parts = [f.get("Model name", "unknown CPU")]
    zen = {"23": "Zen/Zen 2", "25": "Zen 3/Zen 4", "26": "Zen 5"}
    if f.get("Vendor ID") == "AuthenticAMD" and f.get("CPU family") in zen:
        parts.append(zen[f["CPU family"]])
    fam = [f"{k.lower()} {f[k]}" for k in ("CPU family", "Model", "Stepping") if f.get(k)]
    if fam:
        parts.append("(" + ", ".join(fam) + ")")
    if f.get("Socket(s)") and f.get("Core(s) per socket"):
        parts.append(f"{f['Socket(s)']} socket(s) x {f['Core(s) per socket']} cores x "
                     f"{f.get('Thread(s) per core', '1')} threads")
    if f.get("CPU max MHz"):
        parts.append(f"max {float(f['CPU max MHz']):.0f} MHz")
    return ", ".join(parts)


class CpuBaselineLeg:
    """The CPU-baseline leg: every use of the FP64 oracle in this file goes
    through this object (timings of the oracle on the host cores, and the FP64
    reference values that the precision figures are measured against).  With
    --no-cpu-baseline it is not created and none of those figures appear."""

    def __init__(self):
        import oracle
        from oracle import slater
        self.oracle = oracle
        self.slater = slater
        self.threads = len(os.sched_getaffinity(0))
        self.cpu_model = cpu_description()

    def replay_qs(self, lattice, n_grid, coef, start, etas, unis):
        """The oracle's own FP64 chain of quasi-simultaneous steps from the
        same start with the same random numbers: the double-precision
        counterpart of a GPU chain (its inverses from its own FP64 Slater
        matrices).  start [W, 2n, 3]; etas [K, W, 2n, 3]; unis [K, W, 2n].
        Returns (kinetic energies [K, W], accept masks [K, W, 2n])."""
        from oracle import vmc as ovmc
        K, W = etas.shape[0], start.shape[0]
        E = np.empty((K, W))
        acc = np.zeros((K, W, start.shape[1]), dtype=bool)
        for w in range(W):
            pos = start[w].copy()
            D = ovmc.slater_matrices(lattice, n_grid, coef, pos)
            inv = np.stack([np.linalg.inv(D[0]).T, np.linalg.inv(D[1]).T])
            for k in range(K):
                pos, inv, acc[k, w], _, _, E[k, w] = ovmc.qs_step(lattice, n_grid, coef, pos, inv,
                                                                  etas[k, w], unis[k, w])
        return E, acc

    def blocks(self, spec, coef, npos, budget_s=12.0):
        """FP64 oracle on a bounded sample of the same workload, all host
        cores: whole move blocks of the benchmark's shape, as many as fit
        ~budget_s; plus one block on one core (the paper's CPU baseline)."""
        from paper_1204_1121_amd import workloads as wl
        L = spec.norb
        first = wl.move_block(spec, npos, block=1000)
        t0 = time.perf_counter()
        self.oracle.evaluate(spec.lattice, spec.n, coef, first, nthreads=1)
        dt_one = max(time.perf_counter() - t0, 1e-6)
        t0 = time.perf_counter()
        self.oracle.evaluate(spec.lattice, spec.n, coef, first, nthreads=self.threads)
        dt1 = max(time.perf_counter() - t0, 1e-6)
        nblk = int(max(1, min(256, budget_s / dt1)))
        sample = np.concatenate([wl.move_block(spec, npos, block=1000 + b) for b in range(nblk)])
        t0 = time.perf_counter()
        self.oracle.evaluate(spec.lattice, spec.n, coef, sample, nthreads=self.threads)
        dt = time.perf_counter() - t0
        return {"value": sample.shape[0] * L / dt, "unit": UNIT, "cores": self.threads,
                "kind": "oracle", "cpu": self.cpu_model,
                "sample": f"{nblk} move blocks of {npos} positions ({sample.shape[0]} positions "
                          f"x {L} orbitals, val+grad+lap, FP64): {dt:.1f} s on "
                          f"{self.threads} threads",
                "single_core": {"value": npos * L / dt_one, "unit": UNIT, "cores": 1,
                                "sample": f"one block of {npos} positions: {dt_one:.2f} s"}}

    def positions(self, spec, coef, pos, budget_s=8.0, what=""):
        """FP64 oracle on a bounded prefix of the positions pos (val+grad+lap):
        all host cores for about budget_s, and up to 256 positions on one
        core.  Returns a cpu_baseline record in orbital evals/s."""
        L = spec.norb
        probe = pos[: min(len(pos), 256)]
        t0 = time.perf_counter()
        self.oracle.evaluate(spec.lattice, spec.n, coef, probe, kvec=spec.kvec,
                             nthreads=self.threads)
        rate = len(probe) / max(time.perf_counter() - t0, 1e-6)
        n = int(max(len(probe), min(len(pos), rate * budget_s)))
        t0 = time.perf_counter()
        self.oracle.evaluate(spec.lattice, spec.n, coef, pos[:n], kvec=spec.kvec,
                             nthreads=self.threads)
        dt = max(time.perf_counter() - t0, 1e-6)
        t0 = time.perf_counter()
        self.oracle.evaluate(spec.lattice, spec.n, coef, probe, kvec=spec.kvec, nthreads=1)
        dt1 = max(time.perf_counter() - t0, 1e-6)
        return {"value": n * L / dt, "unit": UNIT, "cores": self.threads, "kind": "oracle",
                "cpu": self.cpu_model,
                "sample": f"the first {n} of {len(pos)} positions{what} x {L} orbitals, "
                          f"val+grad+lap, FP64: {dt:.1f} s on {self.threads} threads",
                "single_core": {"value": len(probe) * L / dt1, "unit": UNIT, "cores": 1,
                                "sample": f"{len(probe)} positions: {dt1:.2f} s"}}

    def reference(self, spec, coef, pos, want=("val", "grad", "lap")):
        """FP64 oracle values at pos (all host cores)."""
        return self.oracle.evaluate(spec.lattice, spec.n, coef, pos, kvec=spec.kvec, want=want,
                                    nthreads=self.threads)

    def time_values(self, spec, coef, pos, nthreads=1):
        t0 = time.perf_counter()
        self.oracle.evaluate(spec.lattice, spec.n, coef, pos, kvec=spec.kvec, want=("val",),
                             nthreads=nthreads)
        return time.perf_counter() - t0

    def time_sm(self, inv_t, u_rows, cols):
        t0 = time.perf_counter()
        self.slater.sm_update(inv_t, u_rows, cols)
        return time.perf_counter() - t0

    def blas_threads(self):
        try:
            from threadpoolctl import threadpool_info
            return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:
            return 1


def bench_sm(args, leg=None):
    """Sherman-Morrison update of one spin's inverse after a quasi-simultaneous
    step: n = 768 electrons (one spin of the TiO2 block), K = 384 accepted
    moves (half), in electron order.  Synthetic matrix D = 2I + N(0, 1/n)
    and new rows D + N(0, 0.3^2) as FP32; the kernel does the same arithmetic
    whatever the values.  Every step re-applies the same moves to the updated
    inverse (ratios 1 from the second step on)."""
    import torch
    from paper_1204_1121_amd import blip
    from paper_1204_1121_amd import workloads as wl
    stream = torch.cuda.current_stream()
    n, K = 768, 384
    rng = np.random.default_rng(wl.SEED_BASE + 7)
    D = 2.0 * np.eye(n) + rng.normal(0, 1.0 / np.sqrt(n), (n, n))
    inv_t = np.linalg.inv(D).T.copy()
    U = (D + rng.normal(0, 0.3, (n, n))).astype(np.float32)
    cols = np.sort(rng.permutation(n)[:K]).astype(np.int64)
    inv = torch.from_numpy(inv_t).cuda()
    u = torch.from_numpy(U).cuda()
    ws = blip.sm_workspace(n)
    ratios = torch.empty(K, dtype=torch.float64, device="cuda")

    def step(_):
        blip.sm_update(inv, u, cols, ratios=ratios, workspace=ws, stream=stream)
    steps = max(20, min(args.steps, 200))
    wall, t = time_region(step, [None], steps, 5, stream)
    launches = (K + 31) // 32 + 1
    flop = 4.0 * n * n * K                      # 2 n^2 FMA per move
    res = {"n": n, "accepted_moves": K, "launches_per_step": launches,
           "us_per_step": t * 1e6, "wall_us_per_step": wall / steps * 1e6,
           "moves_per_s": K / t,
           "roofline": {"bound": "alu", "achieved": flop / t / 1e12, "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": flop / t / 1e12 / FP64_PEAK_TFLOPS},
           "b_passes": {"blocked": launches, "rank1_per_move": 2 * K},
           "inputs": "D = 2I + N(0,1/n), new rows D + N(0,0.09) in FP32, 384 of 768 moved"}
    # the batched form: the same step for 64 matrices (32 walkers x 2 spins)
    # in one launch sequence, lists and counts on the device
    nmat = 64
    inv_b = torch.from_numpy(inv_t).cuda().unsqueeze(0).repeat(nmat, 1, 1).contiguous()
    u_b = u.unsqueeze(0).repeat(nmat, 1, 1).contiguous()
    acc = torch.from_numpy(np.tile(cols.astype(np.int32), (nmat, 1))).cuda()
    cnt = torch.full((nmat,), K, dtype=torch.int32, device="cuda")
    ws_b = torch.empty(blip.lib().blip_sm_batched_workspace_size(nmat, n), dtype=torch.uint8,
                       device="cuda")
    rat_b = torch.empty((nmat, K), dtype=torch.float64, device="cuda")

    def step_b(_):
        blip.sm_update_batched(inv_b, u_b, acc, cnt, K, ratios=rat_b, workspace=ws_b,
                               stream=stream)
    steps_b = max(5, min(args.steps // 10, 20))
    _, tb = time_region(step_b, [None], steps_b, 2, stream)
    res["batched"] = {"matrices": nmat, "us_per_step": tb * 1e6,
                      "us_per_matrix_step": tb * 1e6 / nmat,
                      "launches_per_step": 2 * ((K + 31) // 32) + 2,
                      "tflops_fp64": nmat * flop / tb / 1e12,
                      "frac_fp64_peak": nmat * flop / tb / 1e12 / FP64_PEAK_TFLOPS}
    del inv_b, u_b, ws_b
    if leg is not None:
        dt = leg.time_sm(inv_t, U[cols].astype(np.float64), cols)
        res["cpu_baseline"] = {"value": K / dt, "unit": "moves/s", "cores": leg.blas_threads(),
                               "kind": "oracle",
                               "sample": f"one step of {K} moves at n = {n}: {dt:.2f} s"}
    return res


def bench_batched(table, spec, args, nbatch=4, leg=None, coef=None):
    """512 walkers with move blocks of U[1,256] positions on the same table:
    one sorted persistent launch per batch (replayed hipGraph plan), against
    the plain kernel on the concatenation and per-walker launch loops."""
    import torch
    from paper_1204_1121_amd import workloads as wl
    from paper_1204_1121_amd.tuning import TuneCache
    stream = torch.cuda.current_stream()
    bs = [wl.walker_batch(spec, nwalkers=512, max_block=256, batch=q) for q in range(nbatch)]
    cap = max(b.pos.shape[0] for b in bs)
    L = spec.norb
    pos = [torch.from_numpy(b.pos).cuda() for b in bs]
    off = [torch.from_numpy(b.offsets).cuda() for b in bs]
    out = table.alloc_outputs(cap)
    ws = table.workspace(cap)
    cache = TuneCache()
    allr = None
    if not args.retune and cache.apply(table, cap, batched=True):
        best = dict(cache.get(table, cap, True), **{"from": "tuning cache"})
    else:
        best, allr = table.autotune(pos[0], out, offsets=off[0], workspace=ws, capacity=cap)
        cache.put(table, cap, True, best, note="blip_autotune, 512-walker batch")
        best["from"] = "autotuned now"
        if args.save_tuning:
            cache.entries.update(TuneCache(args.save_tuning).entries
                                 if os.path.exists(args.save_tuning) else {})
            cache.put(table, cap, True, best, note="blip_autotune, 512-walker batch")
            cache.save(args.save_tuning)
    log(f"batched shape: P={best['tile_pos']} o={best['vec']} ({best['from']})")
    plans = [table.plan(p, o, out, ws, capacity=p.shape[0]) for p, o in zip(pos, off)]
    steps = max(10, min(args.steps, 50))
    wall, t_b = time_region(lambda i: plans[i].launch(), list(range(nbatch)), steps, 3, stream)
    npos_mean = float(np.mean([b.pos.shape[0] for b in bs]))
    U = [distinct_rows(spec.lattice, spec.n, b.pos) for b in bs]
    b_alg = float(np.mean([u * L * 4 + b.pos.shape[0] * (5 * L * 4 + 24) for u, b in zip(U, bs)]))
    res = {"walkers": 512, "positions_mean": npos_mean, "shape": best, "autotune": allr,
           "value": npos_mean * L * steps / wall, "unit": UNIT,
           "launch_us": t_b * 1e6, "hbm_gbs": b_alg / t_b / 1e9,
           "frac": b_alg / t_b / 1e9 / HBM_PEAK_GBS, "bytes_algorithmic": b_alg,
           "flops_per_launch": npos_mean * L * 296 * 2}
    res["tflops"] = res["flops_per_launch"] / t_b / 1e12

    def plain_all(i):
        table.eval(pos[i], out=tuple(x[: pos[i].shape[0]] for x in out), kernel="plain")
    _, dp = time_launches(plain_all, list(range(nbatch)), 10, 2, stream)
    res["plain_concatenated_us"] = float(np.mean(dp)) * 1e6

    def unsorted_all(i):
        table.eval(pos[i], out=tuple(x[: pos[i].shape[0]] for x in out))
    _, du = time_launches(unsorted_all, list(range(nbatch)), 10, 2, stream)
    res["tiled_unsorted_us"] = float(np.mean(du)) * 1e6
    views = [[(pos[q][int(b.offsets[w]):int(b.offsets[w + 1])],
               tuple(x[int(b.offsets[w]):int(b.offsets[w + 1])] for x in out))
              for w in range(512)] for q, b in enumerate(bs)]

    def per_walker(kernel):
        def f(i):
            for pw, ow in views[i]:
                table.eval(pw, out=ow, kernel=kernel)
        return f
    _, dpw = time_launches(per_walker("plain"), list(range(nbatch)), 3, 1, stream)
    res["per_walker_plain_us"] = float(np.mean(dpw)) * 1e6
    res["speedup_vs_per_walker_plain"] = res["per_walker_plain_us"] / res["launch_us"]
    res["speedup_vs_plain_concatenated"] = res["plain_concatenated_us"] / res["launch_us"]
    for pl in plans:
        pl.free()
    if leg is not None and coef is not None:
        cb = leg.positions(spec, coef, bs[0].pos, what=" of the first batch (walkers in order)")
        cb["gpu_speedup_vs_threads"] = res["value"] / cb["value"]
        cb["gpu_speedup_vs_one_core"] = res["value"] / cb["single_core"]["value"]
        res["cpu_baseline"] = cb
        log(f"batched oracle: {cb['value']:.3e} evals/s on {cb['cores']} threads, "
            f"{cb['single_core']['value']:.3e} on one core")
    log(f"batched: {t_b * 1e6:.0f} us per 512-walker batch; plain(concat) "
        f"{res['plain_concatenated_us']:.0f} us; per-walker plain loop {res['per_walker_plain_us']:.0f} us")
    return res


def bench_block_sizes(table, spec, stream, cache, args, sizes=(1, 8, 64, 256, 1536), reps=200):
    """Move blocks of 1 to 1,536 positions on the 768-orbital table: kernel
    time from per-launch event pairs (median, p99) over blocks rotated as in
    the main figure, and end-to-end latency, host submit to completion, of
    one launch at a time (synchronised before and after).  Each size runs the
    shape cached for its size bucket, autotuned on these blocks if none is."""
    import torch
    from paper_1204_1121_amd import workloads as wl
    L = spec.norb
    rows = []
    for B in sizes:
        blocks = [torch.from_numpy(wl.move_block(spec, B, block=b)).cuda() for b in range(NROT)]
        out = table.alloc_outputs(B)
        if args.retune or not cache.apply(table, B):
            best, _ = table.autotune(torch.cat(blocks).contiguous(), out, rotate=NROT)
            cache.put(table, B, False, best, note=f"blip_autotune rotate={NROT}")
        calls = {id(b): table.bind(b, out) for b in blocks}
        _, durs = time_launches(lambda b: calls[id(b)](), blocks, reps, 20, stream)
        e2e = []
        for i in range(50):
            call = calls[id(blocks[i % NROT])]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            call()
            torch.cuda.synchronize()
            e2e.append(time.perf_counter() - t0)
        med = float(np.median(durs))
        rows.append({"npos": B, "kernel_us_median": med * 1e6,
                     "kernel_us_p99": float(np.percentile(durs, 99)) * 1e6,
                     "e2e_us_median": float(np.median(e2e)) * 1e6,
                     "evals_per_s": B * L / med, "shape": list(table.get_shape(B))})
        log(f"block of {B}: kernel {med * 1e6:.1f} us (p99 {rows[-1]['kernel_us_p99']:.1f}), "
            f"submit-to-completion {rows[-1]['e2e_us_median']:.1f} us")
    return rows


def bench_serving(args, leg=None):
    """Three resident systems (the 768-orbital table; 48^3 x 256; 96x96x64 x
    1024), requests of 1..1536 positions (log-uniform) arriving by Poisson
    process at rates swept around the saturated rate; continuous batching
    with HBM-budget admission.  Latency from the scheduled arrival."""
    import torch
    from paper_1204_1121_amd import blip
    from paper_1204_1121_amd import workloads as wl
    from paper_1204_1121_amd.serve import GpuBackend, Server, ServeRequest
    specs = wl.spec_serving()
    t0 = time.perf_counter()
    tables, coefs = [], []
    for sp in specs:
        c = wl.coefficients(sp)
        tables.append(blip.Table(sp.lattice, sp.n, c, "f32"))
        if leg is not None:
            coefs.append(c)            # the oracle's copy of the served tables
        del c
    resident = sum(t.info()["device_bytes"] for t in tables)
    log(f"serving: {len(tables)} tables, {resident / 1e9:.2f} GB resident "
        f"({time.perf_counter() - t0:.1f} s)")
    norb = [sp.norb for sp in specs]
    nreq = args.serve_requests

    def make(rate, seed, n=nreq, keep_every=0):
        rq = wl.serving_requests(len(specs), n, rate=rate, specs=specs, seed=seed)
        return [ServeRequest(r.rid, r.system, r.pos, arrival=r.arrival,
                             keep=keep_every > 0 and r.rid % keep_every == 0) for r in rq]

    def run(backend, budget, reqs):
        backend.launch_host_s = 0.0
        sv = Server(backend, budget_bytes=budget)
        st = sv.run(reqs)
        ev = sum(r.npos * norb[r.system] for r in reqs if r.status == "done")
        st["evals_per_s"] = ev / st["makespan_s"]
        return st

    out = {"tables_gb": resident / 1e9, "requests_per_point": nreq}
    be = GpuBackend(tables, capacity=16384, max_requests=512, batched=True)
    run(be, 2 << 30, make(1e9, 99, 500))                     # warm-up
    sat = run(be, 2 << 30, make(1e9, 100))                   # all at t=0: saturated
    out["saturated"] = sat
    rate_sat = sat["req_per_s"]
    log(f"serving saturated: {rate_sat:.0f} req/s, {sat['evals_per_s']:.3e} evals/s")
    sweep = []
    for f in (0.25, 0.5, 0.75, 0.9, 1.0, 1.2):
        st = run(be, 2 << 30, make(f * rate_sat, 200 + int(f * 100)))
        st["offered_fraction"] = f
        st["offered_req_per_s"] = f * rate_sat
        sweep.append(st)
        log(f"  rate {f:.2f}x: p50 {st['p50_ms']:.3f} ms p99 {st['p99_ms']:.3f} ms "
            f"(queue wait p50 {st.get('queue_wait_p50_ms', 0):.3f}, in service p50 "
            f"{st.get('in_service_p50_ms', 0):.3f} ms, host {st.get('launch_host_us_mean', 0):.1f} "
            f"us per launch) {st['evals_per_s']:.3e} evals/s")
    out["sweep"] = sweep
    small = run(be, 64 << 20, make(0.9 * rate_sat, 300))
    small["budget_bytes"] = 64 << 20
    out["small_budget_0.9x"] = small
    if leg is not None:
        out["oracle_check"] = serving_oracle_check(leg, be, specs, coefs, make, run)
    be.close()
    # unbatched baseline: one request per launch, plain single-block kernel
    bp = GpuBackend(tables, batched=False, kernel="plain")
    run(bp, 2 << 30, make(1e9, 99, 200))
    psat = run(bp, 2 << 30, make(1e9, 101, max(1000, nreq // 5)))
    out["plain_unbatched_saturated"] = psat
    pl = run(bp, 2 << 30, make(0.5 * psat["req_per_s"], 301, max(1000, nreq // 5)))
    pl["offered_req_per_s"] = 0.5 * psat["req_per_s"]
    out["plain_unbatched_0.5x_of_its_saturation"] = pl
    log(f"plain unbatched saturated: {psat['req_per_s']:.0f} req/s, "
        f"{psat['evals_per_s']:.3e} evals/s")
    bp.close()
    for t in tables:
        t.free()
    return out


def serving_oracle_check(leg, be, specs, coefs, make, run, every=50):
    """The saturated run's request stream served again with one result in
    `every` copied back, each compared with the FP64 oracle (normwise and
    elementwise, per component group and system), and the oracle's time per
    position on those requests (all host cores, and one core)."""
    reqs = make(1e9, 100, keep_every=every)
    run(be, 2 << 30, reqs)
    reqs = [r for r in reqs if r.keep and r.status == "done"]
    per_sys, npos_sys, dt_sys = {}, {}, {}
    for r in reqs:
        sp = specs[r.system]
        t0 = time.perf_counter()
        ref = leg.oracle.evaluate(sp.lattice, sp.n, coefs[r.system], r.pos,
                                  nthreads=leg.threads)
        dt_sys[sp.name] = dt_sys.get(sp.name, 0.0) + time.perf_counter() - t0
        npos_sys[sp.name] = npos_sys.get(sp.name, 0) + r.npos
        per_sys.setdefault(sp.name, []).append(error_figures(r.result, ref))
    res = {"requests_checked": len(reqs), "every": every,
           "errors_by_system": {k: merge_errors(v) for k, v in per_sys.items()},
           "errors": merge_errors([e for v in per_sys.values() for e in v]),
           "oracle_us_per_position": {k: dt_sys[k] / npos_sys[k] * 1e6 for k in dt_sys},
           "oracle_threads": leg.threads}
    one = {}
    for s_idx, sp in enumerate(specs):
        pos = next((r.pos for r in reqs if r.system == s_idx), None)
        if pos is None:
            continue
        pos = pos[:64]
        t0 = time.perf_counter()
        leg.oracle.evaluate(sp.lattice, sp.n, coefs[s_idx], pos, nthreads=1)
        one[sp.name] = (time.perf_counter() - t0) / len(pos) * 1e6
    res["oracle_us_per_position_one_core"] = one
    worst = res["errors"]
    log("serving oracle check: " + f"{len(reqs)} requests, " +
        " ".join(f"{k} {v['norm']:.1e} (p99 elem {v['elem_p99']:.1e})" for k, v in worst.items()))
    return res


def bench_shard_shape(args, coef, spec, cache, full_us, leg=None, shards=8):
    """One GPU's share of the table sharded by orbitals over `shards` GPUs:
    the first 768/shards orbitals of the 768-orbital table on the same
    72x72x48 grid, evaluated at the same 1,536-position blocks with the
    tuned kernel (its own cached or autotuned shape).  B_alg counts the
    shard's distinct rows, its outputs and the positions; the ideal is the
    full table's launch time divided by the number of shards."""
    import torch
    from paper_1204_1121_amd import blip
    from paper_1204_1121_amd import workloads as wl
    stream = torch.cuda.current_stream()
    L = spec.norb // shards
    npos = 1536
    c = np.ascontiguousarray(coef[..., :L])
    t = blip.Table(spec.lattice, spec.n, c, "f32")
    o = t.alloc_outputs(npos)
    blocks_np = [wl.move_block(spec, npos, block=b) for b in range(NROT)]
    blocks = [torch.from_numpy(b).cuda() for b in blocks_np]
    if args.retune or not cache.apply(t, npos):
        best, _ = t.autotune(torch.cat(blocks).contiguous(), o, rotate=NROT)
        cache.put(t, npos, False, best, note=f"blip_autotune rotate={NROT}")
    P, vec = t.get_shape(npos)
    calls = {id(b): t.bind(b, o) for b in blocks}
    _, tk = time_region(lambda b: calls[id(b)](), blocks, max(50, min(args.steps, 200)), 10,
                        stream)
    U = [distinct_rows(spec.lattice, spec.n, b) for b in blocks_np]
    b_alg = float(np.mean([u * L * 4 + npos * (5 * L * 4 + 24) for u in U]))
    res = {"orbitals": L, "shards": shards, "npos": npos, "grid": list(spec.n),
           "shape": {"tile_pos": P, "vec": vec}, "kernel_us": tk * 1e6,
           "evals_per_s": npos * L / tk, "bytes_algorithmic": b_alg,
           "roofline": {"bound": "hbm", "achieved": b_alg / tk / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": b_alg / tk / 1e9 / HBM_PEAK_GBS},
           "full_table_kernel_us": full_us,
           "ideal_shard_us": full_us / shards,
           "shard_efficiency": full_us / shards / (tk * 1e6)}
    if leg is not None:
        ref = leg.reference(spec, c, blocks_np[0])
        v, g, l = t.eval(blocks[0], out=o)
        torch.cuda.synchronize()
        got = {"val": v.cpu().numpy(), "grad": g.cpu().numpy(), "lap": l.cpu().numpy()}
        res["errors"] = error_figures(got, ref)
    t.free()
    log(f"shard shape L={L}: {tk * 1e6:.1f} us per 1,536-block (P={P} o={vec}), "
        f"{res['roofline']['frac']:.3f} of HBM peak on B_alg; full table / {shards} = "
        f"{full_us / shards:.1f} us")
    return res


def bench_precision(args, real_coef, real_spec, cache, leg=None):
    """Storage dtypes at 1,536 positions: the complex k-point table (384
    orbitals) as complex64 / BF16 pairs / FP16 pairs, and the 768-orbital real
    table as FP32 / BF16 / FP16.  For each: kernel time, evals/s and the
    normwise max relative error of val, grad and lap against the FP64 oracle
    on the FP32 master, over the whole block (errors only with the CPU-baseline
    leg, which supplies the oracle's values).  Beside the normwise error, the
    99th percentile and maximum of the elementwise error
    |y - y*| / (|y*| + 1e-3 max|y*|) per component group."""
    import torch
    from paper_1204_1121_amd import blip
    from paper_1204_1121_amd import workloads as wl
    stream = torch.cuda.current_stream()
    out = {}
    cases = [("complex_k", wl.spec_tio2_complex(), None, ("c64", "cbf16", "cf16")),
             ("real", real_spec, real_coef, ("f32", "bf16", "f16"))]
    for label, spec, coef, dtypes in cases:
        if coef is None:
            coef = wl.coefficients(spec)
        blocks = [torch.from_numpy(wl.move_block(spec, 1536, block=b)).cuda() for b in range(NROT)]
        pos0 = wl.move_block(spec, 1536, block=0)
        ref = leg.reference(spec, coef, pos0) if leg is not None else None
        for st in dtypes:
            t = blip.Table(spec.lattice, spec.n, coef, st, kvec=spec.kvec)
            o = t.alloc_outputs(1536)
            if args.retune or not cache.apply(t, 1536):
                best, _ = t.autotune(torch.cat(blocks).contiguous(), o, rotate=NROT)
                cache.put(t, 1536, False, best, note=f"blip_autotune rotate={NROT}")
            calls = {id(b): t.bind(b, o) for b in blocks}
            wall, tk = time_region(lambda b: calls[id(b)](), blocks, 100, 10, stream)
            rb = t.info()["row_bytes"]
            shape = t.get_shape(1536)
            rec = {"kernel_us": tk * 1e6, "evals_per_s": 1536 * spec.norb / tk,
                   "row_bytes": rb, "shape": {"tile_pos": shape[0], "vec": shape[1]}}
            msg = ""
            if ref is not None:
                v, g, l = t.eval(blocks[0], out=o)
                torch.cuda.synchronize()
                got = {"val": v.cpu().numpy(), "grad": g.cpu().numpy(), "lap": l.cpu().numpy()}
                fig = error_figures(got, ref)
                rec["max_rel_err"] = {k: f["norm"] for k, f in fig.items()}
                rec["elementwise_rel_err"] = {k: {"p99": f["elem_p99"], "max": f["elem_max"]}
                                              for k, f in fig.items()}
                msg = ", err " + " ".join(f"{k} {f['norm']:.1e} (p99 elem {f['elem_p99']:.1e})"
                                          for k, f in fig.items())
            out[f"{label}_{st}"] = rec
            log(f"precision {label} {st}: {tk * 1e6:.1f} us{msg}")
            t.free()
    return out


def tune_ratio_pass(wk, table, npos, stream):
    """The sorted ratio pass's launch shape for this step size: every
    (P, o) timed over ten passes at the walkers' current trial positions, the
    fastest kept on the table.  Only the shape changes: the values and
    Laplacian rows are the same at every shape, the ratios the same up to
    FP64 rounding."""
    import torch
    tr = wk.trial.view(npos, 3)
    outs = (wk.ratio, wk.rg, wk.rl, wk.val, wk.lapt)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    found = []
    for P in (1, 2, 4, 8, 16):
        for o in (1, 2, 4):
            table.set_shape(npos, P, o, batched=True, ratio=True)
            wk.ratio_values(tr, outs)
            torch.cuda.synchronize()
            ev[0].record(stream)
            for _ in range(10):
                wk.ratio_values(tr, outs)
            ev[1].record(stream)
            torch.cuda.synchronize()
            found.append({"tile_pos": P, "vec": o, "us": ev[0].elapsed_time(ev[1]) * 100.0})
    best = min(found, key=lambda e: e["us"])
    table.set_shape(npos, best["tile_pos"], best["vec"], batched=True, ratio=True)
    return best


def bench_vmc(args, table, spec, leg=None, cache=None):
    """Quasi-simultaneous Monte Carlo steps on the device.

    Throughput: 16 walkers of the TiO2 system (2 x 768 electrons each, the
    768-orbital table), one full step each time (trial moves, values and
    ratios at the trial positions, accept/reject, batched inverse updates,
    local kinetic energy), with the time of each phase.

    Statistics (the paper's comparison of quasi-simultaneous and
    particle-by-particle updating, Eq. (11.12.23.0b) and Table energy_eval, on a
    synthetic system): 64 walkers of 2 x 8 electrons on a small table,
    both chains from the same start, acceptance and mean local kinetic energy
    with the standard error over the independent walkers."""
    import torch
    from paper_1204_1121_amd import blip
    from paper_1204_1121_amd import vmc
    from paper_1204_1121_amd import workloads as wl
    stream = torch.cuda.current_stream()
    res = {}
    # -- throughput on the TiO2 system
    W, n = 16, spec.norb
    g = torch.Generator(device="cuda").manual_seed(wl.SEED_BASE + 11)
    lat = torch.from_numpy(spec.lattice).cuda()
    pos = torch.rand((W, 2 * n, 3), dtype=torch.float64, device="cuda", generator=g) @ lat
    wk = vmc.Walkers(table, pos, stream=stream)
    sigma = 0.35
    etas = [sigma * torch.randn((W, 2 * n, 3), dtype=torch.float64, device="cuda", generator=g)
            for _ in range(4)]
    unis = [torch.rand((W, 2 * n), dtype=torch.float64, device="cuda", generator=g) for _ in range(4)]
    for i in range(3):
        wk.step(etas[i % 4], unis[i % 4])
    torch.cuda.synchronize()
    npos = W * 2 * n
    shape = None
    if wk.sorted:
        # the sorted ratio pass's shape: from the tuning cache, else measured
        if cache is not None and not args.retune and cache.apply(table, npos, batched=True,
                                                                 ratio=True):
            shape = dict(cache.get(table, npos, True, ratio=True), **{"from": "tuning cache"})
        else:
            shape = dict(tune_ratio_pass(wk, table, npos, stream), **{"from": "measured"})
            if cache is not None:
                cache.put(table, npos, True, shape, ratio=True,
                          note=f"ratio pass sweep, {W}-walker step")
        log(f"vmc: sorted ratio pass, shape P={shape['tile_pos']} o={shape['vec']} "
            f"({shape['from']})")
    steps = 10
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for i in range(steps):
        wk.step(etas[i % 4], unis[i % 4])
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_step = ev[0].elapsed_time(ev[1]) * 1e-3 / steps
    acc = float(wk.acc_count.sum().item()) / (W * 2 * n)
    # phases, each timed alone over the same step inputs
    tr = wk.trial.view(npos, 3)
    phases = {
        "ratios, values and Laplacian rows at the trial positions (one pass)":
            lambda: wk.ratio_values(tr, (wk.ratio, wk.rg, wk.rl, wk.val, wk.lapt)),
        "accepted Laplacian rows carried over": wk.carry_rows,
        "local kinetic energy from the kept rows": wk.kinetic,
    }
    ph = {}
    for name, fn in phases.items():
        fn()
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(steps):
            fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        ph[name] = ev[0].elapsed_time(ev[1]) * 1e3 / steps
    ph["accept + inverse updates + propose (rest of the step)"] = t_step * 1e6 - sum(ph.values())
    assert wk.lap_ok, "the timed steps must run from the kept Laplacian rows"
    res["throughput"] = {"walkers": W, "electrons_per_walker": 2 * n, "orbitals": n,
                         "us_per_step": t_step * 1e6, "walker_steps_per_s": W / t_step,
                         "electron_moves_per_s": W * 2 * n / t_step, "acceptance": acc,
                         "sigma_bohr": sigma, "phases_us": ph,
                         "ratio_pass": ({"launch": "sorted persistent", "shape": shape}
                                        if wk.sorted else {"launch": "block"})}
    del wk
    log(f"vmc: {t_step * 1e6:.0f} us per quasi-simultaneous step of {W} walkers x {2 * n} "
        f"electrons ({W / t_step:.0f} walker-steps/s, acceptance {acc:.2f})")

    # -- two sets of W walkers, each on its own stream, stepped in turn: one
    # set's latency-bound inverse updates overlap the other's ratio pass
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    sets = []
    for k, st in enumerate(streams):
        with torch.cuda.stream(st):
            p0 = torch.rand((W, 2 * n, 3), dtype=torch.float64, device="cuda", generator=g) @ lat
        sets.append(vmc.Walkers(table, p0, stream=st))
    torch.cuda.synchronize()
    for i in range(3):
        for wk2 in sets:
            wk2.step(etas[i % 4], unis[i % 4])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for st in streams:
        st.wait_event(e0)
    for i in range(steps):
        for wk2 in sets:
            wk2.step(etas[i % 4], unis[i % 4])
    for st in streams:
        stream.wait_stream(st)
    e1.record(stream)
    torch.cuda.synchronize()
    t_pair = e0.elapsed_time(e1) * 1e-3 / steps
    res["two_sets_two_streams"] = {"walkers_per_set": W, "sets": 2, "us_per_step_pair": t_pair * 1e6,
                                   "walker_steps_per_s": 2 * W / t_pair,
                                   "gain_over_one_set": (2 * W / t_pair) / (W / t_step)}
    del sets
    log(f"vmc: two sets of {W} walkers on two streams: {t_pair * 1e6:.0f} us per step pair "
        f"({2 * W / t_pair:.0f} walker-steps/s)")

    if args.no_vmc_stats:
        return res
    # -- statistics: quasi-simultaneous against particle-by-particle
    A = np.array([[6.0, 0.3, 0.0], [0.2, 5.0, 0.4], [0.0, -0.3, 5.5]])
    ng, Ls, Ws = (12, 11, 10), 8, 64
    rng = np.random.default_rng(wl.SEED_BASE + 12)
    coef = rng.uniform(-1, 1, ng + (Ls,)).astype(np.float32)
    ts = blip.Table(A, ng, coef, "f32")
    start = torch.from_numpy(rng.uniform(0, 1, (Ws, 2 * Ls, 3)) @ A).cuda()
    chains = {"quasi_simultaneous": vmc.Walkers(ts, start.clone(), stream=stream),
              "particle_by_particle": vmc.Walkers(ts, start.clone(), stream=stream)}
    nequil, nsample, sig = 200, 1000, 0.3
    nrec, wrec = (100, 8) if leg is not None else (0, 0)   # steps replayed on the oracle
    rec = {"eta": [], "uni": [], "e": [], "acc": []}
    stats = {}
    for name, wk in chains.items():
        gs = torch.Generator(device="cuda").manual_seed(wl.SEED_BASE + 13)   # same draws
        esum = torch.zeros(Ws, dtype=torch.float64, device="cuda")
        emax = torch.zeros((), dtype=torch.float64, device="cuda")
        acc_n = torch.zeros((), dtype=torch.float64, device="cuda")
        seq_min = torch.full((), float("inf"), dtype=torch.float64, device="cuda")
        lanes = torch.arange(Ls, device="cuda")[None, :]
        t0 = time.perf_counter()
        for it in range(nequil + nsample):
            eta = sig * torch.randn((Ws, 2 * Ls, 3), dtype=torch.float64, device="cuda",
                                    generator=gs)
            uni = torch.rand((Ws, 2 * Ls), dtype=torch.float64, device="cuda", generator=gs)
            if name == "quasi_simultaneous":
                if it < nrec:
                    before = wk.pos[:wrec].clone()
                cnt, e = wk.step(eta, uni)
                if it < nrec:
                    rec["eta"].append(eta[:wrec].cpu().numpy())
                    rec["uni"].append(uni[:wrec].cpu().numpy())
                    rec["e"].append(e[:wrec].cpu().numpy())
                    rec["acc"].append((wk.pos[:wrec] != before).any(dim=2).cpu().numpy())
                seq = torch.where(lanes < wk.acc_count[:, None], wk.seq.abs(),
                                  torch.full_like(wk.seq, float("inf")))
                seq_min = torch.minimum(seq_min, seq.min())
            else:
                before = wk.pos.clone()
                e = wk.pbp_sweep(eta, uni)
                cnt = (wk.pos != before).any(dim=2).sum()
            if it >= nequil:
                esum += e
                emax = torch.maximum(emax, e.abs().max())
                acc_n += cnt.sum()
        torch.cuda.synchronize()
        ew = (esum / nsample).cpu().numpy()
        stats[name] = {"mean_kinetic_hartree": float(ew.mean()),
                       "stderr": float(ew.std(ddof=1) / np.sqrt(Ws)),
                       "median_walker_mean": float(np.median(ew)),
                       "max_abs_local_energy": float(emax.item()),
                       "acceptance": float(acc_n.item()) / (nsample * Ws * 2 * Ls),
                       "seconds": time.perf_counter() - t0}
        if name == "quasi_simultaneous":
            stats[name]["min_sequential_ratio"] = float(seq_min.item())
    q, c = stats["quasi_simultaneous"], stats["particle_by_particle"]
    diff = q["mean_kinetic_hartree"] - c["mean_kinetic_hartree"]
    err = float(np.hypot(q["stderr"], c["stderr"]))
    stats["difference_in_stderr"] = diff / err
    stats["setup"] = (f"{Ws} walkers x {2 * Ls} electrons, {Ls} orbitals on a {ng} grid, "
                      f"sigma {sig} bohr, {nequil} equilibration + {nsample} sampled steps, the "
                      "same random draws for both chains; stderr over walker means")
    if leg is not None:
        # the paper's single- against double-precision comparison (Table
        # energy_eval), on this system: the GPU chain (FP32 orbitals, FP64
        # inverses) against the oracle's FP64 chain with the same draws
        t0 = time.perf_counter()
        E_o, acc_o = leg.replay_qs(A, ng, coef, start[:wrec].cpu().numpy(),
                                   np.stack(rec["eta"]), np.stack(rec["uni"]))
        E_g, acc_g = np.stack(rec["e"]), np.stack(rec["acc"])
        same = (acc_g == acc_o).all(axis=2)                       # [K, W]
        # steps up to each walker's first differing decision (chains agree there)
        upto = np.where(same.all(axis=0), nrec, np.argmin(same, axis=0))
        mask = np.arange(nrec)[:, None] < upto[None, :]
        dev = np.abs(E_g - E_o)[mask]
        stats["double_precision_replay"] = {
            "walkers": wrec, "steps": nrec,
            "walkers_with_a_differing_decision": int((upto < nrec).sum()),
            "first_differing_step": [int(u) if u < nrec else None for u in upto],
            "max_abs_energy_deviation_hartree": float(dev.max()) if dev.size else None,
            "max_rel_energy_deviation": float((dev / np.abs(E_o[mask])).max()) if dev.size else None,
            "mean_kinetic_gpu": float(E_g[mask].mean()) if dev.size else None,
            "mean_kinetic_oracle_fp64": float(E_o[mask].mean()) if dev.size else None,
            "oracle_seconds": time.perf_counter() - t0}
        dr = stats["double_precision_replay"]
        log(f"vmc replay on the FP64 oracle: {nrec} steps x {wrec} walkers, "
            f"{dr['walkers_with_a_differing_decision']} walkers with a differing decision, "
            f"max |dE| {dr['max_abs_energy_deviation_hartree']} Ha")
    res["statistics"] = stats
    log(f"vmc statistics: Q.S. E_kin {q['mean_kinetic_hartree']:.2f} +- {q['stderr']:.2f} "
        f"(median walker {q['median_walker_mean']:.2f}, max |E_L| {q['max_abs_local_energy']:.3g}, "
        f"acceptance {q['acceptance']:.3f}); PbP {c['mean_kinetic_hartree']:.2f} +- "
        f"{c['stderr']:.2f} (median walker {c['median_walker_mean']:.2f}, max |E_L| "
        f"{c['max_abs_local_energy']:.3g}, acceptance {c['acceptance']:.3f})")
    ts.free()
    return res


PAPER_SYSTEMS = (  # (system, electrons N, orbitals L, the paper's GPU ms per step, CPU ms)
    ("Si 3x3x3", 216, 56, 0.17, 2.77),
    ("TiO2 3x3x3", 648, 168, 0.82, 20.21),
    ("TiO2 4x4x4", 1536, 384, 3.26, 100.00),
)


# The paper's GPU times per Monte Carlo step for its three mappings (Table
# kernel_time0, GTX 480, kernel plus PCIe), quoted for N = 216 and 1,536.
PAPER_MAPPING_MS = {
    216: {"(1)": 6.76, "(2)": 0.43, "(3)": 0.17},
    1536: {"(1)": 68.03, "(2)": 17.83, "(3)": 3.26},
}
MAPPINGS = (  # (reported name, kernel, short label)
    ("(3) quasi-simultaneous, coalesced: tuned tiled kernel", "auto", "(3) tiled"),
    ("(3) quasi-simultaneous, coalesced: plain kernel", "plain", "(3) plain"),
    ("(2) quasi-simultaneous, non-coalesced: site-parallel kernel", "site", "(2)"),
    ("(1) particle-by-particle: N site-parallel launches of one position", "pbp", "(1)"),
)


def time_per_position_launches(table, pos, out, reps=3):
    """GPU seconds for one pass of the particle-by-particle form over a
    block: one site-parallel launch per position, captured once in a graph
    so that the host's enqueue rate does not set the time.  The replayed
    rows must equal one site-parallel launch over the whole block."""
    import torch
    want = table.eval(pos, grad=False, kernel="site")[0]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=side):
        calls = [table.bind(pos[j:j + 1], (out[0][j:j + 1], None, None), kernel="site")
                 for j in range(pos.shape[0])]
        for call in calls:
            call()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    if not torch.equal(out[0], want):
        raise RuntimeError("per-position launches differ from the block launch")
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def bench_paper_sizes(args, cache, leg=None):
    """The paper's own workload shape (Table system_size): complex orbital
    values only, one evaluation of all L orbitals at the N moved electrons of
    a quasi-simultaneous step, for its three (N, L).  Synthetic complex64
    tables on the 72x72x48 grid of the 18x18x12 bohr cell at the k-point of
    the complex workload, so only N and L change between rows.  The paper's
    GTX 480 times (kernel plus PCIe) and single-core CPU times are context."""
    import torch
    from paper_1204_1121_amd import blip
    from paper_1204_1121_amd import workloads as wl
    stream = torch.cuda.current_stream()
    base = wl.spec_tio2_complex()
    rows = []
    for name, N, L, paper_gpu_ms, paper_cpu_ms in PAPER_SYSTEMS:
        spec = wl.TableSpec(f"values_only_N{N}_L{L}c", base.lattice, base.n, L, complex_=True,
                            kvec=base.kvec, seed=base.seed + L)
        coef = wl.coefficients(spec)
        t = blip.Table(spec.lattice, spec.n, coef, "c64", kvec=spec.kvec)
        blocks = [torch.from_numpy(wl.move_block(spec, N, block=b)).cuda() for b in range(NROT)]
        o = t.alloc_outputs(N, grad=False)
        if args.retune or not cache.apply(t, N, values_only=True):
            best, _ = t.autotune(torch.cat(blocks).contiguous(), o, rotate=NROT)
            cache.put(t, N, False, best, note=f"blip_autotune rotate={NROT}, values only",
                      values_only=True)
        times = {}
        for key, kern, _ in MAPPINGS:
            if kern == "pbp":
                times[key] = time_per_position_launches(t, blocks[0], o)
                continue
            calls = {id(b): t.bind(b, o, kernel=kern) for b in blocks}
            steps, warm = (200, 20) if kern != "site" else (20, 3)
            _, times[key] = time_region(lambda b: calls[id(b)](), blocks, steps, warm, stream)
        tk = times[MAPPINGS[0][0]]
        row = {"system": name, "N": N, "L": L, "kernel_us": tk * 1e6,
               "complex_values_per_s": N * L / tk,
               "mappings_us": {k: v * 1e6 for k, v in times.items()},
               "paper_gtx480_ms_kernel_plus_pcie": paper_gpu_ms,
               "paper_gtx480_ms_by_mapping": PAPER_MAPPING_MS.get(N),
               "paper_cpu_1core_ms": paper_cpu_ms}
        msg = ""
        if leg is not None:
            pos0 = wl.move_block(spec, N, block=0)
            dt = leg.time_values(spec, coef, pos0, nthreads=1)
            row["oracle_1core_ms"] = dt * 1e3
            row["speedup_vs_oracle_1core"] = dt / tk
            row["acceleration_vs_oracle_1core"] = {k: dt / v for k, v in times.items()}
            msg = f", FP64 oracle on one core {dt * 1e3:.1f} ms ({dt / tk:.0f}x)"
        rows.append(row)
        log(f"paper size {name} (N={N}, L={L}, complex, values only): {tk * 1e6:.1f} us{msg}; "
            "mappings " + ", ".join(f"{short} {times[key] * 1e6:.1f} us"
                                    for key, _, short in MAPPINGS))
        t.free()
        del coef
    return rows


def stream_read_rate(nbytes=2 << 30, reps=10, grids=(1024, 2048, 4096, 8192, 16384, 32768, 65535)):
    """Achievable HBM read rate on this GPU, the denominator the orbital
    kernel's bound calls for: blip_stream_read over a 2 GiB buffer (more
    than the Infinity Cache holds), event-timed, the best of a few grid
    sizes.  Returns (GB/s, workgroups)."""
    import torch
    from paper_1204_1121_amd import blip
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    part = torch.empty(max(grids), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    best = (0.0, grids[0])
    for nb in grids:
        p = part[:nb]
        for _ in range(2):
            blip.stream_read(x, p)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            blip.stream_read(x, p)
        e1.record(stream)
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) * 1e-3 / reps
        if float(p.sum()) != nbytes // 4:
            raise RuntimeError("stream read probe: partial sums do not cover the buffer")
        log(f"stream read, {nb} workgroups: {nbytes / dt / 1e9:.0f} GB/s")
        best = max(best, (nbytes / dt / 1e9, nb))
    del x, part
    return best


def scattered_read_rate(total_bytes, run_bytes=12288, row_bytes=3072, nbytes=768 << 20,
                        reps=20, grids=(2048, 8192)):
    """Read rate of one launch that reads total_bytes as runs of run_bytes
    at random row-aligned offsets of a table-sized buffer (a block's
    coefficient rows are runs of 4 rows along a3 at scattered offsets):
    blip_stream_read_runs, event-timed, the best of a few grid sizes.
    Returns (GB/s, us per launch, workgroups)."""
    import torch
    from paper_1204_1121_amd import blip
    nruns = max(1, int(round(total_bytes / run_bytes)))
    rng = np.random.default_rng(12041121)
    offs = rng.integers(0, (nbytes - run_bytes) // row_bytes, nruns) * row_bytes
    buf = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    doff = torch.from_numpy(offs.astype(np.int64)).cuda()
    part = torch.empty(max(grids), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    best = (0.0, 0.0, grids[0])
    for nb in grids:
        p = part[:nb]
        for _ in range(3):
            blip.stream_read_runs(buf, doff, run_bytes, p)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            blip.stream_read_runs(buf, doff, run_bytes, p)
        e1.record(stream)
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) * 1e-3 / reps
        if float(p.sum()) != nruns * run_bytes // 4:
            raise RuntimeError("scattered read probe: partial sums do not cover the runs")
        rate = nruns * run_bytes / dt / 1e9
        log(f"scattered read, {nb} workgroups: {rate:.0f} GB/s, {dt * 1e6:.1f} us per launch")
        if rate > best[0]:
            best = (rate, dt * 1e6, nb)
    del buf, doff, part
    return best


def stream_copy_rate(nbytes=1 << 30, reps=10):
    """Achievable HBM rate on this GPU as a second denominator: a 1 GiB
    device-to-device copy (read plus write bytes over the event-timed copy),
    after the kernel measurements so it does not disturb their caches."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        y.copy_(x)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / reps
    del x, y
    return 2 * nbytes / dt / 1e9


def copy_probe(nbytes=1 << 30, reps=5):
    """A plain device copy of known size (calibrates rocprof byte counters)."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return {"bytes_read": nbytes, "bytes_written": nbytes, "gbs": 2 * nbytes / dt / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--npos", type=int, default=1536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-blocks", action="store_true",
                    help="skip the block sizes 1 .. 1,536 (kernel time and submit-to-completion)")
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the cold-cache measurement (profiling runs)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-walker batch")
    ap.add_argument("--shape", default="", help="fixed block launch shape 'P,o' (no tuning)")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner even if the tuning cache has the shapes")
    ap.add_argument("--save-tuning", default="",
                    help="write the shapes chosen by this run to this JSON file")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving sweep")
    ap.add_argument("--no-ratio", action="store_true", help="skip the fused-ratio figure")
    ap.add_argument("--no-sm", action="store_true",
                    help="skip the Sherman-Morrison update figure")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the storage-dtype / complex k-point section")
    ap.add_argument("--no-paper-sizes", action="store_true",
                    help="skip the values-only complex section at the paper's system sizes")
    ap.add_argument("--no-shard", action="store_true",
                    help="skip the one-GPU orbital-shard shape (96 of the 768 orbitals)")
    ap.add_argument("--no-vmc", action="store_true",
                    help="skip the Monte Carlo step throughput and statistics section")
    ap.add_argument("--no-vmc-stats", action="store_true",
                    help="keep the Monte Carlo step throughput, skip its statistics chains")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests per serving rate point")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (rocprof counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1204_1121_amd import blip
    from paper_1204_1121_amd import workloads as wl
    from paper_1204_1121_amd.tuning import TuneCache

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    leg = None if args.no_cpu_baseline else CpuBaselineLeg()

    spec = wl.spec_tio2()
    t0 = time.perf_counter()
    coef = wl.coefficients(spec)
    table = blip.Table(spec.lattice, spec.n, coef, "f32")
    torch.cuda.synchronize()
    log(f"table {spec.name}: {table.info()['device_bytes'] / 1e6:.1f} MB resident "
        f"({time.perf_counter() - t0:.1f} s)")

    npos, L = args.npos, spec.norb
    blocks_np = [wl.move_block(spec, npos, block=b) for b in range(NROT)]
    blocks = [torch.from_numpy(b).cuda() for b in blocks_np]
    out = table.alloc_outputs(npos)

    # launch shape: the cached autotuning result for this table and size, or
    # a fresh run of the library's autotuner rotating over the benchmark's
    # blocks (setup, outside the timed region)
    cache = TuneCache()
    if args.shape:
        P_, o_ = (int(v) for v in args.shape.split(","))
        table.set_shape(npos, P_, o_)
        best = {"tile_pos": P_, "vec": o_, "us": float("nan"), "from": "--shape"}
    elif not args.retune and cache.apply(table, npos):
        best = dict(cache.get(table, npos), **{"from": "tuning cache"})
    else:
        best, _ = table.autotune(torch.cat(blocks).contiguous(), out, rotate=NROT)
        cache.put(table, npos, False, best, note=f"blip_autotune rotate={NROT}")
        best["from"] = "autotuned now"
    log(f"block shape: P={best['tile_pos']} o={best['vec']} ({best['from']})")
    calls = {id(b): table.bind(b, out) for b in blocks}

    def step(pos):
        calls[id(pos)]()

    wall, t_kernel = time_region(step, blocks, args.steps, args.warmup, stream)
    ms_per_step = wall / args.steps * 1e3
    value = npos * L * args.steps / wall
    # per-launch spread, from a separate pass with an event pair per launch
    _, durs = time_launches(step, blocks, args.steps, 4, stream)
    log(f"tuned: {ms_per_step * 1e3:.1f} us/step wall, {t_kernel * 1e6:.1f} us/launch on the "
        f"GPU (per-launch events: median {np.median(durs) * 1e6:.1f}, "
        f"p99 {np.percentile(durs, 99) * 1e6:.1f})")

    # algorithmic bytes per launch: distinct rows + outputs + positions
    row_bytes = L * 4
    U = [distinct_rows(spec.lattice, spec.n, b) for b in blocks_np]
    b_alg = [u * row_bytes + npos * 5 * L * 4 + 24 * npos for u in U]
    b_alg_mean = float(np.mean(b_alg))
    b_gather = 64 * npos * row_bytes + npos * 5 * L * 4 + 24 * npos
    achieved = b_alg_mean / t_kernel / 1e9

    traffic = None
    try:
        with open(COUNTERS) as f:
            cnt = json.load(f)
        if cnt.get("kernel_source_hash") == kernel_source_hash() and cnt.get("npos") == npos:
            traffic = cnt.get("hbm_bytes_per_launch")
    except (OSError, ValueError):
        pass

    result = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"tio2_72x72x48_L768_block{npos}", "grid": list(spec.n),
                   "cell_bohr": [18.0, 18.0, 12.0], "norb": L, "npos": npos,
                   "storage": "f32", "accumulate": "f32", "wrap": "f64",
                   "outputs": "val+grad+lap", "rotating_blocks": NROT,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "kernel_us": {"mean": t_kernel * 1e6,
                      "per_launch_events_median": float(np.median(durs)) * 1e6,
                      "per_launch_events_p99": float(np.percentile(durs, 99)) * 1e6},
        "shape": {"tile_pos": best["tile_pos"], "vec": best["vec"], "from": best["from"]},
        "bytes_per_launch": {"algorithmic": b_alg_mean, "gather_no_reuse": b_gather,
                             "distinct_rows": float(np.mean(U))},
    }

    if not args.no_blocks:
        try:
            result["block_sizes"] = bench_block_sizes(table, spec, stream, cache, args)
            if args.save_tuning:
                cache.save(args.save_tuning)
        except Exception as e:
            result["block_sizes"] = {"error": f"{type(e).__name__}: {e}"}

    if not args.no_plain:
        def plain_step(pos):
            table.eval(pos, out=out, kernel="plain")
        wall_p, tp = time_region(plain_step, blocks, args.steps, args.warmup, stream)
        result["plain"] = {"value": npos * L * args.steps / wall_p,
                           "kernel_us": tp * 1e6,
                           "hbm_gbs": b_alg_mean / tp / 1e9,
                           "speedup_tuned_vs_plain": tp / t_kernel}
        log(f"plain: kernel {tp * 1e6:.1f} us")

    if not args.no_ratio:
        # fused acceptance ratios on the same blocks: two spins x 768
        # electrons, one row of the (transposed) inverse per position
        # (seeded synthetic rows: the timing does not depend on their values)
        g = torch.Generator(device="cuda").manual_seed(wl.SEED_BASE)
        inv_rows = torch.randn((npos, L), dtype=torch.float64, device="cuda", generator=g)
        rout = (torch.empty(npos, dtype=torch.float64, device="cuda"),
                torch.empty((npos, 3), dtype=torch.float64, device="cuda"),
                torch.empty(npos, dtype=torch.float64, device="cuda"))

        def ratio_step(pos):
            table.ratio(pos, inv_rows, out=rout)
        _, tr = time_region(ratio_step, blocks, args.steps, args.warmup, stream)
        b_ratio = float(np.mean(U)) * row_bytes + npos * (24 + 40) + npos * L * 8
        result["ratio"] = {"kernel_us": tr * 1e6, "evals_per_s": npos * L / tr,
                           "bytes_algorithmic": b_ratio, "hbm_gbs": b_ratio / tr / 1e9,
                           "frac": b_ratio / tr / 1e9 / HBM_PEAK_GBS,
                           "outputs": "ratio + grad ratio + lap ratio per position (FP64)"}
        log(f"ratio: {tr * 1e6:.1f} us per block (ratio, grad, lap) vs {t_kernel * 1e6:.1f} us "
            f"for the orbitals")

    if not args.no_sm:
        result["sm_update"] = bench_sm(args, leg)
        sm = result["sm_update"]
        log(f"sm_update: {sm['us_per_step']:.1f} us per step of {sm['accepted_moves']} moves at "
            f"n = {sm['n']} ({sm['launches_per_step']} launches), "
            f"{sm['roofline']['achieved']:.2f} TFLOP/s FP64; batched {sm['batched']['matrices']} "
            f"matrices: {sm['batched']['us_per_matrix_step']:.1f} us per matrix-step, "
            f"{sm['batched']['tflops_fp64']:.2f} TFLOP/s")

    if not args.no_cold:
        # Cold Infinity Cache: read 1 GiB of unrelated data before every
        # launch (outside its event pair) so no table row survives from the
        # previous launch.  Reads leave the cache clean, so the launch pays
        # no write-back of the sweep.  The main figure keeps the natural
        # cache state of back-to-back blocks.
        sweep = torch.ones(256 << 20, dtype=torch.float32, device="cuda")
        sink = torch.empty((), dtype=torch.float32, device="cuda")
        _, durs_c = time_launches(step, blocks, min(args.steps, 50), 2, stream,
                                  pre=lambda: torch.sum(sweep, dim=0, out=sink))
        tc = float(np.mean(durs_c))
        result["cold_cache"] = {"kernel_us": tc * 1e6, "hbm_gbs": b_alg_mean / tc / 1e9,
                                "frac": b_alg_mean / tc / 1e9 / HBM_PEAK_GBS}
        log(f"cold-cache: kernel {tc * 1e6:.1f} us")
        del sweep

    if args.save_tuning:
        cache.save(args.save_tuning)

    if not args.no_precision:
        try:
            result["precision"] = bench_precision(args, coef, spec, cache, leg)
            if args.save_tuning:
                cache.save(args.save_tuning)
        except Exception as e:
            result["precision"] = {"error": f"{type(e).__name__}: {e}"}

    if not args.no_shard:
        try:
            result["shard_shape"] = bench_shard_shape(args, coef, spec, cache, t_kernel * 1e6,
                                                      leg)
            if args.save_tuning:
                cache.save(args.save_tuning)
        except Exception as e:
            result["shard_shape"] = {"error": f"{type(e).__name__}: {e}"}

    if not args.no_vmc:
        try:
            result["vmc"] = bench_vmc(args, table, spec, leg, cache)
            if args.save_tuning:
                cache.save(args.save_tuning)
        except Exception as e:
            result["vmc"] = {"error": f"{type(e).__name__}: {e}"}

    if not args.no_paper_sizes:
        try:
            result["paper_sizes"] = bench_paper_sizes(args, cache, leg)
            if args.save_tuning:
                cache.save(args.save_tuning)
        except Exception as e:
            result["paper_sizes"] = {"error": f"{type(e).__name__}: {e}"}

    if not args.no_batched:
        try:
            result["batched"] = bench_batched(table, spec, args, leg=leg, coef=coef)
        except Exception as e:            # recorded, never fatal for the main line
            result["batched"] = {"error": f"{type(e).__name__}: {e}"}
    table.free()

    if not args.no_serving:
        try:
            result["serving"] = bench_serving(args, leg)
        except Exception as e:
            result["serving"] = {"error": f"{type(e).__name__}: {e}"}

    if args.copy_probe:
        result["copy_probe"] = copy_probe()
    else:
        g = stream_copy_rate()
        result["stream_copy"] = {"gbs": g, "bytes_per_copy": 2 << 30,
                                 "tiled_kernel_frac_of_copy": achieved / g,
                                 "tiled_kernel_traffic_frac_of_copy":
                                     traffic / t_kernel / 1e9 / g if traffic else None}
        log(f"stream copy {g:.0f} GB/s; tiled kernel at {achieved / g:.2f} of it (algorithmic bytes)")
        rd, nb = stream_read_rate()
        result["stream_read"] = {"gbs": rd, "bytes": 2 << 30, "workgroups": nb,
                                 "frac_of_peak": rd / HBM_PEAK_GBS,
                                 "tiled_kernel_frac_of_read": achieved / rd,
                                 "tiled_kernel_traffic_frac_of_read":
                                     traffic / t_kernel / 1e9 / rd if traffic else None}
        log(f"stream read {rd:.0f} GB/s ({nb} workgroups); tiled kernel at {achieved / rd:.2f} "
            f"of it (algorithmic bytes)")
        moved = traffic if traffic else b_gather
        sr, sus, snb = scattered_read_rate(moved)
        result["scattered_read"] = {
            "gbs": sr, "us_per_launch": sus, "workgroups": snb, "run_bytes": 12288,
            "bytes_per_launch": moved,
            "bytes_from": "kernel counters" if traffic else "no-reuse gather count",
            "tiled_kernel_time_frac": sus / (t_kernel * 1e6)}
        log(f"scattered read of {moved / 1e6:.0f} MB in 12 KB runs: {sr:.0f} GB/s, {sus:.1f} us; "
            f"tiled kernel takes {t_kernel * 1e6 / sus:.2f}x that")

    if leg is not None:
        log("timing the FP64 oracle on the host ...")
        result["cpu_baseline"] = leg.blocks(spec, coef, npos)
    del coef

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
