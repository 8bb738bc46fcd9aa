#!/usr/bin/env python3
"""Benchmark: reconstructed bins per second on one MI355X.

Workload ("precision"): a seeded 24-qubit random brickwork circuit (5 layers
of sqrt(X)/sqrt(Y)/sqrt(W) + CZ), cut by 6 wire cuts into a chain of 3
subcircuits; subcircuit outputs from FP64 statevector simulation, cast to
FP32.  One step is the whole hot path on those inputs, already resident in
HBM: attribution of the three subcircuits, bin assignment, merge, the
pairwise contraction into all 2^24 bins, the top-R bins and the FP64 bin sum.

The step is timed for three contraction precisions (FP64 plain, FP32 MFMA,
split-BF16x3 with an FP64-compensated final sum); ``value`` is the path the
precision selector picks at the 1e-6 tolerance, and the fast paths' bins are
also compared with the FP64 GPU path.  The final contraction kernel of every
sixteenth step, and the contraction step before it, are launched with HIP
events recorded by their dispatch inside the timed loop (the final kernel's
live duration, for the roofline fraction); per-step latencies (p50 / p99)
come from a separate pass with an event per step, since per-step events cost
several microseconds.  The CPU baseline is the FP64 oracle
(Eq. 1 evaluated bin by bin) on a bounded sample of bins, timed on the host's
cores before the GPU is touched.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from workloads import configs, qpu  # noqa: E402

METRIC = "reconstructed bins/s & % roofline, MFMA-FP32 vs FP64 plain; p50/p99 latency"
HBM_PEAK = 8.0e12                      # B/s
PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16x3": 2.5e15}  # dense MFMA flop/s
# MFMA products per counted flop: the library counts 2 M N K per GEMM step;
# split-BF16x3 issues three BF16 products for each
MFMA_OPS = {"f64": 1, "f32": 1, "bf16x3": 3}
PREC_ID = {"f64": 0, "f32": 1, "bf16x3": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of bins
# ---------------------------------------------------------------------------

_CPU = {}


def _cpu_worker(chunk):
    from oracle import reconstruction as rc
    t0 = time.perf_counter()
    rc.eval_bins(_CPU["Ts"], _CPU["cc"], chunk)
    return len(chunk), time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cc, var32, seconds: float, n_check: int = 4096):
    """The oracle (Eq. 1 bin by bin, FP64) timed on the host's cores on a
    bounded random sample of the 2^24 outputs.  Also returns the oracle's
    values at n_check of those bins, against which every GPU path's bins are
    compared."""
    import multiprocessing as mp
    from oracle import reconstruction as rc
    Ts = [rc.attribute(cc, i, var32[i].astype(np.float64)) for i in range(cc.n_sub)]
    _CPU["Ts"], _CPU["cc"] = Ts, cc
    # calibrate the per-bin cost on one core
    rng = np.random.default_rng(0)
    probe = rng.integers(0, 1 << cc.n, size=64)
    t0 = time.perf_counter()
    rc.eval_bins(Ts, cc, probe)
    per_bin = (time.perf_counter() - t0) / len(probe)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    # one GPU's share of the host is 16 cores on the GPU machines: never more
    # worker processes than that, nor than the process may run on
    workers = max(1, min(16, affinity))
    per_worker = max(16, int(seconds / per_bin))
    sample = rng.integers(0, 1 << cc.n, size=per_worker * workers)
    chunks = [sample[w * per_worker:(w + 1) * per_worker] for w in range(workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_cpu_worker, chunks)
    wall = time.perf_counter() - t0
    nb = sum(r[0] for r in res)
    check_idx = np.unique(sample[:n_check])
    check_want = rc.eval_bins(Ts, cc, check_idx)
    return {"value": nb / wall, "unit": "bins/s", "cores": workers, "kind": "oracle",
            "sample": f"{nb} bins drawn uniformly from the 2^24 outputs, Eq. 1 evaluated "
                      f"bin by bin (4^6 label assignments each) in FP64 by {workers} worker "
                      f"processes; {wall:.1f} s wall; attribution excluded",
            "cpu_model": cpu_model(), "affinity_cpus": affinity,
            "wall_s": wall, "check_idx": check_idx, "check_want": check_want}


# ---------------------------------------------------------------------------
# GPU
# ---------------------------------------------------------------------------

def run_gpu(cc, var32, steps: int, warmup: int, precs, autotune: bool = True, graph: bool = True, check=None):
    import torch

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU (the HIP library is the only compute path)")
    # a created stream: the steps can then also be recorded into a HIP graph
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        return _run_gpu(cc, var32, steps, warmup, precs, autotune, graph, check)


FINAL_EVERY = 16  # steps per final-contraction launch timed with dispatch events


def _run_gpu(cc, var32, steps, warmup, precs, autotune, graph, check):
    import torch
    from paper_2207_00933_amd import runner, sqc

    s = runner.Session(0, 64 << 20)
    circ = runner.Circuit.from_cut_circuit(s, cc, var32, sqc.F32)
    nbits = cc.n
    M = 1 << nbits
    out = {}
    ref_bins = None
    # bring the device to steady clocks and run every lazy initialisation
    # (kernel loading, timing events, graph capture) before the first timed loop
    for _ in range(20):
        circ.attribute(sqc.F32)
    warm = runner.Recursion(circ, nbits, sqc.F32, 16)
    sqc.ctx_set_timing(s.ctx, sqc.STAGE_FINAL)
    for _ in range(3):
        circ.attribute(sqc.F32)
        warm.run(sqc.F32, M)
    sqc.ctx_set_timing(s.ctx, 0)
    sqc.ctx_timing(s.ctx, sqc.STAGE_FINAL, reset=True)
    sqc.graph_begin(s.ctx)
    warm.run(sqc.F32, M)
    sqc.graph_destroy(sqc.graph_end(s.ctx))
    del warm
    torch.cuda.synchronize()
    # the precision selector's choice for this workload at the stated
    # tolerance (a certified bound of every bin's sum of |terms|)
    circ.attribute(sqc.F32)
    masks = sqc.assign_bins(circ.g.n_data, None, M)
    s.ensure_workspace(sqc.recurse_workspace_bytes(circ.att, circ.g, masks, sqc.AUTO))
    choice, bound = sqc.select_precision(s.ctx, circ.att, circ.g, None, M)
    out["_selector"] = {"choice": {v: k for k, v in PREC_ID.items()}[choice], "bound": bound,
                        "tolerance": 1e-6, "bf16x3_bound": (2.0 ** -13 + 2.0 ** -24) * bound,
                        "f32_bound": (2.0 ** -20 + 2.0 ** -24) * bound}
    log(f"[bench] precision selector: {out['_selector']['choice']} (bound {bound:.3e})")
    for pname in precs:
        prec = PREC_ID[pname]
        att_prec = sqc.F64 if prec == sqc.F64 else sqc.F32
        bins_prec = sqc.F64 if prec == sqc.F64 else sqc.F32
        rec = runner.Recursion(circ, nbits, bins_prec, 16)

        # the step attributes straight into the merged layout of this
        # full-output recursion (sqc_attribute_all_merged: its merge is a
        # transposition, done by the attribution's stores); merged=False is
        # the same step with a separate merge pass, timed below as well
        def step(merged=True):
            circ.attribute(att_prec, merged=merged)
            rec.run(prec, M)

        tune = None
        if autotune:
            # launch choices of this workload's contraction steps (one-time,
            # like a library's tuning cache)
            circ.attribute(att_prec)
            masks = sqc.assign_bins(circ.g.n_data, None, M)
            s.ensure_workspace(sqc.recurse_workspace_bytes(circ.att, circ.g, masks, prec))
            rep = sqc.autotune(s.ctx, circ.att, circ.g, None, M, prec, rec.bins, bins_prec, reps=5)
            tune = {"steps": rep.steps, "candidates": rep.candidates,
                    "default_us": rep.default_us, "tuned_us": rep.tuned_us,
                    "per_step": [{"tile": "16-deep" if rep.step_tile[i] else "64-deep",
                                  "groups": rep.step_groups[i], "nmajor": rep.step_nmajor[i]}
                                 for i in range(min(rep.steps, 64))]}
            log(f"[bench] {pname}: autotune {rep.steps} steps, {rep.default_us:.1f} -> "
                f"{rep.tuned_us:.1f} us")
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        sqc.ctx_timing(s.ctx, sqc.STAGE_FINAL, reset=True)
        torch.cuda.synchronize()
        # timed region: the final contraction of every FINAL_EVERY-th step is
        # launched with HIP events recorded by its dispatch (its live
        # duration); the contraction step before it carries dispatch events
        # too, since without them the final kernel's start stamp falls before
        # the previous kernel has drained (about 3.5 us more on this
        # platform); the other steps carry no instrumentation, which costs
        # several microseconds per step
        t0 = time.perf_counter()
        timed = sqc.STAGE_FINAL | sqc.STAGE_CONTRACT
        for k in range(steps):
            if k % FINAL_EVERY < 2:  # switched on for one step, then off
                sqc.ctx_set_timing(s.ctx, timed if k % FINAL_EVERY == 0 else 0)
            step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sqc.ctx_set_timing(s.ctx, 0)
        fin = sqc.ctx_timing(s.ctx, sqc.STAGE_FINAL, reset=True)
        ms = wall * 1e3 / steps
        # per-step latency (p50 / p99) in a separate pass with an event per step
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        evs[0].record()
        for k in range(steps):
            step()
            evs[k + 1].record()
        torch.cuda.synchronize()
        lat = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(steps))
        # the unfused step (attribution, then the merge kernel), timed the
        # same way (the same dispatch events every FINAL_EVERY-th step)
        for _ in range(warmup):
            step(merged=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            if k % FINAL_EVERY < 2:
                sqc.ctx_set_timing(s.ctx, timed if k % FINAL_EVERY == 0 else 0)
            step(merged=False)
        torch.cuda.synchronize()
        ums = (time.perf_counter() - t0) * 1e3 / steps
        sqc.ctx_set_timing(s.ctx, 0)
        sqc.ctx_timing(s.ctx, sqc.STAGE_FINAL, reset=True)
        log(f"[bench] {pname}: unfused step (separate merge) {ums:.4f} ms/step")
        res = {
            "ms_per_step": ms,
            "bins_per_s": M / (ms * 1e-3),
            "p50_ms": lat[len(lat) // 2],
            "p99_ms": lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)],
            "final_kernel_us": fin.ms * 1e3 / max(1, fin.launches),
            "final_kernel_bytes": fin.bytes / max(1, fin.launches),
            "final_kernel_flops": fin.flops / max(1, fin.launches),
            "bins_sum": rec.sum.item(),
            "autotune": tune,
            "unfused_ms_per_step": ums,
        }
        if graph:
            # the same step recorded once into a HIP graph and replayed: one
            # launch per step instead of one per kernel
            torch.cuda.synchronize()
            sqc.graph_begin(s.ctx)
            step()
            g = sqc.graph_end(s.ctx)
            for _ in range(warmup):
                sqc.graph_launch(s.ctx, g)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                sqc.graph_launch(s.ctx, g)
            torch.cuda.synchronize()
            gms = (time.perf_counter() - t0) * 1e3 / steps
            sqc.graph_destroy(g)
            res["graph"] = {"ms_per_step": gms, "bins_per_s": M / (gms * 1e-3)}
            log(f"[bench] {pname}: graph replay {gms:.4f} ms/step, {M / (gms * 1e-3):.3e} bins/s")
        b = rec.bins.double()
        if prec == sqc.F64:
            ref_bins = b.clone()
        elif ref_bins is not None:
            res["max_abs_vs_fp64_gpu"] = (b - ref_bins).abs().max().item()
        if check is not None:
            got = b[torch.from_numpy(check[0]).to(b.device)].cpu().numpy()
            want = check[1]
            err = np.abs(got - want)
            nz = np.abs(want) > 0
            res["vs_oracle"] = {"bins": int(len(want)), "max_abs": float(err.max()),
                                "max_rel": float((err[nz] / np.abs(want[nz])).max()) if nz.any() else None}
        out[pname] = res
        log(f"[bench] {pname}: {ms:.4f} ms/step, {res['bins_per_s']:.3e} bins/s, "
            f"final kernel {res['final_kernel_us']:.2f} us")
        del rec
    s.close()
    return out


def calib_copy(mib: int):
    """A plain device-to-device copy of known size (reads and writes mib MiB),
    three times; profiler counters of this kernel scale the byte counters of
    the others."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy of {mib} MiB done")
    del src, dst


def measured_traffic():
    """HBM bytes per launch of the final contraction from the committed
    rocprofv3 counter summary, or None when the contraction source changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "final_gemm_precision_traffic.md")
    src = os.path.join(ROOT, "paper_2207_00933_amd", "csrc", "contract.hip")
    try:
        fields = {}
        with open(path) as f:
            for line in f:
                if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_launch", "source_sha256"):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if fields.get("source_sha256") != sha:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# the merging and large workloads: Algorithm 1 on the device
# ---------------------------------------------------------------------------

def replay_bytes(s, circ, M, R, prec, bprec, infos):
    """Algorithmic bytes of a search's recursions (merge reads and writes,
    contraction operands and results, as the stage timing counts them): the
    same Algorithm 1 driven from the host, one sqc_recurse per recursion with
    stage timing on; its records must equal the device search's."""
    import math
    import torch
    from paper_2207_00933_amd import runner, sqc
    stages = sqc.STAGE_MERGE | sqc.STAGE_CONTRACT | sqc.STAGE_FINAL | sqc.STAGE_TOPR
    sqc.ctx_timing(s.ctx, 1, reset=True)
    sqc.ctx_set_timing(s.ctx, stages)
    L, scope, parent, recs = [], None, 1.0, []
    for r in range(R):
        if r > 0 and scope is None:
            break
        rec = runner.Recursion(circ, int(math.log2(M)), bprec, R)
        masks = rec.run(prec, M, scope)
        vals, idx = rec.top_list()
        a = sum(bin(m.active).count("1") for m in masks)
        leaf = all(m.merged == 0 for m in masks)
        recs.append((rec.sum.item(), parent, float(vals[0]), a, leaf))
        if not leaf:
            for q in range(min(R, 1 << a)):
                if vals[q] == vals[q] and vals[q] != -math.inf:
                    L.append((float(vals[q]), r, int(idx[q]), masks))
        L.sort(key=lambda e: (-e[0], e[1], e[2]))
        L = L[:R]
        if not L:
            scope = None
            continue
        e = L.pop(0)
        scope, parent = sqc.bin_scope(e[3], e[2]), e[0]
    sqc.ctx_set_timing(s.ctx, 0)
    nbytes = sum(sqc.ctx_timing(s.ctx, q).bytes for q in (sqc.STAGE_MERGE, sqc.STAGE_CONTRACT, sqc.STAGE_FINAL))
    sqc.ctx_timing(s.ctx, 1, reset=True)
    torch.cuda.synchronize()
    return nbytes, recs == list(infos)


def run_workloads(reps: int = 5, which=("merging", "large", "slicing", "query")):
    """Algorithm 1 (sqc_search, the whole loop on the device) on the merging
    workload (60-qubit QAOA ring, 4 subcircuits, 8 cuts, M = 2^20, R = 12)
    and the large one (200-qubit chain, 16 subcircuits, 24 cuts, M = 2^24,
    R = 20), split-BF16x3 and plain FP64, attributed tensors resident.
    Reports reconstructed bins/s (sum of 2^a over the recursions run, per
    wall second of the whole call: host planning, the enqueue and the final
    wait included) and the HBM roofline fraction of the recursions'
    algorithmic bytes."""
    import torch
    from paper_2207_00933_amd import runner, sqc

    out = {}
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = runner.Session(0, 64 << 20)
        searches = [(name, cc, M, R) for name, cc, M, R in
                    (("merging", lambda: configs.merging(), 1 << 20, 12),
                     ("large", lambda: configs.large(), 1 << 24, 20)) if name in which]
        for name, make, M, R in searches:
            cc = make()
            var = qpu.all_variants(cc)
            circ = runner.Circuit.from_cut_circuit(s, cc, var, sqc.F64)
            res = {"qubits": cc.n, "subcircuits": cc.n_sub, "cuts": len(cc.cuts), "M": M,
                   "max_recursions": R}
            for pname, prec in (("bf16x3", sqc.BF16X3), ("f64", sqc.F64)):
                att = sqc.F64 if prec == sqc.F64 else sqc.F32
                bprec = att
                circ.attribute(att)
                bins = torch.empty(M, dtype=torch.float64 if bprec == sqc.F64 else torch.float32,
                                   device=s.device)
                s.ensure_workspace(sqc.search_workspace_bytes(circ.att, circ.g, M, R, prec))
                sols, infos = sqc.search(s.ctx, circ.att, circ.g, M, R, prec, bins, bprec)  # warm
                nbytes, same = replay_bytes(s, circ, M, R, prec, bprec, infos)
                t0 = time.perf_counter()
                for _ in range(reps):
                    sols, infos = sqc.search(s.ctx, circ.att, circ.g, M, R, prec, bins, bprec)
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t0) / reps
                nb = float(sum(1 << a for (_, _, _, a, _) in infos))
                res[pname] = {"recursions": len(infos), "bins": nb, "ms_per_search": wall * 1e3,
                              "bins_per_s": nb / wall, "algorithmic_bytes": nbytes,
                              "hbm_roofline_frac": nbytes / HBM_PEAK / wall,
                              "solutions": len(sols), "top_prob": sols[0][0] if sols else None,
                              "host_loop_records_equal": same}
                log(f"[workload] {name} {pname}: {len(infos)} recursions, {wall * 1e3:.3f} ms, "
                    f"{nb / wall:.3e} bins/s, HBM fraction {nbytes / HBM_PEAK / wall:.3f}")
            res["speedup_bf16x3_vs_f64"] = res["bf16x3"]["bins_per_s"] / res["f64"]["bins_per_s"]
            out[name] = res
            del circ
        if "slicing" in which:
            out["slicing"] = run_slicing(s, reps)
        if "query" in which:
            out["subset_query"] = run_query(s, reps)
        s.close()
    return out


def run_query(s, reps: int, n_states: int = 1024):
    """Arbitrary-subset queries (Sec. 3) on the precision workload: the
    probabilities of n_states seeded random output states (of 2^24), each a
    recursion with every data bit fixed, batched.  Reports states/s (the
    call waits for the device after every batch)."""
    import torch
    from paper_2207_00933_amd import runner, sqc

    cc = configs.precision()
    var32 = [v.astype(np.float32) for v in qpu.all_variants(cc)]
    circ = runner.Circuit.from_cut_circuit(s, cc, var32, sqc.F32)
    rng = np.random.default_rng(6)
    states = [int(x) for x in rng.integers(0, 1 << cc.n, size=n_states)]
    res = {"workload": "precision: 24 qubits, 3 subcircuits, 6 cuts", "states": n_states}
    for pname, prec in (("bf16x3", sqc.BF16X3), ("f64", sqc.F64)):
        att = sqc.F64 if prec == sqc.F64 else sqc.F32
        circ.attribute(att)
        s.ensure_workspace(sqc.query_states_workspace_bytes(circ.att, circ.g, prec))
        probs = torch.empty(n_states, dtype=torch.float64 if att == sqc.F64 else torch.float32, device=s.device)
        sqc.query_states(s.ctx, circ.att, circ.g, states, prec, probs, att)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sqc.query_states(s.ctx, circ.att, circ.g, states, prec, probs, att)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        res[pname] = {"ms": wall * 1e3, "states_per_s": n_states / wall}
        log(f"[query] {pname}: {n_states} states in {wall * 1e3:.3f} ms, {n_states / wall:.3e} states/s")
    del circ
    return res


def run_slicing(s, reps: int):
    """First-level index slicing (Sec. 6.3) on the precision workload's
    recursion-0 contraction (every data bit active, 2^24 bins): the plain
    contraction against sqc_contract_sliced on the cuts the slicing planner
    picks for a budget of 1/4 and 1/16 of the input floats.  Reports ms per
    contraction, bins/s, the workspace each needs, and the HBM fraction of
    the algorithmic bytes (GEMM operands and results as the stage timing
    counts them, plus each slice's row gathers, read and written once, and
    its FP64 running-sum traffic)."""
    import torch
    from paper_2207_00933_amd import runner, sqc

    cc = configs.precision()
    var32 = [v.astype(np.float32) for v in qpu.all_variants(cc)]
    circ = runner.Circuit.from_cut_circuit(s, cc, var32, sqc.F32)
    g = circ.g
    M = 1 << cc.n
    masks = sqc.assign_bins(g.n_data, None, M)
    cuts = [(c.up_sub, c.down_sub) for c in cc.cuts]
    inputs = sum((4 ** len(cc.incident(i))) << g.n_data[i] for i in range(cc.n_sub))
    res = {"workload": "precision recursion 0: 24 qubits, 3 subcircuits, 6 cuts, 2^24 bins",
           "input_floats": inputs}
    for pname, prec in (("bf16x3", sqc.BF16X3), ("f64", sqc.F64)):
        att = sqc.F64 if prec == sqc.F64 else sqc.F32
        elem = 8 if att == sqc.F64 else 4
        circ.attribute(att)
        merged, bufs = [], []
        for i in range(cc.n_sub):
            n = (4 ** len(cc.incident(i))) << g.n_data[i]
            b = torch.empty(n, dtype=torch.float64 if att == sqc.F64 else torch.float32, device=s.device)
            s.ensure_workspace(sqc.merge_workspace_bytes(circ.att[i], masks[i]))
            merged.append(sqc.merge(s.ctx, circ.att[i], masks[i], b, att))
            bufs.append(b)
        bins = torch.empty(M, dtype=torch.float64 if att == sqc.F64 else torch.float32, device=s.device)
        rows = {}
        for label, budget in (("none", None), ("quarter", inputs / 4), ("sixteenth", inputs / 16)):
            sliced = [] if budget is None else sqc.slice_plan(list(g.n_data), cuts, budget)
            if budget is None:
                ws = sqc.contract_workspace_bytes(merged, g, prec)
                run = lambda: sqc.contract(s.ctx, merged, g, prec, bins, att)  # noqa: E731
            else:
                ws = sqc.contract_sliced_workspace_bytes(merged, g, sliced, prec)
                run = lambda: sqc.contract_sliced(s.ctx, merged, g, sliced, prec, bins, att)  # noqa: E731
            s.ensure_workspace(ws)
            run()
            stages = sqc.STAGE_CONTRACT | sqc.STAGE_FINAL
            sqc.ctx_timing(s.ctx, 1, reset=True)
            sqc.ctx_set_timing(s.ctx, stages)
            run()
            sqc.ctx_set_timing(s.ctx, 0)
            gemm_bytes = sum(sqc.ctx_timing(s.ctx, q).bytes for q in (sqc.STAGE_CONTRACT, sqc.STAGE_FINAL))
            sqc.ctx_timing(s.ctx, 1, reset=True)
            nsl = 4 ** len(sliced)
            gathered = sum(((4 ** (len(cc.incident(i)) - sum(1 for k in sliced if i in cuts[k])))
                            << g.n_data[i]) * elem for i in range(cc.n_sub)
                           if any(i in cuts[k] for k in sliced))
            # per slice: the gathers (read and written once); the final
            # GEMM's running-sum traffic is in the stage bytes above
            extra = nsl * 2 * gathered if sliced else 0.0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                run()
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / reps
            nbytes = gemm_bytes + extra
            rows[label] = {"sliced_cuts": sliced, "slices": nsl, "ms": wall * 1e3, "bins_per_s": M / wall,
                           "workspace_bytes": ws, "algorithmic_bytes": nbytes,
                           "hbm_roofline_frac": nbytes / HBM_PEAK / wall}
            log(f"[slicing] {pname} {label}: cuts {sliced} ({nsl} slices), {wall * 1e3:.3f} ms, "
                f"{M / wall:.3e} bins/s, workspace {ws / 2 ** 20:.1f} MiB, HBM fraction {nbytes / HBM_PEAK / wall:.3f}")
        res[pname] = rows
        del merged, bufs, bins
    del circ
    return res


# ---------------------------------------------------------------------------
# serving: Poisson arrivals of mixed recursions over a resident circuit pool
# ---------------------------------------------------------------------------

def serve_requests(sqc, pool, n_req: int, seed: int):
    """Seeded request mix: a circuit of the pool, a = log2 M in [12, 24]
    (capped by the circuit's unfixed data bits), and for 30% of requests a
    recursion step on a bin of a coarse recursion-0 assignment (the scope of
    a popped bin).  Returns (circuit index, scope, M, active bits)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_req):
        ci = int(rng.integers(len(pool)))
        nd = [s.n_data for s in pool[ci].subs]
        scope, free = None, sum(nd)
        if rng.random() < 0.3:
            m0 = sqc.assign_bins(nd, None, 1 << int(rng.integers(1, 9)))
            a0 = sum(bin(m.active).count("1") for m in m0)
            scope = sqc.bin_scope(m0, int(rng.integers(1 << a0)))
            free -= a0
        a = min(int(rng.integers(12, 25)), free)
        masks = sqc.assign_bins(nd, scope, 1 << a)
        out.append((ci, scope, 1 << a, sum(bin(m.active).count("1") for m in masks)))
    return out


def replay(srv, reqs, arrivals):
    """Submit each request at its arrival time (seconds from the start) and
    record its completion; returns (wall seconds, latencies in ms)."""
    n = len(reqs)
    lat = [0.0] * n
    owner = {}
    i = done = 0
    host = 0.0
    t0 = time.perf_counter()
    while done < n:
        now = time.perf_counter() - t0
        j = i
        while j < n and arrivals[j] <= now:
            j += 1
        if j > i:  # every request that has arrived, in one call
            h0 = time.perf_counter()
            for k, t in enumerate(srv.submit_many(reqs[i:j])):
                owner[t] = i + k
            host += time.perf_counter() - h0
            i = j
        for t in srv.completed():
            k = owner.pop(t)
            lat[k] = (time.perf_counter() - t0 - arrivals[k]) * 1e3
            done += 1
    replay.host_submit_s = host
    return time.perf_counter() - t0, lat


def pct(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))]


def run_serving(n_req: int, slots: int, seed: int = 4, load: float = 0.7):
    import torch
    from paper_2207_00933_amd import runner, sqc

    pool = configs.serving_pool(seed=seed, count=32)
    log(f"[serve] simulating the subcircuit variants of {len(pool)} circuits ...")
    variants = [qpu.all_variants(cc) for cc in pool]
    s = runner.Session(0, 64 << 20)
    circ = {}
    for k, (cc, var) in enumerate(zip(pool, variants)):
        c64 = runner.Circuit.from_cut_circuit(s, cc, var, sqc.F64)
        c64.attribute(sqc.F64)
        c32 = runner.Circuit.from_cut_circuit(s, cc, var, sqc.F64)
        c32.attribute(sqc.F32)
        circ[k] = (c64, c32)
    torch.cuda.synchronize()
    spec = serve_requests(sqc, pool, n_req, seed)
    total_bins = float(sum(1 << a for _, _, _, a in spec))
    fast, plain = sqc.BF16X3, sqc.F64

    def outputs(prec):
        dt = torch.float64 if prec == sqc.F64 else torch.float32
        return [(torch.empty(1 << a, dtype=dt, device="cuda"),
                 torch.empty(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda"),
                 torch.empty(1, dtype=torch.float64, device="cuda")) for _, _, _, a in spec]

    # alone: every request through sqc_recurse one by one, with the per-stage
    # algorithmic byte counts (the ideal time of a request at HBM peak)
    alone = outputs(fast)
    all_stages = (sqc.STAGE_ATTRIBUTE | sqc.STAGE_MERGE | sqc.STAGE_CONTRACT | sqc.STAGE_FINAL
                  | sqc.STAGE_TOPR)
    sqc.ctx_set_timing(s.ctx, all_stages)
    for (ci, scope, M, a), (b, t, bs) in zip(spec, alone):
        c = circ[ci][1]
        s.ensure_workspace(sqc.recurse_workspace_bytes(c.att, c.g, sqc.assign_bins(c.g.n_data, scope, M), fast))
        sqc.recurse(s.ctx, c.att, c.g, scope, M, 16, fast, b, sqc.F32, t, bs)
    torch.cuda.synchronize()
    sqc.ctx_set_timing(s.ctx, 0)
    stage_tot = [sqc.ctx_timing(s.ctx, 1 << q) for q in range(5)]
    ideal_bytes = sum(t.bytes for t in stage_tot)
    # the requests' time at the roof of each stage: HBM bytes or split-BF16x3
    # MFMA work, whichever takes longer (a lower bound on the device time)
    ideal_s = sum(max(t.bytes / HBM_PEAK, t.flops * MFMA_OPS["bf16x3"] / PEAK["bf16x3"]) for t in stage_tot)
    ideal_flops = sum(t.flops for t in stage_tot)
    sqc.ctx_timing(s.ctx, 1, reset=True)
    log(f"[serve] requests at the stage roofs: {ideal_s * 1e3:.3f} ms ({ideal_bytes / 1e9:.2f} GB, "
        f"{ideal_flops * MFMA_OPS['bf16x3'] / 1e12:.2f} TFLOP of BF16 MFMA)")

    def engine(prec, n_slots, max_batch, outs):
        srv = runner.Server(0, n_slots=n_slots, workspace_bytes=8 << 30, max_batch=max_batch)
        ids = {k: srv.register(circ[k][0 if prec == sqc.F64 else 1]) for k in circ}
        bprec = sqc.F64 if prec == sqc.F64 else sqc.F32
        reqs = [srv.request(ids[ci], scope, M, 16, prec, b, bprec, t, bs)
                for (ci, scope, M, a), (b, t, bs) in zip(spec, outs)]
        torch.cuda.synchronize()
        return srv, reqs

    res = {}
    rng = np.random.default_rng(seed + 1)
    gaps = rng.exponential(1.0, n_req)
    lam = None
    # the engine (split-BF16x3, batched), the same engine on the FP64 path,
    # and plain FP64 served one request at a time on one stream
    for name, prec, n_slots, mb in (("engine", fast, slots, 128), ("batched_fp64", plain, slots, 128),
                                    ("serial_fp64", plain, 1, 1)):
        outs = outputs(prec)
        srv, reqs = engine(prec, n_slots, mb, outs)
        # warm-up: the request list once, so the timed replays run with the
        # engine's launch templates cached for every shape (the steady state
        # of a service that sees recurring request shapes)
        replay(srv, reqs, [0.0] * n_req)
        st0 = srv.stats()
        wall_sat, lat_sat = replay(srv, reqs, [0.0] * n_req)
        host_sat = replay.host_submit_s
        st1 = srv.stats()
        sat_plan = st1.plan_seconds - st0.plan_seconds
        sat_launch = st1.launch_seconds - st0.launch_seconds
        sat_batches = st1.batches - st0.batches
        if lam is None:
            lam = load * n_req / wall_sat
        arrivals = np.cumsum(gaps) / lam
        arrivals -= arrivals[0]
        wall, lat = replay(srv, reqs, arrivals.tolist())
        st = srv.stats()
        res[name] = {
            "prec": {sqc.F64: "f64", sqc.F32: "f32", sqc.BF16X3: "bf16x3"}[prec],
            "slots": n_slots, "max_batch": mb,
            "saturation": {"wall_s": wall_sat, "req_per_s": n_req / wall_sat,
                           "bins_per_s": total_bins / wall_sat,
                           "host_submit_s": host_sat, "host_plan_s": sat_plan,
                           "host_launch_s": sat_launch, "batches": sat_batches},
            "poisson": {"lambda_req_per_s": lam, "wall_s": wall, "bins_per_s": total_bins / wall,
                        "p50_ms": pct(lat, 0.50), "p99_ms": pct(lat, 0.99)},
            "max_running": st.max_running, "workspace_peak_bytes": st.workspace_peak,
            "batches": st.batches, "max_batch": st.max_batch,
        }
        log(f"[serve] {name}: saturation {n_req / wall_sat:.0f} req/s "
            f"({total_bins / wall_sat:.3e} bins/s, {host_sat * 1e3:.1f} ms of {wall_sat * 1e3:.1f} "
            f"in submit); Poisson {lam:.0f} req/s: "
            f"p50 {pct(lat, 0.5):.3f} ms p99 {pct(lat, 0.99):.3f} ms; max running {st.max_running}, "
            f"{st.batches} batches (largest {st.max_batch}); burst: {sat_batches} batches, host planning "
            f"{sat_plan * 1e3:.2f} ms, batch launches {sat_launch * 1e3:.2f} ms")
        srv.close()
        if prec == fast:
            same = all(torch.equal(b0, b1) and torch.equal(s0, s1)
                       for (b0, _, s0), (b1, _, s1) in zip(alone, outs))
            fast_outs = outs
        else:
            err = max((b32.double() - b64).abs().max().item()
                      for (b32, _, _), (b64, _, _) in zip(fast_outs, outs))
        del outs
    s.close()
    e = res["engine"]
    return {
        "workload": f"{n_req} requests, Poisson arrivals at {load} x the engine's saturation rate, "
                    "pool of 32 seeded brickwork chains / planted QAOA rings (16-80 qubits, 2-5 "
                    "subcircuits, 2-10 cuts) resident on the device, a = 12..24 active bits, 30% "
                    "recursion steps on a popped bin, top-16",
        "requests": n_req,
        "total_bins": total_bins,
        "engine": e,
        "batched_fp64": res["batched_fp64"],
        "serial_fp64": res["serial_fp64"],
        "speedup_bins_per_s_saturation": e["saturation"]["bins_per_s"]
        / res["serial_fp64"]["saturation"]["bins_per_s"],
        "hbm_roofline_frac_saturation": ideal_bytes / HBM_PEAK / e["saturation"]["wall_s"],
        "roofline_frac_saturation": ideal_s / e["saturation"]["wall_s"],
        "algorithmic_bytes": ideal_bytes,
        "algorithmic_flops": ideal_flops,
        "bitwise_equal_alone": bool(same),
        "max_abs_vs_fp64": err,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU work per worker for the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precs", default="f64,f32,bf16x3")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the contraction launches (sqc_autotune) before timing; off by default "
                         "so that a kernel trace of the command holds only the timed launches")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the HIP-graph replay measurement of the step")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the workloads leg (Algorithm 1 on the device, slicing, queries)")
    ap.add_argument("--workloads", default="merging,large,slicing,query",
                    help="which legs of the workloads leg to run (comma list)")
    ap.add_argument("--workload-reps", type=int, default=5)
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the serving leg (0 skips it)")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration "
                         "for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "reconstruction of one circuit is a single-GPU job here", file=sys.stderr)
        sys.exit(2)

    cc = configs.precision()
    var64 = qpu.all_variants(cc)
    var32 = [v.astype(np.float32) for v in var64]

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        cpu = cpu_baseline(cc, var32, args.cpu_seconds)
        log(f"[bench] CPU oracle: {cpu['value']:.3e} bins/s on {cpu['cores']} cores")

    precs = [p for p in args.precs.split(",") if p]
    if args.calib_copy_mb > 0:
        calib_copy(args.calib_copy_mb)
    gpu = run_gpu(cc, var32, args.steps, args.warmup, precs, autotune=args.autotune,
                  graph=not args.no_graph,
                  check=None if cpu is None else (cpu["check_idx"], cpu["check_want"]))
    selector = gpu.pop("_selector")
    which = [w for w in args.workloads.split(",") if w]
    workloads = None if args.no_workloads or not which else run_workloads(args.workload_reps, which)
    serving = run_serving(args.serve_requests, args.serve_slots) if args.serve_requests > 0 else None
    # the headline path: the one the precision selector picks at the stated
    # tolerance (split-BF16x3 where its bound holds), else the faster fast path
    fast = [p for p in ("bf16x3", "f32") if p in gpu]
    head = selector["choice"] if selector["choice"] in gpu else (
        max(fast, key=lambda p: gpu[p]["bins_per_s"]) if fast else precs[0])
    h = gpu[head]

    def roofline(p):
        x = gpu[p]
        t_hbm = x["final_kernel_bytes"] / HBM_PEAK
        mfma_flops = x["final_kernel_flops"] * MFMA_OPS[p]
        t_mfma = mfma_flops / PEAK[p]
        if t_hbm >= t_mfma:
            r = {"bound": "hbm", "achieved": x["final_kernel_bytes"] / (x["final_kernel_us"] * 1e-6) / 1e9,
                 "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
        else:
            r = {"bound": "mfma", "achieved": mfma_flops / (x["final_kernel_us"] * 1e-6) / 1e12,
                 "peak": PEAK[p] / 1e12, "unit": "TFLOP/s"}
        r["frac"] = r["achieved"] / r["peak"]
        r["traffic"] = measured_traffic() if p == "bf16x3" else None
        r["kernel"] = f"final contraction step ({p})"
        r["kernel_us"] = x["final_kernel_us"]
        return r

    roof = roofline(head)
    for p in ("f32", "bf16x3", "f64"):
        if p in gpu:
            gpu[p]["roofline"] = roofline(p)
    line = {
        "metric": METRIC,
        "value": h["bins_per_s"],
        "unit": "bins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": "precision: 24-qubit random brickwork (5 layers), chain of 3 "
                               "subcircuits, 6 cuts, FP32-cast subcircuit outputs, full 2^24 "
                               "reconstruction (attribution + merge + contraction + top-16 + sum)",
                   "qubits": cc.n, "subcircuits": cc.n_sub, "cuts": len(cc.cuts),
                   "bins": 1 << cc.n},
        "roofline": roof,
        "cpu_baseline": None if cpu is None else {k: cpu[k] for k in
                                                  ("value", "unit", "cores", "kind", "sample", "cpu_model",
                                                   "affinity_cpus")},
        "precision_selector": selector,
        "paper_context": {"note": "context, not the target: the paper gives no kernel times; from its "
                                  "100-qubit runs (5 and 100 recursions, about 50 s and 160 s end to end, "
                                  "QPU time excluded) one 2^20-bin recursion costs about 1.16 s",
                          "bins_per_s": (1 << 20) / 1.16, "hardware": "1 node: 64 CPUs + 1 Nvidia A100",
                          "workload": "100-qubit Supremacy, M = 2^20, random subcircuit outputs"},
        "paths": gpu,
        "latency_ms": {"p50": h["p50_ms"], "p99": h["p99_ms"]},
        "workloads": workloads,
        "serving": serving,
    }
    if "f64" in gpu:
        line["speedup_vs_fp64_gpu"] = h["bins_per_s"] / gpu["f64"]["bins_per_s"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
