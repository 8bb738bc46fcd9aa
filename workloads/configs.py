"""The named synthetic workloads, seeded and shaped like the paper's benchmarks.

* ``tiny``      10-qubit brickwork, 3 x (single-qubit layer + CZ layer), two
                subcircuits of 6 wires joined by 2 cuts (variants 3^2 and 4^2).
* ``precision`` 24-qubit brickwork, 5 x (1q + CZ) layers, chain of three
                subcircuits with 3 + 3 cuts: d = (8, 8, 8), w = (11, 11, 8),
                4^6 label assignments, 2^24 output bins.
* ``merging``   60-qubit p=1 QAOA on a planted-partition 3-regular graph: ring
                of 4 communities (16, 14, 16, 14), 2 cuts between ring
                neighbours (8 cuts), every subcircuit 2 in + 2 out (144
                variants), widths 18/16.  Used with M = 2^20, R = 12.
* ``large``     200-qubit brickwork, 4 x (1q + CZ) layers, chain of 16
                subcircuits with 24 cuts (nine boundaries with 2 cuts, six with
                1), data widths eight 12s and eight 13s.  Used with M = 2^24.
* ``serving pool``  32 seeded brickwork chains and planted QAOA rings
                (16-80 qubits, 2-5 subcircuits, 2-10 cuts).

Every builder asserts the cut count and widths it promises.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .circuits import bernstein_vazirani, brickwork, moving_boundary_schedule, planted_qaoa
from .cutgraph import CutCircuit, build_cut_circuit


def tiny(seed: int = 1) -> CutCircuit:
    sched = moving_boundary_schedule(3, start=[6], end=[4])
    cc = build_cut_circuit(brickwork(10, 3, seed, sched))
    s = cc.summary()
    assert s["K"] == 2 and s["w"] == [6, 6] and s["V"] == [9, 16], s
    cc.meta["name"] = "tiny"
    return cc


def precision(seed: int = 2) -> CutCircuit:
    sched = moving_boundary_schedule(5, start=[11, 19], end=[8, 16])
    cc = build_cut_circuit(brickwork(24, 5, seed, sched))
    s = cc.summary()
    assert s["K"] == 6 and s["d"] == [8, 8, 8] and s["w"] == [11, 11, 8], s
    assert s["V"] == [27, 1728, 64], s
    cc.meta["name"] = "precision"
    return cc


def merging(seed: int = 3) -> CutCircuit:
    cc = build_cut_circuit(planted_qaoa([16, 14, 16, 14], seed, swaps_per_pair=1))
    s = cc.summary()
    assert s["K"] == 8 and s["d"] == [16, 14, 16, 14], s
    assert s["c"] == [4, 4, 4, 4] and s["V"] == [144] * 4, s
    assert max(s["w"]) <= 20, s
    cc.meta["name"] = "merging"
    return cc


def chain_brickwork(n_sub: int, d: List[int], moves: List[int], n_layers: int,
                    seed: int) -> CutCircuit:
    """Chain of ``n_sub`` subcircuits where boundary k moves ``moves[k]``
    qubits towards lower indices, so ``moves[k]`` lines pass from subcircuit k
    into k+1; subcircuit k ends with ``d[k]`` data qubits."""
    assert len(d) == n_sub and len(moves) == n_sub - 1
    ends = list(np.cumsum(d)[:-1])
    starts = [e + m for e, m in zip(ends, moves)]
    n = int(sum(d))
    sched = moving_boundary_schedule(n_layers, start=starts, end=ends)
    cc = build_cut_circuit(brickwork(n, n_layers, seed, sched))
    s = cc.summary()
    assert s["K"] == sum(moves), s
    assert s["d"] == list(d), s
    return cc


def large(seed: int = 5) -> CutCircuit:
    rng = np.random.default_rng(seed)
    d = [12] * 8 + [13] * 8
    rng.shuffle(d)
    moves = [2] * 9 + [1] * 6
    rng.shuffle(moves)
    cc = chain_brickwork(16, [int(v) for v in d], [int(m) for m in moves], 4, seed)
    s = cc.summary()
    assert s["K"] == 24 and s["n"] == 200 and max(s["V"]) <= 144, s
    assert max(s["w"]) <= 24
    cc.meta["name"] = "large"
    return cc


def bv(n_data: int, n_blocks: int, seed: int) -> CutCircuit:
    cc = build_cut_circuit(bernstein_vazirani(n_data, n_blocks, seed))
    cc.meta["name"] = "bv"
    cc.meta["solution"] = cc.circuit.meta["solution"]
    return cc


# Pool anchors: the extremes of the serving pool's ranges, always present.
POOL_QUBITS = (16, 80)
POOL_CUTS = (2, 10)


def serving_pool(seed: int = 4, count: int = 32,
                 max_width: int = 18) -> List[CutCircuit]:
    """Seeded pool of brickwork chains and planted QAOA rings spanning 16-80
    qubits, 2-5 subcircuits and 2-10 cuts, every subcircuit at most
    ``max_width`` wires (so every variant can be simulated).  With
    ``count >= 3`` the pool starts with three anchors at the ranges' ends
    (16 qubits with 2 cuts, 80 qubits, 10 cuts); the rest is drawn at random
    within the ranges, and the realised ranges are checked."""
    rng = np.random.default_rng(seed)
    pool: List[CutCircuit] = []
    if count >= 3:
        for n_sub, d, moves in ((2, [8, 8], [2]), (5, [16] * 5, [1, 1, 1, 1]), (5, [12] * 5, [2, 3, 3, 2])):
            cc = chain_brickwork(n_sub, d, moves, 4, int(rng.integers(1 << 30)))
            cc.meta["name"] = f"pool{len(pool)}"
            pool.append(cc)
    attempt = 0
    while len(pool) < count:
        attempt += 1
        kind = "qaoa" if (len(pool) % 4 == 3) else "brick"
        try:
            if kind == "brick":
                n_sub = int(rng.integers(2, 6))
                moves = [int(rng.integers(1, 3)) for _ in range(n_sub - 1)]
                lo = max(4, -(-16 // n_sub))
                hi = max(lo + 1, min(max_width - 2, 80 // n_sub) + 1)
                d = [int(rng.integers(lo, hi)) for _ in range(n_sub)]
                K = sum(moves)
                if not (2 <= K <= 10) or not (16 <= sum(d) <= 80):
                    continue
                cc = chain_brickwork(n_sub, d, moves, 4, int(rng.integers(1 << 30)))
            else:
                n_sub = int(rng.integers(3, 5))
                sizes = [int(rng.choice([6, 8, 10, 12])) for _ in range(n_sub)]
                if sum(sizes) < 16:
                    continue
                cc = build_cut_circuit(planted_qaoa(sizes, int(rng.integers(1 << 30))))
            s = cc.summary()
            if max(s["w"]) > max_width or not (2 <= s["K"] <= 10):
                continue
            cc.meta["name"] = f"pool{len(pool)}"
            pool.append(cc)
        except (RuntimeError, ValueError):
            continue
        if attempt > 10000:
            raise RuntimeError("could not fill the serving pool")
    ns = [cc.n for cc in pool]
    ks = [len(cc.cuts) for cc in pool]
    subs = [cc.n_sub for cc in pool]
    widths = [max(cc.summary()["w"]) for cc in pool]
    assert POOL_QUBITS[0] <= min(ns) and max(ns) <= POOL_QUBITS[1], ns
    assert POOL_CUTS[0] <= min(ks) and max(ks) <= POOL_CUTS[1], ks
    assert 2 <= min(subs) and max(subs) <= 5 and max(widths) <= max_width
    if count >= 3:
        assert (min(ns), max(ns)) == POOL_QUBITS and (min(ks), max(ks)) == POOL_CUTS, (ns, ks)
    return pool
