"""Pins of the oracle's Algorithms 1-2: partition properties, the shapes the
workloads produce, merged bins against brute force, child bins summing to the
parent, full-state equivalence for M >= 2^n and the n/log2(M) recursion count
of a single-solution circuit (Sec. 4)."""
import itertools

import numpy as np
import pytest

from oracle import reconstruction as rc, states_merging as sm, statevector as sv
from workloads import configs, qpu


def folded(cc):
    var = qpu.all_variants(cc)
    Ts = [rc.attribute(cc, i, var[i]) for i in range(cc.n_sub)]
    return Ts, [rc.fold_half(Ts[i], sum(1 for _, r in cc.incident(i) if r == "out"))
                for i in range(cc.n_sub)]


@pytest.mark.parametrize("n_list,M", [([3, 4, 2], 16), ([5, 5], 8), ([1, 6, 3], 1000),
                                      ([4, 4, 4], 1), ([2, 3], 64)])
def test_partition_properties(n_list, M):
    bins = sm.assign_states(0, None, M, n_list)
    total = 1
    for i, b in enumerate(bins):
        total *= len(b)
        members = sorted(itertools.chain(*b))
        assert members == list(range(1 << n_list[i]))
        sizes = {len(x) for x in b}
        assert len(sizes) == 1
        assert len(b) & (len(b) - 1) == 0  # power of two
    m2 = 1 << int(np.floor(np.log2(M)))
    assert total <= m2
    # maximal: doubling any subcircuit's bin count would exceed M (or its states)
    assert total * 2 > m2 or all(len(b) == (1 << n) for b, n in zip(bins, n_list))


def test_bins_are_low_bit_classes():
    # the j mod l' rule keeps the lowest log2(l') enumeration bits of a state
    bins = sm.assign_states(0, None, 8, [5])
    for k, b in enumerate(bins[0]):
        assert all((x & 7) == k for x in b)
    # and inside a chosen bin the next bits are used
    chosen = [bins[0][5]]
    child = sm.assign_states(1, chosen, 2, [5])
    for k, b in enumerate(child[0]):
        assert all(((x >> 3) & 1) == k and (x & 7) == 5 for x in b)


def test_workload_shapes():
    # merging workload: d = (16, 14, 16, 14), M = 2^20
    b0 = sm.assign_states(0, None, 1 << 20, [16, 14, 16, 14])
    assert [len(b) for b in b0] == [32, 32, 32, 32]
    pick = [b0[i][0] for i in range(4)]
    b1 = sm.assign_states(1, pick, 1 << 20, [16, 14, 16, 14])
    assert [len(b) for b in b1] == [32, 32, 32, 32]
    # large workload: eight 12s and eight 13s, M = 2^24 -> eight 1s and eight 2s
    d = [12, 13] * 8
    a = [len(b) for b in sm.assign_states(0, None, 1 << 24, d)]
    assert sorted(a) == [2] * 8 + [4] * 8


def test_merged_bins_equal_brute_force_sums():
    cc = configs.chain_brickwork(3, [3, 4, 3], [1, 2], 4, 31)
    Ts, Th = folded(cc)
    P = rc.reconstruct_eq1(Ts, cc)  # subcircuit-major
    d = [s.n_data for s in cc.subs]
    bins = sm.assign_states(0, None, 8, d)
    Pm = sm.recursion_bins(Th, cc, bins)
    counts = [len(b) for b in bins]
    for gi in range(len(Pm)):
        ks = sm.split_index(gi, counts)
        tot = 0.0
        for xs in itertools.product(*[bins[i][ks[i]] for i in range(cc.n_sub)]):
            idx = xs[0] + (xs[1] << d[0]) + (xs[2] << (d[0] + d[1]))
            tot += P[idx]
        assert abs(Pm[gi] - tot) <= 1e-13


def test_child_bins_sum_to_parent():
    cc = configs.chain_brickwork(3, [3, 4, 3], [1, 2], 4, 31)
    _, Th = folded(cc)
    d = [s.n_data for s in cc.subs]
    b0 = sm.assign_states(0, None, 8, d)
    P0 = sm.recursion_bins(Th, cc, b0)
    counts = [len(b) for b in b0]
    for k in (0, 3, int(np.argmax(P0))):
        ks = sm.split_index(k, counts)
        states = [b0[i][ks[i]] for i in range(cc.n_sub)]
        b1 = sm.assign_states(1, states, 8, d)
        P1 = sm.recursion_bins(Th, cc, b1)
        assert abs(P1.sum() - P0[k]) <= 1e-14


def test_full_state_when_m_covers_everything():
    cc = configs.tiny()
    Ts, Th = folded(cc)
    res = sm.search(Th, cc, M=1 << cc.n, R=4)
    P = rc.reconstruct_eq1(Ts, cc)
    assert len(res.history) == 1  # one recursion: every bin is a leaf
    assert res.history[0]["a"] == [s.n_data for s in cc.subs]
    top = res.history[0]["top"]
    order = np.argsort(-P, kind="stable")[:4]
    assert [k for k, _ in top] == list(order)
    assert np.allclose([p for _, p in top], P[order], atol=1e-15)


@pytest.mark.parametrize("n_data,blocks,logm", [(11, 3, 4), (11, 2, 3), (15, 4, 4)])
def test_bv_recursion_count(n_data, blocks, logm):
    """A single-solution circuit is found after exactly n / log2(M) recursions
    (Sec. 4; n counts every measured qubit, the ancilla included)."""
    cc = configs.bv(n_data, blocks, seed=n_data + blocks)
    n = cc.n
    assert n % logm == 0
    _, Th = folded(cc)
    res = sm.search(Th, cc, M=1 << logm, R=3 * n)
    assert res.solutions, "no solution found"
    best = max(res.solutions, key=lambda s: s[0])
    assert abs(best[0] - 1) <= 1e-12
    assert sm.global_state(cc, best[1]) == cc.meta["solution"]
    first_leaf = min(h["r"] for h in res.history if h["leaf"])
    assert first_leaf + 1 == n // logm
    # every recursion before it expanded the bin holding the solution
    for h in res.history[:first_leaf + 1]:
        assert abs(h["top"][0][1] - 1) <= 1e-12
