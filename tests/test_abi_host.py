"""The C library without a GPU: it loads, exports every declared symbol, and
its host logic (graph validation, Algorithm 2 as masks, bin scopes, the
Sec. 6.2 cost model, Sec. 6.3 slicing) agrees with the oracle and with the
paper's worked example."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import cost as ocost
from oracle import states_merging as sm
from workloads import configs

sqc = pytest.importorskip("paper_2207_00933_amd.sqc")

HERE = os.path.dirname(os.path.abspath(__file__))
EX = json.load(open(os.path.join(HERE, "golden", "cost_example.json")))


def test_library_exports_every_declared_symbol():
    L = sqc.lib()
    names = sqc.declared_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing
    assert "gfx950" in sqc.version()


def test_binding_types_every_declared_symbol():
    # an untyped ctypes call would pass 64-bit sizes and pointers as int
    missing = sorted(set(sqc.declared_symbols()) - set(sqc.typed_symbols()))
    assert not missing, missing


def test_no_gpu_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(sqc.SqcError) as e:
        sqc.ctx_create(0)
    assert e.value.status == sqc.E_DEVICE


def test_check_graph_accepts_workloads():
    for cc in (configs.tiny(), configs.precision(), configs.merging(), configs.large()):
        sqc.check_graph(sqc.Graph.from_cut_circuit(cc))


@pytest.mark.parametrize("bad,status", [
    ("self_cut", sqc.E_SHAPE), ("wire_range", sqc.E_SHAPE), ("orphan_wire", sqc.E_SHAPE),
    ("double_measure", sqc.E_SHAPE), ("degree", sqc.E_SHAPE), ("sub_range", sqc.E_SHAPE),
])
def test_check_graph_rejects(bad, status):
    n_wires = [3, 3]
    data = [[1, 2], [0, 1, 2]]
    cuts = [(0, 0, 1, 0)]
    if bad == "self_cut":
        cuts = [(0, 0, 0, 1)]
    elif bad == "wire_range":
        cuts = [(0, 5, 1, 0)]
    elif bad == "orphan_wire":
        data = [[2], [0, 1, 2]]
    elif bad == "double_measure":
        cuts = [(0, 0, 1, 0), (0, 0, 1, 1)]
    elif bad == "degree":
        n_wires = [16, 16]
        data = [[], list(range(16))]
        cuts = [(0, k, 1, k) for k in range(16)]
    elif bad == "sub_range":
        cuts = [(0, 0, 2, 0)]
    g = sqc.Graph(n_wires, data, cuts)
    with pytest.raises(sqc.SqcError) as e:
        sqc.check_graph(g)
    assert e.value.status == status
    assert str(e.value)


def _partition_from_masks(m, d):
    """Bins (as sets) described by one subcircuit's masks over d data bits."""
    bins = {}
    for x in range(1 << d):
        if (x & m.fixed) != m.fixed_val:
            continue
        b = 0
        j = 0
        for bit in range(d):
            if (m.active >> bit) & 1:
                b |= ((x >> bit) & 1) << j
                j += 1
        bins.setdefault(b, []).append(x)
    return [sorted(bins[k]) for k in sorted(bins)]


@pytest.mark.parametrize("n_list,M", [([3, 4, 2], 16), ([5, 5], 8), ([1, 6, 3], 1000),
                                      ([4, 4, 4], 1), ([2, 3], 64), ([6, 2, 5, 1], 37)])
def test_assign_bins_equals_algorithm2(n_list, M):
    masks = sqc.assign_bins(n_list, None, M)
    lit = sm.assign_states(0, None, M, n_list)
    for i, d in enumerate(n_list):
        assert _partition_from_masks(masks[i], d) == lit[i]
    # recursion 1 inside a chosen bin
    counts = [len(b) for b in lit]
    for k in (0, int(np.prod(counts)) - 1, int(np.prod(counts)) // 3):
        ks = sm.split_index(k, counts)
        states = [lit[i][ks[i]] for i in range(len(n_list))]
        scope = sqc.bin_scope(masks, k)
        m1 = sqc.assign_bins(n_list, scope, M)
        lit1 = sm.assign_states(1, states, M, n_list)
        for i, d in enumerate(n_list):
            assert _partition_from_masks(m1[i], d) == lit1[i]


def test_assign_bins_workload_shapes():
    m = sqc.assign_bins([16, 14, 16, 14], None, 1 << 20)
    assert [bin(x.active).count("1") for x in m] == [5, 5, 5, 5]
    cc = configs.large()
    d = [s.n_data for s in cc.subs]
    m = sqc.assign_bins(d, None, 1 << 24)
    a = [bin(x.active).count("1") for x in m]
    assert sorted(a) == [1] * 8 + [2] * 8
    # same bin counts as the literal algorithm (on the counts alone)
    lp = [1 << v for v in d]
    while int(np.prod([float(v) for v in lp])) > (1 << 24):
        i = int(np.argmax(lp))
        lp[i] = -(-lp[i] // 2)
    assert [int(np.log2(v)) for v in lp] == a


def test_assign_bins_rejects_bad_scope():
    with pytest.raises(sqc.SqcError):
        sqc.assign_bins([3], [(0b1000, 0, 0, 0)], 4)
    with pytest.raises(sqc.SqcError):
        sqc.assign_bins([3], [(0b001, 0b010, 0, 0)], 4)
    with pytest.raises(sqc.SqcError):
        sqc.assign_bins([3], None, 0)


def test_cost_model_paper_example():
    qubits = EX["graph"]["qubits"]
    cuts = EX["graph"]["cuts"]
    order = [v for p in EX["order"] for v in p]
    c = sqc.plan_cost(qubits, cuts, order)
    assert c.input_floats == EX["input_floats"]
    assert c.plan_mults == sum(EX["step_mults"])
    assert c.naive_mults == EX["naive_mults"]
    assert round(c.naive_mults / c.plan_mults, 1) == EX["naive_over_plan"]
    # the library's own planner finds a plan no worse than the paper's
    c2 = sqc.plan_cost(qubits, cuts, None)
    assert c2.plan_mults <= c.plan_mults


def test_cost_model_matches_oracle_on_workloads():
    for cc in (configs.precision(), configs.merging(), configs.large()):
        d = [s.n_data for s in cc.subs]
        cuts = [(c.up_sub, c.down_sub) for c in cc.cuts]
        c = sqc.plan_cost(d, cuts, None)
        ts = [(frozenset(k for k, _ in cc.incident(i)), 1 << d[i]) for i in range(cc.n_sub)]
        assert c.input_floats == ocost.input_floats(ts)
        order = [(c.order[2 * s], c.order[2 * s + 1]) for s in range(c.n_steps)]
        _, total = ocost.plan_cost(ts, order)
        assert c.plan_mults == pytest.approx(total, rel=1e-12)
        assert c.naive_mults == pytest.approx(ocost.naive_mults(len(cc.cuts), [t[1] for t in ts]),
                                              rel=1e-12)


def _plan_depth(n_sub, order, n_steps):
    """Depth of the contraction tree of a plan given as (position, position)
    pairs over the working list (the result replaces the first position, the
    second is removed)."""
    work, depth = list(range(n_sub)), {i: 0 for i in range(n_sub)}
    nxt, deepest = n_sub, 0
    for s in range(n_steps):
        i, j = order[2 * s], order[2 * s + 1]
        d = max(depth[work[i]], depth[work[j]]) + 1
        deepest = max(deepest, d)
        depth[nxt] = d
        work[i] = nxt
        work.pop(j)
        nxt += 1
    return deepest


def test_planner_keeps_chains_of_small_steps_shallow():
    """The 200-qubit chain (16 subcircuits, 24 cuts) with the active bits of a
    recursion below the first (0 or 1 per subcircuit), where every step is
    small (at most 2^16 result elements): the planner pairs shallow operands
    first, so the tree has depth 5 (size first alone gives depth 11 here, a
    sweep along the chain 15)."""
    cc = configs.large()
    n = cc.n_sub
    cuts = [(c.up_sub, c.down_sub) for c in cc.cuts]
    bits = [0] * 8 + [1] * 8
    c = sqc.plan_cost(bits, cuts, None)
    assert c.n_steps == n - 1
    depth = _plan_depth(n, c.order, c.n_steps)
    assert depth <= 5, depth
    # with large subcircuits the sizes decide: no worse than the sweep
    big = sqc.plan_cost([12] * n, cuts, None)
    assert big.plan_mults <= sqc.plan_cost([12] * n, cuts, [0, 1] * (n - 1)).plan_mults


def test_slicing_paper_example():
    qubits = EX["graph"]["qubits"]
    cuts = EX["graph"]["cuts"]
    chosen = sqc.slice_plan(qubits, cuts, EX["sliced_input_floats"])
    assert len(chosen) == 1 and tuple(cuts[chosen[0]]) == (0, 2)
    ts = [(frozenset(k for k, c in enumerate(cuts) if i in c), 1 << q) for i, q in enumerate(qubits)]
    assert chosen == ocost.greedy_slices(ts, EX["sliced_input_floats"])


def test_slicing_budget_unmet_and_cap():
    """An unreachable budget is an error (SQC_E_NOMEM), not a silent plan
    that misses it; slicing stops at SQC_MAX_SLICED cuts."""
    qubits = EX["graph"]["qubits"]
    cuts = EX["graph"]["cuts"]
    with pytest.raises(sqc.SqcError) as e:  # below the unsliced data floats
        sqc.slice_plan(qubits, cuts, sum(1 << q for q in qubits) - 1)
    assert e.value.status == sqc.E_NOMEM
    # a chain of 12 subcircuits, each pair joined by one cut: meeting the
    # budget of all-sliced inputs would need all 11 cuts, above the cap
    bits = [2] * 12
    chain = [(i, i + 1) for i in range(11)]
    with pytest.raises(sqc.SqcError) as e:
        sqc.slice_plan(bits, chain, 12 * 4)
    assert e.value.status == sqc.E_NOMEM and "SQC_MAX_SLICED" in str(e.value)
    # 120 floats (the total after 8 greedy slices) is met with exactly 8
    # cuts; 119 would need a ninth
    ts = [(frozenset(k for k, c in enumerate(chain) if i in c), 4) for i in range(12)]
    got = sqc.slice_plan(bits, chain, 120)
    assert got == ocost.greedy_slices(ts, 120) and len(got) == sqc.MAX_SLICED
    with pytest.raises(sqc.SqcError) as e:
        sqc.slice_plan(bits, chain, 119)
    assert e.value.status == sqc.E_NOMEM


def _sliced_descs(bits, cuts, prec):
    import torch
    g = sqc.Graph([1] * len(bits), [[] for _ in bits], [(u, 0, v, 0) for u, v in cuts])
    deg = [sum(1 for c in cuts if i in c) for i in range(len(bits))]
    dt = torch.float64 if prec == sqc.F64 else torch.float32
    bufs = [torch.zeros((4 ** deg[i]) << bits[i], dtype=dt) for i in range(len(bits))]
    descs = [sqc.tensor_desc(b, deg[i], bits[i], sqc.F64 if prec == sqc.F64 else sqc.F32, sqc.LAYOUT_MERGED)
             for i, b in enumerate(bufs)]
    return g, descs, bufs


def test_sliced_workspace_layout():
    """Host planning of a sliced contraction (Sec. 6.3): the workspace is the
    sliced network's, the gathered operands and, when something is sliced, two
    FP64 bin vectors (running sums and compensations; the final step adds each
    slice into them, so no slice vector is stored), up to 256-byte
    alignment."""
    bits, cuts = [5, 3, 4], [(0, 1), (0, 1), (1, 2), (1, 2), (1, 2)]
    for prec in (sqc.F64, sqc.F32, sqc.BF16X3):
        g, descs, _ = _sliced_descs(bits, cuts, prec)
        elem = 8 if prec == sqc.F64 else 4
        nb = 1 << sum(bits)
        for sliced in ([], [0], [2, 4], [0, 1, 2, 3, 4]):
            ws = sqc.contract_sliced_workspace_bytes(descs, g, sliced, prec)
            # gathered copies of the tensors touching a sliced cut
            gathered = 0
            for i in range(3):
                deg = sum(1 for c in cuts if i in c)
                s = sum(1 for k in sliced if i in cuts[k])
                if s:
                    gathered += ((4 ** (deg - s)) << bits[i]) * elem
            sums = 2 * nb * 8 if sliced else 0
            rest = [c for k, c in enumerate(cuts) if k not in sliced]
            g2, d2, _ = _sliced_descs(bits, rest, prec)
            own = sqc.contract_workspace_bytes(d2, g2, prec)
            assert own + gathered + sums <= ws <= own + gathered + sums + 256 * 6


@pytest.mark.parametrize("sliced", [[0, 0], [5], [-1], list(range(5)) + [0, 1, 2, 3]])
def test_sliced_rejects_bad_lists(sliced):
    bits, cuts = [5, 3, 4], [(0, 1), (0, 1), (1, 2), (1, 2), (1, 2)]
    g, descs, _ = _sliced_descs(bits, cuts, sqc.F64)
    assert sqc.contract_sliced_workspace_bytes(descs, g, sliced, sqc.F64) == 0


def test_query_workspace_is_fixed_and_validated():
    """Host planning of a subset query (Sec. 3): a fixed workspace whatever
    the number of states; bad tensors are rejected before any launch."""
    import torch
    cc = configs.chain_brickwork(3, [4, 5, 4], [1, 2], 4, 11)
    g = sqc.Graph.from_cut_circuit(cc)
    descs = []
    for i in range(cc.n_sub):
        c = len(cc.incident(i))
        b = torch.zeros((4 ** c) << g.n_data[i], dtype=torch.float64)
        descs.append(sqc.tensor_desc(b, c, g.n_data[i], sqc.F64, sqc.LAYOUT_ATTRIBUTED))
    for prec in (sqc.F64, sqc.F32, sqc.BF16X3):
        assert sqc.query_states_workspace_bytes(descs, g, prec) > 0
    bad = list(descs)
    bad[0] = sqc.tensor_desc(torch.zeros(4), 0, 1, sqc.F64, sqc.LAYOUT_ATTRIBUTED)  # wrong degree
    assert sqc.query_states_workspace_bytes(bad, g, sqc.F64) == 0


def test_sliced_count_limit():
    # ten cuts between two subcircuits: eight may be sliced, nine may not
    bits, cuts = [2, 2], [(0, 1)] * 10
    g, descs, _ = _sliced_descs(bits, cuts, sqc.F32)
    assert sqc.contract_sliced_workspace_bytes(descs, g, list(range(8)), sqc.F32) > 0
    assert sqc.contract_sliced_workspace_bytes(descs, g, list(range(9)), sqc.F32) == 0


def test_search_workspace_covers_every_depth():
    """Host planning of the device search (Algorithm 1): the workspace holds
    the largest recursion of any depth plus the search tables, grows with R,
    and bad arguments are rejected before any launch."""
    import torch
    cc = configs.merging()
    g = sqc.Graph.from_cut_circuit(cc)
    descs = []
    for i in range(cc.n_sub):
        c = len(cc.incident(i))
        descs.append(sqc.tensor_desc(torch.zeros(1), c, g.n_data[i], sqc.F32, sqc.LAYOUT_ATTRIBUTED))
    M = 1 << 20
    masks = sqc.assign_bins(g.n_data, None, M)
    rec = sqc.recurse_workspace_bytes(descs, g, masks, sqc.BF16X3)
    s12 = sqc.search_workspace_bytes(descs, g, M, 12, sqc.BF16X3)
    s20 = sqc.search_workspace_bytes(descs, g, M, 20, sqc.BF16X3)
    # (the recursion query sizes the top-R slots for R = 64)
    assert rec > 0 and s12 > rec - 2 * 64 * 64 * 8 and s20 > s12
    assert sqc.search_workspace_bytes(descs, g, M, 0, sqc.BF16X3) == 0
    assert sqc.search_workspace_bytes(descs, g, M, 65, sqc.BF16X3) == 0
    bad = list(descs)
    bad[1] = sqc.tensor_desc(torch.zeros(1), 1, g.n_data[1], sqc.F32, sqc.LAYOUT_ATTRIBUTED)
    assert sqc.search_workspace_bytes(bad, g, M, 12, sqc.BF16X3) == 0


def _deg10_descs(prec):
    """Two subcircuits joined by ten cuts (degree 10 each; 3 and 4 data
    bits), attributed layout; host planning only, so the buffers are dummies."""
    import torch
    bits, cuts = [3, 4], [(0, 1)] * 10
    g = sqc.Graph([1, 1], [[], []], [(u, 0, v, 0) for u, v in cuts])
    dummy = torch.zeros(1, dtype=torch.float64)
    descs = [sqc.tensor_desc(dummy, 10, b, sqc.F64 if prec == sqc.F64 else sqc.F32, sqc.LAYOUT_ATTRIBUTED)
             for b in bits]
    return g, descs, bits, dummy


@pytest.mark.parametrize("prec", [sqc.F64, sqc.F32, sqc.BF16X3])
def test_recursion_slices_by_memory(prec):
    """Memory-driven slicing of a recursion (Sec. 6.3): nothing is sliced when
    the unsliced plan fits; under a smaller workspace the chooser slices the
    fewest cuts (greedy: largest shrink of the merged inputs, the higher id
    on ties; here every cut ties) whose layout fits, reports a need within the
    budget and below the unsliced need; SQC_E_NOMEM when even SQC_MAX_SLICED
    cuts do not fit."""
    g, descs, bits, _ = _deg10_descs(prec)
    M = 1 << 5
    masks = sqc.assign_bins(bits, None, M)
    assert [bin(m.active).count("1") for m in masks] == [2, 3]
    full = sqc.recurse_workspace_bytes(descs, g, masks, prec)
    sl, need = sqc.recurse_slices(descs, g, masks, prec, sqc.MAX_TOPR, full)
    assert sl == [] and need == full
    eb = 8 if prec == sqc.F64 else 4
    merged = ((4 ** 10) << 2) * eb + ((4 ** 10) << 3) * eb
    assert full >= merged
    budget = 16 << 20
    assert full > budget
    sl, need = sqc.recurse_slices(descs, g, masks, prec, 16, budget)
    s = len(sl)
    assert sl == list(range(9, 9 - s, -1)) and need <= budget < full
    # the layout: each subcircuit's slice of merged rows, two 2^5 FP64 vectors
    assert need >= (merged >> (2 * s)) + 2 * M * 8
    # one cut fewer would not fit: its merged rows alone exceed the budget
    assert s >= 1 and (merged >> (2 * (s - 1))) > budget
    with pytest.raises(sqc.SqcError) as e:
        sqc.recurse_slices(descs, g, masks, prec, 16, 4096)
    assert e.value.status == sqc.E_NOMEM


def test_serve_batching_policy_and_aging():
    """The serving engine's batching policy (host only): requests are taken in
    arrival order while they fit; a later request that fits may pass one that
    does not, each pass counting against the passed one; after 8 passes it
    holds the queue, so it is admitted first once memory frees up (no
    starvation of a large request behind a stream of small ones)."""
    big, small, tab = 1000, 100, 10
    skips = [0, 0, 0]
    # memory for small requests only: the big one (first) is passed over
    picked, held = sqc.serve_pick_batch([big, small, small], [tab] * 3, skips, room=300, max_batch=8)
    assert picked == [1, 2] and not held and skips == [1, 0, 0]
    # a batch of one needs no job table
    picked, _ = sqc.serve_pick_batch([small], [tab], [0], room=small, max_batch=8)
    assert picked == [0]
    # two need both job tables: 2 (small + tab) bytes
    sk = [0, 0]
    picked, _ = sqc.serve_pick_batch([small, small], [tab, tab], sk, room=2 * small + tab, max_batch=8)
    assert picked == [0] and sk == [0, 1]
    picked, _ = sqc.serve_pick_batch([small, small], [tab, tab], [0, 0], room=2 * (small + tab), max_batch=8)
    assert picked == [0, 1]
    # a stream of small requests behind the big one: it is passed 8 times
    skips = [0]
    rounds = 0
    while True:
        sk = skips + [0] * 3
        picked, held = sqc.serve_pick_batch([big] + [small] * 3, [tab] * 4, sk, room=500, max_batch=8)
        skips = sk[:1]
        if held:
            break
        assert picked == [1, 2, 3]
        rounds += 1
        assert rounds <= 8
    assert rounds == 8 and skips == [8] and picked == []
    # once memory frees up it goes first, ahead of the small ones
    sk = [8, 0, 0]
    picked, held = sqc.serve_pick_batch([big, small, small], [tab] * 3, sk, room=big + 2 * small + 3 * tab,
                                        max_batch=8)
    assert picked[0] == 0 and not held
    # max_batch caps the batch; nothing fits: no batch and no skips counted
    sk = [0, 0, 0]
    picked, _ = sqc.serve_pick_batch([small] * 3, [tab] * 3, sk, room=10 ** 6, max_batch=2)
    assert picked == [0, 1]
    sk = [0, 0]
    picked, held = sqc.serve_pick_batch([big, big], [tab] * 2, sk, room=10, max_batch=8)
    assert picked == [] and not held and sk == [0, 0]
    with pytest.raises(sqc.SqcError):
        sqc.serve_pick_batch([small], [tab], [0], room=10, max_batch=0)
