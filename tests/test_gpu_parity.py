"""GPU parity: the HIP library against the CPU oracle on the same seeded
inputs, through the C interface.

Tolerances: FP64 paths <= 1e-12 max-abs (and a relative bound on non-physical
random data); FP32-MFMA and split-BF16x3 paths <= 1e-6 max-abs on physical
data, and within a multiple of their unit roundoff times the sum of |terms|
(the contraction of |T|) on random data."""
import numpy as np
import pytest

from oracle import network, reconstruction as rc, states_merging as sm, statevector as sv
from workloads import configs, qpu
from workloads.circuits import planted_qaoa
from workloads.cutgraph import build_cut_circuit

from gpu_util import TOL_REL, bins_from_masks, error_bound, oracle_attributed, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sqc = pytest.importorskip("paper_2207_00933_amd.sqc")
runner = pytest.importorskip("paper_2207_00933_amd.runner")

PRECS = [("f64", 0), ("f32", 1), ("bf16x3", 2)]
TOL_ABS = {0: 1e-12, 1: 1e-6, 2: 1e-6}


@pytest.fixture(scope="module")
def session():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = runner.Session(0, 64 << 20)
    yield s
    s.close()


def small_cases():
    return {
        "tiny": configs.tiny(),
        "chain3": configs.chain_brickwork(3, [4, 5, 4], [1, 2], 4, 11),
        "chain4": configs.chain_brickwork(4, [3, 4, 3, 4], [2, 1, 1], 4, 12),
        "qaoa3": build_cut_circuit(planted_qaoa([4, 4, 4], seed=5)),
    }


# ---------------------------------------------------------------------------
# attribution
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["tiny", "chain3", "chain4", "qaoa3", "precision"])
@pytest.mark.parametrize("in_prec,out_prec", [(0, 0), (1, 0), (0, 1)])
def test_attribute(session, name, in_prec, out_prec):
    cc = configs.precision() if name == "precision" else small_cases()[name]
    var = qpu.all_variants(cc)
    if in_prec == sqc.F32:
        var = [v.astype(np.float32).astype(np.float64) for v in var]
    say(f"attribute {name} in={in_prec} out={out_prec}")
    circ = runner.Circuit.from_cut_circuit(session, cc, var, in_prec)
    circ.attribute(out_prec)
    torch.cuda.synchronize()
    want = oracle_attributed(cc, var)
    tol = 1e-12 if out_prec == sqc.F64 else 1e-6
    for i in range(cc.n_sub):
        got = circ.attributed_numpy(i)          # [2^d][4^c]
        err = np.abs(got - want[i].T).max()
        assert err <= tol, (i, err)


def test_attribute_direct_path(session):
    """A subcircuit whose per-state variant slice exceeds the LDS stage
    (6 in-cuts + 1 out-cut: 4^6 * 2 > 4096 values per data state) goes through
    the direct kernel.  Random inputs; sampled label rows."""
    # sub 0: wire 0 measured into cut 6, wires 1..6 data, initialised from
    # cuts 0..5; subs 1..6 each have one wire measured into cut k-1, and sub 1's
    # wire is initialised from cut 6
    n_wires = [7, 1, 1, 1, 1, 1, 1]
    data = [[1, 2, 3, 4, 5, 6], [], [], [], [], [], []]
    cuts = [(k + 1, 0, 0, k + 1) for k in range(6)] + [(0, 0, 1, 0)]
    g = sqc.Graph(n_wires, data, cuts)
    sqc.check_graph(g)
    rng = np.random.default_rng(7)
    var0 = rng.random((4 ** 6 * 3, 1 << 7))
    cc = _GraphView(n_wires, data, cuts)
    sig = sorted(rng.choice(4 ** 7, size=200, replace=False).tolist())
    want = rc.fold_half(rc.attribute(cc, 0, var0, sigmas=sig), 1)
    say("attribute direct path")
    vt = torch.from_numpy(var0).cuda()
    out = torch.empty(sqc.attribute_bytes(g, 0, sqc.F64), dtype=torch.uint8, device="cuda")
    d = sqc.attribute(session.ctx, g, 0, vt, sqc.F64, out, sqc.F64)
    torch.cuda.synchronize()
    got = out.view(torch.float64).cpu().numpy().reshape(1 << d.n_bits, 1 << (2 * d.n_labels))
    assert np.abs(got[:, sig] - want.T).max() <= 1e-12


def _hub_graph(n_in, n_out, d_extra, interleave, seed):
    """Subcircuit 0 with n_in in-cuts and n_out out-cuts to single-wire
    partners.  Wires of sub 0: out-cut wires (measured), in-cut wires
    (initialised from a cut, read out as data) and d_extra plain data wires;
    with ``interleave`` the wire order, the data order and the incident cut
    order are shuffled."""
    rng = np.random.default_rng(seed)
    w = n_out + n_in + d_extra
    wires = list(range(w))
    if interleave:
        rng.shuffle(wires)
    out_w, in_w, extra_w = wires[:n_out], wires[n_out:n_out + n_in], wires[n_out + n_in:]
    data0 = in_w + extra_w
    if interleave:
        rng.shuffle(data0)
    n_wires = [w] + [1] * (n_in + n_out)
    data = [data0] + [[] for _ in range(n_in)] + [[0] for _ in range(n_out)]
    cuts = [(1 + k, 0, 0, in_w[k]) for k in range(n_in)] + \
           [(0, out_w[j], 1 + n_in + j, 0) for j in range(n_out)]
    if interleave:
        order = rng.permutation(len(cuts))
        cuts = [cuts[q] for q in order]
    return n_wires, data, cuts


ATTR_GRAPHS = {
    # name: (n_in, n_out, d_extra, interleave)
    "lds_in4": (4, 1, 2, False),       # 4^4 preparations: LDS stage
    "lds_out7": (0, 7, 3, True),       # 2^7 outcomes: LDS stage
    "reg_2_6": (2, 6, 1, False),       # register form, most out-cuts
    "reg_mixed": (2, 2, 3, True),      # register form, scattered wires and labels
    "reg_in3": (3, 0, 4, True),
}


@pytest.mark.parametrize("name", sorted(ATTR_GRAPHS))
@pytest.mark.parametrize("in_prec,out_prec", [(0, 0), (1, 1)])
def test_attribute_graph_paths(session, name, in_prec, out_prec):
    """Random variants on hub graphs that steer attribution through its LDS
    and register forms; all label rows (or 256 sampled) against the oracle."""
    n_in, n_out, d_extra, inter = ATTR_GRAPHS[name]
    n_wires, data, cuts = _hub_graph(n_in, n_out, d_extra, inter, seed=len(name))
    g = sqc.Graph(n_wires, data, cuts)
    sqc.check_graph(g)
    cc = _GraphView(n_wires, data, cuts)
    rng = np.random.default_rng(11)
    var0 = rng.random((4 ** n_in * 3 ** n_out, 1 << n_wires[0]))
    if in_prec == sqc.F32:
        var0 = var0.astype(np.float32).astype(np.float64)
    c = n_in + n_out
    sig = list(range(4 ** c)) if 4 ** c <= 256 else \
        sorted(rng.choice(4 ** c, size=256, replace=False).tolist())
    want = rc.fold_half(rc.attribute(cc, 0, var0, sigmas=sig), n_out)
    say(f"attribute graph {name} in={in_prec} out={out_prec}")
    dt = torch.float64 if in_prec == sqc.F64 else torch.float32
    vt = torch.from_numpy(var0).to(dt).cuda()
    out = torch.empty(sqc.attribute_bytes(g, 0, out_prec), dtype=torch.uint8, device="cuda")
    d = sqc.attribute(session.ctx, g, 0, vt, in_prec, out, out_prec)
    torch.cuda.synchronize()
    odt = torch.float64 if out_prec == sqc.F64 else torch.float32
    got = out.view(odt).double().cpu().numpy().reshape(1 << d.n_bits, 1 << (2 * d.n_labels))
    tol = 1e-12 if out_prec == sqc.F64 else 1e-6 * max(1.0, np.abs(want).max())
    assert np.abs(got[:, sig] - want.T).max() <= tol


class _GraphView:
    """Minimal cut-circuit view for the oracle from plain graph arrays."""

    class _S:
        def __init__(self, w, dw):
            self.n_wires, self.data_wire = w, dw
            self.n_data = len(dw)

    class _C:
        def __init__(self, c):
            self.up_sub, self.up_wire, self.down_sub, self.down_wire = c

    def __init__(self, n_wires, data, cuts):
        self.subs = [self._S(w, dw) for w, dw in zip(n_wires, data)]
        self.cuts = [self._C(c) for c in cuts]
        self.n_sub = len(n_wires)

    def incident(self, i):
        out = []
        for k, c in enumerate(self.cuts):
            if c.down_sub == i:
                out.append((k, "in"))
            elif c.up_sub == i:
                out.append((k, "out"))
        return out


# ---------------------------------------------------------------------------
# merging
# ---------------------------------------------------------------------------

MERGE_CASES = [
    # d, c, masks (fixed, fixed_val, active, merged)
    (8, 2, (0, 0, 0b00011111, 0b11100000)),          # r = 0, few merged (tiles kernel)
    (12, 2, (0, 0, 0b000000001111, 0b111111110000)),  # r = 0, many merged (rows kernel)
    (14, 4, (0b11111, 0b10110, 0b1111100000, 0b11110000000000)),  # r = 1 prefix shape
    (10, 1, (0b1000000001, 0b1, 0b0101010100, 0b0010101010)),     # arbitrary bits
    (9, 3, (0, 0, 0b111111111, 0)),                   # full state (no merged bits)
    (11, 2, (0b111, 0b101, 0, 0b11111111000)),        # no active bit: one bin
    (13, 0, (0, 0, 0b111, 0b1111111111000)),          # subcircuit without cuts
]


@pytest.mark.parametrize("case", range(len(MERGE_CASES)))
@pytest.mark.parametrize("in_prec,out_prec", [(0, 0), (1, 1), (0, 1)])
def test_merge(session, case, in_prec, out_prec):
    d, c, mk = MERGE_CASES[case]
    rng = np.random.default_rng(100 + case)
    T = rng.standard_normal((1 << d, 1 << (2 * c)))  # attributed layout [x][sigma]
    if in_prec == sqc.F32:
        T = T.astype(np.float32).astype(np.float64)
    m = sqc.Masks(*mk)
    bins = bins_from_masks(m, d)
    want = rc.merge_entries(T.T, bins)  # [sigma][b]
    say(f"merge case {case} in={in_prec} out={out_prec}")
    dt = torch.float64 if in_prec == sqc.F64 else torch.float32
    tin = torch.from_numpy(T).to(dt).cuda()
    att = sqc.tensor_desc(tin, c, d, in_prec, sqc.LAYOUT_ATTRIBUTED)
    session.ensure_workspace(sqc.merge_workspace_bytes(att, m))
    odt = torch.float64 if out_prec == sqc.F64 else torch.float32
    out = torch.empty(want.size, dtype=odt, device="cuda")
    desc = sqc.merge(session.ctx, att, m, out, out_prec)
    torch.cuda.synchronize()
    assert desc.n_bits == bin(mk[2]).count("1") and desc.layout == sqc.LAYOUT_MERGED
    got = out.double().cpu().numpy().reshape(want.shape)
    scale = np.abs(T).max() * len(bins[0])
    tol = 1e-12 * max(1.0, scale) if out_prec == sqc.F64 else 2.0 ** -22 * max(1.0, np.abs(want).max())
    assert np.abs(got - want).max() <= tol


def test_merge_rejects_bad_masks(session):
    T = torch.zeros(1 << 6, dtype=torch.float64, device="cuda")
    att = sqc.tensor_desc(T, 0, 6, sqc.F64, sqc.LAYOUT_ATTRIBUTED)
    out = torch.empty(64, dtype=torch.float64, device="cuda")
    for mk in [(0, 0, 0b111, 0b111), (0, 0, 0b111, 0b110000), (0b1, 0b10, 0b111110, 0)]:
        with pytest.raises(sqc.SqcError) as e:
            sqc.merge(session.ctx, att, sqc.Masks(*mk), out, sqc.F64)
        assert e.value.status == sqc.E_SHAPE


# ---------------------------------------------------------------------------
# contraction on random merged tensors (shapes of several compute graphs)
# ---------------------------------------------------------------------------

def _graph(bits, cuts):
    n = len(bits)
    cc = _GraphView([1] * n, [[] for _ in range(n)], [(u, 0, v, 0) for u, v in cuts])
    return cc


CONTRACT_CASES = {
    "pair": ([4, 6], [(0, 1), (0, 1)]),
    "chain3": ([5, 3, 4], [(0, 1), (0, 1), (1, 2), (1, 2), (1, 2)]),
    "ring4": ([3, 2, 3, 2], [(0, 1), (0, 1), (1, 2), (1, 2), (2, 3), (2, 3), (3, 0), (3, 0)]),
    "disconnected": ([3, 4], []),
    "single": ([7], []),
    "zero_bits": ([3, 0, 4], [(0, 1), (1, 2), (2, 1)]),
    "star5": ([2, 3, 1, 2, 3], [(0, 1), (0, 2), (0, 3), (0, 4), (1, 2), (3, 4)]),
    "wide": ([9, 8], [(0, 1)] * 3),
    # random compute graphs (Erdos-Renyi: each pair cut with probability 0.5
    # and 0.35, seeds 1 and 2, redrawn until connected with degree <= 5):
    # neither chains nor rings, so the greedy pairwise planner picks the order
    "erdos6": ([2, 3, 1, 2, 2, 3], [(0, 3), (0, 5), (1, 2), (1, 4), (2, 3), (3, 4), (4, 5)]),
    "erdos8": ([1, 2, 1, 2, 1, 2, 1, 2], [(0, 1), (0, 2), (0, 4), (0, 7), (1, 2), (1, 3), (1, 6), (3, 5),
                                          (3, 6), (4, 7)]),
}


@pytest.mark.parametrize("name", sorted(CONTRACT_CASES))
@pytest.mark.parametrize("pname,prec", PRECS)
def test_contract_random(session, name, pname, prec):
    bits, cuts = CONTRACT_CASES[name]
    cc = _graph(bits, cuts)
    rng = np.random.default_rng(abs(hash(name)) % 1000)
    Ts = [rng.standard_normal((1 << (2 * len(cc.incident(i))), 1 << bits[i])) for i in range(len(bits))]
    if prec != sqc.F64:
        Ts = [T.astype(np.float32).astype(np.float64) for T in Ts]
    want = network.contract_all(Ts, cc)
    bound = error_bound(Ts, cc)
    g = sqc.Graph([1] * len(bits), [[] for _ in bits], [(u, 0, v, 0) for u, v in cuts])
    dt = torch.float64 if prec == sqc.F64 else torch.float32
    bufs = [torch.from_numpy(T).to(dt).cuda() for T in Ts]
    descs = [sqc.tensor_desc(b, len(cc.incident(i)), bits[i], sqc.F64 if prec == sqc.F64 else sqc.F32,
                             sqc.LAYOUT_MERGED) for i, b in enumerate(bufs)]
    session.ensure_workspace(sqc.contract_workspace_bytes(descs, g, prec))
    for bins_prec in (sqc.F64, sqc.F32):
        say(f"contract {name} prec={pname} bins={bins_prec}")
        out = torch.empty(len(want), dtype=torch.float64 if bins_prec == sqc.F64 else torch.float32,
                          device="cuda")
        sqc.contract(session.ctx, descs, g, prec, out, bins_prec)
        torch.cuda.synchronize()
        got = out.double().cpu().numpy()
        tol = TOL_REL[prec] * bound + (2.0 ** -24 * np.abs(want) if bins_prec == sqc.F32 else 0) + 1e-300
        assert np.all(np.abs(got - want) <= tol), np.abs(got - want).max()


# ---------------------------------------------------------------------------
# whole recursions on physical circuits
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["tiny", "chain3", "chain4", "qaoa3"])
@pytest.mark.parametrize("pname,prec", PRECS)
def test_full_state_against_brute_force(session, name, pname, prec):
    cc = small_cases()[name]
    var = qpu.all_variants(cc)
    circ = runner.Circuit.from_cut_circuit(session, cc, var)
    circ.attribute(sqc.F64)
    n = cc.n
    rec = runner.Recursion(circ, n, sqc.F64, 16)
    say(f"full state {name} {pname}")
    masks = rec.run(prec, 1 << n)
    torch.cuda.synchronize()
    assert runner.active_bits(masks) == n
    P_sub = rec.bins.cpu().numpy()
    P = rc.to_qubit_order(P_sub, cc)
    Pb = sv.probabilities(n, cc.circuit.gates)
    assert np.abs(P - Pb).max() <= TOL_ABS[prec]
    vals, idx = rec.top_list()
    order = np.argsort(-P_sub, kind="stable")[:16]
    assert np.allclose(vals, P_sub[order], atol=0, rtol=0)
    assert abs(rec.sum.item() - P_sub.sum()) <= 1e-12
    if prec == sqc.F64:
        assert list(idx) == list(order)


@pytest.mark.parametrize("name", ["tiny", "chain3", "chain4", "qaoa3"])
@pytest.mark.parametrize("pname,prec", PRECS)
def test_recursions_against_oracle(session, name, pname, prec):
    cc = small_cases()[name]
    var = qpu.all_variants(cc)
    Th = oracle_attributed(cc, var)
    circ = runner.Circuit.from_cut_circuit(session, cc, var)
    circ.attribute(sqc.F64 if prec == sqc.F64 else sqc.F32)
    d = [s.n_data for s in cc.subs]
    M = 1 << max(1, cc.n // 2 - 1)
    rec = runner.Recursion(circ, int(np.log2(M)), sqc.F64, 8)
    scope = None
    lit_states = None
    for r in range(3):
        say(f"recursion {name} {pname} r={r}")
        masks = rec.run(prec, M, scope)
        torch.cuda.synchronize()
        a = runner.active_bits(masks)
        got = rec.bins.cpu().numpy()[: 1 << a]
        lit = sm.assign_states(r, lit_states, M, d)
        want = sm.recursion_bins(Th, cc, lit)
        assert np.abs(got - want).max() <= TOL_ABS[prec]
        vals, idx = rec.top_list()
        k = min(8, len(want))
        order = np.argsort(-got, kind="stable")[:k]
        assert np.array_equal(vals[:k], got[order])
        assert abs(rec.sum.item() - want.sum()) <= TOL_ABS[prec] * 10
        if r > 0:
            assert abs(want.sum() - parent_val) <= 1e-12  # children sum to the parent
            assert abs(rec.sum.item() - parent_val) <= TOL_ABS[prec] * 10
        # expand the bin the oracle ranks first (same partition, same label)
        pick = int(np.argmax(want))
        counts = [len(b) for b in lit]
        ks = sm.split_index(pick, counts)
        lit_states = [lit[i][ks[i]] for i in range(cc.n_sub)]
        parent_val = want[pick]
        scope = sqc.bin_scope(masks, pick)
        if all(m.merged == 0 for m in masks):
            break


@pytest.mark.parametrize("pname,prec", PRECS)
def test_search_finds_bv_solution(session, pname, prec):
    cc = configs.bv(11, 3, seed=14)
    var = qpu.all_variants(cc)
    circ = runner.Circuit.from_cut_circuit(session, cc, var)
    circ.attribute(sqc.F64 if prec == sqc.F64 else sqc.F32)
    logm = 4
    bins = torch.empty(1 << logm, dtype=torch.float64, device="cuda")
    masks = sqc.assign_bins(circ.g.n_data, None, 1 << logm)
    session.ensure_workspace(4 * sqc.recurse_workspace_bytes(circ.att, circ.g, masks, prec))
    say(f"search bv {pname}")
    sols, infos = sqc.search(session.ctx, circ.att, circ.g, 1 << logm, 8, prec, bins, sqc.F64)
    assert sols
    best = max(sols, key=lambda s: s[0])
    assert abs(best[0] - 1) <= TOL_ABS[prec]
    assert sm.global_state(cc, best[3]) == cc.meta["solution"]
    first_leaf = min(r for r, inf in enumerate(infos) if inf[4])
    assert first_leaf + 1 == cc.n // logm
    # oracle search on the same circuit expands the same bins
    Th = oracle_attributed(cc, var)
    res = sm.search(Th, cc, 1 << logm, 8)
    for r in range(first_leaf + 1):
        assert abs(infos[r][2] - res.history[r]["top"][0][1]) <= TOL_ABS[prec]
        assert abs(infos[r][0] - res.history[r]["sum"]) <= TOL_ABS[prec] * 10
