"""GPU parity of the sliced contraction (Sec. 6.3, first-level index slicing)
against the oracle's sliced sum, through the C interface.

Small graphs: every element, for several slicings per graph (one cut, cuts on
different subcircuits, a cut on a subcircuit with no data bits, every cut so
the sliced network falls apart into outer products, none), the three
contraction precisions and both bin precisions; tolerances as for the plain
contraction (a multiple of the unit roundoff times the contraction of |T|,
which bounds every slice's error as well, since the slices split its terms).
Full size: the precision workload (2^24 bins) sliced on one and on two cuts,
4096 sampled bins against Eq. 1 evaluated bin by bin by the oracle."""
import numpy as np
import pytest

from oracle import network
from workloads import configs, qpu

from gpu_util import TOL_REL, assert_bound, error_bound, oracle_attributed, sampled_bound, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sqc = pytest.importorskip("paper_2207_00933_amd.sqc")
runner = pytest.importorskip("paper_2207_00933_amd.runner")

PRECS = [("f64", 0), ("f32", 1), ("bf16x3", 2)]


@pytest.fixture(scope="module")
def session():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = runner.Session(0, 64 << 20)
    yield s
    s.close()


class _View:
    """Compute graph from (up, down) subcircuit pairs, for the oracle."""

    class _C:
        def __init__(self, u, v):
            self.up_sub, self.down_sub = u, v

    def __init__(self, n, cuts):
        self.n_sub = n
        self.cuts = [self._C(u, v) for u, v in cuts]

    def incident(self, i):
        return [(k, "in" if c.down_sub == i else "out") for k, c in enumerate(self.cuts)
                if i in (c.up_sub, c.down_sub)]


CASES = {
    "pair": ([4, 6], [(0, 1), (0, 1)], [[0], [1, 0]]),
    "chain3": ([5, 3, 4], [(0, 1), (0, 1), (1, 2), (1, 2), (1, 2)], [[0], [2, 4], [0, 1, 2, 3, 4], []]),
    "ring4": ([3, 2, 3, 2], [(0, 1), (0, 1), (1, 2), (1, 2), (2, 3), (2, 3), (3, 0), (3, 0)], [[0, 4], [7]]),
    "zero_bits": ([3, 0, 4], [(0, 1), (1, 2), (2, 1)], [[1], [0, 2]]),
    "star5": ([2, 3, 1, 2, 3], [(0, 1), (0, 2), (0, 3), (0, 4), (1, 2), (3, 4)], [[0, 5], [3]]),
    "wide": ([9, 8], [(0, 1)] * 3, [[2], [0, 1, 2]]),
    "erdos8": ([1, 2, 1, 2, 1, 2, 1, 2], [(0, 1), (0, 2), (0, 4), (0, 7), (1, 2), (1, 3), (1, 6), (3, 5),
                                          (3, 6), (4, 7)], [[1, 6], [9]]),
}
SLICINGS = [(name, j) for name in sorted(CASES) for j in range(len(CASES[name][2]))]


def _upload(Ts, cc, bits, prec):
    dt = torch.float64 if prec == sqc.F64 else torch.float32
    bufs = [torch.from_numpy(np.ascontiguousarray(T)).to(dt).cuda() for T in Ts]
    descs = [sqc.tensor_desc(b, len(cc.incident(i)), bits[i], sqc.F64 if prec == sqc.F64 else sqc.F32,
                             sqc.LAYOUT_MERGED) for i, b in enumerate(bufs)]
    return bufs, descs


@pytest.mark.parametrize("name,j", SLICINGS)
@pytest.mark.parametrize("pname,prec", PRECS)
def test_contract_sliced_random(session, name, j, pname, prec):
    bits, cuts, slicings = CASES[name]
    sliced = slicings[j]
    cc = _View(len(bits), cuts)
    rng = np.random.default_rng(1000 + 17 * j + len(name))
    Ts = [rng.standard_normal((1 << (2 * len(cc.incident(i))), 1 << bits[i])) for i in range(len(bits))]
    if prec != sqc.F64:
        Ts = [T.astype(np.float32).astype(np.float64) for T in Ts]
    want = network.contract_sliced(Ts, cc, sliced)
    bound = error_bound(Ts, cc)
    g = sqc.Graph([1] * len(bits), [[] for _ in bits], [(u, 0, v, 0) for u, v in cuts])
    bufs, descs = _upload(Ts, cc, bits, prec)
    session.ensure_workspace(sqc.contract_sliced_workspace_bytes(descs, g, sliced, prec))
    for bins_prec in (sqc.F64, sqc.F32):
        say(f"contract_sliced {name} sliced={sliced} prec={pname} bins={bins_prec}")
        out = torch.empty(len(want), dtype=torch.float64 if bins_prec == sqc.F64 else torch.float32,
                          device="cuda")
        sqc.contract_sliced(session.ctx, descs, g, sliced, prec, out, bins_prec)
        torch.cuda.synchronize()
        got = out.double().cpu().numpy()
        tol = TOL_REL[prec] * bound + (2.0 ** -24 * np.abs(want) if bins_prec == sqc.F32 else 0) + 1e-300
        assert np.all(np.abs(got - want) <= tol), np.abs(got - want).max()


def test_contract_sliced_twice_in_a_row(session):
    """The running sums start over on every call: two calls with different
    slicings into the same output both match the oracle."""
    bits, cuts, _ = CASES["chain3"]
    cc = _View(len(bits), cuts)
    rng = np.random.default_rng(7)
    Ts = [rng.standard_normal((1 << (2 * len(cc.incident(i))), 1 << bits[i])) for i in range(len(bits))]
    bound = error_bound(Ts, cc)
    g = sqc.Graph([1] * len(bits), [[] for _ in bits], [(u, 0, v, 0) for u, v in cuts])
    bufs, descs = _upload(Ts, cc, bits, sqc.F64)
    out = torch.empty(1 << sum(bits), dtype=torch.float64, device="cuda")
    for sliced in ([1, 3], [4]):
        session.ensure_workspace(sqc.contract_sliced_workspace_bytes(descs, g, sliced, sqc.F64))
        sqc.contract_sliced(session.ctx, descs, g, sliced, sqc.F64, out, sqc.F64)
        torch.cuda.synchronize()
        want = network.contract_sliced(Ts, cc, sliced)
        assert np.abs(out.cpu().numpy() - want).max() <= 1e-13 * bound.max() + 1e-300


@pytest.mark.parametrize("sliced", [[0, 0], [5], [-1]])
def test_contract_sliced_rejects(session, sliced):
    bits, cuts, _ = CASES["chain3"]
    cc = _View(len(bits), cuts)
    Ts = [np.zeros((1 << (2 * len(cc.incident(i))), 1 << bits[i])) for i in range(len(bits))]
    g = sqc.Graph([1] * len(bits), [[] for _ in bits], [(u, 0, v, 0) for u, v in cuts])
    bufs, descs = _upload(Ts, cc, bits, sqc.F64)
    out = torch.zeros(1 << sum(bits), dtype=torch.float64, device="cuda")
    with pytest.raises(sqc.SqcError) as e:
        sqc.contract_sliced(session.ctx, descs, g, sliced, sqc.F64, out, sqc.F64)
    assert e.value.status == sqc.E_ARG
    assert float(out.abs().max()) == 0.0  # nothing was enqueued


@pytest.mark.timeout(900)
@pytest.mark.parametrize("sliced", [[0], [0, 3]])
def test_precision_sliced_full_size_sampled(session, sliced):
    """The precision workload's recursion-0 contraction (2^24 bins; every
    data bit active, so the attributed entries are the merged tensors),
    sliced, against Eq. 1 at 4096 sampled bins, each within the path's
    a-priori bound (the slices split the terms of the |T| contraction, so it
    bounds the sliced sum as well)."""
    cc = configs.precision()
    var32 = [v.astype(np.float32) for v in qpu.all_variants(cc)]
    Th = oracle_attributed(cc, [v.astype(np.float64) for v in var32])
    bits = [T.shape[1].bit_length() - 1 for T in Th]
    g = sqc.Graph.from_cut_circuit(cc)
    rng = np.random.default_rng(3)
    sample = np.unique(rng.integers(0, 1 << cc.n, size=4096))
    for pname, prec in (("f64", sqc.F64), ("bf16x3", sqc.BF16X3)):
        T_in = Th if prec == sqc.F64 else [T.astype(np.float32).astype(np.float64) for T in Th]
        want = network.eval_bins(T_in, cc, sample)
        bound = sampled_bound(T_in, cc, sample)
        bufs, descs = _upload(T_in, cc, bits, prec)
        bins_prec = sqc.F64 if prec == sqc.F64 else sqc.F32
        session.ensure_workspace(sqc.contract_sliced_workspace_bytes(descs, g, sliced, prec))
        out = torch.empty(1 << cc.n, dtype=torch.float64 if bins_prec == sqc.F64 else torch.float32, device="cuda")
        say(f"precision sliced={sliced} {pname}")
        sqc.contract_sliced(session.ctx, descs, g, sliced, prec, out, bins_prec)
        torch.cuda.synchronize()
        got = out.double().cpu().numpy()
        assert_bound(got[sample], want, bound, prec, bins_prec == sqc.F32, f"sliced {sliced} {pname}")
        # the bins still sum to one (Sec. 3 invariant at recursion 0)
        assert abs(float(out.double().sum()) - 1.0) <= 1e-6
        del bufs, descs, out


def test_contract_sliced_in_a_graph():
    """Recorded into a HIP graph (gathers, contraction steps and additions:
    no memset nodes), every replay matches the oracle, with an eager sliced
    contraction on the same stream and workspace between replays."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bits, cuts, _ = CASES["ring4"]
    cc = _View(len(bits), cuts)
    rng = np.random.default_rng(21)
    Ts = [rng.standard_normal((1 << (2 * len(cc.incident(i))), 1 << bits[i])).astype(np.float32).astype(np.float64)
          for i in range(len(bits))]
    bound = error_bound(Ts, cc)
    want = network.contract_sliced(Ts, cc, [0, 4])
    want_other = network.contract_sliced(Ts, cc, [7])
    tol = TOL_REL[sqc.BF16X3] * bound + 2.0 ** -24 * np.abs(want) + 1e-300
    tol_other = TOL_REL[sqc.BF16X3] * bound + 2.0 ** -24 * np.abs(want_other) + 1e-300
    g = sqc.Graph([1] * len(bits), [[] for _ in bits], [(u, 0, v, 0) for u, v in cuts])
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = runner.Session(0, 64 << 20)
    sqc.ctx_set_stream(s.ctx, st.cuda_stream)
    try:
        with torch.cuda.stream(st):
            bufs, descs = _upload(Ts, cc, bits, sqc.BF16X3)
            s.ensure_workspace(max(sqc.contract_sliced_workspace_bytes(descs, g, [0, 4], sqc.BF16X3),
                                   sqc.contract_sliced_workspace_bytes(descs, g, [7], sqc.BF16X3)))
            out = torch.empty(len(want), dtype=torch.float32, device="cuda")
            other = torch.empty(len(want), dtype=torch.float32, device="cuda")
            st.synchronize()
            sqc.graph_begin(s.ctx)
            sqc.contract_sliced(s.ctx, descs, g, [0, 4], sqc.BF16X3, out, sqc.F32)
            gr = sqc.graph_end(s.ctx)
            try:
                for k in range(4):
                    out.fill_(float("nan"))
                    sqc.graph_launch(s.ctx, gr)
                    st.synchronize()
                    got = out.double().cpu().numpy()
                    say(f"sliced graph replay {k}: max err {np.abs(got - want).max():.3e}")
                    assert np.all(np.abs(got - want) <= tol), k
                    other.fill_(float("nan"))
                    sqc.contract_sliced(s.ctx, descs, g, [7], sqc.BF16X3, other, sqc.F32)
                    st.synchronize()
                    assert np.all(np.abs(other.double().cpu().numpy() - want_other) <= tol_other), k
            finally:
                sqc.graph_destroy(gr)
    finally:
        st.synchronize()
        s.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("pname,prec", PRECS)
def test_recurse_sliced_by_memory_degree_ten(pname, prec):
    """Memory-driven slicing inside a recursion (Sec. 6.3).  Two subcircuits
    joined by ten cuts (degree 10, 4^10 labels; 3 and 4 data bits, random
    signed entries), M = 2^5 so that each subcircuit also merges a bit.  The
    unsliced recursion needs more than the context's 16 MiB workspace; the
    sliced one fits, slices merged straight from the attributed tensors.
    Every bin matches the oracle's sliced sum of the merged entries (and the
    unsliced contraction) within the path's a-priori bound, and the top-R and
    the bin sum are those of the returned bins."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import reconstruction as rc
    from gpu_util import bins_from_masks
    bits, cuts = [3, 4], [(0, 1)] * 10
    cc = _View(2, cuts)
    rng = np.random.default_rng(31 + prec)
    Ts = [rng.standard_normal((4 ** 10, 1 << b)) for b in bits]
    if prec != sqc.F64:
        Ts = [T.astype(np.float32).astype(np.float64) for T in Ts]
    g = sqc.Graph([1, 1], [[0] * b for b in bits], [(u, 0, v, 0) for u, v in cuts])
    M = 1 << 5
    masks = sqc.assign_bins(g.n_data, None, M)
    groups = [bins_from_masks(masks[i], bits[i]) for i in range(2)]
    merged = [rc.merge_entries(Ts[i], groups[i]) for i in range(2)]
    budget = 16 << 20
    aprec = sqc.F64 if prec == sqc.F64 else sqc.F32
    dt = torch.float64 if aprec == sqc.F64 else torch.float32
    bufs = [torch.from_numpy(np.ascontiguousarray(T.T)).to(dt).cuda() for T in Ts]  # [2^d][4^c]
    att = [sqc.tensor_desc(b, 10, bits[i], aprec, sqc.LAYOUT_ATTRIBUTED) for i, b in enumerate(bufs)]
    assert sqc.recurse_workspace_bytes(att, g, masks, prec) > budget
    sliced, need = sqc.recurse_slices(att, g, masks, prec, 8, budget)
    assert sliced and need <= budget
    want = network.contract_sliced(merged, cc, sliced)
    want_full = network.contract_all(merged, cc)
    bound = network.contract_all([rc.merge_entries(np.abs(Ts[i]), groups[i]) for i in range(2)], cc)
    say(f"sliced recursion {pname}: slices {sliced}, workspace {need} of {budget}")
    s = runner.Session(0, budget)
    try:
        for bins_prec in (sqc.F64, sqc.F32):
            bins = torch.full((M,), float("nan"), dtype=torch.float64 if bins_prec == sqc.F64 else torch.float32,
                              device="cuda")
            top = torch.empty(2 * 8, dtype=torch.float64, device="cuda")
            bsum = torch.empty(1, dtype=torch.float64, device="cuda")
            used = sqc.recurse(s.ctx, att, g, None, M, 8, prec, bins, bins_prec, top, bsum)
            torch.cuda.synchronize()
            assert [(m.active, m.merged) for m in used] == [(m.active, m.merged) for m in masks]
            got = bins.double().cpu().numpy()
            tol = TOL_REL[prec] * bound + (2.0 ** -24 * np.abs(want) if bins_prec == sqc.F32 else 0) + 1e-300
            err = np.abs(got - want)
            say(f"  bins {bins_prec}: max |gpu - oracle| {err.max():.3e} (bound {tol.min():.3e}..{tol.max():.3e})")
            assert np.all(err <= tol)
            assert np.all(np.abs(got - want_full) <= 2 * tol)
            rec = top.cpu().numpy().view(np.uint64).reshape(-1, 2)
            vals = top.cpu().numpy().reshape(-1, 2)[:, 0]
            idx = rec[:, 1].astype(np.int64)
            order = sorted(range(M), key=lambda k: (-got[k], k))[:8]
            assert list(idx) == order and np.array_equal(vals, got[order])
            # (the sum is taken over the FP64 values before they are stored)
            rel = 2.0 ** -23 if bins_prec == sqc.F32 else 1e-12
            assert abs(float(bsum.item()) - float(np.sum(got))) <= rel * float(np.sum(np.abs(got))) + 1e-300
    finally:
        s.close()
