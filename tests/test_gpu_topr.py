"""GPU top-R selection and bin sum against a sort of the same bins.

One subcircuit with no cuts and every data bit active makes the bins the
attributed entries themselves (Eq. 1 with an empty label set), so the top-R
stage can be fed any distribution: heavy ties, all-equal bins, negative values,
and bin counts large enough to take its fallback passes (more listed
sub-tiles than fit on chip, a buffer that overflows on ties).

Expected: the R best bins under the strict order "larger value first, lower
index first" (a stable descending sort), and the compensated FP64 sum of all
bins."""
import math

import numpy as np
import pytest

from gpu_util import error_bound, say

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


def planted(name: str) -> np.ndarray:
    rng = np.random.default_rng(sum(map(ord, name)))
    if name == "ties3":
        return rng.integers(0, 3, 1 << 14).astype(np.float64)
    if name == "zeros":
        return np.zeros(1 << 16)
    if name == "negative":
        return rng.standard_normal(1 << 12)
    if name == "smooth":
        return rng.random(1 << 20)
    if name == "one_peak":
        v = rng.random(1 << 18) * 1e-3
        v[123457] = 5.0
        return v
    if name == "flat_big":  # every sub-tile reaches the threshold
        return np.ones(1 << 23)
    if name == "ties_big":  # half the bins tie at the threshold
        return rng.integers(0, 2, 1 << 22).astype(np.float64)
    if name == "tiny":
        return np.array([0.5, 2.0, 2.0, -1.0])
    raise KeyError(name)


def run_topr(session, vals: np.ndarray, R: int, prec: int, bins_prec: int):
    d = int(np.log2(len(vals)))
    g = sqc.Graph([d], [list(range(d))], [])
    in_prec = sqc.F64 if prec == sqc.F64 else sqc.F32
    dt = torch.float64 if in_prec == sqc.F64 else torch.float32
    buf = torch.from_numpy(vals).to(dt).cuda()
    att = [sqc.tensor_desc(buf, 0, d, in_prec, sqc.LAYOUT_ATTRIBUTED)]
    masks = sqc.assign_bins([d], None, 1 << d)
    session.ensure_workspace(sqc.recurse_workspace_bytes(att, g, masks, prec))
    bins = torch.empty(1 << d, dtype=torch.float64 if bins_prec == sqc.F64 else torch.float32,
                       device="cuda")
    top = torch.full((2 * sqc.MAX_TOPR,), 7.0, dtype=torch.float64, device="cuda")
    bsum = torch.empty(1, dtype=torch.float64, device="cuda")
    sqc.recurse(session.ctx, att, g, None, 1 << d, R, prec, bins, bins_prec, top, bsum)
    torch.cuda.synchronize()
    t = top.cpu().numpy()
    return (bins.double().cpu().numpy(), t[0:2 * R:2], t[1:2 * R:2].view(np.uint64),
            bsum.item())


CASES = ["tiny", "ties3", "zeros", "negative", "smooth", "one_peak", "flat_big", "ties_big"]


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("pname,prec", PRECS)
def test_topr_matches_stable_sort(session, name, pname, prec):
    vals = planted(name)
    for R, bins_prec in ((1, sqc.F64), (16, sqc.F32), (64, sqc.F64)):
        say(f"topr {name} {pname} R={R} bins={bins_prec}")
        bins, tv, ti, s = run_topr(session, vals, R, prec, bins_prec)
        if prec == sqc.F64 and bins_prec == sqc.F64:
            assert np.array_equal(bins, vals)
        k = min(R, len(bins))
        order = np.argsort(-bins, kind="stable")[:k]
        assert np.array_equal(tv[:k], bins[order])
        assert np.array_equal(ti[:k], order.astype(np.uint64))
        if k < R:  # fewer bins than R: the rest are empty records
            assert np.all(tv[k:] == -np.inf)
            assert np.all(ti[k:] == np.uint64(0xFFFFFFFFFFFFFFFF))
        # the sum is taken over the accumulated values: the FP64 inputs on the
        # FP64 path, the stored FP32 accumulators on the others
        ref = vals if prec == sqc.F64 else bins
        want = math.fsum(ref.tolist())
        assert abs(s - want) <= 1e-15 * max(1.0, math.fsum(np.abs(ref).tolist())), (s, want)


def test_topr_two_subcircuits_n_panel_order(session):
    """Two subcircuits (7 and 10 data bits, one cut): the final contraction
    has more n than m panels and runs with n panels outermost; the top-R stage
    must address its sub-tiles in that order.  Random attributed entries."""
    rng = np.random.default_rng(21)
    g = sqc.Graph([8, 10], [list(range(7)), list(range(10))], [(0, 7, 1, 0)])
    bufs = [torch.from_numpy(rng.random((1 << 7) * 4)).cuda(),
            torch.from_numpy(rng.random((1 << 10) * 4)).cuda()]
    att = [sqc.tensor_desc(bufs[0], 1, 7, sqc.F64, sqc.LAYOUT_ATTRIBUTED),
           sqc.tensor_desc(bufs[1], 1, 10, sqc.F64, sqc.LAYOUT_ATTRIBUTED)]
    M = 1 << 17
    for pname, prec in PRECS:
        say(f"topr two subs {pname}")
        masks = sqc.assign_bins([7, 10], None, M)
        session.ensure_workspace(sqc.recurse_workspace_bytes(att, g, masks, prec))
        bins = torch.empty(M, dtype=torch.float64, device="cuda")
        top = torch.empty(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda")
        bsum = torch.empty(1, dtype=torch.float64, device="cuda")
        sqc.recurse(session.ctx, att, g, None, M, 32, prec, bins, sqc.F64, top, bsum)
        torch.cuda.synchronize()
        b = bins.cpu().numpy()
        t = top.cpu().numpy()
        order = np.argsort(-b, kind="stable")[:32]
        assert np.array_equal(t[0:64:2], b[order])
        assert np.array_equal(t[1:64:2].view(np.uint64), order.astype(np.uint64))
        assert abs(bsum.item() - math.fsum(b.tolist())) <= 1e-12 * math.fsum(np.abs(b).tolist())


@pytest.mark.parametrize("d0,d1", [(7, 15), (15, 7), (11, 11)])
def test_topr_product_ties(session, d0, d1):
    """Two subcircuits joined by one cut whose attributed entries are small
    integers on label 0 and zero elsewhere: every bin is the product
    A[x0] B[x1], exact in every precision, and a quarter of the bins tie at
    the top value (a flat top spread over every sub-tile, the layout the
    sub-tile pruning and the best-first visit order act on), in both
    orientations of the final contraction."""
    rng = np.random.default_rng(100 + d0)
    g = sqc.Graph([d0 + 1, d1], [list(range(d0)), list(range(d1))], [(0, d0, 1, 0)])
    A = np.zeros(((1 << d0), 4))
    B = np.zeros(((1 << d1), 4))
    A[:, 0] = rng.integers(1, 3, 1 << d0)
    B[:, 0] = rng.integers(1, 3, 1 << d1)
    bufs = [torch.from_numpy(A.reshape(-1)).cuda(), torch.from_numpy(B.reshape(-1)).cuda()]
    att = [sqc.tensor_desc(bufs[0], 1, d0, sqc.F64, sqc.LAYOUT_ATTRIBUTED),
           sqc.tensor_desc(bufs[1], 1, d1, sqc.F64, sqc.LAYOUT_ATTRIBUTED)]
    M = 1 << (d0 + d1)
    for pname, prec in PRECS:
        masks = sqc.assign_bins([d0, d1], None, M)
        session.ensure_workspace(sqc.recurse_workspace_bytes(att, g, masks, prec))
        for R in (1, 2, 16, 64):
            say(f"topr product ties {d0}+{d1} {pname} R={R}")
            bins = torch.empty(M, dtype=torch.float64, device="cuda")
            top = torch.empty(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda")
            bsum = torch.empty(1, dtype=torch.float64, device="cuda")
            sqc.recurse(session.ctx, att, g, None, M, R, prec, bins, sqc.F64, top, bsum)
            torch.cuda.synchronize()
            b = bins.cpu().numpy()
            t = top.cpu().numpy()
            assert np.array_equal(np.sort(b), np.sort(np.outer(A[:, 0], B[:, 0]).ravel()))
            order = np.argsort(-b, kind="stable")[:R]
            assert np.array_equal(t[0:2 * R:2], b[order])
            assert np.array_equal(t[1:2 * R:2].view(np.uint64), order.astype(np.uint64))
            assert bsum.item() == math.fsum(b.tolist())


class _Cuts:
    """Cut-list view for the oracle's contraction (one wire per subcircuit,
    bins taken as given)."""

    class _C:
        def __init__(self, u, v):
            self.up_sub, self.up_wire, self.down_sub, self.down_wire = u, 0, v, 0

    def __init__(self, n, cuts):
        self.n_sub = n
        self.cuts = [self._C(u, v) for u, v in cuts]

    def incident(self, i):
        out = []
        for k, c in enumerate(self.cuts):
            if c.down_sub == i:
                out.append((k, "in"))
            elif c.up_sub == i:
                out.append((k, "out"))
        return out


@pytest.mark.parametrize("pname,prec", PRECS)
def test_topr_interleaved_final_maps(session, pname, prec):
    """Subcircuits 0 and 2 share two cuts and are contracted first, so the
    final contraction's m side holds the bins of subcircuits 0 and 2, which
    are not adjacent in the bin index (two-run index map: the top-R stage's
    general sub-tile addressing).  Random signed tensors; bins against the
    oracle's contraction, top-R against a stable sort of the same bins."""
    from oracle import network
    bits, cuts = [6, 7, 6], [(0, 2), (0, 2), (2, 1)]
    cc = _Cuts(3, cuts)
    rng = np.random.default_rng(77)
    Ts = [rng.standard_normal((1 << (2 * len(cc.incident(i))), 1 << bits[i])) for i in range(3)]
    if prec != sqc.F64:
        Ts = [T.astype(np.float32).astype(np.float64) for T in Ts]
    want = network.contract_all(Ts, cc)
    g = sqc.Graph([1] * 3, [[] for _ in bits], [(u, 0, v, 0) for u, v in cuts])
    in_prec = sqc.F64 if prec == sqc.F64 else sqc.F32
    dt = torch.float64 if in_prec == sqc.F64 else torch.float32
    # attributed layout [x][sigma]: the transpose of the oracle's [sigma][x]
    bufs = [torch.from_numpy(np.ascontiguousarray(T.T)).to(dt).cuda() for T in Ts]
    att = [sqc.tensor_desc(b, len(cc.incident(i)), bits[i], in_prec, sqc.LAYOUT_ATTRIBUTED)
           for i, b in enumerate(bufs)]
    M = 1 << sum(bits)
    masks = sqc.assign_bins(bits, None, M)
    session.ensure_workspace(sqc.recurse_workspace_bytes(att, g, masks, prec))
    # error bound: unit roundoff of the path times the contraction of |T|
    bound = error_bound(Ts, cc) * {sqc.F64: 1e-13, sqc.F32: 2.0 ** -20, sqc.BF16X3: 2.0 ** -13}[prec]
    for R in (1, 16, 64):
        say(f"topr interleaved {pname} R={R}")
        bins = torch.empty(M, dtype=torch.float64, device="cuda")
        top = torch.empty(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda")
        bsum = torch.empty(1, dtype=torch.float64, device="cuda")
        sqc.recurse(session.ctx, att, g, None, M, R, prec, bins, sqc.F64, top, bsum)
        torch.cuda.synchronize()
        b = bins.cpu().numpy()
        assert np.all(np.abs(b - want) <= bound + 1e-300)
        t = top.cpu().numpy()
        order = np.argsort(-b, kind="stable")[:R]
        assert np.array_equal(t[0:2 * R:2], b[order])
        assert np.array_equal(t[1:2 * R:2].view(np.uint64), order.astype(np.uint64))
        assert abs(bsum.item() - math.fsum(b.tolist())) <= 1e-12 * math.fsum(np.abs(b).tolist())
