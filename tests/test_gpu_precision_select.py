"""The precision selector (SQC_AUTO, sqc_select_precision): the certified
bound B = sum_sigma prod_i max_x |T_i[sigma, x]| covers the oracle's exact
sum of |terms| of every bin; split-BF16x3 is picked where 2^-13 B stays within
the tolerance (the 24-qubit workload at 1e-6) and FP32 MFMA where only
2^-20 B does (a planted random network whose terms cancel heavily); FP64 when
neither does.  Each recursion run with SQC_AUTO matches the oracle within the
tolerance and records its choice."""
import numpy as np
import pytest

from oracle import network
from workloads import configs, qpu

from gpu_util import error_bound, oracle_attributed, sampled_bound, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sqc = pytest.importorskip("paper_2207_00933_amd.sqc")
runner = pytest.importorskip("paper_2207_00933_amd.runner")


@pytest.fixture(scope="module")
def session():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = runner.Session(0, 64 << 20)
    yield s
    s.close()


def _auto_recursion(session, att, g, n_bits, bins_prec=sqc.F32):
    M = 1 << n_bits
    masks = sqc.assign_bins(g.n_data, None, M)
    session.ensure_workspace(sqc.recurse_workspace_bytes(att, g, masks, sqc.AUTO))
    bins = torch.empty(M, dtype=torch.float32 if bins_prec == sqc.F32 else torch.float64, device="cuda")
    top = torch.empty(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda")
    bsum = torch.empty(1, dtype=torch.float64, device="cuda")
    sqc.recurse(session.ctx, att, g, None, M, 4, sqc.AUTO, bins, bins_prec, top, bsum)
    torch.cuda.synchronize()
    return bins.double().cpu().numpy(), sqc.ctx_auto_choice(session.ctx)


def test_selector_picks_bf16x3_on_the_precision_workload(session):
    cc = configs.precision()
    var32 = [v.astype(np.float32) for v in qpu.all_variants(cc)]
    Th = oracle_attributed(cc, [v.astype(np.float64) for v in var32])
    circ = runner.Circuit.from_cut_circuit(session, cc, var32, sqc.F32)
    circ.attribute(sqc.F32)
    choice, B = sqc.select_precision(session.ctx, circ.att, circ.g, None, 1 << cc.n)
    exact = float(error_bound(Th, cc).max())
    say(f"precision workload: bound {B:.3e}, exact max {exact:.3e}, choice {choice}")
    assert B >= exact * (1 - 1e-6)  # (FP32-stored entries: the bound uses them)
    assert choice == sqc.BF16X3
    got, (rec_choice, rec_B) = _auto_recursion(session, circ.att, circ.g, cc.n)
    assert rec_choice == sqc.BF16X3 and rec_B == B
    rng = np.random.default_rng(4)
    sample = np.unique(rng.integers(0, 1 << cc.n, size=2048))
    err = np.abs(got[sample] - network.eval_bins(Th, cc, sample)).max()
    say(f"  AUTO recursion max-abs vs oracle {err:.3e}")
    assert err <= 1e-6


class _View:
    class _C:
        def __init__(self, u, v):
            self.up_sub, self.down_sub = u, v

    def __init__(self, n, cuts):
        self.n_sub = n
        self.cuts = [self._C(u, v) for u, v in cuts]

    def incident(self, i):
        return [(k, "in" if c.down_sub == i else "out") for k, c in enumerate(self.cuts)
                if i in (c.up_sub, c.down_sub)]


def _planted(session, scale, seed):
    """Chain of three subcircuits (6, 5, 6 data bits, 2 + 2 cuts) with random
    signed entries: sums of many terms of both signs (heavy cancellation)."""
    bits, cuts = [6, 5, 6], [(0, 1), (0, 1), (1, 2), (1, 2)]
    cc = _View(3, cuts)
    rng = np.random.default_rng(seed)
    Ts = [(scale * rng.standard_normal((4 ** len(cc.incident(i)), 1 << bits[i]))).astype(np.float32)
          .astype(np.float64) for i in range(3)]
    g = sqc.Graph([1] * 3, [[0] * b for b in bits], [(u, 0, v, 0) for u, v in cuts])
    # attributed layout [2^d][4^c] (labels fastest)
    bufs = [torch.from_numpy(np.ascontiguousarray(T.T)).float().cuda() for T in Ts]
    att = [sqc.tensor_desc(b, len(cc.incident(i)), bits[i], sqc.F32, sqc.LAYOUT_ATTRIBUTED)
           for i, b in enumerate(bufs)]
    return cc, Ts, g, att, bufs, sum(bits)


@pytest.mark.parametrize("scale,want", [(0.04, sqc.F32), (2.0, sqc.F64)])
def test_selector_falls_back_on_heavy_cancellation(session, scale, want):
    cc, Ts, g, att, bufs, nbits = _planted(session, scale, seed=17)
    choice, B = sqc.select_precision(session.ctx, att, g, None, 1 << nbits)
    exact_terms = error_bound(Ts, cc)
    say(f"planted scale {scale}: bound {B:.3e}, exact max {exact_terms.max():.3e}, choice {choice}")
    assert B >= exact_terms.max() * (1 - 1e-12)
    assert choice == want
    want_bins = network.contract_all(Ts, cc)
    got, (rec_choice, _) = _auto_recursion(session, att, g, nbits, sqc.F64)
    assert rec_choice == want
    err = np.abs(got - want_bins).max()
    say(f"  AUTO recursion ({rec_choice}) max-abs vs oracle {err:.3e}, |bins| up to {np.abs(want_bins).max():.3e}")
    assert err <= 1e-6
    if want == sqc.F32:
        # what the selector avoided: split-BF16x3 on the same data is not
        # guaranteed within 1e-6 (its a-priori bound exceeds it)
        assert 2.0 ** -13 * B > 1e-6


def test_tolerance_is_validated(session):
    with pytest.raises(sqc.SqcError):
        sqc.ctx_set_tolerance(session.ctx, 0.0)
    sqc.ctx_set_tolerance(session.ctx, 1e-6)


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_input_is_reported(session, bad):
    """A NaN or infinity in an attributed tensor reaches the bound (the row
    maxima keep NaN), and selection fails with SQC_E_NUMERIC before any
    contraction, for sqc_select_precision and sqc_recurse with SQC_AUTO."""
    cc, Ts, g, att, bufs, nbits = _planted(session, 0.04, seed=17)
    bufs[1][7, 3] = bad
    with pytest.raises(sqc.SqcError) as e:
        sqc.select_precision(session.ctx, att, g, None, 1 << nbits)
    assert e.value.status == sqc.E_NUMERIC
    M = 1 << nbits
    masks = sqc.assign_bins(g.n_data, None, M)
    session.ensure_workspace(sqc.recurse_workspace_bytes(att, g, masks, sqc.AUTO))
    bins = torch.zeros(M, dtype=torch.float64, device="cuda")
    top = torch.empty(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda")
    bsum = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(sqc.SqcError) as e:
        sqc.recurse(session.ctx, att, g, None, M, 4, sqc.AUTO, bins, sqc.F64, top, bsum)
    assert e.value.status == sqc.E_NUMERIC
    torch.cuda.synchronize()
    assert float(bins.abs().max()) == 0.0  # nothing was contracted
    # the context still works on finite input afterwards
    bufs[1][7, 3] = 0.5
    choice, B = sqc.select_precision(session.ctx, att, g, None, M)
    assert np.isfinite(B) and choice in (sqc.F32, sqc.F64, sqc.BF16X3)
