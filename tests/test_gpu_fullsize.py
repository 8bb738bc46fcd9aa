"""GPU parity at the full sizes of the three reconstruction workloads, on
sampled outputs the oracle evaluates one by one, plus the invariants that hold
at any size.  Every sampled bin is held to the path's a-priori rounding bound
(a multiple of its unit roundoff times the oracle's contraction of |T| at that
bin) and, as a second check, to the absolute tolerance for physical data.

- precision (24 qubits, 3 subcircuits, 6 cuts, FP32-cast outputs): the
  2^24-bin reconstruction in the launch configuration bench.py times (FP32
  bins on the fast paths), 4096 sampled bins against Eq. 1 evaluated by the
  oracle on the same cast inputs; all 2^24 bins of each fast path against the
  FP64 GPU path at the per-bin bound (the oracle's |T| contraction over the
  whole output); the sum of all bins is 1 to rounding.
- merging (60-qubit QAOA, 4 subcircuits, 8 cuts, M = 2^20): recursions that
  expand the top bin down to single states, with sampled bins of every
  recursion against the oracle's merged entries contracted bin by bin, child
  bins summing to the parent bin, FP32 MFMA and split-BF16x3 against the FP64
  GPU path on every bin; and
  Algorithm 1 on the device with R = 12 (twelve recursions, each summing to the
  bin it expands, FP32 expanding the same bins as FP64).
- large (200 qubits, 16 subcircuits, 24 cuts, M = 2^24): two recursions,
  sampled bins against the oracle's pairwise contraction, child sum = parent,
  split-BF16x3 against the FP64 GPU path.
"""
import numpy as np
import pytest

from oracle import network, reconstruction as rc, states_merging as sm
from workloads import configs, qpu

from gpu_util import TOL_REL, assert_bound, error_bound, oracle_attributed, sampled_bound, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sqc = pytest.importorskip("paper_2207_00933_amd.sqc")
runner = pytest.importorskip("paper_2207_00933_amd.runner")

TOL = {sqc.F64: 1e-12, sqc.F32: 1e-6, sqc.BF16X3: 1e-6}


@pytest.fixture(scope="module")
def session():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = runner.Session(0, 64 << 20)
    yield s
    s.close()


@pytest.mark.timeout(900)
def test_precision_full_reconstruction_sampled(session):
    cc = configs.precision()
    var32 = [v.astype(np.float32) for v in qpu.all_variants(cc)]
    Th = oracle_attributed(cc, [v.astype(np.float64) for v in var32])
    rng = np.random.default_rng(2)
    sample = np.unique(rng.integers(0, 1 << cc.n, size=4096))
    want = network.eval_bins(Th, cc, sample)
    bound = sampled_bound(Th, cc, sample)
    bound_all = error_bound(Th, cc)  # whole output, for the path-to-path check
    circ = runner.Circuit.from_cut_circuit(session, cc, var32, sqc.F32)
    ref64 = None
    for pname, prec in (("f64", sqc.F64), ("f32", sqc.F32), ("bf16x3", sqc.BF16X3)):
        att = sqc.F64 if prec == sqc.F64 else sqc.F32
        bins_prec = sqc.F64 if prec == sqc.F64 else sqc.F32
        say(f"precision full {pname}")
        circ.attribute(att)
        rec = runner.Recursion(circ, cc.n, bins_prec, 16)
        rec.run(prec, 1 << cc.n)
        torch.cuda.synchronize()
        bins = rec.bins.double().cpu().numpy()
        assert_bound(bins[sample], want, bound, prec, prec != sqc.F64, f"{pname} vs oracle, sampled")
        if prec == sqc.F64:
            ref64 = bins
        else:
            # every bin against the FP64 GPU path: the fast path's bound plus
            # the FP64 path's own
            tol = (TOL_REL[prec] + TOL_REL[sqc.F64]) * bound_all + 2.0 ** -24 * np.abs(ref64) + 1e-300
            err = np.abs(bins - ref64)
            bad = np.flatnonzero(~(err <= tol))
            say(f"  {pname} vs FP64 GPU, all {len(bins)} bins: max-abs {err.max():.3e}, "
                f"max err / tol {(err / tol).max():.3f}")
            assert len(bad) == 0, (bad[:8], err[bad[:8]], tol[bad[:8]])
        assert abs(rec.sum.item() - 1.0) <= 1e-6
        vals, idx = rec.top_list()
        assert np.all(np.diff(vals) <= 0)
        assert np.array_equal(vals, bins[idx.astype(np.int64)])
        assert vals[-1] >= np.sort(bins)[-16]
        del rec


def _merged_oracle(Th, cc, lit):
    return [rc.merge_entries(Th[i], lit[i]) for i in range(cc.n_sub)]


def _run_recursions(session, cc, circ, Th, M, n_rec, precs, n_sample, seed, full_bound=True):
    """Recursions expanding the top bin of the FP64 GPU path; every precision
    follows the same bins.  Returns per precision the list of bin vectors
    (and under "bound" the oracle's |T| contraction of every bin)."""
    d = [s.n_data for s in cc.subs]
    rng = np.random.default_rng(seed)
    out = {p: [] for p in precs}
    out["bound"] = []
    scope, lit_states, parent = None, None, None
    for r in range(n_rec):
        lit = sm.assign_states(r, lit_states, M, d)
        counts = [len(b) for b in lit]
        nb = int(np.prod(counts))
        Tm = _merged_oracle(Th, cc, lit)
        sample = np.unique(rng.integers(0, nb, size=n_sample))
        want = network.eval_bins(Tm, cc, sample)
        # rounding scale of a merged bin: the attributed entries are stored in
        # the path's precision before merging, so the bound contracts the
        # merged |T| (not |merged T|)
        absm = [np.abs(T) for T in Th]
        Tabs = _merged_oracle(absm, cc, lit)
        bound = network.eval_bins(Tabs, cc, sample)
        if full_bound:
            out["bound"].append(network.contract_all(Tabs, cc))
        pick = None
        for p in precs:
            att = sqc.F64 if p == sqc.F64 else sqc.F32
            if circ.att and circ.att[0].prec != att or not circ.att:
                circ.attribute(att)
            say(f"recursion r={r} prec={p} bins={nb}")
            rec = runner.Recursion(circ, int(np.log2(M)), sqc.F64, 12)
            masks = rec.run(p, M, scope)
            torch.cuda.synchronize()
            got = rec.bins.cpu().numpy()[:nb]
            assert_bound(got[sample], want, bound, p, False, f"r={r} prec={p} vs oracle, sampled")
            if parent is not None:
                # child bins sum to the parent bin (linearity, any data)
                assert abs(got.sum() - parent) <= max(1e-12, TOL[p] * 10)
                assert abs(rec.sum.item() - got.sum()) <= 1e-12 + 1e-12 * abs(got).sum()
            out[p].append(got)
            if p == sqc.F64:
                pick = int(np.argmax(got))
                pick_masks = masks
            del rec
        ks = sm.split_index(pick, counts)
        lit_states = [lit[i][ks[i]] for i in range(cc.n_sub)]
        parent = float(out[sqc.F64][-1][pick])
        scope = sqc.bin_scope(pick_masks, pick)
        if all(len(b) == 1 for b in lit_states):
            break
    return out


@pytest.mark.timeout(1200)
def test_merging_twelve_recursions(session):
    cc = configs.merging()
    var = qpu.all_variants(cc)
    say("merging: oracle entries")
    Th = oracle_attributed(cc, var)
    circ = runner.Circuit.from_cut_circuit(session, cc, var, sqc.F64)
    out = _run_recursions(session, cc, circ, Th, 1 << 20, 12, [sqc.F64, sqc.F32, sqc.BF16X3], 256, seed=3)
    for p in (sqc.F32, sqc.BF16X3):
        for g64, gp, bnd in zip(out[sqc.F64], out[p], out["bound"]):
            tol = (TOL_REL[p] + TOL_REL[sqc.F64]) * bnd + 1e-300
            err = np.abs(g64 - gp)
            say(f"  prec={p} vs FP64 GPU, all bins: max-abs {err.max():.3e}, max err / tol {(err / tol).max():.3f}")
            assert np.all(err <= tol)
            assert err.max() <= 1e-6
    assert len(out[sqc.F64]) >= 3


@pytest.mark.timeout(1200)
def test_large_chain_two_recursions(session):
    cc = configs.large()
    var = qpu.all_variants(cc)
    say("large: oracle entries")
    Th = oracle_attributed(cc, var)
    circ = runner.Circuit.from_cut_circuit(session, cc, var, sqc.F64)
    out = _run_recursions(session, cc, circ, Th, 1 << 24, 2, [sqc.F64, sqc.BF16X3], 128, seed=5)
    for g64, gb, bnd in zip(out[sqc.F64], out[sqc.BF16X3], out["bound"]):
        tol = (TOL_REL[sqc.BF16X3] + TOL_REL[sqc.F64]) * bnd + 1e-300
        err = np.abs(g64 - gb)
        say(f"  bf16x3 vs fp64 GPU, all bins: max-abs {err.max():.3e}, max err / tol {(err / tol).max():.3f}")
        assert np.all(err <= tol)
        assert err.max() <= 1e-6


@pytest.mark.timeout(900)
def test_merging_search_twelve_recursions(session):
    """Algorithm 1 on the device with R = 12 and M = 2^20: twelve recursions,
    each one's bins summing to the bin it expands; the FP32 MFMA search expands
    the same bins as the FP64 one, to tolerance."""
    cc = configs.merging()
    var = qpu.all_variants(cc)
    circ = runner.Circuit.from_cut_circuit(session, cc, var, sqc.F64)
    M = 1 << 20
    infos = {}
    for pname, prec in (("f64", sqc.F64), ("f32", sqc.F32)):
        circ.attribute(sqc.F64 if prec == sqc.F64 else sqc.F32)
        bins = torch.empty(M, dtype=torch.float64, device="cuda")
        masks = sqc.assign_bins(circ.g.n_data, None, M)
        session.ensure_workspace(4 * sqc.recurse_workspace_bytes(circ.att, circ.g, masks, prec))
        say(f"merging search {pname}")
        sols, inf = sqc.search(session.ctx, circ.att, circ.g, M, 12, prec, bins, sqc.F64)
        torch.cuda.synchronize()
        infos[prec] = inf
        assert len(inf) == 12
        for r, (bsum, parent, top, a, leaf) in enumerate(inf):
            assert abs(bsum - parent) <= (1e-12 if prec == sqc.F64 else 1e-6), (r, bsum, parent)
            assert top <= parent + 1e-12
    for a, b in zip(infos[sqc.F64], infos[sqc.F32]):
        assert abs(a[1] - b[1]) <= 1e-6 and abs(a[2] - b[2]) <= 1e-6 and a[3] == b[3]
