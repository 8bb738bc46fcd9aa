"""Launch autotuner: tuning changes launch choices only.  After tuning, the
recursion's bins and top-R are bitwise those of the untuned run (tile order and
work-group count do not change any bin), the bin sum agrees to rounding (the
work-group count changes how the sum is split), and a reset restores the
untuned bits exactly."""
import numpy as np
import pytest

from workloads import configs, qpu

from gpu_util import say

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
    sqc.autotune_reset()
    s.close()


def run(session, circ, prec, M, scope=None):
    rec = runner.Recursion(circ, int(np.log2(M)), sqc.F32 if prec != sqc.F64 else sqc.F64, 16)
    rec.run(prec, M, scope)
    torch.cuda.synchronize()
    return rec.bins.clone(), rec.top.clone(), rec.sum.item()


@pytest.mark.parametrize("name,prec", [("precision", sqc.BF16X3), ("precision", sqc.F64),
                                       ("merging", sqc.F32)])
def test_tuning_changes_no_bin(session, name, prec):
    cc = configs.precision() if name == "precision" else configs.merging()
    var = qpu.all_variants(cc)
    circ = runner.Circuit.from_cut_circuit(session, cc, var, sqc.F64)
    circ.attribute(sqc.F64 if prec == sqc.F64 else sqc.F32)
    M = 1 << (cc.n if name == "precision" else 20)
    sqc.autotune_reset()
    b0, t0, s0 = run(session, circ, prec, M)
    masks = sqc.assign_bins(circ.g.n_data, None, M)
    session.ensure_workspace(sqc.recurse_workspace_bytes(circ.att, circ.g, masks, prec))
    bins = torch.empty_like(b0)
    rep = sqc.autotune(session.ctx, circ.att, circ.g, None, M, prec, bins,
                       sqc.F32 if prec != sqc.F64 else sqc.F64, reps=3)
    torch.cuda.synchronize()
    say(f"autotune {name} prec={prec}: {rep.steps} steps, {rep.candidates} candidates, "
        f"default {rep.default_us:.1f} us -> tuned {rep.tuned_us:.1f} us")
    assert rep.steps >= 1 and rep.candidates >= rep.steps
    assert rep.tuned_us <= rep.default_us + 1e-9
    assert sqc.autotune_entries() >= rep.steps
    assert torch.equal(bins, b0)  # the tuner's last run leaves the bins
    b1, t1, s1 = run(session, circ, prec, M)
    assert torch.equal(b1, b0)
    k = 2 * 16
    assert torch.equal(t1[:k].view(torch.int64), t0[:k].view(torch.int64))
    assert abs(s1 - s0) <= 1e-14 * max(1.0, abs(s0))
    sqc.autotune_reset()
    assert sqc.autotune_entries() == 0
    b2, t2, s2 = run(session, circ, prec, M)
    assert torch.equal(b2, b0) and s2 == s0


def test_tile_shapes_of_short_contractions(session):
    """The 200-qubit chain (16 subcircuits, every step contracts at most 16
    labels): the tuner times both tile shapes (K staged 64 deep, and the
    narrow 16-deep tile) for every step, records the choice per step, and the
    choice changes no bin (the MFMA steps and their operands are the same)."""
    cc = configs.large()
    var = qpu.all_variants(cc)
    circ = runner.Circuit.from_cut_circuit(session, cc, var, sqc.F64)
    circ.attribute(sqc.F32)
    M = 1 << 20
    sqc.autotune_reset()
    b0, t0, s0 = run(session, circ, sqc.BF16X3, M)
    masks = sqc.assign_bins(circ.g.n_data, None, M)
    session.ensure_workspace(sqc.recurse_workspace_bytes(circ.att, circ.g, masks, sqc.BF16X3))
    bins = torch.empty_like(b0)
    rep = sqc.autotune(session.ctx, circ.att, circ.g, None, M, sqc.BF16X3, bins, sqc.F32, reps=3)
    torch.cuda.synchronize()
    tiles = [rep.step_tile[i] for i in range(rep.steps)]
    say(f"autotune large: {rep.steps} steps, {rep.candidates} candidates, default {rep.default_us:.1f} us "
        f"-> tuned {rep.tuned_us:.1f} us; 16-deep tile chosen for {sum(tiles)} of {rep.steps} steps")
    assert rep.steps == 15 and all(t in (0, 1) for t in tiles)
    assert all(rep.step_groups[i] >= 1 for i in range(rep.steps))
    assert rep.candidates >= 2 * rep.steps  # both shapes timed for every step
    assert rep.tuned_us <= rep.default_us + 1e-9
    b1, t1, s1 = run(session, circ, sqc.BF16X3, M)
    assert torch.equal(b1, b0) and torch.equal(bins, b0)
    assert torch.equal(t1[:32].view(torch.int64), t0[:32].view(torch.int64))
    assert abs(s1 - s0) <= 1e-14 * max(1.0, abs(s0))
    sqc.autotune_reset()
