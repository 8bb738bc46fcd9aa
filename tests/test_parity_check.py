"""The per-bin bound that the full-size GPU parity tests apply can fail: on
the 24-qubit precision workload, a correct result (the oracle's own values at
the sampled bins) passes it on every path, while two swapped bins, or bins
taken from their neighbour inside a 32 x 32 output tile, fail it on every
path, although they stay within the 1e-6 absolute tolerance (bins here are
about 6e-8)."""
import numpy as np
import pytest

from oracle import network
from workloads import configs, qpu

from gpu_util import TOL_ABS, bound_violations, oracle_attributed, sampled_bound


@pytest.fixture(scope="module")
def precision_sample():
    cc = configs.precision()
    var32 = [v.astype(np.float32).astype(np.float64) for v in qpu.all_variants(cc)]
    Th = oracle_attributed(cc, var32)
    rng = np.random.default_rng(2)
    sample = np.unique(rng.integers(0, 1 << cc.n, size=4096))
    want = network.eval_bins(Th, cc, sample)
    bound = sampled_bound(Th, cc, sample)
    return cc, Th, sample, want, bound


@pytest.mark.parametrize("prec,bins_f32", [(0, False), (1, True), (2, True)])
def test_correct_result_passes(precision_sample, prec, bins_f32):
    _, _, _, want, bound = precision_sample
    got = want.astype(np.float32).astype(np.float64) if bins_f32 else want.copy()
    assert len(bound_violations(got, want, bound, prec, bins_f32)) == 0


@pytest.mark.parametrize("prec,bins_f32", [(0, False), (1, True), (2, True)])
def test_swapped_bins_fail(precision_sample, prec, bins_f32):
    _, _, _, want, bound = precision_sample
    got = want.copy()
    # two sampled bins whose values differ by a typical amount
    i, j = 10, 11
    assert abs(want[i] - want[j]) > 1e-9
    got[i], got[j] = want[j], want[i]
    assert np.abs(got - want).max() < TOL_ABS[prec] or prec == 0
    bad = bound_violations(got, want, bound, prec, bins_f32)
    assert set(bad.tolist()) == {i, j}


@pytest.mark.parametrize("prec,bins_f32", [(1, True), (2, True)])
def test_within_tile_permutation_fails(precision_sample, prec, bins_f32):
    """Each sampled bin replaced by its neighbour along the contiguous output
    axis (index XOR 1, the same tile row): the kind of mistake a wrong lane
    or row offset in a tile's staging or store would make."""
    cc, Th, sample, want, bound = precision_sample
    got = network.eval_bins(Th, cc, sample ^ 1)
    assert np.abs(got - want).max() < TOL_ABS[prec]
    bad = bound_violations(got, want, bound, prec, bins_f32)
    assert len(bad) > 0.9 * len(sample)
