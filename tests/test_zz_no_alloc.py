"""The allocation-free recursion (sqc_recurse_noalloc: workspace in a device
array inside the library) against sqc_recurse with a caller workspace: the
same kernels and launch shapes, so the bins, top-R list and bin sum must be
bitwise equal, and within the path's bound of the oracle.  Two calls in a
row share the device array: the 24-qubit precision workload (2^24 bins),
then the smaller 10-qubit circuit; then a recursion whose workspace exceeds
the array is refused with nothing enqueued."""
import numpy as np
import pytest

from oracle import network
from workloads import configs, qpu

from gpu_util import assert_bound, error_bound, oracle_attributed, sampled_bound, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sqc = pytest.importorskip("paper_2207_00933_amd.sqc")
runner = pytest.importorskip("paper_2207_00933_amd.runner")


def _pair(session, cc, var, var_prec, prec, bins_prec, top_r):
    att = sqc.F64 if prec == sqc.F64 else sqc.F32
    circ = runner.Circuit.from_cut_circuit(session, cc, var, var_prec)
    circ.attribute(att)
    dt = torch.float64 if bins_prec == sqc.F64 else torch.float32
    n = 1 << cc.n
    rec = runner.Recursion(circ, cc.n, bins_prec, top_r)
    rec.bins.fill_(float("nan"))
    masks_a = rec.run(prec, n)
    bins_b = torch.full((n,), float("nan"), dtype=dt, device="cuda")
    top_b = torch.empty(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda")
    sum_b = torch.empty(1, dtype=torch.float64, device="cuda")
    masks_b = sqc.recurse_noalloc(session.ctx, circ.att, circ.g, None, n, top_r, prec, bins_b, bins_prec,
                                  top_b, sum_b)
    torch.cuda.synchronize()
    assert [m.as_tuple() for m in masks_a] == [m.as_tuple() for m in masks_b]
    assert torch.equal(rec.bins[:n], bins_b), "bins differ"
    assert torch.equal(rec.top[: 2 * top_r], top_b[: 2 * top_r]), "top-R differs"
    assert torch.equal(rec.sum, sum_b), "bin sum differs"
    return bins_b.double().cpu().numpy()


@pytest.fixture(scope="module")
def session():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = runner.Session(0, 64 << 20)
    yield s
    s.close()


def test_noalloc_equals_recurse_twice(session):
    # first call: the 24-qubit precision workload, FP32-cast outputs
    cc = configs.precision()
    var32 = [v.astype(np.float32) for v in qpu.all_variants(cc)]
    Th = oracle_attributed(cc, [v.astype(np.float64) for v in var32])
    rng = np.random.default_rng(7)
    sample = np.unique(rng.integers(0, 1 << cc.n, size=1024))
    want = network.eval_bins(Th, cc, sample)
    bound = sampled_bound(Th, cc, sample)
    for pname, prec, bp in (("bf16x3", sqc.BF16X3, sqc.F32), ("f64", sqc.F64, sqc.F64)):
        say(f"noalloc precision workload {pname}")
        got = _pair(session, cc, var32, sqc.F32, prec, bp, 16)
        assert_bound(got[sample], want, bound, prec, bp == sqc.F32, f"noalloc precision {pname}")
    # second call, a smaller input in the same device array
    cc = configs.tiny()
    var = qpu.all_variants(cc)
    Th = oracle_attributed(cc, var)
    want = network.contract_all(Th, cc)
    bound = error_bound(Th, cc)
    for pname, prec, bp in (("bf16x3", sqc.BF16X3, sqc.F32), ("f64", sqc.F64, sqc.F64)):
        say(f"noalloc tiny {pname}")
        got = _pair(session, cc, var, sqc.F64, prec, bp, 4)
        assert_bound(got, want, bound, prec, bp == sqc.F32, f"noalloc tiny {pname}")


def test_noalloc_refuses_oversize(session):
    """A chain of three subcircuits with 10, 8 and 10 data bits and 3 + 3
    cuts at M = 2^26 on the FP64 path needs 73 MiB of workspace: refused,
    nothing enqueued (the outputs keep their zeros)."""
    bits, deg = [10, 8, 10], [3, 6, 3]
    cuts = [(0, 1)] * 3 + [(1, 2)] * 3
    g = sqc.Graph([1] * 3, [[0] * b for b in bits], [(u, 0, v, 0) for u, v in cuts])
    rng = np.random.default_rng(9)
    bufs = [torch.from_numpy(rng.standard_normal((1 << bits[i], 4 ** deg[i]))).cuda() for i in range(3)]
    att = [sqc.tensor_desc(b, deg[i], bits[i], sqc.F64, sqc.LAYOUT_ATTRIBUTED) for i, b in enumerate(bufs)]
    M = 1 << 26
    masks = sqc.assign_bins(bits, None, M)
    need = sqc.recurse_workspace_bytes(att, g, masks, sqc.F64)
    say(f"chain [10, 8, 10] FP64 recursion at M = 2^26 needs {need} bytes")
    assert need > sqc.NOALLOC_SCRATCH_BYTES
    bins = torch.zeros(M, dtype=torch.float64, device="cuda")
    top = torch.zeros(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda")
    bsum = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(sqc.SqcError) as e:
        sqc.recurse_noalloc(session.ctx, att, g, None, M, 4, sqc.F64, bins, sqc.F64, top, bsum)
    assert e.value.status == sqc.E_NOMEM
    assert "allocation-free" in str(e.value)
    torch.cuda.synchronize()
    assert float(bins.abs().max()) == 0.0 and float(bsum.abs().max()) == 0.0
    assert float(top.abs().max()) == 0.0
