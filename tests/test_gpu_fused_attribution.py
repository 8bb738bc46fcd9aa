"""Attribution written straight in the merged layout (sqc_attribute_all_merged)
and recursions that read such tensors in place.

The merged tensor of a recursion that keeps every data bit active holds the
attributed entries transposed ([4^c][2^d]); its values must be bitwise those
that sqc_attribute_all followed by sqc_merge stores (both take the same FP64
value to the same storage type), for every circuit and precision pair.  A
recursion that reads them in place must give bitwise the bins, top-R and sum
of the same recursion on attributed tensors, also when only some
subcircuits keep every data bit (the others are merged as usual).  Inputs
that do not fit (bits merged or fixed, another precision, SQC_AUTO) are
refused before anything is enqueued."""
import numpy as np
import pytest

from workloads import configs, qpu
from workloads.circuits import planted_qaoa
from workloads.cutgraph import build_cut_circuit

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
    s.close()


def _circuits():
    return {
        "tiny": configs.tiny(),
        "chain3": configs.chain_brickwork(3, [4, 5, 4], [1, 2], 4, 11),
        "chain4": configs.chain_brickwork(4, [3, 4, 3, 4], [2, 1, 1], 4, 12),
        "qaoa3": build_cut_circuit(planted_qaoa([4, 4, 4], seed=5)),
        "precision": configs.precision(),
    }


def _bits(t):
    return torch.empty((4 ** t.n_labels) << t.n_bits, dtype=torch.float64 if t.prec == sqc.F64 else torch.float32,
                       device="cuda")


@pytest.mark.parametrize("name", ["tiny", "chain3", "chain4", "qaoa3", "precision"])
@pytest.mark.parametrize("in_prec,out_prec", [(sqc.F64, sqc.F64), (sqc.F32, sqc.F32), (sqc.F64, sqc.F32)])
def test_merged_attribution_equals_attribute_then_merge(session, name, in_prec, out_prec):
    cc = _circuits()[name]
    var = qpu.all_variants(cc)
    if in_prec == sqc.F32:
        var = [v.astype(np.float32) for v in var]
    circ = runner.Circuit.from_cut_circuit(session, cc, var, in_prec)
    att = circ.attribute(out_prec)
    masks = sqc.assign_bins(circ.g.n_data, None, 1 << sum(circ.g.n_data))
    want = []
    for i in range(cc.n_sub):
        buf = _bits(att[i])
        session.ensure_workspace(sqc.merge_workspace_bytes(att[i], masks[i]))
        sqc.merge(session.ctx, att[i], masks[i], buf, out_prec)
        want.append(buf)
    bufs = [_bits(att[i]) for i in range(cc.n_sub)]
    got = sqc.attribute_all_merged(session.ctx, circ.g, circ.var, circ.var_prec, bufs, out_prec)
    torch.cuda.synchronize()
    for i in range(cc.n_sub):
        assert got[i].layout == sqc.LAYOUT_MERGED
        assert (got[i].n_labels, got[i].n_bits) == (att[i].n_labels, att[i].n_bits)
        assert torch.equal(bufs[i], want[i]), f"subcircuit {i}"
    say(f"merged attribution {name} in {in_prec} out {out_prec}: bitwise equal, {cc.n_sub} subcircuits")


def _recurse(session, circ, att, M, prec, top_r=16):
    g = circ.g
    bprec = sqc.F64 if prec == sqc.F64 else sqc.F32
    masks = sqc.assign_bins(g.n_data, None, M)
    session.ensure_workspace(sqc.recurse_workspace_bytes(att, g, masks, prec))
    a = sum(bin(m.active).count("1") for m in masks)
    bins = torch.full((1 << a,), -1.0, dtype=torch.float64 if bprec == sqc.F64 else torch.float32, device="cuda")
    top = torch.empty(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda")
    bsum = torch.empty(1, dtype=torch.float64, device="cuda")
    sqc.recurse(session.ctx, att, g, None, M, top_r, prec, bins, bprec, top, bsum)
    torch.cuda.synchronize()
    return bins, top[: 2 * top_r].clone(), bsum.clone(), masks


@pytest.mark.parametrize("name", ["chain4", "qaoa3", "precision"])
@pytest.mark.parametrize("pname,prec", [("f64", sqc.F64), ("f32", sqc.F32), ("bf16x3", sqc.BF16X3)])
def test_recursion_reads_merged_inputs_in_place(session, name, pname, prec):
    cc = _circuits()[name]
    var = [v.astype(np.float32) for v in qpu.all_variants(cc)]
    circ = runner.Circuit.from_cut_circuit(session, cc, var, sqc.F32)
    op = sqc.F64 if prec == sqc.F64 else sqc.F32
    M = 1 << cc.n
    ref = _recurse(session, circ, circ.attribute(op), M, prec)
    got = _recurse(session, circ, circ.attribute(op, merged=True), M, prec)
    for what, x, y in zip(("bins", "top-R", "sum"), ref[:3], got[:3]):
        assert torch.equal(x, y), what
    say(f"recursion {name} {pname}: merged-layout inputs bitwise equal to attributed ones")


def test_recursion_mixes_merged_and_attributed_inputs(session):
    """M = 2^23 on the 24-qubit workload: Algorithm 2 halves subcircuit 0's
    bins (one of its bits merged) and keeps every bit of subcircuits 1 and 2,
    which are then given in the merged layout."""
    cc = configs.precision()
    var = [v.astype(np.float32) for v in qpu.all_variants(cc)]
    circ = runner.Circuit.from_cut_circuit(session, cc, var, sqc.F32)
    M = 1 << (cc.n - 1)
    masks = sqc.assign_bins(circ.g.n_data, None, M)
    full = [m.merged == 0 and m.fixed == 0 for m in masks]
    assert full == [False, True, True], [m.as_tuple() for m in masks]
    att = circ.attribute(sqc.F32)
    ref = _recurse(session, circ, att, M, sqc.BF16X3)
    bufs = [_bits(att[i]) for i in range(cc.n_sub)]
    merged = sqc.attribute_all_merged(session.ctx, circ.g, circ.var, circ.var_prec, bufs, sqc.F32)
    mixed = [att[0], merged[1], merged[2]]
    got = _recurse(session, circ, mixed, M, sqc.BF16X3)
    for what, x, y in zip(("bins", "top-R", "sum"), ref[:3], got[:3]):
        assert torch.equal(x, y), what


def test_merged_inputs_that_do_not_fit_are_refused(session):
    cc = configs.precision()
    var = [v.astype(np.float32) for v in qpu.all_variants(cc)]
    circ = runner.Circuit.from_cut_circuit(session, cc, var, sqc.F32)
    g = circ.g
    merged = circ.attribute(sqc.F32, merged=True)
    bins = torch.zeros(1 << cc.n, dtype=torch.float64, device="cuda")
    top = torch.empty(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda")
    bsum = torch.empty(1, dtype=torch.float64, device="cuda")
    session.ensure_workspace(64 << 20)
    cases = [
        ("a recursion that merges bits", 1 << (cc.n - 1), sqc.BF16X3, sqc.E_ARG),
        ("FP32 merged inputs on the FP64 path", 1 << cc.n, sqc.F64, sqc.E_ARG),
        ("precision selection", 1 << cc.n, sqc.AUTO, sqc.E_ARG),
    ]
    for what, M, prec, status in cases:
        with pytest.raises(sqc.SqcError) as e:
            sqc.recurse(session.ctx, merged, g, None, M, 4, prec, bins, sqc.F64, top, bsum)
        assert e.value.status == status, what
    torch.cuda.synchronize()
    assert float(bins.abs().max()) == 0.0  # nothing was enqueued
    # a merged tensor is not an attributed one
    out = torch.empty(4 ** merged[0].n_labels << merged[0].n_bits, dtype=torch.float32, device="cuda")
    m0 = sqc.assign_bins(g.n_data, None, 1 << cc.n)[0]
    with pytest.raises(sqc.SqcError) as e:
        sqc.merge(session.ctx, merged[0], m0, out, sqc.F32)
    assert e.value.status == sqc.E_SHAPE
