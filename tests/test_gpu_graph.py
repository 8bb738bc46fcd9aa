"""HIP graph recording of the hot path: a recorded attribution + recursion is
replayed several times, with other eager work on the same stream between the
replays, and every replay's bins, top-R and sum are bitwise those of the eager
run (the recorded work has no memset nodes)."""
import numpy as np
import pytest

from workloads import configs, qpu

from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sqc = pytest.importorskip("paper_2207_00933_amd.sqc")
runner = pytest.importorskip("paper_2207_00933_amd.runner")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = runner.Session(0, 64 << 20)
    sqc.ctx_set_stream(s.ctx, st.cuda_stream)
    yield s, st
    st.synchronize()
    s.close()


def snapshot(rec, nb):
    return rec.bins[:nb].clone(), rec.top.clone(), rec.sum.clone()


def same(a, b, top_r):
    return (torch.equal(a[0], b[0]) and torch.equal(a[2], b[2]) and
            torch.equal(a[1][:2 * top_r].view(torch.int64), b[1][:2 * top_r].view(torch.int64)))


@pytest.mark.parametrize("name,prec", [("precision", sqc.BF16X3), ("precision", sqc.F64),
                                       ("tiny", sqc.F32)])
def test_graph_replays_match_eager(env, name, prec):
    s, st = env
    cc = configs.precision() if name == "precision" else configs.tiny()
    var = qpu.all_variants(cc)
    att_prec = sqc.F64 if prec == sqc.F64 else sqc.F32
    bprec = att_prec
    with torch.cuda.stream(st):
        circ = runner.Circuit.from_cut_circuit(s, cc, [v.astype(np.float32) for v in var], sqc.F32)
        M = 1 << cc.n
        rec = runner.Recursion(circ, cc.n, bprec, 16)
        other = runner.Recursion(circ, cc.n, bprec, 8)
        # eager reference (also sizes the workspace before recording)
        circ.attribute(att_prec)
        rec.run(prec, M)
        st.synchronize()
        want = snapshot(rec, M)
        other.run(prec, M >> 3)
        st.synchronize()
        want_other = snapshot(other, M >> 3)
        sqc.graph_begin(s.ctx)
        with pytest.raises(sqc.SqcError):
            sqc.ctx_timing(s.ctx, sqc.STAGE_FINAL)
        circ.attribute(att_prec)
        rec.run(prec, M)
        g = sqc.graph_end(s.ctx)
        try:
            for k in range(4):
                rec.bins.fill_(float("nan"))
                rec.top.fill_(7.0)
                rec.sum.fill_(9.0)
                sqc.graph_launch(s.ctx, g)
                st.synchronize()
                got = snapshot(rec, M)
                say(f"graph {name} prec={prec} replay {k}: equal={same(got, want, 16)}")
                assert same(got, want, 16), k
                # eager work between replays on the same stream
                other.bins.fill_(float("nan"))
                other.run(prec, M >> 3)
                st.synchronize()
                assert same(snapshot(other, M >> 3), want_other, 8), k
        finally:
            sqc.graph_destroy(g)


def test_graph_needs_created_stream():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = runner.Session(0, 1 << 20)
    sqc.ctx_set_stream(s.ctx, None)
    with pytest.raises(sqc.SqcError) as e:
        sqc.graph_begin(s.ctx)
    assert e.value.status == sqc.E_ARG
    s.close()
