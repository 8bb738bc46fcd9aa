"""Serving engine: results of requests run through the engine, in a burst, in
a stream of arrivals and under a workspace too small to hold them all, are
bitwise the same as the same recursions run alone through sqc_recurse (the
alone-versus-mix race test).  Recursion-0 requests of the small circuits are
also checked against the oracle's reconstruction, and admission limits are
checked (footprint larger than the workspace, queueing, overlap)."""
import math

import numpy as np
import pytest

from oracle import network, reconstruction as rc
from workloads import configs, qpu
from workloads.circuits import planted_qaoa
from workloads.cutgraph import build_cut_circuit

from gpu_util import bins_from_masks, oracle_attributed, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sqc = pytest.importorskip("paper_2207_00933_amd.sqc")
runner = pytest.importorskip("paper_2207_00933_amd.runner")

TOL = {sqc.F64: 1e-12, sqc.F32: 1e-6, sqc.BF16X3: 1e-6}


def circuits():
    pool = configs.serving_pool(count=8)
    return {
        "tiny": configs.tiny(),
        "chain3": configs.chain_brickwork(3, [4, 5, 4], [1, 2], 4, 11),
        "qaoa3": build_cut_circuit(planted_qaoa([4, 4, 4], seed=5)),
        "pool7": pool[7],
        "pool5": pool[5],
    }


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = runner.Session(0, 64 << 20)
    ccs = circuits()
    circ = {}
    for name, cc in ccs.items():
        var = qpu.all_variants(cc)
        c64 = runner.Circuit.from_cut_circuit(s, cc, var, sqc.F64)
        c64.attribute(sqc.F64)
        c32 = runner.Circuit.from_cut_circuit(s, cc, var, sqc.F64)
        c32.attribute(sqc.F32)
        circ[name] = (cc, var, {sqc.F64: c64, sqc.F32: c32})
    torch.cuda.synchronize()
    yield s, circ
    s.close()


def request_list(circ, seed, n):
    """Seeded mixed requests: circuit, M, precision, top_r, and a scope taken
    from a bin of a recursion-0 bin assignment (a recursion step) or none."""
    rng = np.random.default_rng(seed)
    names = sorted(circ)
    precs = [sqc.F64, sqc.F32, sqc.BF16X3]
    out = []
    for _ in range(n):
        name = names[int(rng.integers(len(names)))]
        cc = circ[name][0]
        nd = [s.n_data for s in cc.subs]
        a = int(rng.integers(2, min(14, sum(nd)) + 1))
        prec = precs[int(rng.integers(3))]
        top_r = int(rng.integers(1, sqc.MAX_TOPR + 1))
        scope = None
        if rng.random() < 0.4:
            m0 = sqc.assign_bins(nd, None, 1 << int(rng.integers(1, 6)))
            nb = 1 << sum(bin(m.active).count("1") for m in m0)
            scope = sqc.bin_scope(m0, int(rng.integers(nb)))
        out.append((name, a, prec, top_r, scope))
    return out


def buffers(circ, req):
    name, a, prec, top_r, scope = req
    cc = circ[name][0]
    masks = sqc.assign_bins([s.n_data for s in cc.subs], scope, 1 << a)
    nb = 1 << sum(bin(m.active).count("1") for m in masks)
    bprec = sqc.F64 if prec == sqc.F64 else sqc.F32
    dt = torch.float64 if bprec == sqc.F64 else torch.float32
    bins = torch.full((nb,), float("nan"), dtype=dt, device="cuda")
    top = torch.full((2 * sqc.MAX_TOPR,), 3.0, dtype=torch.float64, device="cuda")
    bsum = torch.full((1,), 5.0, dtype=torch.float64, device="cuda")
    return masks, bprec, bins, top, bsum


def run_alone(s, circ, reqs):
    """Each request through sqc_recurse on the session's stream, one by one."""
    res = []
    for req in reqs:
        name, a, prec, top_r, scope = req
        c = circ[name][2][sqc.F64 if prec == sqc.F64 else sqc.F32]
        masks, bprec, bins, top, bsum = buffers(circ, req)
        s.ensure_workspace(sqc.recurse_workspace_bytes(c.att, c.g, masks, prec))
        got = sqc.recurse(s.ctx, c.att, c.g, scope, 1 << a, top_r, prec, bins, bprec, top, bsum)
        assert [m.as_tuple() for m in got] == [m.as_tuple() for m in masks]
        torch.cuda.synchronize()
        res.append((bins.cpu(), top.cpu(), bsum.cpu()))
    return res


def make_server_requests(srv, ids, circ, reqs):
    out = []
    for req in reqs:
        name, a, prec, top_r, scope = req
        masks, bprec, bins, top, bsum = buffers(circ, req)
        r = srv.request(ids[(name, prec)], scope, 1 << a, top_r, prec, bins, bprec, top, bsum,
                        masks_out=True)
        out.append((r, masks, bins, top, bsum))
    # the buffers were filled on torch's stream; the engine's streams do not
    # wait for it
    torch.cuda.synchronize()
    return out


def register_all(srv, circ):
    ids = {}
    for name, (_, _, cs) in circ.items():
        for prec in (sqc.F64, sqc.F32, sqc.BF16X3):
            ids[(name, prec)] = srv.register(cs[sqc.F64 if prec == sqc.F64 else sqc.F32])
    return ids


def check_same(alone, served, reqs):
    for k, ((b0, t0, s0), (r, masks, bins, top, bsum)) in enumerate(zip(alone, served, )):
        name, a, prec, top_r, scope = reqs[k]
        assert [m.as_tuple() for m in r._masks] == [m.as_tuple() for m in masks], k
        assert torch.equal(bins.cpu(), b0), (k, reqs[k][:4])
        # records past the bin count hold index ~0, a NaN as a double: compare bits
        assert torch.equal(top.cpu()[:2 * top_r].view(torch.int64),
                           t0[:2 * top_r].view(torch.int64)), (k, reqs[k][:4])
        assert torch.equal(bsum.cpu(), s0), (k, reqs[k][:4])


def test_alone_equals_burst(setup):
    s, circ = setup
    reqs = request_list(circ, 7, 48)
    say("serve burst: alone pass")
    alone = run_alone(s, circ, reqs)
    srv = runner.Server(0, n_slots=4, workspace_bytes=512 << 20)
    ids = register_all(srv, circ)
    served = make_server_requests(srv, ids, circ, reqs)
    say("serve burst: engine pass")
    tickets = [srv.submit(r[0]) for r in served]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    say(f"  stats submitted={st.submitted} completed={st.completed} max_running={st.max_running} "
        f"peak={st.workspace_peak}")
    assert st.submitted == st.completed == len(reqs)
    assert st.running == 0 and st.queued == 0 and st.workspace_bytes == 0
    assert st.max_running > 1  # requests overlapped on the device
    assert st.max_batch > 1 and st.batches < len(reqs)  # requests shared launches
    check_same(alone, served, reqs)
    srv.close()


def test_alone_equals_submit_many(setup):
    """A burst submitted in one call is shared into batches as a whole (the
    first requests do not leave in batches of one), with results bitwise
    equal to the alone runs; requests of one shape share a cached launch
    template, filled in per request."""
    s, circ = setup
    reqs = request_list(circ, 9, 64) + request_list(circ, 9, 16)  # repeated shapes
    alone = run_alone(s, circ, reqs)
    srv = runner.Server(0, n_slots=2, workspace_bytes=1 << 30)
    ids = register_all(srv, circ)
    served = make_server_requests(srv, ids, circ, reqs)
    tickets = srv.submit_many([r[0] for r in served])
    assert len(tickets) == len(reqs) == len(set(tickets))
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    say(f"  submit_many: {st.batches} batches, largest {st.max_batch}")
    assert st.completed == len(reqs) and st.max_batch >= len(reqs) // 2
    check_same(alone, served, reqs)
    srv.close()


def test_alone_equals_arrivals_small_workspace(setup):
    """Requests arrive while others run; the workspace holds only a few at a
    time, so admission waits for memory as well as slots."""
    s, circ = setup
    reqs = request_list(circ, 8, 40)
    alone = run_alone(s, circ, reqs)
    srv0 = runner.Server(0, n_slots=1, workspace_bytes=64 << 20)
    ids0 = register_all(srv0, circ)
    probe = make_server_requests(srv0, ids0, circ, reqs)
    foot = [srv0.footprint(p[0]) for p in probe]
    srv0.close()
    assert min(foot) > 0
    ws = 2 * max(foot) + 4096
    say(f"serve arrivals: footprints {min(foot)}..{max(foot)}, workspace {ws}")
    srv = runner.Server(0, n_slots=6, workspace_bytes=ws)
    ids = register_all(srv, circ)
    served = make_server_requests(srv, ids, circ, reqs)
    tickets = []
    for k, r in enumerate(served):
        tickets.append(srv.submit(r[0]))
        if k % 3 == 2:  # let some work start, then keep submitting
            srv.poll(tickets[k - 2])
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    say(f"  stats max_running={st.max_running} peak={st.workspace_peak} of {ws}")
    assert st.workspace_peak <= ws
    assert st.completed == len(reqs)
    # the requests do not fit the workspace together, so some waited for
    # memory (however the arrivals interleave with completions)
    assert sum(foot) > ws and st.max_running < len(reqs)
    check_same(alone, served, reqs)
    srv.close()


def test_served_recursion0_matches_oracle(setup):
    """Recursion-0 requests of the small circuits, run in one burst, against
    the oracle's merged entries contracted bin by bin."""
    s, circ = setup
    srv = runner.Server(0, n_slots=3, workspace_bytes=256 << 20)
    ids = register_all(srv, circ)
    work = []
    for name in ("tiny", "chain3", "qaoa3", "pool7"):
        cc, var, _ = circ[name]
        Th = oracle_attributed(cc, var)
        for prec in (sqc.F64, sqc.F32, sqc.BF16X3):
            a = min(10, cc.n)
            req = (name, a, prec, 8, None)
            masks, bprec, bins, top, bsum = buffers(circ, req)
            r = srv.request(ids[(name, prec)], None, 1 << a, 8, prec, bins, bprec, top, bsum)
            work.append((r, name, cc, Th, masks, prec, bins, bsum))
    torch.cuda.synchronize()
    tickets = [srv.submit(w[0]) for w in work]
    for t, (r, name, cc, Th, masks, prec, bins, bsum) in zip(tickets, work):
        srv.wait(t)
        lit = [bins_from_masks(masks[i], cc.subs[i].n_data) for i in range(cc.n_sub)]
        Tm = [rc.merge_entries(Th[i], lit[i]) for i in range(cc.n_sub)]
        nb = bins.numel()
        want = network.eval_bins(Tm, cc, np.arange(nb))
        got = bins.double().cpu().numpy()
        err = np.abs(got - want).max()
        say(f"serve oracle {name} prec={prec} bins={nb} err={err:.3e}")
        assert err <= TOL[prec]
        # the sum is taken over the accumulators before they are stored (FP32
        # storage rounds each by at most 2^-24 relative), so it is within the
        # summed bin errors plus that rounding of the oracle's sum, which is 1
        assert abs(math.fsum(want.tolist()) - 1.0) <= 1e-12
        bound = nb * err + 2.0 ** -24 * math.fsum(np.abs(got).tolist()) + 1e-15
        assert abs(bsum.item() - math.fsum(want.tolist())) <= bound
    srv.close()


def test_footprint_limits(setup):
    s, circ = setup
    srv = runner.Server(0, n_slots=2, workspace_bytes=1 << 16)
    ids = register_all(srv, circ)
    req = ("pool5", 14, sqc.F32, 4, None)
    masks, bprec, bins, top, bsum = buffers(circ, req)
    r = srv.request(ids[("pool5", sqc.F32)], None, 1 << 14, 4, sqc.F32, bins, bprec, top, bsum)
    assert srv.footprint(r) > (1 << 16)
    with pytest.raises(sqc.SqcError) as e:
        srv.submit(r)
    assert e.value.status == sqc.E_NOMEM
    bad = srv.request(ids[("pool5", sqc.F32)], None, 1 << 14, 0, sqc.F32, bins, bprec, top, bsum)
    with pytest.raises(sqc.SqcError) as e:
        srv.submit(bad)
    assert e.value.status == sqc.E_ARG
    st = srv.stats()
    assert st.submitted == 0
    srv.close()


def test_batch_single_subcircuit_and_unit_path(setup):
    """Circuits of one subcircuit and no cuts (the bins are the attributed
    entries summed over merged states; the contraction is against a unit
    tensor), mixed into batches with a multi-subcircuit circuit."""
    s, circ = setup
    rng = np.random.default_rng(31)
    srv = runner.Server(0, n_slots=2, workspace_bytes=256 << 20)
    ids = register_all(srv, circ)
    single = {}
    keep = []
    for d, prec in ((9, sqc.F64), (12, sqc.F32)):
        dt = torch.float64 if prec == sqc.F64 else torch.float32
        buf = torch.from_numpy(rng.random(1 << d)).to(dt).cuda()
        keep.append(buf)
        g = sqc.Graph([d], [list(range(d))], [])
        att = [sqc.tensor_desc(buf, 0, d, prec, sqc.LAYOUT_ATTRIBUTED)]
        torch.cuda.synchronize()
        single[d] = (g, att, sqc.serve_register(srv.srv, att, g))
    work = []
    for k in range(24):
        d = 9 if k % 2 else 12
        g, att, cid = single[d]
        prec = sqc.F64 if d == 9 else (sqc.F32 if k % 4 == 0 else sqc.BF16X3)
        a = int(rng.integers(0, d + 1))
        top_r = int(rng.integers(1, 65))
        bprec = sqc.F64 if prec == sqc.F64 else sqc.F32
        dt = torch.float64 if bprec == sqc.F64 else torch.float32
        masks = sqc.assign_bins([d], None, 1 << a)
        nb = 1 << bin(masks[0].active).count("1")
        outs = [torch.full((nb,), float("nan"), dtype=dt, device="cuda") for _ in range(2)]
        tops = [torch.zeros(2 * sqc.MAX_TOPR, dtype=torch.float64, device="cuda") for _ in range(2)]
        sums = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(2)]
        s.ensure_workspace(sqc.recurse_workspace_bytes(att, g, masks, prec))
        sqc.recurse(s.ctx, att, g, None, 1 << a, top_r, prec, outs[0], bprec, tops[0], sums[0])
        srv.graphs[cid] = g
        r = srv.request(cid, None, 1 << a, top_r, prec, outs[1], bprec, tops[1], sums[1])
        work.append((r, outs, tops, sums, top_r))
    # and a few requests of a multi-subcircuit circuit in the same batches
    reqs = request_list(circ, 9, 8)
    alone = run_alone(s, circ, reqs)
    served = make_server_requests(srv, ids, circ, reqs)
    torch.cuda.synchronize()
    tickets = [srv.submit(w[0]) for w in work] + [srv.submit(r[0]) for r in served]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    say(f"  single-subcircuit batches: {st.batches} for {st.submitted} requests, max batch {st.max_batch}")
    assert st.max_batch > 1
    for r, outs, tops, sums, top_r in work:
        assert torch.equal(outs[0], outs[1])
        assert torch.equal(tops[0][:2 * top_r].view(torch.int64), tops[1][:2 * top_r].view(torch.int64))
        assert torch.equal(sums[0], sums[1])
    check_same(alone, served, reqs)
    srv.close()
