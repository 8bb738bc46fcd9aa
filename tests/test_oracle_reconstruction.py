"""Pins of the oracle's attribution and Eq. 1 reconstruction: brute-force
simulation of the uncut circuit, probability normalisation, product special
cases, and planted mistakes that the pins must catch."""
import numpy as np
import pytest

from oracle import network, reconstruction as rc, statevector as sv
from workloads import configs, qpu
from workloads.circuits import Gate, H, CNOT, brickwork, planted_qaoa
from workloads.cutgraph import build_cut_circuit


def reconstruct(cc):
    var = qpu.all_variants(cc)
    Ts = [rc.attribute(cc, i, var[i]) for i in range(cc.n_sub)]
    return rc.to_qubit_order(rc.reconstruct_eq1(Ts, cc), cc), Ts


def brute(cc):
    return sv.probabilities(cc.n, cc.circuit.gates)


def test_tiny_matches_brute_force():
    cc = configs.tiny()
    P, _ = reconstruct(cc)
    Pb = brute(cc)
    assert np.abs(P - Pb).max() <= 1e-12
    assert abs(P.sum() - 1) <= 1e-12


@pytest.mark.parametrize("seed,d,moves", [
    (11, [4, 5, 4], [1, 2]),
    (12, [3, 4, 3, 4], [2, 1, 1]),
    (13, [5, 5], [2]),
])
def test_brickwork_chains_match_brute_force(seed, d, moves):
    cc = configs.chain_brickwork(len(d), d, moves, 4, seed)
    P, _ = reconstruct(cc)
    assert np.abs(P - brute(cc)).max() <= 1e-12
    assert abs(P.sum() - 1) <= 1e-12


def test_cuts_in_both_directions():
    # boundary moving right: lines pass from subcircuit 1 back into 0
    from workloads.circuits import moving_boundary_schedule
    sched = moving_boundary_schedule(4, start=[4, 9], end=[6, 7])
    cc = build_cut_circuit(brickwork(12, 4, 21, sched))
    assert cc.summary()["K"] == 4
    ups = {(c.up_sub, c.down_sub) for c in cc.cuts}
    assert (1, 0) in ups and (1, 2) in ups
    P, _ = reconstruct(cc)
    assert np.abs(P - brute(cc)).max() <= 1e-12


def test_qaoa_ring_matches_brute_force():
    cc = build_cut_circuit(planted_qaoa([4, 4, 4], seed=5))
    s = cc.summary()
    assert s["K"] == 6 and s["V"] == [144, 144, 144]
    P, _ = reconstruct(cc)
    assert np.abs(P - brute(cc)).max() <= 1e-12


def test_bv_single_state():
    cc = configs.bv(7, 3, seed=3)
    P, _ = reconstruct(cc)
    sol = cc.meta["solution"]
    assert abs(P[sol] - 1) <= 1e-12
    P[sol] = 0
    assert np.abs(P).max() <= 1e-12


def test_no_cut_is_outer_product():
    # two independent blocks: Eq. 1 has one term, the Kronecker product
    cc = build_cut_circuit(brickwork(8, 3, 9, [[4], [4], [4]]))
    assert len(cc.cuts) == 0
    P, Ts = reconstruct(cc)
    p0 = sv.probabilities(4, [g for g in cc.circuit.gates if max(g.qubits) < 4])
    hi = [Gate(g.name, tuple(q - 4 for q in g.qubits), g.mat) for g in cc.circuit.gates if min(g.qubits) >= 4]
    p1 = sv.probabilities(4, hi)
    assert np.abs(P - np.kron(p1, p0)).max() <= 1e-14


def test_identity_wire_cut():
    # a single line cut with nothing after the cut: the downstream side only
    # re-prepares the state, so P is the upstream line's marginal in Z
    circ = brickwork(4, 2, 4, [[4], [4]])
    for g in circ.gates:
        g.sub = 0
    circ.gates.append(Gate("h", (3,), H, 1))
    circ.gates.append(Gate("h", (3,), H, 1))  # identity on the downstream side
    circ.n_sub = 2
    circ.idle_sub = [0, 0, 0, 0]
    cc = build_cut_circuit(circ)
    assert len(cc.cuts) == 1
    P, _ = reconstruct(cc)
    assert np.abs(P - brute(cc)).max() <= 1e-13


def test_network_matches_eq1():
    cc = configs.chain_brickwork(4, [3, 4, 3, 4], [2, 1, 1], 4, 12)
    var = qpu.all_variants(cc)
    Ts = [rc.attribute(cc, i, var[i]) for i in range(cc.n_sub)]
    P = rc.reconstruct_eq1(Ts, cc)
    Th = [rc.fold_half(Ts[i], sum(1 for _, r in cc.incident(i) if r == "out"))
          for i in range(cc.n_sub)]
    P2 = network.contract_all(Th, cc)
    assert np.abs(P - P2).max() <= 1e-14
    idx = np.array([0, 5, 77, len(P) - 1])
    assert np.abs(network.eval_bins(Th, cc, idx) - P[idx]).max() <= 1e-14
    assert np.abs(rc.eval_bins(Ts, cc, idx) - P[idx]).max() <= 1e-14


# ---- planted mistakes: each must break the brute-force pin (tolerance 1e-12)

def _err_with(monkeypatch, attr, value, cc):
    monkeypatch.setattr(rc, attr, value)
    P, _ = reconstruct(cc)
    return np.abs(P - brute(cc)).max()


def test_planted_y_sign_is_caught(monkeypatch):
    cc = configs.tiny()
    bad = rc.MEAS_SIGN.copy()
    bad[2] = -bad[2]
    assert _err_with(monkeypatch, "MEAS_SIGN", bad, cc) > 1e-6


def test_planted_y_prep_is_caught():
    # the downstream Y coefficient written for |-i> instead of |+i> (planted in
    # the oracle's table through a fresh copy)
    cc = configs.tiny()
    old = rc.INIT_COEF.copy()
    try:
        rc.INIT_COEF[2] = [1.0, 1.0, 0.0, -2.0]
        P, _ = reconstruct(cc)
        err = np.abs(P - brute(cc)).max()
    finally:
        rc.INIT_COEF[:] = old
    assert err > 1e-6


def test_planted_dropped_x_term_is_caught(monkeypatch):
    cc = configs.tiny()
    bad = rc.INIT_COEF.copy()
    bad[1] = 0.0
    assert _err_with(monkeypatch, "INIT_COEF", bad, cc) > 1e-6


def test_planted_basis_swap_is_caught(monkeypatch):
    cc = configs.tiny()
    assert _err_with(monkeypatch, "MEAS_BASIS", (0, 2, 1, 0), cc) > 1e-6


def test_precision_config_sampled_brute_force():
    """Degree-6 middle subcircuit (1728 variants) of the 24-qubit workload:
    Eq. 1 at sampled outputs equals the full 24-qubit statevector."""
    cc = configs.precision()
    var = qpu.all_variants(cc)
    Ts = [rc.attribute(cc, i, var[i]) for i in range(cc.n_sub)]
    Pb = brute(cc)
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 1 << 24, size=512)
    vals = rc.eval_bins(Ts, cc, idx)
    # map subcircuit-major indices to qubit order
    y = np.zeros_like(idx)
    shift = 0
    for sub in cc.subs:
        for j, q in enumerate(sub.data_qubit):
            y |= ((idx >> (shift + j)) & 1) << q
        shift += sub.n_data
    assert np.abs(vals - Pb[y]).max() <= 1e-12


# ---- first-level index slicing (Sec. 6.3): the sum over the slices' label
# assignments is Eq. 1's sum split along the sliced cuts, so every slicing of
# a circuit reproduces its brute-force reconstruction

def _chain_half():
    cc = configs.chain_brickwork(4, [3, 4, 3, 4], [2, 1, 1], 4, 12)
    var = qpu.all_variants(cc)
    Ts = [rc.attribute(cc, i, var[i]) for i in range(cc.n_sub)]
    Th = [rc.fold_half(Ts[i], sum(1 for _, r in cc.incident(i) if r == "out"))
          for i in range(cc.n_sub)]
    return cc, Ts, Th


@pytest.mark.parametrize("pick", ["none", "first", "last", "pair", "reversed", "all"])
def test_sliced_contraction_matches_eq1(pick):
    cc, Ts, Th = _chain_half()
    K = len(cc.cuts)
    sliced = {"none": [], "first": [0], "last": [K - 1], "pair": [0, K - 1],
              "reversed": [K - 1, 1, 0], "all": list(range(K))}[pick]
    P = rc.reconstruct_eq1(Ts, cc)
    assert np.abs(network.contract_sliced(Th, cc, sliced) - P).max() <= 1e-14


def test_sliced_contraction_restricts_both_sides():
    """A slice restricted on one side of its cut only (the other side summed
    over all four labels) must not reproduce Eq. 1: the pin above sees it."""
    cc, Ts, Th = _chain_half()
    P = rc.reconstruct_eq1(Ts, cc)
    k = 0
    up = cc.cuts[k].up_sub
    # summing the upstream entries over the cut's labels first, then slicing
    # only the downstream side, gives a different vector
    t = network._sub_tensor(cc, up, Th[up])
    ax = network._cut_axes(cc, up).index(k)
    wrong_up = np.repeat(t.sum(axis=ax, keepdims=True), 4, axis=ax).reshape(Th[up].shape)
    Tw = list(Th)
    Tw[up] = wrong_up
    assert np.abs(network.contract_sliced(Tw, cc, [k]) - P).max() > 1e-6
