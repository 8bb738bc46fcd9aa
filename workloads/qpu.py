"""Stand-in for the quantum processors: runs every variant of a subcircuit.

Variants (paper Fig. 1, Sec. 2.1): each downstream (in-)cut wire of a
subcircuit starts in one of |0>, |1>, |+>, |+i> (digit 0..3, radix 4) and each
upstream (out-)cut wire is measured in the Z, X or Y basis (digit 0..2,
radix 3).  The variant index is mixed-radix over the subcircuit's incident cuts
in global cut order, first incident cut least significant.  Measuring in X
means applying H before a Z measurement; in Y, S^dagger then H.  Outcome bit 0
is the +1 eigenvalue.  All wires are measured; wire t is bit t of the outcome
index.  The result is a ``[V][2^w]`` float64 array of probabilities.

This is input generation (the quantum side of the hybrid workflow), not
post-processing.  ``random_variants`` gives seeded random outputs in the same
shape, the paper's own practice when circuits are too large to run
(Sec. 7.1).
"""
from __future__ import annotations

from typing import List

import numpy as np

from .cutgraph import CutCircuit, Subcircuit

_S2 = 1.0 / np.sqrt(2.0)
# amplitudes of the four preparations on (|0>, |1>)
PREP = np.array([[1, 0], [0, 1], [_S2, _S2], [_S2, 1j * _S2]], dtype=np.complex128)
_H = np.array([[1, 1], [1, -1]], dtype=np.complex128) * _S2
_SDG = np.diag([1, -1j]).astype(np.complex128)
# basis change applied before a Z measurement, for Z, X, Y
MEAS_ROT = np.stack([np.eye(2, dtype=np.complex128), _H, _H @ _SDG])


def _apply(psi: np.ndarray, w: int, mat: np.ndarray, wires) -> np.ndarray:
    """Apply a 1- or 2-wire unitary to a batch of w-wire states ``psi[B, 2^w]``."""
    B = psi.shape[0]
    t = psi.reshape((B,) + (2,) * w)
    axes = [1 + (w - 1 - q) for q in wires]
    # put the gate's wires last: (..., bit of wires[-1], ..., bit of wires[0])
    t = np.moveaxis(t, axes[::-1], list(range(-len(wires), 0)))
    shp = t.shape
    k = 1 << len(wires)
    t = t.reshape(-1, k) @ mat.T
    t = t.reshape(shp)
    t = np.moveaxis(t, list(range(-len(wires), 0)), axes[::-1])
    return np.ascontiguousarray(t).reshape(B, 1 << w)


def simulate_variants(cc: CutCircuit, i: int) -> np.ndarray:
    """Probabilities ``[V_i][2^{w_i}]`` of every variant of subcircuit ``i``."""
    sub: Subcircuit = cc.subs[i]
    w = sub.n_wires
    inc = cc.incident(i)
    in_wires = []   # wire index per in-cut, in incident order
    out_wires = []
    for k, role in inc:
        c = cc.cuts[k]
        if role == "in":
            in_wires.append(c.down_wire)
        else:
            out_wires.append(c.up_wire)
    nin, nout = len(in_wires), len(out_wires)
    # evolve the 2^nin computational-basis inputs on the in-wires
    psi = np.zeros((1 << nin, 1 << w), dtype=np.complex128)
    for e in range(1 << nin):
        idx = 0
        for j, t in enumerate(in_wires):
            if (e >> j) & 1:
                idx |= 1 << t
        psi[e, idx] = 1.0
    for mat, wires in sub.gates:
        psi = _apply(psi, w, mat, wires)
    # combine into the 4^nin preparations: axis j of (2,)*nin is in-cut nin-1-j
    st = psi.reshape((2,) * nin + (1 << w,))
    for j in range(nin):
        ax = nin - 1 - j
        st = np.moveaxis(np.tensordot(PREP, st, axes=([1], [ax])), 0, ax)
    st = st.reshape(4 ** nin, 1 << w)  # index: sum_j s_j 4^j
    # measurement rotations: produce a radix-3 axis per out-cut
    cur = st[:, None, :]  # [4^nin][3^done][2^w]
    for j, t in enumerate(out_wires):
        outs = []
        for b in range(3):
            outs.append(_apply(cur.reshape(-1, 1 << w), w, MEAS_ROT[b], (t,))
                        .reshape(cur.shape))
        # new digit is more significant than the ones already done
        cur = np.stack(outs, axis=1).reshape(cur.shape[0], -1, 1 << w)
    probs = np.abs(cur) ** 2  # [4^nin][3^nout][2^w]
    # split into digits, most significant first: s_{nin-1}..s_0, b_{nout-1}..b_0, x
    t = probs.reshape(tuple([4] * nin) + tuple([3] * nout) + (1 << w,))
    src = []  # source axis of each incident digit, in incident order
    in_j = out_j = 0
    for _, role in inc:
        if role == "in":
            src.append(nin - 1 - in_j)
            in_j += 1
        else:
            src.append(nin + nout - 1 - out_j)
            out_j += 1
    t = np.transpose(t, src[::-1] + [nin + nout])
    V = 4 ** nin * 3 ** nout
    return np.ascontiguousarray(t).reshape(V, 1 << w)


def random_variants(cc: CutCircuit, i: int, seed: int) -> np.ndarray:
    """Seeded random outputs ``[V_i][2^{w_i}]``: Exp(1) draws normalised per
    variant (a stand-in used only where simulation is too large)."""
    rng = np.random.default_rng(seed)
    V = cc.n_variants(i)
    w = cc.subs[i].n_wires
    p = rng.exponential(1.0, size=(V, 1 << w))
    p /= p.sum(axis=1, keepdims=True)
    return p


def all_variants(cc: CutCircuit) -> List[np.ndarray]:
    return [simulate_variants(cc, i) for i in range(cc.n_sub)]
