"""Cut-basis attribution and full-definition reconstruction (paper Sec. 2.1).

Notation.  A cut circuit has K cut edges and n_C subcircuits.  Each cut carries
a label sigma_e in {I, X, Y, Z} (numbered 0, 1, 2, 3).  Subcircuit i touches
c_i cuts; its labels sigma|_i are numbered sum_j sigma_{e_j} 4^j over its
incident cuts e_0, e_1, ... in global cut order.  Its data index x_i runs over
its d_i data qubits, data bit j being ``data_wire[j]``.

Eq. 1 writes the uncut output as the sum over all 4^K label assignments of the
outer product of one entry per subcircuit.  The entry of subcircuit i for an
assignment is obtained from its measured variants (Fig. 1: the upstream side is
measured, the downstream side initialised, in each basis); the physics is the
single-qubit Pauli decomposition

    rho = 1/2 * sum_{P in {I,X,Y,Z}} Tr(P rho) P .

Upstream, Tr(P rho) is a signed sum of outcome probabilities in the eigenbasis
of P (the I term reuses the Z measurement with all signs +1).  Downstream, P is
written as a combination of the four prepared states:
I = |0><0| + |1><1|, Z = |0><0| - |1><1|, X = 2|+><+| - I, Y = 2|+i><+i| - I.

Reading (normalisation): Eq. 1 prints no factor; the decomposition gives 1/2
per cut, so the reconstruction is 2^-K times the sum.  Pinned by brute-force
simulation and by the probabilities summing to 1.
"""
from __future__ import annotations

import itertools
from typing import List, Sequence

import numpy as np

LABELS = ("I", "X", "Y", "Z")
# Downstream: coefficient of each preparation (|0>, |1>, |+>, |+i>) in P.
INIT_COEF = np.array([
    [1.0, 1.0, 0.0, 0.0],    # I
    [-1.0, -1.0, 2.0, 0.0],  # X
    [-1.0, -1.0, 0.0, 2.0],  # Y
    [1.0, -1.0, 0.0, 0.0],   # Z
])
# Upstream: measurement basis digit (0 = Z, 1 = X, 2 = Y) used for each label
MEAS_BASIS = (0, 1, 2, 0)
# Upstream: weight of outcome bit b for each label
MEAS_SIGN = np.array([
    [1.0, 1.0],    # I
    [1.0, -1.0],   # X
    [1.0, -1.0],   # Y
    [1.0, -1.0],   # Z
])


def _bits_to_index(o: np.ndarray, positions: Sequence[int]) -> np.ndarray:
    out = np.zeros_like(o)
    for j, p in enumerate(positions):
        out |= ((o >> p) & 1) << j
    return out


def attribute(cc, i: int, variants: np.ndarray, sigmas=None) -> np.ndarray:
    """Entries T_i[sigma, x] (float64, shape [4^c_i][2^d_i]) of subcircuit i
    for every label assignment of its incident cuts (Sec. 2.1, p_i(k) of
    Eq. 1, without the 1/2-per-cut factor).  With ``sigmas`` (a list of label
    indices) only those rows are evaluated, shape [len(sigmas)][2^d_i].

    ``variants[v][o]``: probability of outcome o (wire t = bit t) in variant v
    (mixed radix over incident cuts: radix 4 preparations for in-cuts, radix 3
    bases for out-cuts, first incident cut least significant).
    """
    sub = cc.subs[i]
    inc = cc.incident(i)
    c = len(inc)
    w, d = sub.n_wires, sub.n_data
    o = np.arange(1 << w, dtype=np.int64)
    x_of_o = _bits_to_index(o, sub.data_wire)
    radix = [4 if role == "in" else 3 for _, role in inc]
    place = [int(np.prod(radix[:j])) for j in range(c)]
    bits_out = {}
    for j, (k, role) in enumerate(inc):
        if role == "out":
            bits_out[j] = (o >> cc.cuts[k].up_wire) & 1
    variants = np.asarray(variants, dtype=np.float64)
    rows = range(4 ** c) if sigmas is None else list(sigmas)
    T = np.zeros((len(rows), 1 << d), dtype=np.float64)
    for row, sigma in enumerate(rows):
        lab = [(sigma >> (2 * j)) & 3 for j in range(c)]
        # outcome weights of the out-cuts and the fixed part of the variant id
        wgt = np.ones(1 << w)
        v_fixed = 0
        choices = []  # per in-cut: list of (digit value, coefficient)
        for j, (_, role) in enumerate(inc):
            if role == "out":
                wgt = wgt * MEAS_SIGN[lab[j]][bits_out[j]]
                v_fixed += MEAS_BASIS[lab[j]] * place[j]
            else:
                choices.append([(j, s, INIT_COEF[lab[j], s]) for s in range(4)
                                if INIT_COEF[lab[j], s] != 0.0])
        for combo in itertools.product(*choices):
            coef = 1.0
            v = v_fixed
            for (j, s, cf) in combo:
                coef *= cf
                v += s * place[j]
            T[row] += coef * np.bincount(x_of_o, weights=wgt * variants[v],
                                         minlength=1 << d)
    return T


def labels_of_sub(cc, i: int, sigma_global: np.ndarray) -> np.ndarray:
    """sigma|_i for global assignments sigma = sum_e sigma_e 4^e."""
    out = np.zeros_like(sigma_global)
    for j, (k, _) in enumerate(cc.incident(i)):
        out |= ((sigma_global >> (2 * k)) & 3) << (2 * j)
    return out


def reconstruct_eq1(Ts: List[np.ndarray], cc) -> np.ndarray:
    """Eq. 1 with the 2^-K normalisation:
    P = 2^-K sum_{sigma in 4^K} T_{n_C-1}[sigma] (x) ... (x) T_0[sigma].
    Output index is subcircuit-major, subcircuit 0 least significant (the
    outer-product order; Sec. 6.4 notes that the order only permutes qubits).
    ``Ts[i]`` may be full ([4^c][2^d]) or merged ([4^c][bins_i]) entries.
    """
    K = len(cc.cuts)
    size = int(np.prod([T.shape[1] for T in Ts]))
    P = np.zeros(size, dtype=np.float64)
    sig = np.arange(4 ** K, dtype=np.int64)
    loc = [labels_of_sub(cc, i, sig) for i in range(cc.n_sub)]
    for s in range(4 ** K):
        term = Ts[cc.n_sub - 1][loc[cc.n_sub - 1][s]]
        for i in range(cc.n_sub - 2, -1, -1):
            term = np.kron(term, Ts[i][loc[i][s]])
        P += term
    return P * (0.5 ** K)


def eval_bins(Ts: List[np.ndarray], cc, bins: np.ndarray) -> np.ndarray:
    """Eq. 1 evaluated at selected output indices only (subcircuit-major index,
    subcircuit 0 least significant): 2^-K sum_sigma prod_i T_i[sigma|_i, x_i]."""
    K = len(cc.cuts)
    sig = np.arange(4 ** K, dtype=np.int64)
    loc = [labels_of_sub(cc, i, sig) for i in range(cc.n_sub)]
    widths = [T.shape[1] for T in Ts]
    out = np.empty(len(bins), dtype=np.float64)
    for b, idx in enumerate(np.asarray(bins, dtype=np.int64)):
        rem = int(idx)
        prod = np.ones(4 ** K)
        for i in range(cc.n_sub):
            xi = rem % widths[i]
            rem //= widths[i]
            prod = prod * Ts[i][loc[i], xi]
        out[b] = prod.sum()
    return out * (0.5 ** K)


def to_qubit_order(P_sub: np.ndarray, cc) -> np.ndarray:
    """Permute a subcircuit-major output into original-qubit order (qubit q =
    bit q), using each subcircuit's data-qubit map (Sec. 6.4)."""
    n = cc.n
    idx = np.arange(1 << n, dtype=np.int64)
    y = np.zeros_like(idx)
    shift = 0
    for sub in cc.subs:
        for j, q in enumerate(sub.data_qubit):
            y |= ((idx >> (shift + j)) & 1) << q
        shift += sub.n_data
    out = np.empty_like(P_sub)
    out[y] = P_sub
    return out


def fold_half(T: np.ndarray, n_out: int) -> np.ndarray:
    """The same entries with the 1/2 per cut moved onto the upstream side:
    multiplying every out-cut's subcircuit by 1/2 gives 2^-K overall."""
    return T * (0.5 ** n_out)


def merge_entries(T: np.ndarray, bins: List[List[int]]) -> np.ndarray:
    """States merging (Sec. 4): the entry of a bin is the sum of the entries of
    the states it contains: Tm[sigma, k] = sum_{x in bins[k]} T[sigma, x]."""
    Tm = np.zeros((T.shape[0], len(bins)), dtype=np.float64)
    for k, states in enumerate(bins):
        for x in states:
            Tm[:, k] += T[:, x]
    return Tm


def abs_bound_entries(Ts: List[np.ndarray]) -> List[np.ndarray]:
    """|T| element-wise: contracting these instead of T bounds the size of the
    terms that are summed for each output (used for a-priori error bounds)."""
    return [np.abs(T) for T in Ts]
