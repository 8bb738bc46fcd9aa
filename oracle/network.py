"""Plain FP64 tensor-network evaluation of a compute graph (paper Sec. 6.1).

Each subcircuit's entries T_i[sigma|_i, x_i] are a tensor with one index of
dimension 4 per incident cut and one output index; contracting all cut indices
gives Eq. 1's sum (Sec. 6.1 shows the two are the same).  This module uses
numpy's einsum as the contraction primitive, with no blocking or reordering of
its own, for graphs whose 4^K terms are too many for ``reconstruction``.
"""
from __future__ import annotations

import string
from typing import List, Sequence

import numpy as np

_LETTERS = string.ascii_letters


def _sub_tensor(cc, i: int, T: np.ndarray) -> np.ndarray:
    """T_i as a tensor with axes (cut labels most significant first ..., x)."""
    c = len(cc.incident(i))
    # T[sigma][x], sigma = sum_j s_j 4^j: C-order axes are s_{c-1} ... s_0
    return T.reshape((4,) * c + (T.shape[1],))


def _cut_axes(cc, i: int) -> List[int]:
    """Global cut id of each label axis of ``_sub_tensor`` (C order)."""
    return [k for k, _ in cc.incident(i)][::-1]


def eval_bins(Ts: Sequence[np.ndarray], cc, bins: Sequence[int]) -> np.ndarray:
    """Output values at selected subcircuit-major indices (subcircuit 0 least
    significant), by contracting the cut indices of the entries sliced at each
    subcircuit's x_i.  ``Ts`` carry the 1/2-per-cut factor already (folded)."""
    K = len(cc.cuts)
    if K > len(_LETTERS):
        raise ValueError("too many cuts for einsum letters")
    widths = [T.shape[1] for T in Ts]
    tens = [_sub_tensor(cc, i, Ts[i]) for i in range(cc.n_sub)]
    axes = [_cut_axes(cc, i) for i in range(cc.n_sub)]
    spec = ",".join("".join(_LETTERS[k] for k in ax) for ax in axes) + "->"
    out = np.empty(len(bins))
    path = None
    for b, idx in enumerate(bins):
        rem = int(idx)
        ops = []
        for i in range(cc.n_sub):
            xi = rem % widths[i]
            rem //= widths[i]
            ops.append(tens[i][..., xi])
        if path is None:
            path = np.einsum_path(spec, *ops, optimize="greedy")[0]
        out[b] = np.einsum(spec, *ops, optimize=path)
    return out


def contract_all(Ts: Sequence[np.ndarray], cc) -> np.ndarray:
    """Whole output vector (subcircuit-major) by one einsum over all cut
    indices and all output indices.  ``Ts`` carry the 1/2-per-cut factor."""
    K = len(cc.cuts)
    if K + cc.n_sub > len(_LETTERS):
        raise ValueError("too many indices for einsum letters")
    tens = [_sub_tensor(cc, i, Ts[i]) for i in range(cc.n_sub)]
    axes = [_cut_axes(cc, i) for i in range(cc.n_sub)]
    outl = [_LETTERS[K + i] for i in range(cc.n_sub)]
    spec = ",".join("".join(_LETTERS[k] for k in ax) + outl[i]
                    for i, ax in enumerate(axes))
    spec += "->" + "".join(outl[::-1])  # subcircuit 0 least significant
    res = np.einsum(spec, *tens, optimize="greedy")
    return res.reshape(-1)


class _WithoutCuts:
    """The compute graph of ``cc`` with the cuts in ``drop`` removed (the
    remaining cuts keep their order and are renumbered from 0)."""

    def __init__(self, cc, drop):
        drop = set(drop)
        self.n_sub = cc.n_sub
        self._keep = [k for k in range(len(cc.cuts)) if k not in drop]
        self.cuts = [cc.cuts[k] for k in self._keep]
        self._new = {k: j for j, k in enumerate(self._keep)}
        self._cc = cc

    def incident(self, i: int):
        return [(self._new[k], role) for k, role in self._cc.incident(i) if k in self._new]


def contract_sliced(Ts: Sequence[np.ndarray], cc, sliced: Sequence[int]) -> np.ndarray:
    """First-level index slicing (Sec. 6.3): the cut indices in ``sliced``
    are written out as an explicit outer sum.  For every label assignment of
    those cuts (the first listed cut the least significant radix-4 digit),
    each subcircuit's entries are restricted to the assigned labels, the graph
    without the sliced cuts is contracted by ``contract_all``, and the slices'
    vectors are added in ascending assignment order.  ``Ts`` carry the
    1/2-per-cut factor."""
    sliced = [int(k) for k in sliced]
    if len(set(sliced)) != len(sliced):
        raise ValueError("a cut is sliced twice")
    rest = _WithoutCuts(cc, sliced)
    total = None
    for q in range(4 ** len(sliced)):
        label = {k: (q >> (2 * j)) & 3 for j, k in enumerate(sliced)}
        parts = []
        for i in range(cc.n_sub):
            t = _sub_tensor(cc, i, Ts[i])
            sel = tuple(label[k] if k in label else slice(None) for k in _cut_axes(cc, i))
            parts.append(t[sel + (slice(None),)].reshape(-1, Ts[i].shape[1]))
        v = contract_all(parts, rest)
        total = v if total is None else total + v
    return total
