"""States merging: Algorithm 2 (states assignment) and Algorithm 1 (the
recursion loop), paper Sec. 3-4, on explicit lists of states.

Readings where the paper is silent (shared with the GPU library's host code):

* enumeration: "the j-th state" of a subcircuit is the j-th smallest state
  index among the states under analysis (ascending order);
* bin labels: the assignment uses the printed 1-based rule k = j mod l'_i; the
  resulting bins are then numbered in ascending order of their smallest member
  (the same partition; only the labels rotate);
* ties in "the subcircuit with the largest l'_i": the lowest subcircuit index
  wins -- parity unpinned, any rule is valid;
* Algorithm 1's list L: a bin is "not yet fully expanded" when it holds more
  than one state; L is ordered by probability (largest first), then earlier
  recursion, then lower bin index -- parity unpinned beyond the recursion count
  of a single-solution circuit; bins of single states are reported as
  solutions (the paper leaves their reporting open);
* "bin is None" means L is empty; R is both the recursion cap and the capacity
  of L, as printed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .reconstruction import merge_entries, reconstruct_eq1


def assign_states(r: int, bin_states: Optional[List[List[int]]], M: int,
                  n_list: List[int]) -> List[List[List[int]]]:
    """Algorithm 2.  Returns, per subcircuit i, its list of bins, each bin the
    ascending list of state indices (over the d_i data qubits) it holds."""
    n_C = len(n_list)
    if r == 0:
        states = [list(range(1 << n_list[i])) for i in range(n_C)]
    else:
        states = [sorted(bin_states[i]) for i in range(n_C)]
    l = [len(s) for s in states]
    lp = list(l)
    total = 1
    for v in lp:
        total *= v
    while total > M:
        i_max = 0
        for i in range(1, n_C):
            if lp[i] > lp[i_max]:
                i_max = i
        lp[i_max] = -(-lp[i_max] // 2)
        total = 1
        for v in lp:
            total *= v
    out = []
    for i in range(n_C):
        bins = [[] for _ in range(lp[i])]
        for j in range(1, l[i] + 1):
            k = j % lp[i]
            bins[k].append(states[i][j - 1])
        bins.sort(key=lambda b: b[0])  # label bins by their smallest member
        out.append(bins)
    return out


def bin_size(bins_per_sub: List[List[List[int]]]) -> int:
    s = 1
    for bins in bins_per_sub:
        s *= len(bins[0])
    return s


@dataclass
class Entry:
    prob: float
    r: int
    index: int
    states: List[List[int]]  # per subcircuit, the states of this bin


@dataclass
class SearchResult:
    solutions: List[tuple] = field(default_factory=list)  # (prob, per-sub states)
    recursions: int = 0
    history: List[dict] = field(default_factory=list)


def recursion_bins(Ts_half: List[np.ndarray], cc, bins_per_sub) -> np.ndarray:
    """One recursion's merged bin probabilities: Eq. 1 on merged entries
    (Sec. 6.1, the inputs' last dimension is each subcircuit's bin count).
    ``Ts_half`` are attributed entries with the 1/2 per cut already folded in,
    so no further normalisation is applied."""
    Tm = [merge_entries(Ts_half[i], bins_per_sub[i]) for i in range(cc.n_sub)]
    return reconstruct_eq1(Tm, cc) * (2.0 ** len(cc.cuts))


def split_index(idx: int, counts: List[int]) -> List[int]:
    out = []
    for c in counts:
        out.append(idx % c)
        idx //= c
    return out


def search(Ts_half: List[np.ndarray], cc, M: int, R: int) -> SearchResult:
    """Algorithm 1 with the cut search and QPU steps replaced by given
    attributed entries (the QPU's merged bins are obtained by summing entries,
    which equals merging measured outcomes because merging touches only data
    qubits)."""
    n_list = [s.n_data for s in cc.subs]
    L: List[Entry] = []
    res = SearchResult()
    r = 0
    chosen: Optional[Entry] = None
    while r < R:
        if r > 0 and chosen is None:
            break
        bins = assign_states(r, None if chosen is None else chosen.states, M, n_list)
        P = recursion_bins(Ts_half, cc, bins)
        counts = [len(b) for b in bins]
        order = sorted(range(len(P)), key=lambda k: (-P[k], k))
        top = order[:R]
        rec = {"r": r, "a": [int(np.log2(c)) for c in counts],
               "leaf": bin_size(bins) == 1,
               "sum": float(P.sum()), "top": [(int(k), float(P[k])) for k in top],
               "parent": None if chosen is None else (chosen.r, chosen.index, chosen.prob)}
        res.history.append(rec)
        if bin_size(bins) > 1:
            for k in top:
                ks = split_index(k, counts)
                L.append(Entry(float(P[k]), r, int(k),
                               [bins[i][ks[i]] for i in range(cc.n_sub)]))
        else:
            for k in top:
                ks = split_index(k, counts)
                res.solutions.append((float(P[k]), [bins[i][ks[i]][0] for i in range(cc.n_sub)]))
        L.sort(key=lambda e: (-e.prob, e.r, e.index))
        L = L[:R]
        chosen = L.pop(0) if L else None
        r += 1
    res.recursions = r
    return res


def global_state(cc, per_sub_states: List[int]) -> int:
    """Original-qubit index (qubit q = bit q) of a leaf given per-subcircuit
    data states."""
    y = 0
    for i, sub in enumerate(cc.subs):
        for j, q in enumerate(sub.data_qubit):
            y |= ((per_sub_states[i] >> j) & 1) << q
    return y
