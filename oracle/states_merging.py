"""States merging on explicit lists of states: the bin assignment of Alg. 2
and the recursion driver of Alg. 1 (Sec. 3-4).  Test infrastructure only.

Each recursion analyses, per subcircuit, an ascending list of data states
(all 2^d_i states at the first recursion, else the states of the bin being
expanded).  Bin counts start at the list lengths; while their product exceeds
M, the largest count is halved, rounding up.  A subcircuit's bins are then the
residue classes of positions in its ordered list modulo its bin count.

Readings where the paper is silent (shared with the library's host code):

* order: a subcircuit's states are enumerated in ascending index order;
* labels: the paper's 1-based residue rule gives the same partition as the
  0-based classes used here; bins are numbered by their smallest member, which
  for residue classes is the class index itself;
* ties between equally large bin counts halve the lowest subcircuit index
  first -- parity unpinned, any rule is valid;
* Alg. 1's candidate list holds bins with more than one state, ordered by
  probability (largest first), then earlier recursion, then lower bin index,
  and is cut to R entries -- parity unpinned beyond the recursion count of a
  single-solution circuit; bins of single states are reported as solutions
  (the paper leaves their reporting open);
* the driver stops when the candidate list is empty or after R recursions
  (R bounds both the recursion count and the list's length).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .reconstruction import merge_entries, reconstruct_eq1


def bin_counts(lengths: List[int], M: int) -> List[int]:
    """Per-subcircuit bin counts of Alg. 2: the list lengths, with the largest
    count (lowest index on ties) halved, rounding up, as long as the product
    of the counts exceeds M."""
    counts = list(lengths)
    while int(np.prod(counts, dtype=object)) > M:
        i = counts.index(max(counts))
        counts[i] = (counts[i] + 1) // 2
    return counts


def assign_states(r: int, bin_states: Optional[List[List[int]]], M: int,
                  n_list: List[int]) -> List[List[List[int]]]:
    """Alg. 2.  Returns, per subcircuit i, its bins, each the ascending list of
    data states (over the d_i data qubits) it holds: bin b of subcircuit i is
    every counts[i]-th state of the ordered list, starting at position b."""
    if r == 0:
        ordered = [list(range(1 << d)) for d in n_list]
    else:
        ordered = [sorted(b) for b in bin_states]
    counts = bin_counts([len(o) for o in ordered], M)
    return [[o[b::c] for b in range(c)] for o, c in zip(ordered, counts)]


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
    """Alg. 1 with the cut search and the QPU runs replaced by given attributed
    entries (summing entries over a bin equals merging the measured outcomes,
    as merging acts on data qubits only).  Each recursion evaluates the bins of
    one parent (the whole output space first), reports the R most probable as
    solutions when they are single states, else adds them to a candidate list
    kept best first and cut to R; the next parent is the list's best."""
    n_list = [s.n_data for s in cc.subs]
    res = SearchResult()
    frontier: List[Entry] = []
    parent: Optional[Entry] = None
    for r in range(R):
        bins = assign_states(r, None if parent is None else parent.states, M, n_list)
        P = recursion_bins(Ts_half, cc, bins)
        counts = [len(b) for b in bins]
        top = sorted(range(len(P)), key=lambda k: (-P[k], k))[:R]
        leaf = bin_size(bins) == 1
        res.history.append({
            "r": r, "a": [int(np.log2(c)) for c in counts], "leaf": leaf,
            "sum": float(P.sum()), "top": [(int(k), float(P[k])) for k in top],
            "parent": None if parent is None else (parent.r, parent.index, parent.prob)})
        picked = [(int(k), split_index(k, counts)) for k in top]
        if leaf:
            res.solutions += [(float(P[k]), [bins[i][ks[i]][0] for i in range(cc.n_sub)])
                              for k, ks in picked]
        else:
            frontier += [Entry(float(P[k]), r, k, [bins[i][ks[i]] for i in range(cc.n_sub)])
                         for k, ks in picked]
            frontier = sorted(frontier, key=lambda e: (-e.prob, e.r, e.index))[:R]
        res.recursions = r + 1
        if not frontier:
            break
        parent = frontier.pop(0)
    return res


def global_state(cc, per_sub_states: List[int]) -> int:
    """Original-qubit index (qubit q = bit q) of a leaf given per-subcircuit
    data states."""
    y = 0
    for i, sub in enumerate(cc.subs):
        for j, q in enumerate(sub.data_qubit):
            y |= ((per_sub_states[i] >> j) & 1) << q
    return y
