"""Cut search model of Sec. 5 (MIP model, constraints and objective), solved by
exhaustive enumeration for tiny circuits.  Test infrastructure only.

The circuit's two-qubit gates are the vertices V of a DAG; each qubit line
between two consecutive two-qubit gates on that qubit is an edge (input and
output vertices are left out, as the paper does).  A partition assigns every
vertex to one of n_C subcircuits.  An edge is cut when its endpoints lie in
different subcircuits; it is an outgoing cut of its tail's subcircuit and an
incoming cut of its head's.  Constraint (Eq. 2): every subcircuit holds at
most alpha |V| gates.  Objective (Eq. 3): the largest number of cut edges on
one subcircuit, L = max_c (I_c + O_c).  Every one of the n_C subcircuits is
non-empty.
"""
from __future__ import annotations

import itertools
import math
from typing import List, Optional, Sequence, Tuple


def dag_edges(gates: Sequence[Tuple[int, int]]) -> List[Tuple[int, int]]:
    """Edges (tail gate, head gate) of the two-qubit-gate DAG: one per qubit
    line between consecutive two-qubit gates on that qubit (a pair of gates
    sharing both qubits gives two edges)."""
    last = {}
    edges = []
    for v, (a, b) in enumerate(gates):
        for q in (a, b):
            if q in last:
                edges.append((last[q], v))
            last[q] = v
    return edges


def degree(assign: Sequence[int], edges, n_sub: int) -> List[int]:
    """I_c + O_c for every subcircuit c."""
    deg = [0] * n_sub
    for u, v in edges:
        if assign[u] != assign[v]:
            deg[assign[u]] += 1
            deg[assign[v]] += 1
    return deg


def objective(assign: Sequence[int], edges, n_sub: int) -> int:
    """Eq. 3."""
    return max(degree(assign, edges, n_sub)) if n_sub > 0 else 0


def feasible(assign: Sequence[int], n_sub: int, alpha: float) -> bool:
    """Eq. 2 and non-empty subcircuits."""
    cap = math.floor(alpha * len(assign) + 1e-9)
    counts = [0] * n_sub
    for c in assign:
        counts[c] += 1
    return all(1 <= k <= cap for k in counts)


def brute_force(gates: Sequence[Tuple[int, int]], n_sub: int, alpha: float) -> Optional[int]:
    """Smallest L over every feasible assignment (None when there is none)."""
    edges = dag_edges(gates)
    best = None
    for assign in itertools.product(range(n_sub), repeat=len(gates)):
        if not feasible(assign, n_sub, alpha):
            continue
        L = objective(assign, edges, n_sub)
        if best is None or L < best:
            best = L
    return best
