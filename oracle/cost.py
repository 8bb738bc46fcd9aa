"""Memory requirement and compute cost of compute-graph contraction (paper
Sec. 6.2) and first-level index slicing sizes (Sec. 6.3).

A compute graph is given as a list of tensors, each a pair (set of cut ids,
output dimension), where a cut id has dimension 4 (labels I, X, Y, Z) and the
output dimension is 2^qubits (full state) or the number of bins (states
merging).
"""
from __future__ import annotations

from typing import FrozenSet, List, Sequence, Tuple

Tensor = Tuple[FrozenSet[int], int]


def size(t: Tensor) -> int:
    """Floats held by one tensor: 4^#cuts * output dimension."""
    return (4 ** len(t[0])) * t[1]


def input_floats(tensors: Sequence[Tensor]) -> int:
    return sum(size(t) for t in tensors)


def contract_pair(a: Tensor, b: Tensor) -> Tuple[Tensor, int]:
    """Result tensor and multiplication count of one pairwise contraction:
    the product of all dimensions involved (shared and free cut indices of both
    tensors, and both output dimensions)."""
    shared = a[0] & b[0]
    union = a[0] | b[0]
    mults = (4 ** len(union)) * a[1] * b[1]
    return (frozenset(union - shared), a[1] * b[1]), mults


def plan_cost(tensors: Sequence[Tensor], order: Sequence[Tuple[int, int]]):
    """Run a contraction order (pairs of positions in a working list; the
    result replaces the first, the second is removed).  Returns per-step
    (floats of the two operands, multiplications) and the totals."""
    work: List[Tensor] = list(tensors)
    steps = []
    for (i, j) in order:
        a, b = work[i], work[j]
        c, m = contract_pair(a, b)
        steps.append({"operand_floats": size(a) + size(b), "mults": m,
                      "result_floats": size(c)})
        work[i] = c
        del work[j]
    return steps, sum(s["mults"] for s in steps)


def naive_mults(n_cuts: int, out_dims: Sequence[int]) -> int:
    """Multiplications of evaluating Eq. 1 directly: for each of the 4^K
    terms, the successive outer products of the subcircuit vectors."""
    per_term = 0
    acc = out_dims[0]
    for d in out_dims[1:]:
        per_term += acc * d
        acc *= d
    return (4 ** n_cuts) * per_term


def slice_edge(tensors: Sequence[Tensor], e: int) -> List[Tensor]:
    """Tensors of each of the 4 sub-graphs obtained by writing out cut e."""
    return [(t[0] - {e}, t[1]) for t in tensors]


def greedy_slices(tensors: Sequence[Tensor], budget_floats: int) -> List[int]:
    """Sec. 6.3 heuristic: repeatedly slice the cut whose removal reduces the
    total input size the most, until the total fits the budget."""
    cur = list(tensors)
    chosen: List[int] = []
    while input_floats(cur) > budget_floats:
        cuts = sorted(set().union(*[t[0] for t in cur]))
        if not cuts:
            break
        best = min(cuts, key=lambda e: (input_floats(slice_edge(cur, e)), e))
        chosen.append(best)
        cur = slice_edge(cur, best)
    return chosen
