"""Seeded circuit generators with a gate-to-subcircuit assignment.

Qubit ``q`` of an ``n``-qubit circuit is bit ``q`` of a basis-state index
(little-endian).  A gate is a :class:`Gate` holding its unitary in the basis
ordered by (bit of ``qubits[0]``) + 2 * (bit of ``qubits[1]``), and the
subcircuit it is assigned to.

Benchmark families (paper Sec. 7.2): ``Supremacy``-like random brickwork
circuits, ``Regular`` (p=1 QAOA on 3-regular graphs with random angles) and
``BV`` (Bernstein-Vazirani, a single solution state).  The generators assign
gates to subcircuits by construction, so that each workload has a fixed,
known cut structure; the library's own cut search of Sec. 5
(``sqc_find_cuts``) partitions an arbitrary circuit's two-qubit gates and is
tested against these assignments.  The assignment follows the paper's rule
that a single-qubit gate belongs to the subcircuit of its neighbouring
two-qubit gate.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_S2 = 1.0 / np.sqrt(2.0)

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PW = (PX + PY) * _S2
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) * _S2


def sqrt_pauli(p: np.ndarray) -> np.ndarray:
    """exp(-i pi/4 P) = (I - iP)/sqrt(2) for a Pauli-like P with P^2 = I."""
    return (I2 - 1j * p) * _S2


SQRT_X = sqrt_pauli(PX)
SQRT_Y = sqrt_pauli(PY)
SQRT_W = sqrt_pauli(PW)
SQRT_GATES = (("sx", SQRT_X), ("sy", SQRT_Y), ("sw", SQRT_W))

CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
# CNOT with control qubits[0] and target qubits[1]; basis index = c + 2 t.
CNOT = np.zeros((4, 4), dtype=np.complex128)
for _c in range(2):
    for _t in range(2):
        CNOT[_c + 2 * (_t ^ _c), _c + 2 * _t] = 1.0


def rx(theta: float) -> np.ndarray:
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def zz_phase(gamma: float) -> np.ndarray:
    """exp(-i gamma Z(x)Z): diagonal with phase exp(-i gamma z0 z1)."""
    d = []
    for idx in range(4):
        z0 = 1 - 2 * (idx & 1)
        z1 = 1 - 2 * ((idx >> 1) & 1)
        d.append(np.exp(-1j * gamma * z0 * z1))
    return np.diag(d).astype(np.complex128)


@dataclass
class Gate:
    name: str
    qubits: Tuple[int, ...]
    mat: np.ndarray
    sub: Optional[int] = None


@dataclass
class Circuit:
    n: int
    gates: List[Gate]
    n_sub: int
    # subcircuit that holds a qubit line carrying no gate at all
    idle_sub: List[int] = field(default_factory=list)
    family: str = ""
    meta: dict = field(default_factory=dict)


def attach_single_qubit_gates(n: int, gates: List[Gate]) -> None:
    """Give every unassigned single-qubit gate the subcircuit of a neighbouring
    two-qubit gate on its line: the preceding one if there is one, otherwise the
    following one (Sec. 5: single-qubit gates follow their closest two-qubit
    neighbour)."""
    last2q: List[Optional[int]] = [None] * n
    pending: List[List[Gate]] = [[] for _ in range(n)]
    for g in gates:
        if len(g.qubits) == 2:
            for q in g.qubits:
                for p in pending[q]:
                    p.sub = g.sub
                pending[q] = []
                last2q[q] = g.sub
        elif g.sub is None:
            q = g.qubits[0]
            if last2q[q] is not None:
                g.sub = last2q[q]
            else:
                pending[q].append(g)
    for q in range(n):
        if pending[q]:
            raise ValueError(f"qubit {q} has single-qubit gates but no two-qubit gate")


# --------------------------------------------------------------------------
# Random brickwork with a moving-boundary partition
# --------------------------------------------------------------------------

def brickwork(n: int, n_layers: int, seed: int,
              schedule: Sequence[Sequence[int]]) -> Circuit:
    """Random brickwork circuit: each layer is a single-qubit layer of seeded
    sqrt(X), sqrt(Y), sqrt(W) gates (never the same gate twice in a row on a
    qubit) followed by CZ on the pairs (i, i+1) with i = layer (mod 2).

    ``schedule[t]`` is the sorted list of block boundaries at layer ``t``:
    subcircuit ``k`` owns qubits ``[b[k-1], b[k])`` during layer ``t``.  Every
    gate of layer ``t`` goes to the owner of its qubits; a CZ that straddles a
    boundary is dropped (boundary thinning), so every cut comes from a boundary
    moving between layers, one cut per qubit line that changes owner.
    """
    if len(schedule) != n_layers:
        raise ValueError("schedule needs one boundary list per layer")
    rng = np.random.default_rng(seed)
    n_sub = len(schedule[0]) + 1
    prev = [-1] * n
    gates: List[Gate] = []

    def owner(t: int, q: int) -> int:
        k = 0
        for b in schedule[t]:
            if q >= b:
                k += 1
        return k

    dropped = 0
    for t in range(n_layers):
        for q in range(n):
            choices = [c for c in range(3) if c != prev[q]]
            c = int(choices[rng.integers(len(choices))])
            prev[q] = c
            name, mat = SQRT_GATES[c]
            gates.append(Gate(name, (q,), mat, owner(t, q)))
        for i in range(t % 2, n - 1, 2):
            oa, ob = owner(t, i), owner(t, i + 1)
            if oa != ob:
                dropped += 1
                continue
            gates.append(Gate("cz", (i, i + 1), CZ, oa))
    return Circuit(n=n, gates=gates, n_sub=n_sub,
                   idle_sub=[owner(0, q) for q in range(n)],
                   family="brickwork",
                   meta={"layers": n_layers, "seed": seed, "dropped_cz": dropped,
                         "schedule": [list(s) for s in schedule]})


def moving_boundary_schedule(n_layers: int, start: Sequence[int],
                             end: Sequence[int]) -> List[List[int]]:
    """A per-layer boundary schedule where boundary ``k`` moves one qubit per
    layer from ``start[k]`` towards ``end[k]``, as late as possible, holding
    still at layer 0 when that avoids a straddling CZ."""
    sched = []
    for t in range(n_layers):
        row = []
        for s, e in zip(start, end):
            moves = abs(s - e)
            if moves > n_layers - 1:
                raise ValueError("boundary must move at most once per layer")
            step = -1 if e < s else 1
            done = max(0, t - (n_layers - 1 - moves))
            row.append(s + step * done)
        sched.append(row)
    return sched


# --------------------------------------------------------------------------
# p=1 QAOA on a planted-partition 3-regular graph
# --------------------------------------------------------------------------

def random_3_regular(nv: int, rng: np.random.Generator) -> List[Tuple[int, int]]:
    """Seeded simple 3-regular graph on ``nv`` vertices (configuration model
    with rejection)."""
    if nv % 2 or nv < 4:
        raise ValueError("3-regular graph needs an even vertex count >= 4")
    for _ in range(10000):
        stubs = np.repeat(np.arange(nv), 3)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        edges = set()
        ok = True
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b:
                ok = False
                break
            e = (min(a, b), max(a, b))
            if e in edges:
                ok = False
                break
            edges.add(e)
        if ok:
            return sorted(edges)
    raise RuntimeError("could not draw a simple 3-regular graph")


def planted_qaoa(sizes: Sequence[int], seed: int,
                 swaps_per_pair: int = 1) -> Circuit:
    """p=1 QAOA (H layer, exp(-i gamma Z_u Z_v) per edge, RX(2 beta) layer,
    gamma, beta ~ U[0, pi]) on a 3-regular graph made of random 3-regular
    communities joined in a ring: between ring neighbours (k, k+1), one
    double-edge swap per ``swaps_per_pair`` replaces an internal edge of each
    community by two cross edges, keeping every degree at 3.

    Cross-edge gates of the pair (k, k+1) are placed in subcircuit ``k`` and are
    the last two-qubit gate on the visiting qubit of community ``k+1``, so each
    cross edge costs exactly one wire cut (from k+1 into k).  Each subcircuit
    therefore has 2*swaps in-cuts and 2*swaps out-cuts.
    """
    rng = np.random.default_rng(seed)
    nc = len(sizes)
    if nc < 3:
        raise ValueError("planted ring needs at least 3 communities")
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    comm_edges = []
    for k, s in enumerate(sizes):
        es = random_3_regular(int(s), rng)
        comm_edges.append([(a + offs[k], b + offs[k]) for a, b in es])
    used_vertices = [set() for _ in range(nc)]
    cross = []  # (host_vertex in k, visitor_vertex in k+1, host community k)
    for k in range(nc):
        k2 = (k + 1) % nc
        for _ in range(swaps_per_pair):
            def pick(c):
                cand = [e for e in comm_edges[c]
                        if e[0] not in used_vertices[c] and e[1] not in used_vertices[c]]
                if not cand:
                    raise RuntimeError("no vertex-disjoint edge left for a swap")
                e = cand[int(rng.integers(len(cand)))]
                comm_edges[c].remove(e)
                used_vertices[c].update(e)
                return e
            a1, a2 = pick(k)
            b1, b2 = pick(k2)
            cross.append((a1, b1, k))
            cross.append((a2, b2, k))
    n = int(offs[-1])
    comm_of = np.zeros(n, dtype=int)
    for k in range(nc):
        comm_of[offs[k]:offs[k + 1]] = k
    gamma = float(rng.uniform(0, np.pi))
    beta = float(rng.uniform(0, np.pi))
    gates: List[Gate] = []
    for q in range(n):
        gates.append(Gate("h", (q,), H, None))
    for k in range(nc):
        for (u, v) in comm_edges[k]:
            gates.append(Gate("zz", (u, v), zz_phase(gamma), k))
    for (u, v, k) in cross:
        gates.append(Gate("zz", (u, v), zz_phase(gamma), k))
    for q in range(n):
        gates.append(Gate("rx", (q,), rx(2 * beta), None))
    attach_single_qubit_gates(n, gates)
    return Circuit(n=n, gates=gates, n_sub=nc, idle_sub=list(comm_of),
                   family="qaoa",
                   meta={"sizes": list(sizes), "seed": seed, "gamma": gamma,
                         "beta": beta, "cross": [(int(a), int(b)) for a, b, _ in cross]})


# --------------------------------------------------------------------------
# Bernstein-Vazirani (single solution state), cut along the ancilla line
# --------------------------------------------------------------------------

def bernstein_vazirani(n_data: int, n_blocks: int, seed: int) -> Circuit:
    """BV with a seeded hidden string: data qubits 0..n_data-1, ancilla qubit
    n_data prepared in |-> and returned to |1> by a final H.  The output is the
    single basis state (s, 1).  Data qubits are split into ``n_blocks``
    contiguous blocks; each block's CNOTs, and the ancilla segment between them,
    form one subcircuit, so the ancilla line is cut once per block boundary."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, 2, size=n_data)
    anc = n_data
    n = n_data + 1
    bounds = np.linspace(0, n_data, n_blocks + 1).round().astype(int)
    block_of = np.zeros(n_data, dtype=int)
    for b in range(n_blocks):
        if bounds[b + 1] <= bounds[b]:
            raise ValueError("every block needs at least one data qubit")
        block_of[bounds[b]:bounds[b + 1]] = b
        # every block holds at least one CNOT so the ancilla visits it
        if not s[bounds[b]:bounds[b + 1]].any():
            s[bounds[b] + int(rng.integers(bounds[b + 1] - bounds[b]))] = 1
    gates: List[Gate] = []
    gates.append(Gate("x", (anc,), PX, None))
    gates.append(Gate("h", (anc,), H, None))
    for q in range(n_data):
        gates.append(Gate("h", (q,), H, int(block_of[q])))
    # blocks that actually hold a CNOT, in order
    for q in range(n_data):
        if s[q]:
            gates.append(Gate("cx", (q, anc), CNOT, int(block_of[q])))
    for q in range(n_data):
        gates.append(Gate("h", (q,), H, int(block_of[q])))
    gates.append(Gate("h", (anc,), H, None))
    attach_single_qubit_gates(n, gates)
    solution = int(sum(int(s[q]) << q for q in range(n_data)) | (1 << anc))
    idle = [int(block_of[q]) for q in range(n_data)] + [n_blocks - 1]
    return Circuit(n=n, gates=gates, n_sub=n_blocks, idle_sub=idle,
                   family="bv", meta={"hidden": [int(v) for v in s],
                                      "solution": solution, "seed": seed})
