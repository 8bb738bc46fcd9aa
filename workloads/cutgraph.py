"""Compute graph of a cut circuit (paper Sec. 5, Fig. 3d).

Given a circuit whose gates each carry a subcircuit id, every qubit line is
split into maximal runs of consecutive gates in one subcircuit (segments).  Each
segment is one wire of that subcircuit; the boundary between two consecutive
segments of a line is one cut edge, directed from the earlier (upstream,
measured) subcircuit to the later (downstream, initialised) one.

Conventions shared with the library's C interface:

* wire ``t`` of a subcircuit is bit ``t`` of its measured outcome index;
  out-cut wires come first (ordered by qubit), then the data wires (wires that
  end in a circuit output, ordered by qubit);
* data bit ``j`` of a subcircuit is wire ``data_wire[j]`` and carries original
  qubit ``data_qubit[j]``;
* the cuts incident to a subcircuit are taken in the order of the global cut
  list; the first incident cut is the least significant digit of both the
  variant index and the cut-label index.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

from .circuits import Circuit


@dataclass
class Wire:
    qubit: int
    seg: int
    start: object  # "input" or the id of the cut it is initialised from
    end: object    # "output" or the id of the cut it is measured into


@dataclass
class Subcircuit:
    wires: List[Wire]
    gates: List[Tuple[np.ndarray, Tuple[int, ...]]]  # (unitary, wire indices)
    data_wire: List[int]
    data_qubit: List[int]

    @property
    def n_wires(self) -> int:
        return len(self.wires)

    @property
    def n_data(self) -> int:
        return len(self.data_wire)


@dataclass
class Cut:
    up_sub: int
    up_wire: int
    down_sub: int
    down_wire: int
    qubit: int


@dataclass
class CutCircuit:
    circuit: Circuit
    subs: List[Subcircuit]
    cuts: List[Cut]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.circuit.n

    @property
    def n_sub(self) -> int:
        return len(self.subs)

    def incident(self, i: int) -> List[Tuple[int, str]]:
        """(cut id, 'in' | 'out') for every cut touching subcircuit ``i``, in
        global cut order."""
        out = []
        for k, c in enumerate(self.cuts):
            if c.down_sub == i:
                out.append((k, "in"))
            elif c.up_sub == i:
                out.append((k, "out"))
        return out

    def n_variants(self, i: int) -> int:
        v = 1
        for _, role in self.incident(i):
            v *= 4 if role == "in" else 3
        return v

    def degree(self, i: int) -> int:
        return len(self.incident(i))

    def summary(self) -> dict:
        return {
            "n": self.n,
            "n_sub": self.n_sub,
            "K": len(self.cuts),
            "w": [s.n_wires for s in self.subs],
            "d": [s.n_data for s in self.subs],
            "c": [self.degree(i) for i in range(self.n_sub)],
            "V": [self.n_variants(i) for i in range(self.n_sub)],
        }


def build_cut_circuit(circ: Circuit) -> CutCircuit:
    """Derive subcircuit wires, gates and cut edges from the gate assignment."""
    n = circ.n
    # segments per qubit: list of (sub, [gate indices])
    segs: List[List[Tuple[int, List[int]]]] = [[] for _ in range(n)]
    for gi, g in enumerate(circ.gates):
        if g.sub is None:
            raise ValueError(f"gate {gi} ({g.name}) has no subcircuit")
        for q in g.qubits:
            if segs[q] and segs[q][-1][0] == g.sub:
                segs[q][-1][1].append(gi)
            else:
                segs[q].append((g.sub, [gi]))
    for q in range(n):
        if not segs[q]:
            segs[q].append((circ.idle_sub[q], []))

    # cuts in (qubit, segment) order
    cuts_raw = []  # (qubit, seg index of upstream)
    for q in range(n):
        for j in range(len(segs[q]) - 1):
            cuts_raw.append((q, j))
    cut_id = {key: k for k, key in enumerate(cuts_raw)}

    n_sub = circ.n_sub
    sub_wires: List[List[Wire]] = [[] for _ in range(n_sub)]
    for q in range(n):
        L = len(segs[q])
        for j, (s, _) in enumerate(segs[q]):
            start = "input" if j == 0 else cut_id[(q, j - 1)]
            end = "output" if j == L - 1 else cut_id[(q, j)]
            sub_wires[s].append(Wire(q, j, start, end))
    # order: out-cut wires first, then data wires, each by (qubit, seg)
    wire_index = {}
    subs: List[Subcircuit] = []
    for s in range(n_sub):
        ws = sub_wires[s]
        outs = sorted([w for w in ws if w.end != "output"], key=lambda w: (w.qubit, w.seg))
        datas = sorted([w for w in ws if w.end == "output"], key=lambda w: (w.qubit, w.seg))
        ordered = outs + datas
        for t, w in enumerate(ordered):
            wire_index[(w.qubit, w.seg)] = (s, t)
        data_wire = [len(outs) + j for j in range(len(datas))]
        data_qubit = [w.qubit for w in datas]
        subs.append(Subcircuit(wires=ordered, gates=[], data_wire=data_wire,
                               data_qubit=data_qubit))
    # gates in time order, mapped to wire indices
    seg_of_gate_on_q = {}
    for q in range(n):
        for j, (_, gl) in enumerate(segs[q]):
            for gi in gl:
                seg_of_gate_on_q[(gi, q)] = j
    for gi, g in enumerate(circ.gates):
        wires = []
        for q in g.qubits:
            s, t = wire_index[(q, seg_of_gate_on_q[(gi, q)])]
            assert s == g.sub
            wires.append(t)
        subs[g.sub].gates.append((g.mat, tuple(wires)))
    cuts: List[Cut] = []
    for (q, j) in cuts_raw:
        su, tu = wire_index[(q, j)]
        sd, td = wire_index[(q, j + 1)]
        if su == sd:
            raise ValueError("a cut must join two different subcircuits")
        cuts.append(Cut(up_sub=su, up_wire=tu, down_sub=sd, down_wire=td, qubit=q))
    for s, sub in enumerate(subs):
        if sub.n_wires == 0:
            raise ValueError(f"subcircuit {s} is empty")
    return CutCircuit(circuit=circ, subs=subs, cuts=cuts)
