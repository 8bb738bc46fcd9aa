"""Pins of the cut-search oracle (Sec. 5 model) against values fixed by the
definitions: hand-counted degrees, closed forms, and the constraint."""
import pytest

from oracle import cut_search as cs


def test_edges_of_a_small_circuit():
    # gates on qubits (0,1), (1,2), (0,1), (2,3): qubit lines between
    # consecutive two-qubit gates on a qubit
    gates = [(0, 1), (1, 2), (0, 1), (2, 3)]
    assert sorted(cs.dag_edges(gates)) == [(0, 1), (0, 2), (1, 2), (1, 3)]


def test_degrees_counted_by_hand():
    gates = [(0, 1), (1, 2), (0, 1), (2, 3)]
    e = cs.dag_edges(gates)
    # gates 0, 2 in subcircuit 0; 1, 3 in subcircuit 1: cut edges (0,1),
    # (1,2); (0,2) and (1,3) stay inside
    assert cs.degree([0, 1, 0, 1], e, 2) == [2, 2]
    assert cs.objective([0, 0, 0, 1], e, 2) == 1


def test_two_qubit_chain_needs_two_cuts():
    # k gates on the same pair of qubits: any split into two non-empty
    # subcircuits cuts at least both lines between some neighbours
    for k in (2, 3, 5):
        assert cs.brute_force([(0, 1)] * k, 2, 1.0) == 2


def test_independent_pairs_need_no_cut():
    # disjoint qubit pairs, one subcircuit each: L = 0
    gates = [(0, 1), (2, 3), (0, 1), (2, 3)]
    assert cs.brute_force(gates, 2, 0.5) == 0


def test_load_constraint_binds():
    # with alpha |V| = 1 every gate is its own subcircuit: every edge is cut
    gates = [(0, 1), (1, 2), (0, 1)]
    e = cs.dag_edges(gates)
    best = cs.brute_force(gates, 3, 1.0 / 3)
    assert best == max(max(cs.degree(list(p), e, 3)) for p in [(0, 1, 2)])
    # no feasible partition when alpha |V| < |V| / n_sub
    assert cs.brute_force(gates, 2, 0.4) is None


def test_feasible_requires_every_subcircuit():
    assert not cs.feasible([0, 0, 0], 2, 1.0)
    assert cs.feasible([0, 1, 0], 2, 1.0)
    assert not cs.feasible([0, 0, 1], 2, 0.5)
