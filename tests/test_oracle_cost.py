"""Pins of the oracle's cost model against the numbers printed in the paper's
worked example (fixture tests/golden/cost_example.json)."""
import json
import os

from oracle import cost

HERE = os.path.dirname(os.path.abspath(__file__))
EX = json.load(open(os.path.join(HERE, "golden", "cost_example.json")))


def graph_tensors():
    qubits = EX["graph"]["qubits"]
    cuts = EX["graph"]["cuts"]
    ts = []
    for i, q in enumerate(qubits):
        ids = frozenset(k for k, (a, b) in enumerate(cuts) if i in (a, b))
        ts.append((ids, 2 ** q))
    return ts


def test_input_floats():
    assert cost.input_floats(graph_tensors()) == EX["input_floats"]


def test_step_costs():
    steps, total = cost.plan_cost(graph_tensors(), [tuple(p) for p in EX["order"]])
    assert [s["mults"] for s in steps] == EX["step_mults"]
    assert steps[1]["operand_floats"] == EX["step2_operand_floats"]


def test_naive_and_ratio():
    ts = graph_tensors()
    naive = cost.naive_mults(len(EX["graph"]["cuts"]), [t[1] for t in ts])
    assert naive == EX["naive_mults"]
    _, total = cost.plan_cost(ts, [tuple(p) for p in EX["order"]])
    assert round(naive / total, 1) == EX["naive_over_plan"]


def test_slicing_one_edge():
    ts = graph_tensors()
    chosen = cost.greedy_slices(ts, EX["sliced_input_floats"])
    assert len(chosen) == 1
    assert 4 ** len(chosen) == EX["sliced_subgraphs"]
    assert cost.input_floats(cost.slice_edge(ts, chosen[0])) == EX["sliced_input_floats"]
    # the slice chosen is one of the two parallel 1-3 edges
    assert tuple(EX["graph"]["cuts"][chosen[0]]) == (0, 2)
