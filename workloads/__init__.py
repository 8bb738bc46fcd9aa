"""Seeded synthetic cut-circuit workloads.

This package is the input side shared by the GPU path's tests and benchmark and
by the CPU oracle's tests.  It holds no post-processing arithmetic (no
attribution, merging, contraction or bin search).  It provides:

* ``circuits``  -- seeded circuit generators shaped like the paper's benchmark
  families (random brickwork "Supremacy"-like circuits, p=1 QAOA on 3-regular
  graphs, Bernstein-Vazirani) together with a gate-to-subcircuit assignment;
* ``cutgraph``  -- derivation of the compute graph (subcircuit wires, data
  qubits and cut edges) from a gate-to-subcircuit assignment, following the
  paper's gate-DAG view (Sec. 5: single-qubit gates follow their two-qubit
  neighbours, every change of subcircuit along a qubit line is one cut);
* ``qpu``       -- the stand-in for the quantum processors: it runs every
  variant of a subcircuit (each upstream cut measured in the Z, X or Y basis,
  each downstream cut initialised in |0>, |1>, |+> or |+i>, Fig. 1) by
  statevector simulation and returns measured probability vectors, or seeded
  random outputs (Sec. 7.1 uses random numbers for the subcircuit outputs);
* ``configs``   -- the five named workloads (tiny, precision, merging, serving
  pool, large chain) built from the above.
"""
