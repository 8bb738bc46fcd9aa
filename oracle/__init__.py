"""CPU FP64 oracle for cut-circuit reconstruction (ScaleQC, arXiv 2207.00933).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg import this package.  The GPU library never calls it, and it
shares no code with the GPU library: the only code both sides use is the seeded
input generator package ``workloads`` (circuits, compute-graph derivation and
the quantum-processor stand-in), which holds none of the post-processing
arithmetic.

Modules (each function cites the passage it follows):

* ``statevector``     plain full-circuit simulator, the brute-force reference;
* ``reconstruction``  cut-basis attribution, Eq. 1 full-definition
                      reconstruction (with the 2^-K normalisation), merged
                      bins, single-bin evaluation, qubit-order permutation;
* ``states_merging``  Algorithm 2 (states assignment) on explicit state lists
                      and Algorithm 1 (the recursion loop);
* ``cost``            the memory / multiplication model of Sec. 6.2 and the
                      index-slicing size of Sec. 6.3;
* ``network``         a plain pairwise FP64 contraction (numpy einsum) for
                      graphs where Eq. 1's 4^K terms are out of reach.

Readings of passages where the paper is silent or ambiguous are listed in the
repository's design notes and repeated at the function they affect.
Parity status: every function is pinned by a test under ``tests/`` against a
closed form, a brute-force simulation or a number printed in the paper, except
the two list conventions marked "parity unpinned" in ``states_merging``
(Algorithm 2's tie rule and Algorithm 1's list ordering), which any choice
satisfies.
"""
