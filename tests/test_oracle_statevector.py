"""Pins of the oracle's statevector simulator: closed forms and a dense-matrix
brute force that shares none of its index arithmetic."""
import numpy as np
import pytest

from oracle import statevector as sv
from workloads import circuits as C
from workloads.circuits import Gate


def dense_unitary(n, gates):
    """Whole-circuit unitary from Kronecker products (qubit q = bit q, so the
    kron factor order is qubit n-1 ... qubit 0)."""
    U = np.eye(1 << n, dtype=np.complex128)
    for g in gates:
        if len(g.qubits) == 1:
            mats = [np.eye(2)] * n
            mats = list(mats)
            mats[g.qubits[0]] = g.mat
            G = np.array([[1.0]])
            for q in range(n - 1, -1, -1):
                G = np.kron(G, mats[q])
        else:
            # permutation-free construction: element-wise over basis states
            G = np.zeros((1 << n, 1 << n), dtype=np.complex128)
            q0, q1 = g.qubits
            for col in range(1 << n):
                b0, b1 = (col >> q0) & 1, (col >> q1) & 1
                j = b0 + 2 * b1
                for k in range(4):
                    row = col & ~((1 << q0) | (1 << q1))
                    row |= (k & 1) << q0
                    row |= (k >> 1) << q1
                    G[row, col] += g.mat[k, j]
        U = G @ U
    return U


def test_bell():
    gates = [Gate("h", (0,), C.H), Gate("cx", (0, 1), C.CNOT)]
    P = sv.probabilities(2, gates)
    assert np.allclose(P, [0.5, 0, 0, 0.5], atol=1e-15)


def test_ghz():
    n = 5
    gates = [Gate("h", (0,), C.H)] + [Gate("cx", (q, q + 1), C.CNOT) for q in range(n - 1)]
    P = sv.probabilities(n, gates)
    want = np.zeros(1 << n)
    want[0] = want[-1] = 0.5
    assert np.allclose(P, want, atol=1e-15)


def test_hadamard_layer_uniform():
    n = 7
    P = sv.probabilities(n, [Gate("h", (q,), C.H) for q in range(n)])
    assert np.allclose(P, 1.0 / (1 << n), atol=1e-15)


def test_sqrt_gates_square_to_pauli():
    for name, mat, pauli in (("sx", C.SQRT_X, C.PX), ("sy", C.SQRT_Y, C.PY), ("sw", C.SQRT_W, C.PW)):
        M = mat @ mat
        # equal up to a global phase
        ph = M[np.unravel_index(np.argmax(np.abs(M)), M.shape)] / pauli[np.unravel_index(np.argmax(np.abs(M)), M.shape)]
        assert np.allclose(M, ph * pauli, atol=1e-15), name
        assert np.allclose(mat @ mat.conj().T, np.eye(2), atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_against_dense_unitary(seed):
    n = 5
    sched = [[5]] * 4
    circ = C.brickwork(n, 4, seed, sched)
    rng = np.random.default_rng(seed)
    # add a non-symmetric two-qubit gate in both orientations
    circ.gates.append(Gate("cx", (3, 1), C.CNOT))
    circ.gates.append(Gate("zz", (0, 4), C.zz_phase(rng.uniform(0, np.pi))))
    psi = sv.amplitudes(n, circ.gates)
    U = dense_unitary(n, circ.gates)
    assert np.allclose(psi, U[:, 0], atol=1e-13)


def test_norm_and_inverse():
    n = 9
    circ = C.brickwork(n, 6, 7, [[n]] * 6)
    psi = sv.amplitudes(n, circ.gates)
    assert abs(np.vdot(psi, psi) - 1) < 1e-13
    inv = [Gate(g.name, g.qubits, g.mat.conj().T) for g in reversed(circ.gates)]
    back = sv.amplitudes(n, circ.gates + inv)
    want = np.zeros(1 << n)
    want[0] = 1
    assert np.allclose(back, want, atol=1e-13)
