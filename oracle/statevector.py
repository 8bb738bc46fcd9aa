"""Plain statevector simulator (the brute-force reference).

Textbook definition: a state of n qubits is a vector of 2^n complex amplitudes,
qubit q is bit q of the index; a gate multiplies the amplitudes of the
sub-space it acts on by its unitary; the output distribution is |psi|^2.
Used only to check reconstructions of whole circuits (the uncut circuit's
output P of Eq. 1, Sec. 2.1).
"""
from __future__ import annotations

import numpy as np


def apply_gate(psi: np.ndarray, n: int, mat: np.ndarray, qubits) -> None:
    """In-place application of a 1- or 2-qubit unitary.  The unitary's basis
    index is bit(qubits[0]) + 2 * bit(qubits[1])."""
    if len(qubits) == 1:
        q = qubits[0]
        v = psi.reshape(1 << (n - q - 1), 2, 1 << q)
        a = v[:, 0, :].copy()
        b = v[:, 1, :].copy()
        v[:, 0, :] = mat[0, 0] * a + mat[0, 1] * b
        v[:, 1, :] = mat[1, 0] * a + mat[1, 1] * b
        return
    q0, q1 = qubits
    lo, hi = min(q0, q1), max(q0, q1)
    v = psi.reshape(1 << (n - hi - 1), 2, 1 << (hi - lo - 1), 2, 1 << lo)
    # amplitudes of the four basis states (bit q0, bit q1)
    def sl(b0, b1):
        bl = b0 if q0 == lo else b1
        bh = b1 if q0 == lo else b0
        return (slice(None), bh, slice(None), bl, slice(None))
    old = [v[sl(k & 1, k >> 1)].copy() for k in range(4)]
    for k in range(4):
        acc = np.zeros_like(old[0])
        for j in range(4):
            if mat[k, j] != 0:
                acc += mat[k, j] * old[j]
        v[sl(k & 1, k >> 1)] = acc


def probabilities(n: int, gates) -> np.ndarray:
    """|<x|U|0...0>|^2 for every x (length 2^n, float64)."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    for g in gates:
        apply_gate(psi, n, g.mat, g.qubits)
    return (psi.real ** 2 + psi.imag ** 2)


def amplitudes(n: int, gates) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    for g in gates:
        apply_gate(psi, n, g.mat, g.qubits)
    return psi
