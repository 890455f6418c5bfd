"""Route B: gate-by-gate application to state vectors (oracle; test infrastructure only).

Each one-qubit gate U = [[Ua, Ub], [Uc, Ud]] on qubit i updates every pair of
amplitudes whose indices differ only in bit i (Appendix A, Eq. 12):
    a[..0_i..] <- Ua a[..0_i..] + Ub a[..1_i..]
    a[..1_i..] <- Uc a[..0_i..] + Ud a[..1_i..]
A controlled gate applies that update only to the pairs whose control bit is 1
(Eq. 7); SWAP exchanges the amplitudes whose bits a and b differ.  A custom
operation M on the range a..a+m-1 (Section 5.2.2) maps, for every fixed value
of the other bits, the 2^m amplitudes indexed by the range bits by M.  Applied to
the columns of the identity this yields the circuit unitary column by column
(U[:, j] = C e_j) without building any step operator, so it is independent of
route A's Kronecker construction and of step formation.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from . import gates as G


def _pair_update(v: np.ndarray, q: int, U: np.ndarray, ctrl: int = -1) -> np.ndarray:
    """Eq. 12 on bit q of the row index of v (shape (N, m)), optionally gated by bit ctrl."""
    N = v.shape[0]
    idx = np.arange(N)
    i0 = idx[((idx >> q) & 1) == 0]
    if ctrl >= 0:
        i0 = i0[((i0 >> ctrl) & 1) == 1]
    i1 = i0 | (1 << q)
    a0 = v[i0].copy()
    a1 = v[i1].copy()
    v[i0] = U[0, 0] * a0 + U[0, 1] * a1
    v[i1] = U[1, 0] * a0 + U[1, 1] * a1
    return v


def _range_update(v: np.ndarray, a: int, M: np.ndarray) -> np.ndarray:
    """Amplitude index i = (hi * 2^m + mid) * 2^a + lo; new[hi, r, lo] = sum_s M[r, s] v[hi, s, lo]."""
    N, cols = v.shape
    W = M.shape[0]
    v4 = v.reshape(N // (W << a), W, 1 << a, cols)
    return np.einsum("rs,hslc->hrlc", M, v4).reshape(N, cols)


def apply_gate(v: np.ndarray, g) -> np.ndarray:
    name, qubits, theta = g[0], g[1], g[2]
    if len(g) == 4:
        if list(qubits) != list(range(min(qubits), max(qubits) + 1)):
            raise ValueError("a custom operation acts on a contiguous ascending range of qubits")
        M = np.asarray(g[3], dtype=np.complex128)
        if M.shape != (1 << len(qubits),) * 2:
            raise ValueError("custom matrix size does not match its qubit range")
        return _range_update(v, qubits[0], M)
    if len(qubits) == 1:
        return _pair_update(v, qubits[0], G.one_qubit(name, theta))
    if name == "SWAP":
        a, b = qubits
        idx = np.arange(v.shape[0])
        ba, bb = (idx >> a) & 1, (idx >> b) & 1
        perm = idx ^ ((ba ^ bb) << a) ^ ((ba ^ bb) << b)
        return v[perm]
    c, t = qubits
    return _pair_update(v, t, G.controlled_target(name, theta), ctrl=c)


def apply_circuit(n: int, gate_list: Sequence, v: np.ndarray) -> np.ndarray:
    """Apply the gates in order to v, a vector of length 2^n or a (2^n, m) block of columns."""
    v = np.array(v, dtype=np.complex128, copy=True)
    squeeze = v.ndim == 1
    if squeeze:
        v = v[:, None]
    if v.shape[0] != (1 << n):
        raise ValueError("state length does not match qubit count")
    for g in gate_list:
        v = apply_gate(v, g)
    return v[:, 0] if squeeze else v


def unitary_columns(n: int, gate_list: Sequence, cols) -> np.ndarray:
    """Columns `cols` of the circuit unitary, shape (2^n, len(cols))."""
    N = 1 << n
    E = np.zeros((N, len(cols)), dtype=np.complex128)
    E[np.asarray(cols), np.arange(len(cols))] = 1.0
    return apply_circuit(n, gate_list, E)


def circuit_unitary(n: int, gate_list: Sequence) -> np.ndarray:
    return apply_circuit(n, gate_list, np.eye(1 << n, dtype=np.complex128))


def final_state(n: int, gate_list: Sequence, psi0=None) -> np.ndarray:
    N = 1 << n
    if psi0 is None:
        psi0 = np.zeros(N, dtype=np.complex128)
        psi0[0] = 1.0
    return apply_circuit(n, gate_list, psi0)
