"""Error metrics used to compare a result with the oracle (test infrastructure only).

The method's result is exact up to rounding (Algorithm 1 computes a fixed
matrix and vector, global phase included), so amplitudes are compared
directly.  Fidelity is phase-blind by definition and is reported beside them.
"""
from __future__ import annotations

import numpy as np


def max_abs_diff(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.size(a) else 0.0


def fidelity(psi, ref) -> float:
    """|<ref|psi>|^2 / (<psi|psi><ref|ref>), accumulated in float64/complex128."""
    psi = np.asarray(psi, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    num = abs(np.vdot(ref, psi)) ** 2
    den = np.vdot(psi, psi).real * np.vdot(ref, ref).real
    return float(num / den)


def unitarity_drift(U) -> tuple:
    """(max |U^H U - I|, ||U^H U - I||_F / sqrt(N)) in complex128 (Section 2.3: U^H = U^{-1})."""
    U = np.asarray(U, dtype=np.complex128)
    D = U.conj().T @ U - np.eye(U.shape[0])
    return float(np.max(np.abs(D))), float(np.linalg.norm(D) / np.sqrt(U.shape[0]))
