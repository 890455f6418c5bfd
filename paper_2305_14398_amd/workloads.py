"""Seeded synthetic circuits: the inputs shared by the HIP path and the oracle.

This module only builds *gate lists* (a gate name, the qubits it touches and,
for rotations and phase gates, an angle).  It holds none of the simulation
arithmetic: no gate matrices, no step operators, no products.  Both sides of
every parity check (the HIP library through the binding, and the CPU oracle)
receive the same plain list and turn it into numbers with their own code.

Qubit convention: little-endian.  Qubit 0 is the least significant bit of a
basis-state index, so |q_{n-1} ... q_1 q_0> has index sum(q_j * 2**j).  This is
the reading under which the paper's QFT figure (Section 2.5, "Quantum Fourier
Transform") computes the discrete Fourier transform; its Bell worked example
(Section 2.4, Eq. 9-11) is convention-invariant.

Gate names (paper Section 2.3, Table 1 and Eq. 7-8; Section 5.2.2 for S, T and
the arbitrary phase gate R):
  one-qubit : H, X, Y, Z, S, T, R(phi), RX(theta), RY(theta), RZ(theta)
  two-qubit : CNOT(c, t), CY(c, t), CZ(c, t), CR(c, t, phi), SWAP(a, b)
For a controlled gate ``qubits == (control, target)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

ONE_QUBIT = ("H", "X", "Y", "Z", "S", "T", "R", "RX", "RY", "RZ")
TWO_QUBIT = ("CNOT", "CY", "CZ", "CR", "SWAP")
ANGLED = ("R", "RX", "RY", "RZ", "CR")
# Largest register: the full-state-vector path (a 2^34 complex64 state); the
# unitary path itself stops at 16.
MAX_QUBITS = 34
# Random-layer gate set, in the order used to index the uniform draw.
RANDOM_1Q = ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ")


@dataclass(frozen=True)
class Gate:
    name: str
    qubits: Tuple[int, ...]
    theta: Optional[float] = None

    def __post_init__(self):
        if self.name in ONE_QUBIT:
            if len(self.qubits) != 1:
                raise ValueError(f"{self.name} takes one qubit, got {self.qubits}")
        elif self.name in TWO_QUBIT:
            if len(self.qubits) != 2 or self.qubits[0] == self.qubits[1]:
                raise ValueError(f"{self.name} takes two distinct qubits, got {self.qubits}")
        else:
            raise ValueError(f"unknown gate {self.name!r}")
        if (self.name in ANGLED) != (self.theta is not None):
            raise ValueError(f"{self.name}: angle {'required' if self.name in ANGLED else 'not allowed'}")

    @property
    def span(self) -> Tuple[int, int]:
        return (min(self.qubits), max(self.qubits))


@dataclass
class Circuit:
    """An ordered gate list over ``n`` qubits (the paper's Circuit(n), Section 5.2.1)."""

    n: int
    gates: List[Gate]
    family: str = "custom"

    def __post_init__(self):
        if not (1 <= self.n <= MAX_QUBITS):
            raise ValueError(f"qubit count {self.n} outside 1..{MAX_QUBITS}")
        for g in self.gates:
            for q in g.qubits:
                if not (0 <= q < self.n):
                    raise ValueError(f"gate {g} touches qubit {q} outside 0..{self.n - 1}")

    # builder methods in the style of the paper's circuit model (Listing "belltornado")
    def _add(self, name, qubits, theta=None):
        g = Gate(name, tuple(int(q) for q in qubits), None if theta is None else float(theta))
        for q in g.qubits:
            if not (0 <= q < self.n):
                raise ValueError(f"qubit {q} outside 0..{self.n - 1}")
        self.gates.append(g)
        return self

    def H(self, q): return self._add("H", (q,))
    def X(self, q): return self._add("X", (q,))
    def Y(self, q): return self._add("Y", (q,))
    def Z(self, q): return self._add("Z", (q,))
    def S(self, q): return self._add("S", (q,))
    def T(self, q): return self._add("T", (q,))
    def R(self, q, phi): return self._add("R", (q,), phi)
    def RX(self, q, t): return self._add("RX", (q,), t)
    def RY(self, q, t): return self._add("RY", (q,), t)
    def RZ(self, q, t): return self._add("RZ", (q,), t)
    def CNOT(self, c, t): return self._add("CNOT", (c, t))
    def CY(self, c, t): return self._add("CY", (c, t))
    def CZ(self, c, t): return self._add("CZ", (c, t))
    def CR(self, c, t, phi): return self._add("CR", (c, t), phi)
    def SWAP(self, a, b): return self._add("SWAP", (a, b))


def new(n: int, family: str = "custom") -> Circuit:
    return Circuit(n, [], family)


# --- families ---------------------------------------------------------------

def bell() -> Circuit:
    """H on qubit 0, then CNOT(0 -> 1) (Section 2.4, Bell-state figure and Listing 'belltornado')."""
    return new(2, "bell").H(0).CNOT(0, 1)


def ghz_chain(n: int) -> Circuit:
    """H(0), then CNOT(i -> i+1) for i = 0..n-2: the nearest-neighbour entangling chain."""
    c = new(n, "ghz_chain").H(0)
    for i in range(n - 1):
        c.CNOT(i, i + 1)
    return c


def ghz_fanout(n: int) -> Circuit:
    """Fully entangled circuit of Section 2.5: H(0), then CNOT(0 -> j) for j = n-1 down to 1."""
    c = new(n, "ghz_fanout").H(0)
    for j in range(n - 1, 0, -1):
        c.CNOT(0, j)
    return c


def dj(n: int, mask: int) -> Circuit:
    """Deutsch-Jozsa (Section 2.5, Deutsch-Jozsa figure) with the oracle f(x) = parity(mask & x).

    Qubit n-1 is the ancilla, qubits 0..n-2 the function inputs.  The ancilla
    starts in |1> in the figure; here an X gate prepares it so that every family
    starts from |0...0>.  The oracle U_f is one CNOT(i -> ancilla) per set bit
    of ``mask`` (ascending i); mask = 0 is the constant function f = 0, any
    nonzero mask a balanced one.
    """
    if n < 2:
        raise ValueError("Deutsch-Jozsa needs at least one input qubit and the ancilla")
    if not (0 <= mask < (1 << (n - 1))):
        raise ValueError(f"mask {mask} does not fit {n - 1} input bits")
    a = n - 1
    c = new(n, "dj").X(a)
    for q in range(n):
        c.H(q)
    for i in range(n - 1):
        if (mask >> i) & 1:
            c.CNOT(i, a)
    for q in range(n - 1):
        c.H(q)
    return c


def qft(n: int) -> Circuit:
    """QFT in the pattern of Section 2.5's QFT figure, generalised to n qubits.

    For j = n-1 down to 0: H(j), then a controlled phase R_phi with
    phi = pi / 2**(j - i) from each lower qubit i = 0..j-1 onto j.  Then
    SWAP(i, n-1-i) for i < n // 2.
    """
    c = new(n, "qft")
    for j in range(n - 1, -1, -1):
        c.H(j)
        for i in range(j):
            c.CR(i, j, math.pi / (1 << (j - i)))
    for i in range(n // 2):
        c.SWAP(i, n - 1 - i)
    return c


def random_layers(n: int, depth: int, rng: np.random.Generator) -> Circuit:
    """Seeded random layered circuit (not in the paper; the precision-sweep workload).

    Per layer, in this draw order:
      1. kinds = rng.integers(0, 9, size=n): qubit q gets RANDOM_1Q[kinds[q]];
      2. for q = 0..n-1 whose gate is RX/RY/RZ: theta = rng.uniform(0, 2*pi);
      3. perm = rng.permutation(n); coins = rng.random(n // 2);
         pair i is (perm[2i], perm[2i+1]): CNOT(perm[2i] -> perm[2i+1]) if
         coins[i] < 0.5, else CZ(perm[2i], perm[2i+1]).
    """
    c = new(n, "random")
    for _ in range(depth):
        kinds = rng.integers(0, len(RANDOM_1Q), size=n)
        for q in range(n):
            name = RANDOM_1Q[int(kinds[q])]
            if name in ("RX", "RY", "RZ"):
                c._add(name, (q,), rng.uniform(0.0, 2.0 * math.pi))
            else:
                c._add(name, (q,))
        perm = rng.permutation(n)
        coins = rng.random(n // 2)
        for i in range(n // 2):
            a, b = int(perm[2 * i]), int(perm[2 * i + 1])
            if coins[i] < 0.5:
                c.CNOT(a, b)
            else:
                c.CZ(a, b)
    return c


def adjoint_gate(g: Gate) -> Gate:
    """Name/angle of the inverse gate (H, X, Y, Z, CNOT, CY, CZ, SWAP are their own inverses)."""
    if g.name in ("H", "X", "Y", "Z", "CNOT", "CY", "CZ", "SWAP"):
        return g
    if g.name == "S":
        return Gate("R", g.qubits, -math.pi / 2)
    if g.name == "T":
        return Gate("R", g.qubits, -math.pi / 4)
    return Gate(g.name, g.qubits, -g.theta)


def mirror(c: Circuit) -> Circuit:
    """The circuit followed by its inverse (adjoint gates in reverse order): its unitary is I."""
    return Circuit(c.n, list(c.gates) + [adjoint_gate(g) for g in reversed(c.gates)], c.family + "_mirror")


def dj_mask(n: int, seed: int) -> int:
    """Seeded balanced Deutsch-Jozsa mask: a uniformly drawn nonzero (n-1)-bit integer."""
    return int(np.random.default_rng(seed).integers(1, 1 << (n - 1)))


MIXED_FAMILIES = ("ghz_chain", "dj", "qft", "random")


def mixed(rng: np.random.Generator, n_lo: int, n_hi: int, d_lo: int, d_hi: int) -> Circuit:
    """One draw of the mixed-family workload: n ~ U{n_lo..n_hi}, family ~ U{MIXED_FAMILIES},
    depth ~ U{d_lo..d_hi} (random layers only; the structured families use their natural size)."""
    n = int(rng.integers(n_lo, n_hi + 1))
    fam = MIXED_FAMILIES[int(rng.integers(0, len(MIXED_FAMILIES)))]
    depth = int(rng.integers(d_lo, d_hi + 1))
    if fam == "ghz_chain":
        return ghz_chain(n)
    if fam == "dj":
        if n < 2:  # Deutsch-Jozsa needs an input qubit besides the ancilla
            return ghz_chain(n)
        return dj(n, int(rng.integers(1, 1 << (n - 1))))
    if fam == "qft":
        return qft(n)
    return random_layers(n, depth, rng)


def batch_mixed(count: int, seed: int, n_lo: int = 4, n_hi: int = 11, d_lo: int = 5, d_hi: int = 30) -> List[Circuit]:
    rng = np.random.default_rng(seed)
    return [mixed(rng, n_lo, n_hi, d_lo, d_hi) for _ in range(count)]


def poisson_trace(count: int, rate_hz: float, seed: int, n_lo: int = 6, n_hi: int = 13,
                  d_lo: int = 10, d_hi: int = 40) -> List[Tuple[float, Circuit]]:
    """Seeded Poisson arrival trace: (arrival time in seconds, circuit) pairs."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    times = np.cumsum(gaps)
    return [(float(t), mixed(rng, n_lo, n_hi, d_lo, d_hi)) for t in times]


def gate_tuples(c: Circuit) -> List[Tuple[str, Tuple[int, ...], Optional[float]]]:
    """The plain (name, qubits, theta) list: the only form the oracle consumes."""
    return [(g.name, g.qubits, g.theta) for g in c.gates]


def random_state(n: int, seed: int) -> np.ndarray:
    """A seeded normalised complex128 vector of length 2**n (an arbitrary initial state)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def random_columns(n: int, count: int, seed: int) -> np.ndarray:
    """Seeded distinct column indices (always including column 0) for sampled checks."""
    N = 1 << n
    rng = np.random.default_rng(seed)
    k = min(count, N)
    cols = rng.choice(N, size=k, replace=False)
    if 0 not in cols:
        cols[0] = 0
    return np.sort(cols)


def random_unitary(m: int, seed: int) -> np.ndarray:
    """A seeded Haar-random 2^m x 2^m unitary (QR of a complex Gaussian matrix with the phases of R's
    diagonal divided out): the data of a custom operation on m qubits."""
    rng = np.random.default_rng(seed)
    D = 1 << m
    z = (rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def with_custom_ops(gates, n: int, m_values, seed: int):
    """Insert custom operations (name, range, None, matrix) on random ranges into a gate list at seeded
    positions; returns the new list (oracle form, 4-tuples for the custom operations)."""
    rng = np.random.default_rng(seed)
    out = list(gates)
    for i, m in enumerate(m_values):
        if m > n:
            continue
        a = int(rng.integers(0, n - m + 1))
        pos = int(rng.integers(0, len(out) + 1))
        out.insert(pos, (f"custom{m}_{seed}_{i}", tuple(range(a, a + m)), None, random_unitary(m, seed * 131 + i)))
    return out
