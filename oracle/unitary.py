"""Route A: the plain unitary-matrix method in complex128 (oracle; test infrastructure only).

Follows the paper's execution flow (Section 5.3, stages 1-6):
  1-3. split the ordered gate list into steps and fetch each operation's data;
  4.   build each step's dense operator by an ordered Kronecker product of the
       step's operands, identities on idle qubits (Algorithm 2; Eq. 9s1);
  5.   result <- A . result over all steps, from result = I (Algorithm 1);
  6.   multiply the circuit unitary by the initial state (Algorithm 1, return).

Qubit order is little-endian (qubit 0 is the least significant index bit), so
the Kronecker operand list runs from qubit n-1 (first, most significant factor)
down to qubit 0.

A two-qubit gate whose qubits are not adjacent becomes one operand over its
whole span [lo, hi] (Section 5.3, the dynamically created non-adjacent
two-qubit matrices).  A controlled gate on the span is built as
P0(control) (x) I + P1(control) (x) U(target), identities elsewhere in the
span; SWAP is built as the product CNOT(a,b) CNOT(b,a) CNOT(a,b) of three such
operands (the paper's operation set has no SWAP; the QFT figure uses it).

A custom operation (Section 5.2.2: data registered with the operation data
provider, applied to a range of qubits) is the 4-tuple
(name, (a, a+1, ..., a+m-1), None, M) with M of size 2^m whose index bit k is
qubit a+k; its range is its span, so M itself is its operand.  ("U2", (q,),
None, M) is the one-qubit case.

Step formation (Section 5.2.1 says only that steps are created dynamically as
gates are added): a gate joins the most recent step if its span is disjoint
from the span of every gate already in that step, otherwise it opens a new
step.  The circuit unitary does not depend on this rule; only the number of
steps does.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import gates as G

GateT = Tuple[str, Tuple[int, ...], object]


def span(g: GateT) -> Tuple[int, int]:
    q = g[1]
    return (min(q), max(q))


def pack_steps(gate_list: Sequence[GateT]) -> List[List[GateT]]:
    """Stages 1-2: group the ordered gates into steps of pairwise disjoint spans."""
    steps: List[List[GateT]] = []
    for g in gate_list:
        lo, hi = span(g)
        if steps and all(hi < span(h)[0] or lo > span(h)[1] for h in steps[-1]):
            steps[-1].append(g)
        else:
            steps.append([g])
    return steps


def _kron_chain(ops: Sequence[np.ndarray]) -> np.ndarray:
    """Algorithm 2: result <- ops[0]; result <- result (x) op for each later operand."""
    result = ops[0]
    for op in ops[1:]:
        result = np.kron(result, op)
    return result


def _span_embed(by_qubit: dict, lo: int, hi: int) -> np.ndarray:
    """Kronecker product over qubits hi..lo of the given 2x2 factors (identity where absent)."""
    return _kron_chain([by_qubit.get(q, G.I2) for q in range(hi, lo - 1, -1)])


def span_operand(g: GateT) -> np.ndarray:
    """Stage 3: the operand a gate contributes to its step, of size 2^m for a span of m qubits."""
    name, qubits, theta = g[0], g[1], g[2]
    if len(g) == 4:
        lo, hi = span(g)
        if list(qubits) != list(range(lo, hi + 1)):
            raise ValueError("a custom operation acts on a contiguous ascending range of qubits")
        M = np.asarray(g[3], dtype=np.complex128)
        if M.shape != (1 << len(qubits),) * 2:
            raise ValueError("custom matrix size does not match its qubit range")
        return M
    if len(qubits) == 1:
        return G.one_qubit(name, theta)
    lo, hi = span(g)
    if name == "SWAP":
        a, b = qubits
        cab = span_operand(("CNOT", (a, b), None))
        cba = span_operand(("CNOT", (b, a), None))
        return cab @ cba @ cab
    c, t = qubits
    U = G.controlled_target(name, theta)
    return _span_embed({c: G.P0}, lo, hi) + _span_embed({c: G.P1, t: U}, lo, hi)


def step_operator(n: int, step: Sequence[GateT]) -> np.ndarray:
    """Stage 4: the dense 2^n x 2^n operator of one step (ordered Kronecker product, Eq. 9s1)."""
    by_top = {span(g)[1]: g for g in step}
    ops = []
    q = n - 1
    while q >= 0:
        if q in by_top:
            g = by_top[q]
            ops.append(span_operand(g))
            q = span(g)[0] - 1
        else:
            ops.append(G.I2)
            q -= 1
    return _kron_chain(ops)


def circuit_unitary(n: int, gate_list: Sequence[GateT], steps=None) -> np.ndarray:
    """Stage 5 (Algorithm 1): result <- I; result <- A . result for each step operator A."""
    if steps is None:
        steps = pack_steps(gate_list)
    result = np.eye(1 << n, dtype=np.complex128)
    for st in steps:
        result = step_operator(n, st) @ result
    return result


def initial_state(n: int) -> np.ndarray:
    """|0...0> as the Kronecker product of single-qubit |0> vectors (Eq. 9)."""
    zero = np.array([1, 0], dtype=np.complex128)
    return _kron_chain([zero] * n)


def simulate_full_state(n: int, gate_list: Sequence[GateT], psi0=None) -> np.ndarray:
    """Stage 6: the circuit unitary applied to the initial state (|0...0> unless given)."""
    U = circuit_unitary(n, gate_list)
    if psi0 is None:
        psi0 = initial_state(n)
    return U @ np.asarray(psi0, dtype=np.complex128)


def probabilities(psi: np.ndarray) -> np.ndarray:
    """Measurement probabilities |psi_i|^2 / sum |psi|^2 (Section 2.2, Eq. 1-3 normalisation)."""
    p = np.abs(psi) ** 2
    return p / p.sum()
