"""CPU oracle for the unitary-matrix simulation method (complex128, numpy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code, tables or constants with the
HIP library; it consumes only the plain ordered gate list
``[(name, qubits, theta), ...]`` that the seeded workload generators produce.

Two independent routes:

* route A (:mod:`oracle.unitary`) follows the paper's plain unitary method:
  one dense step operator per step built by ordered Kronecker products
  (Algorithm 2, Eq. 9s1), the chain ``result <- A . result`` from the identity
  (Algorithm 1), and the final matrix-vector product with the initial state.
* route B (:mod:`oracle.fsv`) applies each gate in place to columns of the
  identity or to a state vector, with the per-amplitude update of the
  full-state-vector method (Appendix A, Eq. 12).

:mod:`oracle.measure` draws measurement outcomes from a state's
probabilities by inverse-CDF sampling with caller-supplied uniforms (the
collapsing method of the Simulator interface, Section 5.2.3).

Parity status: every function here is pinned by the tests in
``tests/test_oracle_pins.py`` (printed matrices of Table 1 and Eq. 8-11,
closed forms for GHZ, QFT and Deutsch-Jozsa, unitarity, brute-force 1-2 qubit
matrices, route A == route B, the error metrics' closed forms on non-unitary
matrices and unnormalised vectors, and for the sampler one-hot, uniform-grid
and Deutsch-Jozsa outcomes).  No function is parity unpinned.
"""
from . import gates, unitary, fsv, metrics, measure  # noqa: F401
