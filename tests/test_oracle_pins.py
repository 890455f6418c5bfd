"""Pins for the CPU oracle: values the paper prints, closed forms, invariants, brute force.

Every check here compares the oracle with something other than itself, so a
plausible slip in it (a dropped term, a wrong sign or index, a transposed
operand, a reversed product) fails at least one test.
"""
import cmath
import math

import numpy as np
import pytest

from oracle import fsv, gates as OG, metrics, unitary as UA
from paper_2305_14398_amd import workloads as W
from tests import golden_io

TOL = 1e-12


# --- Table 1, Eq. 6 and gate identities ---------------------------------------------------

def test_table1_printed_matrices():
    table = golden_io.load_table1()
    for name in ("H", "X", "Y", "Z"):
        np.testing.assert_allclose(OG.one_qubit(name), table[name](), atol=TOL)
    for phi in (0.0, 0.3, math.pi / 2, math.pi, 5.1):
        np.testing.assert_allclose(OG.one_qubit("R", phi), table["R"](phi), atol=TOL)


def test_eq6_pauli_x_swaps_amplitudes():
    a, b = 0.6 + 0.1j, -0.2 + 0.77j
    np.testing.assert_allclose(OG.one_qubit("X") @ np.array([a, b]), [b, a], atol=TOL)


def test_gate_identities():
    H, X, Y, Z, S, T = (OG.one_qubit(g) for g in "HXYZST")
    np.testing.assert_allclose(S @ S, Z, atol=TOL)
    np.testing.assert_allclose(T @ T, S, atol=TOL)
    np.testing.assert_allclose(H @ X @ H, Z, atol=TOL)
    np.testing.assert_allclose(H @ Z @ H, X, atol=TOL)
    np.testing.assert_allclose(S, OG.one_qubit("R", math.pi / 2), atol=TOL)
    np.testing.assert_allclose(T, OG.one_qubit("R", math.pi / 4), atol=TOL)
    np.testing.assert_allclose(OG.one_qubit("RX", math.pi), -1j * X, atol=TOL)
    np.testing.assert_allclose(OG.one_qubit("RY", math.pi), -1j * Y, atol=TOL)
    for th in (0.1, 1.3, 2.9, 4.4):
        np.testing.assert_allclose(OG.one_qubit("RZ", th), cmath.exp(-0.5j * th) * OG.one_qubit("R", th), atol=TOL)
        np.testing.assert_allclose(OG.one_qubit("RX", th), H @ OG.one_qubit("RZ", th) @ H, atol=TOL)
        # RY(a) RY(b) = RY(a + b): rotations compose additively
        np.testing.assert_allclose(OG.one_qubit("RY", th) @ OG.one_qubit("RY", 0.7), OG.one_qubit("RY", th + 0.7), atol=TOL)
    for name in ("H", "X", "Y", "Z", "S", "T"):
        m = OG.one_qubit(name)
        np.testing.assert_allclose(m.conj().T @ m, np.eye(2), atol=TOL)


# --- worked example of Section 2.4 (Eq. 7, 9s1, 10, 11) ------------------------------------

@pytest.mark.parametrize("fixture", ["eq9s1_step1_h_kron_i.txt", "eq10_step2_cnot.txt", "eq7_controlled_u.txt"])
def test_printed_step_matrices(fixture):
    fx = golden_io.load(fixture)
    n, g = fx["qubits"], fx["gates"]
    np.testing.assert_allclose(UA.step_operator(n, g), fx["matrix"], atol=TOL)
    np.testing.assert_allclose(fsv.circuit_unitary(n, g), fx["matrix"], atol=TOL)


def test_eq11_bell_state():
    fx = golden_io.load("eq11_bell_state.txt")
    psi = UA.simulate_full_state(fx["qubits"], fx["gates"])
    np.testing.assert_allclose(psi, fx["state"], atol=TOL)
    # the same vector for H(0), CNOT(0 -> 1) in little-endian order (Listing 'belltornado')
    psi2 = UA.simulate_full_state(2, W.gate_tuples(W.bell()))
    np.testing.assert_allclose(psi2, fx["state"], atol=TOL)
    np.testing.assert_allclose(UA.initial_state(2), [1, 0, 0, 0], atol=0)


# --- brute force: per-element definition of the tensor product, n <= 3 ----------------------

def _bit(x, q):
    return (x >> q) & 1


def brute_step(n, step):
    """S[r][s] from the definition of the Kronecker product on basis indices."""
    N = 1 << n
    busy = set()
    for g in step:
        lo, hi = min(g[1]), max(g[1])
        busy.update(g[1])
    S = np.zeros((N, N), dtype=np.complex128)
    for r in range(N):
        for s in range(N):
            v = 1.0 + 0j
            for q in range(n):
                if q not in busy and _bit(r, q) != _bit(s, q):
                    v = 0
            for name, qs, th in step:
                if len(qs) == 1:
                    v *= OG.one_qubit(name, th)[_bit(r, qs[0]), _bit(s, qs[0])]
                elif name == "SWAP":
                    a, b = qs
                    v *= float(_bit(r, a) == _bit(s, b) and _bit(r, b) == _bit(s, a))
                else:
                    c, t = qs
                    if _bit(r, c) != _bit(s, c):
                        v = 0
                    elif _bit(s, c) == 0:
                        v *= float(_bit(r, t) == _bit(s, t))
                    else:
                        v *= OG.controlled_target(name, th)[_bit(r, t), _bit(s, t)]
            S[r, s] = v
    return S


def _all_single_steps(n):
    one = [(nm, (q,), 0.7 if nm in W.ANGLED else None) for nm in W.ONE_QUBIT for q in range(n)]
    two = []
    for nm in ("CNOT", "CY", "CZ", "CR", "SWAP"):
        for a in range(n):
            for b in range(n):
                if a != b:
                    two.append((nm, (a, b), 1.1 if nm == "CR" else None))
    return [[g] for g in one + two]


@pytest.mark.parametrize("n", [1, 2, 3])
def test_brute_force_every_gate_and_placement(n):
    for step in _all_single_steps(n):
        ref = brute_step(n, step)
        np.testing.assert_allclose(UA.step_operator(n, step), ref, atol=TOL, err_msg=str(step))
        np.testing.assert_allclose(fsv.circuit_unitary(n, step), ref, atol=TOL, err_msg=str(step))


def test_brute_force_multi_gate_steps():
    rng = np.random.default_rng(5)
    for n in (3, 4):
        for _ in range(30):
            c = W.random_layers(n, 2, rng)
            for st in UA.pack_steps(W.gate_tuples(c)):
                np.testing.assert_allclose(UA.step_operator(n, st), brute_step(n, st), atol=TOL)


def test_permutation_steps_have_one_unit_per_row_and_column():
    for n in (3, 4):
        for step in _all_single_steps(n):
            if step[0][0] in ("X", "CNOT", "SWAP"):
                S = UA.step_operator(n, step)
                assert np.all((np.abs(S) < 1e-15) | (np.abs(S - 1) < 1e-15))
                assert np.all(np.abs(S).sum(0) == 1) and np.all(np.abs(S).sum(1) == 1)


# --- closed forms ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", range(1, 9))
def test_ghz_closed_form(n):
    N = 1 << n
    ref = np.zeros(N, dtype=np.complex128)
    ref[0] = ref[N - 1] = 1 / math.sqrt(2)
    for c in (W.ghz_chain(n), W.ghz_fanout(n)):
        g = W.gate_tuples(c)
        np.testing.assert_allclose(UA.simulate_full_state(n, g), ref, atol=TOL)
        np.testing.assert_allclose(fsv.final_state(n, g), ref, atol=TOL)


@pytest.mark.parametrize("n", range(1, 8))
def test_qft_is_the_dft(n):
    N = 1 << n
    j = np.arange(N)
    closed = np.exp(2j * np.pi * np.outer(j, j) / N) / math.sqrt(N)
    U = UA.circuit_unitary(n, W.gate_tuples(W.qft(n)))
    np.testing.assert_allclose(U, closed, atol=1e-12)
    # the same matrix from the library inverse FFT
    np.testing.assert_allclose(U, np.fft.ifft(np.eye(N), axis=0) * math.sqrt(N), atol=1e-12)
    # QFT |0> = uniform superposition
    np.testing.assert_allclose(U[:, 0], np.full(N, 1 / math.sqrt(N)), atol=1e-12)


@pytest.mark.parametrize("n", [2, 3, 5, 7])
def test_deutsch_jozsa_outcome(n):
    N = 1 << n
    half = 1 << (n - 1)
    for mask in [0] + sorted({1, half - 1, W.dj_mask(n, 0), W.dj_mask(n, 1)}):
        psi = UA.simulate_full_state(n, W.gate_tuples(W.dj(n, mask)))
        ref = np.zeros(N, dtype=np.complex128)
        ref[mask] = 1 / math.sqrt(2)
        ref[mask + half] = -1 / math.sqrt(2)
        np.testing.assert_allclose(psi, ref, atol=TOL)
        p = UA.probabilities(psi)
        p_inputs_zero = p[0] + p[half]
        assert p_inputs_zero == pytest.approx(1.0 if mask == 0 else 0.0, abs=1e-12)


# --- invariants ---------------------------------------------------------------------------

def test_unitarity_and_mirror_identity():
    rng = np.random.default_rng(11)
    for n in (2, 4, 6):
        c = W.random_layers(n, 6, rng)
        U = UA.circuit_unitary(n, W.gate_tuples(c))
        mx, fro = metrics.unitarity_drift(U)
        assert mx < 1e-12 and fro < 1e-12
        M = UA.circuit_unitary(n, W.gate_tuples(W.mirror(c)))
        np.testing.assert_allclose(M, np.eye(1 << n), atol=1e-12)
        psi = U @ W.random_state(n, 3)
        assert np.linalg.norm(psi) == pytest.approx(1.0, abs=1e-12)


def _families(n, rng):
    out = [W.ghz_chain(n), W.ghz_fanout(n), W.qft(n), W.random_layers(n, 5, rng)]
    if n >= 2:
        out.append(W.dj(n, int(rng.integers(0, 1 << (n - 1)))))
    return out


@pytest.mark.parametrize("n", range(1, 8))
def test_route_a_equals_route_b(n):
    rng = np.random.default_rng(100 + n)
    for c in _families(n, rng):
        g = W.gate_tuples(c)
        np.testing.assert_allclose(UA.circuit_unitary(n, g), fsv.circuit_unitary(n, g), atol=1e-12, err_msg=c.family)


def test_packing_invariance_and_step_counts():
    rng = np.random.default_rng(7)
    for n in (3, 5):
        for c in _families(n, rng):
            g = W.gate_tuples(c)
            packed = UA.circuit_unitary(n, g)
            one_per_step = UA.circuit_unitary(n, g, steps=[[x] for x in g])
            np.testing.assert_allclose(packed, one_per_step, atol=1e-12)
    # every QFT gate overlaps its predecessor's span: k = n + n(n-1)/2 + floor(n/2)
    for n in (3, 11, 12, 13):
        assert len(UA.pack_steps(W.gate_tuples(W.qft(n)))) == n + n * (n - 1) // 2 + n // 2
    assert len(UA.pack_steps(W.gate_tuples(W.ghz_chain(5)))) == 5
    # one random layer of single-qubit gates fits one step
    c = W.random_layers(6, 1, np.random.default_rng(0))
    assert len(UA.pack_steps(W.gate_tuples(c)[:6])) == 1


def test_sampled_columns_match_full_unitary():
    n = 6
    c = W.random_layers(n, 4, np.random.default_rng(2))
    g = W.gate_tuples(c)
    cols = W.random_columns(n, 9, 4)
    U = UA.circuit_unitary(n, g)
    np.testing.assert_allclose(fsv.unitary_columns(n, g, cols), U[:, cols], atol=1e-12)


def test_metrics():
    psi = W.random_state(5, 1)
    assert metrics.fidelity(np.exp(0.7j) * psi, psi) == pytest.approx(1.0, abs=1e-14)
    assert metrics.max_abs_diff(psi, psi) == 0.0
    assert metrics.unitarity_drift(np.eye(8)) == (0.0, 0.0)
    other = W.random_state(5, 2)
    assert metrics.fidelity(other, psi) == pytest.approx(abs(np.vdot(psi, other)) ** 2, abs=1e-14)


def test_metrics_closed_forms_off_the_unit_sphere():
    """Closed forms of the metrics on non-unitary matrices and unnormalised vectors.

    U^H = U^{-1} characterises a unitary (Section 2.3); the drift measures how far
    U^H U is from I.  For c*I_N, U^H U - I = (|c|^2 - 1) I, so both the largest entry
    and ||.||_F / sqrt(N) equal ||c|^2 - 1|; for the shear [[1, 1], [0, 1]],
    U^H U - I = [[0, 1], [1, 1]]: largest entry 1, Frobenius norm sqrt(3), over
    sqrt(2).  A diagonal matrix with distinct moduli fixes the normalisation by
    sqrt(N) (not N) at N = 4.  Fidelity is invariant under scaling of either
    vector and a global phase, 0 for orthogonal vectors of any length, and 1/2
    for (2, 0) against (3, 3).  The amplitude difference is a modulus, so
    negative and complex differences count by size.
    """
    for n in (1, 3, 5):
        N = 1 << n
        for c in (0.5, 1.25, 0.8 + 0.9j, -1.1j):
            mx, fro = metrics.unitarity_drift(c * np.eye(N))
            assert mx == pytest.approx(abs(abs(c) ** 2 - 1), abs=1e-14)
            assert fro == pytest.approx(abs(abs(c) ** 2 - 1), abs=1e-14)
    mx, fro = metrics.unitarity_drift(np.array([[1.0, 1.0], [0.0, 1.0]]))
    assert mx == pytest.approx(1.0, abs=1e-14)
    assert fro == pytest.approx(math.sqrt(3.0 / 2.0), abs=1e-14)
    d = np.array([1.0, 2.0, 0.5j, 0.0])
    mx, fro = metrics.unitarity_drift(np.diag(d))
    e = np.abs(d) ** 2 - 1  # 0, 3, -0.75, -1
    assert mx == pytest.approx(3.0, abs=1e-14)
    assert fro == pytest.approx(math.sqrt(float(np.sum(e * e)) / 4.0), abs=1e-14)

    psi = W.random_state(4, 3)
    assert metrics.fidelity(2.0 * psi, 3.0 * np.exp(1.9j) * psi) == pytest.approx(1.0, abs=1e-14)
    a = np.zeros(16, dtype=np.complex128)
    b = np.zeros(16, dtype=np.complex128)
    a[3], b[5] = 2.0, 3.0j
    assert metrics.fidelity(a, b) == 0.0
    assert metrics.fidelity(np.array([2.0, 0.0]), np.array([3.0, 3.0])) == pytest.approx(0.5, abs=1e-15)

    assert metrics.max_abs_diff(np.array([1.0, 2.0]), np.array([3.0, 2.5])) == 2.0
    assert metrics.max_abs_diff(np.array([1.0 + 0j, -2.0]), np.array([1.0 + 3.0j, 2.0])) == 4.0
    assert metrics.max_abs_diff(np.array([]), np.array([])) == 0.0


# --- Measurement by inverse-CDF sampling (Section 5.2.3, simulateAndCollapse) -------------

def test_sampler_one_hot_and_zero_probability_outcomes():
    from oracle import measure
    rng = np.random.default_rng(5)
    u = rng.random(1000)
    for N, hot in ((1, 0), (8, 0), (8, 5), (8, 7), (64, 33)):
        p = np.zeros(N)
        p[hot] = 1.0
        assert np.all(measure.sample(p, u) == hot)
    # an outcome with zero probability is never drawn, whatever the uniform
    p = np.array([0.0, 0.25, 0.0, 0.0, 0.75, 0.0])
    s = measure.sample(p, np.linspace(0.0, 1.0, 10001, endpoint=False))
    assert set(np.unique(s)) == {1, 4}


def test_sampler_uniform_grid_closed_form():
    """Uniform p over N outcomes: u = (k + 1/2) / N lands on outcome k, and any u on floor(u N)."""
    from oracle import measure
    for N in (2, 16, 1024):
        p = np.full(N, 1.0 / N)
        k = np.arange(N)
        np.testing.assert_array_equal(measure.sample(p, (k + 0.5) / N), k)
        u = np.random.default_rng(N).random(4096)
        np.testing.assert_array_equal(measure.sample(p * 7.0, u), np.floor(u * N).astype(np.int64))


def test_sampler_grid_counts_equal_probabilities():
    """On the grid u = j / M each outcome receives M * p_i points, to within one, and the map is monotone."""
    from oracle import measure
    rng = np.random.default_rng(11)
    p = rng.random(37) ** 3
    p[[3, 17]] = 0.0
    p /= p.sum()
    M = 200_000
    s = measure.sample(p, np.arange(M) / M)
    assert np.all(np.diff(s) >= 0)
    counts = np.bincount(s, minlength=p.size)
    assert np.max(np.abs(counts - M * p)) <= 1.0 + 1e-9
    assert counts[3] == 0 and counts[17] == 0


def test_sampler_unnormalised_input_is_scaled_by_its_total():
    from oracle import measure
    p = np.array([1.0, 3.0, 0.0, 4.0])
    u = np.array([0.0, 0.124, 0.125, 0.49, 0.5, 0.999])
    np.testing.assert_array_equal(measure.sample(p, u), [0, 0, 1, 1, 3, 3])


@pytest.mark.parametrize("n", [3, 5, 7])
def test_deutsch_jozsa_measurement_reads_the_mask(n):
    """Deutsch-Jozsa (Section 2.5): the input register collapses to |0...0> for the constant
    function; with f(x) = parity(mask & x) it collapses to |mask>, so never to all zeros when
    balanced.  The ancilla stays in (|0> - |1>)/sqrt(2) and reads 0 or 1 with probability 1/2."""
    from oracle import measure
    u = np.random.default_rng(n).random(4000)
    for mask in (0, 1, (1 << (n - 1)) - 1, W.dj_mask(n, 3)):
        psi = UA.simulate_full_state(n, W.gate_tuples(W.dj(n, mask)))
        shots = measure.sample(UA.probabilities(psi), u)
        assert np.all((shots & ((1 << (n - 1)) - 1)) == mask)
        ancilla = (shots >> (n - 1)) & 1
        assert 0.45 < ancilla.mean() < 0.55


def test_collapse_is_the_basis_state():
    from oracle import measure
    psi = measure.collapse(3, 6)
    assert psi[6] == 1.0 and np.count_nonzero(psi) == 1


# --- custom operations on qubit ranges (Section 5.2.2) --------------------------------------

def _relabel(gates, offset):
    return [(nm, tuple(q + offset for q in qs), th) for nm, qs, th in gates]


def test_custom_matches_named_gates():
    n = 5
    H = OG.one_qubit("H")
    # one qubit: the matrix of H is H
    for route in (UA.circuit_unitary, fsv.circuit_unitary):
        np.testing.assert_allclose(route(n, [("U2", (3,), None, H)]), route(n, [("H", (3,), None)]), atol=TOL)
    # two qubits, index bit 0 = qubit a: CNOT(a -> a+1) flips bit 1 where bit 0 is set
    cnot_le = np.zeros((4, 4))
    for s_ in range(4):
        r_ = s_ ^ 2 if s_ & 1 else s_
        cnot_le[r_, s_] = 1
    for a in (0, 2, 3):
        for route in (UA.circuit_unitary, fsv.circuit_unitary):
            np.testing.assert_allclose(route(n, [("cnot", (a, a + 1), None, cnot_le)]),
                                       route(n, [("CNOT", (a, a + 1), None)]), atol=TOL)


@pytest.mark.parametrize("a", [0, 1, 3])
def test_custom_dft_equals_qft_subcircuit(a):
    """A registered 3-qubit DFT matrix (omega^{jk} / sqrt 8) on qubits a..a+2 equals the QFT gates on them."""
    n = 6
    D = 8
    j = np.arange(D)
    dft = np.exp(2j * np.pi * np.outer(j, j) / D) / math.sqrt(D)
    rng = np.random.default_rng(a)
    pre = W.gate_tuples(W.random_layers(n, 2, rng))
    custom = pre + [("dft3", (a, a + 1, a + 2), None, dft)] + [("H", (5,), None)]
    named = pre + _relabel(W.gate_tuples(W.qft(3)), a) + [("H", (5,), None)]
    for route in (UA.circuit_unitary, fsv.circuit_unitary):
        np.testing.assert_allclose(route(n, custom), route(n, named), atol=1e-12)


def test_custom_brute_force_entries():
    """U[r][s] = M[r_range][s_range] * [r and s agree outside the range], entry by entry."""
    n, a, m = 4, 1, 2
    M = W.random_unitary(m, 7)
    U = UA.circuit_unitary(n, [("c", (a, a + 1), None, M)])
    mask = ((1 << m) - 1) << a
    for r_ in range(1 << n):
        for s_ in range(1 << n):
            want = M[(r_ & mask) >> a, (s_ & mask) >> a] if (r_ & ~mask) == (s_ & ~mask) else 0
            assert abs(U[r_, s_] - want) < 1e-14


@pytest.mark.parametrize("n", [3, 6, 8])
def test_custom_route_a_equals_route_b(n):
    g = W.with_custom_ops(W.gate_tuples(W.random_layers(n, 3, np.random.default_rng(n))), n, [1, 2, 3, n], 40 + n)
    A = UA.circuit_unitary(n, g)
    np.testing.assert_allclose(A, fsv.circuit_unitary(n, g), atol=1e-12)
    np.testing.assert_allclose(A.conj().T @ A, np.eye(1 << n), atol=1e-12)


def test_custom_range_checks():
    with pytest.raises(ValueError):
        UA.circuit_unitary(3, [("c", (0, 2), None, np.eye(4))])
    with pytest.raises(ValueError):
        fsv.circuit_unitary(3, [("c", (0, 1), None, np.eye(8))])


def test_chain_association_left_fold_equals_tree():
    """The product of the step operators is associative: Algorithm 1's left fold and a pairwise tree give the
    same matrix (only rounding differs)."""
    n = 6
    steps = UA.pack_steps(W.gate_tuples(W.random_layers(n, 4, np.random.default_rng(12))))
    ops = [UA.step_operator(n, st) for st in steps]
    fold = UA.circuit_unitary(n, W.gate_tuples(W.random_layers(n, 4, np.random.default_rng(12))))
    level = ops
    while len(level) > 1:
        nxt = [level[i + 1] @ level[i] for i in range(0, len(level) - 1, 2)]
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    np.testing.assert_allclose(level[0], fold, atol=1e-12)
