"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances:
* step expansion (stage 4): each entry is a float64 product rounded once to
  float32, so |gpu - oracle| <= 2^-23 |oracle| and structural zeros are exact;
* float32 chains (stage 5) and applied states (stage 6): max |delta| <= 1e-5
  per amplitude / matrix entry (complex64 target);
* float64 drift: the float32 U is exact in float64, so the GPU drift agrees
  with the oracle's drift of the same matrix to 1e-12.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fsv, metrics, unitary as UA  # noqa: E402
from paper_2305_14398_amd import binding as B  # noqa: E402
from paper_2305_14398_amd import workloads as W  # noqa: E402
from tests import gpu_util as G  # noqa: E402

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-5
FP32_PRECS = [B.QSIM_FP32_4M, B.QSIM_FP32_3M]


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


def gpu_step(ctx, n, step, layout=B.QSIM_LAYOUT_ROW):
    out = G.planar(n)
    B.qsim_build_step(ctx, n, step, B.QSIM_FP32_4M, layout, out)
    G.sync()
    return G.to_complex(out, col_major=(layout == B.QSIM_LAYOUT_COL))


def gpu_chain(ctx, n, gates, prec=B.QSIM_FP32_4M, offsets=None):
    U = G.planar(n)
    ws = G.workspace(B.qsim_chain_workspace_bytes(n, prec))
    B.qsim_unitary_chain(ctx, n, gates, prec, U, ws, step_offsets=offsets)
    G.sync()
    return U


def assert_step_close(got, ref):
    assert np.all(got[ref == 0] == 0), "structural zeros must be exact"
    err = np.abs(got - ref)
    assert np.all(err <= 2.0 ** -23 * np.abs(ref) + 1e-30), float(err.max())


# --- stage 4: step expansion ----------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_build_step_every_gate_and_placement(ctx, n):
    names1 = list(W.ONE_QUBIT)
    for q in range(n):
        for nm in names1:
            st = [(nm, (q,), 0.9 if nm in W.ANGLED else None)]
            for layout in (B.QSIM_LAYOUT_ROW, B.QSIM_LAYOUT_COL):
                assert_step_close(gpu_step(ctx, n, st, layout), UA.step_operator(n, st))
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            for nm in ("CNOT", "CY", "CZ", "CR", "SWAP"):
                st = [(nm, (a, b), 1.3 if nm == "CR" else None)]
                for layout in (B.QSIM_LAYOUT_ROW, B.QSIM_LAYOUT_COL):
                    assert_step_close(gpu_step(ctx, n, st, layout), UA.step_operator(n, st))


@pytest.mark.parametrize("n", [4, 7, 9])
def test_build_step_multi_gate_steps(ctx, n):
    rng = np.random.default_rng(n)
    c = W.random_layers(n, 3, rng)
    for st in UA.pack_steps(W.gate_tuples(c)):
        assert_step_close(gpu_step(ctx, n, st), UA.step_operator(n, st))
    # the empty step is the identity
    assert_step_close(gpu_step(ctx, n, []), np.eye(1 << n))


@pytest.mark.parametrize("n", [12, 13])
def test_build_step_full_size_sampled_columns(ctx, n):
    rng = np.random.default_rng(40 + n)
    c = W.random_layers(n, 2, rng)
    steps = UA.pack_steps(W.gate_tuples(c))
    cols = W.random_columns(n, 24, n)
    for st in (steps[0], steps[-1]):
        S = gpu_step(ctx, n, st)
        ref = fsv.unitary_columns(n, st, cols)
        assert_step_close(S[:, cols], ref)


# --- stage 5: a single product --------------------------------------------------------------

@pytest.mark.parametrize("prec", FP32_PRECS)
@pytest.mark.parametrize("n", [1, 3, 4, 5, 6, 7, 8, 10])
def test_step_multiply_random_matrices(ctx, n, prec):
    N = 1 << n
    rng = np.random.default_rng(n + 10 * prec)
    A = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / math.sqrt(N)
    Bm = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / math.sqrt(N)
    A32 = A.astype(np.complex64).astype(np.complex128)
    B32 = Bm.astype(np.complex64).astype(np.complex128)
    dS = G.planar(n, A.T)  # column-major operand
    dU = G.planar(n, Bm)
    dC = G.planar(n)
    B.qsim_step_multiply(ctx, n, prec, dS, dU, dC)
    G.sync()
    ref = A32 @ B32
    err = np.abs(G.to_complex(dC) - ref).max()
    assert err <= 4e-6 * math.sqrt(math.log2(N) + 1), err


@pytest.mark.parametrize("prec", FP32_PRECS)
@pytest.mark.parametrize("n", [11, 13])
def test_step_multiply_full_size_sampled(ctx, n, prec):
    N = 1 << n
    g = torch.Generator(device="cpu").manual_seed(n)
    dS = (torch.randn((2, N, N), generator=g) / math.sqrt(2 * N)).to(G.DEV)
    dU = (torch.randn((2, N, N), generator=g) / math.sqrt(2 * N)).to(G.DEV)
    dC = G.planar(n)
    B.qsim_step_multiply(ctx, n, prec, dS, dU, dC)
    G.sync()
    cols = W.random_columns(n, 32, 7)
    rows = W.random_columns(n, 32, 8)
    S = dS.cpu().numpy().astype(np.float64)
    A = (S[0] + 1j * S[1]).T  # the step operator is stored column-major
    Uc = dU[:, :, cols].cpu().numpy().astype(np.float64)
    ref = A @ (Uc[0] + 1j * Uc[1])
    got = G.to_complex(dC)[:, cols]
    assert np.abs(got - ref).max() <= 2e-5
    # full rows too (exercise every tile column)
    Ur = dU.cpu().numpy().astype(np.float64)
    ref_rows = A[rows] @ (Ur[0] + 1j * Ur[1])
    assert np.abs(G.to_complex(dC)[rows] - ref_rows).max() <= 2e-5


# --- stages 4-5: whole chains ---------------------------------------------------------------

def _families(n, rng):
    out = [W.ghz_chain(n), W.ghz_fanout(n), W.qft(n), W.random_layers(n, 4, rng)]
    if n >= 2:
        out.append(W.dj(n, int(rng.integers(0, 1 << (n - 1)))))
    return out


@pytest.mark.parametrize("prec", FP32_PRECS)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_chain_matches_oracle(ctx, n, prec):
    rng = np.random.default_rng(200 + n)
    for c in _families(n, rng):
        g = W.gate_tuples(c)
        ref = UA.circuit_unitary(n, g)
        U = G.to_complex(gpu_chain(ctx, n, c.gates, prec))
        err = np.abs(U - ref).max()
        assert err <= AMP_TOL, (c.family, err)


def test_chain_edge_cases(ctx):
    # no gates: identity; one step: just the expansion; two steps: one product
    for n in (1, 4, 7):
        np.testing.assert_array_equal(G.to_complex(gpu_chain(ctx, n, [])), np.eye(1 << n))
    for gates in ([("H", (0,), None)], [("H", (0,), None), ("CNOT", (0, 1), None)],
                  [("H", (0,), None), ("CNOT", (0, 1), None), ("X", (1,), None)]):
        n = 6
        ref = UA.circuit_unitary(n, gates)
        assert np.abs(G.to_complex(gpu_chain(ctx, n, gates)) - ref).max() <= 1e-6


def test_chain_caller_offsets_and_packing_invariance(ctx):
    n = 7
    c = W.random_layers(n, 5, np.random.default_rng(3))
    one_per_step = list(range(len(c.gates) + 1))
    U1 = G.to_complex(gpu_chain(ctx, n, c.gates, offsets=one_per_step))
    U2 = G.to_complex(gpu_chain(ctx, n, c.gates))
    ref = UA.circuit_unitary(n, W.gate_tuples(c))
    assert np.abs(U1 - ref).max() <= AMP_TOL and np.abs(U2 - ref).max() <= AMP_TOL


def test_mirror_circuit_gives_identity(ctx):
    for n in (5, 8):
        c = W.mirror(W.random_layers(n, 6, np.random.default_rng(n)))
        U = G.to_complex(gpu_chain(ctx, n, c.gates))
        assert np.abs(U - np.eye(1 << n)).max() <= AMP_TOL


# --- stage 6 and the drift check ------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 4, 7, 8, 10])
def test_apply_state_random_initial_state(ctx, n):
    c = W.random_layers(n, 3, np.random.default_rng(n))
    U = gpu_chain(ctx, n, c.gates)
    psi0 = W.random_state(n, 5)
    d_psi0 = G.planar_vec(psi0)
    d_psi = torch.empty(2 << n, dtype=torch.float32, device=G.DEV)
    d_prob = torch.empty(1 << n, dtype=torch.float64, device=G.DEV)
    norm2 = B.qsim_apply_state(ctx, n, U, d_psi0, d_psi, d_prob)
    psi = G.vec_to_complex(d_psi)
    ref = fsv.final_state(n, W.gate_tuples(c), psi0)
    assert np.abs(psi - ref).max() <= AMP_TOL
    exact = float(np.sum(np.abs(psi) ** 2))  # float32 values squared in float64
    assert norm2 == pytest.approx(exact, rel=1e-12)
    np.testing.assert_allclose(d_prob.cpu().numpy(), np.abs(psi) ** 2 / exact, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("n", [3, 6, 9])
def test_apply_basis_state_equals_first_column_exactly(ctx, n):
    c = W.qft(n)
    U = gpu_chain(ctx, n, c.gates)
    d_psi = torch.empty(2 << n, dtype=torch.float32, device=G.DEV)
    B.qsim_apply_state(ctx, n, U, None, d_psi, None, want_norm2=False)
    G.sync()
    psi = d_psi.cpu().numpy()
    N = 1 << n
    col0 = U[:, :, 0].cpu().numpy()
    np.testing.assert_array_equal(psi[:N], col0[0])
    np.testing.assert_array_equal(psi[N:], col0[1])


@pytest.mark.parametrize("n", [2, 5, 6, 8, 10, 12])  # 12: the 64-wide drift tile
def test_drift_matches_oracle_of_same_matrix(ctx, n):
    c = W.random_layers(n, 4, np.random.default_rng(n))
    U = gpu_chain(ctx, n, c.gates)
    mx, fro = B.qsim_unitarity_drift(ctx, n, U)
    rmx, rfro = metrics.unitarity_drift(G.to_complex(U))
    assert abs(mx - rmx) <= 1e-12 and abs(fro - rfro) <= 1e-12
    assert mx < 1e-5
    # a non-unitary matrix: drift of order one, relative agreement
    N = 1 << n
    rng = np.random.default_rng(1)
    M = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / math.sqrt(N)
    dM = G.planar(n, M)
    mx, fro = B.qsim_unitarity_drift(ctx, n, dM)
    rmx, rfro = metrics.unitarity_drift(G.to_complex(dM))
    assert mx == pytest.approx(rmx, rel=1e-10) and fro == pytest.approx(rfro, rel=1e-10)


# --- the paper's workloads end to end -------------------------------------------------------

def test_fully_entangled_five_qubits(ctx):
    n = 5
    U = gpu_chain(ctx, n, W.ghz_chain(n).gates)
    d_psi = torch.empty(2 << n, dtype=torch.float32, device=G.DEV)
    norm2 = B.qsim_apply_state(ctx, n, U, None, d_psi)
    psi = G.vec_to_complex(d_psi)
    ref = np.zeros(32)
    ref[0] = ref[31] = 1 / math.sqrt(2)
    assert np.abs(psi - ref).max() <= 1e-7
    assert norm2 == pytest.approx(1.0, abs=1e-7)


@pytest.mark.parametrize("prec", FP32_PRECS)
def test_qft_and_deutsch_jozsa_eleven_qubits(ctx, prec):
    n = 11
    N = 1 << n
    circuits = [W.qft(n)] + [W.dj(n, W.dj_mask(n, s)) for s in (0, 1, 2)]
    cols = W.random_columns(n, 64, 11)
    for c in circuits:
        g = W.gate_tuples(c)
        U = gpu_chain(ctx, n, c.gates, prec)
        d_psi = torch.empty(2 * N, dtype=torch.float32, device=G.DEV)
        B.qsim_apply_state(ctx, n, U, None, d_psi)
        psi = G.vec_to_complex(d_psi)
        ref_psi = fsv.final_state(n, g)
        assert np.abs(psi - ref_psi).max() <= AMP_TOL, c.family
        Uc = G.to_complex(U)[:, cols]
        assert np.abs(Uc - fsv.unitary_columns(n, g, cols)).max() <= AMP_TOL, c.family
        if c.family == "qft":
            j = np.arange(N)
            closed = np.exp(2j * np.pi * np.outer(j, cols) / N) / math.sqrt(N)
            assert np.abs(Uc - closed).max() <= AMP_TOL
        mx, _ = B.qsim_unitarity_drift(ctx, n, U)
        assert mx < 1e-4


def test_random_thirteen_qubits_fp32(ctx):
    n = 13
    c = W.random_layers(n, 20, np.random.default_rng(0))
    g = W.gate_tuples(c)
    U = gpu_chain(ctx, n, c.gates, B.QSIM_FP32_4M)
    d_psi = torch.empty(2 << n, dtype=torch.float32, device=G.DEV)
    B.qsim_apply_state(ctx, n, U, None, d_psi)
    psi = G.vec_to_complex(d_psi)
    ref = fsv.final_state(n, g)
    assert np.abs(psi - ref).max() <= AMP_TOL
    assert metrics.fidelity(psi, ref) >= 1 - 1e-6
    cols = W.random_columns(n, 16, 2)
    Uc = U[:, :, cols].cpu().numpy().astype(np.float64)
    assert np.abs((Uc[0] + 1j * Uc[1]) - fsv.unitary_columns(n, g, cols)).max() <= AMP_TOL


# --- maximum sizes --------------------------------------------------------------------------

def test_expand_sixteen_qubits_sixteen_gates(ctx):
    """The largest step: n = 16 (a 32 GiB operator) with 16 gates, one per qubit; sampled columns."""
    n = 16
    rng = np.random.default_rng(16)
    names = ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "R"]
    step = []
    for q in range(n):
        nm = names[int(rng.integers(0, len(names)))]
        step.append((nm, (q,), float(rng.uniform(0, 2 * math.pi)) if nm in W.ANGLED else None))
    S = torch.empty((2, 1 << n, 1 << n), dtype=torch.float32, device=G.DEV)
    B.qsim_build_step(ctx, n, step, B.QSIM_FP32_4M, B.QSIM_LAYOUT_ROW, S)
    G.sync()
    cols = W.random_columns(n, 6, 3)
    ref = fsv.unitary_columns(n, step, cols)
    got = S[:, :, cols].cpu().numpy().astype(np.float64)
    got = got[0] + 1j * got[1]
    assert np.all(np.abs(got - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-30)
    del S
    torch.cuda.empty_cache()


def test_chain_fourteen_qubits_sampled(ctx):
    n = 14
    c = W.random_layers(n, 1, np.random.default_rng(14))  # a few steps of 16384^3 products
    g = W.gate_tuples(c)
    U = gpu_chain(ctx, n, c.gates, B.QSIM_FP32_4M)
    cols = W.random_columns(n, 8, 4)
    Uc = U[:, :, cols].cpu().numpy().astype(np.float64)
    assert np.abs((Uc[0] + 1j * Uc[1]) - fsv.unitary_columns(n, g, cols)).max() <= AMP_TOL
    d_psi = torch.empty(2 << n, dtype=torch.float32, device=G.DEV)
    B.qsim_apply_state(ctx, n, U, None, d_psi)
    assert np.abs(G.vec_to_complex(d_psi) - fsv.final_state(n, g)).max() <= AMP_TOL
    mx, _ = B.qsim_unitarity_drift_probe(ctx, n, U)
    assert mx < 1e-5
    del U
    torch.cuda.empty_cache()


# --- custom operations on qubit ranges (Section 5.2.2) --------------------------------------

@pytest.mark.parametrize("n", [3, 6, 9])
def test_build_step_custom_ranges(ctx, n):
    from tests.custom_ops import lib_gates
    for m in range(1, min(n, 6) + 1):
        for a in sorted({0, n - m, (n - m) // 2}):
            M = W.random_unitary(m, 10 * m + a)
            st = [(f"step_custom_{m}_{a}", tuple(range(a, a + m)), None, M)]
            if a + m < n:
                st.append(("RY", (a + m,), 0.4))
            for layout in (B.QSIM_LAYOUT_ROW, B.QSIM_LAYOUT_COL):
                assert_step_close(gpu_step(ctx, n, lib_gates(st), layout), UA.step_operator(n, st))


@pytest.mark.parametrize("n", [5, 11])
def test_chain_with_custom_ops(ctx, n):
    from tests.custom_ops import lib_gates
    g = W.with_custom_ops(W.gate_tuples(W.random_layers(n, 4, np.random.default_rng(n))), n, [1, 2, 3, 4, 6], 300 + n)
    for prec in FP32_PRECS:
        U = G.to_complex(gpu_chain(ctx, n, lib_gates(g), prec))
        if n <= 6:
            ref = UA.circuit_unitary(n, g)
            assert np.abs(U - ref).max() <= AMP_TOL
        cols = W.random_columns(n, 8, 5)
        assert np.abs(U[:, cols] - fsv.unitary_columns(n, g, cols)).max() <= AMP_TOL


@pytest.mark.parametrize("prec", FP32_PRECS)
def test_tree_of_step_products_equals_chain(ctx, prec):
    """Association (a left fold and a pairwise tree of the same step operators) changes only rounding: both
    GPU results match the oracle to the complex64 tolerance."""
    n = 9
    c = W.random_layers(n, 5, np.random.default_rng(19))
    steps = UA.pack_steps(W.gate_tuples(c))
    level = []
    for st in steps:
        S = G.planar(n)
        B.qsim_build_step(ctx, n, st, B.QSIM_FP32_4M, B.QSIM_LAYOUT_ROW, S)
        level.append(S)
    while len(level) > 1:
        nxt = []
        for i in range(0, len(level) - 1, 2):
            left = level[i + 1].transpose(1, 2).contiguous()  # the left operand is read column-major
            out = G.planar(n)
            B.qsim_step_multiply(ctx, n, prec, left, level[i], out)
            nxt.append(out)
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    G.sync()
    tree = G.to_complex(level[0])
    chain = G.to_complex(gpu_chain(ctx, n, c.gates, prec))
    ref = UA.circuit_unitary(n, W.gate_tuples(c))
    assert np.abs(tree - ref).max() <= AMP_TOL and np.abs(chain - ref).max() <= AMP_TOL


def test_drift_async_equals_synchronous(ctx):
    n = 9
    U = gpu_chain(ctx, n, W.random_layers(n, 3, np.random.default_rng(4)).gates)
    out = torch.full((2,), float("nan"), dtype=torch.float64, device=G.DEV)
    B.qsim_unitarity_drift_async(ctx, n, U, out)
    G.sync()
    assert tuple(out.cpu().tolist()) == B.qsim_unitarity_drift(ctx, n, U)
