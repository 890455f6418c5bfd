"""Fused stages 4 and 5 (Section 5.3 lets a backend change how stages 4-6 compute): one product
C = S . U that computes the step operator S inside the product kernel, and the chain built on it.

Parity:
* with the materialising path, bit for bit: the fused kernel evaluates each entry of S by the same
  rule (float64 product of the gate factors, rounded once to float32) and then runs the same
  product arithmetic, so qsim_step_multiply_fused == qsim_build_step + qsim_step_multiply and
  qsim_unitary_chain_fused == qsim_unitary_chain exactly;
* with the CPU oracle: max |delta| <= 1e-5 per entry (complex64 target).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fsv, unitary as UA  # noqa: E402
from paper_2305_14398_amd import binding as B  # noqa: E402
from paper_2305_14398_amd import workloads as W  # noqa: E402
from tests import gpu_util as G  # noqa: E402
from tests.custom_ops import lib_gates  # noqa: E402

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-5
FP32_PRECS = [B.QSIM_FP32_4M, B.QSIM_FP32_3M]


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


def random_matrix(n, seed):
    rng = np.random.default_rng(seed)
    N = 1 << n
    return (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / np.sqrt(2.0 * N)


def sample_steps(n, seed):
    """Steps of every kind: a random layer with custom operations (all one-qubit kinds, CNOT/CZ
    pairs, dense 2^m blocks), QFT steps (H, controlled phases spanning up to the whole register,
    SWAP) and the empty step."""
    rng = np.random.default_rng(seed)
    g = W.gate_tuples(W.random_layers(n, 2, rng))
    g = W.with_custom_ops(g, n, [1, 2, 3], seed)
    steps = UA.pack_steps(g)
    q = UA.pack_steps(W.gate_tuples(W.qft(n)))
    picks = steps[:3] + [q[0], q[len(q) // 2], q[-1]]
    long_cr = [s for s in q if any(len(t[1]) == 2 and abs(t[1][0] - t[1][1]) == n - 1 for t in s)]
    return picks + long_cr[:1] + [[]]


def materialised(ctx, n, prec, step, Uin):
    S = G.planar(n)
    B.qsim_build_step(ctx, n, lib_gates(step), prec, B.QSIM_LAYOUT_COL, S)
    out = G.planar(n)
    B.qsim_step_multiply(ctx, n, prec, S, Uin, out)
    return out


@pytest.mark.parametrize("prec", FP32_PRECS)
@pytest.mark.parametrize("n", [1, 2, 4, 5, 6, 7, 9, 11])
def test_fused_product_bit_identical_and_matches_oracle(ctx, prec, n):
    U0 = random_matrix(n, 40 + n)
    Uin = G.planar(n, U0)
    for i, step in enumerate(sample_steps(n, 70 + n)):
        out = G.planar(n)
        B.qsim_step_multiply_fused(ctx, n, prec, lib_gates(step), Uin, out)
        ref = materialised(ctx, n, prec, step, Uin)
        G.sync()
        assert torch.equal(out, ref), (n, i, step)
        if n <= 9:
            want = UA.step_operator(n, step) @ U0
            err = np.abs(G.to_complex(out) - want).max()
            assert err <= AMP_TOL, (n, i, err)


@pytest.mark.parametrize("prec", FP32_PRECS)
def test_fused_chain_bit_identical_on_paper_families(ctx, prec):
    for n in (1, 3, 5, 6, 8, 11):
        rng = np.random.default_rng(n)
        circuits = [W.ghz_chain(n), W.qft(n), W.random_layers(n, 5, rng)]
        if n >= 2:
            circuits.append(W.dj(n, W.dj_mask(n, n)))
        custom = W.with_custom_ops(W.gate_tuples(W.random_layers(n, 3, rng)), n, [2, 3], 500 + n)
        for name, gates, ref_gates in [(c.family, c.gates, W.gate_tuples(c)) for c in circuits] + \
                [("custom", lib_gates(custom), custom)]:
            Uf = G.planar(n)
            ws = G.workspace(B.qsim_chain_fused_workspace_bytes(n, prec))
            B.qsim_unitary_chain_fused(ctx, n, gates, prec, Uf, ws)
            Um = G.planar(n)
            wsm = G.workspace(B.qsim_chain_workspace_bytes(n, prec))
            B.qsim_unitary_chain(ctx, n, gates, prec, Um, wsm)
            G.sync()
            assert torch.equal(Uf, Um), (name, n)
            if n <= 8:
                err = np.abs(G.to_complex(Uf) - UA.circuit_unitary(n, ref_gates)).max()
                assert err <= AMP_TOL, (name, n, err)


def test_fused_chain_with_caller_offsets_and_single_step(ctx):
    n = 7
    c = W.qft(n)
    gates = W.gate_tuples(c)
    one_per_step = list(range(len(gates) + 1))
    for prec in FP32_PRECS:
        for offs in (one_per_step, None):
            Uf = G.planar(n)
            B.qsim_unitary_chain_fused(ctx, n, c.gates, prec, Uf,
                                       G.workspace(B.qsim_chain_fused_workspace_bytes(n, prec)), step_offsets=offs)
            Um = G.planar(n)
            B.qsim_unitary_chain(ctx, n, c.gates, prec, Um, G.workspace(B.qsim_chain_workspace_bytes(n, prec)),
                                 step_offsets=offs)
            G.sync()
            assert torch.equal(Uf, Um)
        # a one-step circuit is expanded straight into d_U; no product runs
        Uf = G.planar(n)
        B.qsim_unitary_chain_fused(ctx, n, [("H", (3,), None)], prec, Uf,
                                   G.workspace(B.qsim_chain_fused_workspace_bytes(n, prec)))
        G.sync()
        assert np.abs(G.to_complex(Uf) - UA.circuit_unitary(n, [("H", (3,), None)])).max() <= 2 ** -23


@pytest.mark.parametrize("prec", FP32_PRECS)
def test_fused_product_at_14_qubits(ctx, prec):
    """The largest chain size: 16384^2 operands (2 GiB each); compared with the materialising path on
    the whole output and with the oracle on sampled entries."""
    n = 14
    N = 1 << n
    g = torch.Generator(device=G.DEV).manual_seed(5)
    Uin = torch.randn((2, N, N), device=G.DEV, generator=g) / (2.0 * N) ** 0.5
    step = [("H", (0,), None), ("CR", (1, 12), 0.7), ("RX", (13,), 1.1)]
    out = G.planar(n)
    B.qsim_step_multiply_fused(ctx, n, prec, step, Uin, out)
    ref = materialised(ctx, n, prec, step, Uin)
    G.sync()
    assert torch.equal(out, ref)
    del ref
    # sampled columns from the oracle's gate-by-gate application (route B): C[:, j] = S . U[:, j]
    cols = W.random_columns(n, 4, 10)
    idx = torch.as_tensor(cols, device=G.DEV)
    U = Uin[:, :, idx].detach().cpu().numpy().astype(np.float64)
    got = G.to_complex(out[:, :, idx])
    for i, j in enumerate(cols):
        want = fsv.apply_circuit(n, step, U[0][:, i] + 1j * U[1][:, i])
        assert np.abs(got[:, i] - want).max() <= AMP_TOL, j
    del out, Uin
    torch.cuda.empty_cache()
