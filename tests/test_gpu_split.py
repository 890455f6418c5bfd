"""Split-bf16 / split-fp16 chain products (float32 accumulation) against the oracle.

Bounds (unit-norm rows and columns, as for unitaries): a split operand carries
~16 (bf16) / ~22 (fp16) significant bits and the dropped lo*lo term is
2^-16 / 2^-22 relative, so one product is within ~6e-5 (bf16) / ~2e-6 (fp16)
of the exact product; chains are checked by fidelity >= 1 - 1e-6 and a
per-amplitude bound.
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

SPLITS = [(B.QSIM_SPLIT_BF16, "bf16", 6e-5), (B.QSIM_SPLIT_FP16, "fp16", 2e-6)]


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec,fmt,_", SPLITS)
@pytest.mark.parametrize("n", [1, 3, 6, 9])
def test_build_step_split_planes(ctx, n, prec, fmt, _):
    rng = np.random.default_rng(n)
    c = W.random_layers(n, 2, rng)
    rel = 2.0 ** -16 if fmt == "bf16" else 2.0 ** -21
    for st in UA.pack_steps(W.gate_tuples(c))[:4]:
        ref = UA.step_operator(n, st)
        for layout in (B.QSIM_LAYOUT_ROW, B.QSIM_LAYOUT_COL):
            buf = G.split_buffer(n)
            B.qsim_build_step(ctx, n, st, prec, layout, buf)
            G.sync()
            got = G.unsplit(buf, fmt, col_major=(layout == B.QSIM_LAYOUT_COL))
            assert np.all(got[ref == 0] == 0)
            assert np.all(np.abs(got - ref) <= rel * np.abs(ref) + 1e-12)


def _rand_unit_cols(N, rng):
    M = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    return M / np.linalg.norm(M, axis=0, keepdims=True)


@pytest.mark.parametrize("prec,fmt,tol", SPLITS)
@pytest.mark.parametrize("n", [2, 4, 5, 6, 7, 9])
def test_step_multiply_split(ctx, n, prec, fmt, tol):
    N = 1 << n
    rng = np.random.default_rng(10 + n)
    S = _rand_unit_cols(N, rng).T  # unit-norm rows
    U = _rand_unit_cols(N, rng)   # unit-norm columns
    dS = G.split_planes(S, fmt, col_major=False)
    dU = G.split_planes(U, fmt, col_major=True)
    out = G.planar(n)
    out_split = G.split_buffer(n)
    B.qsim_step_multiply(ctx, n, prec, dS, dU, out, out_split)
    G.sync()
    ref = S @ U
    got = G.to_complex(out)
    assert np.abs(got - ref).max() <= tol
    # the split output is the same product, column-major, re-split from the float32 accumulators
    got_split = G.unsplit(out_split, fmt, col_major=True)
    assert np.abs(got_split - got).max() <= tol


@pytest.mark.parametrize("prec,fmt,_", SPLITS)
@pytest.mark.parametrize("n", [1, 2, 5, 6, 8, 10])
def test_split_chain_matches_oracle(ctx, n, prec, fmt, _):
    rng = np.random.default_rng(300 + n)
    fams = [W.ghz_chain(n), W.qft(n), W.random_layers(n, 5, rng)]
    if n >= 2:
        fams.append(W.dj(n, int(rng.integers(1, 1 << (n - 1)))))
    for c in fams:
        g = W.gate_tuples(c)
        U = G.planar(n)
        ws = G.workspace(B.qsim_chain_workspace_bytes(n, prec))
        B.qsim_unitary_chain(ctx, n, c.gates, prec, U, ws)
        d_psi = torch.empty(2 << n, dtype=torch.float32, device=G.DEV)
        B.qsim_apply_state(ctx, n, U, None, d_psi)
        psi = G.vec_to_complex(d_psi)
        ref = fsv.final_state(n, g)
        assert metrics.fidelity(psi, ref) >= 1 - 1e-6, c.family
        Ug = G.to_complex(U)
        Ur = UA.circuit_unitary(n, g)
        bound = (2e-3 if fmt == "bf16" else 2e-5)
        assert np.abs(Ug - Ur).max() <= bound, (c.family, np.abs(Ug - Ur).max())


@pytest.mark.parametrize("n", [12, 13])
def test_precision_sweep_random_circuits(ctx, n):
    """Seeded random circuits, depth 20: every precision against the float64 oracle (route B)."""
    c = W.random_layers(n, 20, np.random.default_rng(0))
    g = W.gate_tuples(c)
    ref = fsv.final_state(n, g)
    cols = W.random_columns(n, 16, 5)
    refc = fsv.unitary_columns(n, g, cols)
    for prec in (B.QSIM_FP32_4M, B.QSIM_FP32_3M, B.QSIM_SPLIT_BF16, B.QSIM_SPLIT_FP16):
        U = G.planar(n)
        ws = G.workspace(B.qsim_chain_workspace_bytes(n, prec))
        B.qsim_unitary_chain(ctx, n, c.gates, prec, U, ws)
        d_psi = torch.empty(2 << n, dtype=torch.float32, device=G.DEV)
        B.qsim_apply_state(ctx, n, U, None, d_psi)
        psi = G.vec_to_complex(d_psi)
        F = metrics.fidelity(psi, ref)
        err = np.abs(psi - ref).max()
        Uc = U[:, :, cols].cpu().numpy().astype(np.float64)
        errU = np.abs(Uc[0] + 1j * Uc[1] - refc).max()
        print(f"n={n} prec={prec} max|dpsi|={err:.3e} max|dU|={errU:.3e} 1-F={1 - F:.3e}")
        assert F >= 1 - 1e-6
        if prec in (B.QSIM_FP32_4M, B.QSIM_FP32_3M):
            assert err <= 1e-5 and errU <= 1e-5
        del U, ws
        torch.cuda.empty_cache()
