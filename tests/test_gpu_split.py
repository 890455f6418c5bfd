"""Split-bf16 / split-fp16 chain products (float32 accumulation) against the oracle.

Bounds (unit-norm rows and columns, as for unitaries): a split operand carries
~16 (bf16) / ~22 (fp16) significant bits and the dropped lo*lo term is
2^-16 / 2^-22 relative, so one product is within 3 u (u = 2^-16 / 2^-22) plus
float32 rounding of the exact product per entry; the single-product tests allow
6e-5 / 2e-6 on random unit-norm operands.  A chain of P products is held to
gpu_util.split_chain_bound: every column of U and the final state within
3 (u + 2^-24) sqrt(P) in 2-norm of the oracle (the products' roundings add in
quadrature; the unitary steps carry them unchanged in 2-norm), and fidelity
>= 1 - 1e-6 (the target for split precisions).

The three-product (Gauss) forms take Im = T3 - T1 - T2 with T3 over the
operands' float32 sums re + im (|re + im| <= sqrt(2) |x|), so the imaginary
part's per-entry bound is three times the four-product one; the single-product
tests allow 3x and the chain bound carries the same factor.  Their operands have
two more planes (the split of re + im), checked against the float32 sum of the
rounded parts.
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

SPLITS = [(B.QSIM_SPLIT_BF16, "bf16", 6e-5), (B.QSIM_SPLIT_FP16, "fp16", 2e-6),
          (B.QSIM_SPLIT_BF16_3M, "bf16", 1.8e-4), (B.QSIM_SPLIT_FP16_3M, "fp16", 6e-6)]
SPLIT_PRECS = [p for p, _, _ in SPLITS]


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
    gauss = G.split_kind(prec)[1]
    for st in UA.pack_steps(W.gate_tuples(c))[:4]:
        ref = UA.step_operator(n, st)
        for layout in (B.QSIM_LAYOUT_ROW, B.QSIM_LAYOUT_COL):
            buf = G.split_buffer(n, gauss)
            B.qsim_build_step(ctx, n, st, prec, layout, buf)
            G.sync()
            col = layout == B.QSIM_LAYOUT_COL
            got = G.unsplit(buf, fmt, col_major=col)
            assert np.all(got[ref == 0] == 0)
            assert np.all(np.abs(got - ref) <= rel * np.abs(ref) + 1e-12)
            if gauss:  # the sum planes carry re + im of the float32-rounded parts, split the same way
                s32 = (ref.real.astype(np.float32) + ref.imag.astype(np.float32)).astype(np.float64)
                got_s = G.unsplit_sum(buf, fmt, col_major=col)
                assert np.all(got_s[s32 == 0] == 0)
                assert np.all(np.abs(got_s - s32) <= rel * np.abs(s32) + 1e-12)


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
    gauss = G.split_kind(prec)[1]
    dS = G.split_planes(S, fmt, col_major=False, gauss=gauss)
    dU = G.split_planes(U, fmt, col_major=True, gauss=gauss)
    out = G.planar(n)
    out_split = G.split_buffer(n, gauss)
    B.qsim_step_multiply(ctx, n, prec, dS, dU, out, out_split)
    G.sync()
    ref = S @ U
    got = G.to_complex(out)
    assert np.abs(got - ref).max() <= tol
    # the split output is the same product, column-major, re-split from the float32 results
    got_split = G.unsplit(out_split, fmt, col_major=True)
    assert np.abs(got_split - got).max() <= tol
    if gauss:
        s32 = (got.real.astype(np.float32) + got.imag.astype(np.float32)).astype(np.float64)
        assert np.abs(G.unsplit_sum(out_split, fmt, col_major=True) - s32).max() <= tol


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
        bound = G.split_chain_bound(fmt, G.chain_products(n, c.gates), G.split_kind(prec)[1])
        assert G.max_col_err(Ug, Ur) <= bound, (c.family, G.max_col_err(Ug, Ur), bound)
        assert G.max_col_err(psi, ref) <= bound, (c.family, G.max_col_err(psi, ref), bound)


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("n", [12, 13])
def test_precision_sweep_random_circuits(ctx, n, seed):
    """Seeded random circuits random_layers(n, 20, default_rng(seed)), seeds 0-4: every precision against the
    float64 oracle (route B): the final state from |0...0> and 16 sampled columns of U.  float32 chains: max
    |delta| <= 1e-5; split chains: fidelity >= 1 - 1e-6 and the derived 2-norm bound on the state and on every
    sampled column."""
    c = W.random_layers(n, 20, np.random.default_rng(seed))
    g = W.gate_tuples(c)
    P = G.chain_products(n, c.gates)
    ref = fsv.final_state(n, g)
    cols = W.random_columns(n, 16, 5)
    refc = fsv.unitary_columns(n, g, cols)
    for prec in [B.QSIM_FP32_4M, B.QSIM_FP32_3M] + SPLIT_PRECS:
        U = G.planar(n)
        ws = G.workspace(B.qsim_chain_workspace_bytes(n, prec))
        B.qsim_unitary_chain(ctx, n, c.gates, prec, U, ws)
        d_psi = torch.empty(2 << n, dtype=torch.float32, device=G.DEV)
        B.qsim_apply_state(ctx, n, U, None, d_psi)
        psi = G.vec_to_complex(d_psi)
        F = metrics.fidelity(psi, ref)
        err = np.abs(psi - ref).max()
        Uc = U[:, :, cols].cpu().numpy().astype(np.float64)
        Uc = Uc[0] + 1j * Uc[1]
        errU = np.abs(Uc - refc).max()
        print(f"n={n} seed={seed} prec={prec} products={P} max|dpsi|={err:.3e} max|dU|={errU:.3e} "
              f"col2={G.max_col_err(Uc, refc):.3e} 1-F={1 - F:.3e}")
        assert F >= 1 - 1e-6
        if prec in (B.QSIM_FP32_4M, B.QSIM_FP32_3M):
            assert err <= 1e-5 and errU <= 1e-5
        else:
            fmt, gauss = G.split_kind(prec)
            bound = G.split_chain_bound(fmt, P, gauss)
            assert G.max_col_err(psi, ref) <= bound and G.max_col_err(Uc, refc) <= bound
        del U, ws
        torch.cuda.empty_cache()
