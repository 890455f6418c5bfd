"""The allocation-free drift entry point (qsim_unitarity_drift_noalloc) against
the context-based asynchronous one (qsim_unitarity_drift_async).

Both run the same kernels with the same persistent grid and the same
fixed-order reduction of the per-workgroup partial sums; only where the partial
sums live differs (a static per-device array instead of the context's
scratch).  The bar is therefore bit-identical results.  Calls run back to
back, each smaller than the one before, so a call that read a stale partial
sum left by a larger call (2048 pairs at 11 qubits, 3 at 6, 1 at 3) would
disagree with the context-based call.  The oracle's drift of the same float32
matrix (exact in float64) is checked as well, to 1e-12 absolute on unitary
chains and 1e-10 relative on a non-unitary matrix.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import metrics  # noqa: E402
from paper_2305_14398_amd import binding as B  # noqa: E402
from paper_2305_14398_amd import workloads as W  # noqa: E402
from tests import gpu_util as G  # noqa: E402

pytestmark = pytest.mark.gpu


def _chain(ctx, n, gates):
    U = G.planar(n)
    ws = G.workspace(B.qsim_chain_workspace_bytes(n, B.QSIM_FP32_4M))
    B.qsim_unitary_chain(ctx, n, gates, B.QSIM_FP32_4M, U, ws)
    return U


def _both(ctx, n, U):
    ref = torch.full((2,), -1.0, dtype=torch.float64, device=G.DEV)
    got = torch.full((2,), -2.0, dtype=torch.float64, device=G.DEV)
    B.qsim_unitarity_drift_async(ctx, n, U, ref)
    B.qsim_unitarity_drift_noalloc(n, U, got)
    G.sync()
    return tuple(ref.cpu().tolist()), tuple(got.cpu().tolist())


def test_noalloc_drift_equals_context_drift_on_shrinking_inputs():
    with B.Context(0) as ctx:
        for n in (11, 6, 3):  # 2048 partial pairs, then 3, then the one-block kernel
            U = _chain(ctx, n, W.random_layers(n, 6, np.random.default_rng(100 + n)).gates)
            ref, got = _both(ctx, n, U)
            assert got == ref, (n, got, ref)
            rmx, rfro = metrics.unitarity_drift(G.to_complex(U))
            assert abs(got[0] - rmx) <= 1e-12 and abs(got[1] - rfro) <= 1e-12
            assert got[0] < 1e-5


def test_noalloc_drift_non_unitary_then_smaller():
    with B.Context(0) as ctx:
        rng = np.random.default_rng(7)
        for n in (12, 8):  # the 64-wide drift tile, then the 32-wide one
            N = 1 << n
            M = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / math.sqrt(N)
            dM = G.planar(n, M)
            ref, got = _both(ctx, n, dM)
            assert got == ref, (n, got, ref)
            rmx, rfro = metrics.unitarity_drift(G.to_complex(dM))
            assert got[0] == pytest.approx(rmx, rel=1e-10) and got[1] == pytest.approx(rfro, rel=1e-10)
            assert got[0] > 0.1


def test_noalloc_drift_rejects_bad_arguments():
    U = G.planar(4)
    out = torch.empty(2, dtype=torch.float64, device=G.DEV)
    for n in (0, 17):
        with pytest.raises(B.QsimError) as e:
            B.qsim_unitarity_drift_noalloc(n, U, out)
        assert e.value.status == B.QSIM_E_RANGE
    with pytest.raises(B.QsimError) as e:
        B.qsim_unitarity_drift_noalloc(4, U, 0)
    assert e.value.status == B.QSIM_E_INVALID
