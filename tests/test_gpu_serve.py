"""Serving engine (qsim_submit / qsim_poll): continuous batching and the plain FIFO baseline."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fsv, metrics  # noqa: E402
from paper_2305_14398_amd import binding as B  # noqa: E402
from paper_2305_14398_amd import workloads as W  # noqa: E402
from tests import gpu_util as G  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


def serve(ctx, circuits, prec, mode=B.QSIM_SERVE_CONTINUOUS, max_active=64, arena_mib=2048, want_U=False,
          stagger=0.0, policy=B.QSIM_POLICY_ARRIVAL, budget=2.0, aging=0.0):
    arena = torch.empty(arena_mib << 20, dtype=torch.uint8, device=G.DEV)
    psis = [torch.empty(2 << c.n, dtype=torch.float32, device=G.DEV) for c in circuits]
    Us = [G.planar(c.n) if want_U else None for c in circuits]
    G.sync()
    B.qsim_serve_start(ctx, prec, arena, mode=mode, max_active=max_active, policy=policy, iter_budget_tflop=budget,
                       aging_tflop_per_s=aging)
    try:
        ids = []
        for c, p, U in zip(circuits, psis, Us):
            ids.append(B.qsim_submit(ctx, c.n, c.gates, p, d_U=U))
            if stagger:
                time.sleep(stagger)
        results = {}
        t0 = time.time()
        while len(results) < len(ids):
            for i in ids:
                if i not in results:
                    r = B.qsim_poll(ctx, i)
                    if r is not None:
                        results[i] = r
            assert time.time() - t0 < 120, "serving did not finish"
            time.sleep(0.001)
        stats = B.qsim_serve_get_stats(ctx)
    finally:
        B.qsim_serve_stop(ctx)
    G.sync()
    out = [(G.vec_to_complex(p), results[i], G.to_complex(U) if U is not None else None)
           for p, i, U in zip(psis, ids, Us)]
    return out, stats


@pytest.mark.parametrize("prec", [B.QSIM_FP32_4M, B.QSIM_SPLIT_BF16, B.QSIM_SPLIT_BF16_3M])
def test_served_results_match_oracle(ctx, prec):
    circuits = W.batch_mixed(30, seed=21, n_lo=2, n_hi=10, d_lo=2, d_hi=12)
    out, stats = serve(ctx, circuits, prec, want_U=True)
    assert stats["completed"] == len(circuits)
    for c, (psi, res, U) in zip(circuits, out):
        assert res["status"] == B.QSIM_OK
        ref = fsv.final_state(c.n, W.gate_tuples(c))
        assert metrics.fidelity(psi, ref) >= 1 - 1e-6
        if prec == B.QSIM_FP32_4M:
            assert np.abs(psi - ref).max() <= 1e-5
            assert 0 <= res["drift_max"] <= 1e-5
        else:  # the derived split-chain bound on the state (tests/gpu_util.py)
            fmt, gauss = G.split_kind(prec)
            assert G.max_col_err(psi, ref) <= G.split_chain_bound(fmt, G.chain_products(c.n, c.gates), gauss)
        assert res["norm2"] == pytest.approx(float(np.sum(np.abs(psi) ** 2)), rel=1e-12)
        assert res["t_submit_ns"] <= res["t_start_ns"] <= res["t_done_ns"]
        assert res["n_steps"] == len(B.qsim_pack_steps(c.n, c.gates)) - 1


def test_alone_and_in_the_mix_are_identical(ctx):
    probe = W.random_layers(9, 10, np.random.default_rng(4))
    mix = W.batch_mixed(40, seed=5, n_lo=3, n_hi=10, d_lo=5, d_hi=20)
    for prec in (B.QSIM_FP32_4M, B.QSIM_SPLIT_BF16, B.QSIM_SPLIT_BF16_3M):
        alone, _ = serve(ctx, [probe], prec, want_U=True)
        mixed, stats = serve(ctx, mix[:20] + [probe] + mix[20:], prec, want_U=True, stagger=0.0005)
        assert stats["peak_active"] > 1
        np.testing.assert_array_equal(alone[0][0], mixed[20][0])
        np.testing.assert_array_equal(alone[0][2], mixed[20][2])


def test_fifo_baseline_matches_continuous(ctx):
    circuits = [c for c in W.batch_mixed(16, seed=9, n_lo=6, n_hi=10, d_lo=2, d_hi=10)]
    cont, _ = serve(ctx, circuits, B.QSIM_FP32_4M)
    fifo, stats = serve(ctx, circuits, B.QSIM_FP32_4M, mode=B.QSIM_SERVE_FIFO)
    assert stats["peak_active"] == 1 and stats["grouped_launches"] == 0
    for (a, ra, _), (b, rb, _) in zip(cont, fifo):
        np.testing.assert_array_equal(a, b)
        assert ra["norm2"] == rb["norm2"]


def test_admission_waits_for_arena_room(ctx):
    # each 10-qubit request needs 3 x 8 MiB (workspace + U); a 40 MiB arena admits one at a time
    circuits = [W.qft(10), W.dj(10, 77), W.ghz_chain(10), W.random_layers(10, 3, np.random.default_rng(0))]
    out, stats = serve(ctx, circuits, B.QSIM_FP32_4M, arena_mib=40)
    assert stats["peak_active"] == 1
    assert stats["arena_high_water"] <= 40 << 20
    for c, (psi, res, _) in zip(circuits, out):
        assert res["status"] == B.QSIM_OK
        assert np.abs(psi - fsv.final_state(c.n, W.gate_tuples(c))).max() <= 1e-5


def test_errors_full_oom_unknown_and_cancel(ctx):
    arena = torch.empty(4 << 20, dtype=torch.uint8, device=G.DEV)
    B.qsim_serve_start(ctx, B.QSIM_FP32_4M, arena, max_active=1, queue_capacity=2)
    try:
        psi = torch.empty(2 << 10, dtype=torch.float32, device=G.DEV)
        with pytest.raises(B.QsimError) as ei:
            B.qsim_submit(ctx, 10, W.qft(10).gates, psi)  # 24 MiB > 4 MiB arena
        assert ei.value.status == B.QSIM_E_OOM
        with pytest.raises(B.QsimError) as ei:
            B.qsim_poll(ctx, 12345)
        assert ei.value.status == B.QSIM_E_UNKNOWN_ID
        small = torch.empty(2 << 8, dtype=torch.float32, device=G.DEV)
        ids, full = [], False
        for _ in range(50):
            try:
                ids.append(B.qsim_submit(ctx, 8, W.qft(8).gates, small))
            except B.QsimError as e:
                assert e.status == B.QSIM_E_FULL
                full = True
                break
        assert full
    finally:
        B.qsim_serve_stop(ctx)
    with pytest.raises(B.QsimError):
        B.qsim_poll(ctx, ids[0])  # the engine (and its results) are gone


def test_probe_drift_matches_full_check(ctx):
    for n in (4, 8, 11):
        c = W.random_layers(n, 6, np.random.default_rng(n))
        U = G.planar(n)
        ws = G.workspace(B.qsim_chain_workspace_bytes(n, B.QSIM_FP32_4M))
        B.qsim_unitary_chain(ctx, n, c.gates, B.QSIM_FP32_4M, U, ws)
        mx, l2 = B.qsim_unitarity_drift_probe(ctx, n, U)
        Uc = G.to_complex(U)
        N = 1 << n
        j = np.arange(N)
        t = (j * 0.61803398874989484820) % 1.0
        x = np.exp(2j * np.pi * t) / np.sqrt(N)
        d = Uc.conj().T @ (Uc @ x) - x
        assert mx == pytest.approx(np.abs(d).max(), rel=1e-6, abs=1e-15)
        assert l2 == pytest.approx(np.linalg.norm(d), rel=1e-6, abs=1e-15)
        assert mx < 1e-5


def test_large_requests_continuous_equals_fifo(ctx):
    rng = np.random.default_rng(8)
    circuits = [W.random_layers(13, 4, rng), W.qft(12), W.random_layers(12, 6, rng), W.dj(11, 99),
                W.random_layers(7, 12, rng), W.random_layers(11, 8, rng), W.ghz_chain(13), W.qft(9)]
    cont, _ = serve(ctx, circuits, B.QSIM_SPLIT_BF16, arena_mib=24 << 10)
    fifo, _ = serve(ctx, circuits, B.QSIM_SPLIT_BF16, mode=B.QSIM_SERVE_FIFO, arena_mib=24 << 10)
    for c, (a, ra, _), (b, rb, _) in zip(circuits, cont, fifo):
        assert ra["drift_max"] < 1e-3 and rb["drift_max"] < 1e-3, (c.family, c.n, ra["drift_max"], rb["drift_max"])
        np.testing.assert_array_equal(a, b, err_msg=f"{c.family} n={c.n}")


def test_shortest_policy_gives_identical_results_and_finishes_small_first(ctx):
    big = [W.random_layers(12, 6, np.random.default_rng(s)) for s in range(2)]
    small = W.batch_mixed(20, seed=13, n_lo=4, n_hi=8, d_lo=2, d_hi=10)
    circuits = big + small  # the large ones arrive first
    arrival, _ = serve(ctx, circuits, B.QSIM_SPLIT_BF16)
    shortest, stats = serve(ctx, circuits, B.QSIM_SPLIT_BF16, policy=B.QSIM_POLICY_SHORTEST, budget=0.05)
    for (a, ra, _), (b, rb, _) in zip(arrival, shortest):
        np.testing.assert_array_equal(a, b)
        assert rb["status"] == B.QSIM_OK
    # with least-work-first, every small request is done before either large one
    last_small = max(r["t_done_ns"] for _, r, _ in shortest[2:])
    first_big = min(r["t_done_ns"] for _, r, _ in shortest[:2])
    assert last_small <= first_big


def test_aged_policy_identical_results_and_oldest_first_with_large_credit(ctx):
    """With an aging credit far above any request's work, the aged policy serves the oldest request first;
    results are bit-identical to arrival order whatever the policy."""
    big = [W.random_layers(12, 6, np.random.default_rng(s)) for s in range(2)]
    small = W.batch_mixed(12, seed=14, n_lo=4, n_hi=8, d_lo=2, d_hi=10)
    circuits = big + small
    arrival, _ = serve(ctx, circuits, B.QSIM_SPLIT_BF16)
    aged, _ = serve(ctx, circuits, B.QSIM_SPLIT_BF16, policy=B.QSIM_POLICY_AGED, budget=0.05, aging=1e9)
    for (a, _, _), (b, rb, _) in zip(arrival, aged):
        np.testing.assert_array_equal(a, b)
        assert rb["status"] == B.QSIM_OK
    first_big = min(r["t_done_ns"] for _, r, _ in aged[:2])
    assert first_big <= min(r["t_done_ns"] for _, r, _ in aged[2:])


def test_policy_validation(ctx):
    arena = torch.empty(1 << 20, dtype=torch.uint8, device=G.DEV)
    with pytest.raises(B.QsimError, match="policy"):
        B.qsim_serve_start(ctx, B.QSIM_FP32_4M, arena, policy=5)
    with pytest.raises(B.QsimError, match="budget"):
        B.qsim_serve_start(ctx, B.QSIM_FP32_4M, arena, policy=B.QSIM_POLICY_SHORTEST, iter_budget_tflop=0.0)
    with pytest.raises(B.QsimError, match="aging"):
        B.qsim_serve_start(ctx, B.QSIM_FP32_4M, arena, policy=B.QSIM_POLICY_AGED, aging_tflop_per_s=0.0)


def test_served_custom_ops_match_oracle(ctx):
    from types import SimpleNamespace
    from tests.custom_ops import lib_gates
    circuits, refs = [], []
    for i, n in enumerate([4, 8, 10]):
        g = W.with_custom_ops(W.gate_tuples(W.random_layers(n, 3, np.random.default_rng(i))), n, [1, 4, 5], 950 + i)
        circuits.append(SimpleNamespace(n=n, gates=lib_gates(g)))
        refs.append(g)
    out, _ = serve(ctx, circuits, B.QSIM_FP32_4M)
    for c, g, (psi, res, _) in zip(circuits, refs, out):
        assert res["status"] == B.QSIM_OK
        assert np.abs(psi - fsv.final_state(c.n, g)).max() <= 1e-5


def test_full_served_config_sampled_against_oracle(ctx):
    """The served configuration at full size: 200 Poisson arrivals at 200 req/s (seed 0), n ~ U{6..13}, depth
    ~ U{10..40}, split-bf16, least-work-first continuous batching, submitted at the trace's mean spacing.  Every
    request completes with its float64 norm and probe drift; the largest requests and a regular sample match
    the oracle's final state (route B) with fidelity >= 1 - 1e-6."""
    trace = W.poisson_trace(200, 200.0, 0, n_lo=6, n_hi=13, d_lo=10, d_hi=40)
    circuits = [c for _, c in trace]
    out, stats = serve(ctx, circuits, B.QSIM_SPLIT_BF16, arena_mib=48 << 10, policy=B.QSIM_POLICY_SHORTEST,
                       budget=2.0, stagger=0.005)
    assert stats["completed"] == len(circuits)
    for c, (psi, res, _) in zip(circuits, out):
        assert res["status"] == B.QSIM_OK
        assert 0 <= res["drift_max"] <= 1e-3, (c.family, c.n, res["drift_max"])
        assert res["norm2"] == pytest.approx(float(np.sum(np.abs(psi) ** 2)), rel=1e-12)
    largest = sorted(range(len(circuits)), key=lambda i: -circuits[i].n)[:5]
    for i in sorted(set(largest + list(range(0, len(circuits), 25)))):
        c = circuits[i]
        ref = fsv.final_state(c.n, W.gate_tuples(c))
        assert metrics.fidelity(out[i][0], ref) >= 1 - 1e-6, (i, c.family, c.n)
        assert G.max_col_err(out[i][0], ref) <= G.split_chain_bound("bf16", G.chain_products(c.n, c.gates))


def test_served_full_drift_equals_the_synchronous_check(ctx):
    """QSIM_REQ_DRIFT_FULL: the engine runs the full float64 check on each finished unitary; its values equal
    qsim_unitarity_drift of the same returned U (the same kernels and partial counts, so bit for bit), and the
    probe and full flags are exclusive."""
    circuits = W.batch_mixed(12, seed=31, n_lo=4, n_hi=11, d_lo=3, d_hi=10)
    arena = torch.empty(2 << 30, dtype=torch.uint8, device=G.DEV)
    psis = [torch.empty(2 << c.n, dtype=torch.float32, device=G.DEV) for c in circuits]
    Us = [G.planar(c.n) for c in circuits]
    B.qsim_serve_start(ctx, B.QSIM_FP32_3M, arena)
    try:
        with pytest.raises(B.QsimError, match="exclusive"):
            B.qsim_submit(ctx, circuits[0].n, circuits[0].gates, psis[0],
                          flags=B.QSIM_REQ_DRIFT_PROBE | B.QSIM_REQ_DRIFT_FULL)
        ids = [B.qsim_submit(ctx, c.n, c.gates, p, d_U=U, full_drift=True) for c, p, U in zip(circuits, psis, Us)]
        results = {}
        t0 = time.time()
        while len(results) < len(ids):
            for i in ids:
                if i not in results:
                    r = B.qsim_poll(ctx, i)
                    if r is not None:
                        results[i] = r
            assert time.time() - t0 < 120, "serving did not finish"
            time.sleep(0.001)
    finally:
        B.qsim_serve_stop(ctx)
    G.sync()
    for c, i, U in zip(circuits, ids, Us):
        r = results[i]
        assert r["status"] == B.QSIM_OK
        mx, fro = B.qsim_unitarity_drift(ctx, c.n, U)
        assert (r["drift_max"], r["drift_l2"]) == (mx, fro), (c.family, c.n)
        assert mx <= 1e-5
