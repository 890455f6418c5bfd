"""Grouped batches of mixed-size circuits: per-circuit results equal the single-circuit
chain (bit for bit where both use the same tile code), match the oracle, are the same alone
and in the mix, and survive repeated hipGraph replays with eager work in between."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fsv, unitary as UA  # noqa: E402
from paper_2305_14398_amd import binding as B  # noqa: E402
from paper_2305_14398_amd import workloads as W  # noqa: E402
from tests import gpu_util as G  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


def run_batch(ctx, circuits, prec, graph=False, launches=1, between=None):
    outs = [G.planar(c.n) for c in circuits]
    ws = G.workspace(B.qsim_batch_workspace_bytes(circuits, prec))
    plan = B.BatchPlan(ctx, circuits, outs, prec, ws, graph=graph)
    results = []
    for r in range(launches):
        for o in outs:
            o.fill_(float("nan"))
        plan.launch()
        G.sync()
        results.append([G.to_complex(o) for o in outs])
        if between:
            between(r)
    info = plan.info()
    plan.close()
    return results, info


def single(ctx, c, prec):
    U = G.planar(c.n)
    ws = G.workspace(B.qsim_chain_workspace_bytes(c.n, prec))
    B.qsim_unitary_chain(ctx, c.n, c.gates, prec, U, ws)
    G.sync()
    return G.to_complex(U)


PRECS = [B.QSIM_FP32_4M, B.QSIM_FP32_3M, B.QSIM_SPLIT_BF16, B.QSIM_SPLIT_FP16, B.QSIM_SPLIT_BF16_3M,
         B.QSIM_SPLIT_FP16_3M]


@pytest.mark.parametrize("prec", PRECS)
def test_batch_matches_single_and_oracle(ctx, prec):
    circuits = W.batch_mixed(40, seed=7, n_lo=1, n_hi=9, d_lo=1, d_hi=8)
    circuits.append(W.Circuit(3, [], "empty"))
    (res,), info = run_batch(ctx, circuits, prec)
    assert info["iterations"] >= 1
    for c, U in zip(circuits, res):
        ref = UA.circuit_unitary(c.n, W.gate_tuples(c))
        if prec not in (B.QSIM_FP32_4M, B.QSIM_FP32_3M):
            # the derived split-chain bound (column 2-norms; see tests/gpu_util.py)
            fmt, gauss = G.split_kind(prec)
            tol = G.split_chain_bound(fmt, G.chain_products(c.n, c.gates), gauss)
            assert G.max_col_err(U, ref) <= tol, (c.family, c.n, G.max_col_err(U, ref), tol)
        else:
            tol = 1e-5
            assert np.abs(U - ref).max() <= tol, (c.family, c.n)
        S = single(ctx, c, prec)
        if c.n != 5:  # n = 5 runs 32x32 MFMA tiles alone and the whole-product path in a batch
            np.testing.assert_array_equal(U, S, err_msg=f"{c.family} n={c.n}")
        else:
            assert G.max_col_err(U, S) <= 2 * tol


def test_alone_and_in_the_mix_are_identical(ctx):
    mix = W.batch_mixed(24, seed=3, n_lo=4, n_hi=10, d_lo=2, d_hi=10)
    probe = W.qft(10)
    for prec in (B.QSIM_FP32_4M, B.QSIM_SPLIT_BF16, B.QSIM_SPLIT_BF16_3M):
        (alone,), _ = run_batch(ctx, [probe], prec)
        (mixed,), _ = run_batch(ctx, mix[:12] + [probe] + mix[12:], prec)
        np.testing.assert_array_equal(alone[0], mixed[12])


def test_graph_replays_match_eager(ctx):
    circuits = W.batch_mixed(30, seed=11, n_lo=2, n_hi=9, d_lo=2, d_hi=6)
    for prec in (B.QSIM_FP32_4M, B.QSIM_SPLIT_BF16, B.QSIM_SPLIT_BF16_3M):
        (eager,), _ = run_batch(ctx, circuits, prec)
        scratch = torch.empty(1 << 20, device=G.DEV)

        def eager_work(r):
            scratch.normal_()
            float(scratch.sum().item())
            G.sync()

        replays, _ = run_batch(ctx, circuits, prec, graph=True, launches=4, between=eager_work)
        for rep in replays:
            for a, b in zip(rep, eager):
                np.testing.assert_array_equal(a, b)


def test_autotune_records_choices_and_stays_correct(ctx):
    # a range starting below 7 qubits must not give a 6-qubit product a 128-wide tile (that is zero tiles)
    timings = B.qsim_autotune(ctx, B.QSIM_FP32_4M, 4, 10)
    assert min(timings) == 7
    assert B.qsim_tune_get(ctx, B.QSIM_FP32_4M)[6] == 64
    c6 = W.qft(6)
    (res6,), _ = run_batch(ctx, [c6, W.random_layers(8, 3, np.random.default_rng(0))], B.QSIM_FP32_4M)
    assert np.abs(res6[0] - UA.circuit_unitary(6, W.gate_tuples(c6))).max() <= 1e-5
    tiles = B.qsim_tune_get(ctx, B.QSIM_FP32_4M)
    for n in range(7, 11):
        t64, t128 = timings[n]
        assert t64 > 0 and t128 > 0
        assert tiles[n] == (64 if t64 < t128 else 128)
    c = W.random_layers(9, 4, np.random.default_rng(1))
    ref = UA.circuit_unitary(9, W.gate_tuples(c))
    for tile in (64, 128):
        B.qsim_tune_set(ctx, B.QSIM_FP32_4M, 9, tile)
        assert np.abs(single(ctx, c, B.QSIM_FP32_4M) - ref).max() <= 1e-5
        (res,), _ = run_batch(ctx, [c], B.QSIM_FP32_4M)
        assert np.abs(res[0] - ref).max() <= 1e-5
    B.qsim_tune_set(ctx, B.QSIM_FP32_4M, 9, tiles[9])


def test_tile_cache_round_trip_and_rejection(ctx, tmp_path):
    """qsim_tune_save / qsim_tune_load: the table, tuned flags and timings come back as saved; a file from
    another build or device, or with an invalid tile, is rejected and leaves the table unchanged."""
    prec = B.QSIM_SPLIT_BF16_3M
    B.qsim_autotune(ctx, prec, 7, 9)
    saved_tiles = B.qsim_tune_get(ctx, prec)
    saved_ms = B.qsim_tune_ms(ctx, prec)
    assert set(saved_ms) == {7, 8, 9} and all(a > 0 and b > 0 for a, b in saved_ms.values())
    path = tmp_path / "tiles.json"
    B.qsim_tune_save(ctx, str(path))
    text = path.read_text()
    import json
    doc = json.loads(text)
    assert doc["build"] == B.qsim_build_id()
    assert doc["tiles"][prec] == saved_tiles
    other = 64 if saved_tiles[8] == 128 else 128
    B.qsim_tune_set(ctx, prec, 8, other)
    B.qsim_tune_load(ctx, str(path))
    assert B.qsim_tune_get(ctx, prec) == saved_tiles
    assert B.qsim_tune_ms(ctx, prec) == saved_ms
    B.qsim_tune_set(ctx, prec, 8, other)
    for bad in (text.replace(doc["build"], "0" * 16), text.replace(doc["device"], "another device"),
                text.replace('"tiles": [', '"tiles": [\n  [0, 0, 0, 0, 0, 0, 64, 96,', 1)):
        path.write_text(bad)
        with pytest.raises(B.QsimError) as e:
            B.qsim_tune_load(ctx, str(path))
        assert e.value.status == B.QSIM_E_INVALID
        assert B.qsim_tune_get(ctx, prec)[8] == other
    B.qsim_tune_set(ctx, prec, 8, saved_tiles[8])


def test_one_shot_batched_call(ctx):
    circuits = [W.ghz_chain(5), W.dj(7, 5), W.qft(8)]
    outs = [G.planar(c.n) for c in circuits]
    ws = G.workspace(B.qsim_batch_workspace_bytes(circuits, B.QSIM_FP32_4M))
    B.qsim_unitary_chain_batched(ctx, circuits, outs, B.QSIM_FP32_4M, ws)
    for c, o in zip(circuits, outs):
        ref = UA.circuit_unitary(c.n, W.gate_tuples(c))
        assert np.abs(G.to_complex(o) - ref).max() <= 1e-5


@pytest.mark.parametrize("prec", [B.QSIM_FP32_4M, B.QSIM_SPLIT_BF16, B.QSIM_SPLIT_FP16, B.QSIM_SPLIT_BF16_3M,
                                  B.QSIM_SPLIT_FP16_3M])
def test_large_circuits_batch_equals_single(ctx, prec):
    rng = np.random.default_rng(2)
    circuits = [W.random_layers(13, 3, rng), W.qft(12), W.random_layers(12, 4, rng), W.dj(11, 333),
                W.random_layers(11, 5, rng), W.ghz_chain(13)]
    outs = [G.planar(c.n) for c in circuits]
    ws = G.workspace(B.qsim_batch_workspace_bytes(circuits, prec))
    plan = B.BatchPlan(ctx, circuits, outs, prec, ws)
    plan.launch()
    G.sync()
    plan.close()
    del ws
    for c, o in zip(circuits, outs):
        U = G.planar(c.n)
        wss = G.workspace(B.qsim_chain_workspace_bytes(c.n, prec))
        B.qsim_unitary_chain(ctx, c.n, c.gates, prec, U, wss)
        G.sync()
        assert torch.equal(o, U), (c.family, c.n)
        mx, _ = B.qsim_unitarity_drift_probe(ctx, c.n, o)
        assert mx < (1e-3 if prec in (B.QSIM_SPLIT_BF16, B.QSIM_SPLIT_BF16_3M) else 1e-5), (c.family, c.n, mx)
        del U, wss
    torch.cuda.empty_cache()


def test_batch_with_custom_ops_matches_single_and_oracle(ctx):
    """Registered custom operations (Section 5.2.2) inside a mixed batch: bit-identical to the single-circuit
    chain and within the complex64 tolerance of the oracle."""
    from types import SimpleNamespace
    from tests.custom_ops import lib_gates
    circuits, refs = [], []
    for i, n in enumerate([3, 6, 7, 9, 11]):
        g = W.with_custom_ops(W.gate_tuples(W.random_layers(n, 3, np.random.default_rng(i))), n, [2, 3, 6], 900 + i)
        circuits.append(SimpleNamespace(n=n, gates=lib_gates(g), family="custom"))
        refs.append(g)
    (res,), _ = run_batch(ctx, circuits, B.QSIM_FP32_4M)
    for c, g, U in zip(circuits, refs, res):
        cols = W.random_columns(c.n, 8, 3)
        assert np.abs(U[:, cols] - fsv.unitary_columns(c.n, g, cols)).max() <= 1e-5
        np.testing.assert_array_equal(U, single(ctx, c, B.QSIM_FP32_4M))


def test_full_batched_config_sampled_against_oracle(ctx):
    """The batched configuration at full size, in the launch configuration the benchmark times: 512 seeded
    circuits (n ~ U{4..11}, families ghz_chain/dj/qft/random, depth ~ U{5..30}, seed 0), 3M, autotuned tiles,
    one graph-captured plan launched twice.  Every result is checked by a property that holds at any size
    (float64 probe drift); the largest circuits and a regular sample are checked against the oracle (route B)
    on sampled columns; the replay equals the first launch bit for bit."""
    prec = B.QSIM_FP32_3M
    circuits = W.batch_mixed(512, seed=0, n_lo=4, n_hi=11, d_lo=5, d_hi=30)
    B.qsim_autotune(ctx, prec, 7, 11)
    outs = [G.planar(c.n) for c in circuits]
    ws = G.workspace(B.qsim_batch_workspace_bytes(circuits, prec))
    plan = B.BatchPlan(ctx, circuits, outs, prec, ws, graph=True)
    plan.launch()
    G.sync()
    first = [o.clone() for o in outs[:24]]
    plan.launch()
    G.sync()
    plan.close()
    del ws
    for a, o in zip(first, outs[:24]):
        assert torch.equal(a, o)
    for c, o in zip(circuits, outs):
        mx, _ = B.qsim_unitarity_drift_probe(ctx, c.n, o)
        assert mx <= 1e-5, (c.family, c.n, mx)
    largest = sorted(range(len(circuits)), key=lambda i: -circuits[i].n)[:6]
    for i in sorted(set(largest + list(range(0, len(circuits), 48)))):
        c = circuits[i]
        cols = W.random_columns(c.n, 4, i)
        got = G.to_complex(outs[i][:, :, torch.as_tensor(cols, device=G.DEV)])
        ref = fsv.unitary_columns(c.n, W.gate_tuples(c), cols)
        assert np.abs(got - ref).max() <= 1e-5, (i, c.family, c.n)
    del outs, first
    torch.cuda.empty_cache()
