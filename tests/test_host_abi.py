"""Host-side checks of libqsim that need no GPU: loading, exported symbols,
step formation, workspace sizes and argument validation (every call checks
its arguments before touching the device)."""
import math
import os
import re

import numpy as np
import pytest

from oracle import unitary as UA
from paper_2305_14398_amd import binding as B
from paper_2305_14398_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 256 * 4096  # an aligned address that is never dereferenced: validation fails first


def header_functions():
    with open(os.path.join(ROOT, "include", "qsim.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsim_[a-z0-9_]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_function():
    L = B.lib()
    names = header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), f"{name} declared in qsim.h but not exported"
    assert "gfx950" in B.qsim_version()


def test_header_struct_size_matches_binding():
    with open(os.path.join(ROOT, "include", "qsim.h")) as f:
        assert "88 bytes" in f.read()
    assert B.ctypes.sizeof(B.qsim_gate) == 88


def _families(n, rng):
    out = [W.ghz_chain(n), W.ghz_fanout(n), W.qft(n), W.random_layers(n, 6, rng)]
    if n >= 2:
        out.append(W.dj(n, int(rng.integers(0, 1 << (n - 1)))))
    return out


@pytest.mark.parametrize("n", [1, 2, 5, 8, 11, 13, 16])
def test_pack_steps_matches_oracle_rule(n):
    rng = np.random.default_rng(n)
    for c in _families(n, rng):
        off = B.qsim_pack_steps(n, c.gates)
        steps = UA.pack_steps(W.gate_tuples(c))
        ref = [0]
        for st in steps:
            ref.append(ref[-1] + len(st))
        assert off == ref, c.family


def test_pack_step_counts_of_paper_workloads():
    assert len(B.qsim_pack_steps(11, W.qft(11).gates)) - 1 == 71
    assert len(B.qsim_pack_steps(5, W.ghz_chain(5).gates)) - 1 == 5
    # Deutsch-Jozsa: X + H layer share one step, oracle CNOTs one each, final H layer one step
    mask = 0b1011
    k = len(B.qsim_pack_steps(6, W.dj(6, mask).gates)) - 1
    assert k == len(UA.pack_steps(W.gate_tuples(W.dj(6, mask))))


def test_workspace_bytes():
    for n in (1, 5, 11, 13):
        mb = 8 << (2 * n)
        assert B.qsim_chain_workspace_bytes(n, B.QSIM_FP32_4M) == 2 * mb
        assert B.qsim_chain_workspace_bytes(n, B.QSIM_FP32_3M) == 2 * mb
        assert B.qsim_chain_workspace_bytes(n, B.QSIM_SPLIT_BF16) == 3 * mb
        assert B.qsim_chain_workspace_bytes(n, B.QSIM_SPLIT_FP16) == 3 * mb
        # three-product split operands carry six 16-bit planes (12 N^2 bytes)
        assert B.qsim_chain_workspace_bytes(n, B.QSIM_SPLIT_BF16_3M) == 3 * (12 << (2 * n))
        assert B.qsim_chain_workspace_bytes(n, B.QSIM_SPLIT_FP16_3M) == 3 * (12 << (2 * n))
    assert B.qsim_chain_workspace_bytes(0, 0) == 0
    assert B.qsim_chain_workspace_bytes(17, 0) == 0
    assert B.qsim_chain_workspace_bytes(5, 9) == 0
    assert B.qsim_chain_workspace_bytes(5, 6) == 0


def _expect(status, fn, *args, match=None):
    with pytest.raises(B.QsimError) as ei:
        fn(*args)
    assert ei.value.status == status, str(ei.value)
    if match:
        assert re.search(match, ei.value.message), ei.value.message


def test_gate_validation_in_pack():
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 3, [("H", (3,), None)], match="outside")
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 3, [("H", (-1,), None)], match="outside")
    bad = B.gate_record(("CNOT", (0, 1), None))
    bad.control = 0
    bad.target = 0
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 3, [bad], match="control equals target")
    kind = B.gate_record(("H", (0,), None))
    kind.kind = 42
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 3, [kind], match="unknown kind")
    swap = B.gate_record(("SWAP", (0, 1), None))
    swap.control = -1
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 3, [swap], match="SWAP")
    nan = B.gate_record(("RX", (0,), 1.0))
    nan.theta = math.nan
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 3, [nan], match="angle")
    res = B.gate_record(("H", (0,), None))
    res.op_id = 1
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 3, [res], match="op_id")
    _expect(B.QSIM_E_RANGE, B.qsim_pack_steps, 0, [])
    _expect(B.QSIM_E_RANGE, B.qsim_pack_steps, 17, [])


def test_custom_matrix_must_be_unitary():
    r = 1 / math.sqrt(2)
    good = ("U2", (0,), None, [[r, 1j * r], [1j * r, r]])
    assert B.qsim_pack_steps(2, [good]) == [0, 1]
    bad = ("U2", (0,), None, [[1, 1], [0, 1]])
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 2, [bad], match="not unitary")


def test_build_step_validation_without_device():
    g = [("H", (0,), None), ("CNOT", (1, 2), None)]
    # overlapping spans within one step
    _expect(B.QSIM_E_INVALID, B.qsim_build_step, None, 3, [("CNOT", (0, 2), None), ("H", (1,), None)], 0, 0, FAKE,
            match="overlaps")
    _expect(B.QSIM_E_INVALID, B.qsim_build_step, None, 3, g, 0, 0, FAKE + 4, match="aligned")
    _expect(B.QSIM_E_INVALID, B.qsim_build_step, None, 3, g, 0, 7, FAKE, match="layout")
    _expect(B.QSIM_E_INVALID, B.qsim_build_step, None, 3, g, 9, 0, FAKE, match="precision")
    _expect(B.QSIM_E_RANGE, B.qsim_build_step, None, 0, g, 0, 0, FAKE)
    too_many = [("H", (q,), None) for q in range(16)] + [("X", (0,), None)]
    _expect(B.QSIM_E_INVALID, B.qsim_build_step, None, 16, too_many, 0, 0, FAKE)
    # valid arguments and no context: the context check is the last one
    _expect(B.QSIM_E_INVALID, B.qsim_build_step, None, 3, g, 0, 0, FAKE, match="context is NULL")


def test_chain_validation_without_device():
    g = W.qft(4).gates
    mb = 8 << 8
    _expect(B.QSIM_E_RANGE, B.qsim_unitary_chain, None, 4, g, 0, FAKE, FAKE * 4, mb, match="workspace")
    _expect(B.QSIM_E_INVALID, B.qsim_unitary_chain, None, 4, g, 0, FAKE, FAKE, 2 * mb, match="overlaps")
    _expect(B.QSIM_E_INVALID, B.qsim_unitary_chain, None, 4, g, 0, FAKE, FAKE * 4, 2 * mb, [0, 3],
            match="offsets")
    # a step of the caller's offsets that has overlapping spans
    _expect(B.QSIM_E_INVALID, B.qsim_unitary_chain, None, 4, g, 0, FAKE, FAKE * 4, 2 * mb,
            [0, 2] + list(range(3, len(g) + 1)), match="step 0")
    _expect(B.QSIM_E_INVALID, B.qsim_unitary_chain, None, 4, g, 0, FAKE, FAKE * 4, 2 * mb, match="context is NULL")


def test_fused_chain_and_product_validation_without_device():
    g = W.qft(4).gates
    mb = 8 << 8
    # one matrix of workspace: the fused chain stores no step operator
    assert B.qsim_chain_fused_workspace_bytes(4, B.QSIM_FP32_3M) == mb
    assert B.qsim_chain_fused_workspace_bytes(4, B.QSIM_FP32_4M) == mb
    assert B.qsim_chain_workspace_bytes(4, B.QSIM_FP32_3M) == 2 * mb
    assert B.qsim_chain_fused_workspace_bytes(4, B.QSIM_SPLIT_BF16) == 0
    assert B.qsim_chain_fused_workspace_bytes(0, B.QSIM_FP32_4M) == 0
    f = B.qsim_unitary_chain_fused
    _expect(B.QSIM_E_INVALID, f, None, 4, g, B.QSIM_SPLIT_BF16, FAKE, FAKE * 4, 3 * mb, match="float32")
    _expect(B.QSIM_E_RANGE, f, None, 4, g, 0, FAKE, FAKE * 4, mb - 8, match="workspace")
    _expect(B.QSIM_E_INVALID, f, None, 4, g, 0, FAKE, FAKE, mb, match="overlaps")
    _expect(B.QSIM_E_INVALID, f, None, 4, g, 0, FAKE, FAKE * 4, mb, [0, 2] + list(range(3, len(g) + 1)),
            match="step 0")
    _expect(B.QSIM_E_INVALID, f, None, 4, g, 0, FAKE, FAKE * 4, mb, match="context is NULL")
    m = B.qsim_step_multiply_fused
    step = [("H", (0,), None), ("CNOT", (1, 2), None)]
    _expect(B.QSIM_E_INVALID, m, None, 4, B.QSIM_SPLIT_FP16, step, FAKE, FAKE * 2, match="float32")
    _expect(B.QSIM_E_INVALID, m, None, 4, 0, step, FAKE, FAKE, match="aliases")
    _expect(B.QSIM_E_INVALID, m, None, 4, 0, step, FAKE + 8, FAKE * 2, match="aligned")
    _expect(B.QSIM_E_INVALID, m, None, 4, 0, [("H", (1,), None), ("CNOT", (0, 2), None)], FAKE, FAKE * 2)
    _expect(B.QSIM_E_RANGE, m, None, 17, 0, step, FAKE, FAKE * 2)
    _expect(B.QSIM_E_INVALID, m, None, 4, 0, step, FAKE, FAKE * 2, match="context is NULL")


def test_multiply_apply_drift_validation_without_device():
    _expect(B.QSIM_E_INVALID, B.qsim_step_multiply, None, 5, 0, FAKE, FAKE * 2, FAKE, None, match="aliases")
    _expect(B.QSIM_E_INVALID, B.qsim_step_multiply, None, 5, 0, FAKE, FAKE * 2, FAKE * 3, FAKE * 4, match="split")
    _expect(B.QSIM_E_INVALID, B.qsim_step_multiply, None, 5, 0, FAKE + 8, FAKE * 2, FAKE * 3, None, match="aligned")
    _expect(B.QSIM_E_INVALID, B.qsim_apply_state, None, 5, FAKE, FAKE * 2, FAKE * 2, None, match="aliases")
    _expect(B.QSIM_E_INVALID, B.qsim_apply_state, None, 5, FAKE, None, FAKE * 2 + 4, None, match="aligned")
    _expect(B.QSIM_E_RANGE, B.qsim_unitarity_drift, None, 17, FAKE)
    _expect(B.QSIM_E_INVALID, B.qsim_unitarity_drift_async, None, 5, FAKE, FAKE + 4, match="d_out")
    _expect(B.QSIM_E_INVALID, B.qsim_unitarity_drift_async, None, 5, FAKE, FAKE, match="context is NULL")
    _expect(B.QSIM_E_INVALID, B.qsim_unitarity_drift, None, 5, FAKE, match="context is NULL")


def test_sample_validation_without_device():
    _expect(B.QSIM_E_RANGE, B.qsim_sample, None, 0, FAKE, FAKE, 4, FAKE)
    _expect(B.QSIM_E_RANGE, B.qsim_sample, None, 17, FAKE, FAKE, 4, FAKE)
    _expect(B.QSIM_E_INVALID, B.qsim_sample, None, 3, FAKE, FAKE, -1, FAKE, match="negative")
    _expect(B.QSIM_E_INVALID, B.qsim_sample, None, 3, FAKE + 8, FAKE, 4, FAKE, match="aligned")
    _expect(B.QSIM_E_INVALID, B.qsim_sample, None, 3, FAKE, None, 4, FAKE, match="d_uniform")
    _expect(B.QSIM_E_INVALID, B.qsim_sample, None, 3, FAKE, None, 0, None, match="context is NULL")


def test_last_error_is_thread_local_and_resets():
    _expect(B.QSIM_E_RANGE, B.qsim_pack_steps, 0, [])
    msg = B.qsim_last_error()
    assert "n_qubits" in msg
    import threading
    seen = []
    t = threading.Thread(target=lambda: seen.append(B.qsim_last_error()))
    t.start()
    t.join()
    assert seen == ["no error"]
    B.qsim_pack_steps(2, [("H", (0,), None)])
    assert B.qsim_last_error() == "no error"


def test_batch_validation_without_device():
    circuits = [W.qft(5), W.ghz_chain(6)]
    need = B.qsim_batch_workspace_bytes(circuits, B.QSIM_FP32_4M)
    assert need == 2 * (8 << 10) + 2 * (8 << 12)
    assert B.qsim_batch_workspace_bytes(circuits, B.QSIM_SPLIT_BF16) == 3 * (8 << 10) + 3 * (8 << 12)
    assert B.qsim_batch_workspace_bytes(circuits, B.QSIM_SPLIT_FP16_3M) == 3 * (12 << 10) + 3 * (12 << 12)
    outs = [FAKE * 64, FAKE * 65]
    with pytest.raises(B.QsimError, match="workspace"):
        B.BatchPlan(None, circuits, outs, B.QSIM_FP32_4M, FAKE * 4, need - 256)
    with pytest.raises(B.QsimError, match="overlap"):
        B.BatchPlan(None, circuits, [FAKE * 64, FAKE * 64], B.QSIM_FP32_4M, FAKE * 4, need)
    with pytest.raises(B.QsimError, match="overlaps the workspace"):
        B.BatchPlan(None, circuits, [FAKE * 4, FAKE * 65], B.QSIM_FP32_4M, FAKE * 4, need)
    with pytest.raises(B.QsimError, match="context is NULL"):
        B.BatchPlan(None, circuits, outs, B.QSIM_FP32_4M, FAKE * 4, need)
    with pytest.raises(B.QsimError, match="n_qubits"):
        B.qsim_batch_workspace_bytes([(17, [])], 0)


def test_serving_validation_without_device():
    with pytest.raises(B.QsimError, match="context is NULL"):
        B.qsim_serve_start(None, B.QSIM_FP32_4M, FAKE, arena_bytes=1 << 20)
    with pytest.raises(B.QsimError, match="max_active"):
        B.qsim_serve_start(None, B.QSIM_FP32_4M, FAKE, arena_bytes=1 << 20, max_active=0)
    with pytest.raises(B.QsimError, match="arena"):
        B.qsim_serve_start(None, B.QSIM_FP32_4M, FAKE + 8, arena_bytes=1 << 20)
    with pytest.raises(B.QsimError, match="precision"):
        B.qsim_serve_start(None, 7, FAKE, arena_bytes=1 << 20)
    with pytest.raises(B.QsimError, match="aging"):
        B.qsim_serve_start(None, B.QSIM_FP32_4M, FAKE, arena_bytes=1 << 20, policy=B.QSIM_POLICY_AGED)
    with pytest.raises(B.QsimError, match="NULL"):
        B.qsim_submit(None, 3, [("H", (0,), None)], FAKE)
    with pytest.raises(B.QsimError, match="NULL"):
        B.qsim_poll(None, 1)


# --- full-state-vector pass schedule (host only) ---------------------------------------------

DIAGONAL = ("Z", "S", "T", "R", "RZ", "CZ", "CR")


def _check_schedule(n, gates):
    """Passes cover the gates once, in an order where every gate follows each earlier gate sharing a qubit
    with it (unless both are diagonal), and every gate's target (both qubits of a SWAP) is local to its pass."""
    sched, order = B.qsim_fsv_schedule(n, gates, with_order=True)
    assert sorted(order) == list(range(len(gates)))
    pos = {g: i for i, g in enumerate(order)}
    for b, (nb, qb, _) in enumerate(gates):
        for a in range(b):
            na, qa, _ = gates[a]
            if set(qa) & set(qb) and not (na in DIAGONAL and nb in DIAGONAL):
                assert pos[a] < pos[b], (a, b, gates[a], gates[b])
    nxt = 0
    for low, highs, first, cnt in sched:
        assert first == nxt and cnt >= 1
        nxt += cnt
        if low == 0:  # a permutation pass: pairwise disjoint SWAPs on any qubits
            assert n > 12 and highs == ()
            ops = [gates[gi] for gi in order[first:first + cnt]]
            assert all(nm == "SWAP" for nm, _, _ in ops)
            qs = [q for _, pair, _ in ops for q in pair]
            assert len(qs) == len(set(qs))
            continue
        if n <= 12:
            assert low == n and highs == ()
        else:
            assert 6 <= low <= 12 and len(highs) == 12 - low
            assert list(highs) == sorted(set(highs)) and all(low <= q < n for q in highs)
        local = set(range(low)) | set(highs)
        # the pass kernel's per-thread byte offset is 32 bits: local bits 0-7 map to qubits below 30
        bit_qubit = list(range(low)) + list(highs)
        assert all(q < 30 for q in bit_qubit[:8]), (low, highs)
        for gi in order[first:first + cnt]:
            nm, qs, _ = gates[gi]
            need = () if nm in DIAGONAL else (qs if nm == "SWAP" or len(qs) == 1 else qs[1:])
            assert set(need) <= local, (nm, qs, low, highs)
    assert nxt == len(gates)
    return sched


def test_fsv_schedule_high_local_bits():
    # targets on the six highest qubits of 34 force them local with only the six low qubits: local bits 6
    # and 7 are then qubits 28 and 29, the largest a thread index bit can map to
    n = 34
    sched = _check_schedule(n, [("H", (q,), None) for q in range(28, 34)])
    assert sched[0][0] == 6 and sched[0][1] == tuple(range(28, 34))


@pytest.mark.parametrize("n", [1, 5, 12, 13, 20, 34])
def test_fsv_schedule_invariants(n):
    rng = np.random.default_rng(n)
    gates = W.gate_tuples(W.random_layers(n, 4, rng)) + W.gate_tuples(W.qft(min(n, 20)))
    gates.append(("SWAP", (0, n - 1), None) if n > 1 else ("H", (0,), None))
    sched = _check_schedule(n, gates)
    if n <= 12:
        assert len(sched) == 1


def test_fsv_schedule_runs_ahead_on_local_qubits():
    # after H on 13 qubits (12 fit one pass), an X on qubit 0 does not wait for the 13th H
    n = 20
    gates = [("H", (q,), None) for q in range(13)] + [("X", (0,), None)]
    sched, order = B.qsim_fsv_schedule(n, gates, with_order=True)
    assert len(sched) == 2
    assert 13 in order[:sched[0][3]] and 12 not in order[:sched[0][3]]
    # a gate that shares a qubit with a waiting one waits too
    gates = [("H", (q,), None) for q in range(13)] + [("CNOT", (12, 0), None), ("X", (0,), None)]
    sched, order = B.qsim_fsv_schedule(n, gates, with_order=True)
    assert order.index(12) < order.index(13) < order.index(14)
    _check_schedule(n, gates)


def test_fsv_schedule_permutation_passes():
    # the reversal closing a QFT on 30 qubits: 15 disjoint SWAPs over all 30 qubits.  The three on qubits
    # 12-17 ride along in an ordinary pass; the other 12 take one permutation pass (as 12-qubit passes they
    # would take two more): 5 passes in all
    n = 30
    sched = _check_schedule(n, W.gate_tuples(W.qft(n)))
    assert len(sched) == 5 and sched[-1][0] == 0 and sched[-1][3] == 12
    assert all(p[0] != 0 for p in sched[:-1])
    # when only SWAPs are ready and they span more than 12 qubits, they are one permutation pass; two
    # layers sharing qubits are two (a SWAP waits for the earlier one on its qubits)
    layer = [("SWAP", (q, q + 10), None) for q in range(8)]
    swapped = [q for _, pair, _ in layer for q in pair]
    gates = layer + layer + [("H", (q,), None) for q in swapped]
    sched = _check_schedule(n, gates)
    perms = [p for p in sched if p[0] == 0]
    assert len(perms) == 2 and all(p[3] == 8 for p in perms)
    # SWAPs on at most 12 qubits with other gates still to come stay in the ordinary passes
    gates = [("H", (q,), None) for q in range(n)] + [("SWAP", (0, 20), None), ("SWAP", (1, 25), None)] + \
        [("H", (q,), None) for q in range(n)]
    assert all(p[0] != 0 for p in _check_schedule(n, gates))
    # up to 12 qubits there are no permutation passes
    assert all(p[0] != 0 for p in _check_schedule(12, W.gate_tuples(W.qft(12))))


def test_fsv_schedule_random_circuits_with_swap_layers():
    """The planner's invariants on random circuits of every gate kind with bursts of disjoint SWAPs, 13 to 30
    qubits: every gate once, dependency order kept, every target local to its pass, permutation passes made of
    disjoint SWAPs only (the seeded sweeps and the permutation passes are host logic, checked here on the CPU)."""
    rng = np.random.default_rng(2024)
    one = ("H", "X", "Y", "Z", "S", "T", "R", "RX", "RY", "RZ")
    two = ("CNOT", "CY", "CZ", "CR", "SWAP")
    perms = 0
    for _ in range(40):
        n = int(rng.integers(13, 31))
        g = []
        for _ in range(int(rng.integers(1, 100))):
            r = rng.random()
            if r < 0.15:
                qs = [int(x) for x in rng.permutation(n)]
                g += [("SWAP", (qs[2 * i], qs[2 * i + 1]), None) for i in range(int(rng.integers(1, n // 2 + 1)))]
            elif r < 0.55:
                nm = two[int(rng.integers(0, len(two)))]
                a, b = (int(x) for x in rng.choice(n, 2, replace=False))
                g.append((nm, (a, b), float(rng.uniform(0, 2 * math.pi)) if nm in W.ANGLED else None))
            else:
                nm = one[int(rng.integers(0, len(one)))]
                g.append((nm, (int(rng.integers(0, n)),), float(rng.uniform(0, 2 * math.pi)) if nm in W.ANGLED else None))
        perms += sum(1 for p in _check_schedule(n, g) if p[0] == 0)
    assert perms > 0


def test_fsv_schedule_counts():
    # all targets inside 12 qubits: one pass; diagonal gates never split a pass
    assert len(B.qsim_fsv_schedule(30, [("H", (q,), None) for q in range(12)])) == 1
    assert len(B.qsim_fsv_schedule(30, [("H", (0,), None)] + [("RZ", (q,), 0.1) for q in range(30)])) == 1
    # one H per qubit on 30 qubits: 6 low qubits are always local, 6 more per pass -> 4 passes
    assert len(B.qsim_fsv_schedule(30, [("H", (q,), None) for q in range(30)])) == 4
    assert B.qsim_fsv_schedule(5, []) == []


def test_fsv_schedule_validation():
    _expect(B.QSIM_E_RANGE, B.qsim_fsv_schedule, 35, [])
    _expect(B.QSIM_E_RANGE, B.qsim_fsv_schedule, 0, [])
    _expect(B.QSIM_E_INVALID, B.qsim_fsv_schedule, 20, [("H", (20,), None)], match="outside")
    _expect(B.QSIM_E_INVALID, B.FsvPlan, None, 5, [("H", (0,), None)], match="context is NULL")


# --- operation data provider and custom ranges (host only) -----------------------------------

def test_register_and_find_unitary():
    from tests.custom_ops import op_id
    M = W.random_unitary(3, 1)
    i = B.qsim_register_unitary("host_test_u3", M)
    assert i >= 1 and B.qsim_find_unitary("host_test_u3") == (i, 3)
    assert op_id("host_test_u3", M) == i
    _expect(B.QSIM_E_INVALID, B.qsim_register_unitary, "host_test_u3", M, match="already")
    _expect(B.QSIM_E_INVALID, B.qsim_register_unitary, "host_bad", np.ones((4, 4)), match="not unitary")
    _expect(B.QSIM_E_RANGE, B.qsim_register_unitary, "host_big", np.eye(128))
    _expect(B.QSIM_E_UNKNOWN_ID, B.qsim_find_unitary, "no_such_op")
    nan = np.eye(2, dtype=complex)
    nan[0, 0] = np.nan
    _expect(B.QSIM_E_INVALID, B.qsim_register_unitary, "host_nan", nan, match="finite")


def test_custom_gate_validation_and_spans():
    from tests.custom_ops import op_id
    i = op_id("host_span_u2", W.random_unitary(2, 2))
    # a 2-qubit range spans 2 qubits: an H on the next qubit shares the step, one inside does not
    assert B.qsim_pack_steps(5, [("CUSTOM", (1, 2), None, i), ("H", (3,), None)]) == [0, 2]
    assert B.qsim_pack_steps(5, [("CUSTOM", (1, 2), None, i), ("H", (2,), None)]) == [0, 1, 2]
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 3, [("CUSTOM", (2, 3), None, i)], match="range")
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 3, [("CUSTOM", (0, 1), None, 99999)], match="not registered")
    bad = B.gate_record(("H", (0,), None))
    bad.op_id = 1
    _expect(B.QSIM_E_INVALID, B.qsim_pack_steps, 3, [bad], match="op_id")


def test_fsv_schedule_keeps_custom_ranges_local():
    from tests.custom_ops import lib_gates
    n = 24
    g = W.with_custom_ops(W.gate_tuples(W.random_layers(n, 2, np.random.default_rng(3))), n, [2, 3, 6, 6, 1], 77)
    lg = lib_gates(g)
    sched, order = B.qsim_fsv_schedule(n, lg, with_order=True)
    for low, highs, first, cnt in sched:
        local = set(range(low)) | set(highs)
        for x in (lg[i] for i in order[first:first + cnt]):
            if x[0] == "CUSTOM":
                assert set(x[1]) <= local, (x[1], low, highs)


def test_build_id_is_the_hash_of_the_sources_the_library_was_built_from():
    """A tile cache records qsim_build_id and is only loaded by a library built from the same sources."""
    from paper_2305_14398_amd import build
    assert B.qsim_build_id() == build.build_id()
    assert len(B.qsim_build_id()) == 16


def test_fsv_schedule_order_replays_to_the_same_state():
    """The reported order is the one each pass applies (reordered where operations commute); replayed gate by
    gate through the oracle (route B) it gives the circuit's own final state."""
    from oracle import fsv
    n = 14
    gates = W.gate_tuples(W.random_layers(n, 3, np.random.default_rng(11))) + W.gate_tuples(W.qft(n))
    sched, order = B.qsim_fsv_schedule(n, gates, with_order=True)
    assert len(sched) > 1 and order != sorted(order)
    a = fsv.final_state(n, gates)
    b = fsv.final_state(n, [gates[i] for i in order])
    assert np.abs(a - b).max() <= 1e-12
