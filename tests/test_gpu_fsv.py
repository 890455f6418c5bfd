"""Full-state-vector simulation (Appendix A, Eq. 12) on the GPU against the oracle's route B.

Tolerance.  Each operation applies a 2x2 complex matrix rounded to float32
(relative error u = 2^-24 per entry) in float32 fused multiply-adds; for a
unitary matrix that perturbs the state by at most about 7u in 2-norm, and the
later operations are unitary, so after G operations
    ||psi_gpu - psi_exact||_2 <= 8 G u.
The tests check that bound on the whole state (and hence on every amplitude).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fsv  # noqa: E402
from paper_2305_14398_amd import binding as B  # noqa: E402
from paper_2305_14398_amd import workloads as W  # noqa: E402
from tests import gpu_util as G  # noqa: E402

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    c = B.Context(0)
    yield c
    c.close()


def n_ops(gates):
    return len(gates)


def bound(gates):
    return 8 * max(n_ops(gates), 1) * U32


def run_fsv(ctx, n, gates, psi0):
    psi = G.planar_vec(psi0)
    with B.FsvPlan(ctx, n, gates) as plan:
        plan.run(psi)
        G.sync()
        info = plan.info()
    return G.vec_to_complex(psi), info


def all_kinds(n, rng, count):
    """Every gate kind, with controls and SWAP partners drawn from the whole register."""
    out = []
    one = ("H", "X", "Y", "Z", "S", "T", "R", "RX", "RY", "RZ")
    two = ("CNOT", "CY", "CZ", "CR", "SWAP")
    for _ in range(count):
        if n >= 2 and rng.random() < 0.45:
            nm = two[int(rng.integers(0, len(two)))]
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            out.append((nm, (a, b), float(rng.uniform(0, 2 * math.pi)) if nm in W.ANGLED else None))
        else:
            nm = one[int(rng.integers(0, len(one)))]
            out.append((nm, (int(rng.integers(0, n)),), float(rng.uniform(0, 2 * math.pi)) if nm in W.ANGLED else None))
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11, 12, 13, 14, 16])
def test_fsv_matches_route_b_all_kinds(ctx, n):
    rng = np.random.default_rng(500 + n)
    g = all_kinds(n, rng, 40 + 4 * n)
    psi0 = W.random_state(n, n)
    got, info = run_fsv(ctx, n, g, psi0)
    ref = fsv.final_state(n, g, psi0)
    assert np.linalg.norm(got - ref) <= bound(g), (np.linalg.norm(got - ref), bound(g), info)
    assert info["ops"] == n_ops(g)


@pytest.mark.parametrize("n,family", [(13, "qft"), (15, "qft"), (14, "random"), (17, "random"), (18, "ghz_fanout"),
                                      (20, "dj")])
def test_fsv_paper_families(ctx, n, family):
    rng = np.random.default_rng(n)
    c = {"qft": lambda: W.qft(n), "random": lambda: W.random_layers(n, 6, rng),
         "ghz_fanout": lambda: W.ghz_fanout(n), "dj": lambda: W.dj(n, W.dj_mask(n, 5))}[family]()
    g = W.gate_tuples(c)
    psi0 = W.random_state(n, 2 * n)
    got, info = run_fsv(ctx, n, g, psi0)
    ref = fsv.final_state(n, g, psi0)
    assert np.linalg.norm(got - ref) <= bound(g)
    assert info["passes"] == len(B.qsim_fsv_schedule(n, g))


def test_fsv_custom_matrix_equals_named_gate(ctx):
    n = 14
    r = 1 / math.sqrt(2)
    named = [("H", (13,), None), ("CNOT", (13, 2), None), ("H", (5,), None)]
    custom = [("U2", (13,), None, [[r, r], [r, -r]]), ("CNOT", (13, 2), None), ("U2", (5,), None, [[r, r], [r, -r]])]
    psi0 = W.random_state(n, 3)
    a, _ = run_fsv(ctx, n, named, psi0)
    b, _ = run_fsv(ctx, n, custom, psi0)
    np.testing.assert_array_equal(a, b)


def test_fsv_plan_reuse_and_empty(ctx):
    n = 13
    g = W.gate_tuples(W.random_layers(n, 3, np.random.default_rng(9)))
    psi0 = W.random_state(n, 4)
    psi = G.planar_vec(psi0)
    with B.FsvPlan(ctx, n, g) as plan:
        plan.run(psi)
        plan.run(psi)
        G.sync()
    ref = fsv.final_state(n, g + g, psi0)
    assert np.linalg.norm(G.vec_to_complex(psi) - ref) <= bound(g + g)
    # no gates: no passes, state untouched
    before = psi.clone()
    with B.FsvPlan(ctx, n, []) as plan:
        assert plan.info()["passes"] == 0
        plan.run(psi)
        G.sync()
    assert torch.equal(before, psi)


def test_fsv_init_basis_and_norm(ctx):
    for n, b in ((1, 1), (2, 3), (12, 4095), (20, 123457)):
        psi = torch.full((2 << n,), 7.0, dtype=torch.float32, device=G.DEV)
        B.qsim_fsv_init_basis(ctx, n, b, psi)
        G.sync()
        v = G.vec_to_complex(psi)
        e = np.zeros(1 << n)
        e[b] = 1
        np.testing.assert_array_equal(v, e)
        assert B.qsim_fsv_norm2(ctx, n, psi) == 1.0
    psi0 = W.random_state(16, 1) * 3.0
    ref = float(np.sum(np.abs(psi0.astype(np.complex64).astype(np.complex128)) ** 2))
    assert abs(B.qsim_fsv_norm2(ctx, 16, G.planar_vec(psi0)) - ref) <= 1e-12 * ref


# --- full-size states (2-8 GiB), checked against closed forms on the device ------------------

def _err_vs(psi, ref_re, ref_im):
    N = psi.numel() // 2
    d = (psi[:N].double() - ref_re) ** 2 + (psi[N:].double() - ref_im) ** 2
    return math.sqrt(float(d.sum()))


def test_fsv_qft_28_of_basis_state_is_the_dft_column(ctx):
    """QFT|x> has amplitude exp(2 pi i x k / N) / sqrt(N) at k (the DFT, Section 2.5; the closed form
    the oracle is pinned to), evaluated in float64 on the device from exact integer phases."""
    n, x = 28, 91_233_457
    N = 1 << n
    g = W.gate_tuples(W.qft(n))
    psi = torch.empty(2 * N, dtype=torch.float32, device=G.DEV)
    B.qsim_fsv_init_basis(ctx, n, x, psi)
    with B.FsvPlan(ctx, n, g) as plan:
        plan.run(psi)
        G.sync()
    k = torch.arange(N, dtype=torch.int64, device=G.DEV)
    ph = ((k * x) % N).double() * (2 * math.pi / N)
    del k
    err = _err_vs(psi, torch.cos(ph) / math.sqrt(N), torch.sin(ph) / math.sqrt(N))
    assert err <= bound(g), (err, bound(g))
    assert abs(B.qsim_fsv_norm2(ctx, n, psi) - 1.0) <= bound(g)


def test_fsv_diagonals_then_qft_28_closed_form(ctx):
    """Diagonal gates on a basis state only multiply it by a phase (the product of the diagonal entries its bits
    select), and the QFT then gives that phase times the DFT column.  The 80 diagonals draw their qubits from the
    whole register, so in a 12-qubit pass of 28 qubits many read non-local qubits spread over 16 workgroup-number
    bits: grouped records with several table windows, for a local target, a local control and no local qubit.
    The QFT's controlled phases are written with control and target exchanged (the gate is symmetric), so its
    grouped records read a non-local target."""
    from oracle import gates as OG
    n, x = 28, 0b1011_0110_1110_0101_1010_0111_0110
    N = 1 << n
    rng = np.random.default_rng(2828)
    diag, phase = [], 1.0 + 0.0j
    bit = lambda q: (x >> q) & 1
    for _ in range(80):
        nm = str(rng.choice(["CR", "CZ", "T", "S", "RZ", "Z", "R"]))
        th = float(rng.uniform(0, 2 * math.pi)) if nm in W.ANGLED else None
        if nm in ("CR", "CZ"):
            c, t = (int(v) for v in rng.choice(n, 2, replace=False))
            diag.append((nm, (c, t), th))
            if bit(c):
                phase *= OG.controlled_target(nm, th)[bit(t), bit(t)]
        else:
            q = int(rng.integers(0, n))
            diag.append((nm, (q,), th))
            phase *= OG.one_qubit(nm, th)[bit(q), bit(q)]
    qft = []
    for j in range(n - 1, -1, -1):
        qft.append(("H", (j,), None))
        qft += [("CR", (j, i), math.pi / (1 << (j - i))) for i in range(j)]
    qft += [("SWAP", (i, n - 1 - i), None) for i in range(n // 2)]
    g = diag + qft
    assert any(p[0] == 0 for p in B.qsim_fsv_schedule(n, g))
    psi = torch.empty(2 * N, dtype=torch.float32, device=G.DEV)
    B.qsim_fsv_init_basis(ctx, n, x, psi)
    with B.FsvPlan(ctx, n, g) as plan:
        plan.run(psi)
        G.sync()
    k = torch.arange(N, dtype=torch.int64, device=G.DEV)
    ph = ((k * x) % N).double() * (2 * math.pi / N)
    del k
    c, s = torch.cos(ph) / math.sqrt(N), torch.sin(ph) / math.sqrt(N)
    del ph
    err = _err_vs(psi, c * phase.real - s * phase.imag, c * phase.imag + s * phase.real)
    assert err <= bound(g), (err, bound(g))


def test_fsv_mirror_28_returns_to_zero_state(ctx):
    n = 28
    c = W.mirror(W.random_layers(n, 4, np.random.default_rng(28)))
    g = W.gate_tuples(c)
    N = 1 << n
    psi = torch.empty(2 * N, dtype=torch.float32, device=G.DEV)
    B.qsim_fsv_init_basis(ctx, n, 0, psi)
    with B.FsvPlan(ctx, n, g) as plan:
        plan.run(psi)
        G.sync()
    ref_re = torch.zeros(N, dtype=torch.float64, device=G.DEV)
    ref_re[0] = 1.0
    err = _err_vs(psi, ref_re, torch.zeros_like(ref_re))
    assert err <= bound(g), (err, bound(g))


def test_fsv_ghz_30(ctx):
    """GHZ (Section 2.5): (|0...0> + |1...1>)/sqrt(2) on 30 qubits, an 8 GiB state."""
    n = 30
    N = 1 << n
    g = W.gate_tuples(W.ghz_fanout(n))
    psi = torch.empty(2 * N, dtype=torch.float32, device=G.DEV)
    B.qsim_fsv_init_basis(ctx, n, 0, psi)
    with B.FsvPlan(ctx, n, g) as plan:
        plan.run(psi)
        G.sync()
    r = 1 / math.sqrt(2)
    ends = psi[torch.tensor([0, N - 1, N, 2 * N - 1], device=G.DEV)].cpu().numpy()
    assert abs(ends[0] - r) <= 1e-7 and abs(ends[1] - r) <= 1e-7 and ends[2] == 0 and ends[3] == 0
    # the two amplitudes carry the whole norm, so every other amplitude is zero to rounding
    assert abs(B.qsim_fsv_norm2(ctx, n, psi) - 2 * float(ends[0]) * float(ends[0])) <= 1e-6
    del psi
    torch.cuda.empty_cache()


def test_fsv_validation(ctx):
    psi = torch.zeros(64, dtype=torch.float32, device=G.DEV)
    with pytest.raises(B.QsimError, match="basis"):
        B.qsim_fsv_init_basis(ctx, 5, 32, psi)
    with pytest.raises(B.QsimError):
        B.FsvPlan(ctx, 35, [])
    with pytest.raises(B.QsimError, match="outside"):
        B.FsvPlan(ctx, 5, [("H", (5,), None)])


# --- custom operations (Section 5.2.2) ------------------------------------------------------

def custom_bound(gates):
    """8 u per 2x2 operation; a dense 2^m operation in float32 costs about (2^m + 2) 2^(m/2) u."""
    total = 0.0
    for g in gates:
        if len(g) == 4 and g[0] != "U2":
            D = 1 << len(g[1])
            total += 2 * (D + 2) * math.sqrt(D)
        else:
            total += 8
    return total * U32


@pytest.mark.parametrize("n", [4, 9, 12, 14, 17])
def test_fsv_custom_ops_match_route_b(ctx, n):
    from tests.custom_ops import lib_gates
    g = W.with_custom_ops(W.gate_tuples(W.random_layers(n, 3, np.random.default_rng(n))), n, [1, 2, 3, 5, 6, 6],
                          700 + n)
    psi0 = W.random_state(n, 5 * n)
    got, _ = run_fsv(ctx, n, lib_gates(g), psi0)
    ref = fsv.final_state(n, g, psi0)
    assert np.linalg.norm(got - ref) <= custom_bound(g), (np.linalg.norm(got - ref), custom_bound(g))


@pytest.mark.parametrize("n", [14, 17])
def test_fsv_custom_ops_with_swap_layers_and_scaled_forms(ctx, n):
    """Custom operations (passes with a dense operation, the 32 KiB instantiation) among uncontrolled H, RX and RY
    (scaled forms, on both sides of the sine/cosine divide) and layers of disjoint SWAPs over the whole register
    (permutation passes), against route B."""
    from tests.custom_ops import lib_gates
    rng = np.random.default_rng(3100 + n)
    g = []
    for layer in range(3):
        g += W.gate_tuples(W.random_layers(n, 1, rng))
        g += [(("H", "RX", "RY")[int(rng.integers(0, 3))], (q,), None) for q in range(n)]
        g = [(nm, qs, float(rng.uniform(0, 2 * math.pi)) if nm in W.ANGLED and th is None else th)
             for nm, qs, th in g]
        qs = [int(x) for x in rng.permutation(n)]
        g += [("SWAP", (qs[2 * i], qs[2 * i + 1]), None) for i in range(n // 2)]
    g = W.with_custom_ops(g, n, [1, 2, 3, 5], 900 + n)
    g += [("SWAP", (q, n - 1 - q), None) for q in range(n // 2)]  # a closing reversal: one permutation pass
    sched = B.qsim_fsv_schedule(n, lib_gates(g))
    assert sched[-1][0] == 0
    psi0 = W.random_state(n, 6 * n)
    got, _ = run_fsv(ctx, n, lib_gates(g), psi0)
    ref = fsv.final_state(n, g, psi0)
    assert np.linalg.norm(got - ref) <= custom_bound(g), (np.linalg.norm(got - ref), custom_bound(g))


def test_fsv_custom_dft_on_high_qubits_equals_qft_gates(ctx):
    """The 4-qubit DFT registered as one operation on qubits 20..23 of a 24-qubit state equals the
    QFT gates on those qubits (both on the GPU, compared with the bound of each)."""
    from tests.custom_ops import lib_gates
    n, a, D = 24, 20, 16
    j = np.arange(D)
    dft = np.exp(2j * np.pi * np.outer(j, j) / D) / math.sqrt(D)
    pre = [("H", (q,), None) for q in range(0, n, 3)] + [("CNOT", (0, 22), None), ("RY", (21,), 0.7)]
    qft_gates = [(nm, tuple(q + a for q in qs), th) for nm, qs, th in W.gate_tuples(W.qft(4))]
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1
    x, _ = run_fsv(ctx, n, lib_gates(pre + [("dft4_on_20", (20, 21, 22, 23), None, dft)]), psi0)
    y, _ = run_fsv(ctx, n, pre + qft_gates, psi0)
    assert np.linalg.norm(x - y) <= custom_bound(pre + [("d", (20, 21, 22, 23), None, dft)]) + bound(pre + qft_gates)


def test_fsv_ghz_34_maximum_size(ctx):
    """The largest register the full-state path takes: 34 qubits, a 128 GiB state (GHZ, Section 2.5), with
    measurement by sampling on top (every shot is 0 or N-1)."""
    n = B.QSIM_FSV_MAX_QUBITS
    N = 1 << n
    psi = torch.empty(2 * N, dtype=torch.float32, device=G.DEV)
    B.qsim_fsv_init_basis(ctx, n, 0, psi)
    with B.FsvPlan(ctx, n, W.gate_tuples(W.ghz_fanout(n))) as plan:
        plan.run(psi)
        G.sync()
    r = 1 / math.sqrt(2)
    ends = psi[torch.tensor([0, N - 1, N, 2 * N - 1], device=G.DEV)].cpu().numpy()
    assert abs(ends[0] - r) <= 1e-7 and abs(ends[1] - r) <= 1e-7 and ends[2] == 0 and ends[3] == 0
    assert abs(B.qsim_fsv_norm2(ctx, n, psi) - 2 * float(ends[0]) * float(ends[0])) <= 1e-6
    u = torch.rand(4096, dtype=torch.float64, generator=torch.Generator().manual_seed(3)).to(G.DEV)
    out = torch.empty(4096, dtype=torch.int64, device=G.DEV)
    ws = G.workspace(B.qsim_fsv_sample_workspace_bytes(n))
    B.qsim_fsv_sample(ctx, n, psi, u, 4096, out, ws)
    shots = out.cpu().numpy()
    assert set(np.unique(shots)) <= {0, N - 1}
    # X on four qubits, then the reversal SWAP(q, 33 - q): the two amplitudes move to sigma(m) and its
    # complement, through a permutation pass whose addresses need all 34 bits
    m = (1 << 0) | (1 << 7) | (1 << 20) | (1 << 33)
    g = [("X", (q,), None) for q in (0, 7, 20, 33)] + [("SWAP", (q, n - 1 - q), None) for q in range(n // 2)]
    assert any(p[0] == 0 for p in B.qsim_fsv_schedule(n, g))
    with B.FsvPlan(ctx, n, g) as plan:
        plan.run(psi)
        G.sync()
    sm = sum(((m >> q) & 1) << (n - 1 - q) for q in range(n))
    got = psi[torch.tensor([sm, (N - 1) ^ sm, N + sm], device=G.DEV)].cpu().numpy()
    assert got[0] == ends[0] and got[1] == ends[1] and got[2] == 0
    assert abs(B.qsim_fsv_norm2(ctx, n, psi) - 2 * float(ends[0]) * float(ends[0])) <= 1e-6
    del psi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [16, 19])
def test_fsv_diagonal_runs_across_local_and_non_local_qubits(ctx, n):
    """Runs of diagonal operations between Hadamard layers, built to hit every way the planner multiplies them
    out: both qubits local (one table), a local target with a non-local control and the reverse (grouped by
    the local bit, more than five non-local partners per bit so a group spans several tables), one-qubit phases
    and CZ/CR pairs on non-local qubits only (a single factor per workgroup), and a lone diagonal."""
    rng = np.random.default_rng(900 + n)
    g = []
    for layer in range(3):
        g += [("H", (q,), None) for q in range(n)]
        local_t = int(rng.integers(0, 6))
        for c in rng.permutation(np.arange(8, n))[:9]:
            g.append(("CR", (int(c), local_t), float(rng.uniform(0, 2 * math.pi))))  # non-local control
            g.append(("CZ", (local_t + 1, int(c)), None))  # local control, non-local target
        for q in rng.permutation(np.arange(0, 6))[:4]:
            g.append(("RZ", (int(q),), float(rng.uniform(0, 2 * math.pi))))
        for _ in range(6):
            a, b = (int(x) for x in rng.choice(np.arange(12, n), 2, replace=False))
            g.append(("CR", (a, b), float(rng.uniform(0, 2 * math.pi))))
            g.append(("T", (a,), None))
        g.append(("CZ", (0, 1), None))
        g.append(("X", (layer,), None))
        g.append(("S", (n - 1,), None))
    psi0 = W.random_state(n, n + 1)
    got, info = run_fsv(ctx, n, g, psi0)
    ref = fsv.final_state(n, g, psi0)
    assert np.linalg.norm(got - ref) <= bound(g), (np.linalg.norm(got - ref), bound(g), info)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fsv_lane_operations_and_layout_runs(ctx, seed):
    """Runs of one to seven non-diagonal operations aimed at one register group of the 12 local qubits, so that
    the planner applies the short ones across lanes (every lane bit, DPP, swizzle and bpermute exchanges) and
    changes the layout for the long ones; the real, exchange, Y and imaginary off-diagonal forms (the last two take
    the general complex arithmetic across lanes), controls on a lane bit, a wave bit, a register bit and a
    non-local qubit, and diagonal operations between and inside the runs (per-lane phase, register and table
    forms), so pending phases meet both lane operations and layout changes."""
    n = 14
    rng = np.random.default_rng(1300 + seed)
    forms = ("H", "X", "Y", "RX", "RY")
    g = [("H", (q,), None) for q in range(n)]
    for _ in range(40):
        group = int(rng.integers(0, 3))
        for _ in range(int(rng.integers(1, 8))):
            t = 4 * group + int(rng.integers(0, 4))
            nm = forms[int(rng.integers(0, len(forms)))]
            kind = int(rng.integers(0, 5))
            if kind == 0:  # uncontrolled
                g.append((nm, (t,), float(rng.uniform(0, 2 * math.pi)) if nm in W.ANGLED else None))
            else:
                c = int(rng.choice([q for q in range(n) if q != t]))
                two = {"X": "CNOT", "Y": "CY", "H": "CNOT", "RX": "CNOT", "RY": "CY"}[nm]
                g.append((two, (c, t), None))
            if rng.random() < 0.3:  # a phase on the target, then H on it again
                g.append(("R", (t,), float(rng.uniform(0, 2 * math.pi))))
                g.append(("H", (t,), None))
        for _ in range(int(rng.integers(0, 3))):  # diagonals between runs (per-lane phase, register, table)
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            g.append(("CR", (a, b), float(rng.uniform(0, 2 * math.pi))) if rng.random() < 0.5 else ("T", (a,), None))
    psi0 = W.random_state(n, 40 + seed)
    got, info = run_fsv(ctx, n, g, psi0)
    ref = fsv.final_state(n, g, psi0)
    assert np.linalg.norm(got - ref) <= bound(g), (np.linalg.norm(got - ref), bound(g), info)


@pytest.mark.parametrize("n", [7, 12, 14])
def test_fsv_scaled_forms_and_their_growth_limit(ctx, n):
    """H, RX and RY without a control run in a scaled form whose factor (1/sqrt 2 for H) the pass applies when it
    stores.  160 such operations in one pass would grow the values by about 2^80, so past 2^32 the planner keeps
    the unscaled forms: the state still matches route B within the rounding bound, and its norm stays 1.  Angles
    near pi (sine above cosine) take the second rotation forms on register bits and the unscaled form across
    lanes."""
    rng = np.random.default_rng(77 + n)
    g = []
    for i in range(160):
        q = int(rng.integers(0, min(n, 12)))
        kind = i % 5
        if kind < 2:
            g.append(("H", (q,), None))
        elif kind == 2:
            g.append(("RX", (q,), float(rng.uniform(-1.5, 1.5) if i % 2 else rng.uniform(2.0, 4.2))))
        elif kind == 3:
            g.append(("RY", (q,), float(rng.uniform(2.0, 4.2))))  # |sin| > |cos| of the half angle: unscaled
        else:
            g.append(("CNOT", (q, (q + 1) % min(n, 12)), None))
    assert len(B.qsim_fsv_schedule(n, g)) == 1
    psi0 = W.random_state(n, 5 * n)
    got, _ = run_fsv(ctx, n, g, psi0)
    ref = fsv.final_state(n, g, psi0)
    assert np.linalg.norm(got - ref) <= bound(g), (np.linalg.norm(got - ref), bound(g))
    assert abs(np.linalg.norm(got) - 1.0) <= bound(g)


def swap_layers(n, rng, layers):
    """Layers of pairwise disjoint SWAPs on random qubits (a layer of 1 to n/2 pairs)."""
    out = []
    for _ in range(layers):
        qs = [int(x) for x in rng.permutation(n)]
        m = int(rng.integers(1, n // 2 + 1))
        out += [("SWAP", (qs[2 * i], qs[2 * i + 1]), None) for i in range(m)]
    return out


@pytest.mark.parametrize("n,case", [(13, "random"), (14, "random"), (16, "random"), (20, "random"), (13, "reverse"),
                                    (16, "reverse"), (18, "low_only"), (18, "high_only"), (17, "low_high")])
def test_fsv_permutation_passes_are_exact(ctx, n, case):
    """SWAP-only circuits run as permutation passes: the amplitudes move unchanged, so the result equals the
    oracle's exactly (the float32 input permuted)."""
    rng = np.random.default_rng(900 + n)
    g = {"random": lambda: swap_layers(n, rng, 4),
         "reverse": lambda: [("SWAP", (q, n - 1 - q), None) for q in range(n // 2)],
         "low_only": lambda: [("SWAP", (0, 5), None), ("SWAP", (1, 3), None)],  # no row bit exchanged
         "high_only": lambda: [("SWAP", (6, 17), None), ("SWAP", (8, 12), None), ("SWAP", (9, 10), None)],
         "low_high": lambda: [("SWAP", (q, 16 - q), None) for q in range(6)] + [("SWAP", (7, 9), None)]}[case]()
    sched = B.qsim_fsv_schedule(n, g)
    assert any(p[0] == 0 for p in sched)
    psi0 = W.random_state(n, 3 * n).astype(np.complex64)
    got, info = run_fsv(ctx, n, g, psi0)
    ref = fsv.final_state(n, g, psi0.astype(np.complex128))
    np.testing.assert_array_equal(got, ref.astype(np.complex64))
    assert info["passes"] == len(sched)


@pytest.mark.parametrize("n", [16, 20])
def test_fsv_qft_with_permutation_pass(ctx, n):
    """A QFT whose closing reversal runs as a permutation pass, and SWAP layers between rotation layers."""
    rng = np.random.default_rng(40 + n)
    g = W.gate_tuples(W.qft(n))
    assert B.qsim_fsv_schedule(n, g)[-1][0] == 0
    layers = [("SWAP", (q, q + n // 2), None) for q in range(n // 2)]
    g2 = W.gate_tuples(W.random_layers(n, 2, rng)) + layers + W.gate_tuples(W.random_layers(n, 2, rng))
    for gates in (g, g2):
        psi0 = W.random_state(n, 7 + n)
        got, _ = run_fsv(ctx, n, gates, psi0)
        ref = fsv.final_state(n, gates, psi0)
        assert np.linalg.norm(got - ref) <= bound(gates)
