#!/usr/bin/env python
"""Benchmark of the unitary-matrix simulation hot path on one MI355X.

One step = the whole path over one batch of circuits: for each circuit, step
formation on the host, expansion of every step operator (stage 4), the chain
of k-1 complex products (stage 5), the state product with the float64 norm
(stage 6) and the float64 unitarity-drift check.  The batch is the 11-qubit
workload: the QFT (71 steps, 70 products of 2048 x 2048 complex matrices) and
three seeded balanced Deutsch-Jozsa circuits, complex64 (float32 MFMA).

value = complex-GEMM TFLOP/s = sum over circuits of 8 N^3 (k-1) / wall time of
the steps (everything above included).  The JSON line also carries
circuits/s, the live event-timed average of the product kernel against the
float32 MFMA peak, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "complex-GEMM TFLOP/s + circuits/s at 11q; served p50/p99 latency vs plain"
# MFMA peaks of the dtype each product issues, and the MFMA flops issued per 8 N^3 counted
PEAK_TFLOPS = {"fp32_4m": 157.3, "fp32_3m": 157.3, "split_bf16": 2500.0, "split_fp16": 2500.0,
               "split_bf16_3m": 2500.0, "split_fp16_3m": 2500.0}
ISSUED_PER_COUNTED = {"fp32_4m": 1.0, "fp32_3m": 6.0 / 8.0, "split_bf16": 24.0 / 8.0, "split_fp16": 24.0 / 8.0,
                      "split_bf16_3m": 18.0 / 8.0, "split_fp16_3m": 18.0 / 8.0}
# source of each precision's product tile (a committed counter profile counts only while its hash matches)
TILE_SOURCE = {"fp32_4m": "paper_2305_14398_amd/csrc/tile_f32.h", "fp32_3m": "paper_2305_14398_amd/csrc/tile_f32.h",
               "split_bf16": "paper_2305_14398_amd/csrc/tile_split.h",
               "split_fp16": "paper_2305_14398_amd/csrc/tile_split.h",
               "split_bf16_3m": "paper_2305_14398_amd/csrc/tile_split_gauss.h",
               "split_fp16_3m": "paper_2305_14398_amd/csrc/tile_split_gauss.h"}
OPERAND_BYTES_PER_ENTRY = {"fp32_4m": 8, "fp32_3m": 8, "split_bf16": 8, "split_fp16": 8, "split_bf16_3m": 12,
                           "split_fp16_3m": 12}
# probe kind measuring the dtype each precision issues
PROBE_OF = {"fp32_4m": "mfma_f32", "fp32_3m": "mfma_f32", "split_bf16": "mfma_bf16", "split_fp16": "mfma_f16",
            "split_bf16_3m": "mfma_bf16", "split_fp16_3m": "mfma_f16"}
HBM_PEAK_GBS = 8000.0


def workload(n: int):
    from paper_2305_14398_amd import workloads as W
    return [W.qft(n)] + [W.dj(n, W.dj_mask(n, s)) for s in (0, 1, 2)]


def closed_form_error(c, psi):
    """max |psi - closed form| for the QFT (uniform 1/sqrt N) and Deutsch-Jozsa (|mask>|->) states."""
    import numpy as np
    N = psi.size
    ref = np.zeros(N, dtype=np.complex128)
    if c.family == "qft":
        ref[:] = 1 / math.sqrt(N)
    else:
        mask = sum(1 << g.qubits[0] for g in c.gates if g.name == "CNOT")
        ref[mask] = 1 / math.sqrt(2)
        ref[mask + N // 2] = -1 / math.sqrt(2)
    return float(np.abs(psi - ref).max())


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def flops_of(B, c):
    k = len(B.qsim_pack_steps(c.n, c.gates)) - 1
    return 8.0 * (1 << c.n) ** 3 * max(k - 1, 0)


def bench_batched(B, ctx, torch, count: int, seed: int, prec_name: str, reps: int):
    """512 seeded mixed circuits (n 4..11, depth 5..30): one autotuned, graph-captured batch plan vs the same
    circuits one at a time through qsim_unitary_chain."""
    from paper_2305_14398_amd import workloads as W
    prec = B.PRECISIONS[prec_name]
    import tempfile
    circuits = W.batch_mixed(count, seed=seed, n_lo=4, n_hi=11, d_lo=5, d_hi=30)
    B.qsim_autotune(ctx, prec, 7, 11)
    # the choices go through the tile cache (keyed by device and library build) and are read back from it
    cache = os.path.join(tempfile.gettempdir(), f"qsim_tiles_{B.qsim_build_id()}.json")
    B.qsim_tune_save(ctx, cache)
    B.qsim_tune_load(ctx, cache)
    tuning = B.qsim_tune_ms(ctx, prec)
    dev = torch.device("cuda:0")
    outs = [torch.empty((2, 1 << c.n, 1 << c.n), dtype=torch.float32, device=dev) for c in circuits]
    ws = torch.empty(B.qsim_batch_workspace_bytes(circuits, prec), dtype=torch.uint8, device=dev)
    plan = B.BatchPlan(ctx, circuits, outs, prec, ws, graph=True)
    info = plan.info()
    plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.launch()
    torch.cuda.synchronize()
    grouped = (time.perf_counter() - t0) / reps
    plan.close()
    # one at a time (same kernels and precision, no grouping, no graph)
    wss = torch.empty(B.qsim_chain_workspace_bytes(11, prec), dtype=torch.uint8, device=dev)
    for c, o in zip(circuits[:8], outs[:8]):
        B.qsim_unitary_chain(ctx, c.n, c.gates, prec, o, wss)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, o in zip(circuits, outs):
        B.qsim_unitary_chain(ctx, c.n, c.gates, prec, o, wss)
    torch.cuda.synchronize()
    single = time.perf_counter() - t0
    hist = {}
    for c in circuits:
        hist[c.n] = hist.get(c.n, 0) + 1
    return {
        "workload": f"{count} seeded circuits (seed {seed}), n ~ U{{4..11}}, families ghz_chain/dj/qft/random, "
                    f"depth ~ U{{5..30}} for random layers; {prec_name}; grouped persistent launches, autotuned "
                    f"tiles, hipGraph replay",
        "qubit_histogram": {str(k): v for k, v in sorted(hist.items())},
        "iterations": info["iterations"],
        "products": info["products"],
        "tflop": round(info["flops"] / 1e12, 2),
        "grouped_s": round(grouped, 4),
        "grouped_circuits_per_s": round(count / grouped, 1),
        "grouped_tflops": round(info["flops"] / grouped / 1e12, 2),
        "one_at_a_time_s": round(single, 4),
        "one_at_a_time_circuits_per_s": round(count / single, 1),
        "one_at_a_time_tflops": round(info["flops"] / single / 1e12, 2),
        "speedup_vs_one_at_a_time": round(single / grouped, 3),
        "autotune_ms_per_product_64_128": {str(k): [round(a, 4), round(b, 4)] for k, (a, b) in tuning.items()},
        "tiles_chosen": {str(n): B.qsim_tune_get(ctx, prec)[n] for n in range(6, 12)},
        "tile_cache": {"build": B.qsim_build_id(), "file": os.path.basename(cache),
                       "note": "autotuned on seeded dense operands, saved, and loaded back before the timed runs"},
    }


# Drift checks a served request can ask for.
DRIFT_TEXT = {"full": "drift ||U^H U - I|| (max and Frobenius / sqrt(N))",
              "probe": "probe drift ||U^H (U x) - x|| for a fixed unit-modulus x"}


def replay_trace(B, ctx, torch, trace, prec: int, mode: int, arena, max_active: int, policy: int = 0,
                 budget: float = 2.0, aging: float = 0.0, drift: str = "full"):
    import threading
    dev = torch.device("cuda:0")
    psis = [torch.empty(2 << c.n, dtype=torch.float32, device=dev) for _, c in trace]
    torch.cuda.synchronize()
    B.qsim_serve_start(ctx, prec, arena, mode=mode, max_active=max_active, queue_capacity=len(trace) + 1,
                       policy=policy, iter_budget_tflop=budget, aging_tflop_per_s=aging)
    ids = [None] * len(trace)
    t0 = time.monotonic_ns()

    def submitter():
        for i, (t, c) in enumerate(trace):
            target = t0 + int(t * 1e9)
            while True:
                now = time.monotonic_ns()
                if now >= target:
                    break
                time.sleep(min(0.002, (target - now) / 1e9))
            ids[i] = B.qsim_submit(ctx, c.n, c.gates, psis[i], probe=drift == "probe", full_drift=drift == "full")

    th = threading.Thread(target=submitter)
    th.start()
    results = {}
    last_note = time.monotonic()
    while len(results) < len(trace):
        for i in range(len(trace)):
            if ids[i] is not None and i not in results:
                r = B.qsim_poll(ctx, ids[i])
                if r is not None:
                    results[i] = r
        if time.monotonic() - last_note > 30.0:
            progress(f"  served {len(results)}/{len(trace)} requests")
            last_note = time.monotonic()
        time.sleep(0.0005)
    th.join()
    stats = B.qsim_serve_get_stats(ctx)
    B.qsim_serve_stop(ctx)
    lat = sorted((results[i]["t_done_ns"] - (t0 + int(t * 1e9))) / 1e6 for i, (t, _) in enumerate(trace))
    end = max(r["t_done_ns"] for r in results.values())
    span = (end - t0) / 1e9
    flops = sum(flops_of(B, c) for _, c in trace)
    bad = sum(1 for r in results.values() if r["status"] != 0)
    max_drift = max(r["drift_max"] for r in results.values())
    q = lambda p: lat[min(len(lat) - 1, int(round(p * (len(lat) - 1))))]
    return {"p50_ms": round(q(0.50), 2), "p99_ms": round(q(0.99), 2), "max_ms": round(lat[-1], 2),
            "throughput_req_per_s": round(len(trace) / span, 2), "achieved_tflops": round(flops / span / 1e12, 2),
            "makespan_s": round(span, 3), "failed": bad, "drift_check": drift, "max_drift": max_drift,
            "peak_active": stats["peak_active"], "arena_high_water_gib": round(stats["arena_high_water"] / 2**30, 2)}


def bench_served(B, ctx, torch, count: int, rate: float, seed: int, prec_name: str, arena_gib: int,
                 aging: float = 100.0, drift: str = "full"):
    from paper_2305_14398_amd import workloads as W
    prec = B.PRECISIONS[prec_name]
    trace = W.poisson_trace(count, rate, seed, n_lo=6, n_hi=13, d_lo=10, d_hi=40)
    arena = torch.empty(arena_gib << 30, dtype=torch.uint8, device=torch.device("cuda:0"))
    B.qsim_autotune(ctx, prec, 7, 13)
    offered = sum(flops_of(B, c) for _, c in trace) / trace[-1][0]
    cont = replay_trace(B, ctx, torch, trace, prec, B.QSIM_SERVE_CONTINUOUS, arena, 64, drift=drift)
    progress(f"served continuous (arrival order): p50 {cont['p50_ms']} ms p99 {cont['p99_ms']} ms")
    srpt = replay_trace(B, ctx, torch, trace, prec, B.QSIM_SERVE_CONTINUOUS, arena, 64, B.QSIM_POLICY_SHORTEST, 2.0,
                        drift=drift)
    progress(f"served continuous (least work first): p50 {srpt['p50_ms']} ms p99 {srpt['p99_ms']} ms")
    aged = replay_trace(B, ctx, torch, trace, prec, B.QSIM_SERVE_CONTINUOUS, arena, 64, B.QSIM_POLICY_AGED, 2.0,
                        aging, drift=drift)
    progress(f"served continuous (least work first, aged {aging:g} TFLOP/s): p50 {aged['p50_ms']} ms "
             f"p99 {aged['p99_ms']} ms")
    plain = replay_trace(B, ctx, torch, trace, prec, B.QSIM_SERVE_FIFO, arena, 1, drift=drift)
    del arena
    torch.cuda.empty_cache()
    return {
        "workload": f"{count} Poisson arrivals at {rate:g} req/s (seed {seed}), n ~ U{{6..13}}, depth ~ U{{10..40}}, "
                    f"families ghz_chain/dj/qft/random; {prec_name} chains, float64 "
                    f"{DRIFT_TEXT[drift]} and norm per request; arena {arena_gib} GiB",
        "offered_tflops": round(offered / 1e12, 1),
        "continuous_arrival_order": cont,
        "continuous_least_work_first": srpt,
        "continuous_least_work_first_aged": dict(aged, aging_tflop_per_s=aging),
        "plain_fifo": plain,
        "p50_speedup_vs_plain": {"arrival_order": round(plain["p50_ms"] / cont["p50_ms"], 3),
                                 "least_work_first": round(plain["p50_ms"] / srpt["p50_ms"], 3),
                                 "least_work_first_aged": round(plain["p50_ms"] / aged["p50_ms"], 3)},
        "p99_speedup_vs_plain": {"arrival_order": round(plain["p99_ms"] / cont["p99_ms"], 3),
                                 "least_work_first": round(plain["p99_ms"] / srpt["p99_ms"], 3),
                                 "least_work_first_aged": round(plain["p99_ms"] / aged["p99_ms"], 3)},
        "throughput_gain_vs_plain": {"arrival_order": round(cont["throughput_req_per_s"] / plain["throughput_req_per_s"], 3),
                                     "least_work_first": round(srpt["throughput_req_per_s"] / plain["throughput_req_per_s"], 3)},
    }


SWEEP_POLICIES = {"lwf": "continuous_least_work_first", "aged": "continuous_least_work_first_aged",
                  "fifo": "plain_fifo"}


def bench_served_sweep(B, ctx, torch, rates, seconds: float, prec_name: str, arena_gib: int, slo_ms: float,
                       drift: str = "full", policies=("aged", "fifo")):
    """Offered-rate sweep of the served workload: for each Poisson rate, a trace of about `seconds` of arrivals
    run to completion under continuous batching (aged least work first, by default) and under plain FIFO. A rate
    counts as sustained when the p99 latency meets the SLO; the highest rate's achieved TFLOP/s (saturated) gives
    the capacity, and capacity / mean work per request the highest arrival rate any schedule could keep up with."""
    from paper_2305_14398_amd import workloads as W
    prec = B.PRECISIONS[prec_name]
    arena = torch.empty(arena_gib << 30, dtype=torch.uint8, device=torch.device("cuda:0"))
    B.qsim_autotune(ctx, prec, 7, 13)
    rows = []
    for rate in rates:
        count = max(20, int(round(rate * seconds)))
        trace = W.poisson_trace(count, rate, 1, n_lo=6, n_hi=13, d_lo=10, d_hi=40)
        offered = count / trace[-1][0]
        work = sum(flops_of(B, c) for _, c in trace)
        row = {"rate": rate, "requests": count, "offered_req_per_s": round(offered, 2),
               "offered_tflops": round(work / trace[-1][0] / 1e12, 1), "mean_tflop_per_request": round(work / count / 1e12, 2)}
        modes = {"lwf": (B.QSIM_SERVE_CONTINUOUS, 64, B.QSIM_POLICY_SHORTEST),
                 "aged": (B.QSIM_SERVE_CONTINUOUS, 64, B.QSIM_POLICY_AGED),
                 "fifo": (B.QSIM_SERVE_FIFO, 1, 0)}
        for key in policies:
            name = SWEEP_POLICIES[key]
            mode, act, pol = modes[key]
            r = replay_trace(B, ctx, torch, trace, prec, mode, arena, act, pol, 2.0, 100.0, drift)
            r["meets_slo"] = r["p99_ms"] <= slo_ms
            row[name] = r
            progress(f"sweep rate {rate}: {name} p50 {r['p50_ms']} ms p99 {r['p99_ms']} ms "
                     f"{r['throughput_req_per_s']} req/s")
        rows.append(row)
    del arena
    torch.cuda.empty_cache()
    names = [SWEEP_POLICIES[k] for k in policies]
    best = {m: max([r["rate"] for r in rows if r[m]["meets_slo"]] or [0]) for m in names}
    top = rows[-1]
    capacity = max(top[m]["achieved_tflops"] for m in names)
    mean_work = sum(r["mean_tflop_per_request"] * r["requests"] for r in rows) / sum(r["requests"] for r in rows)
    return {"workload": f"Poisson arrivals (seed 1) at each rate for ~{seconds:g} s, n ~ U{{6..13}}, depth ~ "
                        f"U{{10..40}}, {prec_name}, float64 {DRIFT_TEXT[drift]} per request",
            "rates": rows, "slo_p99_ms": slo_ms, "max_rate_meeting_slo": best,
            "capacity_tflops_at_highest_rate": capacity,
            "throughput_bound_rate": round(capacity / mean_work, 2)}


def bench_precision_sweep(B, ctx, torch, sizes, depth: int, seeds, precisions):
    """Config 3: seeded random_layers(n, depth, default_rng(s)) chains, s in `seeds`, at 12 and 13 qubits in every
    precision, timed, with the product's roofline fraction and the float64 drift of each result; and the QFT chain
    at the same n in every precision against its closed form U[j][k] = w^{jk}/sqrt(N) (max |dU| over sampled
    columns, and the fidelity of U e_0 with the uniform state). The QFT chain runs first and also warms the
    kernels. No oracle is involved: random circuits are assessed by drift, QFT by its formula."""
    import numpy as np
    from paper_2305_14398_amd import workloads as W
    dev = torch.device("cuda:0")
    out = {}
    for n in sizes:
        N = 1 << n
        U = torch.empty((2, N, N), dtype=torch.float32, device=dev)
        rands = [W.random_layers(n, depth, np.random.default_rng(s)) for s in seeds]
        qft = W.qft(n)
        cols = W.random_columns(n, 16, 1)
        w = np.exp(2j * np.pi / N)
        closed = np.stack([w ** ((np.arange(N) * c) % N) for c in cols], axis=1) / math.sqrt(N)
        for pname in precisions:
            prec = B.PRECISIONS[pname]
            ws = torch.empty(B.qsim_chain_workspace_bytes(n, prec), dtype=torch.uint8, device=dev)
            B.qsim_unitary_chain(ctx, n, qft.gates, prec, U, ws)
            torch.cuda.synchronize()
            Uc = U[:, :, cols].double().cpu().numpy()
            Uc = Uc[0] + 1j * Uc[1]
            col0 = U[:, :, 0].double().cpu().numpy()
            psi = col0[0] + 1j * col0[1]
            fid = abs(np.sum(psi) / math.sqrt(N)) ** 2 / float(np.sum(np.abs(psi) ** 2))
            walls, drifts, products = [], [], []
            launches = kms = 0.0
            for rand in rands:
                B.qsim_profile_enable(ctx, 1)
                t0 = time.perf_counter()
                B.qsim_unitary_chain(ctx, n, rand.gates, prec, U, ws)
                torch.cuda.synchronize()
                walls.append(time.perf_counter() - t0)
                cnt, tot = B.qsim_profile_read(ctx)["product"]
                B.qsim_profile_enable(ctx, 0)
                launches += cnt
                kms += tot
                products.append(cnt)
                drifts.append(B.qsim_unitarity_drift(ctx, n, U))
            fl = sum(flops_of(B, r) for r in rands)
            per = 8.0 * N ** 3 / (kms / max(launches, 1) * 1e-3) / 1e12
            ceiling = PEAK_TFLOPS[pname] / ISSUED_PER_COUNTED[pname]
            out[f"{n}q_{pname}"] = {
                "seeds": list(seeds), "products_per_seed": products,
                "chain_ms_per_seed": [round(x * 1e3, 2) for x in walls],
                "chain_tflops": round(fl / sum(walls) / 1e12, 1),
                "product_tflops": round(per, 1), "product_frac_of_ceiling": round(per / ceiling, 4),
                "product_issued_tflops": round(per * ISSUED_PER_COUNTED[pname], 1),
                "ceiling_tflops": round(ceiling, 1),
                "random_drift_max_per_seed": [d[0] for d in drifts], "random_drift_fro_per_seed": [d[1] for d in drifts],
                "qft_max_abs_dU_sampled": float(np.abs(Uc - closed).max()), "qft_state_fidelity": fid}
            progress(f"precision sweep {n}q {pname}: {sum(walls)*1e3:.1f} ms over {len(seeds)} seeds, product "
                     f"{per:.1f} TFLOP/s, qft |dU| {out[f'{n}q_{pname}']['qft_max_abs_dU_sampled']:.2e}")
            del ws
        del U
        torch.cuda.empty_cache()
    out["workload"] = (f"random_layers(n, {depth}, default_rng(s)) for s in {list(seeds)} and qft(n), n in "
                       f"{list(sizes)}; chain timing with HIP events per product; errors against closed forms and "
                       f"float64 drift")
    return out


def bench_fsv(B, ctx, torch, n: int, reps: int, which=("qft", "random_layers_20")):
    """Full-state-vector path: qft(n) and random_layers(n, 20) from |0...0>, in place on a 2^n state.
    HBM roofline: every pass reads and writes the state once, 16 bytes per amplitude."""
    import numpy as np
    from paper_2305_14398_amd import workloads as W
    N = 1 << n
    psi = torch.empty(2 * N, dtype=torch.float32, device=torch.device("cuda:0"))
    out = {}
    circuits = {"qft": lambda: W.qft(n), "random_layers_20": lambda: W.random_layers(n, 20, np.random.default_rng(0))}
    for name in which:
        c = circuits[name]()
        g = W.gate_tuples(c)
        with B.FsvPlan(ctx, n, g) as plan:
            info = plan.info()
            B.qsim_fsv_init_basis(ctx, n, 0, psi)
            plan.run(psi)  # warm-up
            torch.cuda.synchronize()
            B.qsim_profile_enable(ctx, 1)
            t0 = time.perf_counter()
            for _ in range(reps):
                plan.run(psi)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / reps
            launches, kernel_ms = B.qsim_profile_read(ctx)["fsv"]
            B.qsim_profile_enable(ctx, 0)
        per_pass_ms = kernel_ms / max(launches, 1)
        achieved = 16.0 * N / (per_pass_ms * 1e-3) / 1e9
        out[name] = {"gates": len(g), "ops": info["ops"], "passes": info["passes"], "ms": round(wall * 1e3, 3),
                     "gates_per_s": round(len(g) / wall, 1), "avg_pass_ms": round(per_pass_ms, 4),
                     "hbm_gb_per_s": round(achieved, 1), "hbm_frac": round(achieved / 8000.0, 4),
                     "one_launch_per_gate_ms_at_peak": round(info["ops"] * 16.0 * N / 8e12 * 1e3, 3)}
        progress(f"fsv {name}({n}): {out[name]['passes']} passes, {out[name]['ms']} ms, {achieved:.0f} GB/s per pass")
    del psi
    torch.cuda.empty_cache()
    out["workload"] = f"full-state-vector simulation of {n} qubits (planar complex64, {8 * N / 2**30:g} GiB), " \
                      f"in place from |0...0>; {reps} runs each"
    out["roofline"] = {"bound": "hbm", "peak": 8000.0, "unit": "GB/s",
                       "traffic_model": "16 bytes per amplitude per pass (read + write of the state)",
                       "traffic": counted_traffic("fsv_pass_qft30_random30.md", "paper_2305_14398_amd/csrc/fsv.hip")
                       if n == 30 else None,
                       "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                       "note": "the pass streams exactly its algorithmic bytes; above the streaming floor its time "
                               "is the issue of the per-operation VALU arithmetic and the scalar dispatch "
                               "(rocprofv3 SQ counters per wave: see the full-state profile summary)"}
    return out


FSV_OP_CASES = {  # one pass of K copies of each (targets on local bits; the pass itself is fixed cost)
    "H": lambda K: [("H", (0,), None)] * K,
    "X": lambda K: [("X", (0,), None)] * K,
    "Y": lambda K: [("Y", (0,), None)] * K,
    "RX": lambda K: [("RX", (0,), 0.3)] * K,
    "RY": lambda K: [("RY", (0,), 0.3)] * K,
    "CNOT_register_control": lambda K: [("CNOT", (1, 0), None)] * K,
    "CNOT_lane_control": lambda K: [("CNOT", (6, 0), None)] * K,
    "CNOT_nonlocal_control": lambda K: [("CNOT", (20, 0), None)] * K,
    "CY_lane_control": lambda K: [("CY", (6, 0), None)] * K,
    "CNOT_alternating_layouts": lambda K: [("CNOT", (0, 4), None) if i % 2 == 0 else ("CNOT", (4, 0), None)
                                           for i in range(K)],
}


def bench_fsv_op_costs(B, ctx, torch, n: int, K: int = 64, reps: int = 3):
    """Marginal time of one full-state operation: a pass of K copies minus a pass of one, over K - 1.  Each case is
    a single pass (its targets are local), so the difference is the operations' own cost (the layout changes
    included for CNOT_alternating_layouts, whose consecutive targets sit in different register groups)."""
    N = 1 << n
    psi = torch.empty(2 * N, dtype=torch.float32, device=torch.device("cuda:0"))

    def time_pass(gates):
        with B.FsvPlan(ctx, n, gates) as plan:
            assert plan.info()["passes"] == 1
            B.qsim_fsv_init_basis(ctx, n, 0, psi)
            plan.run(psi)
            torch.cuda.synchronize()
            B.qsim_profile_enable(ctx, 1)
            for _ in range(reps):
                plan.run(psi)
            torch.cuda.synchronize()
            launches, kernel_ms = B.qsim_profile_read(ctx)["fsv"]
            B.qsim_profile_enable(ctx, 0)
        return kernel_ms / launches

    base = time_pass([("H", (0,), None)])
    out = {"qubits": n, "copies": K, "one_op_pass_us": round(base * 1e3, 2)}
    for name, make in FSV_OP_CASES.items():
        out[name + "_us"] = round((time_pass(make(K)) - base) / (K - 1) * 1e3, 3)
    del psi
    torch.cuda.empty_cache()
    return out


def measure_peaks(B, ctx, torch, copy_mib: int):
    """On-box peaks next to the vendor ones: MFMA issue rate per dtype (independent accumulator chains, random
    and constant operands) and a streaming HBM copy (qsim_probe_mfma / qsim_probe_copy)."""
    vendor = {"mfma_f32": 157.3, "mfma_bf16": 2500.0, "mfma_f16": 2500.0, "mfma_f64": 78.6}
    out = {}
    for name, kind in B.PROBE_KINDS.items():
        rnd = B.qsim_probe_mfma(ctx, kind, True)
        const = B.qsim_probe_mfma(ctx, kind, False)
        out[name] = {"random_operands_tflops": round(rnd, 1), "constant_operands_tflops": round(const, 1),
                     "vendor_tflops": vendor[name], "random_frac_of_vendor": round(rnd / vendor[name], 4)}
    nbytes = copy_mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=torch.device("cuda:0"))
    dst = torch.empty_like(src)
    gbs = B.qsim_probe_copy(ctx, src, dst, nbytes)
    del src, dst
    torch.cuda.empty_cache()
    out["hbm_copy"] = {"gb_per_s": round(gbs, 1), "bytes": nbytes, "vendor_gb_per_s": HBM_PEAK_GBS,
                       "frac_of_vendor": round(gbs / HBM_PEAK_GBS, 4),
                       "note": "read + write bytes of a 16-byte-vector device copy"}
    # the vendor GEMM library on random operands, as a reference for what a tuned dense product reaches here
    lib = {}
    for dtype, name in ((torch.bfloat16, "bf16"), (torch.float16, "fp16"), (torch.float32, "fp32")):
        for m in ((4096, 8192) if name != "fp32" else (8192,)):
            a = torch.randn(m, m, device="cuda:0").to(dtype)
            b = torch.randn(m, m, device="cuda:0").to(dtype)
            for _ in range(2):
                a @ b
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 10 if name != "fp32" else 3
            ev0.record()
            for _ in range(reps):
                a @ b
            ev1.record()
            torch.cuda.synchronize()
            lib[f"{name}_{m}"] = round(2.0 * m ** 3 / (ev0.elapsed_time(ev1) / reps * 1e-3) / 1e12, 1)
            del a, b
    torch.cuda.empty_cache()
    out["library_gemm_tflops"] = lib
    out["method"] = ("MFMA: 2048 workgroups x 256 threads, four independent accumulator chains per wave "
                     "(eight for f64), flops = 2 x M x N x K per instruction; random operands toggle their mantissa bits. "
                     "library_gemm_tflops: torch.matmul (hipBLASLt) on random m x m operands, events over the calls")
    return out


def counted_traffic(profile: str, source: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None when the kernel source changed
    since the counters were taken (the summary stores the source's sha256)."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
        sha = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()
    except OSError:
        return None
    fields = dict(line.strip().split(": ", 1) for line in text.splitlines() if line.startswith("    ") and ": " in line)
    if fields.get("source_sha256") != sha or "hbm_bytes_per_launch" not in fields:
        return None
    return int(fields["hbm_bytes_per_launch"])


def cpu_baseline(n: int, budget_s: float, warmups: int = 3, runs: int = 11):
    """The oracle (route A: dense step operators and complex128 numpy/OpenBLAS products, all host cores) on the
    bench's circuits, after the paper's protocol (Section 6.1: warm-ups, then the mean of the next runs): the
    seeded balanced Deutsch-Jozsa(n) circuit `warmups` times untimed, then the mean of `runs` timed runs; the
    QFT(n) once (its products are 8x more than the Deutsch-Jozsa's); and one product each at n + 1 and n + 2
    qubits, whose time x the product count of random_layers(n', 20) is reported as an extrapolated chain time.
    A single-BLAS-thread run over the first steps of the QFT is the analogue of the paper's single-threaded
    baseline."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import unitary as UA
    from paper_2305_14398_amd import workloads as W

    def chain(steps, nq, limit_s=None):
        t0 = time.perf_counter()
        result = UA.step_operator(nq, steps[0])
        done = 0
        for st in steps[1:]:
            result = UA.step_operator(nq, st) @ result
            done += 1
            if limit_s is not None and time.perf_counter() - t0 > limit_s and done >= 1:
                break
        return time.perf_counter() - t0, done

    N = 1 << n
    per = 8.0 * N ** 3
    dj_steps = UA.pack_steps(W.gate_tuples(W.dj(n, W.dj_mask(n, 0))))
    for _ in range(warmups):
        chain(dj_steps, n)
    times = [chain(dj_steps, n)[0] for _ in range(runs)]
    dj_mean = sum(times) / len(times)
    dj_products = len(dj_steps) - 1
    qft_steps = UA.pack_steps(W.gate_tuples(W.qft(n)))
    t_qft, qft_done = chain(qft_steps, n, limit_s=budget_s)
    threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("internal_api") == "openblas"] or [1])
    per_gemm = {}
    for m in (n + 1, n + 2):
        M = 1 << m
        rl = W.random_layers(m, 20, np.random.default_rng(0))
        steps = UA.pack_steps(W.gate_tuples(rl))
        A = UA.step_operator(m, steps[1])
        X = UA.step_operator(m, steps[0])
        t0 = time.perf_counter()
        A @ X
        dt = time.perf_counter() - t0
        per_gemm[f"{m}q"] = {"gemm_s": round(dt, 3), "tflops": round(8.0 * M ** 3 / dt / 1e12, 3),
                             "random_layers_20_products": len(steps) - 1,
                             "extrapolated_chain_s": round(dt * (len(steps) - 1), 1),
                             "note": "one product timed; the chain time is extrapolated (x products), not measured"}
        del A, X
    with threadpool_limits(limits=1):
        t1, single = chain(qft_steps, n, limit_s=budget_s / 3)
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = [f"{p.get('internal_api')} {p.get('version')}" for p in threadpool_info() if p.get("user_api") == "blas"]
    return {
        "value": per * dj_products / dj_mean / 1e12,
        "unit": "TFLOP/s",
        "host": {"cpu_model": cpu_model, "cpus_visible": os.cpu_count(), "blas": blas},
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"route A over deutsch_jozsa({n}) (mask seed 0, {dj_products} products): {warmups} warm-ups, "
                  f"then the mean of {runs} runs ({dj_mean:.3f} s each); {os.cpu_count()} host CPUs visible",
        "dj_circuits_per_s": round(1.0 / dj_mean, 3),
        "dj_run_s": [round(x, 4) for x in times],
        "qft": {"products": qft_done, "of": len(qft_steps) - 1, "s": round(t_qft, 3),
                "tflops": round(per * qft_done / t_qft / 1e12, 3), "runs": 1},
        "per_gemm": per_gemm,
        "single_thread": {"value": per * single / t1 / 1e12, "unit": "TFLOP/s", "cores": 1,
                          "sample": f"the first {single + 1} steps of qft({n}) with one BLAS thread; {t1:.1f} s"},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp32_3m", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--variant", default="fp32_4m,split_fp16,split_bf16,split_fp16_3m,split_bf16_3m",
                    help="comma-separated further precisions timed on the same workload ('' to skip)")
    ap.add_argument("--fused", default="fp32_3m",
                    help="float32 precisions also timed with stages 4 and 5 fused ('' to skip)")
    ap.add_argument("--qubits", type=int, default=11)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched", type=int, default=512, help="circuits in the batched workload (0: skip)")
    ap.add_argument("--served", type=int, default=200, help="requests in the served trace (0: skip)")
    ap.add_argument("--served-rate", type=float, default=200.0)
    ap.add_argument("--served-prec", default="split_bf16_3m", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--served-drift", default="full", choices=sorted(DRIFT_TEXT),
                    help="drift check per served request: the full ||U^H U - I|| or the two-pass probe")
    ap.add_argument("--fsv", type=int, default=30, help="qubits of the full-state-vector workload (0: skip)")
    ap.add_argument("--fsv-circuits", default="qft,random_layers_20")
    ap.add_argument("--fsv-reps", type=int, default=3)
    ap.add_argument("--fsv-op-costs", type=int, default=26,
                    help="qubits of the per-operation full-state cost cases (0: skip)")
    ap.add_argument("--sweep-qubits", default="12,13", help="qubit counts of the precision sweep ('' to skip)")
    ap.add_argument("--sweep-seeds", default="0,1,2,3,4", help="seeds of the precision sweep's random circuits")
    ap.add_argument("--sweep-precisions", default="fp32_4m,fp32_3m,split_bf16,split_fp16,split_bf16_3m,split_fp16_3m")
    ap.add_argument("--served-sweep", default="8,12,16",
                    help="comma-separated Poisson rates for an offered-rate sweep ('' to skip)")
    ap.add_argument("--served-sweep-seconds", type=float, default=10.0)
    ap.add_argument("--served-sweep-policies", default="aged,fifo", help=f"of {sorted(SWEEP_POLICIES)}")
    ap.add_argument("--served-slo-ms", type=float, default=2500.0)
    ap.add_argument("--peaks", type=int, default=1, help="measure on-box MFMA and HBM peaks (0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a known-size kernel that "
                         "scales the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: --gpus {args.gpus} is not supported (independent circuits would shard "
              f"round-robin over GPUs with no exchange; see the design notes)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2305_14398_amd import binding as B

    n = args.qubits
    N = 1 << n
    prec = B.PRECISIONS[args.prec]
    circuits = workload(n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = B.Context(0)
    U = torch.empty((2, N, N), dtype=torch.float32, device=dev)
    psi = torch.empty(2 * N, dtype=torch.float32, device=dev)
    prob = torch.empty(N, dtype=torch.float64, device=dev)
    records = [B.gate_array(c.gates) for c in circuits]
    gate_lists = [[arr[i] for i in range(ng)] for arr, ng in records]
    ks = [len(B.qsim_pack_steps(n, c.gates)) - 1 for c in circuits]
    flops_per_step = sum(8.0 * N ** 3 * (k - 1) for k in ks)

    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def timed_run(prec_name: str, check: bool, fused: bool = False):
        prec = B.PRECISIONS[prec_name]
        ws_bytes = (B.qsim_chain_fused_workspace_bytes if fused else B.qsim_chain_workspace_bytes)(n, prec)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        chain = B.qsim_unitary_chain_fused if fused else B.qsim_unitary_chain
        results = {}

        drift_dev = torch.empty((len(circuits), 2), dtype=torch.float64, device=dev)

        def one_step(check: bool = False):
            # No host synchronisation inside a step: the float64 norm stays on the device and each drift result
            # goes to its own device slot; the checking step reads them back.
            for ci, (c, gates) in enumerate(zip(circuits, gate_lists)):
                chain(ctx, n, gates, prec, U, ws)
                if not check:
                    B.qsim_apply_state(ctx, n, U, None, psi, prob, want_norm2=False)
                    B.qsim_unitarity_drift_async(ctx, n, U, drift_dev[ci])
                    continue
                norm2 = B.qsim_apply_state(ctx, n, U, None, psi, prob)
                drift = B.qsim_unitarity_drift(ctx, n, U)
                if check:
                    p = psi.cpu().numpy().astype(np.float64)
                    results[c.family + str(len(results))] = {
                        "steps": len(B.qsim_pack_steps(n, c.gates)) - 1, "norm2": norm2, "drift_max": drift[0],
                        "drift_fro": drift[1], "max_abs_err_closed_form": closed_form_error(c, p[:N] + 1j * p[N:])}

        for _ in range(args.warmup):
            one_step()
        torch.cuda.synchronize()
        B.qsim_profile_enable(ctx, True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        for _ in range(args.steps):
            one_step()
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stats = B.qsim_profile_read(ctx)
        B.qsim_profile_enable(ctx, False)
        if check:
            one_step(check=True)
            torch.cuda.synchronize()
        cnt, tot = stats["product"]
        avg_ms = tot / cnt if cnt else float("nan")
        return {"wall": wall, "gpu_ms": ev0.elapsed_time(ev1), "stats": stats, "checks": results,
                "tflops": flops_per_step * args.steps / wall / 1e12, "avg_product_ms": avg_ms, "ws_bytes": ws_bytes}

    main = timed_run(args.prec, check=True)
    wall, gpu_ms, stats, results = main["wall"], main["gpu_ms"], main["stats"], main["checks"]
    variant_names = [v for v in args.variant.split(",") if v and v != args.prec]
    variant_runs = [(v, timed_run(v, check=False)) for v in variant_names]
    fused_names = [v for v in args.fused.split(",") if v]
    fused_runs = [(v, timed_run(v, check=False, fused=True)) for v in fused_names]
    unfused = dict(variant_runs + [(args.prec, main)])

    ms_per_step = wall * 1e3 / args.steps
    tflops = flops_per_step * args.steps / wall / 1e12
    avg_gemm_ms = main["avg_product_ms"]
    achieved = 8.0 * N ** 3 / (avg_gemm_ms * 1e-3) / 1e12
    # ceiling at 8 N^3 counting: the dtype's MFMA peak divided by the MFMA flops issued per counted flop
    peak = PEAK_TFLOPS[args.prec] / ISSUED_PER_COUNTED[args.prec]
    ecnt, etot = stats["expand"]
    out = {
        "metric": METRIC,
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if args.prec.startswith("fp32") else "bf16" if args.prec.startswith("split_bf16") else "fp16",
        "data": "synthetic",
        "config": {
            "workload": f"qft({n}) + 3 seeded balanced deutsch_jozsa({n}); complex64 chains ({args.prec}); "
                        f"expand + chain + apply + fp64 norm + fp64 drift per circuit",
            "qubits": n,
            "circuits_per_step": len(circuits),
            "steps_per_circuit": ks,
            "products_per_step": sum(k - 1 for k in ks),
            "precision": args.prec,
        },
        "circuits_per_s": round(len(circuits) * args.steps / wall, 3),
        "gpu_event_ms_per_step": round(gpu_ms / args.steps, 3),
        "kernel_ms": {k: {"launches": c, "total_ms": round(t, 3), "avg_ms": round(t / c, 5) if c else None}
                      for k, (c, t) in stats.items()},
        "roofline": {
            "bound": "mfma",
            "kernel": f"{'cgemm_f32_kernel' if args.prec.startswith('fp32') else 'cgemm_split_gauss_kernel' if args.prec.endswith('_3m') else 'cgemm_split_kernel'} "
                      f"({args.prec}, complex product of stage 5, 2048^3)",
            "achieved": round(achieved, 2),
            "peak": round(peak, 1),
            "peak_basis": f"{PEAK_TFLOPS[args.prec]} TFLOP/s dense MFMA peak of the issued dtype x 8 N^3 counted / "
                          f"{ISSUED_PER_COUNTED[args.prec] * 8:g} N^3 issued",
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": counted_traffic(f"cgemm_{args.prec}_qft{n}_dj{n}.md", TILE_SOURCE[args.prec]),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE, copy-calibrated)",
            # operands in and result out, each in the precision's format (the last product writes float32)
            "algorithmic_bytes_per_launch": 3 * OPERAND_BYTES_PER_ENTRY[args.prec] * N * N,
        },
        "expand_roofline": {
            "bound": "hbm",
            "achieved": round(8.0 * N * N / (etot / ecnt * 1e-3) / 1e9, 1) if ecnt else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
        },
        "checks": results,
        "variants": [{
            "precision": v,
            "value": round(r["tflops"], 3),
            "ms_per_step": round(r["wall"] * 1e3 / args.steps, 3),
            "avg_product_ms": round(r["avg_product_ms"], 5),
            "product_tflops": round(8.0 * N ** 3 / (r["avg_product_ms"] * 1e-3) / 1e12, 2),
            "product_frac_of_ceiling": round(8.0 * N ** 3 / (r["avg_product_ms"] * 1e-3) / 1e12 /
                                             (PEAK_TFLOPS[v] / ISSUED_PER_COUNTED[v]), 4),
        } for v, r in variant_runs],
        "fused": [{
            "precision": v,
            "workload": "the same steps with stages 4 and 5 fused (qsim_unitary_chain_fused: each step operator "
                        "computed inside the product, never stored)",
            "value": round(r["tflops"], 3),
            "ms_per_step": round(r["wall"] * 1e3 / args.steps, 3),
            "avg_product_ms": round(r["avg_product_ms"], 5),
            "expand_launches": r["stats"]["expand"][0],
            "workspace_bytes": r["ws_bytes"],
            "unfused_workspace_bytes": B.qsim_chain_workspace_bytes(n, B.PRECISIONS[v]),
            "speed_vs_unfused": round(r["tflops"] / unfused[v]["tflops"], 4) if v in unfused else None,
        } for v, r in fused_runs],
        "paper_context": "TornadoQSim reports end-to-end speedups over single-threaded Java of 506.5x (fully "
                         "entangled), 493.10x (Deutsch-Jozsa) and 518.12x (QFT) at 11 qubits on a Quadro GP100; "
                         "different hardware, precision and baseline",
    }
    # The same steps with every final state copied to pinned host memory (the paper's end-to-end timing includes
    # the transfers; here gates travel as kernel arguments and the state is the only bulk transfer).
    host_psi = torch.empty(2 * N, dtype=torch.float32, pin_memory=True)
    prec_main = B.PRECISIONS[args.prec]
    ws_main = torch.empty(B.qsim_chain_workspace_bytes(n, prec_main), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for gates in gate_lists:
            B.qsim_unitary_chain(ctx, n, gates, prec_main, U, ws_main)
            B.qsim_apply_state(ctx, n, U, None, psi, prob, want_norm2=False)
            host_psi.copy_(psi, non_blocking=True)
    torch.cuda.synchronize()
    e2e = time.perf_counter() - t0
    out["e2e_with_state_readback"] = {
        "circuits_per_s": round(len(circuits) * args.steps / e2e, 3),
        "ms_per_circuit": round(e2e * 1e3 / (len(circuits) * args.steps), 3),
        "note": "expand + chain + apply + float64 norm, each state copied to pinned host memory (no drift check)"}
    del ws_main
    progress(f"headline done: {tflops:.1f} TFLOP/s")
    if args.peaks:
        out["peaks"] = measure_peaks(B, ctx, torch, 1024)
        mp = out["peaks"][PROBE_OF[args.prec]]["random_operands_tflops"] / ISSUED_PER_COUNTED[args.prec]
        out["roofline"]["measured_peak"] = round(mp, 1)
        out["roofline"]["frac_of_measured_peak"] = round(achieved / mp, 4)
        progress("peaks done")
    if args.batched:
        out["batched"] = bench_batched(B, ctx, torch, args.batched, 0, "fp32_4m" if args.prec == "fp32_4m"
                                       else args.prec, reps=2)
        progress("batched done")
    if args.served:
        out["served"] = bench_served(B, ctx, torch, args.served, args.served_rate, 0, args.served_prec, 96,
                                     drift=args.served_drift)
        progress("served done")
    if args.sweep_qubits:
        out["precision_sweep"] = bench_precision_sweep(B, ctx, torch, [int(x) for x in args.sweep_qubits.split(",")], 20,
                                                       [int(x) for x in args.sweep_seeds.split(",")],
                                                       [p for p in args.sweep_precisions.split(",") if p])
        progress("precision sweep done")
    if args.served_sweep:
        rates = [float(x) for x in args.served_sweep.split(",") if x]
        out["served_sweep"] = bench_served_sweep(B, ctx, torch, rates, args.served_sweep_seconds, args.served_prec, 96,
                                                 args.served_slo_ms, args.served_drift,
                                                 [p for p in args.served_sweep_policies.split(",") if p])
        progress("served sweep done")
    if args.fsv:
        out["full_state"] = bench_fsv(B, ctx, torch, args.fsv, reps=args.fsv_reps,
                                      which=[x for x in args.fsv_circuits.split(",") if x])
        progress("full-state done")
    if "full_state" in out and "peaks" in out:
        copy = out["peaks"]["hbm_copy"]["gb_per_s"]
        for name in [x for x in args.fsv_circuits.split(",") if x]:
            if name in out["full_state"]:
                out["full_state"][name]["frac_of_measured_copy"] = round(
                    out["full_state"][name]["hbm_gb_per_s"] / copy, 4)
    if args.fsv_op_costs:
        out.setdefault("full_state", {})["op_costs"] = bench_fsv_op_costs(B, ctx, torch, args.fsv_op_costs)
        progress("full-state operation costs done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_seconds)
        progress("cpu baseline done")
        out["speedup_vs_cpu_oracle"] = round(tflops / out["cpu_baseline"]["value"], 1)
    ctx.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
