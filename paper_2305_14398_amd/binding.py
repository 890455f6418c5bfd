"""Thin ctypes binding of libqsim (include/qsim.h): argument marshalling only.

Every function here has the name of the C entry point it forwards to.  Device
buffers may be given as torch tensors (their ``data_ptr()`` is passed) or as
raw integer addresses; ``stream`` defaults to torch's current stream on the
context's device.  Gate lists are ``workloads.Gate`` objects or plain
``(name, qubits, theta)`` tuples and are packed into ``qsim_gate`` records.
No computation happens in Python: a missing library raises instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqsim.so")

QSIM_OK, QSIM_PENDING = 0, 1
QSIM_E_INVALID, QSIM_E_RANGE, QSIM_E_OOM, QSIM_E_DEVICE, QSIM_E_FULL, QSIM_E_UNKNOWN_ID = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "QSIM_OK", 1: "QSIM_PENDING", -1: "QSIM_E_INVALID", -2: "QSIM_E_RANGE", -3: "QSIM_E_OOM",
                -4: "QSIM_E_DEVICE", -5: "QSIM_E_FULL", -6: "QSIM_E_UNKNOWN_ID"}

QSIM_FP32_4M, QSIM_FP32_3M, QSIM_SPLIT_BF16, QSIM_SPLIT_FP16 = 0, 1, 2, 3
QSIM_SPLIT_BF16_3M, QSIM_SPLIT_FP16_3M = 4, 5
PRECISIONS = {"fp32_4m": 0, "fp32_3m": 1, "split_bf16": 2, "split_fp16": 3, "split_bf16_3m": 4, "split_fp16_3m": 5}
QSIM_LAYOUT_ROW, QSIM_LAYOUT_COL = 0, 1

KIND = {"H": 0, "X": 1, "Y": 2, "Z": 3, "S": 4, "T": 5, "R": 6, "RX": 7, "RY": 8, "RZ": 9, "U2": 10, "SWAP": 11,
        "CUSTOM": 12}
QSIM_CUSTOM_MAX_QUBITS = 6
# controlled names -> kind of the gate applied to the target
CONTROLLED = {"CNOT": "X", "CY": "Y", "CZ": "Z", "CR": "R"}


class qsim_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("target", ctypes.c_int32), ("control", ctypes.c_int32),
                ("op_id", ctypes.c_int32), ("theta", ctypes.c_double), ("u", ctypes.c_double * 8)]


assert ctypes.sizeof(qsim_gate) == 88

PROFILE_KINDS = ("expand", "product", "apply", "drift", "fsv")


class qsim_kernel_stats(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64 * 5), ("total_ms", ctypes.c_double * 5)]


QSIM_FSV_MAX_QUBITS = 34
QSIM_FSV_MAX_HIGH = 6


class qsim_fsv_pass_info(ctypes.Structure):
    _fields_ = [("low_qubits", ctypes.c_int32), ("n_high", ctypes.c_int32),
                ("high", ctypes.c_int32 * QSIM_FSV_MAX_HIGH), ("first_op", ctypes.c_int32),
                ("n_ops", ctypes.c_int32), ("permutation", ctypes.c_int32)]


class qsim_circuit_desc(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32), ("gates", ctypes.POINTER(qsim_gate)),
                ("step_offsets", ctypes.POINTER(ctypes.c_int32)), ("n_steps", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("d_U", ctypes.c_void_p)]


QSIM_BATCH_GRAPH = 1
QSIM_SERVE_CONTINUOUS, QSIM_SERVE_FIFO = 0, 1
QSIM_REQ_DRIFT_PROBE = 1
QSIM_REQ_DRIFT_FULL = 2
QSIM_E_CANCELLED = -7
STATUS_NAMES[-7] = "QSIM_E_CANCELLED"


QSIM_POLICY_ARRIVAL, QSIM_POLICY_SHORTEST, QSIM_POLICY_AGED = 0, 1, 2


class qsim_serve_config(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("mode", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int32), ("d_arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("policy", ctypes.c_int32), ("reserved", ctypes.c_int32), ("iter_budget_tflop", ctypes.c_double),
                ("aging_tflop_per_s", ctypes.c_double)]


class qsim_request(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32), ("gates", ctypes.POINTER(qsim_gate)),
                ("d_psi", ctypes.c_void_p), ("d_psi0", ctypes.c_void_p), ("d_U", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class qsim_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_steps", ctypes.c_int32), ("norm2", ctypes.c_double),
                ("drift_max", ctypes.c_double), ("drift_l2", ctypes.c_double), ("t_submit_ns", ctypes.c_uint64),
                ("t_start_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class qsim_serve_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("grouped_launches", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("peak_active", ctypes.c_int64), ("arena_high_water", ctypes.c_uint64)]


class QsimError(RuntimeError):
    def __init__(self, status: int, message: str, call: str):
        super().__init__(f"{call}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


_lib = None


def lib() -> ctypes.CDLL:
    """Load libqsim.so (built in-tree by paper_2305_14398_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2305_14398_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, sz, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
    gp = ctypes.POINTER(qsim_gate)
    ip = ctypes.POINTER(ctypes.c_int32)
    sigs = {
        "qsim_last_error": (ctypes.c_char_p, []),
        "qsim_version": (ctypes.c_char_p, []),
        "qsim_ctx_create": (i32, [i32, ctypes.POINTER(vp)]),
        "qsim_ctx_destroy": (i32, [vp]),
        "qsim_pack_steps": (i32, [i32, gp, i32, ip, ctypes.POINTER(i32)]),
        "qsim_chain_workspace_bytes": (sz, [i32, i32]),
        "qsim_op_bytes": (sz, [i32, i32]),
        "qsim_probe_mfma": (i32, [vp, i32, i32, ctypes.POINTER(dbl)]),
        "qsim_probe_copy": (i32, [vp, vp, vp, sz, ctypes.POINTER(dbl)]),
        "qsim_build_step": (i32, [vp, i32, gp, i32, i32, i32, vp, vp]),
        "qsim_step_multiply": (i32, [vp, i32, i32, vp, vp, vp, vp, vp]),
        "qsim_unitary_chain": (i32, [vp, i32, gp, i32, ip, i32, i32, vp, vp, sz, vp]),
        "qsim_step_multiply_fused": (i32, [vp, i32, i32, gp, i32, vp, vp, vp]),
        "qsim_chain_fused_workspace_bytes": (sz, [i32, i32]),
        "qsim_unitary_chain_fused": (i32, [vp, i32, gp, i32, ip, i32, i32, vp, vp, sz, vp]),
        "qsim_apply_state": (i32, [vp, i32, vp, vp, vp, vp, ctypes.POINTER(dbl), vp]),
        "qsim_unitarity_drift": (i32, [vp, i32, vp, ctypes.POINTER(dbl), vp]),
        "qsim_profile_enable": (i32, [vp, i32]),
        "qsim_batch_workspace_bytes": (i32, [ctypes.POINTER(qsim_circuit_desc), i32, i32, ctypes.POINTER(sz)]),
        "qsim_batch_plan_create": (i32, [vp, ctypes.POINTER(qsim_circuit_desc), i32, i32, vp, sz, i32,
                                         ctypes.POINTER(vp)]),
        "qsim_batch_plan_launch": (i32, [vp, vp]),
        "qsim_batch_plan_info": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(dbl)]),
        "qsim_batch_plan_destroy": (i32, [vp]),
        "qsim_unitary_chain_batched": (i32, [vp, ctypes.POINTER(qsim_circuit_desc), i32, i32, vp, sz, vp]),
        "qsim_autotune": (i32, [vp, i32, i32, i32, ctypes.POINTER(dbl)]),
        "qsim_unitarity_drift_probe": (i32, [vp, i32, vp, ctypes.POINTER(dbl), vp]),
        "qsim_sample": (i32, [vp, i32, vp, vp, i32, vp, vp]),
        "qsim_unitarity_drift_async": (i32, [vp, i32, vp, vp, vp]),
        "qsim_unitarity_drift_noalloc": (i32, [i32, vp, vp, vp]),
        "qsim_register_unitary": (i32, [ctypes.c_char_p, i32, ctypes.POINTER(dbl), ctypes.POINTER(i32)]),
        "qsim_find_unitary": (i32, [ctypes.c_char_p, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "qsim_fsv_schedule": (i32, [i32, vp, i32, ctypes.POINTER(qsim_fsv_pass_info), i32,
                                    ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "qsim_fsv_plan_create": (i32, [vp, i32, vp, i32, ctypes.POINTER(vp)]),
        "qsim_fsv_plan_info": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "qsim_fsv_plan_destroy": (i32, [vp]),
        "qsim_fsv_run": (i32, [vp, vp, vp, vp]),
        "qsim_fsv_init_basis": (i32, [vp, i32, ctypes.c_int64, vp, vp]),
        "qsim_fsv_norm2": (i32, [vp, i32, vp, ctypes.POINTER(dbl), vp]),
        "qsim_fsv_sample_workspace_bytes": (ctypes.c_size_t, [i32]),
        "qsim_fsv_sample": (i32, [vp, i32, vp, vp, i32, vp, vp, ctypes.c_size_t, vp]),
        "qsim_serve_start": (i32, [vp, ctypes.POINTER(qsim_serve_config)]),
        "qsim_serve_stop": (i32, [vp]),
        "qsim_submit": (i32, [vp, ctypes.POINTER(qsim_request), ctypes.POINTER(ctypes.c_uint64)]),
        "qsim_poll": (i32, [vp, ctypes.c_uint64, ctypes.POINTER(qsim_result)]),
        "qsim_serve_get_stats": (i32, [vp, ctypes.POINTER(qsim_serve_stats)]),
        "qsim_tune_get": (i32, [vp, i32, ctypes.POINTER(i32)]),
        "qsim_tune_set": (i32, [vp, i32, i32, i32]),
        "qsim_tune_ms": (i32, [vp, i32, ctypes.POINTER(dbl)]),
        "qsim_tune_save": (i32, [vp, ctypes.c_char_p]),
        "qsim_tune_load": (i32, [vp, ctypes.c_char_p]),
        "qsim_build_id": (ctypes.c_char_p, []),
        "qsim_profile_read": (i32, [vp, ctypes.POINTER(qsim_kernel_stats)]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int, call: str) -> int:
    if status < 0:
        raise QsimError(status, lib().qsim_last_error().decode(), call)
    return status


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream, device: int = 0):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def gate_record(g) -> qsim_gate:
    """Marshal one gate (workloads.Gate, (name, qubits, theta[, u]) or ("CUSTOM", range, None, op_id))
    into a qsim_gate."""
    name, qubits, theta = (g.name, g.qubits, g.theta) if hasattr(g, "name") else (g[0], g[1], g[2])
    rec = qsim_gate()
    rec.op_id = 0
    if name == "CUSTOM":
        rec.kind = KIND["CUSTOM"]
        rec.target = int(qubits[0])
        rec.control = -1
        rec.op_id = int(g[3])
        return rec
    rec.theta = 0.0 if theta is None else float(theta)
    if name in CONTROLLED:
        rec.kind = KIND[CONTROLLED[name]]
        rec.control, rec.target = int(qubits[0]), int(qubits[1])
    elif name == "SWAP":
        rec.kind = KIND["SWAP"]
        rec.target, rec.control = int(qubits[0]), int(qubits[1])
    else:
        rec.kind = KIND[name]
        rec.target = int(qubits[0])
        rec.control = int(qubits[1]) if len(qubits) > 1 else -1
    if name == "U2":
        u = g[3] if not hasattr(g, "name") else g.u
        for i in range(4):
            rec.u[2 * i] = float(complex(u[i // 2][i % 2]).real)
            rec.u[2 * i + 1] = float(complex(u[i // 2][i % 2]).imag)
    return rec


def gate_array(gates: Iterable):
    gl = list(gates)
    arr = (qsim_gate * max(1, len(gl)))()
    for i, g in enumerate(gl):
        arr[i] = g if isinstance(g, qsim_gate) else gate_record(g)
    return arr, len(gl)


class Context:
    """Owns a qsim_ctx handle (qsim_ctx_create / qsim_ctx_destroy)."""

    def __init__(self, device: int = 0):
        self.device = device
        self.handle = qsim_ctx_create(device)

    def close(self):
        if self.handle:
            qsim_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _h(ctx):
    return ctx.handle if isinstance(ctx, Context) else ctx


def _dev(ctx):
    return ctx.device if isinstance(ctx, Context) else 0


# --- entry points (same names as the C ABI) --------------------------------------------------

def qsim_version() -> str:
    return lib().qsim_version().decode()


def qsim_last_error() -> str:
    return lib().qsim_last_error().decode()


def qsim_ctx_create(device: int = 0) -> int:
    out = ctypes.c_void_p()
    _check(lib().qsim_ctx_create(device, ctypes.byref(out)), "qsim_ctx_create")
    return out.value


def qsim_ctx_destroy(handle) -> None:
    _check(lib().qsim_ctx_destroy(handle), "qsim_ctx_destroy")


def qsim_pack_steps(n_qubits: int, gates: Sequence) -> list:
    arr, ng = gate_array(gates)
    off = (ctypes.c_int32 * (ng + 1))()
    ns = ctypes.c_int()
    _check(lib().qsim_pack_steps(n_qubits, arr, ng, off, ctypes.byref(ns)), "qsim_pack_steps")
    return [int(off[i]) for i in range(ns.value + 1)]


def qsim_chain_workspace_bytes(n_qubits: int, prec: int) -> int:
    return int(lib().qsim_chain_workspace_bytes(n_qubits, prec))


def qsim_op_bytes(n_qubits: int, prec: int) -> int:
    return int(lib().qsim_op_bytes(n_qubits, prec))


def qsim_build_step(ctx, n_qubits: int, gates: Sequence, prec: int, layout: int, d_op, stream=None) -> None:
    arr, ng = gate_array(gates)
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_build_step(_h(ctx), n_qubits, arr, ng, prec, layout, _ptr(d_op), st), "qsim_build_step")


def qsim_step_multiply(ctx, n_qubits: int, prec: int, d_S, d_Uin, d_Uout, d_Uout_split=None, stream=None) -> None:
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_step_multiply(_h(ctx), n_qubits, prec, _ptr(d_S), _ptr(d_Uin), _ptr(d_Uout),
                                    _ptr(d_Uout_split), st), "qsim_step_multiply")


def qsim_step_multiply_fused(ctx, n_qubits: int, prec: int, gates: Sequence, d_Uin, d_Uout, stream=None) -> None:
    arr, ng = gate_array(gates)
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_step_multiply_fused(_h(ctx), n_qubits, prec, arr, ng, _ptr(d_Uin), _ptr(d_Uout), st),
           "qsim_step_multiply_fused")


def qsim_chain_fused_workspace_bytes(n_qubits: int, prec: int) -> int:
    return int(lib().qsim_chain_fused_workspace_bytes(n_qubits, prec))


def qsim_unitary_chain_fused(ctx, n_qubits: int, gates: Sequence, prec: int, d_U, d_ws, ws_bytes: Optional[int] = None,
                             step_offsets: Optional[Sequence[int]] = None, stream=None) -> None:
    qsim_unitary_chain(ctx, n_qubits, gates, prec, d_U, d_ws, ws_bytes, step_offsets, stream, _fused=True)


def qsim_unitary_chain(ctx, n_qubits: int, gates: Sequence, prec: int, d_U, d_ws, ws_bytes: Optional[int] = None,
                       step_offsets: Optional[Sequence[int]] = None, stream=None, _fused: bool = False) -> None:
    arr, ng = gate_array(gates)
    if step_offsets is None:
        off_p, ns = None, 0
    else:
        off_p = (ctypes.c_int32 * len(step_offsets))(*step_offsets)
        ns = len(step_offsets) - 1
    if ws_bytes is None:
        ws_bytes = d_ws.numel() * d_ws.element_size() if hasattr(d_ws, "numel") else 0
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    name = "qsim_unitary_chain_fused" if _fused else "qsim_unitary_chain"
    _check(getattr(lib(), name)(_h(ctx), n_qubits, arr, ng, off_p, ns, prec, _ptr(d_U), _ptr(d_ws), ws_bytes, st), name)


def qsim_apply_state(ctx, n_qubits: int, d_U, d_psi0, d_psi, d_prob=None, want_norm2: bool = True,
                     stream=None) -> Optional[float]:
    norm = ctypes.c_double(float("nan"))
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_apply_state(_h(ctx), n_qubits, _ptr(d_U), _ptr(d_psi0), _ptr(d_psi), _ptr(d_prob),
                                  ctypes.byref(norm) if want_norm2 else None, st), "qsim_apply_state")
    return norm.value if want_norm2 else None


def qsim_unitarity_drift(ctx, n_qubits: int, d_U, stream=None) -> tuple:
    out = (ctypes.c_double * 2)()
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_unitarity_drift(_h(ctx), n_qubits, _ptr(d_U), out, st), "qsim_unitarity_drift")
    return float(out[0]), float(out[1])


def qsim_profile_enable(ctx, enable: bool = True) -> None:
    _check(lib().qsim_profile_enable(_h(ctx), 1 if enable else 0), "qsim_profile_enable")


def qsim_profile_read(ctx) -> dict:
    """{kind: (launch count, total milliseconds)} for expand / product / apply / drift."""
    st = qsim_kernel_stats()
    _check(lib().qsim_profile_read(_h(ctx), ctypes.byref(st)), "qsim_profile_read")
    return {k: (int(st.count[i]), float(st.total_ms[i])) for i, k in enumerate(PROFILE_KINDS)}


# --- batches -------------------------------------------------------------------------------

def circuit_descs(circuits: Sequence, outputs: Sequence):
    """Marshal (n_qubits, gates) pairs and their output buffers into a qsim_circuit_desc array.
    Returns the array and the gate arrays it points into (keep both alive across the call)."""
    arr = (qsim_circuit_desc * len(circuits))()
    keep = []
    for i, (c, U) in enumerate(zip(circuits, outputs)):
        n, gates = (c.n, c.gates) if hasattr(c, "n") else c
        g, ng = gate_array(gates)
        keep.append(g)
        arr[i].n_qubits = n
        arr[i].n_gates = ng
        arr[i].gates = ctypes.cast(g, ctypes.POINTER(qsim_gate))
        arr[i].step_offsets = None
        arr[i].n_steps = 0
        arr[i].reserved = 0
        arr[i].d_U = _ptr(U)
    return arr, keep


def qsim_batch_workspace_bytes(circuits: Sequence, prec: int) -> int:
    arr, _keep = circuit_descs(circuits, [0] * len(circuits))
    out = ctypes.c_size_t()
    _check(lib().qsim_batch_workspace_bytes(arr, len(circuits), prec, ctypes.byref(out)), "qsim_batch_workspace_bytes")
    return int(out.value)


class BatchPlan:
    """qsim_batch_plan_create / _launch / _info / _destroy."""

    def __init__(self, ctx, circuits: Sequence, outputs: Sequence, prec: int, d_ws, ws_bytes: Optional[int] = None,
                 graph: bool = False):
        arr, _keep = circuit_descs(circuits, outputs)
        if ws_bytes is None:
            ws_bytes = d_ws.numel() * d_ws.element_size() if hasattr(d_ws, "numel") else 0
        out = ctypes.c_void_p()
        _check(lib().qsim_batch_plan_create(_h(ctx), arr, len(circuits), prec, _ptr(d_ws), ws_bytes,
                                            QSIM_BATCH_GRAPH if graph else 0, ctypes.byref(out)),
               "qsim_batch_plan_create")
        self.handle = out.value
        self.device = _dev(ctx)

    def launch(self, stream=None):
        _check(lib().qsim_batch_plan_launch(self.handle, _stream(stream, self.device)), "qsim_batch_plan_launch")

    def info(self):
        it, pr, fl = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().qsim_batch_plan_info(self.handle, ctypes.byref(it), ctypes.byref(pr), ctypes.byref(fl)),
               "qsim_batch_plan_info")
        return {"iterations": it.value, "products": pr.value, "flops": fl.value}

    def close(self):
        if self.handle:
            _check(lib().qsim_batch_plan_destroy(self.handle), "qsim_batch_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qsim_unitary_chain_batched(ctx, circuits: Sequence, outputs: Sequence, prec: int, d_ws,
                               ws_bytes: Optional[int] = None, stream=None) -> None:
    arr, _keep = circuit_descs(circuits, outputs)
    if ws_bytes is None:
        ws_bytes = d_ws.numel() * d_ws.element_size() if hasattr(d_ws, "numel") else 0
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_unitary_chain_batched(_h(ctx), arr, len(circuits), prec, _ptr(d_ws), ws_bytes, st),
           "qsim_unitary_chain_batched")


def qsim_autotune(ctx, prec: int, n_lo: int = 7, n_hi: int = 11) -> dict:
    """Returns {n: (ms per product with 64-tiles, with 128-tiles)} for n >= 7 and stores the choice in the context."""
    out = (ctypes.c_double * (2 * max(1, n_hi - 6)))()
    _check(lib().qsim_autotune(_h(ctx), prec, n_lo, n_hi, out), "qsim_autotune")
    return {n: (out[2 * (n - 7)], out[2 * (n - 7) + 1]) for n in range(max(7, n_lo), n_hi + 1)}


def qsim_tune_get(ctx, prec: int) -> list:
    out = (ctypes.c_int * 17)()
    _check(lib().qsim_tune_get(_h(ctx), prec, out), "qsim_tune_get")
    return list(out)


def qsim_tune_set(ctx, prec: int, n_qubits: int, tile: int) -> None:
    _check(lib().qsim_tune_set(_h(ctx), prec, n_qubits, tile), "qsim_tune_set")


def qsim_tune_ms(ctx, prec: int) -> dict:
    """{n: (ms per product with 64-wide tiles, with 128-wide tiles)} for the qubit counts the autotuner timed."""
    out = (ctypes.c_double * 34)()
    _check(lib().qsim_tune_ms(_h(ctx), prec, out), "qsim_tune_ms")
    return {n: (out[2 * n], out[2 * n + 1]) for n in range(17) if out[2 * n] >= 0 or out[2 * n + 1] >= 0}


def qsim_tune_save(ctx, path: str) -> None:
    _check(lib().qsim_tune_save(_h(ctx), path.encode()), "qsim_tune_save")


def qsim_tune_load(ctx, path: str) -> None:
    _check(lib().qsim_tune_load(_h(ctx), path.encode()), "qsim_tune_load")


def qsim_build_id() -> str:
    return lib().qsim_build_id().decode()


def qsim_unitarity_drift_async(ctx, n_qubits: int, d_U, d_out, stream=None) -> None:
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_unitarity_drift_async(_h(ctx), n_qubits, _ptr(d_U), _ptr(d_out), st),
           "qsim_unitarity_drift_async")


def qsim_unitarity_drift_noalloc(n_qubits: int, d_U, d_out, stream=None) -> None:
    """Allocation-free drift check on d_U's device (current device, torch's current stream by default)."""
    st = _stream(stream, d_U.device.index if hasattr(d_U, "device") else None)
    _check(lib().qsim_unitarity_drift_noalloc(n_qubits, _ptr(d_U), _ptr(d_out), st), "qsim_unitarity_drift_noalloc")


def qsim_unitarity_drift_probe(ctx, n_qubits: int, d_U, stream=None) -> tuple:
    out = (ctypes.c_double * 2)()
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_unitarity_drift_probe(_h(ctx), n_qubits, _ptr(d_U), out, st), "qsim_unitarity_drift_probe")
    return float(out[0]), float(out[1])


# --- serving -------------------------------------------------------------------------------

def qsim_serve_start(ctx, prec: int, d_arena, arena_bytes: Optional[int] = None, mode: int = QSIM_SERVE_CONTINUOUS,
                     max_active: int = 64, queue_capacity: int = 4096, policy: int = QSIM_POLICY_ARRIVAL,
                     iter_budget_tflop: float = 2.0, aging_tflop_per_s: float = 0.0) -> None:
    if arena_bytes is None:
        arena_bytes = d_arena.numel() * d_arena.element_size() if hasattr(d_arena, "numel") else 0
    cfg = qsim_serve_config(prec, mode, max_active, queue_capacity, _ptr(d_arena), arena_bytes, policy, 0,
                            iter_budget_tflop, aging_tflop_per_s)
    _check(lib().qsim_serve_start(_h(ctx), ctypes.byref(cfg)), "qsim_serve_start")


def qsim_serve_stop(ctx) -> None:
    _check(lib().qsim_serve_stop(_h(ctx)), "qsim_serve_stop")


def qsim_submit(ctx, n_qubits: int, gates: Sequence, d_psi, d_psi0=None, d_U=None, probe: bool = True,
                full_drift: bool = False, flags: Optional[int] = None) -> int:
    """probe: the probe drift check; full_drift: the full float64 check instead; flags: raw request flags."""
    arr, ng = gate_array(gates)
    if flags is None:
        flags = QSIM_REQ_DRIFT_FULL if full_drift else (QSIM_REQ_DRIFT_PROBE if probe else 0)
    req = qsim_request(n_qubits, ng, ctypes.cast(arr, ctypes.POINTER(qsim_gate)), _ptr(d_psi), _ptr(d_psi0),
                       _ptr(d_U), flags, 0)
    rid = ctypes.c_uint64()
    _check(lib().qsim_submit(_h(ctx), ctypes.byref(req), ctypes.byref(rid)), "qsim_submit")
    return int(rid.value)


def qsim_poll(ctx, rid: int) -> Optional[dict]:
    """None while pending; else the result as a dict (its 'status' is the request's own outcome)."""
    res = qsim_result()
    st = lib().qsim_poll(_h(ctx), rid, ctypes.byref(res))
    if st == QSIM_PENDING:
        return None
    _check(st, "qsim_poll")
    return {f: getattr(res, f) for f, _ in qsim_result._fields_}


def qsim_serve_get_stats(ctx) -> dict:
    out = qsim_serve_stats()
    _check(lib().qsim_serve_get_stats(_h(ctx), ctypes.byref(out)), "qsim_serve_get_stats")
    return {f: getattr(out, f) for f, _ in qsim_serve_stats._fields_}


def qsim_sample(ctx, n_qubits: int, d_prob, d_uniform, shots: int, d_out, stream=None) -> None:
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_sample(_h(ctx), n_qubits, _ptr(d_prob), _ptr(d_uniform), shots, _ptr(d_out), st), "qsim_sample")


# --- full-state-vector simulation ---

def qsim_fsv_schedule(n_qubits: int, gates, with_order: bool = False):
    """Pass schedule of a gate list (host only): [(low_qubits, high_qubits, first_op, n_ops), ...], and with
    with_order the execution order (gate indices; pass p runs order[first_op:first_op + n_ops]).
    low_qubits == 0 marks a permutation pass (pairwise disjoint SWAPs on any qubits)."""
    arr, count = gate_array(gates)
    n = ctypes.c_int32(0)
    _check(lib().qsim_fsv_schedule(n_qubits, arr, count, None, 0, ctypes.byref(n), None), "qsim_fsv_schedule")
    buf = (qsim_fsv_pass_info * max(n.value, 1))()
    order = (ctypes.c_int32 * max(count, 1))()
    _check(lib().qsim_fsv_schedule(n_qubits, arr, count, buf, n.value, ctypes.byref(n), order), "qsim_fsv_schedule")
    passes = [(p.low_qubits, tuple(p.high[:p.n_high]), p.first_op, p.n_ops) for p in buf[:n.value]]
    return (passes, [int(order[i]) for i in range(count)]) if with_order else passes


class FsvPlan:
    """Owns a qsim_fsv_plan (qsim_fsv_plan_create / qsim_fsv_plan_destroy)."""

    def __init__(self, ctx, n_qubits: int, gates):
        arr, count = gate_array(gates)
        h = ctypes.c_void_p()
        _check(lib().qsim_fsv_plan_create(_h(ctx), n_qubits, arr, count, ctypes.byref(h)), "qsim_fsv_plan_create")
        self.handle = h.value
        self.ctx = ctx

    def info(self) -> dict:
        n, p, o = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().qsim_fsv_plan_info(self.handle, ctypes.byref(n), ctypes.byref(p), ctypes.byref(o)),
               "qsim_fsv_plan_info")
        return {"n_qubits": n.value, "passes": p.value, "ops": o.value}

    def run(self, d_psi, stream=None) -> None:
        st = _stream(stream, _dev(self.ctx)) if _h(self.ctx) else None
        _check(lib().qsim_fsv_run(_h(self.ctx), self.handle, _ptr(d_psi), st), "qsim_fsv_run")

    def close(self):
        if self.handle:
            _check(lib().qsim_fsv_plan_destroy(self.handle), "qsim_fsv_plan_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def qsim_fsv_init_basis(ctx, n_qubits: int, basis: int, d_psi, stream=None) -> None:
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_fsv_init_basis(_h(ctx), n_qubits, basis, _ptr(d_psi), st), "qsim_fsv_init_basis")


def qsim_fsv_norm2(ctx, n_qubits: int, d_psi, stream=None) -> float:
    out = ctypes.c_double(float("nan"))
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    _check(lib().qsim_fsv_norm2(_h(ctx), n_qubits, _ptr(d_psi), ctypes.byref(out), st), "qsim_fsv_norm2")
    return out.value


# --- operation data provider ---

def qsim_register_unitary(name: str, matrix) -> int:
    """Register a 2^m x 2^m unitary (index bit k = qubit a+k of the range it is applied to); returns its id."""
    import numpy as np
    M = np.asarray(matrix, dtype=np.complex128)
    D = M.shape[0]
    m = D.bit_length() - 1
    if M.shape != (D, D) or (1 << m) != D:
        raise ValueError("custom matrix must be 2^m x 2^m")
    flat = np.empty(2 * D * D, dtype=np.float64)
    flat[0::2] = M.real.ravel()
    flat[1::2] = M.imag.ravel()
    out = ctypes.c_int32(0)
    _check(lib().qsim_register_unitary(name.encode(), m, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       ctypes.byref(out)), "qsim_register_unitary")
    return out.value


def qsim_find_unitary(name: str):
    """(id, qubit count) of a registered operation."""
    i, m = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().qsim_find_unitary(name.encode(), ctypes.byref(i), ctypes.byref(m)), "qsim_find_unitary")
    return i.value, m.value


def qsim_fsv_sample_workspace_bytes(n_qubits: int) -> int:
    return int(lib().qsim_fsv_sample_workspace_bytes(n_qubits))


def qsim_fsv_sample(ctx, n_qubits: int, d_psi, d_uniform, shots: int, d_out, d_ws, ws_bytes=None,
                    stream=None) -> None:
    st = _stream(stream, _dev(ctx)) if _h(ctx) else None
    if ws_bytes is None:
        ws_bytes = d_ws.numel() * d_ws.element_size() if hasattr(d_ws, "numel") else 0
    _check(lib().qsim_fsv_sample(_h(ctx), n_qubits, _ptr(d_psi), _ptr(d_uniform), shots, _ptr(d_out), _ptr(d_ws),
                                 ws_bytes, st), "qsim_fsv_sample")


# --- device peaks (measurement) ---------------------------------------------------------------

PROBE_KINDS = {"mfma_f32": 0, "mfma_bf16": 1, "mfma_f16": 2, "mfma_f64": 3}


def qsim_probe_mfma(ctx, kind: int, random_operands: bool = True) -> float:
    out = ctypes.c_double()
    _check(lib().qsim_probe_mfma(_h(ctx), kind, 1 if random_operands else 0, ctypes.byref(out)), "qsim_probe_mfma")
    return out.value


def qsim_probe_copy(ctx, d_src, d_dst, nbytes: int) -> float:
    out = ctypes.c_double()
    _check(lib().qsim_probe_copy(_h(ctx), _ptr(d_src), _ptr(d_dst), nbytes, ctypes.byref(out)), "qsim_probe_copy")
    return out.value
