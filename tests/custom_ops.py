"""Turns the oracle's custom-operation tuples (name, range, None, matrix) into library gate tuples
("CUSTOM", range, None, op_id), registering each named matrix once per process."""
import numpy as np

from paper_2305_14398_amd import binding as B


_seen = {}


def op_id(name: str, matrix) -> int:
    M = np.asarray(matrix, dtype=np.complex128)
    if name in _seen:
        if not np.array_equal(_seen[name], M):
            raise ValueError(f"{name} is already registered with another matrix")
    else:
        _seen[name] = M.copy()
    try:
        i, m = B.qsim_find_unitary(name)
    except B.QsimError:
        return B.qsim_register_unitary(name, M)
    if (1 << m) != M.shape[0]:
        raise ValueError(f"{name} is registered with another size")
    return i


def lib_gates(gates):
    out = []
    for g in gates:
        if len(g) == 4 and g[0] != "U2":
            out.append(("CUSTOM", g[1], None, op_id(g[0], g[3])))
        else:
            out.append(g)
    return out
