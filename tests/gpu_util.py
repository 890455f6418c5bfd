"""Helpers for the GPU tests: device buffers in the library's planar layouts and
conversions to complex128 numpy arrays for comparison with the oracle."""
import numpy as np
import torch

DEV = "cuda:0"


def planar(n, fill=None):
    N = 1 << n
    t = torch.empty((2, N, N), dtype=torch.float32, device=DEV)
    if fill is not None:
        t.copy_(to_planar(fill))
    return t


def to_planar(M):
    M = np.asarray(M)
    return torch.from_numpy(np.stack([M.real, M.imag]).astype(np.float32))


def planar_vec(v):
    v = np.asarray(v)
    return torch.from_numpy(np.concatenate([v.real, v.imag]).astype(np.float32)).to(DEV)


def to_complex(t, col_major=False):
    a = t.detach().cpu().numpy().astype(np.float64)
    M = a[0] + 1j * a[1]
    return M.T if col_major else M


def vec_to_complex(t):
    a = t.detach().cpu().numpy().astype(np.float64)
    N = a.size // 2
    return a[:N] + 1j * a[N:]


def workspace(nbytes):
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=DEV)


def sync():
    torch.cuda.synchronize()
