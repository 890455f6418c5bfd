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


LO_SCALE = 2.0 ** 12


def _bf16_rne(x32):
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def _bf16_val(h):
    return (h.astype(np.uint32) << 16).view(np.float32)


def split_planes(M, fmt, col_major=False):
    """Host split of a complex matrix into (re_hi, re_lo, im_hi, im_lo) 16-bit planes, row- or column-major."""
    M = np.asarray(M)
    if col_major:
        M = M.T
    out = []
    for part in (M.real, M.imag):
        x = np.ascontiguousarray(part, dtype=np.float32)
        if fmt == "bf16":
            hi = _bf16_rne(x)
            lo = _bf16_rne((x - _bf16_val(hi)).astype(np.float32))
        else:
            h16 = x.astype(np.float16)
            hi = h16.view(np.uint16)
            lo = ((x - h16.astype(np.float32)) * np.float32(LO_SCALE)).astype(np.float16).view(np.uint16)
        out += [hi, lo]
    return torch.from_numpy(np.stack(out).view(np.int16)).to(DEV)


def unsplit(t, fmt, col_major=False):
    """Reconstruct the complex128 value hi + lo * s from 16-bit split planes."""
    a = t.detach().cpu().numpy().view(np.uint16)
    if fmt == "bf16":
        v = [_bf16_val(a[p]).astype(np.float64) for p in range(4)]
        re, im = v[0] + v[1], v[2] + v[3]
    else:
        v = [a[p].view(np.float16).astype(np.float64) for p in range(4)]
        re, im = v[0] + v[1] / LO_SCALE, v[2] + v[3] / LO_SCALE
    M = re + 1j * im
    return M.T if col_major else M


def split_buffer(n):
    N = 1 << n
    return torch.empty((4, N, N), dtype=torch.int16, device=DEV)
