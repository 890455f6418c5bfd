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


def to_blocked(planes):
    """(P, N, N) planes (rows i, contraction index k) -> the fragment-blocked order of the three-product split
    operands for N >= 64: 32 x 16 blocks in row-block-major, k-block-minor order, each holding its P planes as
    1 KiB fragments in MFMA lane order (lane (i % 32) + 32 ((k / 8) % 2), eight consecutive k per lane)."""
    P, N, _ = planes.shape
    return np.ascontiguousarray(planes.reshape(P, N // 32, 32, N // 16, 2, 8).transpose(1, 3, 0, 4, 2, 5)).reshape(P, N, N)


def from_blocked(a):
    P, N, _ = a.shape
    return np.ascontiguousarray(a.reshape(N // 32, N // 16, P, 2, 32, 8).transpose(2, 0, 4, 1, 3, 5)).reshape(P, N, N)


def split_planes(M, fmt, col_major=False, gauss=False):
    """Host split of a complex matrix into (re_hi, re_lo, im_hi, im_lo) 16-bit planes, row- or column-major;
    gauss: also (sum_hi, sum_lo), the split of the float32 sum re + im, in the three-product operand format
    (fragment-blocked from 64 x 64 on)."""
    M = np.asarray(M)
    if col_major:
        M = M.T
    re = np.ascontiguousarray(M.real, dtype=np.float32)
    im = np.ascontiguousarray(M.imag, dtype=np.float32)
    parts = [re, im] + ([(re + im).astype(np.float32)] if gauss else [])
    out = []
    for x in parts:
        if fmt == "bf16":
            hi = _bf16_rne(x)
            lo = _bf16_rne((x - _bf16_val(hi)).astype(np.float32))
        else:
            h16 = x.astype(np.float16)
            hi = h16.view(np.uint16)
            lo = ((x - h16.astype(np.float32)) * np.float32(LO_SCALE)).astype(np.float16).view(np.uint16)
        out += [hi, lo]
    planes = np.stack(out)
    if gauss and planes.shape[1] >= 64:
        planes = to_blocked(planes)
    return torch.from_numpy(planes.view(np.int16)).to(DEV)


def _unsplit_pair(a, p, fmt):
    if fmt == "bf16":
        return _bf16_val(a[p]).astype(np.float64) + _bf16_val(a[p + 1]).astype(np.float64)
    return a[p].view(np.float16).astype(np.float64) + a[p + 1].view(np.float16).astype(np.float64) / LO_SCALE


def _planes(t):
    a = t.detach().cpu().numpy().view(np.uint16)
    if a.shape[0] == 6 and a.shape[1] >= 64:  # three-product operands are fragment-blocked from 64 x 64 on
        a = from_blocked(a)
    return a


def unsplit(t, fmt, col_major=False):
    """Reconstruct the complex128 value hi + lo * s from 16-bit split planes (the first four)."""
    a = _planes(t)
    M = _unsplit_pair(a, 0, fmt) + 1j * _unsplit_pair(a, 2, fmt)
    return M.T if col_major else M


def unsplit_sum(t, fmt, col_major=False):
    """The value carried by the sum planes (4, 5) of a six-plane operand."""
    a = _planes(t)
    S = _unsplit_pair(a, 4, fmt)
    return S.T if col_major else S


def split_buffer(n, gauss=False):
    N = 1 << n
    return torch.empty((6 if gauss else 4, N, N), dtype=torch.int16, device=DEV)


# --- error bounds of split-operand chains --------------------------------------------------
# One split product, per output entry, for operands with unit-norm rows (the step
# operator) and columns (the running product): each float x is carried as
# hi + lo with a residual of at most 2^-16 |x| (bf16: 8 significant bits in hi,
# 8 more in lo) or 2^-22 |x| (fp16: 11 + 11), and the dropped lo*lo term is
# within the same bound, so a real product x*y is off by at most 3 u |x y|; an
# entry sums |x_k||y_k| over k, which Cauchy-Schwarz bounds by 1.  Float32
# accumulation and the float32 result add about 2^-24 more.  The unitary steps
# that follow a product carry its error unchanged in 2-norm, and the roundings of
# different products are independent, so over P products the column (and state)
# error adds in quadrature: ||dU[:, j]||_2 <= 3 (u + 2^-24) sqrt(P), which also
# bounds every entry.  The measured errors sit well inside this (12-13 qubits,
# P ~ 110: max |dU| ~ 1e-6 for bf16, 3e-8 for fp16).
SPLIT_UNIT = {"bf16": 2.0 ** -16, "fp16": 2.0 ** -22}


def split_chain_bound(fmt, products, gauss=False):
    """gauss: the three-product form, whose imaginary part T3 - T1 - T2 sums errors over |x_r + x_i||y_r + y_i|
    (<= 2 |x||y|) and over both real products, so its per-entry bound is 3 times the four-product one."""
    c = 3.0 if gauss else 1.0
    return 3.0 * (c * SPLIT_UNIT[fmt] + 2.0 ** -24) * np.sqrt(max(int(products), 1))


# split precision -> (fmt, gauss)
def split_kind(prec):
    from paper_2305_14398_amd import binding as B
    return {B.QSIM_SPLIT_BF16: ("bf16", False), B.QSIM_SPLIT_FP16: ("fp16", False),
            B.QSIM_SPLIT_BF16_3M: ("bf16", True), B.QSIM_SPLIT_FP16_3M: ("fp16", True)}[prec]


def chain_products(n, gates):
    """Products of a packed chain (k - 1 for k steps; 0 for an empty or one-step circuit)."""
    from paper_2305_14398_amd import binding as B
    return max(len(B.qsim_pack_steps(n, gates)) - 2, 0)


def max_col_err(got, ref):
    """Largest 2-norm over columns of got - ref (matrices) or the 2-norm (vectors)."""
    d = np.asarray(got) - np.asarray(ref)
    if d.ndim == 1:
        return float(np.linalg.norm(d))
    return float(np.sqrt((np.abs(d) ** 2).sum(axis=0)).max())
