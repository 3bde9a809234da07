"""Helpers shared by the GPU parity tests (argument plumbing only)."""
import numpy as np
import torch

from oracle import ntu as O
from paper_2107_06635_amd import ntu

DEV = torch.device("cuda", 0) if torch.cuda.is_available() else None


def to_dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV).contiguous()


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def batched(arrs, dtype=None):
    return to_dev(np.stack(arrs), dtype)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gate_factors_array(pairs, cplx=True):
    """(GA, GB) per bond (dict over O.BONDS) -> (4, 2, d, d, r) array."""
    d, r = pairs['H1'][0].shape[0], pairs['H1'][0].shape[2]
    out = np.zeros((4, 2, d, d, r), dtype=np.complex128 if cplx else np.float64)
    for i, b in enumerate(O.BONDS):
        out[i, 0], out[i, 1] = pairs[b]
    return out


def fit_stat_fields(st, n_iter, D):
    """Split a bond-fit stats row into named fields."""
    return dict(N=st[0], eps_svdu=st[1], eps=st[2], delta=st[3], Dn=int(st[4]), Dk=int(st[5]),
                iters=int(st[6]), n_eig=int(st[7]), nonfinite=st[8],
                eps_hist=st[16:16 + 2 * n_iter], tau_hist=st[16 + 2 * n_iter:16 + 4 * n_iter],
                S=st[16 + 4 * n_iter:16 + 4 * n_iter + D])
