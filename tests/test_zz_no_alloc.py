"""ntu_metric_fix_noalloc (the metric repair for callers that cannot
allocate) through the C ABI against ntu_metric_fix on the same inputs: two
calls in a row, the second with a smaller input, bit for bit (the same
kernels run on the same data; only the scratch space differs)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, batched, rel, to_np
from oracle import ntu as O

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2107_06635_amd import ntu


def _metrics(seed, n, batch, cplx, definite=False):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(batch):
        M = rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if cplx else 0)
        h = (M + M.conj().T) / 2
        if definite:
            h = h + (2.0 * np.sqrt(n) + 1.0) * np.eye(n)
        skew = 1e-6 * (rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if cplx else 0))
        out.append(h + skew)
    return out


@pytest.mark.parametrize("cplx", [True, False])
def test_noalloc_matches_metric_fix(cplx):
    D1, D2 = 8, 3
    ctx = ntu.Context(complex_=cplx, d=2, d_anc=1, r_g=2, max_D=D1, max_batch=4)
    for call, (D, batch, seed, definite) in enumerate(((D1, 3, 70, False), (D2, 2, 71, False), (D2, 2, 72, True))):
        n = (2 * D) ** 2
        gs = _metrics(seed, n, batch, cplx, definite)
        g_ref = batched(gs)
        g_new = g_ref.clone()
        st_ref = ntu.ntu_metric_fix(ctx, g_ref, D, ntu.FIX_HERM_CLIP)
        st_new = torch.full((batch, 8), -7.0, dtype=torch.float64, device=DEV)
        ntu.ntu_metric_fix_noalloc(g_new, ntu.FIX_HERM_CLIP, st_new)
        torch.cuda.synchronize()
        assert torch.equal(g_new, g_ref), call
        a, b = to_np(st_new), to_np(st_ref)
        assert np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)]), call
        # and the oracle's clip, as a check of both
        go, so = O.metric_fix(gs[0])
        assert rel(to_np(g_new)[0], go) < 1e-12, call
    # Hermitisation only, without stats
    gs = _metrics(73, 36, 2, cplx)
    g_ref, g_new = batched(gs), batched(gs)
    ntu.ntu_metric_fix(ctx, g_ref, 3, ntu.FIX_HERM)
    ntu.ntu_metric_fix_noalloc(g_new, ntu.FIX_HERM, None)
    torch.cuda.synchronize()
    assert torch.equal(g_new, g_ref)


def test_noalloc_rejects_beyond_scratch():
    """Requests beyond the scratch array are refused before any launch, with
    a message; the buffer is left unchanged."""
    n = 256
    batch = 17  # 17 complex items of n = 256 need 34 MiB > 32 MiB
    g = torch.zeros(batch, n, n, dtype=torch.complex128, device=DEV)
    with pytest.raises(RuntimeError, match=r"\(-6\).*scratch"):
        ntu.ntu_metric_fix_noalloc(g)
    with pytest.raises(RuntimeError, match=r"\(-2\)"):
        ntu.ntu_metric_fix_noalloc(g[:, :, :100].contiguous())
    with pytest.raises(RuntimeError, match=r"\(-3\)"):
        ntu.ntu_metric_fix_noalloc(g[:2].to(torch.complex64))
    torch.cuda.synchronize()
    assert not g.any()
