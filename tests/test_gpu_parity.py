"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Sizes span several 64-wide tiles with ragged tails (D = 3, 5: R^2 = 36, 100,
D^4 = 81, 625).  Tolerances: FP64 results to ~1e-11 relative (rounding order
only); split-precision metrics against the error budget of their mode.
"""
import numpy as np
import pytest
import torch

from gpu_util import DEV, batched, fit_stat_fields, gate_factors_array, rel, to_dev, to_np
from oracle import ntu as O
from paper_2107_06635_amd import inputs

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2107_06635_amd import ntu


def _ctx(cplx=True, d_anc=1, max_D=6, max_batch=4):
    return ntu.Context(complex_=cplx, d=2, d_anc=d_anc, r_g=2, max_D=max_D, max_batch=max_batch)


def _case(seed, D, p=2, real=False, dt=0.05, hx=3.0):
    rng = np.random.default_rng(seed)
    dtype = np.float64 if real else np.complex128
    X, Y = inputs.random_site_pair(rng, p, D, dtype)
    nbr = inputs.random_neighbours(rng, p, D, dtype)
    G = inputs.bond_gate(inputs.ising_bond_hamiltonian(hx), dt, imaginary=real)
    GA, GB, _ = O.gate_split(G, 2, 2)
    return X, Y, nbr, G, GA, GB


# ------------------------------------------------------------------ boundary

def test_empty_batch_and_argument_errors():
    """C ABI edge cases: batch 0 is a no-op on every compute call (NULL
    descriptors allowed); sizes outside the context, bad enums and NULL
    buffers give their status codes and a message, before any launch."""
    import ctypes
    ctx = _ctx(max_D=3, max_batch=2)
    L, h = ctx.L, ctx.h
    NULL = None
    nbr0 = (ntu.Tensor * 6)()
    fo = ntu.fit_opts(n_iter=3)
    so = ntu.step_opts("f64", n_iter=3)
    OK, ARG, SHAPE, WS = 0, -1, -2, -6
    ctx.bind_stream()
    assert L.ntu_gate_split(h, 0, NULL, NULL, NULL, NULL) == OK
    assert L.ntu_reduce_qr(h, 0, NULL, NULL, 0, NULL, NULL) == OK
    assert L.ntu_env_contract(h, 0, NULL, NULL, nbr0, 3, NULL) == OK
    assert L.ntu_metric_fix(h, 0, NULL, 1, NULL) == OK
    assert L.ntu_bond_fit(h, 0, NULL, NULL, NULL, ctypes.byref(fo), NULL, NULL, NULL) == OK
    assert L.ntu_recombine(h, 0, NULL, NULL, NULL, NULL, NULL, NULL) == OK
    assert L.ntu_trotter_step(h, 0, NULL, NULL, NULL, ctypes.byref(so), NULL) == OK
    # sizes outside the context, negative batch, NULL buffers, bad enums
    site4 = ntu.tensor(torch.zeros(1, 2, 4, 4, 4, 4, dtype=torch.complex128, device=DEV))
    assert L.ntu_reduce_qr(h, 1, ctypes.byref(site4), NULL, 0, NULL, NULL) == SHAPE
    assert L.ntu_reduce_qr(h, 3, NULL, NULL, 0, NULL, NULL) == WS
    assert L.ntu_reduce_qr(h, -1, NULL, NULL, 0, NULL, NULL) == ARG
    assert L.ntu_reduce_qr(h, 1, NULL, NULL, 0, NULL, NULL) == SHAPE
    assert L.ntu_last_error(h).decode()
    assert L.ntu_env_contract(h, 1, NULL, NULL, nbr0, 9, NULL) == ARG
    assert L.ntu_metric_fix(h, 1, NULL, 7, NULL) == ARG
    bad = ntu.step_opts("f64", n_iter=3)
    bad.scheme = 5
    assert L.ntu_trotter_step(h, 1, NULL, NULL, NULL, ctypes.byref(bad), NULL) == ARG
    bad = ntu.step_opts("f64", n_iter=3)
    bad.n_bonds = 9
    assert L.ntu_trotter_step(h, 1, NULL, NULL, NULL, ctypes.byref(bad), NULL) == ARG
    torch.cuda.synchronize()


def test_descriptor_errors_before_launch():
    """Every operand's descriptor is checked on the host before anything is
    launched: wrong element type (NTU_ERR_DTYPE), wrong extent, rank or a
    strided view (NTU_ERR_SHAPE), host memory or a NULL data pointer
    (NTU_ERR_ARG).  Complex64 site tensors pass where the header allows them
    and are refused elsewhere.  After each refusal the buffers are
    untouched and a correct call still works."""
    D, b = 3, 2
    ctx = _ctx(max_D=D, max_batch=b)
    X, Y, nbr, G, GA, GB = _case(330, D)
    A = batched([X, Y])
    B = batched([Y, X])
    gf = to_dev(np.stack([gate_factors_array({bb: (GA, GB) for bb in O.BONDS})] * b))
    opts = ntu.step_opts("f64", n_iter=3)
    A0, B0 = A.clone(), B.clone()

    def step_status(a, bb, g=gf, st=None):
        import ctypes
        ctx.bind_stream()
        return ctx.L.ntu_trotter_step(ctx.h, b, ntu._ref(a), ntu._ref(bb), ntu._ref(g), ctypes.byref(opts),
                                      ntu._ref(st))

    DTYPE, SHAPE, ARG = -3, -2, -1
    # element types: real site tensors in a complex context; gate factors in complex64
    assert step_status(A.real.contiguous(), B.real.contiguous()) == DTYPE
    assert b"element type" in ctx.L.ntu_last_error(ctx.h)
    assert step_status(A, B, gf.to(torch.complex64)) == DTYPE
    # A and B of different element types
    assert step_status(A, B.to(torch.complex64)) == DTYPE
    # extents: D mismatch between A and B, a short batch, a wrong gate rank
    assert step_status(A, B[:, :, :, :, :, :2].contiguous()) == SHAPE
    assert step_status(A[:1], B[:1]) == SHAPE
    assert step_status(A, B, gf[..., :1].contiguous()) == SHAPE
    # a strided (transposed) view of the right shape
    At = A.transpose(3, 4)
    assert not At.is_contiguous()
    assert step_status(At, B) == SHAPE
    assert b"dense row-major" in ctx.L.ntu_last_error(ctx.h)
    # stats of the wrong length
    assert step_status(A, B, st=torch.zeros(b, 4, 5, dtype=torch.float64, device=DEV)) == SHAPE
    # host memory
    assert step_status(A.cpu(), B) == ARG
    assert b"device memory" in ctx.L.ntu_last_error(ctx.h)
    torch.cuda.synchronize()
    assert torch.equal(A, A0) and torch.equal(B, B0)
    # the other entry points check theirs too
    QX, _ = O.reduce_site(X, GA, 'X', 2)
    QY, _ = O.reduce_site(Y, GB, 'Y', 2)
    R = 2 * D
    q = batched([QX.reshape(-1, R)] * b)
    nb = [batched([t, t]) for t in nbr]
    with pytest.raises(RuntimeError, match=r"\(-2\).*QY: shape"):
        ntu.ntu_env_contract(ctx, q, q[:, :, :4].contiguous(), nb)
    with pytest.raises(RuntimeError, match=r"\(-3\).*nbr\[2\]"):
        ntu.ntu_env_contract(ctx, q, q, nb[:2] + [nb[2].to(torch.complex64)] + nb[3:])
    with pytest.raises(RuntimeError, match=r"\(-2\).*site"):
        ntu.ntu_reduce_qr(ctx, A.transpose(2, 3), batched([GA, GA]), 0)
    g = ntu.ntu_env_contract(ctx, q, q, nb)
    with pytest.raises(RuntimeError, match=r"\(-2\)"):
        ntu.ntu_metric_fix(ctx, g[:, :, :30].contiguous())
    with pytest.raises(RuntimeError, match=r"\(-3\).*RX"):
        ntu.ntu_bond_fit(ctx, g, batched([np.eye(R)] * b, torch.complex64), batched([np.eye(R)] * b), D)
    # complex64 site tensors are accepted by the reduction (read with an upcast)
    Q64, R64 = ntu.ntu_reduce_qr(ctx, A.to(torch.complex64), batched([GA, GA]), 0)
    Qo, Ro = O.reduce_site(X.astype(np.complex64).astype(np.complex128), GA, 'X', 2)
    assert rel(to_np(R64)[0], Ro) < 1e-12
    # and a correct step still runs
    assert step_status(A, B) == 0
    torch.cuda.synchronize()


def test_complex64_storage_trotter_step():
    """Complex64 storage of A and B in the Trotter step (configuration 4's
    storage): the step widens them, runs in complex128 and stores the result
    rounded to complex64.  Against the oracle run on the same (widened)
    values: after one H1 update the pair contracted over that bond (gauge
    invariant) within the rounding of complex64 (relative 1e-6); after an
    H1, V1 sweep the cluster energy and <X> within 1e-7; the errors of every
    update at 1e-9."""
    D = 3
    rng = np.random.default_rng(41)
    X, Y = inputs.random_site_pair(rng, 2, D, np.complex64)
    G = inputs.bond_gate(inputs.ising_bond_hamiltonian(3.1), 0.01)
    GA, GB, _ = O.gate_split(G, 2, 2)
    pairs = {bb: (GA, GB) for bb in O.BONDS}
    gf = to_dev(gate_factors_array(pairs)[None])
    ctx = _ctx(max_D=D)
    pair = lambda a, b: np.einsum('ptlbk,qTkBR->ptlbqTBR', a, b).reshape(-1)
    for names, codes in ((('H1',), (0,)), (('H1', 'V1'), (0, 2))):
        Ao, Bo, infos = O.trotter_step(X.astype(np.complex128), Y.astype(np.complex128), pairs, D, n_iter=4,
                                       order=names)
        At, Bt = to_dev(X[None]), to_dev(Y[None])
        assert At.dtype == torch.complex64
        st = to_np(ntu.ntu_trotter_step(ctx, At, Bt, gf, ntu.step_opts("f64", order=codes, n_iter=4)))[0]
        assert At.dtype == torch.complex64 and Bt.dtype == torch.complex64
        An, Bn = to_np(At)[0].astype(np.complex128), to_np(Bt)[0].astype(np.complex128)
        if names == ('H1',):
            assert rel(pair(An, Bn), pair(Ao, Bo)) < 1e-6
        else:
            eo, xo = O.observables(Ao, Bo, 3.1)
            eg, xg = O.observables(An, Bn, 3.1)
            assert abs(eg - eo) < 1e-7 and abs(xg - xo) < 1e-7, (eg - eo, xg - xo)
        for bi, bb in enumerate(names):
            f = fit_stat_fields(st[bi, 8:], 4, D)
            assert abs(f['delta'] - infos[bb]['delta']) <= 1e-9 * infos[bb]['delta'] + 1e-14


# ------------------------------------------------------------------ gate split

@pytest.mark.parametrize("real", [False, True])
def test_gate_split(real):
    G = inputs.bond_gate(inputs.ising_bond_hamiltonian(inputs.H_CRIT), 0.01, imaginary=real)
    GA, GB, s = O.gate_split(G, 2, 2)
    ctx = _ctx(cplx=not real, max_D=2)
    ga, gb, sg = ntu.ntu_gate_split(ctx, batched([G, G]))
    ga, gb, sg = to_np(ga), to_np(gb), to_np(sg)
    for i in range(2):
        assert np.allclose(sg[i], s, atol=1e-14 * s[0])
        assert np.allclose(ga[i], GA, atol=1e-12) and np.allclose(gb[i], GB, atol=1e-12)


# ------------------------------------------------------------------ reduce

@pytest.mark.parametrize("D,p,real", [(2, 2, False), (3, 2, False), (5, 2, False), (3, 4, True)])
def test_reduce_qr(D, p, real):
    X, Y, nbr, G, GA, GB = _case(100 + D, D, p, real)
    ctx = _ctx(cplx=not real, d_anc=p // 2)
    for side, T, gf in ((0, X, GA), (1, Y, GB)):
        Qo, Ro = O.reduce_site(T, gf, 'XY'[side], 2)
        Q, R = ntu.ntu_reduce_qr(ctx, batched([T, T]), batched([gf, gf]), side)
        Q, R = to_np(Q), to_np(R)
        for i in range(2):
            assert rel(Q[i], Qo.reshape(Q[i].shape)) < 1e-12
            assert rel(R[i], Ro) < 1e-12


@pytest.mark.parametrize("D", [4, 6, 8])
def test_reduce_qr_rank_deficient_and_complex64(D):
    # beta = 0 purification (real, p = 4): most columns of W are dependent
    # (rank rule); D = 4, 6, 8 give 256, 864, 2048 rows of W (one and two rows
    # per thread of the register-resident Gram-Schmidt, 512 and 1024 threads)
    A, B = inputs.thermal_product_purification(D)
    G = inputs.bond_gate(inputs.ising_bond_hamiltonian(2.5).real, 0.005, imaginary=True)
    GA, GB, _ = O.gate_split(G, 2, 2)
    ctx = _ctx(cplx=False, d_anc=2, max_D=D)
    for side, T, gf in ((0, A, GA), (1, B, GB)):
        Qo, Ro = O.reduce_site(T, gf, 'XY'[side], 2)
        Q, R = ntu.ntu_reduce_qr(ctx, batched([T]), batched([gf]), side)
        Q, R = to_np(Q)[0], to_np(R)[0]
        zero_cols = np.all(Qo.reshape(Q.shape) == 0, axis=0)
        assert zero_cols.sum() > 0 and np.array_equal(np.all(Q == 0, axis=0), zero_cols)
        assert rel(Q, Qo.reshape(Q.shape)) < 1e-12 and rel(R, Ro) < 1e-12
    # complex, p = 2: the |+> product state padded to D (rank-deficient W of
    # 2 D^3 rows), and a random state with a few of its bond columns zero
    rng = np.random.default_rng(40 + D)
    Gc = inputs.bond_gate(inputs.ising_bond_hamiltonian(3.0), 0.01)
    GA, GB, _ = O.gate_split(Gc, 2, 2)
    Pa, Pb = inputs.plus_product_state(D)
    X, Y = inputs.random_site_pair(rng, 2, D)
    X[..., D // 2:] = 0.0
    ctx = _ctx(max_D=D)
    for T in (Pa.astype(np.complex128), X):
        Qo, Ro = O.reduce_site(T, GA, 'X', 2)
        Q, R = ntu.ntu_reduce_qr(ctx, batched([T]), batched([GA]), 0)
        Q, R = to_np(Q)[0], to_np(R)[0]
        zero_cols = np.all(Qo.reshape(Q.shape) == 0, axis=0)
        assert zero_cols.sum() > 0 and np.array_equal(np.all(Q == 0, axis=0), zero_cols)
        assert rel(Q, Qo.reshape(Q.shape)) < 1e-12 and rel(R, Ro) < 1e-12
    # complex64 storage of the site tensor, upcast on load
    rng = np.random.default_rng(5)
    X, _ = inputs.random_site_pair(rng, 2, 3, np.complex64)
    GA, GB, _ = O.gate_split(inputs.bond_gate(inputs.ising_bond_hamiltonian(3.0), 0.01), 2, 2)
    Qo, Ro = O.reduce_site(X.astype(np.complex128), GA, 'X', 2)
    ctx = _ctx()
    Q, R = ntu.ntu_reduce_qr(ctx, to_dev(X[None]), batched([GA]), 0)
    assert rel(to_np(R)[0], Ro) < 1e-12


# ------------------------------------------------------------------ environment

@pytest.mark.parametrize("D,p,real", [(2, 2, False), (3, 2, False), (5, 2, False), (3, 4, True), (4, 4, True)])
def test_env_contract_f64(D, p, real):
    X, Y, nbr, G, GA, GB = _case(200 + D, D, p, real)
    QX, _ = O.reduce_site(X, GA, 'X', 2)
    QY, _ = O.reduce_site(Y, GB, 'Y', 2)
    go = O.metric(QX, QY, nbr)
    R = D * 2
    ctx = _ctx(cplx=not real, d_anc=p // 2)
    q = lambda Q: batched([Q.reshape(-1, R)] * 2)
    g = ntu.ntu_env_contract(ctx, q(QX), q(QY), [batched([t, t]) for t in nbr], "f64")
    g = to_np(g)
    for i in range(2):
        assert rel(g[i], go) < 1e-12


@pytest.mark.parametrize("prec,tol", [("bf16x3", 3e-5), ("fp16x3", 1e-6), ("bf16x6", 1e-6)])
@pytest.mark.parametrize("D,p,real", [(3, 2, False), (5, 2, False), (5, 4, False), (4, 4, True),
                                      (6, 2, False), (7, 2, False), (8, 2, False), (9, 2, False),
                                      (10, 2, False), (8, 4, True)])
def test_env_contract_mixed(prec, tol, D, p, real):
    """Split-precision metric, element by element against the oracle:
    relative Frobenius error within the mode's budget.  Complex D <= 8 takes
    the fused kernels (D = 5, p = 4: contraction index p D = 20 spans two
    MFMA K steps of the Left/Right blocks; D = 6, 7: D^2 = 36, 49 padded to
    the next multiple of 16; D = 8: no padding); complex D = 9, 10 and every
    real case take the tiled products for Left, Right, L1 and L2.

    FP16x3 (float16 pieces hi + 2^-11 lo, 22 bits, every operand block scaled
    by a power of two, the final assembly from pre-split rows) exists on the
    fused path only: elsewhere the call reports NTU_ERR_UNSUPPORTED.  Its
    budget: 2^-22 per operand value against 2^-24 for BF16x6, the same FP32
    accumulation; asserted at the 1e-6 target."""
    X, Y, nbr, G, GA, GB = _case(300 + D, D, p, real)
    QX, _ = O.reduce_site(X, GA, 'X', 2)
    QY, _ = O.reduce_site(Y, GB, 'Y', 2)
    R = D * 2
    ctx = _ctx(cplx=not real, d_anc=p // 2, max_D=max(D, 6), max_batch=1)
    q = lambda Q: batched([Q.reshape(-1, R)])
    if prec == "fp16x3" and (real or D > 8):
        with pytest.raises(RuntimeError, match=r"\(-7\)"):
            ntu.ntu_env_contract(ctx, q(QX), q(QY), [batched([t]) for t in nbr], prec)
        return
    go = O.metric(QX, QY, nbr)
    g = to_np(ntu.ntu_env_contract(ctx, q(QX), q(QY), [batched([t]) for t in nbr], prec))[0]
    err = rel(g, go)
    print(f"{prec} D={D} p={p} real={real}: metric rel err {err:.3e}")
    assert err < tol


def test_env_tuning(tmp_path):
    """Autotuned schedule of the split-precision metric assembly (K split;
    for FP16x3 also the output tile width): every candidate gives the metric
    within the BF16x6 budget of the oracle; the tuned choice is kept and
    used, set and reset by hand, survives a save / load round trip into a
    fresh context, and refused values raise."""
    D, p = 5, 2
    X, Y, nbr, G, GA, GB = _case(310, D, p, False)
    QX, _ = O.reduce_site(X, GA, 'X', 2)
    QY, _ = O.reduce_site(Y, GB, 'Y', 2)
    go = O.metric(QX, QY, nbr)
    R = D * 2
    q = lambda Q: batched([Q.reshape(-1, R), Q.reshape(-1, R)])
    nb = [batched([t, t]) for t in nbr]
    ctx = _ctx(max_D=D)
    ks, ms = ntu.ntu_tune_env(ctx, q(QX), q(QY), nb, "bf16x6", D=D)
    assert 1 <= ks <= 4 and ms > 0 and ntu.ntu_get_env_ksplit(ctx, D, "bf16x6") == ks
    assert ntu.ntu_get_env_ksplit(ctx, D, "bf16x3") == 0
    for k in (1, 2, 3, 4, 0):
        ntu.ntu_set_env_ksplit(ctx, D, "bf16x6", k)
        assert ntu.ntu_get_env_ksplit(ctx, D, "bf16x6") == k
        g = to_np(ntu.ntu_env_contract(ctx, q(QX), q(QY), nb, "bf16x6"))
        for i in range(2):
            assert rel(g[i], go) < 1e-6, (k, i)
    ntu.ntu_set_env_ksplit(ctx, D, "bf16x6", 3)
    ntu.ntu_set_env_ksplit(ctx, 4, "bf16x3", 2)
    path = tmp_path / "tune.txt"
    ntu.ntu_tune_save(ctx, path)
    fresh = _ctx(max_D=D)
    ntu.ntu_tune_load(fresh, path)
    assert ntu.ntu_get_env_ksplit(fresh, D, "bf16x6") == 3 and ntu.ntu_get_env_ksplit(fresh, 4, "bf16x3") == 2
    with pytest.raises(RuntimeError):
        ntu.ntu_tune_env(ctx, q(QX), q(QY), nb, "f64", D=D)
    # FP16x3 tunes the K split and the width of the assembly's output tiles
    ks, ms = ntu.ntu_tune_env(ctx, q(QX), q(QY), nb, "fp16x3", D=D)
    assert ks >= 1 and ntu.ntu_get_env_ksplit(ctx, D, "fp16x3") == ks
    assert ntu.ntu_get_env_tile(ctx, D, "fp16x3") in (128, 256)
    g = to_np(ntu.ntu_env_contract(ctx, q(QX), q(QY), nb, "fp16x3"))
    for i in range(2):
        assert rel(g[i], go) < 1e-6, i
    for w in (128, 256, 0):
        for k in (1, 3):
            ntu.ntu_set_env_ksplit(ctx, D, "fp16x3", k)
            ntu.ntu_set_env_tile(ctx, D, "fp16x3", w)
            assert ntu.ntu_get_env_tile(ctx, D, "fp16x3") == w
            g = to_np(ntu.ntu_env_contract(ctx, q(QX), q(QY), nb, "fp16x3"))
            for i in range(2):
                assert rel(g[i], go) < 1e-6, (w, k, i)
    ntu.ntu_set_env_tile(ctx, D, "fp16x3", 256)
    ntu.ntu_tune_save(ctx, path)
    fresh = _ctx(max_D=D)
    ntu.ntu_tune_load(fresh, path)
    assert ntu.ntu_get_env_tile(fresh, D, "fp16x3") == 256 and ntu.ntu_get_env_ksplit(fresh, D, "fp16x3") == 3
    for bad in (("bf16x6", 256), ("fp16x3", 64)):
        with pytest.raises(RuntimeError):
            ntu.ntu_set_env_tile(ctx, D, *bad)
    (tmp_path / "bad.txt").write_text("5 2 2 100\n")
    with pytest.raises(RuntimeError):
        ntu.ntu_tune_load(fresh, tmp_path / "bad.txt")


# ------------------------------------------------------------------ metric fix

@pytest.mark.parametrize("real", [False, True])
def test_metric_fix(real):
    rng = np.random.default_rng(9)
    n = 36  # R = 6, D = 3
    M = rng.standard_normal((n, n)) + (0 if real else 1j * rng.standard_normal((n, n)))
    V, _ = np.linalg.qr(M)
    lam = np.linspace(-0.2, 3.0, n)
    g = (V * lam) @ V.conj().T
    skew = 1e-4 * (rng.standard_normal((n, n)) + (0 if real else 1j * rng.standard_normal((n, n))))
    skew = skew - skew.conj().T
    gin = g + skew
    go, so = O.metric_fix(gin)
    ctx = _ctx(cplx=not real, max_D=3)
    gt = batched([gin])
    st = to_np(ntu.ntu_metric_fix(ctx, gt, 3, ntu.FIX_HERM_CLIP))[0]
    assert rel(to_np(gt)[0], go) < 1e-12
    assert abs(st[0] - so['herm_err']) < 1e-13
    assert abs(st[2] - so['lam_min']) < 1e-12 and abs(st[3] - so['lam_max']) < 1e-12 and st[5] == 1.0
    # positive definite input: certified, nothing clipped
    gpd = (V * np.linspace(0.1, 2.0, n)) @ V.conj().T
    gt = batched([gpd])
    st = to_np(ntu.ntu_metric_fix(ctx, gt, 3, ntu.FIX_HERM_CLIP))[0]
    assert st[5] == 0.0 and rel(to_np(gt)[0], O.metric_fix(gpd)[0]) < 1e-13
    # indefinite with exactly zero rows and columns: the eigensolver runs on the
    # nonzero block, here of odd size (a pair with a dummy index in every round)
    for n, D, zero in ((16, 2, (5,)), (64, 4, (0, 17, 40))):
        M = rng.standard_normal((n, n)) + (0 if real else 1j * rng.standard_normal((n, n)))
        gz = (M + M.conj().T) / 2
        for z in zero:
            gz[z, :] = 0.0
            gz[:, z] = 0.0
        go, so = O.metric_fix(gz)
        ctx = _ctx(cplx=not real, max_D=D)
        gt = batched([gz])
        st = to_np(ntu.ntu_metric_fix(ctx, gt, D, ntu.FIX_HERM_CLIP))[0]
        assert rel(to_np(gt)[0], go) < 1e-12 and st[5] == 1.0
        assert abs(st[2] - so['lam_min']) < 1e-12 * abs(so['lam_max'])



@pytest.mark.parametrize("real", [False, True])
def test_metric_fix_eigensolver_full_size(real):
    """The clip at the largest metric of the workloads (n = 256, D = 8, r = 2)
    and on an odd block (n = 144 with one zero row and column).  Complex: the
    Jacobi eigen-solve, each thread taking several chunks of rotation and
    eigenvector updates per round, the pair indices wrapping across rows.
    Real (n >= 128): the sign iteration, (g + g sign(g)) / 2, with the
    clipped mass from traces and no eigenvalues (NaN)."""
    rng = np.random.default_rng(31 + int(real))
    for n, D, zero in ((256, 8, ()), (144, 6, (7,))):
        M = rng.standard_normal((n, n)) + (0 if real else 1j * rng.standard_normal((n, n)))
        g = (M + M.conj().T) / 2
        for z in zero:
            g[z, :] = 0.0
            g[:, z] = 0.0
        go, so = O.metric_fix(g)
        ctx = _ctx(cplx=not real, max_D=D, max_batch=2)
        gt = batched([g, 2.0 * g])
        st = to_np(ntu.ntu_metric_fix(ctx, gt, D, ntu.FIX_HERM_CLIP))
        out = to_np(gt)
        assert rel(out[0], go) < 1e-12 and rel(out[1], 2.0 * go) < 1e-12, (n, rel(out[0], go))
        if real:
            assert np.all(st[:, 5] == 2.0) and np.all(np.isnan(st[:, 2:4]))
            assert abs(st[0, 4] - so['clipped']) < 1e-10 * so['clipped']
            assert abs(st[1, 4] - so['clipped']) < 1e-10 * so['clipped']
        else:
            assert np.all(st[:, 5] == 1.0)
            assert abs(st[0, 2] - so['lam_min']) < 1e-12 * abs(so['lam_max'])


@pytest.mark.parametrize("n, D", [(400, 5), (256, 8)])
def test_metric_fix_sign_iteration_degenerate(n, D):
    """Real metrics of the thermal workloads (n = (D r_g)^2 = 400 for the
    Hermitian purification at D = 5, r_g = 4; 256 at D = 8, r_g = 2): a
    quarter of the spectrum spread over six decades, the rest a null space
    with +-1e-7 noise (the split-precision departure from non-negativity).
    The sign iteration's clip equals the oracle's eigen-decomposition clip
    to 1e-12; in the same batch a positive definite item is certified and
    left alone (the iteration skips it)."""
    rng = np.random.default_rng(41 + n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([np.logspace(0, -6, n // 4), 1e-7 * rng.standard_normal(n - n // 4)])
    g = (Q * lam) @ Q.T
    g = 0.5 * (g + g.T)
    gpd = (Q * np.linspace(0.5, 2.0, n)) @ Q.T
    gpd = 0.5 * (gpd + gpd.T)
    go, so = O.metric_fix(g)
    rg = 4 if n == 400 else 2
    ctx = ntu.Context(complex_=False, d=2, d_anc=2 if rg == 2 else 1, r_g=rg, max_D=D, max_batch=2)
    gt = batched([g, gpd])
    st = to_np(ntu.ntu_metric_fix(ctx, gt, D, ntu.FIX_HERM_CLIP))
    out = to_np(gt)
    assert rel(out[0], go) < 1e-12, rel(out[0], go)
    assert np.array_equal(out[0], out[0].T)
    assert st[0, 5] == 2.0 and abs(st[0, 4] - so['clipped']) < 1e-9 * so['clipped']
    assert st[1, 5] == 0.0 and np.array_equal(out[1], gpd)

# ------------------------------------------------------------------ fit

@pytest.mark.parametrize("D,p,real,n_iter", [(2, 2, False, 20), (3, 2, False, 6), (5, 2, False, 3), (3, 4, True, 6)])
def test_bond_fit(D, p, real, n_iter):
    X, Y, nbr, G, GA, GB = _case(400 + D, D, p, real, dt=0.3)
    QX, RX = O.reduce_site(X, GA, 'X', 2)
    QY, RY = O.reduce_site(Y, GB, 'Y', 2)
    g, _ = O.metric_fix(O.metric(QX, QY, nbr))
    fo = O.bond_fit(g, RX, RY, D, n_iter=n_iter)
    MXb, MYb, S, Dk = O.balance(fo['MX'], fo['MY'], D)
    ctx = _ctx(cplx=not real, d_anc=p // 2)
    MX, MY, st = ntu.ntu_bond_fit(ctx, batched([g]), batched([RX]), batched([RY]), D, ntu.fit_opts(n_iter=n_iter))
    MX, MY = to_np(MX)[0], to_np(MY)[0]
    f = fit_stat_fields(to_np(st)[0], n_iter, D)
    N = fo['N']
    assert abs(f['N'] - N) <= 1e-12 * N
    assert abs(f['eps_svdu'] - fo['eps_svdu']) <= 1e-10 * N
    assert np.allclose(f['eps_hist'], fo['eps'], rtol=1e-7, atol=1e-11 * N)
    assert f['Dn'] == fo['Dn'] and f['Dk'] == Dk
    assert np.allclose(f['S'], S, atol=1e-9)
    # gauge-invariant product of the balanced pair
    assert rel(MX @ MY.T, MXb @ MYb.T) < 1e-8


def test_bond_fit_eckart_young_on_gpu():
    """g = 1: the fit returns the truncated SVD of P (SVDU)."""
    rng = np.random.default_rng(77)
    R, D = 6, 3
    RX = rng.standard_normal((R, R)) + 1j * rng.standard_normal((R, R))
    RY = rng.standard_normal((R, R)) + 1j * rng.standard_normal((R, R))
    ctx = _ctx(max_D=3, max_batch=1)
    MX, MY, st = ntu.ntu_bond_fit(ctx, batched([np.eye(R * R, dtype=complex)]), batched([RX]), batched([RY]), D,
                                  ntu.fit_opts(n_iter=3))
    s = np.linalg.svd(RX @ RY.T, compute_uv=False)
    f = fit_stat_fields(to_np(st)[0], 3, D)
    assert abs(f['eps'] - np.sum(s[D:] ** 2)) <= 1e-11 * np.sum(s ** 2)


# ------------------------------------------------------------------ recombine + full update

@pytest.mark.parametrize("D,p,real", [(3, 2, False), (3, 4, True)])
def test_recombine(D, p, real):
    X, Y, nbr, G, GA, GB = _case(500 + D, D, p, real)
    QX, _ = O.reduce_site(X, GA, 'X', 2)
    QY, _ = O.reduce_site(Y, GB, 'Y', 2)
    rng = np.random.default_rng(3)
    R = 2 * D
    MX = rng.standard_normal((R, D)) + (0 if real else 1j * rng.standard_normal((R, D)))
    MY = rng.standard_normal((R, D)) + (0 if real else 1j * rng.standard_normal((R, D)))
    Xo, Yo = O.recombine(QX, QY, MX, MY)
    ctx = _ctx(cplx=not real, d_anc=p // 2)
    Xn, Yn = ntu.ntu_recombine(ctx, batched([QX.reshape(-1, R)]), batched([QY.reshape(-1, R)]), batched([MX]),
                               batched([MY]), D)
    assert rel(to_np(Xn)[0], Xo) < 1e-13 and rel(to_np(Yn)[0], Yo) < 1e-13


def _gpu_step(ctx, A, B, gf_pairs, n_iter, precision="f64", order=(0, 1, 2, 3), cplx=True, **kw):
    At, Bt = batched([A]), batched([B])
    gf = to_dev(gate_factors_array(gf_pairs, cplx)[None])
    st = ntu.ntu_trotter_step(ctx, At, Bt, gf, ntu.step_opts(precision, order=order, n_iter=n_iter, **kw))
    return to_np(At)[0], to_np(Bt)[0], to_np(st)[0]


def test_single_bond_update_config1():
    """Configuration 1: D = 2, one H1 update, 20 iterations."""
    w = inputs.workload_single_bond(seed=1, D=2)
    GA, GB, _ = O.gate_split(w['gate'], 2, 2)
    X, Y, nbr = O._cluster(True, w['A'], w['B'])
    Xo, Yo, info = O.bond_update(X, Y, nbr, GA, GB, 2, n_iter=20)
    ctx = _ctx(max_D=2)
    pairs = {b: (GA, GB) for b in O.BONDS}
    An, Bn, st = _gpu_step(ctx, w['A'], w['B'], pairs, 20, order=(ntu.BOND_H1,))
    f = fit_stat_fields(st[0, 8:], 20, 2)
    assert abs(f['delta'] - info['delta']) <= 1e-9 * info['delta']
    assert np.allclose(f['eps_hist'], info['eps'], rtol=1e-9)
    assert np.allclose(f['S'], info['S'], atol=1e-10)
    old = np.einsum('ptlbk,qTkBR->ptlbqTBR', Xo, Yo).reshape(-1)
    new = np.einsum('ptlbk,qTkBR->ptlbqTBR', An, Bn).reshape(-1)
    assert rel(new, old) < 1e-9


@pytest.mark.parametrize("D", [2, 3])
def test_trotter_step_quench(D):
    """Configuration 2 prefix: full Trotter sweeps, gauge-invariant comparison
    (errors, singular values, cluster observables)."""
    w = inputs.workload_quench(seed=2, D=D)
    GA, GB, _ = O.gate_split(w['gates'][0], 2, 2)
    pairs = {b: (GA, GB) for b in O.BONDS}
    A, B = w['A'], w['B']
    Ag, Bg = A.copy(), B.copy()
    ctx = _ctx(max_D=D)
    for step in range(3):
        A, B, infos = O.trotter_step(A, B, pairs, D, n_iter=4)
        Ag, Bg, st = _gpu_step(ctx, Ag, Bg, pairs, 4)
        for bi, b in enumerate(O.BONDS):
            f = fit_stat_fields(st[bi, 8:], 4, D)
            assert abs(f['delta'] - infos[b]['delta']) <= 1e-7 * infos[b]['delta'] + 1e-14
            assert np.allclose(f['S'], infos[b]['S'], atol=1e-8)
        eo, xo = O.observables(A, B, inputs.H_CRIT)
        eg, xg = O.observables(Ag, Bg, inputs.H_CRIT)
        assert abs(eg - eo) < 1e-9 and abs(xg - xo) < 1e-9


def test_trotter_step_thermal_prefix():
    """Configuration 3 prefix (D = 3, p = 4, real): from the beta = 0
    purification (zero modes, rank rule) through a few imaginary-time steps."""
    D = 3
    w = inputs.workload_thermal(D=D)
    GA, GB, _ = O.gate_split(w['gates'][0], 2, 2)
    pairs = {b: (GA, GB) for b in O.BONDS}
    A, B = w['A'], w['B']
    Ag, Bg = A.copy(), B.copy()
    ctx = _ctx(cplx=False, d_anc=2, max_D=D)
    for step in range(4):
        A, B, infos = O.trotter_step(A, B, pairs, D, n_iter=3)
        Ag, Bg, st = _gpu_step(ctx, Ag, Bg, pairs, 3, cplx=False)
        for bi, b in enumerate(O.BONDS):
            f = fit_stat_fields(st[bi, 8:], 3, D)
            assert f['Dn'] == infos[b]['Dn'] and f['Dk'] == infos[b]['Dk']
            assert np.allclose(f['S'], infos[b]['S'], atol=1e-9)
        eo, _ = O.observables(A, B, 2.5)
        eg, _ = O.observables(Ag, Bg, 2.5)
        assert abs(eg - eo) < 1e-10


@pytest.mark.parametrize("D, real", [(3, False), (4, False), (3, True)])
def test_svdu_trotter_steps(D, real):
    """SVDU scheme (Fig. 2 without an environment) over Trotter sweeps against
    the oracle: ranks, normalised singular values of every update, and the
    cluster observables of the evolved state (gauge-invariant)."""
    if real:
        w, hx = inputs.workload_thermal(D=D), 2.5
        ctx = _ctx(cplx=False, d_anc=2, max_D=D)
    else:
        w, hx = inputs.workload_quench(seed=2, D=D), inputs.H_CRIT
        ctx = _ctx(max_D=D)
    GA, GB, _ = O.gate_split(w['gates'][0], 2, 2)
    pairs = {b: (GA, GB) for b in O.BONDS}
    A, B = w['A'], w['B']
    Ag, Bg = A.copy(), B.copy()
    for step in range(3):
        A, B, infos = O.trotter_step(A, B, pairs, D, scheme='svdu')
        Ag, Bg, st = _gpu_step(ctx, Ag, Bg, pairs, 2, cplx=not real, scheme="svdu")
        for bi, b in enumerate(O.BONDS):
            f = fit_stat_fields(st[bi, 8:], 2, D)
            assert f['Dn'] == infos[b]['Dn'] and f['Dk'] == infos[b]['Dk']
            assert np.allclose(f['S'], infos[b]['S'], atol=1e-10)
            assert f['N'] == 0.0 and f['eps'] == 0.0 and f['iters'] == 0
        eo, xo = O.observables(A, B, hx)
        eg, xg = O.observables(Ag, Bg, hx)
        assert abs(eg - eo) < 1e-10 and abs(xg - xo) < 1e-10


def test_second_order_sweep():
    """A symmetric sweep H1 H2 V1 V2 V2 V1 H2 H1 of half-time gates (second
    order in the time step) through an 8-entry sweep order, against the
    oracle: the last update of every bond and the observables."""
    D = 2
    w = inputs.workload_quench(seed=2, D=D)
    G_half = inputs.bond_gate(inputs.ising_bond_hamiltonian(inputs.H_CRIT), 0.005)
    GA, GB, _ = O.gate_split(G_half, 2, 2)
    pairs = {b: (GA, GB) for b in O.BONDS}
    names = ('H1', 'H2', 'V1', 'V2', 'V2', 'V1', 'H2', 'H1')
    codes = tuple(O.BONDS.index(b) for b in names)
    A, B = w['A'], w['B']
    Ag, Bg = A.copy(), B.copy()
    ctx = _ctx(max_D=D)
    for step in range(2):
        A, B, infos = O.trotter_step(A, B, pairs, D, n_iter=4, order=names)
        Ag, Bg, st = _gpu_step(ctx, Ag, Bg, pairs, 4, order=codes)
        for bi in range(4, 8):          # the oracle keeps the last update of each bond
            f = fit_stat_fields(st[bi, 8:], 4, D)
            info = infos[names[bi]]
            assert abs(f['delta'] - info['delta']) <= 1e-7 * info['delta'] + 1e-14
            assert np.allclose(f['S'], info['S'], atol=1e-8)
        eo, xo = O.observables(A, B, inputs.H_CRIT)
        eg, xg = O.observables(Ag, Bg, inputs.H_CRIT)
        assert abs(eg - eo) < 1e-9 and abs(xg - xo) < 1e-9


def test_shared_side_stream_matches_own():
    """Two contexts on two streams that share one side stream (ntu_set_aux_stream)
    give the same Trotter steps, bit for bit, as with their own side streams."""
    D = 4
    w = inputs.workload_quench(seed=2, D=D)
    GA, GB, _ = O.gate_split(w['gates'][0], 2, 2)
    pairs = {b: (GA, GB) for b in O.BONDS}
    gf = to_dev(gate_factors_array(pairs)[None])
    opts = ntu.step_opts("bf16x6", n_iter=20, early_stop=True, conv_tol=1e-12)

    def run(shared):
        ctxs = [_ctx(max_D=D, max_batch=1) for _ in range(2)]
        streams = [torch.cuda.Stream() for _ in range(2)]
        aux = torch.cuda.Stream() if shared else None
        states = [(to_dev(w['A'][None]), to_dev(w['B'][None])), (to_dev(w['B'][None]), to_dev(w['A'][None]))]
        torch.cuda.synchronize()
        for c, s, (A, B) in zip(ctxs, streams, states):
            if shared:
                c.set_aux_stream(aux)
            with torch.cuda.stream(s):
                for _ in range(2):
                    ntu.ntu_trotter_step(c, A, B, gf, opts, stats=False)
        torch.cuda.synchronize()
        out = [(to_np(A), to_np(B)) for A, B in states]
        for c in ctxs:
            c.set_aux_stream(None)
            c.close()
        return out

    own, shared = run(False), run(True)
    for (a0, b0), (a1, b1) in zip(own, shared):
        assert np.array_equal(a0, a1) and np.array_equal(b0, b1)
