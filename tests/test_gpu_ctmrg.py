"""GPU parity of the CTMRG expectation values (ntu_ctm_*) against the oracle
and against the closed forms its pins rest on (Onsager's nearest-neighbour
correlation, the h_x = 0 quench value), for pure states, an NTU-evolved
state and the Hermitian purification."""
import numpy as np
import pytest
import torch

from oracle import ctmrg as C
from oracle import hermitian as H
from oracle import ntu as O
from paper_2107_06635_amd import inputs, ntu
from tests.gpu_util import to_dev, to_np
from tests.test_oracle_ctmrg import _bond_peps, onsager_nn

pytestmark = pytest.mark.gpu


def _terms(h, d):
    """Operator-Schmidt terms of a two-site operator (argument preparation:
    the library takes the product terms)."""
    return np.stack([np.stack([a, b]) for a, b in C._two_site_terms(np.asarray(h, complex), d)])


def _gpu(A, B, chi, n_iter, ops):
    p, D = A.shape[0], A.shape[1]
    ctm = ntu.CTM(p, D, chi)
    At, Bt = to_dev(A), to_dev(B)
    ctm.run(At, Bt, n_iter)
    ops1 = to_dev(np.stack([ops['X'], ops['Z']]).astype(complex))
    ops2 = to_dev(_terms(ops['ZZ'], p))
    out = to_np(ctm.expect(At, Bt, ops1, ops2))
    ctm.close()
    return dict(xA=out[0], xB=out[1], zA=out[2], zB=out[3], zz=dict(zip(O.BONDS, out[4:8])))


def _oracle(A, B, chi, n_iter, ops):
    env = C.ctmrg(A, B, chi, n_iter)
    r = C.observables_env(env, A, B, 0.0, 0.0, ops)
    xA = C.expectation_site(env, A, ops['X'], (0, 0))
    xB = C.expectation_site(env, B, ops['X'], (1, 0))
    return dict(xA=xA, xB=xB, zz=r['zz'])


def _compare(g, o, tol):
    assert abs(g['xA'] - o['xA']) < tol and abs(g['xB'] - o['xB']) < tol, (g, o)
    for b in O.BONDS:
        assert abs(g['zz'][b] - o['zz'][b]) < tol, (b, g['zz'][b], o['zz'][b])


def test_product_states():
    """D = 2 padded products (A != B): exact values after a few iterations."""
    th = 0.3
    A = np.zeros((2, 2, 2, 2, 2), complex)
    A[:, 0, 0, 0, 0] = 1 / np.sqrt(2)
    B = np.zeros((2, 2, 2, 2, 2), complex)
    B[0, 0, 0, 0, 0], B[1, 0, 0, 0, 0] = np.cos(th), np.sin(th)
    g = _gpu(A, B, 4, 3, C.pauli_ops())
    assert abs(g['xA'] - 1) < 1e-13 and abs(g['xB'] - np.sin(2 * th)) < 1e-13
    assert abs(g['zB'] - np.cos(2 * th)) < 1e-13
    for v in g['zz'].values():
        assert abs(v) < 1e-13


@pytest.mark.parametrize("K", [0.3, 0.6])
def test_onsager(K):
    """D = 2 Ising PEPS, chi = 16: <ZZ> on all four bonds equals Onsager's
    nearest-neighbour correlation and the oracle's values."""
    A = _bond_peps(np.exp(0.5 * K * np.outer([1, -1], [1, -1])))
    g = _gpu(A, A, 16, 40, C.pauli_ops())
    for v in g['zz'].values():
        assert abs(v - onsager_nn(K)) < 1e-10
    _compare(g, _oracle(A, A, 16, 40, C.pauli_ops()), 1e-10)


@pytest.mark.parametrize("chi", [80, 150])
def test_onsager_large_cut(chi):
    """The Ising PEPS at K = 0.3 with chi = 80 and 150: cuts of n = chi D^2
    = 320 and 600 (the multi-workgroup SVD with its column blocks staged in
    LDS, and read from global memory beyond n = 576; the cuts beyond rank
    chi get the completion rule) still give Onsager's value on every bond to
    1e-10."""
    K = 0.3
    A = _bond_peps(np.exp(0.5 * K * np.outer([1, -1], [1, -1])))
    Z = np.diag([1.0, -1.0]).astype(complex)
    g = _gpu(A, A, chi, 40, dict(X=np.eye(2, dtype=complex), Z=Z, ZZ=np.kron(Z, Z)))
    for b in O.BONDS:
        assert abs(g['zz'][b] - onsager_nn(K)) < 1e-10, (b, g['zz'][b])


def test_quench_closed_form():
    t = 0.2
    A = _bond_peps(np.exp(1j * t * np.outer([1, -1], [1, -1])), 1 / np.sqrt(2))
    g = _gpu(A, A, 16, 40, C.pauli_ops())
    assert abs(g['xA'] - np.cos(2 * t) ** 4) < 1e-11 and abs(g['xB'] - np.cos(2 * t) ** 4) < 1e-11


@pytest.mark.parametrize("D, steps, chi", [(3, 4, 12), (2, 6, 16), (2, 6, 8), (3, 4, 16), (4, 3, 16)])
def test_ntu_quench_state(D, steps, chi):
    """A state of the configuration-2 quench (h_x = 3.04438, dt = 0.05,
    random start, A != B) after some NTU sweeps of the oracle, at chi = 4 D
    (the paper's choice for expectation values) and above: every one-site
    and bond value against the oracle's CTMRG with the same iteration count
    (40: converged to about 1e-11; at 15 iterations the values still move
    by 1e-5 per five iterations and the two sides' unconverged environments
    differ by 2e-8).  At D = 2, chi = 8 the first cuts have rank 4 below
    chi: the directions beyond the rank follow the completion rule both
    sides share (with an arbitrary completion the two sides drift apart by
    about 3e-6)."""
    w = inputs.workload_quench(seed=2, D=D)
    G = inputs.bond_gate(inputs.ising_bond_hamiltonian(inputs.H_CRIT), 0.05)
    GA, GB, _ = O.gate_split(G, 2, 2)
    A, B = w['A'], w['B']
    for _ in range(steps):
        A, B, _ = O.trotter_step(A, B, {b: (GA, GB) for b in O.BONDS}, D, n_iter=5)
    A, B = A / np.abs(A).max(), B / np.abs(B).max()
    g = _gpu(A, B, chi, 40, C.pauli_ops())
    o = _oracle(A, B, chi, 40, C.pauli_ops())
    _compare(g, o, 1e-9)


def test_hermitian_purification():
    """The Hermitian purification at h_x = 0 (exact at D = 2, beta = 0.3):
    <ZZ> of the anticommutator matrices equals Onsager's value at K = beta;
    with fields (D = 3, h_x = 2.9) the values equal the oracle's."""
    dbeta = 0.05
    for D, hx, steps in ((2, 0.0, 6), (3, 2.9, 4)):
        w = inputs.workload_hermitian_thermal(D=D, hx=hx, hz=5e-4 if hx else 0.0, dbeta=dbeta)
        GA, GB, _ = H.gate_factors(w['gate'])
        A, B = w['A'], w['B']
        for _ in range(steps):
            A, B, _ = O.trotter_step(A, B, {b: (GA, GB) for b in O.BONDS}, D, d=4, n_iter=3)
        ops = H.ctmrg_ops()
        g = _gpu(A, B, 4 * D, 40, ops)
        if hx == 0.0:
            for v in g['zz'].values():
                assert abs(v - onsager_nn(steps * dbeta)) < 1e-10
        _compare(g, _oracle(A, B, 4 * D, 40, ops), 1e-9)


def test_errors():
    """Sizes beyond the cut SVD's limit and an evaluation without an
    environment are refused with their codes."""
    with pytest.raises(RuntimeError, match="status -2"):
        ntu.CTM(2, 8, 20)            # chi D^2 = 1280 > 1024
    ctm = ntu.CTM(2, 2, 4)
    A = to_dev(np.zeros((2, 2, 2, 2, 2), complex))
    ops1 = to_dev(np.zeros((1, 2, 2), complex))
    ops2 = to_dev(np.zeros((1, 2, 2, 2), complex))
    with pytest.raises(RuntimeError, match="status -1"):
        ctm.expect(A, A, ops1, ops2)
    with pytest.raises(RuntimeError, match="status -2"):
        ctm.run(to_dev(np.zeros((2, 3, 3, 3, 3), complex)), A, 1)
