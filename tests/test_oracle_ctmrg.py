"""Pins of the CTMRG oracle against facts fixed outside it: exact product
states, decoupled chains (the one-dimensional Ising chain), Onsager's
nearest-neighbour correlation of the square-lattice Ising model, the h_x = 0
quench (Sec. III), and the two thermal purifications evolved at h_x = 0
(Sec. IV), whose squares are classical Ising weights."""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import ellipk

from oracle import ctmrg as C
from oracle import hermitian as H
from oracle import ntu as O
from paper_2107_06635_amd import inputs


def onsager_nn(K):
    """<s_i s_j> of nearest neighbours at coupling K: half the energy per
    site of Onsager's solution, (1/2) coth(2K) [1 + (2/pi)(2 tanh^2(2K) - 1)
    K(k)], k = 2 sinh(2K) / cosh^2(2K)."""
    k = 2 * np.sinh(2 * K) / np.cosh(2 * K) ** 2
    return 0.5 / np.tanh(2 * K) * (1 + (2 / np.pi) * (2 * np.tanh(2 * K) ** 2 - 1) * ellipk(k * k))


def test_onsager_formula_matches_free_energy():
    """The closed form above against a numerical derivative of Onsager's
    free energy, -beta f = ln(2 cosh 2K) + (1/2pi) int_0^pi ln[(1 +
    sqrt(1 - k^2 sin^2 t)) / 2] dt per site: <s_i s_j> is half its K
    derivative (two bonds per site)."""
    def f(K):
        k = 2 * np.sinh(2 * K) / np.cosh(2 * K) ** 2
        i = quad(lambda t: np.log(0.5 * (1 + np.sqrt(1 - k * k * np.sin(t) ** 2))), 0, np.pi,
                 epsabs=1e-14, epsrel=1e-14)[0]
        return np.log(2 * np.cosh(2 * K)) + i / (2 * np.pi)
    for K in (0.3, 0.6):
        h = 1e-4
        assert abs(0.5 * (f(K + h) - f(K - h)) / (2 * h) - onsager_nn(K)) < 1e-7


def _bond_peps(M, scale=1.0):
    """Site tensor whose four legs each carry W with W W^T = M (a bond matrix
    on the spins): the state is prod_bonds M(s_i, s_j)."""
    if np.allclose(np.asarray(M).imag, 0):
        w, U = np.linalg.eigh(np.asarray(M).real)
        W = U * np.sqrt(np.maximum(w, 0))[None, :]
    else:
        U = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
        W = U * np.sqrt(np.diag(U.T @ M @ U).astype(complex))[None, :]
    assert np.allclose(W @ W.T, M)
    return scale * np.einsum('st,sl,sb,sr->stlbr', W, W, W, W).astype(complex)


def test_product_states_exact():
    """D = 1 (and padded to D = 2) products A = |+>, B = cos t|0> + sin t|1>:
    <X> and <Z> are the site means and <ZZ> = z_A z_B on every bond."""
    th = 0.3
    for D in (1, 2):
        A = np.zeros((2, D, D, D, D), complex)
        A[:, 0, 0, 0, 0] = 1 / np.sqrt(2)
        B = np.zeros((2, D, D, D, D), complex)
        B[0, 0, 0, 0, 0], B[1, 0, 0, 0, 0] = np.cos(th), np.sin(th)
        r = C.observables(A, B, 1.5, 4, 3)
        assert abs(r['sx'] - 0.5 * (1 + np.sin(2 * th))) < 1e-14
        assert abs(r['sz'] - 0.5 * np.cos(2 * th)) < 1e-14
        for v in r['zz'].values():
            assert abs(v) < 1e-14


def test_rotation_keeps_every_network():
    """The quarter turn moves corners and edges so that the 3 x 3 network
    around every site keeps its value (random environment)."""
    rng = np.random.default_rng(90)
    D2, chi = 4, 3
    env = {pos: dict(**{c: rng.standard_normal((chi, chi)) for c in ('C1', 'C2', 'C3', 'C4')},
                     **{t: rng.standard_normal((chi, chi, D2)) for t in ('T1', 'T2', 'T3', 'T4')})
           for pos in C.POSITIONS}
    sites = {pos: rng.standard_normal((D2,) * 4) for pos in C.POSITIONS}
    renv, rsites = C.rotate(env, sites)
    for (x, y) in C.POSITIONS:
        q = (y % 2, (-x) % 2)
        v0, v1 = C._site_value(env[(x, y)], sites[(x, y)]), C._site_value(renv[q], rsites[q])
        assert abs(v0 - v1) <= 1e-12 * abs(v0)


@pytest.mark.parametrize("horizontal", [True, False])
def test_decoupled_chains(horizontal):
    """Bond matrix exp(K/2 s s') on one direction and all ones on the other:
    independent Ising chains, <ss'> = tanh K along them and 0 across."""
    K = 0.4
    Wc = np.exp(0.5 * K * np.outer([1, -1], [1, -1]))
    ones = np.ones((2, 2))
    w, U = np.linalg.eigh(Wc)
    Wh = U * np.sqrt(w)[None, :]
    w, U = np.linalg.eigh(ones)
    Wv = U * np.sqrt(np.maximum(w, 0))[None, :]
    if horizontal:
        A = np.einsum('st,sl,sb,sr->stlbr', Wv, Wh, Wv, Wh).astype(complex)
    else:
        A = np.einsum('st,sl,sb,sr->stlbr', Wh, Wv, Wh, Wv).astype(complex)
    r = C.observables(A, A, 0.0, 4, 6)
    along, across = ('H1', 'H2'), ('V1', 'V2')
    if not horizontal:
        along, across = across, along
    for b in along:
        assert abs(r['zz'][b] - np.tanh(K)) < 1e-13
    for b in across:
        assert abs(r['zz'][b]) < 1e-13


@pytest.mark.parametrize("K", [0.3, 0.6])
def test_onsager_nearest_neighbour(K):
    """prod_bonds exp(K/2 s s') at D = 2: |psi|^2 is the Ising weight at
    coupling K, so <ZZ> on every bond equals Onsager's value (disordered
    K = 0.3, ordered K = 0.6, chi = 16)."""
    A = _bond_peps(np.exp(0.5 * K * np.outer([1, -1], [1, -1])))
    r = C.observables(A, A, 0.0, 16, 40)
    for v in r['zz'].values():
        assert abs(v - onsager_nn(K)) < 1e-10


def test_quench_closed_form():
    """Sec. III: the h_x = 0 evolution of |+> under exp(i t ZZ) on every bond
    has <X> = cos^4(2 t) on the square lattice (four neighbours)."""
    t = 0.2
    A = _bond_peps(np.exp(1j * t * np.outer([1, -1], [1, -1])), 1 / np.sqrt(2))
    r = C.observables(A, A, 0.0, 16, 40)
    assert abs(r['sx'] - np.cos(2 * t) ** 4) < 1e-12


def test_hermitian_purification_is_onsager():
    """The Hermitian purification evolved by the oracle's NTU at h_x = 0
    (exact at D = 2) to beta: rho(beta/2)^2 = exp(beta sum ZZ), so the CTMRG
    <ZZ> of the anticommutator matrices is Onsager's value at K = beta and
    <X> = 0."""
    dbeta, steps = 0.05, 6
    w = inputs.workload_hermitian_thermal(D=2, hx=0.0, hz=0.0, dbeta=dbeta)
    GA, GB, _ = H.gate_factors(w['gate'])
    A, B = w['A'], w['B']
    for _ in range(steps):
        A, B, _ = O.trotter_step(A, B, {b: (GA, GB) for b in O.BONDS}, 2, d=4, n_iter=3)
    r = C.observables(A, B, 0.0, 16, 40, ops=H.ctmrg_ops())
    for v in r['zz'].values():
        assert abs(v - onsager_nn(steps * dbeta)) < 1e-10
    assert abs(r['sx']) < 1e-12


def test_ancilla_purification_is_onsager():
    """The physical-plus-ancilla purification evolved by exp(-dbeta h_b) at
    h_x = 0 (exact at D = 2) represents rho = exp(-2 n dbeta H): <ZZ> is
    Onsager's value at K = 2 n dbeta, with Z acting on the physical half of
    p = (s, a)."""
    dbeta, steps = 0.05, 3
    A, B = inputs.thermal_product_purification(2)
    G = inputs.bond_gate(inputs.ising_bond_hamiltonian(0.0).real, dbeta, imaginary=True)
    GA, GB, _ = O.gate_split(G, 2, 2)
    for _ in range(steps):
        A, B, _ = O.trotter_step(A, B, {b: (GA, GB) for b in O.BONDS}, 2, n_iter=3)
    Z = np.kron(np.diag([1.0, -1.0]), np.eye(2))
    X = np.kron(np.array([[0.0, 1.0], [1.0, 0.0]]), np.eye(2))
    ZZ = np.einsum('ij,kl->ikjl', Z, Z).reshape(16, 16)
    r = C.observables(A, B, 0.0, 16, 40, ops=dict(X=X, Z=Z, ZZ=ZZ))
    for v in r['zz'].values():
        assert abs(v - onsager_nn(2 * steps * dbeta)) < 1e-10


def test_isometry_completion_closed_form():
    """Beyond the numerical rank the isometry takes unit vectors in order,
    orthogonalised against what is already there: rank 1 along
    (e_0 + e_1)/sqrt2 gives (e_0 - e_1)/sqrt2 next (e_1 then has nothing
    left and is skipped) and then e_2, e_3; a singular value just above the
    floor is kept, one at the floor is not."""
    n = 6
    u = np.zeros(n)
    u[0] = u[1] = 1 / np.sqrt(2)
    U = np.linalg.qr(np.column_stack([u, np.eye(n)[:, 2:], np.eye(n)[:, 0]]))[0] * -1
    U[:, 0] = u
    s = np.array([2.0, 1e-13, 1e-14, 0, 0, 0])
    Z = C.complete_isometry(U.astype(complex), s, 4)
    want = np.column_stack([u, (np.eye(n)[:, 0] - np.eye(n)[:, 1]) / np.sqrt(2), np.eye(n)[:, 2], np.eye(n)[:, 3]])
    assert np.abs(Z - want).max() < 1e-15
    s2 = np.array([2.0, 2.1e-12, 0, 0, 0, 0])
    Z2 = C.complete_isometry(U.astype(complex), s2, 3)
    assert np.abs(Z2[:, :2] - U[:, :2]).max() == 0
    s3 = np.array([2.0, 2e-12, 0, 0, 0, 0])
    Z3 = C.complete_isometry(U.astype(complex), s3, 3)
    assert np.abs(Z3[:, 1] - want[:, 1]).max() < 1e-15
    assert np.abs(Z3.conj().T @ Z3 - np.eye(3)).max() < 1e-15


def test_pins_catch_planted_mistakes(monkeypatch):
    """A corner turned without its transpose breaks the rotation pin (random
    square environment); the bond between the two sites of the two-site
    network summed on each side separately breaks the chain pin."""
    rng = np.random.default_rng(91)
    chi, D2 = 3, 4
    env = {pos: dict(**{c: rng.standard_normal((chi, chi)) for c in ('C1', 'C2', 'C3', 'C4')},
                     **{t: rng.standard_normal((chi, chi, D2)) for t in ('T1', 'T2', 'T3', 'T4')})
           for pos in C.POSITIONS}
    sites = {pos: rng.standard_normal((D2,) * 4) for pos in C.POSITIONS}
    nenv, nsites = C.rotate(env, sites)
    for q in nenv:
        nenv[q]['C2'] = nenv[q]['C2'].T
    v0, v1 = C._site_value(env[(0, 0)], sites[(0, 0)]), C._site_value(nenv[(0, 0)], nsites[(0, 0)])
    assert abs(v0 - v1) > 1e-3 * abs(v0)

    K = 0.4
    w, U = np.linalg.eigh(np.exp(0.5 * K * np.outer([1, -1], [1, -1])))
    Wh = U * np.sqrt(w)[None, :]
    w, U = np.linalg.eigh(np.ones((2, 2)))
    Wv = U * np.sqrt(np.maximum(w, 0))[None, :]
    A = np.einsum('st,sl,sb,sr->stlbr', Wv, Wh, Wv, Wh).astype(complex)

    def bad_hbond(eL, eR, aL, aR):
        top = C._ein('ab,aRu,RSv,Sc->bcuv', eL['C1'], eL['T1'], eR['T1'], eR['C2'])
        bot = C._ein('ab,bRd,RSe,cS->acde', eL['C4'], eL['T3'], eR['T3'], eR['C3'])
        left = C._ein('bBl,uldm->buBdm', eL['T4'], aL)
        right = C._ein('vmen,cCn->vecC', aR, eR['T2'])
        return C._ein('bcuv,buBdm,vecC,BCde->', top, left, right, bot)

    with monkeypatch.context() as mp:
        mp.setattr(C, '_hbond_value', bad_hbond)
        r = C.observables(A, A, 0.0, 4, 6)
    assert abs(r['zz']['H1'] - np.tanh(K)) > 1e-2
