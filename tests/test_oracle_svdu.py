"""Pins of the oracle's SVDU update (Fig. 2 without an environment).

Closed forms only: the gated pair contracted by an independent einsum, its
singular values from a library SVD of that pair, the Eckart-Young error of the
truncation, the balanced gauge, and the exactly solvable classical Ising
evolution of Sec. III.
"""
import numpy as np

from oracle import ntu as O
from paper_2107_06635_amd import inputs

RNG = np.random.default_rng


def _gated_pair(X, Y, G, d):
    """theta[(s1 a1 t l b), (s2 a2 T B R)]: the two-site gate applied to the
    pair X.r - Y.l contracted over its bond (independent of the oracle)."""
    p, D = X.shape[0], X.shape[1]
    na = p // d
    X6 = X.reshape(d, na, D, D, D, D)
    Y6 = Y.reshape(d, na, D, D, D, D)
    theta = np.einsum('satlbk,cdTkBR->satlbcdTBR', X6, Y6)
    theta = np.einsum('xyuv,uatlbvdTBR->xatlbydTBR', G.reshape(d, d, d, d), theta)
    return theta.reshape(p * D ** 3, p * D ** 3)


def _new_pair(Xn, Yn):
    p = Xn.shape[0]
    D = Xn.shape[1]
    return np.einsum('ptlbk,qTkBR->ptlbqTBR', Xn, Yn).reshape(p * D ** 3, p * D ** 3)


def _case(seed, real):
    rng = RNG(seed)
    p, d, D = 2, 2, 2
    X, Y = inputs.random_site_pair(rng, p, D, np.float64 if real else np.complex128)
    G = inputs.bond_gate(inputs.ising_bond_hamiltonian(2.5), 0.3, imaginary=real)
    GA, GB, _ = O.gate_split(G, d, 4)          # exact split of the gate
    return X, Y, G, GA, GB, d


def test_svdu_without_truncation_reproduces_gated_pair():
    """Fig. 2(b-e): with room for every singular value the SVDU update is
    exact; the new pair equals the gated pair divided by its largest
    singular value (the normalisation of Fig. 5(d))."""
    for seed, real in ((21, False), (22, True)):
        X, Y, G, GA, GB, d = _case(seed, real)
        theta = _gated_pair(X, Y, G, d)
        s = np.linalg.svd(theta, compute_uv=False)
        Dt = 8                                   # D r: every singular value of P fits
        Xn, Yn, info = O.svdu_update(X, Y, GA, GB, Dt, d=d)
        new = _new_pair(Xn, Yn)
        assert np.allclose(new, theta / s[0], atol=1e-12)
        rank = int(np.count_nonzero(s > 1e-10 * s[0]))
        assert info['Dk'] == rank
        assert np.allclose(info['S'][:rank], s[:rank] / s[0], atol=1e-12)


def test_svdu_truncation_is_eckart_young():
    """Fig. 2(c,d): keeping D singular values leaves exactly the discarded
    tail, sqrt(sum_{i >= D} s_i^2) / s_0, between the normalised gated pair
    and the new pair (the reduction's isometries preserve the norm)."""
    for seed, real in ((23, False), (24, True)):
        X, Y, G, GA, GB, d = _case(seed, real)
        theta = _gated_pair(X, Y, G, d)
        s = np.linalg.svd(theta, compute_uv=False)
        for Dt in (1, 2, 3):
            Xn, Yn, info = O.svdu_update(X, Y, GA, GB, Dt, d=d)
            err = np.linalg.norm(theta / s[0] - _new_pair(Xn, Yn))
            assert abs(err - np.sqrt(np.sum(s[Dt:] ** 2)) / s[0]) <= 1e-12


def test_svdu_balanced_gauge():
    """Fig. 5(d): both new factors carry the square roots of the normalised
    singular values, MX^H MX = MY^H MY = diag(S), with S_0 = 1."""
    X, Y, G, GA, GB, d = _case(25, False)
    _, _, info = O.svdu_update(X, Y, GA, GB, 3, d=d)
    S = info['S']
    assert abs(S[0] - 1.0) < 1e-15 and np.all(np.diff(S[:info['Dk']]) <= 0)
    for M in (info['MX'], info['MY']):
        assert np.allclose(M.conj().T @ M, np.diag(S), atol=1e-12)


def test_svdu_classical_ising_exact_D2_evolution():
    """Sec. III: for h_x = 0 the evolution from |+> is an exact D = 2 PEPS, so
    SVDU reproduces it: after n steps every bond's normalised weights are
    (1, tan(n dt))."""
    D, dt, n = 2, 0.05, 4
    A, B = inputs.plus_product_state(D)
    GA, GB, _ = O.gate_split(inputs.zz_gate(dt), 2, 2)
    gf = {b: (GA, GB) for b in O.BONDS}
    for step in range(1, n + 1):
        A, B, infos = O.trotter_step(A, B, gf, D, scheme='svdu')
        for b, info in infos.items():
            assert np.allclose(info['S'], [1.0, np.tan(step * dt)], atol=1e-12), (b, info['S'])
