"""Pins of the Hermitian-purification oracle (Sec. IV, Eqs. (7)-(11), Fig. 8)
against facts fixed outside it: operator synthesis in the Pauli basis,
closed forms of the gate of Eq. (10), product states, and the exact
thermal operator on a 2 x 2 torus."""
import numpy as np
import pytest

from oracle import hermitian as H
from oracle import ntu as O
from paper_2107_06635_amd import inputs
from tests import brute

PAULI = np.stack(H.BASIS)                      # (4, 2, 2): X, Y, Z, 1


def _synth(c, n):
    """Operator sum_a c[a_1..a_n] O^a_1 x ... x O^a_n (n sites) by explicit
    Kronecker products: synthesis only, no trace formula."""
    c = np.asarray(c).reshape((4,) * n)
    M = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    for idx in np.ndindex(*c.shape):
        if c[idx] == 0:
            continue
        P = np.ones((1, 1), dtype=np.complex128)
        for a in idx:
            P = np.kron(P, PAULI[a])
        M += c[idx] * P
    return M


def test_superoperator_by_synthesis():
    """Eq. (11): for a random complex G and random real coefficients c of a
    two-site Hermitian operator rho, S c are the coefficients of G rho G^dag."""
    rng = np.random.default_rng(70)
    G = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    S = H.superoperator(G)
    assert S.dtype == np.float64
    for _ in range(3):
        c = rng.standard_normal(16)
        rho = _synth(c, 2)
        ref = G @ rho @ G.conj().T
        assert np.linalg.norm(_synth(S @ c, 2) - ref) <= 1e-13 * np.linalg.norm(ref)


def test_superoperator_zz_closed_form():
    """For G = 1 + t ZZ (Eq. 10): the identity goes to (1 + t^2) 1 + 2 t ZZ;
    X Y commutes with ZZ, so it goes to XY (1 + t ZZ)^2 = (1 + t^2) XY + 2 t YX
    (XZ = -iY, YZ = iX); X 1 anticommutes with ZZ and goes to (1 - t^2) X 1;
    and the regrouped matrix has the four singular values 4, 4t, 4t, 4t^2
    (terms 1 x 1, the two halves of t(L_ZZ + R_ZZ), and t^2 L_ZZ R_ZZ, with
    orthogonal single-site factors)."""
    t = 0.3
    Z = np.diag([1.0, -1.0])
    G = np.eye(4) + t * np.kron(Z, Z)
    S = H.superoperator(G)
    e = lambda a, b: a * 4 + b
    col = S[:, e(3, 3)]
    ref = np.zeros(16)
    ref[e(3, 3)], ref[e(2, 2)] = 1 + t * t, 2 * t
    assert np.allclose(col, ref, atol=1e-15)
    col = S[:, e(0, 1)]
    ref = np.zeros(16)
    ref[e(0, 1)], ref[e(1, 0)] = 1 + t * t, 2 * t
    assert np.allclose(col, ref, atol=1e-15)
    # X 1 anticommutes with ZZ: G (X 1) G = (X 1)(1 - t ZZ)(1 + t ZZ) = (1 - t^2) X 1
    col = S[:, e(0, 3)]
    ref = np.zeros(16)
    ref[e(0, 3)] = 1 - t * t
    assert np.allclose(col, ref, atol=1e-15)
    _, _, s = O.gate_split(S, 4, 4)
    assert np.allclose(s[:4], [4, 4 * t, 4 * t, 4 * t * t], rtol=1e-13)
    assert s[4] <= 1e-14


def test_gate_of_eq10_is_rank_two_with_fields():
    """The field factors leave the physical bond gate at operator-Schmidt rank
    two and its action at rank four; with h = 0 it is exp(dbeta ZZ / 4)."""
    G = inputs.hermitian_thermal_gate(2.9, 0.2, 0.05)
    M = G.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)
    s = np.linalg.svd(M, compute_uv=False)
    assert s[2] <= 1e-14 * s[0]
    _, _, sS = H.gate_factors(G)
    assert sS[3] > 1e-6 * sS[0] and sS[4] <= 1e-14 * sS[0]
    G0 = inputs.hermitian_thermal_gate(0.0, 0.0, 0.05)
    assert np.allclose(G0, np.diag(np.exp(0.05 / 4 * np.array([1, -1, -1, 1]))), atol=1e-15)


def _product(cA, cB, D=1):
    A = np.zeros((4, D, D, D, D))
    B = np.zeros((4, D, D, D, D))
    A[:, 0, 0, 0, 0], B[:, 0, 0, 0, 0] = cA, cB
    return A, B


def test_observables_product_state():
    """D = 1 product operators rho = (x) rho_A (x) rho_B: the estimator is
    exact, Tr(rho_s^2 O) / Tr(rho_s^2) per site by 2 x 2 matrix arithmetic,
    e = -2 <Z_A><Z_B> - h_x <X> - h_z <Z> (site means)."""
    rng = np.random.default_rng(71)
    cA, cB = rng.standard_normal(4), rng.standard_normal(4)
    A, B = _product(cA, cB, D=2)
    hx, hz = 1.7, 0.4

    def mean(c, op):
        r = _synth(c, 1)
        return float(np.real(np.trace(r @ r @ op) / np.trace(r @ r)))

    X_, Z_ = PAULI[0], PAULI[2]
    xa, xb, za, zb = mean(cA, X_), mean(cB, X_), mean(cA, Z_), mean(cB, Z_)
    e, sx, sz = H.observables(A, B, hx, hz)
    assert abs(sx - 0.5 * (xa + xb)) < 1e-14
    assert abs(sz - 0.5 * (za + zb)) < 1e-14
    assert abs(e - (-2 * za * zb - hx * 0.5 * (xa + xb) - hz * 0.5 * (za + zb))) < 1e-13


def test_observables_pin_catches_planted_mistakes(monkeypatch):
    """A commutator in place of the anticommutator breaks the product-state
    pin."""
    rng = np.random.default_rng(72)
    cA, cB = rng.standard_normal(4), rng.standard_normal(4)
    A, B = _product(cA, cB)
    good = H.observables(A, B, 1.3, 0.5)
    with monkeypatch.context() as mp:
        mp.setattr(H, 'anticommutator_matrix', lambda h: np.real(np.array(
            [[np.trace(H._pair(a // 4, a % 4) @ (h @ H._pair(b // 4, b % 4) - H._pair(b // 4, b % 4) @ h)) / 8
              for b in range(16)] for a in range(16)])))
        bad = H.observables(A, B, 1.3, 0.5)
    assert max(abs(g - b) for g, b in zip(good, bad)) > 1e-3


def _torus_operator(A, B):
    """Operator on the 2 x 2 torus represented by the Hermitian purification
    (A, B): the torus contraction of the iPEPS gives the coefficients, the
    operator follows by synthesis."""
    c = brute.torus_state(A, B, L=2)
    return _synth(c, 4)


def _embed(G, i, j, n=4):
    """Two-site gate G (site 1 = i, site 2 = j) on n spins, sites ordered as
    in the torus helper (site 0 most significant)."""
    G4 = G.reshape(2, 2, 2, 2)
    M = np.eye(2 ** n, dtype=np.complex128).reshape((2,) * (2 * n))
    # apply to the row indices of the identity
    ax = list(range(2 * n))
    out = np.einsum(G4, [n * 2, n * 2 + 1, i, j], M, ax,
                    [*(n * 2 if k == i else n * 2 + 1 if k == j else k for k in range(n)), *range(n, 2 * n)])
    return out.reshape(2 ** n, 2 ** n)


def _exact_sweep(G, L=2):
    """T = product over the bond types in the order H1, H2, V1, V2 of G on
    every bond of that type of the L x L torus: H1 = A.r - B.l, H2 = B.r -
    A.l, V1 = A.t - B.b, V2 = B.t - A.b, A on x + y even; site 1 of a
    horizontal bond is the left site, of a vertical bond the lower one."""
    n = L * L
    T = np.eye(2 ** n, dtype=np.complex128)
    for kind in ('H1', 'H2', 'V1', 'V2'):
        for y in range(L):
            for x in range(L):
                a_site = (x + y) % 2 == 0
                if kind[1] == '1' and not a_site or kind[1] == '2' and a_site:
                    continue
                i = y * L + x
                j = y * L + (x + 1) % L if kind[0] == 'H' else ((y + 1) % L) * L + x
                T = _embed(G, i, j, n) @ T
    return T


def _rel(a, b):
    a, b = a / np.trace(a), b / np.trace(b)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("steps", [1, 4])
def test_classical_exact_D2_torus(steps):
    """h_x = h_z = 0: the gates commute and rho(beta/2) = exp(beta/2 sum ZZ)
    (Eq. 8 with exact exponentials) has bond rank two, so the NTU evolution at
    D = 2 is exact: on the 2 x 2 torus the represented operator equals
    exp((beta/2) sum_b Z_i Z_j) over its eight bonds, beta = steps * dbeta."""
    dbeta = 0.2
    w = inputs.workload_hermitian_thermal(D=2, hx=0.0, hz=0.0, dbeta=dbeta)
    GA, GB, _ = H.gate_factors(w['gate'])
    pairs = {b: (GA, GB) for b in O.BONDS}
    A, B = w['A'], w['B']
    for _ in range(steps):
        A, B, infos = O.trotter_step(A, B, pairs, 2, d=4, n_iter=3)
        for info in infos.values():
            assert info['eps_final'] <= 1e-13 * info['N']
    beta = steps * dbeta
    z = np.array([1.0, -1.0])
    zs = [np.kron(np.kron(np.kron(*(z if k == i else np.ones(2) for k in range(2))),
                          (z if 2 == i else np.ones(2))), (z if 3 == i else np.ones(2))) for i in range(4)]
    # eight bonds of the 2 x 2 torus: each site's right and up bond
    energy = np.zeros(16)
    for y in range(2):
        for x in range(2):
            i = y * 2 + x
            energy += zs[i] * zs[y * 2 + (x + 1) % 2] + zs[i] * zs[((y + 1) % 2) * 2 + x]
    exact = np.diag(np.exp(0.5 * beta * energy))
    assert _rel(_torus_operator(A, B), exact) < 1e-12


def test_one_sweep_exact_D4_torus():
    """With fields, one sweep from rho = 1 adds bond rank at most four per bond
    type, so D = 4 holds it exactly: the represented operator on the 2 x 2
    torus is T T^dagger with T the product of the physical gates in the
    sweep's order (pins the rank-4 split, the order of the bond types and
    the real d^2 = 4 path).  A rank-2 split, or the gate applied as
    G^dagger rho G, fails the same comparison."""
    G = inputs.hermitian_thermal_gate(2.9, 0.7, 0.4)
    w = inputs.workload_hermitian_thermal(D=4)
    GA, GB, _ = H.gate_factors(G)
    A, B, infos = O.trotter_step(w['A'], w['B'], {b: (GA, GB) for b in O.BONDS}, 4, d=4, n_iter=3)
    for info in infos.values():
        assert info['eps_final'] <= 1e-13 * info['N']
    T = _exact_sweep(G)
    exact = T @ T.conj().T
    assert _rel(_torus_operator(A, B), exact) < 1e-12
    # planted: rank-2 split
    GA2, GB2, _ = O.gate_split(H.superoperator(G), 4, 2)
    A2, B2, _ = O.trotter_step(w['A'], w['B'], {b: (GA2, GB2) for b in O.BONDS}, 4, d=4, n_iter=3)
    assert _rel(_torus_operator(A2, B2), exact) > 1e-4
    # planted: the sweep in the reverse order of bond types
    T_rev = np.eye(16, dtype=np.complex128)
    for kind in ('V2', 'V1', 'H2', 'H1'):
        T_rev = _exact_sweep_single(G, kind) @ T_rev
    assert _rel(_torus_operator(A, B), T_rev @ T_rev.conj().T) > 1e-4


def _exact_sweep_single(G, kind, L=2):
    T = np.eye(2 ** (L * L), dtype=np.complex128)
    for y in range(L):
        for x in range(L):
            a_site = (x + y) % 2 == 0
            if kind[1] == '1' and not a_site or kind[1] == '2' and a_site:
                continue
            i = y * L + x
            j = y * L + (x + 1) % L if kind[0] == 'H' else ((y + 1) % L) * L + x
            T = _embed(G, i, j, L * L) @ T
    return T


def test_superoperator_pin_catches_planted_mistake(monkeypatch):
    """The synthesis pin fails for G^dagger P G in place of G P G^dagger."""
    rng = np.random.default_rng(73)
    G = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    c = rng.standard_normal(16)
    ref = G @ _synth(c, 2) @ G.conj().T
    Gd = G.conj().T
    bad = H.superoperator(Gd)     # computes Gd P Gd^dag = G^dag P G
    assert np.linalg.norm(_synth(bad @ c, 2) - ref) > 1e-3 * np.linalg.norm(ref)
