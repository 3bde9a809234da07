"""Plain FP64 CPU oracle of the manifestly Hermitian purification (Sec. IV).

TEST INFRASTRUCTURE ONLY, like ``oracle.ntu``: nothing in the product path
imports it; only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may use it.

The density-matrix half ``rho(beta/2)`` (Eq. 7) is written in the basis of
Hermitian operators of Fig. 8, ``O = (X, Y, Z, 1)``, so that it becomes an
iPEPS with real tensors and a physical index of dimension ``d^2 = 4``.  A gate
``G`` acts as ``rho -> G rho G^dagger``; on two sites that is the real matrix
of Eq. (11), which this module forms from its definition with plain matrix
products.  The NTU update itself is the one of ``oracle.ntu`` with ``d = 4``
and a rank-4 split of that matrix (its operator-Schmidt rank for the gate of
Eq. (10)).

Observables: with ``rho = sum_a c_a O^a`` (a product over sites of such
sums, contracted over the bonds), ``Tr(rho^2 h) / Tr(rho^2)`` is the quadratic
form ``c^T K_h c / c^T c`` with ``K_h`` the matrix of ``X -> (h X + X h) / 2``
in the basis, normalised by ``Tr(O^a O^b) = 2 delta_ab`` per site; the
cluster estimator of ``oracle.ntu.bond_density_matrix`` (with ``d = 4``)
supplies the two-site ``c c^T`` with the environment contracted.
"""
from __future__ import annotations

import numpy as np

from . import ntu as O

# basis of Hermitian operators for spin 1/2, in the order of Fig. 8
BASIS = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
    np.eye(2, dtype=np.complex128),
)


def _pair(a: int, b: int) -> np.ndarray:
    return np.kron(BASIS[a], BASIS[b])


def superoperator(G: np.ndarray) -> np.ndarray:
    """Eq. (11): the real 16 x 16 matrix ``S[(a' b'), (a b)]`` with
    ``G (O^a x O^b) G^dagger = sum_{a'b'} S[(a' b'), (a b)] O^a' x O^b'``.

    The coefficient of ``O^a' x O^b'`` in a two-site operator ``M`` is
    ``Tr((O^a' x O^b') M) / 4`` (the basis is orthogonal with squared norm 2
    per site).  ``G`` is any 4 x 4 matrix on ``(s1, s2)``; the result is real
    because ``G P G^dagger`` is Hermitian for Hermitian ``P``.
    """
    G = np.asarray(G, dtype=np.complex128)
    S = np.zeros((16, 16), dtype=np.complex128)
    for a in range(4):
        for b in range(4):
            M = G @ _pair(a, b) @ G.conj().T
            for ap in range(4):
                for bp in range(4):
                    S[ap * 4 + bp, a * 4 + b] = np.trace(_pair(ap, bp) @ M) / 4.0
    assert np.abs(S.imag).max() <= 1e-12 * max(1.0, np.abs(S).max())
    return S.real.copy()


def anticommutator_matrix(h: np.ndarray) -> np.ndarray:
    """``K[(a b), (a' b')] = Tr((O^a x O^b) {h, O^a' x O^b'}) / 8``: the
    two-site expectation ``Tr(rho^2 h) / Tr(rho^2)`` of the Hermitian
    purification is ``c^T K c / c^T c`` for the real coefficients ``c`` of
    ``rho`` on the bond (``h = 1`` gives the identity)."""
    h = np.asarray(h, dtype=np.complex128)
    K = np.zeros((16, 16), dtype=np.complex128)
    for a in range(4):
        for b in range(4):
            P = _pair(a, b)
            for ap in range(4):
                for bp in range(4):
                    Q = _pair(ap, bp)
                    K[a * 4 + b, ap * 4 + bp] = np.trace(P @ (h @ Q + Q @ h)) / 8.0
    assert np.abs(K.imag).max() <= 1e-12 * max(1.0, np.abs(K).max())
    return K.real.copy()


def anticommutator_matrix_1(h: np.ndarray) -> np.ndarray:
    """One-site form of :func:`anticommutator_matrix`: ``K[a, a'] =
    Tr(O^a {h, O^a'}) / 4`` (``h = 1`` gives the identity)."""
    h = np.asarray(h, dtype=np.complex128)
    K = np.array([[np.trace(BASIS[a] @ (h @ BASIS[b] + BASIS[b] @ h)) / 4.0 for b in range(4)] for a in range(4)])
    assert np.abs(K.imag).max() <= 1e-12 * max(1.0, np.abs(K).max())
    return K.real.copy()


def ctmrg_ops():
    """Operators of the CTMRG expectation values of the Hermitian
    purification on its basis index: ``X``, ``Z`` (one site) and ``ZZ`` (two
    sites) as the matrices of their anticommutators (``<O> = c^T K_O c / c^T
    c``)."""
    X_, Z_ = BASIS[0], BASIS[2]
    return dict(X=anticommutator_matrix_1(X_), Z=anticommutator_matrix_1(Z_),
                ZZ=anticommutator_matrix(np.kron(Z_, Z_)))


def gate_factors(G: np.ndarray):
    """Rank-4 split (Fig. 2(a)) of the action of ``G``: ``(GA, GB, sigma)``
    with ``GA[a', a, k]``, ``GB[b', b, k]`` real."""
    return O.gate_split(superoperator(G), 4, 4)


def observables(A, B, hx, hz=0.0):
    """Energy per site and mean ``<sigma^x>``, ``<sigma^z>`` of the thermal
    state ``rho(beta) = rho(beta/2)^2`` represented by the Hermitian
    purification ``(A, B)`` (legs ``(a, t, l, b, r)``, ``a`` over the basis),
    from the cluster density matrices of the four bonds (Eq. 12 with the bond
    terms of the inputs module)."""
    X_, Z_, I_ = BASIS[0], BASIS[2], BASIS[3]
    hb = (-np.kron(Z_, Z_) - 0.25 * hx * (np.kron(X_, I_) + np.kron(I_, X_))
          - 0.25 * hz * (np.kron(Z_, I_) + np.kron(I_, Z_)))
    Kh = anticommutator_matrix(hb)
    Kx = anticommutator_matrix(0.5 * (np.kron(X_, I_) + np.kron(I_, X_)))
    Kz = anticommutator_matrix(0.5 * (np.kron(Z_, I_) + np.kron(I_, Z_)))
    e = sx = sz = 0.0
    for bond in O.BONDS:
        vertical = bond[0] == 'V'
        a, b = (O.rot_cw(A), O.rot_cw(B)) if vertical else (A, B)
        X, Y, nbr = O._cluster(bond[1] == '1', a, b)
        rho = O.bond_density_matrix(X, Y, nbr, d=4)     # c c^T with the environment, unit trace
        e += 0.5 * float(np.trace(rho @ Kh))
        sx += 0.25 * float(np.trace(rho @ Kx))
        sz += 0.25 * float(np.trace(rho @ Kz))
    return e, sx, sz
