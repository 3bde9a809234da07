"""Pins of the unit-cell sweep oracle against facts fixed outside it: the
cluster of every bond against a network contracted from lattice coordinates
(no roles), the exact evolution by commuting gates on a torus (D = 2 is
exact, so the sweep must reproduce the state vector), and the two-site
sweep as the 2 x 2 cell of the checkerboard pattern for a single bond."""
import itertools

import numpy as np
import pytest

from oracle import cell as CE
from oracle import ntu as O
from paper_2107_06635_amd import inputs


def _rand_cell(rng, Lx, Ly, D, d=2):
    return {(x, y): (rng.standard_normal((d, D, D, D, D)) + 1j * rng.standard_normal((d, D, D, D, D))) / 3
            for x in range(Lx) for y in range(Ly)}


def _coord_norm(T, Lx, Ly, pos):
    """<psi|psi> of the ket network on the lattice positions ``pos`` (not
    reduced modulo the cell): a leg between two positions one step apart is
    contracted (r with l to the right, t with b upwards), every other leg is
    open; tensors taken modulo the cell.  Written from coordinates only."""
    letters = iter('abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ')
    legs = {}
    for P in pos:
        legs[P] = {k: next(letters) for k in ('p', 't', 'l', 'b', 'r')}
    for P in pos:
        x, y = P
        if (x + 1, y) in legs:
            legs[(x + 1, y)]['l'] = legs[P]['r']
        if (x, y + 1) in legs:
            legs[(x, y + 1)]['b'] = legs[P]['t']
    spec = ','.join(''.join(legs[P][k] for k in ('p', 't', 'l', 'b', 'r')) for P in pos)
    ket = np.einsum(spec, *[T[(x % Lx, y % Ly)] for x, y in pos], optimize=True)
    return float(np.vdot(ket, ket).real)


def _role_norm(T, Lx, Ly, x, y, v):
    """The same norm through the oracle's cluster roles and metric, with the
    identity gate: N = y^H g y, y = vec(R_X R_Y^T)."""
    X, Y, nbr = CE.cluster(T, Lx, Ly, x, y, v)
    GA, GB, _ = O.gate_split(np.eye(4, dtype=complex), 2, 2)
    QX, RX = O.reduce_site(X, GA, 'X', 2, O.KAPPA)
    QY, RY = O.reduce_site(Y, GB, 'Y', 2, O.KAPPA)
    g = O.metric(QX, QY, nbr)
    yv = (RX @ RY.T).reshape(-1)
    return float(np.vdot(yv, g @ yv).real)


def _positions(x, y, v):
    if not v:
        return [(x, y), (x + 1, y), (x - 1, y), (x, y + 1), (x, y - 1), (x + 1, y + 1), (x + 1, y - 1), (x + 2, y)]
    return [(x, y), (x, y + 1), (x, y - 1), (x - 1, y), (x + 1, y), (x - 1, y + 1), (x + 1, y + 1), (x, y + 2)]


@pytest.mark.parametrize("v", [0, 1])
def test_cluster_roles_against_coordinates(v):
    """Every bond of a random 3 x 3 cell at D = 2: the cluster norm through
    the roles (turned frame for vertical bonds) equals the network on the
    bond's eight lattice positions contracted by coordinates."""
    rng = np.random.default_rng(70 + v)
    Lx = Ly = 3
    T = _rand_cell(rng, Lx, Ly, 2)
    for x, y in itertools.product(range(Lx), range(Ly)):
        n_roles = _role_norm(T, Lx, Ly, x, y, v)
        n_coord = _coord_norm(T, Lx, Ly, _positions(x, y, v))
        assert abs(n_roles - n_coord) <= 1e-12 * n_coord, (x, y, v, n_roles, n_coord)


def test_planted_role_mistakes_fail():
    """TX and BX exchanged, or the vertical frame turned the wrong way, change
    the cluster norm of a random cell."""
    rng = np.random.default_rng(72)
    T = _rand_cell(rng, 3, 3, 2)
    good = _coord_norm(T, 3, 3, _positions(1, 1, 0))
    X, Y, nbr = CE.cluster(T, 3, 3, 1, 1, 0)
    L, TX, BX, TY, BY, Rn = nbr
    GA, GB, _ = O.gate_split(np.eye(4, dtype=complex), 2, 2)
    QX, RX = O.reduce_site(X, GA, 'X', 2, O.KAPPA)
    QY, RY = O.reduce_site(Y, GB, 'Y', 2, O.KAPPA)
    yv = (RX @ RY.T).reshape(-1)
    bad = float(np.vdot(yv, O.metric(QX, QY, [L, BX, TX, TY, BY, Rn]) @ yv).real)
    assert abs(bad - good) > 1e-3 * good
    good_v = _coord_norm(T, 3, 3, _positions(1, 1, 1))
    ts = [O.rot_ccw(T[s]) for s in CE.cluster_sites(3, 3, 1, 1, True)]
    QX, RX = O.reduce_site(ts[0], GA, 'X', 2, O.KAPPA)
    QY, RY = O.reduce_site(ts[1], GB, 'Y', 2, O.KAPPA)
    yv = (RX @ RY.T).reshape(-1)
    bad_v = float(np.vdot(yv, O.metric(QX, QY, ts[2:]) @ yv).real)
    assert abs(bad_v - good_v) > 1e-3 * good_v


def _torus_vector(T, Lx, Ly):
    """State vector of the Lx x Ly torus the cell tensors wire up (every leg
    contracted with its periodic neighbour), physical legs in the order of
    x + Lx y."""
    letters = iter([chr(c) for c in range(ord('A'), ord('Z') + 1)] + [chr(c) for c in range(ord('a'), ord('z') + 1)]
                   + [chr(c) for c in range(0x3b1, 0x3c9)])
    phys = {s: next(letters) for s in T}
    h = {s: next(letters) for s in T}       # leg from s to its right neighbour
    vv = {s: next(letters) for s in T}      # leg from s to its upper neighbour
    ops, spec = [], []
    for y in range(Ly):
        for x in range(Lx):
            s = (x, y)
            spec.append(phys[s] + vv[s] + h[((x - 1) % Lx, y)] + vv[(x, (y - 1) % Ly)] + h[s])
            ops.append(T[s])
    out = ''.join(phys[(x, y)] for y in range(Ly) for x in range(Lx))
    return np.einsum(','.join(spec) + '->' + out, *ops, optimize=True).reshape(-1)


def test_commuting_gates_exact_on_torus():
    """A 3 x 3 cell of distinct product states, one sweep of the diagonal
    gates exp(i t_b Z x (Z + 0.3)) (X side first, Y side second, an angle
    t_b per bond) on all 18 bonds in the library's order: the update is
    exact at D = 2, so the torus
    vector equals the exact evolution of the product state (overlap 1 to
    1e-12); a sweep with X and Y exchanged on the vertical bonds does not."""
    Lx = Ly = 3
    rng = np.random.default_rng(73)
    th = rng.uniform(0, np.pi, (Lx, Ly))
    T = {}
    for x in range(Lx):
        for y in range(Ly):
            t = np.zeros((2, 2, 2, 2, 2), complex)
            t[0, 0, 0, 0, 0], t[1, 0, 0, 0, 0] = np.cos(th[x, y]), np.sin(th[x, y])
            T[(x, y)] = t
    Z = np.diag([1.0, -1.0])
    M = Z + 0.3 * np.eye(2)
    bonds = inputs.cell_bond_order(Lx, Ly)
    tts = rng.uniform(0.05, 0.3, len(bonds))     # one angle per bond
    gates = [O.gate_split(np.diag(np.exp(1j * t * np.diag(np.kron(Z, M)))), 2, 2)[:2] for t in tts]
    Tn, _ = CE.cell_sweep(T, Lx, Ly, bonds, gates, 2, n_iter=3)
    psi = _torus_vector(Tn, Lx, Ly)
    # exact: product state times the phases of every bond (site index x + Lx y)
    n = Lx * Ly
    z = 1 - 2 * ((np.arange(2 ** n)[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1)
    amp = np.ones(2 ** n, complex)
    for k in range(n):
        x, y = k % Lx, k // Lx
        c, s = np.cos(th[x, y]), np.sin(th[x, y])
        amp *= np.where(z[:, k] == 1, c, s)
    phase = np.zeros(2 ** n)
    for (x, y, v), tt in zip(bonds, tts):
        a = x + Lx * y
        b = ((x + 1) % Lx + Lx * y) if not v else (x + Lx * ((y + 1) % Ly))
        phase += tt * z[:, a] * (z[:, b] + 0.3)
    exact = amp * np.exp(1j * phase)
    ov = abs(np.vdot(exact, psi)) / (np.linalg.norm(exact) * np.linalg.norm(psi))
    assert abs(ov - 1) < 1e-12
    # planted: vertical bonds applied with the gate's sides exchanged
    swapped = [(ga, gb) if v == 0 else (gb, ga) for (_, _, v), (ga, gb) in zip(bonds, gates)]
    Tb, _ = CE.cell_sweep(T, Lx, Ly, bonds, swapped, 2, n_iter=3)
    psib = _torus_vector(Tb, Lx, Ly)
    ovb = abs(np.vdot(exact, psib)) / (np.linalg.norm(exact) * np.linalg.norm(psib))
    assert abs(ovb - 1) > 1e-4


def test_checkerboard_cell_single_bond_is_two_site_update():
    """In the 2 x 2 cell holding the checkerboard pattern, the update of bond
    (0, 0, h) sees the cluster of the two-site sweep's H1 and returns its A',
    B' (bit for bit: the same arithmetic on the same tensors); (0, 0, v) is
    V1."""
    rng = np.random.default_rng(74)
    A, B = inputs.random_site_pair(rng, 2, 2)
    T = {(0, 0): A, (1, 1): A, (1, 0): B, (0, 1): B}
    G = inputs.bond_gate(inputs.ising_bond_hamiltonian(inputs.H_CRIT), 0.05)
    GA, GB, _ = O.gate_split(G, 2, 2)
    for v, name in ((0, 'H1'), (1, 'V1')):
        Tn, _ = CE.cell_sweep(T, 2, 2, [(0, 0, v)], [(GA, GB)], 2, n_iter=4)
        An, Bn, _ = O.trotter_step(A, B, {name: (GA, GB)}, 2, n_iter=4, order=(name,))
        assert np.array_equal(Tn[(0, 0)], An)
        assert np.array_equal(Tn[(1, 0) if v == 0 else (0, 1)], Bn)
