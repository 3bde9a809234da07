"""Seeded synthetic inputs for the NTU bond update.

This module only *draws and defines inputs*: random iPEPS site tensors, the
Ising bond Hamiltonian and its Trotter gate, the beta=0 purification and the
workload descriptions.  It holds none of the arithmetic of the update itself
(no QR, no metric, no fit), so the CPU oracle and the GPU path can both be fed
from it without sharing any of the method's code.

Conventions
-----------
* A site tensor has legs ``(p, t, l, b, r)``: physical block ``p`` (``p = d`` or
  ``p = d * d_anc`` with the ancilla folded in as ``p = s * d_anc + a``), then the
  four virtual legs top, left, bottom, right, each of dimension ``D``.
* A two-site gate is a ``(d*d, d*d)`` matrix with rows ``(s1', s2')`` and
  columns ``(s1, s2)``; site 1 is the left (or lower) site of the bond.
* Transverse-field Ising model (Sec. III, Eq. 6, with the longitudinal bias of
  Sec. V, Eq. 12) written as a sum of bond terms on the square lattice: every
  site has four bonds, so each bond carries a quarter of each on-site field,
  ``h_b = -Z Z - (h_x / 4)(X I + I X) - (h_z / 4)(Z I + I Z)``.
"""
from __future__ import annotations

import numpy as np

PAULI_I = np.eye(2, dtype=np.complex128)
PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)

# critical transverse field of the 2D quantum Ising model quoted in Sec. III
H_CRIT = 3.04438


def ising_bond_hamiltonian(hx: float, hz: float = 0.0) -> np.ndarray:
    """Bond term ``h_b`` of Eqs. (6)/(12) as a 4x4 matrix, rows/cols ``(s1, s2)``."""
    zz = np.kron(PAULI_Z, PAULI_Z)
    xi = np.kron(PAULI_X, PAULI_I) + np.kron(PAULI_I, PAULI_X)
    zi = np.kron(PAULI_Z, PAULI_I) + np.kron(PAULI_I, PAULI_Z)
    return -zz - 0.25 * hx * xi - 0.25 * hz * zi


def bond_gate(h: np.ndarray, dt: float, imaginary: bool = False) -> np.ndarray:
    """Trotter gate ``exp(-i dt h)`` (real time) or ``exp(-dt h)`` (imaginary time).

    ``h`` is Hermitian and 4x4; the exponential is taken through its spectral
    decomposition.  For imaginary time with a real ``h`` the result is real.
    """
    w, v = np.linalg.eigh(h)
    if imaginary:
        gate = (v * np.exp(-dt * w)) @ v.conj().T
        if np.isrealobj(h) or np.allclose(h.imag, 0.0):
            gate = gate.real
        return gate
    return (v * np.exp(-1j * dt * w)) @ v.conj().T


def zz_gate(dt: float) -> np.ndarray:
    """``exp(+i dt Z Z)``: the real-time gate of the classical (h_x = 0) Ising bond."""
    return np.diag(np.exp(1j * dt * np.diag(np.kron(PAULI_Z, PAULI_Z)).real))


def hermitian_thermal_gate(hx: float, hz: float, dbeta: float) -> np.ndarray:
    """Two-site gate of the manifestly Hermitian purification (Sec. IV).

    The non-trivial bond gate of Eq. (10), ``exp(dbeta Z Z / 4)`` (equal to
    ``1 + tanh(dbeta / 4) Z Z`` up to a scale), between the on-site field
    gates ``s = exp((dbeta / 32)(h_x X + h_z Z))`` on both sites, before and
    after: ``(s x s) exp(dbeta Z Z / 4) (s x s)``.  Every site has four bonds,
    so one sweep over the four bond types gives each site ``s^8 =
    exp(dbeta (h_x X + h_z Z) / 4)``, i.e. ``exp(-dbeta H / 4)`` of Eq. (9)
    to first order in ``dbeta``.  The local factors leave the operator-Schmidt
    rank of the bond gate at two (four for its action ``G rho G^dagger``).
    Real, 4 x 4, rows ``(s1', s2')``, columns ``(s1, s2)``.
    """
    w, v = np.linalg.eigh((hx * PAULI_X + hz * PAULI_Z).real)
    s = (v * np.exp(dbeta / 32.0 * w)) @ v.T
    ss = np.kron(s, s)
    zz = np.diag(np.exp(0.25 * dbeta * np.diag(np.kron(PAULI_Z, PAULI_Z)).real))
    return ss @ zz @ ss


def hermitian_identity(D: int) -> tuple[np.ndarray, np.ndarray]:
    """beta = 0 state of the Hermitian purification: ``rho(0/2) = 1`` on every
    site, i.e. coefficient 1 on the fourth basis operator (the identity, in
    the basis ``O = (X, Y, Z, 1)`` of Fig. 8) and bond dimension 1, zero-padded
    to ``D``.  Real, physical dimension ``d^2 = 4``."""
    A = np.zeros((4, D, D, D, D))
    A[3, 0, 0, 0, 0] = 1.0
    return A, A.copy()


def random_site_pair(rng: np.random.Generator, p: int, D: int,
                     dtype=np.complex128) -> tuple[np.ndarray, np.ndarray]:
    """Draw ``A`` then ``B``: i.i.d. ``x + i y`` with ``x, y ~ N(0, 1)``.

    For each tensor the real block is drawn first, then the imaginary block;
    each tensor is scaled to max-abs 1.  ``dtype`` is the storage type (the
    values are drawn in double precision and then cast).
    """
    shape = (p, D, D, D, D)
    out = []
    for _ in range(2):
        re = rng.standard_normal(shape)
        if np.issubdtype(np.dtype(dtype), np.complexfloating):
            im = rng.standard_normal(shape)
            t = re + 1j * im
        else:
            t = re
        t = t / np.max(np.abs(t))
        out.append(t.astype(dtype))
    return out[0], out[1]


def random_neighbours(rng: np.random.Generator, p: int, D: int,
                      dtype=np.complex128) -> list[np.ndarray]:
    """Six independent neighbour tensors ``[L, TX, BX, TY, BY, Rn]``."""
    out = []
    for _ in range(3):
        a, b = random_site_pair(rng, p, D, dtype)
        out += [a, b]
    return out


def thermal_product_purification(D: int, d: int = 2, d_anc: int = 2) -> tuple[np.ndarray, np.ndarray]:
    """beta = 0 purification: ``A[(s, a), 0, 0, 0, 0] = delta_{s a}``, all other
    virtual indices zero-padded to ``D``.  Real, ``p = d * d_anc``."""
    A = np.zeros((d * d_anc, D, D, D, D))
    for s in range(d):
        A[s * d_anc + s, 0, 0, 0, 0] = 1.0
    return A, A.copy()


def plus_product_state(D: int) -> tuple[np.ndarray, np.ndarray]:
    """``|+>`` on every site, bond dimension 1 zero-padded to ``D`` (complex)."""
    A = np.zeros((2, D, D, D, D), dtype=np.complex128)
    A[:, 0, 0, 0, 0] = 1.0 / np.sqrt(2.0)
    return A, A.copy()


# --------------------------------------------------------------------------
# Workloads.  Each returns plain arrays; sizes follow the benchmark configs.
# --------------------------------------------------------------------------

def polarised_x(D: int, dtype=np.complex128):
    """The fully polarised state along x of the quench (Sec. III): A = B =
    |+> on every site, bond dimension 1 padded with zeros to D; legs (p, t,
    l, b, r)."""
    A = np.zeros((2, D, D, D, D), dtype=dtype)
    A[:, 0, 0, 0, 0] = 1.0 / np.sqrt(2.0)
    return A, A.copy()


def cell_bond_order(Lx: int, Ly: int):
    """A sweep order of the 2 Lx Ly bonds of an Lx x Ly cell (triples (x, y,
    dir)) in which bonds that can run side by side are adjacent: horizontal
    bonds by the classes (x mod 4, y mod 3), then vertical bonds by (y mod 4,
    x mod 3).  Within a class, two horizontal bonds are at least four columns
    or three rows apart, so neither touches the other's nearest-neighbour
    cluster when the cell is a multiple of 4 x 3 (the library checks this
    itself and splits where it does not hold)."""
    order = []
    for cx in range(4):
        for cy in range(3):
            order += [(x, y, 0) for y in range(Ly) for x in range(Lx) if x % 4 == cx and y % 3 == cy]
    for cy in range(4):
        for cx in range(3):
            order += [(x, y, 1) for x in range(Lx) for y in range(Ly) if y % 4 == cy and x % 3 == cx]
    return order


def workload_single_bond(seed: int = 1, D: int = 2, hx: float = H_CRIT, dt: float = 0.01):
    """One complex bond update of a random state (configuration 1 at ``D = 2``)."""
    rng = np.random.default_rng(seed)
    A, B = random_site_pair(rng, 2, D)
    gate = bond_gate(ising_bond_hamiltonian(hx), dt)
    return dict(A=A, B=B, gate=gate, D=D, p=2, n_iter=20)


def workload_quench(seed: int = 2, D: int = 4, hx: float = H_CRIT, dt: float = 0.01):
    """Real-time quench of a random complex state (configuration 2)."""
    rng = np.random.default_rng(seed)
    A, B = random_site_pair(rng, 2, D)
    gate = bond_gate(ising_bond_hamiltonian(hx), dt)
    return dict(A=A, B=B, gates=[gate] * 4, D=D, p=2)


def workload_thermal(D: int = 8, hx: float = 2.5, hz: float = 0.0, dbeta: float = 0.005):
    """Imaginary-time evolution of the beta = 0 purification (configuration 3).

    The gate ``exp(-dbeta h_b)`` acts on the physical index only; the ancilla
    is a spectator.  Real arithmetic throughout.
    """
    A, B = thermal_product_purification(D)
    gate = bond_gate(ising_bond_hamiltonian(hx, hz).real, dbeta, imaginary=True)
    return dict(A=A, B=B, gates=[gate] * 4, D=D, p=4)


def workload_hermitian_thermal(D: int = 5, hx: float = 2.9, hz: float = 5e-4, dbeta: float = 0.0025):
    """Imaginary-time evolution of the manifestly Hermitian purification
    (Sec. IV; the field values and the step of Sec. V).  ``gate`` is the
    two-site operator ``G`` of :func:`hermitian_thermal_gate`; the update
    itself uses its action on the basis pairs (Eq. 11), which the library and
    the oracle each form from ``G``.  Real arithmetic, ``p = d^2 = 4``, gate
    rank 4 (``R = 4 D``)."""
    A, B = hermitian_identity(D)
    return dict(A=A, B=B, gate=hermitian_thermal_gate(hx, hz, dbeta), D=D, p=4, hx=hx, hz=hz, dbeta=dbeta)


def workload_batched(seed: int = 4, n: int = 256, D_lo: int = 3, D_hi: int = 8,
                     g_lo: float = 2.5, g_hi: float = 3.5, dt: float = 0.01):
    """Independent horizontal-bond updates of uneven ``D`` (configuration 4).

    Draw order: all ``D_i``, then all ``g_i``, then ``A_i, B_i`` for i = 0..n-1.
    Site tensors are stored as complex64.
    """
    rng = np.random.default_rng(seed)
    Ds = rng.integers(D_lo, D_hi + 1, size=n)
    gs = rng.uniform(g_lo, g_hi, size=n)
    items = []
    for i in range(n):
        A, B = random_site_pair(rng, 2, int(Ds[i]), np.complex64)
        gate = bond_gate(ising_bond_hamiltonian(float(gs[i])), dt)
        items.append(dict(A=A, B=B, gate=gate, D=int(Ds[i]), p=2, g=float(gs[i])))
    return items


def workload_large(seed: int = 5, D: int = 10, hx: float = H_CRIT, dt: float = 0.005):
    """Large single-state quench (configuration 5)."""
    rng = np.random.default_rng(seed)
    A, B = random_site_pair(rng, 2, D)
    gate = bond_gate(ising_bond_hamiltonian(hx), dt)
    return dict(A=A, B=B, gates=[gate] * 4, D=D, p=2)
