"""Pins of the evolution-run oracle (Sec. III) against facts fixed outside
it: the h_x = 0 quench from |+> (every bond gate commutes with every other,
D = 2 is exact, <X> = cos^4(2t) and <ZZ> = 0), exact product-state
energies, and the stop rule of the run (the first measurement that moves
away from the initial energy by more than the tolerance ends it)."""
import numpy as np
import pytest

from oracle import evolve as EV
from oracle import ntu as O
from paper_2107_06635_amd import inputs

X = np.array([[0, 1], [1, 0]], dtype=complex)
Z = np.diag([1.0, -1.0]).astype(complex)


def _gates(hx, dt):
    GA, GB, _ = O.gate_split(inputs.bond_gate(inputs.ising_bond_hamiltonian(hx), dt), 2, 2)
    return {b: (GA, GB) for b in O.BONDS}


def test_hx0_quench_closed_form():
    """h_x = 0 from |+>: after n steps of exp(i dt ZZ) on every bond, <X> =
    cos^4(2 n dt) on both sites and the energy (h_b = -ZZ) stays 0, so the
    0.01 stop never fires; a continued environment gives the same values."""
    dt = 0.05
    A, B = inputs.polarised_x(2)
    for cont in (False, True):
        _, _, hist, steps = EV.evolve(A, B, _gates(0.0, dt), O.BONDS, 2, 6, 2, 16, 30, [X, Z],
                                      inputs.ising_bond_hamiltonian(0.0), ctm_continue=cont, n_iter=3)
        assert steps == 6 and [s for s, _ in hist] == [0, 2, 4, 6]
        for s, r in hist:
            want = np.cos(2 * s * dt) ** 4
            assert np.abs(r['one'][:2] - want).max() < 1e-10, (s, r['one'][:2], want)
            assert np.abs(r['one'][2:]).max() < 1e-10          # <Z> = 0
            assert abs(r['energy']) < 1e-12


def test_product_state_energies():
    """Energy per site = half the sum of the four bond values of
    h_b = -ZZ - (h_x/4)(XI + IX): -h_x for |+> everywhere, -2 for |0>
    everywhere (four bonds of <ZZ> = 1 shared by two sites), and
    -2 cos(2 th)^2 - h_x sin(2 th) for cos th |0> + sin th |1> everywhere
    (<Z> = cos 2 th, <X> = sin 2 th)."""
    hx = 2.5
    hb = inputs.ising_bond_hamiltonian(hx)
    A, B = inputs.polarised_x(2)
    _, rec = EV.measure(A, B, 4, 3, [X, Z], hb)
    assert abs(rec['energy'] + hx) < 1e-13
    Zs = np.zeros((2, 2, 2, 2, 2), complex)
    Zs[0, 0, 0, 0, 0] = 1.0
    _, rec = EV.measure(Zs, Zs.copy(), 4, 3, [X, Z], hb)
    assert abs(rec['energy'] + 2.0) < 1e-13
    th = 0.3
    T = np.zeros((2, 2, 2, 2, 2), complex)
    T[0, 0, 0, 0, 0], T[1, 0, 0, 0, 0] = np.cos(th), np.sin(th)
    _, rec = EV.measure(T, T.copy(), 4, 3, [X, Z], hb)
    x, z = np.sin(2 * th), np.cos(2 * th)
    assert abs(rec['energy'] - (-2 * z * z - hx * x)) < 1e-13


def test_stop_rule():
    """With prescribed energies 0, 0.004, 0.009, 0.0095, 0.012, 0.02 at the
    measurements, tolerance 0.01 ends the run after the fifth measurement
    (steps = 4 every); a rule against the previous measurement, or one that
    fires at equality, would end it elsewhere; tolerance <= 0 runs every
    step."""
    seq = [0.0, 0.004, 0.009, 0.0095, 0.012, 0.02]
    calls = []

    def fake_measure(A, B, chi, ctm_iters, ops1, hb, env=None):
        e = seq[len(calls)]
        calls.append(e)
        return None, dict(one=np.zeros(4), bonds=np.zeros(4), energy=e)

    A, B = inputs.polarised_x(2)
    _, _, hist, steps = EV.evolve(A, B, _gates(0.0, 0.01), O.BONDS, 2, 10, 2, 4, 1, [X, Z],
                                  inputs.ising_bond_hamiltonian(0.0), energy_tol=0.01, n_iter=1,
                                  measure_fn=fake_measure)
    assert steps == 8 and [s for s, _ in hist] == [0, 2, 4, 6, 8]
    calls.clear()
    seq[:] = [0.0, 0.004, 0.01, 0.0101]
    _, _, hist, steps = EV.evolve(A, B, _gates(0.0, 0.01), O.BONDS, 2, 6, 2, 4, 1, [X, Z],
                                  inputs.ising_bond_hamiltonian(0.0), energy_tol=0.01, n_iter=1,
                                  measure_fn=fake_measure)
    assert steps == 6 and len(hist) == 4          # equality does not stop, 0.0101 does
    calls.clear()
    seq[:] = [0.0, 0.5, 1.0]
    _, _, hist, steps = EV.evolve(A, B, _gates(0.0, 0.01), O.BONDS, 2, 4, 2, 4, 1, [X, Z],
                                  inputs.ising_bond_hamiltonian(0.0), energy_tol=0.0, n_iter=1,
                                  measure_fn=fake_measure)
    assert steps == 4 and len(hist) == 3


def test_pins_catch_planted_mistakes(monkeypatch):
    """A measurement that forgets the half (each bond counted for both of
    its sites) breaks the product-state energy; a step that skips the
    vertical bonds breaks the h_x = 0 closed form."""
    hb = inputs.ising_bond_hamiltonian(2.5)
    A, B = inputs.polarised_x(2)
    bonds = EV.bond_values(EV.C.ctmrg(A, B, 4, 3), A, B, hb, 2)
    assert abs(sum(bonds.values()).real + 2.5) > 1.0
    _, _, hist, _ = EV.evolve(A, B, _gates(0.0, 0.05), ['H1', 'H2'], 2, 2, 2, 16, 30, [X, Z],
                              inputs.ising_bond_hamiltonian(0.0), n_iter=3)
    assert abs(hist[-1][1]['one'][0] - np.cos(0.2) ** 4) > 1e-2
