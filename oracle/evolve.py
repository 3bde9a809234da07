"""Plain FP64 CPU oracle of a time-evolution run with CTMRG measurements
(Sec. III: the quench from a polarised state, measured with the CTM
environment at ``chi = 4 D``, each run ended once the energy per site has
moved away from its initial value by more than a tolerance, 0.01 in the
paper).

TEST INFRASTRUCTURE ONLY, like the other oracle modules: nothing in the
product path imports it.

A run is ``n_steps`` Trotter steps (:func:`oracle.ntu.trotter_step`, the
bonds in the order given, e.g. the second-order sweep of half-step gates)
with a measurement before the first step and after every ``every`` steps:
CTMRG from the identity boundary (``ctm_iters`` iterations at ``chi``, or
continued from the previous measurement's environment) and the expectation
values of the one-site operators on A and B and of the bond operator ``hb``
on the four bonds H1, H2, V1, V2.  The energy per site is half the sum of
the four bond values (each site has two of the four bonds of the unit cell
to its right and above it), with ``hb`` carrying its share of the one-site
terms (a quarter of the field on each of its two sites).
"""
from __future__ import annotations

import numpy as np

from . import ctmrg as C
from . import ntu as O


def bond_values(env, A, B, h, d):
    """``<h>`` on the bonds H1, H2, V1, V2 (``h`` on ``(left, right)`` or
    ``(lower, upper)`` site of the bond)."""
    vals = {'H1': C.expectation_hbond(env, A, B, h, (0, 0), d),
            'H2': C.expectation_hbond(env, B, A, h, (1, 0), d)}
    renv, _ = C.rotate(env, {pos: np.zeros((1, 1, 1, 1)) for pos in C.POSITIONS})
    Ar, Br = C._rot_site(A), C._rot_site(B)
    vals['V1'] = C.expectation_hbond(renv, Ar, Br, h, (0, 0), d)
    vals['V2'] = C.expectation_hbond(renv, Br, Ar, h, (1, 0), d)
    return vals


def measure(A, B, chi, ctm_iters, ops1, hb, env=None):
    """One measurement: the environment after ``ctm_iters`` iterations (from
    ``env`` when given), the one-site values ``[<O_k>_A, <O_k>_B]`` per
    operator, the four bond values, and the energy per site."""
    d = A.shape[0]
    env = C.ctmrg(A, B, chi, ctm_iters, env=env)
    one = []
    for Ok in ops1:
        one += [C.expectation_site(env, A, Ok, (0, 0)), C.expectation_site(env, B, Ok, (1, 0))]
    bonds = bond_values(env, A, B, hb, d)
    e = 0.5 * sum(bonds[b] for b in O.BONDS).real
    return env, dict(one=np.array(one), bonds=np.array([bonds[b] for b in O.BONDS]), energy=e)


def evolve(A, B, gate_factors, order, D, n_steps, every, chi, ctm_iters, ops1, hb,
           energy_tol=0.01, ctm_continue=False, n_iter=20, d=2, measure_fn=measure):
    """The run described in the module docstring.  Returns the final ``A,
    B``, the list of measurements ``(step, record)`` and the number of steps
    taken.  A measurement whose energy differs from the first one by more
    than ``energy_tol`` (> 0) ends the run after it."""
    env, rec = measure_fn(A, B, chi, ctm_iters, ops1, hb)
    e0 = rec['energy']
    history = [(0, rec)]
    steps = 0
    for s in range(1, n_steps + 1):
        A, B, _ = O.trotter_step(A, B, gate_factors, D, d=d, n_iter=n_iter, order=order)
        steps = s
        if s % every == 0:
            env, rec = measure_fn(A, B, chi, ctm_iters, ops1, hb, env if ctm_continue else None)
            history.append((s, rec))
            if energy_tol > 0 and abs(rec['energy'] - e0) > energy_tol:
                break
    return A, B, history, steps
