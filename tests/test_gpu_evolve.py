"""GPU parity of the evolution run measured with CTMRG (ntu_evolve, Sec.
III): the h_x = 0 quench against its closed form, the critical quench with
the energy stop against the oracle's run, and the argument checks."""
import numpy as np
import pytest
import torch

from oracle import ctmrg as C
from oracle import evolve as EV
from oracle import hermitian as H
from oracle import ntu as O
from paper_2107_06635_amd import inputs, ntu
from tests.gpu_util import to_dev, to_np
from tests.test_oracle_ctmrg import onsager_nn

pytestmark = pytest.mark.gpu

X = np.array([[0, 1], [1, 0]], dtype=complex)
Z = np.diag([1.0, -1.0]).astype(complex)
CODES = dict(H1=ntu.BOND_H1, H2=ntu.BOND_H2, V1=ntu.BOND_V1, V2=ntu.BOND_V2)
SECOND_ORDER = ['H1', 'H2', 'V1', 'V2', 'V2', 'V1', 'H2', 'H1']
ERR_ARG, ERR_SHAPE, ERR_DTYPE, ERR_UNSUPPORTED = -1, -2, -3, -7  # ntu_status codes


def _terms(h, d=2):
    """Operator-Schmidt terms of the bond operator (argument preparation)."""
    return np.stack([np.stack([a, b]) for a, b in C._two_site_terms(np.asarray(h, complex), d)])


def _setup(hx, dt, D, chi):
    GA, GB, _ = O.gate_split(inputs.bond_gate(inputs.ising_bond_hamiltonian(hx), dt), 2, 2)
    gf_np = np.stack([np.stack([GA, GB])] * 4)[None]
    ctx = ntu.Context(complex_=True, d=2, d_anc=1, r_g=2, max_D=D, max_batch=1)
    ctm = ntu.CTM(2, D, chi)
    A, B = inputs.polarised_x(D)
    return ctx, ctm, A, B, {b: (GA, GB) for b in O.BONDS}, to_dev(gf_np)


def _run(ctx, ctm, A, B, gf, order, hx, n_steps, every, iters, tol, cont=False, n_iter=10):
    At, Bt = to_dev(A[None]), to_dev(B[None])
    step = ntu.step_opts("f64", order=[CODES[b] for b in order], n_iter=n_iter)
    hist, e, steps = ntu.ntu_evolve(ctx, ctm, At, Bt, gf, step, n_steps, every, iters, to_dev(np.stack([X, Z])),
                                    to_dev(_terms(inputs.ising_bond_hamiltonian(hx))), energy_tol=tol,
                                    ctm_continue=cont)
    return to_np(hist), e, steps, to_np(At[0]), to_np(Bt[0])


@pytest.mark.parametrize("cont", [False, True])
def test_hx0_quench_closed_form(cont):
    """h_x = 0 from |+>, D = 2 (exact), dt = 0.05, six steps measured every
    two at chi = 16 after 30 iterations (from the identity boundary, or
    continued): <X> = cos^4(2t) on both sites, <Z> = 0, energy 0, so the
    0.01 stop does not fire."""
    dt = 0.05
    ctx, ctm, A, B, _, gf = _setup(0.0, dt, 2, 16)
    hist, e, steps, _, _ = _run(ctx, ctm, A, B, gf, O.BONDS, 0.0, 6, 2, 30, 0.01, cont=cont, n_iter=3)
    assert steps == 6 and hist.shape[0] == 4 and e.shape == (4,)
    for m in range(4):
        want = np.cos(2 * 2 * m * dt) ** 4
        assert np.abs(hist[m, :2] - want).max() < 1e-10, (m, hist[m, :2], want)
        assert np.abs(hist[m, 2:4]).max() < 1e-10
        assert abs(e[m]) < 1e-12
    ctm.close()


def test_critical_quench_energy_stop_matches_oracle():
    """The quench of Sec. III at h_x = h_c from |+>, D = 2, second-order
    sweep of half-step gates at dt = 0.05, measured every two steps at
    chi = 8 after 20 iterations, run to at most 12 steps with the paper's
    0.01 stop: the oracle's run stops after step 6 (energy moved by 1.3e-2;
    by 1.5e-3 at step 4), and so must the GPU's, with every measured value
    within 1e-8 (the values are the gauge-free comparison of the states:
    each bond update leaves its own gauge on the tensors)."""
    D, dt, hx = 2, 0.05, inputs.H_CRIT
    ctx, ctm, A, B, gd, gf = _setup(hx, dt / 2, D, 8)
    hist, e, steps, _, _ = _run(ctx, ctm, A, B, gf, SECOND_ORDER, hx, 12, 2, 20, 0.01)
    _, _, ohist, osteps = EV.evolve(A, B, gd, SECOND_ORDER, D, 12, 2, 8, 20, [X, Z],
                                      inputs.ising_bond_hamiltonian(hx), energy_tol=0.01, n_iter=10)
    assert osteps == 6 and steps == 6 and hist.shape[0] == len(ohist) == 4
    for m, (s, rec) in enumerate(ohist):
        assert np.abs(hist[m, :4] - rec['one']).max() < 1e-8, (s, hist[m, :4], rec['one'])
        assert np.abs(hist[m, 4:] - rec['bonds']).max() < 1e-8, (s, hist[m, 4:], rec['bonds'])
        assert abs(e[m] - rec['energy']) < 1e-8
    assert abs(e[-1] - e[0]) > 0.011 and abs(e[-2] - e[0]) < 0.009
    ctm.close()


def test_hermitian_purification_run_is_onsager():
    """The run on a real state: the Hermitian purification (d^2 = 4, R = 4 D)
    at h_x = 0, D = 2 (exact), dbeta = 0.05, six steps measured every two at
    chi = 16 after 40 iterations, the bond operator the anticommutator matrix
    of ZZ: <ZZ> on every bond is Onsager's value at K = beta (0.1, 0.2, 0.3),
    0 at beta = 0."""
    D, dbeta = 2, 0.05
    w = inputs.workload_hermitian_thermal(D=D, hx=0.0, hz=0.0, dbeta=dbeta)
    GA, GB, _ = H.gate_factors(w['gate'])
    ctx = ntu.Context(complex_=False, d=4, d_anc=1, r_g=4, max_D=D, max_batch=1)
    ctm = ntu.CTM(4, D, 16)
    gf = to_dev(np.stack([np.stack([GA, GB])] * 4)[None])
    ops = H.ctmrg_ops()
    At, Bt = to_dev(w['A'][None]), to_dev(w['B'][None])
    step = ntu.step_opts("f64", n_iter=3)
    hist, e, steps = ntu.ntu_evolve(ctx, ctm, At, Bt, gf, step, 6, 2, 40,
                                    to_dev(np.stack([ops['X'], ops['Z']]).astype(complex)),
                                    to_dev(_terms(ops['ZZ'], 4)), energy_tol=0.0)
    hist = to_np(hist)
    assert steps == 6 and hist.shape[0] == 4
    assert np.abs(hist[0, 4:]).max() < 1e-12
    for m in range(1, 4):
        want = onsager_nn(2 * m * dbeta)
        assert np.abs(hist[m, 4:] - want).max() < 1e-10, (m, hist[m, 4:], want)
        assert abs(e[m] - 2 * want) < 1e-9
    ctm.close()


def test_errors_before_anything_runs():
    """Refused before any step: complex64 storage, a batch of two, a history
    too short for the measurements, measure_every < 1; the state is left
    untouched."""
    ctx, ctm, A, B, _, gf = _setup(0.0, 0.05, 2, 8)
    step = ntu.step_opts("f64")
    ops1, hb = to_dev(np.stack([X, Z])), to_dev(_terms(inputs.ising_bond_hamiltonian(0.0)))
    At, Bt = to_dev(A[None]), to_dev(B[None])
    L = ntu.load()

    def call(A_, B_, hist, ev):
        n_meas, steps = ntu.ctypes.c_int(-1), ntu.ctypes.c_int(-1)
        return L.ntu_evolve(ctx.h, ctm.h, ntu._ref(A_), ntu._ref(B_), ntu._ref(gf), ntu.ctypes.byref(step),
                            ntu.ctypes.byref(ev), ntu._ref(ops1), ntu._ref(hb), ntu._ref(hist), None,
                            ntu.ctypes.byref(n_meas), ntu.ctypes.byref(steps)), n_meas.value, steps.value

    good = torch.zeros(4, 8, dtype=torch.complex128, device=At.device)
    short = torch.zeros(3, 8, dtype=torch.complex128, device=At.device)
    ev = ntu.EvolveOpts(6, 2, 3, 0, 0.01)
    st, nm, ns = call(At, Bt, short, ev)
    assert st == ERR_SHAPE and nm == 0 and ns == 0
    st, _, _ = call(At.to(torch.complex64), Bt.to(torch.complex64), good, ev)
    assert st == ERR_UNSUPPORTED
    st, _, _ = call(torch.cat([At, At]), torch.cat([Bt, Bt]), good, ev)
    assert st == ERR_SHAPE
    st, _, _ = call(At, Bt, good, ntu.EvolveOpts(6, 0, 3, 0, 0.01))
    assert st == ERR_ARG
    st, _, _ = call(At, Bt, good.to(torch.complex64), ev)
    assert st == ERR_DTYPE
    torch.cuda.synchronize()
    assert np.array_equal(to_np(At[0]), A) and np.array_equal(to_np(Bt[0]), B)
    assert float(good.abs().max()) == 0.0
    ctm.close()
