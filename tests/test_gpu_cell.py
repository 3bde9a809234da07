"""GPU parity of the unit-cell sweep (ntu_cell_step) against the oracle's
one-bond-at-a-time sweep, through gauge-free quantities: the state vector of
the torus the cell wires up (4 x 3 cell), and every bond's norm, errors and
kept singular values (8 x 6 cell, where the library runs groups of several
independent bonds in one chain of launches)."""
import numpy as np
import pytest
import torch

from oracle import cell as CE
from oracle import ntu as O
from paper_2107_06635_amd import inputs, ntu
from tests.gpu_util import to_dev, to_np
from tests.test_oracle_cell import _torus_vector

pytestmark = pytest.mark.gpu

N_ITER = 6


def _cell(rng, Lx, Ly, D):
    T = {}
    for y in range(Ly):
        for x in range(Lx):
            A, _ = inputs.random_site_pair(rng, 2, D)
            T[(x, y)] = A
    return T


def _gates(rng, n, dt):
    """One gate per bond: the critical Ising bond gate with a field that
    varies from bond to bond (so no two updates see the same gate)."""
    out = []
    for _ in range(n):
        hx = inputs.H_CRIT * rng.uniform(0.8, 1.2)
        out.append(O.gate_split(inputs.bond_gate(inputs.ising_bond_hamiltonian(hx), dt), 2, 2)[:2])
    return out


def _gpu(T, Lx, Ly, bonds, gates, D, max_batch, precision="f64"):
    ctx = ntu.Context(complex_=True, d=2, d_anc=1, r_g=2, max_D=D, max_batch=max_batch)
    Tt = to_dev(np.stack([T[(x, y)] for y in range(Ly) for x in range(Lx)]))
    gf = to_dev(np.stack([np.stack([a, b]) for a, b in gates]))
    st, groups = ntu.ntu_cell_step(ctx, Lx, Ly, Tt, bonds, gf, ntu.step_opts(precision, n_iter=N_ITER))
    Tn = to_np(Tt)
    return {(x, y): Tn[x + Lx * y] for y in range(Ly) for x in range(Lx)}, to_np(st), groups


def test_cell_4x3_torus_state_matches_oracle():
    """4 x 3 cell of random complex tensors at D = 2, one sweep of all 24
    bonds (the library's order) with the quench gates at dt = 0.05: the
    torus state vector of the GPU's cell equals the oracle's within 1e-9
    (after the global phase and norm), and every bond's N and final error
    agree to 1e-10 relative."""
    rng = np.random.default_rng(80)
    Lx, Ly, D = 4, 3, 2
    T = _cell(rng, Lx, Ly, D)
    bonds = inputs.cell_bond_order(Lx, Ly)
    gates = _gates(rng, len(bonds), 0.05)
    Tg, st, groups = _gpu(T, Lx, Ly, bonds, gates, D, 8)
    To, infos = CE.cell_sweep(T, Lx, Ly, bonds, gates, D, n_iter=N_ITER)
    pg, po = _torus_vector(Tg, Lx, Ly), _torus_vector(To, Lx, Ly)
    pg, po = pg / np.linalg.norm(pg), po / np.linalg.norm(po)
    ph = np.vdot(pg, po)
    ph /= abs(ph)
    assert np.linalg.norm(pg * ph - po) < 1e-9
    for k, info in enumerate(infos):
        assert abs(st[k, 8] - info['N']) <= 1e-10 * info['N'], k
        assert abs(st[k, 10] - info['eps_final']) <= 1e-10 * info['N'] + 1e-14, k
    assert 1 <= groups <= len(bonds)


@pytest.mark.parametrize("precision, tol", [("f64", 1e-9), ("bf16x6", 1e-5)])
def test_cell_8x6_groups_match_oracle(precision, tol):
    """8 x 6 cell at D = 3 (96 bonds): the library's order forms launch
    groups of several independent bonds (fewer groups than bonds), and every
    bond's N, final error and normalised singular values agree with the
    oracle's sequential sweep (FP64 at 1e-9; BF16x6 environment at 1e-5)."""
    rng = np.random.default_rng(81)
    Lx, Ly, D = 8, 6, 3
    T = _cell(rng, Lx, Ly, D)
    bonds = inputs.cell_bond_order(Lx, Ly)
    gates = _gates(rng, len(bonds), 0.05)
    _, st, groups = _gpu(T, Lx, Ly, bonds, gates, D, 48, precision)
    _, infos = CE.cell_sweep(T, Lx, Ly, bonds, gates, D, n_iter=N_ITER)
    assert groups < len(bonds) // 2
    s0 = 8 + 16 + 4 * N_ITER
    for k, info in enumerate(infos):
        assert abs(st[k, 8] - info['N']) <= tol * info['N'], k
        assert abs(st[k, 10] - info['eps_final']) <= tol * info['N'] + 1e-14, k
        assert np.abs(st[k, s0:s0 + D] - info['S']).max() <= tol, (k, st[k, s0:s0 + D], info['S'])


def test_cell_svdu_sweep_matches_oracle():
    """The SVDU scheme through the cell sweep (no environment): a 4 x 3 cell
    at D = 2 after one sweep of all bonds, by the torus state vector (1e-9
    after phase and norm)."""
    rng = np.random.default_rng(83)
    Lx, Ly, D = 4, 3, 2
    T = _cell(rng, Lx, Ly, D)
    bonds = inputs.cell_bond_order(Lx, Ly)
    gates = _gates(rng, len(bonds), 0.05)
    ctx = ntu.Context(complex_=True, d=2, d_anc=1, r_g=2, max_D=D, max_batch=8)
    Tt = to_dev(np.stack([T[(x, y)] for y in range(Ly) for x in range(Lx)]))
    gf = to_dev(np.stack([np.stack([a, b]) for a, b in gates]))
    ntu.ntu_cell_step(ctx, Lx, Ly, Tt, bonds, gf, ntu.step_opts("f64", scheme="svdu"))
    Tn = to_np(Tt)
    Tg = {(x, y): Tn[x + Lx * y] for y in range(Ly) for x in range(Lx)}
    To, _ = CE.cell_sweep(T, Lx, Ly, bonds, gates, D, scheme='svdu')
    pg, po = _torus_vector(Tg, Lx, Ly), _torus_vector(To, Lx, Ly)
    pg, po = pg / np.linalg.norm(pg), po / np.linalg.norm(po)
    ph = np.vdot(pg, po)
    ph /= abs(ph)
    assert np.linalg.norm(pg * ph - po) < 1e-9


def test_cell_errors_before_anything_runs():
    """Refused before any launch, the cell untouched: a cell of one column,
    a bond outside the cell, an unknown direction, a short work array, gate
    factors of the wrong count."""
    rng = np.random.default_rng(82)
    Lx, Ly, D = 3, 3, 2
    T = _cell(rng, Lx, Ly, D)
    ctx = ntu.Context(complex_=True, d=2, d_anc=1, r_g=2, max_D=D, max_batch=4)
    Tt = to_dev(np.stack([T[(x, y)] for y in range(Ly) for x in range(Lx)]))
    T0 = to_np(Tt).copy()
    bonds = [(0, 0, 0), (1, 1, 1)]
    gf = to_dev(np.stack([np.stack(g) for g in _gates(rng, 2, 0.05)]))
    L = ntu.load()
    opts = ntu.step_opts("f64")

    def call(Lx_, Ly_, bl, g, work):
        flat = (ntu.ctypes.c_int * (3 * len(bl)))(*[v for b in bl for v in b])
        return L.ntu_cell_step(ctx.h, Lx_, Ly_, ntu._ref(Tt), len(bl), flat, ntu._ref(g), ntu.ctypes.byref(opts),
                               ntu._ref(work), None, None)

    nsite = Tt[0].numel()
    good = torch.empty(8 * 4 * nsite, dtype=Tt.dtype, device=Tt.device)
    assert call(1, 9, bonds, gf, good) == -2
    assert call(Lx, Ly, [(3, 0, 0), (1, 1, 1)], gf, good) == -1
    assert call(Lx, Ly, [(0, 0, 2), (1, 1, 1)], gf, good) == -1
    assert call(Lx, Ly, bonds, gf, good[:8 * 4 * nsite - 1]) == -6
    assert call(Lx, Ly, bonds, gf[:1], good) == -2
    assert np.array_equal(to_np(Tt), T0)
    assert call(Lx, Ly, bonds, gf, good) == 0
    assert not np.array_equal(to_np(Tt), T0)
