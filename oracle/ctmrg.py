"""Plain FP64 CPU oracle of CTMRG expectation values (corner transfer matrix
renormalisation group, the environment the paper uses for observables: Sec.
II and the reference it cites for CTM, Sec. III, Sec. V).

TEST INFRASTRUCTURE ONLY, like ``oracle.ntu``: nothing in the product path
imports it.  numpy in float64 / complex128; einsum and SVD as single steps.

Lattice and conventions
-----------------------
* Two-site checkerboard: ``A`` on the sites ``(x, y)`` with ``x + y`` even,
  ``B`` on the others; the ``r`` leg of ``(x, y)`` joins the ``l`` leg of
  ``(x + 1, y)``, the ``t`` leg joins the ``b`` leg of ``(x, y + 1)`` (y grows
  upwards).  Bonds: H1 = A.r - B.l, H2 = B.r - A.l, V1 = A.t - B.b, V2 = B.t -
  A.b.  The unit cell of the environment is 2 x 2 (positions mod 2).
* Double layer of a site tensor ``T[s, t, l, b, r]`` with an operator ``O`` on
  the physical index: ``a[(t t'), (l l'), (b b'), (r r')] = sum_{s s'}
  conj(T[s', t', l', b', r']) O[s', s] T[s, t, l, b, r]`` (``O = 1`` for the
  norm).  The same form covers the ancilla purification (``O`` on ``(s, a)``)
  and the Hermitian purification (real ``T``, ``O`` the matrix of an
  anticommutator on the basis index).
* Environment of each position: corners ``C1`` (top left, legs r, b), ``C2``
  (top right, l, b), ``C3`` (bottom right, t, l), ``C4`` (bottom left, t, r) and
  edges ``T1`` (top, legs l, r, b), ``T2`` (right, t, b, l), ``T3`` (bottom, l,
  r, t), ``T4`` (left, t, b, r); the inner legs of the edges carry the
  double-layer bond.  Initial environment: bond dimension 1, inner legs the
  ket-bra identity (the boundary the cluster estimator closes with).

Algorithm (one iteration = four directional moves)
--------------------------------------------------
The left move absorbs column ``x`` into the left environment of column
``x + 1`` (x = 0, then 1).  For the cut between rows ``y`` and ``y + 1`` the
2 x 2 block of columns ``x, x + 1`` and rows ``y, y + 1`` gives the four
enlarged corners; the upper half ``H_u`` (top-left times top-right) and the
lower half ``H_d`` (bottom-left times bottom-right) meet on the cut's left
index ``i`` and right index ``w``; ``rho[i, j] = sum_w H_u[i, w] H_d[j, w]``,
and the isometry ``Z`` of the cut holds the ``chi`` leading left singular
vectors of ``rho`` (an orthogonal projector ``Z Z^H`` inserted on the cut).
Then ``C1 T1``, ``T4 a`` and ``C4 T3`` are contracted and their fused legs on
each cut replaced through ``Z``.  Moves in the other three directions are the
left move of the lattice rotated by quarter turns (:func:`rotate`).  Every new
tensor is divided by its largest modulus.

Readings (the paper does not specify the CTM variant): isometric projectors
from the half-system density matrix of the 2 x 2 block; identity initial
boundary; a fixed number of iterations (the corner spectra of these states hold
degenerate multiplets whose order does not settle, so observables, not
spectra, are what is compared; :func:`converged_observables` iterates until
they stop moving); directions of a cut beyond the numerical rank of ``rho``
(singular values at most ``RANK_EPS`` times the largest) fixed by Gram-Schmidt
completion with unit vectors in order (:func:`complete_isometry`), since any
orthonormal completion is a valid SVD there and the choice changes the
environment that later iterations build on.
"""
from __future__ import annotations

import numpy as np

POSITIONS = [(0, 0), (1, 0), (0, 1), (1, 1)]


def _ein(spec, *ops):
    """einsum with a contraction order chosen by numpy (pairwise products)."""
    return np.einsum(spec, *ops, optimize=True)


def double_layer(T: np.ndarray, O: np.ndarray | None = None) -> np.ndarray:
    """``a[(t t'), (l l'), (b b'), (r r')]`` of a site tensor (see the module
    docstring); ``O`` acts on the physical index, identity when None."""
    p, D = T.shape[0], T.shape[1]
    OT = T if O is None else _ein('xs,stlbr->xtlbr', O, T)
    a = _ein('xtlbr,xTLBR->tTlLbBrR', np.conj(T), OT)
    return a.reshape(D * D, D * D, D * D, D * D)


def _identity_leg(D: int) -> np.ndarray:
    return np.eye(D).reshape(D * D)


def initial_env(D: int, dtype) -> dict:
    """Bond dimension 1; inner legs closed by the ket-bra identity."""
    e = _identity_leg(D).astype(dtype)
    one = np.ones((1, 1), dtype=dtype)
    env = {}
    for pos in POSITIONS:
        env[pos] = dict(C1=one.copy(), C2=one.copy(), C3=one.copy(), C4=one.copy(),
                        T1=e.reshape(1, 1, -1).copy(), T2=e.reshape(1, 1, -1).copy(),
                        T3=e.reshape(1, 1, -1).copy(), T4=e.reshape(1, 1, -1).copy())
    return env


def _norm(t):
    m = np.abs(t).max()
    return t / m if m > 0 else t


def rotate(env: dict, sites: dict):
    """The lattice and its environment turned a quarter turn clockwise: the
    site at (x, y) goes to (y, -x) mod 2; its double layer's legs (t, l, b, r)
    become (l, b, r, t) of the old tensor; corners and edges move one place
    round (C4 -> C1, C1 -> C2 transposed, C2 -> C3, C3 -> C4 transposed, T4 ->
    T1 with its outer legs swapped, T1 -> T2, T2 -> T3 swapped, T3 -> T4)."""
    nenv, nsites = {}, {}
    for (x, y), e in env.items():
        q = (y % 2, (-x) % 2)
        nenv[q] = dict(C1=e['C4'], C2=e['C1'].T, C3=e['C2'], C4=e['C3'].T,
                       T1=e['T4'].transpose(1, 0, 2), T2=e['T1'], T3=e['T2'].transpose(1, 0, 2), T4=e['T3'])
        nsites[q] = sites[(x, y)].transpose(1, 2, 3, 0)
    return nenv, nsites


def _corners(env, sites, x, y):
    """Enlarged corners of the 2 x 2 block with columns x, x + 1 and rows y,
    y + 1 (positions mod 2), each as a matrix between its two cut indices."""
    x1, y1 = (x + 1) % 2, (y + 1) % 2
    e_tl, a_tl = env[(x, y1)], sites[(x, y1)]
    e_tr, a_tr = env[(x1, y1)], sites[(x1, y1)]
    e_br, a_br = env[(x1, y)], sites[(x1, y)]
    e_bl, a_bl = env[(x, y)], sites[(x, y)]
    # top left: right index (T1.r, a.r), down index (T4.b, a.b)
    q1 = _ein('ab,aRu,bBl,uldr->RrBd', e_tl['C1'], e_tl['T1'], e_tl['T4'], a_tl)
    # top right: left index (T1.l, a.l), down index (T2.b, a.b)
    q2 = _ein('ab,Lau,bBr,uldr->LlBd', e_tr['C2'], e_tr['T1'], e_tr['T2'], a_tr)
    # bottom right: up index (T2.t, a.t), left index (T3.l, a.l)
    q3 = _ein('ab,Tar,Lbd,uldr->TuLl', e_br['C3'], e_br['T2'], e_br['T3'], a_br)
    # bottom left: up index (T4.t, a.t), right index (T3.r, a.r)
    q4 = _ein('ab,Tal,bRd,uldr->TuRr', e_bl['C4'], e_bl['T4'], e_bl['T3'], a_bl)
    s = q1.shape
    Q1 = q1.reshape(s[0] * s[1], s[2] * s[3])
    s = q2.shape
    Q2 = q2.reshape(s[0] * s[1], s[2] * s[3])
    s = q3.shape
    Q3 = q3.reshape(s[0] * s[1], s[2] * s[3])
    s = q4.shape
    Q4 = q4.reshape(s[0] * s[1], s[2] * s[3])
    return Q1, Q2, Q3, Q4


RANK_EPS = 1e-12


def complete_isometry(U: np.ndarray, s: np.ndarray, k: int) -> np.ndarray:
    """The first ``k`` columns of ``U`` whose singular values exceed
    ``RANK_EPS * s[0]``, followed by unit vectors ``e_0, e_1, ...`` (each
    tried once, in order) orthogonalised twice against every column before
    them and kept when at least half of their length is left, until there are
    ``k`` columns."""
    n = U.shape[0]
    r = int(np.sum(s[:k] > RANK_EPS * s[0])) if s.size and s[0] > 0 else 0
    cols = [U[:, j] for j in range(r)]
    unit = 0
    while len(cols) < k:
        v = np.zeros(n, dtype=U.dtype)
        v[unit] = 1.0
        unit += 1
        for _ in range(2):
            for q in cols:
                v = v - q * np.vdot(q, v)
        nv = np.linalg.norm(v)
        if nv > 0.5:
            cols.append(v / nv)
    return np.stack(cols, axis=1)


def cut_isometry(env, sites, x, y, chi):
    """Isometry of the left cut between rows y and y + 1 at column x:
    ``chi`` leading left singular vectors of ``rho = H_u H_d^T`` (completed
    by :func:`complete_isometry` where ``rho`` has smaller rank).  Returns
    ``Z`` (rows: the fused index (edge bond, double-layer bond)) and the
    singular values of ``rho``."""
    Q1, Q2, Q3, Q4 = _corners(env, sites, x, y)
    Hu = Q1.T @ Q2          # [i = Q1 down, w = Q2 down]
    Hd = Q4 @ Q3.T          # [j = Q4 up,   w = Q3 up]
    rho = Hu @ Hd.T
    U, s, _ = np.linalg.svd(rho)
    k = min(chi, U.shape[1])
    return complete_isometry(U, s, k), s


def left_move(env, sites, chi):
    """Absorb column 0 into the left environment of column 1, then column 1
    into that of column 0 (see the module docstring)."""
    for x in (0, 1):
        x1 = (x + 1) % 2
        Z = {}
        for y in (0, 1):
            Z[y], _ = cut_isometry(env, sites, x, y, chi)   # cut between rows y and y + 1
        new = {}
        for y in (0, 1):
            e, a = env[(x, y)], sites[(x, y)]
            zu = Z[y]                 # cut above row y
            zd = Z[(y - 1) % 2]       # cut below row y
            chi_c, D2 = e['C1'].shape[1], e['T1'].shape[2]
            # C1 of (x + 1, y): C1 T1, down legs (C1.b, T1.b) through Z of the cut above
            c1 = _ein('ab,aRu->Rbu', e['C1'], e['T1']).reshape(e['T1'].shape[1], chi_c * D2)
            C1 = c1 @ np.conj(zu)
            # T4 of (x + 1, y): T4 a, up legs through Z above, down legs through Z below
            t4 = _ein('TBl,uldr->TuBdr', e['T4'], a)
            s = t4.shape
            t4 = t4.reshape(s[0] * s[1], s[2] * s[3], s[4])
            T4 = _ein('ik,ijr,jm->kmr', zu, t4, np.conj(zd))
            # C4 of (x + 1, y): C4 T3, up legs (C4.t, T3.t) through Z below
            c4 = _ein('ab,bRd->adR', e['C4'], e['T3'])
            s = c4.shape
            C4 = _ein('ik,iR->kR', zd, c4.reshape(s[0] * s[1], s[2]))
            new[y] = (_norm(C1), _norm(T4), _norm(C4))
        for y in (0, 1):
            C1, T4, C4 = new[y]
            env[(x1, y)]['C1'], env[(x1, y)]['T4'], env[(x1, y)]['C4'] = C1, T4, C4
    return env


def ctmrg(A, B, chi, n_iter, env=None):
    """``n_iter`` iterations (four directional moves each) on the environment
    of the checkerboard state (A, B), from the identity boundary or ``env``.
    Returns the environment in the original orientation.  A fixed count, not
    a convergence test: with the orthogonal projector a cut may fall inside a
    degenerate multiplet of ``rho``, and the corners then keep changing by a
    rotation inside it while every expectation value has converged (they are
    compared instead, see :func:`converged_observables`)."""
    D = A.shape[1]
    dtype = np.result_type(A, B, np.float64)
    sites = {pos: double_layer(A if (pos[0] + pos[1]) % 2 == 0 else B).astype(dtype) for pos in POSITIONS}
    if env is None:
        env = initial_env(D, dtype)
    for _ in range(n_iter):
        for _ in range(4):
            env = left_move(env, sites, chi)
            env, sites = rotate(env, sites)
    return env


# ---------------------------------------------------------------------------
# Expectation values
# ---------------------------------------------------------------------------

def _site_value(e, a):
    """The 3 x 3 network around one site."""
    top = _ein('ab,aRu,Rc->bcu', e['C1'], e['T1'], e['C2'])          # [C1.b, C2.b, u]
    bot = _ein('ab,bRd,cR->acd', e['C4'], e['T3'], e['C3'])          # [C4.t, C3.t, d]
    mid = _ein('bBl,uldr,cCr->bcuBCd', e['T4'], a, e['T2'])          # [T4.t, T2.t, u, T4.b, T2.b, d]
    return _ein('bcu,bcuBCd,BCd->', top, mid, bot)


def _hbond_value(eL, eR, aL, aR):
    """The 3 x 4 network around two horizontally adjacent sites."""
    top = _ein('ab,aRu,RSv,Sc->bcuv', eL['C1'], eL['T1'], eR['T1'], eR['C2'])
    bot = _ein('ab,bRd,RSe,cS->acde', eL['C4'], eL['T3'], eR['T3'], eR['C3'])
    left = _ein('bBl,uldm->buBdm', eL['T4'], aL)                       # [T4.t, u, T4.b, d, m]
    right = _ein('vmen,cCn->vmecC', aR, eR['T2'])                       # [v, m, e, T2.t, T2.b]
    return _ein('bcuv,buBdm,vmecC,BCde->', top, left, right, bot)


def _two_site_terms(h, d):
    """Operator-Schmidt terms of a two-site operator ``h[(s1 s2), (s1' s2')]``
    as pairs of one-site matrices."""
    H = h.reshape(d, d, d, d).transpose(0, 2, 1, 3).reshape(d * d, d * d)
    U, s, Vh = np.linalg.svd(H)
    terms = []
    for k in range(len(s)):
        if s[k] > 1e-14 * s[0]:
            terms.append((s[k] * U[:, k].reshape(d, d), Vh[k].reshape(d, d)))
    return terms


def expectation_site(env, T, O, pos):
    """<O> at position pos (ratio of the 3 x 3 network with O inserted to the
    norm network)."""
    return _site_value(env[pos], double_layer(T, O)) / _site_value(env[pos], double_layer(T))


def expectation_hbond(env, TL, TR, h, pos, d):
    """<h> on the horizontal bond from pos to its right neighbour."""
    x, y = pos
    eL, eR = env[pos], env[((x + 1) % 2, y)]
    den = _hbond_value(eL, eR, double_layer(TL), double_layer(TR))
    num = sum(_hbond_value(eL, eR, double_layer(TL, o1), double_layer(TR, o2))
              for o1, o2 in _two_site_terms(h, d))
    return num / den


def _rot_site(T):
    return T.transpose(0, 2, 3, 4, 1)


def pauli_ops():
    """X, Z and ZZ of spin 1/2."""
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Z = np.diag([1.0, -1.0]).astype(complex)
    return dict(X=X, Z=Z, ZZ=np.kron(Z, Z))


def observables_env(env, A, B, hx, hz=0.0, ops=None):
    """Energy per site and <sigma^x>, <sigma^z> (site means) from a converged
    environment: ``-1/2 sum_b <ZZ>_b - h_x <X> - h_z <Z>`` over the four bonds
    of the unit cell (two per site).  ``ops``: the one-site X, Z and the
    two-site ZZ acting on the physical index (default the Pauli matrices)."""
    if ops is None:
        ops = pauli_ops()
    d = ops['X'].shape[0]
    sx = 0.5 * (expectation_site(env, A, ops['X'], (0, 0)) + expectation_site(env, B, ops['X'], (1, 0)))
    sz = 0.5 * (expectation_site(env, A, ops['Z'], (0, 0)) + expectation_site(env, B, ops['Z'], (1, 0)))
    zz = {'H1': expectation_hbond(env, A, B, ops['ZZ'], (0, 0), d),
          'H2': expectation_hbond(env, B, A, ops['ZZ'], (1, 0), d)}
    # vertical bonds: the lattice turned a quarter turn clockwise puts the
    # upper site of a vertical bond to the right of the lower one
    renv, _ = rotate(env, {pos: np.zeros((1, 1, 1, 1)) for pos in POSITIONS})
    Ar, Br = _rot_site(A), _rot_site(B)
    # V1 = A(0,0).t - B(0,1).b: (0,0) -> (0,0), (0,1) -> (1,0)
    zz['V1'] = expectation_hbond(renv, Ar, Br, ops['ZZ'], (0, 0), d)
    # V2 = B(0,1).t - A(0,2).b: (0,1) -> (1,0), (0,0) -> (0,0)
    zz['V2'] = expectation_hbond(renv, Br, Ar, ops['ZZ'], (1, 0), d)
    e = -0.5 * sum(zz.values()) - hx * sx - hz * sz
    return dict(energy=complex(e), sx=complex(sx), sz=complex(sz), zz=zz)


def observables(A, B, hx, chi, n_iter, hz=0.0, ops=None):
    """:func:`observables_env` after ``n_iter`` CTMRG iterations."""
    env = ctmrg(A, B, chi, n_iter)
    return observables_env(env, A, B, hx, hz, ops)


def converged_observables(A, B, hx, chi, hz=0.0, ops=None, tol=1e-12, step=5, max_iter=200):
    """Iterate in chunks of ``step`` until the energy and both magnetisations
    change by less than ``tol``; returns the observables and the count."""
    env, prev, n = None, None, 0
    while n < max_iter:
        env = ctmrg(A, B, chi, step, env=env)
        n += step
        obs = observables_env(env, A, B, hx, hz, ops)
        cur = np.array([obs['energy'], obs['sx'], obs['sz']])
        if prev is not None and np.abs(cur - prev).max() < tol:
            break
        prev = cur
    obs['iterations'] = n
    return obs
