"""Plain FP64 CPU oracle of a Trotter sweep over a larger unit cell (Sec. II:
each update's environment is the cluster of its nearest neighbours, Fig.
4(b), whatever tensors sit there).

TEST INFRASTRUCTURE ONLY, like the other oracle modules.

The cell holds ``Lx x Ly`` distinct site tensors ``T[(x, y)]`` (legs ``(p,
t, l, b, r)``, ``y`` growing upwards) on the torus the cell repeats on.  A
sweep updates the given bonds one after another with :func:`oracle.ntu.
bond_update`, each from the current tensors.  A horizontal bond ``(x, y, 0)``
joins ``(x, y).r`` to ``(x + 1, y).l``; a vertical bond ``(x, y, 1)`` joins
``(x, y).t`` to ``(x, y + 1).b`` and is updated in the frame turned a quarter
turn clockwise (every tensor of its cluster turned by
:func:`oracle.ntu.rot_cw`, the new tensors turned back), as the vertical bonds
of the two-site sweep.
"""
from __future__ import annotations

from . import ntu as O


def cluster_sites(Lx, Ly, x, y, vertical):
    """Cell coordinates of ``[X, Y, L, TX, BX, TY, BY, Rn]`` of a bond: the
    two sites of the bond, the left neighbour of X, the sites above and below
    X and Y, and the right neighbour of Y, in the bond's frame.  In the turned
    frame of a vertical bond, right is up, up is left and left is down."""
    def at(i, j):
        return (i % Lx, j % Ly)
    if not vertical:
        return [at(x, y), at(x + 1, y), at(x - 1, y), at(x, y + 1), at(x, y - 1),
                at(x + 1, y + 1), at(x + 1, y - 1), at(x + 2, y)]
    return [at(x, y), at(x, y + 1), at(x, y - 1), at(x - 1, y), at(x + 1, y),
            at(x - 1, y + 1), at(x + 1, y + 1), at(x, y + 2)]


def cluster(T, Lx, Ly, x, y, vertical):
    """``X, Y, [L, TX, BX, TY, BY, Rn]`` of a bond in its canonical frame."""
    ts = [T[s] for s in cluster_sites(Lx, Ly, x, y, vertical)]
    if vertical:
        ts = [O.rot_cw(t) for t in ts]
    return ts[0], ts[1], ts[2:]


def cell_sweep(T, Lx, Ly, bonds, gates, D, d=2, n_iter=20, conv_tol=None, clip=True, scheme='ntu'):
    """Update ``bonds`` (triples ``(x, y, dir)``) in order with the gate
    factors ``gates[k] = (GA, GB)`` (GA on X).  Returns the new cell (a dict)
    and the per-bond diagnostics."""
    T = dict(T)
    infos = []
    for k, (x, y, v) in enumerate(bonds):
        GA, GB = gates[k]
        X, Y, nbr = cluster(T, Lx, Ly, x, y, v)
        if scheme == 'svdu':
            Xn, Yn, info = O.svdu_update(X, Y, GA, GB, D, d=d)
        else:
            Xn, Yn, info = O.bond_update(X, Y, nbr, GA, GB, D, d=d, n_iter=n_iter, conv_tol=conv_tol, clip=clip)
        if v:
            Xn, Yn = O.rot_ccw(Xn), O.rot_ccw(Yn)
        sx, sy = cluster_sites(Lx, Ly, x, y, v)[:2]
        T[sx], T[sy] = Xn, Yn
        infos.append(info)
    return T, infos
