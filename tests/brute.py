"""Brute-force metric from the explicit cluster vector (tiny D only).

Independent of the oracle's double-layer contraction: the ket network of the
eight-site cluster (Fig. 4(b)) is built with every physical leg and every
external virtual leg open, and the metric is its Gram matrix
``g[(a' b'), (a b)] = sum_e conj(Phi_{a'b'}(e)) Phi_{ab}(e)``.
"""
from __future__ import annotations

import numpy as np


def cluster_vector_chunks(QX, QY, nbr):
    """Yield ``Phi`` as ``(R*R, n_e)`` matrices, one chunk per physical index of
    ``L`` (rows ``(a, b)``; every chunk a disjoint slice of ``e``)."""
    L, TX, BX, TY, BY, Rn = nbr
    R = QX.shape[-1]
    for pl in range(L.shape[0]):
        Lp = L[pl]
        # QX legs (p t l b a): t-TX.b, l-L.r, b-BX.t ; QY legs (p t b r b): t-TY.b, b-BY.t, r-Rn.l
        phi = np.einsum(
            'xtlba,TUVl,ABCtv,DbEFw,GHvIJ,KMwLN,yIMrc,OPrQS->acxyABCDEFGHJKLNOPQSTUV',
            QX, Lp, TX, BX, TY, BY, QY, Rn, optimize=True)
        # a/c: bond pair; x/y: X/Y physical; t,l,b: X.t-TX.b, X.l-L.r, X.b-BX.t;
        # I,M,r: Y.t-TY.b, Y.b-BY.t, Y.r-Rn.l; v,w: TX.r-TY.l, BX.r-BY.l;
        # every other letter is an open physical or external leg
        yield phi.reshape(R * R, -1)


def brute_metric(QX, QY, nbr):
    R = QX.shape[-1]
    g = np.zeros((R * R, R * R), dtype=np.result_type(QX, QY, *nbr))
    for phi in cluster_vector_chunks(QX, QY, nbr):
        g += phi.conj() @ phi.T
    return g


def bond_density_matrix_brute(X, Y, nbr, d=2):
    """Two-site reduced density matrix of the bond X.r - Y.l from the explicit
    eight-site ket (Fig. 4(b) cluster with the full site tensors X, Y and the
    bond between them contracted): every leg except the physical indices of
    X and Y is an environment index ``e`` (the neighbours' physical legs,
    the external virtual legs and the ancillas of X and Y), and
    ``rho[(s1 s2), (s1' s2')] = sum_e Phi(e; s1, s2) conj(Phi(e; s1', s2'))``,
    normalised to unit trace."""
    L, TX, BX, TY, BY, Rn = nbr
    p, D = X.shape[0], X.shape[1]
    na = p // d
    X6 = X.reshape(d, na, D, D, D, D)
    Y6 = Y.reshape(d, na, D, D, D, D)
    rho = np.zeros((d * d, d * d), dtype=np.result_type(X, Y, *nbr))
    for pl in range(L.shape[0]):
        for pr in range(Rn.shape[0]):
            # X legs (s, anc, t, l, b, k), Y legs (s, anc, t, k, b, r), k = the bond;
            # one chunk per physical index of L and of Rn
            phi = np.einsum(
                'xatlbk,TUVl,ABCtv,DbEFw,GHvIJ,KMwLN,ycIkMr,PrQS->xyacABCDEFGHJKLNPQSTUV',
                X6, L[pl], TX, BX, TY, BY, Y6, Rn[pr], optimize=True)
            phi = phi.reshape(d * d, -1)
            rho += phi @ phi.conj().T
    return rho / np.trace(rho)


def torus_state(A, B, L=4):
    """State vector of the two-site checkerboard iPEPS on an L x L torus (L
    even), every bond contracted: ``A`` on the sites (x, y) with x + y even,
    ``B`` on the others, legs (p, t, l, b, r); the r leg of (x, y) joins the l
    leg of (x + 1, y), the t leg joins the b leg of (x, y + 1).  Returns
    ``psi[s]`` with the physical indices ordered row by row (y, then x)."""
    p, D = A.shape[0], A.shape[1]
    rows = []
    for y in range(L):
        # row tensor: horizontal bonds of the ring contracted one site at a time
        T0 = A if y % 2 == 0 else B
        # (s, t, b, l0, r); then s, t, b grow one site at a time
        cur = T0.transpose(0, 1, 3, 2, 4)
        for x in range(1, L):
            T = A if (x + y) % 2 == 0 else B
            # contract cur's r with T's l
            cur = np.einsum('STBlk,ptkbr->SpTtBblr', cur, T)
            n = cur.shape
            cur = cur.reshape(n[0] * n[1], n[2] * n[3], n[4] * n[5], n[6], n[7])
        # close the ring: r of the last site with l0 of the first
        rows.append(np.einsum('STBll->STB', cur))              # (s_row, t_row, b_row)
    # stack rows: t of row y joins b of row y + 1; b of row 0 joins t of row L-1
    st = rows[0]                                               # (S, T, B0)
    for y in range(1, L):
        st = np.einsum('STO,stT->SstO', st, rows[y])
        n = st.shape
        st = st.reshape(n[0] * n[1], n[2], n[3])
    return np.einsum('STT->S', st)
