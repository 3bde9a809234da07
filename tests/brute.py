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
