"""TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Truncated singular value decomposition of a TensorMap, Alg. "Abelian tensor
decomposition": permute A into the matrix form (p; q), decompose the matrix
of every coupled charge c on its own (the grouping isomorphism is unitary, so
the blocks' SVDs together are an SVD of the whole map), and give the new bond
space W one sector per coupled charge, whose degeneracy is the number of
singular values kept there.  Truncation (the truncated SVD of the two-site
benchmark, Alg. "Two-site Benchmark"): the largest singular values over all
sectors are kept, at most max_dim of them and only those above cutoff; the
truncation error is the norm of the discarded ones.

A = U o S o Vh with U : cod <- W, S : W <- W (diagonal, descending per
sector), Vh : W <- dom.  A library SVD (numpy) is the per-block step.
"""
from __future__ import annotations

import numpy as np

from . import blockwise
from .graded import Space, Structure


def svd_trunc(st: Structure, vec, p, q, max_dim=None, cutoff=0.0):
    """Returns (stU, u), (stS, s), (stV, vh), trunc_err, kept, where kept maps
    each coupled charge to its kept singular values (descending)."""
    stT, v = blockwise.permute_storage(st, vec, p, q)
    pieces = {}
    allv = []
    for c in stT.sectors:
        M = stT.sector_matrix(v, c)
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
        pieces[c] = (U, s, Vt)
        allv += [(float(x), n, j) for j, x in enumerate(s) for n in [stT.sectors.index(c)]]
    # largest first; ties by sector order, then index
    allv.sort(key=lambda t: (-t[0], t[1], t[2]))
    keep = [t for t in allv if t[0] > cutoff]
    if max_dim is not None and max_dim >= 0:
        keep = keep[:max_dim]
    dropped = allv[len(keep):] if len(keep) < len(allv) else []
    kset = {}
    for x, n, j in keep:
        kset.setdefault(stT.sectors[n], []).append(j)
    kept_c = [c for c in stT.sectors if c in kset]
    W = Space(kept_c, [len(kset[c]) for c in kept_c])
    stU = Structure(st.sym, stT.cod, (W,))
    stS = Structure(st.sym, (W,), (W,))
    stV = Structure(st.sym, (W,), stT.dom)
    u = np.zeros(stU.size)
    s = np.zeros(stS.size)
    vh = np.zeros(stV.size)
    kept = {}
    for c in kept_c:
        js = sorted(kset[c])              # numpy orders each block's values descending
        U, sv, Vt = pieces[c]
        R, k = U.shape[0], len(js)
        o = stU.sector_offset[c]
        u[o:o + R * k] = U[:, js].reshape(-1, order="F")
        o = stS.sector_offset[c]
        s[o:o + k * k] = np.diag(sv[js]).reshape(-1, order="F")
        o = stV.sector_offset[c]
        C = Vt.shape[1]
        vh[o:o + k * C] = Vt[js, :].reshape(-1, order="F")
        kept[c] = sv[js]
    err = float(np.sqrt(sum(x * x for x, _, _ in dropped)))
    return (stU, u), (stS, s), (stV, vh), err, kept
