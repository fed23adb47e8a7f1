"""O2: plain blockwise permute and contraction (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A tensor is (Structure, {(cod_tuple, dom_tuple): block}) where the key holds
the sector index of every leg and the block is the reduced array of that
fusion channel with axes codomain legs then domain legs.

permute  : Alg. "Abelian Tensor Permutation": for every fusion channel
           (a_1..; b_1..), y = permute(x, (p.., q..)) and the output channel is
           (e; f) with e_i the p_i-th element of (a..; b*..) and f_j the q_j-th
           of (a*..; b..).  Here keys are sector indices of the underlying
           spaces, so the conjugation is carried by the flipped dual flag of
           the output space (the labels follow).  Fermionic symmetries multiply
           by (-1)^{|x||y|} for every pair of legs whose bra-ket order is
           exchanged (R^{JJ}_I = -1).
compose  : eq. abelian_compostion, C^c = A^c B^c per coupled charge; a coupled
           charge with an empty K range gives a zero block.  Fermionic: every
           contracted leg whose space (codomain of B~) is a dual space closes an
           (X, X*) pair and contributes (-1)^{|x|} (the pushed-twist pairing
           |v><w| -> (-1)^{|v||w|} delta_vw); pairs on normal spaces are
           sign free.
contract : Alg. "Abelian tensor contraction": A~ = permute(A, (pA, qA)),
           B~ = permute(B, (pB, qB)) (the paper prints q^A in the second call;
           q^B is meant), C~ = A~ o B~, C = permute(C~, (pAB, qAB)).
"""
from __future__ import annotations

import numpy as np

from .graded import Structure, fparity, is_fermionic, linearized_order, permute_spaces


def koszul_parity(sym: str, cod, dom, tup, p, q) -> int:
    """Parity of  sum over exchanged leg pairs (x, y) of |x||y|  for the
    channel whose legs carry the sector indices tup (cod legs then dom legs)."""
    if not is_fermionic(sym):
        return 0
    spaces = tuple(cod) + tuple(dom)
    pi = [fparity(sym, spaces[l].sectors[tup[l]]) for l in range(len(spaces))]
    lin_in = linearized_order(len(cod), len(dom))
    pos_in = {leg: i for i, leg in enumerate(lin_in)}
    src = tuple(p) + tuple(q)                       # output leg n <- input leg src[n]
    lin_out = linearized_order(len(p), len(q))
    pos_out = {src[n]: i for i, n in enumerate(lin_out)}
    s = 0
    for x in range(len(spaces)):
        for y in range(len(spaces)):
            if pos_in[x] < pos_in[y] and pos_out[x] > pos_out[y]:
                s += pi[x] * pi[y]
    return s & 1


def permute(st: Structure, blocks: dict, p, q):
    """Alg. "Abelian Tensor Permutation".  Returns (Structure, blocks)."""
    p, q = tuple(p), tuple(q)
    ncod, ndom = permute_spaces(st.cod, st.dom, p, q)
    out_st = Structure(st.sym, ncod, ndom)
    src = p + q
    out = {}
    for (a, b), x in blocks.items():
        tup = tuple(a) + tuple(b)
        y = np.transpose(x, src)
        if koszul_parity(st.sym, st.cod, st.dom, tup, p, q):
            y = -y
        e = tuple(tup[i] for i in p)
        f = tuple(tup[j] for j in q)
        out[(e, f)] = y
    return out_st, out


def twist_parity(sym: str, spaces, tup) -> int:
    """Parity of sum |x| over the legs whose space is dual (the pushed twist of
    an (X, X*) pair closed by a composition)."""
    if not is_fermionic(sym):
        return 0
    return sum(fparity(sym, spaces[l].sectors[tup[l]]) for l in range(len(spaces))
               if spaces[l].dual) & 1


def compose(stA: Structure, bA: dict, stB: Structure, bB: dict):
    """C~ = A~ o B~, block by block per coupled charge."""
    if stA.sym != stB.sym:
        raise ValueError("symmetry mismatch")
    if stA.dom != stB.cod:
        raise ValueError("domain(A~) != codomain(B~)")
    sym = stA.sym
    stC = Structure(sym, stA.cod, stB.dom)
    vA = stA.from_blocks(bA)
    bB2 = {}
    for (a, b), x in bB.items():
        bB2[(a, b)] = -x if twist_parity(sym, stB.cod, a) else x
    vB = stB.from_blocks(bB2)
    vC = np.zeros(stC.size)
    for c in stC.sectors:
        off = stC.sector_offset[c]
        M, N = stC.rows[c].total, stC.cols[c].total
        if c in stA.sectors and c in stB.sectors:
            Cm = stA.sector_matrix(vA, c) @ stB.sector_matrix(vB, c)
        else:
            Cm = np.zeros((M, N))          # K range empty: zero block
        vC[off:off + M * N] = Cm.reshape(-1, order="F")
    return stC, stC.to_blocks(vC)


def contract(stA, bA, pA, qA, stB, bB, pB, qB, pAB, qAB):
    """Alg. "Abelian tensor contraction".  Returns (Structure, blocks)."""
    stAt, bAt = permute(stA, bA, pA, qA)
    stBt, bBt = permute(stB, bB, pB, qB)
    stCt, bCt = compose(stAt, bAt, stBt, bBt)
    return permute(stCt, bCt, pAB, qAB)


def adjoint(st: Structure, blocks: dict):
    """Blockwise Hermitian conjugate; codomain and domain exchange (the
    grouping maps are permutation matrices, section "Adjoint")."""
    out_st = Structure(st.sym, st.dom, st.cod)
    n1 = st.N1
    out = {}
    for (a, b), x in blocks.items():
        n = x.ndim
        out[(b, a)] = np.conj(np.transpose(x, tuple(range(n1, n)) + tuple(range(n1))))
    return out_st, out


def contract_storage(stA: Structure, vA, pA, qA, stB: Structure, vB, pB, qB, pAB, qAB,
                     alpha=1.0, beta=0.0, vC=None):
    """Storage-vector form:  C = alpha * contract(A, B) + beta * C."""
    stC, bC = contract(stA, stA.to_blocks(vA), pA, qA, stB, stB.to_blocks(vB), pB, qB, pAB, qAB)
    out = alpha * stC.from_blocks(bC)
    if beta != 0.0:
        out = out + beta * np.asarray(vC)
    return stC, out


def permute_storage(st: Structure, v, p, q):
    stC, bC = permute(st, st.to_blocks(v), p, q)
    return stC, stC.from_blocks(bC)


def useful_flops(stA: Structure, pA, qA, stB: Structure, pB, qB) -> int:
    """sum over coupled charges of 2 M_c N_c K_c for the composition A~ o B~
    (only sectors with K_c > 0 do arithmetic)."""
    Acod, Adom = permute_spaces(stA.cod, stA.dom, pA, qA)
    Bcod, Bdom = permute_spaces(stB.cod, stB.dom, pB, qB)
    sA = Structure(stA.sym, Acod, Adom)
    sB = Structure(stB.sym, Bcod, Bdom)
    f = 0
    for c in sA.sectors:
        if c in sB.sectors:
            f += 2 * sA.rows[c].total * sA.cols[c].total * sB.cols[c].total
    return f
