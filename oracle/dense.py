"""O1: dense definitions of permute and contraction (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Bosonic symmetries (Z1, Z2, U1): the symmetric algorithms reach exactly the
dense result.  Permute is the array transpose C_{I;J} = A_{I';J'} (section
"Permutations", with tau_{ij;kl} = delta_il delta_jk); a pairwise contraction
is permute-permute-compose-permute where composition is the matrix product
C_{I;J} = A_{I;K} B_{K;J} (eq. tm_composition, Alg. "Tensor Contraction").
Densified, that is one einsum.

Fermionic symmetries (FZ2, U1xFZ2): a tensor network is evaluated as a graph
under the "twist pushed into the right evaluation" convention of section
"Fermions and fusion categories":
  * a TensorMap W_1..W_N2 -> V_1..V_N1 is the tensor in
    V_1 (x)..(x) V_N1 (x) W*_N2 (x)..(x) W*_1 (eq. homtobraket), the stored
    coefficients unchanged; a leg is "dual" in this order iff its space is
    dual xor it sits in the domain;
  * every crossing of two lines is the braiding tau with R^{JJ}_I = -1 and
    R = +1 otherwise (Deligne product: the U(1) factor is trivial), so
    reordering legs multiplies an entry by (-1)^{|x||y|} for every pair of
    legs whose order is exchanged;
  * a contracted pair is closed with the left evaluation  V* (x) V -> C,
    <i|j> = delta_ij, after placing the dual leg first; closing it the other
    way round is the pushed-twist pairing  V (x) V* -> C,
    |v><w| -> (-1)^{|v||w|} delta_vw, which is the same thing.
The evaluator below builds the einsum of all tensors, one (-1)^{pi_x pi_y}
factor per exchanged pair of legs, and a shared index per contracted pair.
"""
from __future__ import annotations

import numpy as np

from .graded import Space, fparity, is_fermionic, linearized_order, permute_spaces


# ---------------------------------------------------------------------------
# bosonic definitions
# ---------------------------------------------------------------------------
def permute_bosonic(T: np.ndarray, p, q) -> np.ndarray:
    """C_{I;J} = A_{I';J'}: output leg n is input leg (p+q)[n]."""
    return np.transpose(T, tuple(p) + tuple(q))


def contract_bosonic(A: np.ndarray, pA, qA, B: np.ndarray, pB, qB, pAB, qAB) -> np.ndarray:
    """Dense pairwise contraction: legs qA of A are summed against legs pB of
    B (k-th with k-th); the free legs pA then qB are reordered by pAB + qAB."""
    if len(qA) != len(pB):
        raise ValueError("contracted leg lists differ in length")
    la = list(range(A.ndim))
    lb = list(range(A.ndim, A.ndim + B.ndim))
    for ka, kb in zip(qA, pB):
        lb[kb] = la[ka]
    free = [la[i] for i in pA] + [lb[i] for i in qB]
    out = [free[i] for i in tuple(pAB) + tuple(qAB)]
    return np.einsum(A, la, B, lb, out, optimize=True)


def adjoint_dense(T: np.ndarray, N1: int) -> np.ndarray:
    """A^dagger_{j;i} = conj(A_{i;j}) (section "Orthogonality and Adjoints")."""
    n = T.ndim
    return np.conj(np.transpose(T, tuple(range(N1, n)) + tuple(range(N1))))


# ---------------------------------------------------------------------------
# fermionic graph evaluator
# ---------------------------------------------------------------------------
def _lin_dual(sp: Space, in_domain: bool) -> bool:
    return bool(sp.dual) ^ bool(in_domain)


def graph_evaluate(sym: str, tensors, pairs, out_cod, out_dom):
    """Evaluate a fermionic (or bosonic) tensor network as a graph.

    tensors : list of (T, cod_spaces, dom_spaces); T dense, axes cod then dom.
    pairs   : list of ((t, leg), (t', leg')) contracted with each other.
    out_cod, out_dom : lists of (t, leg) -- the free legs in the output's
              codomain and domain order.
    Returns (dense output with axes out_cod + out_dom, cod spaces, dom spaces).
    """
    legs = []            # joint order: each tensor's legs in bra-ket order
    info = {}
    for ti, (T, cod, dom) in enumerate(tensors):
        N1, N2 = len(cod), len(dom)
        if T.shape != tuple(s.dim for s in tuple(cod) + tuple(dom)):
            raise ValueError(f"tensor {ti}: dense shape does not match its spaces")
        sp = tuple(cod) + tuple(dom)
        for l in linearized_order(N1, N2):
            key = (ti, l)
            legs.append(key)
            info[key] = dict(space=sp[l], lin_dual=_lin_dual(sp[l], l >= N1),
                             par=sp[l].parity_of_index(sym))
    used = [k for pr in pairs for k in pr] + list(out_cod) + list(out_dom)
    if sorted(used) != sorted(legs):
        raise ValueError("every leg must be contracted or free exactly once")

    target = []
    for x, y in pairs:
        sx, sy = info[x]["space"], info[y]["space"]
        if sx.sectors != sy.sectors or sx.degs != sy.degs:
            raise ValueError(f"contracted legs {x}, {y} carry different spaces")
        if info[x]["lin_dual"] == info[y]["lin_dual"]:
            raise ValueError(f"contracted legs {x}, {y} are not a vector/co-vector pair")
        target += [x, y] if info[x]["lin_dual"] else [y, x]
    out_lin = list(out_cod) + list(reversed(list(out_dom)))
    target += out_lin
    target_pos = {k: i for i, k in enumerate(target)}

    # index letters: one per leg, shared within a contracted pair
    letter = {}
    for n, k in enumerate(legs):
        letter[k] = n
    for x, y in pairs:
        letter[y] = letter[x]

    operands = []
    for ti, (T, cod, dom) in enumerate(tensors):
        operands += [T, [letter[(ti, l)] for l in range(T.ndim)]]
    if is_fermionic(sym):
        for i, x in enumerate(legs):
            for y in legs[i + 1:]:
                if target_pos[x] > target_pos[y]:          # this pair is exchanged
                    px, py = info[x]["par"], info[y]["par"]
                    if px.any() and py.any():
                        S = np.where(np.outer(px, py) % 2 == 1, -1.0, 1.0)
                        operands += [S, [letter[x], letter[y]]]
    out_letters = [letter[k] for k in list(out_cod) + list(out_dom)]
    res = np.einsum(*operands, out_letters, optimize=True)

    ocod = tuple(Space(info[k]["space"].sectors, info[k]["space"].degs, info[k]["lin_dual"])
                 for k in out_cod)
    odom = tuple(Space(info[k]["space"].sectors, info[k]["space"].degs, not info[k]["lin_dual"])
                 for k in out_dom)
    return res, ocod, odom


def permute_dense(sym: str, T: np.ndarray, cod, dom, p, q):
    """Dense permute under the graph semantics (bosonic: plain transpose)."""
    ncod, ndom = permute_spaces(cod, dom, p, q)
    if not is_fermionic(sym):
        return permute_bosonic(T, p, q), ncod, ndom
    res, c2, d2 = graph_evaluate(sym, [(T, cod, dom)], [], [(0, i) for i in p], [(0, j) for j in q])
    assert c2 == ncod and d2 == ndom
    return res, ncod, ndom


def contract_dense(sym: str, A, Acod, Adom, pA, qA, B, Bcod, Bdom, pB, qB, pAB, qAB):
    """Dense pairwise contraction, Alg. "Tensor Contraction" semantics: the
    k-th leg of qA meets the k-th leg of pB; C~ has legs pA then qB, and C is
    C~ reordered by (pAB, qAB).  Returns (C, cod, dom)."""
    _, Adom_t = permute_spaces(Acod, Adom, pA, qA)
    Bcod_t, _ = permute_spaces(Bcod, Bdom, pB, qB)
    if Adom_t != Bcod_t:
        raise ValueError("domain(A~) != codomain(B~)")
    free = [(0, i) for i in pA] + [(1, j) for j in qB]
    out_cod = [free[i] for i in pAB]
    out_dom = [free[i] for i in qAB]
    pairs = [((0, a), (1, b)) for a, b in zip(qA, pB)]
    if not is_fermionic(sym):
        C = contract_bosonic(A, pA, qA, B, pB, qB, pAB, qAB)
        Bt_dom = permute_spaces(Bcod, Bdom, pB, qB)[1]
        At_cod = permute_spaces(Acod, Adom, pA, qA)[0]
        ocod, odom = permute_spaces(At_cod, Bt_dom, pAB, qAB)
        return C, ocod, odom
    return graph_evaluate(sym, [(A, Acod, Adom), (B, Bcod, Bdom)], pairs, out_cod, out_dom)


def trace_dense(sym: str, T: np.ndarray, cod, dom, p, q, t1, t2):
    """Partial trace (Alg. "Abelian Tensor Trace") as a graph: legs t1[i] and
    t2[i] of the one tensor are a contracted pair (closed with the dual leg
    first, as every pair of the evaluator), the free legs are the output's
    codomain p and domain q.  For a bosonic symmetry this is the einsum with
    a repeated index per pair.  Returns (C, cod, dom)."""
    pairs = [((0, a), (0, b)) for a, b in zip(t1, t2)]
    return graph_evaluate(sym, [(T, cod, dom)], pairs, [(0, i) for i in p], [(0, j) for j in q])


# ---------------------------------------------------------------------------
# adjacent-swap decomposition (used by the tests to pin the exchange sign)
# ---------------------------------------------------------------------------
def permute_linear_by_swaps(sym: str, T: np.ndarray, spaces, perm, rng=None):
    """Reorder the axes of a linearized tensor T (axes in bra-ket order, with
    the given spaces) so that output axis n is input axis perm[n], by a chain
    of adjacent swaps tau^(k,k+1), each multiplying by R = (-1)^{|x||y|}
    (footnote on the bubble-sort decomposition in section "Permutations").
    rng=None sweeps left to right (bubble sort); otherwise every step picks a
    random adjacent inverted pair, giving a different decomposition."""
    order = list(range(T.ndim))            # current axis -> original leg
    want = {leg: n for n, leg in enumerate(perm)}
    pars = [sp.parity_of_index(sym) for sp in spaces]
    X = T.copy()
    while True:
        inv = [k for k in range(len(order) - 1) if want[order[k]] > want[order[k + 1]]]
        if not inv:
            break
        k = inv[0] if rng is None else inv[int(rng.integers(len(inv)))]
        ax = list(range(X.ndim))
        ax[k], ax[k + 1] = ax[k + 1], ax[k]
        X = np.transpose(X, ax)
        a, b = order[k], order[k + 1]
        if is_fermionic(sym):
            S = np.where(np.outer(pars[b], pars[a]) % 2 == 1, -1.0, 1.0)
            shape = [1] * X.ndim
            shape[k], shape[k + 1] = S.shape
            X = X * S.reshape(shape)
        order[k], order[k + 1] = b, a
    return X

