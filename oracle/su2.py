"""TEST INFRASTRUCTURE ONLY -- never imported by the product path.

SU(2)-symmetric tensor maps and their leg permutations, Section "Non-abelian
symmetries" (fusion trees; the canonical expansion of a tensor map over
fusion-splitting tree pairs) and Alg. "Non-abelian Tensor Transformation".

Conventions (shared with the HIP path only through this description):

* Spins are stored as twice their value (tj = 2j).  A leg is a list of
  (tj, deg) sectors with distinct tj, ascending.
* A splitting tree of legs a_1..a_N is canonical (left to right, eq. of the
  canonical splitting): e_1 = a_1, e_k in e_{k-1} x a_k, e_N = c.  Its dense
  form X[m_1..m_N, m_c] is built from Clebsch-Gordan coefficients
  <e_{k-1} m, a_k m_k | e_k m'>; index m of spin j runs over j, j-1, .., -j.
  A domain tree is the adjoint of a splitting tree of the domain legs.
* t = sum over tree pairs (s, f) with the same coupled spin c of
  X_s . X_f^T (summed over m_c) (x) t^(s,f), the reduced array t^(s,f) having
  the degeneracies of the outer sectors as its axes.
* Storage: one column-major matrix per coupled spin c (ascending, only those
  with rows and columns); rows are the splitting trees of c, columns the
  domain trees of c, each tree taking the product of its outer degeneracies
  (first leg fastest).  Trees of one c are ordered by outer sectors (colex,
  first leg fastest), then by intermediates e_2..e_{N-1} (colex).
* permute(t, (p, q)) moves output codomain leg k to input leg p[k] and
  output domain leg k to input leg q[k]; here every p[k] is a codomain leg
  and every q[k] a domain leg (braids within each side).
* Dual legs (section "Duality Fusion Tree Manipulations"): a leg may carry
  the dual space V_j* of its sectors.  The canonical trees keep spin j on
  such a leg and add the isomorphism between V_j* and V_j on the outer line
  (Z^dagger on a splitting tree, Z on a fusion tree); here Z maps the dual
  basis vector of m to (-1)^(j-m) times the vector of -m, so on a dual leg
  the dense index of m (position i = j - m) holds (-1)^i times the tree's
  value at -m, on either side.  For SU(2) the Frobenius-Schur phase of spin j
  is (-1)^(2j).
* transpose(t, (p, q)) (the generalised transpose and permute of the
  paper: any legs may cross between codomain and domain, a crossing leg
  turning into the dual space): on dense arrays a bend is the identity on
  components (coevaluation and evaluation pair a basis with its dual basis),
  so the transformed map is the array with its axes reordered to (p, q),
  projected onto the canonical trees of the new structure.  Its
  coefficients per pair of trees are computed the same way on the dense
  form of one tree pair (pair_coeffs) and applied to the reduced arrays.

The transformation coefficients are the overlaps of each permuted tree with
the canonical trees (the projection method of Section "Fusion Tree
Manipulations": trees form an orthonormal basis), computed from their dense
forms.  SU(2) braiding is symmetric and its coefficients are real.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np


def _fact(n2: int) -> int:
    """Factorial of n2 / 2 (n2 even and >= 0)."""
    assert n2 % 2 == 0 and n2 >= 0
    return math.factorial(n2 // 2)


def triangle(ta: int, tb: int, tc: int) -> bool:
    """Spin c appears in a x b (all twice their value)."""
    return abs(ta - tb) <= tc <= ta + tb and (ta + tb + tc) % 2 == 0


def cg(tj1, tm1, tj2, tm2, tJ, tM) -> float:
    """Clebsch-Gordan coefficient <j1 m1, j2 m2 | J M> (Condon-Shortley
    phases), by Racah's closed formula; arguments are twice their value."""
    if tm1 + tm2 != tM or not triangle(tj1, tj2, tJ):
        return 0.0
    if abs(tm1) > tj1 or abs(tm2) > tj2 or abs(tM) > tJ:
        return 0.0
    pre = Fraction((tJ + 1) * _fact(tJ + tj1 - tj2) * _fact(tJ - tj1 + tj2) * _fact(tj1 + tj2 - tJ),
                   _fact(tj1 + tj2 + tJ + 2))
    pre *= (_fact(tJ + tM) * _fact(tJ - tM) * _fact(tj1 - tm1) * _fact(tj1 + tm1)
            * _fact(tj2 - tm2) * _fact(tj2 + tm2))
    s = Fraction(0)
    for k in range(0, tj1 + tj2 + 1):
        args = [tj1 + tj2 - tJ - 2 * k, tj1 - tm1 - 2 * k, tj2 + tm2 - 2 * k,
                tJ - tj2 + tm1 + 2 * k, tJ - tj1 - tm2 + 2 * k]
        if min(args) < 0:
            continue
        den = math.factorial(k)
        for a in args:
            den *= _fact(a)
        s += Fraction((-1) ** k, den)
    return float(s) * math.sqrt(pre)


def mvals(tj: int):
    """m = j, j-1, .., -j (twice their value): the order of a spin's index."""
    return list(range(tj, -tj - 1, -2))


def cg_tensor(ta: int, tb: int, tc: int) -> np.ndarray:
    """X[ma, mb, mc] = <a ma, b mb | c mc>: the splitting tensor c -> a x b."""
    X = np.zeros((ta + 1, tb + 1, tc + 1))
    for i, ma in enumerate(mvals(ta)):
        for j, mb in enumerate(mvals(tb)):
            for k, mc in enumerate(mvals(tc)):
                X[i, j, k] = cg(ta, ma, tb, mb, tc, mc)
    return X


def spin_ops(tj: int):
    """J_z and J_+ on spin j in the basis m = j..-j (for invariance pins)."""
    ms = mvals(tj)
    n = tj + 1
    Jz = np.diag([m / 2.0 for m in ms])
    Jp = np.zeros((n, n))
    for i in range(1, n):  # J+ |m> = sqrt(j(j+1) - m(m+1)) |m+1>
        m = ms[i] / 2.0
        j = tj / 2.0
        Jp[i - 1, i] = math.sqrt(j * (j + 1) - m * (m + 1))
    return Jz, Jp


def trees(outer):
    """Canonical splitting trees for outer spins (tj per leg): a list of
    (intermediates e_2..e_{N-1}, coupled c), in the storage order for one
    outer tuple (intermediates colex, e_2 fastest)."""
    N = len(outer)
    if N == 1:
        return [((), outer[0])]
    res = []

    def rec(k, e, inter):
        if k == N:
            res.append((tuple(inter[:-1]), inter[-1]))
            return
        for tf in range(abs(e - outer[k]), e + outer[k] + 1, 2):
            rec(k + 1, tf, inter + [tf])

    rec(1, outer[0], [])
    # colex over (e_2..e_{N-1}), first intermediate fastest
    res.sort(key=lambda t: (t[1], tuple(reversed(t[0]))))
    return res


def tree_tensor(outer, inter, tc) -> np.ndarray:
    """Dense splitting tree X[m_1..m_N, m_c] (eq. of the canonical splitting)."""
    T = np.eye(outer[0] + 1)  # [m_1, m_e1]
    es = [outer[0]] + list(inter) + [tc] if len(outer) > 1 else [tc]
    for k in range(1, len(outer)):
        X = cg_tensor(es[k - 1], outer[k], es[k])
        T = np.tensordot(T, X, axes=([T.ndim - 1], [0]))
    return T


def dualize(T, axes):
    """Puts the isomorphism Z between V_j* and V_j on the given axes of a dense
    tree or tree pair: along each axis, entry i becomes (-1)^i times entry
    2j - i (m = j - i goes to -m)."""
    for ax in axes:
        n = T.shape[ax]
        sign = np.array([(-1.0) ** i for i in range(n)])
        shape = [1] * T.ndim
        shape[ax] = n
        T = np.flip(T, axis=ax) * sign.reshape(shape)
    return T


def pair_tensor(cod_outer, dom_outer, s_inter, f_inter, tc, duals=()) -> np.ndarray:
    """Dense tree pair X_s . X_f^T summed over m_c, axes [m_cod.., m_dom..],
    with Z on the legs listed in duals (global leg numbers)."""
    X = tree_tensor(cod_outer, s_inter, tc)
    Y = tree_tensor(dom_outer, f_inter, tc)
    G = np.tensordot(X, Y, axes=([len(cod_outer)], [len(dom_outer)]))
    return dualize(G, duals)


class SU2Map:
    """Structure of t : cod <- dom (legs as lists of (tj, deg)); dual lists
    the legs (0-based, codomain then domain) that carry the dual space."""

    def __init__(self, cod, dom, dual=()):
        self.cod = [sorted(l) for l in cod]
        self.dom = [sorted(l) for l in dom]
        self.N1, self.N2 = len(self.cod), len(self.dom)
        self.dual = tuple(sorted(dual))
        assert self.N1 >= 1 and self.N2 >= 1
        rows = self._side(self.cod)
        cols = self._side(self.dom)
        self.blocks = {}  # tc -> (offset, R, C)
        self.rows, self.cols = {}, {}  # tc -> list of (outer sector idx, inter, r0, dims)
        off = 0
        for tc in sorted(set(rows) & set(cols)):
            R = sum(int(np.prod(d)) for *_, d in rows[tc])
            C = sum(int(np.prod(d)) for *_, d in cols[tc])
            self.blocks[tc] = (off, R, C)
            self.rows[tc], self.cols[tc] = rows[tc], cols[tc]
            off += R * C
        self.size = off

    @staticmethod
    def _side(legs):
        out = {}
        ranges = [range(len(l)) for l in legs]
        # colex over outer sector indices: first leg fastest
        tuples = sorted(itertools.product(*ranges), key=lambda t: tuple(reversed(t)))
        for idx in tuples:
            outer = [legs[k][i][0] for k, i in enumerate(idx)]
            dims = tuple(legs[k][i][1] for k, i in enumerate(idx))
            for inter, tc in trees(outer):
                lst = out.setdefault(tc, [])
                r0 = sum(int(np.prod(d)) for *_, d in lst)
                lst.append((idx, inter, r0, dims))
        return out

    def pairs(self):
        """Every tree pair: (tc, s, f) with s, f entries of rows/cols."""
        for tc in self.blocks:
            for s in self.rows[tc]:
                for f in self.cols[tc]:
                    yield tc, s, f

    def get(self, vec, tc, s, f) -> np.ndarray:
        """The reduced array t^(s,f), axes = codomain then domain
        degeneracies (element (i; j) sits at row r0(s) + colex(i), column
        c0(f) + colex(j) of the block of c)."""
        off, R, C = self.blocks[tc]
        M = vec[off:off + R * C].reshape(C, R).T
        nr, nc = int(np.prod(s[3])), int(np.prod(f[3]))
        return M[s[2]:s[2] + nr, f[2]:f[2] + nc].reshape(tuple(s[3]) + tuple(f[3]), order="F")

    def add(self, vec, tc, s, f, arr):
        """Adds arr (axes as get returns them) to t^(s,f) in vec."""
        off, R, C = self.blocks[tc]
        M = vec[off:off + R * C].reshape(C, R).T
        nr, nc = int(np.prod(s[3])), int(np.prod(f[3]))
        M[s[2]:s[2] + nr, f[2]:f[2] + nc] += arr.reshape((nr, nc), order="F")

    def outer(self, s, side):
        legs = self.cod if side == 0 else self.dom
        return [legs[k][i][0] for k, i in enumerate(s[0])]


def permute_legs(st: SU2Map, p, q) -> SU2Map:
    """Structure of permute(t, (p, q)) for braids within each side."""
    N1 = st.N1
    assert sorted(p) == list(range(N1)) and sorted(q) == list(range(N1, N1 + st.N2)), \
        "only permutations within the codomain and within the domain"
    return SU2Map([st.cod[k] for k in p], [st.dom[k - N1] for k in q])


def tree_coeffs(outer, inter, tc, perm):
    """Coefficients of the permuted splitting tree (legs reordered so that
    new leg k is old leg perm[k]) in the canonical trees of the new outer
    spins: {(new inter): coefficient}, by overlap of the dense forms."""
    X = tree_tensor(outer, inter, tc)
    Y = X.transpose(list(perm) + [len(outer)])
    new_outer = [outer[k] for k in perm]
    res = {}
    for ninter, ntc in trees(new_outer):
        if ntc != tc:
            continue
        Z = tree_tensor(new_outer, ninter, tc)
        # trees are orthonormal: <Z|Y> summed over all m, divided by d_c
        v = float(np.sum(Z * Y)) / (tc + 1)
        if abs(v) > 1e-13:
            res[ninter] = v
    return res


def permute(st: SU2Map, vec, p, q):
    """Alg. "Non-abelian Tensor Transformation": for every tree pair (s, f) of
    t and every output pair (s', f') its transform reaches with coefficient
    c_s c_f, y^(s',f') += c_s c_f permute(x^(s,f)).  Returns (structure, data)."""
    N1 = st.N1
    out = permute_legs(st, p, q)
    qd = [k - N1 for k in q]
    y = np.zeros(out.size)
    rowpos = {tc: {(r[0], r[1]): r for r in out.rows[tc]} for tc in out.blocks}
    colpos = {tc: {(c[0], c[1]): c for c in out.cols[tc]} for tc in out.blocks}
    cache = {}
    for tc, s, f in st.pairs():
        x = st.get(vec, tc, s, f)
        xp = x.transpose(list(p) + [N1 + k for k in qd])
        key_s = (tuple(st.outer(s, 0)), s[1], tc, tuple(p))
        key_f = (tuple(st.outer(f, 1)), f[1], tc, tuple(qd))
        for key, o, i, perm in ((key_s, st.outer(s, 0), s[1], p), (key_f, st.outer(f, 1), f[1], qd)):
            if key not in cache:
                cache[key] = tree_coeffs(o, i, tc, perm)
        sidx = tuple(s[0][k] for k in p)
        fidx = tuple(f[0][k] for k in qd)
        for si, cs in cache[key_s].items():
            for fi, cf in cache[key_f].items():
                out.add(y, tc, rowpos[tc][(sidx, si)], colpos[tc][(fidx, fi)], cs * cf * xp)
    return out, y


def leg_dense_index(leg):
    """Dense basis of one leg: sectors in order, within a sector the
    degeneracy index slowest and m fastest.  Returns per sector its offset."""
    offs, o = [], 0
    for tj, d in leg:
        offs.append(o)
        o += d * (tj + 1)
    return offs, o


def to_dense(st: SU2Map, vec) -> np.ndarray:
    """The full array t[i_1..i_N1; j_1..j_N2] (canonical expansion)."""
    legs = st.cod + st.dom
    info = [leg_dense_index(l) for l in legs]
    T = np.zeros([n for _, n in info])
    for tc, s, f in st.pairs():
        G = pair_tensor(st.outer(s, 0), st.outer(f, 1), s[1], f[1], tc, st.dual)  # [m_cod.., m_dom..]
        r = st.get(vec, tc, s, f)  # [i_cod.., j_dom..]
        N = st.N1 + st.N2
        # block[i_1, m_1, i_2, m_2, ...] = r[i..] * G[m..]
        blk = np.multiply.outer(r, G)
        blk = blk.transpose([a for k in range(N) for a in (k, N + k)])
        idx = list(s[0]) + list(f[0])
        sl = []
        for k in range(N):
            tj, d = legs[k][idx[k]]
            o = info[k][0][idx[k]]
            sl.append(slice(o, o + d * (tj + 1)))
        shape = [legs[k][idx[k]][1] * (legs[k][idx[k]][0] + 1) for k in range(N)]
        T[tuple(sl)] += blk.reshape(shape)
    return T


def from_dense(st: SU2Map, T) -> np.ndarray:
    """Projects a dense symmetric array onto the canonical tree pairs:
    t^(s,f) = (X_s^T T X_f) traced over m_c, divided by d_c."""
    legs = st.cod + st.dom
    info = [leg_dense_index(l) for l in legs]
    N = st.N1 + st.N2
    vec = np.zeros(st.size)
    for tc, s, f in st.pairs():
        G = pair_tensor(st.outer(s, 0), st.outer(f, 1), s[1], f[1], tc, st.dual)
        idx = list(s[0]) + list(f[0])
        sl, shape = [], []
        for k in range(N):
            tj, d = legs[k][idx[k]]
            o = info[k][0][idx[k]]
            sl.append(slice(o, o + d * (tj + 1)))
            shape += [d, tj + 1]
        blk = T[tuple(sl)].reshape(shape)
        r = np.tensordot(blk, G, axes=(list(range(1, 2 * N, 2)), list(range(N))))
        st.add(vec, tc, s, f, r / (tc + 1))
    return vec


def transpose_legs(st: SU2Map, p, q) -> SU2Map:
    """Structure of transpose(t, (p, q)): output codomain leg k is input leg
    p[k], output domain leg k input leg q[k]; a leg that changes sides carries
    the dual of its space."""
    N1 = st.N1
    legs = st.cod + st.dom
    assert sorted(list(p) + list(q)) == list(range(len(legs))) and len(p) >= 1 and len(q) >= 1
    dual = []
    for k, g in enumerate(list(p) + list(q)):
        crossed = (g < N1) != (k < len(p))
        if (g in st.dual) != crossed:
            dual.append(k)
    return SU2Map([legs[g] for g in p], [legs[g] for g in q], dual)


def pair_coeffs(st: SU2Map, out: SU2Map, cod_outer, dom_outer, s_inter, f_inter, tc, p, q):
    """Coefficients of one input tree pair, its dense form with axes
    reordered to (p, q), in the canonical tree pairs of the output with the
    same outer spins: {(s_inter', f_inter', tc'): coefficient}."""
    order = list(p) + list(q)
    G = pair_tensor(cod_outer, dom_outer, s_inter, f_inter, tc, st.dual).transpose(order)
    outer = list(cod_outer) + list(dom_outer)
    oc, od = [outer[g] for g in p], [outer[g] for g in q]
    res = {}
    for si, c1 in trees(oc):
        for fi, c2 in trees(od):
            if c1 != c2:
                continue
            H = pair_tensor(oc, od, si, fi, c1, out.dual)
            v = float(np.sum(H * G)) / (c1 + 1)  # tree pairs are orthonormal: d_c per pair
            if abs(v) > 1e-13:
                res[(si, fi, c1)] = v
    return res


def transpose(st: SU2Map, vec, p, q):
    """transpose(t, (p, q)) by coefficients: every input pair (s, f) adds
    coefficient times its reduced array, axes reordered to (p, q), to every
    output pair it reaches.  Returns (structure, data)."""
    out = transpose_legs(st, p, q)
    order = list(p) + list(q)
    y = np.zeros(out.size)
    rowpos = {tc: {(r[0], r[1]): r for r in out.rows[tc]} for tc in out.blocks}
    colpos = {tc: {(c[0], c[1]): c for c in out.cols[tc]} for tc in out.blocks}
    cache = {}
    for tc, s, f in st.pairs():
        co, do = st.outer(s, 0), st.outer(f, 1)
        key = (tuple(co), tuple(do), s[1], f[1], tc)
        if key not in cache:
            cache[key] = pair_coeffs(st, out, co, do, s[1], f[1], tc, p, q)
        xp = st.get(vec, tc, s, f).transpose(order)
        idx = list(s[0]) + list(f[0])
        sidx = tuple(idx[g] for g in p)
        fidx = tuple(idx[g] for g in q)
        for (si, fi, c2), cf in cache[key].items():
            out.add(y, c2, rowpos[c2][(sidx, si)], colpos[c2][(fidx, fi)], cf * xp)
    return out, y


def transpose_dense(st: SU2Map, vec, p, q):
    """The definition: the dense array with its axes reordered to (p, q),
    projected onto the output's canonical tree pairs."""
    out = transpose_legs(st, p, q)
    return out, from_dense(out, to_dense(st, vec).transpose(list(p) + list(q)))
