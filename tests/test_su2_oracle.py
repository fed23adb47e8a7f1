"""Pins of the SU(2) oracle (oracle/su2.py) against what the mathematics and
the paper fix: Clebsch-Gordan closed forms and orthonormality, SU(2)
invariance and orthonormality of the dense fusion trees (section "Fusion
trees"), the worked permutation and trace matrices of the section "Index
Manipulations", and the permutation computed densely (build the full array,
transpose it, project back)."""
import math
import os

import numpy as np
import pytest

from oracle import su2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
V = [(0, 1), (1, 1)]  # V_0 + V_1/2, degeneracy 1 each


def test_cg_closed_forms():
    for tj in range(0, 7):
        # stretched state: <j j, j' j' | j+j', j+j'> = 1
        for tk in range(0, 5):
            assert su2.cg(tj, tj, tk, tk, tj + tk, tj + tk) == pytest.approx(1.0, abs=1e-15)
        # singlet: <j m, j -m | 0 0> = (-1)^(j-m) / sqrt(2j+1)
        for tm in su2.mvals(tj):
            want = (-1) ** ((tj - tm) // 2) / math.sqrt(tj + 1)
            assert su2.cg(tj, tm, tj, -tm, 0, 0) == pytest.approx(want, abs=1e-15)
    # two spin-1/2: the triplet m = 0 state and the singlet
    assert su2.cg(1, 1, 1, -1, 2, 0) == pytest.approx(1 / math.sqrt(2), abs=1e-15)
    assert su2.cg(1, -1, 1, 1, 2, 0) == pytest.approx(1 / math.sqrt(2), abs=1e-15)
    assert su2.cg(1, 1, 1, -1, 0, 0) == pytest.approx(1 / math.sqrt(2), abs=1e-15)
    assert su2.cg(1, -1, 1, 1, 0, 0) == pytest.approx(-1 / math.sqrt(2), abs=1e-15)
    # spin 1 x spin 1/2 -> 3/2, m = 1/2: sqrt(2/3) and sqrt(1/3)
    assert su2.cg(2, 0, 1, 1, 3, 1) == pytest.approx(math.sqrt(2 / 3), abs=1e-15)
    assert su2.cg(2, 2, 1, -1, 3, 1) == pytest.approx(math.sqrt(1 / 3), abs=1e-15)


@pytest.mark.parametrize("ta,tb", [(1, 1), (2, 1), (2, 3), (3, 4)])
def test_cg_unitary(ta, tb):
    rows = []
    for tc in range(abs(ta - tb), ta + tb + 1, 2):
        X = su2.cg_tensor(ta, tb, tc)
        rows.append(X.reshape((ta + 1) * (tb + 1), tc + 1))
    U = np.concatenate(rows, axis=1)  # (ma mb) x (c mc): square and orthogonal
    assert U.shape[0] == U.shape[1]
    np.testing.assert_allclose(U.T @ U, np.eye(U.shape[0]), atol=1e-14)


def _total(ops, tjs, which):
    """sum_k J^(k) on the tensor product of spins tjs."""
    n = int(np.prod([t + 1 for t in tjs]))
    out = np.zeros((n, n))
    for k, t in enumerate(tjs):
        m = np.eye(1)
        for l, u in enumerate(tjs):
            m = np.kron(m, ops(u)[which] if l == k else np.eye(u + 1))
        out += m
    return out


@pytest.mark.parametrize("outer", [[1, 1, 1], [2, 1, 3], [1, 2, 2, 1], [3, 3, 2]])
def test_trees_invariant_and_orthonormal(outer):
    ts = su2.trees(outer)
    assert ts
    Xs = {}
    for inter, tc in ts:
        X = su2.tree_tensor(outer, inter, tc)
        M = X.reshape(-1, tc + 1)
        for w in (0, 1):  # J_z and J_+ commute with the tree: (sum_k J^(k)) X = X J^(c)
            np.testing.assert_allclose(_total(su2.spin_ops, outer, w) @ M, M @ su2.spin_ops(tc)[w], atol=1e-13)
        Xs[(inter, tc)] = M
    # orthonormality of the trees (equation after the canonical basis)
    for a, Ma in Xs.items():
        for b, Mb in Xs.items():
            G = Ma.T @ Mb if a[1] == b[1] else None
            if G is not None:
                np.testing.assert_allclose(G, np.eye(a[1] + 1) if a == b else 0 * G, atol=1e-13)
    # completeness: the trees span the product space
    assert sum(tc + 1 for _, tc in ts) == int(np.prod([t + 1 for t in outer]))


def _storage_matrix(st, fn, n_out):
    M = np.zeros((n_out, st.size))
    for j in range(st.size):
        e = np.zeros(st.size)
        e[j] = 1.0
        M[:, j] = fn(e)
    return M


def test_paper_permutation_matrix():
    want = np.loadtxt(os.path.join(GOLDEN, "su2_permute_matrix.txt"))
    st = su2.SU2Map([V, V], [V, V])
    assert st.size == 9
    M = _storage_matrix(st, lambda e: su2.permute(st, e, [1, 0], [3, 2])[1], 9)
    np.testing.assert_allclose(M, want, atol=1e-14)


def _trace_fixture():
    lines = open(os.path.join(GOLDEN, "su2_trace_matrix.txt")).read().splitlines()
    lines = [l for l in lines if l and not l.startswith("#")]
    i, j = lines.index("matrix"), lines.index("formula")
    mat = np.array([[float(x) for x in l.split()] for l in lines[i + 1:j]])
    form = np.zeros((9, 2))
    for l in lines[j + 1:]:
        lhs, rhs = l.split("=")
        for term in rhs.split("+"):
            c, ch = term.strip().split("*")
            form[int(ch) - 1, int(lhs) - 1] = float(c)
    return mat, form


def _dense_trace(st, vec, leg):
    """Partial trace of codomain leg `leg` with domain leg `leg` on the dense
    array, projected back onto V <- V."""
    T = su2.to_dense(st, vec)  # axes (i1, i2; j1, j2)
    Tt = np.einsum("abad->bd", T) if leg == 0 else np.einsum("abcb->ac", T)
    out = su2.SU2Map([V], [V])
    return su2.from_dense(out, Tt)


def test_paper_trace_matrix_and_formula():
    mat, form = _trace_fixture()
    st = su2.SU2Map([V, V], [V, V])
    first = _storage_matrix(st, lambda e: _dense_trace(st, e, 0), 2).T
    second = _storage_matrix(st, lambda e: _dense_trace(st, e, 1), 2).T
    np.testing.assert_allclose(first, mat, atol=1e-14)
    np.testing.assert_allclose(second, form, atol=1e-14)


CASES = [
    ([[(0, 2), (1, 1)], [(1, 2), (2, 1)]], [[(1, 1), (2, 2)], [(0, 1), (1, 2)]], [1, 0], [2, 3]),
    ([[(0, 1), (1, 2)], [(1, 1), (2, 2)], [(1, 2), (3, 1)]],
     [[(1, 2), (2, 1)], [(0, 1), (1, 2), (2, 1)], [(1, 1), (3, 1)]], [2, 0, 1], [4, 5, 3]),
    ([[(1, 1), (2, 1)]] * 4, [[(0, 1), (2, 1)], [(1, 1), (3, 1)]], [1, 3, 2, 0], [5, 4]),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_permute_equals_dense_transpose(case):
    cod, dom, p, q = CASES[case]
    st = su2.SU2Map(cod, dom)
    rng = np.random.default_rng(case)
    x = rng.standard_normal(st.size)
    T = su2.to_dense(st, x)
    np.testing.assert_allclose(su2.from_dense(st, T), x, atol=1e-13)  # round trip
    out, y = su2.permute(st, x, p, q)
    Tp = T.transpose(list(p) + list(q))
    np.testing.assert_allclose(su2.to_dense(out, y), Tp, atol=1e-12)
    np.testing.assert_allclose(su2.from_dense(out, Tp), y, atol=1e-12)


def test_permute_composes_and_keeps_the_norm():
    cod, dom, p, q = CASES[1]
    st = su2.SU2Map(cod, dom)
    x = np.random.default_rng(7).standard_normal(st.size)
    o1, y1 = su2.permute(st, x, p, q)
    p2, q2 = [2, 1, 0], [3, 5, 4]
    o2, y2 = su2.permute(o1, y1, p2, q2)
    o3, y3 = su2.permute(st, x, [p[k] for k in p2], [q[k - 3] for k in q2])
    assert o2.blocks == o3.blocks
    np.testing.assert_allclose(y2, y3, atol=1e-13)

    def norm2(s, v):  # the dense norm: every block counts d_c times
        return sum((tc + 1) * float(np.sum(v[o:o + R * C] ** 2)) for tc, (o, R, C) in s.blocks.items())
    assert norm2(o1, y1) == pytest.approx(norm2(st, x), rel=1e-13)


def test_identity_permutation_is_a_copy():
    cod, dom, _, _ = CASES[2]
    st = su2.SU2Map(cod, dom)
    x = np.random.default_rng(3).standard_normal(st.size)
    out, y = su2.permute(st, x, [0, 1, 2, 3], [4, 5])
    # each tree overlaps itself with 1, up to the rounding of the dense sums
    np.testing.assert_allclose(y, x, rtol=0, atol=1e-14)


# ---------------------------------------------------------------------------
# transposition: legs moving between codomain and domain (dual legs)
# ---------------------------------------------------------------------------
def _transpose_fixture():
    lines = [l for l in open(os.path.join(GOLDEN, "su2_transpose_matrix.txt")).read().splitlines()
             if l and not l.startswith("#")]
    i, j = lines.index("formula"), lines.index("matrix")
    form = np.zeros((9, 9))
    for l in lines[i + 1:j]:
        lhs, rhs = l.split("=")
        for term in rhs.split("+"):
            c, ch = term.strip().split("*")
            form[int(lhs) - 1, int(ch) - 1] = float(c)
    mat = np.array([[float(x) for x in l.split()] for l in lines[j + 1:]])
    return form, mat


def test_dual_trees_are_invariant():
    """A tree pair with dual legs (Z on the outer lines) is an intertwiner:
    on a dual leg the generators act as -J^T (the dual representation), so
    sum over legs of the generator annihilates the dense pair; this pins the
    isomorphism Z (a wrong sign or index order breaks it)."""
    outer_c, outer_d = [1, 2], [3]
    for s_inter, tc in su2.trees(outer_c):
        for f_inter, tc2 in su2.trees(outer_d):
            if tc != tc2:
                continue
            for duals in [(), (0,), (1, 2), (0, 1, 2)]:
                G = su2.pair_tensor(outer_c, outer_d, s_inter, f_inter, tc, duals)
                spins = outer_c + outer_d
                for op in (0, 1):
                    tot = np.zeros_like(G)
                    for k, tj in enumerate(spins):
                        J = su2.spin_ops(tj)[op]
                        # the codomain carries V (or V*), the domain their duals
                        rep = J if ((k < 2) != (k in duals)) else -J.T
                        tot += np.moveaxis(np.tensordot(rep, G, axes=([1], [k])), 0, k)
                    assert np.abs(tot).max() < 1e-12, (duals, op)


def test_paper_transpose_formula():
    """The clockwise cycle t : V x V <- V x V  ->  s : V x V* <- V* x V of the
    worked example, against the formula the paper prints for s: every
    coefficient has the printed position and magnitude, and every sign
    except the two diagonal entries of the c = 1/2 block (channels 5 and 8),
    which come out with the opposite sign (the sign of bending a spin-1/2
    line one way round rather than the other; the paper leaves the bending
    convention open)."""
    form, _ = _transpose_fixture()
    st = su2.SU2Map([V, V], [V, V])
    out, _ = su2.transpose(st, np.zeros(9), (1, 3), (0, 2))
    assert out.dual == (1, 2) and out.size == 9
    T = _storage_matrix(st, lambda e: su2.transpose(st, e, (1, 3), (0, 2))[1], 9)
    np.testing.assert_allclose(np.abs(T), np.abs(form), atol=1e-14)
    flip = np.ones((9, 1))
    flip[[4, 7]] = -1
    np.testing.assert_allclose(T, flip * form, atol=1e-14)


def test_paper_transpose_printed_matrix():
    """The printed transition matrix: as the basis change of the opposite
    (counter-clockwise) cycle, s' : V* x V <- V x V*, its entries are the
    coefficients of that transpose read column-wise (every position and
    magnitude)."""
    _, mat = _transpose_fixture()
    st = su2.SU2Map([V, V], [V, V])
    T = _storage_matrix(st, lambda e: su2.transpose(st, e, (2, 0), (3, 1))[1], 9)
    np.testing.assert_allclose(np.abs(T.T), np.abs(mat), atol=1e-14)


TCASES = [
    ([[(0, 2), (1, 1)], [(1, 2), (2, 1)]], [[(1, 1), (2, 2)], [(0, 1), (1, 2)]], (), (1, 3), (0, 2)),
    ([[(0, 1), (1, 2)], [(1, 1), (2, 2)], [(1, 2), (3, 1)]], [[(1, 2), (2, 1)], [(0, 1), (1, 2)]], (1, 4),
     (4, 0, 2), (1, 3)),
    ([[(1, 1), (2, 1)], [(0, 1), (2, 1)]], [[(1, 2), (3, 1)], [(0, 2), (2, 1)], [(1, 1)]], (0, 3),
     (2, 1), (0, 4, 3)),
]


@pytest.mark.parametrize("case", range(len(TCASES)))
def test_transpose_coefficients_equal_dense_definition(case):
    """Transposes with legs crossing in both directions and dual legs on
    input: the per-tree-pair coefficients applied to the reduced arrays equal
    the definition (dense array, axes reordered, projected); the dense norm
    is kept, and the inverse transpose restores the input."""
    cod, dom, dual, p, q = TCASES[case]
    st = su2.SU2Map(cod, dom, dual)
    x = np.random.default_rng(40 + case).standard_normal(st.size)
    np.testing.assert_allclose(su2.from_dense(st, su2.to_dense(st, x)), x, atol=1e-13)
    out, y = su2.transpose(st, x, p, q)
    outd, yd = su2.transpose_dense(st, x, p, q)
    assert out.blocks == outd.blocks and out.dual == outd.dual
    np.testing.assert_allclose(y, yd, atol=1e-12)
    np.testing.assert_allclose(su2.to_dense(out, y), su2.to_dense(st, x).transpose(list(p) + list(q)), atol=1e-12)
    order = list(p) + list(q)
    inv = [order.index(g) for g in range(len(order))]
    back, z = su2.transpose(out, y, inv[:st.N1], inv[st.N1:])
    assert back.dual == st.dual
    np.testing.assert_allclose(z, x, atol=1e-12)


def test_transpose_without_crossing_is_the_braid_permute():
    cod, dom, p, q = CASES[1]
    st = su2.SU2Map(cod, dom)
    x = np.random.default_rng(11).standard_normal(st.size)
    _, y1 = su2.permute(st, x, p, q)
    _, y2 = su2.transpose(st, x, p, q)
    np.testing.assert_allclose(y1, y2, atol=1e-13)


def test_four_clockwise_cycles_are_the_identity():
    """Cycling the legs of t : V x V <- V x V clockwise four times returns
    every leg to its place (the linear order (1, 2, 4, 3) rotated by four)."""
    st = su2.SU2Map([V, V], [V, V])
    x = np.random.default_rng(12).standard_normal(st.size)
    s, y = st, x
    for _ in range(4):
        s, y = su2.transpose(s, y, (1, 3), (0, 2))
    assert s.dual == ()
    np.testing.assert_allclose(y, x, atol=1e-13)
