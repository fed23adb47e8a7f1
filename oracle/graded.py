"""Sectors, graded spaces and the block storage layout of a TensorMap (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Symmetries
----------
Z1      no symmetry: every space has the single trivial sector ().
Z2      bosonic Z2: sectors (p,), p in {0, 1}, fusion p xor p'; the worked
        example of the abelian grouping section uses it.
FZ2     fermion parity (the category SVect of section "Fermions and fusion
        categories"): sectors (p,), J = (1,) is the odd object, J x J = I.
U1      U(1) charges (q,), fusion q + q', dual -q (abelian group irreps are
        one-dimensional, N^{ab}_c = delta_{c, ab}).
U1xFZ2  Deligne product Rep U(1) x SVect (section "Deligne Product
        Categories"): sectors (q, p), componentwise fusion; the braiding sign
        is the product of the components' R-symbols, i.e. the SVect one.

Leg labels
----------
A leg stores the sectors of its underlying space plus a dual flag.  The
charge used for block keys and charge conservation is the sector itself on a
normal space and its conjugate on a dual space (a dual graded space is graded
by the conjugate irreps and its pairing is diagonal in the charges, section
"Transpositions" of the abelian chapter).  Conservation for a map
W_1..W_N2 -> V_1..V_N1 is  fuse(labels of the codomain) == fuse(labels of the
domain)  (eq. abeliantensorzeros).

Storage layout (reading of eq. abeliangrouping, whose channel order is left
"arbitrary but fixed")
----------------------------------------------------------------------------
* Coupled charges c present on both sides are stored one after the other in
  ascending tuple order; each as an R_c x C_c column-major matrix.
* The rows of t^(c) are the codomain channels (tuples of sector indices, one
  per leg, with fused label c), enumerated with the FIRST leg varying fastest
  (the column-major rule of eq. linearindex applied to sector indices); each
  channel contributes prod(degeneracies) rows.  Columns likewise for the
  domain.  The worked Z2 example of the grouping section fixes this order:
  t^(+) has rows/cols (++, --) and t^(-) has rows/cols (-+, +-).
* Inside a channel the entries are ordered by eq. linearindex (first index
  fastest) on each side: element (i_1..i_N1; j_1..j_N2) of channel block
  (a; b) sits at  sector_offset + (col_off(b) + lin(j)) * R_c + row_off(a) +
  lin(i).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SYMMETRIES = ("Z1", "Z2", "FZ2", "U1", "U1xFZ2")
_NCOMP = {"Z1": 0, "Z2": 1, "FZ2": 1, "U1": 1, "U1xFZ2": 2}


def ncomp(sym: str) -> int:
    return _NCOMP[sym]


def is_fermionic(sym: str) -> bool:
    """SVect and products with it carry R^{JJ}_I = -1."""
    return sym in ("FZ2", "U1xFZ2")


def unit(sym: str) -> tuple:
    return (0,) * _NCOMP[sym]


def fuse(sym: str, a: tuple, b: tuple) -> tuple:
    if sym == "Z1":
        return ()
    if sym in ("Z2", "FZ2"):
        return ((a[0] + b[0]) % 2,)
    if sym == "U1":
        return (a[0] + b[0],)
    return (a[0] + b[0], (a[1] + b[1]) % 2)


def conj(sym: str, a: tuple) -> tuple:
    """Dual irrep: U(1) charge q -> -q; Z2 / parity labels are self-dual."""
    if sym == "U1":
        return (-a[0],)
    if sym == "U1xFZ2":
        return (-a[0], a[1])
    return tuple(a)


def fparity(sym: str, a: tuple) -> int:
    """Fermion parity |a| (0 for bosonic symmetries)."""
    if sym == "FZ2":
        return a[0]
    if sym == "U1xFZ2":
        return a[1]
    return 0


def valid_sector(sym: str, a: tuple) -> bool:
    if len(a) != _NCOMP[sym]:
        return False
    if sym in ("Z2", "FZ2"):
        return a[0] in (0, 1)
    if sym == "U1xFZ2":
        return a[1] in (0, 1)
    return True


@dataclass(frozen=True)
class Space:
    """Graded space  (+)_a C^{N_a} (x) V^(a)  with a dual flag."""
    sectors: tuple
    degs: tuple
    dual: bool = False

    def __post_init__(self):
        object.__setattr__(self, "sectors", tuple(tuple(int(x) for x in s) for s in self.sectors))
        object.__setattr__(self, "degs", tuple(int(d) for d in self.degs))
        if len(self.sectors) != len(self.degs):
            raise ValueError("sectors and degeneracies differ in length")
        if len(set(self.sectors)) != len(self.sectors):
            raise ValueError("repeated sector")
        if any(d <= 0 for d in self.degs):
            raise ValueError("degeneracies must be positive")

    @property
    def dim(self) -> int:
        return int(sum(self.degs))

    def flip(self) -> "Space":
        return Space(self.sectors, self.degs, not self.dual)

    def label(self, sym: str, k: int) -> tuple:
        s = self.sectors[k]
        return conj(sym, s) if self.dual else s

    def starts(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.degs)[:-1]]).astype(np.int64)

    def sector_of_index(self) -> np.ndarray:
        """Dense index -> sector index (sectors listed in order, each
        contiguous over its degeneracy)."""
        return np.repeat(np.arange(len(self.degs)), self.degs)

    def parity_of_index(self, sym: str) -> np.ndarray:
        par = np.array([fparity(sym, s) for s in self.sectors], dtype=np.int64)
        return np.repeat(par, self.degs)


def check_space(sym: str, sp: Space):
    for s in sp.sectors:
        if not valid_sector(sym, s):
            raise ValueError(f"sector {s} invalid for {sym}")


def _label_arrays(sym: str, sp: Space) -> np.ndarray:
    """(nsect, ncomp) effective labels of one leg."""
    return np.array([sp.label(sym, k) for k in range(len(sp.sectors))],
                    dtype=np.int64).reshape(len(sp.sectors), _NCOMP[sym])


def enumerate_side(sym: str, spaces):
    """All sector-index tuples of one side, first leg fastest.

    Returns (idx (n, N) int64, labels (n, ncomp) int64, size (n,) int64)
    where size is the product of the degeneracies."""
    N = len(spaces)
    if N == 0:
        return (np.zeros((1, 0), np.int64), np.zeros((1, _NCOMP[sym]), np.int64),
                np.ones(1, np.int64))
    shape = tuple(len(sp.sectors) for sp in spaces)
    # np.indices in Fortran order = colexicographic = first leg fastest.
    idx = np.indices(shape).reshape(N, -1, order="F").T.astype(np.int64)
    lab = np.zeros((idx.shape[0], _NCOMP[sym]), np.int64)
    size = np.ones(idx.shape[0], np.int64)
    for leg, sp in enumerate(spaces):
        la = _label_arrays(sym, sp)[idx[:, leg]]
        lab += la
        size *= np.asarray(sp.degs, np.int64)[idx[:, leg]]
    if sym in ("Z2", "FZ2"):
        lab[:, 0] %= 2
    elif sym == "U1xFZ2":
        lab[:, 1] %= 2
    return idx, lab, size


@dataclass
class SideGroup:
    idx: np.ndarray      # (n, N) sector indices of the channels with this label
    size: np.ndarray     # (n,) entries per channel on this side
    off: np.ndarray      # (n,) row (or column) offset inside t^(c)
    total: int           # R_c (or C_c)


def group_side(sym: str, spaces) -> dict:
    idx, lab, size = enumerate_side(sym, spaces)
    out = {}
    if lab.shape[1] == 0:
        keys = [()] * idx.shape[0]
        uniq = [()]
        inv = np.zeros(idx.shape[0], np.int64)
    else:
        uniq_arr, inv = np.unique(lab, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        uniq = [tuple(int(x) for x in u) for u in uniq_arr]
    for gi, key in enumerate(uniq):
        sel = np.nonzero(inv == gi)[0]          # keeps colex order
        sz = size[sel]
        off = np.concatenate([[0], np.cumsum(sz)[:-1]]).astype(np.int64)
        out[key] = SideGroup(idx[sel], sz, off, int(sz.sum()))
    return out


class Structure:
    """Block structure of a TensorMap  W_1..W_N2 -> V_1..V_N1."""

    def __init__(self, sym: str, cod, dom):
        if sym not in SYMMETRIES:
            raise ValueError(sym)
        self.sym = sym
        self.cod = tuple(cod)
        self.dom = tuple(dom)
        for sp in self.cod + self.dom:
            check_space(sym, sp)
        self.rows = group_side(sym, self.cod)
        self.cols = group_side(sym, self.dom)
        self.sectors = sorted(k for k in self.rows if k in self.cols)
        self.sector_offset = {}
        off = 0
        for c in self.sectors:
            self.sector_offset[c] = off
            off += self.rows[c].total * self.cols[c].total
        self.size = off

    @property
    def N1(self):
        return len(self.cod)

    @property
    def N2(self):
        return len(self.dom)

    def spaces(self):
        return self.cod + self.dom

    def degs(self, leg: int) -> np.ndarray:
        return np.asarray(self.spaces()[leg].degs, np.int64)

    def channels(self):
        """Yield (c, cod_tuple, dom_tuple, offset_of_block, R_c) in storage
        order: sector by sector, columns outer, rows inner."""
        for c in self.sectors:
            rg, cg = self.rows[c], self.cols[c]
            base = self.sector_offset[c]
            for j in range(len(cg.size)):
                for i in range(len(rg.size)):
                    yield (c, tuple(int(x) for x in rg.idx[i]), tuple(int(x) for x in cg.idx[j]),
                           base + int(cg.off[j]) * rg.total + int(rg.off[i]), rg.total)

    def block_dims(self, cod_t, dom_t):
        sp = self.spaces()
        t = tuple(cod_t) + tuple(dom_t)
        return tuple(sp[l].degs[t[l]] for l in range(len(t)))

    # -- storage <-> blocks -------------------------------------------------
    def to_blocks(self, vec: np.ndarray) -> dict:
        vec = np.asarray(vec)
        if vec.shape != (self.size,):
            raise ValueError(f"storage has {vec.shape}, expected ({self.size},)")
        out = {}
        for c, a, b, off, R in self.channels():
            dims = self.block_dims(a, b)
            r = int(np.prod(dims[:self.N1], dtype=np.int64))
            cc = int(np.prod(dims[self.N1:], dtype=np.int64))
            # rows off..off+r of columns spaced by R  (column-major t^(c))
            cols = [vec[off + j * R: off + j * R + r] for j in range(cc)]
            mat = np.stack(cols, axis=1) if cc else np.zeros((r, 0), vec.dtype)
            out[(a, b)] = mat.reshape(dims, order="F")
        return out

    def from_blocks(self, blocks: dict, dtype=np.float64) -> np.ndarray:
        vec = np.zeros(self.size, dtype)
        for c, a, b, off, R in self.channels():
            blk = blocks.get((a, b))
            if blk is None:
                continue
            dims = self.block_dims(a, b)
            r = int(np.prod(dims[:self.N1], dtype=np.int64))
            cc = int(np.prod(dims[self.N1:], dtype=np.int64))
            mat = np.asarray(blk).reshape((r, cc), order="F")
            for j in range(cc):
                vec[off + j * R: off + j * R + r] = mat[:, j]
        return vec

    # -- storage <-> dense ----------------------------------------------------
    def dense_shape(self):
        return tuple(sp.dim for sp in self.spaces())

    def to_dense(self, vec: np.ndarray) -> np.ndarray:
        """Expand to the dense array t_{i_1..i_N1; j_1..j_N2}; entries outside
        every fusion channel are zero (eq. abeliantensorzeros)."""
        T = np.zeros(self.dense_shape(), np.asarray(vec).dtype)
        starts = [sp.starts() for sp in self.spaces()]
        sp = self.spaces()
        for (a, b), blk in self.to_blocks(vec).items():
            t = a + b
            sl = tuple(slice(starts[l][t[l]], starts[l][t[l]] + sp[l].degs[t[l]]) for l in range(len(t)))
            T[sl] = blk
        return T

    def allowed_mask(self) -> np.ndarray:
        """Boolean dense mask of entries that belong to a stored channel."""
        return self.to_dense(np.ones(self.size)) != 0

    def from_dense(self, T: np.ndarray, check_zero: bool = True) -> np.ndarray:
        T = np.asarray(T)
        if T.shape != self.dense_shape():
            raise ValueError("dense shape mismatch")
        if check_zero:
            mask = self.allowed_mask()
            bad = np.abs(T[~mask]).max() if (~mask).any() else 0.0
            if bad != 0:
                raise ValueError(f"dense tensor violates charge conservation (|x|={bad})")
        starts = [sp.starts() for sp in self.spaces()]
        sp = self.spaces()
        blocks = {}
        for c, a, b, off, R in self.channels():
            t = a + b
            sl = tuple(slice(starts[l][t[l]], starts[l][t[l]] + sp[l].degs[t[l]]) for l in range(len(t)))
            blocks[(a, b)] = T[sl]
        return self.from_blocks(blocks, T.dtype)

    # -- sector matrices ------------------------------------------------------
    def sector_matrix(self, vec: np.ndarray, c) -> np.ndarray:
        off = self.sector_offset[c]
        R, C = self.rows[c].total, self.cols[c].total
        return np.asarray(vec)[off:off + R * C].reshape((R, C), order="F")


def permute_spaces(cod, dom, p, q):
    """Space assignment of Alg. "Tensor Permute" (and its abelian form):
    V'_i = p_i-th space of (V_1.., W_1*..);  W'_j = q_j-th of (V_1*.., W_1..).
    Legs are 0-based here; the paper counts from 1."""
    cod, dom = tuple(cod), tuple(dom)
    N1 = len(cod)
    allsp = cod + dom
    p, q = tuple(p), tuple(q)
    if sorted(p + q) != list(range(len(allsp))):
        raise ValueError("(p, q) is not a permutation of the legs")
    ncod = tuple(allsp[i] if i < N1 else allsp[i].flip() for i in p)
    ndom = tuple(allsp[i].flip() if i < N1 else allsp[i] for i in q)
    return ncod, ndom


def linearized_order(N1: int, N2: int):
    """Legs in bra-ket order: codomain first, domain reversed
    (t in V_1..V_N1 (x) W*_N2 .. W*_1, eq. homtobraket)."""
    return list(range(N1)) + list(range(N1 + N2 - 1, N1 - 1, -1))
