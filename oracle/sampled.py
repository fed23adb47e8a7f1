"""TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Oracle pieces for sizes at which the whole-tensor oracles are too slow:

* `codomain_channels`: the storage layout of a tensor whose legs all sit in
  the codomain (a single coupled sector, the unit): its fusion channels in
  storage order with their sizes and offsets (eq. abeliangrouping and the
  column-major block rule; channels ordered colexicographically, first leg
  fastest).  Built by enumerating the first and the second half of the legs
  separately and pairing halves whose labels fuse to the unit, instead of
  enumerating every sector tuple of all legs.
* `graph_entries`: selected entries of a network evaluated as a graph
  (section "Fermionic tensor networks"; pushed-twist semantics): outer
  product of the tensors in bra-ket (linearized) order, Koszul sign of the
  reordering that brings every contracted pair together (dual-in-linearized-
  order leg first) followed by the free legs in the output's linearized
  order, and the pairing of each contracted pair -- summed over the values
  of the contracted indices, one output entry at a time.
"""
from __future__ import annotations

import itertools

import numpy as np

from .graded import Space, conj, enumerate_side, is_fermionic, linearized_order


def codomain_channels(sym: str, spaces):
    """Channels of W <- V_1..V_N (N2 = 0) in storage order.

    Returns (idx (n, N) sector indices, size (n,), off (n,) storage offset).
    """
    spaces = tuple(spaces)
    N = len(spaces)
    h = N // 2
    i1, l1, s1 = enumerate_side(sym, spaces[:h])
    i2, l2, s2 = enumerate_side(sym, spaces[h:])
    n1 = i1.shape[0]                     # rows of enumerate_side are in colex order
    by_label = {}
    for r, lab in enumerate(map(tuple, l1.tolist())):
        by_label.setdefault(lab, []).append(r)
    by_label = {k: np.asarray(v, np.int64) for k, v in by_label.items()}
    keys, sizes, r1s, r2s = [], [], [], []
    for r2, lab in enumerate(map(tuple, l2.tolist())):
        need = conj(sym, lab) if lab else ()       # the first half must cancel this label
        r1 = by_label.get(tuple(need))
        if r1 is None:
            continue
        r1s.append(r1)
        r2s.append(np.full(r1.shape, r2, np.int64))
    if not r1s:
        return np.zeros((0, N), np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64)
    r1 = np.concatenate(r1s)
    r2 = np.concatenate(r2s)
    key = r1 + n1 * r2                   # colex key over all N legs
    order = np.argsort(key, kind="stable")
    r1, r2 = r1[order], r2[order]
    idx = np.concatenate([i1[r1], i2[r2]], axis=1)
    size = s1[r1] * s2[r2]
    off = np.concatenate([[0], np.cumsum(size)[:-1]]).astype(np.int64)
    return idx, size, off


def positions_to_dense(spaces, idx, size, off, pos):
    """Storage positions -> dense index tuples (n, N) for the layout of
    `codomain_channels` (inside a channel: colex over the legs' local
    indices, first leg fastest)."""
    spaces = tuple(spaces)
    pos = np.asarray(pos, np.int64)
    ch = np.searchsorted(off, pos, side="right") - 1
    local = pos - off[ch]
    out = np.zeros((pos.shape[0], len(spaces)), np.int64)
    for leg, sp in enumerate(spaces):
        degs = np.asarray(sp.degs, np.int64)
        d = degs[idx[ch, leg]]
        out[:, leg] = sp.starts()[idx[ch, leg]] + local % d
        local //= d
    return out


def dense_to_positions(sym: str, spaces, idx, size, off, dense):
    """Dense index tuples -> storage positions, or -1 where the tuple lies in
    no channel (a structurally zero entry)."""
    spaces = tuple(spaces)
    dense = np.asarray(dense, np.int64)
    nl = [len(sp.sectors) for sp in spaces]
    sec = np.stack([sp.sector_of_index()[dense[:, l]] for l, sp in enumerate(spaces)], axis=1)
    key_all = np.zeros(dense.shape[0], np.int64)
    key_ch = np.zeros(idx.shape[0], np.int64)
    mul = 1
    for l in range(len(spaces)):
        key_all += sec[:, l] * mul
        key_ch += idx[:, l] * mul
        mul *= nl[l]
    j = np.searchsorted(key_ch, key_all)
    j = np.minimum(j, max(0, key_ch.shape[0] - 1))
    found = (key_ch.shape[0] > 0) & (key_ch[j] == key_all)
    local = np.zeros(dense.shape[0], np.int64)
    mul = np.ones(dense.shape[0], np.int64)
    for l, sp in enumerate(spaces):
        degs = np.asarray(sp.degs, np.int64)
        d = degs[sec[:, l]]
        local += (dense[:, l] - sp.starts()[sec[:, l]]) * mul
        mul *= d
    return np.where(found, off[j] + local, -1)


def _lin_dual(sp: Space, in_domain: bool) -> bool:
    return bool(sp.dual) ^ bool(in_domain)


def graph_output_spaces(tensor_spaces, out_cod, out_dom):
    """Spaces of the network's output legs: a free leg keeps its space, with
    the dual flag it has in linearized order (flipped again for the output's
    domain)."""
    info = {}
    for ti, (cod, dom) in enumerate(tensor_spaces):
        sp = tuple(cod) + tuple(dom)
        for l in range(len(sp)):
            info[(ti, l)] = (sp[l], _lin_dual(sp[l], l >= len(cod)))
    ocod = tuple(Space(info[k][0].sectors, info[k][0].degs, info[k][1]) for k in out_cod)
    odom = tuple(Space(info[k][0].sectors, info[k][0].degs, not info[k][1]) for k in out_dom)
    return ocod, odom


def graph_entries(sym: str, tensors, pairs, out_cod, out_dom, out_index):
    """Entries of the graph value at the output index tuples `out_index`
    ((S, n_out), axes out_cod then out_dom).

    tensors : list of (T dense, cod spaces, dom spaces)
    pairs   : list of ((t, leg), (t', leg')) contracted with each other
    """
    out_index = np.asarray(out_index, np.int64)
    legs, info = [], {}
    for ti, (T, cod, dom) in enumerate(tensors):
        N1, N2 = len(cod), len(dom)
        sp = tuple(cod) + tuple(dom)
        for l in linearized_order(N1, N2):
            legs.append((ti, l))
            info[(ti, l)] = dict(space=sp[l], lin_dual=_lin_dual(sp[l], l >= N1),
                                 par=sp[l].parity_of_index(sym))
    target = []
    for x, y in pairs:
        if info[x]["lin_dual"] == info[y]["lin_dual"]:
            raise ValueError("contracted legs must be a vector / co-vector pair")
        target += [x, y] if info[x]["lin_dual"] else [y, x]
    target += list(out_cod) + list(reversed(list(out_dom)))
    tpos = {k: i for i, k in enumerate(target)}
    exchanged = []
    if is_fermionic(sym):
        for i, x in enumerate(legs):
            for y in legs[i + 1:]:
                if tpos[x] > tpos[y]:
                    exchanged.append((x, y))
    S = out_index.shape[0]
    value = {}
    for n, k in enumerate(list(out_cod) + list(out_dom)):
        value[k] = out_index[:, n]
    total = np.zeros(S, np.result_type(*[T.dtype for T, _, _ in tensors]))
    ranges = [range(info[x]["space"].dim) for x, _ in pairs]
    for combo in itertools.product(*ranges):
        for (x, y), v in zip(pairs, combo):
            value[x] = np.full(S, v, np.int64)
            value[y] = value[x]
        term = np.ones(S, total.dtype)
        for ti, (T, cod, dom) in enumerate(tensors):
            term = term * T[tuple(value[(ti, l)] for l in range(T.ndim))]
        par = np.zeros(S, np.int64)
        for x, y in exchanged:
            par += info[x]["par"][value[x]] * info[y]["par"][value[y]]
        total += np.where(par % 2 == 1, -term, term)
    return total
