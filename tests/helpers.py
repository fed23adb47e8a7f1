"""Glue between the seeded workload descriptions and the oracle / library."""
from __future__ import annotations

import itertools

import numpy as np

from oracle import blockwise
from oracle.graded import Space, Structure, permute_spaces
from paper_2508_10076_amd import synth


def ospace(spec) -> Space:
    return Space(spec.sectors, spec.degs, spec.dual)


def ostruct(t: dict) -> Structure:
    return Structure(t["sym"], [ospace(s) for s in t["cod"]], [ospace(s) for s in t["dom"]])


Z2_LABEL = {"+": (0,), "-": (1,)}


def read_golden(name: str):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    lines = []
    with open(path) as fh:
        for ln in fh:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                lines.append(ln.split())
    return lines


def brute_channels(sym_fuse, unit, spaces_cod, spaces_dom, label):
    """Fusion channels by brute force over every sector tuple (pure Python)."""
    out = []
    cod_t = list(itertools.product(*[range(len(s.sectors)) for s in spaces_cod]))
    dom_t = list(itertools.product(*[range(len(s.sectors)) for s in spaces_dom]))
    for a in cod_t:
        la = unit
        for l, k in enumerate(a):
            la = sym_fuse(la, label(spaces_cod[l], k))
        for b in dom_t:
            lb = unit
            for l, k in enumerate(b):
                lb = sym_fuse(lb, label(spaces_dom[l], k))
            if la == lb:
                out.append((la, a, b))
    return out


def int_data(n, rng, lo=-3, hi=3):
    return rng.integers(lo, hi + 1, size=n).astype(np.float64)


def trace_case(rng, sym: str, npairs: int = 1, max_free: int = 3):
    """A random tensor with npairs traceable leg pairs (each a vector /
    co-vector pair over one space: a codomain and a domain leg over X, or X
    and X* on the same side) plus up to max_free free legs, and a random
    arrangement of the free legs.  Returns (tensor dict, p, q, t1, t2)."""
    from paper_2508_10076_amd import synth
    while True:
        cod, dom, pairs = [], [], []
        for _ in range(npairs):
            X = synth.random_space(rng, sym, max_deg=3)
            kind = int(rng.integers(0, 3))
            if kind == 0:
                cod.append(("t", X)), dom.append(("t", X))
            elif kind == 1:
                cod.append(("t", X)), cod.append(("t", synth.dual(X)))
            else:
                dom.append(("t", X)), dom.append(("t", synth.dual(X)))
            pairs.append(kind)
        for _ in range(int(rng.integers(0, max_free + 1))):
            (cod if rng.random() < 0.5 else dom).append(("f", synth.random_space(rng, sym, max_deg=3)))
        if len(cod) > 4 or len(dom) > 4:
            continue
        cod = [cod[i] for i in rng.permutation(len(cod))] if cod else cod
        dom = [dom[i] for i in rng.permutation(len(dom))] if dom else dom
        legs = cod + dom
        # pair the traced legs: an X leg with its partner (same space, opposite reading)
        used, t1, t2 = set(), [], []
        for a in range(len(legs)):
            if legs[a][0] != "t" or a in used:
                continue
            for b in range(a + 1, len(legs)):
                if legs[b][0] != "t" or b in used:
                    continue
                A, B = legs[a][1], legs[b][1]
                if A.sectors != B.sectors or A.degs != B.degs:
                    continue
                da = A.dual != (a >= len(cod))
                db = B.dual != (b >= len(cod))
                if da != db:
                    used |= {a, b}
                    t1.append(a)
                    t2.append(b)
                    break
        if len(t1) != npairs:
            continue
        free = [l for l in range(len(legs)) if l not in used]
        free = [free[i] for i in rng.permutation(len(free))] if free else free
        n1 = int(rng.integers(0, len(free) + 1))
        t = dict(sym=sym, cod=[s for _, s in cod], dom=[s for _, s in dom])
        if ostruct(t).size == 0:
            continue
        return t, tuple(free[:n1]), tuple(free[n1:]), tuple(t1), tuple(t2)


def wide_n_case(rng, sym):
    """Small K (<= 8 per sector) against free legs of B wide enough that the
    sectors have well over 64 columns (output-stationary small-K path)."""
    while True:
        kl = synth.random_space(rng, sym, max_deg=2)
        tA = dict(sym=sym, cod=[synth.random_space(rng, sym, max_deg=3) for _ in range(2)], dom=[kl])
        wide = [synth.random_space(rng, sym, max_sect=3, max_deg=4) for _ in range(2)]
        wide = [synth.space(w.sectors, [d + 8 for d in w.degs], w.dual) for w in wide]
        tB = dict(sym=sym, cod=[synth.SpaceSpec(kl.sectors, kl.degs, kl.dual)], dom=wide)
        if not (ostruct(tA).size and ostruct(tB).size):
            continue
        oc = [int(x) for x in rng.permutation(4)]
        n1 = int(rng.integers(0, 5))
        return tA, (0, 1), (2,), tB, (0,), (1, 2), oc[:n1], oc[n1:]


def random_tdict(rng, sym, n1, n2, **kw):
    while True:
        t = dict(sym=sym, cod=[synth.random_space(rng, sym, **kw) for _ in range(n1)],
                 dom=[synth.random_space(rng, sym, **kw) for _ in range(n2)])
        if ostruct(t).size:
            return t


def plan_case(rng, sym, max_deg=3):
    """A random valid contraction: A over 1-2 + 1-2 random legs, contracted
    over a random subset, B built around the contracted spaces with 0-2 free
    legs, random leg orders and codomain / domain splits for B~ and C."""
    while True:
        tA = random_tdict(rng, sym, int(rng.integers(1, 3)), int(rng.integers(1, 3)), max_deg=max_deg)
        stA = ostruct(tA)
        nA = stA.N1 + stA.N2
        k = int(rng.integers(1, nA + 1))
        legs = [int(x) for x in rng.permutation(nA)]
        qA, pA = legs[:k], legs[k:]
        _, Adom = permute_spaces(stA.cod, stA.dom, pA, qA)
        free = [synth.random_space(rng, sym, max_deg=max_deg) for _ in range(int(rng.integers(0, 3)))]
        Bt = dict(sym=sym, cod=[synth.SpaceSpec(s.sectors, s.degs, s.dual) for s in Adom], dom=free)
        stBt = ostruct(Bt)
        if not stBt.size:
            continue
        nB = k + len(free)
        order = [int(x) for x in rng.permutation(nB)]
        n1B = int(rng.integers(0, nB + 1))
        stB, _ = blockwise.permute(stBt, {}, order[:n1B], order[n1B:])
        inv = [0] * nB
        for n, l in enumerate(order):
            inv[l] = n
        pB, qB = inv[:k], inv[k:]
        tB = dict(sym=sym, cod=[synth.SpaceSpec(s.sectors, s.degs, s.dual) for s in stB.cod],
                  dom=[synth.SpaceSpec(s.sectors, s.degs, s.dual) for s in stB.dom])
        if not stB.size:
            continue
        nC = len(pA) + len(qB)
        oc = [int(x) for x in rng.permutation(nC)]
        n1C = int(rng.integers(0, nC + 1))
        return tA, pA, qA, tB, pB, qB, oc[:n1C], oc[n1C:]
