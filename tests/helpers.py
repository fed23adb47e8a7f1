"""Glue between the seeded workload descriptions and the oracle / library."""
from __future__ import annotations

import itertools

import numpy as np

from oracle.graded import Space, Structure


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
