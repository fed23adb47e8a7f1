"""Seeded synthetic workloads (spaces, contraction calls, random data).

This module is the only code shared by the tests' oracle side and the HIP
side.  It holds no arithmetic of the method: it only describes graded spaces
as plain (sectors, degeneracies, dual) data, names the contraction calls of
each workload, and draws random numbers.  Storage vectors are drawn as flat
arrays whose length the caller takes from the tensor's block structure, so
the oracle and the library each interpret the same numbers through their own
layout code.

The paper benchmarks DMRG effective-Hamiltonian applications on spaces that
it takes from converged MPSKit ground states; those are not available, so
Gaussian charge profiles of the same total dimension stand in for them.
"""
from __future__ import annotations

from collections import namedtuple

import numpy as np

SpaceSpec = namedtuple("SpaceSpec", "sectors degs dual")
SEED_BASE = 250810076


def space(sectors, degs, dual=False) -> SpaceSpec:
    return SpaceSpec(tuple(tuple(int(x) for x in s) for s in sectors), tuple(int(d) for d in degs), bool(dual))


def dual(sp: SpaceSpec) -> SpaceSpec:
    return SpaceSpec(sp.sectors, sp.degs, not sp.dual)


def rng(config: int, stream: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE + config, stream])


def gaussian_degeneracies(D: int, qmax: int, sigma: float, floor: int = 1):
    """Degeneracies over charges -qmax..qmax with deg(q) ~ exp(-q^2/2 sigma^2):
    shares of D rounded by largest remainder to sum exactly to D (ties:
    smaller |q|, then smaller q); a charge left below `floor` is raised to it
    and the excess is taken from the largest degeneracies."""
    qs = np.arange(-qmax, qmax + 1)
    n = len(qs)
    if D < floor * n:
        raise ValueError("D too small for the floor")
    w = np.exp(-qs.astype(float) ** 2 / (2.0 * sigma * sigma))
    share = w / w.sum() * D
    degs = np.floor(share).astype(np.int64)
    frac = share - degs
    left = D - int(degs.sum())
    order = sorted(range(n), key=lambda i: (-frac[i], abs(qs[i]), qs[i]))
    for i in order[:left]:
        degs[i] += 1
    excess = int(np.maximum(floor - degs, 0).sum())
    degs = np.maximum(degs, floor)
    while excess > 0:
        i = max(range(n), key=lambda j: (degs[j], -abs(qs[j]), -qs[j]))
        degs[i] -= 1
        excess -= 1
    assert int(degs.sum()) == D
    return [int(q) for q in qs], [int(d) for d in degs]


def u1_space(charges, degs, dual_=False) -> SpaceSpec:
    return space([(q,) for q in charges], degs, dual_)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
P_U1 = u1_space([0, 1], [1, 1])
WM_U1 = u1_space([-1, 0, 1], [1, 3, 1])


def config1(seed_stream: int = 0):
    """U(1) A[l,p,m] . B[m,q,r] over m; virtual charges -2..2 with
    degeneracies drawn from U{2..10}."""
    g = rng(1, seed_stream)
    degs = [int(x) for x in g.integers(2, 11, size=5)]
    V = u1_space(range(-2, 3), degs)
    A = dict(sym="U1", cod=(V, P_U1), dom=(V,))
    B = dict(sym="U1", cod=(V, P_U1), dom=(V,))
    call = dict(pA=(0, 1), qA=(2,), pB=(0,), qB=(1, 2), pAB=(0, 1), qAB=(2, 3))
    return dict(name="u1_rank3_pair", tensors=dict(A=A, B=B), calls=[("C", "A", "B", call)])


def heff_spaces(D: int, qmax: int, sigma: float):
    q, d = gaussian_degeneracies(D, qmax, sigma)
    V = u1_space(q, d)
    x = dict(sym="U1", cod=(V, P_U1), dom=(V,))
    L = dict(sym="U1", cod=(V,), dom=(V, WM_U1))
    W = dict(sym="U1", cod=(WM_U1, P_U1), dom=(P_U1, WM_U1))
    R = dict(sym="U1", cod=(WM_U1, V), dom=(V,))
    return V, dict(x=x, L=L, W=W, R=R)


HEFF_CALLS = [
    ("T1", "L", "x", dict(pA=(0, 2), qA=(1,), pB=(0,), qB=(1, 2), pAB=(0, 3), qAB=(1, 2))),
    ("T2", "T1", "W", dict(pA=(0, 1), qA=(2, 3), pB=(0, 2), qB=(1, 3), pAB=(0, 2), qAB=(3, 1))),
    ("y", "T2", "R", dict(pA=(0, 1), qA=(2, 3), pB=(0, 1), qB=(2,), pAB=(0, 1), qAB=(2,))),
]


def heff_config(D: int, qmax: int, sigma: float, config_id: int):
    """Single-site effective Hamiltonian  y = L . W . x . R  (Alg.
    "Single-site Benchmark") as three pairwise contractions."""
    V, t = heff_spaces(D, qmax, sigma)
    return dict(name=f"heff_u1_D{D}", config=config_id, tensors=t, calls=HEFF_CALLS,
                inputs=("x", "L", "W", "R"), output="y")


# Two-site H_eff: x2[a', p1'; b', p2'] with the second physical leg in the
# domain as P* (type V x P <- V x P*), contracted with L, W twice and R.
HEFF2_CALLS = [
    ("T1", "L", "x", dict(pA=(0, 2), qA=(1,), pB=(0,), qB=(1, 2, 3), pAB=(0, 3, 4), qAB=(1, 2))),
    ("T2", "T1", "W", dict(pA=(0, 1, 2), qA=(3, 4), pB=(0, 2), qB=(1, 3), pAB=(0, 3, 1), qAB=(4, 2))),
    ("T3", "T2", "W", dict(pA=(0, 1, 2), qA=(3, 4), pB=(0, 2), qB=(1, 3), pAB=(0, 1, 3), qAB=(4, 2))),
    ("y", "T3", "R", dict(pA=(0, 1, 2), qA=(3, 4), pB=(0, 1), qB=(2,), pAB=(0, 1), qAB=(3, 2))),
]


def heff2_spaces(D: int, qmax: int, sigma: float):
    V, t = heff_spaces(D, qmax, sigma)
    t = dict(t)
    t["x"] = dict(sym="U1", cod=(V, P_U1), dom=(V, dual(P_U1)))
    return V, t


def heff2_config(D: int, qmax: int, sigma: float, config_id: int):
    """Two-site effective Hamiltonian  y = L . W . W . x2 . R  (Alg.
    "Two-site Benchmark"; x2 : V x P <- V x P*) as four pairwise
    contractions."""
    V, t = heff2_spaces(D, qmax, sigma)
    return dict(name=f"heff2_u1_D{D}", config=config_id, tensors=t, calls=HEFF2_CALLS,
                inputs=("x", "L", "W", "R"), output="y")


def config2():
    return heff_config(1024, 8, 3.0, 2)


def config3():
    return heff_config(4096, 12, 4.5, 3)


def config4(n: int = 64, dmin: int = 256, dmax: int = 2048):
    """Batch of n independent U(1) rank-3 x rank-4 contractions
    C_i = A_i[a; a', w] . B_i[a', w, p; b] with uneven sector structures."""
    g = rng(4, 0)
    items = []
    for i in range(n):
        D = int(g.integers(dmin, dmax + 1))
        qr = int(g.integers(4, 11))
        sigma = 3.0 * qr / 8.0
        q, d = gaussian_degeneracies(D, qr, sigma)
        V = u1_space(q, d)
        A = dict(sym="U1", cod=(V,), dom=(V, WM_U1))
        B = dict(sym="U1", cod=(V, WM_U1, P_U1), dom=(V,))
        items.append(dict(D=D, qmax=qr, A=A, B=B))
    call = dict(pA=(0,), qA=(1, 2), pB=(0, 1), qB=(2, 3), pAB=(0, 1), qAB=(2,))
    return dict(name=f"batch{n}_u1_rank3x4", items=items, call=call)


def peps_virtual(pattern):
    """U(1) x fZ2 virtual space: for each parity, charges -k..k with the
    given degeneracies (k = len(pattern)//2)."""
    k = len(pattern) // 2
    sectors, degs = [], []
    for par in (0, 1):
        for i, q in enumerate(range(-k, k + 1)):
            sectors.append((q, par))
            degs.append(pattern[i])
    return space(sectors, degs)


P_PEPS = space([(0, 0), (1, 1), (2, 0)], [1, 2, 1])     # spinful site, d = 4


def config5(pattern=(1, 2, 2, 2, 1)):
    """Fermionic U(1) x fZ2 PEPS double layer  E = A^dagger o A  over the
    physical leg, then interleaved ket/bra virtual legs (rank 8)."""
    V = peps_virtual(pattern)
    A = dict(sym="U1xFZ2", cod=(P_PEPS,), dom=(V, V, dual(V), dual(V)))
    call = dict(pA=(0, 1, 2, 3), qA=(4,), pB=(0,), qB=(1, 2, 3, 4),
                pAB=(0, 4, 1, 5, 2, 6, 3, 7), qAB=())
    return dict(name=f"peps_u1xfz2_D{2 * sum(pattern)}", tensors=dict(A=A), call=call)


# ---------------------------------------------------------------------------
# data
# ---------------------------------------------------------------------------
def normal(n: int, config: int, stream: int) -> np.ndarray:
    return rng(config, 1000 + stream).standard_normal(int(n))


def small_ints(n: int, config: int, stream: int, lo: int = -3, hi: int = 3) -> np.ndarray:
    """Integers in [lo, hi] as float64: products and partial sums stay exact
    in fp64, fp32 and bf16 for the sizes the tests use."""
    return rng(config, 2000 + stream).integers(lo, hi + 1, size=int(n)).astype(np.float64)


def signs(n: int, config: int, stream: int) -> np.ndarray:
    """Random +-1 weights as float64 (for projections of a whole tensor)."""
    return rng(config, 3000 + stream).integers(0, 2, size=int(n)).astype(np.float64) * 2.0 - 1.0


def random_space(g: np.random.Generator, sym: str, max_sect: int = 3, max_deg: int = 3,
                 qrange: int = 2, dual_prob: float = 0.5) -> SpaceSpec:
    """A small random graded space for property tests."""
    if sym == "Z1":
        cands = [()]
    elif sym in ("Z2", "FZ2"):
        cands = [(0,), (1,)]
    elif sym == "U1":
        cands = [(q,) for q in range(-qrange, qrange + 1)]
    else:
        cands = [(q, p) for q in range(-qrange, qrange + 1) for p in (0, 1)]
    ns = int(g.integers(1, min(max_sect, len(cands)) + 1))
    pick = sorted(g.choice(len(cands), size=ns, replace=False).tolist())
    secs = [cands[i] for i in pick]
    degs = [int(g.integers(1, max_deg + 1)) for _ in secs]
    return space(secs, degs, bool(g.random() < dual_prob))


# ---- SU(2) spin-1 chain -------------------------------------------------------
# The SU(2) benchmark of the paper is the spin-1 Heisenberg chain: physical
# leg spin 1, virtual legs with integer spins.  Synthetic virtual leg: spins
# j = 0..jmax with multiplicities ~ exp(-j^2 / 2 sigma^2) summing to Dred
# (the number of multiplets); the dense dimension is sum deg(j) (2j + 1).
SU2_PHYS = [(2, 1)]  # (twice the spin, degeneracy): spin 1


def su2_virtual(Dred: int, jmax: int, sigma: float):
    """Virtual leg as [(2j, deg)], j = 0..jmax (largest-remainder rounding of
    the Gaussian shares; every spin keeps at least one multiplet)."""
    js = np.arange(0, jmax + 1)
    w = np.exp(-js.astype(float) ** 2 / (2.0 * sigma * sigma))
    share = w / w.sum() * Dred
    d = np.maximum(np.floor(share).astype(np.int64), 1)
    left = Dred - int(d.sum())
    order = sorted(range(len(js)), key=lambda i: (-(share[i] - np.floor(share[i])), i))
    for i in order[:max(0, left)]:
        d[i] += 1
    return [(2 * int(j), int(x)) for j, x in zip(js, d)]


def su2_two_site(Dred: int, jmax: int, sigma: float):
    """x2 : V (x) P (x) P <- V and the swap of its two physical legs
    (codomain (0, 2, 1), domain (3)): the braid of a two-site gate."""
    V = su2_virtual(Dred, jmax, sigma)
    return dict(cod=[V, SU2_PHYS, SU2_PHYS], dom=[V], p=[0, 2, 1], q=[3])
