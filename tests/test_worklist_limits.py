"""Host replay of the LDS indices of the zero-range and output-run kernels.

Both kernels stage one workgroup's items (ranges of C to zero, or output runs
of the small-K sectors) in LDS arrays of kMax + 1 entries and give each of its
at most kChunk elements its item through an LDS index map (one mark per item,
then a running maximum).  Those indices are safe only if the planner's work
lists keep their limits.  These tests read the lists of real plans (the PEPS
double layer at D = 6, 8 and 16, and random wide small-K contractions) and
recompute, in numpy, every index the kernels form from them: item counts per
workgroup, the relative starts written to the map, the map entries, the
dimension records and the multiply-high decode of each run's linear index.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2508_10076_amd import synth
from tests.helpers import wide_n_case

tk = pytest.importorskip("paper_2508_10076_amd.tk")

RUN_CHUNK, RUN_MAX = 4096, 128      # kRunChunk, kRunMax (tk_internal.h)
ZERO_CHUNK, ZERO_MAX = 8192, 256    # kZeroChunk, kZeroMax


def peps_plan(pattern):
    cfg = synth.config5(pattern)
    t, call = cfg["tensors"]["A"], cfg["call"]
    A = tk.tensor_create(None, t["sym"], t["cod"], t["dom"])
    Ad = tk.tensor_create_adjoint(None, A)
    E = tk.tensor_create_contracted(None, Ad, call["pA"], call["qA"], A, call["pB"], call["qB"], call["pAB"],
                                    call["qAB"])
    P = tk.Plan(None, Ad, call["pA"], call["qA"], A, call["pB"], call["qB"], call["pAB"], call["qAB"], E)
    return P, E.nelem


def check_list(wl, chunk, kmax, nelem_out=None, every_element=False):
    """Replays the kernels' per-workgroup staging; returns the element count."""
    vs, ln, first, ws = wl["vstart"], wl["len"], wl["first"], wl["wstart"]
    n_items = vs.size
    if n_items == 0:
        assert first.size == 0 and ws.size == 0
        return 0
    total = int(vs[-1] + ln[-1])
    # items are laid end to end, each with at least one element
    assert np.all(ln >= 1)
    assert vs[0] == 0 and np.array_equal(vs[1:], np.cumsum(ln)[:-1])
    assert ws[0] == 0 and ws[-1] == total and first.size == ws.size
    c0, c1 = ws[:-1], ws[1:]
    n = c1 - c0
    assert np.all(n >= 1) and np.all(n <= chunk), "workgroup size out of [1, chunk]"
    r0 = first[:-1].astype(np.int64)
    r1 = np.minimum(n_items, first[1:].astype(np.int64) + 1)
    nr = r1 - r0
    assert np.all(np.diff(first) >= 0)
    # the kernel clamps nr to kmax + 1: the clamp must never bite
    assert np.all(nr >= 1) and np.all(nr <= kmax + 1), f"max staged items {nr.max()} > {kmax + 1}"
    # item 0 of a workgroup holds its first element: relative start <= 0
    assert np.all(vs[r0] <= c0) and np.all(vs[r0] + ln[r0] > c0)
    # every element of the workgroup lies in a staged item: the item holding
    # its last element is among r0 .. r1 - 1
    last_item = np.searchsorted(vs, c1 - 1, side="right") - 1
    assert np.all(last_item < r1) and np.all(last_item >= r0)
    # staged items i >= 1 have relative starts in (0, n]; the map's entries
    # are item numbers below nr (8-bit map for runs, 16-bit for zero ranges)
    for w in (range(len(n)) if every_element else np.linspace(0, len(n) - 1, 64).astype(int)):
        idx = np.arange(r0[w], r1[w])
        rel = vs[idx] - c0[w]
        s_r = np.maximum(rel, 0)
        assert s_r[0] == 0 and np.all(s_r[1:] > 0) and np.all(s_r[1:] <= n[w])
        # the kernel's map: mark each item's first element, running maximum
        mark = np.zeros(int(n[w]), np.int64)
        for i in range(1, len(idx)):
            if 0 < s_r[i] < n[w]:
                mark[s_r[i]] = i
        m = np.maximum.accumulate(mark)
        assert m.max() < len(idx) and m.max() < (255 if kmax == RUN_MAX else 65535)
        holder = np.searchsorted(vs, c0[w] + np.arange(n[w]), side="right") - 1
        assert np.array_equal(idx[m], holder), f"workgroup {w}: element mapped to the wrong item"
    return total


def check_runs(wl):
    """Dimension records and the multiply-high decode of every run's linear
    index range (the kernel's 32-bit mulhi and 24-bit products)."""
    rec, shape, lin0, ln = wl["dimrec"], wl["shape"], wl["lin0"].astype(np.int64), wl["len"]
    if shape.size == 0:
        return
    assert np.all(shape >= 0) and np.all(shape < rec.shape[0])
    nd = rec[:, 0]
    assert np.all(nd >= 0) and np.all(nd <= 8)
    ext = rec[:, 1::3].astype(np.int64)
    mag = rec[:, 2::3].astype(np.int64) & 0xFFFFFFFF
    shr = rec[:, 3::3].astype(np.int64)
    used = np.arange(8)[None, :] < nd[:, None]
    assert np.all(ext[used] >= 2), "records hold only extents above 1"
    size = np.prod(np.where(used, ext, 1), axis=1)
    assert np.all(size < 1 << 24)
    # every element of a run lies in its block
    assert np.all(lin0 >= 0) and np.all(lin0 + ln <= size[shape])
    # the magic division is exact on every index the kernel can see (< block size)
    for r in range(rec.shape[0]):
        for d in range(nd[r]):
            x = np.arange(int(size[r]), dtype=np.int64)
            assert np.array_equal((x * mag[r, d]) >> shr[r, d], x // ext[r, d]), (r, d)


@pytest.mark.parametrize("pattern", [(1, 1, 1), (1, 2, 1), (1, 2, 2, 2, 1)])
def test_peps_worklists_keep_lds_limits(pattern):
    P, nelem = peps_plan(pattern)
    every = sum(pattern) <= 4
    n0 = check_list(P.worklist(0), ZERO_CHUNK, ZERO_MAX, every_element=every)
    nruns = 0
    for K in range(1, 9):
        wl = P.worklist(K)
        nruns += check_list(wl, RUN_CHUNK, RUN_MAX, every_element=every)
        check_runs(wl)
    # at D = 16 the layer writes E through zero ranges and output runs only
    # (at D = 6 and 8 the blocks are too small for runs: block tasks write them)
    assert n0 > 0
    if pattern == (1, 2, 2, 2, 1):
        assert P.counts()["smallk_runs"] > 0
        assert n0 + nruns == nelem


def test_wide_small_k_worklists_keep_lds_limits():
    """Random small-K contractions with wide outputs (runs of every K and
    zero ranges), through the same replay."""
    rng = np.random.default_rng(5501)
    seen = 0
    for _ in range(12):
        tA, pA, qA, tB, pB, qB, pAB, qAB = wide_n_case(rng, "U1xFZ2")
        A = tk.tensor_create(None, tA["sym"], tA["cod"], tA["dom"])
        B = tk.tensor_create(None, tB["sym"], tB["cod"], tB["dom"])
        Cn = tk.tensor_create_contracted(None, A, pA, qA, B, pB, qB, pAB, qAB)
        P = tk.Plan(None, A, pA, qA, B, pB, qB, pAB, qAB, Cn)
        check_list(P.worklist(0), ZERO_CHUNK, ZERO_MAX, every_element=True)
        for K in range(1, 9):
            wl = P.worklist(K)
            seen += wl["vstart"].size
            check_list(wl, RUN_CHUNK, RUN_MAX, every_element=True)
            check_runs(wl)
    assert seen > 0


def test_replay_rejects_broken_lists():
    """The replay itself fails on lists that break a limit (a workgroup
    longer than the chunk, too many staged items, a wrong first item)."""
    P, _ = peps_plan((1, 2, 2, 2, 1))
    wl = P.worklist(1)
    check_list(wl, RUN_CHUNK, RUN_MAX)
    for broken in ("chunk", "items", "first"):
        bad = {k: v.copy() for k, v in wl.items()}
        if broken == "chunk":        # merge two workgroups into one
            w = int(np.argmax(np.diff(bad["wstart"]) < RUN_CHUNK // 2))
            bad["wstart"] = np.delete(bad["wstart"], w + 1)
            bad["first"] = np.delete(bad["first"], w + 1)
            chunk, kmax = RUN_CHUNK // 2 + 1, RUN_MAX
        elif broken == "items":      # a smaller item budget than the planner used
            chunk, kmax = RUN_CHUNK, 1
        else:                        # first item one too far
            w = int(np.argmax(bad["first"][:-1] < bad["first"][1:]))
            bad["first"][w] += 1
            chunk, kmax = RUN_CHUNK, RUN_MAX
        with pytest.raises(AssertionError):
            check_list(bad, chunk, kmax)
