"""GPU parity at the sizes and in the launch configurations that bench.py
times, against the CPU oracle.

* The batch of 64 independent contractions (D ~ U{256..2048}), in fp64 and
  fp32 storage, as one persistent grouped launch captured in a HIP graph and
  replayed, under the autotuner's shipped tile and under every tile shape.
* The single-site H_eff apply at D = 4096 under every tile shape (fp64), and
  its fp32 and split-BF16x3 modes under every tile they support.
* The two-site H_eff apply at D = 4096 with the shipped tiles.
* The Jacobi SVD on sector matrices taller than 512 rows (the two-pass
  path) and on rank-deficient sectors.
* The fermionic PEPS double layer in split-BF16x3: exact on integer data at
  D = 6, 8 and 16, and within a stated bound on Gaussian data at D = 16.

Bounds.  fp64: 1e-12 normwise and entrywise relative to (|A||B|)_ij (a
length-K fp64 dot product errs by at most K u (|A||B|)_ij, u = 2^-53).
fp32 storage: inputs are fp32 numbers, only the accumulation rounds, so
|C - C*|_ij <= (K + 2) 2^-24 (|A||B|)_ij.  split-BF16x3: a = hi + lo + r with
|r| <= 2^-16 |a| (bf16 keeps 8 significant bits), dropping lo*lo' and the
residuals costs at most 3 * 2^-16 per product, the fp32 accumulation adds
K 2^-24: 2^-14 (|A||B|)_ij for K <= 2.
"""
import numpy as np
import pytest

from oracle import blockwise, dense, sampled
from oracle.graded import Structure
from paper_2508_10076_amd import autotune, synth
from tests.helpers import ostruct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_10076_amd import tk  # noqa: E402
from tests.gpu_util import assert_close, download, fill, upload  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = tk.Context(0)
    yield c
    torch.cuda.synchronize()


def make(ctx, t, vec=None, dtype="f64"):
    T = tk.tensor_create(ctx, t["sym"], t["cod"], t["dom"], dtype=dtype)
    if vec is not None:
        upload(T, vec)
    return T


def int_vec(rng, n):
    return rng.integers(-3, 4, size=n).astype(np.float64)


def say(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------
# the batch of 64 contractions, one grouped launch replayed from a graph
# ---------------------------------------------------------------------------
def batch_setup(ctx, cfg, data, dtype):
    call = cfg["call"]
    plans, As, Bs, Cs = [], [], [], []
    for it, (a, b) in zip(cfg["items"], data):
        A, B = make(ctx, it["A"], a, dtype), make(ctx, it["B"], b, dtype)
        Cg = tk.tensor_create_contracted(ctx, A, call["pA"], call["qA"], B, call["pB"], call["qB"], call["pAB"],
                                         call["qAB"])
        plans.append(tk.Plan(ctx, A, call["pA"], call["qA"], B, call["pB"], call["qB"], call["pAB"], call["qAB"],
                             Cg))
        As.append(A)
        Bs.append(B)
        Cs.append(Cg)
    batch = tk.Batch(ctx, plans, As, Bs, Cs)
    mnk = [g for P in plans for g in P.gemms().tolist()]
    return batch, plans, As, Bs, Cs, mnk


def batch_oracle(cfg, data):
    call = cfg["call"]
    out = []
    for it, (a, b) in zip(cfg["items"], data):
        stA, stB = ostruct(it["A"]), ostruct(it["B"])
        out.append(blockwise.contract_storage(stA, a, call["pA"], call["qA"], stB, b, call["pB"], call["qB"],
                                              call["pAB"], call["qAB"])[1])
    return out


def replays(batch, Cs, s, check, nrep=2):
    """Capture the batch, then replay it nrep times with garbage written to
    every output in between; check(i, got) for every member after each."""
    batch.capture(s)
    for rep in range(nrep):
        for Cg in Cs:
            fill(Cg)
        torch.cuda.synchronize()
        batch.replay(s)
        s.synchronize()
        for i, Cg in enumerate(Cs):
            check(i, download(Cg), rep)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_config4_batch_every_tile_integer_exact(ctx, dtype):
    """All 64 members, integer data (exact in fp64 and fp32, partial sums
    below 2^24), bit-exact against the oracle after graph replays under the
    shipped tuned tile and under every tile shape."""
    cfg = synth.config4()
    rng = np.random.default_rng(4400)
    data = [(int_vec(rng, ostruct(it["A"]).size), int_vec(rng, ostruct(it["B"]).size)) for it in cfg["items"]]
    refs = batch_oracle(cfg, data)
    batch, plans, As, Bs, Cs, mnk = batch_setup(ctx, cfg, data, dtype)
    assert len(Cs) == 64
    tuned = autotune.lookup(mnk, (dtype, "native"))
    assert tuned is not None, "the timed batch's shape class has a shipped tile"
    s = torch.cuda.Stream()
    for tile in [tuned] + [t for t in tk.tile_shapes() if t != tuned]:
        say(f"case config4 {dtype} tile {tile}")
        batch.set_tile(*tile)

        def check(i, got, rep, tile=tile):
            assert np.array_equal(got, refs[i]), (dtype, tile, i, rep)
        replays(batch, Cs, s, check)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_config4_batch_gaussian_bound(ctx, dtype):
    """All 64 members on the bench's Gaussian data under the shipped tile,
    replayed from the graph: fp64 within 1e-12, fp32 storage within
    (K + 2) 2^-24, both entrywise relative to (|A||B|)_ij."""
    cfg = synth.config4()
    data = []
    for i, it in enumerate(cfg["items"]):
        a = synth.normal(ostruct(it["A"]).size, 4, 2 * i)
        b = synth.normal(ostruct(it["B"]).size, 4, 2 * i + 1)
        if dtype == "f32":   # the oracle sees the fp32 numbers the GPU holds
            a, b = a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
        data.append((a, b))
    refs = batch_oracle(cfg, data)
    absr = batch_oracle(cfg, [(np.abs(a), np.abs(b)) for a, b in data])
    batch, plans, As, Bs, Cs, mnk = batch_setup(ctx, cfg, data, dtype)
    batch.set_tile(*autotune.lookup(mnk, (dtype, "native")))
    kmax = [int(P.gemms()[:, 2].max()) for P in plans]
    worst = []

    def check(i, got, rep):
        tol = 1e-12 if dtype == "f64" else (kmax[i] + 2) * 2.0 ** -24
        assert_close(got, refs[i], absr[i], tol=tol)
        worst.append(float(np.max(np.abs(got - refs[i]) / (absr[i] + 1e-300))))
    replays(batch, Cs, torch.cuda.Stream(), check)
    say(f"config4 {dtype}: max entrywise error / (|A||B|) = {max(worst):.3e}")


# ---------------------------------------------------------------------------
# H_eff applications at D = 4096
# ---------------------------------------------------------------------------
def heff_data(cfg, cid):
    return {k: synth.normal(ostruct(cfg["tensors"][k]).size, cid, i) for i, k in enumerate(cfg["inputs"])}


def heff_oracle(cfg, data):
    st = {k: ostruct(cfg["tensors"][k]) for k in cfg["inputs"]}
    v = dict(data)
    for out, a, b, call in cfg["calls"]:
        st[out], v[out] = blockwise.contract_storage(st[a], v[a], call["pA"], call["qA"], st[b], v[b], call["pB"],
                                                     call["qB"], call["pAB"], call["qAB"])
    return v


class HeffChain:
    """The application as the bench runs it: one plan per contraction."""

    def __init__(self, ctx, cfg, data, precision="native"):
        self.T = {k: make(ctx, cfg["tensors"][k], data[k]) for k in cfg["inputs"]}
        self.plans = []
        for out, a, b, call in cfg["calls"]:
            T = self.T
            T[out] = tk.tensor_create_contracted(ctx, T[a], call["pA"], call["qA"], T[b], call["pB"], call["qB"],
                                                 call["pAB"], call["qAB"])
            P = tk.Plan(ctx, T[a], call["pA"], call["qA"], T[b], call["pB"], call["qB"], call["pAB"], call["qAB"],
                        T[out], precision=precision)
            self.plans.append((out, P, T[a], T[b], T[out]))
        self.mfma = [x for x in self.plans if x[1].gemms()[:, 2].max() > 64]

    def run(self):
        for out, P, A, B, Cc in self.plans:
            fill(Cc)
            P.execute(A, B, Cc)
        torch.cuda.synchronize()


@pytest.fixture(scope="module")
def heff4096():
    cfg = synth.config3()
    data = heff_data(cfg, 3)
    ref = heff_oracle(cfg, data)
    refabs = heff_oracle(cfg, {k: np.abs(x) for k, x in data.items()})
    return cfg, data, ref, refabs


def test_heff_d4096_every_tile_fp64(ctx, heff4096):
    """Every intermediate of the D = 4096 application under every tile shape
    (the bench times the shipped one), fp64 within 1e-12."""
    cfg, data, ref, refabs = heff4096
    H = HeffChain(ctx, cfg, data)
    assert len(H.mfma) == 2
    for tile in tk.tile_shapes():
        say(f"case heff_d4096 fp64 tile {tile}")
        for _, P, *_r in H.mfma:
            P.set_tile(*tile)
        H.run()
        for k in ("T1", "T2", "y"):
            assert_close(download(H.T[k]), ref[k], refabs[k])


@pytest.mark.parametrize("precision,tol", [("f32", 2e-5), ("bf16x3", 2e-4)])
def test_heff_d4096_reduced_precision_every_tile(ctx, heff4096, precision, tol):
    """The fp32 and split-BF16x3 modes at D = 4096 under every tile shape
    they support (the shipped one included): normwise error of y within the
    bound of the D = 1024 test (fp32 keeps 24 bits, sums of K <= 1807 terms;
    bf16x3 keeps ~16 bits per operand), and not below fp64 accuracy."""
    cfg, data, ref, refabs = heff4096
    H = HeffChain(ctx, cfg, data, precision=precision)
    tuned = [autotune.lookup(P.gemms().tolist(), ("f64", precision)) for _, P, *_r in H.mfma]
    errs = {}
    for tile in tk.tile_shapes():
        try:
            for _, P, *_r in H.mfma:
                P.set_tile(*tile)
        except tk.TkError:
            assert precision == "bf16x3" and tile[2] % 32, tile   # bf16 stages are 32 deep
            continue
        say(f"case heff_d4096 {precision} tile {tile}")
        H.run()
        y = download(H.T["y"])
        err = np.linalg.norm(y - ref["y"]) / np.linalg.norm(ref["y"])
        errs[tile] = err
        assert err <= tol and err > 1e-12, (tile, err)
    assert all(t in errs for t in tuned)
    say(f"heff_d4096 {precision}: normwise errors {({k: f'{v:.2e}' for k, v in errs.items()})}")


def test_heff2_d4096_fp64_shipped_tiles(ctx):
    """The two-site application at D = 4096 (four contractions) with the
    shipped tiles the bench uses: every intermediate within 1e-12."""
    cfg = synth.heff2_config(4096, 12, 4.5, 7)
    data = heff_data(cfg, 7)
    ref = heff_oracle(cfg, data)
    refabs = heff_oracle(cfg, {k: np.abs(x) for k, x in data.items()})
    H = HeffChain(ctx, cfg, data)
    for _, P, *_r in H.mfma:
        t = autotune.lookup(P.gemms().tolist(), ("f64", "native"))
        if t:
            P.set_tile(*t)
    say("case heff2_d4096 fp64")
    H.run()
    for k in ("T1", "T2", "T3", "y"):
        assert_close(download(H.T[k]), ref[k], refabs[k])


# ---------------------------------------------------------------------------
# truncated SVD: tall sectors (two-pass Jacobi path) and rank deficiency
# ---------------------------------------------------------------------------
def svd_compare(ctx, t, a, p, q, max_dim=-1, cutoff=0.0, rank=None):
    from oracle import decomp
    st = ostruct(t)
    A = make(ctx, t, a)
    U, S, Vh, err, info = tk.tensor_svd(ctx, A, p, q, max_dim=max_dim, cutoff=cutoff, info=True)
    (stU, u), (stS, sv), (stV, vh), err_o, kept = decomp.svd_trunc(st, a, p, q, None if max_dim < 0 else max_dim,
                                                                  cutoff)
    assert 0 < info["max_sweeps"] < 60
    assert U.nelem == stU.size and S.nelem == stS.size and Vh.nelem == stV.size
    gu, gs, gv = download(U), download(S), download(Vh)
    scale = max(float(np.max(np.abs(kept[c]))) for c in kept)
    assert abs(err - err_o) <= 1e-12 * scale
    assert np.allclose(gs, sv, rtol=0, atol=1e-12 * scale)
    for c in stU.sectors:
        Ug, Uo = stU.sector_matrix(gu, c), stU.sector_matrix(u, c)
        Vg, Vo = stV.sector_matrix(gv, c), stV.sector_matrix(vh, c)
        assert np.allclose(Ug.T @ Ug, np.eye(Ug.shape[1]), atol=1e-12)
        assert np.allclose(Vg @ Vg.T, np.eye(Vg.shape[0]), atol=1e-12)
        sg = np.sign(np.sum(Ug * Uo, axis=0))
        assert np.allclose(Ug * sg, Uo, atol=1e-10) and np.allclose(Vg * sg[:, None], Vo, atol=1e-10)
    return info, err


def test_svd_sectors_taller_than_512_rows(ctx):
    """Sector matrices of 700 x 200 and 300 x 530 (transposed to 530 x 300)
    take the two-pass Jacobi loop (m > 512), beside a small one on the
    register path; all against the oracle's library SVD."""
    V1 = synth.u1_space([-1, 0, 1], [700, 300, 90])
    V2 = synth.u1_space([-1, 0, 1], [200, 530, 70])
    t = dict(sym="U1", cod=[V1], dom=[V2])
    a = synth.normal(ostruct(t).size, 95, 0)
    say("case svd tall sectors 700x200, 300x530, 90x70")
    info, _ = svd_compare(ctx, t, a, (0,), (1,))
    assert info["nsectors"] == 3


def test_svd_rank_deficient_sectors(ctx):
    """Every sector matrix has rank 12 (a product of Gaussian factors): the
    values past the rank are at rounding level on both sides; truncating
    below 1e-8 of the largest keeps exactly the rank, and those factors match
    the oracle's."""
    V1 = synth.u1_space([-1, 0, 1], [60, 640, 40])
    V2 = synth.u1_space([-1, 0, 1], [50, 90, 45])
    t = dict(sym="U1", cod=[V1], dom=[V2])
    st = ostruct(t)
    rng = np.random.default_rng(96)
    a = np.zeros(st.size)
    for c in st.sectors:
        R, C = st.rows[c].total, st.cols[c].total
        M = rng.standard_normal((R, 12)) @ rng.standard_normal((12, C))
        o = st.sector_offset[c]
        a[o:o + R * C] = M.reshape(-1, order="F")
    A = make(ctx, t, a)
    _, S, _, _ = tk.tensor_svd(ctx, A, (0,), (1,))
    s_all = np.sort(download(S)[download(S) != 0])[::-1]
    big = s_all[0]
    assert np.count_nonzero(s_all > 1e-8 * big) == 12 * len(st.sectors)
    say("case svd rank-deficient sectors")
    info, err = svd_compare(ctx, t, a, (0,), (1,), cutoff=1e-8 * big)
    assert info["nkept"] == 12 * len(st.sectors)
    assert err <= 1e-12 * big


# ---------------------------------------------------------------------------
# fermionic PEPS double layer in split-BF16x3
# ---------------------------------------------------------------------------
def peps_gpu(ctx, cfg, a, precision):
    tA, call = cfg["tensors"]["A"], cfg["call"]
    A = make(ctx, tA, a)
    Ad = tk.tensor_adjoint(ctx, A)
    E = tk.tensor_contract(ctx, Ad, call["pA"], call["qA"], A, call["pB"], call["qB"], call["pAB"], call["qAB"],
                           precision=precision)
    return download(E)


@pytest.mark.parametrize("pattern", [(1, 1, 1), (1, 2, 1)])
def test_peps_bf16x3_integer_exact_against_graph_evaluator(ctx, pattern):
    """Integers in [-3, 3] are exact in bf16 (hi = x, lo = 0) and K <= 2, so
    the split-BF16x3 layer equals the dense graph evaluator exactly."""
    cfg = synth.config5(pattern)
    tA, call = cfg["tensors"]["A"], cfg["call"]
    stA = ostruct(tA)
    a = int_vec(np.random.default_rng(700 + sum(pattern)), stA.size)
    say(f"case peps bf16x3 pattern {pattern}")
    got = peps_gpu(ctx, cfg, a, "bf16x3")
    sAd, bAd = blockwise.adjoint(stA, stA.to_blocks(a))
    D, dcod, ddom = dense.contract_dense("U1xFZ2", sAd.to_dense(sAd.from_blocks(bAd)), sAd.cod, sAd.dom,
                                         call["pA"], call["qA"], stA.to_dense(a), stA.cod, stA.dom, call["pB"],
                                         call["qB"], call["pAB"], call["qAB"])
    assert np.array_equal(Structure("U1xFZ2", dcod, ddom).to_dense(got), D)


def test_peps_d16_bf16x3_integer_every_block_exact(ctx):
    """D = 16 in split-BF16x3 on the integer data of the fp64 fingerprint
    test: every block's projections, entry count, nonzero count and sum of
    squares equal the oracle's exactly."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "peps_d16_fingerprint.txt")
    ref = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            ref[k] = float(v)
    cfg = synth.config5()
    a = synth.small_ints(ostruct(cfg["tensors"]["A"]).size, 5, 16)
    say("case peps D16 bf16x3 integer")
    e = peps_gpu(ctx, cfg, a, "bf16x3")
    assert e.shape[0] == int(ref["size"])
    assert int(np.count_nonzero(e)) == int(ref["nonzero"])
    assert float(np.dot(e, e)) == ref["sum_sq"]
    for k in range(4):
        assert float(np.dot(synth.signs(e.shape[0], 5, k), e)) == ref[f"proj{k}"], k


def test_peps_d16_bf16x3_gaussian_sampled_bound(ctx):
    """D = 16 in split-BF16x3 on the bench's Gaussian data: 10^6 stored
    entries against the graph value of the network at that entry (fp64),
    within 2^-14 (|A^dagger| |A|)_ij; the measured maximum is printed."""
    cfg = synth.config5()
    tA, call = cfg["tensors"]["A"], cfg["call"]
    stA = ostruct(tA)
    a = synth.normal(stA.size, 5, 0)
    say("case peps D16 bf16x3 gaussian")
    e = peps_gpu(ctx, cfg, a, "bf16x3")
    sAd, bAd = blockwise.adjoint(stA, stA.to_blocks(a))
    Ad = sAd.to_dense(sAd.from_blocks(bAd))
    Ax = stA.to_dense(a)
    free = [(0, i) for i in call["pA"]] + [(1, j) for j in call["qB"]]
    out_cod = [free[i] for i in call["pAB"]]
    pairs = [((0, x), (1, y)) for x, y in zip(call["qA"], call["pB"])]
    ocod, _ = sampled.graph_output_spaces([(sAd.cod, sAd.dom), (stA.cod, stA.dom)], out_cod, [])
    idx, size, off = sampled.codomain_channels("U1xFZ2", ocod)
    rng = np.random.default_rng(51601)
    pos = rng.integers(0, e.shape[0], size=1_000_000)
    di = sampled.positions_to_dense(ocod, idx, size, off, pos)
    ref = sampled.graph_entries("U1xFZ2", [(Ad, sAd.cod, sAd.dom), (Ax, stA.cod, stA.dom)], pairs, out_cod, [], di)
    # (|A^dagger||A|) at the same entries: output legs interleave ket and bra
    # legs (A^dagger leg 0, A leg 1, A^dagger leg 1, ...), summed over p
    absum = np.zeros(pos.shape[0])
    for p in range(Ax.shape[0]):
        absum += np.abs(Ad[di[:, 0], di[:, 2], di[:, 4], di[:, 6], p]) * np.abs(Ax[p, di[:, 1], di[:, 3], di[:, 5],
                                                                                   di[:, 7]])
    err = np.abs(e[pos] - ref)
    assert np.all(err <= 2.0 ** -14 * absum + 1e-300)
    nz = absum > 0
    say(f"peps D16 bf16x3: max |err| / (|A+||A|) = {np.max(err[nz] / absum[nz]):.3e}, "
        f"normwise over the sample {np.linalg.norm(err) / np.linalg.norm(ref):.3e}")
    assert np.max(err) > 0     # the reduced precision really was used


# ---------------------------------------------------------------------------
# split-BF16x3 operand planes (written by the operand permute)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("sym", ["U1", "U1xFZ2"])
def test_bf16x3_planes_random_contractions_integer_exact(ctx, sym):
    """Random contractions with degeneracies up to 12, so coupled sectors
    with K > 8 (split operand planes, MFMA) and K <= 8 (small-K path) mix in
    one plan, with random leg orders (identity permutations and dual
    contracted legs included): integers are exact in bf16 and every partial
    sum stays below 2^24, so the split-BF16x3 mode equals the oracle."""
    from tests.helpers import plan_case
    rng = np.random.default_rng(3300 + len(sym))
    mfma = 0
    for trial in range(24):
        tA, pA, qA, tB, pB, qB, pAB, qAB = plan_case(rng, sym, max_deg=12)
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        P = tk.Plan(ctx, A, pA, qA, B, pB, qB, pAB, qAB, Cg, precision="bf16x3")
        mfma += int((P.gemms()[:, 2] > 8).sum()) if P.info()["ngemm"] else 0
        fill(Cg)
        P.execute(A, B, Cg)
        _, ref = blockwise.contract_storage(stA, a, pA, qA, stB, b, pB, qB, pAB, qAB)
        assert np.array_equal(download(Cg), ref), (sym, trial)
    assert mfma >= 4


def test_bf16x3_planes_identity_and_twist(ctx):
    """Operands that need no permute (their planes come from an identity
    permute) and a contracted dual odd leg (the composition twist folded
    into B~'s planes), U(1) x fZ2, integer data, exact."""
    V = synth.space([(q, p) for p in (0, 1) for q in (-1, 0, 1)], [5, 9, 6, 7, 4, 11])
    W = synth.space([(0, 0), (1, 1), (-1, 1)], [13, 10, 12])
    rng = np.random.default_rng(3310)
    for dual in (False, True):
        Wk = synth.dual(W) if dual else W
        tA = dict(sym="U1xFZ2", cod=[V], dom=[Wk, V])
        tB = dict(sym="U1xFZ2", cod=[Wk, V], dom=[W])
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        for pAB, qAB in (((0,), (1,)), ((1,), (0,)), ((0, 1), ())):
            Cg = tk.tensor_create_contracted(ctx, A, (0,), (1, 2), B, (0, 1), (2,), pAB, qAB)
            fill(Cg)
            tk.tensor_contract(ctx, A, (0,), (1, 2), B, (0, 1), (2,), pAB, qAB, precision="bf16x3", C_=Cg)
            _, ref = blockwise.contract_storage(stA, a, (0,), (1, 2), stB, b, (0, 1), (2,), pAB, qAB)
            assert np.array_equal(download(Cg), ref), (dual, pAB, qAB)


def test_bf16x3_batch_config4_integer_exact(ctx):
    """The 64-contraction batch in split-BF16x3 (per-member operand planes
    in the batch's buffer table), replayed from a graph: exact on integers."""
    cfg = synth.config4()
    rng = np.random.default_rng(4410)
    data = [(int_vec(rng, ostruct(it["A"]).size), int_vec(rng, ostruct(it["B"]).size)) for it in cfg["items"]]
    refs = batch_oracle(cfg, data)
    call = cfg["call"]
    plans, As, Bs, Cs = [], [], [], []
    for it, (a, b) in zip(cfg["items"], data):
        A, B = make(ctx, it["A"], a), make(ctx, it["B"], b)
        Cg = tk.tensor_create_contracted(ctx, A, call["pA"], call["qA"], B, call["pB"], call["qB"], call["pAB"],
                                         call["qAB"])
        plans.append(tk.Plan(ctx, A, call["pA"], call["qA"], B, call["pB"], call["qB"], call["pAB"], call["qAB"],
                             Cg, precision="bf16x3"))
        As.append(A)
        Bs.append(B)
        Cs.append(Cg)
    batch = tk.Batch(ctx, plans, As, Bs, Cs)
    say("case config4 bf16x3 batch")

    def check(i, got, rep):
        assert np.array_equal(got, refs[i]), (i, rep)
    replays(batch, Cs, torch.cuda.Stream(), check)


# ---------------------------------------------------------------------------
# LDS-staged block permutes (source and destination contiguous along
# different legs)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tile_permute_every_leg_order_exact(ctx, dtype):
    """A U(1) tensor with long legs (17..131, ragged against the 64-wide
    tiles) permuted into every leg order and codomain / domain split: the
    blocks whose fastest source and destination legs differ go through LDS
    tiles, the rest through the output-order walk; bit-exact in fp64 and
    fp32 (a permute moves values, it does not round them)."""
    import itertools
    V = synth.u1_space([-1, 0, 1], [17, 131, 64])
    W = synth.u1_space([0, 1], [70, 23])
    t = dict(sym="U1", cod=[V, W], dom=[V])
    st = ostruct(t)
    v = np.random.default_rng(61).standard_normal(st.size)
    if dtype == "f32":
        v = v.astype(np.float32).astype(np.float64)
    A = make(ctx, t, v, dtype)
    tiles = 0
    for perm in itertools.permutations(range(3)):
        for n1 in range(4):
            p, q = perm[:n1], perm[n1:]
            Cg = tk.tensor_create_permuted(ctx, A, p, q)
            fill(Cg)
            tk.tensor_permute(ctx, A, p, q, Cg)
            _, ref = blockwise.permute_storage(st, v, p, q)
            assert np.array_equal(download(Cg), ref), (p, q)
            tiles += 1
    assert tiles == 24


def test_tile_permute_after_gemm_alpha_beta(ctx):
    """An output permute that cannot be fused (five row legs in C~) runs after
    the sector GEMMs, here through LDS tiles (C~ is contiguous along X, C
    along W, both 16..20 long), with alpha = 2 and beta = -1: integer data,
    exact against the oracle."""
    X = synth.u1_space([0, 1], [17, 20])
    Y = synth.u1_space([0], [2])
    Kl = synth.u1_space([-1, 0, 1], [9, 12, 10])
    Wl = synth.u1_space([0, 1], [16, 19])
    tA = dict(sym="U1", cod=[X, Y, X], dom=[Y, Y, Kl])
    stA = ostruct(tA)
    pA, qA = (0, 1, 2, 3, 4), (5,)
    from oracle.graded import permute_spaces
    _, Adom = permute_spaces(stA.cod, stA.dom, pA, qA)
    tB = dict(sym="U1", cod=[synth.SpaceSpec(s.sectors, s.degs, s.dual) for s in Adom], dom=[Wl])
    stB = ostruct(tB)
    rng = np.random.default_rng(62)
    a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
    A, B = make(ctx, tA, a), make(ctx, tB, b)
    pAB, qAB = (5, 0, 4), (1, 3, 2)
    Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, (0,), (1,), pAB, qAB)
    c0 = int_vec(rng, Cg.nelem)
    upload(Cg, c0)
    tk.tensor_contract(ctx, A, pA, qA, B, (0,), (1,), pAB, qAB, alpha=2.0, beta=-1.0, C_=Cg)
    _, ref = blockwise.contract_storage(stA, a, pA, qA, stB, b, (0,), (1,), pAB, qAB, alpha=2.0, beta=-1.0, vC=c0)
    assert np.array_equal(download(Cg), ref)
