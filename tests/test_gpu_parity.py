"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Integer and index work (block structure, placement, signs) is checked
bit-exactly: permutes on any data, contractions on small-integer data (exact
in fp64).  Gaussian fp64 data is held to 1e-12 normwise and entrywise
relative to |A||B| (an fp64 dot product of length K has error below
K u (|A||B|)_ij with u = 2^-53, i.e. < 3e-13 for every K used here).
"""
import numpy as np
import pytest

from oracle import blockwise, dense
from oracle.graded import Structure, permute_spaces
from paper_2508_10076_amd import synth
from tests.helpers import ospace, ostruct, wide_n_case as _wide_n_case

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


def random_tdict(rng, sym, n1, n2, **kw):
    while True:
        t = dict(sym=sym, cod=[synth.random_space(rng, sym, **kw) for _ in range(n1)],
                 dom=[synth.random_space(rng, sym, **kw) for _ in range(n2)])
        if ostruct(t).size:
            return t


def int_vec(rng, n):
    return rng.integers(-3, 4, size=n).astype(np.float64)


# ---------------------------------------------------------------------------
# permute (Alg. "Abelian Tensor Permutation")
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("sym", ["Z1", "Z2", "FZ2", "U1", "U1xFZ2"])
def test_permute_bit_exact(ctx, sym):
    rng = np.random.default_rng(1000 + len(sym))
    for trial in range(12):
        n1, n2 = int(rng.integers(0, 4)), int(rng.integers(0, 4))
        if n1 + n2 == 0:
            continue
        t = random_tdict(rng, sym, n1, n2, max_deg=4)
        st = ostruct(t)
        v = rng.standard_normal(st.size)
        perm = [int(x) for x in rng.permutation(n1 + n2)]
        k = int(rng.integers(0, n1 + n2 + 1))
        p, q = perm[:k], perm[k:]
        A = make(ctx, t, v)
        Cg = tk.tensor_create_permuted(ctx, A, p, q)
        fill(Cg)
        tk.tensor_permute(ctx, A, p, q, Cg)
        _, ref = blockwise.permute_storage(st, v, p, q)
        got = download(Cg)
        assert np.array_equal(got, ref), (sym, trial, p, q)


def test_permute_large_blocks(ctx):
    """Blocks larger than one workgroup chunk, odd sizes, all strides."""
    rng = np.random.default_rng(5)
    V = synth.u1_space([-1, 0, 1], [37, 101, 53])
    W = synth.u1_space([0, 1], [3, 5])
    t = dict(sym="U1", cod=[V, W], dom=[V])
    st = ostruct(t)
    v = rng.standard_normal(st.size)
    A = make(ctx, t, v)
    for p, q in [((2, 0), (1,)), ((1,), (2, 0)), ((0, 2, 1), ()), ((), (1, 0, 2))]:
        Cg = tk.tensor_create_permuted(ctx, A, p, q)
        fill(Cg)
        tk.tensor_permute(ctx, A, p, q, Cg)
        _, ref = blockwise.permute_storage(st, v, p, q)
        assert np.array_equal(download(Cg), ref), (p, q)


def test_adjoint_bit_exact(ctx):
    rng = np.random.default_rng(6)
    for sym in ("U1", "U1xFZ2"):
        t = random_tdict(rng, sym, 2, 3, max_deg=5)
        st = ostruct(t)
        v = rng.standard_normal(st.size)
        A = make(ctx, t, v)
        Cg = tk.tensor_adjoint(ctx, A)
        sta, b = blockwise.adjoint(st, st.to_blocks(v))
        assert np.array_equal(download(Cg), sta.from_blocks(b))


# ---------------------------------------------------------------------------
# contraction (Alg. "Abelian tensor contraction")
# ---------------------------------------------------------------------------
def _contract_case(rng, sym, max_deg=4):
    from tests.test_abi_host import _plan_case  # same generator as the host tests
    return _plan_case(rng, sym)


@pytest.mark.parametrize("sym", ["Z1", "Z2", "FZ2", "U1", "U1xFZ2"])
def test_contract_random_integer_bit_exact(ctx, sym):
    rng = np.random.default_rng(2000 + len(sym))
    for trial in range(10):
        tA, pA, qA, tB, pB, qB, pAB, qAB = _contract_case(rng, sym)
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        fill(Cg)
        tk.tensor_contract(ctx, A, pA, qA, B, pB, qB, pAB, qAB, C_=Cg)
        _, ref = blockwise.contract_storage(stA, a, pA, qA, stB, b, pB, qB, pAB, qAB)
        assert np.array_equal(download(Cg), ref), (sym, trial)


def _wide_case(rng, sym, kdeg):
    """C~ with five row legs (beyond the fused-scatter limit of four legs per
    side), so the output permute runs after the sector GEMMs; kdeg bounds the
    degeneracies of the contracted leg (small: K <= 8 stream; large: MFMA)."""
    while True:
        kl = synth.random_space(rng, sym, max_deg=kdeg)
        if kdeg > 8:  # every sector of the contracted leg longer than the small-K limit
            kl = synth.space(kl.sectors, [d + 8 for d in kl.degs], kl.dual)
        tA = dict(sym=sym, cod=[synth.random_space(rng, sym, max_deg=2) for _ in range(3)],
                  dom=[synth.random_space(rng, sym, max_deg=2) for _ in range(2)] + [kl])
        stA = ostruct(tA)
        if not stA.size:
            continue
        pA, qA = (0, 1, 2, 3, 4), (5,)
        _, Adom = permute_spaces(stA.cod, stA.dom, pA, qA)
        tB = dict(sym=sym, cod=[synth.SpaceSpec(s.sectors, s.degs, s.dual) for s in Adom],
                  dom=[synth.random_space(rng, sym, max_deg=3)])
        if not ostruct(tB).size:
            continue
        return tA, pA, qA, tB, (0,), (1,), (5, 0, 4), (1, 3, 2)


@pytest.mark.parametrize("sym", ["Z2", "U1", "U1xFZ2"])
@pytest.mark.parametrize("kdeg", [2, 12])
def test_contract_wide_output_permuted_after(ctx, sym, kdeg):
    rng = np.random.default_rng(4100 + kdeg + len(sym))
    for trial in range(4):
        tA, pA, qA, tB, pB, qB, pAB, qAB = _wide_case(rng, sym, kdeg)
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        c0 = int_vec(rng, Cg.nelem)
        upload(Cg, c0)
        tk.tensor_contract(ctx, A, pA, qA, B, pB, qB, pAB, qAB, alpha=2.0, beta=-1.0, C_=Cg)
        _, ref = blockwise.contract_storage(stA, a, pA, qA, stB, b, pB, qB, pAB, qAB, alpha=2.0, beta=-1.0, vC=c0)
        assert np.array_equal(download(Cg), ref), (sym, kdeg, trial)


@pytest.mark.parametrize("sym", ["Z1", "Z2", "FZ2", "U1", "U1xFZ2"])
def test_contract_small_k_many_columns(ctx, sym):
    rng = np.random.default_rng(4700 + len(sym))
    seen_wide = seen_runs = 0
    for trial in range(6):
        tA, pA, qA, tB, pB, qB, pAB, qAB = _wide_n_case(rng, sym)
        if trial == 0:
            pAB, qAB = [0, 1], [2, 3]        # identity output layout
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        P = tk.Plan(ctx, A, pA, qA, B, pB, qB, pAB, qAB, Cg)
        g = P.gemms()
        seen_wide += int(len(g) > 0 and g[:, 1].max() > 64 and g[:, 2].max() <= 8)
        seen_runs += int(P.counts()["smallk_runs"] > 0)
        c0 = int_vec(rng, Cg.nelem)
        upload(Cg, c0)
        tk.tensor_contract(ctx, A, pA, qA, B, pB, qB, pAB, qAB, alpha=2.0, beta=-1.0, C_=Cg)
        _, ref = blockwise.contract_storage(stA, a, pA, qA, stB, b, pB, qB, pAB, qAB, alpha=2.0, beta=-1.0, vC=c0)
        assert np.array_equal(download(Cg), ref), (sym, trial)
    assert seen_wide >= 3
    assert seen_runs >= 3


def _short_run_case(rng, sym, swap):
    """Small K against wide columns, where the rows of A~ come in channels of
    one row each (two codomain legs of degeneracy 1 with several sectors):
    the output blocks are single rows, too short for output runs, so the
    planner keeps the per-block tasks.  swap reverses the two row legs in the
    output (fused permute) instead of the identity layout."""
    cands = {"Z1": [()], "Z2": [(0,), (1,)], "FZ2": [(0,), (1,)], "U1": [(q,) for q in range(-2, 3)],
             "U1xFZ2": [(q, p) for q in range(-1, 2) for p in (0, 1)]}[sym]
    while True:
        rows = [synth.space(cands, [1] * len(cands), bool(rng.random() < 0.5)) for _ in range(2)]
        kl = synth.random_space(rng, sym, max_deg=2)
        tA = dict(sym=sym, cod=rows, dom=[kl])
        wide = synth.random_space(rng, sym, max_sect=3, max_deg=4)
        wide = synth.space(wide.sectors, [d + 70 for d in wide.degs], wide.dual)
        tB = dict(sym=sym, cod=[synth.SpaceSpec(kl.sectors, kl.degs, kl.dual)], dom=[wide])
        if ostruct(tA).size and ostruct(tB).size:
            return tA, (0, 1), (2,), tB, (0,), (1,), ((1, 0) if swap else (0, 1)), (2,)


@pytest.mark.parametrize("sym", ["Z2", "U1", "U1xFZ2"])
@pytest.mark.parametrize("swap", [False, True])
def test_contract_small_k_short_runs_use_block_tasks(ctx, sym, swap):
    rng = np.random.default_rng(5100 + len(sym) + 7 * swap)
    seen_blocks = 0
    for trial in range(3):
        tA, pA, qA, tB, pB, qB, pAB, qAB = _short_run_case(rng, sym, swap)
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        P = tk.Plan(ctx, A, pA, qA, B, pB, qB, pAB, qAB, Cg)
        cnt = P.counts()
        seen_blocks += int(cnt["smallk_tasks"] > 0 and cnt["smallk_runs"] == 0)
        c0 = int_vec(rng, Cg.nelem)
        upload(Cg, c0)
        P.execute(A, B, Cg, alpha=-1.0, beta=2.0)
        _, ref = blockwise.contract_storage(stA, a, pA, qA, stB, b, pB, qB, pAB, qAB, alpha=-1.0, beta=2.0, vC=c0)
        assert np.array_equal(download(Cg), ref), (sym, swap, trial)
    assert seen_blocks >= 1


@pytest.mark.parametrize("sym", ["U1", "U1xFZ2"])
def test_contract_small_k_wide_columns_permuted_after(ctx, sym):
    """Small K, wide columns and five row legs: the output permute runs after
    the small-K blocks, which then write C~ in its own layout."""
    rng = np.random.default_rng(5300 + len(sym))
    for trial in range(3):
        tA, pA, qA, tB, pB, qB, pAB, qAB = _wide_case(rng, sym, 2)
        w = tB["dom"][0]
        tB = dict(tB, dom=[synth.space(w.sectors, [d + 70 for d in w.degs], w.dual)])
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        P = tk.Plan(ctx, A, pA, qA, B, pB, qB, pAB, qAB, Cg)
        assert P.counts()["smallk_runs"] == 0
        c0 = int_vec(rng, Cg.nelem)
        upload(Cg, c0)
        P.execute(A, B, Cg, alpha=2.0, beta=-1.0)
        _, ref = blockwise.contract_storage(stA, a, pA, qA, stB, b, pB, qB, pAB, qAB, alpha=2.0, beta=-1.0, vC=c0)
        assert np.array_equal(download(Cg), ref), (sym, trial)


def test_contract_fermionic_against_graph_evaluator(ctx):
    """U(1) x fZ2: the GPU result against the dense graph evaluator (O1)."""
    rng = np.random.default_rng(77)
    sym = "U1xFZ2"
    for trial in range(10):
        tA, pA, qA, tB, pB, qB, pAB, qAB = _contract_case(rng, sym)
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        Cg = tk.tensor_contract(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        D, dcod, ddom = dense.contract_dense(sym, stA.to_dense(a), stA.cod, stA.dom, pA, qA,
                                             stB.to_dense(b), stB.cod, stB.dom, pB, qB, pAB, qAB)
        stC = Structure(sym, dcod, ddom)
        assert np.array_equal(stC.to_dense(download(Cg)), D), trial


def test_contract_alpha_beta(ctx):
    rng = np.random.default_rng(8)
    tA, pA, qA, tB, pB, qB, pAB, qAB = _contract_case(rng, "U1")
    stA, stB = ostruct(tA), ostruct(tB)
    a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
    A, B = make(ctx, tA, a), make(ctx, tB, b)
    Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
    c0 = int_vec(rng, Cg.nelem)
    upload(Cg, c0)
    tk.tensor_contract(ctx, A, pA, qA, B, pB, qB, pAB, qAB, alpha=2.0, beta=-1.0, C_=Cg)
    _, ref = blockwise.contract_storage(stA, a, pA, qA, stB, b, pB, qB, pAB, qAB, alpha=2.0, beta=-1.0, vC=c0)
    assert np.array_equal(download(Cg), ref)


@pytest.mark.parametrize("sym", ["Z1", "Z2", "FZ2", "U1", "U1xFZ2"])
def test_outer_product_bit_exact(ctx, sym):
    """Contraction over no legs (K = 1 sector GEMMs through the small-K
    path): GPU against the blockwise oracle, random output arrangements."""
    rng = np.random.default_rng(9300 + len(sym))
    done = 0
    while done < 4:
        tA = dict(sym=sym, cod=[synth.random_space(rng, sym, max_deg=3) for _ in range(2)],
                  dom=[synth.random_space(rng, sym, max_deg=3)])
        tB = dict(sym=sym, cod=[synth.random_space(rng, sym, max_deg=3)],
                  dom=[synth.random_space(rng, sym, max_deg=3)])
        stA, stB = ostruct(tA), ostruct(tB)
        if stA.size == 0 or stB.size == 0:
            continue
        perm = [int(x) for x in rng.permutation(5)]
        n1 = int(rng.integers(0, 5))
        pAB, qAB = perm[:n1], perm[n1:]
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        Cg = tk.tensor_contract(ctx, A, (0, 1, 2), (), B, (), (0, 1), pAB, qAB)
        _, ref = blockwise.contract_storage(stA, a, (0, 1, 2), (), stB, b, (), (0, 1), pAB, qAB)
        assert np.array_equal(download(Cg), ref), (sym, pAB, qAB)
        done += 1


def test_empty_operands(ctx):
    """An operand without any channel: C = beta * C exactly (every coupled
    charge of C has an empty K range), and operations on a zero-size tensor
    launch nothing and succeed."""
    V = synth.u1_space([-1, 0, 1], [2, 3, 2])
    W = synth.u1_space([7], [2])
    tE = dict(sym="U1", cod=[W], dom=[V])            # charge 7 never meets -1..1: no channel
    tB = dict(sym="U1", cod=[V], dom=[V])
    assert ostruct(tE).size == 0
    rng = np.random.default_rng(77)
    E = make(ctx, tE)
    B = make(ctx, tB, int_vec(rng, ostruct(tB).size))
    C0 = tk.tensor_create_contracted(ctx, E, (0,), (1,), B, (0,), (1,), (0,), (1,))
    assert C0.nelem == 0
    tk.tensor_contract(ctx, E, (0,), (1,), B, (0,), (1,), (0,), (1,), C_=C0)
    tk.tensor_permute(ctx, E, (), (0, 1))
    # a C with entries, fed by an operand whose sectors never couple
    tA = dict(sym="U1", cod=[V], dom=[synth.u1_space([5], [3])])
    tB2 = dict(sym="U1", cod=[synth.u1_space([5], [3])], dom=[V])
    A = make(ctx, tA, int_vec(rng, ostruct(tA).size))
    Cg = tk.tensor_create_contracted(ctx, A, (0,), (1,), make(ctx, tB2), (0,), (1,), (0,), (1,))
    assert ostruct(tA).size == 0 and Cg.nelem > 0
    c0 = int_vec(rng, Cg.nelem)
    upload(Cg, c0)
    tk.tensor_contract(ctx, A, (0,), (1,), make(ctx, tB2), (0,), (1,), (0,), (1,), alpha=3.0, beta=-2.0, C_=Cg)
    assert np.array_equal(download(Cg), -2.0 * c0)
    upload(Cg, c0)
    tk.tensor_contract(ctx, A, (0,), (1,), make(ctx, tB2), (0,), (1,), (0,), (1,), alpha=3.0, beta=0.0, C_=Cg)
    assert np.array_equal(download(Cg), np.zeros_like(c0))


def test_empty_k_sectors_are_zero(ctx):
    """A coupled charge present in codomain(A~) and domain(B~) but not in the
    contracted space gives a zero block (remark after eq. abelian_compostion)."""
    V = synth.u1_space([-1, 0, 1], [2, 3, 2])
    K = synth.u1_space([0], [4])
    tA = dict(sym="U1", cod=[V], dom=[K])
    tB = dict(sym="U1", cod=[K], dom=[V])
    rng = np.random.default_rng(9)
    stA, stB = ostruct(tA), ostruct(tB)
    a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
    A, B = make(ctx, tA, a), make(ctx, tB, b)
    for pAB, qAB in [((0,), (1,)), ((1,), (0,))]:     # in place, and scattered
        Cg = tk.tensor_create_contracted(ctx, A, [0], [1], B, [0], [1], pAB, qAB)
        fill(Cg)
        tk.tensor_contract(ctx, A, [0], [1], B, [0], [1], pAB, qAB, C_=Cg)
        stC, ref = blockwise.contract_storage(stA, a, (0,), (1,), stB, b, (0,), (1,), pAB, qAB)
        got = download(Cg)
        assert np.array_equal(got, ref)
        assert len(stC.sectors) == 3 and (got == 0).sum() >= 2 * 2 * 2


def test_config1_gaussian(ctx):
    cfg = synth.config1()
    tA, tB = cfg["tensors"]["A"], cfg["tensors"]["B"]
    stA, stB = ostruct(tA), ostruct(tB)
    a, b = synth.normal(stA.size, 1, 0), synth.normal(stB.size, 1, 1)
    A, B = make(ctx, tA, a), make(ctx, tB, b)
    _, _, _, call = cfg["calls"][0]
    Cg = tk.tensor_contract(ctx, A, call["pA"], call["qA"], B, call["pB"], call["qB"], call["pAB"], call["qAB"])
    _, ref = blockwise.contract_storage(stA, a, call["pA"], call["qA"], stB, b, call["pB"], call["qB"],
                                        call["pAB"], call["qAB"])
    _, refabs = blockwise.contract_storage(stA, np.abs(a), call["pA"], call["qA"], stB, np.abs(b), call["pB"],
                                           call["qB"], call["pAB"], call["qAB"])
    assert_close(download(Cg), ref, refabs)


# ---------------------------------------------------------------------------
# effective Hamiltonian chains
# ---------------------------------------------------------------------------
def run_heff_gpu(ctx, cfg, data, precision="native"):
    T = {k: make(ctx, cfg["tensors"][k], data[k]) for k in cfg["inputs"]}
    for out, a, b, call in cfg["calls"]:
        T[out] = tk.tensor_contract(ctx, T[a], call["pA"], call["qA"], T[b], call["pB"], call["qB"], call["pAB"],
                                    call["qAB"], precision=precision)
    return T


def run_heff_oracle(cfg, data):
    st = {k: ostruct(cfg["tensors"][k]) for k in cfg["inputs"]}
    v = dict(data)
    for out, a, b, call in cfg["calls"]:
        st[out], v[out] = blockwise.contract_storage(st[a], v[a], call["pA"], call["qA"], st[b], v[b], call["pB"],
                                                     call["qB"], call["pAB"], call["qAB"])
    return st, v


def heff_data(cfg, cid, ints=False, rng=None):
    out = {}
    for i, k in enumerate(cfg["inputs"]):
        n = ostruct(cfg["tensors"][k]).size
        out[k] = int_vec(rng, n) if ints else synth.normal(n, cid, i)
    return out


def test_heff_small_integer_bit_exact(ctx):
    cfg = synth.heff_config(96, 4, 1.6, 90)
    rng = np.random.default_rng(90)
    data = heff_data(cfg, 90, ints=True, rng=rng)
    T = run_heff_gpu(ctx, cfg, data)
    _, v = run_heff_oracle(cfg, data)
    for k in ("T1", "T2", "y"):
        assert np.array_equal(download(T[k]), v[k]), k


@pytest.mark.parametrize("cfgfn,cid", [(synth.config2, 2), (synth.config3, 3)])
def test_heff_full_size_fp64(ctx, cfgfn, cid):
    cfg = cfgfn()
    data = heff_data(cfg, cid)
    T = run_heff_gpu(ctx, cfg, data)
    _, v = run_heff_oracle(cfg, data)
    absdata = {k: np.abs(x) for k, x in data.items()}
    _, vabs = run_heff_oracle(cfg, absdata)
    for k in ("T1", "T2", "y"):
        assert_close(download(T[k]), v[k], vabs[k])


# ---------------------------------------------------------------------------
# partial trace (Alg. "Abelian Tensor Trace")
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("sym", ["Z1", "Z2", "FZ2", "U1", "U1xFZ2"])
def test_trace_against_dense_oracle(ctx, sym):
    """GPU partial trace against the dense graph oracle: one and two traced
    pairs in every orientation, random free-leg arrangements (including a
    full trace to a scalar), small-integer data, alpha/beta, bit-exact."""
    from tests.helpers import trace_case
    rng = np.random.default_rng(8200 + len(sym))
    for trial in range(10):
        t, p, q, t1, t2 = trace_case(rng, sym, npairs=1 + trial % 2)
        st = ostruct(t)
        a = int_vec(rng, st.size)
        A = make(ctx, t, a)
        Cg = tk.tensor_create_traced(ctx, A, p, q, t1, t2)
        D, ocod, odom = dense.trace_dense(sym, st.to_dense(a), st.cod, st.dom, p, q, t1, t2)
        stC = Structure(sym, ocod, odom)
        assert stC.size == Cg.nelem
        c0 = int_vec(rng, Cg.nelem)
        upload(Cg, c0)
        tk.tensor_trace(ctx, A, p, q, t1, t2, alpha=2.0, beta=-1.0, C_=Cg)
        want = 2.0 * stC.from_dense(D, check_zero=True) - c0
        assert np.array_equal(download(Cg), want), (sym, trial, p, q, t1, t2)


def test_trace_large_u1_fp64(ctx):
    """A U(1) tensor V (x) Wm <- V (x) Wm (D=1024) traced over the Wm pair,
    against the dense oracle's blocks, fp64 within 1e-12."""
    q, d = synth.gaussian_degeneracies(1024, 8, 3.0)
    V = synth.u1_space(q, d)
    t = dict(sym="U1", cod=[V, synth.WM_U1], dom=[V, synth.WM_U1])
    st = ostruct(t)
    a = synth.normal(st.size, 9, 0)
    A = make(ctx, t, a)
    Cg = tk.tensor_trace(ctx, A, (0,), (2,), (1,), (3,))
    # blockwise reference: C[a; b] = sum_w A[a, w; b, w], channel by channel
    ref = np.zeros(Cg.nelem)
    stA = st
    stC = Structure("U1", [stA.cod[0]], [stA.dom[0]])
    dense_idx = {}
    for c, ai, bi, off, R in stA.channels():
        if ai[1] != bi[1]:
            continue
        dw = stA.cod[1].degs[ai[1]]
        da, db = stA.cod[0].degs[ai[0]], stA.dom[0].degs[bi[0]]
        blk = a[off + np.arange(da)[:, None, None, None] + da * np.arange(dw)[None, :, None, None]
                + R * (np.arange(db)[None, None, :, None] + db * np.arange(dw)[None, None, None, :])]
        dense_idx.setdefault((ai[0], bi[0]), np.zeros((da, db)))
        dense_idx[(ai[0], bi[0])] += np.einsum("awbw->ab", blk)
    for c, ai, bi, off, R in stC.channels():
        blk = dense_idx.get((ai[0], bi[0]))
        if blk is not None:
            da, db = blk.shape
            ref[off + np.arange(da)[:, None] + R * np.arange(db)[None, :]] = blk
    assert_close(download(Cg), ref, np.abs(ref) + 1.0)


# ---------------------------------------------------------------------------
# truncated SVD (Alg. "Abelian tensor decomposition")
# ---------------------------------------------------------------------------
def _svd_check(ctx, t, a, p, q, max_dim=-1, cutoff=0.0):
    from oracle import decomp
    st = ostruct(t)
    A = make(ctx, t, a)
    U, S, Vh, err = tk.tensor_svd(ctx, A, p, q, max_dim=max_dim, cutoff=cutoff)
    (stU, u), (stS, sv), (stV, vh), err_o, kept = decomp.svd_trunc(st, a, p, q, None if max_dim < 0 else max_dim,
                                                                  cutoff)
    assert U.nelem == stU.size and S.nelem == stS.size and Vh.nelem == stV.size
    gu, gs, gv = download(U), download(S), download(Vh)
    scale = max(float(np.max(np.abs(kept[c]))) for c in kept)
    assert abs(err - err_o) <= 1e-12 * scale
    # same singular values per coupled charge (descending), within fp64 accuracy
    assert np.allclose(gs, sv, rtol=0, atol=1e-12 * scale)
    for c in stU.sectors:
        Ug, Uo = stU.sector_matrix(gu, c), stU.sector_matrix(u, c)
        Vg, Vo = stV.sector_matrix(gv, c), stV.sector_matrix(vh, c)
        assert np.allclose(Ug.T @ Ug, np.eye(Ug.shape[1]), atol=1e-12)
        assert np.allclose(Vg @ Vg.T, np.eye(Vg.shape[0]), atol=1e-12)
        # vectors of distinct singular values agree up to a sign
        sg = np.sign(np.sum(Ug * Uo, axis=0))
        assert np.allclose(Ug * sg, Uo, atol=1e-10) and np.allclose(Vg * sg[:, None], Vo, atol=1e-10)
    return err


@pytest.mark.parametrize("sym", ["Z1", "Z2", "FZ2", "U1", "U1xFZ2"])
def test_svd_against_oracle(ctx, sym):
    """Blockwise Jacobi SVD against the oracle's per-sector library SVD:
    singular values, orthonormal and (up to sign) equal singular vectors,
    with the matrix form taken across every leg split."""
    rng = np.random.default_rng(9600 + len(sym))
    done = 0
    while done < 4:
        t = dict(sym=sym, cod=[synth.random_space(rng, sym, max_deg=4) for _ in range(2)],
                 dom=[synth.random_space(rng, sym, max_deg=4) for _ in range(2)])
        st = ostruct(t)
        if st.size == 0:
            continue
        perm = [int(x) for x in rng.permutation(4)]
        n1 = int(rng.integers(1, 4))
        _svd_check(ctx, t, rng.standard_normal(st.size), tuple(perm[:n1]), tuple(perm[n1:]))
        done += 1


def test_svd_truncated_two_site(ctx):
    """The truncation of the two-site algorithm: x2 : V x P <- V x P* (D=256)
    split between (a, p1) and (b, p2), keeping the 200 largest singular
    values over all charges; error and factors against the oracle."""
    cfg = synth.heff2_config(256, 6, 2.2, 94)
    t = cfg["tensors"]["x"]
    a = synth.normal(ostruct(t).size, 94, 0)
    err = _svd_check(ctx, t, a, (0, 1), (2, 3), max_dim=200)
    assert err > 0


def test_heff2_small_integer_bit_exact(ctx):
    """Two-site H_eff chain (four contractions, two of them skinny) on
    small-integer data: every intermediate equals the oracle's exactly."""
    cfg = synth.heff2_config(64, 3, 1.2, 92)
    rng = np.random.default_rng(92)
    data = heff_data(cfg, 92, ints=True, rng=rng)
    T = run_heff_gpu(ctx, cfg, data)
    _, v = run_heff_oracle(cfg, data)
    for k in ("T1", "T2", "T3", "y"):
        assert np.array_equal(download(T[k]), v[k]), k


def test_heff2_d1024_fp64(ctx):
    cfg = synth.heff2_config(1024, 8, 3.0, 6)
    data = heff_data(cfg, 6)
    T = run_heff_gpu(ctx, cfg, data)
    _, v = run_heff_oracle(cfg, data)
    absdata = {k: np.abs(x) for k, x in data.items()}
    _, vabs = run_heff_oracle(cfg, absdata)
    for k in ("T1", "T2", "T3", "y"):
        assert_close(download(T[k]), v[k], vabs[k])


# ---------------------------------------------------------------------------
# batches and graphs
# ---------------------------------------------------------------------------
def test_batch_graph_replays(ctx):
    cfg = synth.config4(n=6, dmin=64, dmax=300)
    call = cfg["call"]
    rng = np.random.default_rng(44)
    plans, As, Bs, Cs, refs = [], [], [], [], []
    for it in cfg["items"]:
        stA, stB = ostruct(it["A"]), ostruct(it["B"])
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, it["A"], a), make(ctx, it["B"], b)
        Cg = tk.tensor_create_contracted(ctx, A, call["pA"], call["qA"], B, call["pB"], call["qB"], call["pAB"],
                                         call["qAB"])
        plans.append(tk.Plan(ctx, A, call["pA"], call["qA"], B, call["pB"], call["qB"], call["pAB"], call["qAB"], Cg))
        As.append(A)
        Bs.append(B)
        Cs.append(Cg)
        refs.append(blockwise.contract_storage(stA, a, call["pA"], call["qA"], stB, b, call["pB"], call["qB"],
                                               call["pAB"], call["qAB"])[1])
    batch = tk.Batch(ctx, plans, As, Bs, Cs)
    batch.launch()
    for Cg, ref in zip(Cs, refs):
        assert np.array_equal(download(Cg), ref)
    s = torch.cuda.Stream()
    batch.capture(s)
    for rep in range(3):
        for Cg in Cs:
            fill(Cg)
        torch.cuda.synchronize()
        batch.replay(s)
        s.synchronize()
        for Cg, ref in zip(Cs, refs):
            assert np.array_equal(download(Cg), ref), rep


def test_batch_small_k_output_runs(ctx):
    """A batch of small-K contractions with wide columns: the members' output
    runs and decoders are merged into one run list per K."""
    rng = np.random.default_rng(5500)
    plans, As, Bs, Cs, refs = [], [], [], [], []
    for m in range(4):
        tA, pA, qA, tB, pB, qB, pAB, qAB = _wide_n_case(rng, "U1xFZ2")
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        P = tk.Plan(ctx, A, pA, qA, B, pB, qB, pAB, qAB, Cg)
        if P.counts()["smallk_runs"] == 0:
            continue
        plans.append(P)
        As.append(A)
        Bs.append(B)
        Cs.append(Cg)
        refs.append(blockwise.contract_storage(stA, a, pA, qA, stB, b, pB, qB, pAB, qAB)[1])
    assert len(plans) >= 2
    for Cg in Cs:
        fill(Cg)
    batch = tk.Batch(ctx, plans, As, Bs, Cs)
    batch.launch()
    torch.cuda.synchronize()
    for Cg, ref in zip(Cs, refs):
        assert np.array_equal(download(Cg), ref)


def test_heff_chain_graph_replays_match_eager(ctx):
    """The three contractions of H_eff (D=1024) captured in one HIP graph
    (plans execute on the capturing stream) and replayed three times, with
    eager work and synchronizations between the replays: every replay equals
    the eager result bit-exactly, and the oracle within fp64 tolerance."""
    cfg = synth.config2()
    data = heff_data(cfg, 2)
    s = torch.cuda.Stream()
    T = {k: make(ctx, cfg["tensors"][k], data[k]) for k in cfg["inputs"]}
    plans = []
    for out, a, b, call in cfg["calls"]:
        T[out] = tk.tensor_create_contracted(ctx, T[a], call["pA"], call["qA"], T[b], call["pB"], call["qB"],
                                             call["pAB"], call["qAB"])
        plans.append((tk.Plan(ctx, T[a], call["pA"], call["qA"], T[b], call["pB"], call["qB"], call["pAB"],
                              call["qAB"], T[out]), T[a], T[b], T[out]))

    def step():
        for P, A, B, Cc in plans:
            P.execute(A, B, Cc, stream=s)

    with torch.cuda.stream(s):
        step()
    s.synchronize()
    y_eager = download(T[cfg["output"]])
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step()
    for rep in range(3):
        for _, _, _, Cc in plans:          # eager work between replays: garbage in every output
            fill(Cc)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        s.synchronize()
        assert np.array_equal(download(T[cfg["output"]]), y_eager), rep
    _, v = run_heff_oracle(cfg, data)
    ref = v[cfg["output"]]
    assert np.linalg.norm(y_eager - ref) <= 1e-12 * np.linalg.norm(ref)


def test_split_k_tall_k_exact_and_repeatable(ctx):
    """Few tiles with a long K range take the split-K path (partials reduced
    by the last arriving unit); repeated launches must reset its counters."""
    V = synth.u1_space([-1, 0, 1], [40, 60, 40])
    Kb = synth.u1_space([-1, 0, 1], [900, 1200, 900])
    tA = dict(sym="U1", cod=[V], dom=[Kb])
    tB = dict(sym="U1", cod=[Kb], dom=[V])
    rng = np.random.default_rng(12)
    stA, stB = ostruct(tA), ostruct(tB)
    a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
    A, B = make(ctx, tA, a), make(ctx, tB, b)
    _, ref = blockwise.contract_storage(stA, a, (0,), (1,), stB, b, (0,), (1,), (0,), (1,))
    _, reft = blockwise.contract_storage(stA, a, (0,), (1,), stB, b, (0,), (1,), (1,), (0,))
    for pAB, qAB, want in [((0,), (1,), ref), ((1,), (0,), reft)]:
        Cg = tk.tensor_create_contracted(ctx, A, [0], [1], B, [0], [1], pAB, qAB)
        for rep in range(3):
            fill(Cg)
            tk.tensor_contract(ctx, A, [0], [1], B, [0], [1], pAB, qAB, C_=Cg)
            assert np.array_equal(download(Cg), want), (pAB, rep)


# ---------------------------------------------------------------------------
# precision variants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["f32", "bf16x3"])
def test_precision_modes_exact_on_integers(ctx, precision):
    """Integers in [-3, 3] are exact in fp32 and in bf16 (hi = x, lo = 0), and
    every partial sum stays below 2^24, so both modes must be bit-exact."""
    rng = np.random.default_rng(3000 + len(precision))
    for trial in range(8):
        tA, pA, qA, tB, pB, qB, pAB, qAB = _contract_case(rng, "U1xFZ2" if trial % 2 else "U1")
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a), make(ctx, tB, b)
        Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        fill(Cg)
        tk.tensor_contract(ctx, A, pA, qA, B, pB, qB, pAB, qAB, precision=precision, C_=Cg)
        _, ref = blockwise.contract_storage(stA, a, pA, qA, stB, b, pB, qB, pAB, qAB)
        assert np.array_equal(download(Cg), ref), (precision, trial)
    # MFMA-sized sectors too (the random cases are small)
    cfg = synth.heff_config(160, 4, 1.6, 91)
    data = heff_data(cfg, 91, ints=True, rng=rng)
    T = run_heff_gpu(ctx, cfg, data, precision=precision)
    _, v = run_heff_oracle(cfg, data)
    assert np.array_equal(download(T["T1"]), v["T1"])


def test_fp32_storage_exact_on_integers(ctx):
    rng = np.random.default_rng(3100)
    for trial in range(6):
        tA, pA, qA, tB, pB, qB, pAB, qAB = _contract_case(rng, "U1")
        stA, stB = ostruct(tA), ostruct(tB)
        a, b = int_vec(rng, stA.size), int_vec(rng, stB.size)
        A, B = make(ctx, tA, a, dtype="f32"), make(ctx, tB, b, dtype="f32")
        Cg = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        fill(Cg)
        tk.tensor_contract(ctx, A, pA, qA, B, pB, qB, pAB, qAB, C_=Cg)
        _, ref = blockwise.contract_storage(stA, a, pA, qA, stB, b, pB, qB, pAB, qAB)
        assert np.array_equal(download(Cg), ref), trial


@pytest.mark.parametrize("precision,tol", [("f32", 2e-5), ("bf16x3", 2e-4)])
def test_heff_precision_error_bound(ctx, precision, tol):
    """Gaussian D = 1024 H_eff apply.  Bounds from the arithmetic: fp32 keeps
    24 bits (products exact to 2^-24, sums of K <= 700 terms add ~sqrt(K)
    2^-24); bf16x3 keeps 16 bits of each operand (hi + lo) and drops lo*lo,
    ~2^-15 per product.  The measured error is printed for the record."""
    cfg = synth.config2()
    data = heff_data(cfg, 2)
    T = run_heff_gpu(ctx, cfg, data, precision=precision)
    _, v = run_heff_oracle(cfg, data)
    got = download(T["y"])
    err = np.linalg.norm(got - v["y"]) / np.linalg.norm(v["y"])
    print(f"{precision}: normwise error of y {err:.3e}")
    assert err <= tol
    assert err > 1e-12      # the reduced precision really was used


# ---------------------------------------------------------------------------
# fermionic PEPS double layer (reduced sizes; full size in test_gpu_peps.py)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pattern", [(1, 1, 1), (1, 2, 1)])
def test_peps_double_layer_against_graph_evaluator(ctx, pattern):
    """E = A^dagger o A over the physical leg, interleaved ket/bra (rank 8,
    U(1) x fZ2), against the dense graph evaluator; integer data, exact."""
    cfg = synth.config5(pattern)
    tA, call = cfg["tensors"]["A"], cfg["call"]
    stA = ostruct(tA)
    rng = np.random.default_rng(500 + sum(pattern))
    a = int_vec(rng, stA.size)
    A = make(ctx, tA, a)
    Ad = tk.tensor_adjoint(ctx, A)
    E = tk.tensor_contract(ctx, Ad, call["pA"], call["qA"], A, call["pB"], call["qB"], call["pAB"], call["qAB"])
    sAd, bAd = blockwise.adjoint(stA, stA.to_blocks(a))
    vAd = sAd.from_blocks(bAd)
    D, dcod, ddom = dense.contract_dense("U1xFZ2", sAd.to_dense(vAd), sAd.cod, sAd.dom, call["pA"], call["qA"],
                                         stA.to_dense(a), stA.cod, stA.dom, call["pB"], call["qB"],
                                         call["pAB"], call["qAB"])
    stE = Structure("U1xFZ2", dcod, ddom)
    assert stE.size == E.nelem
    got = stE.to_dense(download(E))
    assert np.array_equal(got, D)
    # the interleave really moves odd legs past each other: the bosonic
    # (sign-free) result differs
    Db = np.einsum(sAd.to_dense(vAd), [0, 1, 2, 3, 8], stA.to_dense(a), [8, 4, 5, 6, 7], [0, 4, 1, 5, 2, 6, 3, 7])
    assert not np.array_equal(Db, D) and np.array_equal(np.abs(Db), np.abs(D))


# ---------------------------------------------------------------------------
# config 5 at full size (D = 16): E has 243M stored entries in 4.9M blocks
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def peps_d16(ctx):
    cfg = synth.config5()
    tA, call = cfg["tensors"]["A"], cfg["call"]
    stA = ostruct(tA)
    a = synth.small_ints(stA.size, 5, 16)
    A = make(ctx, tA, a)
    Ad = tk.tensor_adjoint(ctx, A)
    E = tk.tensor_contract(ctx, Ad, call["pA"], call["qA"], A, call["pB"], call["qB"], call["pAB"], call["qAB"])
    e = download(E)
    del E, Ad, A
    return cfg, stA, a, e


def test_peps_d16_sampled_entries_against_graph_definition(peps_d16):
    """10^6 stored entries of E drawn uniformly (the structurally zero blocks
    included) and 2x10^5 uniformly random dense index tuples, each against
    the graph value of the network at that entry (definition evaluated
    pointwise, independent of the blockwise path); layout from the oracle's
    channel enumeration.  Integer data: exact."""
    from oracle import sampled
    cfg, stA, a, e = peps_d16
    call = cfg["call"]
    sAd, bAd = blockwise.adjoint(stA, stA.to_blocks(a))
    Ad = sAd.to_dense(sAd.from_blocks(bAd))
    Ax = stA.to_dense(a)
    tensors = [(Ad, sAd.cod, sAd.dom), (Ax, stA.cod, stA.dom)]
    free = [(0, i) for i in call["pA"]] + [(1, j) for j in call["qB"]]
    out_cod = [free[i] for i in call["pAB"]]
    pairs = [((0, x), (1, y)) for x, y in zip(call["qA"], call["pB"])]
    ocod, odom = sampled.graph_output_spaces([(sAd.cod, sAd.dom), (stA.cod, stA.dom)], out_cod, [])
    assert odom == ()
    idx, size, off = sampled.codomain_channels("U1xFZ2", ocod)
    assert int(off[-1] + size[-1]) == e.shape[0] == 243409664
    rng = np.random.default_rng(51600)
    pos = rng.integers(0, e.shape[0], size=1_000_000)
    dense_idx = sampled.positions_to_dense(ocod, idx, size, off, pos)
    ref = sampled.graph_entries("U1xFZ2", tensors, pairs, out_cod, [], dense_idx)
    assert np.array_equal(e[pos], ref)
    assert np.count_nonzero(ref == 0) > 100_000 and np.count_nonzero(ref) > 100_000
    rnd = np.stack([rng.integers(0, sp.dim, size=200_000) for sp in ocod], axis=1)
    p2 = sampled.dense_to_positions("U1xFZ2", ocod, idx, size, off, rnd)
    v2 = sampled.graph_entries("U1xFZ2", tensors, pairs, out_cod, [], rnd)
    assert np.all(v2[p2 < 0] == 0)                      # outside every stored block: zero
    assert np.array_equal(e[p2[p2 >= 0]], v2[p2 >= 0])


def test_peps_d16_every_block_against_oracle_fingerprint(peps_d16):
    """Every block of E through projections onto seeded +-1 vectors, against
    the values the blockwise oracle produced over every block (written by
    tests/golden/make_peps_d16_fingerprint.py).  Integer data: the entries
    and the projections are exact integers, so the comparison is exact."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "peps_d16_fingerprint.txt")
    ref = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            ref[k] = float(v)
    _, _, _, e = peps_d16
    assert e.shape[0] == int(ref["size"])
    assert int(np.count_nonzero(e)) == int(ref["nonzero"])
    assert float(np.dot(e, e)) == ref["sum_sq"]
    for k in range(4):
        w = synth.signs(e.shape[0], 5, k)
        assert float(np.dot(w, e)) == ref[f"proj{k}"], k
