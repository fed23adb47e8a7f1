"""The per-operand permute stages (TK_STAGE_PERMUTE_A / _B) through the
C-ABI: enqueued apart, in either order, on one stream or on two streams
joined by an event, a contraction equals the whole-plan execution bit for
bit (fp64 and split-BF16x3, random contractions whose operands both need a
permute); and the H_eff chain of the bench, with the input permutes of the
later contractions on a second stream, equals the same chain run on one
stream, eagerly and replayed from a HIP graph."""
import numpy as np
import pytest

from paper_2508_10076_amd import synth
from tests.helpers import plan_case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_10076_amd import tk  # noqa: E402
from tests.gpu_util import download, fill, upload  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = tk.Context(0)
    yield c
    c.close()


def _identity(p, q, n1):
    return list(p) == list(range(n1)) and list(q) == list(range(n1, n1 + len(q)))


def _case(ctx, rng, sym, precision):
    """A random contraction in which A and B both have permute work (in
    split-BF16x3 both operands are always written as planes)."""
    while True:
        tA, pA, qA, tB, pB, qB, pAB, qAB = plan_case(rng, sym, max_deg=6)
        if precision != "bf16x3" and (_identity(pA, qA, len(tA["cod"])) or _identity(pB, qB, len(tB["cod"]))):
            continue
        A = tk.tensor_create(ctx, sym, tA["cod"], tA["dom"])
        B = tk.tensor_create(ctx, sym, tB["cod"], tB["dom"])
        C = tk.tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
        P = tk.Plan(ctx, A, pA, qA, B, pB, qB, pAB, qAB, C, precision=precision)
        if P.counts()["pre_tasks"] == 0 or not P.gemms().size:
            continue
        upload(A, rng.integers(-3, 4, A.nelem).astype(np.float64))
        upload(B, rng.integers(-3, 4, B.nelem).astype(np.float64))
        return A, B, C, P


@pytest.mark.parametrize("precision", ["native", "bf16x3"])
@pytest.mark.parametrize("sym", ["U1", "FZ2"])
def test_operand_stages_equal_whole_plan(ctx, sym, precision):
    rng = np.random.default_rng(31 + len(sym) + len(precision))
    done = 0
    for trial in range(40):
        A, B, C, P = _case(ctx, rng, sym, precision)
        print(f"{sym} {precision} trial {trial}: {A.nelem} x {B.nelem} -> {C.nelem}", flush=True)
        fill(C, np.nan)
        P.execute(A, B, C)
        torch.cuda.synchronize()
        want = download(C)
        # A then B, one stream
        fill(C, np.nan)
        P.execute_stages(A, B, C, tk.STAGE_PERMUTE_A)
        P.execute_stages(A, B, C, tk.STAGE_PERMUTE_B)
        P.execute_stages(A, B, C, tk.STAGE_GEMM | tk.STAGE_ZERO)
        torch.cuda.synchronize()
        assert np.array_equal(download(C), want, equal_nan=True)
        # B on a second stream, A on the first, joined by an event
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        fill(C, np.nan)
        torch.cuda.synchronize()
        P.execute_stages(A, B, C, tk.STAGE_PERMUTE_B, stream=s2)
        ev = torch.cuda.Event()
        ev.record(s2)
        P.execute_stages(A, B, C, tk.STAGE_PERMUTE_A, stream=s1)
        s1.wait_event(ev)
        P.execute_stages(A, B, C, tk.STAGE_GEMM | tk.STAGE_ZERO, stream=s1)
        s1.synchronize()
        assert np.array_equal(download(C), want, equal_nan=True)
        done += 1
        if done == 6:
            break
    assert done == 6


def test_stage_mask_is_checked(ctx):
    rng = np.random.default_rng(5)
    A, B, C, P = _case(ctx, rng, "U1", "native")
    with pytest.raises(tk.TkError):
        P.execute_stages(A, B, C, 32)


@pytest.mark.parametrize("precision", ["native", "bf16x3"])
def test_heff_two_stream_step_equals_one_stream(ctx, precision):
    import bench
    cfg = synth.config2()
    s = torch.cuda.Stream()
    H = bench.Heff(tk, torch, cfg, 2, ctx, s, precision, overlap=True)
    assert H.side_stages, "the chain has input permutes after its first contraction"
    y_out = H.T[cfg["output"]]
    # one stream, whole plans
    with torch.cuda.stream(s):
        for P, A, B, Cc, _ in H.plans:
            P.execute(A, B, Cc, stream=s)
    s.synchronize()
    want = H.output()
    fill(y_out, np.nan)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        H.step()
    s.synchronize()
    assert np.array_equal(H.output(), want)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        H.step()
    for rep in range(3):
        fill(y_out, np.nan)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        s.synchronize()
        assert np.array_equal(H.output(), want), rep
