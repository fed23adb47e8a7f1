"""Helpers for the GPU parity tests: move seeded storage vectors in and out
of library tensors and compare with the oracle."""
from __future__ import annotations

import numpy as np


def upload(T, vec):
    import torch
    vec = np.asarray(vec)
    n = T.nelem
    assert vec.shape == (n,), (vec.shape, n)
    dt = T.storage.dtype
    T.storage[:n].copy_(torch.from_numpy(vec).to(dt))


def download(T):
    import torch
    torch.cuda.synchronize()
    return T.storage[:T.nelem].double().cpu().numpy()


def fill(T, value=np.nan):
    T.storage.fill_(float(value))


def normwise(got, ref):
    d = np.linalg.norm(got - ref)
    r = np.linalg.norm(ref)
    return d / r if r > 0 else d


def assert_close(got, ref, refabs=None, tol=1e-12):
    """Normwise  |C - C*|_F / |C*|_F <= tol  and, when the entrywise bound
    (|A| |B|)_ij is given,  |C - C*|_ij <= tol (|A||B|)_ij."""
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got)), "non-finite output (an element was never written?)"
    nw = normwise(got, ref)
    assert nw <= tol, f"normwise error {nw:.3e} > {tol}"
    if refabs is not None:
        bad = np.abs(got - ref) > tol * refabs + 1e-300
        assert not bad.any(), f"{bad.sum()} entries above the entrywise bound"
