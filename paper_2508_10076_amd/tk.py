"""Thin Python binding of the C-ABI in include/tk.h (argument marshalling only).

The library is loaded from libtk.so next to this file; importing this module
raises if it is missing (there is no fallback of any kind).  Device memory
comes from torch (tensors wrap torch buffers); every numerical step runs in
the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# TK_LIBRARY selects another build of the same library (the sanitized one)
LIB_PATH = os.environ.get("TK_LIBRARY") or os.path.join(_HERE, "libtk.so")

SYM = {"Z1": 0, "Z2": 1, "FZ2": 2, "U1": 3, "U1xFZ2": 4}
NCOMP = {0: 0, 1: 1, 2: 1, 3: 1, 4: 2}
DTYPE = {"f64": 0, "f32": 1}
PREC = {"native": 0, "f32": 1, "bf16x3": 2}
STAGE_PERMUTE, STAGE_GEMM, STAGE_ZERO, STAGE_ALL = 1, 2, 4, 7
STAGE_PERMUTE_A, STAGE_PERMUTE_B = 8, 16
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "SPACE_MISMATCH", 3: "CHARGE", 4: "DTYPE", 5: "UNSUPPORTED",
          6: "OOM", 7: "HIP"}


class TkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tk error {STATUS.get(status, status)}: {msg}")
        self.status = status


class tk_space(C.Structure):
    _fields_ = [("nsect", C.c_int32), ("charges", C.POINTER(C.c_int32)),
                ("degeneracies", C.POINTER(C.c_int64)), ("isdual", C.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2508_10076_amd.build.build()")
# torch provides device memory and streams; loading it first makes libtk.so
# bind to the HIP runtime torch already uses (same SONAME), so one process
# never holds two HIP runtimes.
import torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)

_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_SIGS = {
    "tk_context_create": [C.c_int32, C.POINTER(_P)],
    "tk_context_destroy": [_P],
    "tk_tensor_create": [_P, C.c_int32, C.c_int32, C.POINTER(tk_space), C.c_int32, C.POINTER(tk_space), C.c_int32,
                         _P, C.c_uint64, C.POINTER(_P)],
    "tk_tensor_destroy": [_P],
    "tk_tensor_info": [_P, _I32P, _I32P, _I32P, _I32P, _I64P, _I64P, _I64P],
    "tk_tensor_blocks": [_P, C.c_int64, C.c_int64, _I32P, _I64P, _I64P],
    "tk_tensor_sectors": [_P, C.c_int64, C.c_int64, _I32P, _I64P, _I64P, _I64P],
    "tk_tensor_space": [_P, C.c_int32, C.POINTER(tk_space)],
    "tk_tensor_data": [_P, C.POINTER(_P), C.POINTER(C.c_uint64)],
    "tk_tensor_create_permuted": [_P, _P, _I32P, C.c_int32, _I32P, C.c_int32, _P, C.c_uint64, C.POINTER(_P)],
    "tk_tensor_create_contracted": [_P, _P, _I32P, C.c_int32, _I32P, C.c_int32, _P, _I32P, C.c_int32, _I32P,
                                    C.c_int32, _I32P, C.c_int32, _I32P, C.c_int32, _P, C.c_uint64, C.POINTER(_P)],
    "tk_tensor_create_adjoint": [_P, _P, _P, C.c_uint64, C.POINTER(_P)],
    "tk_tensor_permute": [_P, _P, _I32P, C.c_int32, _I32P, C.c_int32, _P, _P],
    "tk_svd_create": [_P, _P, _I32P, C.c_int32, _I32P, C.c_int32, C.c_int64, C.c_double, _P, C.POINTER(_P)],
    "tk_svd_create_factor": [_P, _P, C.c_int32, _P, C.c_uint64, C.POINTER(_P)],
    "tk_svd_finish": [_P, _P, _P, _P, C.POINTER(C.c_double), _P],
    "tk_svd_info": [_P, _I64P, _I64P, _I32P],
    "tk_svd_destroy": [_P],
    "tk_tensor_create_traced": [_P, _P, _I32P, C.c_int32, _I32P, C.c_int32, _I32P, _I32P, C.c_int32, _P,
                                C.c_uint64, C.POINTER(_P)],
    "tk_tensor_trace": [_P, _P, _I32P, C.c_int32, _I32P, C.c_int32, _I32P, _I32P, C.c_int32, C.c_double,
                        C.c_double, _P, _P],
    "tk_tensor_contract": [_P, _P, _I32P, C.c_int32, _I32P, C.c_int32, _P, _I32P, C.c_int32, _I32P, C.c_int32,
                           _I32P, C.c_int32, _I32P, C.c_int32, C.c_double, C.c_double, C.c_int32, _P, _P],
    "tk_tensor_contract_noalloc": [_P, _P, _I32P, C.c_int32, _I32P, C.c_int32, _P, _I32P, C.c_int32, _I32P,
                                   C.c_int32, _I32P, C.c_int32, _I32P, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                   _P, _P],
    "tk_tensor_adjoint": [_P, _P, _P, _P],
    "tk_plan_contract": [_P, _P, _I32P, C.c_int32, _I32P, C.c_int32, _P, _I32P, C.c_int32, _I32P, C.c_int32,
                         _I32P, C.c_int32, _I32P, C.c_int32, C.c_int32, _P, C.POINTER(_P)],
    "tk_plan_execute": [_P, _P, _P, _P, C.c_double, C.c_double, _P],
    "tk_plan_destroy": [_P],
    "tk_plan_execute_stages": [_P, _P, _P, _P, C.c_double, C.c_double, C.c_int32, _P],
    "tk_plan_info": [_P, _I64P, C.POINTER(C.c_double), _I64P, _I64P, _I32P, _I32P, _I32P],
    "tk_plan_gemms": [_P, C.c_int64, C.c_int64, _I64P],
    "tk_plan_counts": [_P, _I64P],
    "tk_plan_worklist": [_P, C.c_int32, _I64P, _I64P, _I64P, _I32P, _I32P, _I32P, _I64P, _I32P],
    "tk_permute_map": [_P, _I32P, C.c_int32, _I32P, C.c_int32, _P, _I64P, _I32P],
    "tk_batch_create": [_P, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.c_int32, C.c_double,
                        C.c_double, C.POINTER(_P)],
    "tk_batch_launch": [_P, _P],
    "tk_batch_capture": [_P, _P],
    "tk_batch_replay": [_P, _P],
    "tk_batch_info": [_P, _I64P, _I64P, C.POINTER(C.c_double), _I32P, _I32P, _I32P],
    "tk_batch_destroy": [_P],
    "tk_tile_shapes": [_I32P, _I32P],
    "tk_plan_set_tile": [_P, C.c_int32, C.c_int32, C.c_int32],
    "tk_su2_plan_create": [C.c_int32, C.c_int32, _I32P, _I32P, _I64P, _I32P, _I32P, C.POINTER(_P)],
    "tk_su2_plan_create_dual": [C.c_int32, C.c_int32, _I32P, _I32P, _I64P, _I32P, _I32P, C.c_int32, _I32P,
                                C.c_int32, C.POINTER(_P)],
    "tk_su2_plan_legs": [_P, _I32P, _I32P, _I32P],
    "tk_su2_plan_info": [_P, _I64P, _I64P, _I64P],
    "tk_su2_plan_contribs": [_P, C.c_int64, _I64P, _I64P, C.POINTER(C.c_double)],
    "tk_su2_permute": [_P, C.c_int32, _P, _P, C.c_double, C.c_double, _P],
    "tk_su2_plan_destroy": [_P],
    "tk_batch_set_tile": [_P, C.c_int32, C.c_int32, C.c_int32],
}
for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int32
lib.tk_last_error.restype = C.c_char_p
lib.tk_last_error.argtypes = []
lib.tk_version.restype = C.c_char_p
lib.tk_version.argtypes = []
lib.tk_device_alloc_count.restype = C.c_uint64
lib.tk_device_alloc_count.argtypes = []
SCRATCH_BYTES = 64 << 20   # TK_SCRATCH_BYTES


def _check(st):
    if st != 0:
        raise TkError(st, lib.tk_last_error().decode())


def _ilist(v):
    v = [int(x) for x in v]
    arr = (C.c_int32 * max(1, len(v)))(*v)
    return arr, len(v)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class _SpaceArray:
    """Keeps the ctypes arrays of a list of spaces alive."""

    def __init__(self, sym: int, spaces):
        self.keep = []
        self.arr = (tk_space * max(1, len(spaces)))()
        nc = NCOMP[sym]
        for i, sp in enumerate(spaces):
            sectors, degs, dual = sp[0], sp[1], sp[2]
            flat = [int(x) for s in sectors for x in s][: len(sectors) * nc] if nc else []
            ch = (C.c_int32 * max(1, len(flat)))(*flat)
            dg = (C.c_int64 * len(degs))(*[int(d) for d in degs])
            self.keep += [ch, dg]
            self.arr[i].nsect = len(degs)
            self.arr[i].charges = ch if nc else None
            self.arr[i].degeneracies = dg
            self.arr[i].isdual = 1 if dual else 0
        self.n = len(spaces)


class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib.tk_context_create(device, C.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib.tk_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tensor:
    """A TensorMap handle.  With a context its storage is a torch tensor on
    the context's device (allocated here unless `storage` is given)."""

    def __init__(self, handle, ctx=None, storage=None):
        self.h = handle
        self.ctx = ctx
        self.storage = storage

    # -- construction --------------------------------------------------------
    @classmethod
    def create(cls, ctx, sym, cod, dom, dtype="f64", storage=None):
        symi = SYM[sym] if isinstance(sym, str) else int(sym)
        dt = DTYPE[dtype] if isinstance(dtype, str) else int(dtype)
        sc, sd = _SpaceArray(symi, cod), _SpaceArray(symi, dom)
        if ctx is None:
            h = C.c_void_p()
            _check(lib.tk_tensor_create(None, symi, dt, sc.arr, sc.n, sd.arr, sd.n, None, 0, C.byref(h)))
            return cls(h)
        # ask the structure for its size first, then wrap a torch buffer
        probe = C.c_void_p()
        _check(lib.tk_tensor_create(None, symi, dt, sc.arr, sc.n, sd.arr, sd.n, None, 0, C.byref(probe)))
        n = C.c_int64()
        _check(lib.tk_tensor_info(probe, None, None, None, None, C.byref(n), None, None))
        lib.tk_tensor_destroy(probe)
        storage = _alloc(ctx, n.value, dt) if storage is None else storage
        h = C.c_void_p()
        _check(lib.tk_tensor_create(ctx.h, symi, dt, sc.arr, sc.n, sd.arr, sd.n, C.c_void_p(storage.data_ptr()),
                                    storage.numel() * storage.element_size(), C.byref(h)))
        return cls(h, ctx, storage)

    @classmethod
    def _derived(cls, ctx, fn, *args):
        probe = C.c_void_p()
        _check(fn(None, *args, None, 0, C.byref(probe)))
        if ctx is None:
            return cls(probe)
        n = C.c_int64()
        dt = C.c_int32()
        st = lib.tk_tensor_info(probe, None, C.byref(dt), None, None, C.byref(n), None, None)
        lib.tk_tensor_destroy(probe)
        _check(st)
        storage = _alloc(ctx, n.value, dt.value)
        h = C.c_void_p()
        _check(fn(ctx.h, *args, C.c_void_p(storage.data_ptr()), storage.numel() * storage.element_size(),
                  C.byref(h)))
        return cls(h, ctx, storage)

    def close(self):
        if self.h:
            lib.tk_tensor_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries -------------------------------------------------------------
    def _info(self):
        sym, dt, n1, n2 = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        ne, nb, ns = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib.tk_tensor_info(self.h, C.byref(sym), C.byref(dt), C.byref(n1), C.byref(n2), C.byref(ne),
                                  C.byref(nb), C.byref(ns)))
        return sym.value, dt.value, n1.value, n2.value, ne.value, nb.value, ns.value

    @property
    def sym(self):
        return self._info()[0]

    @property
    def dtype(self):
        return self._info()[1]

    @property
    def ncod(self):
        return self._info()[2]

    @property
    def ndom(self):
        return self._info()[3]

    @property
    def nelem(self):
        return self._info()[4]

    @property
    def nblocks(self):
        return self._info()[5]

    @property
    def nsectors(self):
        return self._info()[6]

    def blocks(self, first=0, count=None):
        """(sector indices (count, rank), offsets, ld) of channels in storage order."""
        _, _, n1, n2, _, nb, _ = self._info()
        count = nb - first if count is None else count
        idx = np.zeros((count, n1 + n2), np.int32)
        off = np.zeros(count, np.int64)
        ld = np.zeros(count, np.int64)
        _check(lib.tk_tensor_blocks(self.h, first, count, idx.ctypes.data_as(_I32P), off.ctypes.data_as(_I64P),
                                    ld.ctypes.data_as(_I64P)))
        return idx, off, ld

    def sectors(self):
        sym, _, _, _, _, _, ns = self._info()
        nc = NCOMP[sym]
        ch = np.zeros((ns, max(1, nc)), np.int32)
        r, c, o = (np.zeros(ns, np.int64) for _ in range(3))
        _check(lib.tk_tensor_sectors(self.h, 0, ns, ch.ctypes.data_as(_I32P), r.ctypes.data_as(_I64P),
                                     c.ctypes.data_as(_I64P), o.ctypes.data_as(_I64P)))
        return ch[:, :nc], r, c, o

    def space(self, leg):
        s = tk_space()
        _check(lib.tk_tensor_space(self.h, leg, C.byref(s)))
        nc = NCOMP[self.sym]
        degs = [s.degeneracies[k] for k in range(s.nsect)]
        if nc:
            sect = [tuple(s.charges[nc * k + c] for c in range(nc)) for k in range(s.nsect)]
        else:
            sect = [()] * s.nsect
        return sect, degs, bool(s.isdual)

    def data_ptr(self):
        p = C.c_void_p()
        _check(lib.tk_tensor_data(self.h, C.byref(p), None))
        return p.value


def _alloc(ctx, n, dtype):
    import torch
    tdt = torch.float64 if int(dtype) == 0 else torch.float32
    return torch.empty(max(1, int(n)), dtype=tdt, device=f"cuda:{ctx.device}")


# ---------------------------------------------------------------------------
# operations (names as in the C-ABI)
# ---------------------------------------------------------------------------
def tensor_create(ctx, sym, cod, dom, dtype="f64", storage=None):
    return Tensor.create(ctx, sym, cod, dom, dtype, storage)


def tensor_create_permuted(ctx, A, p, q):
    pa, npa = _ilist(p)
    qa, nqa = _ilist(q)
    return Tensor._derived(ctx, lambda c, *r: lib.tk_tensor_create_permuted(c, A.h, pa, npa, qa, nqa, *r))


def tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB):
    lists = [_ilist(v) for v in (pA, qA, pB, qB, pAB, qAB)]
    (a1, n1), (a2, n2), (b1, m1), (b2, m2), (c1, k1), (c2, k2) = lists
    return Tensor._derived(ctx, lambda c, *r: lib.tk_tensor_create_contracted(
        c, A.h, a1, n1, a2, n2, B.h, b1, m1, b2, m2, c1, k1, c2, k2, *r))


def tensor_create_traced(ctx, A, p, q, t1, t2):
    (pa, npa), (qa, nqa), (a, na), (b, nb) = [_ilist(v) for v in (p, q, t1, t2)]
    if na != nb:
        raise ValueError("t1 and t2 differ in length")
    return Tensor._derived(ctx, lambda c, *r: lib.tk_tensor_create_traced(c, A.h, pa, npa, qa, nqa, a, b, na, *r))


def tensor_trace(ctx, A, p, q, t1, t2, alpha=1.0, beta=0.0, C_=None, stream=None):
    if C_ is None:
        C_ = tensor_create_traced(ctx, A, p, q, t1, t2)
    (pa, npa), (qa, nqa), (a, na), (b, nb) = [_ilist(v) for v in (p, q, t1, t2)]
    if na != nb:
        raise ValueError("t1 and t2 differ in length")
    _check(lib.tk_tensor_trace(ctx.h, A.h, pa, npa, qa, nqa, a, b, na, float(alpha), float(beta), C_.h,
                               _stream(stream)))
    return C_


def tensor_svd(ctx, A, p, q, max_dim=-1, cutoff=0.0, stream=None, info=False):
    """Truncated SVD A~ = U o S o Vh of A~ = permute(A, (p, q)); returns
    (U, S, Vh, truncation error), and with info=True also a dict with the
    number of sector matrices, of kept values and the largest sweep count."""
    (pa, npa), (qa, nqa) = _ilist(p), _ilist(q)
    h = C.c_void_p()
    _check(lib.tk_svd_create(ctx.h, A.h, pa, npa, qa, nqa, int(max_dim), float(cutoff), _stream(stream),
                             C.byref(h)))
    try:
        ns, nk, sw = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib.tk_svd_info(h, C.byref(ns), C.byref(nk), C.byref(sw)))
        U, S, Vh = (Tensor._derived(ctx, lambda c, *r, w=w: lib.tk_svd_create_factor(c, h, w, *r)) for w in range(3))
        err = C.c_double()
        _check(lib.tk_svd_finish(h, U.h, S.h, Vh.h, C.byref(err), _stream(stream)))
    finally:
        lib.tk_svd_destroy(h)
    if info:
        return U, S, Vh, err.value, dict(nsectors=ns.value, nkept=nk.value, max_sweeps=sw.value)
    return U, S, Vh, err.value


class SU2Plan:
    """permute(A, (p, q)) of an SU(2) tensor map cod <- dom whose legs are
    lists of (twice the spin, degeneracy); p and q permute the codomain and
    the domain legs (numbered as in tk_su2_plan_create)."""

    def __init__(self, cod, dom, p, q, dual=()):
        legs = [sorted(l) for l in list(cod) + list(dom)]
        nsec, nl = _ilist([len(l) for l in legs])
        tj, _ = _ilist([x for l in legs for x, _ in l])
        deg = (C.c_int64 * max(1, sum(len(l) for l in legs)))(*[d for l in legs for _, d in l])
        isd, _ = _ilist([1 if k in set(dual) else 0 for k in range(len(legs))])
        (pa, npa), (qa, nqa) = _ilist(p), _ilist(q)
        self.h = C.c_void_p()
        _check(lib.tk_su2_plan_create_dual(len(cod), len(dom), nsec, tj, deg, isd, pa, npa, qa, nqa,
                                           C.byref(self.h)))
        a, b, n = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib.tk_su2_plan_info(self.h, C.byref(a), C.byref(b), C.byref(n)))
        self.in_size, self.out_size, self.ncontrib = a.value, b.value, n.value
        o1, o2 = C.c_int32(), C.c_int32()
        od = (C.c_int32 * len(legs))()
        _check(lib.tk_su2_plan_legs(self.h, C.byref(o1), C.byref(o2), od))
        self.out_dual = tuple(k for k in range(len(legs)) if od[k])

    def contribs(self):
        """Host table: (output array start, input array start, coefficient)."""
        n = max(1, self.ncontrib)
        d, s_, c = (C.c_int64 * n)(), (C.c_int64 * n)(), (C.c_double * n)()
        _check(lib.tk_su2_plan_contribs(self.h, self.ncontrib, d, s_, c))
        return [(d[i], s_[i], c[i]) for i in range(self.ncontrib)]

    def permute(self, A, C_=None, alpha=1.0, beta=0.0, stream=None):
        """C = alpha * permute(A) + beta * C on device tensors (fp64 or fp32)."""
        dt = {torch.float64: 0, torch.float32: 1}[A.dtype]
        if A.numel() != self.in_size:
            raise ValueError("A has %d elements, the plan needs %d" % (A.numel(), self.in_size))
        if C_ is None:
            C_ = torch.zeros(self.out_size, dtype=A.dtype, device=A.device)
        if C_.numel() != self.out_size or C_.dtype != A.dtype or not (A.is_contiguous() and C_.is_contiguous()):
            raise ValueError("C must be a contiguous tensor of the output size and A's dtype")
        _check(lib.tk_su2_permute(self.h, dt, C.c_void_p(A.data_ptr()), C.c_void_p(C_.data_ptr()), float(alpha),
                                  float(beta), _stream(stream)))
        return C_

    def __del__(self, _destroy=lib.tk_su2_plan_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


def tensor_create_adjoint(ctx, A):
    return Tensor._derived(ctx, lambda c, *r: lib.tk_tensor_create_adjoint(c, A.h, *r))


def tensor_permute(ctx, A, p, q, C_=None, stream=None):
    if C_ is None:
        C_ = tensor_create_permuted(ctx, A, p, q)
    pa, npa = _ilist(p)
    qa, nqa = _ilist(q)
    _check(lib.tk_tensor_permute(ctx.h, A.h, pa, npa, qa, nqa, C_.h, _stream(stream)))
    return C_


def tensor_contract(ctx, A, pA, qA, B, pB, qB, pAB, qAB, alpha=1.0, beta=0.0, precision="native", C_=None,
                    stream=None):
    if C_ is None:
        C_ = tensor_create_contracted(ctx, A, pA, qA, B, pB, qB, pAB, qAB)
    (a1, n1), (a2, n2), (b1, m1), (b2, m2), (c1, k1), (c2, k2) = [_ilist(v) for v in (pA, qA, pB, qB, pAB, qAB)]
    prec = PREC[precision] if isinstance(precision, str) else int(precision)
    _check(lib.tk_tensor_contract(ctx.h, A.h, a1, n1, a2, n2, B.h, b1, m1, b2, m2, c1, k1, c2, k2, float(alpha),
                                  float(beta), prec, C_.h, _stream(stream)))
    return C_


def tensor_contract_noalloc(ctx, A, pA, qA, B, pB, qB, pAB, qAB, C_, alpha=1.0, beta=0.0, precision="native",
                            stream=None):
    """tk_tensor_contract_noalloc: the contraction into the existing tensor
    C_, with the library's tables and workspaces in its per-device scratch
    array (no device allocation)."""
    (a1, n1), (a2, n2), (b1, m1), (b2, m2), (c1, k1), (c2, k2) = [_ilist(v) for v in (pA, qA, pB, qB, pAB, qAB)]
    prec = PREC[precision] if isinstance(precision, str) else int(precision)
    _check(lib.tk_tensor_contract_noalloc(ctx.h, A.h, a1, n1, a2, n2, B.h, b1, m1, b2, m2, c1, k1, c2, k2,
                                          float(alpha), float(beta), prec, C_.h, _stream(stream)))
    return C_


def device_alloc_count():
    return int(lib.tk_device_alloc_count())


def tensor_adjoint(ctx, A, C_=None, stream=None):
    if C_ is None:
        C_ = tensor_create_adjoint(ctx, A)
    _check(lib.tk_tensor_adjoint(ctx.h, A.h, C_.h, _stream(stream)))
    return C_


def permute_map(A, p, q, C_):
    pa, npa = _ilist(p)
    qa, nqa = _ilist(q)
    nb = A.nblocks
    dst = np.zeros(nb, np.int64)
    sg = np.zeros(nb, np.int32)
    _check(lib.tk_permute_map(A.h, pa, npa, qa, nqa, C_.h, dst.ctypes.data_as(_I64P), sg.ctypes.data_as(_I32P)))
    return dst, sg


class Plan:
    def __init__(self, ctx, A, pA, qA, B, pB, qB, pAB, qAB, C_, precision="native"):
        (a1, n1), (a2, n2), (b1, m1), (b2, m2), (c1, k1), (c2, k2) = [_ilist(v) for v in (pA, qA, pB, qB, pAB, qAB)]
        prec = PREC[precision] if isinstance(precision, str) else int(precision)
        h = C.c_void_p()
        _check(lib.tk_plan_contract(ctx.h if ctx else None, A.h, a1, n1, a2, n2, B.h, b1, m1, b2, m2, c1, k1, c2, k2,
                                    prec, C_.h, C.byref(h)))
        self.h = h

    def execute(self, A, B, C_, alpha=1.0, beta=0.0, stream=None):
        _check(lib.tk_plan_execute(self.h, A.h, B.h, C_.h, float(alpha), float(beta), _stream(stream)))

    def execute_stages(self, A, B, C_, stages, alpha=1.0, beta=0.0, stream=None):
        _check(lib.tk_plan_execute_stages(self.h, A.h, B.h, C_.h, float(alpha), float(beta), int(stages),
                                          _stream(stream)))

    def info(self):
        ng, nz, ws = C.c_int64(), C.c_int64(), C.c_int64()
        fl = C.c_double()
        tm, tn, tkk = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib.tk_plan_info(self.h, C.byref(ng), C.byref(fl), C.byref(nz), C.byref(ws), C.byref(tm),
                                C.byref(tn), C.byref(tkk)))
        return dict(ngemm=ng.value, flops=fl.value, nzero=nz.value, workspace_bytes=ws.value,
                    tile=(tm.value, tn.value, tkk.value))

    def counts(self):
        out = np.zeros(14, np.int64)
        _check(lib.tk_plan_counts(self.h, out.ctypes.data_as(_I64P)))
        keys = ("pre_tasks", "pre_wgs", "zero_tasks", "zero_wgs", "smallk_tasks", "smallk_wgs", "gemm_descs",
                "tiles", "gemm_wgs", "split_groups", "split_slots", "makespan_stages", "smallk_runs", "run_wgs")
        return dict(zip(keys, out.tolist()))

    def worklist(self, kind):
        """Host copy of the zero-range (kind 0) or K-output-run (kind K) work
        list: dict of numpy arrays (see tk_plan_worklist)."""
        cnt = np.zeros(3, np.int64)
        _check(lib.tk_plan_worklist(self.h, int(kind), cnt.ctypes.data_as(_I64P), None, None, None, None, None,
                                    None, None))
        n, nwg, nrec = (int(x) for x in cnt)
        out = dict(vstart=np.zeros(n, np.int64), len=np.zeros(n, np.int64), lin0=np.zeros(n, np.int32),
                   shape=np.zeros(n, np.int32), first=np.zeros(nwg + 1 if nwg else 0, np.int32),
                   wstart=np.zeros(nwg + 1 if nwg else 0, np.int64), dimrec=np.zeros((nrec, 25), np.int32))
        _check(lib.tk_plan_worklist(self.h, int(kind), cnt.ctypes.data_as(_I64P),
                                    out["vstart"].ctypes.data_as(_I64P), out["len"].ctypes.data_as(_I64P),
                                    out["lin0"].ctypes.data_as(_I32P), out["shape"].ctypes.data_as(_I32P),
                                    out["first"].ctypes.data_as(_I32P), out["wstart"].ctypes.data_as(_I64P),
                                    out["dimrec"].ctypes.data_as(_I32P)))
        return out

    def gemms(self):
        n = self.info()["ngemm"]
        out = np.zeros((n, 3), np.int64)
        if n:
            _check(lib.tk_plan_gemms(self.h, 0, n, out.ctypes.data_as(_I64P)))
        return out

    def set_tile(self, tm, tn, tk_):
        _check(lib.tk_plan_set_tile(self.h, int(tm), int(tn), int(tk_)))

    def close(self):
        if self.h:
            lib.tk_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    def __init__(self, ctx, plans, As, Bs, Cs, alpha=1.0, beta=0.0):
        n = len(plans)
        arr = lambda xs: (C.c_void_p * n)(*[x.h.value for x in xs])
        self._keep = (plans, As, Bs, Cs)
        h = C.c_void_p()
        _check(lib.tk_batch_create(ctx.h, arr(plans), arr(As), arr(Bs), arr(Cs), n, float(alpha), float(beta),
                                   C.byref(h)))
        self.h = h

    def launch(self, stream=None):
        _check(lib.tk_batch_launch(self.h, _stream(stream)))

    def capture(self, stream):
        _check(lib.tk_batch_capture(self.h, _stream(stream)))

    def replay(self, stream=None):
        _check(lib.tk_batch_replay(self.h, _stream(stream)))

    def set_tile(self, tm, tn, tk_):
        _check(lib.tk_batch_set_tile(self.h, int(tm), int(tn), int(tk_)))

    def info(self):
        ng, nt = C.c_int64(), C.c_int64()
        fl = C.c_double()
        tm, tn, tkk = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib.tk_batch_info(self.h, C.byref(ng), C.byref(nt), C.byref(fl), C.byref(tm), C.byref(tn),
                                 C.byref(tkk)))
        return dict(ngemm=ng.value, ntiles=nt.value, flops=fl.value, tile=(tm.value, tn.value, tkk.value))

    def close(self):
        if self.h:
            lib.tk_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tile_shapes():
    n = C.c_int32()
    _check(lib.tk_tile_shapes(C.byref(n), None))
    arr = (C.c_int32 * (3 * n.value))()
    _check(lib.tk_tile_shapes(C.byref(n), arr))
    return [(arr[3 * i], arr[3 * i + 1], arr[3 * i + 2]) for i in range(n.value)]


def version():
    return lib.tk_version().decode()
