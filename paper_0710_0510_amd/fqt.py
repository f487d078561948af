"""Python binding of libfqt.so (the C ABI in include/fqt.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  torch supplies device memory (tensor data pointers) and the
current HIP stream.  The binding never falls back to any other
implementation: if the library is missing it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfqt.so")

FQT_OK = 0
STATUS_NAMES = {
    0: "FQT_OK", 1: "FQT_ERR_INVALID_ARG", 2: "FQT_ERR_BOUNDS", 3: "FQT_ERR_NOT_PRIME",
    4: "FQT_ERR_REDUCIBLE", 5: "FQT_ERR_UNSUPPORTED", 6: "FQT_ERR_DEVICE", 7: "FQT_ERR_OOM",
}
PATHS = {"auto": 0, "packed": 1, "int8": 2, "plain": 3}
PATH_NAMES = {v: k for k, v in PATHS.items()}
UNPACK_POLY, UNPACK_FIELD = 0, 1

EXPORTED = [
    "fqt_field_create", "fqt_field_destroy", "fqt_field_tables", "fqt_params", "fqt_pack",
    "fqt_unpack_redq", "fqt_unpack_redq_u64", "fqt_polymul_batch", "fqt_gemm_gfpk",
    "fqt_gemm_gfpk_ex", "fqt_gemm_gfpk_batched", "fqt_gemm_gfpk_batched_ex", "fqt_autotune",
    "fqt_tile_count", "fqt_last_error", "fqt_version", "fqt_polymul_dfqt", "fqt_polymul_delayed",
    "fqt_log_info", "fqt_to_log", "fqt_from_log", "fqt_log_add", "fqt_gemm_log",
    "fqt_gemm_winograd", "fqt_polymul_dfqt_batched", "fqt_autotune_polymul",
    "fqt_polymul_dfqt_batched_noalloc",
]


class FqtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))


class GemmOpts(ctypes.Structure):
    _fields_ = [("log2q", ctypes.c_uint32), ("n_q", ctypes.c_uint32),
                ("tile", ctypes.c_uint32), ("boundary", ctypes.c_uint32),
                ("centered", ctypes.c_uint32)]


class PolyDesc(ctypes.Structure):
    """fqt_poly_desc: c (la + lb - 1 coefficients) = a (la) * b (lb)."""
    _fields_ = [("la", ctypes.c_int64), ("lb", ctypes.c_int64), ("a", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("c", ctypes.c_void_p)]


class GemmDesc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64), ("ldc", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           f"`python paper_0710_0510_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    c_int, c_u32, c_u64, c_i64, c_sz = (ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                                       ctypes.c_int64, ctypes.c_size_t)
    vp = ctypes.c_void_p
    sig = {
        "fqt_field_create": (c_int, [c_u32, c_u32, ctypes.POINTER(c_u32), ctypes.POINTER(vp)]),
        "fqt_field_destroy": (None, [vp]),
        "fqt_field_tables": (c_int, [vp, c_u64, vp, vp, ctypes.POINTER(c_sz)]),
        "fqt_params": (c_int, [c_u32, c_u32, c_u64, c_int, c_int, ctypes.POINTER(c_u64),
                               ctypes.POINTER(c_u64)]),
        "fqt_pack": (c_int, [vp, c_u64, vp, c_sz, vp, vp]),
        "fqt_unpack_redq": (c_int, [vp, c_u64, vp, c_sz, c_u32, c_int, vp, vp]),
        "fqt_unpack_redq_u64": (c_int, [vp, c_u64, vp, c_sz, c_u32, c_int, vp, vp]),
        "fqt_polymul_batch": (c_int, [c_u32, c_u32, c_u64, vp, vp, c_sz, vp, vp]),
        "fqt_polymul_dfqt": (c_int, [c_u32, c_u32, c_u32, c_u32, c_u32, c_u32, vp, vp, c_i64,
                                     c_i64, vp, vp]),
        "fqt_polymul_delayed": (c_int, [c_u32, vp, vp, c_i64, c_i64, vp, vp]),
        "fqt_polymul_dfqt_batched": (c_int, [c_u32, c_u32, c_u32, c_u32, c_u32, c_u32, c_i64,
                                             ctypes.POINTER(PolyDesc), vp]),
        "fqt_polymul_dfqt_batched_noalloc": (c_int, [c_u32, c_u32, c_u32, c_u32, c_u32, c_u32,
                                                     c_i64, ctypes.POINTER(PolyDesc), vp]),
        "fqt_autotune_polymul": (c_int, [c_u32, c_i64, ctypes.POINTER(PolyDesc),
                                         ctypes.c_char_p, ctypes.POINTER(c_u32),
                                         ctypes.POINTER(c_u32), ctypes.POINTER(c_u32), vp]),
        "fqt_gemm_gfpk": (c_int, [vp, c_int, c_i64, c_i64, c_i64, vp, c_i64, vp, c_i64, vp,
                                  c_i64, vp]),
        "fqt_gemm_gfpk_ex": (c_int, [vp, c_int, ctypes.POINTER(GemmOpts), c_i64, c_i64, c_i64,
                                     vp, c_i64, vp, c_i64, vp, c_i64, vp]),
        "fqt_gemm_gfpk_batched": (c_int, [vp, c_int, c_i64, ctypes.POINTER(GemmDesc), vp]),
        "fqt_gemm_gfpk_batched_ex": (c_int, [vp, c_int, ctypes.POINTER(GemmOpts), c_i64,
                                             ctypes.POINTER(GemmDesc), vp]),
        "fqt_autotune": (c_int, [vp, c_int, c_i64, ctypes.POINTER(GemmDesc), ctypes.c_char_p,
                                 ctypes.POINTER(c_int), ctypes.POINTER(GemmOpts), vp]),
        "fqt_gemm_winograd": (c_int, [vp, c_int, ctypes.POINTER(GemmOpts), c_u32, c_i64, c_i64,
                                      c_i64, vp, c_i64, vp, c_i64, vp, c_i64, vp]),
        "fqt_log_info": (c_int, [vp, ctypes.POINTER(c_u32), ctypes.POINTER(c_u32)]),
        "fqt_to_log": (c_int, [vp, vp, c_i64, vp, vp]),
        "fqt_from_log": (c_int, [vp, vp, c_i64, vp, vp]),
        "fqt_log_add": (c_int, [vp, vp, vp, c_i64, vp, vp]),
        "fqt_gemm_log": (c_int, [vp, ctypes.POINTER(GemmOpts), c_i64, c_i64, c_i64, vp, c_i64,
                                 vp, c_i64, vp, c_i64, vp]),
        "fqt_tile_count": (c_u32, [c_int]),
        "fqt_last_error": (ctypes.c_char_p, []),
        "fqt_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int) -> None:
    if status != FQT_OK:
        raise FqtError(status, lib().fqt_last_error().decode())


def last_error() -> str:
    return lib().fqt_last_error().decode()


def version() -> str:
    return lib().fqt_version().decode()


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def params(p: int, k: int, n_q: int, pow2: bool = True, carry_in: bool = False) -> Tuple[int, int]:
    """(q, largest n_q for q) from eq. (2); raises FqtError(FQT_ERR_BOUNDS)."""
    q, nq = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib().fqt_params(p, k, n_q, int(pow2), int(carry_in), ctypes.byref(q), ctypes.byref(nq)))
    return q.value, nq.value


def params_raw(p: int, k: int, n_q: int, pow2: bool = True, carry_in: bool = False):
    """(status, q, nq_max) without raising."""
    q, nq = ctypes.c_uint64(0), ctypes.c_uint64(0)
    st = lib().fqt_params(p, k, n_q, int(pow2), int(carry_in), ctypes.byref(q), ctypes.byref(nq))
    return st, q.value, nq.value


class Field:
    """GF(p^k) with defining polynomial X^k + sum P_low[i] X^i."""

    def __init__(self, p: int, k: int, P_low: Sequence[int] = ()):
        arr = (ctypes.c_uint32 * max(k, 1))(*([int(x) for x in P_low] or [0] * k))
        h = ctypes.c_void_p(0)
        _check(lib().fqt_field_create(p, k, arr if P_low else None, ctypes.byref(h)))
        self.handle = h
        self.p, self.k, self.P_low = p, k, tuple(P_low)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().fqt_field_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tables(self, q: int):
        """Host copies (L, H) of the Thm. 3 tables as lists of uint32."""
        n = ctypes.c_size_t(0)
        _check(lib().fqt_field_tables(self.handle, q, None, None, ctypes.byref(n)))
        L = (ctypes.c_uint32 * n.value)()
        H = (ctypes.c_uint32 * n.value)()
        _check(lib().fqt_field_tables(self.handle, q, L, H, ctypes.byref(n)))
        return list(L), list(H)


def create_field_status(p: int, k: int, P_low: Sequence[int]):
    """Status code of fqt_field_create (the handle is destroyed)."""
    arr = (ctypes.c_uint32 * max(k, 1))(*([int(x) for x in P_low] or [0] * max(k, 1)))
    h = ctypes.c_void_p(0)
    st = lib().fqt_field_create(p, k, arr if P_low else None, ctypes.byref(h))
    if st == FQT_OK:
        lib().fqt_field_destroy(h)
    return st


# ---- device entry points (torch tensors on the current device) -----------------

def pack(field: Field, q: int, coeffs, out=None, stream=None):
    import torch
    n = coeffs.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=coeffs.device)
    _check(lib().fqt_pack(field.handle, q, _ptr(coeffs), n, _ptr(out), _stream(stream)))
    return out


def unpack_redq(field: Field, q: int, packed, ndigits: int, mode: int, out=None, stream=None):
    import torch
    n = packed.shape[0]
    ob = ndigits if mode == UNPACK_POLY else field.k
    if out is None:
        out = torch.empty((n, ob), dtype=torch.uint8, device=packed.device)
    fn = lib().fqt_unpack_redq_u64 if packed.dtype == torch.int64 else lib().fqt_unpack_redq
    _check(fn(field.handle, q, _ptr(packed), n, ndigits, mode, _ptr(out), _stream(stream)))
    return out


def polymul_batch(p: int, k: int, q: int, a, b, out=None, stream=None):
    import torch
    n = a.shape[0]
    if out is None:
        out = torch.empty((n, 2 * k - 1), dtype=torch.uint8, device=a.device)
    _check(lib().fqt_polymul_batch(p, k, q, _ptr(a), _ptr(b), n, _ptr(out), _stream(stream)))
    return out


def _poly_operands(a, b, name: str):
    """count x len uint8 device tensors, rows contiguous."""
    import torch
    for t in (a, b):
        if t.dtype != torch.uint8 or t.dim() != 2 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name}: operands must be contiguous (count, len) uint8 device tensors")
    if a.shape != b.shape:
        raise ValueError(f"{name}: operand shapes differ: {tuple(a.shape)} vs {tuple(b.shape)}")


def polymul_dfqt(p: int, d: int, a, b, log2q: int = 0, n_q: int = 0, boundary: int = 0,
                 out=None, stream=None, centered: int = 0):
    """d-FQT products of long polynomials (Section 6): out[i] = a[i] * b[i];
    centered=1 packs centred chunks (about twice the products per block)."""
    import torch
    _poly_operands(a, b, "polymul_dfqt")
    count, length = a.shape
    if out is None:
        out = torch.empty((count, max(2 * length - 1, 0)), dtype=torch.uint8, device=a.device)
    _check(lib().fqt_polymul_dfqt(p, d, log2q, n_q, boundary, centered, _ptr(a), _ptr(b), count,
                                  length, _ptr(out), _stream(stream)))
    return out


def make_poly_descs(As, Bs, Cs):
    """Descriptors of an uneven polynomial batch: A[i], B[i] 1-D uint8 device
    tensors (any lengths), C[i] of len(A[i]) + len(B[i]) - 1 bytes (or 0)."""
    arr = (PolyDesc * len(As))()
    for i, (a, b, c) in enumerate(zip(As, Bs, Cs)):
        for t, name in ((a, "A"), (b, "B"), (c, "C")):
            if t.dim() != 1 or not t.is_cuda or not t.is_contiguous() or t.element_size() != 1:
                raise ValueError(f"{name}[{i}]: expected a contiguous 1-D uint8 device tensor")
        la, lb = a.shape[0], b.shape[0]
        want = la + lb - 1 if la and lb else 0
        if c.shape[0] != want:
            raise ValueError(f"pair {i}: C holds {c.shape[0]} coefficients, not {want}")
        arr[i] = PolyDesc(la, lb, a.data_ptr(), b.data_ptr(), c.data_ptr())
    return arr


def poly_descs_flat(a, b, c, lens):
    """Descriptors of an uneven batch held in three flat device buffers:
    pair i reads la_i bytes of ``a`` and lb_i of ``b`` at the running sums of
    the earlier lengths and writes la_i + lb_i - 1 bytes of ``c`` (none when a
    length is 0) at the running sum of the earlier output lengths.
    ``lens`` is a host count x 2 integer array of (la, lb)."""
    lens = np.asarray(lens, dtype=np.int64).reshape(-1, 2)
    la, lb = lens[:, 0], lens[:, 1]
    lc = np.where((la > 0) & (lb > 0), la + lb - 1, 0)
    for t, need, name in ((a, la.sum(), "a"), (b, lb.sum(), "b"), (c, lc.sum(), "c")):
        if t.dim() != 1 or not t.is_cuda or not t.is_contiguous() or t.element_size() != 1:
            raise ValueError(f"{name}: expected a contiguous 1-D uint8 device tensor")
        if t.shape[0] < need:
            raise ValueError(f"{name}: {t.shape[0]} bytes, the lengths need {need}")
    off = lambda v: np.concatenate(([0], np.cumsum(v)[:-1])).astype(np.uint64)
    rec = np.zeros(len(lens), dtype=[("la", "<i8"), ("lb", "<i8"), ("a", "<u8"), ("b", "<u8"),
                                     ("c", "<u8")])
    rec["la"], rec["lb"] = la, lb
    rec["a"] = np.uint64(a.data_ptr()) + off(la)
    rec["b"] = np.uint64(b.data_ptr()) + off(lb)
    rec["c"] = np.uint64(c.data_ptr()) + off(lc)
    assert rec.dtype.itemsize == ctypes.sizeof(PolyDesc)
    return (PolyDesc * len(lens)).from_buffer_copy(rec.tobytes())


def polymul_dfqt_batched(p: int, d: int, descs, log2q: int = 0, n_q: int = 0,
                         boundary: int = 0, centered: int = 0, stream=None):
    """d-FQT (Section 6) over an uneven batch described by ``make_poly_descs``,
    in one persistent launch replayed from a captured graph."""
    _check(lib().fqt_polymul_dfqt_batched(p, d, log2q, n_q, boundary, centered, len(descs),
                                          descs, _stream(stream)))


def polymul_dfqt_batched_noalloc(p: int, d: int, descs, log2q: int = 0, n_q: int = 0,
                                 boundary: int = 0, centered: int = 0, stream=None):
    """As ``polymul_dfqt_batched`` without any device allocation: the
    descriptors go to the library's static per-GPU array, no plan, no graph."""
    _check(lib().fqt_polymul_dfqt_batched_noalloc(p, d, log2q, n_q, boundary, centered,
                                                  len(descs), descs, _stream(stream)))


def autotune_polymul(p: int, descs, cache_path: Optional[str] = None, stream=None):
    """The fastest (d, centered, boundary) for an uneven batch; returns a dict."""
    d, cen, bnd = ctypes.c_uint32(0), ctypes.c_uint32(0), ctypes.c_uint32(0)
    _check(lib().fqt_autotune_polymul(p, len(descs), descs,
                                      cache_path.encode() if cache_path else None,
                                      ctypes.byref(d), ctypes.byref(cen), ctypes.byref(bnd),
                                      _stream(stream)))
    return {"d": d.value, "centered": cen.value, "boundary": bnd.value}


def polymul_delayed(p: int, a, b, out=None, stream=None):
    """The classical product with delayed reduction (eq. (3)), the comparator."""
    import torch
    _poly_operands(a, b, "polymul_delayed")
    count, length = a.shape
    if out is None:
        out = torch.empty((count, max(2 * length - 1, 0)), dtype=torch.uint8, device=a.device)
    _check(lib().fqt_polymul_delayed(p, _ptr(a), _ptr(b), count, length, _ptr(out),
                                     _stream(stream)))
    return out


def _opts(opts) -> Optional[ctypes.POINTER(GemmOpts)]:
    if opts is None:
        return None
    if isinstance(opts, GemmOpts):
        return ctypes.pointer(opts)
    return ctypes.pointer(GemmOpts(int(opts.get("log2q", 0)), int(opts.get("n_q", 0)),
                                   int(opts.get("tile", 0)), int(opts.get("boundary", 0)),
                                   int(opts.get("centered", 0))))


def _ld(t, k: int) -> int:
    """Leading dimension in elements of a rows x cols x k tensor (the row
    length when the stride carries no information: empty or one row)."""
    rows, cols = t.shape[0], t.shape[1]
    if t.numel() == 0 or rows <= 1:
        return max(cols, 1)
    return t.stride(0) // k


def _matrix(t, k: int, name: str):
    """A rows x cols x k uint8 device tensor whose elements are k consecutive
    bytes and whose rows are equally spaced (any row stride)."""
    import torch
    if t.dtype != torch.uint8 or t.dim() != 3 or t.shape[2] != k:
        raise ValueError(f"{name}: expected a uint8 tensor of shape (rows, cols, {k})")
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a device tensor")
    if t.numel() and ((t.shape[2] > 1 and t.stride(2) != 1) or
                      (t.shape[1] > 1 and t.stride(1) != k)):
        raise ValueError(f"{name}: elements within a row must be contiguous")


def gemm(field: Field, A, B, C=None, path: str = "auto", opts=None, stream=None):
    """C = A B over the field; A is M x K x k, B is K x N x k (uint8)."""
    import torch
    M, K = A.shape[0], A.shape[1]
    N = B.shape[1]
    if C is None:
        C = torch.empty((M, N, field.k), dtype=torch.uint8, device=A.device)
    for t, name in ((A, "A"), (B, "B"), (C, "C")):
        _matrix(t, field.k, name)
    if B.shape[0] != K or tuple(C.shape[:2]) != (M, N):
        raise ValueError(f"shapes do not chain: A {tuple(A.shape)}, B {tuple(B.shape)}, "
                         f"C {tuple(C.shape)}")
    lda, ldb, ldc = _ld(A, field.k), _ld(B, field.k), _ld(C, field.k)
    _check(lib().fqt_gemm_gfpk_ex(field.handle, PATHS[path], _opts(opts), M, N, K, _ptr(A),
                                  lda, _ptr(B), ldb, _ptr(C), ldc, _stream(stream)))
    return C


def gemm_winograd(field: Field, A, B, C=None, levels: int = 1, path: str = "packed", opts=None,
                  stream=None):
    """C = A B over the field with `levels` levels of Winograd's recursion;
    the block products run on `path` with `opts`."""
    import torch
    M, K = A.shape[0], A.shape[1]
    N = B.shape[1]
    if C is None:
        C = torch.empty((M, N, field.k), dtype=torch.uint8, device=A.device)
    for t, name in ((A, "A"), (B, "B"), (C, "C")):
        _matrix(t, field.k, name)
    if B.shape[0] != K or tuple(C.shape[:2]) != (M, N):
        raise ValueError(f"shapes do not chain: A {tuple(A.shape)}, B {tuple(B.shape)}, "
                         f"C {tuple(C.shape)}")
    _check(lib().fqt_gemm_winograd(field.handle, PATHS[path], _opts(opts), levels, M, N, K,
                                   _ptr(A), _ld(A, field.k), _ptr(B), _ld(B, field.k), _ptr(C),
                                   _ld(C, field.k), _stream(stream)))
    return C


def make_descs(field: Field, As, Bs, Cs):
    arr = (GemmDesc * len(As))()
    for i, (A, B, C) in enumerate(zip(As, Bs, Cs)):
        for t, name in ((A, "A"), (B, "B"), (C, "C")):
            _matrix(t, field.k, f"{name}[{i}]")
        if B.shape[0] != A.shape[1] or tuple(C.shape[:2]) != (A.shape[0], B.shape[1]):
            raise ValueError(f"product {i}: shapes do not chain")
        arr[i] = GemmDesc(A.shape[0], B.shape[1], A.shape[1], _ld(A, field.k),
                          _ld(B, field.k), _ld(C, field.k),
                          A.data_ptr(), B.data_ptr(), C.data_ptr())
    return arr


def gemm_batched(field: Field, descs, path: str = "auto", opts=None, stream=None):
    """Run a batch described by ``make_descs`` (the descriptor array)."""
    _check(lib().fqt_gemm_gfpk_batched_ex(field.handle, PATHS[path], _opts(opts), len(descs),
                                          descs, _stream(stream)))


def autotune(field: Field, descs, cache_path: Optional[str] = None, only: str = "auto",
             stream=None):
    """Tune (path, q, tile) on the problem described by ``descs``; ``only``
    restricts the candidates to one path ("packed" or "int8")."""
    path = ctypes.c_int(0)
    best = GemmOpts()
    _check(lib().fqt_autotune(field.handle, PATHS[only], len(descs), descs,
                              cache_path.encode() if cache_path else None, ctypes.byref(path),
                              ctypes.byref(best), _stream(stream)))
    return PATH_NAMES[path.value], {"log2q": best.log2q, "n_q": best.n_q, "tile": best.tile,
                                    "boundary": best.boundary, "centered": best.centered}


def tile_count(path: str) -> int:
    return lib().fqt_tile_count(PATHS[path])


# ---- discrete-log representation (Alg. 4) -------------------------------------


def log_info(field: Field) -> Tuple[int, int]:
    """(base-p index of the generator g, code of zero m = p^k - 1)."""
    g, m = ctypes.c_uint32(0), ctypes.c_uint32(0)
    _check(lib().fqt_log_info(field.handle, ctypes.byref(g), ctypes.byref(m)))
    return g.value, m.value


def _codes(t, name: str):
    import torch
    if t.dtype != torch.uint16 or not t.is_cuda:
        raise ValueError(f"{name}: expected a uint16 device tensor")


def to_log(field: Field, coeffs, out=None, stream=None):
    """Codes of the elements of an (..., k) uint8 device tensor."""
    import torch
    if coeffs.dtype != torch.uint8 or not coeffs.is_cuda or coeffs.shape[-1] != field.k \
            or not coeffs.is_contiguous():
        raise ValueError(f"coeffs: expected a contiguous (..., {field.k}) uint8 device tensor")
    n = coeffs.numel() // field.k
    if out is None:
        out = torch.empty(coeffs.shape[:-1], dtype=torch.uint16, device=coeffs.device)
    _codes(out, "out")
    if out.numel() != n or not out.is_contiguous():
        raise ValueError("out: one contiguous code per element")
    _check(lib().fqt_to_log(field.handle, _ptr(coeffs), n, _ptr(out), _stream(stream)))
    return out


def from_log(field: Field, codes, out=None, stream=None):
    """Coefficient form (..., k) uint8 of a uint16 device tensor of codes."""
    import torch
    _codes(codes, "codes")
    if not codes.is_contiguous():
        raise ValueError("codes: expected a contiguous tensor")
    n = codes.numel()
    if out is None:
        out = torch.empty(tuple(codes.shape) + (field.k,), dtype=torch.uint8, device=codes.device)
    if out.dtype != torch.uint8 or out.numel() != n * field.k or not out.is_contiguous():
        raise ValueError(f"out: expected a contiguous uint8 tensor of {n} x {field.k} bytes")
    _check(lib().fqt_from_log(field.handle, _ptr(codes), n, _ptr(out), _stream(stream)))
    return out


def log_add(field: Field, a, b, out=None, stream=None):
    """a + b in the field, element-wise on codes (Zech table)."""
    import torch
    _codes(a, "a")
    _codes(b, "b")
    if a.shape != b.shape or not a.is_contiguous() or not b.is_contiguous():
        raise ValueError("a, b: contiguous tensors of one shape")
    if out is None:
        out = torch.empty_like(a)
    _codes(out, "out")
    if out.shape != a.shape or not out.is_contiguous():
        raise ValueError("out: a contiguous tensor of the operands' shape")
    _check(lib().fqt_log_add(field.handle, _ptr(a), _ptr(b), a.numel(), _ptr(out),
                             _stream(stream)))
    return out


def _code_matrix(t, name: str):
    _codes(t, name)
    if t.dim() != 2:
        raise ValueError(f"{name}: expected a 2-D tensor of codes")
    if t.numel() and t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name}: codes within a row must be contiguous")


def gemm_log(field: Field, A, B, C=None, opts=None, stream=None):
    """C = A B over the field on codes (M x K and K x N uint16 device tensors)."""
    import torch
    M, K = A.shape[0], A.shape[1]
    N = B.shape[1]
    if C is None:
        C = torch.empty((M, N), dtype=torch.uint16, device=A.device)
    for t, name in ((A, "A"), (B, "B"), (C, "C")):
        _code_matrix(t, name)
    if B.shape[0] != K or tuple(C.shape) != (M, N):
        raise ValueError(f"shapes do not chain: A {tuple(A.shape)}, B {tuple(B.shape)}, "
                         f"C {tuple(C.shape)}")
    ld = lambda t: max(t.shape[1], 1) if t.numel() == 0 or t.shape[0] <= 1 else t.stride(0)
    _check(lib().fqt_gemm_log(field.handle, _opts(opts), M, N, K, _ptr(A), ld(A), _ptr(B), ld(B),
                              _ptr(C), ld(C), _stream(stream)))
    return C
