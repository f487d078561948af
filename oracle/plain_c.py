"""ctypes binding of oracle/plain_gf.c (TEST AND BENCHMARK INFRASTRUCTURE ONLY).

The multi-core schoolbook comparator: textbook field products (Section 1's
classical method; Section 7's field arithmetic), threaded with OpenMP over
rows or over the products of a batch.  Only the tests, ``bench.py`` and the
build step use it; the HIP library never does.

``build()`` compiles ``libgfplain.so`` beside the source with gcc; ``lib()``
loads it and builds it first when it is missing or older than the source.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "plain_gf.c")
LIB = os.path.join(HERE, "libgfplain.so")

_lib = None


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall", SRC, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"gcc failed for {SRC}:\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        u8p, i64 = ctypes.c_void_p, ctypes.c_int64
        L.gf_plain_gemm.argtypes = [ctypes.c_int, ctypes.c_int, u8p, i64, i64, i64, u8p, i64,
                                    u8p, i64, u8p, i64, ctypes.c_int]
        L.gf_plain_gemm_batched.argtypes = [ctypes.c_int, ctypes.c_int, u8p, i64, u8p, u8p,
                                            u8p, u8p, ctypes.c_int]
        L.gf_plain_polymul.argtypes = [ctypes.c_int, ctypes.c_int, i64, u8p, u8p, u8p,
                                       ctypes.c_int]
        L.gf_plain_threads.argtypes = []
        for fn in (L.gf_plain_gemm, L.gf_plain_gemm_batched, L.gf_plain_polymul,
                   L.gf_plain_threads):
            fn.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"{what}: invalid arguments")


def threads_used() -> int:
    """OpenMP threads of the last call."""
    return lib().gf_plain_threads()


def gemm(A: np.ndarray, B: np.ndarray, p: int, P_low, threads: int = 0) -> np.ndarray:
    """C = A B over GF(p^k); A is M x K x k, B is K x N x k (uint8, C order)."""
    A = np.ascontiguousarray(A, dtype=np.uint8)
    B = np.ascontiguousarray(B, dtype=np.uint8)
    k = len(P_low)
    M, K, N = A.shape[0], A.shape[1], B.shape[1]
    assert A.shape[2] == k and B.shape[0] == K and B.shape[2] == k
    C = np.zeros((M, N, k), dtype=np.uint8)
    P = np.asarray(P_low, dtype=np.uint8)
    _check(lib().gf_plain_gemm(p, k, _ptr(P), M, N, K, _ptr(A), K, _ptr(B), N, _ptr(C), N,
                               threads), "gf_plain_gemm")
    return C


def gemm_batched(As, Bs, p: int, P_low, threads: int = 0):
    """Independent products C_g = A_g B_g over GF(p^k)."""
    k = len(P_low)
    As = [np.ascontiguousarray(a, dtype=np.uint8) for a in As]
    Bs = [np.ascontiguousarray(b, dtype=np.uint8) for b in Bs]
    Cs = [np.zeros((a.shape[0], b.shape[1], k), dtype=np.uint8) for a, b in zip(As, Bs)]
    mnk = np.array([(a.shape[0], b.shape[1], a.shape[1]) for a, b in zip(As, Bs)],
                   dtype=np.int64).reshape(-1)
    ptrs = lambda xs: np.array([x.ctypes.data for x in xs], dtype=np.uint64)  # noqa: E731
    pa, pb, pc = ptrs(As), ptrs(Bs), ptrs(Cs)
    P = np.asarray(P_low, dtype=np.uint8)
    _check(lib().gf_plain_gemm_batched(p, k, _ptr(P), len(As), _ptr(mnk), _ptr(pa), _ptr(pb),
                                       _ptr(pc), threads), "gf_plain_gemm_batched")
    return Cs


def polymul_batch(a: np.ndarray, b: np.ndarray, p: int, threads: int = 0) -> np.ndarray:
    """out[r] = a[r] b[r] in GF(p)[X] for n x k coefficient arrays."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    n, k = a.shape
    c = np.zeros((n, 2 * k - 1), dtype=np.uint8)
    _check(lib().gf_plain_polymul(p, k, n, _ptr(a), _ptr(b), _ptr(c), threads),
           "gf_plain_polymul")
    return c
