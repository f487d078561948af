"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every entry point that include/fqt.h declares,
and reject every invalid argument synchronously, before touching a device.
Its Thm. 3 tables are compared with the oracle's, built independently.
"""
import ctypes
import itertools
import os
import re

import pytest

from oracle import gf
from paper_0710_0510_amd import fqt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CONFIG_FIELDS = [(7, 2, (1, 0)), (3, 4, (2, 0, 0, 2)), (5, 3, (3, 3, 0)), (3, 2, (1, 0))]


def header_functions():
    text = open(os.path.join(ROOT, "include", "fqt.h")).read()
    return sorted(set(re.findall(r"\b(fqt_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = fqt.lib()
    declared = header_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(fqt.EXPORTED)


def test_version_string():
    assert "gfx950" in fqt.version()


@pytest.mark.parametrize("p,k", [(7, 2), (3, 4), (5, 3), (3, 2), (5, 3), (2, 3), (11, 1)])
def test_params_match_oracle(p, k):
    q, nq = fqt.params(p, k, 1, pow2=True)
    assert (q, nq) == gf.max_pow2_q(p, k)
    assert gf.eq2_holds(p, k, q, nq) and not gf.eq2_holds(p, k, q, nq + 1)
    st, _, _ = fqt.params_raw(p, k, nq + 1, pow2=True)
    assert fqt.STATUS_NAMES[st] == "FQT_ERR_BOUNDS"
    # general q: largest integer q with q^(2k-1) < 2^53
    qg, nqg = fqt.params(p, k, 1, pow2=False)
    assert qg ** (2 * k - 1) < 2 ** 53 <= (qg + 1) ** (2 * k - 1)
    assert gf.eq2_holds(p, k, qg, nqg) and not gf.eq2_holds(p, k, qg, nqg + 1)


def test_params_survey_values():
    assert fqt.params(7, 2, 1)[0] == 2 ** 17 and fqt.params(7, 2, 1)[1] == 1820
    assert fqt.params(3, 4, 1) == (128, 7)
    assert fqt.params(3, 4, 1, pow2=False) == (190, 11)
    assert fqt.params(5, 3, 1) == (1024, 21)
    assert fqt.params(5, 3, 1, pow2=False) == (1552, 32)
    assert fqt.params(3, 2, 1) == (2 ** 17, 16383)


def test_params_carry_in():
    q, nq = fqt.params(5, 3, 1, pow2=True, carry_in=True)
    assert q > nq * 3 * 16 + 4 and not q > (nq + 1) * 3 * 16 + 4


def test_params_errors():
    st, _, _ = fqt.params_raw(4, 2, 1)
    assert fqt.STATUS_NAMES[st] == "FQT_ERR_NOT_PRIME"
    st, _, _ = fqt.params_raw(7, 2, 0)
    assert fqt.STATUS_NAMES[st] == "FQT_ERR_INVALID_ARG"
    assert "n_q" in fqt.last_error()


@pytest.mark.parametrize("p,k,P,want", [
    (4, 2, (1, 0), "FQT_ERR_NOT_PRIME"),
    (9, 2, (1, 0), "FQT_ERR_NOT_PRIME"),
    (3, 2, (2, 0), "FQT_ERR_REDUCIBLE"),      # X^2 + 2 = (X+1)(X+2)
    (5, 3, (0, 0, 1), "FQT_ERR_REDUCIBLE"),   # X^3 + X^2
    (7, 2, (6, 0), "FQT_ERR_REDUCIBLE"),      # X^2 - 1
    (3, 5, (1, 2, 0, 0, 0), "FQT_ERR_UNSUPPORTED"),
    (131, 2, (1, 0), "FQT_ERR_UNSUPPORTED"),
    (7, 2, (7, 0), "FQT_ERR_INVALID_ARG"),
    (3, 0, (), "FQT_ERR_UNSUPPORTED"),
])
def test_field_create_errors(p, k, P, want):
    assert fqt.STATUS_NAMES[fqt.create_field_status(p, k, P)] == want


def test_field_create_accepts_every_irreducible_quadratic_gf5():
    for low in itertools.product(range(5), repeat=2):
        st = fqt.create_field_status(5, 2, low)
        assert (st == 0) == gf.is_irreducible(list(low), 5), low


@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
@pytest.mark.parametrize("which_q", ["pow2", "general", "other"])
def test_tables_match_oracle(p, k, P, which_q):
    f = fqt.Field(p, k, P)
    q = {"pow2": fqt.params(p, k, 1)[0], "general": fqt.params(p, k, 1, pow2=False)[0],
         "other": 10 ** 6}[which_q]
    L, H = f.tables(q)
    cb = max(1, (p - 1).bit_length())
    assert len(L) == len(H) == 1 << (k * cb)
    seen = set()
    for w in itertools.product(range(p), repeat=k):
        idx = gf.binary_index(w, p)
        seen.add(idx)
        want_L = gf.table_L(list(w), q, p)
        want_H = gf.table_H(list(w), q, p, P)
        assert [(L[idx] >> (8 * s)) & 0xFF for s in range(k)] == want_L
        assert [(H[idx] >> (8 * s)) & 0xFF for s in range(k)] == want_H
        assert L[idx] >> (8 * k) == 0 and H[idx] >> (8 * k) == 0
    for idx in range(len(L)):
        if idx not in seen:
            assert L[idx] == 0 and H[idx] == 0


def test_k1_prime_field_tables():
    f = fqt.Field(11, 1, (0,))
    L, H = f.tables(2 ** 52)
    for u in range(11):
        assert L[u] == 0 and H[u] == u


# ---- argument validation happens before any device work -------------------------

BOGUS = 0x1000  # never dereferenced: every call below must fail validation first


def _gemm_status(field, path, M, N, K, lda, ldb, ldc, A=BOGUS, B=BOGUS + (1 << 30),
                 C=BOGUS + (1 << 31), opts=None):
    L = fqt.lib()
    return fqt.STATUS_NAMES[L.fqt_gemm_gfpk_ex(
        field.handle, fqt.PATHS[path], fqt._opts(opts), M, N, K, ctypes.c_void_p(A), lda,
        ctypes.c_void_p(B), ldb, ctypes.c_void_p(C), ldc, None)]


def test_gemm_validation_errors():
    f = fqt.Field(7, 2, (1, 0))
    assert _gemm_status(f, "packed", -1, 4, 4, 4, 4, 4) == "FQT_ERR_INVALID_ARG"
    assert _gemm_status(f, "packed", 4, 4, 8, 4, 4, 4) == "FQT_ERR_INVALID_ARG"   # lda < K
    assert _gemm_status(f, "packed", 4, 8, 4, 4, 4, 8) == "FQT_ERR_INVALID_ARG"   # ldb < N
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4, A=0) == "FQT_ERR_INVALID_ARG"
    # C overlapping A
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4, A=BOGUS, C=BOGUS + 8) == "FQT_ERR_INVALID_ARG"
    # eq. (2): n_q above the bound for q = 2^17 (1820) and q above 2^17
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4, opts={"n_q": 1821}) == "FQT_ERR_BOUNDS"
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4, opts={"log2q": 18}) == "FQT_ERR_BOUNDS"
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4, opts={"tile": 99}) == "FQT_ERR_INVALID_ARG"
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4,
                        opts={"log2q": 3}) in ("FQT_ERR_BOUNDS", "FQT_ERR_UNSUPPORTED")


def test_direct_tiles_refuse_several_blocks():
    # register-direct tiles other than 11 hold no per-element block state:
    # K > n_q is refused on the host; tile 11 carries it
    f = fqt.Field(3, 4, (2, 0, 0, 2))          # q = 2^7, n_q <= 7
    for tile in (7, 8, 9, 10, 12):
        assert _gemm_status(f, "packed", 4, 4, 64, 64, 4, 4,
                            opts={"tile": tile}) == "FQT_ERR_UNSUPPORTED"
    g = fqt.Field(7, 2, (1, 0))                # q = 2^17, n_q <= 1820
    assert _gemm_status(g, "packed", 4, 4, 1821, 1821, 4, 4,
                        opts={"tile": 7}) == "FQT_ERR_UNSUPPORTED"


def test_buffered_tile_refuses_extents_beyond_32_bits():
    # tile 12 addresses A and B through 32-bit byte offsets: an operand that
    # spans 2^31 bytes or more is refused before any device work
    f = fqt.Field(7, 2, (1, 0))
    big_ld = 1 << 21                           # (1023 * 2^21 + 1024) * 2 bytes > 2^31
    assert _gemm_status(f, "packed", 1024, 4, 1024, big_ld, 4, 4, A=BOGUS, B=BOGUS + (1 << 33),
                        C=BOGUS + (1 << 34), opts={"tile": 12}) == "FQT_ERR_UNSUPPORTED"
    assert _gemm_status(f, "packed", 4, 1024, 1024, 1024, big_ld, 1024, A=BOGUS,
                        B=BOGUS + (1 << 33), C=BOGUS + (1 << 40),
                        opts={"tile": 12}) == "FQT_ERR_UNSUPPORTED"


def test_int8_tile_ids_and_lds_refusal():
    f = fqt.Field(7, 2, (1, 0))
    assert _gemm_status(f, "int8", 4, 4, 4, 4, 4, 4, opts={"tile": 12}) == "FQT_ERR_INVALID_ARG"
    # id 11 (strips of 16 outputs, B' built in LDS) runs k = 4 fields only
    assert _gemm_status(f, "int8", 4, 4, 4, 4, 4, 4, opts={"tile": 11}) == "FQT_ERR_UNSUPPORTED"
    # GF(13^3): a 12-bit table index, 4096 entries of 16 bytes; with the
    # 128 x 128 operand tiles of id 5 that exceeds one CU's LDS
    g = fqt.Field(13, 3, (1, 0, 4))
    assert _gemm_status(g, "int8", 4, 4, 4, 4, 4, 4, opts={"tile": 5}) == "FQT_ERR_UNSUPPORTED"


def test_split_tiles_validation():
    # d-split tiles: k = 3 or 4 only, q = 2^17 only, n_q <= (2^17 - 1) / (w (p-1)^2)
    # (w = 8 for k = 4: 4095 for p = 3), blocks of at least 16 products
    g = fqt.Field(7, 2, (1, 0))
    for tile in (13, 14):
        assert _gemm_status(g, "packed", 4, 4, 4, 4, 4, 4, opts={"tile": tile}) == "FQT_ERR_UNSUPPORTED"
    f = fqt.Field(3, 4, (2, 0, 0, 2))
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4,
                        opts={"tile": 13, "log2q": 16}) == "FQT_ERR_INVALID_ARG"
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4,
                        opts={"tile": 13, "n_q": 4096}) == "FQT_ERR_BOUNDS"
    assert _gemm_status(f, "packed", 4, 4, 64, 64, 4, 4,
                        opts={"tile": 14, "n_q": 8}) == "FQT_ERR_UNSUPPORTED"


def test_gemm_n_q_bound_cfg4():
    f = fqt.Field(5, 3, (3, 3, 0))
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4, opts={"log2q": 10, "n_q": 22}) == "FQT_ERR_BOUNDS"


def test_polymul_validation_errors():
    L = fqt.lib()
    v = ctypes.c_void_p(BOGUS)
    w = ctypes.c_void_p(BOGUS + (1 << 30))
    o = ctypes.c_void_p(BOGUS + (1 << 31))
    name = lambda st: fqt.STATUS_NAMES[st]
    # q = 48 = k (p-1)^2 breaks q > n_q k (p-1)^2 for p = 5, k = 3
    assert name(L.fqt_polymul_batch(5, 3, 48, v, w, 10, o, None)) == "FQT_ERR_BOUNDS"
    # q^(2k-1) >= 2^53
    assert name(L.fqt_polymul_batch(5, 3, 2 ** 11, v, w, 10, o, None)) == "FQT_ERR_BOUNDS"
    assert name(L.fqt_polymul_batch(6, 3, 64, v, w, 10, o, None)) == "FQT_ERR_NOT_PRIME"
    assert name(L.fqt_polymul_batch(5, 3, 64, v, w, 10, v, None)) == "FQT_ERR_INVALID_ARG"
    assert name(L.fqt_polymul_batch(5, 9, 64, v, w, 10, o, None)) == "FQT_ERR_UNSUPPORTED"


def test_unpack_pack_validation_errors():
    f = fqt.Field(5, 3, (3, 3, 0))
    L = fqt.lib()
    v = ctypes.c_void_p(BOGUS)
    o = ctypes.c_void_p(BOGUS + (1 << 30))
    name = lambda st: fqt.STATUS_NAMES[st]
    # (10^4)^5 > 2^53: the binary64 path refuses; the uint64 path needs q^(ndigits-1) < 2^64
    assert name(L.fqt_unpack_redq(f.handle, 10 ** 4, v, 4, 5, 0, o, None)) == "FQT_ERR_BOUNDS"
    assert name(L.fqt_unpack_redq_u64(f.handle, 10 ** 4, v, 4, 7, 0, o, None)) == "FQT_ERR_BOUNDS"
    assert name(L.fqt_unpack_redq(f.handle, 64, v, 4, 6, 1, o, None)) == "FQT_ERR_INVALID_ARG"
    assert name(L.fqt_unpack_redq(f.handle, 64, v, 4, 0, 0, o, None)) == "FQT_ERR_UNSUPPORTED"
    # ndigits in [1, 15]: 16 digits of q = 2 fit 2^53 but are refused
    assert name(L.fqt_unpack_redq(f.handle, 2, v, 4, 16, 0, o, None)) == "FQT_ERR_UNSUPPORTED"
    assert name(L.fqt_pack(f.handle, 2 ** 30, v, 4, o, None)) == "FQT_ERR_BOUNDS"
    # GF(5^2) at q = 2^36: packed values stay below 2^53, but q^k = 2^72 is refused
    f2 = fqt.Field(5, 2, (2, 0))
    assert name(L.fqt_pack(f2.handle, 2 ** 36, v, 4, o, None)) == "FQT_ERR_BOUNDS"
    assert name(L.fqt_pack(f.handle, 1, v, 4, o, None)) == "FQT_ERR_INVALID_ARG"


def test_autotune_argument_errors():
    f = fqt.Field(7, 2, (1, 0))
    L = fqt.lib()
    name = lambda st: fqt.STATUS_NAMES[st]
    assert name(L.fqt_autotune(f.handle, 0, 0, None, None, None, None, None)) == "FQT_ERR_INVALID_ARG"
    bad = (fqt.GemmDesc * 1)()
    bad[0] = fqt.GemmDesc(4, 4, 8, 4, 4, 4, BOGUS, BOGUS + (1 << 30), BOGUS + (1 << 31))  # lda < K
    assert name(L.fqt_autotune(f.handle, 0, 1, bad, None, None, None, None)) == "FQT_ERR_INVALID_ARG"


def test_tile_counts():
    assert fqt.tile_count("packed") == 15
    assert fqt.tile_count("int8") == 11


def test_autotune_rejects_plain_only():
    f = fqt.Field(7, 2, (1, 0))
    d = (fqt.GemmDesc * 1)()
    d[0] = fqt.GemmDesc(4, 4, 4, 4, 4, 4, BOGUS, BOGUS + (1 << 30), BOGUS + (1 << 31))
    assert fqt.STATUS_NAMES[fqt.lib().fqt_autotune(f.handle, 3, 1, d, None, None, None, None)] == "FQT_ERR_INVALID_ARG"



@pytest.mark.skipif(os.path.exists("/dev/kfd"),
                    reason="the fallback launches on BOGUS pointers once a GPU is present")
def test_tuned_options_refused_at_larger_k_fall_back_to_defaults(tmp_path):
    # GF(7^2): direct tile 12 holds no block state, so it is admissible at
    # K = 1500 (one K-block of n_q = 1820 at q = 2^17) but not at K = 2000,
    # which falls in the same power-of-two shape class (K bucket 2048).  A
    # tuned entry for the class must not make the AUTO call at K = 2000 fail:
    # the refusal (host side) falls back to the packed defaults, which pass
    # every host check and reach the device (FQT_ERR_DEVICE without a GPU).
    f = fqt.Field(7, 2, (1, 0))
    L = fqt.lib()
    cache = tmp_path / "tune.jsonl"
    for count in (1, 2):
        key = f"p7_k2_c{count}_1024_1024_2048"
        with open(cache, "a") as fp:
            fp.write('{"key": "%s", "path": 1, "log2q": 17, "n_q": 0, "tile": 12, '
                     '"boundary": 0, "centered": 0, "ms": 1.0}\n' % key)
        d = (fqt.GemmDesc * count)()
        for i in range(count):
            d[i] = fqt.GemmDesc(1024, 1024, 1500, 1500, 1024, 1024, BOGUS + i * (1 << 24),
                                BOGUS + (1 << 30) + i * (1 << 24),
                                BOGUS + (1 << 31) + i * (1 << 24))
        bp = ctypes.c_int(0)
        best = fqt.GemmOpts()
        st = L.fqt_autotune(f.handle, 0, count, d, str(cache).encode(), ctypes.byref(bp),
                            ctypes.byref(best), None)
        assert fqt.STATUS_NAMES[st] == "FQT_OK", fqt.last_error()   # from the cache alone
        assert best.tile == 12 and bp.value == 1
        # the tuned options themselves are refused at K = 2000
        assert _gemm_status(f, "packed", 1024, 1024, 2000, 2000, 1024, 1024,
                            opts={"log2q": 17, "tile": 12}) == "FQT_ERR_UNSUPPORTED"
        for i in range(count):
            d[i].K = 2000
            d[i].lda = 2000
        if count == 1:
            st = _gemm_status(f, "auto", 1024, 1024, 2000, 2000, 1024, 1024)
        else:
            st = fqt.STATUS_NAMES[L.fqt_gemm_gfpk_batched_ex(f.handle, 0, None, count, d, None)]
        assert st == "FQT_ERR_DEVICE", (count, st, fqt.last_error())


# ---- d-FQT long polynomials: every refusal happens before device work -------

def _dfqt_status(p, d, log2q, n_q, boundary, count, length, a=BOGUS, b=BOGUS + (1 << 30),
                 c=BOGUS + (1 << 31), centered=0):
    L = fqt.lib()
    return fqt.STATUS_NAMES[L.fqt_polymul_dfqt(p, d, log2q, n_q, boundary, centered,
                                               ctypes.c_void_p(a), ctypes.c_void_p(b), count,
                                               length, ctypes.c_void_p(c), None)]


def test_dfqt_centred_validation_errors():
    assert _dfqt_status(2, 1, 0, 0, 0, 1, 10, centered=1) == "FQT_ERR_UNSUPPORTED"
    assert _dfqt_status(3, 4, 0, 0, 0, 1, 10, centered=2) == "FQT_ERR_INVALID_ARG"
    # p = 3, d = 4, q = 2^5: centred blocks hold 3 chunk products, not 4
    assert _dfqt_status(3, 4, 0, 4, 0, 1, 10, centered=1) == "FQT_ERR_BOUNDS"
    assert _dfqt_status(3, 4, 0, 2, 0, 1, 10, centered=0) == "FQT_ERR_BOUNDS"


def test_dfqt_validation_errors():
    assert _dfqt_status(4, 1, 0, 0, 0, 1, 10) == "FQT_ERR_NOT_PRIME"
    assert _dfqt_status(131, 1, 0, 0, 0, 1, 10) == "FQT_ERR_UNSUPPORTED"       # p > 127
    assert _dfqt_status(3, 8, 0, 0, 0, 1, 10) == "FQT_ERR_UNSUPPORTED"         # d > 7
    assert _dfqt_status(3, 1, 0, 0, 0, -1, 10) == "FQT_ERR_INVALID_ARG"
    assert _dfqt_status(3, 1, 0, 0, 0, 1, 0) == "FQT_ERR_INVALID_ARG"
    assert _dfqt_status(3, 1, 0, 0, 0, 1, 10, a=0) == "FQT_ERR_INVALID_ARG"
    assert _dfqt_status(3, 0, 0, 0, 0, 1, 1025) == "FQT_ERR_UNSUPPORTED"       # > 1024 chunks
    assert _dfqt_status(3, 1, 0, 0, 3, 1, 10) == "FQT_ERR_INVALID_ARG"         # boundary 3
    # q^(2d+1) < 2^53: d = 4 allows q up to 2^5
    assert _dfqt_status(3, 4, 6, 0, 0, 1, 10) == "FQT_ERR_BOUNDS"
    # q > n_q (d+1)(p-1)^2: p = 3, d = 4, q = 32 allows n_q = 1 only
    assert _dfqt_status(3, 4, 0, 2, 0, 1, 10) == "FQT_ERR_BOUNDS"
    # p = 127, d = 4: q = 32 is below (d+1)(p-1)^2, no block fits
    assert _dfqt_status(127, 4, 0, 0, 0, 1, 10) == "FQT_ERR_BOUNDS"
    # several blocks need the largest q (d = 1: q = 2^17), and q = 2^16 with
    # n_q = 2 < 6 chunks would need them
    assert _dfqt_status(3, 1, 16, 2, 0, 1, 12) == "FQT_ERR_UNSUPPORTED"
    # digit sums need q <= 2^12: d = 1 has q = 2^17 when several blocks are forced
    assert _dfqt_status(3, 1, 0, 2, 2, 1, 12) == "FQT_ERR_UNSUPPORTED"
    # output overlapping an input
    assert _dfqt_status(3, 1, 0, 0, 0, 4, 10, c=BOGUS + 8) == "FQT_ERR_INVALID_ARG"


def test_delayed_validation_errors():
    L = fqt.lib()
    v, w, o = (ctypes.c_void_p(BOGUS), ctypes.c_void_p(BOGUS + (1 << 30)),
               ctypes.c_void_p(BOGUS + (1 << 31)))
    name = lambda st: fqt.STATUS_NAMES[st]
    assert name(L.fqt_polymul_delayed(9, v, w, 1, 10, o, None)) == "FQT_ERR_NOT_PRIME"
    assert name(L.fqt_polymul_delayed(3, v, w, 1, 8193, o, None)) == "FQT_ERR_UNSUPPORTED"
    assert name(L.fqt_polymul_delayed(3, v, w, 1, 0, o, None)) == "FQT_ERR_INVALID_ARG"
    assert name(L.fqt_polymul_delayed(3, v, w, 4, 10, v, None)) == "FQT_ERR_INVALID_ARG"


# ---- discrete-log representation -------------------------------------------

@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS + [(2, 2, (1, 1)), (13, 3, (1, 0, 4)),
                                                   (7, 4, (1, 0, 0, 1)), (11, 1, (9,))])
def test_log_generator_matches_oracle(p, k, P):
    # host-only query: the library's generator search against the oracle's
    f = fqt.Field(p, k, P)
    g, m = fqt.log_info(f)
    assert m == p ** k - 1
    assert g == gf.log_generator(p, P)


def test_log_validation_errors():
    f = fqt.Field(5, 3, (3, 3, 0))
    L = fqt.lib()
    v = ctypes.c_void_p(BOGUS)
    w = ctypes.c_void_p(BOGUS + (1 << 30))
    o = ctypes.c_void_p(BOGUS + (1 << 31))
    name = lambda st: fqt.STATUS_NAMES[st]
    assert name(L.fqt_to_log(f.handle, v, -1, o, None)) == "FQT_ERR_INVALID_ARG"
    assert name(L.fqt_to_log(f.handle, v, 10, None, None)) == "FQT_ERR_INVALID_ARG"
    assert name(L.fqt_to_log(f.handle, v, 10, ctypes.c_void_p(BOGUS + 4), None)) == "FQT_ERR_INVALID_ARG"
    assert name(L.fqt_from_log(f.handle, v, 10, ctypes.c_void_p(BOGUS + 8), None)) == "FQT_ERR_INVALID_ARG"
    # log_add: in place is allowed, a partial overlap is not
    assert name(L.fqt_log_add(f.handle, v, w, 10, ctypes.c_void_p(BOGUS + 2), None)) == "FQT_ERR_INVALID_ARG"
    assert name(L.fqt_log_add(f.handle, v, w, -3, o, None)) == "FQT_ERR_INVALID_ARG"

    def gemm_log(M, N, K, lda, ldb, ldc, A=BOGUS, B=BOGUS + (1 << 30), C=BOGUS + (1 << 31),
                 opts=None):
        return name(L.fqt_gemm_log(f.handle, fqt._opts(opts), M, N, K, ctypes.c_void_p(A), lda,
                                   ctypes.c_void_p(B), ldb, ctypes.c_void_p(C), ldc, None))
    assert gemm_log(4, 4, 8, 4, 4, 4) == "FQT_ERR_INVALID_ARG"             # lda < K
    assert gemm_log(-1, 4, 4, 4, 4, 4) == "FQT_ERR_INVALID_ARG"
    assert gemm_log(4, 4, 4, 4, 4, 4, C=BOGUS + 6) == "FQT_ERR_INVALID_ARG"  # C overlaps A (2-byte codes)
    assert gemm_log(4, 4, 4, 4, 4, 4, opts={"tile": 2}) == "FQT_ERR_UNSUPPORTED"
    assert gemm_log(4, 4, 4, 4, 4, 4, opts={"tile": 13}) == "FQT_ERR_UNSUPPORTED"
    assert gemm_log(4, 4, 4, 4, 4, 4, opts={"n_q": 100}) == "FQT_ERR_BOUNDS"
    # tiles 7 and 9 take one K-block (q = 2^10, n_q = 21 for GF(5^3))
    assert gemm_log(4, 4, 64, 64, 4, 4, opts={"tile": 7}) == "FQT_ERR_UNSUPPORTED"


def test_winograd_validation_errors():
    f = fqt.Field(7, 2, (1, 0))
    L = fqt.lib()
    name = lambda st: fqt.STATUS_NAMES[st]

    def wg(levels, M, N, K, lda, ldb, ldc, path=1, C=BOGUS + (1 << 31)):
        return name(L.fqt_gemm_winograd(f.handle, path, None, levels, M, N, K, ctypes.c_void_p(BOGUS),
                                        lda, ctypes.c_void_p(BOGUS + (1 << 30)), ldb,
                                        ctypes.c_void_p(C), ldc, None))
    assert wg(7, 4, 4, 4, 4, 4, 4) == "FQT_ERR_INVALID_ARG"        # levels above 6
    assert wg(1, 4, 4, 8, 4, 4, 4) == "FQT_ERR_INVALID_ARG"        # lda < K
    assert wg(1, 4, 4, 4, 4, 4, 4, path=9) == "FQT_ERR_INVALID_ARG"
    assert wg(1, 4, 4, 4, 4, 4, 4, C=BOGUS + 8) == "FQT_ERR_INVALID_ARG"  # C overlaps A


def test_centred_validation_errors():
    # centred packing: odd p only, staged tiles 1..6 only, n_q up to
    # (q/2 - 1) / (k ((p-1)/2)^2): 15 for GF(3^4) at q = 2^7
    g2 = fqt.Field(2, 3, (1, 0, 1))
    assert _gemm_status(g2, "packed", 4, 4, 4, 4, 4, 4, opts={"centered": 1}) == "FQT_ERR_UNSUPPORTED"
    f = fqt.Field(3, 4, (2, 0, 0, 2))
    for tile in (7, 11, 13):
        assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4,
                            opts={"centered": 1, "tile": tile}) == "FQT_ERR_UNSUPPORTED"
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4,
                        opts={"centered": 1, "n_q": 16}) == "FQT_ERR_BOUNDS"
    # without centring the same n_q breaks eq. (2)
    assert _gemm_status(f, "packed", 4, 4, 4, 4, 4, 4, opts={"n_q": 15}) == "FQT_ERR_BOUNDS"


# ---- d-FQT over uneven batches: every refusal happens before device work ----

def _dfqt_batch_status(p, d, pairs, log2q=0, n_q=0, boundary=0, centered=0):
    L = fqt.lib()
    arr = (fqt.PolyDesc * len(pairs))()
    for i, (la, lb, a, b, c) in enumerate(pairs):
        arr[i] = fqt.PolyDesc(la, lb, a, b, c)
    return fqt.STATUS_NAMES[L.fqt_polymul_dfqt_batched(p, d, log2q, n_q, boundary, centered,
                                                       len(pairs), arr, None)]


def test_dfqt_batched_validation_errors():
    ok_pair = (10, 20, BOGUS, BOGUS + (1 << 20), BOGUS + (1 << 30))
    assert _dfqt_batch_status(4, 1, [ok_pair]) == "FQT_ERR_NOT_PRIME"
    assert _dfqt_batch_status(131, 1, [ok_pair]) == "FQT_ERR_UNSUPPORTED"
    assert _dfqt_batch_status(3, 8, [ok_pair]) == "FQT_ERR_UNSUPPORTED"
    assert _dfqt_batch_status(2, 1, [ok_pair], centered=1) == "FQT_ERR_UNSUPPORTED"
    assert _dfqt_batch_status(3, 1, [ok_pair], centered=2) == "FQT_ERR_INVALID_ARG"
    assert _dfqt_batch_status(3, 1, [ok_pair], boundary=3) == "FQT_ERR_INVALID_ARG"
    # negative length; a null operand of a non-empty pair
    assert _dfqt_batch_status(3, 1, [(-1, 5, BOGUS, BOGUS, BOGUS)]) == "FQT_ERR_INVALID_ARG"
    assert _dfqt_batch_status(3, 1, [(3, 5, 0, BOGUS, BOGUS + (1 << 30))]) == "FQT_ERR_INVALID_ARG"
    # more chunks than one wave's LDS holds: 1024 (d + 1) coefficients at most
    assert _dfqt_batch_status(3, 1, [(2049, 5, BOGUS, BOGUS + (1 << 20),
                                      BOGUS + (1 << 30))]) == "FQT_ERR_UNSUPPORTED"
    # the output overlaps its own operand
    assert _dfqt_batch_status(3, 1, [(10, 10, BOGUS, BOGUS + (1 << 20),
                                      BOGUS + 5)]) == "FQT_ERR_INVALID_ARG"
    # eq. (2): p = 3, d = 4 at q = 2^5 holds one chunk product per block, not 2
    assert _dfqt_batch_status(3, 4, [ok_pair], n_q=2) == "FQT_ERR_BOUNDS"
    # empty pairs only: nothing to do, nothing refused
    assert _dfqt_batch_status(3, 1, [(0, 7, 0, 0, 0)]) == "FQT_OK"
    assert _dfqt_batch_status(3, 1, []) == "FQT_OK"


def test_dfqt_batched_noalloc_validation_errors():
    # the same host checks as the planned batch, and its own maximum of
    # 16384 pairs with output, all before any device work
    L = fqt.lib()

    def status(p, d, pairs, centered=0):
        arr = (fqt.PolyDesc * len(pairs))()
        for i, (la, lb, a, b, c) in enumerate(pairs):
            arr[i] = fqt.PolyDesc(la, lb, a, b, c)
        return fqt.STATUS_NAMES[L.fqt_polymul_dfqt_batched_noalloc(p, d, 0, 0, 0, centered,
                                                                  len(pairs), arr, None)]

    ok_pair = (10, 20, BOGUS, BOGUS + (1 << 20), BOGUS + (1 << 30))
    assert status(4, 1, [ok_pair]) == "FQT_ERR_NOT_PRIME"
    assert status(3, 8, [ok_pair]) == "FQT_ERR_UNSUPPORTED"
    assert status(2, 1, [ok_pair], centered=1) == "FQT_ERR_UNSUPPORTED"
    assert status(3, 1, [(-1, 5, BOGUS, BOGUS, BOGUS)]) == "FQT_ERR_INVALID_ARG"
    assert status(3, 1, [(2049, 5, BOGUS, BOGUS + (1 << 20), BOGUS + (1 << 30))]) == \
        "FQT_ERR_UNSUPPORTED"
    many = [(1, 1, BOGUS + 4 * i, BOGUS + (1 << 20) + 4 * i, BOGUS + (1 << 30) + 4 * i)
            for i in range(16385)]
    assert status(3, 4, many) == "FQT_ERR_UNSUPPORTED"
    assert "16384" in fqt.last_error()
    assert status(3, 4, [(0, 5, 0, 0, 0)]) == "FQT_OK"


def test_wave_tile_refuses_unaligned_c_and_far_c_rows():
    # tile 15 stores elements as words through a buffer bounded by C: C must
    # be 4-byte aligned and (M + 32) ldc k below 2^30 bytes
    f = fqt.Field(3, 4, (2, 0, 0, 2))
    opts = {"tile": 15}
    assert _gemm_status(f, "packed", 8, 8, 8, 8, 8, 8, C=BOGUS + (1 << 31) + 1,
                        opts=opts) == "FQT_ERR_UNSUPPORTED"
    assert "aligned" in fqt.last_error()
    big = 1 << 23                                  # (8 + 32) * 2^23 * 4 >= 2^30
    assert _gemm_status(f, "packed", 8, 8, 8, 8, 8, big, C=BOGUS + (1 << 33),
                        opts=opts) == "FQT_ERR_UNSUPPORTED"
    assert "2^30" in fqt.last_error()
