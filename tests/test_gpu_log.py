"""Parity of the discrete-log representation (Alg. 4) with the oracle,
through the C ABI: conversions between coefficient form and codes, the Zech
addition, and the GEMM on codes.  Bit-exact: codes are unique.

A code e < m = p^k - 1 stands for g^e (g the first element of full order in
base-p order), m for zero; codes above m read as zero.
"""
import sys

import numpy as np
import pytest

from oracle import gf
from paper_0710_0510_amd import fqt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELDS = [(7, 2, (1, 0)), (3, 4, (2, 0, 0, 2)), (5, 3, (3, 3, 0)), (3, 2, (1, 0)),
          (2, 1, (1,)), (13, 1, (11,)), (2, 4, (1, 0, 0, 1)), (13, 3, (1, 0, 4))]


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fqt.lib()
    yield
    torch.cuda.synchronize()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def antilog_table(p, k, P):
    _, expo, _ = gf.log_tables(p, P)
    return np.array([gf.elem_from_index(i, p, k) for i in expo] + [[0] * k], dtype=np.uint8)


@pytest.mark.parametrize("p,k,P", FIELDS)
def test_conversions_every_element(p, k, P):
    note(f"log conversions GF({p}^{k})")
    f = fqt.Field(p, k, P)
    m = p ** k - 1
    anti = antilog_table(p, k, P)
    codes = np.arange(m + 1, dtype=np.uint16)
    # from_log: every code, plus codes above m (read as zero)
    extra = np.array([m + 1, 65535, m + 7], dtype=np.uint16)
    got = host(fqt.from_log(f, dev(np.concatenate([codes, extra]))))
    assert np.array_equal(got[:m + 1], anti)
    assert not got[m + 1:].any()
    # to_log: every element in coefficient form
    elems = np.array(list(gf.all_elements(p, k)), dtype=np.uint8)
    want = np.array([gf.to_log(e, p, P) for e in elems.tolist()], dtype=np.uint16)
    assert np.array_equal(host(fqt.to_log(f, dev(elems))), want)


@pytest.mark.parametrize("p,k,P", FIELDS)
def test_log_add(p, k, P):
    note(f"log add GF({p}^{k})")
    f = fqt.Field(p, k, P)
    m = p ** k - 1
    Z = gf.zech_table(p, P)
    if m + 1 <= 130:
        a, b = np.meshgrid(np.arange(m + 1), np.arange(m + 1))
        a, b = a.ravel(), b.ravel()
    else:
        rng = np.random.default_rng(p * k)
        a, b = rng.integers(0, m + 1, 20000), rng.integers(0, m + 1, 20000)
    a, b = a.astype(np.uint16), b.astype(np.uint16)
    want = np.array([gf.log_add(int(x), int(y), Z) for x, y in zip(a, b)], dtype=np.uint16)
    da, db = dev(a), dev(b)
    assert np.array_equal(host(fqt.log_add(f, da, db)), want)
    # in place, and codes above m read as zero
    fqt.log_add(f, da, db, out=da)
    assert np.array_equal(host(da), want)
    big = np.full_like(a, 65535)
    assert np.array_equal(host(fqt.log_add(f, dev(big), db)), b)


# the GEMM needs n_q >= 4 (one MFMA k-group) at the largest power-of-two q;
# GF(13^3) has n_q = 2 there and is refused like in coefficient form
GEMM_FIELDS = [f for f in FIELDS if fqt.params(f[0], f[1], 1)[1] >= 4]


def test_gemm_log_refuses_fields_without_a_k_group():
    f = fqt.Field(13, 3, (1, 0, 4))
    with pytest.raises(fqt.FqtError) as ei:
        fqt.gemm_log(f, dev(np.zeros((4, 4), np.uint16)), dev(np.zeros((4, 4), np.uint16)))
    assert ei.value.name == "FQT_ERR_UNSUPPORTED"


def refused(status, fn):
    """The host refuses the call with `status` before any launch."""
    with pytest.raises(fqt.FqtError) as ei:
        fn()
    assert ei.value.name == status, str(ei.value)


def run(p, k, P, M, N, K, seed, opts=None, adversarial=False, lda_pad=0):
    f = fqt.Field(p, k, P)
    m = p ** k - 1
    rng = np.random.default_rng(seed)
    if adversarial:
        full = gf.to_log([p - 1] * k, p, P)
        A = np.full((M, K + lda_pad), full, dtype=np.uint16)
        B = np.full((K, N), full, dtype=np.uint16)
    else:
        A = rng.integers(0, m + 1, size=(M, K + lda_pad)).astype(np.uint16)
        B = rng.integers(0, m + 1, size=(K, N)).astype(np.uint16)
    dA = dev(A)[:, :K]
    C = host(fqt.gemm_log(f, dA, dev(B), opts=opts))
    return C, gf.gemm_log(A[:, :K], B, p, P)


SHAPES = [(1, 1, 1), (17, 33, 45), (64, 64, 64), (100, 70, 300), (33, 130, 16), (5, 7, 0),
          (130, 200, 301), (200, 72, 33), (129, 257, 17)]


@pytest.mark.parametrize("p,k,P", GEMM_FIELDS)
@pytest.mark.parametrize("tile", [0, 7, 9, 11])
def test_gemm_log_shapes(p, k, P, tile):
    _, nq = fqt.params(p, k, 1)
    nq4 = nq // 4 * 4
    f = fqt.Field(p, k, P)
    for (M, N, K) in SHAPES:
        note(f"gemm_log GF({p}^{k}) tile={tile} {M}x{N}x{K}")
        if tile in (7, 9) and K > nq4:
            with pytest.raises(fqt.FqtError) as ei:
                fqt.gemm_log(f, dev(np.zeros((M, K), np.uint16)), dev(np.zeros((K, N), np.uint16)),
                             opts={"tile": tile})
            assert ei.value.name == "FQT_ERR_UNSUPPORTED"
            continue
        C, want = run(p, k, P, M, N, K, seed=M + N + K, opts={"tile": tile} if tile else None)
        assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("p,k,P", FIELDS[:4])
@pytest.mark.parametrize("boundary", [1, 2])
def test_gemm_log_blocks(p, k, P, boundary):
    q, nq = fqt.params(p, k, 1)
    for (M, N, K, nqc) in [(40, 50, 97, 4), (64, 128, 256, 8), (33, 129, 1001, 0)]:
        note(f"gemm_log blocks GF({p}^{k}) boundary={boundary} n_q={nqc} {M}x{N}x{K}")
        case = lambda: run(p, k, P, M, N, K, seed=K,
                           opts={"tile": 11, "n_q": nqc, "boundary": boundary})
        block = (nqc or nq) // 4 * 4  # the direct tiles round n_q down to whole MFMA groups
        if nqc > nq:  # eq. (2) fails for this n_q at the largest q
            refused("FQT_ERR_BOUNDS", case)
        elif boundary == 2 and q > 2 ** 12 and K > block:  # digit-sum fields above 24 bits
            refused("FQT_ERR_UNSUPPORTED", case)
        else:
            C, want = case()
            assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("p,k,P", FIELDS[:4])
def test_gemm_log_adversarial(p, k, P):
    # every element has all coefficients p-1: K = n_q reaches eq. (2)'s bound
    _, nq = fqt.params(p, k, 1)
    nq4 = min(nq // 4 * 4, 2000)
    for (K, tile) in [(nq4, 7), (nq4, 9), (3 * nq4 + 5, 11)]:
        note(f"gemm_log adversarial GF({p}^{k}) tile={tile} K={K}")
        C, want = run(p, k, P, 48, 96, K, seed=0, adversarial=True, opts={"tile": tile})
        assert np.array_equal(C, want), (K, tile)


def test_gemm_log_strided_and_codes_above_zero():
    p, k, P = 5, 3, (3, 3, 0)
    m = p ** k - 1
    # odd lda: rows off 4-byte boundaries take the byte-gather loads
    note("gemm_log strided")
    C, want = run(p, k, P, 70, 75, 91, seed=4, lda_pad=3)
    assert np.array_equal(C, want)
    # codes above m read as zero
    note("gemm_log codes above m")
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(5)
    A = rng.integers(0, 65536, size=(64, 40)).astype(np.uint16)
    B = rng.integers(0, m + 1, size=(40, 64)).astype(np.uint16)
    Ac = np.where(A > m, m, A).astype(np.uint16)
    C = host(fqt.gemm_log(f, dev(A), dev(B)))
    assert np.array_equal(C, gf.gemm_log(Ac, B, p, P))


def test_gemm_log_agrees_with_coefficient_path_1024():
    # the headline shape: log form against the coefficient form of the same
    # product (both complete, every entry), and sampled entries against Alg. 4
    p, k, P = 7, 2, (1, 0)
    f = fqt.Field(p, k, P)
    m = p ** k - 1
    rng = np.random.default_rng(2)
    Ac = rng.integers(0, p, size=(1024, 1024, k), dtype=np.uint8)
    Bc = rng.integers(0, p, size=(1024, 1024, k), dtype=np.uint8)
    dAc, dBc = dev(Ac), dev(Bc)
    note("gemm_log 1024^3 GF(7^2)")
    Al, Bl = fqt.to_log(f, dAc), fqt.to_log(f, dBc)
    Cl = fqt.gemm_log(f, Al, Bl)
    Cc = fqt.gemm(f, dAc, dBc, path="packed")
    assert torch.equal(fqt.to_log(f, Cc), Cl)
    Alh, Blh, Clh = host(Al), host(Bl), host(Cl)
    q, nq = gf.max_pow2_q(p, k)
    for i, j in rng.integers(0, 1024, size=(6, 2)).tolist():
        want = gf.gemm_log_alg4(Alh[i:i + 1].tolist(), Blh[:, j:j + 1].tolist(), p, P, q, nq)
        assert Clh[i, j] == want[0][0]
