"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every comparison is bit-exact: the method is exact integer arithmetic and
the canonical representative of a result is unique.
"""
import itertools
import sys

import numpy as np
import pytest

from oracle import gf
from paper_0710_0510_amd import fqt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CONFIG_FIELDS = [(7, 2, (1, 0)), (3, 4, (2, 0, 0, 2)), (5, 3, (3, 3, 0)), (3, 2, (1, 0))]


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


def refused(status, fn):
    """The host refuses the call with `status` before any launch."""
    with pytest.raises(fqt.FqtError) as ei:
        fn()
    assert ei.value.name == status, str(ei.value)


# ---- Alg. 1: batched polynomial products -------------------------------------

def test_polymul_cfg1_exhaustive():
    p, k, q = 5, 3, 64
    note("polymul exhaustive GF(5) k=3 q=64")
    elems = np.array([e for e in gf.all_elements(p, k)], dtype=np.uint8)
    a = np.repeat(elems, len(elems), axis=0)
    b = np.tile(elems, (len(elems), 1))
    out = host(fqt.polymul_batch(p, k, q, dev(a), dev(b)))
    assert np.array_equal(out, gf.polymul_batch(a, b, p))


@pytest.mark.parametrize("name", ["polymul-gf5-k3", "polymul-gf5-k3-2^24"])
def test_polymul_cfg1_workload(name):
    from paper_0710_0510_amd import workloads as W
    w = W.WORKLOADS[name]
    a, b = W.polymul_inputs(w)
    note(f"polymul workload {name}")
    out = host(fqt.polymul_batch(w.p, w.k, w.q, dev(a), dev(b)))
    assert np.array_equal(out, gf.polymul_batch(a, b, w.p))


def test_polymul_example1_general_q():
    note("polymul example 1 q=100")
    a = np.array([[1, 1]], dtype=np.uint8)
    b = np.array([[2, 1]], dtype=np.uint8)
    out = host(fqt.polymul_batch(3, 2, 100, dev(a), dev(b)))
    assert out.tolist() == [[2, 0, 1]]


@pytest.mark.parametrize("p,k,q,n", [(3, 2, 100, 1000), (7, 2, 2 ** 17, 257), (5, 3, 1552, 255),
                                     (3, 4, 190, 999), (2, 7, 8, 4097), (11, 1, 2 ** 40, 33),
                                     (13, 3, 1000, 700), (127, 2, 2 ** 15, 300),
                                     (127, 2, 32259, 300), (2, 5, 8, 3000), (3, 6, 25, 2100)])
def test_polymul_params(p, k, q, n):
    note(f"polymul p={p} k={k} q={q} n={n}")
    assert gf.eq2_holds(p, k, q, 1)
    rng = np.random.default_rng(p * 1000 + k)
    a = rng.integers(0, p, size=(n, k), dtype=np.uint8)
    b = rng.integers(0, p, size=(n, k), dtype=np.uint8)
    a[0] = p - 1
    b[0] = p - 1
    out = host(fqt.polymul_batch(p, k, q, dev(a), dev(b)))
    assert np.array_equal(out, gf.polymul_batch(a, b, p))


@pytest.mark.parametrize("p,k,q,n", [(5, 3, 64, 1), (5, 3, 64, 2), (5, 3, 64, 3), (5, 3, 64, 4),
                                     (5, 3, 64, 1029), (5, 3, 64, 4 * 256 * 3 + 2),
                                     (2, 5, 8, 3001), (3, 3, 16, 1002), (5, 2, 64, 777),
                                     (13, 2, 512, 3), (127, 1, 2 ** 14, 4099), (2, 1, 2, 5),
                                     (2, 4, 8, 2048), (7, 2, 2 ** 10, 4097), (3, 2, 2 ** 8, 999),
                                     (3, 1, 2 ** 32, 10)])
def test_polymul_32bit_words(p, k, q, n):
    # q = 2^b with (2k - 1) b <= 32 and word-aligned buffers: every pair's
    # product and digits stay below 2^32 (four pairs per thread, the last
    # thread of a ragged batch byte by byte); all-maximal rows put the
    # largest r of the batch through the floor division by p
    b = q.bit_length() - 1
    assert q == 1 << b and (2 * k - 1) * b <= 32 and gf.eq2_holds(p, k, q, 1)
    note(f"polymul 32-bit words p={p} k={k} q={q} n={n}")
    rng = np.random.default_rng(p * 31 + k * 7 + n)
    a = rng.integers(0, p, size=(n, k), dtype=np.uint8)
    b_ = rng.integers(0, p, size=(n, k), dtype=np.uint8)
    a[-1] = p - 1
    b_[-1] = p - 1
    a[0] = p - 1
    b_[0] = p - 1
    out = host(fqt.polymul_batch(p, k, q, dev(a), dev(b_)))
    assert np.array_equal(out, gf.polymul_batch(a, b_, p))


@pytest.mark.parametrize("p,k,q,n", [(3, 3, 256, 2049), (3, 4, 64, 1024), (2, 8, 9, 1025),
                                     (5, 1, 2 ** 20, 5000), (2, 4, 8, 1031), (5, 3, 64, 1030)])
def test_polymul_unaligned_views(p, k, q, n):
    # operands and output start one row into their buffers (k and 2k - 1
    # bytes: not 16-byte aligned), and the batch ends inside a workgroup
    assert gf.eq2_holds(p, k, q, 1)
    note(f"polymul unaligned views k={k} n={n}")
    rng = np.random.default_rng(k * 7 + n)
    a = rng.integers(0, p, size=(n + 1, k), dtype=np.uint8)
    b = rng.integers(0, p, size=(n + 1, k), dtype=np.uint8)
    cbig = torch.full((n + 1, 2 * k - 1), 255, dtype=torch.uint8, device="cuda")
    fqt.polymul_batch(p, k, q, dev(a)[1:], dev(b)[1:], out=cbig[1:])
    got = host(cbig)
    assert np.array_equal(got[1:], gf.polymul_batch(a[1:], b[1:], p))
    assert (got[0] == 255).all()  # nothing written before the output view


def test_polymul_empty():
    out = fqt.polymul_batch(5, 3, 64, torch.empty((0, 3), dtype=torch.uint8, device="cuda"),
                            torch.empty((0, 3), dtype=torch.uint8, device="cuda"))
    assert out.shape == (0, 5)


# ---- DQT pack / REDQ unpack ---------------------------------------------------

@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
@pytest.mark.parametrize("qkind", ["pow2", "general"])
def test_pack(p, k, P, qkind):
    q = fqt.params(p, k, 1, pow2=(qkind == "pow2"))[0]
    note(f"pack GF({p}^{k}) q={q}")
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(5)
    n = 3001
    c = rng.integers(0, p, size=(n, k), dtype=np.uint8)
    out = host(fqt.pack(f, q, dev(c)))
    want = np.array([float(gf.dqt(row.tolist(), q)) for row in c])
    assert np.array_equal(out, want)


@pytest.mark.parametrize("p,k", [(2, 1), (127, 1), (7, 2), (5, 3), (3, 4), (13, 2)])
def test_pack_word_kernel_largest_q(p, k):
    # q = 2^b, the largest b the host admits (packed values exact in
    # binary64, q^k at most 2^70); 1027 elements end inside a thread's group
    # of four; then the same bytes one element into their buffer (not
    # word-aligned unless k = 4) packed into an output view one value into
    # its buffer
    b = max(bb for bb in range(1, 64)
            if (p - 1) * sum(2 ** (bb * j) for j in range(k)) <= 2 ** 53 and bb * k <= 70)
    q = 1 << b
    note(f"pack word kernel GF({p}^{k}) q=2^{b}")
    f = fqt.Field(p, k, _first_irreducible(p, k))
    rng = np.random.default_rng(p + k)
    n = 1027
    c = rng.integers(0, p, size=(n + 1, k), dtype=np.uint8)
    c[1] = p - 1
    c[-1] = p - 1
    want = np.array([float(gf.dqt(row.tolist(), q)) for row in c])
    out = host(fqt.pack(f, q, dev(c)))
    assert np.array_equal(out, want)
    big = torch.full((n + 1,), -1.0, dtype=torch.float64, device="cuda")
    fqt.pack(f, q, dev(c)[1:], out=big[1:])
    got = host(big)
    assert np.array_equal(got[1:], want[1:]) and got[0] == -1.0


def _random_packed(rng, n, nd, q):
    digits = rng.integers(0, q, size=(n, nd), dtype=np.int64)
    digits[0] = q - 1
    vals = [gf.dqt(row.tolist(), q) for row in digits]
    return digits, vals


@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
@pytest.mark.parametrize("qkind", ["pow2", "general"])
def test_unpack_poly_and_field(p, k, P, qkind):
    q = fqt.params(p, k, 1, pow2=(qkind == "pow2"))[0]
    nd = 2 * k - 1
    note(f"unpack GF({p}^{k}) q={q} nd={nd}")
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(7)
    digits, vals = _random_packed(rng, 2500, nd, q)
    assert max(vals) < 2 ** 53
    packed = dev(np.array(vals, dtype=np.float64))
    poly = host(fqt.unpack_redq(f, q, packed, nd, fqt.UNPACK_POLY))
    want_poly = np.array([gf.dqt_inverse(v, q, nd, p) for v in vals], dtype=np.uint8)
    assert np.array_equal(poly, want_poly)
    field = host(fqt.unpack_redq(f, q, packed, nd, fqt.UNPACK_FIELD))
    want_field = np.array([gf.poly_rem(row.tolist(), P, p) for row in want_poly], dtype=np.uint8)
    assert np.array_equal(field, want_field)
    # an output view one row into its buffer (not 16-byte aligned)
    big = torch.full((2501, nd), 255, dtype=torch.uint8, device="cuda")
    fqt.unpack_redq(f, q, packed, nd, fqt.UNPACK_POLY, out=big[1:])
    got = host(big)
    assert np.array_equal(got[1:], want_poly) and (got[0] == 255).all()
    # the uint64 variant agrees on the same values
    packed64 = dev(np.array(vals, dtype=np.int64))
    assert np.array_equal(host(fqt.unpack_redq(f, q, packed64, nd, fqt.UNPACK_POLY)), want_poly)
    assert np.array_equal(host(fqt.unpack_redq(f, q, packed64, nd, fqt.UNPACK_FIELD)), want_field)


def _first_irreducible(p, k):
    for idx in range(p ** k):
        P = [(idx // p ** j) % p for j in range(k)]
        if P[0] != 0 and gf.is_irreducible(P, p):
            return tuple(P)
    raise AssertionError("no irreducible polynomial")


def _edge_values(rng, n, top, p):
    # uniform values below top, then the largest ones, zero and multiples of p
    vals = [int(v) for v in rng.integers(0, top, size=n, dtype=np.int64)]
    edges = [top - 1, top - 2, 0, 1, p, top - 1 - (top - 1) % p]
    vals[:len(edges)] = edges
    vals[-1] = top - 1
    return vals


@pytest.mark.parametrize("nd", list(range(1, 16)))
def test_unpack_poly_word_kernel_every_ndigits(nd):
    # q = 2^b with q^nd <= 2^53: the word-direct kernel (four values per
    # thread, NR = nd digits fixed at compile time); 1001 values end inside
    # a thread's group of four
    p, k, P = 5, 3, (3, 3, 0)
    b = min(53 // nd, 40)
    q = 1 << b
    note(f"unpack POLY word kernel nd={nd} q=2^{b}")
    f = fqt.Field(p, k, P)
    vals = _edge_values(np.random.default_rng(nd), 1001, q ** nd, p)
    out = host(fqt.unpack_redq(f, q, dev(np.array(vals, dtype=np.float64)), nd, fqt.UNPACK_POLY))
    want = np.array([gf.dqt_inverse(v, q, nd, p) for v in vals], dtype=np.uint8)
    assert np.array_equal(out, want)


@pytest.mark.parametrize("p,k", [(2, 1), (127, 1), (3, 2), (7, 2), (13, 2), (2, 3), (5, 3),
                                 (2, 4), (3, 4)])
def test_unpack_field_word_kernel_every_k(p, k):
    P = _first_irreducible(p, k)
    nr = 2 * k - 1
    b = 53 // nr
    q = 1 << b
    note(f"unpack FIELD word kernel GF({p}^{k}) q=2^{b}")
    f = fqt.Field(p, k, P)
    vals = _edge_values(np.random.default_rng(p * 10 + k), 1003, q ** nr, p)
    out = host(fqt.unpack_redq(f, q, dev(np.array(vals, dtype=np.float64)), nr, fqt.UNPACK_FIELD))
    want = np.array([gf.poly_rem(gf.dqt_inverse(v, q, nr, p), P, p) for v in vals],
                    dtype=np.uint8)
    assert np.array_equal(out, want)


def test_unpack_field_fewer_digits_than_residues():
    # FIELD mode with ndigits < 2k - 1 at a q whose (2k-1)-th power is far
    # above 2^64: the residues past the value are zero
    p, k, P = 5, 3, (3, 3, 0)
    q, nd = 2 ** 17, 3
    note("unpack FIELD ndigits 3 of 5 at q=2^17")
    f = fqt.Field(p, k, P)
    vals = _edge_values(np.random.default_rng(17), 999, q ** nd, p)
    out = host(fqt.unpack_redq(f, q, dev(np.array(vals, dtype=np.float64)), nd, fqt.UNPACK_FIELD))
    want = np.array([gf.poly_rem(gf.dqt_inverse(v, q, 2 * k - 1, p), P, p) for v in vals],
                    dtype=np.uint8)
    assert np.array_equal(out, want)


def test_unpack_example2_uint64():
    note("unpack example 2 (uint64, q=10^4)")
    from golden_io import load
    g = load("ex2_redq_p_divides_q.txt")
    f = fqt.Field(5, 3, (3, 3, 0))
    packed = dev(np.array([g["product"]], dtype=np.int64))
    out = host(fqt.unpack_redq(f, g["q"], packed, 5, fqt.UNPACK_POLY))
    assert out.tolist() == [g["result"]]


def test_unpack_near_2_53():
    # q^nd = 2^53 exactly: the largest binary64 values
    p, k, P = 3, 2, (1, 0)
    f = fqt.Field(p, k, P)
    q, nd = 2 ** 53, 1
    note("unpack near 2^53")
    vals = [2 ** 53 - 1, 2 ** 53 - 2, 2 ** 52, 2 ** 52 + 1, 0, 1, 2]
    out = host(fqt.unpack_redq(f, q, dev(np.array(vals, dtype=np.float64)), nd, fqt.UNPACK_POLY))
    assert out[:, 0].tolist() == [v % p for v in vals]


# ---- GEMM over GF(p^k) ----------------------------------------------------------

def _gemm_case(p, k, P, M, N, K, seed, path="packed", opts=None, adversarial=False):
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(seed)
    if adversarial:
        A = np.full((M, K, k), p - 1, dtype=np.uint8)
        B = np.full((K, N, k), p - 1, dtype=np.uint8)
    else:
        A = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        B = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
    C = host(fqt.gemm(f, dev(A), dev(B), path=path, opts=opts))
    want = gf.gemm_gfpk_planes(A, B, p, P)
    return C, want


SHAPES = [(1, 1, 1), (17, 33, 45), (64, 64, 64), (100, 70, 300), (33, 130, 16), (5, 7, 0)]


@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6])
def test_gemm_packed_shapes(p, k, P, tile):
    for (M, N, K) in SHAPES:
        note(f"gemm packed GF({p}^{k}) tile={tile} {M}x{N}x{K}")
        C, want = _gemm_case(p, k, P, M, N, K, seed=M + N + K, opts={"tile": tile})
        assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
@pytest.mark.parametrize("nq", [4, 8, 12, 20])
@pytest.mark.parametrize("boundary", [1, 2])
def test_gemm_packed_multiblock(p, k, P, nq, boundary):
    q, nqmax = fqt.params(p, k, 1)
    for (M, N, K) in [(40, 50, 97), (64, 64, 256)]:
        note(f"gemm packed multiblock GF({p}^{k}) n_q={nq} boundary={boundary} {M}x{N}x{K}")
        case = lambda: _gemm_case(p, k, P, M, N, K, seed=nq,
                                  opts={"n_q": nq, "tile": 2, "boundary": boundary})
        if nq > nqmax:  # eq. (2) fails for this n_q at the largest q
            refused("FQT_ERR_BOUNDS", case)
        elif boundary == 2 and q > 2 ** 12:  # digit-sum fields of 2b bits exceed 24
            refused("FQT_ERR_UNSUPPORTED", case)
        else:
            C, want = case()
            assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("tile", [1, 4])
def test_gemm_packed_lane_folding_residues(tile):
    # 10000 K-blocks of 4 products: the 16-bit residue lanes must be folded
    p, k, P = 7, 2, (1, 0)
    for adversarial in (True, False):
        note(f"gemm packed folding residues tile={tile} adversarial={adversarial}")
        C, want = _gemm_case(p, k, P, 33, 40, 40000, seed=7, adversarial=adversarial,
                             opts={"n_q": 4, "tile": tile, "boundary": 1})
        assert np.array_equal(C, want)


@pytest.mark.parametrize("tile", [1, 2])
def test_gemm_packed_field_folding_digits(tile):
    # GF(3^4), q = 2^7, blocks of 7: 14-bit digit fields hold 146 blocks of
    # digit sums (7*16 each); K = 3000 is 429 blocks, so the fields are folded
    p, k, P = 3, 4, (2, 0, 0, 2)
    for adversarial in (True, False):
        note(f"gemm packed folding digits tile={tile} adversarial={adversarial}")
        C, want = _gemm_case(p, k, P, 33, 40, 3000, seed=8, adversarial=adversarial,
                             opts={"tile": tile, "boundary": 2})
        assert np.array_equal(C, want)


@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
@pytest.mark.parametrize("boundary", [1, 2])
def test_gemm_adversarial_bound(p, k, P, boundary):
    q, nqmax = fqt.params(p, k, 1)
    nq4 = nqmax - nqmax % 4
    for K in [nq4, 3 * nq4 + 5]:
        K = min(K, 3000)
        note(f"gemm adversarial GF({p}^{k}) K={K} n_q={nq4} boundary={boundary}")
        if boundary == 2 and K > nq4 and 2 * (q.bit_length() - 1) > 24:
            # digit sums of q = 2^b need fields of 2b <= 24 bits: refused on the host
            with pytest.raises(fqt.FqtError) as ei:
                _gemm_case(p, k, P, 32, 48, K, seed=0, adversarial=True,
                           opts={"tile": 2, "boundary": boundary})
            assert ei.value.name == "FQT_ERR_UNSUPPORTED"
            continue
        C, want = _gemm_case(p, k, P, 32, 48, K, seed=0, adversarial=True,
                             opts={"tile": 2, "boundary": boundary})
        assert np.array_equal(C, want)


@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
def test_gemm_plain(p, k, P):
    for (M, N, K) in [(17, 33, 45), (64, 80, 130)]:
        note(f"gemm plain GF({p}^{k}) {M}x{N}x{K}")
        C, want = _gemm_case(p, k, P, M, N, K, seed=3, path="plain")
        assert np.array_equal(C, want)


def test_gemm_strided_and_unaligned():
    p, k, P = 7, 2, (1, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(9)
    Abig = rng.integers(0, p, size=(70, 91, k), dtype=np.uint8)   # odd ld: unaligned rows
    Bbig = rng.integers(0, p, size=(91, 75, k), dtype=np.uint8)
    A = dev(Abig)[:50, :61]
    B = dev(Bbig)[:61, :40]
    note("gemm strided/unaligned")
    C = host(fqt.gemm(f, A, B, path="packed"))
    want = gf.gemm_gfpk_planes(Abig[:50, :61], Bbig[:61, :40], p, P)
    assert np.array_equal(C, want)


def test_gemm_cross_path_identity_medium():
    p, k, P = 5, 3, (3, 3, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(12)
    A = dev(rng.integers(0, p, size=(300, 700, k), dtype=np.uint8))
    B = dev(rng.integers(0, p, size=(700, 260, k), dtype=np.uint8))
    note("gemm cross-path 300x260x700")
    outs = [host(fqt.gemm(f, A, B, path="plain"))]
    for tile in (1, 2, 3, 4, 5, 6):
        outs.append(host(fqt.gemm(f, A, B, path="packed", opts={"tile": tile})))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    want = gf.gemm_gfpk_planes(host(A), host(B), p, P)
    assert np.array_equal(outs[0], want)


# ---- batched --------------------------------------------------------------------

def test_gemm_batched_replay():
    p, k, P = 3, 4, (2, 0, 0, 2)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(31)
    shapes = rng.integers(1, 90, size=(40, 3))
    shapes[0] = (200, 150, 256)
    As, Bs, Cs, hostA, hostB = [], [], [], [], []
    for (M, N, K) in shapes.tolist():
        a = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        b = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
        hostA.append(a)
        hostB.append(b)
        As.append(dev(a))
        Bs.append(dev(b))
        Cs.append(torch.zeros((M, N, k), dtype=torch.uint8, device="cuda"))
    descs = fqt.make_descs(f, As, Bs, Cs)
    wants = [gf.gemm_gfpk_planes(a, b, p, P) for a, b in zip(hostA, hostB)]
    for rep in range(3):
        note(f"batched replay {rep}")
        for c in Cs:
            c.zero_()
        fqt.gemm_batched(f, descs, path="packed")
        torch.cuda.synchronize()
        for c, w in zip(Cs, wants):
            assert np.array_equal(host(c), w)
    for tile in range(1, 11):
        for rep in range(2):
            note(f"batched int8 tile {tile} replay {rep}")
            for c in Cs:
                c.zero_()
            fqt.gemm_batched(f, descs, path="int8", opts={"tile": tile})
            torch.cuda.synchronize()
            for c, w in zip(Cs, wants):
                assert np.array_equal(host(c), w)
    note("batched plain")
    for c in Cs:
        c.zero_()
    fqt.gemm_batched(f, descs, path="plain")
    for c, w in zip(Cs, wants):
        assert np.array_equal(host(c), w)


# ---- INT8 coefficient-wise path -------------------------------------------------

@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
@pytest.mark.parametrize("tile", list(range(1, 11)))
def test_gemm_int8_shapes(p, k, P, tile):
    for (M, N, K) in SHAPES + [(130, 200, 257)]:
        note(f"gemm int8 GF({p}^{k}) tile={tile} {M}x{N}x{K}")
        C, want = _gemm_case(p, k, P, M, N, K, seed=M + 2 * N + K, path="int8",
                             opts={"tile": tile})
        assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("tile", list(range(1, 11)))
def test_gemm_int8_prime_field(tile):
    # k = 1: GF(13), B' is B itself (1 x 1 multiplication matrices)
    p, k, P = 13, 1, (11,)
    for (M, N, K) in [(17, 33, 45), (100, 70, 300), (129, 257, 130)]:
        note(f"gemm int8 GF(13) tile={tile} {M}x{N}x{K}")
        C, want = _gemm_case(p, k, P, M, N, K, seed=M + K, path="int8", opts={"tile": tile})
        assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
@pytest.mark.parametrize("tile", [None, 4, 7, 9])
def test_gemm_int8_adversarial(p, k, P, tile):
    note(f"gemm int8 adversarial GF({p}^{k}) tile={tile}")
    C, want = _gemm_case(p, k, P, 40, 50, 3001, seed=0, adversarial=True, path="int8",
                         opts={"tile": tile} if tile else None)
    assert np.array_equal(C, want)


@pytest.mark.parametrize("tile", [None, 4, 8, 10])
def test_gemm_int8_delayed_reduction_gf61_2(tile):
    # K k (p-1)^2 far above 2^31: the INT32 accumulators are reduced mod p
    # every few thousand K-tiles (eq. (3) with n_d (p-1)^2 < 2^31).
    p, P = 61, (59, 0)   # X^2 - 2, irreducible since 2 is a non-residue mod 61
    assert gf.is_irreducible(P, p)
    note(f"gemm int8 delayed reduction GF(61^2) K=300000 tile={tile}")
    for adversarial in (True, False):
        C, want = _gemm_case(p, 2, P, 16, 24, 300000, seed=5, adversarial=adversarial,
                             path="int8", opts={"tile": tile} if tile else None)
        assert np.array_equal(C, want)


@pytest.mark.parametrize("tile", [None, 4, 5, 6, 7, 8, 9, 10])
def test_gemm_int8_strided_unaligned(tile):
    p, k, P = 5, 3, (3, 3, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(19)
    Abig = rng.integers(0, p, size=(70, 93, k), dtype=np.uint8)
    Bbig = rng.integers(0, p, size=(93, 75, k), dtype=np.uint8)
    note(f"gemm int8 strided/unaligned tile={tile}")
    C = host(fqt.gemm(f, dev(Abig)[:50, :61], dev(Bbig)[:61, :40], path="int8",
                      opts={"tile": tile} if tile else None))
    assert np.array_equal(C, gf.gemm_gfpk_planes(Abig[:50, :61], Bbig[:61, :40], p, P))


def test_gemm_int8_fused_table_too_large():
    # GF(13^3): 12-bit table index, 4096 entries of 16 bytes beside the
    # 128 x 128 operand tiles of id 5 exceed the LDS; id 4 fits
    p, k, P = 13, 3, (1, 0, 4)
    assert gf.is_irreducible(P, p)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(23)
    A = rng.integers(0, p, size=(70, 90, k), dtype=np.uint8)
    B = rng.integers(0, p, size=(90, 50, k), dtype=np.uint8)
    with pytest.raises(fqt.FqtError):
        fqt.gemm(f, dev(A), dev(B), path="int8", opts={"tile": 5})
    C = host(fqt.gemm(f, dev(A), dev(B), path="int8", opts={"tile": 4}))
    assert np.array_equal(C, gf.gemm_gfpk_planes(A, B, p, P))


@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
def test_gemm_three_paths_identical(p, k, P):
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(44)
    A = dev(rng.integers(0, p, size=(257, 513, k), dtype=np.uint8))
    B = dev(rng.integers(0, p, size=(513, 300, k), dtype=np.uint8))
    note(f"three paths GF({p}^{k}) 257x300x513")
    outs = [host(fqt.gemm(f, A, B, path=path)) for path in ("plain", "packed", "int8")]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    assert np.array_equal(outs[0], gf.gemm_gfpk_planes(host(A), host(B), p, P))


# ---- autotuner ------------------------------------------------------------------

def test_autotune_single_and_cache(tmp_path):
    p, k, P = 5, 3, (3, 3, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(61)
    Ah = rng.integers(0, p, size=(200, 300, k), dtype=np.uint8)
    Bh = rng.integers(0, p, size=(300, 150, k), dtype=np.uint8)
    A, B = dev(Ah), dev(Bh)
    C = torch.zeros((200, 150, k), dtype=torch.uint8, device="cuda")
    descs = fqt.make_descs(f, [A], [B], [C])
    cache = str(tmp_path / "tune.jsonl")
    note("autotune single GEMM")
    path, opts = fqt.autotune(f, descs, cache)
    assert path in ("packed", "int8") and opts["tile"] >= 1
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"key"' in lines[0]
    # second tuning reads the cache, writes nothing new
    f2 = fqt.Field(p, k, P)
    assert fqt.autotune(f2, fqt.make_descs(f2, [A], [B], [C]), cache) == (path, opts)
    assert len(open(cache).read().strip().splitlines()) == 1
    want = gf.gemm_gfpk_planes(Ah, Bh, p, P)
    for field in (f, f2):
        out = host(fqt.gemm(field, A, B, path="auto"))
        assert np.array_equal(out, want)


def test_autotune_batched():
    p, k, P = 3, 4, (2, 0, 0, 2)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(62)
    shapes = rng.integers(16, 120, size=(24, 3))
    As, Bs, Cs, wants = [], [], [], []
    for (M, N, K) in shapes.tolist():
        a = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        b = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
        As.append(dev(a)); Bs.append(dev(b))
        Cs.append(torch.zeros((M, N, k), dtype=torch.uint8, device="cuda"))
        wants.append(gf.gemm_gfpk_planes(a, b, p, P))
    descs = fqt.make_descs(f, As, Bs, Cs)
    note("autotune batched")
    path, opts = fqt.autotune(f, descs)
    assert path in ("packed", "int8") and opts["tile"] >= 1
    assert fqt.autotune(f, descs, only="packed")[0] == "packed"
    assert fqt.autotune(f, descs, only="int8")[0] == "int8"
    for c in Cs:
        c.zero_()
    fqt.gemm_batched(f, descs, path="auto")
    for c, w in zip(Cs, wants):
        assert np.array_equal(host(c), w)


@pytest.mark.parametrize("p,k,P", CONFIG_FIELDS)
@pytest.mark.parametrize("nq", [5, 6, 7, 13, 15])
@pytest.mark.parametrize("boundary", [1, 2])
def test_gemm_packed_padded_blocks(p, k, P, nq, boundary):
    # n_q not a multiple of 4: blocks of n_q products padded to 8 or 16 MFMA slots
    q, nqmax = fqt.params(p, k, 1)
    for tile in (1, 3):
        for (M, N, K) in [(40, 50, 97), (64, 64, 256), (17, 9, 7 * nq + 3)]:
            note(f"gemm padded GF({p}^{k}) n_q={nq} boundary={boundary} tile={tile} {M}x{N}x{K}")
            case = lambda: _gemm_case(p, k, P, M, N, K, seed=nq + K,
                                      opts={"n_q": nq, "tile": tile, "boundary": boundary})
            if nq > nqmax:
                refused("FQT_ERR_BOUNDS", case)
            elif boundary == 2 and q > 2 ** 12:  # every K here exceeds n_q: several blocks
                refused("FQT_ERR_UNSUPPORTED", case)
            else:
                C, want = case()
                assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("boundary", [1, 2])
def test_gemm_padded_adversarial_gf81(boundary):
    # GF(3^4), q = 2^7: n_q = 7 is the largest block eq. (2) admits
    p, k, P = 3, 4, (2, 0, 0, 2)
    note(f"gemm padded adversarial GF(3^4) boundary={boundary}")
    C, want = _gemm_case(p, k, P, 48, 40, 256, seed=0, adversarial=True,
                         opts={"n_q": 7, "boundary": boundary})
    assert np.array_equal(C, want)
