"""Parity of the INT8 strip tile (INT8 id 11, k = 4 fields) with the CPU
oracle, through the C ABI.  Bit-exact.

One workgroup per strip of 16 output elements of a product: B' of every
K-tile built in LDS from the multiplication-matrix table and shared by all
rows; operands through buffer resources whose out-of-range reads are zero.
The cases cover edge strips and row chunks, K not a multiple of the 64-element
K-tile, K = 0, more than 256 rows (row groups), strided operands, the
binary64 reduction of large INT32 sums, batches replayed from the graph and
the host's refusals.
"""
import itertools
import sys

import numpy as np
import pytest

from oracle import gf
from paper_0710_0510_amd import fqt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TILE = 11
GF81 = (3, 4, (2, 0, 0, 2))      # X^4 + 2X^3 + 2
GF16 = (2, 4, (1, 1, 0, 0))      # X^4 + X + 1


def first_irreducible_quartic(p):
    for low in itertools.product(range(p), repeat=4):
        if low[0] and gf.is_irreducible(low, p):
            return tuple(low)
    raise AssertionError(p)


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
    with pytest.raises(fqt.FqtError) as ei:
        fn()
    assert ei.value.name == status, str(ei.value)


def case(field, M, N, K, seed, fill=None):
    p, k, P = field
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(seed)
    if fill is None:
        A = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        B = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
    else:
        A = np.full((M, K, k), fill, dtype=np.uint8)
        B = np.full((K, N, k), fill, dtype=np.uint8)
    C = host(fqt.gemm(f, dev(A), dev(B), path="int8", opts={"tile": TILE}))
    return C, gf.gemm_gfpk_planes(A, B, p, P)


SHAPES = [(1, 1, 1), (17, 33, 45), (32, 16, 64), (33, 17, 65), (100, 70, 300), (5, 7, 0),
          (256, 48, 129), (300, 20, 77), (16, 16, 4)]


@pytest.mark.parametrize("field", [GF81, GF16, "gf7^4"])
def test_i8strip_shapes(field):
    if field == "gf7^4":
        field = (7, 4, first_irreducible_quartic(7))
    p, k, _ = field
    for (M, N, K) in SHAPES:
        note(f"int8 strip GF({p}^{k}) {M}x{N}x{K}")
        C, want = case(field, M, N, K, seed=M + N + K)
        assert np.array_equal(C, want), (M, N, K)


def test_i8strip_adversarial_and_large_sums():
    # all coefficients p - 1; GF(7^4) with K = 240000 puts the INT32 sums
    # above 2^25, so the epilogue takes the binary64 reduction
    for field, K in ((GF81, 3001), ((7, 4, first_irreducible_quartic(7)), 240000)):
        p = field[0]
        note(f"int8 strip adversarial GF({p}^4) K={K}")
        C, want = case(field, 8, 20, K, seed=0, fill=p - 1)
        assert np.array_equal(C, want), K


def test_i8strip_strided():
    p, k, P = GF81
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(5)
    Abig = rng.integers(0, p, size=(70, 93, k), dtype=np.uint8)
    Bbig = rng.integers(0, p, size=(93, 75, k), dtype=np.uint8)
    note("int8 strip strided")
    C = host(fqt.gemm(f, dev(Abig)[:50, :61], dev(Bbig)[:61, :40], path="int8",
                      opts={"tile": TILE}))
    assert np.array_equal(C, gf.gemm_gfpk_planes(Abig[:50, :61], Bbig[:61, :40], p, P))


def test_i8strip_batched_replays():
    p, k, P = GF81
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(41)
    shapes = rng.integers(1, 140, size=(50, 3))
    shapes[0] = (256, 256, 256)
    shapes[1] = (3, 2, 0)
    As, Bs, Cs, wants = [], [], [], []
    for (M, N, K) in shapes.tolist():
        a = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        b = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
        As.append(dev(a))
        Bs.append(dev(b))
        Cs.append(torch.zeros((M, N, k), dtype=torch.uint8, device="cuda"))
        wants.append(gf.gemm_gfpk_planes(a, b, p, P))
    descs = fqt.make_descs(f, As, Bs, Cs)
    for rep in range(3):
        note(f"int8 strip batched replay {rep}")
        for c in Cs:
            c.fill_(0xEE)
        fqt.gemm_batched(f, descs, path="int8", opts={"tile": TILE})
        torch.cuda.synchronize()
        for i, (c, w) in enumerate(zip(Cs, wants)):
            assert np.array_equal(host(c), w), (rep, i, shapes[i])


def test_i8strip_refusals():
    note("int8 strip refusals")
    f2 = fqt.Field(7, 2, (1, 0))
    A2 = torch.zeros((8, 8, 2), dtype=torch.uint8, device="cuda")
    refused("FQT_ERR_UNSUPPORTED", lambda: fqt.gemm(f2, A2, A2, path="int8", opts={"tile": TILE}))
    p, k, P = GF81
    f = fqt.Field(p, k, P)
    flat = torch.zeros(8 * 8 * k + 1, dtype=torch.uint8, device="cuda")
    B = torch.zeros((8, 8, k), dtype=torch.uint8, device="cuda")
    refused("FQT_ERR_UNSUPPORTED", lambda: fqt.gemm(f, flat[1:].view(8, 8, k), B, path="int8",
                                                     opts={"tile": TILE}))
