"""Parity of the wave-persistent packed tile (id 15, k = 4 fields, q = 2^7)
with the CPU oracle, through the C ABI.  Bit-exact.

Every wave computes 32 x 32 outputs of one product alone; K-blocks of
4 n_q/4 products (at most 16) end in a digit-sum block step; operands come
through buffer resources whose out-of-range reads return 0.  The cases
cover edge tiles of every size, K not a multiple of the block, K = 0,
folds of the digit-sum fields, both extreme centred digit signs,
strided operands, batches replayed from the captured graph, and the host's
refusals.
"""
import sys

import numpy as np
import pytest

from oracle import gf
from paper_0710_0510_amd import fqt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GF81 = (3, 4, (2, 0, 0, 2))      # X^4 + 2X^3 + 2
GF16 = (2, 4, (1, 1, 0, 0))      # X^4 + X + 1
TILE = 15


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


def nq_max(p, k, centered):
    q = 2 ** 7
    if centered:
        return gf.centred_nq_max(p, k, q)
    return (q - 1) // (k * (p - 1) ** 2)


def case(field, M, N, K, seed, opts, fill=None):
    p, k, P = field
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(seed)
    if fill is None:
        A = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        B = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
    else:
        A = np.full((M, K, k), fill, dtype=np.uint8)
        B = np.full((K, N, k), fill, dtype=np.uint8)
    C = host(fqt.gemm(f, dev(A), dev(B), path="packed", opts=opts))
    return C, gf.gemm_gfpk_planes(A, B, p, P)


SHAPES = [(1, 1, 1), (17, 33, 45), (32, 32, 12), (33, 31, 13), (64, 96, 48), (100, 70, 300),
          (5, 7, 0), (16, 16, 4), (130, 47, 257)]


@pytest.mark.parametrize("field,centered", [(GF81, 0), (GF81, 1), (GF16, 0)])
@pytest.mark.parametrize("nq", [4, 8, 12, 16])
def test_wave_shapes(field, centered, nq):
    p, k, _ = field
    for (M, N, K) in SHAPES:
        note(f"wave GF({p}^{k}) centered={centered} n_q={nq} {M}x{N}x{K}")
        run = lambda: case(field, M, N, K, seed=M + N + K + nq,
                           opts={"tile": TILE, "n_q": nq, "centered": centered})
        if nq > nq_max(p, k, centered):
            refused("FQT_ERR_BOUNDS", run)
            continue
        C, want = run()
        assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("field,centered", [(GF81, 0), (GF81, 1), (GF16, 0)])
def test_wave_default_nq_long_k_folds(field, centered):
    # the digit-sum fields (14 bits) are folded mod p every ~126 blocks; with
    # blocks of 4 (GF(3^4) uncentred) K = 2001 is 501 blocks
    p, k, _ = field
    for K in (2001, 1024):
        note(f"wave GF({p}^{k}) centered={centered} default n_q K={K}")
        C, want = case(field, 40, 36, K, seed=K, opts={"tile": TILE, "centered": centered})
        assert np.array_equal(C, want), K


@pytest.mark.parametrize("field,centered", [(GF81, 0), (GF81, 1), (GF16, 0)])
def test_wave_adversarial(field, centered):
    # all coefficients p - 1 (centred: -h) and, centred, all 1 (+h): every
    # digit of every block at its bound, at the largest n_q, across folds
    p, k, _ = field
    nq = nq_max(p, k, centered)
    fills = [p - 1] + ([1] if centered else [])
    for fill in fills:
        for K in (nq, 4 * nq + 3, 1500):
            note(f"wave adversarial GF({p}^{k}) centered={centered} fill={fill} K={K}")
            C, want = case(field, 33, 34, K, seed=0, fill=fill,
                           opts={"tile": TILE, "centered": centered})
            assert np.array_equal(C, want), (fill, K)


def test_wave_strided_operands():
    p, k, P = GF81
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(9)
    Abig = rng.integers(0, p, size=(70, 93, k), dtype=np.uint8)
    Bbig = rng.integers(0, p, size=(93, 75, k), dtype=np.uint8)
    for cen in (0, 1):
        note(f"wave strided centered={cen}")
        C = host(fqt.gemm(f, dev(Abig)[:50, :61], dev(Bbig)[:61, :40], path="packed",
                          opts={"tile": TILE, "centered": cen}))
        assert np.array_equal(C, gf.gemm_gfpk_planes(Abig[:50, :61], Bbig[:61, :40], p, P))


def test_wave_batched_replays():
    p, k, P = GF81
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(37)
    shapes = rng.integers(1, 120, size=(60, 3))
    shapes[0] = (256, 256, 256)
    shapes[1] = (1, 1, 0)
    As, Bs, Cs, wants = [], [], [], []
    for (M, N, K) in shapes.tolist():
        a = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        b = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
        As.append(dev(a))
        Bs.append(dev(b))
        Cs.append(torch.zeros((M, N, k), dtype=torch.uint8, device="cuda"))
        wants.append(gf.gemm_gfpk_planes(a, b, p, P))
    descs = fqt.make_descs(f, As, Bs, Cs)
    for cen in (0, 1):
        for rep in range(3):
            note(f"wave batched centered={cen} replay {rep}")
            for c in Cs:
                c.fill_(0xEE)
            fqt.gemm_batched(f, descs, path="packed", opts={"tile": TILE, "centered": cen})
            torch.cuda.synchronize()
            for i, (c, w) in enumerate(zip(Cs, wants)):
                assert np.array_equal(host(c), w), (cen, rep, i, shapes[i])


def test_wave_refusals():
    p, k, P = GF81
    f = fqt.Field(p, k, P)
    A = torch.zeros((8, 8, k), dtype=torch.uint8, device="cuda")
    B = torch.zeros((8, 8, k), dtype=torch.uint8, device="cuda")
    note("wave refusals")
    refused("FQT_ERR_UNSUPPORTED", lambda: fqt.gemm(f, A, B, path="packed",
                                                     opts={"tile": TILE, "boundary": 1}))
    refused("FQT_ERR_UNSUPPORTED", lambda: fqt.gemm(f, A, B, path="packed",
                                                     opts={"tile": TILE, "log2q": 6}))
    refused("FQT_ERR_BOUNDS", lambda: fqt.gemm(f, A, B, path="packed",
                                               opts={"tile": TILE, "n_q": 8}))
    # k = 2 fields are not this tile's
    f2 = fqt.Field(7, 2, (1, 0))
    A2 = torch.zeros((8, 8, 2), dtype=torch.uint8, device="cuda")
    refused("FQT_ERR_UNSUPPORTED", lambda: fqt.gemm(f2, A2, A2, path="packed",
                                                     opts={"tile": TILE}))
    # centring needs an odd p
    p2, k2, P2 = GF16
    f16 = fqt.Field(p2, k2, P2)
    refused("FQT_ERR_UNSUPPORTED", lambda: fqt.gemm(f16, A, B, path="packed",
                                                     opts={"tile": TILE, "centered": 1}))
    # operands read as words: a view one byte into a buffer is refused
    flat = torch.zeros(8 * 8 * k + 1, dtype=torch.uint8, device="cuda")
    Av = flat[1:].view(8, 8, k)
    refused("FQT_ERR_UNSUPPORTED", lambda: fqt.gemm(f, Av, B, path="packed",
                                                     opts={"tile": TILE}))
