"""Parity of centred packing in the LDS-staged packed kernels (tiles 1..6,
opts centered = 1) with the oracle, through the C ABI.  Bit-exact.

Coefficients above (p-1)/2 enter the DQT as c - p; every K-block starts from
2^52 + sum (q/2) q^i so the shifted digits stay in [0, q); the residues of
that shift, n_blocks times, are taken off as one constant element.
"""
import sys

import numpy as np
import pytest

from oracle import gf
from paper_0710_0510_amd import fqt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELDS = [(3, 4, (2, 0, 0, 2)), (5, 3, (3, 3, 0)), (7, 2, (1, 0)), (3, 2, (1, 0)), (13, 1, (11,))]


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


def centred_nq(p, k, b=0):
    q = 2 ** b if b else fqt.params(p, k, 1)[0]
    return gf.centred_nq_max(p, k, q)


def run(p, k, P, M, N, K, seed, opts, A=None, B=None):
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(seed)
    if A is None:
        A = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        B = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
    C = host(fqt.gemm(f, dev(A), dev(B), path="packed", opts=opts))
    return C, gf.gemm_gfpk_planes(A, B, p, P)


SHAPES = [(1, 1, 1), (17, 33, 45), (64, 64, 64), (100, 70, 300), (5, 7, 0), (130, 200, 301),
          (33, 129, 1001)]


@pytest.mark.parametrize("p,k,P", FIELDS)
@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6])
def test_centred_shapes(p, k, P, tile):
    for (M, N, K) in SHAPES:
        note(f"centred GF({p}^{k}) tile={tile} {M}x{N}x{K}")
        C, want = run(p, k, P, M, N, K, seed=M + N + K, opts={"tile": tile, "centered": 1})
        assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("p,k,P", FIELDS[:4])
@pytest.mark.parametrize("boundary", [1, 2])
@pytest.mark.parametrize("nq", [0, 4, 8])
def test_centred_blocks(p, k, P, boundary, nq):
    q = fqt.params(p, k, 1)[0]
    block = nq or centred_nq(p, k)  # products per K-block (a multiple of 4 here)
    for (M, N, K) in [(40, 50, 97), (64, 128, 256), (33, 129, 1001)]:
        note(f"centred blocks GF({p}^{k}) boundary={boundary} n_q={nq} {M}x{N}x{K}")
        case = lambda: run(p, k, P, M, N, K, seed=K + nq,
                           opts={"tile": 2, "centered": 1, "boundary": boundary, "n_q": nq})
        if boundary == 2 and q > 2 ** 12 and K > block:
            # several blocks with digit-sum fields of 2b > 24 bits
            refused("FQT_ERR_UNSUPPORTED", case)
        else:
            C, want = case()
            assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("p,k,P", FIELDS[:4])
@pytest.mark.parametrize("boundary", [1, 2])
def test_centred_adversarial(p, k, P, boundary):
    # the extreme digit sums: every coefficient h against h (+h^2 per term)
    # and h against -h (-h^2), one block at the centred bound and many blocks
    q = fqt.params(p, k, 1)[0]
    h = (p - 1) // 2
    block = centred_nq(p, k)
    nq = min(block, 3000)
    for K in (nq, 3 * nq + 5):
        for bval in (h, p - h):
            note(f"centred adversarial GF({p}^{k}) boundary={boundary} K={K} b={bval}")
            A = np.full((48, K, k), h, dtype=np.uint8)
            B = np.full((K, 96, k), bval, dtype=np.uint8)
            case = lambda: run(p, k, P, 48, 96, K, 0,
                               {"tile": 2, "centered": 1, "boundary": boundary}, A, B)
            if boundary == 2 and q > 2 ** 12 and K > block:
                refused("FQT_ERR_UNSUPPORTED", case)
            else:
                C, want = case()
                assert np.array_equal(C, want), (K, bval)


@pytest.mark.parametrize("p,k,P", FIELDS[:2])
def test_centred_batched_replay(p, k, P):
    # the batched workload's shape mix, one persistent launch, graph replays
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(60 + p)
    shapes = rng.integers(16, 257, size=(30, 3))
    shapes[0] = (256, 130, 700)
    shapes[1] = (3, 300, 5)
    As, Bs, Cs, wants = [], [], [], []
    for (M, N, K) in shapes.tolist():
        a = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        b = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
        As.append(dev(a))
        Bs.append(dev(b))
        Cs.append(torch.zeros((M, N, k), dtype=torch.uint8, device="cuda"))
        wants.append(gf.gemm_gfpk_planes(a, b, p, P))
    descs = fqt.make_descs(f, As, Bs, Cs)
    for boundary in (1, 2):
        for rep in range(2):
            note(f"centred batched GF({p}^{k}) boundary={boundary} replay {rep}")
            for c in Cs:
                c.zero_()
            torch.cuda.synchronize()
            fqt.gemm_batched(f, descs, path="packed",
                             opts={"tile": 2, "centered": 1, "boundary": boundary})
            torch.cuda.synchronize()
            for c, w in zip(Cs, wants):
                assert np.array_equal(host(c), w)
