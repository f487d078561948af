"""Parity of the d-split packed kernels (tile ids 13 and 14, k = 3 or 4) with
the oracle, through the C ABI.  Bit-exact: the canonical field element is
unique.

Every element is cut into two chunks of 2 coefficients packed at q = 2^17;
the three chunk-pair sums are contracted on the matrix cores and the middle
one is recovered digit by digit (one Karatsuba step).  One block holds
n_q = (2^17 - 1) / (w (p-1)^2) products (w = 8 for k = 4, 4 for k = 3);
longer K restarts every block from its digits mod p.
"""
import sys

import numpy as np
import pytest

from oracle import gf
from paper_0710_0510_amd import fqt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (p, k, P_low): the workload fields GF(3^4) and GF(5^3), p = 2, and the
# largest p the binary table index allows for k = 4 and k = 3
FIELDS = [(3, 4, (2, 0, 0, 2)), (5, 3, (3, 3, 0)), (2, 4, (1, 0, 0, 1)), (2, 3, (1, 0, 1)),
          (7, 4, (1, 0, 0, 1)), (13, 3, (1, 0, 4))]
SPLIT = [13, 14]


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


def nq_split(p, k):
    """Products of one d-split block: S_K's digits grow by w (p-1)^2 per k."""
    w = 8 if k == 4 else 4
    return (2 ** 17 - 1) // (w * (p - 1) ** 2)


def run(p, k, P, M, N, K, tile, seed, adversarial=False, opts=None):
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(seed)
    if adversarial:
        A = np.full((M, K, k), p - 1, dtype=np.uint8)
        B = np.full((K, N, k), p - 1, dtype=np.uint8)
    else:
        A = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        B = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
    o = {"tile": tile}
    o.update(opts or {})
    C = host(fqt.gemm(f, dev(A), dev(B), path="packed", opts=o))
    return C, gf.gemm_gfpk_planes(A, B, p, P)


# ragged M, N against the 32 x 128 and 64 x 64 workgroup tiles, K tails of
# every residue mod 16, empty K, and K past one block for the large p
SHAPES = [(1, 1, 1), (17, 33, 45), (64, 64, 64), (100, 70, 300), (33, 130, 16), (5, 7, 0),
          (130, 200, 301), (64, 128, 1000), (200, 72, 33), (129, 257, 17), (16, 16, 250)]


@pytest.mark.parametrize("p,k,P", FIELDS)
@pytest.mark.parametrize("tile", SPLIT)
def test_split_shapes(p, k, P, tile):
    for (M, N, K) in SHAPES:
        note(f"split GF({p}^{k}) tile={tile} {M}x{N}x{K}")
        C, want = run(p, k, P, M, N, K, tile, seed=M + N + K)
        assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("p,k,P", FIELDS[:2] + FIELDS[4:])
@pytest.mark.parametrize("tile", SPLIT)
def test_split_adversarial(p, k, P, tile):
    # every coefficient p-1: K = n_q fills one block to eq. (2)'s bound for
    # the chunks; 2 n_q + 37 runs three blocks, each restarted near its bound
    nq = nq_split(p, k)
    for K in (nq, 2 * nq + 37):
        note(f"split adversarial GF({p}^{k}) tile={tile} K={K}")
        C, want = run(p, k, P, 48, 96, K, tile, seed=0, adversarial=True)
        assert np.array_equal(C, want), K


@pytest.mark.parametrize("nq", [16, 40, 100])
def test_split_short_blocks(nq):
    # a smaller n_q: blocks of floor(n_q / 16) 16-k steps
    p, k, P = 3, 4, (2, 0, 0, 2)
    for (M, N, K) in [(40, 50, 97), (64, 128, 256), (33, 129, 1001)]:
        note(f"split short blocks n_q={nq} {M}x{N}x{K}")
        C, want = run(p, k, P, M, N, K, 13, seed=nq + K, opts={"n_q": nq})
        assert np.array_equal(C, want), (M, N, K)


def test_split_long_k_gf125():
    # GF(5^3): n_q = 2047, K = 4096 (the 4096^3 workload's K) takes 3 blocks
    p, k, P = 5, 3, (3, 3, 0)
    for adversarial in (False, True):
        note(f"split GF(5^3) K=4096 adversarial={adversarial}")
        C, want = run(p, k, P, 40, 72, 4096, 14, seed=5, adversarial=adversarial)
        assert np.array_equal(C, want)


@pytest.mark.parametrize("tile", SPLIT)
def test_split_strided_and_unaligned(tile):
    # odd row strides: rows off 4-byte boundaries take the byte-gather loads
    p, k, P = 5, 3, (3, 3, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(9)
    for (rows, cols) in [((70, 91), (91, 75)), ((130, 300), (300, 260))]:
        Abig = rng.integers(0, p, size=rows + (k,), dtype=np.uint8)
        Bbig = rng.integers(0, p, size=cols + (k,), dtype=np.uint8)
        m, kk, n = rows[0] - 5, rows[1] - 7, cols[1] - 3
        note(f"split strided/unaligned tile={tile} {m}x{n}x{kk}")
        C = host(fqt.gemm(f, dev(Abig)[:m, :kk], dev(Bbig)[:kk, :n], path="packed",
                          opts={"tile": tile}))
        want = gf.gemm_gfpk_planes(Abig[:m, :kk], Bbig[:kk, :n], p, P)
        assert np.array_equal(C, want)


def test_split_output_strided():
    # C with a row stride wider than N; nothing is written past column N
    p, k, P = 3, 4, (2, 0, 0, 2)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(21)
    A = rng.integers(0, p, size=(96, 20, k), dtype=np.uint8)
    B = rng.integers(0, p, size=(20, 130, k), dtype=np.uint8)
    for ldc in (130, 131, 200):
        note(f"split strided C ldc={ldc}")
        Cbig = torch.zeros((96, ldc, k), dtype=torch.uint8, device="cuda")
        fqt.gemm(f, dev(A), dev(B), Cbig[:, :130], path="packed", opts={"tile": 13})
        out = host(Cbig)
        assert np.array_equal(out[:, :130], gf.gemm_gfpk_planes(A, B, p, P))
        assert not out[:, 130:].any()


@pytest.mark.parametrize("p,k,P", FIELDS[:2])
@pytest.mark.parametrize("tile", SPLIT)
def test_split_batched_replay(p, k, P, tile):
    # one persistent launch over uneven products (16..256 like the batched
    # workload, plus tiny and long-K ones), captured in a graph and replayed
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(50 + tile + p)
    shapes = rng.integers(16, 257, size=(30, 3))
    shapes[0] = (256, 130, 3000)
    shapes[1] = (3, 300, 5)
    shapes[2] = (1, 1, 1)
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
        note(f"split batched GF({p}^{k}) tile={tile} replay {rep}")
        for c in Cs:
            c.zero_()
        torch.cuda.synchronize()
        fqt.gemm_batched(f, descs, path="packed", opts={"tile": tile})
        torch.cuda.synchronize()
        for c, w in zip(Cs, wants):
            assert np.array_equal(host(c), w)


def test_split_matches_other_tiles():
    # the d-split tiles give the same bytes as the single-q tiles
    p, k, P = 3, 4, (2, 0, 0, 2)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(13)
    A = dev(rng.integers(0, p, size=(200, 700, k), dtype=np.uint8))
    B = dev(rng.integers(0, p, size=(700, 300, k), dtype=np.uint8))
    ref = host(fqt.gemm(f, A, B, path="packed", opts={"tile": 2}))
    for tile in SPLIT:
        note(f"split vs tile 2 GF(3^4) tile={tile}")
        assert np.array_equal(host(fqt.gemm(f, A, B, path="packed", opts={"tile": tile})), ref)
