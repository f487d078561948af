"""Parity of the register-direct packed kernels (tile ids 7..12) with the
oracle, through the C ABI.  Bit-exact: the canonical field element is unique.

Tiles 7, 8 and 12 split the K-steps across the waves of a workgroup (4, 2
and 4 ways; tile 12 runs 8 waves, two per SIMD) and combine the partial
accumulators at the end; tiles 9..11 give every wave its own output tile.
All but tile 11 take one K-block (K <= n_q); tile 11 also carries several
(both boundary modes).
"""
import sys

import numpy as np
import pytest

from oracle import gf
from paper_0710_0510_amd import fqt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELDS = [(7, 2, (1, 0)), (3, 4, (2, 0, 0, 2)), (5, 3, (3, 3, 0)), (3, 2, (1, 0)),
          (2, 1, (1,)), (13, 1, (11,))]
DIRECT = [7, 8, 9, 10, 11, 12]
SINGLE_ONLY = {7, 8, 9, 10, 12}


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


def nq_direct(p, k):
    """Products per K-block of the direct tiles: eq. (2)'s bound at the
    largest q, rounded down to whole MFMA k-groups of 4."""
    return fqt.params(p, k, 1)[1] // 4 * 4


def refused(status, fn):
    """The host refuses the call with `status` before any launch."""
    with pytest.raises(fqt.FqtError) as ei:
        fn()
    assert ei.value.name == status, str(ei.value)


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


SHAPES = [(1, 1, 1), (17, 33, 45), (64, 64, 64), (100, 70, 300), (33, 130, 16), (5, 7, 0),
          (130, 200, 300), (64, 128, 1000), (200, 72, 33), (129, 257, 17)]


@pytest.mark.parametrize("p,k,P", FIELDS)
@pytest.mark.parametrize("tile", DIRECT)
def test_direct_shapes(p, k, P, tile):
    nq = nq_direct(p, k)
    for (M, N, K) in SHAPES:
        note(f"direct GF({p}^{k}) tile={tile} {M}x{N}x{K}")
        if tile in SINGLE_ONLY and K > nq:
            with pytest.raises(fqt.FqtError) as ei:
                run(p, k, P, M, N, K, tile, seed=M + N + K)
            assert ei.value.name == "FQT_ERR_UNSUPPORTED"
            continue
        C, want = run(p, k, P, M, N, K, tile, seed=M + N + K)
        assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("tile", [7, 8, 11, 12])
def test_direct_split_k_edges(tile):
    # K-steps of 16 shared by 4 (tiles 7, 12) or 2 (tile 8) waves: fewer steps
    # than waves, a ragged last step, steps that do not divide evenly
    p, k, P = 7, 2, (1, 0)
    for K in [0, 1, 3, 15, 16, 17, 31, 32, 48, 63, 64, 65, 80, 127, 1819, 1820]:
        note(f"direct split-K edges tile={tile} K={K}")
        C, want = run(p, k, P, 70, 136, K, tile, seed=K)
        assert np.array_equal(C, want), K


@pytest.mark.parametrize("p,k,P", FIELDS[:4])
@pytest.mark.parametrize("tile", [7, 8, 9, 11, 12])
def test_direct_adversarial_single_block(p, k, P, tile):
    # every coefficient p-1 and K = n_q: the packed sums reach eq. (2)'s bound
    nq = min(nq_direct(p, k), 3000)
    note(f"direct adversarial GF({p}^{k}) tile={tile} K={nq}")
    C, want = run(p, k, P, 64, 128, nq, tile, seed=0, adversarial=True)
    assert np.array_equal(C, want)


@pytest.mark.parametrize("p,k,P", FIELDS[:4])
@pytest.mark.parametrize("nq", [4, 8, 12, 20])
@pytest.mark.parametrize("boundary", [1, 2])
def test_direct_multiblock(p, k, P, nq, boundary):
    q, nqmax = fqt.params(p, k, 1)
    for (M, N, K) in [(40, 50, 97), (64, 128, 256), (33, 129, 1001)]:
        note(f"direct multiblock GF({p}^{k}) n_q={nq} boundary={boundary} {M}x{N}x{K}")
        case = lambda: run(p, k, P, M, N, K, 11, seed=nq + K,
                           opts={"n_q": nq, "boundary": boundary})
        if nq > nqmax:  # eq. (2) fails for this n_q at the largest q
            refused("FQT_ERR_BOUNDS", case)
        elif boundary == 2 and q > 2 ** 12:  # every K here exceeds n_q: several blocks
            refused("FQT_ERR_UNSUPPORTED", case)
        else:
            C, want = case()
            assert np.array_equal(C, want), (M, N, K)


@pytest.mark.parametrize("p,k,P", [(3, 4, (2, 0, 0, 2)), (5, 3, (3, 3, 0))])
@pytest.mark.parametrize("boundary", [1, 2])
def test_direct_multiblock_adversarial(p, k, P, boundary):
    # default n_q of the direct tiles (rounded down to a multiple of 4), all p-1
    nq = nq_direct(p, k)
    for K in [3 * nq + 5, 777]:
        note(f"direct multiblock adversarial GF({p}^{k}) boundary={boundary} K={K}")
        C, want = run(p, k, P, 48, 128, K, 11, seed=0, adversarial=True,
                      opts={"boundary": boundary})
        assert np.array_equal(C, want)


def test_direct_lane_folding_residues():
    # 10000 blocks of 4 products: the 16-bit residue lanes are folded mod p
    p, k, P = 7, 2, (1, 0)
    for adversarial in (True, False):
        note(f"direct folding residues adversarial={adversarial}")
        C, want = run(p, k, P, 33, 72, 40000, 11, seed=7, adversarial=adversarial,
                      opts={"n_q": 4, "boundary": 1})
        assert np.array_equal(C, want)


def test_direct_field_folding_digits():
    # GF(3^4), q = 2^7, blocks of 4: K = 3000 is 750 blocks, the 14-bit digit
    # fields are folded mod p on the way
    p, k, P = 3, 4, (2, 0, 0, 2)
    for adversarial in (True, False):
        note(f"direct folding digits adversarial={adversarial}")
        C, want = run(p, k, P, 33, 72, 3000, 11, seed=8, adversarial=adversarial,
                      opts={"boundary": 2})
        assert np.array_equal(C, want)


@pytest.mark.parametrize("tile", [7, 9, 11])
def test_direct_strided_and_unaligned(tile):
    p, k, P = 7, 2, (1, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(9)
    for (rows, cols) in [((70, 91), (91, 75)), ((130, 300), (300, 260))]:
        Abig = rng.integers(0, p, size=rows + (k,), dtype=np.uint8)   # odd ld: unaligned rows
        Bbig = rng.integers(0, p, size=cols + (k,), dtype=np.uint8)
        m, kk, n = rows[0] - 5, rows[1] - 7, cols[1] - 3
        note(f"direct strided/unaligned tile={tile} {m}x{n}x{kk}")
        C = host(fqt.gemm(f, dev(Abig)[:m, :kk], dev(Bbig)[:kk, :n], path="packed",
                          opts={"tile": tile}))
        want = gf.gemm_gfpk_planes(Abig[:m, :kk], Bbig[:kk, :n], p, P)
        assert np.array_equal(C, want)


def test_direct_output_strided():
    # C with a row stride wider than N, one that is not a multiple of 4 bytes
    p, k, P = 5, 3, (3, 3, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(21)
    A = rng.integers(0, p, size=(96, 20, k), dtype=np.uint8)
    B = rng.integers(0, p, size=(20, 130, k), dtype=np.uint8)
    for ldc in (130, 131, 200):
        note(f"direct strided C ldc={ldc}")
        Cbig = torch.zeros((96, ldc, k), dtype=torch.uint8, device="cuda")
        fqt.gemm(f, dev(A), dev(B), Cbig[:, :130], path="packed", opts={"tile": 11})
        out = host(Cbig)
        assert np.array_equal(out[:, :130], gf.gemm_gfpk_planes(A, B, p, P))
        assert not out[:, 130:].any()  # nothing written beyond the N columns


def test_direct_all_tiles_identical():
    p, k, P = 7, 2, (1, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(12)
    Ah = rng.integers(0, p, size=(300, 1000, k), dtype=np.uint8)
    Bh = rng.integers(0, p, size=(1000, 260, k), dtype=np.uint8)
    A, B = dev(Ah), dev(Bh)
    want = gf.gemm_gfpk_planes(Ah, Bh, p, P)
    for tile in range(1, 13):  # every tile but the d-split ones, which need k >= 3
        note(f"all tiles identical GF(7^2) tile={tile}")
        assert np.array_equal(host(fqt.gemm(f, A, B, path="packed", opts={"tile": tile})), want)


@pytest.mark.parametrize("tile", DIRECT)
def test_direct_batched_replay(tile):
    # one persistent launch over uneven products, captured in a graph and replayed
    p, k, P = 7, 2, (1, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(40 + tile)
    shapes = rng.integers(1, 200, size=(30, 3))
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
    for rep in range(3):
        note(f"direct batched tile={tile} replay {rep}")
        for c in Cs:
            c.zero_()
        fqt.gemm_batched(f, descs, path="packed", opts={"tile": tile})
        torch.cuda.synchronize()
        for c, w in zip(Cs, wants):
            assert np.array_equal(host(c), w)


def test_direct_batched_multiblock_gf81():
    # GF(3^4): every product with K > 4 has several K-blocks; tile 11 only
    p, k, P = 3, 4, (2, 0, 0, 2)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(77)
    shapes = rng.integers(16, 200, size=(25, 3))
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
            note(f"direct batched GF(3^4) boundary={boundary} replay {rep}")
            for c in Cs:
                c.zero_()
            fqt.gemm_batched(f, descs, path="packed", opts={"tile": 11, "boundary": boundary})
            torch.cuda.synchronize()
            for c, w in zip(Cs, wants):
                assert np.array_equal(host(c), w)
