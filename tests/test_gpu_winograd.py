"""Parity of Winograd's recursion over GF(p^k) (fqt_gemm_winograd) with the
oracle, through the C ABI.  Bit-exact: the canonical field element is unique.

Per level, seven block products on the chosen path and fifteen block
additions mod p; odd dimensions are peeled (last row, last column, last k).
"""
import sys

import numpy as np
import pytest

from oracle import gf
from paper_0710_0510_amd import fqt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELDS = [(7, 2, (1, 0)), (3, 4, (2, 0, 0, 2)), (5, 3, (3, 3, 0)), (2, 1, (1,))]


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


SHAPES = [(2, 2, 2), (64, 64, 64), (65, 63, 67), (128, 130, 96), (33, 257, 200), (1, 5, 9),
          (200, 1, 30), (40, 50, 1), (96, 96, 0)]


@pytest.mark.parametrize("p,k,P", FIELDS)
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_winograd_shapes(p, k, P, levels):
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(p + 10 * levels)
    for (M, N, K) in SHAPES:
        note(f"winograd GF({p}^{k}) levels={levels} {M}x{N}x{K}")
        A = rng.integers(0, p, size=(M, K, k), dtype=np.uint8)
        B = rng.integers(0, p, size=(K, N, k), dtype=np.uint8)
        C = host(fqt.gemm_winograd(f, dev(A), dev(B), levels=levels, path="packed"))
        assert np.array_equal(C, gf.gemm_gfpk_planes(A, B, p, P)), (M, N, K)


@pytest.mark.parametrize("path,opts", [("packed", {"tile": 9}), ("packed", {"tile": 7}),
                                       ("packed", {"tile": 2}), ("int8", None), ("plain", None)])
def test_winograd_base_paths(path, opts):
    p, k, P = 7, 2, (1, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(3)
    A = rng.integers(0, p, size=(150, 210, k), dtype=np.uint8)
    B = rng.integers(0, p, size=(210, 170, k), dtype=np.uint8)
    note(f"winograd base path {path} {opts}")
    C = host(fqt.gemm_winograd(f, dev(A), dev(B), levels=2, path=path, opts=opts))
    assert np.array_equal(C, gf.gemm_gfpk_planes(A, B, p, P))


def test_winograd_strided_operands_and_output():
    p, k, P = 5, 3, (3, 3, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(8)
    Abig = rng.integers(0, p, size=(100, 91, k), dtype=np.uint8)
    Bbig = rng.integers(0, p, size=(91, 130, k), dtype=np.uint8)
    Cbig = torch.zeros((90, 131, k), dtype=torch.uint8, device="cuda")
    note("winograd strided")
    fqt.gemm_winograd(f, dev(Abig)[:90, :85], dev(Bbig)[:85, :120], Cbig[:, :120], levels=2,
                      path="packed")
    out = host(Cbig)
    assert np.array_equal(out[:, :120], gf.gemm_gfpk_planes(Abig[:90, :85], Bbig[:85, :120], p, P))
    assert not out[:, 120:].any()


def test_winograd_1024_equals_the_single_call():
    # the headline shape, every byte: one and two levels against one call of
    # the packed path, twice in a row (the temporaries are reused)
    p, k, P = 7, 2, (1, 0)
    f = fqt.Field(p, k, P)
    rng = np.random.default_rng(2)
    A = dev(rng.integers(0, p, size=(1024, 1024, k), dtype=np.uint8))
    B = dev(rng.integers(0, p, size=(1024, 1024, k), dtype=np.uint8))
    ref = fqt.gemm(f, A, B, path="packed", opts={"tile": 7})
    for levels in (1, 2, 1):
        note(f"winograd 1024^3 levels={levels}")
        C = fqt.gemm_winograd(f, A, B, levels=levels, path="packed", opts={"tile": 7})
        torch.cuda.synchronize()
        assert torch.equal(C, ref), levels
