"""Parity of the d-FQT product of long polynomials (Section 6) and of its
delayed-reduction comparator with the oracle's product definition, through
the C ABI.  Bit-exact."""
import sys

import numpy as np
import pytest

from oracle import gf
from paper_0710_0510_amd import fqt
from paper_0710_0510_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def want_rows(a, b, p):
    return np.array([gf.polymul_long(x.tolist(), y.tolist(), p) for x, y in zip(a, b)],
                    dtype=np.uint8).reshape(a.shape[0], 2 * a.shape[1] - 1)


# (p, d) pairs eq. (2) admits at the largest q; one block or several
PD = [(2, 0), (2, 1), (2, 5), (3, 0), (3, 1), (3, 2), (3, 3), (3, 4), (5, 2), (5, 3), (7, 1),
      (13, 1), (127, 0), (127, 1)]


@pytest.mark.parametrize("p,d", PD)
def test_dfqt_matches_product_definition(p, d):
    rng = np.random.default_rng(p * 100 + d)
    lens = sorted({1, 2, d + 1, d + 2, 37, 255, 256, 257, 501, min(1024 * (d + 1), 3000)})
    for length in lens:
        for count in (1, 5):
            note(f"dfqt p={p} d={d} len={length} count={count}")
            a = rng.integers(0, p, size=(count, length), dtype=np.uint8)
            b = rng.integers(0, p, size=(count, length), dtype=np.uint8)
            out = host(fqt.polymul_dfqt(p, d, dev(a), dev(b)))
            assert np.array_equal(out, want_rows(a, b, p)), (length, count)


@pytest.mark.parametrize("p,d,nq", [(3, 2, 1), (3, 2, 2), (3, 2, 7), (3, 2, 85), (3, 4, 1),
                                    (7, 1, 1), (7, 1, 5), (5, 3, 3)])
@pytest.mark.parametrize("boundary", [1, 2])
def test_dfqt_block_modes(p, d, nq, boundary):
    q, nqmax = gf.max_pow2_q(p, d + 1)
    zeros = dev(np.zeros((1, 1000), np.uint8))
    if nq > nqmax:  # eq. (2) fails for this n_q with k = d + 1 at the largest q
        refused("FQT_ERR_BOUNDS", lambda: fqt.polymul_dfqt(p, d, zeros, zeros, n_q=nq,
                                                             boundary=boundary))
        return
    if boundary == 2 and q > 2 ** 12:
        refused("FQT_ERR_UNSUPPORTED", lambda: fqt.polymul_dfqt(p, d, zeros, zeros, n_q=nq,
                                                                  boundary=2))
        return
    rng = np.random.default_rng(nq * 10 + d)
    for length in (255, 1000, 1024 * (d + 1)):
        note(f"dfqt blocks p={p} d={d} n_q={nq} boundary={boundary} len={length}")
        a = rng.integers(0, p, size=(3, length), dtype=np.uint8)
        b = rng.integers(0, p, size=(3, length), dtype=np.uint8)
        out = host(fqt.polymul_dfqt(p, d, dev(a), dev(b), n_q=nq, boundary=boundary))
        assert np.array_equal(out, want_rows(a, b, p))


@pytest.mark.parametrize("p,d,boundary", [(3, 4, 1), (3, 4, 2), (3, 2, 2), (7, 1, 1), (5, 3, 2)])
def test_dfqt_adversarial_longest(p, d, boundary):
    # every coefficient p-1 at the longest length: blocks reach eq. (2)'s
    # bound, and with d = 4 the 10-bit digit fields are folded mod p
    length = 1024 * (d + 1)
    note(f"dfqt adversarial p={p} d={d} boundary={boundary} len={length}")
    a = np.full((2, length), p - 1, dtype=np.uint8)
    out = host(fqt.polymul_dfqt(p, d, dev(a), dev(a), boundary=boundary))
    assert np.array_equal(out, want_rows(a, a, p))


def test_dfqt_smaller_q_single_block():
    # q = 2^14 < 2^17 for d = 1: allowed while one block holds every product
    p, d = 3, 1
    rng = np.random.default_rng(4)
    a = rng.integers(0, p, size=(4, 300), dtype=np.uint8)
    b = rng.integers(0, p, size=(4, 300), dtype=np.uint8)
    note("dfqt single block q=2^14")
    out = host(fqt.polymul_dfqt(p, d, dev(a), dev(b), log2q=14))
    assert np.array_equal(out, want_rows(a, b, p))


def test_dfqt_empty_batch():
    out = fqt.polymul_dfqt(3, 4, torch.empty((0, 501), dtype=torch.uint8, device="cuda"),
                           torch.empty((0, 501), dtype=torch.uint8, device="cuda"))
    assert out.shape == (0, 1001)


@pytest.mark.parametrize("p", [2, 3, 7, 127])
def test_delayed_matches_product_definition(p):
    rng = np.random.default_rng(p)
    for length in (1, 2, 3, 64, 255, 256, 257, 501, 2000, 8192):
        count = 3 if length > 1000 else 5
        note(f"delayed p={p} len={length}")
        a = rng.integers(0, p, size=(count, length), dtype=np.uint8)
        b = rng.integers(0, p, size=(count, length), dtype=np.uint8)
        out = host(fqt.polymul_delayed(p, dev(a), dev(b)))
        assert np.array_equal(out, want_rows(a, b, p)), length
    a = np.full((2, 8192), p - 1, dtype=np.uint8)
    assert np.array_equal(host(fqt.polymul_delayed(p, dev(a), dev(a))), want_rows(a, a, p))


def test_dfqt_workload_sampled():
    # the benchmark's batch (p = 3, N = 500, d = 4, 16384 pairs) in the launch
    # configuration it times, against the oracle on sampled products; the
    # comparator agrees on every product
    w = W.WORKLOADS["dfqt-gf3-n500-d4"]
    a_h, b_h = W.poly_long_inputs(w)
    a, b = dev(a_h), dev(b_h)
    note("dfqt workload")
    out = fqt.polymul_dfqt(w.p, w.d, a, b)
    ref = fqt.polymul_delayed(w.p, a, b)
    out_h = host(out)
    assert torch.equal(out, ref)
    rng = np.random.default_rng(11)
    picks = sorted({0, w.count - 1} | set(rng.integers(0, w.count, size=64).tolist()))
    assert np.array_equal(out_h[picks], want_rows(a_h[picks], b_h[picks], w.p))


# ---- centred chunks ------------------------------------------------------------

CPD = [(p, d) for (p, d) in PD if p % 2 == 1]


@pytest.mark.parametrize("p,d", CPD)
def test_dfqt_centred_matches_product_definition(p, d):
    rng = np.random.default_rng(p * 1000 + d)
    for length in sorted({1, 2, d + 1, 37, 256, 501, min(1024 * (d + 1), 3000)}):
        note(f"dfqt centred p={p} d={d} len={length}")
        a = rng.integers(0, p, size=(3, length), dtype=np.uint8)
        b = rng.integers(0, p, size=(3, length), dtype=np.uint8)
        out = host(fqt.polymul_dfqt(p, d, dev(a), dev(b), centered=1))
        assert np.array_equal(out, want_rows(a, b, p)), length


@pytest.mark.parametrize("p,d", [(3, 4), (3, 3), (5, 2), (7, 1)])
@pytest.mark.parametrize("boundary", [1, 2])
def test_dfqt_centred_extremes(p, d, boundary):
    # every coefficient h against h (+h^2 per term) and against -h (-h^2): the
    # block digits reach both ends of [-q/2, q/2) at the centred n_q
    q = 2 ** (52 // (2 * d + 1))
    h = (p - 1) // 2
    length = 501
    chunks = -(-length // (d + 1))
    several = chunks > gf.centred_nq_max(p, d + 1, q)  # blocks per longest S_t above one
    for bv in (h, p - h):
        note(f"dfqt centred extremes p={p} d={d} boundary={boundary} b={bv}")
        a = np.full((2, length), h, dtype=np.uint8)
        b = np.full((2, length), bv, dtype=np.uint8)
        case = lambda: fqt.polymul_dfqt(p, d, dev(a), dev(b), boundary=boundary, centered=1)
        if boundary == 2 and q > 2 ** 12 and several:
            refused("FQT_ERR_UNSUPPORTED", case)
        else:
            assert np.array_equal(host(case()), want_rows(a, b, p)), bv


def test_dfqt_centred_workload_sampled():
    from paper_0710_0510_amd import workloads as W
    w = W.WORKLOADS["dfqt-gf3-n500-d4"]
    a_h, b_h = W.poly_long_inputs(w)
    a, b = dev(a_h), dev(b_h)
    note("dfqt centred workload")
    plain = fqt.polymul_dfqt(w.p, w.d, a, b)
    cen = fqt.polymul_dfqt(w.p, w.d, a, b, centered=1)
    torch.cuda.synchronize()
    assert torch.equal(plain, cen)
    rng = np.random.default_rng(5)
    out = host(cen)
    for i in rng.integers(0, w.count, size=8).tolist():
        assert out[i].tolist() == gf.polymul_long(a_h[i].tolist(), b_h[i].tolist(), w.p)
