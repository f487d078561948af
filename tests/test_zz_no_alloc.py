"""The allocation-free d-FQT batch (fqt_polymul_dfqt_batched_noalloc)
against the planned one (fqt_polymul_dfqt_batched), through the C ABI.
Bit-exact.

Two calls in a row on the same static per-GPU scratch array, the first at
the largest batch it takes (16384 pairs), the second smaller: the second must
not see the first's descriptors.  Then the refusal beyond the
maximum, before any device work.
"""
import sys

import numpy as np
import pytest

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


def batch(p, lens, seed):
    rng = np.random.default_rng(seed)
    la, lb = lens[:, 0], lens[:, 1]
    lc = np.where((la > 0) & (lb > 0), la + lb - 1, 0)
    a = torch.from_numpy(rng.integers(0, p, size=int(la.sum()), dtype=np.uint8)).cuda()
    b = torch.from_numpy(rng.integers(0, p, size=int(lb.sum()), dtype=np.uint8)).cuda()
    c_ref = torch.full((int(lc.sum()) + 1,), 0xEE, dtype=torch.uint8, device="cuda")
    c_new = torch.full((int(lc.sum()) + 1,), 0x11, dtype=torch.uint8, device="cuda")
    return (a, b, fqt.poly_descs_flat(a, b, c_ref, lens), c_ref,
            fqt.poly_descs_flat(a, b, c_new, lens), c_new)


@pytest.mark.parametrize("p,d,centered", [(3, 4, 0), (3, 4, 1), (7, 1, 0), (2, 5, 0)])
def test_noalloc_matches_planned_batch_two_calls(p, d, centered):
    big = W.poly_uneven_lengths(21 + p + d, 16384, 1, 1024)
    big[5] = (0, 9)  # an empty pair: no output, and not scheduled
    small = W.poly_uneven_lengths(22 + p + d, 700, 1, 300)
    for name, lens in (("first, 16384 pairs", big), ("second, 700 pairs", small)):
        note(f"noalloc p={p} d={d} centered={centered} {name}")
        a, b, d_ref, c_ref, d_new, c_new = batch(p, lens, seed=len(lens) + p)
        fqt.polymul_dfqt_batched(p, d, d_ref, centered=centered)
        fqt.polymul_dfqt_batched_noalloc(p, d, d_new, centered=centered)
        torch.cuda.synchronize()
        assert torch.equal(c_ref[:-1], c_new[:-1]), name
        assert int(c_ref[-1]) == 0xEE and int(c_new[-1]) == 0x11, name


def test_noalloc_refuses_beyond_its_maximum():
    note("noalloc refusal")
    lens = np.ones((16385, 2), dtype=np.int64)
    a = torch.zeros(16385, dtype=torch.uint8, device="cuda")
    b = torch.zeros(16385, dtype=torch.uint8, device="cuda")
    c = torch.zeros(16385, dtype=torch.uint8, device="cuda")
    descs = fqt.poly_descs_flat(a, b, c, lens)
    with pytest.raises(fqt.FqtError) as ei:
        fqt.polymul_dfqt_batched_noalloc(3, 4, descs)
    assert ei.value.name == "FQT_ERR_UNSUPPORTED", str(ei.value)
