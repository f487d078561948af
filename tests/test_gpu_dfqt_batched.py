"""Parity of the d-FQT over batches of uneven polynomial pairs (Section 6,
one persistent launch replayed from a captured graph) with the oracle's
product definition, through the C ABI.  Bit-exact, every product.

Both operand lengths of every pair are drawn independently, uniform in
1..1024 (and up to the 1024 (d+1) maximum); pairs with an empty operand sit
in between and write nothing; the cases cover single-block and several-block
modes (both block-boundary modes, explicit n_q), centred chunks, graph
replays of one plan beside a second plan, the autotuner, and the host's
refusals.
"""
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


def refused(status, fn):
    """The host refuses the call with `status` before any launch."""
    with pytest.raises(fqt.FqtError) as ei:
        fn()
    assert ei.value.name == status, str(ei.value)


class Batch:
    """An uneven batch in three flat device buffers, with the oracle's
    products of every pair."""

    def __init__(self, p, lens, seed):
        rng = np.random.default_rng(seed)
        self.p = p
        self.lens = np.asarray(lens, dtype=np.int64).reshape(-1, 2)
        la, lb = self.lens[:, 0], self.lens[:, 1]
        self.a_h = rng.integers(0, p, size=int(la.sum()), dtype=np.uint8)
        self.b_h = rng.integers(0, p, size=int(lb.sum()), dtype=np.uint8)
        self.lc = np.where((la > 0) & (lb > 0), la + lb - 1, 0)
        self.a = torch.from_numpy(self.a_h).cuda()
        self.b = torch.from_numpy(self.b_h).cuda()
        # one spare byte past the end: a write beyond the last product shows
        self.c = torch.full((int(self.lc.sum()) + 1,), 0xEE, dtype=torch.uint8, device="cuda")
        self.descs = fqt.poly_descs_flat(self.a, self.b, self.c, self.lens)
        self.oa = np.concatenate(([0], np.cumsum(la)))
        self.ob = np.concatenate(([0], np.cumsum(lb)))
        self.oc = np.concatenate(([0], np.cumsum(self.lc)))
        self.want = [np.asarray(gf.polymul_long(self.a_h[self.oa[i]:self.oa[i + 1]].tolist(),
                                                self.b_h[self.ob[i]:self.ob[i + 1]].tolist(), p),
                                dtype=np.uint8)
                     for i in range(len(self.lens))]

    def check(self, what):
        torch.cuda.synchronize()
        c = self.c.cpu().numpy()
        assert c[-1] == 0xEE, (what, "write past the last product")
        for i, w in enumerate(self.want):
            got = c[self.oc[i]:self.oc[i + 1]]
            assert np.array_equal(got, w), (what, i, tuple(self.lens[i]))

    def clear(self):
        self.c.fill_(0xEE)


def uneven_lengths(seed, count, hi=1024, zeros=True):
    lens = W.poly_uneven_lengths(seed, count, 1, hi)
    if zeros:  # a few empty operands among the others
        lens[3] = (0, 17)
        lens[7] = (40, 0)
        lens[11] = (0, 0)
    lens[0] = (1, 1)
    lens[1] = (1, hi)
    lens[2] = (hi, 1)
    return lens


@pytest.mark.parametrize("p,d,centered", [(3, 4, 0), (3, 4, 1), (3, 1, 0), (3, 2, 1), (2, 5, 0),
                                          (5, 3, 1), (7, 1, 0), (13, 1, 1), (127, 0, 0)])
def test_dfqt_batched_uneven_every_product(p, d, centered):
    bt = Batch(p, uneven_lengths(100 * p + 10 * d + centered, 300), seed=p + d)
    note(f"dfqt batched p={p} d={d} centered={centered} pairs=300")
    fqt.polymul_dfqt_batched(p, d, bt.descs, centered=centered)
    bt.check((p, d, centered))


@pytest.mark.parametrize("p,d", [(3, 2), (7, 1), (2, 5)])
def test_dfqt_batched_largest_lengths(p, d):
    # 1024 (d + 1) coefficients per operand: 1024 chunks, the LDS maximum
    m = 1024 * (d + 1)
    lens = [(m, m), (m, 1), (1, m), (m - 1, m - d), (m, 513), (3, 5)]
    bt = Batch(p, lens, seed=m)
    note(f"dfqt batched largest p={p} d={d} len={m}")
    fqt.polymul_dfqt_batched(p, d, bt.descs)
    bt.check((p, d))


@pytest.mark.parametrize("p,d,nq", [(3, 2, 1), (3, 2, 2), (3, 2, 7), (7, 1, 5), (5, 3, 3),
                                    (3, 4, 1)])
@pytest.mark.parametrize("boundary", [1, 2])
def test_dfqt_batched_block_modes(p, d, nq, boundary):
    q, nqmax = gf.max_pow2_q(p, d + 1)
    bt = Batch(p, uneven_lengths(nq * 10 + boundary, 60, hi=700), seed=nq)
    if nq > nqmax:
        refused("FQT_ERR_BOUNDS",
                lambda: fqt.polymul_dfqt_batched(p, d, bt.descs, n_q=nq, boundary=boundary))
        return
    if boundary == 2 and q > 2 ** 12:  # digit-sum fields hold digits of q <= 2^12 only
        refused("FQT_ERR_UNSUPPORTED",
                lambda: fqt.polymul_dfqt_batched(p, d, bt.descs, n_q=nq, boundary=2))
        return
    note(f"dfqt batched blocks p={p} d={d} n_q={nq} boundary={boundary}")
    fqt.polymul_dfqt_batched(p, d, bt.descs, n_q=nq, boundary=boundary)
    bt.check((p, d, nq, boundary))


def test_dfqt_batched_adversarial_all_top_coefficients():
    # every coefficient p - 1: every block at its bound (centred: -h)
    for p, d, cen in ((3, 4, 0), (3, 4, 1), (7, 1, 0), (127, 0, 0)):
        m = 1024 * (d + 1)
        lens = np.array([(m, m), (m // 2 + 1, m), (m, 7)], dtype=np.int64)
        bt = Batch(p, lens, seed=0)
        bt.a_h[:] = p - 1
        bt.b_h[:] = p - 1
        bt.a.copy_(torch.from_numpy(bt.a_h))
        bt.b.copy_(torch.from_numpy(bt.b_h))
        bt.want = [np.asarray(gf.polymul_long([p - 1] * int(x), [p - 1] * int(y), p),
                              dtype=np.uint8) for x, y in lens.tolist()]
        note(f"dfqt batched adversarial p={p} d={d} centered={cen}")
        fqt.polymul_dfqt_batched(p, d, bt.descs, centered=cen)
        bt.check((p, d, cen))


def test_dfqt_batched_replays_and_two_plans():
    one = Batch(3, uneven_lengths(5, 500), seed=5)
    two = Batch(3, uneven_lengths(6, 123, hi=300), seed=6)
    for rep in range(3):
        for bt, name in ((one, "one"), (two, "two")):
            note(f"dfqt batched replay {rep} plan {name}")
            bt.clear()
            fqt.polymul_dfqt_batched(3, 4, bt.descs)
            bt.check((rep, name))
    # same descriptors, other chunk length: a plan of its own
    note("dfqt batched replay d=2")
    one.clear()
    fqt.polymul_dfqt_batched(3, 2, one.descs, centered=1)
    one.check("d=2 centred")


def test_dfqt_batched_full_workload_sampled():
    # the benchmark's batch: 16384 pairs, lengths uniform in 1..1024, d = 4;
    # sampled pairs against the oracle, and every byte against the padded
    # equal-length d-FQT of the same pairs
    w = W.WORKLOADS["dfqt-uneven-gf3-1024"]
    lens, a_h, b_h = W.poly_uneven_inputs(w)
    a, b = torch.from_numpy(a_h).cuda(), torch.from_numpy(b_h).cuda()
    la, lb = lens[:, 0], lens[:, 1]
    lc = la + lb - 1
    c = torch.full((int(lc.sum()),), 0xEE, dtype=torch.uint8, device="cuda")
    descs = fqt.poly_descs_flat(a, b, c, lens)
    note("dfqt batched full workload")
    fqt.polymul_dfqt_batched(w.p, w.d, descs)
    torch.cuda.synchronize()
    c_h = c.cpu().numpy()
    oa = np.concatenate(([0], np.cumsum(la)))
    ob = np.concatenate(([0], np.cumsum(lb)))
    oc = np.concatenate(([0], np.cumsum(lc)))
    rng = np.random.default_rng(11)
    picks = set(rng.integers(0, w.count, size=200).tolist()) | {int(np.argmax(la * lb)),
                                                                int(np.argmin(la * lb))}
    for i in sorted(picks):
        want = gf.polymul_long(a_h[oa[i]:oa[i + 1]].tolist(), b_h[ob[i]:ob[i + 1]].tolist(), w.p)
        assert c_h[oc[i]:oc[i + 1]].tolist() == want, i
    # padded to 1024 coefficients: the same products followed by zeros
    hi = w.hi
    A = np.zeros((w.count, hi), np.uint8)
    B = np.zeros((w.count, hi), np.uint8)
    for i in range(w.count):
        A[i, :la[i]] = a_h[oa[i]:oa[i + 1]]
        B[i, :lb[i]] = b_h[ob[i]:ob[i + 1]]
    ref = fqt.polymul_dfqt(w.p, w.d, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
    ref_h = ref.cpu().numpy()
    for i in range(w.count):
        assert np.array_equal(c_h[oc[i]:oc[i + 1]], ref_h[i, :lc[i]]), i
        assert not ref_h[i, lc[i]:].any(), i


def test_dfqt_batched_autotune():
    bt = Batch(3, uneven_lengths(9, 400), seed=9)
    note("dfqt batched autotune")
    best = fqt.autotune_polymul(3, bt.descs)
    assert 0 <= best["d"] <= 7 and best["centered"] in (0, 1) and best["boundary"] in (1, 2)
    bt.clear()
    fqt.polymul_dfqt_batched(3, best["d"], bt.descs, centered=best["centered"],
                             boundary=best["boundary"])
    bt.check(best)


def test_dfqt_batched_refusals():
    note("dfqt batched refusals")
    bt = Batch(3, [(2049, 5)], seed=1)  # 2049 coefficients are 1025 chunks at d = 1
    refused("FQT_ERR_UNSUPPORTED", lambda: fqt.polymul_dfqt_batched(3, 1, bt.descs))
    refused("FQT_ERR_UNSUPPORTED", lambda: fqt.polymul_dfqt_batched(3, 8, bt.descs))
    refused("FQT_ERR_NOT_PRIME", lambda: fqt.polymul_dfqt_batched(9, 2, bt.descs))
    refused("FQT_ERR_UNSUPPORTED", lambda: fqt.polymul_dfqt_batched(2, 2, bt.descs, centered=1))
