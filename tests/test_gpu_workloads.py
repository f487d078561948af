"""The benchmark's full-size workloads, run the way the benchmark times them
(each path autotuned, then called with the tuned q / n_q / tile), checked
against the oracle on every output byte by Freivalds' test (C x = A (B x)
for 20 random vectors x over the field: a wrong C survives one vector with
probability at most 1/p^k), plus exact samples: whole columns of C through
the oracle's plane products and single entries through its one-entry dot
product.  Batched: Freivalds on every product, whole sampled products and
single entries of others.
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


@pytest.mark.parametrize("name", ["gemm-gf7^2-1024", "gemm-gf5^3-4096", "gemm-gf3^2-8192"])
@pytest.mark.parametrize("path", ["packed", "int8"])
def test_workload_gemm_sampled(name, path):
    w = W.WORKLOADS[name]
    A_h, B_h = W.gemm_inputs(w)
    f = fqt.Field(w.p, w.k, w.P_low)
    A = torch.from_numpy(A_h).cuda()
    B = torch.from_numpy(B_h).cuda()
    C = torch.empty((w.M, w.N, w.k), dtype=torch.uint8, device="cuda")
    note(f"workload {name} path={path}: autotune")
    tuned = fqt.autotune(f, fqt.make_descs(f, [A], [B], [C]), only=path)
    note(f"workload {name} path={path}: run {tuned}")
    C.fill_(255)
    fqt.gemm(f, A, B, C, path=path)
    Ch = C.cpu().numpy()
    rng = np.random.default_rng(2024)
    note(f"workload {name} path={path}: Freivalds, 20 vectors")
    assert gf.freivalds(A_h, B_h, Ch, w.p, w.P_low, rng)
    cols = sorted({0, w.N - 1} | set(rng.integers(0, w.N, size=2).tolist()))
    note(f"workload {name} path={path}: oracle columns {cols}")
    assert np.array_equal(Ch[:, cols], gf.gemm_gfpk_planes(A_h, B_h[:, cols], w.p, w.P_low))
    entries = [(0, 0), (w.M - 1, w.N - 1), (w.M - 1, 0), (0, w.N - 1)]
    entries += [tuple(x) for x in rng.integers(0, [w.M, w.N], size=(28, 2)).tolist()]
    note(f"workload {name} path={path}: {len(entries)} oracle entries")
    for i, j in entries:
        assert gf.gemm_entry(A_h[i], B_h[:, j], w.p, w.P_low) == Ch[i, j].tolist(), (i, j)


def _pack(arrays, align=256):
    """One device buffer holding every array at 256-byte aligned offsets."""
    offs, total = [], 0
    for a in arrays:
        offs.append(total)
        total += (a.nbytes + align - 1) // align * align
    buf = np.zeros(max(total, 1), dtype=np.uint8)
    for a, o in zip(arrays, offs):
        buf[o:o + a.nbytes] = a.reshape(-1)
    return torch.from_numpy(buf).cuda(), offs


@pytest.mark.parametrize("path", ["packed", "int8"])
def test_workload_batched_sampled(path):
    w = W.WORKLOADS["batched-gf3^4-4096"]
    mnk, As, Bs = W.batched_inputs(w)
    f = fqt.Field(w.p, w.k, w.P_low)
    k = w.k
    dA, offA = _pack(As)
    dB, offB = _pack(Bs)
    dC, offC = _pack([np.zeros((M, N, k), dtype=np.uint8) for (M, N, K) in mnk.tolist()])
    descs = (fqt.GemmDesc * len(As))()
    for i, (M, N, K) in enumerate(mnk.tolist()):
        descs[i] = fqt.GemmDesc(M, N, K, K, N, N, dA.data_ptr() + offA[i],
                                dB.data_ptr() + offB[i], dC.data_ptr() + offC[i])
    note(f"workload batched path={path}: autotune")
    tuned = fqt.autotune(f, descs, only=path)
    rng = np.random.default_rng(77)
    whole = rng.choice(len(As), size=24, replace=False).tolist()
    whole += np.argsort(-mnk[:, 2])[:2].tolist()          # the longest K
    singles = rng.integers(0, len(As), size=200).tolist()
    for rep in range(2):                                   # graph capture, then replay
        note(f"workload batched path={path} {tuned} replay {rep}")
        dC.fill_(255)
        fqt.gemm_batched(f, descs, path=path)
        Ch = dC.cpu().numpy()
        if rep == 0:
            note(f"workload batched path={path}: Freivalds on all {len(As)} products")
            for g in range(len(As)):
                M, N, K = mnk[g].tolist()
                got = Ch[offC[g]:offC[g] + M * N * k].reshape(M, N, k)
                assert gf.freivalds(As[g], Bs[g], got, w.p, w.P_low, rng), g
        for g in whole:
            M, N, K = mnk[g].tolist()
            got = Ch[offC[g]:offC[g] + M * N * k].reshape(M, N, k)
            assert np.array_equal(got, gf.gemm_gfpk_planes(As[g], Bs[g], w.p, w.P_low)), g
        for g in singles:
            M, N, K = mnk[g].tolist()
            got = Ch[offC[g]:offC[g] + M * N * k].reshape(M, N, k)
            i, j = int(rng.integers(0, M)), int(rng.integers(0, N))
            assert gf.gemm_entry(As[g][i], Bs[g][:, j], w.p, w.P_low) == got[i, j].tolist(), g
