"""GPU parity of data with fewer spatial dimensions (Sec. 4; Eq. 6 over D axes).

Records, slot permutations and decoded values must equal the oracle's, byte for
byte and bit for bit: single frames of D = 1 and 2 with and without
supplementary fields (ragged sizes, several block sizes), a batch of
independent 2-D frames in one call, multi-frame 2-D and 1-D streams (temporal
runs of one- and two-field frames) one call and frame by frame, and a 2-D frame
of 2^20 particles.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lcp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_00761_amd import lcp as L
    L.lib()
    return L


def bits_equal(a, b) -> bool:
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32),
                          np.asarray(b, np.float32).view(np.uint32))


def frame(F, n, seed, hi=100.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, hi, size=(F, n)).astype(np.float32)


@pytest.mark.parametrize("D,F,n,k", [(2, 2, 5001, 6), (2, 4, 4099, 4), (1, 1, 7003, 8),
                                     (1, 3, 3000, 10), (2, 2, 65537, 0)])
def test_single_frame_parity(lcp, D, F, n, k):
    x = frame(F, n, seed=D * 10 + F)
    eb = 1e-3
    plan = lcp.Plan(eb, lcp.EB_ABS, n_fields=F, block_log2=k, max_particles=n, n_dims=D)
    out, offs, _, perms = plan.compress([torch.from_numpy(x).cuda()], want_perm=True)
    got = out[:offs[1]].cpu().numpy().tobytes()
    want, perm, _ = O.compress_s(x, O.grids_for(x, O.EB_ABS, eb), k, dims=D)
    assert got == want, (len(got), len(want))
    assert got[52] == D
    assert np.array_equal(perms[0].cpu().numpy().astype(np.uint32), perm)
    dec = plan.decompress(out, offs)[0].cpu().numpy()
    wdec, _ = O.decompress(want)
    for f in range(F):
        assert bits_equal(dec[f], wdec[f]), f
        assert np.abs(dec[f].astype(np.float64) - x[f][perm].astype(np.float64)).max() <= eb


def test_batch_of_2d_frames(lcp):
    xs = [frame(3, n, seed=40 + j) for j, n in enumerate([3000, 777, 12345, 1, 4096])]
    plan = lcp.Plan(1e-3, lcp.EB_ABS, n_fields=3, block_log2=5, max_particles=12345,
                    n_dims=2, max_batch_frames=8)
    out, offs, _, _ = plan.compress([torch.from_numpy(x).cuda() for x in xs])
    buf = out[:offs[-1]].cpu().numpy().tobytes()
    for j, x in enumerate(xs):
        # a plan numbers its frames: frame j of a fresh plan's first call is seq j
        want, _, _ = O.compress_s(x, O.grids_for(x, O.EB_ABS, 1e-3), 5, seq=j, dims=2)
        assert buf[offs[j]:offs[j + 1]] == want, j
    dec = plan.decompress(out, offs)
    for j, rec in enumerate([buf[offs[j]:offs[j + 1]] for j in range(len(xs))]):
        w, _ = O.decompress(rec)
        for f in range(3):
            assert bits_equal(dec[j][f].cpu().numpy(), w[f]), (j, f)


@pytest.mark.parametrize("D,F,n", [(2, 2, 20000), (1, 2, 20003), (1, 1, 20000)])
@pytest.mark.parametrize("one_call", [True, False])
def test_stream_parity(lcp, D, F, n, one_call):
    rng = np.random.default_rng(D + 3 * F)
    x = rng.uniform(0.0, 50.0, size=(F, n)).astype(np.float32)
    xs = [x]
    for _ in range(11):
        xs.append((xs[-1] + rng.normal(0, 0.003, size=x.shape)).astype(np.float32))
    eb = 0.01
    ost = O.Stream(O.EB_ABS, eb, n_fields=F, batch_size=4, block_log2=4, max_n=n, n_dims=D)
    want = [ost.compress(f_) for f_ in xs]
    kw = dict(n_fields=F, multi_frame=True, batch_size=4, block_log2=4, max_particles=n, n_dims=D)
    plan = lcp.Plan(eb, lcp.EB_ABS, **kw)
    dev = [torch.from_numpy(f_).cuda() for f_ in xs]
    if one_call:
        out, offs, used, _ = plan.compress(dev)
        recs = [out[offs[t]:offs[t + 1]] for t in range(len(xs))]
    else:
        recs, used = [], []
        for f_ in dev:
            o, of, u, _ = plan.compress([f_])
            recs.append(o[:of[1]])
            used += u
    for t, (rec, wused, _) in enumerate(want):
        assert used[t] == wused, t
        assert recs[t].cpu().numpy().tobytes() == rec, t
    assert O.METHOD_T in used
    dplan = lcp.Plan(eb, lcp.EB_ABS, **kw)
    buf = torch.cat(recs)
    offs = np.concatenate([[0], np.cumsum([r.numel() for r in recs])]).tolist()
    dec = dplan.decompress(buf, offs)
    dst = O.Stream(O.EB_ABS, eb, n_fields=F, batch_size=4, block_log2=4, max_n=n, n_dims=D)
    for t, (rec, _, _) in enumerate(want):
        w = dst.decompress(rec)
        for f in range(F):
            assert bits_equal(dec[t][f].cpu().numpy(), w[f]), (t, f)


def test_2d_frame_2p20(lcp):
    n = 1 << 20
    x = frame(2, n, seed=77, hi=1000.0)
    plan = lcp.Plan(1e-3, lcp.EB_REL_GLOBAL, n_fields=2, block_log2=-1, max_particles=n, n_dims=2,
                    sample=torch.from_numpy(x).cuda())
    k = plan.block_log2
    assert k == O.search_k(x, O.EB_REL_GLOBAL, 1e-3, dims=2)[0]
    out, offs, _, _ = plan.compress([torch.from_numpy(x).cuda()])
    want, _, _ = O.compress_s(x, O.grids_for(x, O.EB_REL_GLOBAL, 1e-3), k, dims=2)
    assert out[:offs[1]].cpu().numpy().tobytes() == want
