"""GPU checks at the workloads' full sizes and on damaged records.

* A full 4,194,304-particle frame of the MD trajectory: byte parity with the
  oracle (which finishes it in seconds).
* The 134,217,728-particle, six-field cosmology snapshot: properties that hold at
  any size -- every value within its field's bound, the slot order is a
  permutation that sorts particles by block id stably (checked on samples), and
  sampled particles' decoded values equal the oracle's Eq. 5 reconstruction of
  the same input computed one by one.
* Damaged records are rejected with LCP_ERR_CORRUPT (or decode to some values)
  and never fault: every read the decoder makes is bounds-checked.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2411_00761_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lcp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_00761_amd import lcp as L
    L.lib()
    return L


def test_md_frame_full_size_parity(lcp):
    traj = datagen.MDTrajectory(1 << 22, dims=(256, 128, 128), seed=2)
    x = traj.next_frame()
    xd = torch.from_numpy(x).cuda()
    plan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, block_log2=-1, max_particles=1 << 22, sample=xd)
    k = plan.block_log2
    out, offs, _, perms = plan.compress([xd], want_perm=True)
    rec = out[offs[0]:offs[1]].cpu().numpy().tobytes()
    grids = O.grids_for(x, O.EB_REL_GLOBAL, 1e-4)
    want, wperm, _ = O.compress_s(x, grids, k, 10, 0)
    assert rec == want
    assert np.array_equal(perms[0].cpu().numpy().astype(np.uint32), wperm)
    dec = plan.decompress(out, offs)[0]
    wdec, _ = O.decompress(want)
    for f in range(3):
        assert np.array_equal(dec[f].cpu().numpy().view(np.uint32), wdec[f].view(np.uint32))


def test_cosmology_snapshot_full_size_properties(lcp):
    n = 1 << 27
    x = datagen.cosmology_snapshot(n, seed=3)
    xd = torch.from_numpy(x).cuda()
    del x
    plan = lcp.Plan(1e-4, lcp.EB_REL_PER_FIELD, n_fields=6, block_log2=3, max_particles=n)
    out, offs, _, perms = plan.compress([xd], want_perm=True)
    size = offs[1]
    dec = plan.decompress(out, offs)[0]
    perm = perms[0].long()
    lo = xd.amin(dim=1).double()
    hi = xd.amax(dim=1).double()
    eb = (1e-4 * (hi - lo)).cpu().numpy()
    for f in range(6):
        err = (dec[f].double() - xd[f][perm].double()).abs().max().item()
        assert err <= eb[f], (f, err, eb[f])
    # perm is a permutation
    seen = torch.zeros(n, dtype=torch.int32, device="cuda")
    seen.index_add_(0, perm, torch.ones(n, dtype=torch.int32, device="cuda"))
    assert int(seen.min()) == 1 and int(seen.max()) == 1
    # sampled particles: the oracle's one-by-one Eq. 5 reconstruction matches
    rng = np.random.default_rng(7)
    idx = rng.integers(0, n, size=4096)
    xs = xd[:, perm[torch.from_numpy(idx).cuda()]].cpu().numpy()
    ds = dec[:, torch.from_numpy(idx).cuda()].cpu().numpy()
    lo_c, hi_c = lo.cpu().numpy().astype(np.float32), hi.cpu().numpy().astype(np.float32)
    for f in range(6):
        g = O.make_grid(lo_c[f], hi_c[f], float(eb[f]))
        want = O.reconstruct(O.quantize(xs[f], g), g)
        assert np.array_equal(want.view(np.uint32), ds[f].view(np.uint32)), f
    # block order is stable: within sampled consecutive slot pairs of one block the
    # input indices increase, and block keys never decrease
    q = [O.quantize(xd[d][perm[:1 << 20]].cpu().numpy(), O.make_grid(lo_c[d], hi_c[d], float(eb[d])))
         for d in range(3)]
    qmax = [int(O.quantize(np.array([hi_c[d]], np.float32), O.make_grid(lo_c[d], hi_c[d], float(eb[d])))[0])
            for d in range(3)]
    bn = [(qm >> 3) + 1 for qm in qmax]
    key = (q[0] >> 3) + bn[0] * ((q[1] >> 3) + bn[1] * (q[2] >> 3))
    assert np.all(np.diff(key) >= 0)
    p = perm[:1 << 20].cpu().numpy()
    same = np.diff(key) == 0
    assert np.all(np.diff(p)[same] > 0)
    print(f"cosmology snapshot: {n} particles x 6 fields, {size} bytes, CR {n * 24 / size:.3f}")


@pytest.mark.parametrize("seed", range(6))
def test_corrupted_records_fail_cleanly(lcp, seed):
    n = 50000
    traj = datagen.MDTrajectory(n, seed=51, step=0.002)
    xs = [torch.from_numpy(traj.next_frame()).cuda() for _ in range(3)]
    plan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=0, block_log2=5,
                    max_particles=n)
    out, offs, used, _ = plan.compress(xs)
    host = out[: offs[-1]].cpu().numpy().copy()
    rng = np.random.default_rng(seed)
    for trial in range(8):
        bad = host.copy()
        j = int(rng.integers(0, 3))
        lo, hi = offs[j], offs[j + 1]
        for _ in range(int(rng.integers(1, 6))):
            bad[int(rng.integers(lo + (80 if seed % 2 else 0), hi))] ^= np.uint8(rng.integers(1, 256))
        buf = torch.from_numpy(bad).cuda()
        dplan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=0, block_log2=5,
                         max_particles=n)
        try:
            dplan.decompress(buf, offs)
        except lcp.LCPError as e:
            assert e.status in (lcp.ERR_CORRUPT, lcp.ERR_NO_REFERENCE, lcp.ERR_ARG), e
    # a truncated record
    dplan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=0, block_log2=5,
                     max_particles=n)
    with pytest.raises(lcp.LCPError):
        dplan.decompress(out, [0, offs[1] - 8])
    torch.cuda.synchronize()
