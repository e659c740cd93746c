"""GPU tests of the served form: requests of several multi-frame streams run
concurrently (several workers, scratch carved from a shared arena), with or
without merging the temporal requests of different streams into shared
launches, must give each stream exactly the records and decoded frames a
standalone plan gives for the same calls, and those records must equal the
oracle's.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2411_00761_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = [3000, 20000, 777, 50000, 12345, 100000]
FRAMES = 6
BATCH = 4


@pytest.fixture(scope="module")
def lcp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_00761_amd import lcp as L
    L.lib()
    return L


def stream_frames(j, n, jump=False):
    traj = datagen.MDTrajectory(n, seed=60 + j, step=0.002 * (1 + j % 3))
    xs = [traj.next_frame() for _ in range(FRAMES)]
    if jump:
        # the last frame loses its temporal correlation: same extent, positions
        # redrawn, so its LCP-T record is far larger than the last LCP-S one
        rng = np.random.default_rng(900 + j)
        x = xs[-1]
        lo, hi = x.min(axis=1, keepdims=True), x.max(axis=1, keepdims=True)
        xs[-1] = (lo + (hi - lo) * rng.random(x.shape)).astype(np.float32)
    return xs


def eb_of(j):
    return 1e-3 if j % 2 == 0 else 1e-4


def standalone(lcp, j, xs, k):
    n = xs[0].shape[1]
    plan = lcp.Plan(eb_of(j), lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=BATCH, block_log2=k,
                    max_particles=n)
    dplan = lcp.Plan(eb_of(j), lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=BATCH, block_log2=k,
                     max_particles=n)
    recs, decs = [], []
    for x in xs:
        out, offs, _, _ = plan.compress([torch.from_numpy(x).cuda()])
        recs.append(out[:offs[1]].cpu().numpy().tobytes())
        decs.append(dplan.decompress(out, offs)[0].cpu().numpy())
    return recs, decs


def serve(lcp, streams, workers, arena, batch_frames=0, batch_particles=0, counts=None):
    srv = lcp.Server(arena, workers=workers, batch_frames=batch_frames,
                     batch_particles=batch_particles)
    ids, outs, decs, tickets = [], [], [], []
    for j, xs in enumerate(streams):
        n = xs[0].shape[1]
        k = 4 if j % 3 else -1
        sid = srv.open_stream(eb_of(j), lcp.EB_REL_GLOBAL, batch_size=BATCH, block_log2=k,
                              max_particles=n, sample=torch.from_numpy(xs[0]).cuda() if k < 0 else None)
        ids.append(sid)
        cap = 40 * n + 4096  # above the record bound for three fields
        outs.append([torch.zeros(cap, dtype=torch.uint8, device="cuda") for _ in xs])
        decs.append([torch.empty((3, n), dtype=torch.float32, device="cuda") for _ in xs])
    frames = [[torch.from_numpy(x).cuda() for x in xs] for xs in streams]
    # interleave: frame t of every stream, compress then decompress
    sizes = [[None] * FRAMES for _ in streams]
    for t in range(FRAMES):
        # each burst is queued whole before the workers look at it, so that
        # merging (when enabled) sees every stream's request
        srv.hold(True)
        ct = [srv.compress(ids[j], frames[j][t], outs[j][t]) for j in range(len(streams))]
        srv.hold(False)
        for j, tk in enumerate(ct):
            r = srv.wait(tk)
            assert r["status"] == 0, (j, t, r)
            sizes[j][t] = r["bytes"]
        srv.hold(True)
        tickets += [(j, t, srv.decompress(ids[j], outs[j][t], 0, sizes[j][t], decs[j][t]))
                    for j in range(len(streams))]
        srv.hold(False)
    for j, t, tk in tickets:
        r = srv.wait(tk)
        assert r["status"] == 0 and r["bytes"] == streams[j][0].shape[1], (j, t, r)
    torch.cuda.synchronize()
    recs = [[outs[j][t][:sizes[j][t]].cpu().numpy().tobytes() for t in range(FRAMES)]
            for j in range(len(streams))]
    dec = [[decs[j][t].cpu().numpy() for t in range(FRAMES)] for j in range(len(streams))]
    if counts is not None:
        counts.update(srv.counts())
    srv.close()
    return recs, dec, ids


def check(lcp, workers, arena_of, jump=(), **batch):
    streams = [stream_frames(j, n, j in jump) for j, n in enumerate(SIZES)]
    arena = arena_of(lcp)
    counts = {}
    recs, dec, _ = serve(lcp, streams, workers, arena, counts=counts, **batch)
    for j, xs in enumerate(streams):
        print(f"stream {j} n={SIZES[j]}", flush=True)
        k = 4 if j % 3 else O.search_k(xs[0], O.EB_REL_GLOBAL, eb_of(j))[0]
        wrecs, wdecs = standalone(lcp, j, xs, k)
        for t in range(FRAMES):
            assert recs[j][t] == wrecs[t], (j, t)
            assert np.array_equal(dec[j][t].view(np.uint32), wdecs[t].view(np.uint32)), (j, t)
    # the records are the oracle's too (two streams)
    for j in (1, 2):
        ost = O.Stream(O.EB_REL_GLOBAL, eb_of(j), batch_size=BATCH, block_log2=4, max_n=SIZES[j])
        for t, x in enumerate(streams[j]):
            want, _, _ = ost.compress(x)
            assert recs[j][t] == want, (j, t)
    return counts


def test_served_mix_equals_standalone(lcp):
    check(lcp, 4, lambda L: 4 * max(L.scratch_bytes(max_particles=n) for n in SIZES))


def test_served_arena_for_one_request(lcp):
    # room for exactly one of the largest requests: admission serialises them
    check(lcp, 4, lambda L: max(L.scratch_bytes(max_particles=n) for n in SIZES))


def test_served_budget_refuses_stream(lcp):
    arena = lcp.scratch_bytes(max_particles=1000)
    srv = lcp.Server(arena, workers=1, hbm_budget_bytes=arena + 1000)
    with pytest.raises(lcp.LCPError):
        srv.open_stream(1e-3, lcp.EB_ABS, block_log2=4, max_particles=1000)
    srv.close()


def test_served_batched_equals_standalone(lcp):
    """Temporal requests of the six streams share launches; every record and
    decoded frame is still the stream's own, and the oracle's."""
    c = check(lcp, 4, lambda L: 4 * max(L.scratch_bytes(max_particles=n) for n in SIZES),
              batch_frames=8, batch_particles=sum(SIZES))
    print(c, flush=True)
    assert c["merged_requests"] > 0 and c["merged_launches"] < c["merged_requests"], c


def test_served_batched_capacity_split_and_requeue(lcp):
    """Two frames or 60,000 particles per launch set split the groups; a frame
    that loses its temporal correlation is put back and coded alone, as its own
    call would code it."""
    c = check(lcp, 2, lambda L: 2 * max(L.scratch_bytes(max_particles=n) for n in SIZES),
              jump=(1, 4), batch_frames=2, batch_particles=60000)
    print(c, flush=True)
    assert c["merged_requests"] > 0 and c["requeued"] > 0, c


def test_served_batched_forced_t_capacity(lcp):
    """A forced LCP-T request whose record does not fit its buffer is put back
    and fails alone with the status and size its own call gives; both streams
    then go on exactly like standalone plans given the same calls."""
    n = 20000
    xs = stream_frames(3, n)
    srv = lcp.Server(4 * lcp.scratch_bytes(max_particles=n), workers=2, batch_frames=4,
                     batch_particles=4 * n)
    kw = dict(batch_size=BATCH, block_log2=4, max_particles=n)
    plans = [lcp.Plan(1e-3, lcp.EB_REL_GLOBAL, multi_frame=True, **kw) for _ in range(2)]
    sids = [srv.open_stream(1e-3, lcp.EB_REL_GLOBAL, **kw) for _ in range(2)]
    big = 40 * n + 4096
    frames = [torch.from_numpy(x).cuda() for x in xs]
    for t in range(5):
        method = lcp.METHOD_AUTO if t == 0 else lcp.METHOD_T
        caps = [big, 64 if t == 2 else big]
        outs = [torch.zeros(c, dtype=torch.uint8, device="cuda") for c in caps]
        srv.hold(True)
        tks = [srv.compress(sid, frames[t], outs[i], method=method) for i, sid in enumerate(sids)]
        srv.hold(False)
        res = [srv.wait(tk) for tk in tks]
        for i in range(2):
            wout = torch.zeros(caps[i], dtype=torch.uint8, device="cuda")
            try:
                _, woffs, _, _ = plans[i].compress([frames[t]], methods=[method], out=wout)
                want = (0, woffs[1])
            except lcp.LCPError as e:
                want = (lcp.ERR_CAPACITY, None)
                assert "needs" in str(e)
            torch.cuda.synchronize()
            assert res[i]["status"] == want[0], (t, i, res[i])
            if want[0] == 0:
                assert res[i]["bytes"] == want[1]
                assert outs[i][:want[1]].cpu().numpy().tobytes() == \
                    wout[:want[1]].cpu().numpy().tobytes(), (t, i)
    c = srv.counts()
    print(c, flush=True)
    assert c["merged_requests"] > 0 and c["requeued"] > 0, c
    srv.close()
