"""GPU parity of multi-frame streams compressed in one lcp_compress call.

While LCP-FSM stays in its T state the library enqueues temporal frames in runs
and reads their outcomes back once per run; a frame whose outcome differs from
the prediction is coded again by the per-frame path.  Whatever the run does,
each record, method and slot permutation must be the oracle stream's, frame by
frame: across batch anchors (Alg. 1), where a jump sends a frame through the
spatial comparison part-way into a run (both when the temporal record still
wins and when the spatial one does), where a frame leaves the reference grid's
range, with forced methods, and with a buffer too small for the runs' bounds.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2411_00761_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 20000
EB = 1e-4


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


def trajectory(count, seed=5, step=0.002):
    tr = datagen.MDTrajectory(N, seed=seed, step=step)
    return [tr.next_frame() for _ in range(count)]


def eb_abs(xs):
    return EB * (float(xs[0].max()) - float(xs[0].min()))


def jump(x, sigma, seed):
    rng = np.random.default_rng(seed)
    return (x + rng.normal(0.0, sigma, size=x.shape)).astype(np.float32)


def oracle_stream(xs, batch, methods):
    ost = O.Stream(O.EB_REL_GLOBAL, EB, batch_size=batch, block_log2=4, max_n=N)
    out = []
    for t, x in enumerate(xs):
        out.append(ost.compress(x, method=methods[t] if methods else O.METHOD_AUTO))
    return out


def check_one_call(lcp, xs, batch, methods=None):
    want = oracle_stream(xs, batch, methods)
    plan = lcp.Plan(EB, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=batch, block_log2=4,
                    max_particles=N)
    out, offs, used, perms = plan.compress([torch.from_numpy(x).cuda() for x in xs],
                                           methods=methods, want_perm=True)
    buf = out[:offs[-1]].cpu().numpy().tobytes()
    for t, (rec, wused, wperm) in enumerate(want):
        print(f"frame {t}: method {wused}, {len(rec)} bytes", flush=True)
        assert used[t] == wused, (t, used[t], wused)
        assert buf[offs[t]:offs[t + 1]] == rec, f"frame {t}: {offs[t + 1] - offs[t]} vs {len(rec)} bytes"
        assert np.array_equal(perms[t].cpu().numpy().astype(np.uint32), wperm), t
    dplan = lcp.Plan(EB, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=batch, block_log2=4,
                     max_particles=N)
    dec = dplan.decompress(out, offs)
    ost = O.Stream(O.EB_REL_GLOBAL, EB, batch_size=batch, block_log2=4, max_n=N)
    for t, (rec, _, _) in enumerate(want):
        w = ost.decompress(rec)
        assert all(bits_equal(dec[t][f].cpu().numpy(), w[f]) for f in range(3)), t
    return used


@pytest.mark.parametrize("batch", [0, 8])
def test_stream_in_one_call(lcp, batch):
    """Long temporal runs; with batches of 8 the first frame of each batch is
    coded against the batch anchor inside a run."""
    used = check_one_call(lcp, trajectory(32), batch)
    assert used.count(lcp.METHOD_T) >= 24


def test_runs_broken_part_way(lcp):
    """Frame 6 jumps by 200 eb: its temporal record is larger than the last
    spatial one, so the run stops there and the frame is coded again, and the
    temporal record still wins, coded against the codes of frame 5, whose slot
    a later frame of the run had reused.  Frame 13 jumps by 400 eb (spatial
    wins, LCP-FSM leaves T); frame 22 leaves the reference grid's range."""
    xs = trajectory(32)
    e = eb_abs(xs)
    xs[6] = jump(xs[6], 200 * e, 61)
    xs[13] = jump(xs[13], 400 * e, 62)
    xs[22] = (xs[22] * np.float32(3.0)).astype(np.float32)
    used = check_one_call(lcp, xs, 0)
    assert used[6] == lcp.METHOD_T and used[13] == lcp.METHOD_S and used[22] == lcp.METHOD_S


def test_forced_methods_in_one_call(lcp):
    A, S, T = O.METHOD_AUTO, O.METHOD_S, O.METHOD_T
    methods = [S, T, T, T, A, A, T, S, A, A, A, T, T, A, A, A, S, T, T, T]
    check_one_call(lcp, trajectory(len(methods), seed=6), 4, methods)


def test_tight_buffer_stops_at_the_frame_that_does_not_fit(lcp):
    """The buffer holds ten records and part of the eleventh.  Runs only take
    frames whose worst-case records fit, so here every frame goes through the
    per-frame path: the call stops at frame 10 and reports the bytes it needs,
    and the ten records before it are in place."""
    xs = trajectory(16, seed=7)
    want = oracle_stream(xs, 0, None)
    sizes = [len(r) for r, _, _ in want]
    assert all(u == O.METHOD_T for _, u, _ in want[3:11])
    cap = sum(sizes[:10]) + sizes[10] - 4
    plan = lcp.Plan(EB, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=0, block_log2=4,
                    max_particles=N)
    out = torch.empty(cap, dtype=torch.uint8, device="cuda")
    with pytest.raises(lcp.LCPError) as ei:
        plan.compress([torch.from_numpy(x).cuda() for x in xs], out=out)
    assert ei.value.status == lcp.ERR_CAPACITY
    assert f"needs {sum(sizes[:11])} bytes" in str(ei.value)
    buf = out.cpu().numpy().tobytes()
    assert buf[:sum(sizes[:10])] == b"".join(r for r, _, _ in want[:10])


@pytest.mark.parametrize("n,batch", [(20003, 4), (4096 * 3 + 1, 0)])
def test_runs_ragged_size_and_segments(lcp, n, batch):
    """Runs on the residual kernel's one-slot-per-thread path (n not a multiple
    of four), split into segments where Alg. 1 turns to the anchor (batches of
    four) or one unbounded chain: records, methods and permutations against
    the oracle stream, and the stream decoded in one call."""
    tr = datagen.MDTrajectory(n, seed=17, step=0.002)
    xs = [tr.next_frame() for _ in range(30)]
    ost = O.Stream(O.EB_REL_GLOBAL, EB, batch_size=batch, block_log2=4, max_n=n)
    plan = lcp.Plan(EB, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=batch, block_log2=4,
                    max_particles=n)
    out, offs, used, perms = plan.compress([torch.from_numpy(x).cuda() for x in xs], want_perm=True)
    recs = []
    for t, x in enumerate(xs):
        want, wused, wperm = ost.compress(x)
        assert used[t] == wused, t
        assert out[offs[t]:offs[t + 1]].cpu().numpy().tobytes() == want, t
        assert np.array_equal(perms[t].cpu().numpy().astype(np.uint32), wperm), t
        recs.append(want)
    assert sum(1 for u in used if u == lcp.METHOD_T) >= 20
    dplan = lcp.Plan(EB, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=batch, block_log2=4,
                     max_particles=n)
    dec = dplan.decompress(out, offs)
    dst = O.Stream(O.EB_REL_GLOBAL, EB, batch_size=batch, block_log2=4, max_n=n)
    for t in range(len(xs)):
        w = dst.decompress(recs[t])
        assert all(bits_equal(dec[t][f].cpu().numpy(), w[f]) for f in range(3)), t
