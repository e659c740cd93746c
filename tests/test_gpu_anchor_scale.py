"""GPU parity of the anchor error-bound scale (Sec. 7.4.2).

Streams with anchor_scale = 5 must give the oracle stream's records, methods,
slot permutations and decoded values, byte for byte and bit for bit, whether
the frames go one per call or all in one call (temporal runs), including a
run that breaks inside a chain of frames scaled from an anchor (the library
then rebuilds the last committed frame's codes by following the chain from
the anchor), the correlation gate turning scaling off, the vector and scalar
paths (n divisible by 4 or not), and the served form with merged launches.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_2411_00761_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EB = 1e-4
S = 5


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


def break_stream(n, seed=41):
    """Smooth frames 0-5, frame 6 moved by noise of 0.5 (its temporal record,
    coded against frame 5 on the grid of the scaled anchor 0, is larger than the
    last spatial record yet smaller than its own spatial one), then smooth
    again; batch 4."""
    traj = datagen.MDTrajectory(n, step=0.002, seed=seed)
    fr = [traj.next_frame() for _ in range(6)]
    rng = np.random.default_rng(5)
    fr.append((fr[-1] + rng.normal(0, 0.5, size=fr[-1].shape)).astype(np.float32))
    for _ in range(5):
        fr.append((fr[-1] + rng.normal(0, 0.002, size=fr[-1].shape)).astype(np.float32))
    return fr


def gate_stream(n):
    """Eight copies of one uniform frame, then five unrelated uniform frames."""
    rng = np.random.default_rng(77)
    a = rng.uniform(0.0, 100.0, size=(3, n)).astype(np.float32)
    return [a.copy() for _ in range(8)] + [
        rng.uniform(0.0, 100.0, size=(3, n)).astype(np.float32) for _ in range(5)]


def oracle_records(xs, eb_mode, eb, batch, k):
    ost = O.Stream(eb_mode, eb, batch_size=batch, block_log2=k, max_n=xs[0].shape[1],
                   anchor_scale=S)
    return [ost.compress(x) for x in xs]


def check(lcp, xs, eb_mode, eb, batch=4, k=4, one_call=True):
    n = xs[0].shape[1]
    want = oracle_records(xs, eb_mode, eb, batch, k)
    kw = dict(multi_frame=True, batch_size=batch, block_log2=k, max_particles=n, anchor_scale=S)
    plan = lcp.Plan(eb, eb_mode, **kw)
    dev = [torch.from_numpy(x).cuda() for x in xs]
    if one_call:
        out, offs, used, perms = plan.compress(dev, want_perm=True)
        recs = [out[offs[t]:offs[t + 1]] for t in range(len(xs))]
    else:
        recs, used, perms = [], [], []
        for x in dev:
            o, of, u, p = plan.compress([x], want_perm=True)
            recs.append(o[:of[1]])
            used += u
            perms += p
    scaled_t = 0
    for t, (rec, wused, wperm) in enumerate(want):
        got = recs[t].cpu().numpy().tobytes()
        print(f"frame {t}: method {wused}, {len(rec)} bytes, step {rec[11]}", flush=True)
        assert used[t] == wused, (t, used[t], wused)
        assert got == rec, f"frame {t}: {len(got)} vs {len(rec)} bytes"
        assert np.array_equal(perms[t].cpu().numpy().astype(np.uint32), wperm), t
        scaled_t += rec[6] == 1 and rec[11] == S
    # the decoder, all records in one call, against the oracle's decoder
    buf = torch.cat(recs)
    offs = np.concatenate([[0], np.cumsum([r.numel() for r in recs])]).tolist()
    dplan = lcp.Plan(eb, eb_mode, **kw)
    dec = dplan.decompress(buf, offs)
    ost = O.Stream(eb_mode, eb, batch_size=batch, block_log2=k, max_n=n, anchor_scale=S)
    for t, (rec, _, wperm) in enumerate(want):
        w = ost.decompress(rec)
        d = dec[t].cpu().numpy()
        for f in range(3):
            assert bits_equal(d[f], w[f]), (t, f)
    return want, scaled_t


@pytest.mark.parametrize("n", [20000, 20003])
@pytest.mark.parametrize("one_call", [True, False])
def test_scaled_chain_and_run_break(lcp, n, one_call):
    xs = break_stream(n)
    want, scaled_t = check(lcp, xs, O.EB_REL_GLOBAL, EB, one_call=one_call)
    methods = "".join("S" if u == O.METHOD_S else "T" for _, u, _ in want)
    assert methods.startswith("SST") and scaled_t >= 3, (methods, scaled_t)


def test_gate_turns_scaling_off(lcp):
    xs = gate_stream(3000)
    want, _ = check(lcp, xs, O.EB_ABS, 0.01, k=3)
    # anchors at frames 0 and 8 scaled, at 12 not (a spatial record's grid
    # shows it: eb_q below eb / 5, or above eb / 2)
    import struct
    ebq = [struct.unpack_from("<f", rec, 84)[0] for rec, _, _ in want]
    assert ebq[0] < 0.01 / S and ebq[8] < 0.01 / S and ebq[12] > 0.01 / 2


def test_served_scaled_streams_match_standalone(lcp):
    n = 12000
    xs = [break_stream(n, seed=41 + j)[:8] for j in range(3)]
    srv = lcp.Server(4 * lcp.scratch_bytes(max_particles=n), workers=2, batch_frames=4,
                     batch_particles=4 * n)
    sids = [srv.open_stream(EB, lcp.EB_REL_GLOBAL, batch_size=4, block_log2=4, max_particles=n,
                            anchor_scale=S) for _ in xs]
    outs = [[torch.zeros(40 * n + 4096, dtype=torch.uint8, device="cuda") for _ in range(8)]
            for _ in xs]
    frames = [[torch.from_numpy(x).cuda() for x in s] for s in xs]
    sizes = [[0] * 8 for _ in xs]
    for t in range(8):
        srv.hold(True)
        tks = [srv.compress(sids[j], frames[j][t], outs[j][t]) for j in range(len(xs))]
        srv.hold(False)
        for j, tk in enumerate(tks):
            r = srv.wait(tk)
            assert r["status"] == 0, (j, t, r)
            sizes[j][t] = r["bytes"]
    torch.cuda.synchronize()
    for j, s in enumerate(xs):
        want = oracle_records(s, O.EB_REL_GLOBAL, EB, 4, 4)
        for t in range(8):
            assert outs[j][t][:sizes[j][t]].cpu().numpy().tobytes() == want[t][0], (j, t)
    c = srv.counts()
    print(c, flush=True)
    assert c["merged_requests"] > 0
    srv.close()
