"""GPU parity of int32 fields (Sec. 3: the data may be integers).

Records, slot permutations and decoded values must equal the oracle's, byte for
byte and bit for bit: single frames of fixed-point MD positions under the three
bound modes (lossless, small and wide bins; ragged sizes; several block
sizes), a batch of independent frames in one call, values at both ends of the
int32 range (the saturating reconstruction), multi-frame streams one call
(temporal runs) and frame by frame, anchors with an error-bound scale and the
fallback when an integer bin cannot be split, a 2-D stream with a
supplementary field, served streams of both element types merged into shared
launches, the entry point without allocation, the container of int32 records
(packed bytes and retrievals in several orders), and the refusals (a range past
the code limit, a record of the other type).
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


MODES = {0: O.EB_ABS, 1: O.EB_REL_GLOBAL, 2: O.EB_REL_PER_FIELD}


def md_ints(n, frames=1, seed=3, step=0.01, units=1000.0, F=3):
    traj = datagen.MDTrajectory(n, step=step, seed=seed)
    out = []
    for _ in range(frames):
        x = datagen.fixed_point(traj.next_frame(), units)
        if F > 3:  # supplementary integer fields (e.g. species, charge counts)
            rng = np.random.default_rng(seed + 100 + len(out))
            x = np.concatenate([x, rng.integers(-500, 500, size=(F - 3, n), dtype=np.int32)])
        out.append(np.ascontiguousarray(x[:F]))
    return out


def dev(x):
    return torch.from_numpy(x).cuda()


@pytest.mark.parametrize("n,k,mode,eb", [(5001, 4, 0, 0.5), (4099, 6, 0, 3.0), (20000, 8, 0, 250.0),
                                         (7003, 5, 1, 1e-4), (3000, 3, 2, 1e-3), (1, 0, 0, 2.0),
                                         (65537, 10, 0, 17.5)])
def test_single_frame_parity(lcp, n, k, mode, eb):
    x = md_ints(n, seed=n % 97)[0]
    plan = lcp.Plan(eb, mode, block_log2=k, max_particles=n, dtype=lcp.DTYPE_I32)
    out, offs, _, perms = plan.compress([dev(x)], want_perm=True)
    got = out[:offs[1]].cpu().numpy().tobytes()
    want, perm, _ = O.compress_s(x, O.grids_for(x, MODES[mode], eb), k)
    assert got == want, (len(got), len(want))
    assert got[53] == 1
    assert np.array_equal(perms[0].cpu().numpy().astype(np.uint32), perm)
    dec = plan.decompress(out, offs)[0]
    assert dec.dtype == torch.int32
    dec = dec.cpu().numpy()
    wdec, _ = O.decompress(want)
    for f in range(3):
        assert np.array_equal(dec[f], wdec[f]), f


def test_batch_of_frames_with_supplementary_fields(lcp):
    sizes = [3000, 777, 12345, 1, 4096]
    xs = [md_ints(n, seed=40 + j, F=5)[0] for j, n in enumerate(sizes)]
    plan = lcp.Plan(6.0, lcp.EB_ABS, n_fields=5, block_log2=5, max_particles=max(sizes),
                    max_batch_frames=8, dtype=lcp.DTYPE_I32)
    out, offs, _, _ = plan.compress([dev(x) for x in xs])
    buf = out[:offs[-1]].cpu().numpy().tobytes()
    for j, x in enumerate(xs):
        want, _, _ = O.compress_s(x, O.grids_for(x, O.EB_ABS, 6.0), 5, seq=j)
        assert buf[offs[j]:offs[j + 1]] == want, j
    dec = plan.decompress(out, offs)
    for j in range(len(xs)):
        w, _ = O.decompress(buf[offs[j]:offs[j + 1]])
        for f in range(5):
            assert np.array_equal(dec[j][f].cpu().numpy(), w[f]), (j, f)


@pytest.mark.parametrize("lo,eb", [(2147483647 - 40000, 10.0), (-2147483648, 3.0)])
def test_int32_range_ends(lcp, lo, eb):
    rng = np.random.default_rng(8)
    n = 10000
    x = (lo + rng.integers(0, 40001, size=(3, n))).astype(np.int32)
    x[:, 0] = lo  # the extreme itself
    x[:, 1] = lo + 40000
    plan = lcp.Plan(eb, lcp.EB_ABS, block_log2=6, max_particles=n, dtype=lcp.DTYPE_I32)
    out, offs, _, _ = plan.compress([dev(x)])
    want, perm, _ = O.compress_s(x, O.grids_for(x, O.EB_ABS, eb), 6)
    assert out[:offs[1]].cpu().numpy().tobytes() == want
    dec = plan.decompress(out, offs)[0].cpu().numpy()
    wdec, _ = O.decompress(want)
    for f in range(3):
        assert np.array_equal(dec[f], wdec[f])
        assert np.abs(dec[f].astype(np.int64) - x[f][perm].astype(np.int64)).max() <= eb


def test_refusals(lcp):
    x = np.array([[-2147483648, 2147483647, 0]] * 3, np.int32)
    plan = lcp.Plan(0.5, lcp.EB_ABS, block_log2=0, max_particles=3, dtype=lcp.DTYPE_I32)
    with pytest.raises(lcp.LCPError) as e:
        plan.compress([dev(x)])
    assert e.value.status == lcp.ERR_RANGE
    with pytest.raises(O.OracleError) as e2:
        O.compress_s(x, O.grids_for(x, O.EB_ABS, 0.5), 0)
    assert e2.value.status == O.ERR_RANGE
    # a record decodes only through a plan of its element type
    y = md_ints(500, seed=2)[0]
    ip = lcp.Plan(2.0, lcp.EB_ABS, block_log2=4, max_particles=500, dtype=lcp.DTYPE_I32)
    out, offs, _, _ = ip.compress([dev(y)])
    fp = lcp.Plan(2.0, lcp.EB_ABS, block_log2=4, max_particles=500)
    with pytest.raises(lcp.LCPError) as e:
        fp.decompress(out, offs, outs=[torch.empty((3, 500), dtype=torch.float32, device="cuda")])
    assert e.value.status == lcp.ERR_ARG
    with pytest.raises(lcp.LCPError):
        lcp.Plan(2.0, lcp.EB_ABS, block_log2=4, max_particles=500, dtype=2)


def stream_check(lcp, xs, eb, mode=0, F=3, D=0, one_call=True, anchor_scale=0, batch=4):
    n = xs[0].shape[1]
    ost = O.Stream(MODES[mode], eb, n_fields=F, batch_size=batch, block_log2=4, max_n=n,
                   n_dims=D, anchor_scale=anchor_scale, dtype=O.DTYPE_I32)
    want = [ost.compress(x) for x in xs]
    kw = dict(n_fields=F, multi_frame=True, batch_size=batch, block_log2=4, max_particles=n,
              n_dims=D, anchor_scale=anchor_scale, dtype=lcp.DTYPE_I32)
    plan = lcp.Plan(eb, mode, **kw)
    dx = [dev(x) for x in xs]
    if one_call:
        out, offs, used, _ = plan.compress(dx)
        recs = [out[offs[t]:offs[t + 1]] for t in range(len(xs))]
    else:
        recs, used = [], []
        for x in dx:
            o, of, u, _ = plan.compress([x])
            recs.append(o[:of[1]])
            used += u
    for t, (rec, wused, _) in enumerate(want):
        print(f"frame {t} used {used[t]}", flush=True)
        assert used[t] == wused, t
        assert recs[t].cpu().numpy().tobytes() == rec, t
    dplan = lcp.Plan(eb, mode, **kw)
    buf = torch.cat(recs)
    offs = np.concatenate([[0], np.cumsum([r.numel() for r in recs])]).tolist()
    dec = dplan.decompress(buf, offs)
    dst = O.Stream(MODES[mode], eb, n_fields=F, batch_size=batch, block_log2=4, max_n=n,
                   n_dims=D, anchor_scale=anchor_scale, dtype=O.DTYPE_I32)
    for t, (rec, _, _) in enumerate(want):
        w = dst.decompress(rec)
        for f in range(F):
            assert np.array_equal(dec[t][f].cpu().numpy(), w[f]), (t, f)
    return used, [r.cpu().numpy().tobytes() for r in recs]


@pytest.mark.parametrize("one_call", [True, False])
@pytest.mark.parametrize("n,eb,mode", [(20000, 4.0, 0), (20003, 0.5, 0), (30000, 1e-4, 1)])
def test_stream_parity(lcp, n, eb, mode, one_call):
    xs = md_ints(n, frames=12, seed=n % 13, step=0.004)
    used, _ = stream_check(lcp, xs, eb, mode=mode, one_call=one_call)
    assert lcp.METHOD_T in used


def test_stream_2d_with_supplementary(lcp):
    xs = [x[[0, 1, 3]] for x in md_ints(20000, frames=10, seed=5, step=0.004, F=4)]
    for j in range(1, len(xs)):  # the supplementary field changes little between frames
        xs[j][2] = xs[0][2] + (j % 3)
    used, _ = stream_check(lcp, xs, 2.0, F=3, D=2)
    assert lcp.METHOD_T in used


@pytest.mark.parametrize("eb", [12.0, 1.0])
def test_anchor_scale(lcp, eb):
    xs = md_ints(20000, frames=13, seed=21, step=0.003)
    used, recs = stream_check(lcp, xs, eb, anchor_scale=5)
    scales = [r[11] for r in recs]
    if eb == 1.0:  # bins of 3 integers cannot be split five ways
        assert all(s == 0 for s in scales)
    else:
        assert any(s == 5 for s in scales)


def test_static_entry_point(lcp):
    xs = md_ints(50000, frames=3, seed=9)
    xs[1] = xs[1][:, :20001].copy()
    out, offs, perms = lcp.compress_static([dev(x) for x in xs], 5.0, lcp.EB_ABS, block_log2=5,
                                           max_particles=50000, want_perm=True,
                                           dtype=lcp.DTYPE_I32)
    buf = out[:offs[-1]].cpu().numpy().tobytes()
    for j, x in enumerate(xs):
        want, wperm, _ = O.compress_s(x, O.grids_for(x, O.EB_ABS, 5.0), 5, seq=j)
        assert buf[offs[j]:offs[j + 1]] == want, j
        assert np.array_equal(perms[j].cpu().numpy().astype(np.uint32), wperm), j


def test_served_mixed_types(lcp):
    """int32 and float32 streams served together, temporal requests merged into
    shared launches: every record equals the oracle stream's."""
    n = 20000
    FR = 6
    ints_ = md_ints(n, frames=FR, seed=31, step=0.004)
    traj = datagen.MDTrajectory(n, step=0.004, seed=32)
    flts = [traj.next_frame() for _ in range(FR)]
    streams = [(ints_, lcp.DTYPE_I32, 4.0), (flts, lcp.DTYPE_F32, 1e-3),
               (ints_, lcp.DTYPE_I32, 9.0)]
    srv = lcp.Server(4 * lcp.scratch_bytes(max_particles=n), workers=2, batch_frames=4,
                     batch_particles=4 * n)
    sids = [srv.open_stream(eb, lcp.EB_ABS, batch_size=4, block_log2=4, max_particles=n,
                            dtype=dt) for (_, dt, eb) in streams]
    recs = [[] for _ in streams]
    for t in range(FR):
        outs = [torch.zeros(40 * n + 4096, dtype=torch.uint8, device="cuda") for _ in streams]
        srv.hold(True)
        tks = [srv.compress(sid, dev(xs[t]), outs[i]) for i, (sid, (xs, _, _)) in
               enumerate(zip(sids, streams))]
        srv.hold(False)
        for i, tk in enumerate(tks):
            r = srv.wait(tk)
            assert r["status"] == 0, (t, i, r)
            recs[i].append(outs[i][:r["bytes"]].cpu().numpy().tobytes())
    c = srv.counts()
    srv.close()
    for i, (xs, dt, eb) in enumerate(streams):
        ost = O.Stream(O.EB_ABS, eb, batch_size=4, block_log2=4, max_n=n,
                       dtype=O.DTYPE_I32 if dt == lcp.DTYPE_I32 else O.DTYPE_F32)
        for t, x in enumerate(xs):
            assert recs[i][t] == ost.compress(x)[0], (i, t)
    assert c["merged_requests"] > 0, c


def test_frame_2p20(lcp):
    n = 1 << 20
    xs = md_ints(n, frames=3, seed=44, step=0.004)
    eb = 3.0
    plan = lcp.Plan(eb, lcp.EB_ABS, multi_frame=True, batch_size=16, block_log2=-1,
                    max_particles=n, sample=dev(xs[0]), dtype=lcp.DTYPE_I32)
    k = plan.block_log2
    assert k == O.search_k(xs[0], O.EB_ABS, eb)[0]
    out, offs, used, _ = plan.compress([dev(x) for x in xs])
    ost = O.Stream(O.EB_ABS, eb, batch_size=16, block_log2=k, max_n=n, dtype=O.DTYPE_I32)
    for t, x in enumerate(xs):
        rec, u, _ = ost.compress(x)
        assert used[t] == u, t
        assert out[offs[t]:offs[t + 1]].cpu().numpy().tobytes() == rec, t


def test_container_of_int_records(lcp):
    """int32 records packed for random access: the bytes, and every retrieval
    (frames in any order), equal the oracle's."""
    n, batch = 20003, 4
    xs = md_ints(n, frames=14, seed=23, step=0.004)
    kw = dict(multi_frame=True, batch_size=batch, block_log2=4, max_particles=n,
              dtype=lcp.DTYPE_I32)
    plan = lcp.Plan(4.0, lcp.EB_ABS, **kw)
    out, offs, _, _ = plan.compress([dev(x) for x in xs])
    recs = [out[offs[j]:offs[j + 1]].cpu().numpy().tobytes() for j in range(len(xs))]
    want = O.container_pack(recs, batch)
    cont = lcp.Container.pack(out, offs, batch)
    assert cont.cpu().numpy().tobytes() == want
    C = lcp.Container(cont)
    dplan = lcp.Plan(4.0, lcp.EB_ABS, **kw)
    for req in ([13], [2, 9, 5, 6], list(range(14))[::-1]):
        outs = [torch.empty((3, n), dtype=torch.int32, device="cuda") for _ in req]
        decoded = C.retrieve(dplan, req, outs)
        wout, wdec = O.container_retrieve(want, req, O.EB_ABS, 4.0, block_log2=4,
                                          dtype=O.DTYPE_I32)
        assert decoded == wdec
        for k, o in zip(req, outs):
            got = o.cpu().numpy()
            for f in range(3):
                assert np.array_equal(got[f], wout[k][f]), (k, f)
    C.close()
