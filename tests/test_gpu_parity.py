"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Bit-exact on every record byte (which fixes the quantisation codes, block order,
every symbol stream and coder choice), on the slot permutation, and on the
decoded float32 values (0 ULP: both sides evaluate fmaf((float)(2q+1), eb_q, m)).
"""
from __future__ import annotations

import numpy as np
import pytest

import fmt_ref
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


def diff_report(got: bytes, want: bytes) -> str:
    if got == want:
        return "equal"
    msg = [f"sizes {len(got)} vs {len(want)}"]
    try:
        a, b = fmt_ref.parse(got), fmt_ref.parse(want)
        for key in ("mode", "n", "B", "k", "bn", "seq", "ref_seq", "grids"):
            if a[key] != b[key]:
                msg.append(f"{key}: {a[key]} vs {b[key]}")
        for i, (da, db) in enumerate(zip(a["dirs"], b["dirs"])):
            if da != db:
                msg.append(f"array {i} dir {da} vs {db}")
            if a["arrays"][i] != b["arrays"][i]:
                j = next(t for t, (u, v) in enumerate(zip(a["arrays"][i], b["arrays"][i])) if u != v) \
                    if len(a["arrays"][i]) == len(b["arrays"][i]) else -1
                msg.append(f"array {i} values differ first at {j}")
    except Exception as e:  # noqa: BLE001
        msg.append(f"parse failed: {e!r}")
    return "; ".join(msg)


def bits_equal(a, b) -> bool:
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32), np.asarray(b, np.float32).view(np.uint32))


def run_s(lcp, x, eb_mode, eb, k, chunk_log2=10):
    plan = lcp.Plan(eb, eb_mode, n_fields=x.shape[0], block_log2=k, chunk_log2=chunk_log2,
                    max_particles=x.shape[1])
    xd = torch.from_numpy(x).cuda()
    out, offs, used, perms = plan.compress([xd], want_perm=True)
    torch.cuda.synchronize()
    rec = out[offs[0]:offs[1]].cpu().numpy().tobytes()
    dec = plan.decompress(out, offs)[0].cpu().numpy()
    return rec, perms[0].cpu().numpy().astype(np.uint32), dec


S_CASES = [
    # (n, seed, hi, eb, k, chunk_log2)
    (1, 1, 100.0, 1e-3, 4, 10),
    (2, 2, 100.0, 1e-3, 0, 10),
    (37, 3, 10.0, 0.05, 2, 5),
    (1000, 4, 100.0, 1e-3, 10, 10),
    (4097, 5, 100.0, 1e-3, 16, 10),
    (65537, 6, 100.0, 1e-3, 8, 10),
    (100000, 7, 1.0, 1e-4, 3, 9),
]


@pytest.mark.parametrize("n,seed,hi,eb,k,cl", S_CASES)
def test_spatial_parity_uniform(lcp, n, seed, hi, eb, k, cl):
    print(f"case n={n} seed={seed} k={k} cl={cl}", flush=True)
    x = datagen.uniform_frame(n, hi=hi, seed=seed)
    rec, perm, dec = run_s(lcp, x, lcp.EB_ABS, eb, k, cl)
    grids = O.grids_for(x, O.EB_ABS, eb)
    want, wperm, _ = O.compress_s(x, grids, k, cl, 0)
    assert rec == want, diff_report(rec, want)
    assert np.array_equal(perm, wperm)
    wdec, _ = O.decompress(want)
    for f in range(3):
        assert bits_equal(dec[f], wdec[f])
        assert np.max(np.abs(dec[f].astype(np.float64) - x[f][perm].astype(np.float64))) <= eb


def test_spatial_parity_identical_points(lcp):
    x = np.full((3, 5000), 7.25, np.float32)
    x[:, 0] = 0.0
    rec, perm, dec = run_s(lcp, x, lcp.EB_ABS, 0.01, 4)
    want, wperm, _ = O.compress_s(x, O.grids_for(x, O.EB_ABS, 0.01), 4, 10, 0)
    assert rec == want, diff_report(rec, want)
    assert np.array_equal(perm, wperm)


def test_spatial_parity_cosmology_six_fields(lcp):
    x = datagen.cosmology_snapshot(200000, box=256.0, n_halos=50, seed=3)
    rec, perm, dec = run_s(lcp, x, lcp.EB_REL_PER_FIELD, 1e-4, 3)
    grids = O.grids_for(x, O.EB_REL_PER_FIELD, 1e-4)
    want, wperm, _ = O.compress_s(x, grids, 3, 10, 0)
    assert rec == want, diff_report(rec, want)
    assert np.array_equal(perm, wperm)
    wdec, _ = O.decompress(want)
    for f in range(6):
        assert bits_equal(dec[f], wdec[f])
        assert np.max(np.abs(dec[f].astype(np.float64) - x[f][perm].astype(np.float64))) <= grids[f].eb


def test_block_size_search_matches_oracle(lcp):
    x = datagen.uniform_frame(1 << 18, seed=1)  # the 262,144-particle uniform frame, eb 1e-3
    xd = torch.from_numpy(x).cuda()
    plan = lcp.Plan(1e-3, lcp.EB_ABS, block_log2=-1, max_particles=x.shape[1], sample=xd)
    k, sizes = O.search_k(x, O.EB_ABS, 1e-3)
    assert plan.block_log2 == k
    out, offs, _, perms = plan.compress([xd], want_perm=True)
    rec = out[offs[0]:offs[1]].cpu().numpy().tobytes()
    want, wperm, _ = O.compress_s(x, O.grids_for(x, O.EB_ABS, 1e-3), k, 10, 0)
    assert rec == want, diff_report(rec, want)
    assert len(rec) == int(sizes[k])
    dec = plan.decompress(out, offs)[0].cpu().numpy()
    wdec, _ = O.decompress(want)
    assert all(bits_equal(dec[f], wdec[f]) for f in range(3))


@pytest.mark.parametrize("batch", [4, 0])
def test_multi_frame_stream_parity(lcp, batch):
    n, frames = 50000, 12
    traj = datagen.MDTrajectory(n, seed=21, step=0.002)
    xs = [traj.next_frame() for _ in range(frames)]
    ost = O.Stream(O.EB_REL_GLOBAL, 1e-4, batch_size=batch, block_log2=4, max_n=n)
    plan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=batch, block_log2=4,
                    max_particles=n)
    dplan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=batch, block_log2=4,
                     max_particles=n)
    eb = 1e-4 * (float(xs[0].max()) - float(xs[0].min()))
    for t, x in enumerate(xs):
        assert plan.select() == ost.select(), t
        want, wused, wperm = ost.compress(x)
        out, offs, used, perms = plan.compress([torch.from_numpy(x).cuda()], want_perm=True)
        rec = out[offs[0]:offs[1]].cpu().numpy().tobytes()
        assert used[0] == wused, (t, used, wused)
        assert rec == want, f"frame {t}: " + diff_report(rec, want)
        assert np.array_equal(perms[0].cpu().numpy().astype(np.uint32), wperm)
        dec = dplan.decompress(out, offs)[0].cpu().numpy()
        wdec = ost.decompress(want)
        for f in range(3):
            assert bits_equal(dec[f], wdec[f]), (t, f)
            assert np.max(np.abs(dec[f].astype(np.float64) - x[f][wperm].astype(np.float64))) <= eb


def test_forced_temporal_identical_frame(lcp):
    n = 30000
    x = datagen.uniform_frame(n, seed=9)
    plan = lcp.Plan(1e-3, lcp.EB_ABS, multi_frame=True, batch_size=0, block_log2=6, max_particles=n)
    xd = torch.from_numpy(x).cuda()
    out, offs, used, _ = plan.compress([xd, xd], methods=[lcp.METHOD_S, lcp.METHOD_T])
    assert used == [lcp.METHOD_S, lcp.METHOD_T]
    rec_t = out[offs[1]:offs[2]].cpu().numpy().tobytes()
    P = fmt_ref.parse(rec_t)
    assert P["mode"] == 1 and all(d["nbytes"] == 0 for d in P["dirs"])
    dplan = lcp.Plan(1e-3, lcp.EB_ABS, multi_frame=True, batch_size=0, block_log2=6, max_particles=n)
    d0, d1 = dplan.decompress(out, offs)
    assert torch.equal(d0, d1)


def test_temporal_infeasible_falls_back_to_spatial(lcp):
    """A frame that leaves the reference grid's float32 margin cannot be coded by
    LCP-T; the stream codes it spatially, exactly as the oracle does."""
    n = 20000
    traj = datagen.MDTrajectory(n, seed=31, step=0.001)
    xs = [traj.next_frame() for _ in range(6)]
    xs[4] = xs[4] * np.float32(3.0)  # |x| crosses into a higher binade
    ost = O.Stream(O.EB_REL_GLOBAL, 1e-4, batch_size=0, block_log2=4, max_n=n)
    plan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=0, block_log2=4,
                    max_particles=n)
    for t, x in enumerate(xs):
        want, wused, _ = ost.compress(x)
        out, offs, used, _ = plan.compress([torch.from_numpy(x).cuda()])
        rec = out[offs[0]:offs[1]].cpu().numpy().tobytes()
        assert used[0] == wused, t
        assert rec == want, f"frame {t}: " + diff_report(rec, want)
    assert fmt_ref.parse(want)["mode"] in (0, 1)


def test_batched_decompress_equals_per_frame(lcp):
    n, frames = 40000, 20
    traj = datagen.MDTrajectory(n, seed=41, step=0.003)
    xs = [torch.from_numpy(traj.next_frame()).cuda() for _ in range(frames)]
    plan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=8, block_log2=5,
                    max_particles=n)
    out, offs, used, _ = plan.compress(xs)
    assert lcp.METHOD_T in used and lcp.METHOD_S in used
    d_all = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=8, block_log2=5,
                     max_particles=n)
    d_one = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=8, block_log2=5,
                     max_particles=n)
    batch = d_all.decompress(out, offs)
    ost = O.Stream(O.EB_REL_GLOBAL, 1e-4, batch_size=8, block_log2=5, max_n=n)
    for j in range(frames):
        one = d_one.decompress(out, offs[j:j + 2])[0]
        assert torch.equal(one.view(torch.int32), batch[j].view(torch.int32)), j
        rec = out[offs[j]:offs[j + 1]].cpu().numpy().tobytes()
        w = ost.decompress(rec)
        assert all(bits_equal(batch[j][f].cpu().numpy(), w[f]) for f in range(3)), j


def test_temporal_residuals_need_the_length_limit(lcp):
    """Residual counts following the Fibonacci numbers make a Huffman tree 22
    deep, so the 13-bit limit halves the counts; every residual symbol is
    below 64, the alphabet the one-wave code builder handles."""
    fib = [1, 1]
    while len(fib) < 23:
        fib.append(fib[-1] + fib[-2])
    n = sum(fib)
    rng = np.random.default_rng(77)
    x0 = datagen.uniform_frame(n, hi=50.0, seed=78)
    grids = O.grids_for(x0, O.EB_ABS, 1e-3)
    r = np.repeat(np.arange(23, dtype=np.int64), fib)
    x1 = np.empty_like(x0)
    for f in range(3):
        rr = rng.permutation(r) if f else r[rng.permutation(n)]
        x1[f] = O.reconstruct(O.quantize(x0[f], grids[f]) + rr, grids[f])
    ost = O.Stream(O.EB_ABS, 1e-3, batch_size=0, block_log2=6, max_n=n)
    plan = lcp.Plan(1e-3, lcp.EB_ABS, multi_frame=True, batch_size=0, block_log2=6, max_particles=n)
    for t, (x, m) in enumerate([(x0, O.METHOD_S), (x1, O.METHOD_T)]):
        want, wused, _ = ost.compress(x, method=m)
        out, offs, used, _ = plan.compress([torch.from_numpy(x).cuda()], methods=[m])
        rec = out[offs[0]:offs[1]].cpu().numpy().tobytes()
        assert used[0] == wused == m, t
        assert rec == want, f"frame {t}: " + diff_report(rec, want)
    P = fmt_ref.parse(want)
    assert P["mode"] == 1 and any(d["coder"] == 1 for d in P["dirs"])


def test_temporal_residuals_above_a_byte_fixed_length(lcp):
    """Residuals uniform in [-512, 512): zigzag values reach 1023, beyond what
    one byte holds, and the flat distribution makes the fixed-length coder the
    shorter one."""
    n = 40000
    rng = np.random.default_rng(91)
    x0 = datagen.uniform_frame(n, hi=50.0, seed=92)
    grids = O.grids_for(x0, O.EB_ABS, 1e-3)
    x1 = np.empty_like(x0)
    for f in range(3):
        r = rng.integers(-512, 512, size=n)
        x1[f] = O.reconstruct(O.quantize(x0[f], grids[f]) + r, grids[f])
    ost = O.Stream(O.EB_ABS, 1e-3, batch_size=0, block_log2=6, max_n=n)
    plan = lcp.Plan(1e-3, lcp.EB_ABS, multi_frame=True, batch_size=0, block_log2=6, max_particles=n)
    for t, (x, m) in enumerate([(x0, O.METHOD_S), (x1, O.METHOD_T)]):
        want, wused, _ = ost.compress(x, method=m)
        out, offs, used, _ = plan.compress([torch.from_numpy(x).cuda()], methods=[m])
        rec = out[offs[0]:offs[1]].cpu().numpy().tobytes()
        assert used[0] == wused == m, t
        assert rec == want, f"frame {t}: " + diff_report(rec, want)
    P = fmt_ref.parse(want)
    assert P["mode"] == 1 and all(d["coder"] == 0 and d["param"] >= 9 for d in P["dirs"])


def temporal_pair(lcp, n, cl, resid, seed, arrays=True):
    """Frame 0 spatial, frame 1 forced temporal with the given residuals per
    field; both records and the decoded frame 1 against the oracle."""
    x0 = datagen.uniform_frame(n, hi=50.0, seed=seed)
    grids = O.grids_for(x0, O.EB_ABS, 1e-3)
    x1 = np.empty_like(x0)
    for f in range(3):
        x1[f] = O.reconstruct(O.quantize(x0[f], grids[f]) + resid[f], grids[f])
    ost = O.Stream(O.EB_ABS, 1e-3, batch_size=0, block_log2=6, chunk_log2=cl, max_n=n)
    plan = lcp.Plan(1e-3, lcp.EB_ABS, multi_frame=True, batch_size=0, block_log2=6, chunk_log2=cl,
                    max_particles=n)
    recs = []
    for t, (x, m) in enumerate([(x0, O.METHOD_S), (x1, O.METHOD_T)]):
        want, wused, _ = ost.compress(x, method=m)
        out, offs, used, _ = plan.compress([torch.from_numpy(x).cuda()], methods=[m])
        rec = out[offs[0]:offs[1]].cpu().numpy().tobytes()
        assert used[0] == wused == m, t
        assert rec == want, f"frame {t}: " + diff_report(rec, want)
        recs.append(want)
    dplan = lcp.Plan(1e-3, lcp.EB_ABS, multi_frame=True, batch_size=0, block_log2=6,
                     chunk_log2=cl, max_particles=n)
    buf = np.frombuffer(b"".join(recs), np.uint8)
    offs = [0, len(recs[0]), len(recs[0]) + len(recs[1])]
    dec = dplan.decompress(torch.from_numpy(buf.copy()).cuda(), offs)
    dst = O.Stream(O.EB_ABS, 1e-3, batch_size=0, block_log2=6, chunk_log2=cl, max_n=n)
    for t in range(2):
        w = dst.decompress(recs[t])
        assert all(bits_equal(dec[t][f].cpu().numpy(), w[f]) for f in range(3)), t
    return fmt_ref.parse(recs[1], arrays)


@pytest.mark.parametrize("cl", [5, 6, 7, 8, 9, 10, 11, 12])
def test_temporal_chunk_sizes_ragged(lcp, cl):
    """Small residuals (the byte path; nine in ten zero, so that Huffman wins
    even with 32-value chunks) at every chunk size, with a ragged last chunk and
    a length that is not a multiple of 16, so that the second and third
    fields' bytes start unaligned."""
    n = 40 * (1 << cl) + 37
    rng = np.random.default_rng(100 + cl)
    resid = [np.where(rng.random(n) < 0.9, 0, rng.integers(-3, 4, size=n)) for _ in range(3)]
    print(f"case cl={cl} n={n}", flush=True)
    P = temporal_pair(lcp, n, cl, resid, seed=200 + cl)
    # with 32-value chunks the chunk index alone costs a bit per value: fixed wins
    assert P["mode"] == 1 and all(d["coder"] == (1 if cl >= 6 else 0) for d in P["dirs"])


@pytest.mark.parametrize("cl", [6, 8, 10])
def test_temporal_escapes_and_many_rounds(lcp, cl):
    """Mostly small residuals with one in a thousand far out (zigzag values
    past a byte, some past the direct symbols, so raw extra bits follow their
    codes), over enough chunks that each packing wave takes several rounds."""
    n = (4100 << cl) // 4 * 4 + 11 if cl < 10 else (1 << 20) + 11
    rng = np.random.default_rng(300 + cl)
    resid = []
    for f in range(3):
        r = rng.integers(-2, 3, size=n)
        far = rng.random(n) < 1e-3
        r[far] = rng.integers(-6000, 6000, size=int(far.sum()))
        resid.append(r)
    assert min(int(np.abs(r).max()) for r in resid) >= 2048  # zigzag values past 4096
    print(f"case cl={cl} n={n}", flush=True)
    P = temporal_pair(lcp, n, cl, resid, seed=400 + cl, arrays=False)
    assert all(d["coder"] == 1 for d in P["dirs"])


def test_temporal_sixty_symbols(lcp):
    """Residuals spread over [-31, 31] (each value at least once, the rest
    Gaussian with sigma 8): 63 symbols, all below 64, for the one-wave code
    builder with nearly every lane in use."""
    n = 50000
    rng = np.random.default_rng(501)
    resid = []
    for _ in range(3):
        r = np.clip(np.rint(rng.normal(0.0, 8.0, size=n)), -31, 31).astype(np.int64)
        r[:63] = np.arange(-31, 32)
        resid.append(r)
    P = temporal_pair(lcp, n, 10, resid, seed=502)
    assert all(d["coder"] == 1 and d["used"] == 63 for d in P["dirs"])


def test_temporal_run_with_one_wide_frame(lcp):
    """Forced temporal frames coded in one call (back-to-back runs), one of
    them with residuals far past 64 symbols: the frames before it, that frame
    and the many after it (those first with the separate code build, later
    again with the packing kernel building the code) all match the oracle."""
    n, frames, wide, cl = 6000, 80, 5, 7
    rng = np.random.default_rng(611)
    x0 = datagen.uniform_frame(n, hi=50.0, seed=612)
    grids = O.grids_for(x0, O.EB_ABS, 1e-3)
    q = [O.quantize(x0[f], grids[f]) for f in range(3)]
    xs = [x0]
    for t in range(1, frames):
        x = np.empty_like(x0)
        for f in range(3):
            r = rng.integers(-2, 3, size=n)
            if t == wide:
                far = rng.random(n) < 0.01
                r[far] = rng.integers(-3000, 3000, size=int(far.sum()))
            q[f] = q[f] + r
            x[f] = O.reconstruct(q[f], grids[f])
        xs.append(x)
    ost = O.Stream(O.EB_ABS, 1e-3, batch_size=0, block_log2=6, chunk_log2=cl, max_n=n)
    plan = lcp.Plan(1e-3, lcp.EB_ABS, multi_frame=True, batch_size=0, block_log2=6, chunk_log2=cl,
                    max_particles=n)
    methods = [O.METHOD_S] + [O.METHOD_T] * (frames - 1)
    out, offs, used, _ = plan.compress([torch.from_numpy(x).cuda() for x in xs], methods=methods)
    assert list(used) == methods
    for t, x in enumerate(xs):
        want, wused, _ = ost.compress(x, method=methods[t])
        assert wused == methods[t], t
        rec = out[offs[t]:offs[t + 1]].cpu().numpy().tobytes()
        assert rec == want, f"frame {t}: " + diff_report(rec, want)
        if t == wide:
            assert max(d["param"] for d in fmt_ref.parse(want)["dirs"]) > 6
    # decoded in one call: chains of up to 16 temporal frames, one of them
    # with escaped residuals
    dplan = lcp.Plan(1e-3, lcp.EB_ABS, multi_frame=True, batch_size=0, block_log2=6,
                     chunk_log2=cl, max_particles=n)
    dec = dplan.decompress(out, offs)
    dst = O.Stream(O.EB_ABS, 1e-3, batch_size=0, block_log2=6, chunk_log2=cl, max_n=n)
    for t in range(frames):
        w = dst.decompress(out[offs[t]:offs[t + 1]].cpu().numpy().tobytes())
        assert all(bits_equal(dec[t][f].cpu().numpy(), w[f]) for f in range(3)), t
