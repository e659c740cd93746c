"""GPU parity of the batched form: independent frames compressed together (one
extent pass, one sort, one set of coding launches per batch) must give, record
by record, the oracle's bytes for each frame compressed alone, the oracle's
slot permutation, and bit-exact decoded values.
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


def bits_equal(a, b) -> bool:
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32), np.asarray(b, np.float32).view(np.uint32))


def mixed_frames():
    """Sizes from one particle to several workgroup tiles with ragged tails;
    uniform and clustered frames alternate."""
    sizes = [1, 2, 37, 1000, 4097, 20000, 65537, 3, 300000, 255, 256, 257]
    rng = np.random.default_rng(11)
    xs = []
    for j, n in enumerate(sizes):
        if j % 2 == 0:
            xs.append(datagen.uniform_frame(n, hi=100.0, seed=100 + j))
        else:
            xs.append(datagen.clustered_positions(rng, n, 100.0, 20, 0.3))
    return xs


def check_batch(lcp, xs, eb_mode, eb, k, decode_frames=None, **plan_kw):
    n_max = max(x.shape[1] for x in xs)
    plan = lcp.Plan(eb, eb_mode, n_fields=xs[0].shape[0], block_log2=k, max_particles=n_max,
                    **plan_kw)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    out, offs, used, perms = plan.compress(xd, want_perm=True)
    assert used == [lcp.METHOD_S] * len(xs)
    buf = out[:offs[-1]].cpu().numpy().tobytes()
    for j, x in enumerate(xs):
        print(f"frame {j} n={x.shape[1]}", flush=True)
        rec = buf[offs[j]:offs[j + 1]]
        want, wperm, _ = O.compress_s(x, O.grids_for(x, eb_mode, eb), k, 10, j)
        assert rec == want, f"frame {j}: {len(rec)} vs {len(want)} bytes"
        assert np.array_equal(perms[j].cpu().numpy().astype(np.uint32), wperm), j
    dec = plan.decompress(out, offs)
    for j in (decode_frames if decode_frames is not None else range(len(xs))):
        wdec, _ = O.decompress(buf[offs[j]:offs[j + 1]])
        got = dec[j].cpu().numpy()
        assert all(bits_equal(got[f], wdec[f]) for f in range(xs[j].shape[0])), j
    return plan, offs


def test_batch_of_mixed_frames(lcp):
    xs = mixed_frames()
    check_batch(lcp, xs, lcp.EB_REL_GLOBAL, 1e-4, 5,
                max_batch_particles=sum(x.shape[1] for x in xs), max_batch_frames=len(xs))


def test_batches_split_by_frame_count(lcp):
    xs = mixed_frames()
    check_batch(lcp, xs, lcp.EB_REL_GLOBAL, 1e-4, 3,
                max_batch_particles=sum(x.shape[1] for x in xs), max_batch_frames=3)


def test_batches_split_by_particle_count(lcp):
    # default batch capacity: max_particles per batch
    check_batch(lcp, mixed_frames(), lcp.EB_ABS, 1e-3, 7)


def test_batch_with_wide_keys(lcp):
    """20 bits of block id per axis at k = 0: 60-bit keys, eight radix passes,
    32 frames sorted side by side within their own segments."""
    xs = [datagen.uniform_frame(100, hi=1.0e6, seed=200 + j) for j in range(32)]
    check_batch(lcp, xs, lcp.EB_ABS, 0.5, 0, max_batch_particles=3200, max_batch_frames=32)


def test_batch_six_fields(lcp):
    xs = [datagen.cosmology_snapshot(n, box=64.0, n_halos=10, seed=300 + j)
          for j, n in enumerate([5000, 3, 12345, 777])]
    check_batch(lcp, xs, lcp.EB_REL_PER_FIELD, 1e-4, 4,
                max_batch_particles=sum(x.shape[1] for x in xs))


def test_batch_errors_leave_no_partial_state(lcp):
    xs = mixed_frames()[:4]
    bad = xs[2].copy()
    bad[1, 5] = np.nan
    plan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, block_log2=4, max_particles=5000,
                    max_batch_particles=10000)
    with pytest.raises(lcp.LCPError):
        plan.compress([torch.from_numpy(x).cuda() for x in [xs[0], xs[1], bad, xs[3]]])
    # the plan still works and numbers records from where it stood
    out, offs, _, _ = plan.compress([torch.from_numpy(x).cuda() for x in xs])
    rec = out[offs[0]:offs[1]].cpu().numpy().tobytes()
    want, _, _ = O.compress_s(xs[0], O.grids_for(xs[0], O.EB_REL_GLOBAL, 1e-4), 4, 10, 0)
    assert rec == want


def test_graph_replays_tunings_and_autotune(lcp):
    """Batches of one launch shape: the first call captures the kernels into a
    graph, later calls replay it on other frames of the same sizes (other
    values, grids and block counts) -- every record and permutation is the
    oracle's for its frame and sequence number.  Other launch shapes (tile,
    persistent grids), graphs switched off, and the autotuner's choice give
    the same bytes."""
    sizes = [5000, 70001, 3, 20000, 131072, 777]
    rng = np.random.default_rng(23)

    def frames(seed):
        r = np.random.default_rng(seed)
        return [datagen.uniform_frame(n, hi=100.0, seed=seed + j) if j % 2 == 0
                else datagen.clustered_positions(r, n, 100.0, 15, 0.3) for j, n in enumerate(sizes)]

    A, B = frames(31), frames(57)
    tot = sum(sizes)
    plan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, block_log2=5, max_particles=max(sizes),
                    max_batch_particles=tot, max_batch_frames=len(sizes))
    out = torch.empty(sum(plan.bound(n) + 4 for n in sizes), dtype=torch.uint8, device="cuda")
    seq = 0

    def check(xs, label):
        nonlocal seq
        xd = [torch.from_numpy(x).cuda() for x in xs]
        _, offs, used, perms = plan.compress(xd, out=out, want_perm=True)
        buf = out[:offs[-1]].cpu().numpy().tobytes()
        for j, x in enumerate(xs):
            want, wperm, _ = O.compress_s(x, O.grids_for(x, O.EB_REL_GLOBAL, 1e-4), 5, 10, seq + j)
            assert buf[offs[j]:offs[j + 1]] == want, (label, j)
            assert np.array_equal(perms[j].cpu().numpy().astype(np.uint32), wperm), (label, j)
        seq += len(xs)

    for rep, xs in enumerate([A, B, A, B]):  # capture, then replays
        check(xs, f"graph {rep}")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for t in [(4096, 0, 0, True), (2048, 8 * cus, 16 * cus, True), (256, 2, 1, True),
              (1024, 0, 0, False), (16384, 32 * cus, 0, False)]:
        plan.set_tuning(*t)
        assert plan.tuning() == {"tile": t[0], "grid": t[1], "slot_grid": t[2], "graphs": t[3]}
        check(B, f"tuning {t}")
    with pytest.raises(lcp.LCPError):
        plan.set_tuning(1000, 0, 0, True)  # not a multiple of 256
    tuned = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, block_log2=5, max_particles=max(sizes),
                     max_batch_particles=tot, max_batch_frames=len(sizes))
    xd = [torch.from_numpy(x).cuda() for x in A]
    choice, best, dflt = tuned.autotune(xd, out, reps=1)
    assert best <= dflt and choice["tile"] in (1024, 2048, 4096)
    _, offs, _, _ = tuned.compress(xd, out=out)
    buf = out[:offs[-1]].cpu().numpy().tobytes()
    for j, x in enumerate(A):  # the autotuner left the sequence numbers as they were
        want, _, _ = O.compress_s(x, O.grids_for(x, O.EB_REL_GLOBAL, 1e-4), 5, 10, j)
        assert buf[offs[j]:offs[j + 1]] == want, j
