"""Pins of the oracle's anchor error-bound scale (Sec. 7.4.2) that do not restate
its code.

Reading: an anchor frame (first in its batch, coded by LCP-S) is coded at eb / s
(s odd, the paper's 5) while the stream's frames are temporally correlated; a
temporal frame chained to such an anchor is coded at eb on the anchor's finer
grid, its code moving from the reference's by a multiple of s.

* Exact arithmetic: every reconstructed value of a scaled temporal frame is
  within eb of its input (fractions, no rounding), and the bound is not met by
  accident of a finer step (some errors exceed the anchor's own eb / s).
* Brute force: each code is the one value congruent to the reference's modulo
  s that lies within (s - 1) / 2 of the value's own bin, found by searching
  the candidates with exact bin positions.
* s = 1 gives the unscaled record byte for byte; the header carries s; a
  record with an even or spatial scale byte is refused.
* Alg. 1 + LCP-FSM + the correlation gate: a stream built so that the decision
  and scale of every frame follow by hand from the readings.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import fmt_ref
import oracle as O
from paper_2411_00761_amd import datagen


def exact_bin(x, g):
    """Exact position of x in bins of the grid: (x - m) / (2 eb_q) as a Fraction."""
    return (Fraction(float(x)) - Fraction(float(g.m))) / (2 * Fraction(float(g.eb_q)))


def recon_exact(Q, g):
    return (2 * Q + 1) * Fraction(float(g.eb_q)) + Fraction(float(g.m))


def scaled_pair(n=400, s=5, eb=0.05, seed=3, step=0.03):
    """An anchor coded by S at eb / s and the next frame coded by T against it."""
    traj = datagen.MDTrajectory(n, step=step, seed=seed)
    x0, x1 = traj.next_frame(), traj.next_frame()
    lo, hi = x0.min(axis=1), x0.max(axis=1)
    grids = [O.make_grid(lo[f], hi[f], eb / s) for f in range(3)]
    _, perm, q0 = O.compress_s(x0, grids, 2)
    rec, q1 = O.compress_t(x1, grids, perm, q0, ref_seq=0, seq=1, scale=s)
    return x1, grids, perm, q0, rec, q1


@pytest.mark.parametrize("s", [3, 5, 7])
def test_scaled_temporal_bound_exact(s):
    eb = 0.05
    x1, grids, perm, q0, rec, q1 = scaled_pair(s=s, eb=eb)
    out, qd = O.decompress(rec, ref_q=q0, ref_seq=0)
    assert np.array_equal(qd, q1)
    worst = Fraction(0)
    for f in range(3):
        for j in range(x1.shape[1]):
            xv = Fraction(float(x1[f][perm[j]]))
            err = abs(Fraction(float(out[f][j])) - xv)
            assert err <= Fraction(eb), (f, j)
            worst = max(worst, err)
            # the float32 output is the exact bin centre rounded once
            assert np.float32(float(recon_exact(int(q1[f][j]), grids[f]))) == out[f][j]
    # a coarse step is in use: errors beyond the anchor grid's own bound occur
    assert worst > Fraction(eb) / s


@pytest.mark.parametrize("s", [3, 5])
def test_scaled_codes_brute_force(s):
    x1, grids, perm, q0, _rec, q1 = scaled_pair(n=150, s=s, eb=0.05, seed=9, step=0.05)
    h = (s - 1) // 2
    moved = 0
    for f in range(3):
        for j in range(x1.shape[1]):
            t = exact_bin(x1[f][perm[j]], grids[f])
            q = int(t // 1)  # the value's own bin
            ref = int(q0[f][j])
            cands = [c for c in range(ref - 10 * s - q, ref + 10 * s - q + 1)]
            ok = [q + c for c in cands if (q + c - ref) % s == 0 and abs(c) <= h]
            assert len(ok) == 1
            assert int(q1[f][j]) == ok[0], (f, j)
            moved += int(q1[f][j]) != ref
    assert moved > 0


def test_scale_one_is_the_plain_record():
    traj = datagen.MDTrajectory(300, step=0.02, seed=4)
    x0, x1 = traj.next_frame(), traj.next_frame()
    lo, hi = x0.min(axis=1), x0.max(axis=1)
    grids = [O.make_grid(lo[f], hi[f], 0.01) for f in range(3)]
    _, perm, q0 = O.compress_s(x0, grids, 3)
    a, qa = O.compress_t(x1, grids, perm, q0, ref_seq=0, seq=1)
    b, qb = O.compress_t(x1, grids, perm, q0, ref_seq=0, seq=1, scale=1)
    assert a == b and np.array_equal(qa, qb)
    assert a[11] == 0 and fmt_ref.parse(a, arrays=False)["scale"] == 1


def test_scale_in_header_and_refusals():
    _x1, _g, _p, q0, rec, _q1 = scaled_pair(s=5)
    assert rec[11] == 5 and O.record_info(rec).scale == 5
    assert fmt_ref.parse(rec, arrays=False)["scale"] == 5
    bad = bytearray(rec)
    bad[11] = 4
    with pytest.raises(O.OracleError) as e:
        O.record_info(bytes(bad))
    assert e.value.status == O.ERR_CORRUPT
    traj = datagen.MDTrajectory(200, step=0.02, seed=5)
    x0 = traj.next_frame()
    lo, hi = x0.min(axis=1), x0.max(axis=1)
    srec, _, _ = O.compress_s(x0, [O.make_grid(lo[f], hi[f], 0.01) for f in range(3)], 2)
    bad = bytearray(srec)
    bad[11] = 5
    with pytest.raises(O.OracleError):
        O.record_info(bytes(bad))
    with pytest.raises(O.OracleError):
        O.compress_t(traj.next_frame(), [O.make_grid(lo[f], hi[f], 0.01) for f in range(3)],
                     np.arange(200, dtype=np.uint32), np.zeros((3, 200), np.int32), 0, scale=2)


# ------------------------------------------------------------------ gate trace
def gate_stream_frames(n=3000):
    """Eight copies of one uniform frame A, then five unrelated uniform frames."""
    rng = np.random.default_rng(77)

    def rand():
        return rng.uniform(0.0, 100.0, size=(3, n)).astype(np.float32)

    a = rand()
    return [a.copy() for _ in range(8)] + [rand() for _ in range(5)]


# Batch size 4, s = 5.  From the readings of Sec. 7.2 (LCP-FSM), Alg. 1 and the
# gate (an anchor is scaled at the stream's start, or when at least half of the
# frames since the last anchor were coded by T):
#  0 first in batch, no reference: S; anchor, nothing coded yet -> scaled
#  1 countdown 1: S at eb (not first in batch)
#  2 compare: T against frame 1 (same values: zero residuals) wins -> T, scale 1
#  3 T kept, scale 1
#  4 first in batch, T against anchor 0 (same values on its grid): kept, scale 5
#  5..7 T kept, chained to frame 4: scale 5
#  8 first in batch, unrelated: T against anchor 0 loses; S wins -> anchor;
#    since anchor 0: frames 1..7, six by T -> scaled
#  9 compare (S1X): unrelated, S wins -> S2X
# 10 countdown: S
# 11 compare: S wins -> S4X
# 12 first in batch, countdown: S -> anchor; since anchor 8 no frame by T -> not scaled
GATE_METHODS = "S S T T T T T T S S S S S".split()
GATE_SCALES = [5, 1, 1, 1, 5, 5, 5, 5, 5, 1, 1, 1, 1]


def test_gate_trace_written_by_hand():
    frames = gate_stream_frames()
    eb = 0.01
    st = O.Stream(O.EB_ABS, eb, batch_size=4, block_log2=3, max_n=frames[0].shape[1],
                  anchor_scale=5)
    dst = O.Stream(O.EB_ABS, eb, batch_size=4, block_log2=3, max_n=frames[0].shape[1],
                   anchor_scale=5)
    methods, scales = [], []
    for t, x in enumerate(frames):
        rec, used, perm = st.compress(x)
        P = fmt_ref.parse(rec, arrays=False)
        methods.append("S" if used == O.METHOD_S else "T")
        if P["mode"] == 0:
            # an S record's scale shows in its grid: eb_q below eb / 5, or above eb / 2
            ebq = P["grids"][0][1]
            assert ebq < eb / 5 or ebq > eb / 2
            scales.append(5 if ebq < eb / 5 else 1)
        else:
            scales.append(P["scale"])
            assert P["ref_seq"] == (0 if t == 4 else t - 1)
        out = dst.decompress(rec)
        for f in range(3):
            err = np.abs(out[f].astype(np.float64) - x[f][perm].astype(np.float64))
            assert err.max() <= eb
    assert methods == GATE_METHODS
    assert scales == GATE_SCALES


def test_gate_off_without_scale():
    frames = gate_stream_frames(1000)
    a = O.Stream(O.EB_ABS, 0.01, batch_size=4, block_log2=3, max_n=1000, anchor_scale=0)
    b = O.Stream(O.EB_ABS, 0.01, batch_size=4, block_log2=3, max_n=1000, anchor_scale=1)
    for x in frames:
        assert a.compress(x)[0] == b.compress(x)[0]
