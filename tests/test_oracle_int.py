"""Pins of the oracle's integer-typed fields that do not restate its code.

Reading (Sec. 3 allows the data to be integers; the paper gives no quantiser
for them): with b = floor(eb), a bin is a run of w = 2b + 1 consecutive
integers from the field's minimum, a value is reconstructed as the integer at
its run's centre (held to the int32 range), and a temporal frame chained to an
anchor made with the step s uses the largest odd w with s w <= 2b + 1.

* Values worked by hand (tests/golden/int_grid_cases.json): codes and
  reconstructions of a spatial frame and of a temporal frame on its grid, the
  scaled bin widths and the int32 clamps.
* Brute force: every reconstruction is an integer within floor(eb) of its
  value, and the bins are the widest that allow it (a run of L integers takes
  ceil(L / (2b + 1)) codes; no run of 2b + 2 integers has a centre within b of
  both ends).
* Records: the dtype byte and the integer grid slots parsed by the test-side
  reader; a spatial record's codes, read back by that reader, are the floor
  divisions; decoding gives int32 values within the bound.
* Streams (Alg. 1 + LCP-FSM): fixed-point MD frames coded by S and T decode
  within the bound; eb < 1 is lossless; a constant field under a relative
  bound is kept exactly; anchors scaled by s keep the bound, and fall back to
  the stream's bound when a bin cannot be split.
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import fmt_ref
import oracle as O
from paper_2411_00761_amd import datagen

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "int_grid_cases.json")))


def ints(*rows):
    return np.ascontiguousarray(np.array(rows, dtype=np.int32))


# ------------------------------------------------------------------ worked by hand
def test_worked_spatial_and_temporal():
    S, T = GOLD["spatial"], GOLD["temporal_on_that_grid"]
    g = O.make_grid_i(S["m"], S["eb"])
    assert (g.mi, 2 * g.hb + 1) == (S["m"], S["w"])
    assert [O.quant_i(x, g) for x in S["x"]] == S["q"]
    assert [O.recon_i(q, g) for q in S["q"]] == S["recon"]
    assert [abs(r - x) for r, x in zip(S["recon"], S["x"])] == S["err"]
    assert [O.quant_i(x, g) for x in T["x"]] == T["q"]
    assert [O.recon_i(q, g) for q in T["q"]] == T["recon"]
    assert [abs(r - x) for r, x in zip(T["recon"], T["x"])] == T["err"]
    # the same values through the record path: a one-field record with D = 1
    x = ints(S["x"])
    grids = O.grids_for(x, O.EB_ABS, S["eb"])
    rec, perm, q = O.compress_s(x, grids, 0, dims=1)
    assert [int(v) for v in q[0]] == [S["q"][i] for i in perm]
    out, _ = O.decompress(rec)
    assert out[0].dtype == np.int32
    assert [int(v) for v in out[0]] == [S["recon"][i] for i in perm]
    trec, tq = O.compress_t(ints(T["x"]), grids, perm, q, ref_seq=0, seq=1)
    tout, _ = O.decompress(trec, ref_q=q, ref_seq=0)
    assert [int(v) for v in tout[0]] == [T["recon"][i] for i in perm]


@pytest.mark.parametrize("case", GOLD["scaled_widths"], ids=lambda c: f"eb{c['eb']}-s{c['s']}")
def test_scaled_widths(case):
    if case["w"] is None:
        with pytest.raises(O.OracleError) as e:
            O.make_grid_i(0, case["eb"], case["s"])
        assert e.value.status == O.ERR_EB_TOO_SMALL
        return
    g = O.make_grid_i(0, case["eb"], case["s"])
    assert (2 * g.hb + 1, g.hb) == (case["w"], case["hb"])


@pytest.mark.parametrize("i", range(3))
def test_clamps(i):
    c = GOLD["clamps"][i]
    g = O.make_grid_i(c["m"], c["eb"])
    assert O.quant_i(c["x"], g) == c["q"]
    assert O.recon_i(c["q"], g) == c["recon"]
    assert abs(c["recon"] - c["x"]) <= c["eb"]


def test_full_range_lossless_is_refused():
    c = GOLD["clamps"][3]
    x = ints([c["m"], c["x"], 0])
    with pytest.raises(O.OracleError) as e:
        O.compress_s(x, O.grids_for(x, O.EB_ABS, 0.5), 0, dims=1)
    assert e.value.status == O.ERR_RANGE


# ------------------------------------------------------------------ brute force
@pytest.mark.parametrize("eb", [0.3, 1.0, 2.5, 3.0, 7.99, 40.0])
@pytest.mark.parametrize("m", [-37, 0, 1000])
def test_bound_and_widest_bins(eb, m):
    g = O.make_grid_i(m, eb)
    b = int(np.floor(eb))
    xs = list(range(m - 3 * (2 * b + 1) - 2, m + 6 * (2 * b + 1) + 3))
    codes = [O.quant_i(x, g) for x in xs]
    for x, q in zip(xs, codes):
        r = O.recon_i(q, g)
        assert abs(r - x) <= eb, (x, q, r)
    # codes never decrease, and a run of L integers from the origin takes
    # ceil(L / (2b + 1)) of them: the widest bins the bound allows
    assert all(a <= c for a, c in zip(codes, codes[1:]))
    for L in range(1, 4 * (2 * b + 1)):
        assert len({O.quant_i(x, g) for x in range(m, m + L)}) == -(-L // (2 * b + 1))
    # no run of 2b + 2 integers has an integer within b of both ends
    assert not any(abs(c - m) <= b and abs(c - (m + 2 * b + 1)) <= b
                   for c in range(m - 2 * b - 2, m + 4 * b + 4))


@pytest.mark.parametrize("s", [3, 5, 7, 9, 15])
@pytest.mark.parametrize("eb", [4.0, 7.5, 12.0, 31.0])
def test_scaled_step_bound_brute_force(s, eb):
    """Every value against every reference code: the temporal code moves from
    the reference's by the multiple of s nearest the value's own code; the
    reconstruction stays within eb (and the width is the largest that does)."""
    b = int(np.floor(eb))
    if 2 * b + 1 < s:
        pytest.skip("no finer bin")
    g = O.make_grid_i(0, eb, s)
    w = 2 * g.hb + 1
    assert w % 2 == 1 and s * w <= 2 * b + 1 < s * (w + 2)
    h = (s - 1) // 2
    worst = 0
    for ref in range(-2 * s, 2 * s + 1):
        for x in range(-4 * s * w, 4 * s * w + 1):
            q = O.quant_i(x, g)
            # candidates congruent to ref modulo s within h of q: exactly one
            ok = [c for c in range(q - h, q + h + 1) if (c - ref) % s == 0]
            assert len(ok) == 1
            err = abs(O.recon_i(ok[0], g) - x)
            assert err <= eb
            worst = max(worst, err)
    # the worst case is reached: the width could not be larger
    assert worst == (s * w - 1) // 2


# ------------------------------------------------------------------ records
def md_ints(n=600, frames=6, seed=11, step=0.02, units=1000.0):
    traj = datagen.MDTrajectory(n, step=step, seed=seed)
    return [datagen.fixed_point(traj.next_frame(), units) for _ in range(frames)]


def test_record_header_and_codes():
    x = md_ints(frames=1)[0]
    eb = 6.0
    grids = O.grids_for(x, O.EB_ABS, eb)
    rec, perm, q = O.compress_s(x, grids, 4)
    P = fmt_ref.parse(rec)
    assert P["dtype"] == 1 and rec[53] == 1
    lo = x.min(axis=1)
    assert P["grids"] == [(int(lo[f]), 6) for f in range(3)]
    codes, _, _, _ = fmt_ref.s_codes(rec)
    for f in range(3):
        want = [(int(x[f][i]) - int(lo[f])) // 13 for i in perm]  # Python's // rounds down
        assert codes[f] == want
    out, qd = O.decompress(rec)
    assert np.array_equal(qd, q)
    for f in range(3):
        assert out[f].dtype == np.int32
        assert np.abs(out[f].astype(np.int64) - x[f][perm].astype(np.int64)).max() <= eb


def test_record_refusals():
    x = md_ints(frames=1)[0]
    rec, _, _ = O.compress_s(x, O.grids_for(x, O.EB_ABS, 3.0), 3)
    bad = bytearray(rec)
    bad[53] = 2
    with pytest.raises(O.OracleError) as e:
        O.record_info(bytes(bad))
    assert e.value.status == O.ERR_CORRUPT
    bad = bytearray(rec)
    bad[80 + 7] = 0x80  # half width 2^31 + 3
    with pytest.raises(O.OracleError) as e:
        O.record_info(bytes(bad))
    assert e.value.status == O.ERR_CORRUPT
    # a float grid for int32 fields (or mixed grids) is refused
    g = O.grids_for(x, O.EB_ABS, 3.0)
    gf = O.grids_for(x.astype(np.float32), O.EB_ABS, 3.0)
    with pytest.raises(O.OracleError):
        O.compress_s(x, [g[0], gf[1], g[2]], 3)


def test_float_record_has_zero_dtype_byte():
    x = datagen.uniform_frame(300, seed=3)
    rec, _, _ = O.compress_s(x, O.grids_for(x, O.EB_ABS, 1e-3), 3)
    assert rec[53] == 0 and fmt_ref.parse(rec, arrays=False)["dtype"] == 0


# ------------------------------------------------------------------ streams
def run_stream(frames, eb_mode, eb, **kw):
    n = frames[0].shape[1]
    st = O.Stream(eb_mode, eb, max_n=n, dtype=O.DTYPE_I32, **kw)
    dst = O.Stream(eb_mode, eb, max_n=n, dtype=O.DTYPE_I32, **kw)
    for x in frames:
        rec, u, perm = st.compress(x)
        yield x, rec, u, perm, dst.decompress(rec)


@pytest.mark.parametrize("eb", [0.5, 4.0, 25.0])
def test_stream_bound(eb):
    frames = md_ints(frames=8)
    used = []
    for x, rec, u, perm, out in run_stream(frames, O.EB_ABS, eb, batch_size=4, block_log2=4):
        used.append(u)
        for f in range(3):
            err = np.abs(out[f].astype(np.int64) - x[f][perm].astype(np.int64))
            assert err.max() <= eb
            if eb < 1:
                assert err.max() == 0
    assert O.METHOD_T in used


def test_relative_bound_and_constant_field():
    frames = md_ints(frames=3)
    for x in frames:
        x[2][:] = 77  # one constant field: its relative bound is 0
    # a stream's relative bound is taken on its first frame
    eb0 = 1e-3 * float(int(frames[0][0].max()) - int(frames[0][0].min()))
    for x, rec, u, perm, out in run_stream(frames, O.EB_REL_PER_FIELD, 1e-3, batch_size=4,
                                           block_log2=4):
        P = fmt_ref.parse(rec, arrays=False)
        assert P["mode"] == 1 or P["grids"][2] == (77, 0)
        assert np.array_equal(out[2], x[2][perm])
        assert np.abs(out[0].astype(np.int64) - x[0][perm]).max() <= eb0


def test_anchor_scale_bound_and_fallback():
    frames = md_ints(frames=9, step=0.01)
    eb = 12.0
    scaled = 0
    for x, rec, u, perm, out in run_stream(frames, O.EB_ABS, eb, batch_size=4, block_log2=4,
                                           anchor_scale=5):
        P = fmt_ref.parse(rec, arrays=False)
        if P["mode"] == 0 and P["grids"][0][1] == 2:  # w = 5 = 25 / 5
            scaled += 1
        if P["mode"] == 1 and P["scale"] == 5:
            scaled += 1
        for f in range(3):
            assert np.abs(out[f].astype(np.int64) - x[f][perm].astype(np.int64)).max() <= eb
    assert scaled >= 2
    # eb = 1: bins of 3 integers cannot be split five ways: every record at eb
    for x, rec, u, perm, out in run_stream(frames[:5], O.EB_ABS, 1.0, batch_size=4,
                                           block_log2=4, anchor_scale=5):
        P = fmt_ref.parse(rec, arrays=False)
        assert P["scale"] == 1
        if P["mode"] == 0:
            assert P["grids"][0][1] == 1
        for f in range(3):
            assert np.abs(out[f].astype(np.int64) - x[f][perm].astype(np.int64)).max() <= 1


def test_stream_dtype_mismatch_refused():
    x = md_ints(frames=1)[0]
    st = O.Stream(O.EB_ABS, 2.0, max_n=x.shape[1], dtype=O.DTYPE_I32)
    rec, _, _ = st.compress(x)
    fl = O.Stream(O.EB_ABS, 2.0, max_n=x.shape[1])
    with pytest.raises(O.OracleError) as e:
        fl.decompress(rec)
    assert e.value.status == O.ERR_ARG


def test_search_k_on_integers():
    x = md_ints(n=3000, frames=1)[0]
    k, sizes = O.search_k(x, O.EB_ABS, 8.0)
    assert sizes[k] == min(int(v) for v in sizes if v)
    rec, _, _ = O.compress_s(x, O.grids_for(x, O.EB_ABS, 8.0), k)
    # the search samples every value here (n < 2^20): its size is the record's
    assert sizes[k] == len(rec)
