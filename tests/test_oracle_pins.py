"""Pins of the oracle that do not restate its own code.

* Quantisation grids: float32 bit patterns of eb_q worked by hand in exact
  arithmetic (tests/golden/grid_cases.json), across binades, a negative range,
  an all-zero field, and the eb-too-small boundary.
* Length-limited Huffman: two cases worked by hand, round by round
  (tests/golden/huffman_limit.json), checked against the oracle's lengths and
  against fmt_ref's independent two-queue builder, halving count included.
* Coder choice in both directions: fmt_ref recomputes the exact byte cost of
  both coders, and the oracle must pick the shorter, fixed on a tie.
* LCP-FSM (Sec. 7.2) and Alg. 1 with an unbounded batch: a stream built so that
  T wins, keeps winning, loses to S once, wins again, and S wins a comparison;
  the decision before every frame and the method used are written by hand.
"""
from __future__ import annotations

import json
import os
import struct

import numpy as np
import pytest

import fmt_ref
import oracle as O
from paper_2411_00761_amd import datagen

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def f32_hex(v) -> str:
    return struct.pack(">f", float(v)).hex()


# ------------------------------------------------------------------ grids
GRID = json.load(open(os.path.join(HERE, "grid_cases.json")))


@pytest.mark.parametrize("case", GRID["cases"], ids=lambda c: f"{c['lo']}:{c['hi']}:{c['eb']}")
def test_grid_bit_patterns_worked_by_hand(case):
    g = O.make_grid(np.float32(case["lo"]), np.float32(case["hi"]), case["eb"])
    assert g.E == case["E"]
    assert f32_hex(g.eb_q) == case["eb_q_hex"], case["derivation"]
    assert g.m == np.float32(case["lo"])
    # the bin width is 2 eb_q; its reciprocal is the one double rounding of 1/(2 eb_q)
    assert g.inv == 0.5 / float(g.eb_q)


@pytest.mark.parametrize("case", GRID["too_small"], ids=lambda c: str(c["eb"]))
def test_grid_eb_too_small_boundary(case):
    if case.get("ok"):
        O.make_grid(np.float32(case["lo"]), np.float32(case["hi"]), case["eb"])
    else:
        with pytest.raises(O.OracleError) as e:
            O.make_grid(np.float32(case["lo"]), np.float32(case["hi"]), case["eb"])
        assert e.value.status == O.ERR_EB_TOO_SMALL


# ------------------------------------------------------------------ Huffman length limit
LIMIT = json.load(open(os.path.join(HERE, "huffman_limit.json")))


@pytest.mark.parametrize("case", LIMIT["cases"], ids=lambda c: c["name"])
def test_length_limit_worked_by_hand(case):
    counts = np.zeros(O.ALPHABET, np.uint64)
    counts[: len(case["counts"])] = case["counts"]
    ln = O.huffman_lengths(counts)
    assert list(ln[: len(case["counts"])]) == case["lengths"]
    assert int(ln[len(case["counts"]):].sum()) == 0
    # the independent builder agrees, with the same number of halvings
    lengths, halvings = fmt_ref.huffman_lengths(dict(enumerate(case["counts"])))
    assert [lengths[s] for s in range(len(case["counts"]))] == case["lengths"]
    assert halvings == case["halvings"]


# ------------------------------------------------------------------ coder choice
def choice_cases():
    rng = np.random.default_rng(11)
    # exact tie: 42 values of 7 -> fixed 4 ceil(126/32) = 16 bytes; Huffman one
    # symbol of 1 bit: table 4 + one chunk offset 4 + 2 payload words 8 = 16
    yield "tie-fixed", np.full(42, 7, np.uint64), 10, 0
    # one value more: fixed 20 bytes, Huffman still 16
    yield "huffman-by-4", np.full(43, 7, np.uint64), 10, 1
    yield "skewed", np.where(rng.random(5000) < 0.85, 2, rng.integers(0, 200, 5000)).astype(np.uint64), 10, None
    yield "flat-8bit", rng.integers(0, 256, 5000).astype(np.uint64), 10, None
    yield "escapes", np.concatenate([np.zeros(3000, np.uint64),
                                     rng.integers(4096, 1 << 40, 300, dtype=np.uint64)]), 7, None
    yield "small-chunks", rng.geometric(0.4, 3000).astype(np.uint64), 5, None
    yield "wide", rng.integers(0, 1 << 62, 200, dtype=np.uint64), 10, None
    yield "two-values", rng.integers(0, 2, 999).astype(np.uint64) * 1000, 6, None


@pytest.mark.parametrize("name,v,cl,want", list(choice_cases()), ids=lambda x: x if isinstance(x, str) else "")
def test_coder_choice_both_directions(name, v, cl, want):
    fixed, huff, lengths = fmt_ref.coder_costs(v, cl)
    data, coder, param, used = O.encode_array(v, cl)
    expect = 1 if huff < fixed else 0  # the shorter coder; a tie keeps fixed
    if want is not None:
        assert expect == want, (fixed, huff)
    assert coder == expect, (name, fixed, huff)
    assert len(data) == (huff if coder else fixed)
    if coder:
        # the stored table is the independent builder's code
        tab = struct.unpack_from("<%dI" % used, data, 0)
        assert {e & 0xFFFF: e >> 16 for e in tab} == lengths
        assert param == max(lengths.values())
    else:
        assert param == (int(v.max()).bit_length() if len(v) else 0)


# ------------------------------------------------------------------ LCP-FSM trace
def fsm_stream_frames(n=2000):
    """Frames built for a known LCP-FSM path: four coherent trajectory frames,
    then an unrelated uniform frame (T against the previous frame is larger than
    the last S record, and larger than S), two small moves of it, two unrelated
    uniform frames, a third, and two small moves of that."""
    traj = datagen.MDTrajectory(n, step=0.001, seed=31)
    rng = np.random.default_rng(32)

    def rand():
        return rng.uniform(0.0, 12.0, size=(3, n)).astype(np.float32)

    def near(x):
        return (x + rng.normal(0.0, 0.001, size=x.shape)).astype(np.float32)

    fr = [traj.next_frame() for _ in range(4)]
    fr.append(rand())
    fr.append(near(fr[-1]))
    fr.append(near(fr[-1]))
    fr.append(rand())
    fr.append(rand())
    fr.append(rand())
    fr.append(near(fr[-1]))
    fr.append(near(fr[-1]))
    return fr


# The path, frame by frame, from the reading of Sec. 7.2 (S states S1X..S16X
# with a countdown of untested frames; a comparison runs both and the smaller
# wins, ties to S; in T, T runs and is kept while it is not larger than the
# last S record, else S runs too, the smaller is kept, and S returns to S1X):
#  0 no reference: S, counted as an S win        -> S2X, countdown 1
#  1 countdown 1: S                              -> countdown 0
#  2 countdown 0: compare, T smaller             -> T
#  3 T, not larger than the last S               -> T
#  4 T (unrelated frame) larger than last S; S runs and is smaller -> S1X, countdown 0
#  5 compare (small move of frame 4): T smaller  -> T
#  6 T kept                                      -> T
#  7 T loses (unrelated frame)                   -> S1X
#  8 compare (unrelated frame): S smaller        -> S2X, countdown 1
#  9 countdown 1: S                              -> countdown 0
# 10 compare (small move of frame 9): T smaller  -> T
# 11 T kept
FSM_DECISIONS = "S S C T T C T T C S C T".split()
FSM_METHODS = "S S T T S T T S S S T T".split()


def test_fsm_trace_written_by_hand():
    frames = fsm_stream_frames()
    st = O.Stream(O.EB_ABS, 1e-2, batch_size=0, block_log2=3, max_n=frames[0].shape[1])
    name = {O.DECIDE_S: "S", O.DECIDE_T: "T", O.DECIDE_COMPARE: "C"}
    decisions, methods, recs = [], [], []
    for x in frames:
        decisions.append(name[st.select()])
        rec, used, _ = st.compress(x)
        methods.append("S" if used == O.METHOD_S else "T")
        recs.append(rec)
    assert decisions == FSM_DECISIONS
    assert methods == FSM_METHODS
    # Alg. 1 with one unbounded batch: every temporal record refers to the frame
    # just before it
    for t, rec in enumerate(recs):
        P = fmt_ref.parse(rec, arrays=False)
        assert P["seq"] == t and P["mode"] == (1 if methods[t] == "T" else 0)
        if P["mode"] == 1:
            assert P["ref_seq"] == t - 1
