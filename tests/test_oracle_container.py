"""Pins of the oracle's multi-frame container (Sec. 7.3, Alg. 1) that do not
restate its code.

* Layout: the anchors (first-in-batch frames coded by LCP-S) sit in an array of
  their own after the batches; every record is stored once, byte for byte; the
  sizes add up.
* Closures written by hand from the stream's known methods: a frame needs its
  references back to a spatial frame, and never more than the frames of its
  batch up to it plus one anchor (the paper's worst case).
* Retrieval of any set of frames, in any order, gives bit for bit the frames a
  plain sequential decode of the whole stream gives, and decodes as many
  records as the hand-counted closures.
"""
from __future__ import annotations

import struct

import numpy as np
import pytest

import oracle as O
from test_oracle_anchor_scale import GATE_METHODS, gate_stream_frames

B = 4
EB = 0.01


@pytest.fixture(scope="module")
def stream():
    frames = gate_stream_frames(1500)
    st = O.Stream(O.EB_ABS, EB, batch_size=B, block_log2=3, max_n=1500, anchor_scale=5)
    recs = [st.compress(x)[0] for x in frames]
    dst = O.Stream(O.EB_ABS, EB, batch_size=B, block_log2=3, max_n=1500, anchor_scale=5)
    seq = [dst.decompress(r) for r in recs]
    return frames, recs, seq


def test_layout(stream):
    _, recs, _ = stream
    cont = O.container_pack(recs, B)
    n, batch, ents = O.container_entries(cont)
    assert n == len(recs) and batch == B
    # anchors by hand: frames 0, 8 and 12 are first in their batch and spatial
    anchors = [j for j, e in enumerate(ents) if e[5]]
    assert anchors == [0, 8, 12]
    assert struct.unpack_from("<Q", cont, 24)[0] == 3
    table_end = 64 + 32 * n
    a_off = struct.unpack_from("<Q", cont, 40)[0]
    assert struct.unpack_from("<Q", cont, 48)[0] == len(cont) == table_end + sum(map(len, recs))
    # batches in stream order, anchors after them, each record once
    pos = table_end
    for j in [j for j in range(n) if j not in anchors] + anchors:
        if j == anchors[0]:
            assert pos == a_off
        assert ents[j][0] == pos and ents[j][1] == len(recs[j])
        assert cont[pos:pos + len(recs[j])] == recs[j]
        pos += len(recs[j])
    assert [e[4] for e in ents] == [0 if m == "S" else 1 for m in GATE_METHODS]


# From the methods S S T T | T T T T | S S S S | S (batch 4): frames 2, 3 refer
# to the frame before; frame 4 (a batch start coded by T) to anchor 0; 5-7 to
# the frame before; 8-12 are spatial.
CLOSURES = {0: [0], 1: [1], 2: [1, 2], 3: [1, 2, 3], 4: [0, 4], 5: [0, 4, 5], 7: [0, 4, 5, 6, 7],
            8: [8], 11: [11], 12: [12]}


def test_closures_by_hand(stream):
    _, recs, _ = stream
    cont = O.container_pack(recs, B)
    for k, want in CLOSURES.items():
        assert O.container_closure(cont, k) == want, k
    for k in range(len(recs)):
        assert len(O.container_closure(cont, k)) <= k % B + 2  # batch up to k plus one anchor


@pytest.mark.parametrize("req,decoded", [([7], 5), ([12, 3, 5], 1 + 6), ([3, 2, 1], 3 + 2 + 1),
                                         ([0, 4, 7, 8, 12], 7), (list(range(13)), 13)])
def test_retrieval_equals_sequential_decode(stream, req, decoded):
    _, recs, seq = stream
    cont = O.container_pack(recs, B)
    out, count = O.container_retrieve(cont, req, O.EB_ABS, EB, block_log2=3, anchor_scale=5)
    assert count == decoded
    assert sorted(out) == sorted(set(req))
    for k in req:
        for f in range(3):
            assert np.array_equal(out[k][f].view(np.uint32), seq[k][f].view(np.uint32)), (k, f)


def test_refusals(stream):
    _, recs, _ = stream
    with pytest.raises(O.OracleError) as e:
        O.container_pack([recs[1], recs[0]], B)  # not one stream from its start
    assert e.value.status == O.ERR_ARG
    cont = bytearray(O.container_pack(recs, B))
    with pytest.raises(O.OracleError):
        O.container_closure(bytes(cont), 13)
    cont[0] ^= 1
    with pytest.raises(O.OracleError) as e:
        O.container_closure(bytes(cont), 3)
    assert e.value.status == O.ERR_CORRUPT
