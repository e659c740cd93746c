"""Pins of the oracle's spatial coder on data of fewer dimensions (Sec. 4: the
design carries over to other dimensions; Eq. 6 over the D spatial axes).

* Brute force in exact arithmetic on small frames of D = 1 and 2 spatial
  dimensions, with and without supplementary fields: every code is the exact
  Eq. 5 floor; block ids follow Eq. 6 over the D axes; the order is numpy's
  stable sort of the ids; absent axes count one block; the header carries D.
* D = 3 given explicitly is the plain record byte for byte.
* Round trips: every decoded value within eb, spatial and temporal frames.
"""
from __future__ import annotations

import math
from fractions import Fraction as fr

import numpy as np
import pytest

import fmt_ref
import oracle as O


def exact_floor_bin(x, g):
    return math.floor((fr(float(x)) - fr(float(g.m))) / (2 * fr(float(g.eb_q))))


@pytest.mark.parametrize("D,F,n,k,seed", [(2, 2, 60, 2, 1), (2, 4, 90, 3, 2), (1, 1, 70, 2, 3),
                                          (1, 3, 50, 0, 4), (2, 2, 200, 16, 5)])
def test_low_dimensional_record_brute_force(D, F, n, k, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 10.0, size=(F, n)).astype(np.float32)
    x[:, 7] = x[:, 3]  # a repeated point
    grids = O.grids_for(x, O.EB_ABS, 0.05)
    rec, perm, q = O.compress_s(x, grids, k, dims=D)
    assert rec[52] == (0 if D == 3 else D)
    qs, ids, cnts, P = fmt_ref.s_codes(rec)
    assert P["dims"] == D and P["F"] == F and len(P["arrays"]) == F + 2
    for s in range(n):
        for f in range(F):
            assert qs[f][s] == exact_floor_bin(x[f][perm[s]], grids[f]) == q[f][s]
    bn = [(exact_floor_bin(x[d].max(), grids[d]) >> k) + 1 if d < D else 1 for d in range(3)]
    assert list(P["bn"]) == bn
    blocks = [[exact_floor_bin(x[d][i], grids[d]) >> k for d in range(D)] + [0] * (3 - D)
              for i in range(n)]
    keys = np.array([b[0] + bn[0] * (b[1] + bn[1] * b[2]) for b in blocks], np.int64)
    assert np.array_equal(perm, np.argsort(keys, kind="stable"))
    u, c = np.unique(keys, return_counts=True)
    assert list(u) == ids and list(c) == cnts
    out, _ = O.decompress(rec)
    for f in range(F):
        err = max(abs(fr(float(out[f][s])) - fr(float(x[f][perm[s]]))) for s in range(n))
        assert err <= fr(0.05)


def test_three_dimensions_explicit_is_plain():
    rng = np.random.default_rng(9)
    x = rng.uniform(0.0, 10.0, size=(4, 300)).astype(np.float32)
    grids = O.grids_for(x, O.EB_ABS, 0.01)
    a = O.compress_s(x, grids, 3)[0]
    b = O.compress_s(x, grids, 3, dims=3)[0]
    assert a == b and a[52] == 0


def test_dimension_refusals():
    x = np.zeros((2, 10), np.float32)
    grids = O.grids_for(x, O.EB_ABS, 0.1)
    with pytest.raises(O.OracleError):
        O.compress_s(x, grids, 2, dims=3)  # fewer fields than dimensions
    rng = np.random.default_rng(1)
    y = rng.uniform(0, 1, size=(2, 40)).astype(np.float32)
    rec = bytearray(O.compress_s(y, O.grids_for(y, O.EB_ABS, 0.01), 2, dims=2)[0])
    rec[52] = 3  # 3 is written as 0
    with pytest.raises(O.OracleError):
        O.record_info(bytes(rec))


@pytest.mark.parametrize("D,F", [(2, 2), (1, 2)])
def test_low_dimensional_stream_round_trip(D, F):
    rng = np.random.default_rng(20 + D)
    n = 2000
    x = rng.uniform(0.0, 50.0, size=(F, n)).astype(np.float32)
    frames = [x]
    for _ in range(7):
        frames.append((frames[-1] + rng.normal(0, 0.002, size=x.shape)).astype(np.float32))
    st = O.Stream(O.EB_ABS, 0.01, n_fields=F, batch_size=4, block_log2=3, max_n=n, n_dims=D)
    dst = O.Stream(O.EB_ABS, 0.01, n_fields=F, batch_size=4, block_log2=3, max_n=n, n_dims=D)
    methods = []
    for f_ in frames:
        rec, used, perm = st.compress(f_)
        methods.append(used)
        out = dst.decompress(rec)
        for f in range(F):
            assert np.abs(out[f].astype(np.float64) - f_[f][perm].astype(np.float64)).max() <= 0.01
    assert O.METHOD_T in methods and O.METHOD_S in methods
