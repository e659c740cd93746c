"""Golden fixtures: a hand-worked example and oracle-written regression records."""
import json
import os
import struct

import numpy as np

import fmt_ref
import oracle as O

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_worked_example_by_hand():
    W = json.load(open(os.path.join(HERE, "worked_example.json")))
    x = np.array(W["x"], np.float32)
    grids = O.grids_for(x, O.EB_ABS, W["eb"])
    assert struct.pack(">f", grids[0].eb_q).hex() == W["eb_q_hex"]
    rec, perm, q = O.compress_s(x, grids, W["k"])
    assert list(perm) == W["perm"]
    assert len(rec) == W["total_bytes"]
    P = fmt_ref.parse(rec)
    assert list(P["bn"]) == W["bn"] and P["B"] == len(W["ids"])
    qs, ids, cnts, _ = fmt_ref.s_codes(rec)
    assert ids == W["ids"] and cnts == W["counts"]
    for d in range(3):
        assert [qs[d][s] for s in range(5)] == [W["q"][d][i] for i in W["perm"]]
    for a, (w, word) in enumerate(zip(W["widths"], W["words"])):
        dd = P["dirs"][a]
        assert dd["coder"] == 0 and dd["param"] == w and dd["nbytes"] == 4
        assert rec[dd["off"]:dd["off"] + 4] == struct.pack("<I", int(word, 16))


def test_golden_records_reproduce():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    for name, rec in mg.cases():
        stored = bytes.fromhex(open(os.path.join(HERE, name + ".hex")).read().strip())
        assert rec == stored, name
        fmt_ref.parse(stored)
