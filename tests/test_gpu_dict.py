"""GPU parity of the dictionary stage (order-0 rANS over coded bytes, the last
coding step of Sec. 6.2.2 and Sec. 7.1).

The GPU stream must equal the oracle's byte for byte, and decode (on the GPU)
to the input: skewed, uniform and constant bytes at ragged sizes and three
block sizes, the empty input, the records of an MD trajectory coded by the
library (one compress call), the oracle's own streams decoded on the GPU, and
the refusals (a damaged stream, a small output, small scratch).
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
    from paper_2411_00761_amd import lcp as L
    L.lib()
    return L


def sample(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "skewed":
        return rng.geometric(0.45, n).clip(1, 255).astype(np.uint8) - 1
    if kind == "uniform":
        return rng.integers(0, 256, n, dtype=np.uint8)
    if kind == "runs":
        return np.repeat(rng.integers(0, 8, n // 100 + 1, dtype=np.uint8), 100)[:n]
    return np.full(n, 0xA5, np.uint8)  # constant


def round_trip(lcp, data: np.ndarray, bl: int):
    print(f"case dict n={len(data)} block_log2={bl}", flush=True)
    dev = torch.from_numpy(data.copy() if len(data) else np.zeros(4, np.uint8)).cuda()
    out, size = lcp.dict_encode(dev, n=len(data), block_log2=bl)
    got = out[:size].cpu().numpy().tobytes()
    want = O.dict_encode(data.tobytes(), block_log2=bl)
    assert got == want, (len(got), len(want))
    dec = lcp.dict_decode(out, size, len(data), block_log2=bl)
    assert dec.cpu().numpy().tobytes() == data.tobytes()
    # the oracle's stream decodes on the GPU as well
    ost = torch.from_numpy(np.frombuffer(want, np.uint8).copy()).cuda()
    assert lcp.dict_decode(ost, len(want), len(data)).cpu().numpy().tobytes() == data.tobytes()
    return size


@pytest.mark.parametrize("kind", ["skewed", "uniform", "runs", "constant"])
@pytest.mark.parametrize("n,bl", [(1, 12), (4097, 12), (65_536 * 3 + 17, 12), (300_001, 16),
                                  (5_000, 13), (200_000, 20)])
def test_dict_parity(lcp, kind, n, bl):
    round_trip(lcp, sample(kind, n, n + bl), bl)


def test_dict_empty(lcp):
    assert round_trip(lcp, np.zeros(0, np.uint8), 12) == 4 + 4 + 8 + 512


def test_dict_of_trajectory_records(lcp):
    """The records of eight 2^22-particle frames of the MD trajectory, coded
    by one lcp_compress call, through the stage (the temporal records shrink a
    few percent: their Huffman streams are close to incompressible)."""
    n = 1 << 22
    traj = datagen.MDTrajectory(n, dims=(256, 128, 128), seed=2)
    frames = [torch.from_numpy(traj.next_frame()).cuda() for _ in range(8)]
    plan = lcp.Plan(1e-4, lcp.EB_REL_GLOBAL, multi_frame=True, batch_size=16, block_log2=12,
                    max_particles=n)
    out, offs, used, _ = plan.compress(frames)
    rec = out[:offs[-1]].cpu().numpy()
    size = round_trip(lcp, rec, 12)
    assert size < len(rec)


def test_dict_refusals(lcp):
    data = sample("skewed", 10_000, 5)
    dev = torch.from_numpy(data).cuda()
    with pytest.raises(lcp.LCPError) as e:  # the worst case must fit
        lcp.dict_encode(dev, block_log2=12,
                        out=torch.empty(100, dtype=torch.uint8, device="cuda"))
    assert e.value.status == lcp.ERR_CAPACITY
    with pytest.raises(lcp.LCPError) as e:
        lcp.dict_encode(dev, block_log2=12, scratch=torch.empty(256, dtype=torch.uint8,
                                                                 device="cuda"))
    assert e.value.status == lcp.ERR_BUDGET
    out, size = lcp.dict_encode(dev, block_log2=12)
    bad = out[:size].clone()
    bad[0] ^= 1  # not a dictionary stream
    with pytest.raises(lcp.LCPError) as e:
        lcp.dict_decode(bad, size, len(data))
    assert e.value.status == lcp.ERR_CORRUPT
    with pytest.raises(lcp.LCPError) as e:  # sizes that do not add up to the stream
        lcp.dict_decode(out, size - 1, len(data))
    assert e.value.status == lcp.ERR_CORRUPT
    bad = out[:size].clone()
    bad[16] ^= 1  # a table that does not sum to 4096
    with pytest.raises(lcp.LCPError) as e:
        lcp.dict_decode(bad, size, len(data))
    assert e.value.status == lcp.ERR_CORRUPT
    with pytest.raises(lcp.LCPError) as e:
        lcp.dict_decode(out, size, len(data), out=torch.empty(10, dtype=torch.uint8,
                                                               device="cuda"))
    assert e.value.status == lcp.ERR_CAPACITY


def test_dict_table_rules(lcp):
    """The normalisation's special rules on the GPU: a shortfall on a tie goes to
    the smaller value, an excess from many rare values comes off the largest
    frequency (the tables the oracle's pins work by hand)."""
    tie = np.array([5, 9, 2], np.uint8)
    round_trip(lcp, tie, 12)
    excess = np.concatenate([np.zeros(10_000, np.uint8), np.arange(1, 201, dtype=np.uint8)])
    excess = np.random.default_rng(9).permutation(excess)
    round_trip(lcp, excess, 12)
    # the stream's tables are the hand-worked ones
    out, size = lcp.dict_encode(torch.from_numpy(np.concatenate([tie, np.zeros(1, np.uint8)])).cuda(),
                                n=3, block_log2=12)
    f = np.frombuffer(out[16:16 + 512].cpu().numpy().tobytes(), np.uint16)
    assert (f[2], f[5], f[9]) == (1366, 1365, 1365)
    out, size = lcp.dict_encode(torch.from_numpy(excess).cuda(), block_log2=12)
    f = np.frombuffer(out[16:16 + 512].cpu().numpy().tobytes(), np.uint16)
    assert f[0] == 4015 - 119 and (f[1:201] == 1).all()
