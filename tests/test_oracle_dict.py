"""Pins of the oracle's dictionary stage (order-0 rANS over coded bytes, the
last coding step of Sec. 6.2.2 and Sec. 7.1): hand-worked frequency tables,
the closed form of a constant block, the exact coding cost of rANS, round
trips over ragged blocks and the stream's own consistency checks."""
import math

import numpy as np
import pytest

import oracle as O

HDR = 4 + 4 + 8 + 2 * 256


def counts_of(pairs):
    c = np.zeros(256, np.uint64)
    for s, k in pairs.items():
        c[s] = k
    return c


def test_normalise_hand_cases():
    # 3 : 1 splits 4096 exactly
    f = O.dict_normalise(counts_of({0: 3, 1: 1}))
    assert f[0] == 3072 and f[1] == 1024 and f.sum() == 4096
    # one value takes everything
    f = O.dict_normalise(counts_of({200: 7}))
    assert f[200] == 4096 and f.sum() == 4096
    # three equal counts: 1365 each, the missing 1 to the smallest value
    f = O.dict_normalise(counts_of({5: 1, 9: 1, 2: 1}))
    assert (f[2], f[5], f[9]) == (1366, 1365, 1365)
    # 10,000 of one value and one each of 200 others: 4096 * 10000 // 10200 = 4015,
    # the others rounded up to 1 (200 in all), so 119 too many come off the largest
    c = counts_of({0: 10000, **{s: 1 for s in range(1, 201)}})
    f = O.dict_normalise(c)
    assert f[0] == 4015 - 119 and all(f[s] == 1 for s in range(1, 201)) and f.sum() == 4096
    # every byte value once: 16 each
    f = O.dict_normalise(np.ones(256, np.uint64))
    assert (f == 16).all()
    # nothing to code: no table
    assert O.dict_normalise(np.zeros(256, np.uint64)).sum() == 0


LANES = 64
STATE = bytes([0x00, 0x00, 0x80, 0x00])  # 2^23, little-endian
BLOCK_CONST = (4).to_bytes(2, "little") * LANES + STATE * LANES


def test_constant_block_closed_form():
    # one value at frequency 4096: x -> (x / 4096) * 4096 + x % 4096 = x, so every
    # lane's state stays at 2^23 and no byte is written; a block is 64 lane sizes
    # of 4 and 64 states (lanes without bytes keep the initial state too)
    for n in (1, 300, 4096):
        st = O.dict_encode(bytes([0x5A]) * n, block_log2=12)
        assert len(st) == HDR + 4 + len(BLOCK_CONST)
        assert st[:4] == (0x4450434C).to_bytes(4, "little")
        assert int.from_bytes(st[8:16], "little") == n
        assert int.from_bytes(st[16 + 2 * 0x5A:18 + 2 * 0x5A], "little") == 4096
        assert st[HDR:HDR + 4] == len(BLOCK_CONST).to_bytes(4, "little")
        assert st[HDR + 4:] == BLOCK_CONST
    # and the hand-built stream (two blocks) decodes to the bytes
    hand = bytearray(HDR + 8)
    hand[0:4] = (0x4450434C).to_bytes(4, "little")
    hand[4:8] = (12).to_bytes(4, "little")
    hand[8:16] = (4096 + 37).to_bytes(8, "little")
    hand[16 + 2 * 3:18 + 2 * 3] = (4096).to_bytes(2, "little")
    hand[HDR:HDR + 4] = len(BLOCK_CONST).to_bytes(4, "little")
    hand[HDR + 4:HDR + 8] = len(BLOCK_CONST).to_bytes(4, "little")
    hand += BLOCK_CONST * 2
    assert O.dict_decode(bytes(hand)) == bytes([3]) * (4096 + 37)


def test_coding_cost_is_the_table_cross_entropy():
    # rANS codes a byte of frequency f in log2(4096 / f) bits up to the state's
    # few bytes per lane: the payload is that sum over the input, within 4
    # bytes of state and 1 byte of rounding per lane (and the lanes' sizes)
    rng = np.random.default_rng(1)
    for p, n, bl in (([0.75, 0.125, 0.125], 300_000, 14), ([0.5] + [0.5 / 40] * 40, 123_457, 12)):
        data = rng.choice(len(p), size=n, p=p).astype(np.uint8)
        st = O.dict_encode(data.tobytes(), block_log2=bl)
        freq = np.frombuffer(st[16:HDR], np.uint16).astype(np.float64)
        counts = np.bincount(data, minlength=256)
        bits = sum(counts[s] * math.log2(4096 / freq[s]) for s in range(256) if counts[s])
        nb = (n + (1 << bl) - 1) >> bl
        payload = len(st) - HDR - 4 * nb - 2 * LANES * nb
        assert abs(payload - bits / 8) <= 5 * LANES * nb, (payload, bits / 8)
        assert O.dict_decode(st) == data.tobytes()


@pytest.mark.parametrize("n,bl", [(0, 12), (1, 12), (63, 12), (64, 12), (65, 12), (4097, 12),
                                  (70_001, 12), (1 << 16, 16), (300_001, 13)])
def test_round_trip_ragged_blocks(n, bl):
    rng = np.random.default_rng(n + bl)
    # runs of one value, a skewed range and uniform bytes, one after the other
    parts = [np.repeat(rng.integers(0, 256, max(1, n // 64), dtype=np.uint8), 16),
             rng.geometric(0.4, n).clip(0, 255).astype(np.uint8),
             rng.integers(0, 256, n, dtype=np.uint8)]
    data = np.concatenate(parts)[:n].tobytes()
    st = O.dict_encode(data, block_log2=bl)
    nb = (n + (1 << bl) - 1) >> bl
    assert len(st) <= O.dict_bound(n, bl)
    sizes = np.frombuffer(st[HDR:HDR + 4 * nb], np.uint32)
    assert len(st) == HDR + 4 * nb + int(sizes.sum())
    assert O.dict_decode(st) == data


def test_uniform_bytes_cost_eight_bits():
    # 256 values of frequency 16 each: 8 bits per byte
    data = np.random.default_rng(3).permutation(np.repeat(np.arange(256, dtype=np.uint8), 64))
    st = O.dict_encode(data.tobytes(), block_log2=14)
    assert abs((len(st) - HDR - 4 - 2 * LANES) - len(data)) <= 5 * LANES


def test_stream_checks():
    data = bytes(np.random.default_rng(4).integers(0, 5, 5000, dtype=np.uint8))
    st = bytearray(O.dict_encode(data, block_log2=12))
    with pytest.raises(O.OracleError):
        O.dict_decode(bytes(st[:-1]))  # a block cut short
    bad = bytearray(st)
    bad[0] ^= 1
    with pytest.raises(O.OracleError):
        O.dict_decode(bytes(bad))  # not a dictionary stream
    bad = bytearray(st)
    bad[16] ^= 1  # the frequencies no longer sum to 4096
    with pytest.raises(O.OracleError):
        O.dict_decode(bytes(bad))
