"""Independent pure-Python reader of the LCP frame record (test helper).

Written from the record layout itself (header fields, grid slots, array
directory, fixed-length and chunked Huffman arrays), not from either implementation, so that a record written by the C oracle or by the GPU
library can be taken apart and checked field by field.  Slow: small inputs only.
"""
from __future__ import annotations

import struct

MAGIC = b"LCP1"
DIRECT = 4096
FIRST_CLASS_BITS = 13
MAX_LEN = 13


class Bits:
    """MSB-first reader over little-endian 32-bit words."""

    def __init__(self, data: bytes, start_word: int, end_word: int):
        self.words = struct.unpack_from("<%dI" % (end_word - start_word), data, 4 * start_word)
        self.pos = 0
        self.end = 32 * len(self.words)

    def bit(self) -> int:
        if self.pos >= self.end:
            raise ValueError("read past end")
        w = self.words[self.pos >> 5]
        b = (w >> (31 - (self.pos & 31))) & 1
        self.pos += 1
        return b

    def bits(self, n: int) -> int:
        v = 0
        for _ in range(n):
            v = (v << 1) | self.bit()
        return v


def canonical(lengths: dict[int, int]) -> dict[int, tuple[int, int]]:
    """symbol -> (code, length): shorter codes first, ties by symbol."""
    order = sorted(lengths, key=lambda s: (lengths[s], s))
    codes, code, prev = {}, 0, None
    for s in order:
        l = lengths[s]
        if prev is not None:
            code = (code + 1) << (l - prev)
        else:
            code = 0
        codes[s] = (code, l)
        prev = l
    return codes


def decode_array(data: bytes, n: int, coder: int, param: int, used: int, chunk_log2: int):
    if coder == 0:
        w = param
        nwords = (n * w + 31) // 32
        assert len(data) == 4 * nwords
        r = Bits(data, 0, nwords)
        return [r.bits(w) for _ in range(n)]
    assert coder == 1
    table = struct.unpack_from("<%dI" % used, data, 0)
    lengths = {}
    for e in table:
        assert e >> 24 == 0
        lengths[e & 0xFFFF] = (e >> 16) & 0xFF
    assert list(lengths) == sorted(lengths)
    assert max(lengths.values()) == param <= MAX_LEN
    codes = canonical(lengths)
    lookup = {(c, l): s for s, (c, l) in codes.items()}
    C = 1 << chunk_log2
    nchunks = (n + C - 1) // C
    ends = struct.unpack_from("<%dI" % nchunks, data, 4 * used)
    base = used + nchunks
    payload_words = len(data) // 4 - base
    assert len(data) % 4 == 0 and (nchunks == 0 or ends[-1] == payload_words)
    out, start = [], 0
    for c in range(nchunks):
        r = Bits(data, base + start, base + ends[c])
        for _ in range(min(C, n - c * C)):
            code, l = 0, 0
            while (code, l) not in lookup:
                code = (code << 1) | r.bit()
                l += 1
                assert l <= MAX_LEN
            s = lookup[(code, l)]
            if s < DIRECT:
                out.append(s)
            else:
                e = s - DIRECT + FIRST_CLASS_BITS - 1
                out.append((1 << e) + r.bits(e))
        start = ends[c]
    return out


def unzigzag(z: int) -> int:
    return -(z >> 1) - 1 if z & 1 else z >> 1


def parse(rec: bytes, arrays: bool = True) -> dict:
    """Header, grids, directory and (unless arrays is False) the decoded symbol
    arrays of one record."""
    assert rec[:4] == MAGIC
    version, mode, F, k, cl, A, flags, hdr = struct.unpack_from("<HBBBBBBI", rec, 4)
    n, B, total = struct.unpack_from("<QQQ", rec, 16)
    bn = struct.unpack_from("<3I", rec, 40)
    seq, ref_seq = struct.unpack_from("<QQ", rec, 56)
    assert version == 1 and total == len(rec) and hdr == 80 + 8 * F + 32 * A
    assert A == (F + 2 if mode == 0 else F)
    # byte 53: element type of the fields (0 float32, 1 int32); an int32 grid
    # slot holds the origin and the half width of the integer bins
    dtype = rec[53]
    assert dtype in (0, 1)
    grids = [struct.unpack_from("<iI" if dtype else "<ff", rec, 80 + 8 * f) for f in range(F)]
    want_arrays, arrays, dirs, off = arrays, [], [], hdr
    for a in range(A):
        coder, param, _r, used, an, aoff, anb = struct.unpack_from("<BBHIQQQ", rec, 80 + 8 * F + 32 * a)
        assert aoff == off
        dirs.append(dict(coder=coder, param=param, used=used, n=an, off=aoff, nbytes=anb))
        if want_arrays:
            arrays.append(decode_array(rec[aoff:aoff + anb], an, coder, param, used, cl))
        off += anb
    assert off == total
    # byte 11: the step of a temporal record's residuals (0 meaning 1); zero in S records
    assert (flags == 0) if mode == 0 else (flags == 0 or flags % 2 == 1)
    # byte 52: a spatial record's dimensions (0 meaning 3); zero in T records
    dims = rec[52] if rec[52] else 3
    assert rec[52] in (0, 1, 2) and (mode == 0 or rec[52] == 0)
    return dict(mode=mode, F=F, k=k, chunk_log2=cl, n=n, B=B, bn=bn, seq=seq, ref_seq=ref_seq,
                grids=grids, dirs=dirs, arrays=arrays, scale=flags if flags else 1, dims=dims,
                dtype=dtype)


def s_codes(rec: bytes):
    """Quantisation codes in slot order ([F][n] lists) of a spatial record, plus
    the block ids and counts: inverse delta coding, block expansion, corner +
    relative position."""
    P = parse(rec)
    assert P["mode"] == 0
    F, n, k, B = P["F"], P["n"], P["k"], P["B"]
    p = 1 << k
    bnx, bny, _ = P["bn"]
    ids, cnts, acc_id, acc_c = [], [], 0, 0
    for b in range(B):
        acc_id += P["arrays"][0][b]
        acc_c += unzigzag(P["arrays"][1][b])
        ids.append(acc_id)
        cnts.append(acc_c)
    D = P["dims"]
    q = [[0] * n for _ in range(F)]
    rel = [0, 0, 0]
    s = 0
    for b in range(B):
        i = ids[b]
        corner = (i % bnx, (i // bnx) % bny, i // (bnx * bny))
        for _ in range(cnts[b]):
            for d in range(D):
                rel[d] = (rel[d] + P["arrays"][2 + d][s]) % p
                q[d][s] = corner[d] * p + rel[d]
            s += 1
    assert s == n
    for f in range(D, F):
        q[f] = list(P["arrays"][2 + f])
    return q, ids, cnts, P


def t_codes(rec: bytes, ref_q):
    P = parse(rec)
    assert P["mode"] == 1
    return [[int(ref_q[f][s]) + unzigzag(P["arrays"][f][s]) for s in range(P["n"])]
            for f in range(P["F"])], P


# ------------------------------------------------------------------ coder cost
# The writer side of the array coding, for pins of the coder choice: symbols of
# values (values below 4096 are symbols themselves; a larger value is a length
# class followed by its bits below the leading one), length-limited Huffman
# lengths under the stated tie rules, and the exact byte cost of both coders.
def symbol(v: int) -> tuple[int, int]:
    """(symbol, raw bits after its code)."""
    if v < DIRECT:
        return v, 0
    b = v.bit_length()
    return DIRECT + b - FIRST_CLASS_BITS, b - 1


def huffman_lengths(counts: dict[int, int], limit: int = MAX_LEN) -> tuple[dict[int, int], int]:
    """symbol -> code length, and the number of halvings it took.  Leaves in
    (count, symbol) order; internal nodes queue in creation order; a merge takes
    the lighter head twice, the leaf when the two heads weigh the same."""
    cnt = {s: c for s, c in counts.items() if c > 0}
    halvings = 0
    while True:
        leaves = sorted(cnt, key=lambda s: (cnt[s], s))
        if len(leaves) == 1:
            return {leaves[0]: 1}, halvings
        weight = [cnt[s] for s in leaves]
        kids: list[tuple[int, int]] = []
        li, ii = 0, 0  # heads of the leaf queue and of the internal queue
        for _ in range(len(leaves) - 1):
            pair = []
            for _ in range(2):
                leaf_ok = li < len(leaves)
                int_ok = ii < len(kids)
                if leaf_ok and (not int_ok or weight[li] <= weight[len(leaves) + ii]):
                    pair.append(li)
                    li += 1
                else:
                    pair.append(len(leaves) + ii)
                    ii += 1
            weight.append(weight[pair[0]] + weight[pair[1]])
            kids.append((pair[0], pair[1]))
        depth = [0] * len(weight)
        for j in range(len(kids) - 1, -1, -1):  # root last: walk down from it
            node = len(leaves) + j
            for c in kids[j]:
                depth[c] = depth[node] + 1
        lengths = {leaves[i]: depth[i] for i in range(len(leaves))}
        if max(lengths.values()) <= limit:
            return lengths, halvings
        cnt = {s: (c + 1) // 2 for s, c in cnt.items()}
        halvings += 1


def coder_costs(values, chunk_log2: int) -> tuple[int, int, dict[int, int]]:
    """(fixed bytes, Huffman bytes, Huffman lengths) of one array: fixed =
    4 ceil(n w / 32) with w the bit width of the largest value; Huffman = 4 per
    table entry + 4 per chunk offset + 4 per payload word, each chunk of
    2^chunk_log2 values starting on a fresh word."""
    vals = [int(v) for v in values]
    n = len(vals)
    w = max(vals).bit_length() if n else 0
    fixed = 4 * ((n * w + 31) // 32)
    if n == 0:
        return fixed, 0, {}
    counts: dict[int, int] = {}
    for v in vals:
        s, _ = symbol(v)
        counts[s] = counts.get(s, 0) + 1
    lengths, _ = huffman_lengths(counts)
    C = 1 << chunk_log2
    words = 0
    for c0 in range(0, n, C):
        bits = 0
        for v in vals[c0:c0 + C]:
            s, e = symbol(v)
            bits += lengths[s] + e
        words += (bits + 31) // 32
    nchunks = (n + C - 1) // C
    return fixed, 4 * len(lengths) + 4 * nchunks + 4 * words, lengths
