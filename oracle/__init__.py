"""ctypes binding of the plain-C LCP oracle (lcp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the benchmark's
CPU-baseline leg.  The product library never imports this package and shares no
code with it.  Every function here only marshals numpy arrays to the C oracle.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lcp_oracle.c")
_LIB = os.path.join(_HERE, "liblcp_oracle.so")

OK, ERR_ARG, ERR_EB_TOO_SMALL, ERR_RANGE, ERR_CAPACITY, ERR_CORRUPT, ERR_NO_REFERENCE = range(7)
EB_ABS, EB_REL_GLOBAL, EB_REL_PER_FIELD = 0, 1, 2
METHOD_AUTO, METHOD_S, METHOD_T = 0, 1, 2
DECIDE_S, DECIDE_T, DECIDE_COMPARE = 1, 2, 3
DTYPE_F32, DTYPE_I32 = 0, 1
MAX_F = 8
ALPHABET = 4148


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "lcp_oracle.h"))
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-shared",
             "-fPIC", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("eb_mode", C.c_int), ("eb", C.c_double), ("n_fields", C.c_int),
                ("multi_frame", C.c_int), ("batch_size", C.c_int), ("block_log2", C.c_int),
                ("chunk_log2", C.c_int), ("anchor_scale", C.c_int), ("n_dims", C.c_int),
                ("dtype", C.c_int)]


class Grid(C.Structure):
    _fields_ = [("m", C.c_float), ("eb_q", C.c_float), ("inv", C.c_double),
                ("eb", C.c_double), ("E", C.c_int), ("dtype", C.c_int), ("mi", C.c_int32),
                ("hb", C.c_int64)]


class Info(C.Structure):
    _fields_ = [("mode", C.c_int), ("F", C.c_int), ("k", C.c_int), ("chunk_log2", C.c_int),
                ("n_arrays", C.c_int), ("n", C.c_uint64), ("B", C.c_uint64),
                ("total_bytes", C.c_uint64), ("seq", C.c_uint64), ("ref_seq", C.c_uint64),
                ("bn", C.c_uint32 * 3), ("m", C.c_float * MAX_F), ("eb_q", C.c_float * MAX_F),
                ("coder", C.c_int * (MAX_F + 2)), ("param", C.c_int * (MAX_F + 2)),
                ("used", C.c_uint32 * (MAX_F + 2)), ("arr_n", C.c_uint64 * (MAX_F + 2)),
                ("arr_off", C.c_uint64 * (MAX_F + 2)), ("arr_bytes", C.c_uint64 * (MAX_F + 2)),
                ("scale", C.c_int), ("dims", C.c_int), ("dtype", C.c_int),
                ("mi", C.c_int32 * MAX_F), ("hb", C.c_int64 * MAX_F)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        P = C.c_void_p
        L.lco_extent.argtypes = [P, C.c_int, C.c_uint64, C.c_int, P, P]
        L.lco_field_eb.argtypes = [C.c_int, C.c_double, C.c_int, P, P, C.c_int, P]
        L.lco_make_grid.argtypes = [C.c_float, C.c_float, C.c_double, C.POINTER(Grid)]
        L.lco_make_grid_i.argtypes = [C.c_int32, C.c_double, C.c_int, C.POINTER(Grid)]
        L.lco_quant.argtypes = [C.c_float, C.POINTER(Grid)]
        L.lco_quant.restype = C.c_int64
        L.lco_recon.argtypes = [C.c_int64, C.POINTER(Grid)]
        L.lco_recon.restype = C.c_float
        L.lco_quant_i.argtypes = [C.c_int32, C.POINTER(Grid)]
        L.lco_quant_i.restype = C.c_int64
        L.lco_recon_i.argtypes = [C.c_int64, C.POINTER(Grid)]
        L.lco_recon_i.restype = C.c_int32
        L.lco_quantize.argtypes = [P, C.c_uint64, C.POINTER(Grid), P]
        L.lco_quantize.restype = None
        L.lco_reconstruct.argtypes = [P, C.c_uint64, C.POINTER(Grid), P]
        L.lco_reconstruct.restype = None
        L.lco_huffman_lengths.argtypes = [P, C.c_int, P]
        L.lco_encode_array.argtypes = [P, C.c_uint64, C.c_int, P, C.c_uint64,
                                       C.POINTER(C.c_uint64), C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), C.POINTER(C.c_uint32)]
        L.lco_decode_array.argtypes = [P, C.c_uint64, C.c_uint64, C.c_int, C.c_int,
                                       C.c_uint32, C.c_int, P]
        L.lco_compress_s.argtypes = [P, C.c_int, C.c_int, C.c_uint64, P, C.c_int, C.c_int, C.c_uint64,
                                     P, C.c_uint64, C.POINTER(C.c_uint64), P, P]
        L.lco_compress_t.argtypes = [P, C.c_int, C.c_uint64, P, P, P, C.c_uint64, C.c_int,
                                     C.c_int, C.c_uint64, P, C.c_uint64, C.POINTER(C.c_uint64),
                                     P]
        L.lco_record_info.argtypes = [P, C.c_uint64, C.POINTER(Info)]
        L.lco_container_pack.argtypes = [P, P, C.c_uint64, C.c_int, P, C.c_uint64,
                                         C.POINTER(C.c_uint64)]
        L.lco_container_closure.argtypes = [P, C.c_uint64, C.c_uint64, P, C.c_uint64,
                                            C.POINTER(C.c_uint64)]
        L.lco_decompress.argtypes = [P, C.c_uint64, P, C.c_uint64, C.c_uint64, P, C.c_uint64,
                                     C.POINTER(C.c_uint64), P]
        L.lco_stream_create.argtypes = [C.POINTER(Params), C.c_uint64]
        L.lco_stream_create.restype = P
        L.lco_stream_destroy.argtypes = [P]
        L.lco_stream_destroy.restype = None
        L.lco_stream_select.argtypes = [P, C.POINTER(C.c_int)]
        L.lco_stream_compress.argtypes = [P, P, C.c_uint64, C.c_int, P, C.c_uint64,
                                          C.POINTER(C.c_uint64), C.POINTER(C.c_int), P]
        L.lco_stream_decompress.argtypes = [P, P, C.c_uint64, P, C.c_uint64,
                                            C.POINTER(C.c_uint64)]
        L.lco_search_k.argtypes = [P, C.c_int, C.c_uint64, C.POINTER(Params),
                                   C.POINTER(C.c_int), P]
        L.lco_bound.argtypes = [C.c_int, C.c_uint64, C.c_int]
        L.lco_bound.restype = C.c_uint64
        L.lco_dict_bound.argtypes = [C.c_uint64, C.c_int]
        L.lco_dict_bound.restype = C.c_uint64
        L.lco_dict_normalise.argtypes = [P, P]
        L.lco_dict_encode.argtypes = [P, C.c_uint64, C.c_int, P, C.c_uint64,
                                      C.POINTER(C.c_uint64)]
        L.lco_dict_decode.argtypes = [P, C.c_uint64, P, C.c_uint64, C.POINTER(C.c_uint64)]
    return _lib


def _check(st: int, what: str):
    if st != OK:
        raise OracleError(st, what)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def dtype_of(fields) -> int:
    """DTYPE_I32 for int32 fields, DTYPE_F32 otherwise (converted to float32)."""
    return DTYPE_I32 if np.asarray(fields[0]).dtype == np.int32 else DTYPE_F32


def _fields(fields):
    """Contiguous float32 (or int32) arrays + a C array of their pointers (kept alive)."""
    dt = np.int32 if dtype_of(fields) == DTYPE_I32 else np.float32
    arrs = [np.ascontiguousarray(f, dtype=dt) for f in fields]
    ptrs = (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    return arrs, ptrs


def _grids(grids):
    arr = (Grid * len(grids))()
    for i, g in enumerate(grids):
        arr[i] = g
    return arr


# ---------------------------------------------------------------- steps
def extent(fields):
    """Per-field minima and maxima as float64 (exact for either type)."""
    arrs, ptrs = _fields(fields)
    F = len(arrs)
    lo = np.zeros(F, np.float64)
    hi = np.zeros(F, np.float64)
    _check(lib().lco_extent(ptrs, F, len(arrs[0]), dtype_of(fields), _ptr(lo), _ptr(hi)),
           "extent")
    return lo, hi


def field_eb(eb_mode, eb, lo, hi, dtype=DTYPE_F32):
    F = len(lo)
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    out = np.zeros(F, np.float64)
    _check(lib().lco_field_eb(eb_mode, eb, F, _ptr(lo), _ptr(hi), dtype, _ptr(out)), "field_eb")
    return out


def make_grid(lo, hi, eb_f) -> Grid:
    g = Grid()
    _check(lib().lco_make_grid(float(lo), float(hi), float(eb_f), C.byref(g)), "make_grid")
    return g


def make_grid_i(lo, eb_f, s=1) -> Grid:
    g = Grid()
    _check(lib().lco_make_grid_i(int(lo), float(eb_f), s, C.byref(g)), "make_grid_i")
    return g


def quant_i(x, g: Grid) -> int:
    return int(lib().lco_quant_i(int(x), C.byref(g)))


def recon_i(q, g: Grid) -> int:
    return int(lib().lco_recon_i(int(q), C.byref(g)))


def quantize(x, g: Grid) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    q = np.zeros(len(x), np.int64)
    lib().lco_quantize(_ptr(x), len(x), C.byref(g), _ptr(q))
    return q


def reconstruct(q, g: Grid) -> np.ndarray:
    q = np.ascontiguousarray(q, np.int64)
    out = np.zeros(len(q), np.float32)
    lib().lco_reconstruct(_ptr(q), len(q), C.byref(g), _ptr(out))
    return out


def huffman_lengths(counts) -> np.ndarray:
    c = np.ascontiguousarray(counts, np.uint64)
    ln = np.zeros(len(c), np.uint8)
    lib().lco_huffman_lengths(_ptr(c), len(c), _ptr(ln))
    return ln


def encode_array(values, chunk_log2=10):
    v = np.ascontiguousarray(values, np.uint64)
    nb, coder, param, used = C.c_uint64(), C.c_int(), C.c_int(), C.c_uint32()
    L = lib()
    _check(L.lco_encode_array(_ptr(v), len(v), chunk_log2, None, 0, C.byref(nb),
                              C.byref(coder), C.byref(param), C.byref(used)), "encode size")
    out = np.zeros(max(nb.value, 1), np.uint8)
    _check(L.lco_encode_array(_ptr(v), len(v), chunk_log2, _ptr(out), nb.value, C.byref(nb),
                              C.byref(coder), C.byref(param), C.byref(used)), "encode")
    return out[: nb.value].tobytes(), coder.value, param.value, used.value


def decode_array(data: bytes, n, coder, param, used, chunk_log2=10) -> np.ndarray:
    buf = np.frombuffer(data, np.uint8).copy() if len(data) else np.zeros(1, np.uint8)
    v = np.zeros(max(n, 1), np.uint64)
    _check(lib().lco_decode_array(_ptr(buf), len(data), n, coder, param, used, chunk_log2,
                                  _ptr(v)), "decode_array")
    return v[:n]


def bound(F, n, chunk_log2=10) -> int:
    return int(lib().lco_bound(F, n, chunk_log2))


def grids_for(fields, eb_mode, eb, s=1):
    """Grids of a frame (float32 grids at eb / s, int32 grids with step s)."""
    lo, hi = extent(fields)
    dt = dtype_of(fields)
    ebf = field_eb(eb_mode, eb, lo, hi, dt)
    if dt == DTYPE_I32:
        return [make_grid_i(int(lo[f]), ebf[f], s) for f in range(len(fields))]
    return [make_grid(lo[f], hi[f], ebf[f] / s) for f in range(len(fields))]


def compress_s(fields, grids, k, chunk_log2=10, seq=0, dims=3):
    arrs, ptrs = _fields(fields)
    F, n = len(arrs), len(arrs[0])
    cap = bound(F, n, chunk_log2)
    out = np.zeros(cap, np.uint8)
    perm = np.zeros(n, np.uint32)
    q = np.zeros((F, n), np.int32)
    size = C.c_uint64()
    _check(lib().lco_compress_s(ptrs, F, dims, n, _grids(grids), k, chunk_log2, seq, _ptr(out), cap,
                                C.byref(size), _ptr(perm), _ptr(q)), "compress_s")
    return out[: size.value].tobytes(), perm, q


def compress_t(fields, grids, ref_perm, ref_q, ref_seq, chunk_log2=10, seq=1, scale=1):
    arrs, ptrs = _fields(fields)
    F, n = len(arrs), len(arrs[0])
    cap = bound(F, n, chunk_log2)
    out = np.zeros(cap, np.uint8)
    q = np.zeros((F, n), np.int32)
    rp = np.ascontiguousarray(ref_perm, np.uint32)
    rq = np.ascontiguousarray(ref_q, np.int32)
    size = C.c_uint64()
    _check(lib().lco_compress_t(ptrs, F, n, _grids(grids), _ptr(rp), _ptr(rq), ref_seq, scale,
                                chunk_log2, seq, _ptr(out), cap, C.byref(size), _ptr(q)),
           "compress_t")
    return out[: size.value].tobytes(), q


def record_info(rec: bytes) -> Info:
    buf = np.frombuffer(rec, np.uint8).copy()
    info = Info()
    _check(lib().lco_record_info(_ptr(buf), len(rec), C.byref(info)), "record_info")
    return info


def _out_dtype(info):
    return np.int32 if info.dtype == DTYPE_I32 else np.float32


def decompress(rec: bytes, ref_q=None, ref_seq=0):
    """Returns (fields [F][n] float32 or int32 in slot order, q [F][n] int32)."""
    info = record_info(rec)
    F, n = info.F, info.n
    buf = np.frombuffer(rec, np.uint8).copy()
    outs = [np.zeros(n, _out_dtype(info)) for _ in range(F)]
    optrs = (C.c_void_p * F)(*[o.ctypes.data for o in outs])
    q = np.zeros((F, n), np.int32)
    nout = C.c_uint64()
    if ref_q is not None:
        rq = np.ascontiguousarray(ref_q, np.int32)
        rqp, rn = _ptr(rq), rq.shape[1]
    else:
        rqp, rn = None, 0
    _check(lib().lco_decompress(_ptr(buf), len(rec), rqp, ref_seq, rn, optrs, n, C.byref(nout),
                                _ptr(q)), "decompress")
    return outs, q


def search_k(fields, eb_mode, eb, chunk_log2=10, dims=3):
    arrs, ptrs = _fields(fields)
    p = Params(eb_mode, eb, len(arrs), 0, 0, 0, chunk_log2, 0, dims, dtype_of(fields))
    k = C.c_int()
    sizes = np.zeros(17, np.uint64)
    _check(lib().lco_search_k(ptrs, len(arrs), len(arrs[0]), C.byref(p), C.byref(k),
                              _ptr(sizes)), "search_k")
    return k.value, sizes


class Stream:
    """Alg. 1 multi-frame driver with LCP-FSM (compress and decompress sides)."""

    def __init__(self, eb_mode, eb, n_fields=3, multi_frame=1, batch_size=16, block_log2=4,
                 chunk_log2=10, max_n=1 << 20, anchor_scale=0, n_dims=0, dtype=DTYPE_F32):
        self.p = Params(eb_mode, eb, n_fields, multi_frame, batch_size, block_log2, chunk_log2,
                        anchor_scale, n_dims, dtype)
        self.F = n_fields
        self.max_n = max_n
        self.h = lib().lco_stream_create(C.byref(self.p), max_n)
        if not self.h:
            raise OracleError(ERR_ARG, "stream_create")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().lco_stream_destroy(h)
            self.h = None

    def select(self) -> int:
        d = C.c_int()
        _check(lib().lco_stream_select(self.h, C.byref(d)), "select")
        return d.value

    def compress(self, fields, method=METHOD_AUTO):
        arrs, ptrs = _fields(fields)
        n = len(arrs[0])
        cap = bound(self.F, n, self.p.chunk_log2)
        out = np.zeros(cap, np.uint8)
        size, used = C.c_uint64(), C.c_int()
        perm = np.zeros(n, np.uint32)
        _check(lib().lco_stream_compress(self.h, ptrs, n, method, _ptr(out), cap, C.byref(size),
                                         C.byref(used), _ptr(perm)), "stream_compress")
        return out[: size.value].tobytes(), used.value, perm

    def decompress(self, rec: bytes):
        info = record_info(rec)
        buf = np.frombuffer(rec, np.uint8).copy()
        outs = [np.zeros(info.n, _out_dtype(info)) for _ in range(info.F)]
        optrs = (C.c_void_p * info.F)(*[o.ctypes.data for o in outs])
        nout = C.c_uint64()
        _check(lib().lco_stream_decompress(self.h, _ptr(buf), len(rec), optrs, info.n,
                                           C.byref(nout)), "stream_decompress")
        return outs


# ---------------------------------------------------------------- container (Sec. 7.3)
CONTAINER_HDR, CONTAINER_ENTRY = 64, 32


def container_pack(records, batch_size: int) -> bytes:
    """Records of one stream (frames 0..n-1 in order) packed for random access."""
    bufs = [np.frombuffer(r, np.uint8).copy() for r in records]
    n = len(bufs)
    ptrs = (C.c_void_p * n)(*[b.ctypes.data for b in bufs])
    sizes = np.array([len(r) for r in records], np.uint64)
    size = C.c_uint64()
    _check(lib().lco_container_pack(ptrs, _ptr(sizes), n, batch_size, None, 0, C.byref(size)),
           "container_pack")
    out = np.zeros(size.value, np.uint8)
    _check(lib().lco_container_pack(ptrs, _ptr(sizes), n, batch_size, _ptr(out), size.value,
                                    C.byref(size)), "container_pack")
    return out.tobytes()


def container_closure(cont: bytes, k: int):
    buf = np.frombuffer(cont, np.uint8).copy()
    frames = np.zeros(1 << 16, np.uint64)
    count = C.c_uint64()
    _check(lib().lco_container_closure(_ptr(buf), len(cont), k, _ptr(frames), len(frames),
                                       C.byref(count)), "container_closure")
    return [int(v) for v in frames[: count.value]]


def container_entries(cont: bytes):
    """(frames, batch_size, [(offset, size, ref_seq, n, mode, anchor)])"""
    import struct
    n = struct.unpack_from("<Q", cont, 16)[0]
    batch = struct.unpack_from("<I", cont, 8)[0]
    ents = [struct.unpack_from("<QQQIBB", cont, CONTAINER_HDR + CONTAINER_ENTRY * j)
            for j in range(n)]
    return n, batch, ents


def container_passes(frames):
    """Requests in the caller's order, split into passes of increasing frame
    numbers: each pass decodes the union of its requests' closures in stream
    order on a fresh decoder."""
    passes, cur = [], []
    for k in frames:
        if cur and k <= cur[-1]:
            passes.append(cur)
            cur = []
        cur.append(k)
    if cur:
        passes.append(cur)
    return passes


def container_retrieve(cont: bytes, frames, eb_mode, eb, n_fields=3, block_log2=4,
                       anchor_scale=0, dtype=DTYPE_F32):
    """{frame: decoded fields [F][n] in slot order} for the requested frames, and
    the number of records decoded."""
    n, batch, ents = container_entries(cont)
    out, decoded = {}, 0
    for ps in container_passes(frames):
        need = sorted(set(j for k in ps for j in container_closure(cont, k)))
        st = Stream(eb_mode, eb, n_fields=n_fields, batch_size=batch, block_log2=block_log2,
                    max_n=max(e[3] for e in ents), anchor_scale=anchor_scale, dtype=dtype)
        for j in need:
            off, size = ents[j][0], ents[j][1]
            dec = st.decompress(cont[off:off + size])
            decoded += 1
            if j in ps:
                out[j] = dec
    return out, decoded


# ---- dictionary stage: order-0 rANS over bytes (lcp_oracle.h) ----
DICT_MAGIC = 0x4450434C


def dict_normalise(counts) -> np.ndarray:
    """Byte counts [256] -> frequencies [256] summing to 4096 (0 for absent values)."""
    c = np.ascontiguousarray(counts, np.uint64)
    assert c.shape == (256,)
    f = np.zeros(256, np.uint16)
    _check(lib().lco_dict_normalise(_ptr(c), _ptr(f)), "lco_dict_normalise")
    return f


def dict_bound(n: int, block_log2: int = 12) -> int:
    return int(lib().lco_dict_bound(n, block_log2))


def dict_encode(data: bytes, block_log2: int = 12) -> bytes:
    a = np.frombuffer(bytes(data), np.uint8)
    cap = dict_bound(len(a), block_log2)
    out = np.zeros(max(cap, 1), np.uint8)
    size = C.c_uint64(0)
    _check(lib().lco_dict_encode(_ptr(a) if len(a) else None, len(a), block_log2, _ptr(out), cap,
                                 C.byref(size)), "lco_dict_encode")
    return out[:size.value].tobytes()


def dict_decode(stream: bytes) -> bytes:
    a = np.frombuffer(bytes(stream), np.uint8)
    n = int(np.frombuffer(a[8:16].tobytes(), np.uint64)[0]) if len(a) >= 16 else 0
    out = np.zeros(max(n, 1), np.uint8)
    got = C.c_uint64(0)
    _check(lib().lco_dict_decode(_ptr(a), len(a), _ptr(out), n, C.byref(got)), "lco_dict_decode")
    return out[:got.value].tobytes()
