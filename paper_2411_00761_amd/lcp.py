"""Python binding of the LCP C ABI (include/lcp.h), same names as the C calls.

Argument marshalling only: every step of compression and decompression runs in
the HIP library liblcp_hip.so.  torch supplies device memory and the current HIP
stream.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblcp_hip.so")

MAX_FIELDS = 8
(OK, ERR_ARG, ERR_EB_TOO_SMALL, ERR_RANGE, ERR_CAPACITY, ERR_CORRUPT, ERR_NO_REFERENCE,
 ERR_BUDGET, ERR_DEVICE) = range(9)
EB_ABS, EB_REL_GLOBAL, EB_REL_PER_FIELD = 0, 1, 2
METHOD_AUTO, METHOD_S, METHOD_T = 0, 1, 2
DECIDE_S, DECIDE_T, DECIDE_COMPARE = 1, 2, 3
DTYPE_F32, DTYPE_I32 = 0, 1

EXPORTED = ["lcp_plan", "lcp_plan_destroy", "lcp_plan_reset", "lcp_plan_block_log2", "lcp_bound", "lcp_compress",
            "lcp_decompress", "lcp_select", "lcp_status_string", "lcp_kernel_timer_set",
            "lcp_kernel_timer_read", "lcp_server_create", "lcp_server_destroy",
            "lcp_server_open_stream", "lcp_server_submit", "lcp_server_wait",
            "lcp_scratch_bytes", "lcp_compress_static", "lcp_plan_set_tuning",
            "lcp_plan_get_tuning", "lcp_plan_autotune", "lcp_server_counts",
            "lcp_server_hold", "lcp_container_pack", "lcp_container_open",
            "lcp_container_info", "lcp_container_closure", "lcp_container_retrieve",
            "lcp_container_close", "lcp_dict_bound", "lcp_dict_scratch_bytes",
            "lcp_dict_encode", "lcp_dict_decode"]
REQ_COMPRESS, REQ_DECOMPRESS = 1, 2


class LCPError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = lib().lcp_status_string(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})")
        self.status = status


class lcp_params(C.Structure):
    _fields_ = [("eb_mode", C.c_int), ("eb", C.c_double), ("n_fields", C.c_int),
                ("multi_frame", C.c_int), ("batch_size", C.c_int), ("block_log2", C.c_int),
                ("chunk_log2", C.c_int), ("max_particles", C.c_uint64),
                ("hbm_budget_bytes", C.c_uint64), ("device", C.c_int),
                ("max_batch_particles", C.c_uint64), ("max_batch_frames", C.c_int),
                ("anchor_scale", C.c_int), ("n_dims", C.c_int), ("dtype", C.c_int)]


class lcp_tuning(C.Structure):
    _fields_ = [("tile", C.c_uint32), ("grid", C.c_uint32), ("slot_grid", C.c_uint32),
                ("graphs", C.c_int)]


class lcp_frame_in(C.Structure):
    _fields_ = [("fields", C.c_void_p * MAX_FIELDS), ("n", C.c_uint64), ("method", C.c_int)]


class lcp_blob(C.Structure):
    _fields_ = [("data", C.c_void_p), ("size", C.c_uint64)]


class lcp_frame_out(C.Structure):
    _fields_ = [("fields", C.c_void_p * MAX_FIELDS), ("capacity", C.c_uint64)]


# the descriptor arrays are filled as u64 tables of these widths
_FRAME_IN_WORDS = C.sizeof(lcp_frame_in) // 8
_FRAME_OUT_WORDS = C.sizeof(lcp_frame_out) // 8
assert C.sizeof(lcp_frame_in) == 8 * (MAX_FIELDS + 2) and C.sizeof(lcp_blob) == 16
assert C.sizeof(lcp_frame_out) == 8 * (MAX_FIELDS + 1)


# Descriptor arrays for a call, filled as one u64 table each (setting ctypes
# fields, or indexing a tensor, per field costs microseconds, i.e. hundreds on
# a call of many frames).  Each returns the ctypes array and the table that
# backs it (keep the table alive for the call).
def frame_in_table(frames, F, methods=None):
    """lcp_frame_in per contiguous (F, n) frame: field k starts k rows after the first."""
    nf = len(frames)
    base = np.array([f.data_ptr() for f in frames], np.uint64)
    ns = np.array([f.shape[1] for f in frames], np.uint64)
    tab = np.zeros((nf, _FRAME_IN_WORDS), np.uint64)
    for k in range(F):
        tab[:, k] = base + np.uint64(4 * k) * ns
    tab[:, MAX_FIELDS] = ns
    tab[:, MAX_FIELDS + 1] = (METHOD_AUTO if methods is None
                              else np.asarray(methods, np.int64).astype(np.uint64))
    return (lcp_frame_in * nf).from_buffer(tab), tab


def blob_table(base, offsets, sizes=None):
    """lcp_blob per record buf[offsets[j]:offsets[j+1]] (or of sizes[j] bytes)."""
    ofs = np.asarray(offsets, np.uint64)
    nf = len(offsets) - 1
    tab = np.empty((nf, 2), np.uint64)
    tab[:, 0] = np.uint64(base) + ofs[:-1]
    tab[:, 1] = np.asarray(sizes, np.uint64)[:nf] if sizes is not None else ofs[1:] - ofs[:-1]
    return (lcp_blob * nf).from_buffer(tab), tab


def frame_out_table(outs, F):
    """lcp_frame_out per (F, n) output with unit column stride."""
    nf = len(outs)
    ob = np.array([o.data_ptr() for o in outs], np.uint64)
    row = np.array([o.element_size() * o.stride(0) for o in outs], np.uint64)
    tab = np.zeros((nf, _FRAME_OUT_WORDS), np.uint64)
    for k in range(F):
        tab[:, k] = ob + np.uint64(k) * row
    tab[:, MAX_FIELDS] = [o.shape[1] for o in outs]
    return (lcp_frame_out * nf).from_buffer(tab), tab


class lcp_server_params(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("scratch_bytes", C.c_uint64),
                ("workers", C.c_int), ("device", C.c_int), ("batch_frames", C.c_int),
                ("batch_particles", C.c_uint64)]


class lcp_request(C.Structure):
    _fields_ = [("kind", C.c_int), ("stream", C.c_int), ("frame", lcp_frame_in),
                ("out", C.c_void_p), ("out_cap", C.c_uint64), ("blob", lcp_blob),
                ("dst", lcp_frame_out), ("after", C.c_void_p)]


class lcp_result(C.Structure):
    _fields_ = [("status", C.c_int), ("method", C.c_int), ("bytes", C.c_uint64),
                ("t_submit_ns", C.c_uint64), ("t_start_ns", C.c_uint64), ("t_end_ns", C.c_uint64),
                ("group", C.c_int)]


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950); there is no fallback")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.lcp_plan.argtypes = [C.POINTER(lcp_params), P, C.c_uint64, C.POINTER(P)]
        L.lcp_plan_destroy.argtypes = [P]
        L.lcp_plan_destroy.restype = None
        L.lcp_plan_reset.argtypes = [P]
        L.lcp_plan_block_log2.argtypes = [P]
        L.lcp_bound.argtypes = [P, C.c_uint64]
        L.lcp_bound.restype = C.c_uint64
        L.lcp_compress.argtypes = [P, C.c_uint64, P, P, C.c_uint64, P, P, P, P]
        L.lcp_decompress.argtypes = [P, C.c_uint64, P, P, P, P]
        L.lcp_select.argtypes = [P, C.POINTER(C.c_int)]
        L.lcp_status_string.argtypes = [C.c_int]
        L.lcp_status_string.restype = C.c_char_p
        L.lcp_kernel_timer_set.argtypes = [P, C.c_char_p]
        L.lcp_kernel_timer_read.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_uint64),
                                            C.POINTER(C.c_uint64)]
        L.lcp_scratch_bytes.argtypes = [C.POINTER(lcp_params), C.POINTER(C.c_uint64)]
        L.lcp_compress_static.argtypes = [C.POINTER(lcp_params), C.c_uint64, P, P, C.c_uint64, P,
                                          P, P]
        L.lcp_plan_set_tuning.argtypes = [P, C.POINTER(lcp_tuning)]
        L.lcp_plan_get_tuning.argtypes = [P, C.POINTER(lcp_tuning)]
        L.lcp_plan_autotune.argtypes = [P, C.c_uint64, P, P, C.c_uint64, C.c_int, P,
                                        C.POINTER(lcp_tuning), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.lcp_server_create.argtypes = [C.POINTER(lcp_server_params), C.POINTER(P)]
        L.lcp_server_destroy.argtypes = [P]
        L.lcp_server_destroy.restype = None
        L.lcp_server_open_stream.argtypes = [P, C.POINTER(lcp_params), P, C.c_uint64,
                                             C.POINTER(C.c_int)]
        L.lcp_server_submit.argtypes = [P, C.POINTER(lcp_request), C.POINTER(C.c_uint64)]
        L.lcp_server_wait.argtypes = [P, C.c_uint64, C.POINTER(lcp_result)]
        L.lcp_server_counts.argtypes = [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_uint64)]
        L.lcp_server_hold.argtypes = [P, C.c_int]
        L.lcp_container_pack.argtypes = [P, C.c_uint64, C.c_int, P, C.c_uint64,
                                         C.POINTER(C.c_uint64), P]
        L.lcp_container_open.argtypes = [P, C.c_uint64, P, C.POINTER(P)]
        L.lcp_container_info.argtypes = [P, C.POINTER(C.c_uint64), C.POINTER(C.c_int),
                                         C.POINTER(C.c_uint64), C.POINTER(C.c_int)]
        L.lcp_container_closure.argtypes = [P, C.c_uint64, P, C.c_uint64, C.POINTER(C.c_uint64)]
        L.lcp_container_retrieve.argtypes = [P, P, C.c_uint64, P, P, C.POINTER(C.c_uint64), P]
        L.lcp_container_close.argtypes = [P]
        L.lcp_container_close.restype = None
        _lib = L
    return _lib


def _stream_handle():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(st: int, what: str):
    if st != OK:
        raise LCPError(st, what)


class Plan:
    """lcp_plan / lcp_compress / lcp_decompress / lcp_select on one device.

    frames are torch CUDA tensors shaped (F, n) (rows contiguous): float32, or
    int32 for a plan made with dtype=DTYPE_I32."""

    def __init__(self, eb: float, eb_mode: int = EB_ABS, n_fields: int = 3,
                 multi_frame: bool = False, batch_size: int = 16, block_log2: int = -1,
                 chunk_log2: int = 10, max_particles: int = 1 << 20, hbm_budget_bytes: int = 0,
                 device: int = 0, sample=None, max_batch_particles: int = 0,
                 max_batch_frames: int = 0, anchor_scale: int = 0, n_dims: int = 0,
                 dtype: int = DTYPE_F32):
        import torch
        self.F = n_fields
        self.device = device
        self.tdtype = torch.int32 if dtype == DTYPE_I32 else torch.float32
        self.params = lcp_params(eb_mode, eb, n_fields, int(multi_frame), batch_size, block_log2,
                                 chunk_log2, max_particles, hbm_budget_bytes, device,
                                 max_batch_particles, max_batch_frames, anchor_scale, n_dims,
                                 dtype)
        ptrs = None
        sn = 0
        if sample is not None:
            sample = sample.contiguous()
            ptrs = (C.c_void_p * n_fields)(*[sample[f].data_ptr() for f in range(n_fields)])
            sn = sample.shape[1]
        h = C.c_void_p()
        with torch.cuda.device(device):
            _check(lib().lcp_plan(C.byref(self.params), ptrs, sn, C.byref(h)), "lcp_plan")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().lcp_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        _check(lib().lcp_plan_reset(self.h), "lcp_plan_reset")

    @property
    def block_log2(self) -> int:
        return lib().lcp_plan_block_log2(self.h)

    def bound(self, n: int) -> int:
        return int(lib().lcp_bound(self.h, n))

    def select(self) -> int:
        d = C.c_int()
        _check(lib().lcp_select(self.h, C.byref(d)), "lcp_select")
        return d.value

    def compress(self, frames: Sequence, methods=None, want_perm: bool = False, out=None):
        """Returns (out uint8 tensor, offsets list, methods_used list, perms list|None)."""
        import torch
        nf = len(frames)
        frames = [f if f.is_contiguous() else f.contiguous() for f in frames]
        for f in frames:
            assert f.dtype == self.tdtype and f.is_cuda and f.shape[0] == self.F
        arr, tab = frame_in_table(frames, self.F, methods)
        cap = 0
        bounds = {}
        for n in tab[:, MAX_FIELDS].tolist():
            b = bounds.get(n)
            if b is None:
                b = bounds[n] = (self.bound(n) + 3) & ~3
            cap += b
        if out is None:
            out = torch.empty(max(cap, 4), dtype=torch.uint8, device=f"cuda:{self.device}")
        offs = (C.c_uint64 * (nf + 1))()
        used = (C.c_int * max(nf, 1))()
        perms = None
        pptr = None
        if want_perm:
            perms = [torch.empty(f.shape[1], dtype=torch.int32, device=f.device) for f in frames]
            pptr = (C.c_void_p * nf)(*[p.data_ptr() for p in perms])
        st = lib().lcp_compress(self.h, nf, arr, C.c_void_p(out.data_ptr()), out.numel(), offs, used,
                                pptr, _stream_handle())
        if st == ERR_CAPACITY:
            raise LCPError(st, f"lcp_compress needs {offs[nf]} bytes")
        _check(st, "lcp_compress")
        return out, [int(offs[j]) for j in range(nf + 1)], [int(used[j]) for j in range(nf)], perms

    def decompress(self, buf, offsets, sizes=None, outs=None):
        """Decode records at buf[offsets[j]:offsets[j+1]]; returns (F, n) tensors of
        the plan's element type."""
        import torch
        nf = len(offsets) - 1
        offsets = [int(o) for o in offsets]
        blobs, btab = blob_table(buf.data_ptr(), offsets, sizes)
        if outs is None:
            outs = []
            for j in range(nf):
                n = self.record_n(buf, offsets[j])
                outs.append(torch.empty((self.F, n), dtype=self.tdtype, device=buf.device))
        for o in outs:
            assert o.dtype == self.tdtype and o.stride(1) == 1
        fo, otab = frame_out_table(outs, self.F)
        n_out = (C.c_uint64 * max(nf, 1))()
        _check(lib().lcp_decompress(self.h, nf, blobs, fo, n_out, _stream_handle()),
               "lcp_decompress")
        return [o if o.shape[1] == n_out[j] else o[:, : int(n_out[j])] for j, o in enumerate(outs)]

    @staticmethod
    def record_n(buf, offset: int) -> int:
        """Particle count from a record header (bytes 16..23, little-endian)."""
        b = buf[offset + 16: offset + 24].cpu().numpy().tobytes()
        return int.from_bytes(b, "little")

    def set_tuning(self, tile: int = 1024, grid: int = 0, slot_grid: int = 0, graphs: bool = True):
        t = lcp_tuning(tile, grid, slot_grid, int(graphs))
        _check(lib().lcp_plan_set_tuning(self.h, C.byref(t)), "lcp_plan_set_tuning")

    def tuning(self) -> dict:
        t = lcp_tuning()
        _check(lib().lcp_plan_get_tuning(self.h, C.byref(t)), "lcp_plan_get_tuning")
        return {"tile": t.tile, "grid": t.grid, "slot_grid": t.slot_grid, "graphs": bool(t.graphs)}

    def autotune(self, frames: Sequence, out, reps: int = 2):
        """lcp_plan_autotune on these frames; returns (choice dict, best ms, default ms)."""
        import torch
        frames = [f if f.is_contiguous() else f.contiguous() for f in frames]
        fin, keep = frame_in_table(frames, self.F)
        t, best, dflt = lcp_tuning(), C.c_double(), C.c_double()
        _check(lib().lcp_plan_autotune(self.h, len(frames), fin, out.data_ptr(), out.numel(), reps,
                                       torch.cuda.current_stream(self.device).cuda_stream,
                                       C.byref(t), C.byref(best), C.byref(dflt)),
               "lcp_plan_autotune")
        return ({"tile": t.tile, "grid": t.grid, "slot_grid": t.slot_grid,
                 "graphs": bool(t.graphs)}, best.value, dflt.value)

    def timer_set(self, name):
        _check(lib().lcp_kernel_timer_set(self.h, None if name is None else name.encode()),
               "lcp_kernel_timer_set")

    def timer_read(self):
        ms, la, by = C.c_double(), C.c_uint64(), C.c_uint64()
        _check(lib().lcp_kernel_timer_read(self.h, C.byref(ms), C.byref(la), C.byref(by)),
               "lcp_kernel_timer_read")
        return ms.value, la.value, by.value


def compress_static(frames: Sequence, eb: float, eb_mode: int = EB_ABS, n_fields: int = 3,
                    block_log2: int = 4, chunk_log2: int = 10, max_particles: int = 0,
                    max_batch_particles: int = 0, max_batch_frames: int = 0, out=None,
                    want_perm: bool = False, device: int = 0, dtype: int = DTYPE_F32):
    """lcp_compress_static: LCP-S records of independent frames on the library's
    static scratch (no plan, no allocation inside the call).  Returns
    (out uint8 tensor, offsets list, perms list|None)."""
    import torch
    nf = len(frames)
    frames = [f if f.is_contiguous() else f.contiguous() for f in frames]
    n_max = max(int(f.shape[1]) for f in frames)
    p = lcp_params(eb_mode, eb, n_fields, 0, 0, block_log2, chunk_log2,
                   max_particles or n_max, 0, device, max_batch_particles, max_batch_frames, 0, 0,
                   dtype)
    if out is None:
        def bound(n):  # worst-case record bytes (what lcp_bound gives)
            w = lambda bits: (bits + 31) // 32  # noqa: E731
            return (80 + 8 * n_fields + 32 * (n_fields + 2) + 4 * w(63 * n) + 4 * w(33 * n)
                    + 4 * n_fields * w(25 * n))
        out = torch.empty(sum(bound(int(f.shape[1])) for f in frames), dtype=torch.uint8,
                          device=frames[0].device)
    fin, keep = frame_in_table(frames, n_fields)
    offs = (C.c_uint64 * (nf + 1))()
    perms = None
    pp = None
    if want_perm:
        perms = [torch.empty(int(f.shape[1]), dtype=torch.int32, device=f.device) for f in frames]
        pp = (C.c_void_p * nf)(*[t.data_ptr() for t in perms])
    st = lib().lcp_compress_static(C.byref(p), nf, fin, out.data_ptr(), out.numel(), offs, pp,
                                   torch.cuda.current_stream(device).cuda_stream)
    _check(st, "lcp_compress_static")
    return out, [int(v) for v in offs], perms


def scratch_bytes(n_fields: int = 3, multi_frame: bool = True, max_particles: int = 1 << 20,
                  chunk_log2: int = 10, max_batch_particles: int = 0, max_batch_frames: int = 0) -> int:
    """Device scratch of one call of a plan with these sizes (lcp_scratch_bytes)."""
    p = lcp_params(EB_ABS, 1.0, n_fields, int(multi_frame), 16, 0, chunk_log2, max_particles, 0, 0,
                   max_batch_particles, max_batch_frames)
    b = C.c_uint64()
    _check(lib().lcp_scratch_bytes(C.byref(p), C.byref(b)), "lcp_scratch_bytes")
    return b.value


class Server:
    """lcp_server_*: multi-frame streams served concurrently on one device.

    Frames are torch float32 (or int32) CUDA tensors shaped (F, n); records and outputs are
    caller tensors kept alive here until their request is waited for."""

    def __init__(self, scratch_bytes: int, workers: int = 4, hbm_budget_bytes: int = 0,
                 device: int = 0, batch_frames: int = 0, batch_particles: int = 0):
        import torch
        self.device = device
        p = lcp_server_params(hbm_budget_bytes, scratch_bytes, workers, device, batch_frames,
                              batch_particles)
        h = C.c_void_p()
        with torch.cuda.device(device):
            _check(lib().lcp_server_create(C.byref(p), C.byref(h)), "lcp_server_create")
        self.h = h
        self.F = {}
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            lib().lcp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def open_stream(self, eb: float, eb_mode: int = EB_ABS, n_fields: int = 3, batch_size: int = 16,
                    block_log2: int = -1, chunk_log2: int = 10, max_particles: int = 1 << 20,
                    sample=None, anchor_scale: int = 0, n_dims: int = 0,
                    dtype: int = DTYPE_F32) -> int:
        params = lcp_params(eb_mode, eb, n_fields, 1, batch_size, block_log2, chunk_log2,
                            max_particles, 0, self.device, 0, 0, anchor_scale, n_dims, dtype)
        ptrs, sn = None, 0
        if sample is not None:
            sample = sample.contiguous()
            ptrs = (C.c_void_p * n_fields)(*[sample[f].data_ptr() for f in range(n_fields)])
            sn = sample.shape[1]
        sid = C.c_int()
        _check(lib().lcp_server_open_stream(self.h, C.byref(params), ptrs, sn, C.byref(sid)),
               "lcp_server_open_stream")
        self.F[sid.value] = n_fields
        return sid.value

    def _submit(self, rq, keep) -> int:
        import torch
        # the request waits for the work torch has queued on the buffers so far
        rq.after = torch.cuda.current_stream(self.device).cuda_stream
        t = C.c_uint64()
        _check(lib().lcp_server_submit(self.h, C.byref(rq), C.byref(t)), "lcp_server_submit")
        self._keep[t.value] = keep
        return t.value

    def compress(self, stream: int, frame, out, method: int = METHOD_AUTO) -> int:
        """Queue the stream's next frame; the record goes to out (uint8 CUDA tensor)."""
        rq = lcp_request()
        rq.kind = REQ_COMPRESS
        rq.stream = stream
        if not frame.is_contiguous():
            frame = frame.contiguous()
        base, n = frame.data_ptr(), frame.shape[1]
        for k in range(self.F[stream]):
            rq.frame.fields[k] = base + 4 * n * k
        rq.frame.n = n
        rq.frame.method = method
        rq.out = out.data_ptr()
        rq.out_cap = out.numel()
        return self._submit(rq, (frame, out))

    def decompress(self, stream: int, buf, offset: int, size: int, out) -> int:
        """Queue the decoding of the stream's next record buf[offset:offset+size] into out (F, n)."""
        rq = lcp_request()
        rq.kind = REQ_DECOMPRESS
        rq.stream = stream
        rq.blob.data = buf.data_ptr() + offset
        rq.blob.size = size
        assert out.element_size() == 4 and out.stride(1) == 1
        ob, row = out.data_ptr(), 4 * out.stride(0)
        for k in range(self.F[stream]):
            rq.dst.fields[k] = ob + row * k
        rq.dst.capacity = out.shape[1]
        return self._submit(rq, (buf, out))

    def wait(self, ticket: int) -> dict:
        r = lcp_result()
        _check(lib().lcp_server_wait(self.h, ticket, C.byref(r)), "lcp_server_wait")
        self._keep.pop(ticket, None)
        return {"status": r.status, "method": r.method, "bytes": r.bytes,
                "t_submit_ns": r.t_submit_ns, "t_start_ns": r.t_start_ns, "t_end_ns": r.t_end_ns,
                "group": r.group}

    def hold(self, on: bool = True):
        """lcp_server_hold: while on, workers start no further request."""
        _check(lib().lcp_server_hold(self.h, int(on)), "lcp_server_hold")

    def counts(self) -> dict:
        """Launch sets run on batch scratch, requests they finished, requests put back."""
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(lib().lcp_server_counts(self.h, C.byref(a), C.byref(b), C.byref(c)),
               "lcp_server_counts")
        return {"merged_launches": a.value, "merged_requests": b.value, "requeued": c.value}


class Container:
    """lcp_container_*: a multi-frame stream's records packed for random access
    (Sec. 7.3).  buf is the container, a uint8 CUDA tensor kept alive here."""

    @staticmethod
    def pack(buf, offsets, batch_size: int):
        """Records buf[offsets[j]:offsets[j+1]] (frames 0..n-1 of one stream) -> container tensor."""
        import torch
        offsets = [int(o) for o in offsets]
        blobs, _tab = blob_table(buf.data_ptr(), offsets)
        n = len(offsets) - 1
        size = C.c_uint64()
        _check(lib().lcp_container_pack(blobs, n, batch_size, None, 0, C.byref(size),
                                        _stream_handle()), "lcp_container_pack")
        out = torch.empty(size.value, dtype=torch.uint8, device=buf.device)
        _check(lib().lcp_container_pack(blobs, n, batch_size, C.c_void_p(out.data_ptr()),
                                        out.numel(), C.byref(size), _stream_handle()),
               "lcp_container_pack")
        return out

    def __init__(self, buf):
        self.buf = buf
        h = C.c_void_p()
        _check(lib().lcp_container_open(C.c_void_p(buf.data_ptr()), buf.numel(), _stream_handle(),
                                        C.byref(h)), "lcp_container_open")
        self.h = h
        fr, b, a, F = C.c_uint64(), C.c_int(), C.c_uint64(), C.c_int()
        _check(lib().lcp_container_info(h, C.byref(fr), C.byref(b), C.byref(a), C.byref(F)),
               "lcp_container_info")
        self.frames, self.batch_size, self.anchors, self.F = fr.value, b.value, a.value, F.value

    def close(self):
        if getattr(self, "h", None):
            lib().lcp_container_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def closure(self, frame: int):
        arr = (C.c_uint64 * 4096)()
        cnt = C.c_uint64()
        _check(lib().lcp_container_closure(self.h, frame, arr, 4096, C.byref(cnt)),
               "lcp_container_closure")
        return [int(arr[i]) for i in range(cnt.value)]

    def retrieve(self, plan, frames, outs):
        """Decode frames (list of ints) into outs (list of (F, n) CUDA tensors of the
        plan's element type);
        returns the number of records decoded."""
        n = len(frames)
        fr = (C.c_uint64 * max(n, 1))(*frames)
        fo, _o = frame_out_table(outs, self.F)
        dec = C.c_uint64()
        _check(lib().lcp_container_retrieve(self.h, plan.h, n, fr, fo, C.byref(dec),
                                            _stream_handle()), "lcp_container_retrieve")
        return dec.value


# ---- dictionary stage (lcp_dict_*): marshalling only ----
def _dict_lib():
    L = lib()
    if not getattr(L, "_dict_types", False):
        P = C.c_void_p
        L.lcp_dict_bound.argtypes = [C.c_uint64, C.c_int]
        L.lcp_dict_bound.restype = C.c_uint64
        L.lcp_dict_scratch_bytes.argtypes = [C.c_uint64, C.c_int, C.c_int, C.POINTER(C.c_uint64)]
        L.lcp_dict_encode.argtypes = [P, C.c_uint64, C.c_int, P, C.c_uint64, P, C.c_uint64,
                                      C.POINTER(C.c_uint64), P]
        L.lcp_dict_decode.argtypes = [P, C.c_uint64, P, C.c_uint64, P, C.c_uint64,
                                      C.POINTER(C.c_uint64), P]
        L._dict_types = True
    return L


def dict_bound(n: int, block_log2: int = 12) -> int:
    return int(_dict_lib().lcp_dict_bound(n, block_log2))


def dict_scratch_bytes(n: int, block_log2: int = 12, encode: bool = True) -> int:
    b = C.c_uint64(0)
    _check(_dict_lib().lcp_dict_scratch_bytes(n, block_log2, 1 if encode else 0, C.byref(b)),
           "lcp_dict_scratch_bytes")
    return b.value


def dict_encode(buf, n: int = None, block_log2: int = 12, out=None, scratch=None):
    """lcp_dict_encode on the first n bytes of a device uint8 tensor; returns
    (stream uint8 tensor, stream size)."""
    import torch
    n = buf.numel() if n is None else int(n)
    if out is None:
        out = torch.empty(dict_bound(n, block_log2), dtype=torch.uint8, device=buf.device)
    if scratch is None:
        scratch = torch.empty(dict_scratch_bytes(n, block_log2, True), dtype=torch.uint8,
                              device=buf.device)
    size = C.c_uint64(0)
    _check(_dict_lib().lcp_dict_encode(buf.data_ptr(), n, block_log2, out.data_ptr(), out.numel(),
                                       scratch.data_ptr(), scratch.numel(), C.byref(size),
                                       torch.cuda.current_stream(buf.device).cuda_stream),
           "lcp_dict_encode")
    return out, size.value


def dict_decode(stream, size: int, n: int, block_log2: int = 12, out=None, scratch=None):
    """lcp_dict_decode of a stream of size bytes holding n bytes (block_log2 as
    encoded); returns the decoded uint8 tensor."""
    import torch
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.uint8, device=stream.device)
    if scratch is None:
        scratch = torch.empty(dict_scratch_bytes(n, block_log2, False), dtype=torch.uint8,
                              device=stream.device)
    got = C.c_uint64(0)
    _check(_dict_lib().lcp_dict_decode(stream.data_ptr(), size, out.data_ptr(), out.numel(),
                                       scratch.data_ptr(), scratch.numel(), C.byref(got),
                                       torch.cuda.current_stream(stream.device).cuda_stream),
           "lcp_dict_decode")
    return out[:got.value]
