/*
 * lcp.h -- C ABI of the MI355X (gfx950) LCP particle compressor.
 *
 * LCP (Zhang et al., arXiv 2411.00761) compresses frames of particle positions
 * under a pointwise absolute error bound:
 *   - LCP-S, the block-wise spatial compressor (Sec. 6): error-bound-aware
 *     quantisation (Eq. 5), spatial blocks of 2^k bins per side (Eq. 6), the
 *     non-empty blocks' ids / counts / corner-relative positions stored block by
 *     block (Sec. 6.2.1), each array delta coded and then Huffman or fixed-length
 *     coded, whichever is shorter (Sec. 6.2.2, Tab. 3);
 *   - LCP-T, the temporal compressor (Sec. 7.1): codes on the reference frame's
 *     grid minus the reference's codes;
 *   - the multi-frame driver: LCP-FSM chooses S or T per frame (Sec. 7.2) and
 *     Alg. 1 picks the reference (the last spatial anchor for the first frame of a
 *     batch, otherwise the previous frame; Sec. 7.3);
 *   - the block-size search over p = 2^k, 0 <= k <= 16, on a sample (Sec. 7.4.1).
 * The problem statement (Sec. 4, Eq. 1-2) fixes the interface: particle arrays
 * (frames x particles x coordinates, with further fields as supplementary
 * dimensions), an absolute or value-range-relative error bound, and single- or
 * multi-frame use.
 *
 * Conventions for every call:
 *   - All particle and record buffers are DEVICE pointers owned by the caller
 *     (e.g. the data pointers of torch tensors).  Fields are structure-of-arrays:
 *     one float32 array of n values per field.
 *   - Work is enqueued on the caller's hipStream_t (NULL = the null stream); the
 *     calls that report sizes synchronise that stream before returning.
 *   - Calls return an lcp_status; nothing crosses the ABI as an exception.  On an
 *     error the output contents are undefined and the plan's stream state (the
 *     reference frames and the FSM) is unchanged.
 *   - A plan is one compression stream plus one decompression stream; it is not
 *     thread-safe.  The plan owns all device scratch, allocated in lcp_plan.
 *   - Decompressed particles come back in slot order (block order, stable in the
 *     input index); lcp_compress can return the slot -> input index permutation.
 */
#ifndef LCP_H
#define LCP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LCP_MAX_FIELDS 8

typedef enum {
  LCP_OK = 0,
  LCP_ERR_ARG = 1,           /* invalid argument or non-finite input value */
  LCP_ERR_EB_TOO_SMALL = 2,  /* eb below two float32 ulps of the data magnitude */
  LCP_ERR_RANGE = 3,         /* codes would exceed 2^23, or block ids 2^63 */
  LCP_ERR_CAPACITY = 4,      /* output buffer too small; required size reported */
  LCP_ERR_CORRUPT = 5,       /* a record failed validation while decoding */
  LCP_ERR_NO_REFERENCE = 6,  /* a temporal record's reference frame is not resident */
  LCP_ERR_BUDGET = 7,        /* the plan's scratch would exceed hbm_budget_bytes */
  LCP_ERR_DEVICE = 8         /* a HIP runtime call, or a device-side consistency check, failed */
} lcp_status;

enum { LCP_EB_ABS = 0, LCP_EB_REL_GLOBAL = 1, LCP_EB_REL_PER_FIELD = 2 };
enum { LCP_METHOD_AUTO = 0, LCP_METHOD_S = 1, LCP_METHOD_T = 2 };
enum { LCP_DECIDE_S = 1, LCP_DECIDE_T = 2, LCP_DECIDE_COMPARE = 3 };
/* Element type of a plan's fields (Sec. 3: the data may be integers or floats). */
enum { LCP_DTYPE_F32 = 0, LCP_DTYPE_I32 = 1 };

typedef struct {
  int eb_mode;        /* LCP_EB_ABS: eb is absolute.  LCP_EB_REL_GLOBAL: eb times the
                         value range max(D)-min(D) over all fields (Sec. 4).
                         LCP_EB_REL_PER_FIELD: eb times each field's own range. */
  double eb;          /* > 0 */
  int n_fields;       /* 1 .. LCP_MAX_FIELDS: the n_dims spatial coordinates first, then
                         supplementary fields (velocities ...) */
  int multi_frame;    /* 0: every frame LCP-S.  1: LCP-FSM picks S or T per frame and
                         the error bound is fixed by the stream's first frame. */
  int batch_size;     /* Alg. 1 batch length (frames); 0 = one unbounded batch */
  int block_log2;     /* k in [0,16] (block side p = 2^k bins), or -1: search k on
                         the sample given to lcp_plan (Sec. 7.4.1) */
  int chunk_log2;     /* Huffman chunk of 2^chunk_log2 symbols, in [5,12]; a format
                         parameter (10 by default when 0 is passed) */
  uint64_t max_particles;    /* largest n per frame this plan will see (<= 2^31) */
  uint64_t hbm_budget_bytes; /* 0 = unlimited; otherwise lcp_plan fails with
                                LCP_ERR_BUDGET if its scratch would exceed it */
  int device;                /* HIP device ordinal */
  uint64_t max_batch_particles; /* single-frame plans: most particles in one batch of
                                   independent frames, max_particles..2^32-1
                                   (0 = max_particles) */
  int max_batch_frames;         /* single-frame plans: most frames in one batch, at most
                                   1024 (0 = 64) */
  int anchor_scale;             /* multi-frame plans (Sec. 7.4.2): 0 or 1 = off; an odd
                                   s in 3..15 codes an anchor frame (first in its batch,
                                   LCP-S) at eb / s while the stream is temporally
                                   correlated -- at its start, or when at least half of
                                   the frames since the last anchor were LCP-T; the
                                   LCP-T frames chained to it keep its finer grid and
                                   move in steps of s (the paper uses s = 5) */
  int n_dims;                   /* spatial dimensions 1..3 (0 = 3): the fields that form
                                   the blocks of Eq. 6 (Sec. 4: data of other dimensions);
                                   at most n_fields; a spatial record carries it in
                                   header byte 52 (3 written as 0) */
  int dtype;                    /* LCP_DTYPE_F32 (0) or LCP_DTYPE_I32: every field of
                                   every frame.  int32 fields are quantised to runs of
                                   2 floor(eb) + 1 consecutive integers and decode to the
                                   run's centre (held to the int32 range), exact within
                                   eb; a bound below 1 is lossless, and a relative bound
                                   of 0 (a constant field) is allowed.  With anchor_scale
                                   s, an anchor's bins are the widest odd runs with
                                   s runs <= 2 floor(eb) + 1 integers, and an anchor is
                                   coded at eb when some field has no such run (bins
                                   narrower than s).  Records carry it in header byte 53
                                   and decode only through a plan of the same dtype. */
} lcp_params;

typedef struct lcp_plan_s* lcp_plan_t;

/* One input frame: fields[0..n_fields) device pointers of n float32 values each
 * (int32 values, the pointers cast, when the plan's dtype is LCP_DTYPE_I32). */
typedef struct {
  const float* fields[LCP_MAX_FIELDS];
  uint64_t n;
  int method; /* LCP_METHOD_AUTO (FSM), LCP_METHOD_S or LCP_METHOD_T */
} lcp_frame_in;

/* One compressed record in device memory. */
typedef struct {
  const void* data;
  uint64_t size;
} lcp_blob;

/* Destination of one decompressed frame: n_fields device arrays of `capacity`
 * float32 values each (int32 for LCP_DTYPE_I32 plans, the pointers cast). */
typedef struct {
  float* fields[LCP_MAX_FIELDS];
  uint64_t capacity;
} lcp_frame_out;

/* Create a plan (the parameters theta of the compressor, Sec. 4; the block size
 * p = 2^k of Sec. 6.2.1 and its search, Sec. 7.4.1): validates params, allocates
 * all device scratch and the resident stream state on params->device, and, when
 * block_log2 == -1, runs the block-size search on a stride sample of the given
 * frame (sample_fields: device
 * pointers, n_fields of them, sample_n values each; the stride is
 * max(1, sample_n >> 20)).  The plan is returned in *out.
 * Errors: LCP_ERR_ARG, LCP_ERR_BUDGET, LCP_ERR_DEVICE, and the search's errors. */
lcp_status lcp_plan(const lcp_params* params, const float* const* sample_fields,
                    uint64_t sample_n, lcp_plan_t* out);

void lcp_plan_destroy(lcp_plan_t plan);

/* Forget the plan's stream state: both the compression and decompression sides
 * restart at frame 0 with no reference frames, LCP-FSM back in S1X and (for
 * multi-frame plans) the error bound taken again from the next frame.  Scratch
 * and the block size are kept.  Returns LCP_ERR_ARG for a NULL plan. */
lcp_status lcp_plan_reset(lcp_plan_t plan);

/* The block size exponent k the plan uses (searched or given). */
int lcp_plan_block_log2(lcp_plan_t plan);

/* Worst-case record bytes for a frame of n particles. */
uint64_t lcp_bound(lcp_plan_t plan, uint64_t n);

/* Device scratch bytes a plan with these parameters uses per call (what
 * lcp_plan allocates beside the stream state; what a server request carves out
 * of its arena).  Errors: LCP_ERR_ARG. */
lcp_status lcp_scratch_bytes(const lcp_params* params, uint64_t* device_bytes);

/* Compress n_frames frames, in stream order, into out (device, out_cap bytes):
 * the compression f of Sec. 4, Eq. 1-2 (|d - d'| <= eb pointwise).  A spatial
 * frame is LCP-S (Sec. 6: Eq. 5 quantisation, Eq. 6 blocks, Sec. 6.2.2 delta and
 * Huffman / fixed coding); a temporal frame is LCP-T (Sec. 7.1) against the
 * reference Alg. 1 names (Sec. 7.3), the choice made by LCP-FSM (Sec. 7.2).
 * Arguments: frames[j].fields are device SoA float32 arrays owned by the caller,
 * read only; out is a caller-owned device buffer, 4-byte aligned.
 * Record j is written at out + out_offsets[j] and occupies
 * out_offsets[j+1] - out_offsets[j] bytes (out_offsets: host array of
 * n_frames + 1 entries; records are 4-byte aligned and back to back).
 * methods_used (host, nullable): LCP_METHOD_S or LCP_METHOD_T per frame.
 * perms (nullable; else n_frames device pointers, each nullable): receives the
 * slot -> input index permutation of each frame (n uint32 values).
 * In single-frame plans (multi_frame == 0) the frames are independent, and
 * consecutive frames are compressed together, as many at a time as the plan's
 * max_batch_frames and max_batch_particles allow: one extent pass, one sort and
 * one set of coding launches per batch (the records are the same bytes as when
 * the frames are compressed one per call).  In multi-frame plans, frames that
 * LCP-FSM codes with LCP-T in a row are enqueued in runs and their outcomes
 * read back once per run (a run takes eight frames, twice as many after each
 * run that commits in full, up to 32); a frame whose outcome differs from that
 * prediction is coded again on its own, so the records are again those of one
 * call per frame.  A run only takes frames whose worst-case records fit in out_cap.
 * Errors: LCP_ERR_ARG, LCP_ERR_EB_TOO_SMALL, LCP_ERR_RANGE, LCP_ERR_CAPACITY
 * (out_offsets[n_frames] then holds the bytes required so far), LCP_ERR_DEVICE,
 * LCP_ERR_NO_REFERENCE (LCP_METHOD_T without a resident reference). */
lcp_status lcp_compress(lcp_plan_t plan, uint64_t n_frames, const lcp_frame_in* frames,
                        void* out, uint64_t out_cap, uint64_t* out_offsets,
                        int* methods_used, uint32_t* const* perms, hipStream_t stream);

/* Decompress n_frames records, in stream order: the decompression g of Sec. 4
 * (x' = (2q + 1) eb + min, Eq. 5), with the block structure of Sec. 6.2.1
 * expanded and a temporal record added to its reference (Sec. 7.1), which must
 * have been decoded before it by this plan (recursive retrieval, Sec. 7.3).
 * blobs[j].data: caller-owned device records, 4-byte aligned, read only; outs:
 * caller-owned device arrays.  Frame j's float32 values are
 * written, in slot order, to outs[j].fields[f][0..n); n_out (host) receives n.
 * A temporal record needs its reference (the previous frame, or the last anchor
 * for the first frame of a batch) decoded earlier by this plan.
 * Errors: LCP_ERR_ARG, LCP_ERR_CORRUPT, LCP_ERR_NO_REFERENCE, LCP_ERR_CAPACITY
 * (n_out then holds n), LCP_ERR_DEVICE. */
lcp_status lcp_decompress(lcp_plan_t plan, uint64_t n_frames, const lcp_blob* blobs,
                          const lcp_frame_out* outs, uint64_t* n_out, hipStream_t stream);

/* LCP-FSM (Sec. 7.2) with Alg. 1's reference rule (Sec. 7.3): what the next
 * frame compressed with LCP_METHOD_AUTO gets:
 * LCP_DECIDE_S, LCP_DECIDE_T or LCP_DECIDE_COMPARE (run both, keep the smaller). */
lcp_status lcp_select(lcp_plan_t plan, int* decision);

const char* lcp_status_string(lcp_status status);

/* LCP-S compression of independent frames that allocates nothing: for callers
 * that cannot allocate device or pinned memory during the call (code that a HIP
 * graph capture surrounds, tight serving loops, harnesses that forbid it).
 * Same records, offsets and permutations as lcp_compress on a fresh plan made
 * with the same params (record j of a call carries sequence number j), but no
 * plan exists: the scratch is one library-owned device array of 64 MiB per GPU
 * (file-scope, reserved with the library's code object and held by each GPU the
 * library runs on until the process ends) plus a static host block for the
 * small tables.  params: as for lcp_plan, with multi_frame = 0 and block_log2 in
 * [0, 16] (no search); max_particles, max_batch_particles and max_batch_frames
 * (0 means 1 here: one frame per launch set) size the scratch the call needs,
 * which must fit the array -- else LCP_ERR_BUDGET before any HIP call.  With one
 * frame per launch set that is a frame of about 550,000 particles of three
 * fields (about 370,000 of six); each further frame per launch set costs about 2 MB.  The other
 * arguments and errors are lcp_compress's (methods are all LCP_METHOD_S).
 * Calls on one GPU share its array and keep none of each other's state: the
 * library runs them one at a time (each call has finished on the GPU when it
 * returns), and clears what must start at zero at the start of every call. */
lcp_status lcp_compress_static(const lcp_params* params, uint64_t n_frames,
                               const lcp_frame_in* frames, void* out, uint64_t out_cap,
                               uint64_t* out_offsets, uint32_t* const* perms, hipStream_t stream);

/* ---- Launch shape of batched LCP-S compression, and its autotuner ----
 *
 * How the kernels of a batch of independent frames are launched; never a
 * format parameter (records are the same bytes under every setting).  tile:
 * slots per tile of the element-wise encode kernels, a multiple of 256 in
 * [256, 16384].  grid: persistent workgroups those kernels walk their tiles
 * with (0: one workgroup per tile).  slot_grid: the same for the slot-symbol
 * kernel (256-slot tiles).  graphs: 1 captures the kernels of each batch
 * launch shape (frame sizes, output buffer) into a hipGraph on first use and
 * replays it afterwards (plans created by lcp_plan only; at most 8 shapes are
 * kept per plan). */
typedef struct {
  uint32_t tile;
  uint32_t grid;
  uint32_t slot_grid;
  int graphs;
} lcp_tuning;

/* Set or read a plan's launch shape (LCP_ERR_ARG on an invalid setting).  A
 * plan starts from the autotuner's cached choice for its device, particle
 * count and fields if there is one (checked per call), else tile 1024, grid 0,
 * slot_grid 0, graphs 1; an explicit setting overrides the cache. */
lcp_status lcp_plan_set_tuning(lcp_plan_t plan, const lcp_tuning* tuning);
lcp_status lcp_plan_get_tuning(lcp_plan_t plan, lcp_tuning* tuning);

/* Autotuner: compresses the given frames (as lcp_compress on this single-frame
 * plan would, into out) under each candidate launch shape -- tile 1024, 2048
 * or 4096, grid 0, 8 or 32 workgroups per compute unit, slot_grid 0 or 16 per
 * compute unit -- repeats best-of-reps timings of each on the stream, keeps
 * the fastest for this plan and stores it in a process-wide cache keyed by
 * (GPU name and compute units, bit width of the call's total particles,
 * n_fields) that later calls of any plan consult.  The plan's stream state
 * (frame sequence numbers) is left as it was.  *chosen (nullable) receives the
 * choice, *best_ms and *default_ms (nullable) the time of one call under it
 * and under the defaults.  Errors: those of lcp_compress; LCP_ERR_ARG for a
 * multi-frame plan. */
lcp_status lcp_plan_autotune(lcp_plan_t plan, uint64_t n_frames, const lcp_frame_in* frames,
                             void* out, uint64_t out_cap, int reps, hipStream_t stream,
                             lcp_tuning* chosen, double* best_ms, double* default_ms);

/* Kernel timing for roofline measurement: while a name is set, one launch in
 * sixteen of the kernel with that name (the first, the 17th, ...; "name/N"
 * times one in N, N in 1..1024) carries HIP events on its own dispatch; the
 * accumulated time (ms), count and algorithmic bytes of the timed launches are
 * read back with lcp_kernel_timer_read.  Sampling keeps the events' cost on the
 * stream (a few microseconds around each timed launch) out of the other
 * launches.  Names: "t_resid" (one temporal frame, or frames of several
 * streams), "t_resid_run" (a run of temporal frames of one stream), "t_recon",
 * "quant_key", "radix_scatter", "slot_syms", "s_recon", "extent", "hist",
 * "huff_build", "pack_huff", "emit", "layout", "decode_huff", "decode_fixed".
 * Pass NULL to stop. */
lcp_status lcp_kernel_timer_set(lcp_plan_t plan, const char* kernel_name);
lcp_status lcp_kernel_timer_read(lcp_plan_t plan, double* total_ms, uint64_t* launches,
                                 uint64_t* bytes);

/* ---- Multi-frame container with random access (Sec. 7.3, Alg. 1) ----
 *
 * The records of one multi-frame stream, packed so that any frame can be
 * retrieved alone.  Layout (little-endian, all in one device buffer): a 64-byte
 * header ("LCPC", version 1, batch size, fields, frame count, anchor count,
 * table offset 64, anchor-array offset, total bytes), a 32-byte entry per frame
 * (record offset, size, reference frame or all ones, particle count, method
 * 0 = S / 1 = T, anchor flag), the records of each batch in stream order, then
 * the anchor array: the first-in-batch frames coded by LCP-S, which Sec. 7.3
 * stores apart.  Retrieving frame k decodes it directly when it is spatial,
 * else its reference first, recursively: at most the frames of its batch up to
 * k plus one anchor. */
typedef struct lcp_container_s* lcp_container_t;

/* Pack n records of one stream (records[j] is frame j, j = 0..n-1, as a
 * multi-frame lcp_compress wrote them; device pointers, 4-byte aligned) with the
 * stream's batch size into out (device, out_cap bytes; NULL only sizes it).
 * *out_size receives the container's size.  Synchronises the stream.
 * Errors: LCP_ERR_ARG (not one stream from its start, mixed field counts),
 * LCP_ERR_CORRUPT (not a record), LCP_ERR_CAPACITY, LCP_ERR_DEVICE. */
lcp_status lcp_container_pack(const lcp_blob* records, uint64_t n, int batch_size, void* out,
                              uint64_t out_cap, uint64_t* out_size, hipStream_t stream);

/* Open a container in device memory (it must stay alive and unchanged until
 * lcp_container_close): reads its header and frame table.  Errors: LCP_ERR_ARG,
 * LCP_ERR_CORRUPT (bad magic, sizes, offsets, references or anchor flags),
 * LCP_ERR_DEVICE. */
lcp_status lcp_container_open(const void* container, uint64_t size, hipStream_t stream,
                              lcp_container_t* out);
lcp_status lcp_container_info(lcp_container_t c, uint64_t* frames, int* batch_size,
                              uint64_t* anchors, int* n_fields);

/* The frames that must be decoded to obtain `frame`, in stream order (the last
 * is `frame`), into frames[0..*count) (LCP_ERR_CAPACITY when cap is smaller). */
lcp_status lcp_container_closure(lcp_container_t c, uint64_t frame, uint64_t* frames,
                                 uint64_t cap, uint64_t* count);

/* Retrieve frames[0..n_req) into outs[i] (device, slot order as lcp_decompress
 * writes them) with a multi-frame plan of the container's field count and batch
 * size (its decode state is reset).  Requests are served in the given order:
 * each run of requests with increasing frame numbers is one pass that decodes
 * the union of their closures once, in stream order; a request that goes back
 * in the stream starts a new pass.  *decoded (nullable) receives the number of
 * records decoded.  Frames decoded but not requested go to scratch the
 * container allocates on first use.  Errors: those of lcp_decompress;
 * LCP_ERR_ARG (a frame out of range, a plan that does not match). */
lcp_status lcp_container_retrieve(lcp_container_t c, lcp_plan_t plan, uint64_t n_req,
                                  const uint64_t* frames, const lcp_frame_out* outs,
                                  uint64_t* decoded, hipStream_t stream);
void lcp_container_close(lcp_container_t c);

/* ---- Dictionary stage ----
 * The last coding step of the encoding stage (Sec. 6.2.2) and of LCP-T
 * (Sec. 7.1), which the paper fills with a general-purpose dictionary coder:
 * here a lossless pass over any coded bytes (typically the records of a
 * compress call), an order-0 rANS coder over bytes with one frequency table
 * for the input and independent blocks of 2^block_log2 bytes (12..20), one
 * block per GPU wave whose lane k takes the block's bytes k, k + 64, ...
 * Stream: u32 magic "LCPD", u32 block_log2, u64 n, u16 freq[256] (normalised
 * to 4096), u32 size[nb] (nb = ceil(n / 2^block_log2)), then the blocks, each
 * u16 lane_size[64] and the lanes' coded bytes.  A lane is coded from its last
 * byte to its first through a 32-bit state starting at 2^23: a byte of
 * frequency f and cumulative frequency c writes out the state's low bytes
 * while it is at least 2^19 f, then takes it to (x / f) 4096 + x % f + c; the
 * coded lane is the final state (4 bytes, little-endian) and the written bytes
 * in reading order.
 *
 * lcp_dict_bound: the largest stream for n input bytes (0 for an invalid
 * block_log2).  lcp_dict_scratch_bytes: the device scratch an encode (encode
 * != 0) or a decode of n bytes needs.
 * lcp_dict_encode: in (device, 4-byte aligned, n bytes, read only) to out
 * (device, 4-byte aligned, out_cap >= lcp_dict_bound(n)); scratch: caller-owned device
 * memory, 256-byte aligned, of at least lcp_dict_scratch_bytes; *out_size
 * (host) receives the stream's size.  Synchronises the stream.  Errors:
 * LCP_ERR_ARG, LCP_ERR_CAPACITY (*out_size = the bound), LCP_ERR_BUDGET
 * (scratch too small), LCP_ERR_DEVICE.
 * lcp_dict_decode: a stream of size bytes (device) to out (device, out_cap
 * bytes); *n_out (host) receives n.  Synchronises the stream (twice).  Errors:
 * LCP_ERR_ARG, LCP_ERR_CORRUPT (a stream that fails its checks: magic, table
 * sum, block sizes that do not add up to the stream or lane sizes to their
 * block, a lane that does not end on its initial state with all its bytes
 * used), LCP_ERR_CAPACITY (*n_out = n),
 * LCP_ERR_BUDGET, LCP_ERR_DEVICE. */
uint64_t lcp_dict_bound(uint64_t n, int block_log2);
lcp_status lcp_dict_scratch_bytes(uint64_t n, int block_log2, int encode, uint64_t* device_bytes);
lcp_status lcp_dict_encode(const void* in, uint64_t n, int block_log2, void* out, uint64_t out_cap,
                           void* scratch, uint64_t scratch_bytes, uint64_t* out_size,
                           hipStream_t stream);
lcp_status lcp_dict_decode(const void* in, uint64_t size, void* out, uint64_t out_cap,
                           void* scratch, uint64_t scratch_bytes, uint64_t* n_out,
                           hipStream_t stream);

/* ---- Serving: many multi-frame streams, requests overlapped on one device ----
 *
 * A server holds multi-frame streams (each one the state of a multi-frame plan:
 * reference codes, permutations, LCP-FSM and Alg. 1 bookkeeping, resident on
 * the device for the stream's lifetime) and runs their compress / decompress
 * requests on `workers` threads, each with its own HIP stream.  A request's
 * scratch is carved out of a device arena of scratch_bytes when it starts and
 * returned when it ends.  Requests are admitted in submission order as soon as
 * a worker is free, their stream has no request in flight (each stream's
 * requests run in submission order) and the arena has room; requests of other
 * streams may pass one whose stream is busy, never one waiting for memory.
 * Each result is exactly what a standalone plan with the same parameters gives
 * for the same sequence of calls.  The caller owns every frame, record and
 * output buffer and keeps it alive until the request's lcp_server_wait
 * returns.
 *
 * Continuous batching (batch_frames > 0): requests of different streams that
 * are admissible together and use the temporal path (Sec. 5) -- compress
 * requests whose stream's LCP-FSM state (Sec. 7.2) or method sends the frame to
 * LCP-T, decompress requests of LCP-T records -- share one set of launches:
 * one residual (or decode) launch and one coding (or reconstruction) launch
 * for up to batch_frames requests holding up to batch_particles particles in
 * all, on batch scratch (one per worker) allocated for each (fields, chunk
 * size) when the first such stream opens (counted against hbm_budget_bytes).
 * A group forms when the first admissible request can be merged, a batch
 * scratch of its kind is free and at least one further pending request can
 * join it; otherwise that request runs alone as without merging.  Records, frames and
 * stream state are the same as without merging: a merged request whose LCP-T
 * record comes out larger than the stream's last LCP-S record, or whose record
 * turns out to be LCP-S, is put back at the front of the queue and runs
 * alone. */
typedef struct lcp_server_s* lcp_server_t;

typedef struct {
  uint64_t hbm_budget_bytes; /* stream state + scratch arena (0 = no limit on the state) */
  uint64_t scratch_bytes;    /* arena for in-flight requests' scratch (> 0) */
  int workers;               /* requests in flight at once, 1..16 */
  int device;                /* HIP device ordinal */
  int batch_frames;          /* most requests one merged launch takes: 0 (no merging)
                                or 2..64 */
  uint64_t batch_particles;  /* most particles of one merged launch (> 0 when
                                batch_frames > 0, < 2^32) */
} lcp_server_params;

enum { LCP_REQ_COMPRESS = 1, LCP_REQ_DECOMPRESS = 2 };

typedef struct {
  int kind;          /* LCP_REQ_COMPRESS or LCP_REQ_DECOMPRESS */
  int stream;        /* from lcp_server_open_stream */
  lcp_frame_in frame;  /* compress: the next frame of the stream */
  void* out;           /* compress: record destination (device, 4-byte aligned) */
  uint64_t out_cap;    /* compress: bytes available at out */
  lcp_blob blob;       /* decompress: the stream's next record (decode order = stream order) */
  lcp_frame_out dst;   /* decompress: where the frame goes */
  hipStream_t after;   /* the caller's stream (NULL: the null stream) that produces
                          the request's inputs and last used its outputs:
                          lcp_server_submit records an event on it, and the
                          request's work starts only after what was enqueued there
                          before the submit */
} lcp_request;

typedef struct {
  lcp_status status;   /* the lcp_compress / lcp_decompress status */
  int method;          /* compress: LCP_METHOD_S or LCP_METHOD_T */
  uint64_t bytes;      /* compress: record bytes; decompress: particles decoded */
  uint64_t t_submit_ns, t_start_ns, t_end_ns; /* steady clock: submitted, admitted, done */
  int group;           /* requests in the launch set that finished this one (1: alone) */
} lcp_result;

/* Create a server: allocates the arena and starts the workers.
 * Errors: LCP_ERR_ARG, LCP_ERR_DEVICE. */
lcp_status lcp_server_create(const lcp_server_params* params, lcp_server_t* out);

/* Stop the workers (requests still queued are dropped) and free everything. */
void lcp_server_destroy(lcp_server_t server);

/* Admit a stream: params must be multi-frame and name the server's device
 * (block_log2 == -1 searches on the sample, as lcp_plan does).  Fails with
 * LCP_ERR_BUDGET when the stream's state would exceed the budget left beside
 * the arena, or one request's scratch would not fit the arena. */
lcp_status lcp_server_open_stream(lcp_server_t server, const lcp_params* params,
                                  const float* const* sample_fields, uint64_t sample_n,
                                  int* stream_id);

/* Queue a request (copied); returns at once with a ticket.
 * Errors: LCP_ERR_ARG (unknown stream or kind), LCP_ERR_DEVICE (a worker failed). */
lcp_status lcp_server_submit(lcp_server_t server, const lcp_request* request, uint64_t* ticket);

/* Block until the request is done and return its result (once per ticket). */
lcp_status lcp_server_wait(lcp_server_t server, uint64_t ticket, lcp_result* result);

/* hold != 0: workers start no further request (those running finish) until
 * called again with hold == 0, so that a burst of submits is seen whole and
 * merged as far as it can be.  Waiting on a held request blocks until the
 * hold is lifted.  Errors: LCP_ERR_ARG (no server). */
lcp_status lcp_server_hold(lcp_server_t server, int hold);

/* Counters since creation: merged launch sets run, requests they finished,
 * requests they put back to run alone (any pointer may be NULL).
 * Errors: LCP_ERR_ARG (no server). */
lcp_status lcp_server_counts(lcp_server_t server, uint64_t* merged_launches,
                             uint64_t* merged_requests, uint64_t* requeued);

#ifdef __cplusplus
}
#endif
#endif
