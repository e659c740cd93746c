// lcp_internal.h -- host-side launchers of the LCP kernels (one translation unit
// per kernel family) and the plain-old-data structs passed to them by value.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include "../../include/lcp.h"
#include "lcp_common.h"

namespace lcp {

struct FieldPtrs {
  const float* p[kMaxF];
};
struct OutPtrs {
  float* p[kMaxF];
};

// Quantisation grid of every field, by value in kernel arguments.  int32
// grids keep the bits of their origin in m and of their half width in eb_q
// (the words the record stores).
struct GridDev {
  float m[kMaxF];
  float eb_q[kMaxF];
  double md[kMaxF];   // quantisation origin (see quantise)
  double inv[kMaxF];
  // temporal frames on a float32 grid: the largest |x| whose value keeps the
  // grid's rounding margin (|x| + 2 eb < 2^E in double arithmetic)
  float xmax[kMaxF];
  // temporal frames: the step of the codes on this grid (1, or the scale of
  // the anchor the grid was made for, Sec. 7.4.2)
  int32_t scale;
  int32_t dtype;  // kDtypeF32 or kDtypeI32
};

// One symbol array to be coded: u64 or u32 values; its length is n, or
// *n_dev when n_dev is set (block count known only on the device).
struct ArrIn {
  const void* v;
  int is64;
  const uint32_t* n_dev;
  uint64_t n;
  // non-null: v holds one byte per value, and 255 means the value is esc[i]
  // (temporal residuals, which are nearly all small)
  const uint32_t* esc;
};
constexpr int kWordParts = 16;
// Per-array coder workspace in device memory.
struct ArrWork {
  uint32_t hist[kAlphabet];
  uint32_t lc[kAlphabet];     // code | length << 16 (0 = unused symbol)
  uint32_t table[kAlphabet];  // used symbols in ascending order: symbol | length << 16
  unsigned long long maxv;
  uint32_t n, U, L, coder, w, nchunks;
  unsigned long long nbytes, off;
  // packed Huffman payload words, summed by the packing workgroups into
  // kWordParts spread totals (workgroup b adds to part b % kWordParts): a
  // device-scope atomic on one address is serialised across the chip, so a
  // single total would cost every packing workgroup one turn in that queue
  unsigned long long huff_words[kWordParts];
  unsigned long long huff_bits;  // code + raw bits of all symbols (no chunk padding)
  uint32_t cand, pad;            // Huffman may be the shorter coding: pack it
};

// Header fields of a record being written.
struct RecHdr {
  int mode, F, k, chunk_log2, A;
  int scale;  // temporal records: residual step (byte 11; 1 is written as 0)
  int dims;   // spatial records: spatial dimensions (byte 52; 3 is written as 0)
  int dtype;  // element type of the fields (byte 53)
  uint64_t n, seq, ref_seq;
  uint32_t bn[3];
  float m[kMaxF], eb_q[kMaxF];
};

// Encoder tables (device memory).  One launch set codes every array of every
// record of a call; workgroups find their array through per-launch prefix
// tables of workgroup counts (binary search), as the decoder does.
struct EncArr {
  ArrIn in;
  uint32_t rec;     // record of the call the array belongs to
  uint32_t copy0;   // first of its spread histogram copies in hist_part
  uint32_t copies;  // number of spread copies
  uint32_t pad;
  uint64_t cw0;     // first of its chunk words / look-back states
  uint64_t stage0;  // first word of its Huffman payload staging
};
struct EncRec {
  RecHdr h;
  const uint32_t* B_dev;  // spatial records: the block count (device)
  uint32_t a0, pad;       // first array of the record
  unsigned long long size, off;  // written by the layout kernel
};
// Workgroups given to an array of (at most) n values in each encode launch, its
// spread histogram copies, and its Huffman payload staging (words).
uint32_t enc_hist_blocks(uint64_t n);
uint32_t enc_hist_copies(uint64_t n);
uint32_t enc_chunk_blocks(uint64_t n, int chunk_log2, bool bytes);
uint32_t enc_copy_blocks(uint64_t n, int chunk_log2);
uint32_t enc_fixed_blocks(uint64_t n);
uint32_t enc_slot_words(bool is64, int chunk_log2);
uint64_t enc_stage_words(uint64_t n, bool is64, int chunk_log2);

// One frame of a spatial batch (device table).  Frames are concatenated: frame
// r owns slots [off, off + n) of every batch-wide array.  Per-particle kernels
// give each frame whole workgroups (first workgroup from a prefix table).
struct SegDev {
  const float* x[kMaxF];
  float m[kMaxF], eb_q[kMaxF];
  double md[kMaxF], inv[kMaxF];
  uint64_t n, off;
  uint64_t bn0, bn1;  // Eq. 6 block grid (1 along axes the data does not have)
  int k, D;           // block size log2, spatial dimensions (fields 0..D-1)
  int dtype, pad;     // kDtypeF32 or kDtypeI32
};
// One frame of a spatial decode batch (device table): frame r owns slots
// [off, off + n) and blocks [boff, boff + B) of the batch-wide arrays.
struct DSegDev {
  float* out[kMaxF];
  float m[kMaxF], eb_q[kMaxF];
  uint64_t n, off, B, boff, total_blocks;
  uint64_t bn0, bn1;
  int k, D;       // block size log2, spatial dimensions
  int dtype, pad;  // kDtypeF32 or kDtypeI32
};
constexpr int kMaxBatch = 1024;       // frames per spatial batch
constexpr uint32_t kSegExtCap = 256;  // extent workgroups per frame (at most)
constexpr uint32_t kSeg1k = 1024;     // slots per workgroup, element-wise kernels (decode side;
                                      // the encode side's tile is tuned, see TileShape)
constexpr uint32_t kSeg256 = 256;     // slots per workgroup, slot symbol kernel
uint32_t seg_ext_blocks(uint64_t n);

// One array of a record being decoded.
struct DecArr {
  const uint8_t* data;
  uint64_t nbytes, n;
  int coder, param;
  uint32_t used;
  void* out;
  int mode;        // 0 u64, 1 unzigzag -> int64 in u64, 2 u32, 3 unzigzag -> int32 in u32,
                   // 4 unzigzag -> int8 in out, -128 marking a value kept in esc (int32)
  uint64_t limit;  // raw values >= limit are corrupt
  int32_t* esc;    // mode 4: where values outside [-127, 127] go (same index)
};

// Device error word bits.
enum : uint32_t {
  kErrNonFinite = 1u,
  kErrCorrupt = 2u,
  kErrCapacity = 4u,
  kErrRange = 8u,  // a temporal frame left its reference grid's range
  // a temporal frame whose packing was to build its own code found an alphabet
  // beyond one wave's (the frame is coded again with the separate build)
  kErrRebuild = 16u,
};

// ---- kernel timer (lcp_host.hip) ----
// When the named kernel is being timed, ktimer_events hands out the pair of HIP
// events for one launch and records `bytes`, the launch's algorithmic traffic.
// The events ride on the kernel's own dispatch (hipExtLaunchKernel), so they
// time the kernel alone and add no marker packets between kernels.
bool ktimer_events(const char* name, uint64_t bytes, hipEvent_t* start, hipEvent_t* stop);
template <typename K, typename... A>
inline void launch_timed(const char* name, uint64_t bytes, K kernel, dim3 grid, dim3 block,
                         uint32_t shm, hipStream_t s, A... args) {
  hipEvent_t a, b;
  if (ktimer_events(name, bytes, &a, &b))
    hipExtLaunchKernelGGL(kernel, grid, block, shm, s, a, b, 0, args...);
  else
    kernel<<<grid, block, shm, s>>>(args...);
}

// ---- lcp_host.hip: the server's merged temporal launches ----
// A batch plan holds the scratch of one merged launch: up to `frames` temporal
// frames of different streams with F fields and chunk size chunk_log2, and
// `particles` particles in all.
lcp_status serve_batch_create(int F, int chunk_log2, int frames, uint64_t particles, int device,
                              lcp_plan_s** out);
size_t serve_batch_bytes(lcp_plan_s* B);
int serve_batch_fields(lcp_plan_s* B);
int serve_batch_frames(lcp_plan_s* B);
uint64_t serve_batch_particles(lcp_plan_s* B);
int plan_fields(lcp_plan_s* P);
int plan_chunk_log2(lcp_plan_s* P);
// Whether the stream's last decoded record was LCP-T (its next one likely is).
bool plan_decoding_t(lcp_plan_s* P);
bool plan_multi_frame(lcp_plan_s* P);
int plan_batch_size(lcp_plan_s* P);
uint64_t plan_max_particles(lcp_plan_s* P);
// Whether a compress request of the stream can join a merged launch (its frame
// goes to LCP-T against a resident reference whatever the size comparison).
bool serve_t_eligible(lcp_plan_s* P, const lcp_frame_in& fr);
// K requests of K different streams (plans[i], its next frame or record): one
// residual (or decode) launch, one coding (or reconstruction) launch for all.
// done[i]: request i is finished exactly as the stream's own lcp_compress /
// lcp_decompress would have finished it (stream state committed; size or
// particle count in sizes / n_out); otherwise nothing of its stream changed
// and it must take its own call.
lcp_status serve_t_compress(lcp_plan_s* B, int K, lcp_plan_s* const* plans,
                            const lcp_frame_in* frames, void* const* outs, const uint64_t* caps,
                            bool* done, uint64_t* sizes, hipStream_t s);
lcp_status serve_t_decompress(lcp_plan_s* B, int K, lcp_plan_s* const* plans,
                              const lcp_blob* blobs, const lcp_frame_out* dsts, bool* done,
                              uint64_t* n_out, hipStream_t s);

// ---- lcp_host.hip: plans whose scratch is bound per call (the server) ----
// A plan with its stream state but no scratch; the block-size search, if asked
// for, runs on temporary scratch.  Before each call, plan_bind points the plan
// at plan_scratch_bytes of device memory and plan_host_bytes of pinned host
// memory (and clears what must start at zero, on stream s).
lcp_status plan_create_unbound(const lcp_params* params, const float* const* sample_fields,
                               uint64_t sample_n, lcp_plan_s** out);
size_t plan_scratch_bytes(lcp_plan_s* P);
size_t plan_host_bytes(lcp_plan_s* P);
size_t plan_state_bytes(lcp_plan_s* P);
void plan_bind(lcp_plan_s* P, void* dev, void* host, hipStream_t s);
// Marks the plan's scratch as gone (its memory returned to the server's arena):
// compress and decompress then fail with LCP_ERR_ARG until the next plan_bind.
void plan_unbind(lcp_plan_s* P);

// ---- kernels_core.hip ----
// Spatial batch front end.  pre_* are device prefix tables (R + 1 entries) of
// the workgroups each frame gets: seg_ext_blocks(n), ceil(n / kSeg1k),
// ceil(n / kSeg256) and ceil(n / kSortTile).  ext receives R x 2F sortable keys (min, max per field).
void launch_extent_b(const SegDev* S, const uint32_t* pre_ext, uint32_t ext_blocks, int R, int F,
                     uint32_t* ext, uint32_t* part, uint32_t* err, uint64_t bytes, hipStream_t s);
// rec receives, per particle in input order, a record of slot_rec_words(F, D)
// words: its D in-block offsets (16 bits apart; word 0 for up to two axes,
// words 0-1 for three) and its supplementary fields' codes after them.
int slot_rec_words(int F, int D);
// The element-wise encode kernels of a batch walk `tiles` tiles of `tile`
// slots (a multiple of 256; the prefix tables count tiles per frame) with a
// persistent grid of `grid` workgroups (0: one workgroup per tile).  Launch
// shape only: the results do not depend on it.
struct TileShape {
  uint32_t tile, tiles, grid;
};
void launch_quant_key_b(const SegDev* S, const uint32_t* pre_tile, const TileShape& ts, int R,
                        int F, int D, uint64_t* keys, uint32_t* vals, uint32_t* rec, uint64_t ntot,
                        bool key32, hipStream_t s);
// Non-empty blocks of every frame: ids, global start slots,
// rstart[r] (first block of frame r; rstart[R] = all blocks) and Bs[r].
void launch_runs_b(const uint64_t* keys, const SegDev* S, const uint32_t* pre_tile,
                   const TileShape& ts, int R, uint64_t ntot, uint32_t* flags_scan, uint64_t* ids,
                   uint32_t* starts, uint32_t* rstart, uint32_t* Bs, uint32_t* tmp32,
                   bool key32, hipStream_t s);
// Block symbols of frame r go to v_id / v_cnt + S[r].off.
void launch_block_syms_b(const uint64_t* ids, const uint32_t* starts, const uint32_t* rstart,
                         int R, const SegDev* S, uint64_t ntot, uint64_t* v_id, uint64_t* v_cnt,
                         hipStream_t s);
// v_rel: [3][ntot], v_sup: [F-3][ntot]; q_slot (nullable): [F][ntot]; keys:
// the sorted block keys (slot order).
void launch_slot_syms_b(const SegDev* S, const uint32_t* pre_256, uint32_t tiles, uint32_t grid,
                        int R, int F, int D, const uint32_t* perm, const uint64_t* keys,
                        const uint32_t* rec, uint64_t ntot, uint32_t* v_rel, uint32_t* v_sup,
                        int32_t* q_slot, bool key32, hipStream_t s);
// dst[r] (device table of device pointers, entries may be null) <- perm slice of frame r.
void launch_copy_perm_b(const uint32_t* perm, const SegDev* S, const uint32_t* pre_tile,
                        const TileShape& ts, int R, uint32_t* const* dst, hipStream_t s);

// Keys are u32 (key32: every block id below 2^32) or u64 in the same buffers.
// Stable LSD radix sort of (key, value) by the low `bits` key bits, within
// each frame of the SegDev table (pre_tile: ceil(n / kSortTile) tiles per
// frame, ntiles in all; hist: 256 * ntiles u32).  Returns the buffer index
// (0: k0/v0, 1: k1/v1) that holds the result.
constexpr uint32_t kSortTile = 4096;
// The buffer (0: k0/v0, 1: k1/v1) a sort of `bits` key bits leaves its result in.
int radix_result(int bits);
int radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, const SegDev* S,
               const uint32_t* pre_tile, uint32_t ntiles, int R, uint64_t ntot, int bits,
               uint32_t* hist, uint32_t* tmp32, bool key32, hipStream_t s);
template <typename T>
void scan_device(T* data, uint64_t n, const uint32_t* n_dev, bool exclusive, T* tmp,
                 hipStream_t s);
// Inclusive scans of nd <= 4 u32 arrays of length n in one set of launches
// (tmp: scan_tmp_elems(n) u64 of scratch, as for scan_device).
void scan_device4(uint32_t* const* arrs, int nd, uint64_t n, uint32_t* tmp, hipStream_t s);
size_t scan_tmp_elems(uint64_t n);
// Spatial batch decode.  seg_rebase turns batch-wide inclusive scans of nd
// arrays (X + d * stride) into per-frame ones (segments by slot or, with
// by_block, by block; pre: ceil(len / kSeg1k) workgroups per frame; bases:
// nd * R scratch values).
template <typename T>
void seg_rebase(T* X, uint64_t stride, int nd, const DSegDev* D, const uint32_t* pre,
                uint32_t blocks, int R, bool by_block, T* bases, hipStream_t s);
void launch_s_blocks_b(const uint64_t* ids, const uint64_t* cnt, const uint64_t* cum,
                       const DSegDev* D, const uint32_t* pre_blk, uint32_t blocks, int R,
                       uint64_t Btot, uint64_t ntot, uint32_t* corner, uint32_t* mark,
                       uint32_t* err, hipStream_t s);
void launch_s_recon_b(const uint32_t* blk, const uint32_t* corner, const uint32_t* v,
                      const DSegDev* D, const uint32_t* pre_slot, uint32_t blocks, int R, int F,
                      uint64_t Btot, uint64_t ntot, uint32_t* err, hipStream_t s);
// LCP-T residuals; err gets kErrNonFinite / kErrRange when the frame cannot be
// coded on the reference grid.
// The residual symbols of field f are also counted into array f's spread
// histogram copies (hist_part / hist_max, as launch_encode expects them).
// Residuals go to v8 as bytes (255: the value is in v_res, written for such
// values only), or to v_res as u32 when v8 is null.  zero_words (may be null):
// the F work records whose Huffman word totals are cleared for the packing
// that builds its own code.
void launch_t_resid(const FieldPtrs& x, int F, uint64_t n, const GridDev& g,
                    const uint32_t* perm_ref, const int32_t* q_ref, uint8_t* v8, uint32_t* v_res,
                    int32_t* q_new, uint32_t* err, uint32_t* hist_part,
                    unsigned long long* hist_max, ArrWork* zero_words, hipStream_t s);
// A temporal run: up to kRunMax frames coded as a chain on one reference grid
// and slot order in one launch (frame j's fields fr.x[j]); see k_t_resid_run.
constexpr int kRunMax = 32;
// Frames one run launch can take at F fields (kRunMax, or fewer for wide F).
int run_launch_frames(int F);
struct RunFrames {
  const float* x[kRunMax][kMaxF];
};
void launch_t_resid_run(const RunFrames& fr, int J, int F, uint64_t n, const GridDev& g,
                        const uint32_t* perm, const int32_t* q_ref, int32_t* q_last, uint8_t* v8,
                        uint32_t* vesc, uint64_t astride, int a0, uint32_t* hist_part,
                        unsigned long long* hist_max, int copies, ArrWork* zero_words,
                        uint32_t* err, int err_stride, hipStream_t s);
// Temporal frames of different streams in one launch (the served form): each
// frame has its own size, reference grid, slot order and reference codes, and
// its own residual buffers; workgroups find their frame through a prefix table
// of per-frame workgroup counts.  Frame r's arrays are r * F + f of the launch
// (histogram copies [(r F + f) copies, +copies), work records zw[r F + f]).
struct TFrameDev {
  const float* x[kMaxF];
  const uint32_t* perm;   // reference slot -> input index
  const int32_t* q_ref;   // reference codes [F][n]
  int32_t* q_new;         // the frame's codes [F][n]
  uint8_t* v8;            // residual bytes, field f at v8 + f * n
  uint32_t* esc;          // escaped residuals, field f at esc + f * n
  uint32_t* err;          // the frame's error word
  uint64_t n;
  int vec, pad;
  GridDev g;
};
uint32_t t_multi_blocks(uint64_t n, int vec);
void launch_t_resid_multi(const TFrameDev* frames, const uint32_t* pre, uint32_t blocks, int R,
                          int F, uint32_t* hist_part, unsigned long long* hist_max, int copies,
                          ArrWork* zero_words, uint64_t bytes, hipStream_t s);
// Temporal frames of different streams reconstructed in one launch: frame r's
// residual bytes (-128: the int32 residual is in out[f] at the same index) are
// added to its reference codes; the values go to out, the codes to q_new.
struct TReconDev {
  const int32_t* q_ref;
  int32_t* q_new;
  const int8_t* r8;  // field f at r8 + f * n
  float* out[kMaxF];
  uint64_t n;
  float m[kMaxF], eb_q[kMaxF];
  int32_t scale, dtype;
};
void launch_t_recon_multi(const TReconDev* frames, const uint32_t* pre, uint32_t blocks, int R,
                          int F, uint32_t* err, uint64_t bytes, hipStream_t s);
void launch_s_blocks(const uint64_t* ids, const uint64_t* cnt, uint64_t* cum, uint64_t B,
                     uint64_t n, uint64_t total_blocks, const uint32_t* bn, int k,
                     uint32_t* corner, uint32_t* mark, uint32_t* err, hipStream_t s);
// Reconstruction in place: out.p[f] holds the decoded u32 symbols (scanned
// relative positions for f < 3, codes for supplementary fields) and receives
// the float32 values.
void launch_s_recon(const uint32_t* blk, const uint32_t* corner, uint64_t B, int F, int D, uint64_t n,
                    int k, const GridDev& g, const OutPtrs& out, int32_t* q_slot, uint32_t* err,
                    hipStream_t s);
// The codes the last of J temporal frames leaves as the next reference: with
// step 1 (g.scale) they are its own Eq. 5 codes (only frame J - 1 is read,
// q_ref is unused); with a larger step they follow the chain of frames from
// the codes q_ref of the frames' first reference.
void launch_t_codes(const RunFrames& fr, int J, int F, uint64_t n, const GridDev& g,
                    const uint32_t* perm_ref, const int32_t* q_ref, int32_t* q_new,
                    uint32_t* err, hipStream_t s);
void launch_t_recon(const int32_t* q_ref, int F, uint64_t n, const GridDev& g,
                    const OutPtrs& out, int32_t* q_slot, uint32_t* err, hipStream_t s);
// Copies `bytes` (a multiple of 4) from host memory to device memory through
// kernel arguments, kInstallWords words per launch (the host buffer may be
// reused as soon as this returns).
constexpr int kInstallWords = 512;
void launch_install(const void* src, void* dst, size_t bytes, hipStream_t s);
// The same for a table in pinned host memory (bytes a multiple of 4) that one
// kernel reads itself: the source must stay untouched until the stream has
// passed the launch, and the launch must not be captured into a graph.
void launch_fetch_host(const void* host_src, void* dst, size_t bytes, hipStream_t s);
// A chain of up to kChainMax temporal frames reconstructed in one pass:
// out.p[j][f] holds frame j's int32 residuals and receives its values; frame
// 0's reference codes are q_ref; q_last (nullable) receives the last frame's.
constexpr int kChainMax = 16;
struct ChainOut {
  float* p[kChainMax][kMaxF];
  // non-null: the frame's residuals as int8 (-128: the int32 residual is in p
  // at the same index); null: the int32 residuals are in p itself
  const int8_t* r8[kChainMax][kMaxF];
};
void launch_t_recon_chain(const int32_t* q_ref, int F, uint64_t n, const GridDev& g,
                          const ChainOut& out, int J, int32_t* q_last, uint32_t* err,
                          hipStream_t s);
void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
// tab: nrec (device pointer, byte size) pairs; dst: nrec * stage bytes.
void launch_gather_headers(const uint64_t* tab, int nrec, int stage, uint8_t* dst, hipStream_t s);
void launch_copy_perm(const uint32_t* src, uint32_t* dst, uint64_t n, hipStream_t s);
// Record r (src bytes [offs[r], offs[r+1])) to the device pointer tab[2r] when
// its size is at most tab[2r + 1].
void launch_scatter_records(const unsigned long long* offs, const uint8_t* src, const uint64_t* tab,
                            int R, hipStream_t s);

// ---- kernels_codec.hip ----
// Workgroups per array in the histogram pass (at most); their counts meet in
// up to kHistCopies spread copies per array (hist_part: kAlphabet u32 per copy,
// hist_max: one u64 per copy), zero between uses.
constexpr int kHistBlocks = 1024;
constexpr int kHistCopies = 32;
// Candidate halving counts built side by side (huff_lens: arrays * 32 *
// kAlphabet bytes, huff_maxd: arrays * 32 u32).
constexpr int kHuffCandidates = 32;
// One encode launch set: NA arrays of R records (tables in device memory);
// pre_dev holds three prefix tables of NA + 1 workgroup counts (histogram,
// chunk, fixed-length pack), whose totals are given.  Records are placed back
// to back at out + offs[r] (offs: R + 1 device values, offs[R] = total bytes);
// a total beyond cap sets kErrCapacity and nothing is packed.  With hist_done
// the histograms are already in the spread copies.
struct EncLaunch {
  const EncArr* arrs;
  EncRec* recs;     // the layout writes every record's size and offset here
  EncRec rec0;      // the first record's header (the only one read when R == 1)
  const uint32_t* pre;
  int NA, R;
  uint32_t hist_blocks, chunk_blocks, fixed_blocks, copy_blocks;
  uint64_t values;  // sum of the arrays' lengths (bounds), for the kernel timer
  int all_bytes;    // every array holds bytes with escapes (temporal residuals)
  // temporal record whose packing builds the code itself (all_bytes, a chunk
  // per wave): no build launch; the emit clears the histogram copies
  int fused;
  // non-null: a record whose packing could not build its code flags
  // kErrRebuild at err_rec + record * err_stride instead of in the launch's
  // error word (a run of temporal records learns which frame it was)
  uint32_t* err_rec;
  int err_stride;
};
// Coding scratch of a launch set: a word count per chunk and the staging of
// the Huffman payloads before they move into their records.
struct EncScratch {
  uint32_t* chunk_words;  // word count per chunk
  uint32_t* stage;        // one slot per chunk (enc_slot_words)
  uint32_t* hist_part;
  unsigned long long* hist_max;
  uint8_t* huff_lens;
  uint32_t* huff_maxd;
};
// Records go to out + offs[r]; with `base` (device, nullable) the first
// record starts at *base rather than at 0, cap bounding the end either way.
void launch_encode(const EncLaunch& L, int chunk_log2, ArrWork* work, const EncScratch& X,
                   uint8_t* out, uint64_t cap, unsigned long long* offs, uint32_t* err,
                   const unsigned long long* base, bool hist_done, hipStream_t s);
// Workgroups needed by one array in the Huffman (huff=true) or fixed-length
// decode launch (0 when the array uses the other coder).
uint32_t decode_blocks(const DecArr& d, int chunk_log2, bool huff);
// Decode A arrays (descriptors in device memory).  *_prefix_dev[a] is the first
// workgroup of array a in each launch (A entries); lut holds 2^13 entries per array.
// lut_log2: the longest Huffman code among the arrays (sizes the LDS table).
void launch_decode(const DecArr* arrs_dev, int A, const uint32_t* huff_prefix_dev,
                   uint32_t huff_blocks, const uint32_t* fixed_prefix_dev, uint32_t fixed_blocks,
                   int chunk_log2, int lut_log2, uint64_t bytes, uint32_t* lut, uint32_t* err,
                   hipStream_t s);

}  // namespace lcp
