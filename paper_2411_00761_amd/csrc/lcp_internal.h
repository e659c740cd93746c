// lcp_internal.h -- host-side launchers of the LCP kernels (one translation unit
// per kernel family) and the plain-old-data structs passed to them by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lcp_common.h"

namespace lcp {

struct FieldPtrs {
  const float* p[kMaxF];
};
struct OutPtrs {
  float* p[kMaxF];
};

// Quantisation grid of every field, by value in kernel arguments.
struct GridDev {
  float m[kMaxF];
  float eb_q[kMaxF];
  double inv[kMaxF];
  double eb2[kMaxF];  // 2 * the user's bound (temporal feasibility check)
  double lim[kMaxF];  // 2^E: |x| + 2 eb must stay below it on this grid
};

// One symbol array to be coded: u64 or u32 values; its length is n, or
// *n_dev when n_dev is set (block count known only on the device).
struct ArrIn {
  const void* v;
  int is64;
  const uint32_t* n_dev;
  uint64_t n;
};
struct ArrSet {
  ArrIn a[kMaxArrays];
  int A;
};

// Per-array coder workspace in device memory.
struct ArrWork {
  uint32_t hist[kAlphabet];
  uint32_t lc[kAlphabet];     // code | length << 16 (0 = unused symbol)
  uint32_t table[kAlphabet];  // used symbols in ascending order: symbol | length << 16
  unsigned long long maxv;
  uint32_t n, U, L, coder, w, nchunks;
  unsigned long long huff_words, nbytes, off;
};

// Header fields of a record being written.
struct RecHdr {
  int mode, F, k, chunk_log2, A;
  uint64_t n, seq, ref_seq;
  uint32_t bn[3];
  float m[kMaxF], eb_q[kMaxF];
};

// One array of a record being decoded.
struct DecArr {
  const uint8_t* data;
  uint64_t nbytes, n;
  int coder, param;
  uint32_t used;
  void* out;
  int mode;        // 0 u64, 1 unzigzag -> int64 in u64, 2 u32, 3 unzigzag -> int32 in u32
  uint64_t limit;  // raw values >= limit are corrupt
};

// Device error word bits.
enum : uint32_t {
  kErrNonFinite = 1u,
  kErrCorrupt = 2u,
  kErrCapacity = 4u,
  kErrRange = 8u,  // a temporal frame left its reference grid's range
};

// ---- kernel timer (lcp_host.hip) ----
// When the named kernel is being timed, its launches are bracketed by HIP events
// on their stream; `bytes` is the launch's algorithmic traffic.
bool ktimer_on(const char* name);
void ktimer_begin(hipStream_t s);
void ktimer_end(hipStream_t s, uint64_t bytes);
#define LCP_TIMED(name, bytes, stream, ...)        \
  do {                                             \
    bool timed_ = ::lcp::ktimer_on(name);          \
    if (timed_) ::lcp::ktimer_begin(stream);       \
    __VA_ARGS__;                                   \
    if (timed_) ::lcp::ktimer_end(stream, (bytes)); \
  } while (0)

// ---- kernels_core.hip ----
// Per-field extent as sortable keys ext[2f] (min), ext[2f+1] (max); part holds
// 2 * F * 256 partials; err gets kErrNonFinite for NaN/Inf input (it is not cleared).
void launch_extent(const FieldPtrs& x, int F, uint64_t n, uint32_t* ext, uint32_t* part,
                   uint32_t* err, hipStream_t s);
void launch_quant_key(const FieldPtrs& x, uint64_t n, const GridDev& g, int k, uint64_t bn0,
                      uint64_t bn1, uint64_t* keys, uint32_t* vals, hipStream_t s);
// Stable LSD radix sort of (key, value) by the low `bits` key bits.  Returns the
// buffer index (0: k0/v0, 1: k1/v1) that holds the result.
int radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint64_t n, int bits,
               uint32_t* hist, uint32_t* tmp32, hipStream_t s);
template <typename T>
void scan_device(T* data, uint64_t n, const uint32_t* n_dev, bool exclusive, T* tmp,
                 hipStream_t s);
size_t scan_tmp_elems(uint64_t n);
void launch_runs(const uint64_t* keys, uint64_t n, uint32_t* flags_scan, uint64_t* ids,
                 uint32_t* starts, uint32_t* B_dev, uint32_t* tmp32, hipStream_t s);
void launch_block_syms(const uint64_t* ids, const uint32_t* starts, const uint32_t* B_dev,
                       uint64_t n, uint64_t* v_id, uint64_t* v_cnt, hipStream_t s);
void launch_slot_syms(const FieldPtrs& x, int F, uint64_t n, const GridDev& g, int k,
                      const uint32_t* perm, uint32_t* v_rel, uint32_t* v_sup, int32_t* q_slot,
                      hipStream_t s);
// LCP-T residuals; err gets kErrNonFinite / kErrRange when the frame cannot be
// coded on the reference grid.
// The residual symbols of field f are also counted into array f's spread
// histogram copies (hist_part / hist_max, as launch_encode expects them).
void launch_t_resid(const FieldPtrs& x, int F, uint64_t n, const GridDev& g,
                    const uint32_t* perm_ref, const int32_t* q_ref, uint32_t* v_res,
                    int32_t* q_new, uint32_t* err, uint32_t* hist_part,
                    unsigned long long* hist_max, hipStream_t s);
void launch_s_blocks(const uint64_t* ids, const uint64_t* cnt, uint64_t* cum, uint64_t B,
                     uint64_t n, uint64_t total_blocks, const uint32_t* bn, int k,
                     uint32_t* corner, uint32_t* mark, uint32_t* err, hipStream_t s);
// Reconstruction in place: out.p[f] holds the decoded u32 symbols (scanned
// relative positions for f < 3, codes for supplementary fields) and receives
// the float32 values.
void launch_s_recon(const uint32_t* blk, const uint32_t* corner, uint64_t B, int F, uint64_t n,
                    int k, const GridDev& g, const OutPtrs& out, int32_t* q_slot, uint32_t* err,
                    hipStream_t s);
// out.p[f] holds int32 residuals; q_slot receives q_ref + residual.
void launch_t_recon(const int32_t* q_ref, int F, uint64_t n, const GridDev& g,
                    const OutPtrs& out, int32_t* q_slot, uint32_t* err, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
// tab: nrec (device pointer, byte size) pairs; dst: nrec * stage bytes.
void launch_gather_headers(const uint64_t* tab, int nrec, int stage, uint8_t* dst, hipStream_t s);
void launch_copy_perm(const uint32_t* src, uint32_t* dst, uint64_t n, hipStream_t s);

// ---- kernels_codec.hip ----
// Workgroups per array in the histogram pass; their counts meet in kHistCopies
// spread copies per array (hist_part: kMaxArrays * kHistCopies * kAlphabet u32,
// hist_max: kMaxArrays * kHistCopies u64), zero between uses.
constexpr int kHistBlocks = 1024;
constexpr int kHistCopies = 32;
// Candidate halving counts built side by side (huff_lens: kMaxArrays * 32 *
// kAlphabet bytes, huff_maxd: kMaxArrays * 32 u32).
constexpr int kHuffCandidates = 32;
void launch_encode(const ArrSet& set, uint64_t max_n, int chunk_log2, ArrWork* work,
                   uint32_t* chunk_words, uint64_t max_chunks, uint32_t* hist_part,
                   unsigned long long* hist_max, uint8_t* huff_lens, uint32_t* huff_maxd,
                   const RecHdr& h, const uint32_t* B_dev, uint8_t* out, uint64_t cap,
                   unsigned long long* size_dev, uint32_t* err, bool hist_done, hipStream_t s);
// Workgroups needed by one array in the Huffman (huff=true) or fixed-length
// decode launch (0 when the array uses the other coder).
uint32_t decode_blocks(const DecArr& d, int chunk_log2, bool huff);
// Decode A arrays (descriptors in device memory).  *_prefix_dev[a] is the first
// workgroup of array a in each launch (A entries); lut holds 2^13 entries per array.
void launch_decode(const DecArr* arrs_dev, int A, const uint32_t* huff_prefix_dev,
                   uint32_t huff_blocks, const uint32_t* fixed_prefix_dev, uint32_t fixed_blocks,
                   int chunk_log2, uint64_t bytes, uint32_t* lut, uint32_t* err, hipStream_t s);

}  // namespace lcp
