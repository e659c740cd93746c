// lcp_host.hip -- the C ABI declared in include/lcp.h: plans, the LCP-S and
// LCP-T pipelines, LCP-FSM (Sec. 7.2) with Alg. 1's reference/anchor rule
// (Sec. 7.3), block-size search (Sec. 7.4.1), decode, and the kernel timer.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <initializer_list>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lcp.h"
#include "lcp_internal.h"

using namespace lcp;

namespace {

// Temporal frames coded back to back before the host reads their outcomes: a
// run starts at kTRunStart frames and doubles after each run that commits in
// full, up to kTRun; a run broken part-way starts over at kTRunStart, so the
// work a misprediction throws away stays small while long T stretches pay one
// host round trip per kTRun frames.
constexpr int kTRun = 32;
constexpr int kTRunStart = 8;
// The kernel timer brackets one launch in kTimerStride (or the stride the
// name asks for) of the named kernel: each timed launch costs the stream some
// microseconds on either side (the events' own packets), which a sampled
// average keeps out of the rest.
constexpr uint64_t kTimerStride = 16;
// Temporal frames whose residuals one decode launch keeps as bytes.
constexpr int kDecSlots = kChainMax;

// ------------------------------------------------------------------ grids
// int32 grids (dtype kDtypeI32) keep the bits of their origin in m and of
// their half width in eb_q: the two words the record stores.
struct HostGrid {
  float m, eb_q;
  double md, inv, eb;
  int E;
  int dtype;
};

// Eq. 5 with a float32 output.  Every reconstruction of the field lies below
// 2^E in magnitude, where 2^E is the first power of two above the double sum
// top = max(|lo|, |hi|) + 2 eb (E at least -100).  Rounding an exact bin centre
// to float32 there costs at most half an ulp of the binade [2^(E-1), 2^E),
// i.e. 2^(E-24), so the half bin width eb_q is the largest float32 not above
// eb - 2^(E-24); a bound below two such half ulps is refused.  The exponents
// and the rounding toward zero are read off the IEEE-754 bit fields.
lcp_status make_grid(float lo, float hi, double eb, HostGrid* g) {
  if (!isfinite(lo) || !isfinite(hi) || !(eb > 0) || !isfinite(eb)) return LCP_ERR_ARG;
  const double alo = lo < 0 ? -(double)lo : (double)lo;
  const double ahi = hi < 0 ? -(double)hi : (double)hi;
  const double top = (alo > ahi ? alo : ahi) + 2.0 * eb;
  uint64_t tb;
  memcpy(&tb, &top, 8);
  const int top_biased = (int)((tb >> 52) & 0x7FF);
  if (top_biased == 0x7FF) return LCP_ERR_RANGE;  // the bound overflows the double range
  // top = 1.f x 2^(biased - 1023) < 2^(biased - 1022); a subnormal or zero top
  // is far below the floor of -100
  int E = top_biased == 0 ? -100 : top_biased - 1022;
  if (E < -100) E = -100;
  uint64_t db = (uint64_t)(E - 24 + 1023) << 52;  // 2^(E-24), a normal double here
  double half_ulp;
  memcpy(&half_ulp, &db, 8);
  if (eb < half_ulp * 2) return LCP_ERR_EB_TOO_SMALL;
  // exact: half_ulp is a power of two no larger than eb / 2
  const double t = eb - half_ulp;
  uint64_t u;
  memcpy(&u, &t, 8);
  const int te = (int)((u >> 52) & 0x7FF) - 1023;  // t in [2^te, 2^(te+1))
  uint32_t fb;
  if (te > 127) fb = 0x7F7FFFFFu;  // above every float32: the largest one
  else if (te < -126) return LCP_ERR_EB_TOO_SMALL;
  else fb = ((uint32_t)(te + 127) << 23) | (uint32_t)((u >> 29) & 0x7FFFFFu);  // truncate
  float e;
  memcpy(&e, &fb, 4);
  g->m = lo;
  g->eb_q = e;
  g->md = (double)lo;
  g->inv = 0.5 / (double)e;  // 2 e is exact, so this is the rounding of 1 / (2 e)
  g->eb = eb;
  g->E = E;
  g->dtype = kDtypeF32;
  return LCP_OK;
}

// int32 fields (Sec. 3 allows integer data): a bin is a run of w = 2 hb + 1
// consecutive integers from the field's minimum and decodes to its centre, an
// integer within hb of every member, so no rounding margin is needed and
// hb = floor(eb) (at most 2^31 - 1, enough for any int32 range) is the widest
// bin the bound allows.  For an anchor whose temporal frames move by s bins
// (Sec. 7.4.2) their error reaches (s w - 1) / 2, so w is the largest odd
// integer with s w <= 2 floor(eb) + 1; none exists when that is below s.
lcp_status make_grid_i(int32_t lo, double eb, int s, HostGrid* g) {
  if (!(eb >= 0) || s < 1 || !(s & 1)) return LCP_ERR_ARG;
  const uint64_t b = eb >= 2147483647.0 ? 2147483647ull : (uint64_t)eb;  // eb >= 0: floor
  uint64_t w = (2 * b + 1) / (uint64_t)s;
  if (w == 0) return LCP_ERR_EB_TOO_SMALL;
  if (!(w & 1)) w -= 1;
  const uint32_t hb = (uint32_t)((w - 1) / 2);
  memcpy(&g->m, &lo, 4);
  memcpy(&g->eb_q, &hb, 4);
  g->md = (double)lo - 0.5;  // see quantise: floor((x - m + 1/2) / w) = floor((x - m) / w)
  g->inv = 1.0 / (double)w;
  g->eb = eb;
  g->E = 0;
  g->dtype = kDtypeI32;
  return LCP_OK;
}

// The code of an extent value (float32 or int32, exact in double), as the
// device computes it.
int64_t host_quant(double x, const HostGrid& g) {
  return (int64_t)floor((x - g.md) * g.inv);
}

// ------------------------------------------------------------------ device buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct RefState {
  bool valid = false;
  int scale = 1;  // the grid's step against the stream's bound: 1, or an anchor's scale
  uint64_t seq = 0, n = 0;
  HostGrid grid[kMaxF];
  int q = -1;     // index into the q pool
  int perm = -1;  // index into the perm pool (compress side)
};

}  // namespace

struct lcp_plan_s {
  lcp_params p{};
  int k = 0;
  int F = 3;
  int chunk_log2 = 10;
  uint64_t N = 0;   // max particles per frame
  uint64_t NB = 0;  // max particles per spatial batch (>= N)
  int RB = 1;       // max frames per spatial batch
  int NAmax = 0;    // max coded arrays per encode launch set
  uint64_t hist_copies = 0, cw_cap = 0, stage_cap = 0;
  // memory: scratch (device + pinned host tables) is either owned (standalone
  // plans) or bound per call by a server; the stream state is always owned
  void* own_dev = nullptr;   // owned device scratch block
  void* own_host = nullptr;  // owned pinned host block
  void* state_dev = nullptr; // reference codes and permutations
  // the scratch pointers below address live memory: set by bind_scratch,
  // cleared when a server takes the memory back (or the search's temporary
  // scratch is freed); compress and decompress refuse to run without it
  bool bound = false;
  // scratch laid out for LCP-S compression only (no decode tables): the
  // library's static scratch, which must stay small
  bool compress_only = false;
  // scratch of a server's merged temporal launches: up to RB frames of
  // different streams, NB particles in all (residual bytes, escapes, coder,
  // decoder and frame tables; no spatial buffers)
  bool serve_batch = false;
  TFrameDev *tfr_host = nullptr, *tfr_dev = nullptr;
  TReconDev *trc_host = nullptr, *trc_dev = nullptr;
  uint32_t *spre_host = nullptr, *spre_dev = nullptr;        // [RB + 1] workgroup prefix
  unsigned long long *sret_host = nullptr, *sret_dev = nullptr;  // [RB] errs, [RB + 1] offsets, launch err
  uint64_t *sdst_host = nullptr, *sdst_dev = nullptr;        // [RB] (destination, capacity)
  size_t scratch_bytes = 0, host_bytes = 0, state_bytes = 0;

  // scratch (batch-wide arrays hold NB slots)
  uint64_t *keys0, *keys1, *ids, *v_id, *v_cnt;
  uint32_t* slot_rec;  // per particle: in-block offsets and supplementary codes
  uint32_t *vals0, *vals1, *hist, *flags, *starts, *v_slot, *chunk_words, *lut, *corner;
  uint8_t* v_byte;  // temporal residuals as bytes (multi-frame plans; escapes in v_slot)
  int8_t* dres8;    // decoded temporal residuals as bytes, kDecSlots frames (multi-frame)
  uint32_t* stage;  // Huffman payload staging, one slot per chunk
  uint64_t* scan_tmp;
  size_t scan_tmp_n;
  ArrWork* work;
  // device return block (one read back per sync): [0] error word, [1, RB + 2)
  // record offsets, then RB x 2F extent keys; ret_host is its pinned mirror
  unsigned long long *ret_dev, *ret_host;
  uint32_t* err;  // the error word (low half of ret_dev[0])
  bool err_clean = false;  // the error word is known to be zero at the stream's tail
  bool run_clean = false;  // ... and so is a run's return block (cleared behind its read-back)
  bool host_pinned = true;  // the bound host tables are pinned (a kernel may read them)
  int run_len = kTRunStart;  // frames the next temporal run may take
  // temporal frames left to code with the separate code build, after a frame
  // whose residual alphabet outgrew the packing kernel's own build
  int fuse_skip = 0;
  // temporal runs (frames coded back to back, one read-back per run): per
  // frame [4k] error word; then the records' offsets (kTRun + 1) and the run's
  // own error word
  unsigned long long *run_dev, *run_host;
  // frames one run codes at once (0: no runs) and their buffers: residual
  // bytes and escaped residuals of [run_max][F] arrays of run_stride values
  int run_max = 0;
  uint64_t run_stride = 0;
  uint8_t* run_v8 = nullptr;
  uint32_t* run_esc = nullptr;
  uint8_t* rec_tmp;  // second record (temporal candidate)
  uint64_t rec_tmp_cap;
  uint32_t* ext_part;    // extent partials
  uint32_t* hist_part;   // spread histogram copies
  unsigned long long* hist_max;
  uint8_t* huff_lens;    // candidate code lengths per (array, halving count)
  uint32_t* huff_maxd;
  // spatial batch tables (pinned host staging + device mirrors)
  SegDev *seg_host, *seg_dev;
  uint32_t *segpre_host, *segpre_dev;  // [4][RB + 1]
  uint32_t* ext_dev;                   // [RB][2F] extent keys (in ret_dev)
  uint32_t *rstart, *Bs;               // [RB + 1], [RB]
  uint32_t **permdst_host, **permdst_dev;
  // spatial decode batch tables
  DSegDev *dseg_host, *dseg_dev;
  uint32_t *dpre_host, *dpre_dev;  // [2][kMaxBatchFrames + 1]: slot and block workgroups
  unsigned long long* segbase;     // [3][kMaxBatchFrames] scan bases
  // encoder tables
  EncArr *earr_host, *earr_dev;
  EncRec *erec_host, *erec_dev;
  uint32_t *epre_host, *epre_dev;  // [4][NAmax + 1]
  unsigned long long* offs_dev;  // [RB + 1] record offsets (in ret_dev)
  // batched decode staging (pinned host + device mirrors)
  uint8_t *hdr_host, *hdr_dev;
  uint64_t *blobtab_host, *blobtab_dev;
  DecArr *arrtab_host, *arrtab_dev;
  uint32_t *prefix_host, *prefix_dev;

  // resident stream state
  int32_t* qpool[4] = {nullptr, nullptr, nullptr, nullptr};
  uint32_t* ppool[3] = {nullptr, nullptr, nullptr};
  int32_t* dqpool[3] = {nullptr, nullptr, nullptr};
  RefState prev, anchor, dprev, danchor;
  RefState sr_state_tmp;  // reference state of the spatial candidate of the current frame
  // the encoder array and prefix tables last uploaded (valid while the scratch
  // stays bound)
  std::vector<uint8_t> enc_cache;
  bool enc_cache_ok = false;
  bool have_eb = false;
  double eb_f[kMaxF];
  uint64_t seq = 0;
  // LCP-FSM
  uint8_t fsm_state = 0;  // S1X (see the LCP-FSM table)
  int untested = 0;
  uint64_t last_s = 0;
  bool have_last_s = false;
  bool dec_last_t = false;  // the last record decoded was LCP-T
  int D = 3;  // spatial dimensions: fields 0..D-1 form the blocks (Eq. 6)
  // frames coded since the last anchor, and how many of them by LCP-T (the
  // temporal-correlation gate of the anchor scale, Sec. 7.4.2)
  uint64_t n_since_anchor = 0, t_since_anchor = 0;

  // launch shape of the batch encode kernels (tuned, or the defaults) and the
  // graphs captured for batches of LCP-S frames, keyed by their launch shape
  lcp_tuning tune{1024, 0, 0, 1};
  bool tune_set = false;  // set by lcp_plan_autotune / lcp_plan_set_tuning
  std::string dev_key;    // GPU name and compute units, for the tuning cache
  std::vector<std::pair<std::vector<uint64_t>, hipGraphExec_t>> graphs;
  hipStream_t cap_stream = nullptr;
  bool capturing = false;  // kernels are being captured: no timer events
  uint64_t graph_launches = 0, graph_captures = 0;

  // kernel timer
  char timer_name[64] = {0};
  uint64_t timer_every = kTimerStride;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  std::vector<uint64_t> ev_bytes;
  double timer_ms = 0;
  uint64_t timer_launches = 0, timer_bytes = 0;
  uint64_t timer_seen = 0;  // launches of the named kernel since the name was set
};

namespace {

thread_local lcp_plan_s* g_timer_plan = nullptr;  // plan whose call this thread runs

struct TimerScope {
  explicit TimerScope(lcp_plan_s* p) { g_timer_plan = p; }
  ~TimerScope() { g_timer_plan = nullptr; }
};

// A failed HIP call becomes LCP_ERR_DEVICE; with LCP_DEBUG set in the
// environment the call and the runtime's message go to stderr.
lcp_status hip_fail(hipError_t e, const char* what, int line) {
  static const bool dbg = getenv("LCP_DEBUG") != nullptr;
  if (dbg) fprintf(stderr, "lcp: %s failed at lcp_host.hip:%d: %s\n", what, line, hipGetErrorString(e));
  return LCP_ERR_DEVICE;
}
#define HIP_OK(x)                                              \
  do {                                                         \
    hipError_t e_ = (x);                                       \
    if (e_ != hipSuccess) return hip_fail(e_, #x, __LINE__);   \
  } while (0)

void drop_graphs(lcp_plan_s* P) {
  for (auto& e : P->graphs) (void)hipGraphExecDestroy(e.second);
  P->graphs.clear();
}

// Host table -> device: small tables through kernel arguments (a copy-engine
// transfer costs tens of microseconds on the stream), large ones by copy from
// pinned memory (the source must then stay untouched until the stream syncs).
lcp_status upload(const void* host, void* dev, size_t bytes, hipStream_t s) {
  if (bytes == 0) return LCP_OK;
  if (bytes % 4 == 0 && bytes <= 4 * (size_t)kInstallWords * 4) {
    launch_install(host, dev, bytes, s);
    return LCP_OK;
  }
  HIP_OK(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, s));
  return LCP_OK;
}

// Uploads tables that are adjacent, in the same order and at the same
// relative offsets, on the host and on the device: the whole span in one
// transfer when it is small, else each table's used part on its own.
struct Part {
  const void* host;
  void* dev;
  size_t bytes;  // used bytes
};
lcp_status upload_group(std::initializer_list<Part> parts, hipStream_t s) {
  const Part& a = *parts.begin();
  const Part& z = *(parts.end() - 1);
  const size_t span = (size_t)(static_cast<const uint8_t*>(z.host) - static_cast<const uint8_t*>(a.host)) + z.bytes;
  if (span <= 4 * (size_t)kInstallWords * 4) return upload(a.host, a.dev, (span + 3) & ~(size_t)3, s);
  for (const Part& p : parts) {
    lcp_status st = upload(p.host, p.dev, p.bytes, s);
    if (st) return st;
  }
  return LCP_OK;
}

// Reads back the first `words` u64 of the return block and waits for the stream.
// The error word is cleared right behind the read-back (on the GPU while the
// host waits), so the next call need not start with a clearing launch.
lcp_status read_ret(lcp_plan_s* P, size_t words, hipStream_t s) {
  HIP_OK(hipMemcpyAsync(P->ret_host, P->ret_dev, words * 8, hipMemcpyDeviceToHost, s));
  launch_fill_u32(P->err, 1, 0u, s);
  HIP_OK(hipStreamSynchronize(s));
  P->err_clean = true;
  return LCP_OK;
}

// Before kernels that may set the error word: zero it unless already known zero.
void clear_err(lcp_plan_s* P, hipStream_t s) {
  if (!P->err_clean) launch_fill_u32(P->err, 1, 0u, s);
  P->err_clean = false;
}
uint32_t host_err(const lcp_plan_s* P) { return (uint32_t)(P->ret_host[0] & 0xFFFFFFFFull); }

void timer_collect(lcp_plan_s* P) {
  for (size_t i = 0; i < P->ev_pending.size(); i++) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, P->ev_pending[i].first, P->ev_pending[i].second);
    P->timer_ms += ms;
    P->timer_launches++;
    P->timer_bytes += P->ev_bytes[i];
    P->ev_free.push_back(P->ev_pending[i].first);
    P->ev_free.push_back(P->ev_pending[i].second);
  }
  P->ev_pending.clear();
  P->ev_bytes.clear();
}

hipEvent_t timer_event(lcp_plan_s* P) {
  if (!P->ev_free.empty()) {
    hipEvent_t e = P->ev_free.back();
    P->ev_free.pop_back();
    return e;
  }
  hipEvent_t e;
  (void)hipEventCreate(&e);
  return e;
}

uint64_t bound_bytes(int F, uint64_t n) {
  auto words = [](uint64_t bits) { return (bits + 31) / 32; };
  uint64_t b = kHdrBytes + 8ull * F + (uint64_t)kDirBytes * (F + 2);
  b += 4 * words(n * 63) + 4 * words(n * 33);
  b += (uint64_t)F * 4 * words(n * 25);
  return b;
}

GridDev to_dev(const HostGrid* g, int F) {
  GridDev d;
  memset(&d, 0, sizeof(d));
  d.scale = 1;
  d.dtype = g[0].dtype;
  for (int f = 0; f < F; f++) {
    d.m[f] = g[f].m;
    d.eb_q[f] = g[f].eb_q;
    d.md[f] = g[f].md;
    d.inv[f] = g[f].inv;
  }
  return d;
}

// ------------------------------------------------------------------ spatial batch tables
// The caller fills seg_host[r].x and .n; frames are placed back to back.
struct SegLayout {
  uint32_t ext_blocks = 0, blocks_1k = 0, blocks_256 = 0, tiles = 0;
  uint64_t ntot = 0;
};

lcp_status upload_segs(lcp_plan_s* P, int R, SegLayout* L, hipStream_t s) {
  uint32_t* pe = P->segpre_host;
  uint32_t* p1 = pe + (R + 1);
  uint32_t* p2 = p1 + (R + 1);
  uint32_t* pt = p2 + (R + 1);
  SegLayout l;
  for (int r = 0; r < R; r++) {
    SegDev& g = P->seg_host[r];
    g.off = l.ntot;
    l.ntot += g.n;
    pe[r] = l.ext_blocks;
    p1[r] = l.blocks_1k;
    p2[r] = l.blocks_256;
    pt[r] = l.tiles;
    l.ext_blocks += seg_ext_blocks(g.n);
    l.blocks_1k += (uint32_t)((g.n + P->tune.tile - 1) / P->tune.tile);
    l.blocks_256 += (uint32_t)((g.n + kSeg256 - 1) / kSeg256);
    l.tiles += (uint32_t)((g.n + kSortTile - 1) / kSortTile);
  }
  pe[R] = l.ext_blocks;
  p1[R] = l.blocks_1k;
  p2[R] = l.blocks_256;
  pt[R] = l.tiles;
  if (l.ntot > P->NB) return LCP_ERR_ARG;
  lcp_status st = upload_group({{P->seg_host, P->seg_dev, sizeof(SegDev) * R},
                                 {P->segpre_host, P->segpre_dev, sizeof(uint32_t) * 4 * (R + 1)}},
                                s);
  if (st) return st;
  *L = l;
  return LCP_OK;
}

// ------------------------------------------------------------------ extent
// Per-field minima and maxima of R frames (seg_host[r].x / .n), one sync.
lcp_status extent_batch(lcp_plan_s* P, int R, double (*lo)[kMaxF], double (*hi)[kMaxF],
                        hipStream_t s) {
  const int F = P->F;
  const int is_int = P->p.dtype == LCP_DTYPE_I32;
  for (int r = 0; r < R; r++) P->seg_host[r].dtype = P->p.dtype;
  SegLayout L;
  lcp_status st = upload_segs(P, R, &L, s);
  if (st) return st;
  clear_err(P, s);
  launch_extent_b(P->seg_dev, P->segpre_dev, L.ext_blocks, R, F, P->ext_dev, P->ext_part,
                  P->err, (uint64_t)F * L.ntot * 4, s);
  const size_t ext_word0 = (size_t)(reinterpret_cast<unsigned long long*>(P->ext_dev) - P->ret_dev);
  if ((st = read_ret(P, ext_word0 + ((size_t)R * 2 * F + 1) / 2, s))) return st;
  if (host_err(P) & kErrNonFinite) return LCP_ERR_ARG;
  const uint32_t* ext = reinterpret_cast<const uint32_t*>(P->ret_host + ext_word0);
  for (int r = 0; r < R; r++)
    for (int f = 0; f < F; f++) {
      const uint32_t ka = ext[(size_t)r * 2 * F + 2 * f], kb = ext[(size_t)r * 2 * F + 2 * f + 1];
      if (is_int) {
        lo[r][f] = (double)(int32_t)(ka ^ 0x80000000u);
        hi[r][f] = (double)(int32_t)(kb ^ 0x80000000u);
        continue;
      }
      float a = key_float(ka), b = key_float(kb);
      lo[r][f] = a == 0.0f ? 0.0 : (double)a;  // one zero: +0
      hi[r][f] = b == 0.0f ? 0.0 : (double)b;
    }
  return LCP_OK;
}

// Absolute bound per field.  An int32 field may get 0 (a constant field under
// a relative bound): it is then kept exactly.
lcp_status field_eb(const lcp_params& p, int F, const double* lo, const double* hi, double* eb) {
  if (!(p.eb > 0) || !isfinite(p.eb)) return LCP_ERR_ARG;
  if (p.eb_mode == LCP_EB_ABS) {
    for (int f = 0; f < F; f++) eb[f] = p.eb;
  } else if (p.eb_mode == LCP_EB_REL_GLOBAL) {
    double a = lo[0], b = hi[0];
    for (int f = 1; f < F; f++) {
      a = lo[f] < a ? lo[f] : a;
      b = hi[f] > b ? hi[f] : b;
    }
    for (int f = 0; f < F; f++) eb[f] = p.eb * (b - a);
  } else if (p.eb_mode == LCP_EB_REL_PER_FIELD) {
    for (int f = 0; f < F; f++) eb[f] = p.eb * (hi[f] - lo[f]);
  } else {
    return LCP_ERR_ARG;
  }
  const bool is_int = p.dtype == LCP_DTYPE_I32;
  for (int f = 0; f < F; f++)
    if (is_int ? !(eb[f] >= 0) : !(eb[f] > 0)) return LCP_ERR_EB_TOO_SMALL;
  return LCP_OK;
}

// The grids of one frame: float32 grids at eb / s, int32 grids with step s.
lcp_status make_grids(const lcp_params& p, int F, const double* lo, const double* hi,
                      const double* eb, int s, HostGrid* g) {
  for (int f = 0; f < F; f++) {
    lcp_status st = p.dtype == LCP_DTYPE_I32
                        ? make_grid_i((int32_t)lo[f], eb[f], s, &g[f])
                        : make_grid((float)lo[f], (float)hi[f], eb[f] / (double)s, &g[f]);
    if (st) return st;
  }
  return LCP_OK;
}

// ------------------------------------------------------------------ encoder tables
struct EncBuild {
  int NA = 0, R = 0;
  uint32_t copies = 0;
  uint64_t cw = 0, values = 0, stage = 0;
  std::vector<uint32_t> hb, cb, fb, kb;
  bool fused = false;  // the packing builds the code (temporal record, a chunk per wave)
  // the tables go up by one kernel that reads them from pinned host memory
  // (launch sets the host waits for before it writes the tables again, never captured)
  bool fetch = false;
};

// Adds one array of at most nb values to record rec; copy0 < 0 places its
// spread histogram copies after the previous array's.
lcp_status enc_add(lcp_plan_s* P, EncBuild& B, const ArrIn& in, uint64_t nb, int rec, int copy0,
                   uint32_t copies) {
  if (B.NA >= P->NAmax) return LCP_ERR_ARG;
  EncArr& e = P->earr_host[B.NA];
  memset(&e, 0, sizeof(e));
  e.in = in;
  e.rec = (uint32_t)rec;
  if (copy0 < 0) {
    e.copy0 = B.copies;
    e.copies = enc_hist_copies(nb);
    B.copies += e.copies;
  } else {
    e.copy0 = (uint32_t)copy0;
    e.copies = copies;
    if ((uint32_t)copy0 + copies > B.copies) B.copies = (uint32_t)copy0 + copies;
  }
  e.cw0 = B.cw;
  B.cw += (nb + (1ull << P->chunk_log2) - 1) >> P->chunk_log2;
  e.stage0 = B.stage;
  B.stage += enc_stage_words(nb, in.is64 != 0, P->chunk_log2);
  if (B.copies > P->hist_copies || B.cw > P->cw_cap || B.stage > P->stage_cap) return LCP_ERR_ARG;
  B.hb.push_back(enc_hist_blocks(nb));
  B.cb.push_back(enc_chunk_blocks(nb, P->chunk_log2, in.esc != nullptr));
  B.kb.push_back(enc_copy_blocks(nb, P->chunk_log2));
  B.fb.push_back(enc_fixed_blocks(nb));
  B.values += nb;
  B.NA++;
  return LCP_OK;
}

constexpr uint64_t kFusedPackBlocks = 4096;  // total packing workgroups of a fused launch
constexpr uint64_t kFusedCopyBlocks = 4096;  // ... emit workgroups of its Huffman arrays
constexpr uint64_t kFusedFixedBlocks = 1024;  // ... and of its fixed-length ones (rare)

// The host side of an encode launch set: prefix tables, and the record, array
// and prefix tables uploaded on stream s unless the device already holds them.
lcp_status enc_prepare(lcp_plan_s* P, EncBuild& B, EncLaunch* Lo, hipStream_t s) {
  const int NA = B.NA;
  EncLaunch L;
  L.arrs = P->earr_dev;
  L.recs = P->erec_dev;
  L.pre = P->epre_dev;
  L.NA = NA;
  L.R = B.R;
  uint32_t* ph = P->epre_host;
  uint32_t* pc = ph + (NA + 1);
  uint32_t* pf = pc + (NA + 1);
  uint32_t* pk = pf + (NA + 1);
  // a launch of many arrays whose packing builds each array's code (the
  // records of a run): fewer workgroups per array, so that what each one does
  // once (that build, and the emit's sum of the chunk counts before its range)
  // is shared by more chunks; the grid stays several workgroups per compute unit
  if (B.fused && NA > 1) {
    const uint32_t per_pack = (uint32_t)((kFusedPackBlocks + NA - 1) / NA);
    const uint32_t per_copy = (uint32_t)((kFusedCopyBlocks + NA - 1) / NA);
    const uint32_t per_fixed = (uint32_t)((kFusedFixedBlocks + NA - 1) / NA);
    for (int a = 0; a < NA; a++) {
      if (B.cb[a] > per_pack) B.cb[a] = per_pack;
      if (B.kb[a] > per_copy) B.kb[a] = per_copy;
      if (B.fb[a] > per_fixed) B.fb[a] = per_fixed;
    }
  }
  uint32_t h = 0, c = 0, f = 0, k = 0;
  for (int a = 0; a < NA; a++) {
    ph[a] = h;
    pc[a] = c;
    pf[a] = f;
    pk[a] = k;
    h += B.hb[a];
    c += B.cb[a];
    f += B.fb[a];
    k += B.kb[a];
  }
  ph[NA] = h;
  pc[NA] = c;
  pf[NA] = f;
  pk[NA] = k;
  L.hist_blocks = h;
  L.chunk_blocks = c;
  L.fixed_blocks = f;
  L.copy_blocks = k;
  L.values = B.values;
  L.all_bytes = 1;
  L.fused = B.fused ? 1 : 0;
  L.err_rec = nullptr;
  L.err_stride = 0;
  for (int a = 0; a < NA; a++) L.all_bytes &= P->earr_host[a].in.esc != nullptr ? 1 : 0;
  // A single record travels to the layout kernel as an argument; the array and
  // prefix tables are not uploaded again while the device holds the same bytes
  // (consecutive temporal frames of one size)
  L.rec0 = P->erec_host[0];
  const size_t arr_bytes = sizeof(EncArr) * NA, pre_bytes = sizeof(uint32_t) * 4 * (NA + 1);
  const bool same = P->enc_cache_ok && P->enc_cache.size() == arr_bytes + pre_bytes &&
                    !memcmp(P->enc_cache.data(), P->earr_host, arr_bytes) &&
                    !memcmp(P->enc_cache.data() + arr_bytes, P->epre_host, pre_bytes);
  lcp_status st = LCP_OK;
  if (B.fetch && B.R > 1 && P->host_pinned) {
    // the record table and, unless the device holds them, the array and prefix
    // tables after it: one span, the same offsets on both sides
    const uint8_t* h0 = reinterpret_cast<const uint8_t*>(P->erec_host);
    const uint8_t* hz = same ? h0 + sizeof(EncRec) * B.R
                             : reinterpret_cast<const uint8_t*>(P->epre_host) + pre_bytes;
    const size_t span = (size_t)(hz - h0);
    if (reinterpret_cast<const uint8_t*>(P->earr_host) - h0 !=
            reinterpret_cast<const uint8_t*>(P->earr_dev) - reinterpret_cast<const uint8_t*>(P->erec_dev) ||
        reinterpret_cast<const uint8_t*>(P->epre_host) - h0 !=
            reinterpret_cast<const uint8_t*>(P->epre_dev) - reinterpret_cast<const uint8_t*>(P->erec_dev))
      return LCP_ERR_DEVICE;  // the layouts keep these tables in the same order and spacing
    launch_fetch_host(h0, P->erec_dev, (span + 3) & ~(size_t)3, s);
  } else if (B.R > 1 && same) st = upload(P->erec_host, P->erec_dev, sizeof(EncRec) * B.R, s);
  else if (B.R > 1)
    st = upload_group({{P->erec_host, P->erec_dev, sizeof(EncRec) * B.R},
                       {P->earr_host, P->earr_dev, arr_bytes},
                       {P->epre_host, P->epre_dev, pre_bytes}},
                      s);
  else if (!same)
    st = upload_group({{P->earr_host, P->earr_dev, arr_bytes}, {P->epre_host, P->epre_dev, pre_bytes}},
                      s);
  if (st) return st;
  if (!same) {
    P->enc_cache.resize(arr_bytes + pre_bytes);
    memcpy(P->enc_cache.data(), P->earr_host, arr_bytes);
    memcpy(P->enc_cache.data() + arr_bytes, P->epre_host, pre_bytes);
    P->enc_cache_ok = true;
  }
  *Lo = L;
  return LCP_OK;
}

// The kernels of an encode launch set (tables in place).  Errors go to err and
// record offsets to offs (the plan's return block unless given); with base
// (device) the first record starts at *base.
void enc_enqueue(lcp_plan_s* P, const EncLaunch& L, uint8_t* out, uint64_t cap, bool hist_done,
                 hipStream_t s, uint32_t* err = nullptr, unsigned long long* offs = nullptr,
                 const unsigned long long* base = nullptr) {
  EncScratch X;
  X.chunk_words = P->chunk_words;
  X.stage = P->stage;
  X.hist_part = P->hist_part;
  X.hist_max = P->hist_max;
  X.huff_lens = P->huff_lens;
  X.huff_maxd = P->huff_maxd;
  launch_encode(L, P->chunk_log2, P->work, X, out, cap, offs ? offs : P->offs_dev,
                err ? err : P->err, base, hist_done, s);
}

lcp_status enc_launch(lcp_plan_s* P, EncBuild& B, uint8_t* out, uint64_t cap, bool hist_done,
                      hipStream_t s, uint32_t* err = nullptr, unsigned long long* offs = nullptr,
                      const unsigned long long* base = nullptr, uint32_t* err_rec = nullptr,
                      int err_stride = 0) {
  EncLaunch L;
  lcp_status st = enc_prepare(P, B, &L, s);
  if (st) return st;
  L.err_rec = err_rec;
  L.err_stride = err_stride;
  enc_enqueue(P, L, out, cap, hist_done, s, err, offs, base);
  return LCP_OK;
}

// Waits for the encode launch set: record offsets offs[0..R] (host) and the
// device error word.
lcp_status finish_records(lcp_plan_s* P, int R, uint64_t* offs, uint32_t* flags, hipStream_t s) {
  lcp_status st = read_ret(P, 2 + (size_t)R, s);
  if (st) return st;
  if (g_timer_plan == P) timer_collect(P);
  for (int r = 0; r <= R; r++) offs[r] = P->ret_host[1 + r];
  if (flags) *flags = host_err(P);
  if (host_err(P) & kErrCapacity) return LCP_ERR_CAPACITY;
  // the encoder's own consistency checks (a chunk beyond its staging slot)
  if (host_err(P) & kErrCorrupt) return LCP_ERR_DEVICE;
  return LCP_OK;
}

RecHdr make_hdr(int mode, int F, int k, int cl, int A, uint64_t n, uint64_t seq, uint64_t ref_seq,
                const HostGrid* g, int scale = 1, int dims = 3) {
  RecHdr h;
  memset(&h, 0, sizeof(h));
  h.mode = mode;
  h.scale = scale;
  h.dims = dims;
  h.F = F;
  h.k = k;
  h.chunk_log2 = cl;
  h.A = A;
  h.n = n;
  h.seq = seq;
  h.ref_seq = ref_seq;
  h.dtype = g[0].dtype;
  for (int f = 0; f < F; f++) {
    h.m[f] = g[f].m;
    h.eb_q[f] = g[f].eb_q;
  }
  return h;
}

// ------------------------------------------------------------------ graphs
// The kernels of one launch shape, captured on the plan's own stream into a
// graph (a fill kernel clears the error word first; no copies or memsets are
// recorded) and instantiated.
constexpr size_t kMaxGraphs = 8;
template <typename K>
lcp_status capture_graph(lcp_plan_s* P, K& kernels, hipGraphExec_t* exec) {
  if (!P->cap_stream) HIP_OK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
  HIP_OK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
  P->capturing = true;
  launch_fill_u32(P->err, 1, 0u, P->cap_stream);
  kernels(P->cap_stream);
  P->capturing = false;
  hipGraph_t graph = nullptr;
  HIP_OK(hipStreamEndCapture(P->cap_stream, &graph));
  const hipError_t e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate", __LINE__);
  P->graph_captures++;
  return LCP_OK;
}

// LCP-S on R independent frames (seg_host[r].x / .n) in one set of launches.
// g[r] are frame r's grids, hi[r] its maxima.  Records go back to back to out;
// offs (host, R + 1) receives their offsets.  q_slot (R == 1 only) receives
// the slot-order codes; perm_dst (nullable, R device pointers, each nullable)
// the slot -> input permutations; *perm_res the batch's permutation array.
lcp_status compress_s_batch(lcp_plan_s* P, int R, const HostGrid (*g)[kMaxF],
                            const double (*hi)[kMaxF], int k, uint64_t seq0, uint8_t* out,
                            uint64_t cap, int32_t* q_slot, uint32_t* const* perm_dst,
                            uint64_t* offs, const uint32_t** perm_res, hipStream_t s) {
  const int F = P->F;
  if (R < 1 || R > P->RB || (q_slot && R != 1)) return LCP_ERR_ARG;
  std::vector<int> kb(R);
  std::vector<RecHdr> hdr(R);
  for (int r = 0; r < R; r++) {
    SegDev& sg = P->seg_host[r];
    uint64_t bn[3];
    unsigned __int128 tot = 1;
    const int D = P->D;
    bn[0] = bn[1] = bn[2] = 1;  // an axis the data does not have: one block
    for (int f = 0; f < F; f++) {
      int64_t qm = host_quant(hi[r][f], g[r][f]);
      if (qm >= kQLimit) return LCP_ERR_RANGE;
      if (f < D) {
        bn[f] = (uint64_t)((qm >> k) + 1);
        tot *= bn[f];
      }
      sg.m[f] = g[r][f].m;
      sg.eb_q[f] = g[r][f].eb_q;
      sg.md[f] = g[r][f].md;
      sg.inv[f] = g[r][f].inv;
    }
    sg.dtype = g[r][0].dtype;
    if (tot >= ((unsigned __int128)1 << 63)) return LCP_ERR_RANGE;
    kb[r] = bitwidth64((uint64_t)tot - 1);
    sg.bn0 = bn[0];
    sg.bn1 = bn[1];
    sg.k = k;
    sg.D = D;
    hdr[r] = make_hdr(0, F, k, P->chunk_log2, F + 2, sg.n, seq0 + r, ~0ull, g[r], 1, D);
    for (int d = 0; d < 3; d++) hdr[r].bn[d] = (uint32_t)bn[d];
  }
  int sort_bits = 0;
  for (int r = 0; r < R; r++) sort_bits = kb[r] > sort_bits ? kb[r] : sort_bits;
  // host side first: frame tables, encoder tables, permutation destinations,
  // all uploaded on s; then the kernels, which read only device tables
  SegLayout L;
  lcp_status st = upload_segs(P, R, &L, s);
  if (st) return st;
  const uint64_t ntot = L.ntot;
  uint32_t* v_rel = P->v_slot;                       // fields 0..D-1
  uint32_t* v_sup = P->v_slot + (uint64_t)P->D * ntot;  // fields D..F-1
  EncBuild B;
  B.R = R;
  for (int r = 0; r < R; r++) {
    const SegDev& sg = P->seg_host[r];
    const uint64_t n = sg.n, o = sg.off;
    EncRec& rc = P->erec_host[r];
    memset(&rc, 0, sizeof(rc));
    rc.h = hdr[r];
    rc.B_dev = P->Bs + r;
    rc.a0 = (uint32_t)B.NA;
    if ((st = enc_add(P, B, ArrIn{P->v_id + o, 1, P->Bs + r, n}, n, r, -1, 0))) return st;
    if ((st = enc_add(P, B, ArrIn{P->v_cnt + o, 1, P->Bs + r, n}, n, r, -1, 0))) return st;
    for (int d = 0; d < P->D; d++)
      if ((st = enc_add(P, B, ArrIn{v_rel + (uint64_t)d * ntot + o, 0, nullptr, n}, n, r, -1, 0)))
        return st;
    for (int f = P->D; f < F; f++)
      if ((st = enc_add(P, B, ArrIn{v_sup + (uint64_t)(f - P->D) * ntot + o, 0, nullptr, n}, n, r, -1, 0)))
        return st;
  }
  EncLaunch EL;
  if ((st = enc_prepare(P, B, &EL, s))) return st;
  bool perm_copy = false;
  if (perm_dst) {
    for (int r = 0; r < R; r++) {
      P->permdst_host[r] = perm_dst[r];
      perm_copy |= perm_dst[r] != nullptr;
    }
    if (perm_copy && (st = upload(P->permdst_host, P->permdst_dev, sizeof(uint32_t*) * R, s)))
      return st;
  }
  // the sort leaves keys and permutation in one of two buffers, fixed by the
  // number of 8-bit passes
  const int cur = radix_result(sort_bits);
  const uint64_t* keys = cur ? P->keys1 : P->keys0;
  const uint32_t* perm = cur ? P->vals1 : P->vals0;
  const uint32_t* pre_tile = P->segpre_dev + (R + 1);
  const uint32_t* pre_256 = P->segpre_dev + 2 * (R + 1);
  const TileShape ts{P->tune.tile, L.blocks_1k, P->tune.grid};
  const bool key32 = sort_bits <= 32;  // every block id fits 32 bits
  auto kernels = [&](hipStream_t q) {
    launch_quant_key_b(P->seg_dev, pre_tile, ts, R, F, P->D, P->keys0, P->vals0, P->slot_rec,
                       ntot, key32, q);
    uint32_t* tmp32 = reinterpret_cast<uint32_t*>(P->scan_tmp);
    radix_sort(P->keys0, P->vals0, P->keys1, P->vals1, P->seg_dev, P->segpre_dev + 3 * (R + 1),
               L.tiles, R, ntot, sort_bits, P->hist, tmp32, key32, q);
    launch_runs_b(keys, P->seg_dev, pre_tile, ts, R, ntot, P->flags, P->ids, P->starts, P->rstart,
                  P->Bs, tmp32, key32, q);
    launch_block_syms_b(P->ids, P->starts, P->rstart, R, P->seg_dev, ntot, P->v_id, P->v_cnt, q);
    launch_slot_syms_b(P->seg_dev, pre_256, L.blocks_256, P->tune.slot_grid, R, F, P->D, perm, keys,
                       P->slot_rec, ntot, v_rel, v_sup, q_slot, key32, q);
    enc_enqueue(P, EL, out, cap, false, q);
    if (perm_copy) launch_copy_perm_b(perm, P->seg_dev, pre_tile, ts, R, P->permdst_dev, q);
  };
  // A batch of frames from a plan that owns its scratch replays the graph of
  // its launch shape (captured on first use); everything that differs between
  // batches of one shape is in the tables uploaded above.
  const bool graph = P->tune.graphs && R >= 2 && P->own_dev && !q_slot;
  if (graph) {
    std::vector<uint64_t> key = {(uint64_t)R, (uint64_t)F, (uint64_t)P->chunk_log2,
                                 (uint64_t)sort_bits, P->tune.tile, P->tune.grid,
                                 P->tune.slot_grid, (uint64_t)(uintptr_t)out, cap, perm_copy};
    for (int r = 0; r < R; r++) key.push_back(P->seg_host[r].n);
    hipGraphExec_t exec = nullptr;
    for (auto& e : P->graphs)
      if (e.first == key) exec = e.second;
    if (!exec) {
      if ((st = capture_graph(P, kernels, &exec))) return st;
      if (P->graphs.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(P->graphs.front().second);
        P->graphs.erase(P->graphs.begin());
      }
      P->graphs.push_back({key, exec});
    }
    HIP_OK(hipGraphLaunch(exec, s));
    P->graph_launches++;
    P->err_clean = false;
  } else {
    clear_err(P, s);
    kernels(s);
  }
  if (perm_res) *perm_res = perm;
  return finish_records(P, R, offs, nullptr, s);
}

// LCP-S on one frame (a batch of one).
struct SResult {
  uint64_t size = 0;
  const uint32_t* perm = nullptr;  // device, slot -> input index
};

lcp_status compress_s(lcp_plan_s* P, const float* const* x, uint64_t n, const HostGrid* g,
                      const double* hi, int k, uint64_t seq, uint8_t* out, uint64_t cap,
                      int32_t* q_slot, SResult* res, hipStream_t s) {
  for (int f = 0; f < P->F; f++) P->seg_host[0].x[f] = x[f];
  P->seg_host[0].n = n;
  HostGrid g1[1][kMaxF];
  double h1[1][kMaxF];
  memcpy(g1[0], g, sizeof(HostGrid) * P->F);
  memcpy(h1[0], hi, sizeof(double) * P->F);
  uint64_t offs[2] = {0, 0};
  lcp_status st = compress_s_batch(P, 1, g1, h1, k, seq, out, cap, q_slot, nullptr, offs,
                                   &res->perm, s);
  res->size = offs[1];
  return st;
}

lcp_status extent(lcp_plan_s* P, const float* const* x, uint64_t n, double* lo, double* hi,
                  hipStream_t s) {
  for (int f = 0; f < P->F; f++) P->seg_host[0].x[f] = x[f];
  P->seg_host[0].n = n;
  double l1[1][kMaxF], h1[1][kMaxF];
  lcp_status st = extent_batch(P, 1, l1, h1, s);
  if (st) return st;
  memcpy(lo, l1[0], sizeof(double) * P->F);
  memcpy(hi, h1[0], sizeof(double) * P->F);
  return LCP_OK;
}

// LCP-T on one frame against a resident reference.  Whether the frame fits the
// reference grid (finite values, float32 margin, code range) is checked by the
// residual kernel itself, so no extent pass is needed.
// The largest float32 x >= 0 with x + eb2 < lim in double arithmetic (the
// temporal frames' margin test of a float32 grid; -1 when no x passes).  The
// double sum is monotone in x, so the floats that pass are one interval from
// 0, and a bisection over the float bit patterns (ordered as integers for
// x >= 0) finds its end with the same IEEE double addition the test uses.
float margin_xmax(double eb2, double lim) {
  auto ok = [&](uint32_t bits) {
    float x;
    memcpy(&x, &bits, 4);
    return (double)x + eb2 < lim;
  };
  if (!ok(0u)) return -1.0f;
  uint32_t lo = 0u, hi = 0x7F800000u;  // ok(lo); hi (infinity) fails
  while (hi - lo > 1u) {
    const uint32_t mid = lo + (hi - lo) / 2u;
    if (ok(mid)) lo = mid;
    else hi = mid;
  }
  float x;
  memcpy(&x, &lo, 4);
  return x;
}

GridDev t_grid(const RefState& ref, int F) {
  GridDev gd = to_dev(ref.grid, F);
  gd.scale = ref.scale;
  for (int f = 0; f < F; f++) {
    // int32 grids: exact integer reconstructions, no float32 margin to keep
    const HostGrid& hg = ref.grid[f];
    gd.xmax[f] = hg.dtype == kDtypeI32 ? HUGE_VALF
                                       : margin_xmax(2.0 * hg.eb, ldexp(1.0, hg.E));
  }
  return gd;
}

FieldPtrs field_ptrs(const float* const* x, int F) {
  FieldPtrs fp;
  memset(&fp, 0, sizeof(fp));
  for (int f = 0; f < F; f++) fp.p[f] = x[f];
  return fp;
}

// Enqueues LCP-T of one frame against `ref` (Sec. 4): residual kernel, then
// the coder launches.  Errors go to err, the record's start and end to
// offs[0..1] (from *base when given).
lcp_status launch_t(lcp_plan_s* P, const float* const* x, uint64_t n, const RefState& ref,
                    uint64_t seq, uint8_t* out, uint64_t cap, int32_t* q_new, uint32_t* err,
                    unsigned long long* offs, const unsigned long long* base, hipStream_t s) {
  const int F = P->F;
  // residual alphabets are short: unless one recently was not, the packing
  // kernel builds the code (the residual kernel zeroes the word totals)
  const bool fused = P->fuse_skip == 0 && n > 0 && P->chunk_log2 >= 6 && P->chunk_log2 <= 10;
  if (P->fuse_skip > 0) P->fuse_skip--;
  launch_t_resid(field_ptrs(x, F), F, n, t_grid(ref, F), P->ppool[ref.perm], P->qpool[ref.q],
                 P->v_byte, P->v_slot, q_new, err, P->hist_part, P->hist_max,
                 fused ? P->work : nullptr, s);
  EncBuild B;
  B.R = 1;
  B.fused = fused;
  EncRec& rc = P->erec_host[0];
  memset(&rc, 0, sizeof(rc));
  rc.h = make_hdr(1, F, 0, P->chunk_log2, F, n, seq, ref.seq, ref.grid, ref.scale);
  rc.a0 = 0;
  lcp_status st;
  // the residual kernel counts field f into spread copies f * kHistCopies ...
  for (int f = 0; f < F; f++)
    if ((st = enc_add(P, B,
                      ArrIn{P->v_byte + (uint64_t)f * n, 0, nullptr, n, P->v_slot + (uint64_t)f * n},
                      n, 0, f * kHistCopies, kHistCopies)))
      return st;
  return enc_launch(P, B, out, cap, true, s, err, offs, base);
}

// After a temporal frame whose packing could not build its code (an alphabet
// past one wave's): its histogram copies hold counts past the bins the emit
// clears, so all are cleared, and the next frames use the separate build.
constexpr int kFuseBackoff = 64;
void fused_fallback(lcp_plan_s* P, hipStream_t s) {
  launch_fill_u32(P->hist_part, P->hist_copies * kAlphabet, 0u, s);
  launch_fill_u32(reinterpret_cast<uint32_t*>(P->hist_max), 2 * P->hist_copies, 0u, s);
  P->fuse_skip = kFuseBackoff;
}

lcp_status compress_t(lcp_plan_s* P, const float* const* x, uint64_t n, const RefState& ref,
                      uint64_t seq, uint8_t* out, uint64_t cap, int32_t* q_new, uint64_t* size,
                      hipStream_t s) {
  clear_err(P, s);
  lcp_status st = launch_t(P, x, n, ref, seq, out, cap, q_new, P->err, P->offs_dev, nullptr, s);
  if (st) return st;
  uint32_t flags = 0;
  uint64_t offs[2] = {0, 0};
  st = finish_records(P, 1, offs, &flags, s);
  if (flags & kErrRebuild) {
    fused_fallback(P, s);
    if (!(flags & (kErrNonFinite | kErrRange))) {
      // the frame again, with the separate build
      clear_err(P, s);
      if ((st = launch_t(P, x, n, ref, seq, out, cap, q_new, P->err, P->offs_dev, nullptr, s)))
        return st;
      flags = 0;
      st = finish_records(P, 1, offs, &flags, s);
    }
  }
  *size = offs[1];
  if (flags & kErrNonFinite) return LCP_ERR_ARG;
  if (flags & kErrRange) return LCP_ERR_RANGE;
  return st;
}

// ------------------------------------------------------------------ LCP-FSM
// Sec. 7.2 as a transition table.  States: S1X, S2X, S4X, S8X, S16X (LCP-S,
// with a comparison of both methods on every 1st, 2nd, ... 16th frame) and T
// (LCP-T, its size checked against the last LCP-S record).  `untested` counts
// the S frames still to go before the next comparison.  The size of a frame's
// outcome picks the event; the event picks the next state:
//   no reference (the stream's first frame, or a batch start without anchor):
//     coded with S and taken as a won comparison;
//   an S state's untested frame;
//   a comparison won by S (ties go to S) or by T;
//   a T frame no larger than the last S record (kept), or larger (S is run as
//     well and the smaller kept: either way the machine leaves T for S1X when
//     S wins, and stays in T when T is still the smaller).
bool first_in_batch(const lcp_plan_s* P, uint64_t seq) {
  return P->p.batch_size == 0 ? seq == 0 : seq % (uint64_t)P->p.batch_size == 0;
}

const RefState* reference_for(const lcp_plan_s* P, uint64_t n) {
  if (!P->p.multi_frame) return nullptr;
  const RefState* r = first_in_batch(P, P->seq) ? &P->anchor : &P->prev;
  if (!r->valid || r->n != n) return nullptr;
  return r;
}

enum : uint8_t { kFsmS1, kFsmS2, kFsmS4, kFsmS8, kFsmS16, kFsmT, kFsmStates };
enum : uint8_t { kEvNoRef, kEvUntested, kEvCmpS, kEvCmpT, kEvTKept, kEvTLost, kFsmEvents };
constexpr uint8_t kFsmNone = 0xFF;  // an event the state cannot see
constexpr uint8_t kFsmNext[kFsmStates][kFsmEvents] = {
    //        no ref  untested  cmp S    cmp T   T kept    T lost
    /* S1  */ {kFsmS2, kFsmS1, kFsmS2, kFsmT, kFsmNone, kFsmNone},
    /* S2  */ {kFsmS4, kFsmS2, kFsmS4, kFsmT, kFsmNone, kFsmNone},
    /* S4  */ {kFsmS8, kFsmS4, kFsmS8, kFsmT, kFsmNone, kFsmNone},
    /* S8  */ {kFsmS16, kFsmS8, kFsmS16, kFsmT, kFsmNone, kFsmNone},
    /* S16 */ {kFsmS16, kFsmS16, kFsmS16, kFsmT, kFsmNone, kFsmNone},
    /* T   */ {kFsmS2, kFsmNone, kFsmNone, kFsmNone, kFsmT, kFsmS1},
};
// Frames between comparisons in each S state, once entered by an S win.
constexpr int kFsmGap[kFsmStates] = {0, 1, 3, 7, 15, 0};

int fsm_decide(const lcp_plan_s* P, bool have_ref) {
  if (!P->p.multi_frame || !have_ref) return LCP_DECIDE_S;
  if (P->fsm_state == kFsmT) return LCP_DECIDE_T;
  return P->untested > 0 ? LCP_DECIDE_S : LCP_DECIDE_COMPARE;
}

// One frame's outcome: what was decided, whether a reference existed, and
// which method's record was kept.
void fsm_update(lcp_plan_s* P, int decision, bool have_ref, bool chose_t) {
  uint8_t ev;
  if (!have_ref) ev = kEvNoRef;
  else if (decision == LCP_DECIDE_S) ev = kEvUntested;
  else if (decision == LCP_DECIDE_COMPARE) ev = chose_t ? kEvCmpT : kEvCmpS;
  else ev = chose_t ? kEvTKept : kEvTLost;
  const uint8_t next = kFsmNext[P->fsm_state][ev];
  if (next == kFsmNone) return;  // not reachable: decisions follow the state
  if (ev == kEvUntested) P->untested--;
  else if (next != kFsmT) P->untested = ev == kEvTLost ? 0 : kFsmGap[next];
  P->fsm_state = next;
}

int free_q(const lcp_plan_s* P, int avoid) {
  for (int i = 0; i < 4; i++)
    if (i != avoid && !(P->prev.valid && P->prev.q == i) && !(P->anchor.valid && P->anchor.q == i))
      return i;
  return -1;
}
int free_perm(const lcp_plan_s* P) {
  for (int i = 0; i < 3; i++)
    if (!(P->prev.valid && P->prev.perm == i) && !(P->anchor.valid && P->anchor.perm == i))
      return i;
  return -1;
}

// One frame through Alg. 1 + LCP-FSM (or plain LCP-S for single-frame plans).
// The extent pass and the spatial grid are computed only when LCP-S runs.
lcp_status compress_frame(lcp_plan_s* P, const lcp_frame_in& fr, uint8_t* out, uint64_t cap,
                          uint64_t* size, int* used, uint32_t* perm_out, hipStream_t s) {
  const int F = P->F;
  const uint64_t n = fr.n;
  if (n == 0 || n > P->N || fr.method < 0 || fr.method > 2) return LCP_ERR_ARG;
  for (int f = 0; f < F; f++)
    if (!fr.fields[f]) return LCP_ERR_ARG;
  const bool multi = P->p.multi_frame != 0;
  const RefState* ref = reference_for(P, n);
  int decision;
  if (fr.method == LCP_METHOD_S) decision = LCP_DECIDE_S;
  else if (fr.method == LCP_METHOD_T) decision = LCP_DECIDE_T;
  else decision = fsm_decide(P, ref != nullptr);
  if (decision != LCP_DECIDE_S && !ref) return LCP_ERR_NO_REFERENCE;

  lcp_status st = LCP_OK;
  int qt_i = -1, qs_i = -1, ps_i = -1;
  uint64_t size_s = 0, size_t_ = 0;
  bool have_s = false, have_t = false;
  // A frame decided T is coded straight into `out` when it can hold any record
  // (a spatial fallback then goes to the spare buffer); otherwise the temporal
  // candidate goes to the spare buffer and the spatial one to `out`.
  const bool t_direct = decision == LCP_DECIDE_T && cap >= bound_bytes(F, n);
  uint8_t* t_buf = t_direct ? out : P->rec_tmp;
  uint8_t* s_buf = t_direct ? P->rec_tmp : out;
  const uint64_t s_cap = t_direct ? P->rec_tmp_cap : cap;
  if (decision != LCP_DECIDE_S) {
    qt_i = free_q(P, -1);
    st = compress_t(P, fr.fields, n, *ref, P->seq, t_buf, t_direct ? cap : P->rec_tmp_cap,
                    P->qpool[qt_i], &size_t_, s);
    if (st == LCP_OK) have_t = true;
    else if (st == LCP_ERR_RANGE && fr.method != LCP_METHOD_T) st = LCP_OK;  // T infeasible
    else return st;
  }
  bool need_s = decision != LCP_DECIDE_T || !have_t ||
                (fr.method == LCP_METHOD_AUTO && (!P->have_last_s || size_t_ > P->last_s));
  SResult sr;
  double eb_f[kMaxF];
  // Sec. 7.4.2: a frame that would become an anchor (first in its batch, coded
  // by S) is coded at eb / s while the stream is temporally correlated: at its
  // start (no frame since an anchor yet), or when at least half of the frames
  // since the last anchor were coded by T
  int s_scale = 1;
  if (multi && P->p.anchor_scale > 1 && first_in_batch(P, P->seq) &&
      (P->n_since_anchor == 0 || 2 * P->t_since_anchor >= P->n_since_anchor))
    s_scale = P->p.anchor_scale;
  if (need_s) {
    double lo[kMaxF], hi[kMaxF];
    if ((st = extent(P, fr.fields, n, lo, hi, s))) return st;
    if (multi && P->have_eb) memcpy(eb_f, P->eb_f, sizeof(eb_f));
    else if ((st = field_eb(P->p, F, lo, hi, eb_f))) return st;
    // an int32 bin holds at least one integer: when a field's unscaled bin has
    // fewer than s integers there is no finer anchor grid, and the anchor is
    // coded at the stream's bound
    for (int f = 0; f < F && s_scale > 1 && P->p.dtype == LCP_DTYPE_I32; f++)
      if (2.0 * floor(fmin(eb_f[f], 2147483647.0)) + 1.0 < (double)s_scale) s_scale = 1;
    HostGrid sg[kMaxF];
    if ((st = make_grids(P->p, F, lo, hi, eb_f, s_scale, sg))) return st;
    if (multi) {
      qs_i = free_q(P, qt_i);
      ps_i = free_perm(P);
    }
    st = compress_s(P, fr.fields, n, sg, hi, P->k, P->seq, s_buf, s_cap,
                    multi ? P->qpool[qs_i] : nullptr, &sr, s);
    if (st == LCP_ERR_CAPACITY && have_t && size_t_ < sr.size) {
      st = LCP_OK;  // the temporal record is the smaller one and may still fit
    } else if (st) {
      if (st == LCP_ERR_CAPACITY) *size = sr.size;
      return st;
    } else {
      have_s = true;
      size_s = sr.size;
      if (multi) {
        RefState r;
        r.valid = true;
        r.scale = s_scale;
        r.seq = P->seq;
        r.n = n;
        memcpy(r.grid, sg, sizeof(sg));
        r.q = qs_i;
        r.perm = ps_i;
        P->sr_state_tmp = r;
      }
    }
  }
  const bool chose_t = have_t && (!have_s || size_t_ < size_s);
  const uint64_t chosen = chose_t ? size_t_ : size_s;
  if (chosen > cap) {
    *size = chosen;
    return LCP_ERR_CAPACITY;
  }
  if (chose_t && t_buf != out)
    HIP_OK(hipMemcpyAsync(out, t_buf, size_t_, hipMemcpyDeviceToDevice, s));
  if (!chose_t && s_buf != out)
    HIP_OK(hipMemcpyAsync(out, s_buf, size_s, hipMemcpyDeviceToDevice, s));
  *size = chosen;
  if (used) *used = chose_t ? LCP_METHOD_T : LCP_METHOD_S;
  // the estimate of S is an S record at the stream's bound; an anchor coded at
  // eb / s stands in only until there is one
  if (have_s && (s_scale == 1 || !P->have_last_s)) {
    P->last_s = size_s;
    P->have_last_s = true;
  }
  if (multi && fr.method == LCP_METHOD_AUTO) fsm_update(P, decision, ref != nullptr, chose_t);
  if (multi) {
    // Alg. 1 bookkeeping: the previous frame; anchors are first-in-batch S frames
    if (!chose_t) {
      launch_copy_perm(sr.perm, P->ppool[ps_i], n, s);
      P->prev = P->sr_state_tmp;
      if (first_in_batch(P, P->seq)) P->anchor = P->sr_state_tmp;
    } else {
      RefState r = *ref;  // a T frame keeps its reference's grid and slot order
      r.seq = P->seq;
      r.q = qt_i;
      P->prev = r;
    }
    if (!P->have_eb && have_s) {
      memcpy(P->eb_f, eb_f, sizeof(eb_f));  // the first frame is always spatial
      P->have_eb = true;
    }
  }
  if (perm_out) {
    const uint32_t* src = chose_t ? P->ppool[P->prev.perm] : (multi ? P->ppool[ps_i] : sr.perm);
    launch_copy_perm(src, perm_out, n, s);
  }
  if (!chose_t && first_in_batch(P, P->seq)) {
    P->n_since_anchor = 0;
    P->t_since_anchor = 0;
  } else {
    P->n_since_anchor++;
    P->t_since_anchor += chose_t ? 1 : 0;
  }
  P->seq++;
  return LCP_OK;
}

// ------------------------------------------------------------------ temporal runs
// While LCP-FSM stays in its T state every frame is coded with LCP-T against
// the frame before it (Alg. 1: the batch anchor for the first frame of a
// batch), and the host only needs a frame's outcome to learn that it still
// holds.  A run therefore enqueues several such frames back to back, each
// with its own error word and offsets, each record placed on the device right
// behind the previous one, and reads the outcomes back once.  Frames are then
// taken in order; the first whose outcome differs from the prediction (an
// error flag, a record beyond capacity, a size above the last spatial one) and
// every frame after it are left to the per-frame path, which codes that frame
// again from the state the run committed.  Codes of a run frame go to one of
// the two q slots that are neither the committed reference nor the anchor,
// alternating, so the committed reference survives the run; the last
// committed frame's codes, if a later frame reused their slot, are rebuilt
// from its input.
struct RunFrame {
  RefState ref;  // reference the frame is coded against
  int q;         // q slot of its codes
  bool chain;    // the reference is the run frame just before (same grid and slot order)
};

// Frames that would be coded as T in a row if each of them stays T.
int plan_run(const lcp_plan_s* P, const lcp_frame_in* fr, uint64_t nf, uint64_t cap,
             RunFrame* rf) {
  if (!P->p.multi_frame) return 0;
  int spare[2], ns = 0;
  for (int i = 0; i < 4 && ns < 2; i++)
    if (!(P->prev.valid && P->prev.q == i) && !(P->anchor.valid && P->anchor.q == i))
      spare[ns++] = i;
  if (ns < 2) return 0;
  RefState prev = P->prev;
  uint64_t seq = P->seq, used = 0;
  int D = 0;
  const int dmax = P->run_len < P->run_max ? P->run_len : P->run_max;
  if (dmax < 2) return 0;
  for (; D < dmax && (uint64_t)D < nf; D++) {
    const lcp_frame_in& f = fr[D];
    if (f.n == 0 || f.n > P->N || f.method < 0 || f.method > 2) break;
    bool ok = true;
    for (int k = 0; k < P->F; k++) ok = ok && f.fields[k] != nullptr;
    if (!ok) break;
    if (f.method == LCP_METHOD_S || (f.method == LCP_METHOD_AUTO && P->fsm_state != kFsmT)) break;
    const bool first = P->p.batch_size == 0 ? seq == 0 : seq % (uint64_t)P->p.batch_size == 0;
    const RefState& ref = first ? P->anchor : prev;
    if (!ref.valid || ref.n != f.n) break;
    if (D > 0 && f.n != fr[0].n) break;  // a run's frames share one size
    used += bound_bytes(P->F, f.n);
    if (used > cap) break;
    rf[D].ref = ref;
    rf[D].q = spare[D & 1];
    rf[D].chain = D > 0 && !first;
    RefState r = ref;
    r.seq = seq;
    r.q = rf[D].q;
    prev = r;
    seq++;
  }
  return D;
}

// Runs D planned frames; ends[k] receives frame k's record end (relative to
// out) for the committed frames, *committed how many there are.  The frames'
// residuals come from one launch per segment of frames chained on one
// reference (a segment ends where Alg. 1 turns to the anchor), and all D
// records from one encode launch set, placed back to back from out.
constexpr int kRunCopies = 8;    // spread histogram copies per array of a run
constexpr int kServeCopies = 2;  // ... and per array of a server's merged launch
lcp_status run_t(lcp_plan_s* P, const lcp_frame_in* fr, int D, const RunFrame* rf, uint8_t* out,
                 uint64_t cap, uint32_t* const* perms, uint64_t* ends, int* committed,
                 hipStream_t s) {
  *committed = 0;
  const int F = P->F;
  const uint64_t n = fr[0].n;
  uint32_t* words = reinterpret_cast<uint32_t*>(P->run_dev);
  unsigned long long* offs = P->run_dev + 4 * kTRun;
  uint32_t* run_err = reinterpret_cast<uint32_t*>(offs + kTRun + 1);
  const size_t run_words = 4 * kTRun + kTRun + 2;
  if (!P->run_clean) launch_fill_u32(words, 2 * run_words, 0u, s);
  P->run_clean = false;
  // residual alphabets are short: unless one recently was not, the packing
  // kernel builds each array's code (the residual kernel zeroes the word totals)
  const bool fused = P->fuse_skip == 0 && P->chunk_log2 >= 6 && P->chunk_log2 <= 10;
  if (P->fuse_skip > 0) P->fuse_skip = P->fuse_skip > D ? P->fuse_skip - D : 0;
  for (int k0 = 0; k0 < D;) {
    int k1 = k0 + 1;
    while (k1 < D && rf[k1].chain) k1++;
    RunFrames rx;
    memset(&rx, 0, sizeof(rx));
    for (int j = k0; j < k1; j++)
      for (int f = 0; f < F; f++) rx.x[j - k0][f] = fr[j].fields[f];
    const RefState& ref = rf[k0].ref;
    launch_t_resid_run(rx, k1 - k0, F, n, t_grid(ref, F), P->ppool[ref.perm], P->qpool[ref.q],
                       P->qpool[rf[k1 - 1].q], P->run_v8, P->run_esc, P->run_stride, k0,
                       P->hist_part, P->hist_max, kRunCopies, fused ? P->work : nullptr,
                       words + 8 * k0, 8, s);
    k0 = k1;
  }
  EncBuild B;
  B.R = D;
  B.fused = fused;
  B.fetch = true;  // the host waits for the run below before it writes the tables again
  lcp_status st;
  for (int k = 0; k < D; k++) {
    EncRec& rc = P->erec_host[k];
    memset(&rc, 0, sizeof(rc));
    rc.h = make_hdr(1, F, 0, P->chunk_log2, F, n, P->seq + k, rf[k].ref.seq, rf[k].ref.grid,
                    rf[k].ref.scale);
    rc.a0 = (uint32_t)B.NA;
    for (int f = 0; f < F; f++) {
      const uint64_t a = (uint64_t)k * F + f;
      if ((st = enc_add(P, B, ArrIn{P->run_v8 + a * P->run_stride, 0, nullptr, n,
                                    P->run_esc + a * P->run_stride},
                        n, k, (int)(a * kRunCopies), kRunCopies)))
        return st;
    }
  }
  if ((st = enc_launch(P, B, out, cap, true, s, run_err, offs, nullptr, words, 8))) return st;
  HIP_OK(hipMemcpyAsync(P->run_host, P->run_dev, 8 * run_words, hipMemcpyDeviceToHost, s));
  // the next run's return block is cleared while the host waits
  launch_fill_u32(words, 2 * run_words, 0u, s);
  P->run_clean = true;
  HIP_OK(hipStreamSynchronize(s));
  if (g_timer_plan == P) timer_collect(P);
  const uint32_t launch_err = (uint32_t)(P->run_host[4 * kTRun + kTRun + 1] & 0xFFFFFFFFull);
  // the encoder's own consistency checks (a chunk beyond its staging slot)
  if (launch_err & kErrCorrupt) return LCP_ERR_DEVICE;
  // a frame flagged for the separate code build ends the commits there; the
  // per-frame path codes it again
  for (int k = 0; k < D; k++)
    if ((uint32_t)(P->run_host[4 * k] & 0xFFFFFFFFull) & kErrRebuild) {
      fused_fallback(P, s);
      break;
    }
  const unsigned long long* ho = P->run_host + 4 * kTRun;
  int c = 0;
  for (; c < D && !(launch_err & kErrCapacity); c++) {
    const uint32_t flags = (uint32_t)(P->run_host[4 * c] & 0xFFFFFFFFull);
    const uint64_t size = ho[c + 1] - ho[c];
    if (flags) break;
    if (fr[c].method == LCP_METHOD_AUTO && (!P->have_last_s || size > P->last_s)) break;
    // committed: LCP-FSM stays in T; Alg. 1 bookkeeping as for any T frame
    RefState r = rf[c].ref;
    r.seq = P->seq;
    r.q = rf[c].q;
    P->prev = r;
    if (perms && perms[c]) launch_copy_perm(P->ppool[r.perm], perms[c], fr[c].n, s);
    P->n_since_anchor++;
    P->t_since_anchor++;
    P->seq++;
    ends[c] = ho[c + 1];
  }
  *committed = c;
  P->run_len = c < D ? kTRunStart : (D == P->run_len && D < kTRun ? 2 * D : P->run_len);
  // only the last frame of each segment left its codes, and a later segment
  // may have reused that slot: after a break, the last committed frame's codes
  // are rebuilt from its input (and, on a scaled grid, from the frames of its
  // segment before it, starting at the segment's reference, whose slot the run
  // never writes: the run's starting reference or the anchor)
  if (c >= 1 && c < D) {
    int k0 = c - 1;
    while (k0 > 0 && rf[k0].chain) k0--;
    RunFrames rx;
    memset(&rx, 0, sizeof(rx));
    for (int j = k0; j < c; j++)
      for (int f = 0; f < F; f++) rx.x[j - k0][f] = fr[j].fields[f];
    launch_t_codes(rx, c - k0, F, fr[c - 1].n, t_grid(P->prev, F), P->ppool[P->prev.perm],
                   P->qpool[rf[k0].ref.q], P->qpool[P->prev.q], P->err, s);
    P->err_clean = false;
  }
  return LCP_OK;
}

// ------------------------------------------------------------------ decode
struct ParsedHdr {
  int mode, F, k, cl, A;
  int scale;  // temporal records: residual step (Sec. 7.4.2); 1 for spatial ones
  int dims;   // spatial records: spatial dimensions (byte 52; 3 for temporal ones)
  int dtype;  // element type of the fields (byte 53)
  uint64_t n, B, total, seq, ref_seq;
  uint32_t bn[3];
  float m[kMaxF], eb_q[kMaxF];
  int coder[kMaxArrays], param[kMaxArrays];
  uint32_t used[kMaxArrays];
  uint64_t an[kMaxArrays], aoff[kMaxArrays], anb[kMaxArrays];
};

uint32_t rd32(const uint8_t* b, size_t o) {
  uint32_t v;
  memcpy(&v, b + o, 4);
  return v;
}
uint64_t rd64(const uint8_t* b, size_t o) {
  uint64_t v;
  memcpy(&v, b + o, 8);
  return v;
}

lcp_status parse_header(const uint8_t* b, uint64_t size, ParsedHdr* h) {
  if (size < (uint64_t)kHdrBytes || rd32(b, 0) != kMagic || (rd32(b, 4) & 0xFFFF) != kVersion)
    return LCP_ERR_CORRUPT;
  h->mode = b[6];
  h->F = b[7];
  h->k = b[8];
  h->cl = b[9];
  h->A = b[10];
  h->scale = b[11] ? b[11] : 1;
  if ((h->mode == 0 && b[11] != 0) || h->scale > 15 || h->scale % 2 == 0) return LCP_ERR_CORRUPT;
  h->dims = b[52] ? b[52] : 3;
  if (b[52] > 2 || (h->mode == 1 && b[52] != 0)) return LCP_ERR_CORRUPT;
  h->dtype = b[53];
  if (h->dtype != kDtypeF32 && h->dtype != kDtypeI32) return LCP_ERR_CORRUPT;
  if (h->mode > 1 || h->F < (h->mode == 0 ? h->dims : 1) || h->F > kMaxF || h->k > 16 ||
      h->cl < 5 || h->cl > 16)
    return LCP_ERR_CORRUPT;
  int A = h->mode == 0 ? h->F + 2 : h->F;
  uint64_t hdr = (uint64_t)kHdrBytes + 8ull * h->F + (uint64_t)kDirBytes * A;
  if (h->A != A || rd32(b, 12) != hdr || size < hdr) return LCP_ERR_CORRUPT;
  h->n = rd64(b, 16);
  h->B = rd64(b, 24);
  h->total = rd64(b, 32);
  for (int d = 0; d < 3; d++) h->bn[d] = rd32(b, 40 + 4 * d);
  h->seq = rd64(b, 56);
  h->ref_seq = rd64(b, 64);
  if (h->total > size || h->n == 0 || h->n > (1ull << 31)) return LCP_ERR_CORRUPT;
  if (h->mode == 0 && (h->B == 0 || h->B > h->n)) return LCP_ERR_CORRUPT;
  for (int f = 0; f < h->F; f++) {
    uint32_t mb = rd32(b, kHdrBytes + 8 * f), eb = rd32(b, kHdrBytes + 8 * f + 4);
    memcpy(&h->m[f], &mb, 4);
    memcpy(&h->eb_q[f], &eb, 4);
    if (h->dtype == kDtypeI32) {
      if (eb > 0x7FFFFFFFu) return LCP_ERR_CORRUPT;  // integer half width below 2^31
      continue;
    }
    if (!isfinite(h->m[f]) || !(h->eb_q[f] > 0) || !isfinite(h->eb_q[f])) return LCP_ERR_CORRUPT;
  }
  uint64_t off = hdr;
  for (int a = 0; a < A; a++) {
    size_t d = kHdrBytes + 8 * h->F + kDirBytes * a;
    h->coder[a] = b[d];
    h->param[a] = b[d + 1];
    h->used[a] = rd32(b, d + 4);
    h->an[a] = rd64(b, d + 8);
    h->aoff[a] = rd64(b, d + 16);
    h->anb[a] = rd64(b, d + 24);
    uint64_t expect = (h->mode == 0 && a < 2) ? h->B : h->n;
    if (h->an[a] != expect || h->aoff[a] != off || h->anb[a] > h->total - off || h->coder[a] > 1)
      return LCP_ERR_CORRUPT;
    if (h->anb[a] % 4) return LCP_ERR_CORRUPT;
    const uint64_t n = h->an[a];
    if (h->coder[a] == 0) {
      if (h->param[a] > 64 || h->used[a] != 0 || h->anb[a] != 4 * ((n * (uint64_t)h->param[a] + 31) / 32))
        return LCP_ERR_CORRUPT;
    } else {
      uint64_t nchunks = (n + (1ull << h->cl) - 1) >> h->cl;
      if (n == 0 || h->used[a] == 0 || h->used[a] > (uint32_t)kAlphabet || h->param[a] < 1 ||
          h->param[a] > kMaxLen || h->anb[a] < 4ull * h->used[a] + 4 * nchunks)
        return LCP_ERR_CORRUPT;
    }
    off += h->anb[a];
  }
  if (off != h->total) return LCP_ERR_CORRUPT;
  return LCP_OK;
}

constexpr int kMaxBatchFrames = 64;
constexpr int kHdrStage = 512;  // header bytes staged per record
constexpr int kMaxBatchArrays = kMaxBatchFrames * kMaxF + 2;

// Decode one group of arrays (descriptors staged at arrtab_host[base..base+A))
// through the batched kernels; the LUT slots start at array `base`.
lcp_status decode_arrays(lcp_plan_s* P, int base, int A, int cl, uint64_t bytes, hipStream_t s) {
  // Huffman arrays with the most bits per value first: a chunk is decoded by
  // one lane from start to end, so their workgroups take longest, and started
  // first they overlap the rest instead of trailing the launch
  auto density = [](const DecArr& d) {
    return d.coder == 1 && d.n ? (double)d.nbytes / (double)d.n : -1.0;
  };
  std::stable_sort(P->arrtab_host + base, P->arrtab_host + base + A,
                   [&](const DecArr& x, const DecArr& y) { return density(x) > density(y); });
  uint32_t* hp = P->prefix_host + 2 * base;
  uint32_t* fp = hp + A;
  uint32_t hb = 0, fb = 0;
  int lut_log2 = 1;
  for (int a = 0; a < A; a++) {
    const DecArr& d = P->arrtab_host[base + a];
    hp[a] = hb;
    fp[a] = fb;
    hb += decode_blocks(d, cl, true);
    fb += decode_blocks(d, cl, false);
    if (d.coder == 1 && d.param > lut_log2) lut_log2 = d.param;
  }
  lcp_status st = upload(P->arrtab_host + base, P->arrtab_dev + base, sizeof(DecArr) * A, s);
  if (!st) st = upload(hp, P->prefix_dev + 2 * base, sizeof(uint32_t) * 2 * A, s);
  if (st) return st;
  launch_decode(P->arrtab_dev + base, A, P->prefix_dev + 2 * base, hb,
                P->prefix_dev + 2 * base + A, fb, cl, lut_log2, bytes,
                P->lut + ((uint64_t)base << kMaxLen),
                P->err, s);
  return LCP_OK;
}

// Single-frame plans: spatial records j0..j1 decoded as one batch (slot and
// block arrays concatenated, per-frame scans by rebasing batch-wide scans).
lcp_status decompress_s_batch(lcp_plan_s* P, const ParsedHdr* H, const lcp_blob* blobs,
                              const lcp_frame_out* outs, int R, hipStream_t s) {
  const int F = P->F;
  const int cl = H[0].cl;
  uint64_t ntot = 0, Btot = 0, bytes = 0;
  int A = 0;
  uint32_t* ps = P->dpre_host;
  uint32_t* pb = ps + (R + 1);
  uint32_t bs = 0, bb = 0;
  for (int r = 0; r < R; r++) {
    const ParsedHdr& h = H[r];
    unsigned __int128 tot = (unsigned __int128)h.bn[0] * h.bn[1] * h.bn[2];
    if (h.bn[0] == 0 || h.bn[1] == 0 || h.bn[2] == 0 || tot >= ((unsigned __int128)1 << 63))
      return LCP_ERR_CORRUPT;
    DSegDev& g = P->dseg_host[r];
    memset(&g, 0, sizeof(g));
    g.dtype = h.dtype;
    for (int f = 0; f < F; f++) {
      g.out[f] = outs[r].fields[f];
      g.m[f] = h.m[f];
      g.eb_q[f] = h.eb_q[f];
    }
    g.n = h.n;
    g.off = ntot;
    g.B = h.B;
    g.boff = Btot;
    g.total_blocks = (uint64_t)tot;
    g.bn0 = h.bn[0];
    g.bn1 = h.bn[1];
    g.k = h.k;
    g.D = h.dims;
    if (h.dims != H[0].dims) return LCP_ERR_ARG;  // one batch, one dimensionality
    ps[r] = bs;
    pb[r] = bb;
    bs += (uint32_t)((h.n + kSeg1k - 1) / kSeg1k);
    bb += (uint32_t)((h.B + kSeg1k - 1) / kSeg1k);
    ntot += h.n;
    Btot += h.B;
  }
  ps[R] = bs;
  pb[R] = bb;
  // every array of every record in one decode launch set
  for (int r = 0; r < R; r++) {
    const ParsedHdr& h = H[r];
    const DSegDev& g = P->dseg_host[r];
    const uint8_t* rec = reinterpret_cast<const uint8_t*>(blobs[r].data);
    for (int a = 0; a < h.A; a++) {
      DecArr& d = P->arrtab_host[A++];
      d.data = rec + h.aoff[a];
      d.nbytes = h.anb[a];
      d.n = h.an[a];
      d.coder = h.coder[a];
      d.param = h.param[a];
      d.used = h.used[a];
      if (a == 0) {
        d.out = P->v_id + g.boff;
        d.mode = 0;
        d.limit = g.total_blocks;
      } else if (a == 1) {
        d.out = P->v_cnt + g.boff;
        d.mode = 1;
        d.limit = ~0ull;
      } else {
        const int f = a - 2;
        d.out = P->v_slot + (uint64_t)f * ntot + g.off;
        d.mode = 2;
        d.limit = f < h.dims ? (1ull << h.k) : (uint64_t)kQLimit;
      }
      bytes += h.anb[a] + (a < 2 ? 8 : 4) * h.an[a];
    }
  }
  lcp_status st = upload_group({{P->dseg_host, P->dseg_dev, sizeof(DSegDev) * R},
                                 {P->dpre_host, P->dpre_dev, sizeof(uint32_t) * 2 * (R + 1)}},
                                s);
  if (!st) st = decode_arrays(P, 0, A, cl, bytes, s);
  if (st) return st;
  const uint32_t* pre_slot = P->dpre_dev;
  const uint32_t* pre_blk = P->dpre_dev + (R + 1);
  uint64_t* ids = P->v_id;
  uint64_t* cnt = P->v_cnt;
  uint64_t* cum = P->ids;
  // ids and counts: per-frame inclusive scans; slot ends: batch-wide scan of counts
  scan_device<uint64_t>(ids, Btot, nullptr, false, P->scan_tmp, s);
  seg_rebase<uint64_t>(ids, 0, 1, P->dseg_dev, pre_blk, bb, R, true,
                       reinterpret_cast<uint64_t*>(P->segbase), s);
  scan_device<uint64_t>(cnt, Btot, nullptr, false, P->scan_tmp, s);
  seg_rebase<uint64_t>(cnt, 0, 1, P->dseg_dev, pre_blk, bb, R, true,
                       reinterpret_cast<uint64_t*>(P->segbase), s);
  HIP_OK(hipMemcpyAsync(cum, cnt, Btot * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
  scan_device<uint64_t>(cum, Btot, nullptr, false, P->scan_tmp, s);
  launch_fill_u32(P->flags, ntot, 0u, s);
  launch_s_blocks_b(ids, cnt, cum, P->dseg_dev, pre_blk, bb, R, Btot, ntot, P->corner, P->flags,
                    P->err, s);
  uint32_t* tmp32 = reinterpret_cast<uint32_t*>(P->scan_tmp);
  const int D = H[0].dims;
  uint32_t* arrs[4] = {P->flags, P->v_slot, P->v_slot + ntot, P->v_slot + 2 * ntot};
  scan_device4(arrs, 1 + D, ntot, tmp32, s);
  seg_rebase<uint32_t>(P->v_slot, ntot, D, P->dseg_dev, pre_slot, bs, R, false,
                       reinterpret_cast<uint32_t*>(P->segbase), s);
  launch_s_recon_b(P->flags, P->corner, P->v_slot, P->dseg_dev, pre_slot, bs, R, F, Btot, ntot,
                   P->err, s);
  return LCP_OK;
}

// Decompress up to kMaxBatchFrames records: headers in one gather + copy, the
// entropy decoding of every position / residual array in one set of launches,
// then the per-frame reconstruction in stream order (temporal frames need the
// codes of their reference).  Stream state is committed only on success.
lcp_status decompress_group(lcp_plan_s* P, uint64_t nf, const lcp_blob* blobs,
                            const lcp_frame_out* outs, uint64_t* n_out, hipStream_t s) {
  const int F = P->F;
  const bool multi = P->p.multi_frame != 0;
  for (uint64_t j = 0; j < nf; j++) {
    if (!blobs[j].data || ((uintptr_t)blobs[j].data & 3)) return LCP_ERR_ARG;
    P->blobtab_host[2 * j] = (uint64_t)(uintptr_t)blobs[j].data;
    P->blobtab_host[2 * j + 1] = blobs[j].size;
  }
  {
    lcp_status st = upload(P->blobtab_host, P->blobtab_dev, 16 * nf, s);
    if (st) return st;
  }
  launch_gather_headers(P->blobtab_dev, (int)nf, kHdrStage, P->hdr_dev, s);
  HIP_OK(hipMemcpyAsync(P->hdr_host, P->hdr_dev, (size_t)kHdrStage * nf, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));

  std::vector<ParsedHdr> H(nf);
  std::vector<int> refq(nf, -1), dq(nf, -1);
  RefState sp = P->dprev, sa = P->danchor;
  for (uint64_t j = 0; j < nf; j++) {
    lcp_status st = parse_header(P->hdr_host + (size_t)kHdrStage * j, blobs[j].size, &H[j]);
    if (st) return st;
    const ParsedHdr& h = H[j];
    // a record of the other element type cannot go to this plan's outputs
    if (h.F != F || h.cl > 12 || h.n > P->N || h.dtype != P->p.dtype) return LCP_ERR_ARG;
    n_out[j] = h.n;
    if (h.n > outs[j].capacity) return LCP_ERR_CAPACITY;
    for (int f = 0; f < F; f++)
      if (!outs[j].fields[f]) return LCP_ERR_ARG;
    if (h.mode == 1) {
      if (sp.valid && sp.seq == h.ref_seq && sp.n == h.n) refq[j] = sp.q;
      else if (sa.valid && sa.seq == h.ref_seq && sa.n == h.n) refq[j] = sa.q;
      else return LCP_ERR_NO_REFERENCE;
    }
    if (multi) {
      for (int i = 0; i < 3; i++)
        if (!(sp.valid && sp.q == i) && !(sa.valid && sa.q == i)) {
          dq[j] = i;
          break;
        }
      RefState r;
      r.valid = true;
      r.seq = h.seq;
      r.n = h.n;
      r.q = dq[j];
      sp = r;
      if (h.mode == 0 && first_in_batch(P, h.seq)) sa = r;
    }
  }
  clear_err(P, s);
  if (!multi) {
    // independent spatial records: batches of at most NB particles
    for (uint64_t j0 = 0; j0 < nf;) {
      uint64_t j1 = j0, tot = 0;
      while (j1 < nf && tot + H[j1].n <= P->NB && (j1 == j0 || H[j1].cl == H[j0].cl)) tot += H[j1++].n;
      lcp_status st = decompress_s_batch(P, &H[j0], blobs + j0, outs + j0, (int)(j1 - j0), s);
      if (st) return st;
      j0 = j1;
    }
  } else {
  // ---- frames in sub-groups with at most kDecSlots temporal frames: one
  // decode launch for every array of the sub-group that lands in an output
  // buffer (a temporal frame's residuals go to a byte slot, escapes to its
  // output buffer), then reconstruction in stream order.  Consecutive
  // temporal frames each coded against the previous one form a chain
  // reconstructed in one pass; only the chain's last codes are kept (a later
  // record can only reference the frame just before it or an anchor, which is
  // spatial).
  int cl = nf ? H[0].cl : 10;
  bool same_cl = true;
  for (uint64_t j = 0; j < nf; j++) same_cl &= H[j].cl == cl;
  const int cap_arrays = kMaxBatchArrays + 2 * kMaxBatchFrames;
  int next = 0;  // descriptor slots used by this call
  ChainOut chain;
  memset(&chain, 0, sizeof(chain));
  int chain_len = 0, chain_ref = -1;
  uint64_t chain_last = 0;
  GridDev chain_g;
  memset(&chain_g, 0, sizeof(chain_g));
  auto flush_chain = [&]() {
    if (chain_len)
      launch_t_recon_chain(P->dqpool[chain_ref], F, H[chain_last].n, chain_g, chain, chain_len,
                           P->dqpool[dq[chain_last]], P->err, s);
    chain_len = 0;
  };
  // the arrays of frame j that land in its output buffers; tslot >= 0 puts a
  // temporal frame's residuals into that byte slot
  auto add_arrays = [&](uint64_t j, int tslot, uint64_t* bytes) {
    const ParsedHdr& h = H[j];
    const uint8_t* rec = reinterpret_cast<const uint8_t*>(blobs[j].data);
    for (int a = (h.mode == 0 ? 2 : 0); a < h.A; a++) {
      const int f = h.mode == 0 ? a - 2 : a;
      DecArr& d = P->arrtab_host[next++];
      d.data = rec + h.aoff[a];
      d.nbytes = h.anb[a];
      d.n = h.an[a];
      d.coder = h.coder[a];
      d.param = h.param[a];
      d.used = h.used[a];
      d.out = outs[j].fields[f];
      d.esc = nullptr;
      d.mode = h.mode == 0 ? 2 : 3;
      if (h.mode == 1 && tslot >= 0) {
        d.mode = 4;
        d.out = P->dres8 + ((uint64_t)tslot * F + f) * P->N;
        d.esc = reinterpret_cast<int32_t*>(outs[j].fields[f]);
      }
      d.limit = h.mode == 0 ? (f < h.dims ? (1ull << h.k) : (uint64_t)kQLimit) : (1ull << 25);
      if (bytes) *bytes += h.anb[a] + 4 * h.an[a];
    }
  };
  for (uint64_t g0 = 0; g0 < nf;) {
    uint64_t g1 = g0;
    for (int nt = 0; g1 < nf && (H[g1].mode == 0 || nt < kDecSlots); g1++) nt += H[g1].mode;
    std::vector<int> tslot(g1 - g0, -1);
    if (same_cl) {
      const int a0 = next;
      uint64_t bytes = 0;
      int t = 0;
      for (uint64_t j = g0; j < g1; j++) {
        if (next + kMaxArrays > cap_arrays) return LCP_ERR_ARG;
        if (H[j].mode == 1) tslot[j - g0] = t++;
        add_arrays(j, tslot[j - g0], &bytes);
      }
      lcp_status st = decode_arrays(P, a0, next - a0, cl, bytes, s);
      if (st) return st;
    }
    for (uint64_t j = g0; j < g1; j++) {
      const ParsedHdr& h = H[j];
      const uint64_t n = h.n;
      const uint8_t* rec = reinterpret_cast<const uint8_t*>(blobs[j].data);
      GridDev gd;
      memset(&gd, 0, sizeof(gd));
      gd.scale = h.scale;
      gd.dtype = h.dtype;
      for (int f = 0; f < F; f++) {
        gd.m[f] = h.m[f];
        gd.eb_q[f] = h.eb_q[f];
      }
      OutPtrs op;
      memset(&op, 0, sizeof(op));
      for (int f = 0; f < F; f++) op.p[f] = outs[j].fields[f];
      int32_t* q_slot = multi ? P->dqpool[dq[j]] : nullptr;
      if (next + kMaxArrays + 2 > cap_arrays) return LCP_ERR_ARG;
      if (!same_cl) {  // mixed chunk sizes: decode this frame's arrays on their own
        const int a0 = next;
        add_arrays(j, -1, nullptr);
        lcp_status st = decode_arrays(P, a0, next - a0, h.cl, 0, s);
        if (st) return st;
      }
      if (h.mode == 0) {
        flush_chain();
        const uint64_t B = h.B;
        unsigned __int128 tot = (unsigned __int128)h.bn[0] * h.bn[1] * h.bn[2];
        if (h.bn[0] == 0 || h.bn[1] == 0 || h.bn[2] == 0 || tot >= ((unsigned __int128)1 << 63))
          return LCP_ERR_CORRUPT;
        const uint64_t total_blocks = (uint64_t)tot;
        for (int a = 0; a < 2; a++) {
          DecArr& d = P->arrtab_host[next + a];
          d.data = rec + h.aoff[a];
          d.nbytes = h.anb[a];
          d.n = h.an[a];
          d.coder = h.coder[a];
          d.param = h.param[a];
          d.used = h.used[a];
          d.out = a == 0 ? (void*)P->v_id : (void*)P->v_cnt;
          d.esc = nullptr;
          d.mode = a;  // ids raw, counts unzigzagged
          d.limit = a == 0 ? total_blocks : ~0ull;
        }
        lcp_status st = decode_arrays(P, next, 2, h.cl, 0, s);
        if (st) return st;
        next += 2;
        uint64_t* ids = P->v_id;
        uint64_t* cnt = P->v_cnt;
        uint64_t* cum = P->ids;
        scan_device<uint64_t>(ids, B, nullptr, false, P->scan_tmp, s);
        scan_device<uint64_t>(cnt, B, nullptr, false, P->scan_tmp, s);
        HIP_OK(hipMemcpyAsync(cum, cnt, B * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        scan_device<uint64_t>(cum, B, nullptr, false, P->scan_tmp, s);
        launch_fill_u32(P->flags, n, 0u, s);
        launch_s_blocks(ids, cnt, cum, B, n, total_blocks, h.bn, h.k, P->corner, P->flags,
                        P->err, s);
        uint32_t* tmp32 = reinterpret_cast<uint32_t*>(P->scan_tmp);
        uint32_t* arrs[4] = {P->flags, nullptr, nullptr, nullptr};
        for (int d = 0; d < h.dims; d++) arrs[1 + d] = reinterpret_cast<uint32_t*>(outs[j].fields[d]);
        scan_device4(arrs, 1 + h.dims, n, tmp32, s);
        launch_s_recon(P->flags, P->corner, B, F, h.dims, n, h.k, gd, op, q_slot, P->err, s);
      } else {
        const bool extend = chain_len > 0 && chain_len < kChainMax && j > g0 &&
                            chain_last == j - 1 && refq[j] == dq[j - 1] && H[j - 1].n == n &&
                            memcmp(&chain_g, &gd, sizeof(gd)) == 0;
        if (!extend) {
          flush_chain();
          chain_ref = refq[j];
          chain_g = gd;
        }
        const int t = tslot[j - g0];
        for (int f = 0; f < F; f++) {
          chain.p[chain_len][f] = outs[j].fields[f];
          chain.r8[chain_len][f] = t >= 0 ? P->dres8 + ((uint64_t)t * F + f) * P->N : nullptr;
        }
        chain_len++;
        chain_last = j;
      }
    }
    flush_chain();
    g0 = g1;
  }
  }
  {
    lcp_status st = read_ret(P, 1, s);
    if (st) return st;
  }
  if (g_timer_plan == P) timer_collect(P);
  if (host_err(P) & kErrCorrupt) return LCP_ERR_CORRUPT;
  if (multi) {
    P->dprev = sp;
    P->danchor = sa;
    P->dec_last_t = nf > 0 && H[nf - 1].mode == 1;
  }
  return LCP_OK;
}

// A list of buffers placed back to back (256-byte aligned) in one block.
struct Layout {
  struct Item {
    void** ptr;
    size_t bytes;
  };
  std::vector<Item> items;
  size_t total = 0;
  template <typename T>
  void add(T** p, size_t elems) {
    size_t b = elems * sizeof(T);
    b = b ? (b + 255) & ~(size_t)255 : 256;
    items.push_back({reinterpret_cast<void**>(p), b});
    total += b;
  }
  void place(void* base) const {
    size_t o = 0;
    for (const Item& it : items) {
      *it.ptr = static_cast<uint8_t*>(base) + o;
      o += it.bytes;
    }
  }
};

// Scratch of one call: device buffers (D) and pinned host tables (H).  Sizes
// follow from the plan's particle capacities; nothing in them outlives a call
// except that the spread histogram copies must be zero between calls.
void layout_scratch(lcp_plan_s* P, Layout& D, Layout& H) {
  const uint64_t N = P->N, NB = P->NB;
  const int F = P->F, RB = P->RB;
  const uint64_t ntiles = (NB + kSortTile - 1) / kSortTile + RB;  // tiles never cross frames
  P->NAmax = RB * (F + 2);
  if (P->run_max * F > P->NAmax) P->NAmax = P->run_max * F;  // a run's arrays
  const uint64_t NA = (uint64_t)P->NAmax;
  const uint64_t RR = (uint64_t)(RB > P->run_max ? RB : P->run_max);  // records per launch set
  // spread histogram copies: enc_hist_copies(n) <= 1 + (1 + n / 8192) / 16 per
  // array; the residual kernel uses kHistCopies per field
  uint64_t hc = 2 * NA + (uint64_t)(F + 2) * NB / 131072 + 1;
  if (hc > NA * kHistCopies) hc = NA * kHistCopies;
  if (hc < (uint64_t)kMaxF * kHistCopies) hc = (uint64_t)kMaxF * kHistCopies;
  if (hc < (uint64_t)P->run_max * F * kRunCopies) hc = (uint64_t)P->run_max * F * kRunCopies;
  if (P->serve_batch && hc < (uint64_t)RB * F * kServeCopies) hc = (uint64_t)RB * F * kServeCopies;
  P->hist_copies = hc;
  P->cw_cap = (uint64_t)(F + 2) * NB / (1ull << P->chunk_log2) + NA + 1;
  // staging: enc_stage_words summed over a batch's arrays; per array type a
  // batch has at most NB / C + RB chunks (ids and counts are 64-bit, the rest
  // 32-bit)
  P->stage_cap = ((uint64_t)2 * enc_slot_words(true, P->chunk_log2) +
                  (uint64_t)F * enc_slot_words(false, P->chunk_log2)) *
                 ((NB >> P->chunk_log2) + RB + 1);
  // a run's arrays: run_max * F byte arrays of at most N values
  const uint64_t run_chunks = (uint64_t)P->run_max * F * ((N >> P->chunk_log2) + 1);
  if (P->cw_cap < run_chunks + NA + 1) P->cw_cap = run_chunks + NA + 1;
  if (P->stage_cap < run_chunks * enc_slot_words(false, P->chunk_log2))
    P->stage_cap = run_chunks * enc_slot_words(false, P->chunk_log2);
  P->run_stride = (N + 63) & ~(uint64_t)63;
  uint64_t sn = NB > 256 * ntiles ? NB : 256 * ntiles;
  P->scan_tmp_n = scan_tmp_elems(sn);
  P->rec_tmp_cap = bound_bytes(F, N);
  const bool sb = P->serve_batch;
  const uint64_t NS = sb ? 0 : NB;  // the spatial path's per-particle buffers
  D.add(&P->keys0, NS);
  D.add(&P->keys1, NS);
  D.add(&P->ids, NS);
  D.add(&P->v_id, NS);
  D.add(&P->v_cnt, NS);
  D.add(&P->slot_rec, NS * (uint64_t)slot_rec_words(F, P->D));
  D.add(&P->vals0, NS);
  D.add(&P->vals1, NS);
  D.add(&P->hist, sb ? 0 : 256 * ntiles);
  D.add(&P->flags, NS);
  D.add(&P->starts, NS);
  D.add(&P->v_slot, (uint64_t)F * NB);
  if (P->p.multi_frame || sb) {
    D.add(&P->v_byte, (uint64_t)F * NB);
    D.add(&P->dres8, (uint64_t)(sb ? 1 : kDecSlots) * F * NB);
  } else {
    P->v_byte = nullptr;
    P->dres8 = nullptr;
  }
  D.add(&P->chunk_words, P->cw_cap);
  D.add(&P->stage, P->stage_cap);
  // decode-only tables: 2^13 LUT entries per array of a decode launch, header
  // staging, descriptor tables, block corners
  const uint64_t dec_arrays = P->compress_only ? 0 : kMaxBatchArrays + 2 * kMaxBatchFrames;
  const uint64_t dec_frames = P->compress_only ? 0 : (sb && RB > kMaxBatchFrames ? (uint64_t)RB : kMaxBatchFrames);
  D.add(&P->lut, dec_arrays << kMaxLen);
  D.add(&P->ext_part, (uint64_t)2 * kMaxF * kSegExtCap * RB);
  D.add(&P->hist_part, hc * kAlphabet);
  D.add(&P->hist_max, hc);
  D.add(&P->huff_lens, NA * kHuffCandidates * kAlphabet);
  D.add(&P->huff_maxd, NA * kHuffCandidates);
  D.add(&P->hdr_dev, (uint64_t)kHdrStage * dec_frames);
  D.add(&P->blobtab_dev, 2 * dec_frames);
  D.add(&P->arrtab_dev, dec_arrays);
  D.add(&P->prefix_dev, 2 * dec_arrays);
  D.add(&P->corner, P->compress_only || sb ? 0 : 3 * NB);
  D.add(&P->scan_tmp, P->scan_tmp_n);
  D.add(&P->work, NA);
  D.add(&P->ret_dev, 2 + (uint64_t)RB + (uint64_t)RB * F);
  D.add(&P->run_dev, 4 * kTRun + kTRun + 2);
  D.add(&P->run_v8, (uint64_t)P->run_max * F * P->run_stride);
  D.add(&P->run_esc, (uint64_t)P->run_max * F * P->run_stride);
  // tables uploaded together are adjacent, with the same sizes as their host
  // staging (seg + segpre, dseg + dpre, erec + earr + epre)
  D.add(&P->seg_dev, RB);
  D.add(&P->segpre_dev, 4 * ((uint64_t)RB + 1));
  D.add(&P->dseg_dev, dec_frames);
  D.add(&P->dpre_dev, P->compress_only ? 0 : 2 * (kMaxBatchFrames + 1));
  D.add(&P->erec_dev, RR);
  D.add(&P->earr_dev, NA);
  D.add(&P->epre_dev, 4 * (NA + 1));
  D.add(&P->rstart, (uint64_t)RB + 1);
  D.add(&P->Bs, RB);
  D.add(&P->permdst_dev, RB);
  D.add(&P->segbase, 3 * dec_frames);
  if (sb) P->rec_tmp_cap = bound_bytes(F, NB) + 4096ull * RB;  // records of a merged launch
  D.add(&P->rec_tmp, P->compress_only ? 0 : P->rec_tmp_cap);
  D.add(&P->tfr_dev, sb ? RB : 0);
  D.add(&P->trc_dev, sb ? RB : 0);
  D.add(&P->spre_dev, sb ? (uint64_t)RB + 1 : 0);
  D.add(&P->sret_dev, sb ? 2 * (uint64_t)RB + 2 : 0);
  D.add(&P->sdst_dev, sb ? 2 * (uint64_t)RB : 0);
  H.add(&P->ret_host, 2 + (size_t)RB + (size_t)RB * F);
  H.add(&P->run_host, 4 * kTRun + kTRun + 2);
  H.add(&P->hdr_host, (size_t)kHdrStage * dec_frames);
  H.add(&P->blobtab_host, 2 * dec_frames);
  H.add(&P->arrtab_host, dec_arrays);
  H.add(&P->prefix_host, 2 * dec_arrays);
  H.add(&P->seg_host, RB);
  H.add(&P->segpre_host, 4 * ((size_t)RB + 1));
  H.add(&P->dseg_host, dec_frames);
  H.add(&P->dpre_host, P->compress_only ? 0 : 2 * (kMaxBatchFrames + 1));
  H.add(&P->erec_host, RR);
  H.add(&P->earr_host, NA);
  H.add(&P->epre_host, 4 * (NA + 1));
  H.add(&P->permdst_host, RB);
  H.add(&P->tfr_host, sb ? RB : 0);
  H.add(&P->trc_host, sb ? RB : 0);
  H.add(&P->spre_host, sb ? (size_t)RB + 1 : 0);
  H.add(&P->sret_host, sb ? 2 * (size_t)RB + 2 : 0);
  H.add(&P->sdst_host, sb ? 2 * (size_t)RB : 0);
}

// Resident stream state of multi-frame plans: the compressor's candidate and
// reference codes and permutations, the decompressor's reference codes.
void layout_state(lcp_plan_s* P, Layout& S) {
  if (!P->p.multi_frame) return;
  const uint64_t N = P->N;
  const int F = P->F;
  for (int i = 0; i < 4; i++) S.add(&P->qpool[i], (uint64_t)F * N);
  for (int i = 0; i < 3; i++) S.add(&P->ppool[i], N);
  for (int i = 0; i < 3; i++) S.add(&P->dqpool[i], (uint64_t)F * N);
}

// Points the plan's scratch at a device block (layout_scratch's D.total bytes)
// and a pinned host block (H.total bytes), and clears the spread histogram
// copies on stream s.
void bind_scratch(lcp_plan_s* P, void* dev, void* host, hipStream_t s) {
  Layout D, H;
  layout_scratch(P, D, H);
  D.place(dev);
  H.place(host);
  P->enc_cache_ok = false;
  drop_graphs(P);  // they hold the scratch pointers of the last binding
  P->err = reinterpret_cast<uint32_t*>(P->ret_dev);
  P->offs_dev = P->ret_dev + 1;
  P->ext_dev = reinterpret_cast<uint32_t*>(P->ret_dev + 2 + P->RB);
  memset(P->seg_host, 0, sizeof(SegDev) * P->RB);
  launch_fill_u32(P->hist_part, P->hist_copies * kAlphabet, 0u, s);
  launch_fill_u32(reinterpret_cast<uint32_t*>(P->hist_max), 2 * P->hist_copies, 0u, s);
  launch_fill_u32(P->err, 1, 0u, s);
  P->err_clean = true;
  P->bound = true;
}

lcp_status alloc_state(lcp_plan_s* P) {
  Layout S;
  layout_state(P, S);
  P->state_bytes = S.items.empty() ? 0 : S.total;
  if (P->state_bytes) {
    HIP_OK(hipMalloc(&P->state_dev, P->state_bytes));
    S.place(P->state_dev);
  }
  return LCP_OK;
}

// Frames a temporal run of a multi-frame plan codes at once: as many as keep
// the run's buffers (residual bytes, escapes, staging, histogram copies) within
// kRunBytes, at most kRunMax; fewer than two means no runs.
constexpr uint64_t kRunBytes = 4ull << 30;
int run_frames_for(const lcp_plan_s* P) {
  if (!P->p.multi_frame) return 0;
  const uint64_t N = P->N, F = (uint64_t)P->F;
  const uint64_t chunks = (N >> P->chunk_log2) + 1;
  const uint64_t per = F * ((N + 63) & ~63ull) * 5 + F * chunks * 4 * (enc_slot_words(false, P->chunk_log2) + 1) +
                       F * kRunCopies * kAlphabet * 4ull;
  uint64_t d = kRunBytes / per;
  if (d > (uint64_t)run_launch_frames(P->F)) d = run_launch_frames(P->F);
  return d < 2 ? 0 : (int)d;
}

lcp_status alloc_plan(lcp_plan_s* P) {
  Layout D, H, S;
  P->run_max = run_frames_for(P);
  layout_scratch(P, D, H);
  layout_state(P, S);
  const size_t state = S.items.empty() ? 0 : S.total;
  // within a budget, temporal runs get fewer frames, then none, before the plan fails
  while (P->p.hbm_budget_bytes && D.total + state > P->p.hbm_budget_bytes && P->run_max > 0) {
    P->run_max = P->run_max > 2 ? P->run_max / 2 : 0;
    D = Layout();
    H = Layout();
    layout_scratch(P, D, H);
  }
  P->scratch_bytes = D.total;
  P->host_bytes = H.total;
  const size_t need = D.total + state;
  if (P->p.hbm_budget_bytes && need > P->p.hbm_budget_bytes) return LCP_ERR_BUDGET;
  HIP_OK(hipMalloc(&P->own_dev, D.total));
  HIP_OK(hipHostMalloc(&P->own_host, H.total, 0));
  lcp_status st = alloc_state(P);
  if (st) return st;
  bind_scratch(P, P->own_dev, P->own_host, nullptr);
  HIP_OK(hipStreamSynchronize(nullptr));
  return LCP_OK;
}

void free_plan(lcp_plan_s* P) {
  drop_graphs(P);
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
  if (P->own_dev) (void)hipFree(P->own_dev);
  if (P->state_dev) (void)hipFree(P->state_dev);
  if (P->own_host) (void)hipHostFree(P->own_host);
  for (auto e : P->ev_free) (void)hipEventDestroy(e);
  for (auto& pr : P->ev_pending) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  delete P;
}

// Block-size search (Sec. 7.4.1): every feasible k in [0,16] codes the stride
// sample; the smallest record wins, ties to the smaller k.
lcp_status search_k(lcp_plan_s* P, const float* const* sample, uint64_t sn, hipStream_t s) {
  const int F = P->F;
  uint64_t stride = sn >> 20;
  if (stride < 1) stride = 1;
  const uint64_t ns = (sn + stride - 1) / stride;
  std::vector<float*> tmp(F, nullptr);
  const float* xs[kMaxF];
  lcp_status st = LCP_OK;
  for (int f = 0; f < F && !st; f++) {
    if (stride == 1) {
      xs[f] = sample[f];
      continue;
    }
    if (hipMalloc((void**)&tmp[f], ns * sizeof(float)) != hipSuccess) st = LCP_ERR_DEVICE;
    else if (hipMemcpy2DAsync(tmp[f], sizeof(float), sample[f], stride * sizeof(float),
                              sizeof(float), ns, hipMemcpyDeviceToDevice, s) != hipSuccess)
      st = LCP_ERR_DEVICE;
    xs[f] = tmp[f];
  }
  double lo[kMaxF], hi[kMaxF];
  double eb[kMaxF];
  HostGrid g[kMaxF];
  if (!st) st = extent(P, xs, ns, lo, hi, s);
  if (!st) st = field_eb(P->p, F, lo, hi, eb);
  if (!st) st = make_grids(P->p, F, lo, hi, eb, 1, g);
  int best = -1;
  uint64_t best_size = 0;
  for (int k = 0; k <= 16 && !st; k++) {
    SResult r;
    lcp_status s2 = compress_s(P, xs, ns, g, hi, k, 0, P->rec_tmp, P->rec_tmp_cap, nullptr, &r, s);
    if (s2 == LCP_OK && (best < 0 || r.size < best_size)) {
      best = k;
      best_size = r.size;
    } else if (s2 != LCP_OK && s2 != LCP_ERR_RANGE) {
      st = s2;
    }
  }
  for (float* p : tmp)
    if (p) (void)hipFree(p);
  if (st) return st;
  if (best < 0) return LCP_ERR_RANGE;
  P->k = best;
  return LCP_OK;
}

// Single-frame plans: R independent frames through one extent pass and one
// LCP-S launch set.  offs (host, R + 1) receives the records' offsets from out.
lcp_status compress_group(lcp_plan_s* P, int R, const lcp_frame_in* fr, uint8_t* out,
                          uint64_t cap, uint64_t* offs, uint32_t* const* perms, hipStream_t s) {
  const int F = P->F;
  for (int r = 0; r < R; r++) {
    for (int f = 0; f < F; f++) P->seg_host[r].x[f] = fr[r].fields[f];
    P->seg_host[r].n = fr[r].n;
  }
  std::vector<double> lo((size_t)R * kMaxF), hi((size_t)R * kMaxF);
  double(*lo2)[kMaxF] = reinterpret_cast<double(*)[kMaxF]>(lo.data());
  double(*hi2)[kMaxF] = reinterpret_cast<double(*)[kMaxF]>(hi.data());
  lcp_status st = extent_batch(P, R, lo2, hi2, s);
  if (st) return st;
  std::vector<HostGrid> g((size_t)R * kMaxF);
  HostGrid(*g2)[kMaxF] = reinterpret_cast<HostGrid(*)[kMaxF]>(g.data());
  for (int r = 0; r < R; r++) {
    double eb[kMaxF];
    if ((st = field_eb(P->p, F, lo2[r], hi2[r], eb))) return st;
    if ((st = make_grids(P->p, F, lo2[r], hi2[r], eb, 1, g2[r]))) return st;
  }
  st = compress_s_batch(P, R, g2, hi2, P->k, P->seq, out, cap, nullptr, perms, offs, nullptr, s);
  if (st) return st;
  P->seq += (uint64_t)R;
  return LCP_OK;
}

// The autotuner's choices, shared by every plan of the process: (GPU name and
// compute units, bit width of a call's total particles, fields) -> shape.
std::mutex g_tune_mu;
std::map<std::tuple<std::string, int, int>, lcp_tuning> g_tune_cache;
const lcp_tuning kDefaultTuning{1024, 0, 0, 1};

std::tuple<std::string, int, int> tune_key(const lcp_plan_s* P, uint64_t particles) {
  return std::make_tuple(P->dev_key, bitwidth64(particles), P->F);
}

// The launch shape for a call of `particles` particles: the plan's own
// setting, else the cached choice for its key, else the defaults.
void pick_tuning(lcp_plan_s* P, uint64_t particles) {
  if (P->tune_set) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune_cache.find(tune_key(P, particles));
  P->tune = it != g_tune_cache.end() ? it->second : kDefaultTuning;
}

// Single-frame plans: independent frames in batches of up to RB frames and
// NB particles, each batch one extent pass and one LCP-S launch set.
lcp_status compress_independent(lcp_plan_s* plan, uint64_t n_frames, const lcp_frame_in* frames,
                                uint8_t* o, uint64_t out_cap, uint64_t* out_offsets,
                                int* methods_used, uint32_t* const* perms, hipStream_t stream) {
  uint64_t off = 0;
  out_offsets[0] = 0;
  std::vector<uint64_t> offs((size_t)plan->RB + 1);
  uint64_t particles = 0;
  for (uint64_t j = 0; j < n_frames; j++) particles += frames[j].n;
  pick_tuning(plan, particles);
  for (uint64_t j = 0; j < n_frames;) {
    int R = 0;
    uint64_t tot = 0;
    while (j + R < n_frames && R < plan->RB) {
      const lcp_frame_in& fr = frames[j + R];
      if (fr.n == 0 || fr.n > plan->N || fr.method < 0 || fr.method > 2) return LCP_ERR_ARG;
      for (int f = 0; f < plan->F; f++)
        if (!fr.fields[f]) return LCP_ERR_ARG;
      if (fr.method == LCP_METHOD_T) return LCP_ERR_NO_REFERENCE;
      if (tot + fr.n > plan->NB) break;
      tot += fr.n;
      R++;
    }
    uint64_t cap = out_cap > off ? out_cap - off : 0;
    lcp_status st = compress_group(plan, R, frames + j, o + off, cap, offs.data(),
                                   perms ? perms + j : nullptr, stream);
    if (st == LCP_ERR_CAPACITY) {
      for (int r = 0; r < R; r++) out_offsets[j + r + 1] = off + offs[r + 1];
      out_offsets[n_frames] = off + offs[R];  // the bytes required so far
      return st;
    }
    if (st) return st;
    for (int r = 0; r < R; r++) {
      if (methods_used) methods_used[j + r] = LCP_METHOD_S;
      out_offsets[j + r + 1] = off + offs[r + 1];
    }
    off += offs[R];
    j += (uint64_t)R;
  }
  timer_collect(plan);
  return LCP_OK;
}

}  // namespace

namespace {
lcp_status plan_check(const lcp_params& p, const float* const* sample_fields, uint64_t sample_n) {
  const int cl = p.chunk_log2 == 0 ? 10 : p.chunk_log2;
  if (p.n_fields < 1 || p.n_fields > LCP_MAX_FIELDS || cl < 5 || cl > 12 || p.batch_size < 0 ||
      p.n_dims < 0 || p.n_dims > 3 || p.n_fields < (p.n_dims ? p.n_dims : 3) ||
      p.block_log2 < -1 || p.block_log2 > 16 || p.max_particles == 0 ||
      p.max_particles > (1ull << 31) || !(p.eb > 0) || p.eb_mode < 0 || p.eb_mode > 2 ||
      p.max_batch_frames < 0 || p.max_batch_frames > kMaxBatch ||
      (p.max_batch_particles != 0 &&
       (p.max_batch_particles < p.max_particles || p.max_batch_particles > 0xFFFFFFFFull)) ||
      p.anchor_scale < 0 || p.anchor_scale > 15 || (p.anchor_scale > 1 && p.anchor_scale % 2 == 0) ||
      (p.dtype != LCP_DTYPE_F32 && p.dtype != LCP_DTYPE_I32))
    return LCP_ERR_ARG;
  if (p.block_log2 == -1 && (!sample_fields || sample_n == 0 || sample_n > p.max_particles))
    return LCP_ERR_ARG;
  return LCP_OK;
}

// The plan's sizes and parameters from checked params (no memory).
void plan_fill(lcp_plan_s* P, const lcp_params& p) {
  const int cl = p.chunk_log2 == 0 ? 10 : p.chunk_log2;
  P->p = p;
  P->p.chunk_log2 = cl;
  P->chunk_log2 = cl;
  P->F = p.n_fields;
  P->D = p.n_dims ? p.n_dims : 3;
  P->N = p.max_particles;
  if (p.multi_frame) {
    P->RB = 1;
    P->NB = P->N;
  } else {
    P->RB = p.max_batch_frames == 0 ? 64 : p.max_batch_frames;
    P->NB = p.max_batch_particles == 0 ? P->N : p.max_batch_particles;
  }
  P->k = p.block_log2 < 0 ? 0 : p.block_log2;
}

// Validates params and fills the plan's sizes (no device memory).
lcp_status plan_setup(const lcp_params* params, const float* const* sample_fields,
                      uint64_t sample_n, lcp_plan_s** out) {
  if (!params || !out) return LCP_ERR_ARG;
  *out = nullptr;
  lcp_status st = plan_check(*params, sample_fields, sample_n);
  if (st) return st;
  if (hipSetDevice(params->device) != hipSuccess) return LCP_ERR_DEVICE;
  lcp_plan_s* P = new lcp_plan_s();
  plan_fill(P, *params);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, params->device) == hipSuccess)
    P->dev_key = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
  *out = P;
  return LCP_OK;
}
}  // namespace

namespace lcp {
bool ktimer_events(const char* name, uint64_t bytes, hipEvent_t* start, hipEvent_t* stop) {
  lcp_plan_s* P = g_timer_plan;
  if (!P || P->capturing || !P->timer_name[0] || strcmp(P->timer_name, name) != 0) return false;
  if (P->timer_seen++ % P->timer_every != 0) return false;
  *start = timer_event(P);
  *stop = timer_event(P);
  P->ev_pending.push_back({*start, *stop});
  P->ev_bytes.push_back(bytes);
  return true;
}

lcp_status plan_create_unbound(const lcp_params* params, const float* const* sample_fields,
                               uint64_t sample_n, lcp_plan_t* out) {
  lcp_plan_s* P = nullptr;
  lcp_status st = plan_setup(params, sample_fields, sample_n, &P);
  if (st) return st;
  Layout D, H;
  layout_scratch(P, D, H);
  P->scratch_bytes = D.total;
  P->host_bytes = H.total;
  st = alloc_state(P);
  if (!st && params->block_log2 == -1) {
    // the search needs scratch once; it is released afterwards
    void *dev = nullptr, *host = nullptr;
    hipError_t e = hipMalloc(&dev, D.total);
    if (e == hipSuccess) e = hipHostMalloc(&host, H.total, 0);
    if (e != hipSuccess) {
      st = hip_fail(e, "scratch for the block-size search", __LINE__);
    } else {
      bind_scratch(P, dev, host, nullptr);
      TimerScope ts(P);
      st = search_k(P, sample_fields, sample_n, nullptr);
      e = hipStreamSynchronize(nullptr);
      if (e != hipSuccess && !st) st = hip_fail(e, "hipStreamSynchronize", __LINE__);
    }
    if (dev) (void)hipFree(dev);
    if (host) (void)hipHostFree(host);
    P->bound = false;
  }
  if (st) {
    free_plan(P);
    return st;
  }
  *out = P;
  return LCP_OK;
}

size_t plan_scratch_bytes(lcp_plan_t P) { return P->scratch_bytes; }
size_t plan_host_bytes(lcp_plan_t P) { return P->host_bytes; }
size_t plan_state_bytes(lcp_plan_t P) { return P->state_bytes; }
void plan_bind(lcp_plan_t P, void* dev, void* host, hipStream_t s) { bind_scratch(P, dev, host, s); }
void plan_unbind(lcp_plan_t P) { P->bound = false; }

}  // namespace lcp

// ================================================================== C ABI
extern "C" {

const char* lcp_status_string(lcp_status st) {
  switch (st) {
    case LCP_OK: return "ok";
    case LCP_ERR_ARG: return "invalid argument";
    case LCP_ERR_EB_TOO_SMALL: return "error bound too small for float32 data";
    case LCP_ERR_RANGE: return "quantisation codes or block ids out of range";
    case LCP_ERR_CAPACITY: return "output buffer too small";
    case LCP_ERR_CORRUPT: return "corrupt record";
    case LCP_ERR_NO_REFERENCE: return "reference frame not resident";
    case LCP_ERR_BUDGET: return "HBM budget exceeded";
    case LCP_ERR_DEVICE: return "HIP runtime error";
  }
  return "unknown status";
}


lcp_status lcp_plan(const lcp_params* params, const float* const* sample_fields,
                    uint64_t sample_n, lcp_plan_t* out) {
  lcp_plan_s* P = nullptr;
  lcp_status st = plan_setup(params, sample_fields, sample_n, &P);
  if (st) return st;
  st = alloc_plan(P);
  if (!st && params->block_log2 == -1) {
    TimerScope ts(P);
    st = search_k(P, sample_fields, sample_n, nullptr);
  }
  if (st) {
    free_plan(P);
    return st;
  }
  *out = P;
  return LCP_OK;
}

void lcp_plan_destroy(lcp_plan_t plan) {
  if (plan) free_plan(plan);
}

int lcp_plan_block_log2(lcp_plan_t plan) { return plan ? plan->k : -1; }

lcp_status lcp_plan_reset(lcp_plan_t plan) {
  if (!plan) return LCP_ERR_ARG;
  plan->prev = RefState();
  plan->anchor = RefState();
  plan->dprev = RefState();
  plan->danchor = RefState();
  plan->dec_last_t = false;
  plan->have_eb = false;
  plan->seq = 0;
  plan->fsm_state = kFsmS1;
  plan->untested = 0;
  plan->last_s = 0;
  plan->have_last_s = false;
  plan->n_since_anchor = 0;
  plan->t_since_anchor = 0;
  return LCP_OK;
}

uint64_t lcp_bound(lcp_plan_t plan, uint64_t n) { return plan ? bound_bytes(plan->F, n) : 0; }

lcp_status lcp_scratch_bytes(const lcp_params* params, uint64_t* device_bytes) {
  if (!device_bytes) return LCP_ERR_ARG;
  lcp_plan_s* P = nullptr;
  lcp_params q;
  if (!params) return LCP_ERR_ARG;
  q = *params;
  if (q.block_log2 == -1) q.block_log2 = 0;  // the search does not change the sizes
  lcp_status st = plan_setup(&q, nullptr, 0, &P);
  if (st) return st;
  Layout D, H;
  layout_scratch(P, D, H);
  *device_bytes = (D.total + 255) & ~(uint64_t)255;
  delete P;
  return LCP_OK;
}

lcp_status lcp_compress(lcp_plan_t plan, uint64_t n_frames, const lcp_frame_in* frames,
                        void* out, uint64_t out_cap, uint64_t* out_offsets, int* methods_used,
                        uint32_t* const* perms, hipStream_t stream) {
  if (!plan || (!frames && n_frames) || !out_offsets || (!out && n_frames)) return LCP_ERR_ARG;
  if ((uintptr_t)out & 3 || !plan->bound) return LCP_ERR_ARG;
  TimerScope ts(plan);
  uint8_t* o = reinterpret_cast<uint8_t*>(out);
  uint64_t off = 0;
  out_offsets[0] = 0;
  if (!plan->p.multi_frame)
    return compress_independent(plan, n_frames, frames, o, out_cap, out_offsets, methods_used,
                                perms, stream);
  bool one = false;  // the next frame goes through the per-frame path
  for (uint64_t j = 0; j < n_frames;) {
    uint64_t cap = out_cap > off ? out_cap - off : 0;
    RunFrame rf[kTRun];
    const int D = one ? 0 : plan_run(plan, frames + j, n_frames - j, cap, rf);
    if (D >= 2) {
      uint64_t ends[kTRun];
      int c = 0;
      lcp_status st = run_t(plan, frames + j, D, rf, o + off, cap, perms ? perms + j : nullptr,
                            ends, &c, stream);
      if (st) return st;
      for (int k = 0; k < c; k++) {
        if (methods_used) methods_used[j + k] = LCP_METHOD_T;
        out_offsets[j + k + 1] = off + ends[k];
      }
      if (c) off += ends[c - 1];
      j += (uint64_t)c;
      one = c < D;
      continue;
    }
    one = false;
    uint64_t size = 0;
    int used = 0;
    lcp_status st = compress_frame(plan, frames[j], o + off, cap, &size, &used,
                                   perms ? perms[j] : nullptr, stream);
    if (st) {
      out_offsets[j + 1] = off + size;
      if (st == LCP_ERR_CAPACITY) out_offsets[n_frames] = off + size;
      return st;
    }
    if (methods_used) methods_used[j] = used;
    off += (size + 3) & ~3ull;
    out_offsets[j + 1] = off;
    j++;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return LCP_ERR_DEVICE;
  timer_collect(plan);
  return LCP_OK;
}

lcp_status lcp_decompress(lcp_plan_t plan, uint64_t n_frames, const lcp_blob* blobs,
                          const lcp_frame_out* outs, uint64_t* n_out, hipStream_t stream) {
  if (!plan || (n_frames && (!blobs || !outs || !n_out)) || !plan->bound) return LCP_ERR_ARG;
  TimerScope ts(plan);
  for (uint64_t j = 0; j < n_frames; j += kMaxBatchFrames) {
    uint64_t g = n_frames - j < (uint64_t)kMaxBatchFrames ? n_frames - j : kMaxBatchFrames;
    lcp_status st = decompress_group(plan, g, blobs + j, outs + j, n_out + j, stream);
    if (st) return st;
  }
  timer_collect(plan);
  return LCP_OK;
}

lcp_status lcp_select(lcp_plan_t plan, int* decision) {
  if (!plan || !decision) return LCP_ERR_ARG;
  bool have_ref = false;
  if (plan->p.multi_frame) {
    const RefState* r = first_in_batch(plan, plan->seq) ? &plan->anchor : &plan->prev;
    have_ref = r->valid;
  }
  *decision = fsm_decide(plan, have_ref);
  return LCP_OK;
}

lcp_status lcp_plan_set_tuning(lcp_plan_t plan, const lcp_tuning* t) {
  if (!plan || !t || t->tile < 256 || t->tile > 16384 || t->tile % 256 || t->grid > (1u << 20) ||
      t->slot_grid > (1u << 20) || (t->graphs != 0 && t->graphs != 1))
    return LCP_ERR_ARG;
  plan->tune = *t;
  plan->tune_set = true;
  return LCP_OK;
}

lcp_status lcp_plan_get_tuning(lcp_plan_t plan, lcp_tuning* t) {
  if (!plan || !t) return LCP_ERR_ARG;
  *t = plan->tune;
  return LCP_OK;
}

lcp_status lcp_plan_autotune(lcp_plan_t plan, uint64_t n_frames, const lcp_frame_in* frames,
                             void* out, uint64_t out_cap, int reps, hipStream_t stream,
                             lcp_tuning* chosen, double* best_ms, double* default_ms) {
  if (!plan || plan->p.multi_frame || !frames || n_frames == 0 || !out || ((uintptr_t)out & 3) ||
      !plan->bound || reps < 1)
    return LCP_ERR_ARG;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, plan->p.device) != hipSuccess ||
      cus < 1)
    return LCP_ERR_DEVICE;
  std::vector<lcp_tuning> cand;
  for (uint32_t tile : {1024u, 2048u, 4096u})
    for (uint32_t g : {0u, 8u, 32u})
      for (uint32_t sg : {0u, 16u}) cand.push_back(lcp_tuning{tile, g * cus, sg * cus, 1});
  std::vector<uint64_t> offs(n_frames + 1);
  const uint64_t seq0 = plan->seq;
  const lcp_tuning saved = plan->tune;
  const bool saved_set = plan->tune_set;
  TimerScope ts(plan);
  // best-of-reps wall time of one call (each call waits for its records), the
  // first call of a shape capturing its graph untimed
  auto time_of = [&](const lcp_tuning& t, double* ms) -> lcp_status {
    plan->tune = t;
    plan->tune_set = true;
    double best = 1e30;
    for (int r = -1; r < reps; r++) {
      plan->seq = seq0;
      const auto t0 = std::chrono::steady_clock::now();
      lcp_status st = compress_independent(plan, n_frames, frames, reinterpret_cast<uint8_t*>(out),
                                           out_cap, offs.data(), nullptr, nullptr, stream);
      const auto t1 = std::chrono::steady_clock::now();
      if (st) return st;
      if (r >= 0) best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    *ms = best;
    return LCP_OK;
  };
  double dflt = 0, best = 1e30;
  lcp_tuning pick = kDefaultTuning;
  lcp_status st = time_of(kDefaultTuning, &dflt);
  best = dflt;
  for (size_t i = 0; !st && i < cand.size(); i++) {
    double ms = 0;
    st = time_of(cand[i], &ms);
    if (!st && ms < best) {
      best = ms;
      pick = cand[i];
    }
  }
  plan->seq = seq0;
  if (st) {
    plan->tune = saved;
    plan->tune_set = saved_set;
    return st;
  }
  plan->tune = pick;
  plan->tune_set = true;
  uint64_t particles = 0;
  for (uint64_t j = 0; j < n_frames; j++) particles += frames[j].n;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[tune_key(plan, particles)] = pick;
  }
  if (chosen) *chosen = pick;
  if (best_ms) *best_ms = best;
  if (default_ms) *default_ms = dflt;
  return LCP_OK;
}

lcp_status lcp_kernel_timer_set(lcp_plan_t plan, const char* kernel_name) {
  if (!plan) return LCP_ERR_ARG;
  plan->timer_every = kTimerStride;
  if (!kernel_name) {
    plan->timer_name[0] = 0;
  } else {
    // "name" or "name/N": one launch in N (1..1024) is timed
    const char* slash = strchr(kernel_name, '/');
    const size_t len = slash ? (size_t)(slash - kernel_name) : strlen(kernel_name);
    if (len == 0 || len >= sizeof(plan->timer_name)) return LCP_ERR_ARG;
    if (slash) {
      char* end = nullptr;
      const long every = strtol(slash + 1, &end, 10);
      if (!end || *end || every < 1 || every > 1024) return LCP_ERR_ARG;
      plan->timer_every = (uint64_t)every;
    }
    memcpy(plan->timer_name, kernel_name, len);
    plan->timer_name[len] = 0;
  }
  plan->timer_ms = 0;
  plan->timer_launches = 0;
  plan->timer_seen = 0;
  plan->timer_bytes = 0;
  return LCP_OK;
}

lcp_status lcp_kernel_timer_read(lcp_plan_t plan, double* total_ms, uint64_t* launches,
                                 uint64_t* bytes) {
  if (!plan) return LCP_ERR_ARG;
  timer_collect(plan);
  if (total_ms) *total_ms = plan->timer_ms;
  if (launches) *launches = plan->timer_launches;
  if (bytes) *bytes = plan->timer_bytes;
  return LCP_OK;
}

}  // extern "C"


// ================================================================== served form: merged launches
// A server merges the temporal requests of different streams into one set of
// launches on a batch plan (serve_batch scratch for up to RB frames).  The
// records and stream states are exactly those of each stream's own calls.
namespace lcp {

lcp_status serve_batch_create(int F, int chunk_log2, int frames, uint64_t particles, int device,
                              lcp_plan_s** out) {
  lcp_params p{};
  p.eb_mode = LCP_EB_ABS;
  p.eb = 1.0;
  p.n_fields = F;
  p.chunk_log2 = chunk_log2;
  p.max_particles = particles;
  p.max_batch_particles = particles;
  p.max_batch_frames = frames;
  p.device = device;
  lcp_plan_s* P = nullptr;
  lcp_status st = plan_setup(&p, nullptr, 0, &P);
  if (st) return st;
  P->serve_batch = true;
  st = alloc_plan(P);
  if (st) {
    free_plan(P);
    return st;
  }
  *out = P;
  return LCP_OK;
}

size_t serve_batch_bytes(lcp_plan_s* B) { return B->scratch_bytes; }
int serve_batch_fields(lcp_plan_s* B) { return B->F; }
int serve_batch_frames(lcp_plan_s* B) { return B->RB; }
uint64_t serve_batch_particles(lcp_plan_s* B) { return B->NB; }
int plan_fields(lcp_plan_s* P) { return P->F; }
int plan_chunk_log2(lcp_plan_s* P) { return P->chunk_log2; }
bool plan_decoding_t(lcp_plan_s* P) { return P->p.multi_frame && P->dec_last_t; }
bool plan_multi_frame(lcp_plan_s* P) { return P->p.multi_frame != 0; }
int plan_batch_size(lcp_plan_s* P) { return P->p.batch_size; }
uint64_t plan_max_particles(lcp_plan_s* P) { return P->N; }

// Whether the stream's next compress request can join a merged launch: its
// frame will be coded by LCP-T (LCP-FSM in its T state, or forced T) against a
// resident reference of the same size, so that the merged launch decides it
// (kept if no larger than the last LCP-S record) as the stream's own call would.
bool serve_t_eligible(lcp_plan_s* P, const lcp_frame_in& fr) {
  if (!P->p.multi_frame || fr.n == 0 || fr.n > P->N) return false;
  if (fr.method == LCP_METHOD_S || fr.method < 0 || fr.method > 2) return false;
  if (fr.method == LCP_METHOD_AUTO && (P->fsm_state != kFsmT || !P->have_last_s)) return false;
  for (int f = 0; f < P->F; f++)
    if (!fr.fields[f]) return false;
  return reference_for(P, fr.n) != nullptr && free_q(P, -1) >= 0;
}

lcp_status serve_t_compress(lcp_plan_s* B, int K, lcp_plan_s* const* plans,
                            const lcp_frame_in* frames, void* const* outs, const uint64_t* caps,
                            bool* done, uint64_t* sizes, hipStream_t s) {
  const int F = B->F;
  if (K < 1 || K > B->RB) return LCP_ERR_ARG;
  TimerScope ts(B);
  std::vector<RefState> refs(K);
  std::vector<int> qsel(K);
  uint64_t off = 0, bytes = 0;
  uint32_t blocks = 0;
  for (int i = 0; i < K; i++) {
    lcp_plan_s* P = plans[i];
    const lcp_frame_in& fr = frames[i];
    done[i] = false;
    const RefState* ref = reference_for(P, fr.n);
    if (P->F != F || P->chunk_log2 != B->chunk_log2 || !ref) return LCP_ERR_ARG;
    refs[i] = *ref;
    qsel[i] = free_q(P, -1);
    TFrameDev& t = B->tfr_host[i];
    memset(&t, 0, sizeof(t));
    for (int f = 0; f < F; f++) t.x[f] = fr.fields[f];
    t.perm = P->ppool[ref->perm];
    t.q_ref = P->qpool[ref->q];
    t.q_new = P->qpool[qsel[i]];
    t.v8 = B->v_byte + (uint64_t)F * off;
    t.esc = B->v_slot + (uint64_t)F * off;
    t.err = reinterpret_cast<uint32_t*>(B->sret_dev + i);
    t.n = fr.n;
    // the vector path stores four residual bytes and four codes at a time
    auto a16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
    t.vec = fr.n % 4 == 0 && ((uintptr_t)t.v8 & 3) == 0 && a16(t.q_ref) && a16(t.q_new) &&
            a16(t.perm);
    t.g = t_grid(*ref, F);
    B->spre_host[i] = blocks;
    blocks += t_multi_blocks(fr.n, t.vec);
    off += fr.n;
    bytes += fr.n * (4 + 12ull * F);
  }
  B->spre_host[K] = blocks;
  if (off > B->NB) return LCP_ERR_ARG;
  lcp_status st = upload(B->tfr_host, B->tfr_dev, sizeof(TFrameDev) * K, s);
  if (!st) st = upload(B->spre_host, B->spre_dev, sizeof(uint32_t) * (K + 1), s);
  if (st) return st;
  unsigned long long* offs = B->sret_dev + K;
  uint32_t* launch_err = reinterpret_cast<uint32_t*>(B->sret_dev + 2 * K + 1);
  launch_fill_u32(reinterpret_cast<uint32_t*>(B->sret_dev), 2 * (2 * (uint64_t)K + 2), 0u, s);
  const bool fused = B->fuse_skip == 0 && B->chunk_log2 >= 6 && B->chunk_log2 <= 10;
  if (B->fuse_skip > 0) B->fuse_skip = B->fuse_skip > K ? B->fuse_skip - K : 0;
  launch_t_resid_multi(B->tfr_dev, B->spre_dev, blocks, K, F, B->hist_part, B->hist_max,
                       kServeCopies, fused ? B->work : nullptr, bytes, s);
  EncBuild EB;
  EB.R = K;
  EB.fused = fused;
  off = 0;
  for (int i = 0; i < K; i++) {
    const uint64_t n = frames[i].n;
    EncRec& rc = B->erec_host[i];
    memset(&rc, 0, sizeof(rc));
    rc.h = make_hdr(1, F, 0, B->chunk_log2, F, n, plans[i]->seq, refs[i].seq, refs[i].grid,
                    refs[i].scale);
    rc.a0 = (uint32_t)EB.NA;
    for (int f = 0; f < F; f++) {
      const uint64_t a = (uint64_t)i * F + f;
      if ((st = enc_add(B, EB, ArrIn{B->v_byte + (uint64_t)F * off + (uint64_t)f * n, 0, nullptr, n,
                                     B->v_slot + (uint64_t)F * off + (uint64_t)f * n},
                        n, i, (int)(a * kServeCopies), kServeCopies)))
        return st;
    }
    off += n;
  }
  if ((st = enc_launch(B, EB, B->rec_tmp, B->rec_tmp_cap, true, s, launch_err, offs, nullptr,
                       reinterpret_cast<uint32_t*>(B->sret_dev), 2)))
    return st;
  for (int i = 0; i < K; i++) {
    B->sdst_host[2 * i] = (uint64_t)(uintptr_t)outs[i];
    B->sdst_host[2 * i + 1] = caps[i];
  }
  if ((st = upload(B->sdst_host, B->sdst_dev, sizeof(uint64_t) * 2 * K, s))) return st;
  launch_scatter_records(offs, B->rec_tmp, B->sdst_dev, K, s);
  HIP_OK(hipMemcpyAsync(B->sret_host, B->sret_dev, 8 * (2 * (size_t)K + 2), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (g_timer_plan == B) timer_collect(B);
  const uint32_t lerr = (uint32_t)(B->sret_host[2 * K + 1] & 0xFFFFFFFFull);
  if (lerr & kErrCorrupt) return LCP_ERR_DEVICE;
  for (int i = 0; i < K; i++)
    if ((uint32_t)(B->sret_host[i] & 0xFFFFFFFFull) & kErrRebuild) {
      fused_fallback(B, s);
      break;
    }
  for (int i = 0; i < K; i++) {
    lcp_plan_s* P = plans[i];
    const uint32_t flags = (uint32_t)(B->sret_host[i] & 0xFFFFFFFFull);
    const uint64_t size = B->sret_host[K + i + 1] - B->sret_host[K + i];
    if (flags || (lerr & kErrCapacity) || size > caps[i]) continue;
    if (frames[i].method == LCP_METHOD_AUTO && size > P->last_s) continue;
    // committed as the stream's own call commits a kept temporal frame
    if (frames[i].method == LCP_METHOD_AUTO) fsm_update(P, LCP_DECIDE_T, true, true);
    RefState r = refs[i];
    r.seq = P->seq;
    r.q = qsel[i];
    P->prev = r;
    P->n_since_anchor++;
    P->t_since_anchor++;
    P->seq++;
    sizes[i] = size;
    done[i] = true;
  }
  return LCP_OK;
}

lcp_status serve_t_decompress(lcp_plan_s* B, int K, lcp_plan_s* const* plans,
                              const lcp_blob* blobs, const lcp_frame_out* dsts, bool* done,
                              uint64_t* n_out, hipStream_t s) {
  const int F = B->F;
  if (K < 1 || K > B->RB) return LCP_ERR_ARG;
  TimerScope ts(B);
  for (int i = 0; i < K; i++) {
    done[i] = false;
    if (!blobs[i].data || ((uintptr_t)blobs[i].data & 3)) return LCP_ERR_ARG;
    B->blobtab_host[2 * i] = (uint64_t)(uintptr_t)blobs[i].data;
    B->blobtab_host[2 * i + 1] = blobs[i].size;
  }
  lcp_status st = upload(B->blobtab_host, B->blobtab_dev, 16ull * K, s);
  if (st) return st;
  launch_gather_headers(B->blobtab_dev, K, kHdrStage, B->hdr_dev, s);
  HIP_OK(hipMemcpyAsync(B->hdr_host, B->hdr_dev, (size_t)kHdrStage * K, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  std::vector<ParsedHdr> H(K);
  std::vector<int> dq(K, -1), take;
  uint64_t off = 0, bytes = 0;
  uint32_t blocks = 0;
  int A = 0;
  for (int i = 0; i < K; i++) {
    lcp_plan_s* P = plans[i];
    ParsedHdr& h = H[i];
    if (parse_header(B->hdr_host + (size_t)kHdrStage * i, blobs[i].size, &h)) continue;
    if (h.mode != 1 || h.F != F || h.cl != B->chunk_log2 || P->F != F || h.n > P->N ||
        h.dtype != P->p.dtype || h.n > dsts[i].capacity || off + h.n > B->NB)
      continue;
    bool fields = true;
    for (int f = 0; f < F; f++) fields = fields && dsts[i].fields[f];
    if (!fields) continue;
    int refq = -1;
    if (P->dprev.valid && P->dprev.seq == h.ref_seq && P->dprev.n == h.n) refq = P->dprev.q;
    else if (P->danchor.valid && P->danchor.seq == h.ref_seq && P->danchor.n == h.n) refq = P->danchor.q;
    if (refq < 0) continue;
    for (int q = 0; q < 3; q++)
      if (!(P->dprev.valid && P->dprev.q == q) && !(P->danchor.valid && P->danchor.q == q)) {
        dq[i] = q;
        break;
      }
    if (dq[i] < 0) continue;
    const uint8_t* rec = reinterpret_cast<const uint8_t*>(blobs[i].data);
    for (int f = 0; f < F; f++) {
      DecArr& d = B->arrtab_host[A++];
      d.data = rec + h.aoff[f];
      d.nbytes = h.anb[f];
      d.n = h.an[f];
      d.coder = h.coder[f];
      d.param = h.param[f];
      d.used = h.used[f];
      d.out = B->dres8 + (uint64_t)F * off + (uint64_t)f * h.n;
      d.esc = reinterpret_cast<int32_t*>(dsts[i].fields[f]);
      d.mode = 4;
      d.limit = 1ull << 25;
      bytes += h.anb[f] + 4 * h.an[f];
    }
    TReconDev& t = B->trc_host[take.size()];
    memset(&t, 0, sizeof(t));
    t.q_ref = P->dqpool[refq];
    t.q_new = P->dqpool[dq[i]];
    t.scale = h.scale;
    t.dtype = h.dtype;
    t.r8 = reinterpret_cast<const int8_t*>(B->dres8 + (uint64_t)F * off);
    for (int f = 0; f < F; f++) {
      t.out[f] = dsts[i].fields[f];
      t.m[f] = h.m[f];
      t.eb_q[f] = h.eb_q[f];
    }
    t.n = h.n;
    B->spre_host[take.size()] = blocks;
    blocks += (uint32_t)((h.n + kSeg1k - 1) / kSeg1k);
    off += h.n;
    take.push_back(i);
  }
  if (take.empty()) return LCP_OK;
  const int KT = (int)take.size();
  B->spre_host[KT] = blocks;
  clear_err(B, s);
  if ((st = decode_arrays(B, 0, A, B->chunk_log2, bytes, s))) return st;
  if ((st = upload(B->trc_host, B->trc_dev, sizeof(TReconDev) * KT, s))) return st;
  if ((st = upload(B->spre_host, B->spre_dev, sizeof(uint32_t) * (KT + 1), s))) return st;
  launch_t_recon_multi(B->trc_dev, B->spre_dev, blocks, KT, F, B->err, off * 16ull * F, s);
  if ((st = read_ret(B, 1, s))) return st;
  if (g_timer_plan == B) timer_collect(B);
  if (host_err(B) & kErrCorrupt) return LCP_OK;  // each goes its own way, which reports it
  for (int j = 0; j < KT; j++) {
    const int i = take[j];
    lcp_plan_s* P = plans[i];
    RefState r;
    r.valid = true;
    r.seq = H[i].seq;
    r.n = H[i].n;
    r.q = dq[i];
    P->dprev = r;
    P->dec_last_t = true;
    n_out[i] = H[i].n;
    done[i] = true;
  }
  return LCP_OK;
}

}  // namespace lcp

// ================================================================== no-allocation entry point
// lcp_compress_static runs the single-frame LCP-S path of lcp_compress on
// scratch that already exists: one file-scope device array per GPU (reserved
// with the code object, held until the process ends) and a static host block
// for the plan's small tables.  In host code `scratch` names a host-side
// stand-in of the array, never its device memory: the device address comes
// from hipGetSymbolAddress on the first call on each device, and only that
// address is handed to kernels and fills.
namespace {

constexpr size_t kStaticScratchBytes = 64ull << 20;
constexpr size_t kStaticHostBytes = 256ull << 10;
constexpr int kStaticDevices = 16;

static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

struct StaticSlot {
  std::mutex mu;           // calls on one device run one at a time
  void* dev = nullptr;     // this device's address of `scratch`
  bool looked_up = false;
  lcp_plan_s plan;         // sizes and table pointers of the current call
  alignas(256) uint8_t host[kStaticHostBytes];
};
StaticSlot g_static[kStaticDevices];

}  // namespace

extern "C" lcp_status lcp_compress_static(const lcp_params* params, uint64_t n_frames,
                                          const lcp_frame_in* frames, void* out, uint64_t out_cap,
                                          uint64_t* out_offsets, uint32_t* const* perms,
                                          hipStream_t stream) {
  if (!params || (!frames && n_frames) || !out_offsets || (!out && n_frames) || ((uintptr_t)out & 3))
    return LCP_ERR_ARG;
  if (params->multi_frame || params->block_log2 < 0) return LCP_ERR_ARG;
  lcp_status st = plan_check(*params, nullptr, 0);
  if (st) return st;
  if (params->device < 0 || params->device >= kStaticDevices) return LCP_ERR_ARG;
  StaticSlot& S = g_static[params->device];
  std::lock_guard<std::mutex> lk(S.mu);
  lcp_plan_s* P = &S.plan;
  lcp_params q = *params;
  if (q.max_batch_frames == 0) q.max_batch_frames = 1;  // one frame per launch set
  plan_fill(P, q);
  P->compress_only = true;
  P->seq = 0;
  P->timer_name[0] = 0;
  Layout D, H;
  layout_scratch(P, D, H);
  // refused before any HIP call
  if (D.total > kStaticScratchBytes || H.total > kStaticHostBytes) return LCP_ERR_BUDGET;
  if (hipSetDevice(params->device) != hipSuccess) return LCP_ERR_DEVICE;
  if (!S.looked_up) {
    // the device copy of the array on this (current) device
    hipError_t e = hipGetSymbolAddress(&S.dev, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !S.dev) return hip_fail(e, "hipGetSymbolAddress(scratch)", __LINE__);
    S.looked_up = true;
  }
  // binding clears what must start at zero (histogram copies, error word)
  bind_scratch(P, S.dev, S.host, stream);
  P->host_pinned = false;  // a static host block: tables go up as kernel arguments
  TimerScope ts(P);
  st = compress_independent(P, n_frames, frames, reinterpret_cast<uint8_t*>(out), out_cap,
                            out_offsets, nullptr, perms, stream);
  P->bound = false;
  return st;
}
