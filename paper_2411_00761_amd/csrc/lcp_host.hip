// lcp_host.hip -- the C ABI declared in include/lcp.h: plans, the LCP-S and
// LCP-T pipelines, LCP-FSM (Sec. 7.2) with Alg. 1's reference/anchor rule
// (Sec. 7.3), block-size search (Sec. 7.4.1), decode, and the kernel timer.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/lcp.h"
#include "lcp_internal.h"

using namespace lcp;

namespace {

// ------------------------------------------------------------------ grids
struct HostGrid {
  float m, eb_q;
  double inv, eb;
  int E;
};

// Eq. 5 with a float32 output: the exact bin centre is within eb_q of x and the
// float32 rounding of the centre adds at most half an ulp of the top binade
// 2^E, where |x| + 2 eb < 2^E; eb_q = eb - 2^(E-24), rounded down to float,
// keeps every reconstruction within eb.
lcp_status make_grid(float lo, float hi, double eb, HostGrid* g) {
  if (!isfinite(lo) || !isfinite(hi) || !(eb > 0) || !isfinite(eb)) return LCP_ERR_ARG;
  double M = fmax(fabs((double)lo), fabs((double)hi)) + 2.0 * eb;
  int E;
  frexp(M, &E);
  if (E < -100) E = -100;
  double delta = ldexp(1.0, E - 24);
  if (!(eb >= 2.0 * delta)) return LCP_ERR_EB_TOO_SMALL;
  double t = eb - delta;
  float e = (float)t;
  if ((double)e > t) e = nextafterf(e, 0.0f);
  if (!(e > 0.0f)) return LCP_ERR_EB_TOO_SMALL;
  g->m = lo;
  g->eb_q = e;
  g->inv = 1.0 / (2.0 * (double)e);
  g->eb = eb;
  g->E = E;
  return LCP_OK;
}

int64_t host_quant(float x, const HostGrid& g) {
  return (int64_t)floor(((double)x - (double)g.m) * g.inv);
}

// ------------------------------------------------------------------ device buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct RefState {
  bool valid = false;
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
  uint64_t N = 0;           // max particles
  uint64_t max_chunks = 0;  // per array
  std::vector<void*> allocs;
  size_t allocated = 0;

  // scratch
  uint64_t *keys0, *keys1, *ids, *v_id, *v_cnt;
  uint32_t *vals0, *vals1, *hist, *flags, *starts, *v_slot, *chunk_words, *lut, *corner;
  uint64_t* scan_tmp;
  size_t scan_tmp_n;
  ArrWork* work;
  uint32_t* small;  // [0] B, [1] err, [2..2+2F) extent keys
  unsigned long long* size_dev;
  uint8_t* rec_tmp;  // second record (temporal candidate)
  uint64_t rec_tmp_cap;
  uint32_t* host_small;  // pinned mirror of `small`
  unsigned long long* host_size;
  uint32_t* ext_part;    // extent partials
  uint32_t* hist_part;   // per-workgroup histograms
  unsigned long long* hist_max;
  uint8_t* huff_lens;    // candidate code lengths per (array, halving count)
  uint32_t* huff_maxd;
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
  bool have_eb = false;
  double eb_f[kMaxF];
  uint64_t seq = 0;
  // LCP-FSM
  bool fsm_t = false;
  int interval = 1, countdown = 0;
  uint64_t last_s = 0;
  bool have_last_s = false;

  // kernel timer
  char timer_name[64] = {0};
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  std::vector<uint64_t> ev_bytes;
  double timer_ms = 0;
  uint64_t timer_launches = 0, timer_bytes = 0;
};

namespace {

lcp_plan_s* g_timer_plan = nullptr;  // plan whose call is running (one at a time)

struct TimerScope {
  explicit TimerScope(lcp_plan_s* p) { g_timer_plan = p; }
  ~TimerScope() { g_timer_plan = nullptr; }
};

#define HIP_OK(x)                          \
  do {                                     \
    if ((x) != hipSuccess) return LCP_ERR_DEVICE; \
  } while (0)

template <typename T>
lcp_status dalloc(lcp_plan_s* P, T** out, size_t elems) {
  size_t bytes = elems * sizeof(T);
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~(size_t)255;
  if (P->p.hbm_budget_bytes && P->allocated + bytes > P->p.hbm_budget_bytes) return LCP_ERR_BUDGET;
  void* ptr = nullptr;
  if (hipMalloc(&ptr, bytes) != hipSuccess) return LCP_ERR_DEVICE;
  P->allocs.push_back(ptr);
  P->allocated += bytes;
  *out = reinterpret_cast<T*>(ptr);
  return LCP_OK;
}

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
  b += 3 * 4 * words(n * 25);
  if (F > 3) b += (uint64_t)(F - 3) * 4 * words(n * 25);
  return b;
}

GridDev to_dev(const HostGrid* g, int F) {
  GridDev d;
  memset(&d, 0, sizeof(d));
  for (int f = 0; f < F; f++) {
    d.m[f] = g[f].m;
    d.eb_q[f] = g[f].eb_q;
    d.inv[f] = g[f].inv;
  }
  return d;
}

// ------------------------------------------------------------------ extent
lcp_status extent(lcp_plan_s* P, const float* const* x, uint64_t n, float* lo, float* hi,
                  hipStream_t s) {
  FieldPtrs fp;
  memset(&fp, 0, sizeof(fp));
  for (int f = 0; f < P->F; f++) fp.p[f] = x[f];
  launch_fill_u32(P->small + 1, 1, 0u, s);
  launch_extent(fp, P->F, n, P->small + 2, P->ext_part, P->small + 1, s);
  HIP_OK(hipMemcpyAsync(P->host_small, P->small, sizeof(uint32_t) * (2 + 2 * P->F),
                        hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (P->host_small[1] & kErrNonFinite) return LCP_ERR_ARG;
  for (int f = 0; f < P->F; f++) {
    float a = key_float(P->host_small[2 + 2 * f]);
    float b = key_float(P->host_small[3 + 2 * f]);
    lo[f] = a == 0.0f ? 0.0f : a;  // one zero: +0
    hi[f] = b == 0.0f ? 0.0f : b;
  }
  return LCP_OK;
}

lcp_status field_eb(const lcp_params& p, int F, const float* lo, const float* hi, double* eb) {
  if (!(p.eb > 0) || !isfinite(p.eb)) return LCP_ERR_ARG;
  if (p.eb_mode == LCP_EB_ABS) {
    for (int f = 0; f < F; f++) eb[f] = p.eb;
  } else if (p.eb_mode == LCP_EB_REL_GLOBAL) {
    float a = lo[0], b = hi[0];
    for (int f = 1; f < F; f++) {
      a = lo[f] < a ? lo[f] : a;
      b = hi[f] > b ? hi[f] : b;
    }
    double r = (double)b - (double)a;
    for (int f = 0; f < F; f++) eb[f] = p.eb * r;
  } else if (p.eb_mode == LCP_EB_REL_PER_FIELD) {
    for (int f = 0; f < F; f++) eb[f] = p.eb * ((double)hi[f] - (double)lo[f]);
  } else {
    return LCP_ERR_ARG;
  }
  for (int f = 0; f < F; f++)
    if (!(eb[f] > 0)) return LCP_ERR_EB_TOO_SMALL;
  return LCP_OK;
}

// ------------------------------------------------------------------ encode driver
lcp_status finish_record(lcp_plan_s* P, uint64_t* size, uint32_t* flags, hipStream_t s) {
  HIP_OK(hipMemcpyAsync(P->host_size, P->size_dev, sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(P->host_small + 1, P->small + 1, sizeof(uint32_t),
                        hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (g_timer_plan == P) timer_collect(P);
  *size = *P->host_size;
  if (flags) *flags = P->host_small[1];
  if (P->host_small[1] & kErrCapacity) return LCP_ERR_CAPACITY;
  return LCP_OK;
}

struct SResult {
  uint64_t size = 0;
  const uint32_t* perm = nullptr;  // device, slot -> input index
};

// LCP-S on one frame.  grids[] come from this frame's extent; hi[] its maxima.
lcp_status compress_s(lcp_plan_s* P, const float* const* x, uint64_t n, const HostGrid* g,
                      const float* hi, int k, uint64_t seq, uint8_t* out, uint64_t cap,
                      int32_t* q_slot, SResult* res, hipStream_t s) {
  const int F = P->F;
  uint32_t bn[3];
  unsigned __int128 tot = 1;
  for (int f = 0; f < F; f++) {
    int64_t qm = host_quant(hi[f], g[f]);
    if (qm >= kQLimit) return LCP_ERR_RANGE;
    if (f < 3) {
      bn[f] = (uint32_t)((qm >> k) + 1);
      tot *= bn[f];
    }
  }
  if (tot >= ((unsigned __int128)1 << 63)) return LCP_ERR_RANGE;
  const uint64_t total_blocks = (uint64_t)tot;
  int bits = bitwidth64(total_blocks - 1);

  FieldPtrs fp;
  memset(&fp, 0, sizeof(fp));
  for (int f = 0; f < F; f++) fp.p[f] = x[f];
  GridDev gd = to_dev(g, F);
  launch_quant_key(fp, n, gd, k, bn[0], bn[1], P->keys0, P->vals0, s);
  int cur = radix_sort(P->keys0, P->vals0, P->keys1, P->vals1, n, bits, P->hist,
                       reinterpret_cast<uint32_t*>(P->scan_tmp), s);
  uint64_t* keys = cur ? P->keys1 : P->keys0;
  uint32_t* perm = cur ? P->vals1 : P->vals0;
  uint32_t* B_dev = P->small;
  launch_runs(keys, n, P->flags, P->ids, P->starts, B_dev,
              reinterpret_cast<uint32_t*>(P->scan_tmp), s);
  launch_block_syms(P->ids, P->starts, B_dev, n, P->v_id, P->v_cnt, s);
  uint32_t* v_rel = P->v_slot;
  uint32_t* v_sup = P->v_slot + 3 * n;
  launch_slot_syms(fp, F, n, gd, k, perm, v_rel, v_sup, q_slot, s);

  ArrSet set;
  memset(&set, 0, sizeof(set));
  set.A = F + 2;
  set.a[0] = ArrIn{P->v_id, 1, B_dev, n};
  set.a[1] = ArrIn{P->v_cnt, 1, B_dev, n};
  for (int d = 0; d < 3; d++) set.a[2 + d] = ArrIn{v_rel + (uint64_t)d * n, 0, nullptr, n};
  for (int f = 3; f < F; f++) set.a[2 + f] = ArrIn{v_sup + (uint64_t)(f - 3) * n, 0, nullptr, n};
  RecHdr h;
  memset(&h, 0, sizeof(h));
  h.mode = 0;
  h.F = F;
  h.k = k;
  h.chunk_log2 = P->chunk_log2;
  h.A = F + 2;
  h.n = n;
  h.seq = seq;
  h.ref_seq = ~0ull;
  for (int d = 0; d < 3; d++) h.bn[d] = bn[d];
  for (int f = 0; f < F; f++) {
    h.m[f] = g[f].m;
    h.eb_q[f] = g[f].eb_q;
  }
  HIP_OK(hipMemsetAsync(P->small + 1, 0, sizeof(uint32_t), s));
  launch_encode(set, n, P->chunk_log2, P->work, P->chunk_words, P->max_chunks, P->hist_part,
                P->hist_max, P->huff_lens, P->huff_maxd, h, B_dev, out,
                cap, P->size_dev, P->small + 1, false, s);
  res->perm = perm;
  return finish_record(P, &res->size, nullptr, s);
}

// LCP-T on one frame against a resident reference.  Whether the frame fits the
// reference grid (finite values, float32 margin, code range) is checked by the
// residual kernel itself, so no extent pass is needed.
lcp_status compress_t(lcp_plan_s* P, const float* const* x, uint64_t n, const RefState& ref,
                      uint64_t seq, uint8_t* out, uint64_t cap, int32_t* q_new, uint64_t* size,
                      hipStream_t s) {
  const int F = P->F;
  FieldPtrs fp;
  memset(&fp, 0, sizeof(fp));
  for (int f = 0; f < F; f++) fp.p[f] = x[f];
  GridDev gd = to_dev(ref.grid, F);
  for (int f = 0; f < F; f++) {
    gd.eb2[f] = 2.0 * ref.grid[f].eb;
    gd.lim[f] = ldexp(1.0, ref.grid[f].E);
  }
  launch_fill_u32(P->small + 1, 1, 0u, s);
  launch_t_resid(fp, F, n, gd, P->ppool[ref.perm], P->qpool[ref.q], P->v_slot, q_new,
                 P->small + 1, P->hist_part, P->hist_max, s);
  ArrSet set;
  memset(&set, 0, sizeof(set));
  set.A = F;
  for (int f = 0; f < F; f++) set.a[f] = ArrIn{P->v_slot + (uint64_t)f * n, 0, nullptr, n};
  RecHdr h;
  memset(&h, 0, sizeof(h));
  h.mode = 1;
  h.F = F;
  h.k = 0;
  h.chunk_log2 = P->chunk_log2;
  h.A = F;
  h.n = n;
  h.seq = seq;
  h.ref_seq = ref.seq;
  for (int f = 0; f < F; f++) {
    h.m[f] = ref.grid[f].m;
    h.eb_q[f] = ref.grid[f].eb_q;
  }
  launch_encode(set, n, P->chunk_log2, P->work, P->chunk_words, P->max_chunks, P->hist_part,
                P->hist_max, P->huff_lens, P->huff_maxd, h, P->small,
                out, cap, P->size_dev, P->small + 1, true, s);
  uint32_t flags = 0;
  lcp_status st = finish_record(P, size, &flags, s);
  if (flags & kErrNonFinite) return LCP_ERR_ARG;
  if (flags & kErrRange) return LCP_ERR_RANGE;
  return st;
}

// ------------------------------------------------------------------ LCP-FSM
// S state with a test interval (S1X, S2X, ... S16X) and a countdown of frames
// coded with S untested; T state.  A frame with no reference counts as an S win.
bool first_in_batch(const lcp_plan_s* P, uint64_t seq) {
  return P->p.batch_size == 0 ? seq == 0 : seq % (uint64_t)P->p.batch_size == 0;
}

const RefState* reference_for(const lcp_plan_s* P, uint64_t n) {
  if (!P->p.multi_frame) return nullptr;
  const RefState* r = first_in_batch(P, P->seq) ? &P->anchor : &P->prev;
  if (!r->valid || r->n != n) return nullptr;
  return r;
}

int fsm_decide(const lcp_plan_s* P, bool have_ref) {
  if (!P->p.multi_frame || !have_ref) return LCP_DECIDE_S;
  if (P->fsm_t) return LCP_DECIDE_T;
  return P->countdown > 0 ? LCP_DECIDE_S : LCP_DECIDE_COMPARE;
}

void fsm_s_win(lcp_plan_s* P) {
  P->interval = P->interval * 2 > 16 ? 16 : P->interval * 2;
  P->countdown = P->interval - 1;
}

void fsm_update(lcp_plan_s* P, int decision, bool have_ref, bool chose_t) {
  if (!have_ref) {
    if (P->fsm_t) {
      P->fsm_t = false;
      P->interval = 1;
    }
    fsm_s_win(P);
  } else if (decision == LCP_DECIDE_S) {
    P->countdown--;
  } else if (decision == LCP_DECIDE_COMPARE) {
    if (chose_t) P->fsm_t = true;
    else fsm_s_win(P);
  } else if (!chose_t) {
    P->fsm_t = false;
    P->interval = 1;
    P->countdown = 0;
  }
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
  if (decision != LCP_DECIDE_S) {
    qt_i = free_q(P, -1);
    st = compress_t(P, fr.fields, n, *ref, P->seq, P->rec_tmp, P->rec_tmp_cap, P->qpool[qt_i],
                    &size_t_, s);
    if (st == LCP_OK) have_t = true;
    else if (st == LCP_ERR_RANGE && fr.method != LCP_METHOD_T) st = LCP_OK;  // T infeasible
    else return st;
  }
  bool need_s = decision != LCP_DECIDE_T || !have_t ||
                (fr.method == LCP_METHOD_AUTO && (!P->have_last_s || size_t_ > P->last_s));
  SResult sr;
  double eb_f[kMaxF];
  if (need_s) {
    float lo[kMaxF], hi[kMaxF];
    if ((st = extent(P, fr.fields, n, lo, hi, s))) return st;
    if (multi && P->have_eb) memcpy(eb_f, P->eb_f, sizeof(eb_f));
    else if ((st = field_eb(P->p, F, lo, hi, eb_f))) return st;
    HostGrid sg[kMaxF];
    for (int f = 0; f < F; f++)
      if ((st = make_grid(lo[f], hi[f], eb_f[f], &sg[f]))) return st;
    if (multi) {
      qs_i = free_q(P, qt_i);
      ps_i = free_perm(P);
    }
    st = compress_s(P, fr.fields, n, sg, hi, P->k, P->seq, out, cap,
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
  if (chose_t) HIP_OK(hipMemcpyAsync(out, P->rec_tmp, size_t_, hipMemcpyDeviceToDevice, s));
  *size = chosen;
  if (used) *used = chose_t ? LCP_METHOD_T : LCP_METHOD_S;
  if (have_s) {
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
  P->seq++;
  return LCP_OK;
}

// ------------------------------------------------------------------ decode
struct ParsedHdr {
  int mode, F, k, cl, A;
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
  if (h->mode > 1 || h->F < 3 || h->F > kMaxF || h->k > 16 || h->cl < 5 || h->cl > 16)
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
  uint32_t* hp = P->prefix_host + 2 * base;
  uint32_t* fp = hp + A;
  uint32_t hb = 0, fb = 0;
  for (int a = 0; a < A; a++) {
    hp[a] = hb;
    fp[a] = fb;
    hb += decode_blocks(P->arrtab_host[base + a], cl, true);
    fb += decode_blocks(P->arrtab_host[base + a], cl, false);
  }
  HIP_OK(hipMemcpyAsync(P->arrtab_dev + base, P->arrtab_host + base, sizeof(DecArr) * A,
                        hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(P->prefix_dev + 2 * base, hp, sizeof(uint32_t) * 2 * A,
                        hipMemcpyHostToDevice, s));
  launch_decode(P->arrtab_dev + base, A, P->prefix_dev + 2 * base, hb,
                P->prefix_dev + 2 * base + A, fb, cl, bytes, P->lut + ((uint64_t)base << kMaxLen),
                P->small + 1, s);
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
  HIP_OK(hipMemcpyAsync(P->blobtab_dev, P->blobtab_host, 16 * nf, hipMemcpyHostToDevice, s));
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
    if (h.F != F || h.cl > 12 || h.n > P->N) return LCP_ERR_ARG;
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
  // ---- entropy decoding of every array that lands in the output buffers
  launch_fill_u32(P->small + 1, 1, 0u, s);
  int A = 0;
  uint64_t bytes = 0;
  int cl = nf ? H[0].cl : 10;
  bool same_cl = true;
  for (uint64_t j = 0; j < nf; j++) same_cl &= H[j].cl == cl;
  for (uint64_t j = 0; j < nf && same_cl; j++) {
    const ParsedHdr& h = H[j];
    const uint8_t* rec = reinterpret_cast<const uint8_t*>(blobs[j].data);
    for (int a = (h.mode == 0 ? 2 : 0); a < h.A; a++) {
      const int f = h.mode == 0 ? a - 2 : a;
      DecArr& d = P->arrtab_host[A++];
      d.data = rec + h.aoff[a];
      d.nbytes = h.anb[a];
      d.n = h.an[a];
      d.coder = h.coder[a];
      d.param = h.param[a];
      d.used = h.used[a];
      d.out = outs[j].fields[f];
      d.mode = h.mode == 0 ? 2 : 3;
      d.limit = h.mode == 0 ? (f < 3 ? (1ull << h.k) : (uint64_t)kQLimit) : (1ull << 25);
      bytes += h.anb[a] + 4 * h.an[a];
    }
  }
  if (same_cl) {
    lcp_status st = decode_arrays(P, 0, A, cl, bytes, s);
    if (st) return st;
  }
  // ---- reconstruction in stream order
  int extra = A;  // staging slots for the id / count arrays of spatial frames
  for (uint64_t j = 0; j < nf; j++) {
    const ParsedHdr& h = H[j];
    const uint64_t n = h.n;
    const uint8_t* rec = reinterpret_cast<const uint8_t*>(blobs[j].data);
    GridDev gd;
    memset(&gd, 0, sizeof(gd));
    for (int f = 0; f < F; f++) {
      gd.m[f] = h.m[f];
      gd.eb_q[f] = h.eb_q[f];
    }
    OutPtrs op;
    memset(&op, 0, sizeof(op));
    for (int f = 0; f < F; f++) op.p[f] = outs[j].fields[f];
    int32_t* q_slot = multi ? P->dqpool[dq[j]] : nullptr;
    // staging slots: at most kMaxF + 2 per frame beyond the batched arrays
    if (extra + kMaxF + 2 > kMaxBatchArrays + 2 * kMaxBatchFrames) return LCP_ERR_ARG;
    if (!same_cl) {  // mixed chunk sizes: decode this frame's arrays on their own
      int a0 = extra;
      for (int a = (h.mode == 0 ? 2 : 0); a < h.A; a++) {
        const int f = h.mode == 0 ? a - 2 : a;
        DecArr& d = P->arrtab_host[extra++];
        d.data = rec + h.aoff[a];
        d.nbytes = h.anb[a];
        d.n = h.an[a];
        d.coder = h.coder[a];
        d.param = h.param[a];
        d.used = h.used[a];
        d.out = outs[j].fields[f];
        d.mode = h.mode == 0 ? 2 : 3;
        d.limit = h.mode == 0 ? (f < 3 ? (1ull << h.k) : (uint64_t)kQLimit) : (1ull << 25);
      }
      lcp_status st = decode_arrays(P, a0, extra - a0, h.cl, 0, s);
      if (st) return st;
    }
    if (h.mode == 0) {
      const uint64_t B = h.B;
      unsigned __int128 tot = (unsigned __int128)h.bn[0] * h.bn[1] * h.bn[2];
      if (h.bn[0] == 0 || h.bn[1] == 0 || h.bn[2] == 0 || tot >= ((unsigned __int128)1 << 63))
        return LCP_ERR_CORRUPT;
      const uint64_t total_blocks = (uint64_t)tot;
      for (int a = 0; a < 2; a++) {
        DecArr& d = P->arrtab_host[extra + a];
        d.data = rec + h.aoff[a];
        d.nbytes = h.anb[a];
        d.n = h.an[a];
        d.coder = h.coder[a];
        d.param = h.param[a];
        d.used = h.used[a];
        d.out = a == 0 ? (void*)P->v_id : (void*)P->v_cnt;
        d.mode = a;  // ids raw, counts unzigzagged
        d.limit = a == 0 ? total_blocks : ~0ull;
      }
      lcp_status st = decode_arrays(P, extra, 2, h.cl, 0, s);
      if (st) return st;
      extra += 2;
      uint64_t* ids = P->v_id;
      uint64_t* cnt = P->v_cnt;
      uint64_t* cum = P->ids;
      scan_device<uint64_t>(ids, B, nullptr, false, P->scan_tmp, s);
      scan_device<uint64_t>(cnt, B, nullptr, false, P->scan_tmp, s);
      HIP_OK(hipMemcpyAsync(cum, cnt, B * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
      scan_device<uint64_t>(cum, B, nullptr, false, P->scan_tmp, s);
      launch_fill_u32(P->flags, n, 0u, s);
      launch_s_blocks(ids, cnt, cum, B, n, total_blocks, h.bn, h.k, P->corner, P->flags,
                      P->small + 1, s);
      uint32_t* tmp32 = reinterpret_cast<uint32_t*>(P->scan_tmp);
      scan_device<uint32_t>(P->flags, n, nullptr, false, tmp32, s);
      for (int d = 0; d < 3; d++)
        scan_device<uint32_t>(reinterpret_cast<uint32_t*>(outs[j].fields[d]), n, nullptr, false,
                              tmp32, s);
      launch_s_recon(P->flags, P->corner, B, F, n, h.k, gd, op, q_slot, P->small + 1, s);
    } else {
      launch_t_recon(P->dqpool[refq[j]], F, n, gd, op, q_slot, P->small + 1, s);
    }
  }
  HIP_OK(hipMemcpyAsync(P->host_small + 1, P->small + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (g_timer_plan == P) timer_collect(P);
  if (P->host_small[1] & kErrCorrupt) return LCP_ERR_CORRUPT;
  if (multi) {
    P->dprev = sp;
    P->danchor = sa;
  }
  return LCP_OK;
}

lcp_status alloc_plan(lcp_plan_s* P) {
  const uint64_t N = P->N;
  const int F = P->F;
  const uint64_t ntiles = (N + 4095) / 4096;
  lcp_status st;
#define A_(ptr, cnt) \
  if ((st = dalloc(P, &(ptr), (cnt)))) return st
  A_(P->keys0, N);
  A_(P->keys1, N);
  A_(P->ids, N);
  A_(P->v_id, N);
  A_(P->v_cnt, N);
  A_(P->vals0, N);
  A_(P->vals1, N);
  A_(P->hist, 256 * ntiles);
  A_(P->flags, N);
  A_(P->starts, N);
  A_(P->v_slot, (uint64_t)F * N);
  P->max_chunks = (N + (1ull << P->chunk_log2) - 1) >> P->chunk_log2;
  A_(P->chunk_words, (uint64_t)kMaxArrays * P->max_chunks + 1);
  A_(P->lut, (uint64_t)(kMaxBatchArrays + 2 * kMaxBatchFrames) << kMaxLen);
  A_(P->ext_part, 2 * kMaxF * 256);
  A_(P->hist_part, (uint64_t)kMaxArrays * kHistCopies * kAlphabet);
  A_(P->hist_max, (uint64_t)kMaxArrays * kHistCopies);
  A_(P->huff_lens, (uint64_t)kMaxArrays * kHuffCandidates * kAlphabet);
  A_(P->huff_maxd, (uint64_t)kMaxArrays * kHuffCandidates);
  A_(P->hdr_dev, (uint64_t)kHdrStage * kMaxBatchFrames);
  A_(P->blobtab_dev, 2 * kMaxBatchFrames);
  A_(P->arrtab_dev, kMaxBatchArrays + 2 * kMaxBatchFrames);
  A_(P->prefix_dev, 2 * (kMaxBatchArrays + 2 * kMaxBatchFrames));
  A_(P->corner, 3 * N);
  uint64_t sn = N > 256 * ntiles ? N : 256 * ntiles;
  P->scan_tmp_n = scan_tmp_elems(sn);
  A_(P->scan_tmp, P->scan_tmp_n);
  A_(P->work, kMaxArrays);
  A_(P->small, 64);
  A_(P->size_dev, 1);
  P->rec_tmp_cap = bound_bytes(F, N);
  A_(P->rec_tmp, P->rec_tmp_cap);
  if (P->p.multi_frame) {
    for (int i = 0; i < 4; i++) A_(P->qpool[i], (uint64_t)F * N);
    for (int i = 0; i < 3; i++) A_(P->ppool[i], N);
    for (int i = 0; i < 3; i++) A_(P->dqpool[i], (uint64_t)F * N);
  }
#undef A_
  if (hipMemset(P->hist_part, 0, sizeof(uint32_t) * kMaxArrays * kHistCopies * kAlphabet) != hipSuccess ||
      hipMemset(P->hist_max, 0, sizeof(unsigned long long) * kMaxArrays * kHistCopies) != hipSuccess)
    return LCP_ERR_DEVICE;
  if (hipHostMalloc((void**)&P->host_small, 64 * sizeof(uint32_t), 0) != hipSuccess)
    return LCP_ERR_DEVICE;
  if (hipHostMalloc((void**)&P->host_size, sizeof(unsigned long long), 0) != hipSuccess)
    return LCP_ERR_DEVICE;
  if (hipHostMalloc((void**)&P->hdr_host, (size_t)kHdrStage * kMaxBatchFrames, 0) != hipSuccess ||
      hipHostMalloc((void**)&P->blobtab_host, 16 * kMaxBatchFrames, 0) != hipSuccess ||
      hipHostMalloc((void**)&P->arrtab_host, sizeof(DecArr) * (kMaxBatchArrays + 2 * kMaxBatchFrames), 0) != hipSuccess ||
      hipHostMalloc((void**)&P->prefix_host, 8 * (kMaxBatchArrays + 2 * kMaxBatchFrames), 0) != hipSuccess)
    return LCP_ERR_DEVICE;
  return LCP_OK;
}

void free_plan(lcp_plan_s* P) {
  for (void* p : P->allocs) (void)hipFree(p);
  if (P->host_small) (void)hipHostFree(P->host_small);
  if (P->host_size) (void)hipHostFree(P->host_size);
  for (void* hp : {(void*)P->hdr_host, (void*)P->blobtab_host, (void*)P->arrtab_host, (void*)P->prefix_host})
    if (hp) (void)hipHostFree(hp);
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
  float lo[kMaxF], hi[kMaxF];
  double eb[kMaxF];
  HostGrid g[kMaxF];
  if (!st) st = extent(P, xs, ns, lo, hi, s);
  if (!st) st = field_eb(P->p, F, lo, hi, eb);
  for (int f = 0; f < F && !st; f++) st = make_grid(lo[f], hi[f], eb[f], &g[f]);
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

}  // namespace

namespace lcp {
bool ktimer_on(const char* name) {
  return g_timer_plan && g_timer_plan->timer_name[0] && strcmp(g_timer_plan->timer_name, name) == 0;
}
void ktimer_begin(hipStream_t s) {
  lcp_plan_s* P = g_timer_plan;
  hipEvent_t a = timer_event(P), b = timer_event(P);
  (void)hipEventRecord(a, s);
  P->ev_pending.push_back({a, b});
  P->ev_bytes.push_back(0);
}
void ktimer_end(hipStream_t s, uint64_t bytes) {
  lcp_plan_s* P = g_timer_plan;
  (void)hipEventRecord(P->ev_pending.back().second, s);
  P->ev_bytes.back() = bytes;
}
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
  if (!params || !out) return LCP_ERR_ARG;
  *out = nullptr;
  const lcp_params& p = *params;
  int cl = p.chunk_log2 == 0 ? 10 : p.chunk_log2;
  if (p.n_fields < 3 || p.n_fields > LCP_MAX_FIELDS || cl < 5 || cl > 12 || p.batch_size < 0 ||
      p.block_log2 < -1 || p.block_log2 > 16 || p.max_particles == 0 ||
      p.max_particles > (1ull << 31) || !(p.eb > 0) || p.eb_mode < 0 || p.eb_mode > 2)
    return LCP_ERR_ARG;
  if (p.block_log2 == -1 && (!sample_fields || sample_n == 0)) return LCP_ERR_ARG;
  if (hipSetDevice(p.device) != hipSuccess) return LCP_ERR_DEVICE;
  lcp_plan_s* P = new lcp_plan_s();
  P->p = p;
  P->p.chunk_log2 = cl;
  P->chunk_log2 = cl;
  P->F = p.n_fields;
  P->N = p.max_particles;
  P->k = p.block_log2 < 0 ? 0 : p.block_log2;
  lcp_status st = alloc_plan(P);
  if (!st && p.block_log2 == -1) {
    if (sample_n > P->N) st = LCP_ERR_ARG;
    else {
      TimerScope ts(P);
      st = search_k(P, sample_fields, sample_n, nullptr);
    }
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
  plan->have_eb = false;
  plan->seq = 0;
  plan->fsm_t = false;
  plan->interval = 1;
  plan->countdown = 0;
  plan->last_s = 0;
  plan->have_last_s = false;
  return LCP_OK;
}

uint64_t lcp_bound(lcp_plan_t plan, uint64_t n) { return plan ? bound_bytes(plan->F, n) : 0; }

lcp_status lcp_compress(lcp_plan_t plan, uint64_t n_frames, const lcp_frame_in* frames,
                        void* out, uint64_t out_cap, uint64_t* out_offsets, int* methods_used,
                        uint32_t* const* perms, hipStream_t stream) {
  if (!plan || (!frames && n_frames) || !out_offsets || (!out && n_frames)) return LCP_ERR_ARG;
  if ((uintptr_t)out & 3) return LCP_ERR_ARG;
  TimerScope ts(plan);
  uint8_t* o = reinterpret_cast<uint8_t*>(out);
  uint64_t off = 0;
  out_offsets[0] = 0;
  for (uint64_t j = 0; j < n_frames; j++) {
    uint64_t size = 0;
    int used = 0;
    uint64_t cap = out_cap > off ? out_cap - off : 0;
    lcp_status st = compress_frame(plan, frames[j], o + off, cap, &size, &used,
                                   perms ? perms[j] : nullptr, stream);
    if (st) {
      out_offsets[j + 1] = off + size;
      return st;
    }
    if (methods_used) methods_used[j] = used;
    off += (size + 3) & ~3ull;
    out_offsets[j + 1] = off;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return LCP_ERR_DEVICE;
  timer_collect(plan);
  return LCP_OK;
}

lcp_status lcp_decompress(lcp_plan_t plan, uint64_t n_frames, const lcp_blob* blobs,
                          const lcp_frame_out* outs, uint64_t* n_out, hipStream_t stream) {
  if (!plan || (n_frames && (!blobs || !outs || !n_out))) return LCP_ERR_ARG;
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

lcp_status lcp_kernel_timer_set(lcp_plan_t plan, const char* kernel_name) {
  if (!plan) return LCP_ERR_ARG;
  if (!kernel_name) {
    plan->timer_name[0] = 0;
  } else {
    if (strlen(kernel_name) >= sizeof(plan->timer_name)) return LCP_ERR_ARG;
    strcpy(plan->timer_name, kernel_name);
  }
  plan->timer_ms = 0;
  plan->timer_launches = 0;
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
