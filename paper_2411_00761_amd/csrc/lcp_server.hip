// lcp_server.hip -- serving many multi-frame streams on one device.
//
// Each stream is a multi-frame plan whose resident state (reference codes and
// permutations, LCP-FSM and Alg. 1 bookkeeping) lives on the device for the
// stream's lifetime; its scratch is not owned but carved, per request, out of
// one device arena.  Worker threads, each with its own HIP stream and pinned
// host tables, take requests in arrival order: a request is admitted when a
// worker is free, its stream has no request in flight (a stream's requests run
// in submission order), and the arena has room for its scratch.  Requests of
// different streams therefore overlap on the device, and the memory a finished
// request releases admits the next one.
//
// Continuous batching: with batch plans enabled, the temporal requests that
// are admissible together -- compress requests whose stream's next frame goes
// to LCP-T, decompress requests of streams with the same fields and chunk size
// -- are merged into one set of launches on a batch plan (one residual or
// decode launch, one coding or reconstruction launch for all of them) instead
// of one set per request.  A merged request finishes exactly as its stream's
// own call would; one the merged launch cannot finish (its temporal record is
// larger than the last spatial one, or it is a spatial record) goes back to
// the front of the queue and takes its own call.
#include <algorithm>
#include <chrono>
#include <memory>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string.h>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lcp.h"
#include "lcp_internal.h"

using namespace lcp;

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct ServedStream {
  lcp_plan_s* plan = nullptr;
  size_t scratch = 0;  // arena bytes one request needs
  bool busy = false;
};

struct Ticket {
  lcp_request req;
  lcp_result res;
  bool solo = false;  // takes its own call (a merged launch could not finish it)
  // recorded on req.after at submit: the worker's stream waits for it, so the
  // request reads inputs and overwrites outputs only after the caller's
  // earlier work on them
  hipEvent_t ready = nullptr;
  bool done = false;
};

// First-fit allocator over [0, size) with coalescing frees (256-byte units).
struct Arena {
  std::map<size_t, size_t> free;  // offset -> bytes
  void init(size_t size) {
    free.clear();
    if (size) free[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free.begin(); it != free.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free.erase(it);
      if (rest) free[at] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

}  // namespace

// The scratch of merged launches for streams of one (fields, chunk size).
struct BatchSlot {
  int F = 0, cl = 0;
  lcp_plan_s* plan = nullptr;
  bool busy = false;
};

struct lcp_server_s {
  lcp_server_params p{};
  std::deque<BatchSlot> batches;  // one per worker and key; stable addresses
  uint64_t merged_launches = 0, merged_requests = 0, requeued = 0;
  void* arena_mem = nullptr;
  Arena arena;
  size_t state_used = 0;
  size_t host_bytes = 0;  // pinned tables per worker
  std::vector<ServedStream> streams;
  std::deque<uint64_t> pending;  // tickets in submission order
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  bool hold = false;  // workers take no new request
  std::vector<std::thread> workers;
  lcp_status worker_error = LCP_OK;
};

namespace {

// A free batch scratch for the request's (fields, chunk size), if any.
BatchSlot* free_batch_for(lcp_server_s* S, const Ticket& t) {
  if (t.solo) return nullptr;
  lcp_plan_s* P = S->streams[t.req.stream].plan;
  for (BatchSlot& b : S->batches)
    if (!b.busy && b.F == plan_fields(P) && b.cl == plan_chunk_log2(P)) return &b;
  return nullptr;
}

bool same_key(lcp_server_s* S, const Ticket& t, const BatchSlot* b) {
  lcp_plan_s* P = S->streams[t.req.stream].plan;
  return !t.solo && b->F == plan_fields(P) && b->cl == plan_chunk_log2(P);
}

// Particles a request brings into a merged launch (at most).
uint64_t particles_of(const Ticket& t) {
  return t.req.kind == LCP_REQ_COMPRESS ? t.req.frame.n : t.req.dst.capacity;
}

bool mergeable(lcp_server_s* S, const Ticket& t) {
  if (t.req.kind == LCP_REQ_COMPRESS) return serve_t_eligible(S->streams[t.req.stream].plan, t.req.frame);
  // decompress: whether the record is temporal shows once its header is read;
  // a stream whose last record was temporal most likely sends another
  return plan_decoding_t(S->streams[t.req.stream].plan);
}

// Next work (lock held), taken in arrival order among requests whose stream
// is idle and has no earlier pending request.  When the first such request
// can be merged and a batch scratch of its kind is free, it leads a group
// joined by the further such requests of the same kind and batch key, up to
// the frame and particle capacity; a group of two or more runs merged.
// Otherwise that first request runs alone (single) on scratch from the arena;
// memory is admitted strictly in order, so a large request is not starved by
// smaller ones behind it.
bool pick(lcp_server_s* S, std::vector<uint64_t>* group, BatchSlot** slot, uint64_t* single,
          size_t* off) {
  std::vector<char> blocked(S->streams.size(), 0);
  group->clear();
  *slot = nullptr;
  int kind = 0;
  uint64_t parts = 0;
  auto first = S->pending.end();
  for (auto it = S->pending.begin(); it != S->pending.end(); ++it) {
    const Ticket& t = S->tickets[*it];
    const int sid = t.req.stream;
    if (blocked[sid]) continue;
    blocked[sid] = 1;
    if (S->streams[sid].busy) continue;
    if (first == S->pending.end()) {
      first = it;
      BatchSlot* b = free_batch_for(S, t);
      if (!b || !mergeable(S, t) || particles_of(t) > serve_batch_particles(b->plan)) break;
      *slot = b;
      kind = t.req.kind;
      parts = particles_of(t);
      group->push_back(*it);
      continue;
    }
    if ((int)group->size() >= serve_batch_frames((*slot)->plan)) break;
    if (t.req.kind != kind || !same_key(S, t, *slot) || !mergeable(S, t)) continue;
    if (parts + particles_of(t) > serve_batch_particles((*slot)->plan)) continue;
    parts += particles_of(t);
    group->push_back(*it);
  }
  if (group->size() >= 2) {
    for (uint64_t id : *group) {
      S->streams[S->tickets[id].req.stream].busy = true;
      S->pending.erase(std::find(S->pending.begin(), S->pending.end(), id));
    }
    (*slot)->busy = true;
    return true;
  }
  group->clear();
  *slot = nullptr;
  if (first == S->pending.end()) return false;
  ServedStream& st = S->streams[S->tickets[*first].req.stream];
  if (!S->arena.alloc(st.scratch, off)) return false;
  st.busy = true;
  *single = *first;
  S->pending.erase(first);
  return true;
}

// A merged launch of the group's requests on the worker's stream; the ones it
// finished complete, the others go back to the front of the queue in order.
void run_group(lcp_server_s* S, const std::vector<uint64_t>& group, BatchSlot* slot,
               hipStream_t hs) {
  const int K = (int)group.size();
  std::vector<lcp_plan_s*> plans(K);
  std::vector<lcp_frame_in> frames(K);
  std::vector<void*> outs(K);
  std::vector<uint64_t> caps(K), sizes(K, 0), nout(K, 0);
  std::vector<lcp_blob> blobs(K);
  std::vector<lcp_frame_out> dsts(K);
  std::unique_ptr<bool[]> done(new bool[K]());
  int kind = 0;
  bool ok = true;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    const uint64_t now = now_ns();
    for (int i = 0; i < K; i++) {
      Ticket& t = S->tickets[group[i]];
      t.res.t_start_ns = now;
      kind = t.req.kind;
      plans[i] = S->streams[t.req.stream].plan;
      frames[i] = t.req.frame;
      outs[i] = t.req.out;
      caps[i] = t.req.out_cap;
      blobs[i] = t.req.blob;
      dsts[i] = t.req.dst;
      if (t.ready && hipStreamWaitEvent(hs, t.ready, 0) != hipSuccess) ok = false;
    }
  }
  lcp_status st = LCP_ERR_DEVICE;
  if (ok)
    st = kind == LCP_REQ_COMPRESS
             ? serve_t_compress(slot->plan, K, plans.data(), frames.data(), outs.data(), caps.data(),
                                done.get(), sizes.data(), hs)
             : serve_t_decompress(slot->plan, K, plans.data(), blobs.data(), dsts.data(), done.get(),
                                  nout.data(), hs);
  const uint64_t end = now_ns();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->merged_launches++;
    for (int i = K - 1; i >= 0; i--) {
      Ticket& t = S->tickets[group[i]];
      S->streams[t.req.stream].busy = false;
      if (st == LCP_OK && done[i]) {
        t.res.status = LCP_OK;
        t.res.method = kind == LCP_REQ_COMPRESS ? LCP_METHOD_T : 0;
        t.res.bytes = kind == LCP_REQ_COMPRESS ? sizes[i] : nout[i];
        t.res.t_end_ns = end;
        t.res.group = K;
        if (t.ready) (void)hipEventDestroy(t.ready);
        t.ready = nullptr;
        t.done = true;
        S->merged_requests++;
      } else {
        t.solo = true;  // back to the front of the queue, in order
        S->pending.push_front(group[i]);
        S->requeued++;
      }
    }
    slot->busy = false;
  }
}

void run_request(lcp_plan_s* plan, const lcp_request& rq, hipStream_t hs, lcp_result* res) {
  if (rq.kind == LCP_REQ_COMPRESS) {
    uint64_t offs[2] = {0, 0};
    int method = 0;
    res->status = lcp_compress(plan, 1, &rq.frame, rq.out, rq.out_cap, offs, &method, nullptr, hs);
    res->method = method;
    res->bytes = offs[1];
  } else {
    uint64_t n = 0;
    res->status = lcp_decompress(plan, 1, &rq.blob, &rq.dst, &n, hs);
    res->method = 0;
    res->bytes = n;
  }
}

void worker_main(lcp_server_s* S) {
  hipStream_t hs = nullptr;
  void* host = nullptr;
  lcp_status init = LCP_OK;
  if (hipSetDevice(S->p.device) != hipSuccess ||
      hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc(&host, S->host_bytes, 0) != hipSuccess)
    init = LCP_ERR_DEVICE;
  for (;;) {
    uint64_t tk = 0;
    size_t off = 0;
    std::vector<uint64_t> group;
    BatchSlot* slot = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (init != LCP_OK) S->worker_error = init;
      S->cv_work.wait(lk, [&] {
        return S->stop || (init == LCP_OK && !S->hold && pick(S, &group, &slot, &tk, &off));
      });
      if (S->stop && tk == 0 && group.empty()) break;
    }
    if (!group.empty()) {
      run_group(S, group, slot, hs);
      S->cv_done.notify_all();
      S->cv_work.notify_all();
      continue;
    }
    Ticket* t;
    lcp_plan_s* plan;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      t = &S->tickets[tk];
      plan = S->streams[t->req.stream].plan;
      t->res.t_start_ns = now_ns();
    }
    lcp_result res = t->res;
    res.group = 1;
    if (t->ready && hipStreamWaitEvent(hs, t->ready, 0) != hipSuccess) {
      res.status = LCP_ERR_DEVICE;
    } else {
      plan_bind(plan, static_cast<uint8_t*>(S->arena_mem) + off, host, hs);
      run_request(plan, t->req, hs, &res);
      plan_unbind(plan);
    }
    if (t->ready) (void)hipEventDestroy(t->ready);
    t->ready = nullptr;
    res.t_end_ns = now_ns();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->arena.release(off, S->streams[t->req.stream].scratch);
      S->streams[t->req.stream].busy = false;
      t->res = res;
      t->done = true;
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  if (host) (void)hipHostFree(host);
  if (hs) (void)hipStreamDestroy(hs);
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

lcp_status lcp_server_create(const lcp_server_params* params, lcp_server_t* out) {
  if (!params || !out) return LCP_ERR_ARG;
  *out = nullptr;
  const lcp_server_params& p = *params;
  if (p.workers < 1 || p.workers > 16 || p.scratch_bytes == 0 ||
      (p.hbm_budget_bytes && p.scratch_bytes > p.hbm_budget_bytes) || p.batch_frames < 0 ||
      p.batch_frames > 64 || p.batch_frames == 1 || p.batch_particles > 0xFFFFFFFFull ||
      (p.batch_frames > 0 && p.batch_particles == 0))
    return LCP_ERR_ARG;
  if (hipSetDevice(p.device) != hipSuccess) return LCP_ERR_DEVICE;
  lcp_server_s* S = new lcp_server_s();
  S->p = p;
  S->p.scratch_bytes = round256(p.scratch_bytes);
  // pinned tables of the largest multi-frame plan (they do not depend on n)
  lcp_params q{};
  q.eb_mode = LCP_EB_ABS;
  q.eb = 1.0;
  q.n_fields = LCP_MAX_FIELDS;
  q.multi_frame = 1;
  q.block_log2 = 0;
  q.max_particles = 1;
  q.device = p.device;
  lcp_plan_s* probe = nullptr;
  lcp_status st = plan_create_unbound(&q, nullptr, 0, &probe);
  if (st) {
    delete S;
    return st;
  }
  S->host_bytes = plan_host_bytes(probe);
  lcp_plan_destroy(probe);
  if (hipMalloc(&S->arena_mem, S->p.scratch_bytes) != hipSuccess) {
    delete S;
    return LCP_ERR_DEVICE;
  }
  S->arena.init(S->p.scratch_bytes);
  for (int w = 0; w < p.workers; w++) S->workers.emplace_back(worker_main, S);
  *out = S;
  return LCP_OK;
}

void lcp_server_destroy(lcp_server_t S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& th : S->workers) th.join();
  for (auto& st : S->streams) lcp_plan_destroy(st.plan);
  for (auto& b : S->batches) lcp_plan_destroy(b.plan);
  for (auto& kv : S->tickets)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  if (S->arena_mem) (void)hipFree(S->arena_mem);
  delete S;
}

lcp_status lcp_server_open_stream(lcp_server_t S, const lcp_params* params,
                                  const float* const* sample_fields, uint64_t sample_n,
                                  int* stream_id) {
  if (!S || !params || !stream_id || !params->multi_frame || params->device != S->p.device)
    return LCP_ERR_ARG;
  lcp_plan_s* plan = nullptr;
  lcp_status st = plan_create_unbound(params, sample_fields, sample_n, &plan);
  if (st) return st;
  const size_t scratch = round256(plan_scratch_bytes(plan));
  const size_t state = plan_state_bytes(plan);
  std::lock_guard<std::mutex> lk(S->mu);
  if (scratch > S->p.scratch_bytes ||
      (S->p.hbm_budget_bytes && S->state_used + state + S->p.scratch_bytes > S->p.hbm_budget_bytes)) {
    lcp_plan_destroy(plan);
    return LCP_ERR_BUDGET;
  }
  S->state_used += state;
  if (S->p.batch_frames > 0) {
    bool have = false;
    for (const BatchSlot& b : S->batches)
      have |= b.F == plan_fields(plan) && b.cl == plan_chunk_log2(plan);
    // one batch scratch per worker for a new (fields, chunk size)
    for (int w = 0; !have && w < S->p.workers; w++) {
      BatchSlot b;
      b.F = plan_fields(plan);
      b.cl = plan_chunk_log2(plan);
      st = serve_batch_create(b.F, b.cl, S->p.batch_frames, S->p.batch_particles, S->p.device,
                              &b.plan);
      if (st == LCP_OK && S->p.hbm_budget_bytes &&
          S->state_used + serve_batch_bytes(b.plan) + S->p.scratch_bytes > S->p.hbm_budget_bytes)
        st = LCP_ERR_BUDGET;
      if (st) {
        if (b.plan) lcp_plan_destroy(b.plan);
        while (!S->batches.empty() && S->batches.back().F == b.F && S->batches.back().cl == b.cl) {
          S->state_used -= serve_batch_bytes(S->batches.back().plan);
          lcp_plan_destroy(S->batches.back().plan);
          S->batches.pop_back();
        }
        S->state_used -= state;
        lcp_plan_destroy(plan);
        return st;
      }
      S->state_used += serve_batch_bytes(b.plan);
      S->batches.push_back(b);
    }
  }
  ServedStream ss;
  ss.plan = plan;
  ss.scratch = scratch;
  S->streams.push_back(ss);
  *stream_id = (int)S->streams.size() - 1;
  return LCP_OK;
}

lcp_status lcp_server_submit(lcp_server_t S, const lcp_request* req, uint64_t* ticket) {
  if (!S || !req || !ticket) return LCP_ERR_ARG;
  if (req->kind != LCP_REQ_COMPRESS && req->kind != LCP_REQ_DECOMPRESS) return LCP_ERR_ARG;
  hipEvent_t ready = nullptr;
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) return LCP_ERR_DEVICE;
  if (hipEventRecord(ready, req->after) != hipSuccess) {
    (void)hipEventDestroy(ready);
    return LCP_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  lcp_status bad = S->worker_error;
  if (!bad && (req->stream < 0 || req->stream >= (int)S->streams.size())) bad = LCP_ERR_ARG;
  if (bad) {
    if (ready) (void)hipEventDestroy(ready);
    return bad;
  }
  const uint64_t id = S->next_ticket++;
  Ticket& t = S->tickets[id];
  t.req = *req;
  t.ready = ready;
  memset(&t.res, 0, sizeof(t.res));
  t.res.t_submit_ns = now_ns();
  S->pending.push_back(id);
  *ticket = id;
  S->cv_work.notify_one();
  return LCP_OK;
}

lcp_status lcp_server_wait(lcp_server_t S, uint64_t ticket, lcp_result* res) {
  if (!S || !res) return LCP_ERR_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return LCP_ERR_ARG;
  S->cv_done.wait(lk, [&] { return S->tickets[ticket].done || S->worker_error != LCP_OK; });
  Ticket& t = S->tickets[ticket];
  if (!t.done) return S->worker_error;
  *res = t.res;
  S->tickets.erase(ticket);
  return LCP_OK;
}

lcp_status lcp_server_hold(lcp_server_t S, int hold) {
  if (!S) return LCP_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->hold = hold != 0;
  }
  S->cv_work.notify_all();
  return LCP_OK;
}

lcp_status lcp_server_counts(lcp_server_t S, uint64_t* merged_launches, uint64_t* merged_requests,
                             uint64_t* requeued) {
  if (!S) return LCP_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  if (merged_launches) *merged_launches = S->merged_launches;
  if (merged_requests) *merged_requests = S->merged_requests;
  if (requeued) *requeued = S->requeued;
  return LCP_OK;
}

}  // extern "C"
