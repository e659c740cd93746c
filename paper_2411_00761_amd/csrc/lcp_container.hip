// Multi-frame container with random access (Sec. 7.3, Alg. 1).
//
// The records of one multi-frame stream are packed so that any frame can be
// retrieved alone: a 64-byte header, a 32-byte entry per frame (offset, size,
// reference, particle count, method, anchor flag), the records of each batch in
// stream order, and the spatial anchor frames -- first in their batch, coded by
// LCP-S -- in an array of their own after the batches (Sec. 7.3).  A frame is
// retrieved by decoding it directly when it is spatial, else its reference
// first, recursively: at most the frames of its batch up to it plus one anchor.
// Retrieval decodes the union of the requested frames' closures once, in stream
// order, through a multi-frame plan's decoder (whose resident references carry
// the chain), in the caller's order of requests (a new pass, on a reset
// decoder, wherever a request goes back in the stream).  All decoding is the
// library's GPU path; this file is host-side bookkeeping.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/lcp.h"
#include "lcp_internal.h"

using namespace lcp;

namespace {

constexpr uint64_t kCHdr = 64, kCEntry = 32;
constexpr uint32_t kCMagic = 0x4350434Cu;  // bytes "LCPC"
constexpr int kSlots = 16;                 // frames decoded per call

struct Entry {
  uint64_t off = 0, size = 0, ref = ~0ull;
  uint32_t n = 0;
  uint8_t mode = 0, anchor = 0;
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
void wr32(uint8_t* b, size_t o, uint32_t v) { memcpy(b + o, &v, 4); }
void wr64(uint8_t* b, size_t o, uint64_t v) { memcpy(b + o, &v, 8); }

bool first_of_batch(int batch, uint64_t seq) {
  return batch == 0 ? seq == 0 : seq % (uint64_t)batch == 0;
}

}  // namespace

struct lcp_container_s {
  int batch = 0, F = 0;
  uint64_t frames = 0, anchors = 0, total = 0;
  const uint8_t* base = nullptr;  // device
  std::vector<Entry> ent;
  float* scratch = nullptr;  // kSlots frames of F fields for frames not requested
  uint64_t scratch_n = 0;
};

namespace {

// The frames needed to obtain frame k, in stream order.
lcp_status closure_of(const lcp_container_s* C, uint64_t k, std::vector<uint64_t>* out) {
  out->clear();
  if (k >= C->frames) return LCP_ERR_ARG;
  for (uint64_t j = k;;) {
    out->push_back(j);
    const Entry& e = C->ent[j];
    if (e.mode == 0) break;
    j = e.ref;  // checked at open: below j
  }
  std::reverse(out->begin(), out->end());
  return LCP_OK;
}

}  // namespace

extern "C" {

lcp_status lcp_container_pack(const lcp_blob* records, uint64_t n, int batch_size, void* out,
                              uint64_t out_cap, uint64_t* out_size, hipStream_t stream) {
  if (!records || n == 0 || batch_size < 0 || !out_size || ((uintptr_t)out & 3)) return LCP_ERR_ARG;
  // the fixed part of every record's header, read back once
  std::vector<uint8_t> hdr(n * (uint64_t)kHdrBytes, 0);
  for (uint64_t j = 0; j < n; j++) {
    if (!records[j].data || records[j].size < (uint64_t)kHdrBytes || (records[j].size & 3))
      return LCP_ERR_ARG;
    if (hipMemcpyAsync(hdr.data() + j * kHdrBytes, records[j].data, kHdrBytes,
                       hipMemcpyDeviceToHost, stream) != hipSuccess)
      return LCP_ERR_DEVICE;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return LCP_ERR_DEVICE;
  std::vector<Entry> ent(n);
  int F = 0;
  uint64_t anchors = 0;
  for (uint64_t j = 0; j < n; j++) {
    const uint8_t* h = hdr.data() + j * kHdrBytes;
    if (rd32(h, 0) != kMagic || (rd32(h, 4) & 0xFFFF) != (uint32_t)kVersion) return LCP_ERR_CORRUPT;
    const int mode = h[6], f = h[7];
    const uint64_t nn = rd64(h, 16), total = rd64(h, 32), seq = rd64(h, 56), ref = rd64(h, 64);
    if (j == 0) F = f;
    // one stream from its start: record j is frame j, references go back
    if (mode > 1 || f != F || seq != j || total != records[j].size || nn == 0 ||
        nn > (1ull << 31) || (mode == 1 && ref >= j))
      return LCP_ERR_ARG;
    ent[j].size = total;
    ent[j].n = (uint32_t)nn;
    ent[j].mode = (uint8_t)mode;
    ent[j].ref = mode == 1 ? ref : ~0ull;
    ent[j].anchor = first_of_batch(batch_size, j) && mode == 0;
    anchors += ent[j].anchor;
  }
  uint64_t off = kCHdr + kCEntry * n;
  for (uint64_t j = 0; j < n; j++)
    if (!ent[j].anchor) {
      ent[j].off = off;
      off += ent[j].size;
    }
  const uint64_t anchor_off = off;
  for (uint64_t j = 0; j < n; j++)
    if (ent[j].anchor) {
      ent[j].off = off;
      off += ent[j].size;
    }
  *out_size = off;
  if (!out) return LCP_OK;
  if (off > out_cap) return LCP_ERR_CAPACITY;
  std::vector<uint8_t> head(kCHdr + kCEntry * n, 0);
  wr32(head.data(), 0, kCMagic);
  wr32(head.data(), 4, 1u);  // version 1, reserved 0
  wr32(head.data(), 8, (uint32_t)batch_size);
  wr32(head.data(), 12, (uint32_t)F);
  wr64(head.data(), 16, n);
  wr64(head.data(), 24, anchors);
  wr64(head.data(), 32, kCHdr);
  wr64(head.data(), 40, anchor_off);
  wr64(head.data(), 48, off);
  for (uint64_t j = 0; j < n; j++) {
    uint8_t* e = head.data() + kCHdr + kCEntry * j;
    wr64(e, 0, ent[j].off);
    wr64(e, 8, ent[j].size);
    wr64(e, 16, ent[j].ref);
    wr32(e, 24, ent[j].n);
    e[28] = ent[j].mode;
    e[29] = ent[j].anchor;
  }
  uint8_t* o = static_cast<uint8_t*>(out);
  if (hipMemcpyAsync(o, head.data(), head.size(), hipMemcpyHostToDevice, stream) != hipSuccess)
    return LCP_ERR_DEVICE;
  for (uint64_t j = 0; j < n; j++)
    if (hipMemcpyAsync(o + ent[j].off, records[j].data, ent[j].size, hipMemcpyDeviceToDevice,
                       stream) != hipSuccess)
      return LCP_ERR_DEVICE;
  // the header buffer is host memory that goes away on return
  if (hipStreamSynchronize(stream) != hipSuccess) return LCP_ERR_DEVICE;
  return LCP_OK;
}

lcp_status lcp_container_open(const void* container, uint64_t size, hipStream_t stream,
                              lcp_container_t* out) {
  if (!container || !out || size < kCHdr || ((uintptr_t)container & 3)) return LCP_ERR_ARG;
  *out = nullptr;
  uint8_t h[kCHdr];
  if (hipMemcpyAsync(h, container, kCHdr, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return LCP_ERR_DEVICE;
  const uint64_t n = rd64(h, 16);
  if (rd32(h, 0) != kCMagic || rd32(h, 4) != 1u || n == 0 || rd64(h, 32) != kCHdr ||
      n > (size - kCHdr) / kCEntry || rd64(h, 48) != size || rd32(h, 12) < 1 ||
      rd32(h, 12) > LCP_MAX_FIELDS || rd32(h, 8) > 0x7FFFFFFFu)
    return LCP_ERR_CORRUPT;
  std::vector<uint8_t> tab(kCEntry * n);
  if (hipMemcpyAsync(tab.data(), static_cast<const uint8_t*>(container) + kCHdr, tab.size(),
                     hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return LCP_ERR_DEVICE;
  lcp_container_s* C = new lcp_container_s();
  C->batch = (int)rd32(h, 8);
  C->F = (int)rd32(h, 12);
  C->frames = n;
  C->anchors = rd64(h, 24);
  C->total = size;
  C->base = static_cast<const uint8_t*>(container);
  C->ent.resize(n);
  uint64_t anchors = 0;
  bool ok = true;
  for (uint64_t j = 0; j < n && ok; j++) {
    const uint8_t* e = tab.data() + kCEntry * j;
    Entry& x = C->ent[j];
    x.off = rd64(e, 0);
    x.size = rd64(e, 8);
    x.ref = rd64(e, 16);
    x.n = rd32(e, 24);
    x.mode = e[28];
    x.anchor = e[29];
    anchors += x.anchor;
    ok = x.mode <= 1 && x.anchor <= 1 && x.off >= kCHdr + kCEntry * n && x.size >= (uint64_t)kHdrBytes &&
         x.off <= size && x.size <= size - x.off && !(x.off & 3) && !(x.size & 3) && x.n > 0 &&
         (x.mode == 0 ? x.ref == ~0ull : x.ref < j) &&
         x.anchor == (first_of_batch(C->batch, j) && x.mode == 0);
  }
  if (!ok || anchors != C->anchors) {
    delete C;
    return LCP_ERR_CORRUPT;
  }
  *out = C;
  return LCP_OK;
}

lcp_status lcp_container_info(lcp_container_t C, uint64_t* frames, int* batch_size,
                              uint64_t* anchors, int* n_fields) {
  if (!C) return LCP_ERR_ARG;
  if (frames) *frames = C->frames;
  if (batch_size) *batch_size = C->batch;
  if (anchors) *anchors = C->anchors;
  if (n_fields) *n_fields = C->F;
  return LCP_OK;
}

lcp_status lcp_container_closure(lcp_container_t C, uint64_t frame, uint64_t* frames,
                                 uint64_t cap, uint64_t* count) {
  if (!C || !count) return LCP_ERR_ARG;
  std::vector<uint64_t> cl;
  lcp_status st = closure_of(C, frame, &cl);
  if (st) return st;
  *count = cl.size();
  if (cl.size() > cap || (!frames && cap)) return LCP_ERR_CAPACITY;
  for (size_t i = 0; i < cl.size(); i++) frames[i] = cl[i];
  return LCP_OK;
}

lcp_status lcp_container_retrieve(lcp_container_t C, lcp_plan_t plan, uint64_t n_req,
                                  const uint64_t* frames, const lcp_frame_out* outs,
                                  uint64_t* decoded, hipStream_t stream) {
  if (!C || !plan || (n_req && (!frames || !outs))) return LCP_ERR_ARG;
  if (!plan_multi_frame(plan) || plan_fields(plan) != C->F || plan_batch_size(plan) != C->batch)
    return LCP_ERR_ARG;
  uint64_t nmax = 0;
  for (uint64_t j = 0; j < C->frames; j++) nmax = std::max<uint64_t>(nmax, C->ent[j].n);
  if (nmax > plan_max_particles(plan)) return LCP_ERR_ARG;
  for (uint64_t i = 0; i < n_req; i++)
    if (frames[i] >= C->frames) return LCP_ERR_ARG;
  if (C->scratch_n < nmax) {
    if (C->scratch) (void)hipFree(C->scratch);
    C->scratch = nullptr;
    C->scratch_n = 0;
    if (hipMalloc(&C->scratch, sizeof(float) * nmax * C->F * kSlots) != hipSuccess)
      return LCP_ERR_DEVICE;
    C->scratch_n = nmax;
  }
  uint64_t count = 0;
  // passes: runs of requests with increasing frame numbers, in the caller's order
  for (uint64_t p0 = 0; p0 < n_req;) {
    uint64_t p1 = p0 + 1;
    while (p1 < n_req && frames[p1] > frames[p1 - 1]) p1++;
    std::vector<uint64_t> need, cl;
    for (uint64_t i = p0; i < p1; i++) {
      lcp_status st = closure_of(C, frames[i], &cl);
      if (st) return st;
      need.insert(need.end(), cl.begin(), cl.end());
    }
    std::sort(need.begin(), need.end());
    need.erase(std::unique(need.begin(), need.end()), need.end());
    lcp_status st = lcp_plan_reset(plan);
    if (st) return st;
    for (size_t g0 = 0; g0 < need.size(); g0 += kSlots) {
      const size_t g1 = std::min(need.size(), g0 + kSlots);
      lcp_blob blobs[kSlots];
      lcp_frame_out fo[kSlots];
      uint64_t n_out[kSlots];
      for (size_t g = g0; g < g1; g++) {
        const uint64_t j = need[g];
        const Entry& e = C->ent[j];
        blobs[g - g0].data = C->base + e.off;
        blobs[g - g0].size = e.size;
        // a requested frame goes to its own output, the others to scratch
        const uint64_t* hit = std::find(frames + p0, frames + p1, j);
        if (hit != frames + p1) {
          fo[g - g0] = outs[hit - frames];
        } else {
          memset(&fo[g - g0], 0, sizeof(lcp_frame_out));
          float* s = C->scratch + (g - g0) * C->F * nmax;
          for (int f = 0; f < C->F; f++) fo[g - g0].fields[f] = s + (uint64_t)f * nmax;
          fo[g - g0].capacity = nmax;
        }
      }
      st = lcp_decompress(plan, g1 - g0, blobs, fo, n_out, stream);
      if (st) return st;
      for (size_t g = g0; g < g1; g++)
        if (n_out[g - g0] != C->ent[need[g]].n) return LCP_ERR_CORRUPT;
      count += g1 - g0;
    }
    p0 = p1;
  }
  if (decoded) *decoded = count;
  return LCP_OK;
}

void lcp_container_close(lcp_container_t C) {
  if (!C) return;
  if (C->scratch) (void)hipFree(C->scratch);
  delete C;
}

}  // extern "C"
