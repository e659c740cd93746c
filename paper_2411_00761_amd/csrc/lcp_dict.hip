// Dictionary stage: the last coding step of Sec. 6.2.2 and Sec. 7.1 (which
// the paper fills with a general-purpose dictionary coder), here an order-0
// range-asymmetric numeral system (rANS) coder over the bytes of coded
// records.  One frequency table for the whole input (normalised to 4096) and
// independent blocks of 2^block_log2 bytes, each coded by one wave whose lane
// k takes the block's bytes k, k + 64, ... (so the lanes read and write
// neighbouring bytes): a lane's bytes go from last to first through a 32-bit
// state that starts at 2^23; a byte s of frequency f and cumulative frequency
// c first writes out the low bytes of the state while it is at least 2^19 f,
// then takes it to (x / f) 4096 + x % f + c.  A coded lane is the final state
// (4 bytes, little-endian) followed by the written bytes in reading order.
// Stream: u32 magic "LCPD", u32 block_log2, u64 n, u16 freq[256], u32
// size[nb], then the blocks (u16 lane_size[64], then the lanes' bytes).
//
// Encode: byte histogram; the table (one thread: normalisation, header);
// blocks coded into per-lane staging (each wave also writes its block's size
// into the stream's size table); the sizes scanned into offsets (the
// library's device scan); blocks gathered into the stream, a wave per block.
// Decode: one header read-back, the sizes scanned and checked against the
// stream's size, the slot-to-byte map built once, blocks decoded a wave each.
#include <hip/hip_runtime.h>
#include <string.h>

#include "../../include/lcp.h"
#include "lcp_internal.h"

namespace {

constexpr uint32_t kDMagic = 0x4450434Cu;  // bytes "LCPD"
constexpr int kDScale = 12;
constexpr uint32_t kDM = 1u << kDScale;
constexpr uint32_t kDL = 1u << 23;
constexpr uint64_t kDHdr = 4 + 4 + 8 + 2 * 256;
constexpr int kDThreads = 256;
constexpr int kDLanes = 64;  // lanes of a block (one wave)

enum : uint32_t { kDErrCorrupt = 1u };

__host__ __device__ inline uint64_t dict_blocks(uint64_t n, int bl) { return (n + (1ull << bl) - 1) >> bl; }
// a lane's staging: at most 1.5 bytes per byte, its state and a byte of rounding
__host__ __device__ inline uint64_t dict_lane_cap(int bl) {
  const uint64_t per = (1ull << bl) / kDLanes;
  return (per + per / 2 + 8 + 15) & ~15ull;
}

// Scratch of one call (device, 256-byte aligned pieces).
struct DictScratch {
  unsigned long long* counts;  // [256]
  uint32_t* freq;              // [256]
  uint32_t* cum;               // [257]
  uint32_t* sizes;             // [nb]
  uint64_t* offs;              // [nb + 1]
  unsigned long long* total;   // [1] stream bytes
  uint32_t* err;               // [1]
  uint64_t* tmp;               // scan scratch
  uint32_t* sym;               // [4096 / 4] decode: the slot-to-byte map, four slots a word
  uint32_t* lane;              // [nb][64] encode: the lanes' coded sizes
  uint8_t* stage;              // [nb][64][lane_cap] (encode only)
};
uint64_t align256(uint64_t b) { return (b + 255) & ~255ull; }
uint64_t dict_scratch(uint64_t nb, int bl, bool enc, DictScratch* S, uint8_t* base) {
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    uint8_t* p = base ? base + o : nullptr;
    o += align256(bytes ? bytes : 1);
    return p;
  };
  DictScratch x;
  x.counts = reinterpret_cast<unsigned long long*>(take(8 * 256));
  x.freq = reinterpret_cast<uint32_t*>(take(4 * 256));
  x.cum = reinterpret_cast<uint32_t*>(take(4 * 257));
  x.sizes = reinterpret_cast<uint32_t*>(take(4 * nb));
  x.offs = reinterpret_cast<uint64_t*>(take(8 * (nb + 1)));
  x.total = reinterpret_cast<unsigned long long*>(take(8));
  x.err = reinterpret_cast<uint32_t*>(take(4));
  x.tmp = reinterpret_cast<uint64_t*>(take(8 * lcp::scan_tmp_elems(nb + 1)));
  x.sym = reinterpret_cast<uint32_t*>(take(kDM));
  x.lane = reinterpret_cast<uint32_t*>(take(enc ? 4 * kDLanes * nb : 0));
  x.stage = take(enc ? nb * kDLanes * dict_lane_cap(bl) : 0);
  if (S) *S = x;
  return o;
}

__global__ __launch_bounds__(kDThreads) void k_dict_clear(DictScratch S) {
  const uint32_t t = threadIdx.x;
  S.counts[t] = 0;
  if (t == 0) {
    *S.total = 0;
    *S.err = 0;
  }
}

// Byte histogram: per-workgroup bins in LDS, merged once.
__global__ __launch_bounds__(kDThreads) void k_dict_hist(const uint8_t* in, uint64_t n,
                                                         DictScratch S) {
  __shared__ uint32_t bins[256];
  bins[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t words = n / 4;
  const uint32_t* w = reinterpret_cast<const uint32_t*>(in);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) {
    const uint32_t v = w[i];
#pragma unroll
    for (int k = 0; k < 4; k++) atomicAdd(&bins[(v >> (8 * k)) & 255u], 1u);
  }
  if (blockIdx.x == 0 && threadIdx.x < (n & 3)) atomicAdd(&bins[in[4 * words + threadIdx.x]], 1u);
  __syncthreads();
  if (bins[threadIdx.x]) atomicAdd(&S.counts[threadIdx.x], (unsigned long long)bins[threadIdx.x]);
}

// The table and the stream header: one workgroup, a thread per byte value;
// the rare excess (many values rounded up to 1) is taken off by one thread.
__global__ __launch_bounds__(kDThreads) void k_dict_table(uint64_t n, int bl, DictScratch S,
                                                          uint8_t* out) {
  __shared__ uint32_t f[256];
  __shared__ unsigned long long red[kDThreads];
  const uint32_t t = threadIdx.x;
  const unsigned long long c = S.counts[t];
  // c * 4096 / n without overflow: c < 2^52 for any input below 2^52 bytes
  const unsigned long long q = c ? (c << kDScale) / n : 0ull;
  f[t] = c ? (q < 1 ? 1u : (uint32_t)q) : 0u;
  red[t] = f[t];
  __syncthreads();
  for (int d = kDThreads / 2; d > 0; d >>= 1) {
    if ((int)t < d) red[t] += red[t + d];
    __syncthreads();
  }
  const int64_t sum = (int64_t)red[0];
  __syncthreads();
  if (n && sum < (int64_t)kDM) {
    // the most frequent value, ties to the smaller: (count, 255 - value) maximised
    red[t] = c ? (c << 8) | (255u - t) : 0ull;
    __syncthreads();
    for (int d = kDThreads / 2; d > 0; d >>= 1) {
      if ((int)t < d && red[t + d] > red[t]) red[t] = red[t + d];
      __syncthreads();
    }
    if (t == 0) f[255u - (uint32_t)(red[0] & 255u)] += (uint32_t)((int64_t)kDM - sum);
    __syncthreads();
  }
  if (t == 0) {
    int64_t excess = n ? sum - (int64_t)kDM : 0;
    while (excess > 0) {
      int best = -1;
      for (int s = 0; s < 256; s++)
        if (f[s] > 1 && (best < 0 || f[s] > f[best])) best = s;
      if (best < 0) break;  // not reachable: 256 values of at least 1 sum below 4096
      const int64_t d = (int64_t)(f[best] - 1) < excess ? (int64_t)(f[best] - 1) : excess;
      f[best] -= (uint32_t)d;
      excess -= d;
    }
    uint32_t run = 0;
    for (int s = 0; s < 256; s++) {
      S.cum[s] = run;
      run += f[s];
    }
    S.cum[256] = run;
    const uint32_t head[4] = {kDMagic, (uint32_t)bl, (uint32_t)n, (uint32_t)(n >> 32)};
    for (int i = 0; i < 16; i++) out[i] = (uint8_t)(head[i / 4] >> (8 * (i % 4)));
  }
  __syncthreads();
  S.freq[t] = f[t];
  out[16 + 2 * t] = (uint8_t)f[t];
  out[17 + 2 * t] = (uint8_t)(f[t] >> 8);
}

__device__ inline uint32_t wave_excl_sum(uint32_t v) {
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < kDLanes; d <<= 1) {
    const uint32_t o = (uint32_t)__shfl_up((int)incl, d, kDLanes);
    if ((int)(threadIdx.x % kDLanes) >= d) incl += o;
  }
  return incl - v;
}

// One block per wave (workgroup of 64): lane k codes the block's bytes k,
// k + 64, ... from the last into the end of its staging region.
__global__ __launch_bounds__(kDLanes) void k_dict_encode(const uint8_t* in, uint64_t n, int bl,
                                                         uint64_t nb, DictScratch S,
                                                         uint8_t* out) {
  __shared__ uint32_t freq[256], cum[256];
  for (int s = threadIdx.x; s < 256; s += kDLanes) {
    freq[s] = S.freq[s];
    cum[s] = S.cum[s];
  }
  __syncthreads();
  const uint64_t b = blockIdx.x;
  const uint32_t k = threadIdx.x;
  const uint64_t B = 1ull << bl, cap = dict_lane_cap(bl);
  const uint64_t i0 = b * B, len = n - i0 < B ? n - i0 : B;
  const uint64_t cnt = k < len ? (len - k + kDLanes - 1) / kDLanes : 0;
  uint8_t* const lo = S.stage + (b * kDLanes + k) * cap;
  uint8_t* const end = lo + cap;
  uint8_t* p = end;
  uint32_t x = kDL;
  bool over = false;
  for (uint64_t m = cnt; m-- > 0 && !over;) {
    const uint32_t s = in[i0 + k + kDLanes * m], f = freq[s];
    const uint32_t x_max = ((kDL >> kDScale) << 8) * f;
    while (x >= x_max) {
      if (p - lo <= 4) {  // never taken: a lane codes into at most 1.5 bytes per byte + 5
        over = true;
        break;
      }
      *--p = (uint8_t)(x & 0xFFu);
      x >>= 8;
    }
    x = (x / f) * kDM + x % f + cum[s];
  }
  uint32_t size = 0;
  if (!over) {
    p -= 4;
    p[0] = (uint8_t)x;
    p[1] = (uint8_t)(x >> 8);
    p[2] = (uint8_t)(x >> 16);
    p[3] = (uint8_t)(x >> 24);
    size = (uint32_t)(end - p);
  } else {
    atomicOr(S.err, kDErrCorrupt);
  }
  S.lane[b * kDLanes + k] = size;
  // the block's size: the lanes' table and their bytes
  uint32_t tot = size;
#pragma unroll
  for (int d = kDLanes / 2; d > 0; d >>= 1) tot += (uint32_t)__shfl_xor((int)tot, d, kDLanes);
  if (k == 0) {
    const uint32_t bsize = 2 * kDLanes + tot;
    S.sizes[b] = bsize;
    S.offs[b] = bsize;
    reinterpret_cast<uint32_t*>(out + kDHdr)[b] = bsize;  // the stream's size table
  }
}

// The block sizes as u64 (decoding: from the stream), to be scanned in place.
__global__ __launch_bounds__(kDThreads) void k_dict_widen(uint64_t nb, DictScratch S) {
  const uint64_t j = (uint64_t)blockIdx.x * kDThreads + threadIdx.x;
  if (j < nb) S.offs[j] = S.sizes[j];
}

// After the exclusive scan: offs[nb] and the stream's total size; when
// decoding the sizes must add up to the stream.
__global__ void k_dict_total(uint64_t nb, DictScratch S, uint64_t check_total) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const unsigned long long run = nb ? S.offs[nb - 1] + S.sizes[nb - 1] : 0ull;
  S.offs[nb] = run;
  const unsigned long long total = kDHdr + 4 * nb + run;
  *S.total = total;
  if (check_total && total != check_total) atomicOr(S.err, kDErrCorrupt);
}

// Coded blocks into the stream, a wave per block: the lanes' size table, then
// each lane's bytes copied by the whole wave in turn.
__global__ __launch_bounds__(kDThreads) void k_dict_gather(uint64_t nb, int bl, DictScratch S,
                                                           uint8_t* out) {
  const uint64_t b = (uint64_t)blockIdx.x * (kDThreads / kDLanes) + threadIdx.x / kDLanes;
  if (b >= nb) return;
  const uint32_t k = threadIdx.x % kDLanes;
  const uint64_t cap = dict_lane_cap(bl);
  const uint32_t size = S.lane[b * kDLanes + k];
  const uint32_t off = wave_excl_sum(size);
  uint8_t* dst = out + kDHdr + 4 * nb + S.offs[b];
  dst[2 * k] = (uint8_t)size;
  dst[2 * k + 1] = (uint8_t)(size >> 8);
  for (uint32_t j = 0; j < kDLanes; j++) {
    const uint32_t sj = (uint32_t)__shfl((int)size, (int)j, kDLanes);
    const uint32_t oj = (uint32_t)__shfl((int)off, (int)j, kDLanes);
    const uint8_t* src = S.stage + (b * kDLanes + j) * cap + cap - sj;
    uint8_t* d = dst + 2 * kDLanes + oj;
    // four bytes per lane requested together
    for (uint32_t i = k; i < sj; i += 4 * kDLanes) {
      uint8_t v[4];
#pragma unroll
      for (int u = 0; u < 4; u++) v[u] = i + u * kDLanes < sj ? src[i + u * kDLanes] : 0;
#pragma unroll
      for (int u = 0; u < 4; u++)
        if (i + u * kDLanes < sj) d[i + u * kDLanes] = v[u];
    }
  }
}

// The slot-to-byte map of a stream's table (slot i belongs to the byte whose
// interval [cum, cum + freq) holds it), built once for the decode workgroups;
// a table that does not sum to 4096 flags the stream.
__global__ __launch_bounds__(kDThreads) void k_dict_slots(const uint8_t* in, DictScratch S) {
  __shared__ uint32_t cum[257];
  if (threadIdx.x == 0) {
    uint32_t c = 0;
    for (int s = 0; s < 256; s++) {
      cum[s] = c;
      c += (uint32_t)in[16 + 2 * s] | (uint32_t)in[17 + 2 * s] << 8;
    }
    cum[256] = c;
    if (c != kDM && blockIdx.x == 0) atomicOr(S.err, kDErrCorrupt);
  }
  __syncthreads();
  if (cum[256] != kDM) return;
  // four consecutive slots per thread, packed into one word
  const uint32_t w = blockIdx.x * kDThreads + threadIdx.x;  // < kDM / 4
  uint32_t packed = 0;
  for (uint32_t k = 0; k < 4; k++) {
    const uint32_t i = 4 * w + k;
    uint32_t lo = 0, hi = 256;  // cum[lo] <= i < cum[hi]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (cum[mid] <= i) lo = mid;
      else hi = mid;
    }
    packed |= lo << (8 * k);
  }
  S.sym[w] = packed;
}

// One block per wave: lane k finds its bytes through the block's lane sizes,
// reads its state from their first four, then per byte the slot x mod 4096
// names the byte, the state steps back and takes in bytes while it is below
// 2^23; the byte goes to the block's position k + 64 m.  Every lane must end
// on the initial state with all its bytes used, and the lanes' sizes must
// fill the block.
__global__ __launch_bounds__(kDLanes) void k_dict_decode(const uint8_t* in, uint64_t n, int bl,
                                                         uint64_t nb, DictScratch S,
                                                         uint8_t* out) {
  __shared__ uint32_t freq[256], cum[257];
  __shared__ uint32_t sym4[kDM / 4];
  const uint8_t* sym = reinterpret_cast<const uint8_t*>(sym4);
  for (int s = threadIdx.x; s < 256; s += kDLanes)
    freq[s] = (uint32_t)in[16 + 2 * s] | (uint32_t)in[17 + 2 * s] << 8;
  for (uint32_t i = threadIdx.x; i < kDM / 4; i += kDLanes) sym4[i] = S.sym[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t c = 0;
    for (int s = 0; s < 256; s++) {
      cum[s] = c;
      c += freq[s];
    }
    cum[256] = c;
  }
  __syncthreads();
  const uint64_t b = blockIdx.x;
  const uint32_t k = threadIdx.x;
  const uint64_t B = 1ull << bl;
  const uint64_t i0 = b * B, len = n - i0 < B ? n - i0 : B;
  const uint64_t bsize = S.sizes[b];
  const uint8_t* blk = in + kDHdr + 4 * nb + S.offs[b];
  if (bsize < 2 * kDLanes) {  // the whole wave sees the same size
    if (k == 0) atomicOr(S.err, kDErrCorrupt);
    return;
  }
  const uint32_t lsize = (uint32_t)blk[2 * k] | (uint32_t)blk[2 * k + 1] << 8;
  const uint32_t loff = wave_excl_sum(lsize);
  uint32_t tot = lsize;
#pragma unroll
  for (int d = kDLanes / 2; d > 0; d >>= 1) tot += (uint32_t)__shfl_xor((int)tot, d, kDLanes);
  if ((uint64_t)tot + 2 * kDLanes != bsize) {
    if (k == 0) atomicOr(S.err, kDErrCorrupt);
    return;
  }
  if (lsize < 4) {
    atomicOr(S.err, kDErrCorrupt);
    return;
  }
  const uint8_t* p = blk + 2 * kDLanes + loff;
  const uint64_t cnt = k < len ? (len - k + kDLanes - 1) / kDLanes : 0;
  uint32_t x = (uint32_t)p[0] | (uint32_t)p[1] << 8 | (uint32_t)p[2] << 16 | (uint32_t)p[3] << 24;
  uint32_t r = 4;
  for (uint64_t m = 0; m < cnt; m++) {
    const uint32_t slot = x & (kDM - 1);
    const uint32_t s = sym[slot];
    x = freq[s] * (x >> kDScale) + slot - cum[s];
    while (x < kDL) {
      if (r >= lsize) {
        atomicOr(S.err, kDErrCorrupt);
        return;
      }
      x = (x << 8) | p[r++];
    }
    out[i0 + k + kDLanes * m] = (uint8_t)s;
  }
  if (x != kDL || r != lsize) atomicOr(S.err, kDErrCorrupt);
}

lcp_status dict_args(int bl) { return bl < 12 || bl > 20 ? LCP_ERR_ARG : LCP_OK; }

}  // namespace

extern "C" {

uint64_t lcp_dict_bound(uint64_t n, int block_log2) {
  if (dict_args(block_log2)) return 0;
  const uint64_t nb = dict_blocks(n, block_log2);
  return kDHdr + 4 * nb + n + n / 2 + nb * (2 * kDLanes + 8 * kDLanes);
}

lcp_status lcp_dict_scratch_bytes(uint64_t n, int block_log2, int encode, uint64_t* device_bytes) {
  if (!device_bytes || dict_args(block_log2)) return LCP_ERR_ARG;
  *device_bytes = dict_scratch(dict_blocks(n, block_log2), block_log2, encode != 0, nullptr, nullptr);
  return LCP_OK;
}

lcp_status lcp_dict_encode(const void* in, uint64_t n, int block_log2, void* out, uint64_t out_cap,
                           void* scratch, uint64_t scratch_bytes, uint64_t* out_size,
                           hipStream_t stream) {
  if (!out_size || !out || !scratch || (n && !in) || dict_args(block_log2)) return LCP_ERR_ARG;
  if (((uintptr_t)in & 3) || ((uintptr_t)out & 3) || ((uintptr_t)scratch & 255)) return LCP_ERR_ARG;
  const uint64_t nb = dict_blocks(n, block_log2);
  if (nb > 0x7FFFFFFFull) return LCP_ERR_ARG;
  DictScratch S;
  if (dict_scratch(nb, block_log2, true, &S, static_cast<uint8_t*>(scratch)) > scratch_bytes)
    return LCP_ERR_BUDGET;
  const uint64_t bound = lcp_dict_bound(n, block_log2);
  *out_size = bound;
  // the worst case must fit: blocks are placed before their sizes are known
  if (out_cap < bound) return LCP_ERR_CAPACITY;
  uint8_t* o = static_cast<uint8_t*>(out);
  const uint8_t* src = static_cast<const uint8_t*>(in);
  k_dict_clear<<<1, kDThreads, 0, stream>>>(S);
  if (n) {
    const uint64_t hb = (n / 4 + kDThreads * 16 - 1) / (kDThreads * 16);
    k_dict_hist<<<(uint32_t)(hb < 1 ? 1 : (hb > 4096 ? 4096 : hb)), kDThreads, 0, stream>>>(src, n,
                                                                                            S);
  }
  k_dict_table<<<1, kDThreads, 0, stream>>>(n, block_log2, S, o);
  if (nb) {
    k_dict_encode<<<(uint32_t)nb, kDLanes, 0, stream>>>(src, n, block_log2, nb, S, o);
    lcp::scan_device<uint64_t>(S.offs, nb, nullptr, true, S.tmp, stream);
  }
  k_dict_total<<<1, 64, 0, stream>>>(nb, S, 0);
  if (nb)
    k_dict_gather<<<(uint32_t)((nb + kDThreads / kDLanes - 1) / (kDThreads / kDLanes)), kDThreads,
                    0, stream>>>(nb, block_log2, S, o);
  unsigned long long total = 0;
  uint32_t err = 0;
  if (hipMemcpyAsync(&total, S.total, 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemcpyAsync(&err, S.err, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return LCP_ERR_DEVICE;
  *out_size = total;
  return err ? LCP_ERR_DEVICE : LCP_OK;
}

lcp_status lcp_dict_decode(const void* in, uint64_t size, void* out, uint64_t out_cap,
                           void* scratch, uint64_t scratch_bytes, uint64_t* n_out,
                           hipStream_t stream) {
  if (!in || !n_out || !scratch || size < kDHdr || ((uintptr_t)scratch & 255))
    return LCP_ERR_ARG;
  if (size > (1ull << 40)) return LCP_ERR_ARG;
  uint32_t head[4];
  if (hipMemcpyAsync(head, in, 16, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return LCP_ERR_DEVICE;
  if (head[0] != kDMagic || dict_args((int)head[1])) return LCP_ERR_CORRUPT;
  const int bl = (int)head[1];
  const uint64_t n = (uint64_t)head[2] | (uint64_t)head[3] << 32;
  *n_out = n;
  const uint64_t nb = dict_blocks(n, bl);
  if (nb > (size - kDHdr) / 4) return LCP_ERR_CORRUPT;
  if (n > out_cap || (n && !out)) return LCP_ERR_CAPACITY;
  DictScratch S;
  if (dict_scratch(nb, bl, false, &S, static_cast<uint8_t*>(scratch)) > scratch_bytes)
    return LCP_ERR_BUDGET;
  const uint8_t* src = static_cast<const uint8_t*>(in);
  k_dict_clear<<<1, kDThreads, 0, stream>>>(S);
  // the stream's sizes (at byte offset kDHdr), copied into scratch
  if (nb && hipMemcpyAsync(S.sizes, src + kDHdr, 4 * nb, hipMemcpyDeviceToDevice, stream) != hipSuccess)
    return LCP_ERR_DEVICE;
  if (nb) {
    k_dict_widen<<<(uint32_t)((nb + kDThreads - 1) / kDThreads), kDThreads, 0, stream>>>(nb, S);
    lcp::scan_device<uint64_t>(S.offs, nb, nullptr, true, S.tmp, stream);
  }
  k_dict_total<<<1, 64, 0, stream>>>(nb, S, size);
  // an empty stream has no table (nothing to decode)
  if (nb) k_dict_slots<<<kDM / 4 / kDThreads, kDThreads, 0, stream>>>(src, S);
  uint32_t err = 0;
  if (hipMemcpyAsync(&err, S.err, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return LCP_ERR_DEVICE;
  if (err) return LCP_ERR_CORRUPT;  // blocks past the stream, or a table not summing to 4096
  if (nb)
    k_dict_decode<<<(uint32_t)nb, kDLanes, 0, stream>>>(src, n, bl, nb, S,
                                                       static_cast<uint8_t*>(out));
  if (hipMemcpyAsync(&err, S.err, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return LCP_ERR_DEVICE;
  return err ? LCP_ERR_CORRUPT : LCP_OK;
}

}  // extern "C"
