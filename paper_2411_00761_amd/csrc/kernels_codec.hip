// kernels_codec.hip -- block coding (Sec. 6.2.2, Tab. 3) on gfx950.
//
// Encode, per symbol array: histogram (LDS-privatised) -> canonical, length-
// limited Huffman code built on the device by one workgroup (leaves sorted by
// (count, symbol), two-queue merge, pointer-jumping depths) -> exact size of the
// Huffman coding (table + chunk index + chunks padded to 32-bit words) against
// fixed-length coding -> record layout -> MSB-first bit packing (one wave per
// chunk, bit offsets by wave prefix scan, bits OR-ed into an LDS chunk image,
// then written out coalesced).
// Decode: a 2^L-entry lookup table per Huffman array, one thread per chunk with
// the table in LDS; fixed-length arrays one thread per value.
#include "lcp_internal.h"

namespace lcp {

namespace {

constexpr int kThreads = 256;
constexpr int kHT = 1024;  // Huffman-build workgroup

__device__ inline uint64_t arr_len(const ArrIn& a) {
  return a.n_dev ? min((uint64_t)*a.n_dev, a.n) : a.n;
}
__device__ inline uint64_t arr_load(const ArrIn& a, uint64_t i) {
  return a.is64 ? ((const uint64_t*)a.v)[i] : (uint64_t)((const uint32_t*)a.v)[i];
}
__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = (uint32_t)__shfl_xor((int)lo, m, kWave);
  hi = (uint32_t)__shfl_xor((int)hi, m, kWave);
  return ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------------------------------ histogram
__global__ __launch_bounds__(kThreads) void k_enc_init(ArrWork* W, ArrSet set) {
  ArrWork& w = W[blockIdx.x];
  for (int j = threadIdx.x; j < kAlphabet; j += blockDim.x) w.hist[j] = 0;
  if (threadIdx.x == 0) {
    w.maxv = 0;
    w.n = 0;
  }
}

// Lanes of a wave holding the same symbol are grouped by 13 ballots (one per
// symbol bit); the lowest lane of each group adds the group's size, so a wave
// of identical symbols (e.g. zero residuals) costs one LDS atomic, not 64.
__global__ __launch_bounds__(kThreads) void k_hist(ArrSet set, ArrWork* W) {
  __shared__ uint32_t h[kAlphabet];
  const ArrIn a = set.a[blockIdx.y];
  ArrWork& w = W[blockIdx.y];
  const uint64_t n = arr_len(a);
  for (int j = threadIdx.x; j < kAlphabet; j += kThreads) h[j] = 0;
  __syncthreads();
  uint64_t mx = 0;
  const uint64_t lt = lanemask_lt();
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t base = (uint64_t)blockIdx.x * kThreads + wave_id() * kWave; base < n;
       base += stride) {
    const uint64_t i = base + lane_id();
    const bool valid = i < n;
    uint64_t v = valid ? arr_load(a, i) : 0;
    int e;
    const uint32_t sym = (uint32_t)symbol_of(v, &e);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 13; b++) {
      uint64_t bal = __ballot((sym >> b) & 1u);
      peers &= ((sym >> b) & 1u) ? bal : ~bal;
    }
    if (valid && (peers & lt) == 0) atomicAdd(&h[sym], (uint32_t)__popcll(peers));
    mx = v > mx ? v : mx;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kAlphabet; j += kThreads)
    if (h[j]) atomicAdd(&w.hist[j], h[j]);
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    uint64_t o = shfl_xor_u64(mx, d);
    mx = o > mx ? o : mx;
  }
  if (lane_id() == 0 && mx) atomicMax(&w.maxv, (unsigned long long)mx);
  if (blockIdx.x == 0 && threadIdx.x == 0) w.n = (uint32_t)n;
}

// ------------------------------------------------------------------ Huffman build
// LDS layout of the 64 KB buffer (U <= 4148 used symbols):
//   [0, 16592)      leaf weights u32 [U]        -> later depths u16 [2U-1]
//   [16592, 24888)  leaf symbols u16 [U]
//   [24888, 41480)  internal weights u32 [U-1]  -> later ancestors u16 [2U-1]
//   [41480, 58072)  parents u16 [2U-1]
//   [58080, 62228)  code lengths u8 [4148]
//   [62464, 62720)  small scratch u32 [64]
// During the sort the whole buffer holds up to 8192 u64 keys (count << 13 | symbol).
constexpr int kOffLeafSym = 16592;
constexpr int kOffInt = 24888;
constexpr int kOffParent = 41480;
constexpr int kOffLens = 58080;
constexpr int kOffMisc = 62464;

__device__ inline uint32_t block_max_u32(uint32_t v, uint32_t* misc) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, kWave));
  __syncthreads();
  if (lane_id() == 0) misc[wave_id()] = v;
  __syncthreads();
  uint32_t t = 0;
  for (int j = 0; j < (int)(blockDim.x / kWave); j++) t = max(t, misc[j]);
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kHT) void k_huffman(ArrWork* W) {
  __shared__ uint64_t sm64[8192];
  uint8_t* smb = reinterpret_cast<uint8_t*>(sm64);
  uint32_t* leafw = reinterpret_cast<uint32_t*>(smb);
  uint16_t* dist = reinterpret_cast<uint16_t*>(smb);
  uint16_t* leafsym = reinterpret_cast<uint16_t*>(smb + kOffLeafSym);
  uint32_t* intw = reinterpret_cast<uint32_t*>(smb + kOffInt);
  uint16_t* anc = reinterpret_cast<uint16_t*>(smb + kOffInt);
  uint16_t* parent = reinterpret_cast<uint16_t*>(smb + kOffParent);
  uint8_t* lens = smb + kOffLens;
  uint32_t* misc = reinterpret_cast<uint32_t*>(smb + kOffMisc);

  ArrWork& w = W[blockIdx.x];
  const int t = threadIdx.x;
  const uint32_t n = w.n;
  if (n == 0) {
    for (int s = t; s < kAlphabet; s += kHT) w.lc[s] = 0;
    if (t == 0) {
      w.U = 0;
      w.L = 0;
    }
    return;
  }
  constexpr int kPer = (kAlphabet + kHT - 1) / kHT;  // 5 symbols per thread
  uint32_t U = 0;
  for (int halvings = 0;; halvings++) {
    // ---- leaves: used symbols with their (halved) counts
    uint32_t c[kPer];
    uint32_t mine = 0;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      int s = t + kHT * j;
      uint32_t cc = s < kAlphabet ? w.hist[s] : 0u;
      for (int h = 0; h < halvings && cc; h++) cc = (cc + 1u) >> 1;
      c[j] = cc;
      mine += cc ? 1u : 0u;
    }
    // exclusive position of this thread's leaves
    uint32_t incl = wave_incl_scan(mine);
    __syncthreads();
    if (lane_id() == kWave - 1) misc[wave_id()] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int j = 0; j < kHT / kWave; j++) {
      uint32_t v = misc[j];
      if (j < wave_id()) before += v;
      total += v;
    }
    __syncthreads();
    U = total;
    uint32_t pos = before + incl - mine;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      int s = t + kHT * j;
      if (c[j]) sm64[pos++] = ((uint64_t)c[j] << 13) | (uint64_t)s;
    }
    if (U == 1) {
      __syncthreads();
      uint32_t only = (uint32_t)(sm64[0] & 0x1FFFu);
      __syncthreads();
      for (int s = t; s < kAlphabet; s += kHT) lens[s] = (uint32_t)s == only ? 1 : 0;
      __syncthreads();
      break;
    }
    uint32_t P = 2;
    while (P < U) P <<= 1;
    for (uint32_t i = U + t; i < P; i += kHT) sm64[i] = ~0ull;
    __syncthreads();
    // ---- bitonic sort of the (count, symbol) keys; all keys distinct
    for (uint32_t size = 2; size <= P; size <<= 1) {
      for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
        for (uint32_t i = t; i < P / 2; i += kHT) {
          uint32_t lo = 2 * i - (i & (stride - 1));
          uint32_t hi = lo + stride;
          bool asc = (lo & size) == 0;
          uint64_t a = sm64[lo], b = sm64[hi];
          if ((a > b) == asc) {
            sm64[lo] = b;
            sm64[hi] = a;
          }
        }
        __syncthreads();
      }
    }
    // ---- unpack leaves to weights and symbols
    uint64_t kr[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      uint32_t i = t + kHT * j;
      kr[j] = i < U ? sm64[i] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; j++) {
      uint32_t i = t + kHT * j;
      if (i < U) {
        leafw[i] = (uint32_t)(kr[j] >> 13);
        leafsym[i] = (uint16_t)(kr[j] & 0x1FFFu);
      }
    }
    __syncthreads();
    // ---- two-queue merge: leaves in sorted order, internal nodes FIFO in
    // creation order; the lighter head is taken, the leaf on a tie.
    if (t == 0) {
      uint32_t li = 0, ii = 0, nxt = 0;
      for (uint32_t step = 0; step + 1 < U; step++) {
        uint32_t node0, node1, w0, w1;
        {
          bool leaf = li < U && (ii >= nxt || leafw[li] <= intw[ii]);
          if (leaf) { node0 = li; w0 = leafw[li]; li++; }
          else { node0 = U + ii; w0 = intw[ii]; ii++; }
        }
        {
          bool leaf = li < U && (ii >= nxt || leafw[li] <= intw[ii]);
          if (leaf) { node1 = li; w1 = leafw[li]; li++; }
          else { node1 = U + ii; w1 = intw[ii]; ii++; }
        }
        intw[nxt] = w0 + w1;
        parent[node0] = (uint16_t)(U + nxt);
        parent[node1] = (uint16_t)(U + nxt);
        nxt++;
      }
    }
    __syncthreads();
    // ---- depths by pointer jumping (13 rounds cover any depth < 8192)
    const uint32_t nodes = 2 * U - 1, root = 2 * U - 2;
    {
      uint16_t av[9], dv[9];
#pragma unroll
      for (int j = 0; j < 9; j++) {
        uint32_t i = t + kHT * j;
        av[j] = i < nodes ? (i == root ? (uint16_t)root : parent[i]) : 0;
        dv[j] = (i < nodes && i != root) ? 1 : 0;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 9; j++) {
        uint32_t i = t + kHT * j;
        if (i < nodes) {
          anc[i] = av[j];
          dist[i] = dv[j];
        }
      }
      __syncthreads();
    }
    for (int it = 0; it < 13; it++) {
      uint16_t av[9], dv[9];
#pragma unroll
      for (int j = 0; j < 9; j++) {
        uint32_t i = t + kHT * j;
        if (i < nodes) {
          uint16_t a = anc[i];
          dv[j] = (uint16_t)(dist[i] + dist[a]);
          av[j] = anc[a];
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 9; j++) {
        uint32_t i = t + kHT * j;
        if (i < nodes) {
          anc[i] = av[j];
          dist[i] = dv[j];
        }
      }
      __syncthreads();
    }
    uint32_t md = 0;
#pragma unroll
    for (int j = 0; j < 5; j++) {
      uint32_t i = t + kHT * j;
      if (i < U) md = max(md, (uint32_t)dist[i]);
    }
    md = block_max_u32(md, misc);
    if (md <= (uint32_t)kMaxLen) {
      for (int s = t; s < kAlphabet; s += kHT) lens[s] = 0;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 5; j++) {
        uint32_t i = t + kHT * j;
        if (i < U) lens[leafsym[i]] = (uint8_t)dist[i];
      }
      __syncthreads();
      break;
    }
    __syncthreads();
  }
  // ---- canonical codes: shorter first, then by symbol (RFC 1951 order)
  uint32_t* wcnt = reinterpret_cast<uint32_t*>(smb);  // [16 waves][16]
  uint32_t* blc = misc;                               // [16] code-length counts
  uint32_t* first = misc + 16;                        // [16] first code per length
  uint32_t* run = misc + 32;                          // [16] codes given so far / table size
  if (t < 48) misc[t] = 0;
  __syncthreads();
  uint32_t lmax = 0;
  for (int s = t; s < kAlphabet; s += kHT) {
    uint32_t l = lens[s];
    if (l) atomicAdd(&blc[l], 1u);
    lmax = max(lmax, l);
  }
  __syncthreads();
  if (t == 0) {
    uint32_t code = 0;
    for (int l = 1; l <= kMaxLen; l++) {
      code = (code + blc[l - 1]) << 1;
      first[l] = code;
    }
  }
  lmax = block_max_u32(lmax, misc + 48);
  const uint64_t lt = lanemask_lt();
  for (int slab = 0; slab * kHT < kAlphabet; slab++) {
    const int s = slab * kHT + t;
    const uint32_t l = s < kAlphabet ? lens[s] : 0u;
    uint32_t rank = 0, urank = 0;
    for (uint32_t L = 1; L <= (uint32_t)kMaxLen; L++) {
      uint64_t m = __ballot(l == L);
      if (l == L) rank = (uint32_t)__popcll(m & lt);
      if (lane_id() == 0) wcnt[wave_id() * 16 + L] = (uint32_t)__popcll(m);
    }
    {
      uint64_t m = __ballot(l != 0);
      urank = (uint32_t)__popcll(m & lt);
      if (lane_id() == 0) wcnt[wave_id() * 16 + 0] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (s < kAlphabet) {
      if (l) {
        uint32_t r = run[l] + rank, u = run[0] + urank;
        for (int j = 0; j < wave_id(); j++) {
          r += wcnt[j * 16 + l];
          u += wcnt[j * 16 + 0];
        }
        w.lc[s] = (first[l] + r) | (l << 16);
        w.table[u] = (uint32_t)s | (l << 16);
      } else {
        w.lc[s] = 0;
      }
    }
    __syncthreads();
    if (t < 14) {
      uint32_t add = 0;
      for (int j = 0; j < kHT / kWave; j++) add += wcnt[j * 16 + t];
      run[t] += add;
    }
    __syncthreads();
  }
  if (t == 0) {
    w.U = run[0];
    w.L = lmax;
  }
}

// ------------------------------------------------------------------ chunk sizes
__global__ __launch_bounds__(kThreads) void k_chunk_bits(ArrSet set, const ArrWork* W,
                                                         int chunk_log2, uint32_t* cw,
                                                         uint64_t max_chunks) {
  const int a = blockIdx.y;
  const ArrIn in = set.a[a];
  const ArrWork& w = W[a];
  const uint64_t n = w.n;
  const uint64_t C = 1ull << chunk_log2;
  const uint64_t nchunks = (n + C - 1) >> chunk_log2;
  const uint64_t c = (uint64_t)blockIdx.x * (kThreads / kWave) + wave_id();
  if (c >= nchunks || w.U == 0) return;
  const uint64_t end = min(n, (c + 1) * C);
  uint32_t bits = 0;
  for (uint64_t i = c * C + lane_id(); i < end; i += kWave) {
    int e;
    int sym = symbol_of(arr_load(in, i), &e);
    bits += (w.lc[sym] >> 16) + (uint32_t)e;
  }
  bits = wave_sum(bits);
  if (lane_id() == 0) cw[(uint64_t)a * max_chunks + c] = (bits + 31u) >> 5;
}

// Inclusive scan of one array's chunk word counts (one workgroup per array).
__global__ __launch_bounds__(kHT) void k_chunk_scan(ArrWork* W, int chunk_log2, uint32_t* cw,
                                                    uint64_t max_chunks) {
  __shared__ uint32_t sm[kHT / kWave + 1];
  const int a = blockIdx.x;
  ArrWork& w = W[a];
  const uint64_t n = w.n;
  const uint64_t nchunks = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  uint32_t* p = cw + (uint64_t)a * max_chunks;
  uint64_t carry = 0;
  if (w.U != 0) {
    for (uint64_t base = 0; base < nchunks; base += (uint64_t)kHT * 4) {
      uint32_t v[4], loc = 0;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        uint64_t i = base + (uint64_t)threadIdx.x * 4 + j;
        v[j] = i < nchunks ? p[i] : 0u;
        loc += v[j];
      }
      uint32_t tot;
      uint32_t inc = block_incl_scan(loc, sm, &tot);
      uint64_t r = carry + inc - loc;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        uint64_t i = base + (uint64_t)threadIdx.x * 4 + j;
        r += v[j];
        if (i < nchunks) p[i] = (uint32_t)r;
      }
      carry += tot;
    }
  }
  if (threadIdx.x == 0) {
    w.nchunks = (uint32_t)nchunks;
    w.huff_words = carry;
  }
}

// ------------------------------------------------------------------ layout
__device__ inline void put32(uint8_t* base, uint64_t off, uint32_t v) {
  *reinterpret_cast<uint32_t*>(base + off) = v;
}
__device__ inline void put64(uint8_t* base, uint64_t off, uint64_t v) {
  put32(base, off, (uint32_t)v);
  put32(base, off + 4, (uint32_t)(v >> 32));
}

// Chooses each array's coder (the shorter; a tie keeps fixed length), places
// the arrays and writes header, grids and directory.
__global__ void k_layout(ArrWork* W, RecHdr h, const uint32_t* B_dev, uint8_t* out,
                         uint64_t cap, unsigned long long* size_dev, uint32_t* err) {
  if (threadIdx.x != 0) return;
  const int A = h.A;
  uint64_t off = (uint64_t)kHdrBytes + 8ull * h.F + (uint64_t)kDirBytes * A;
  const uint64_t hdr = off;
  for (int a = 0; a < A; a++) {
    ArrWork& w = W[a];
    uint64_t n = w.n;
    int wd = bitwidth64(w.maxv);
    uint64_t fixed = 4 * ((n * (uint64_t)wd + 31) / 32);
    uint64_t huff = 4ull * w.U + 4ull * w.nchunks + 4ull * w.huff_words;
    bool use_h = w.U != 0 && huff < fixed;
    w.coder = use_h ? 1u : 0u;
    w.w = (uint32_t)wd;
    w.nbytes = use_h ? huff : fixed;
    w.off = off;
    off += w.nbytes;
  }
  *size_dev = off;
  if (off > cap) {
    atomicOr(err, kErrCapacity);
    return;
  }
  for (uint64_t o = 0; o < hdr; o += 4) put32(out, o, 0u);
  put32(out, 0, kMagic);
  put32(out, 4, (uint32_t)kVersion | ((uint32_t)h.mode << 16) | ((uint32_t)h.F << 24));
  put32(out, 8, (uint32_t)h.k | ((uint32_t)h.chunk_log2 << 8) | ((uint32_t)A << 16));
  put32(out, 12, (uint32_t)hdr);
  put64(out, 16, h.n);
  put64(out, 24, h.mode == 0 ? (uint64_t)*B_dev : 0ull);
  put64(out, 32, off);
  for (int d = 0; d < 3; d++) put32(out, 40 + 4 * d, h.bn[d]);
  put64(out, 56, h.seq);
  put64(out, 64, h.ref_seq);
  for (int f = 0; f < h.F; f++) {
    put32(out, kHdrBytes + 8 * f, __float_as_uint(h.m[f]));
    put32(out, kHdrBytes + 8 * f + 4, __float_as_uint(h.eb_q[f]));
  }
  for (int a = 0; a < A; a++) {
    const ArrWork& w = W[a];
    uint64_t d = (uint64_t)kHdrBytes + 8ull * h.F + (uint64_t)kDirBytes * a;
    uint32_t param = w.coder ? w.L : w.w;
    put32(out, d, w.coder | (param << 8));
    put32(out, d + 4, w.coder ? w.U : 0u);
    put64(out, d + 8, w.n);
    put64(out, d + 16, w.off);
    put64(out, d + 24, w.nbytes);
  }
}

// ------------------------------------------------------------------ packing
__global__ __launch_bounds__(kThreads) void k_pack_fixed(ArrSet set, const ArrWork* W,
                                                         uint8_t* out, const uint32_t* err) {
  const int a = blockIdx.y;
  const ArrWork& w = W[a];
  if (w.coder != 0 || w.w == 0 || (*err & kErrCapacity)) return;
  const ArrIn in = set.a[a];
  const uint64_t n = w.n, wd = w.w;
  const uint64_t nwords = (n * wd + 31) / 32;
  uint32_t* dst = reinterpret_cast<uint32_t*>(out + w.off);
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x; j < nwords; j += stride) {
    const uint64_t bit0 = 32 * j;
    const uint64_t i0 = bit0 / wd;
    uint64_t i1 = (bit0 + 31) / wd;
    if (i1 > n - 1) i1 = n - 1;
    uint32_t word = 0;
    for (uint64_t i = i0; i <= i1; i++) {
      const uint64_t pos = i * wd;
      const uint64_t lo = pos > bit0 ? pos : bit0;
      const uint64_t hi = min(pos + wd, bit0 + 32);
      if (lo >= hi) continue;
      const uint64_t nb = hi - lo;
      const uint64_t v = arr_load(in, i);
      const uint64_t part = (v >> (pos + wd - hi)) & (nb >= 32 ? 0xFFFFFFFFull : ((1ull << nb) - 1));
      word |= (uint32_t)(part << (bit0 + 32 - hi));
    }
    dst[j] = word;
  }
}

__device__ inline void put_bits_lds(uint32_t* buf, uint32_t pos, uint64_t val, int nbits) {
  while (nbits > 0) {
    uint32_t wi = pos >> 5, o = pos & 31u;
    int room = 32 - (int)o;
    int take = nbits < room ? nbits : room;
    uint32_t part = (uint32_t)((val >> (nbits - take)) & ((1ull << take) - 1));
    atomicOr(&buf[wi], part << (room - take));
    pos += (uint32_t)take;
    nbits -= take;
  }
}

// One wave per chunk; the chunk's words are assembled in LDS.
__global__ void k_pack_huff(ArrSet set, const ArrWork* W, int chunk_log2, const uint32_t* cw,
                            uint64_t max_chunks, uint32_t max_words, uint8_t* out,
                            const uint32_t* err) {
  extern __shared__ uint32_t lds[];
  const int a = blockIdx.y;
  const ArrWork& w = W[a];
  if (w.coder != 1 || (*err & kErrCapacity)) return;
  const ArrIn in = set.a[a];
  const uint64_t n = w.n, nchunks = w.nchunks, U = w.U;
  uint32_t* tab = reinterpret_cast<uint32_t*>(out + w.off);
  uint32_t* offs = tab + U;
  uint32_t* payload = offs + nchunks;
  const uint32_t* ce = cw + (uint64_t)a * max_chunks;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t gstride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = gid; j < U; j += gstride) tab[j] = w.table[j];
  for (uint64_t c = gid; c < nchunks; c += gstride) offs[c] = ce[c];

  const int waves = (int)(blockDim.x / kWave);
  const uint64_t c = (uint64_t)blockIdx.x * waves + wave_id();
  const bool active = c < nchunks;
  const uint32_t wbeg = active ? (c ? ce[c - 1] : 0u) : 0u;
  const uint32_t nw = active ? ce[c] - wbeg : 0u;
  uint32_t* buf = lds + (uint64_t)wave_id() * max_words;
  const bool fits = nw <= max_words;
  for (uint32_t j = lane_id(); j < nw && fits; j += kWave) buf[j] = 0;
  __syncthreads();
  if (active && fits) {
    const uint64_t C = 1ull << chunk_log2;
    const uint64_t end = min(n, (c + 1) * C);
    uint32_t run = 0;
    for (uint64_t i0 = c * C; i0 < end; i0 += kWave) {
      const uint64_t i = i0 + lane_id();
      const bool valid = i < end;
      uint64_t v = valid ? arr_load(in, i) : 0;
      int e;
      int sym = symbol_of(v, &e);
      uint32_t lc = valid ? w.lc[sym] : 0u;
      uint32_t len = lc >> 16;
      uint32_t bits = valid ? len + (uint32_t)e : 0u;
      uint32_t incl = wave_incl_scan(bits);
      uint32_t pos = run + incl - bits;
      run += (uint32_t)__shfl((int)incl, kWave - 1, kWave);
      if (valid) {
        put_bits_lds(buf, pos, lc & 0xFFFFu, (int)len);
        if (e) put_bits_lds(buf, pos + len, v - (1ull << e), e);
      }
    }
  }
  __syncthreads();
  for (uint32_t j = lane_id(); j < nw && fits; j += kWave) payload[wbeg + j] = buf[j];
}

// ------------------------------------------------------------------ decode
// Every array of every record in a call is described by a DecArr in device
// memory.  Workgroups are assigned to arrays through a prefix of per-array
// workgroup counts (binary search), so one launch decodes all arrays of all
// frames: the entropy decoding of a batch does not depend on the reference
// chain, only the reconstruction that follows does.
__device__ inline uint32_t array_of_block(const uint32_t* prefix, int A, uint32_t b) {
  int lo = 0, hi = A - 1;  // largest a with prefix[a] <= b
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return (uint32_t)lo;
}

__global__ __launch_bounds__(kHT) void k_lut(const DecArr* arrs, uint32_t* lut_all, uint32_t* err) {
  __shared__ uint32_t wcnt[kHT / kWave * 16];
  __shared__ uint32_t misc[64];
  const int a = blockIdx.x;
  const DecArr d = arrs[a];
  if (d.coder != 1) return;
  const int t = threadIdx.x;
  const uint32_t U = d.used;
  const int L = d.param;
  uint32_t* lut = lut_all + (uint64_t)a * (1u << kMaxLen);
  if (L < 1 || L > kMaxLen || U < 1 || U > (uint32_t)kAlphabet) {
    if (t == 0) atomicOr(err, kErrCorrupt);
    return;
  }
  const uint32_t* tab = reinterpret_cast<const uint32_t*>(d.data);
  for (uint32_t i = t; i < (1u << L); i += kHT) lut[i] = 0;
  if (t < 64) misc[t] = 0;
  __syncthreads();
  uint32_t* blc = misc;  // [16]
  uint32_t* first = misc + 16;
  uint32_t* run = misc + 32;
  uint32_t* flags = misc + 48;  // [0] malformed entry, [1] has length L, [2] Kraft sum
  for (uint32_t j = t; j < U; j += kHT) {
    uint32_t e = tab[j];
    uint32_t sy = e & 0xFFFFu, l = (e >> 16) & 0xFFu;
    bool bad = (e >> 24) != 0 || sy >= (uint32_t)kAlphabet || l < 1 || l > (uint32_t)L ||
               (j > 0 && (tab[j - 1] & 0xFFFFu) >= sy);
    if (bad) atomicOr(&flags[0], 1u);
    else {
      atomicAdd(&blc[l], 1u);
      atomicAdd(&flags[2], 1u << (L - l));
      if (l == (uint32_t)L) flags[1] = 1u;
    }
  }
  __syncthreads();
  if (flags[0] || !flags[1] || flags[2] > (1u << L)) {
    if (t == 0) atomicOr(err, kErrCorrupt);
    return;
  }
  if (t == 0) {
    uint32_t code = 0;
    for (int l = 1; l <= kMaxLen; l++) {
      code = (code + blc[l - 1]) << 1;
      first[l] = code;
    }
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  for (uint32_t slab = 0; slab * kHT < U; slab++) {
    const uint32_t j = slab * kHT + t;
    const uint32_t e = j < U ? tab[j] : 0u;
    const uint32_t l = (e >> 16) & 0xFFu;
    uint32_t rank = 0;
    for (uint32_t q = 1; q <= (uint32_t)kMaxLen; q++) {
      uint64_t m = __ballot(l == q);
      if (l == q) rank = (uint32_t)__popcll(m & lt);
      if (lane_id() == 0) wcnt[wave_id() * 16 + q] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (j < U) {
      uint32_t r = run[l] + rank;
      for (int w2 = 0; w2 < wave_id(); w2++) r += wcnt[w2 * 16 + l];
      uint32_t code = first[l] + r;
      if (code < (1u << l)) {
        uint32_t span = 1u << (L - l), start = code << (L - l);
        uint32_t entry = (e & 0xFFFFu) | (l << 16);
        for (uint32_t q = 0; q < span; q++) lut[start + q] = entry;
      } else {
        atomicOr(err, kErrCorrupt);
      }
    }
    __syncthreads();
    if (t >= 1 && t <= kMaxLen) {
      uint32_t add = 0;
      for (int w2 = 0; w2 < kHT / kWave; w2++) add += wcnt[w2 * 16 + t];
      run[t] += add;
    }
    __syncthreads();
  }
}

__device__ inline bool store_value(const DecArr& d, uint64_t i, uint64_t v) {
  if (v >= d.limit) return false;
  switch (d.mode) {
    case 0: reinterpret_cast<uint64_t*>(d.out)[i] = v; break;
    case 1: reinterpret_cast<uint64_t*>(d.out)[i] = (uint64_t)unzigzag64(v); break;
    case 2: reinterpret_cast<uint32_t*>(d.out)[i] = (uint32_t)v; break;
    default: reinterpret_cast<uint32_t*>(d.out)[i] = (uint32_t)(int32_t)unzigzag64(v); break;
  }
  return true;
}

// One thread per chunk; the array's lookup table is staged in LDS.
__global__ __launch_bounds__(kThreads) void k_decode_huff(const DecArr* arrs,
                                                          const uint32_t* prefix, int A,
                                                          int chunk_log2,
                                                          const uint32_t* lut_all,
                                                          uint32_t* err) {
  __shared__ uint32_t lut[1u << kMaxLen];
  const uint32_t a = array_of_block(prefix, A, blockIdx.x);
  const DecArr d = arrs[a];
  if (d.coder != 1 || d.param < 1 || d.param > kMaxLen || (*err & kErrCorrupt)) return;
  const int L = d.param;
  const uint32_t* src = lut_all + (uint64_t)a * (1u << kMaxLen);
  for (uint32_t i = threadIdx.x; i < (1u << L); i += kThreads) lut[i] = src[i];
  __syncthreads();
  const uint64_t C = 1ull << chunk_log2;
  const uint64_t nchunks = (d.n + C - 1) >> chunk_log2;
  const uint64_t c = (uint64_t)(blockIdx.x - prefix[a]) * kThreads + threadIdx.x;
  if (c >= nchunks) return;
  const uint32_t* offs = reinterpret_cast<const uint32_t*>(d.data) + d.used;
  const uint32_t* payload = offs + nchunks;
  const uint64_t payload_words = d.nbytes / 4 - d.used - nchunks;
  const uint64_t wbeg = c ? offs[c - 1] : 0, wend = offs[c];
  if (wbeg > wend || wend > payload_words || (c == nchunks - 1 && wend != payload_words)) {
    atomicOr(err, kErrCorrupt);
    return;
  }
  uint64_t buf = 0;
  int nb = 0;
  uint64_t wp = wbeg;
  const uint64_t end = min(d.n, (c + 1) * C);
  for (uint64_t i = c * C; i < end; i++) {
    while (nb <= 32 && wp < wend) {
      buf |= (uint64_t)payload[wp] << (32 - nb);
      wp++;
      nb += 32;
    }
    const uint32_t e = lut[(uint32_t)(buf >> (64 - L))];
    const int l = (int)((e >> 16) & 0xFFu);
    if (l == 0 || l > nb) {
      atomicOr(err, kErrCorrupt);
      return;
    }
    const uint32_t sym = e & 0xFFFFu;
    buf <<= l;
    nb -= l;
    uint64_t v = sym;
    if (sym >= (uint32_t)kDirect) {
      const int eb = (int)sym - kDirect + kFirstClassBits - 1;
      uint64_t x = 0;
      int rem = eb;
      while (rem > 0) {
        while (nb <= 32 && wp < wend) {
          buf |= (uint64_t)payload[wp] << (32 - nb);
          wp++;
          nb += 32;
        }
        const int take = rem < 32 ? rem : 32;
        if (take > nb) {
          atomicOr(err, kErrCorrupt);
          return;
        }
        x = (x << take) | (buf >> (64 - take));
        buf <<= take;
        nb -= take;
        rem -= take;
      }
      v = (1ull << eb) + x;
    }
    if (!store_value(d, i, v)) {
      atomicOr(err, kErrCorrupt);
      return;
    }
  }
}

constexpr int kFixedPerBlock = kThreads * 4;

__global__ __launch_bounds__(kThreads) void k_decode_fixed(const DecArr* arrs,
                                                           const uint32_t* prefix, int A,
                                                           uint32_t* err) {
  const uint32_t a = array_of_block(prefix, A, blockIdx.x);
  const DecArr d = arrs[a];
  if (d.coder != 0) return;
  const uint64_t w = (uint64_t)d.param;
  const uint64_t nwords = (d.n * w + 31) / 32;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(d.data);
  const uint64_t i0 = (uint64_t)(blockIdx.x - prefix[a]) * kFixedPerBlock;
  for (uint64_t i = i0 + threadIdx.x; i < d.n && i < i0 + kFixedPerBlock; i += kThreads) {
    uint64_t v = 0;
    if (w) {
      const uint64_t pos = i * w, w0 = pos >> 5;
      const uint32_t o = (uint32_t)(pos & 31);
      const uint64_t a0 = src[w0];
      const uint64_t a1 = w0 + 1 < nwords ? src[w0 + 1] : 0;
      const uint64_t a2 = w0 + 2 < nwords ? src[w0 + 2] : 0;
      uint64_t t = ((a0 << 32) | a1) << o;
      if (o) t |= a2 >> (32 - o);
      v = w == 64 ? t : t >> (64 - w);
    }
    if (!store_value(d, i, v)) atomicOr(err, kErrCorrupt);
  }
}

inline uint32_t gclamp(uint64_t g, uint32_t cap) {
  if (g < 1) g = 1;
  return (uint32_t)(g > cap ? cap : g);
}

}  // namespace

void launch_encode(const ArrSet& set, uint64_t max_n, int chunk_log2, ArrWork* work,
                   uint32_t* chunk_words, uint64_t max_chunks, const RecHdr& h,
                   const uint32_t* B_dev, uint8_t* out, uint64_t cap,
                   unsigned long long* size_dev, uint32_t* err, hipStream_t s) {
  const int A = set.A;
  k_enc_init<<<A, kThreads, 0, s>>>(work, set);
  {
    dim3 g(gclamp((max_n + 4 * kThreads - 1) / (4 * kThreads), 512), A);
    LCP_TIMED("hist", max_n * 4ull * A, s, k_hist<<<g, kThreads, 0, s>>>(set, work));
  }
  k_huffman<<<A, kHT, 0, s>>>(work);
  const uint64_t chunks = (max_n + (1ull << chunk_log2) - 1) >> chunk_log2;
  {
    dim3 g(gclamp((chunks + 3) / 4, 1u << 30), A);
    k_chunk_bits<<<g, kThreads, 0, s>>>(set, work, chunk_log2, chunk_words, max_chunks);
  }
  k_chunk_scan<<<A, kHT, 0, s>>>(work, chunk_log2, chunk_words, max_chunks);
  k_layout<<<1, 64, 0, s>>>(work, h, B_dev, out, cap, size_dev, err);
  {
    const uint64_t max_words = (max_n * 64 + 31) / 32;
    dim3 g(gclamp((max_words + kThreads - 1) / kThreads, 1u << 16), A);
    LCP_TIMED("pack_fixed", max_n * 6ull * A, s,
              k_pack_fixed<<<g, kThreads, 0, s>>>(set, work, out, err));
  }
  {
    const uint32_t C = 1u << chunk_log2;
    const uint32_t max_words = (C * (kMaxLen + 63) + 31) / 32 + 1;
    int waves = (int)((64 * 1024) / (max_words * 4));
    if (waves > 4) waves = 4;
    if (waves < 1) waves = 1;
    dim3 g(gclamp((chunks + waves - 1) / waves, 1u << 30), A);
    LCP_TIMED("pack_huff", max_n * 6ull * A, s,
              k_pack_huff<<<g, waves * kWave, (size_t)waves * max_words * 4, s>>>(
                  set, work, chunk_log2, chunk_words, max_chunks, max_words, out, err));
  }
}

uint32_t decode_blocks(const DecArr& d, int chunk_log2, bool huff) {
  if (huff) {
    if (d.coder != 1) return 0;
    uint64_t nchunks = (d.n + (1ull << chunk_log2) - 1) >> chunk_log2;
    return (uint32_t)((nchunks + kThreads - 1) / kThreads);
  }
  if (d.coder != 0) return 0;
  return (uint32_t)((d.n + kFixedPerBlock - 1) / kFixedPerBlock);
}

void launch_decode(const DecArr* arrs_dev, int A, const uint32_t* huff_prefix_dev,
                   uint32_t huff_blocks, const uint32_t* fixed_prefix_dev, uint32_t fixed_blocks,
                   int chunk_log2, uint64_t bytes, uint32_t* lut, uint32_t* err, hipStream_t s) {
  if (A == 0) return;
  k_lut<<<A, kHT, 0, s>>>(arrs_dev, lut, err);
  if (huff_blocks)
    LCP_TIMED("decode_huff", bytes, s,
              k_decode_huff<<<huff_blocks, kThreads, 0, s>>>(arrs_dev, huff_prefix_dev, A,
                                                            chunk_log2, lut, err));
  if (fixed_blocks)
    LCP_TIMED("decode_fixed", bytes, s,
              k_decode_fixed<<<fixed_blocks, kThreads, 0, s>>>(arrs_dev, fixed_prefix_dev, A, err));
}

}  // namespace lcp
