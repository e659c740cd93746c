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
typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));

// Byte arrays (temporal residuals, mode 4) with codes of at most kMW bits
// also get a table of kMW-bit windows: the bytes of up to six leading codes
// whose values are small (residuals -8..7) and the bits they take.  It sits
// in the array's slot of the lookup tables, after the 2^kMaxLen-entry area's
// first kMOff words (the 32-bit table of such an array has at most 2^kMW).
constexpr int kMW = 10;
constexpr uint32_t kMOff = 4096;
static_assert((1u << kMW) <= kMOff && kMOff + 2 * (1u << kMW) <= (1u << kMaxLen), "window table fits");

__device__ inline uint64_t arr_len(const ArrIn& a) {
  return a.n_dev ? min((uint64_t)*a.n_dev, a.n) : a.n;
}
__device__ inline uint64_t arr_load(const ArrIn& a, uint64_t i) {
  if (a.esc) {
    const uint32_t b = ((const uint8_t*)a.v)[i];
    return b == 255u ? a.esc[i] : b;
  }
  return a.is64 ? ((const uint64_t*)a.v)[i] : (uint64_t)((const uint32_t*)a.v)[i];
}
__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = (uint32_t)__shfl_xor((int)lo, m, kWave);
  hi = (uint32_t)__shfl_xor((int)hi, m, kWave);
  return ((uint64_t)hi << 32) | lo;
}

// LDS accesses of this wave issued so far are complete; a compiler barrier too.
__device__ inline void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Array of workgroup b: the largest a < A with prefix[a] <= b.
__device__ inline uint32_t array_of_block(const uint32_t* prefix, int A, uint32_t b) {
  int lo = 0, hi = A - 1;  // largest a with prefix[a] <= b
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return (uint32_t)lo;
}
// The same for A <= 8 with the prefixes read together (one round of loads, not
// a chain): the number of a in [1, A) with prefix[a] <= b.
__device__ inline uint32_t array_of_block_few(const uint32_t* prefix, int A, uint32_t b) {
  if (A > 8) return array_of_block(prefix, A, b);
  uint32_t a = 0;
#pragma unroll
  for (int i = 1; i < 8; i++) a += (i < A && prefix[i] <= b) ? 1u : 0u;
  return a;
}

// ------------------------------------------------------------------ histogram
// Each workgroup counts its share of one array in LDS (wave_hist_add: the
// wave's most common case, the first lane's symbol, in one update, the other
// lanes by LDS atomics), symbols below kPrivBins in a private histogram per
// wave and the rest in the workgroup's shared one, then adds the non-zero bins
// up to its largest value's symbol into one of the array's spread copies in
// global memory; k_huff_build sums the copies.
constexpr int kPrivBins = 256;
constexpr int kHistVals = 8;  // values per lane per iteration, loads issued together

__device__ inline int sym_bound(unsigned long long mx) {
  int e;
  return symbol_of(mx, &e);
}

__global__ __launch_bounds__(kThreads) void k_hist(const EncArr* E, const uint32_t* pre, int NA,
                                                   uint32_t* part, unsigned long long* part_max) {
  __shared__ uint32_t h[kAlphabet];
  __shared__ uint32_t hpriv[kThreads / kWave][kPrivBins];
  __shared__ unsigned long long smax[kThreads / kWave];
  const uint32_t ai = array_of_block(pre, NA, blockIdx.x);
  const EncArr& e = E[ai];
  const uint32_t lb = blockIdx.x - pre[ai], nb = pre[ai + 1] - pre[ai];
  const ArrIn a = e.in;
  const uint64_t n = arr_len(a);
  for (int j = threadIdx.x; j < kAlphabet; j += kThreads) h[j] = 0;
  for (int j = threadIdx.x; j < kPrivBins * (kThreads / kWave); j += kThreads) (&hpriv[0][0])[j] = 0;
  __syncthreads();
  uint32_t* hp = hpriv[wave_id()];
  uint64_t mx = 0;
  const uint64_t stride = (uint64_t)nb * kThreads * kHistVals;
  for (uint64_t base = ((uint64_t)lb * kThreads + wave_id() * kWave) * kHistVals; base < n;
       base += stride) {
    uint64_t v[kHistVals];
#pragma unroll
    for (int j = 0; j < kHistVals; j++) {
      const uint64_t i = base + (uint64_t)j * kWave + lane_id();
      v[j] = i < n ? arr_load(a, i) : 0;
    }
#pragma unroll
    for (int j = 0; j < kHistVals; j++) {
      int ex;
      const bool valid = base + (uint64_t)j * kWave + lane_id() < n;
      wave_hist_add(h, hp, kPrivBins, (uint32_t)symbol_of(v[j], &ex), valid);
      mx = v[j] > mx ? v[j] : mx;
    }
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    uint64_t o = shfl_xor_u64(mx, d);
    mx = o > mx ? o : mx;
  }
  if (lane_id() == 0) smax[wave_id()] = mx;
  __syncthreads();
  unsigned long long bm = 0;
  for (int w = 0; w < kThreads / kWave; w++) bm = smax[w] > bm ? smax[w] : bm;
  const int top = sym_bound(bm);
  // add the non-zero bins into one of the array's spread copies (few
  // workgroups share an address, so the atomics do not queue)
  const uint32_t copy = e.copy0 + lb % e.copies;
  uint32_t* dst = part + (uint64_t)copy * kAlphabet;
  for (int j = threadIdx.x; j <= top; j += kThreads) {
    uint32_t t = h[j];
    if (j < kPrivBins)
      for (int w = 0; w < kThreads / kWave; w++) t += hpriv[w][j];
    if (t) atomicAdd(&dst[j], t);
  }
  if (threadIdx.x == 0 && bm) atomicMax(&part_max[copy], bm);
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

// Code lengths from this thread's counts c[j] (symbols t + kHT * j): one
// Huffman build.  Leaves are the used symbols sorted by (count, symbol)
// (bitonic sort), merged by one thread with two queues (leaves in order,
// internal nodes FIFO, the lighter head first and the leaf on a tie), depths
// by pointer jumping.  The lengths go to lens_g (global) and to LDS at
// kOffLens; returns the longest code (block-uniform).
constexpr int kPer = (kAlphabet + kHT - 1) / kHT;  // 5 symbols per thread
constexpr int kHalvings = 32;  // counts < 2^31: after 31 halvings every count is 1

__device__ uint32_t huff_build(const uint32_t* c, int nsym, uint8_t* smb, uint8_t* lens_g) {
  uint64_t* sm64 = reinterpret_cast<uint64_t*>(smb);
  uint32_t* leafw = reinterpret_cast<uint32_t*>(smb);
  uint16_t* dist = reinterpret_cast<uint16_t*>(smb);
  uint16_t* leafsym = reinterpret_cast<uint16_t*>(smb + kOffLeafSym);
  uint32_t* intw = reinterpret_cast<uint32_t*>(smb + kOffInt);
  uint16_t* anc = reinterpret_cast<uint16_t*>(smb + kOffInt);
  uint16_t* parent = reinterpret_cast<uint16_t*>(smb + kOffParent);
  uint8_t* lens_l = smb + kOffLens;
  uint32_t* misc = reinterpret_cast<uint32_t*>(smb + kOffMisc);
  const int t = threadIdx.x;
  // ---- leaves: used symbols with their counts
  uint32_t mine = 0;
#pragma unroll
  for (int j = 0; j < kPer; j++) mine += c[j] ? 1u : 0u;
  uint32_t incl = wave_incl_scan(mine);
  __syncthreads();
  if (lane_id() == kWave - 1) misc[wave_id()] = incl;
  __syncthreads();
  uint32_t before = 0, U = 0;
  for (int j = 0; j < kHT / kWave; j++) {
    uint32_t v = misc[j];
    if (j < wave_id()) before += v;
    U += v;
  }
  __syncthreads();
  uint32_t pos = before + incl - mine;
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    int s = t + kHT * j;
    if (c[j]) sm64[pos++] = ((uint64_t)c[j] << 13) | (uint64_t)s;
  }
  __syncthreads();
  if (U == 1) {
    uint32_t only = (uint32_t)(sm64[0] & 0x1FFFu);
    __syncthreads();
    for (int s = t; s < nsym; s += kHT) {
      const uint8_t l = (uint32_t)s == only ? 1 : 0;
      lens_g[s] = l;
      lens_l[s] = l;
    }
    __syncthreads();
    return 1;
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
        uint64_t x = sm64[lo], y = sm64[hi];
        if ((x > y) == asc) {
          sm64[lo] = y;
          sm64[hi] = x;
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
  // ---- two-queue merge; the four candidates of a step are loaded together, a
  // missing one reads as +inf
  if (t == 0) {
    constexpr uint32_t kInf = 0xFFFFFFFFu;
    uint32_t li = 0, ii = 0, nxt = 0;
    for (uint32_t step = 0; step + 1 < U; step++) {
      const uint32_t L0 = li < U ? leafw[li] : kInf;
      const uint32_t L1 = li + 1 < U ? leafw[li + 1] : kInf;
      const uint32_t I0 = ii < nxt ? intw[ii] : kInf;
      const uint32_t I1 = ii + 1 < nxt ? intw[ii + 1] : kInf;
      uint32_t node0, node1, w0, w1, lh, ih;
      if (L0 <= I0) {
        node0 = li++;
        w0 = L0;
        lh = L1;
        ih = I0;
      } else {
        node0 = U + ii++;
        w0 = I0;
        lh = L0;
        ih = I1;
      }
      if (lh <= ih) {
        node1 = li++;
        w1 = lh;
      } else {
        node1 = U + ii++;
        w1 = ih;
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
        uint16_t an = anc[i];
        dv[j] = (uint16_t)(dist[i] + dist[an]);
        av[j] = anc[an];
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
  for (int s = t; s < nsym; s += kHT) {
    lens_g[s] = 0;
    lens_l[s] = 0;
  }
  __syncthreads();
  uint32_t md = 0;
#pragma unroll
  for (int j = 0; j < 5; j++) {
    uint32_t i = t + kHT * j;
    if (i < U) {
      md = max(md, (uint32_t)dist[i]);
      const uint8_t l = (uint8_t)(dist[i] > 255 ? 255 : dist[i]);
      lens_g[leafsym[i]] = l;
      lens_l[leafsym[i]] = l;
    }
  }
  md = block_max_u32(md, misc);
  return md;
}

// Canonical codes from code lengths in LDS: shorter first, ties by symbol
// (RFC 1951 order), and the table of used symbols; returns the number of used
// symbols.  wcnt: kHT / kWave * 16 u32 and misc: 64 u32 of LDS scratch.
__device__ uint32_t huff_codes(ArrWork& w, int nsym, const uint8_t* lens, uint32_t* wcnt,
                               uint32_t* misc) {
  const int t = threadIdx.x;
  uint32_t* blc = misc;        // [16] code-length counts
  uint32_t* first = misc + 16; // [16] first code per length
  uint32_t* run = misc + 32;   // [16] codes given so far / table size
  __syncthreads();
  if (t < 48) misc[t] = 0;
  __syncthreads();
  uint32_t lmax = 0;
  for (int s = t; s < nsym; s += kHT) {
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
  for (int slab = 0; slab * kHT < nsym; slab++) {
    const int s = slab * kHT + t;
    const uint32_t l = s < nsym ? lens[s] : 0u;
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
    if (s < nsym) {
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
  const uint32_t U = run[0];
  if (t == 0) {
    w.U = U;
    w.L = lmax;
  }
  return U;
}

__device__ inline void empty_codes(ArrWork& w) {
  if (threadIdx.x == 0) {
    w.U = 0;
    w.L = 0;
  }
}

// Code of an array whose symbols are all below 64 (temporal residuals, short
// arrays), built by one wave without barriers: lane s holds symbol s's count;
// the leaves are sorted by (count, symbol) with a lane bitonic sort, the
// two-queue merge runs with wave-uniform indices over node values kept in
// registers (readlane / writelane), depths are assigned in reverse creation
// order, and the canonical codes come from a second lane sort by (length,
// symbol).  Same lengths and codes as the workgroup build.  Counts are halved
// (c -> ceil(c / 2)) until the longest code fits.  Writes lc, table, U, L;
// returns this lane's symbol's code length.
__device__ inline uint32_t lane_u32(uint32_t v, uint32_t l);

// Lane i receives the i-th smallest key of the lanes in `used` (their keys
// distinct), lanes from popc(used) on the other lanes' keys in lane order.
// Each used lane's rank counts the used keys below its own, taken one lane at
// a time by broadcast (used lanes are few: no shuffle network), and the keys
// are placed by rank through the wave's 64-entry LDS scratch.
__device__ inline uint64_t lane_sort_used(uint64_t key, uint64_t used, uint64_t* scratch) {
  const uint32_t lane = (uint32_t)lane_id();
  uint32_t r = 0;
  for (uint64_t m = used; m; m &= m - 1) {
    const uint32_t j = (uint32_t)__builtin_ctzll(m);
    const uint64_t kj = ((uint64_t)lane_u32((uint32_t)(key >> 32), j) << 32) | lane_u32((uint32_t)key, j);
    r += kj < key ? 1u : 0u;
  }
  const uint32_t U = (uint32_t)__popcll(used);
  const uint32_t rank = (used >> lane) & 1 ? r : U + (uint32_t)__popcll(~used & lanemask_lt());
  scratch[rank] = key;
  wave_lds_sync();
  const uint64_t out = scratch[lane];
  wave_lds_sync();
  return out;
}

__device__ inline uint32_t lane_u32(uint32_t v, uint32_t l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}

// Lengths of one wave's code with `h` halvings (c -> ceil(c / 2), h times) of
// lane s's count; returns the longest, sets this lane's length (0 if unused).
__device__ uint32_t small_lengths(uint32_t count, int h, uint32_t* len_out, uint64_t* scratch) {
  const uint32_t lane = (uint32_t)lane_id();
  const uint64_t used = __ballot(count != 0);
  const uint32_t U = (uint32_t)__popcll(used);
  if (U == 1) {
    *len_out = count ? 1u : 0u;
    return 1;
  }
  uint32_t c = count;
  for (int j = 0; j < h && c > 1; j++) c = (c + 1u) >> 1;
  // leaves in (count, symbol) order; unused symbols sort last
  const uint64_t key = lane_sort_used(c ? (((uint64_t)c << 13) | lane) : ~0ull, used, scratch);
  const uint32_t lw = (uint32_t)(key >> 13);   // leaf weight (lane i = leaf i)
  const uint32_t ls = (uint32_t)(key & 0x1FFFu);
  uint32_t iw = 0;     // internal node weights (lane k = internal node k)
  uint32_t lpar = 0;   // parent of leaf i (a node id: internal k is U + k)
  uint32_t ipar = 0;   // parent of internal node k
  uint32_t li = 0, ii = 0;
  constexpr uint32_t kInf = 0xFFFFFFFFu;
  for (uint32_t nxt = 0; nxt + 1 < U; nxt++) {
    const uint32_t L0 = li < U ? lane_u32(lw, li) : kInf;
    const uint32_t L1 = li + 1 < U ? lane_u32(lw, li + 1) : kInf;
    const uint32_t I0 = ii < nxt ? lane_u32(iw, ii) : kInf;
    const uint32_t I1 = ii + 1 < nxt ? lane_u32(iw, ii + 1) : kInf;
    uint32_t node0, node1, w0, w1, lh, ih;
    if (L0 <= I0) {
      node0 = li++;
      w0 = L0;
      lh = L1;
      ih = I0;
    } else {
      node0 = U + ii++;
      w0 = I0;
      lh = L0;
      ih = I1;
    }
    if (lh <= ih) {
      node1 = li++;
      w1 = lh;
    } else {
      node1 = U + ii++;
      w1 = ih;
    }
    if (lane == nxt) iw = w0 + w1;
    if (node0 < U) {
      if (lane == node0) lpar = U + nxt;
    } else if (lane == node0 - U) {
      ipar = U + nxt;
    }
    if (node1 < U) {
      if (lane == node1) lpar = U + nxt;
    } else if (lane == node1 - U) {
      ipar = U + nxt;
    }
  }
  // depths: the root (internal U - 2) is 0; parents are created after
  // their children
  uint32_t idep = 0;
  for (int k = (int)U - 3; k >= 0; k--) {
    const uint32_t p = lane_u32(ipar, (uint32_t)k) - U;
    const uint32_t d = lane_u32(idep, p) + 1;
    if (lane == (uint32_t)k) idep = d;
  }
  // (every lane takes part in the shuffle; only leaves keep the result)
  const uint32_t pd = (uint32_t)__shfl((int)idep, lane < U ? (int)(lpar - U) : 0, kWave);
  const uint32_t ldep = lane < U ? pd + 1 : 0;
  uint32_t md = ldep;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) md = max(md, (uint32_t)__shfl_xor((int)md, d, kWave));
  // lengths back to symbol lanes: leaf i carries symbol ls
  uint32_t* s32 = reinterpret_cast<uint32_t*>(scratch);
  s32[lane] = 0;
  wave_lds_sync();
  if (lane < U) s32[ls] = ldep;
  wave_lds_sync();
  *len_out = s32[lane];
  wave_lds_sync();
  return md;
}

// Canonical codes of one wave's lengths (shorter first, ties by symbol);
// writes lc, table, U, L and the depth md.
__device__ void small_codes(ArrWork& w, uint32_t count, uint32_t len, uint32_t md,
                            uint32_t* maxd_out) {
  const uint32_t lane = (uint32_t)lane_id();
  const uint64_t used = __ballot(count != 0);
  const uint32_t U = (uint32_t)__popcll(used);
  uint32_t first = 0, before = 0;
  {
    uint32_t code = 0;
    for (uint32_t l = 1; l <= (uint32_t)kMaxLen; l++) {
      const uint32_t prev = l > 1 ? (uint32_t)__popcll(__ballot(len == l - 1)) : 0u;
      code = (code + prev) << 1;
      if (len == l) first = code;
    }
  }
  const uint64_t lt = lanemask_lt();
  for (uint32_t l = 1; l <= (uint32_t)kMaxLen; l++) {
    const uint64_t m = __ballot(len == l);
    if (len == l) before = (uint32_t)__popcll(m & lt);
  }
  uint32_t lmax = len;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) lmax = max(lmax, (uint32_t)__shfl_xor((int)lmax, d, kWave));
  if (count) {
    w.lc[lane] = (first + before) | (len << 16);
    w.table[(uint32_t)__popcll(used & lt)] = lane | (len << 16);
  }
  if (lane == 0) {
    w.U = U;
    w.L = lmax;
    *maxd_out = md;
  }
}

// ------------------------------------------------------------------ Huffman size
// After the code is built: the exact code + raw bits of all the array's
// symbols (chunk padding aside) bound the Huffman coding from below.  When that
// bound is not below the fixed-length size, fixed length wins and the array is
// never packed as Huffman; otherwise it is a candidate, packed with its word
// total starting from zero.
__device__ inline int extra_bits(int s) { return s >= kDirect ? s - kDirect + kFirstClassBits - 1 : 0; }

__device__ inline uint32_t huff_candidate(uint32_t U, uint64_t n, uint64_t maxv,
                                          unsigned long long bits, int chunk_log2) {
  const uint64_t nchunks = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  const uint64_t lower = 4ull * U + 4ull * nchunks + 4ull * ((bits + 31) / 32);
  const uint64_t fixed = 4ull * ((n * (uint64_t)bitwidth64(maxv) + 31) / 32);
  return (U != 0 && lower < fixed) ? 1u : 0u;
}

// All kHT threads: `part` is this thread's share of the bits; U the number of
// used symbols, n and maxv the array's length and largest value.
__device__ void finish_block(ArrWork& w, unsigned long long part, uint32_t U, uint64_t n,
                             uint64_t maxv, int chunk_log2, unsigned long long* red) {
  __syncthreads();
  if (threadIdx.x == 0) red[0] = 0;
  __syncthreads();
  atomicAdd(red, part);
  __syncthreads();
  const unsigned long long bits = red[0];
  if (threadIdx.x == 0) {
    w.huff_bits = bits;
    w.cand = huff_candidate(U, n, maxv, bits, chunk_log2);
    w.nchunks = (uint32_t)((n + (1ull << chunk_log2) - 1) >> chunk_log2);
  }
  if (threadIdx.x < kWordParts) w.huff_words[threadIdx.x] = 0;
}

// One wave (the small-alphabet path): `part` is this lane's share.
__device__ void finish_wave(ArrWork& w, unsigned long long part, uint32_t U, uint64_t n,
                            uint64_t maxv, int chunk_log2) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) part += shfl_xor_u64(part, d);
  if (lane_id() == 0) {
    w.huff_bits = part;
    w.cand = huff_candidate(U, n, maxv, part, chunk_log2);
    w.nchunks = (uint32_t)((n + (1ull << chunk_log2) - 1) >> chunk_log2);
  }
  if (lane_id() < kWordParts) w.huff_words[lane_id()] = 0;
}

// One array per workgroup: sums its spread histogram copies (only the bins up
// to the largest value's symbol can be non-zero) and clears them, then builds
// the code: by one wave when every symbol is below 64, else by the workgroup
// with no halving, and with inline halvings when `inline_halve` is set (short
// alphabets, as temporal residuals have).  maxd_all[a][0] tells the fallback
// launches (candidate halvings side by side) whether they are needed.
__global__ __launch_bounds__(kHT) void k_huff_build(const EncArr* E, uint32_t* part,
                                                    unsigned long long* part_max, ArrWork* W,
                                                    uint8_t* lens_all, uint32_t* maxd_all,
                                                    int inline_halve, int chunk_log2) {
  __shared__ uint64_t sm64[8192];
  __shared__ unsigned long long smx[kHT / kWave];
  __shared__ unsigned long long red[1];
  uint8_t* smb = reinterpret_cast<uint8_t*>(sm64);
  const int a = blockIdx.x, t = threadIdx.x;
  ArrWork& w = W[a];
  // the array's fields, read once: the stores below could alias them, and
  // each reread would wait for all loads in flight
  const uint32_t copies = E[a].copies, copy0 = E[a].copy0;
  const uint64_t n = arr_len(E[a].in);
  // largest value over the copies (and clear them)
  unsigned long long mx = 0;
  for (uint32_t c = t; c < copies; c += kHT) {
    const unsigned long long v = part_max[copy0 + c];
    mx = v > mx ? v : mx;
    part_max[copy0 + c] = 0;
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    const unsigned long long o = shfl_xor_u64(mx, d);
    mx = o > mx ? o : mx;
  }
  if (lane_id() == 0) smx[wave_id()] = mx;
  __syncthreads();
  mx = 0;
  for (int j = 0; j < kHT / kWave; j++) mx = smx[j] > mx ? smx[j] : mx;
  const int top = n ? sym_bound(mx) : -1;
  // only symbols up to the largest value's can occur; every loop below stops
  // there (entries past it are never read)
  const int nsym = top + 1;
  uint32_t cnt[kPer];
  uint32_t* src = part + (uint64_t)copy0 * kAlphabet;
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const int s = t + kHT * j;
    uint32_t v = 0;
    if (s < nsym) {
      uint32_t x[kHistCopies];
#pragma unroll
      for (int c = 0; c < kHistCopies; c++)
        x[c] = (uint32_t)c < copies ? src[(uint64_t)c * kAlphabet + s] : 0u;
#pragma unroll
      for (int c = 0; c < kHistCopies; c++) {
        v += x[c];
        if ((uint32_t)c < copies) src[(uint64_t)c * kAlphabet + s] = 0;
      }
      w.hist[s] = v;
    }
    cnt[j] = v;
  }
  if (t == 0) {
    w.maxv = mx;
    w.n = (uint32_t)n;
  }
  uint32_t* maxd = maxd_all + (uint64_t)a * kHalvings;
  if (n == 0) {
    empty_codes(w);
    if (t == 0) {
      maxd[0] = 0;
      w.cand = 0;
    }
    return;
  }
  if (nsym <= kWave) {
    // wave h tries h halvings, side by side; the fewest that fit win (the
    // result of halving one step at a time)
    __shared__ uint32_t s_cnt[kWave], s_md[kHT / kWave];
    if (wave_id() == 0) s_cnt[lane_id()] = cnt[0];
    __syncthreads();
    const uint32_t c = s_cnt[lane_id()];
    uint32_t len;
    uint64_t* scratch = sm64 + wave_id() * kWave;  // the small path leaves sm64 free
    const uint32_t md = small_lengths(c, wave_id(), &len, scratch);
    if (lane_id() == 0) s_md[wave_id()] = md;
    __syncthreads();
    int pick = -1;
    for (int h = 0; h < kHT / kWave && pick < 0; h++)
      if (s_md[h] <= (uint32_t)kMaxLen) pick = h;
    if (pick < 0 && wave_id() == 0) {  // more halvings than waves: one at a time
      uint32_t mdh = kMaxLen + 1;
      for (int h = kHT / kWave; h < kHalvings && mdh > (uint32_t)kMaxLen; h++)
        mdh = small_lengths(c, h, &len, scratch);
      small_codes(w, c, len, mdh, maxd);
      finish_wave(w, (unsigned long long)c * len, (uint32_t)__popcll(__ballot(c != 0)), n, mx,
                  chunk_log2);
    } else if (wave_id() == pick) {
      small_codes(w, c, len, md, maxd);
      finish_wave(w, (unsigned long long)c * len, (uint32_t)__popcll(__ballot(c != 0)), n, mx,
                  chunk_log2);
    }
    return;
  }
  uint32_t orig[kPer];
#pragma unroll
  for (int j = 0; j < kPer; j++) orig[j] = cnt[j];
  uint32_t md = huff_build(cnt, nsym, smb, lens_all + (uint64_t)a * kHalvings * kAlphabet);
  for (int h = 1; inline_halve && md > (uint32_t)kMaxLen && h < kHalvings; h++) {
#pragma unroll
    for (int j = 0; j < kPer; j++) cnt[j] = cnt[j] > 1 ? (cnt[j] + 1u) >> 1 : cnt[j];
    md = huff_build(cnt, nsym, smb, lens_all + (uint64_t)a * kHalvings * kAlphabet);
  }
  if (t == 0) maxd[0] = md;
  if (md > (uint32_t)kMaxLen) return;
  const uint32_t U = huff_codes(w, nsym, smb + kOffLens, reinterpret_cast<uint32_t*>(smb),
                                reinterpret_cast<uint32_t*>(smb + kOffMisc));
  unsigned long long part_bits = 0;
  const uint8_t* lens_l = smb + kOffLens;
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const int s = t + kHT * j;
    if (s < nsym) part_bits += (unsigned long long)orig[j] * (lens_l[s] + extra_bits(s));
  }
  finish_block(w, part_bits, U, n, mx, chunk_log2, red);
}

// Fallback for arrays whose plain build is too deep (the oracle's loop halves
// the counts, c -> ceil(c / 2), until the longest code fits): workgroup (a, h)
// builds with h = blockIdx.y + h0 halvings, candidates side by side.
// A launch builds the candidates from h0 halvings on; one from h0 > 1 skips
// the arrays for which fewer halvings already fit (the pick below never reads
// past the first count that fits, so those entries need not be written).
constexpr int kFirstHalvings = 8;  // candidates built first; the rest only when none fits
// Below this many candidate workgroups (arrays x 31) all are built in one launch.
constexpr uint64_t kOneLaunchCandidates = 1024;

__global__ __launch_bounds__(kHT) void k_huff_lengths(const ArrWork* W, uint8_t* lens_all,
                                                      uint32_t* maxd_all, int h0) {
  __shared__ uint64_t sm64[8192];
  const int a = blockIdx.x, halvings = blockIdx.y + h0;
  if (maxd_all[(uint64_t)a * kHalvings] <= (uint32_t)kMaxLen) return;
  for (int h = 1; h < h0; h++)
    if (maxd_all[(uint64_t)a * kHalvings + h] <= (uint32_t)kMaxLen) return;
  const ArrWork& w = W[a];
  const int t = threadIdx.x;
  const int nsym = sym_bound(w.maxv) + 1;
  uint32_t c[kPer];
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    int s = t + kHT * j;
    uint32_t cc = s < nsym ? w.hist[s] : 0u;
    for (int h = 0; h < halvings && cc > 1; h++) cc = (cc + 1u) >> 1;
    c[j] = cc;
  }
  const uint32_t md = huff_build(c, nsym, reinterpret_cast<uint8_t*>(sm64),
                                 lens_all + ((uint64_t)a * kHalvings + halvings) * kAlphabet);
  if (t == 0) maxd_all[(uint64_t)a * kHalvings + halvings] = md;
}

// Fallback codes: the fewest halvings whose longest code fits (31 always fit).
__global__ __launch_bounds__(kHT) void k_huff_codes(const EncArr* E, ArrWork* W,
                                                    const uint8_t* lens_all,
                                                    const uint32_t* maxd_all, int chunk_log2) {
  __shared__ uint8_t lens[kAlphabet];
  __shared__ uint32_t wcnt[kHT / kWave * 16];
  __shared__ uint32_t misc[64];
  __shared__ unsigned long long red[1];
  const int a = blockIdx.x;
  if (maxd_all[(uint64_t)a * kHalvings] <= (uint32_t)kMaxLen) return;
  ArrWork& w = W[a];
  int hsel = kHalvings - 1;
  for (int h = 1; h < kHalvings - 1; h++)
    if (maxd_all[(uint64_t)a * kHalvings + h] <= (uint32_t)kMaxLen) {
      hsel = h;
      break;
    }
  const int nsym = sym_bound(w.maxv) + 1;
  const uint8_t* src = lens_all + ((uint64_t)a * kHalvings + hsel) * kAlphabet;
  for (int s = threadIdx.x; s < nsym; s += kHT) lens[s] = src[s];
  const uint32_t U = huff_codes(w, nsym, lens, wcnt, misc);
  unsigned long long part_bits = 0;
  for (int s = threadIdx.x; s < nsym; s += kHT)
    part_bits += (unsigned long long)w.hist[s] * (lens[s] + extra_bits(s));
  finish_block(w, part_bits, U, w.n, w.maxv, chunk_log2, red);
}

// ------------------------------------------------------------------ chunk sizes
// One workgroup per chunk; thread t holds the chunk's symbols [t*r, t*r + r)
// with r = C / 256 (at least 1), loaded together.
constexpr int kMaxRun = 16;  // chunk_log2 <= 12

// The array's code table in LDS, up to its largest value's symbol (no symbol
// above it occurs).
__device__ inline void load_codes(const ArrWork& w, uint32_t* lc_lds) {
  const int nsym = sym_bound(w.maxv) + 1;
  for (int j = threadIdx.x; j < nsym; j += blockDim.x) lc_lds[j] = w.lc[j];
}

// Thread t's run of chunk c: values [c*C + t*run, ...) of an array of T.
// Past the run's end the loads repeat the array's last value (n >= 1): they
// are unconditional, so they stay in flight until first used, and callers
// mask them.  Global (not flat) loads, so that waiting for LDS does not wait
// for them.
template <int RUN, typename T>
__device__ inline void load_run(const void* v, uint64_t n, int chunk_log2, uint64_t run,
                                uint32_t c, uint64_t* vals) {
  const uint64_t cend = min(n, (uint64_t)(c + 1) << chunk_log2);
  const uint64_t i0 = min(cend, ((uint64_t)c << chunk_log2) + threadIdx.x * run);
  const uint64_t last = n - 1;
  const __attribute__((address_space(1))) T* p = (const __attribute__((address_space(1))) T*)v;
#pragma unroll
  for (int j = 0; j < RUN; j++) vals[j] = (uint64_t)p[min(i0 + j, last)];
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS accesses
// (global loads stay in flight across it) and for the other waves.  The
// memory clobber keeps the compiler from moving accesses across it.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Inclusive workgroup scan with LDS-only barriers; every thread reads the
// per-wave totals itself.  `sm` (kThreads / kWave words) must not be written
// again before another barrier.
__device__ inline uint32_t block_scan_lds(uint32_t v, uint32_t* sm, uint32_t* total) {
  const uint32_t x = wave_incl_scan(v);
  if (lane_id() == kWave - 1) sm[wave_id()] = x;
  lds_barrier();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / kWave; w++) {
    const uint32_t t = sm[w];
    before += w < wave_id() ? t : 0u;
    tot += t;
  }
  *total = tot;
  return x + before;
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
// the arrays, sizes the records and places them back to back (from *base_dev
// when given), then writes each header, grid and directory that fits in the
// output, with NT threads.
// Records are taken NT / kMaxArrays at a time: thread j reads record j's
// header, thread (j, a) = (t / kMaxArrays, t % kMaxArrays) reads and decides
// array a of record j, record threads turn the array sizes into offsets, and a
// workgroup scan of the record sizes places the records.  Each phase is one
// round of independent loads.  Every record size is a multiple of 4 bytes.
template <int NT>
constexpr size_t layout_lds_bytes() {
  return 8 * (NT / kWave + 1) + 8 * (NT / kMaxArrays) * (kMaxArrays + 2) + 12 * (NT / kMaxArrays);
}

__device__ inline void write_header(const RecHdr& h, uint64_t B, uint64_t size, uint8_t* out) {
  const uint64_t hdr = (uint64_t)kHdrBytes + 8ull * h.F + (uint64_t)kDirBytes * h.A;
  put32(out, 0, kMagic);
  put32(out, 4, (uint32_t)kVersion | ((uint32_t)h.mode << 16) | ((uint32_t)h.F << 24));
  // byte 11: a temporal record's residual step (Sec. 7.4.2), 0 standing for 1
  const uint32_t step = h.scale > 1 ? (uint32_t)h.scale : 0u;
  put32(out, 8, (uint32_t)h.k | ((uint32_t)h.chunk_log2 << 8) | ((uint32_t)h.A << 16) | (step << 24));
  put32(out, 12, (uint32_t)hdr);
  put64(out, 16, h.n);
  put64(out, 24, B);
  put64(out, 32, size);
  for (int d = 0; d < 3; d++) put32(out, 40 + 4 * d, h.bn[d]);
  // byte 52: a spatial record's dimensions (3 written as 0); byte 53: the
  // fields' element type (0 float32, 1 int32); the rest reserved
  put32(out, 52, (h.mode == 0 && h.dims != 3 ? (uint32_t)h.dims : 0u) | ((uint32_t)h.dtype << 8));
  put64(out, 56, h.seq);
  put64(out, 64, h.ref_seq);
  put64(out, 72, 0ull);
#pragma unroll
  for (int f = 0; f < kMaxF; f++) {
    if (f < h.F) {
      put32(out, kHdrBytes + 8 * f, __float_as_uint(h.m[f]));
      put32(out, kHdrBytes + 8 * f + 4, __float_as_uint(h.eb_q[f]));
    }
  }
}

// An array's coder: Huffman when it is a candidate and strictly shorter than
// fixed length, which wins ties.
struct ArrChoice {
  uint32_t coder, param, U, wd;
  uint64_t n, nbytes;
};
__device__ inline ArrChoice choose_coder(const ArrWork& w) {
  ArrChoice c;
  c.n = w.n;
  const uint64_t mv = w.maxv;
  const uint32_t L = w.L, cand = w.cand, nc = w.nchunks, U = w.U;
  uint64_t hw = 0;
#pragma unroll
  for (int q = 0; q < kWordParts; q++) hw += w.huff_words[q];
  c.wd = (uint32_t)bitwidth64(mv);
  const uint64_t fixed = 4 * ((c.n * (uint64_t)c.wd + 31) / 32);
  const uint64_t huff = 4ull * U + 4ull * nc + 4ull * hw;
  const bool use_h = cand && huff < fixed;
  c.coder = use_h ? 1u : 0u;
  c.param = use_h ? L : c.wd;
  c.U = use_h ? U : 0u;
  c.nbytes = use_h ? huff : fixed;
  return c;
}

__device__ inline void write_dir(uint8_t* o, int F, int a, const ArrChoice& c, uint64_t aoff) {
  const uint64_t d = (uint64_t)kHdrBytes + 8ull * F + (uint64_t)kDirBytes * a;
  put32(o, d, c.coder | (c.param << 8));
  put32(o, d + 4, c.U);
  put64(o, d + 8, c.n);
  put64(o, d + 16, aoff);
  put64(o, d + 24, c.nbytes);
}

template <int NT>
__device__ void layout_records(ArrWork* W, EncRec* recs, const EncRec& rec0, int R, uint8_t* out,
                               uint64_t cap, unsigned long long* offs,
                               const unsigned long long* base_dev, uint32_t* err, uint8_t* lds) {
  constexpr int kLayRecs = NT / kMaxArrays;
  unsigned long long* sm = reinterpret_cast<unsigned long long*>(lds);
  unsigned long long(*s_nb)[kMaxArrays] =
      reinterpret_cast<unsigned long long(*)[kMaxArrays]>(sm + NT / kWave + 1);  // bytes, then offsets
  unsigned long long* s_roff = reinterpret_cast<unsigned long long*>(s_nb + kLayRecs);
  unsigned long long* s_size = s_roff + kLayRecs;
  uint32_t* s_a0 = reinterpret_cast<uint32_t*>(s_size + kLayRecs);
  int* s_A = reinterpret_cast<int*>(s_a0 + kLayRecs);
  int* s_F = s_A + kLayRecs;
  const int t = (int)threadIdx.x;
  const int j = t / kMaxArrays, a = t % kMaxArrays;
  unsigned long long carry = base_dev ? *base_dev : 0ull;
  for (int base = 0; base < R; base += kLayRecs) {
    const int r = base + t;
    const bool hv = t < kLayRecs && r < R;
    RecHdr h;
    uint64_t B = 0;
    if (hv) {
      const EncRec& rc = R == 1 ? rec0 : recs[r];  // a single record comes as an argument
      h = rc.h;
      s_a0[t] = rc.a0;
      s_A[t] = h.A;
      s_F[t] = h.F;
      if (h.mode == 0) B = *rc.B_dev;
    }
    __syncthreads();
    const bool av = j < kLayRecs && base + j < R && a < s_A[j];
    ArrChoice ch{};
    if (av) {
      ArrWork& w = W[s_a0[j] + a];
      ch = choose_coder(w);
      w.coder = ch.coder;
      w.w = ch.wd;
      w.nbytes = ch.nbytes;
      s_nb[j][a] = ch.nbytes;
    }
    __syncthreads();
    unsigned long long size = 0;
    if (hv) {
      uint64_t off = (uint64_t)kHdrBytes + 8ull * h.F + (uint64_t)kDirBytes * h.A;
      for (int q = 0; q < h.A; q++) {
        const unsigned long long bq = s_nb[t][q];
        s_nb[t][q] = off;
        off += bq;
      }
      size = off;
    }
    unsigned long long tot;
    const unsigned long long incl = block_incl_scan(size, sm, &tot);
    if (hv) {
      const unsigned long long roff = carry + incl - size;
      s_roff[t] = roff;
      s_size[t] = size;
      recs[r].size = size;
      recs[r].off = roff;
      offs[r] = roff;
      if (roff + size <= cap) write_header(h, B, size, out + roff);
    }
    __syncthreads();
    if (av) {
      const uint64_t aoff = s_nb[j][a];
      W[s_a0[j] + a].off = aoff;
      const unsigned long long roff = s_roff[j];
      if (roff + s_size[j] <= cap) write_dir(out + roff, s_F[j], a, ch, aoff);
    }
    carry += tot;
    __syncthreads();
  }
  if (t == 0) offs[R] = carry;
  if (carry > cap && t == 0) atomicOr(err, kErrCapacity);
}

// ------------------------------------------------------------------ packing
// Workgroup lb of the nb that pack fixed-length array a.
// Where an array goes, as the layout decided: its coder and fixed width, and
// its first byte in the output (valid when the record fits).
struct ArrPlace {
  uint32_t coder, wd;
  uint8_t* dst;
  bool fits;
};

__device__ inline void pack_fixed_block(const EncArr* E, const ArrWork* W, uint32_t a,
                                        const ArrPlace& pl, uint32_t lb, uint32_t nb) {
  if (pl.coder != 0 || pl.wd == 0 || !pl.fits) return;
  const ArrWork& w = W[a];
  const ArrIn in = E[a].in;
  const uint64_t n = w.n, wd = pl.wd;
  const uint64_t nwords = (n * wd + 31) / 32;
  uint32_t* dst = reinterpret_cast<uint32_t*>(pl.dst);
  const uint64_t stride = (uint64_t)nb * kThreads;
  for (uint64_t j = (uint64_t)lb * kThreads + threadIdx.x; j < nwords; j += stride) {
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
      const uint64_t nbits = hi - lo;
      const uint64_t v = arr_load(in, i);
      const uint64_t part = (v >> (pos + wd - hi)) & (nbits >= 32 ? 0xFFFFFFFFull : ((1ull << nbits) - 1));
      word |= (uint32_t)(part << (bit0 + 32 - hi));
    }
    dst[j] = word;
  }
}

// Bits are appended MSB-first to a 64-bit accumulator and flushed one 32-bit
// word at a time into the chunk image in LDS (OR, since the first and last word
// of a lane's run are shared with its neighbours).
struct BitSink {
  uint64_t acc;
  int accb;
  uint32_t wi;
  uint32_t* buf;
  __device__ inline void push(uint64_t val, int nb) {  // nb <= 32
    if (nb == 0) return;
    acc = (acc << nb) | val;
    accb += nb;
    if (accb >= 32) {
      atomicOr(&buf[wi], (uint32_t)(acc >> (accb - 32)));
      wi++;
      accb -= 32;
      acc &= accb ? ((1ull << accb) - 1) : 0ull;
    }
  }
  __device__ inline void flush() {
    if (accb > 0) atomicOr(&buf[wi], (uint32_t)(acc << (32 - accb)));
  }
};

// Chunks of a Huffman candidate are independent: thread t packs the t-th run
// of C/256 consecutive symbols at the bit offset given by a workgroup scan of
// the runs' lengths into the chunk's image in LDS, which goes to the chunk's
// own slot of the array's staging area (a slot holds C symbols of the longest
// code and the most extra bits, enc_slot_words).  The chunk's word count goes
// to cnt[c] and, summed per workgroup, into the array's total; where each
// chunk lands in the record is settled by the copy once all are packed, so no
// workgroup waits on another.
// Packs chunk c from its values vin (thread t's run) into the chunk's slot;
// with esc (byte arrays), a value 255 is replaced by esc at its index first.
template <int RUN>
__device__ inline void pack_chunk(uint32_t c, const uint64_t* vin, const uint32_t* esc,
                                  uint64_t n, uint64_t C, uint64_t run, const uint32_t* lc,
                                  uint32_t* buf, uint32_t* sm, uint32_t* cnta, uint32_t* pay,
                                  uint32_t slot, unsigned long long* words, uint32_t* err) {
  const uint64_t cend = min(n, (uint64_t)(c + 1) * C);
  const uint64_t i0 = min(cend, (uint64_t)c * C + threadIdx.x * run);
  const uint64_t i1 = min(cend, i0 + run);
  uint64_t v[RUN];
#pragma unroll
  for (int j = 0; j < RUN; j++) {
    v[j] = vin[j];
    if (esc && v[j] == 255u && i0 + j < i1) v[j] = esc[i0 + j];
  }
  // each value's code (code | length << 16) and raw extra bits, once
  uint32_t cl[RUN];
  int exb[RUN];
  uint32_t bits = 0, extra = 0;
#pragma unroll
  for (int j = 0; j < RUN; j++) {
    const int sym = symbol_of(v[j], &exb[j]);
    const bool in = i0 + j < i1;
    cl[j] = in ? lc[sym] : 0u;
    exb[j] = in ? exb[j] : 0;
    bits += (cl[j] >> 16) + (uint32_t)exb[j];
    extra |= (uint32_t)exb[j];
  }
  uint32_t total;
  const uint32_t start = block_scan_lds(bits, sm, &total) - bits;
  const uint32_t nw = (total + 31u) >> 5;
  // a chunk beyond its slot would mean the code and the data disagree:
  // flagged, never written
  const bool fits = nw <= slot;
  if (threadIdx.x == 0) {
    if (!fits) atomicOr(err, kErrCorrupt);
    cnta[c] = nw;
    *words += nw;
  }
  for (uint32_t j = threadIdx.x; j < nw && fits; j += kThreads) buf[j] = 0;
  lds_barrier();
  if (bits && fits) {
    if (bits <= 32 && !extra) {
      // the run's codes fit one register: placed MSB first at bit `start`,
      // they touch at most two words
      uint64_t str = 0;
#pragma unroll
      for (int j = 0; j < RUN; j++) str = (str << (cl[j] >> 16)) | (cl[j] & 0xFFFFu);
      const uint64_t part = (str << (64 - bits)) >> (start & 31u);
      const uint32_t w0 = start >> 5;
      atomicOr(&buf[w0], (uint32_t)(part >> 32));
      if ((uint32_t)part) atomicOr(&buf[w0 + 1], (uint32_t)part);
    } else {
      BitSink sk{0ull, (int)(start & 31u), start >> 5, buf};
#pragma unroll
      for (int j = 0; j < RUN; j++) {
        if (i0 + j >= i1) break;
        sk.push(cl[j] & 0xFFFFu, (int)(cl[j] >> 16));
        const int ex = exb[j];
        if (ex) {
          const uint64_t x = v[j] - (1ull << ex);
          if (ex > 32) {
            sk.push(x >> 32, ex - 32);
            sk.push(x & 0xFFFFFFFFull, 32);
          } else {
            sk.push(x, ex);
          }
        }
      }
      sk.flush();
    }
  }
  lds_barrier();
  uint32_t* dst = pay + (uint64_t)c * slot;
  for (uint32_t j = threadIdx.x; j < nw && fits; j += kThreads) dst[j] = buf[j];
  lds_barrier();
}

// The workgroup's chunks lb, lb + nb, ... of an array of T, with two value
// buffers: the next chunk's values are loaded while one is packed.
template <int RUN, typename T>
__device__ inline void pack_chunks(const void* v, const uint32_t* esc, uint64_t n, int chunk_log2,
                                   uint32_t lb, uint32_t nb, const uint32_t* lc, uint32_t* buf,
                                   uint32_t* sm, uint32_t* cnta, uint32_t* pay, uint32_t slot,
                                   unsigned long long* words, uint32_t* err) {
  const uint64_t C = 1ull << chunk_log2;
  const uint32_t nchunks = (uint32_t)((n + C - 1) >> chunk_log2);
  const uint64_t run = C >= (uint64_t)kThreads ? C / kThreads : 1;
  uint64_t va[RUN], vb[RUN];
  load_run<RUN, T>(v, n, chunk_log2, run, min(lb, nchunks - 1), va);
  for (uint32_t c = lb; c < nchunks; c += 2 * nb) {
    load_run<RUN, T>(v, n, chunk_log2, run, min(c + nb, nchunks - 1), vb);
    pack_chunk<RUN>(c, va, esc, n, C, run, lc, buf, sm, cnta, pay, slot, words, err);
    if (c + nb >= nchunks) break;
    load_run<RUN, T>(v, n, chunk_log2, run, min(c + 2 * nb, nchunks - 1), va);
    pack_chunk<RUN>(c + nb, vb, esc, n, C, run, lc, buf, sm, cnta, pay, slot, words, err);
  }
}

template <int RUN>
__global__ __launch_bounds__(kThreads) void k_pack_huff(const EncArr* E, ArrWork* W,
                                                        const uint32_t* pre, int NA,
                                                        int chunk_log2, uint32_t* cnt,
                                                        uint32_t* stage, uint32_t slot32,
                                                        uint32_t slot64, uint32_t* err) {
  extern __shared__ uint32_t buf[];
  __shared__ uint32_t sm[kThreads / kWave];
  __shared__ uint32_t lc[kAlphabet];
  const uint32_t a = array_of_block(pre, NA, blockIdx.x);
  const uint32_t lb = blockIdx.x - pre[a], nb = pre[a + 1] - pre[a];
  ArrWork& w = W[a];
  if (!w.cand) return;
  load_codes(w, lc);
  __syncthreads();
  const EncArr& e = E[a];
  const uint64_t n = w.n;
  uint32_t* cnta = cnt + e.cw0;
  uint32_t* pay = stage + e.stage0;
  unsigned long long words = 0;  // thread 0: this workgroup's share of the array
  if (e.in.esc)
    pack_chunks<RUN, uint8_t>(e.in.v, e.in.esc, n, chunk_log2, lb, nb, lc, buf, sm, cnta, pay,
                              slot32, &words, err);
  else if (e.in.is64)
    pack_chunks<RUN, uint64_t>(e.in.v, nullptr, n, chunk_log2, lb, nb, lc, buf, sm, cnta, pay,
                               slot64, &words, err);
  else
    pack_chunks<RUN, uint32_t>(e.in.v, nullptr, n, chunk_log2, lb, nb, lc, buf, sm, cnta, pay,
                               slot32, &words, err);
  if (threadIdx.x == 0 && words) atomicAdd(&w.huff_words[blockIdx.x % kWordParts], words);
}

// Byte arrays (temporal residuals, whose codes are nearly all a few bits
// long) pack one chunk per wave: lane l takes the chunk's values
// [l * RUN, l * RUN + RUN) with RUN = C / 64, the lanes' bit offsets come from
// a wave scan, and the chunk image is assembled in the wave's own LDS slot, so
// a chunk needs no workgroup barrier.  Chunk images, word counts and staging
// slots are those of k_pack_huff.
constexpr int kPackWaves = kThreads / kWave;
constexpr int kPackDepth = 4;  // whole chunks a wave has in flight
// s_waitcnt immediate for vmcnt(0) alone (gfx9 encoding: vmcnt in bits 3:0
// and 15:14, expcnt 6:4, lgkmcnt 11:8; the other counters at their maxima)
constexpr int kWaitVm0 = 0x0F70;
constexpr bool pack_by_wave(int chunk_log2) { return chunk_log2 >= 6 && chunk_log2 <= 10; }


// A lane's RUN bytes, packed four to a word (RUN < 4: one word), kept packed
// until they are coded so that a prefetched chunk costs few registers.
template <int RUN>
struct ByteRun {
  static constexpr int kWords = RUN >= 4 ? RUN / 4 : 1;
  uint32_t w[kWords];
  __device__ inline uint32_t at(int j) const { return (w[j >> 2] >> (8 * (j & 3))) & 255u; }
};

// One vector load (RUN = 4, 8 or 16; i0 + RUN <= n and v + i0 aligned to RUN
// bytes).
template <int RUN>
__device__ inline void load_bytes_vec(const uint8_t* v, uint64_t i0, ByteRun<RUN>& b) {
  if constexpr (RUN == 16) {
    typedef const __attribute__((address_space(1))) U32x4* G4;
    const U32x4 x = *(G4)(v + i0);
    b.w[0] = x[0];
    b.w[1] = x[1];
    b.w[2] = x[2];
    b.w[3] = x[3];
  } else if constexpr (RUN == 8) {
    typedef uint32_t U32x2 __attribute__((ext_vector_type(2)));
    typedef const __attribute__((address_space(1))) U32x2* G2;
    const U32x2 x = *(G2)(v + i0);
    b.w[0] = x[0];
    b.w[1] = x[1];
  } else {
    b.w[0] = *(const __attribute__((address_space(1))) uint32_t*)(v + i0);
  }
}

// One load per byte, clamped to the last value (masked later).
template <int RUN>
__device__ inline void load_bytes_clamped(const uint8_t* v, uint64_t i0, uint64_t n,
                                          ByteRun<RUN>& b) {
  const __attribute__((address_space(1))) uint8_t* p = (const __attribute__((address_space(1))) uint8_t*)v;
#pragma unroll
  for (int q = 0; q < ByteRun<RUN>::kWords; q++) b.w[q] = 0;
#pragma unroll
  for (int j = 0; j < RUN; j++) b.w[j >> 2] |= (uint32_t)p[min(i0 + j, n - 1)] << (8 * (j & 3));
}

static_assert(offsetof(ArrWork, lc) % 16 == 0 && sizeof(ArrWork) % 16 == 0,
              "an array's code table is 16-byte aligned");
// The code of symbol s as length | code << 16 (the table's halves swapped, so
// that the length is the low bits a 64-bit shift takes): the first kPackLcLds
// entries are in LDS, the rest (escaped values only) are read from the table.
constexpr int kPackLcLds = 256;
static_assert(kPackLcLds == kThreads && kAlphabet >= kPackLcLds, "one table entry per thread");
typedef const __attribute__((address_space(1))) uint32_t* GWordsIn;
__device__ inline uint32_t swap_halves(uint32_t x) { return (x >> 16) | (x << 16); }
__device__ inline uint32_t code_of(uint32_t s, const uint32_t* lc_lds, GWordsIn lc_glb) {
  return s < (uint32_t)kPackLcLds ? lc_lds[s] : swap_halves(lc_glb[s]);
}
// Non-zero iff one of the word's four bytes is 255.
__device__ inline uint32_t has_ff(uint32_t w) { return ((w & 0x7F7F7F7Fu) + 0x01010101u) & w & 0x80808080u; }

// Inclusive sum over the wave's 64 lanes with DPP row shifts and row
// broadcasts (no LDS round trips).
__device__ inline uint32_t wave_incl_sum_dpp(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

// Packs chunk c of a byte array from this lane's bytes b; returns the chunk's
// word count (written to cnta[c] by lane 0).  FULL: the chunk has all C values.
template <int RUN, bool FULL>
__device__ inline uint32_t pack_chunk_wave(uint32_t c, const ByteRun<RUN>& b, GWordsIn esc,
                                           uint64_t n, uint64_t C, const uint32_t* lc,
                                           GWordsIn lc_glb, uint32_t* buf, uint32_t* cnta,
                                           uint32_t* pay, uint32_t slot, uint32_t* err) {
  const uint32_t lane = (uint32_t)lane_id();
  const uint64_t cend = FULL ? (uint64_t)(c + 1) * C : min(n, (uint64_t)(c + 1) * C);
  const uint64_t i0 = (uint64_t)c * C + lane * RUN;
  uint32_t cl[RUN];  // length | code << 16
  uint32_t bits = 0;
  // an escaped value (byte 255) sends the lane's codes and raw bits down the
  // general path; the check is per word (unused bytes of a short run are 0)
  uint32_t ff = 0;
#pragma unroll
  for (int q = 0; q < ByteRun<RUN>::kWords; q++) ff |= has_ff(b.w[q]);
  const bool slow = ff != 0;
  if (__ballot(slow) == 0) {
#pragma unroll
    for (int j = 0; j < RUN; j++) {
      cl[j] = (FULL || i0 + j < cend) ? lc[b.at(j)] : 0u;
      bits += cl[j] & 0xFFu;
    }
  } else {
#pragma unroll
    for (int j = 0; j < RUN; j++) {
      const bool in = FULL || i0 + j < cend;
      const uint32_t bj = b.at(j);
      uint32_t code = 0;
      int ex = 0;
      if (in && bj == 255u) code = code_of((uint32_t)symbol_of(esc[i0 + j], &ex), lc, lc_glb);
      else code = lc[bj];
      cl[j] = in ? code : 0u;
      bits += (cl[j] & 0xFFu) + (uint32_t)ex;
    }
  }
  const uint32_t incl = wave_incl_sum_dpp(bits);
  const uint32_t start = incl - bits;
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
  const uint32_t nw = (total + 31u) >> 5;
  // a chunk beyond its slot would mean the code and the data disagree:
  // flagged, never written
  if (nw > slot) {
    if (lane == 0) {
      atomicOr(err, kErrCorrupt);
      cnta[c] = nw;
    }
    return nw;
  }
  for (uint32_t j = lane; j < nw; j += kWave) buf[j] = 0;
  wave_lds_sync();
  if (bits && !slow && bits <= 64) {
    // the lane's codes in one register, placed MSB first at bit `start`:
    // they touch at most three words
    uint64_t str = 0;
#pragma unroll
    for (int j = 0; j < RUN; j++) str = (str << (cl[j] & 63u)) | (cl[j] >> 16);
    const uint64_t t = str << (64 - bits);
    const uint32_t o = start & 31u, w0 = start >> 5;
    atomicOr(&buf[w0], (uint32_t)(t >> (32 + o)));
    if (o + bits > 32) atomicOr(&buf[w0 + 1], (uint32_t)(t >> o));
    if (o + bits > 64) atomicOr(&buf[w0 + 2], (uint32_t)(t << (32 - o)));
  } else if (bits) {
    BitSink sk{0ull, (int)(start & 31u), start >> 5, buf};
#pragma unroll
    for (int j = 0; j < RUN; j++) {
      if (!FULL && i0 + j >= cend) break;
      sk.push(cl[j] >> 16, (int)(cl[j] & 0xFFu));
      if (b.at(j) == 255u) {
        const uint64_t val = esc[i0 + j];
        int ex = 0;
        symbol_of(val, &ex);
        if (ex) sk.push(val - (1ull << ex), ex);  // ex <= 31: the value is 32-bit
      }
    }
    sk.flush();
  }
  wave_lds_sync();
  uint32_t* dst = pay + (uint64_t)c * slot;
  for (uint32_t j = lane; j < nw; j += kWave) dst[j] = buf[j];
  if (lane == 0) cnta[c] = nw;
  return nw;
}

// Workgroup lb of the nb packing byte array a: wave g = lb * kPackWaves + w
// takes chunks g, g + G, ... (G = nb * kPackWaves).  Whole chunks of an array
// whose bytes start 16-byte aligned load with vector loads, the next chunk's
// while one is packed; the ragged last chunk (and every chunk otherwise) loads
// byte by byte.
// With `build` (temporal records of a run) every workgroup first builds the
// array's code itself from the residual kernel's spread histogram copies, as
// the one-wave builder of k_huff_build does (wave h tries h halvings), so
// that no build launch sits between the residuals and the packing; workgroup
// 0 of the array stores what the emit needs (used-symbol table, sizes,
// candidate flag).  An array with symbols past kWave flags kErrRebuild.
template <int RUN>
__global__ __launch_bounds__(kThreads) void k_pack_wave(const EncArr* E, ArrWork* W,
                                                        const uint32_t* pre, int NA,
                                                        int chunk_log2, uint32_t* cnt,
                                                        uint32_t* stage, uint32_t slot,
                                                        uint32_t* err, const uint32_t* hpart,
                                                        const unsigned long long* hmax,
                                                        int build, uint32_t* err_rec,
                                                        int err_stride) {
  extern __shared__ uint32_t bufs[];
  __shared__ uint32_t lc[kPackLcLds];
  __shared__ unsigned long long wsum[kPackWaves];
  const uint32_t a = array_of_block_few(pre, NA, blockIdx.x);
  const uint32_t lb = blockIdx.x - pre[a], nb = pre[a + 1] - pre[a];
  ArrWork& w = W[a];
  const EncArr& e = E[a];
  // the table's first kPackLcLds entries, requested with the array's fields
  // (entries past the largest value's symbol are never looked up)
  const uint32_t lc_t = build ? 0u : ((GWordsIn)w.lc)[threadIdx.x];
  if (!build && !w.cand) return;
  const uint64_t n = build ? arr_len(e.in) : (uint64_t)w.n;
  const uint8_t* v = static_cast<const uint8_t*>(e.in.v);
  GWordsIn esc = (GWordsIn)e.in.esc;
  GWordsIn lc_glb = (GWordsIn)w.lc;
  uint32_t* cnta = cnt + e.cw0;
  uint32_t* pay = stage + e.stage0;
  // the wave index is uniform: loops over chunks stay scalar
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane(wave_id());
  uint32_t* buf = bufs + (uint64_t)wv * slot;
  const uint64_t C = 1ull << chunk_log2;
  const uint32_t nchunks = (uint32_t)((n + C - 1) >> chunk_log2);
  const uint32_t g = lb * kPackWaves + wv, G = nb * kPackWaves;
  const uint64_t lane_off = (uint64_t)lane_id() * RUN;
  const bool vec = RUN >= 4 && ((uintptr_t)v & 15u) == 0;
  const uint32_t nfull = vec ? (uint32_t)(n >> chunk_log2) : 0u;
  unsigned long long words = 0;
  // the wave's first kPackDepth whole chunks are in flight with the code
  // table's entries; later rounds load their kPackDepth chunks at once too, so
  // a round waits for memory once (the loads are unconditional, so that
  // waiting for the table's does not wait for the chunks': a wave without
  // whole chunks reads the table's words)
  ByteRun<RUN> q[kPackDepth];
  const bool deep = RUN >= 4 && g < nfull;
  if constexpr (RUN >= 4) {
    const uint8_t* src = deep ? v : reinterpret_cast<const uint8_t*>(w.lc);
#pragma unroll
    for (int k = 0; k < kPackDepth; k++)
      load_bytes_vec<RUN>(src, deep ? ((uint64_t)min(g + k * G, nfull - 1) << chunk_log2) + lane_off
                                    : lane_off,
                          q[k]);
  }
  if (build) {
    __shared__ uint32_t s_cb[kWave], s_mdb[kPackWaves], s_cand;
    __shared__ unsigned long long s_mx;
    __shared__ uint64_t s_scr[kPackWaves][kWave];
    const uint32_t copies = e.copies, copy0 = e.copy0;
    const int lane = lane_id();
    lc[threadIdx.x] = 0;  // symbols past the alphabet: never looked up
    if (wave_id() == 0) {
      // largest value over the copies; counts of symbols below kWave (bins
      // past the largest symbol are zero: every build clears what it used)
      unsigned long long m = (uint32_t)lane < copies ? hmax[copy0 + lane] : 0ull;
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) {
        const unsigned long long o = shfl_xor_u64(m, d);
        m = o > m ? o : m;
      }
      uint32_t x[kHistCopies];
#pragma unroll
      for (int c = 0; c < kHistCopies; c++)
        x[c] = (uint32_t)c < copies ? hpart[(uint64_t)(copy0 + c) * kAlphabet + lane] : 0u;
      uint32_t sum = 0;
#pragma unroll
      for (int c = 0; c < kHistCopies; c++) sum += x[c];
      s_cb[lane] = sum;
      if (lane == 0) s_mx = m;
    }
    __syncthreads();
    const unsigned long long mx = s_mx;
    if (n == 0 || sym_bound(mx) + 1 > kWave) {
      // the array is laid out as fixed length meanwhile (its fields within
      // its input) and the frame is coded again
      if (threadIdx.x == 0) {
        atomicOr(err_rec ? err_rec + (uint64_t)e.rec * err_stride : err, kErrRebuild);
        if (lb == 0) {
          w.U = 0;
          w.L = 0;
          w.maxv = mx;
          w.n = (uint32_t)n;
          w.nchunks = nchunks;
          w.huff_bits = 0;
          w.cand = 0;
        }
      }
      return;
    }
    const uint32_t c = s_cb[lane];
    uint32_t len;
    uint32_t md = small_lengths(c, wave_id(), &len, s_scr[wave_id()]);
    if (lane == 0) s_mdb[wave_id()] = md;
    __syncthreads();
    int pick = -1;
    for (int h = 0; h < kPackWaves && pick < 0; h++)
      if (s_mdb[h] <= (uint32_t)kMaxLen) pick = h;
    if (pick < 0) pick = 0;  // wave 0 goes on halving, one count at a time
    if ((int)wave_id() == pick) {
      for (int h = kPackWaves; md > (uint32_t)kMaxLen && h < kHalvings; h++)
        md = small_lengths(c, h, &len, s_scr[pick]);
      // canonical codes (shorter first, ties by symbol), as small_codes
      const uint64_t used = __ballot(c != 0);
      const uint32_t U = (uint32_t)__popcll(used);
      uint32_t first = 0, before = 0, code = 0;
      for (uint32_t l = 1; l <= (uint32_t)kMaxLen; l++) {
        const uint32_t prev = l > 1 ? (uint32_t)__popcll(__ballot(len == l - 1)) : 0u;
        code = (code + prev) << 1;
        if (len == l) first = code;
      }
      const uint64_t lt = lanemask_lt();
      for (uint32_t l = 1; l <= (uint32_t)kMaxLen; l++) {
        const uint64_t m = __ballot(len == l);
        if (len == l) before = (uint32_t)__popcll(m & lt);
      }
      uint32_t lmax = len;
      unsigned long long bits = (unsigned long long)c * len;
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) {
        lmax = max(lmax, (uint32_t)__shfl_xor((int)lmax, d, kWave));
        bits += shfl_xor_u64(bits, d);
      }
      lc[lane] = c ? (len | ((first + before) << 16)) : 0u;  // length in the low half
      const uint32_t cand = huff_candidate(U, n, mx, bits, chunk_log2);
      if (lb == 0) {
        if (c) w.table[(uint32_t)__popcll(used & lt)] = (uint32_t)lane | (len << 16);
        if (lane == 0) {
          w.U = U;
          w.L = lmax;
          w.maxv = mx;
          w.n = (uint32_t)n;
          w.nchunks = nchunks;
          w.huff_bits = bits;
          w.cand = cand;
        }
      }
      if (lane == 0) s_cand = cand;
    }
    __syncthreads();
    if (!s_cand) return;
  } else {
    lc[threadIdx.x] = swap_halves(lc_t);
  }
  __syncthreads();
  if constexpr (RUN >= 4) {
    if (deep) {
      for (uint32_t c0 = g;;) {
        // the round's chunks are in (and the last round's stores done): one
        // wait, where the compiler would otherwise wait before each chunk for
        // the stores of the one before, which share the loads' counter
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
#pragma unroll
        for (int k = 0; k < kPackDepth; k++) {
          const uint32_t c = c0 + k * G;
          if (c < nfull)
            words += pack_chunk_wave<RUN, true>(c, q[k], esc, n, C, lc, lc_glb, buf, cnta, pay,
                                                slot, err);
        }
        c0 += kPackDepth * G;
        if (c0 >= nfull) break;
#pragma unroll
        for (int k = 0; k < kPackDepth; k++)
          load_bytes_vec<RUN>(v, ((uint64_t)min(c0 + k * G, nfull - 1) << chunk_log2) + lane_off,
                              q[k]);
      }
    }
  }
  // chunks from nfull on that belong to this wave
  for (uint32_t c = nfull + (g + G - nfull % G) % G; c < nchunks; c += G) {
    ByteRun<RUN> vt;
    load_bytes_clamped<RUN>(v, ((uint64_t)c << chunk_log2) + lane_off, n, vt);
    words += pack_chunk_wave<RUN, false>(c, vt, esc, n, C, lc, lc_glb, buf, cnta, pay, slot, err);
  }
  if (lane_id() == 0) wsum[wv] = words;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
#pragma unroll
    for (int k = 0; k < kPackWaves; k++) tot += wsum[k];
    if (tot) atomicAdd(&w.huff_words[blockIdx.x % kWordParts], tot);
  }
}

__global__ __launch_bounds__(kHT) void k_layout(ArrWork* W, EncRec* recs, const EncRec rec0,
                                                int R, uint8_t* out, uint64_t cap,
                                                unsigned long long* offs,
                                                const unsigned long long* base_dev,
                                                uint32_t* err) {
  __shared__ __align__(8) uint8_t lds[layout_lds_bytes<kHT>()];
  layout_records<kHT>(W, recs, rec0, R, out, cap, offs, base_dev, err, lds);
}

// Huffman arrays the layout kept: code table, chunk end offsets and the
// payload gathered from the chunks' slots into the record.  Workgroup lb of
// the array's nb handles a contiguous range of chunks: it sums the word counts
// before its range (eight loads in flight per thread), then takes the range
// 256 chunks at a time, scanning their counts and copying their words as one
// flat range (a word finds its chunk by binary search over the tile's
// offsets), so that loads of different chunks overlap.
__device__ inline void copy_huff_block(const EncArr* E, const ArrWork* W, uint32_t a,
                                       const ArrPlace& pl, uint32_t lb, uint32_t nb,
                                       const uint32_t* cnt, const uint32_t* stage,
                                       uint32_t slot32, uint32_t slot64, const uint32_t* err) {
  __shared__ unsigned long long sm[kThreads / kWave + 1];
  __shared__ uint32_t c_end[kThreads];  // inclusive word ends inside the tile
  const ArrWork& w = W[a];
  if (pl.coder != 1 || !pl.fits || (*err & kErrCorrupt)) return;
  const EncArr& e = E[a];
  const uint32_t U = w.U, nchunks = w.nchunks;
  const uint32_t slot = e.in.is64 ? slot64 : slot32;
  uint32_t* dst = reinterpret_cast<uint32_t*>(pl.dst);
  uint32_t* dpay = dst + U + nchunks;
  const uint32_t* cnta = cnt + e.cw0;
  const uint32_t* pay = stage + e.stage0;
  if (lb == 0)
    for (uint32_t j = threadIdx.x; j < U; j += kThreads) dst[j] = w.table[j];
  const uint32_t per = (nchunks + nb - 1) / nb;
  const uint32_t c0 = min(nchunks, lb * per), c1 = min(nchunks, c0 + per);
  if (c0 >= c1) return;
  constexpr int kPf = 16;  // one round of loads covers 4096 chunks
  unsigned long long part = 0;
  for (uint32_t j0 = 0; j0 < c0; j0 += kThreads * kPf) {
    uint32_t v[kPf];
#pragma unroll
    for (int q = 0; q < kPf; q++) {
      const uint32_t j = j0 + q * kThreads + threadIdx.x;
      v[q] = j < c0 ? cnta[j] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kPf; q++) part += v[q];
  }
  unsigned long long base;
  block_incl_scan(part, sm, &base);
  for (uint32_t t0 = c0; t0 < c1; t0 += kThreads) {
    const uint32_t c = t0 + threadIdx.x;
    const uint32_t m = min((uint32_t)kThreads, c1 - t0);
    const unsigned long long k = c < c1 ? cnta[c] : 0u;
    unsigned long long tot;
    const unsigned long long incl = block_incl_scan(k, sm, &tot);
    if (c < c1) {
      dst[U + c] = (uint32_t)(base + incl);
      c_end[threadIdx.x] = (uint32_t)incl;
    }
    __syncthreads();
    // wave w copies the tile's chunks w, w + kPackWaves, ...: the first 64
    // words of kCopyAhead chunks are loaded together, longer chunks finish
    // word by word
    uint32_t* d = dpay + base;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane(wave_id()), lane = lane_id();
    constexpr int kCopyAhead = 8;
    for (uint32_t i0 = wv; i0 < m; i0 += kPackWaves * kCopyAhead) {
      uint32_t val[kCopyAhead], s0[kCopyAhead], nw[kCopyAhead];
#pragma unroll
      for (int q = 0; q < kCopyAhead; q++) {
        const uint32_t i = i0 + q * kPackWaves;
        s0[q] = i < m && i ? c_end[i - 1] : 0u;
        nw[q] = i < m ? c_end[i] - s0[q] : 0u;
        val[q] = lane < nw[q] ? pay[(uint64_t)(t0 + i) * slot + lane] : 0u;
      }
#pragma unroll
      for (int q = 0; q < kCopyAhead; q++) {
        const uint32_t i = i0 + q * kPackWaves;
        if (lane < nw[q]) d[s0[q] + lane] = val[q];
        for (uint32_t j = kWave + lane; j < nw[q]; j += kWave)
          d[s0[q] + j] = pay[(uint64_t)(t0 + i) * slot + j];
      }
    }
    base += tot;
    __syncthreads();
  }
}

// The arrays' payloads once the layout has placed them: workgroups below
// fixed_blocks pack fixed-length arrays, the rest copy Huffman arrays.
// Fixed-length arrays are packed in place and the Huffman payloads gathered
// from their staging.  A launch of one record (fold) has no layout kernel:
// every workgroup decides the record's layout itself from the arrays' sizes
// (a few loads) and workgroup 0 writes what the layout kernel would have (the
// header, the directory, the record's offsets, the coder decisions and the
// capacity error).
__global__ __launch_bounds__(kThreads) void k_emit(const EncArr* E, ArrWork* W, EncRec* recs,
                                                   const EncRec rec0, int fold,
                                                   const uint32_t* pre_fixed,
                                                   uint32_t fixed_blocks, const uint32_t* pre_copy,
                                                   int NA, const uint32_t* cnt,
                                                   const uint32_t* stage, uint32_t slot32,
                                                   uint32_t slot64, uint8_t* out, uint64_t cap,
                                                   unsigned long long* offs,
                                                   const unsigned long long* base_dev,
                                                   uint32_t* err, uint32_t* clear_part,
                                                   unsigned long long* clear_max) {
  const bool fixed = blockIdx.x < fixed_blocks;
  const uint32_t b = fixed ? blockIdx.x : blockIdx.x - fixed_blocks;
  const uint32_t* pre = fixed ? pre_fixed : pre_copy;
  const uint32_t a = array_of_block_few(pre, NA, b);
  const uint32_t lb = b - pre[a], nb = pre[a + 1] - pre[a];
  ArrPlace pl;
  if (fold) {
    __shared__ ArrChoice s_ch[kMaxArrays];
    __shared__ unsigned long long s_aoff[kMaxArrays + 1], s_roff;
    const int t = threadIdx.x, A = rec0.h.A, F = rec0.h.F;
    const unsigned long long carry = base_dev ? *base_dev : 0ull;
    if (t < A) s_ch[t] = choose_coder(W[rec0.a0 + t]);
    __syncthreads();
    if (t == 0) {
      uint64_t off = (uint64_t)kHdrBytes + 8ull * F + (uint64_t)kDirBytes * A;
      for (int q = 0; q < A; q++) {
        s_aoff[q] = off;
        off += s_ch[q].nbytes;
      }
      s_aoff[A] = off;  // the record's size
      s_roff = carry;
    }
    __syncthreads();
    const uint64_t size = s_aoff[A], roff = s_roff;
    const bool fits = roff + size <= cap;
    if (blockIdx.x == 0) {
      if (t < A) {
        ArrWork& w = W[rec0.a0 + t];
        w.coder = s_ch[t].coder;
        w.w = s_ch[t].wd;
        w.nbytes = s_ch[t].nbytes;
        w.off = s_aoff[t];
        if (fits) write_dir(out + roff, F, t, s_ch[t], s_aoff[t]);
      }
      if (t == 0) {
        recs[0].size = size;
        recs[0].off = roff;
        offs[0] = roff;
        offs[1] = roff + size;
        if (fits) write_header(rec0.h, rec0.h.mode == 0 ? *rec0.B_dev : 0ull, size, out + roff);
        else atomicOr(err, kErrCapacity);
      }
    }
    const uint32_t q = a - rec0.a0;
    pl = ArrPlace{s_ch[q].coder, s_ch[q].wd, out + roff + s_aoff[q], fits};
  } else {
    const ArrWork& w = W[a];
    pl = ArrPlace{w.coder, w.w, out + recs[E[a].rec].off + w.off, !(*err & kErrCapacity)};
  }
  // a record whose packing built its code: the histogram copies (symbols below
  // kWave, which are all it used) start from zero for the next residuals
  if (clear_part && fixed && lb == 0) {
    const uint32_t copies = E[a].copies, copy0 = E[a].copy0;
    for (uint32_t i = threadIdx.x; i < copies * kWave; i += kThreads)
      clear_part[(uint64_t)(copy0 + i / kWave) * kAlphabet + i % kWave] = 0;
    if (threadIdx.x < copies) clear_max[copy0 + threadIdx.x] = 0;
  }
  if (fixed)
    pack_fixed_block(E, W, a, pl, lb, nb);
  else
    copy_huff_block(E, W, a, pl, lb, nb, cnt, stage, slot32, slot64, err);
}

// ------------------------------------------------------------------ decode
// Every array of every record in a call is described by a DecArr in device
// memory.  Workgroups are assigned to arrays through a prefix of per-array
// workgroup counts (binary search), so one launch decodes all arrays of all
// frames: the entropy decoding of a batch does not depend on the reference
// chain, only the reconstruction that follows does.

// Lookup table of one Huffman array: entry i (an L-bit window) holds the
// symbol and length of the code that prefixes it.  The table is validated
// (ascending symbols, lengths 1..L, some code of length L, Kraft sum <= 1),
// the canonical codes are laid out in (length, symbol) order, and each of the
// 2^L entries finds its code by binary search over the codes' left-justified
// starts, so no thread fills a long run of entries.
__global__ __launch_bounds__(kHT) void k_lut(const DecArr* arrs, uint32_t* lut_all, uint32_t* err) {
  __shared__ uint32_t wcnt[kHT / kWave * 16];
  __shared__ uint32_t misc[80];
  __shared__ uint32_t cstart[kAlphabet], centry[kAlphabet];
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
  if (t < 80) misc[t] = 0;
  __syncthreads();
  uint32_t* blc = misc;  // [16] codes per length
  uint32_t* first = misc + 16;  // [16] first code per length
  uint32_t* run = misc + 32;    // [16] codes of each length placed so far
  uint32_t* flags = misc + 48;  // [0] malformed entry, [1] has length L, [2] Kraft sum
  uint32_t* cbase = misc + 64;  // [16] canonical index of each length's first code
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
    uint32_t code = 0, base = 0;
    for (int l = 1; l <= kMaxLen; l++) {
      code = (code + blc[l - 1]) << 1;
      first[l] = code;
      cbase[l] = base;
      base += blc[l];
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
      const uint32_t code = first[l] + r;
      if (code < (1u << l)) {
        cstart[cbase[l] + r] = code << (L - l);
        centry[cbase[l] + r] = (e & 0xFFFFu) | (l << 16);
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
  // codes that overflowed their length were flagged above; the starts of the
  // rest ascend in canonical order
  for (uint32_t i = t; i < (1u << L); i += kHT) {
    int lo = 0, hi = (int)U - 1;  // last code starting at or before i
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (cstart[mid] <= i) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t e = centry[lo];
    const uint32_t l = e >> 16;
    lut[i] = (cstart[lo] <= i && i - cstart[lo] < (1u << (L - l))) ? e : 0u;
  }
  if (d.mode != 4 || L > kMW) return;
  __syncthreads();  // the table above is read back
  // window x: codes taken one after another while the next L bits (zero
  // padded past the window) name a code that ends inside it and a value
  // below 16 (and the limit); their residuals as bytes, count and bits
  uint64_t* win = reinterpret_cast<uint64_t*>(lut + kMOff);
  const uint32_t lim = d.limit > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)d.limit;
  for (uint32_t x = t; x < (1u << kMW); x += kHT) {
    uint64_t bytes = 0;
    uint32_t n = 0, pos = 0;
    while (n < 6 && pos < (uint32_t)kMW) {
      const uint32_t idx = pos + L <= (uint32_t)kMW ? (x >> (kMW - pos - L)) & ((1u << L) - 1u)
                                                    : (x << (pos + L - kMW)) & ((1u << L) - 1u);
      const uint32_t e = lut[idx], l = e >> 16, sym = e & 0xFFFFu;
      if (e == 0 || l > (uint32_t)kMW - pos || sym >= 16u || sym >= lim) break;
      const int32_t r = (int32_t)unzigzag64(sym);
      bytes |= (uint64_t)(uint8_t)(int8_t)r << (8 * n);
      n++;
      pos += l;
    }
    win[x] = bytes | ((uint64_t)n << 48) | ((uint64_t)pos << 52);
  }
}

__device__ inline bool store_value(const DecArr& d, uint64_t i, uint64_t v) {
  if (v >= d.limit) return false;
  switch (d.mode) {
    case 0: reinterpret_cast<uint64_t*>(d.out)[i] = v; break;
    case 1: reinterpret_cast<uint64_t*>(d.out)[i] = (uint64_t)unzigzag64(v); break;
    case 2: reinterpret_cast<uint32_t*>(d.out)[i] = (uint32_t)v; break;
    case 4: {
      const int32_t r = (int32_t)unzigzag64(v);
      const bool small = r >= -127 && r <= 127;
      reinterpret_cast<int8_t*>(d.out)[i] = small ? (int8_t)r : (int8_t)-128;
      if (!small) d.esc[i] = r;
      break;
    }
    default: reinterpret_cast<uint32_t*>(d.out)[i] = (uint32_t)(int32_t)unzigzag64(v); break;
  }
  return true;
}

// One thread per chunk.  The array's lookup table is staged in LDS with 16-bit
// entries (length << 12 | symbol; 0 for a length-class symbol or an invalid
// window, which then take the 32-bit table in global memory).  Each thread
// decodes its chunk in rounds of kRound symbols and reads its payload through
// a ring of kRing words in LDS: every round every thread commits the K words
// it loaded in the round before into its ring (if they are the next ones and
// fit) and loads the following K, unconditionally, so those loads are waited
// for one round later, and a refill of the bit buffer only reads LDS.  No
// workgroup barrier follows the table fill: waves decode independently.  A
// ring that runs dry (a round that needs more than K words) reads the next
// word from global memory directly.  Payload reads and output stores use
// global, not flat, addressing: flat accesses also count as LDS traffic, so
// every table lookup would wait for them.
constexpr int kRound = 16;
constexpr int kRing = 16;
// Per wave: the staged payload of its 64 chunks (or the lanes' rings).
constexpr int kStageWords = 3072;  // 48 words (1536 bits) per chunk on average
constexpr int kStageBatch = 8;  // words per lane loaded together while staging
static_assert(kStageWords >= kRing * kWave, "a wave's area holds its lanes' rings");
static_assert(kThreads / kWave * kStageWords * 4 + (2 << kMaxLen) <= 65536, "decoder LDS");
constexpr int kWinLog2Max = 12;  // longest code of a launch that leaves room for windows
static_assert(kThreads / kWave * kStageWords * 4 + (2 << kWinLog2Max) + (8 << kMW) <= 65536,
              "decoder LDS with the window table");
typedef const __attribute__((address_space(1))) uint32_t* GWords;
typedef __attribute__((address_space(1))) uint64_t* GOut64;
typedef __attribute__((address_space(1))) uint32_t* GOut32;
typedef __attribute__((address_space(1))) U32x4* GOut128;

// One chunk's bits, MSB first: buf holds nb valid bits; words [rpos, wpos)
// are in the ring; cw words in the chunk.
struct RingReader {
  uint64_t buf;
  int nb;
  uint32_t rpos, wpos, cw;
  GWords pay;          // the chunk's first word
  uint32_t* ring;      // slot s of this thread at ring[s * kWave] (the wave's own area)
  __device__ inline void refill() {
    if (nb <= 32 && rpos < cw) {
      uint32_t w;
      if (rpos < wpos) {
        w = ring[(rpos & (kRing - 1)) * kWave];
      } else {
        w = pay[rpos];
        wpos = rpos + 1;
      }
      buf |= (uint64_t)w << (32 - nb);
      nb += 32;
      rpos++;
    }
  }
};

// A chunk whose payload words all sit in LDS (staged by its wave).
struct StageReader {
  uint64_t buf;
  int nb;
  uint32_t rpos, cw;
  const uint32_t* w;  // the chunk's first word in LDS
  __device__ inline void refill() {
    if (nb <= 32 && rpos < cw) {
      buf |= (uint64_t)w[rpos] << (32 - nb);
      nb += 32;
      rpos++;
    }
  }
};

// Raw bits that follow a length-class symbol (rare): up to 63 bits.
template <typename Reader>
__device__ inline bool read_extra(Reader& r, int eb, uint64_t* x) {
  uint64_t v = 0;
  int rem = eb;
  while (rem > 0) {
    r.refill();
    const int take = rem < 32 ? rem : 32;
    if (take > r.nb) return false;
    v = (v << take) | (r.buf >> (64 - take));
    r.buf <<= take;
    r.nb -= take;
    rem -= take;
  }
  *x = v;
  return true;
}

// One symbol; false on a malformed stream.  A refill leaves at least 33 bits
// unless the chunk ends, so one test covers the code itself (at most 13 bits).
template <typename Reader>
__device__ inline bool decode_symbol(Reader& r, const uint16_t* lut, const uint32_t* glut,
                                     int L, const DecArr& d, uint64_t* out) {
  if (r.nb <= 32) r.refill();
  const uint32_t win = (uint32_t)(r.buf >> (64 - L));
  const uint32_t e16 = lut ? lut[win] : 0u;
  uint32_t e = ((e16 >> 12) << 16) | (e16 & 0xFFFu);
  if (e16 == 0) e = glut[win];
  const int l = (int)(e >> 16);
  if (l == 0 || l > r.nb) return false;
  const uint32_t sym = e & 0xFFFFu;
  r.buf <<= l;
  r.nb -= l;
  uint64_t v = sym;
  if (sym >= (uint32_t)kDirect) {
    const int eb = (int)sym - kDirect + kFirstClassBits - 1;
    uint64_t x;
    if (!read_extra(r, eb, &x)) return false;
    v = (1ull << eb) + x;
  }
  if (v >= d.limit) return false;
  *out = v;
  return true;
}

template <int MODE>
__device__ inline uint64_t out_value(uint64_t v) {
  return (MODE == 1 || MODE >= 3) ? (uint64_t)unzigzag64(v) : v;
}

// Mode 4: a residual as int8, or -128 with the value kept in esc.
__device__ inline uint32_t byte_of(uint32_t r, const DecArr& d, uint64_t i) {
  const int32_t v = (int32_t)r;
  if (v >= -127 && v <= 127) return (uint32_t)(uint8_t)(int8_t)v;
  ((__attribute__((address_space(1))) int32_t*)d.esc)[i] = v;
  return 0x80u;
}

// A round's values (cnt of them from index i0) to the output array of mode
// 2..4; vec: the output is 16-byte aligned.
template <int MODE>
__device__ inline void store_round(const DecArr& d, const uint32_t* vals, int cnt, uint64_t i0,
                                   bool vec) {
  typedef __attribute__((address_space(1))) uint8_t* GOut8;
  if (MODE == 4) {
    // bytes: four values to a word, one 16-byte store per round
    uint32_t b[kRound];
#pragma unroll
    for (int j = 0; j < kRound; j++) b[j] = j < cnt ? byte_of(vals[j], d, i0 + j) : 0u;
    if (vec && cnt == kRound) {
      uint32_t wd[kRound / 4];
#pragma unroll
      for (int q = 0; q < kRound / 4; q++)
        wd[q] = b[4 * q] | (b[4 * q + 1] << 8) | (b[4 * q + 2] << 16) | (b[4 * q + 3] << 24);
      *(GOut128)((GOut8)d.out + i0) = U32x4{wd[0], wd[1], wd[2], wd[3]};
    } else {
#pragma unroll
      for (int j = 0; j < kRound; j++)
        if (j < cnt) ((GOut8)d.out)[i0 + j] = (uint8_t)b[j];
    }
  } else if (vec && cnt == kRound) {
    GOut128 o = (GOut128)((GOut32)d.out + i0);
#pragma unroll
    for (int q = 0; q < kRound / 4; q++)
      o[q] = U32x4{vals[4 * q], vals[4 * q + 1], vals[4 * q + 2], vals[4 * q + 3]};
  } else {
#pragma unroll
    for (int j = 0; j < kRound; j++)
      if (j < cnt) ((GOut32)d.out)[i0 + j] = vals[j];
  }
}

template <int MODE, int K>
__device__ inline void decode_chunk(const DecArr& d, const uint16_t* lut, const uint32_t* glut,
                                    int L, uint64_t c, int chunk_log2, uint32_t* ring,
                                    uint32_t* err) {
  const uint64_t C = 1ull << chunk_log2;
  const uint64_t nchunks = (d.n + C - 1) >> chunk_log2;
  const GWords offs = (GWords)d.data + d.used;
  const uint64_t payload_words = d.nbytes / 4 - d.used - nchunks;
  const uint64_t wbeg = c ? offs[c - 1] : 0, wend = offs[c];
  // a chunk holds at least one symbol, so at least one word
  if (wbeg >= wend || wend > payload_words || (c == nchunks - 1 && wend != payload_words)) {
    atomicOr(err, kErrCorrupt);
    return;
  }
  RingReader r;
  r.pay = offs + nchunks + wbeg;
  r.cw = (uint32_t)(wend - wbeg);
  r.ring = ring + lane_id();
  r.buf = 0;
  r.nb = 0;
  r.rpos = 0;
  const uint64_t last = payload_words - 1 - wbeg;  // loads past the chunk stay in the payload
  {
    uint32_t w0[kRing];
#pragma unroll
    for (int j = 0; j < kRing; j++) w0[j] = r.pay[min((uint64_t)j, last)];
#pragma unroll
    for (int j = 0; j < kRing; j++) r.ring[j * kWave] = w0[j];
  }
  r.wpos = min((uint32_t)kRing, r.cw);
  uint32_t pf[K];
  uint32_t pfpos = r.wpos;
#pragma unroll
  for (int j = 0; j < K; j++) pf[j] = r.pay[min((uint64_t)pfpos + j, last)];
  const uint64_t cbeg = c * C, cend = min(d.n, cbeg + C);
  const bool vec = MODE >= 2 && (reinterpret_cast<uintptr_t>(d.out) & 15) == 0;
  typedef __attribute__((address_space(1))) uint8_t* GOut8;
  const uint32_t lim = d.limit > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)d.limit;
  static_assert(2 * kMaxLen <= 32, "two codes fit the bits one top-up guarantees");
  const int P = L <= 4 ? 8 : L <= 8 ? 4 : 2;  // symbols per top-up of the bit buffer
  const uint32_t pmask = (uint32_t)P - 1u;
  const int group_bits = P * L;
  for (uint64_t i0 = cbeg; i0 < cend; i0 += kRound) {
    if (pfpos == r.wpos && r.wpos < r.cw && r.wpos + K <= r.rpos + kRing) {
#pragma unroll
      for (int j = 0; j < K; j++) r.ring[((r.wpos + j) & (kRing - 1)) * kWave] = pf[j];
      r.wpos = min(r.wpos + K, r.cw);
    }
    pfpos = r.wpos;
#pragma unroll
    for (int j = 0; j < K; j++) pf[j] = r.pay[min((uint64_t)pfpos + j, last)];
    const int cnt = (int)min((uint64_t)kRound, cend - i0);
    if (MODE < 2) {
      for (int j = 0; j < cnt; j++) {
        uint64_t v;
        if (!decode_symbol(r, lut, glut, L, d, &v)) {
          atomicOr(err, kErrCorrupt);
          return;
        }
        ((GOut64)d.out)[i0 + j] = out_value<MODE>(v);
      }
    } else {
      uint32_t vals[kRound];
      // A full round first without branches: the ring word is always read and
      // appended where the buffer needs it; anything else (ring dry, escape
      // entry, code longer than the bits left, value over the limit, a short
      // round) marks the lane, which then starts the round again on the
      // careful path.
      // The buffer is topped up once per group of P symbols: after a top-up it
      // holds at least 33 bits (unless the chunk's words ran out), and P codes
      // of at most L bits fit in 32, so within a group no symbol needs a
      // refill or a length check (P = 8, 4, 2 for L up to 4, 8, 13).
      const uint64_t buf0 = r.buf;
      const int nb0 = r.nb;
      const uint32_t rpos0 = r.rpos, wpos0 = r.wpos;
      bool redo = cnt < kRound || lut == nullptr;  // no 16-bit table: the careful path only
      if (!redo) {
#pragma unroll
        for (int j = 0; j < kRound; j++) {
          if ((j & pmask) == 0) {
            const bool need = r.nb <= 32 && r.rpos < r.cw;
            const bool have = r.rpos < r.wpos;
            const bool app = need && have;
            const uint32_t w = r.ring[(r.rpos & (kRing - 1)) * kWave];
            const int sh = app ? 32 - r.nb : 0;
            r.buf |= app ? ((uint64_t)w << sh) : 0ull;
            r.nb += app ? 32 : 0;
            r.rpos += app ? 1u : 0u;
            redo |= (need && !have) || r.nb < group_bits;
          }
          const uint32_t e16 = lut[(uint32_t)(r.buf >> (64 - L))];
          const int l = (int)(e16 >> 12);
          const uint32_t sym = e16 & 0xFFFu;
          redo |= e16 == 0 || sym >= lim;
          r.buf <<= l;
          r.nb -= l;
          vals[j] = (uint32_t)out_value<MODE>(sym);
        }
      }
      if (redo) {
        r.buf = buf0;
        r.nb = nb0;
        r.rpos = rpos0;
        r.wpos = wpos0;
#pragma unroll
        for (int j = 0; j < kRound; j++) {
          vals[j] = 0;
          if (j < cnt) {
            uint64_t v;
            if (!decode_symbol(r, lut, glut, L, d, &v)) {
              atomicOr(err, kErrCorrupt);
              return;
            }
            vals[j] = (uint32_t)out_value<MODE>(v);
          }
        }
      }
      store_round<MODE>(d, vals, cnt, i0, vec);
    }
  }
}

// A chunk of an array of mode 2..4 whose cw payload words the wave has staged
// in LDS at w: the same rounds as decode_chunk (a branch-free full round, the
// careful path for anything unusual), with no loads from global memory.
template <int MODE>
__device__ inline void decode_chunk_staged(const DecArr& d, const uint16_t* lut,
                                           const uint32_t* glut, const uint64_t* win, int L,
                                           uint64_t c, int chunk_log2, const uint32_t* w,
                                           uint32_t cw, uint32_t* err) {
  const uint64_t C = 1ull << chunk_log2;
  StageReader r{0ull, 0, 0u, cw, w};
  const uint64_t cbeg = c * C, cend = min(d.n, cbeg + C);
  const bool vec = (reinterpret_cast<uintptr_t>(d.out) & 15) == 0;
  const uint32_t lim = d.limit > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)d.limit;
  const int P = L <= 4 ? 8 : L <= 8 ? 4 : 2;  // symbols per top-up of the bit buffer
  const uint32_t pmask = (uint32_t)P - 1u;
  const int group_bits = P * L;
  // window path (MODE 4 with a window table): bytes decoded past a round's 16
  // are carried into the next one
  uint64_t carry = 0;
  int cc = 0;
  for (uint64_t i0 = cbeg; i0 < cend; i0 += kRound) {
    const int cnt = (int)min((uint64_t)kRound, cend - i0);
    uint32_t vals[kRound];
    const uint64_t buf0 = r.buf;
    const int nb0 = r.nb;
    const uint32_t rpos0 = r.rpos;
    bool redo = cnt < kRound || (lut == nullptr && win == nullptr);
    if (MODE == 4 && win) {
      uint64_t a0 = carry, a1 = 0, a2 = 0;
      int p = cc;
      while (!redo && p < kRound) {
        const bool app = r.nb <= 32 && r.rpos < r.cw;
        const uint32_t wd = w[min(r.rpos, r.cw - 1u)];
        const int sh = app ? 32 - r.nb : 0;
        r.buf |= app ? ((uint64_t)wd << sh) : 0ull;
        r.nb += app ? 32 : 0;
        r.rpos += app ? 1u : 0u;
        const uint64_t e = win[(uint32_t)(r.buf >> (64 - kMW))];
        const int n = (int)((e >> 48) & 15u), bits = (int)(e >> 52);
        redo = n == 0 || bits > r.nb;
        const uint64_t v = redo ? 0ull : (e & 0xFFFFFFFFFFFFull);
        const int s8 = 8 * (p & 7);
        const uint64_t lo = v << s8, hi = s8 ? v >> (64 - s8) : 0ull;
        const bool first = p < 8;
        a0 |= first ? lo : 0ull;
        a1 |= first ? hi : lo;
        a2 |= first ? 0ull : hi;
        r.buf <<= redo ? 0 : bits;
        r.nb -= redo ? 0 : bits;
        p += redo ? 0 : n;
      }
      if (!redo) {
        if (vec) {
          *(GOut128)((__attribute__((address_space(1))) uint8_t*)d.out + i0) =
              U32x4{(uint32_t)a0, (uint32_t)(a0 >> 32), (uint32_t)a1, (uint32_t)(a1 >> 32)};
        } else {
#pragma unroll
          for (int j = 0; j < kRound; j++)
            ((__attribute__((address_space(1))) uint8_t*)d.out)[i0 + j] =
                (uint8_t)((j < 8 ? a0 : a1) >> (8 * (j & 7)));
        }
        carry = a2;
        cc = p - kRound;
        continue;
      }
      // the careful path: the carried values first, then one code at a time
      r.buf = buf0;
      r.nb = nb0;
      r.rpos = rpos0;
#pragma unroll
      for (int j = 0; j < kRound; j++) {
        vals[j] = 0;
        if (j < cnt && j < cc) {
          vals[j] = (uint32_t)(int32_t)(int8_t)(uint8_t)(carry >> (8 * j));
        } else if (j < cnt) {
          uint64_t v;
          if (!decode_symbol(r, lut, glut, L, d, &v)) {
            atomicOr(err, kErrCorrupt);
            return;
          }
          vals[j] = (uint32_t)out_value<MODE>(v);
        }
      }
      carry = 0;
      cc = 0;
      store_round<MODE>(d, vals, cnt, i0, vec);
      continue;
    }
    if (!redo) {
#pragma unroll
      for (int j = 0; j < kRound; j++) {
        if ((j & pmask) == 0) {
          const bool app = r.nb <= 32 && r.rpos < r.cw;
          const uint32_t wd = w[min(r.rpos, r.cw - 1u)];
          const int sh = app ? 32 - r.nb : 0;
          r.buf |= app ? ((uint64_t)wd << sh) : 0ull;
          r.nb += app ? 32 : 0;
          r.rpos += app ? 1u : 0u;
          redo |= r.nb < group_bits;
        }
        const uint32_t e16 = lut[(uint32_t)(r.buf >> (64 - L))];
        const int l = (int)(e16 >> 12);
        const uint32_t sym = e16 & 0xFFFu;
        redo |= e16 == 0 || sym >= lim;
        r.buf <<= l;
        r.nb -= l;
        vals[j] = (uint32_t)out_value<MODE>(sym);
      }
    }
    if (redo) {
      r.buf = buf0;
      r.nb = nb0;
      r.rpos = rpos0;
#pragma unroll
      for (int j = 0; j < kRound; j++) {
        vals[j] = 0;
        if (j < cnt) {
          uint64_t v;
          if (!decode_symbol(r, lut, glut, L, d, &v)) {
            atomicOr(err, kErrCorrupt);
            return;
          }
          vals[j] = (uint32_t)out_value<MODE>(v);
        }
      }
    }
    store_round<MODE>(d, vals, cnt, i0, vec);
  }
}

// Words to load per round: about one and a half times the array's average
// (payload words per kRound symbols), rounded up to a power of two, at most 8.
__device__ inline int ring_words(const DecArr& d, uint64_t nchunks) {
  const uint64_t pw = d.nbytes / 4 - d.used - nchunks;
  const uint64_t need = (pw * kRound * 3 / 2 + d.n - 1) / d.n + 1;
  return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 8;
}

template <int MODE>
__device__ inline void decode_chunk_k(int K, const DecArr& d, const uint16_t* lut,
                                      const uint32_t* glut, int L, uint64_t c, int chunk_log2,
                                      uint32_t* ring, uint32_t* err) {
  switch (K) {
    case 1: decode_chunk<MODE, 1>(d, lut, glut, L, c, chunk_log2, ring, err); break;
    case 2: decode_chunk<MODE, 2>(d, lut, glut, L, c, chunk_log2, ring, err); break;
    case 4: decode_chunk<MODE, 4>(d, lut, glut, L, c, chunk_log2, ring, err); break;
    default: decode_chunk<MODE, 8>(d, lut, glut, L, c, chunk_log2, ring, err); break;
  }
}

// Dynamic LDS: an area of kStageWords words per wave (its chunks' staged
// payload, or its lanes' rings), then the 16-bit table of 2^lut_log2 entries
// (lut_log2: the longest code among the launch's arrays), then, when lut_log2
// <= kWinLog2Max, the 2^kMW-entry window table of a short-code byte array;
// 64 KB at most.
__global__ __launch_bounds__(kThreads) void k_decode_huff(const DecArr* arrs,
                                                          const uint32_t* prefix, int A,
                                                          int chunk_log2,
                                                          const uint32_t* lut_all, int lut_log2,
                                                          uint32_t* err) {
  extern __shared__ uint32_t dyn[];
  uint16_t* lut = reinterpret_cast<uint16_t*>(dyn + kThreads / kWave * kStageWords);
  const uint32_t a = array_of_block(prefix, A, blockIdx.x);
  const DecArr d = arrs[a];
  if (d.coder != 1 || d.param < 1 || d.param > kMaxLen || (*err & kErrCorrupt)) return;
  const int L = d.param;
  if (L > lut_log2) {
    if (threadIdx.x == 0) atomicOr(err, kErrCorrupt);
    return;
  }
  const uint64_t C = 1ull << chunk_log2;
  const uint64_t nchunks = (d.n + C - 1) >> chunk_log2;
  if (d.nbytes / 4 < (uint64_t)d.used + nchunks + 1) {  // no payload word
    if (threadIdx.x == 0) atomicOr(err, kErrCorrupt);
    return;
  }
  const uint32_t* src = lut_all + (uint64_t)a * (1u << kMaxLen);
  for (uint32_t i = threadIdx.x; i < (1u << L); i += kThreads) {
    const uint32_t e = src[i], sym = e & 0xFFFFu, l = e >> 16;
    lut[i] = (uint16_t)(sym < (uint32_t)kDirect && l ? (l << 12) | sym : 0u);
  }
  // byte arrays with short codes also take the window table, when the
  // launch's longest code leaves room for it (lut_log2 <= kWinLog2Max)
  const bool use_win = lut_log2 <= kWinLog2Max && d.mode == 4 && L <= kMW;
  uint64_t* win_lds = reinterpret_cast<uint64_t*>(lut + (((1u << lut_log2) + 3u) & ~3u));
  if (use_win) {
    const uint64_t* wsrc = reinterpret_cast<const uint64_t*>(src + kMOff);
    for (uint32_t i = threadIdx.x; i < (1u << kMW); i += kThreads) win_lds[i] = wsrc[i];
  }
  __syncthreads();
  // The wave's chunks are consecutive, so their payloads are one range of
  // words: when it fits the wave's area it is copied there with coalesced
  // loads (one request per 64 words, where a lane reading its own chunk would
  // touch a line per lane per word) and every lane decodes from LDS; else the
  // lanes read through their rings.
  const uint64_t c = (uint64_t)(blockIdx.x - prefix[a]) * kThreads + threadIdx.x;
  const bool valid = c < nchunks;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane(wave_id());
  uint32_t* area = dyn + (uint64_t)wv * kStageWords;
  const uint64_t vmask = __ballot(valid);
  if (vmask == 0) return;
  const GWords offs = (GWords)d.data + d.used;
  const uint64_t payload_words = d.nbytes / 4 - d.used - nchunks;
  const uint64_t wbeg = valid ? (c ? offs[c - 1] : 0) : 0, wend = valid ? offs[c] : 0;
  // a chunk holds at least one symbol, so at least one word
  const bool bad = valid && (wbeg >= wend || wend > payload_words ||
                             (c == nchunks - 1 && wend != payload_words));
  const uint32_t last_lane = 63u - (uint32_t)__builtin_clzll(vmask);
  const uint64_t r0 = (uint64_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)wbeg) |
                      ((uint64_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(wbeg >> 32)) << 32);
  const uint64_t r1 = (uint64_t)__builtin_amdgcn_readlane((int)(uint32_t)wend, last_lane) |
                      ((uint64_t)__builtin_amdgcn_readlane((int)(uint32_t)(wend >> 32), last_lane) << 32);
  const int K = ring_words(d, nchunks);
  if ((d.mode >= 2) && __ballot(bad) == 0 && r1 > r0 && r1 - r0 <= (uint64_t)kStageWords) {
    const uint32_t S = (uint32_t)(r1 - r0);
    const GWords src_w = offs + nchunks + r0;
    const uint32_t lane = (uint32_t)lane_id();
    for (uint32_t j0 = 0; j0 < S; j0 += kWave * kStageBatch) {
      uint32_t v[kStageBatch];
#pragma unroll
      for (int q = 0; q < kStageBatch; q++) {
        const uint32_t j = j0 + q * kWave + lane;
        v[q] = j < S ? src_w[j] : 0u;
      }
#pragma unroll
      for (int q = 0; q < kStageBatch; q++) {
        const uint32_t j = j0 + q * kWave + lane;
        if (j < S) area[j] = v[q];
      }
    }
    wave_lds_sync();
    if (!valid) return;
    const uint32_t* wch = area + (uint32_t)(wbeg - r0);
    const uint32_t cw = (uint32_t)(wend - wbeg);
    switch (d.mode) {
      case 2: decode_chunk_staged<2>(d, lut, src, nullptr, L, c, chunk_log2, wch, cw, err); break;
      case 3: decode_chunk_staged<3>(d, lut, src, nullptr, L, c, chunk_log2, wch, cw, err); break;
      default:
        decode_chunk_staged<4>(d, lut, src, use_win ? win_lds : nullptr, L, c, chunk_log2, wch,
                               cw, err);
        break;
    }
    return;
  }
  if (!valid) return;
  switch (d.mode) {
    case 0: decode_chunk_k<0>(K, d, lut, src, L, c, chunk_log2, area, err); break;
    case 1: decode_chunk_k<1>(K, d, lut, src, L, c, chunk_log2, area, err); break;
    case 2: decode_chunk_k<2>(K, d, lut, src, L, c, chunk_log2, area, err); break;
    case 3: decode_chunk_k<3>(K, d, lut, src, L, c, chunk_log2, area, err); break;
    default: decode_chunk_k<4>(K, d, lut, src, L, c, chunk_log2, area, err); break;
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

uint32_t enc_hist_blocks(uint64_t n) { return gclamp((n + 8191) / 8192, kHistBlocks); }
uint32_t enc_hist_copies(uint64_t n) {
  const uint32_t c = (enc_hist_blocks(n) + 15) / 16;
  return c > (uint32_t)kHistCopies ? (uint32_t)kHistCopies : c;
}
uint32_t enc_chunk_blocks(uint64_t n, int chunk_log2, bool bytes) {
  // byte arrays pack one chunk per wave (k_pack_wave), others one per workgroup
  const uint64_t nchunks = (n + (1ull << chunk_log2) - 1) >> chunk_log2;
  return bytes && pack_by_wave(chunk_log2) ? gclamp((nchunks + kPackWaves - 1) / kPackWaves, 256)
                                            : gclamp(nchunks, 512);
}
uint32_t enc_copy_blocks(uint64_t n, int chunk_log2) {
  return gclamp((n + (1ull << chunk_log2) - 1) >> chunk_log2, 256);
}
// Fixed-length packing loops over its words, so a few workgroups per array
// suffice; every emit workgroup of a single record also lays the record out,
// which workgroups that find their array Huffman-coded would only repeat.
uint32_t enc_fixed_blocks(uint64_t n) { return gclamp((n + 2047) / 2048, 128); }

uint32_t enc_slot_words(bool is64, int chunk_log2) {
  // per symbol at most the longest code and, for values from kDirect up, one
  // raw bit fewer than the value's width
  return (uint32_t)(((1ull << chunk_log2) * (uint64_t)(kMaxLen + (is64 ? 63 : 31)) + 31) / 32);
}
uint64_t enc_stage_words(uint64_t n, bool is64, int chunk_log2) {
  return ((n + (1ull << chunk_log2) - 1) >> chunk_log2) * enc_slot_words(is64, chunk_log2);
}

void launch_encode(const EncLaunch& L, int chunk_log2, ArrWork* work, const EncScratch& X,
                   uint8_t* out, uint64_t cap, unsigned long long* offs, uint32_t* err,
                   const unsigned long long* base, bool hist_done, hipStream_t s) {
  const int NA = L.NA;
  const uint32_t* pre_hist = L.pre;
  const uint32_t* pre_chunk = L.pre + (NA + 1);
  const uint32_t* pre_fixed = L.pre + 2 * (NA + 1);
  const uint32_t* pre_copy = L.pre + 3 * (NA + 1);
  if (!hist_done)
    launch_timed("hist", L.values * 4ull, k_hist, L.hist_blocks, kThreads, 0, s,
               L.arrs, pre_hist, NA, X.hist_part, X.hist_max);
  // the plain build (and its codes) per array; the halving candidates and their
  // codes only run for arrays whose plain build is too deep.  Temporal residual
  // arrays (hist_done) halve inline: their alphabets are short and the fallback
  // launches would cost more than they save.
  const int fused = L.fused && L.all_bytes && pack_by_wave(chunk_log2);
  if (!fused)
    launch_timed("huff_build", 0, k_huff_build, NA, kHT, 0, s, L.arrs, X.hist_part, X.hist_max,
                 work, X.huff_lens, X.huff_maxd, hist_done ? 1 : 0, chunk_log2);
  if (!hist_done) {
    if ((uint64_t)NA * (kHalvings - 1) <= kOneLaunchCandidates) {
      // few arrays: every candidate in one launch (the GPU is far from full
      // either way, and a second launch would cost its own latency)
      k_huff_lengths<<<dim3(NA, kHalvings - 1), kHT, 0, s>>>(work, X.huff_lens, X.huff_maxd, 1);
    } else {
      k_huff_lengths<<<dim3(NA, kFirstHalvings), kHT, 0, s>>>(work, X.huff_lens, X.huff_maxd, 1);
      k_huff_lengths<<<dim3(NA, kHalvings - 1 - kFirstHalvings), kHT, 0, s>>>(
          work, X.huff_lens, X.huff_maxd, 1 + kFirstHalvings);
    }
    k_huff_codes<<<NA, kHT, 0, s>>>(L.arrs, work, X.huff_lens, X.huff_maxd, chunk_log2);
  }
  const uint32_t slot32 = enc_slot_words(false, chunk_log2), slot64 = enc_slot_words(true, chunk_log2);
  if (L.all_bytes && pack_by_wave(chunk_log2)) {
    // one chunk per wave: C / 64 values per lane
    const size_t shm = (size_t)kPackWaves * slot32 * 4;
    auto* kernel = k_pack_wave<16>;
    switch (chunk_log2) {
      case 6: kernel = k_pack_wave<1>; break;
      case 7: kernel = k_pack_wave<2>; break;
      case 8: kernel = k_pack_wave<4>; break;
      case 9: kernel = k_pack_wave<8>; break;
      default: break;
    }
    launch_timed("pack_huff", L.values * 6ull, kernel, L.chunk_blocks, kThreads, shm, s, L.arrs,
                 work, pre_chunk, NA, chunk_log2, X.chunk_words, X.stage, slot32, err,
                 X.hist_part, X.hist_max, fused, L.err_rec, L.err_stride);
  } else {
    const size_t shm = (size_t)slot64 * 4;
    const uint32_t g = L.chunk_blocks;
    auto* kernel = k_pack_huff<1>;
    switch (chunk_log2) {
      case 9: kernel = k_pack_huff<2>; break;
      case 10: kernel = k_pack_huff<4>; break;
      case 11: kernel = k_pack_huff<8>; break;
      case 12: kernel = k_pack_huff<16>; break;
      default: break;
    }
    launch_timed("pack_huff", L.values * 6ull, kernel, g, kThreads, shm, s, L.arrs, work,
                 pre_chunk, NA, chunk_log2, X.chunk_words, X.stage, slot32, slot64, err);
  }
  const uint32_t emit_blocks = L.fixed_blocks + L.copy_blocks;
  const int fold = L.R == 1 && emit_blocks > 0;  // the emit workgroups lay the record out
  if (!fold)
    launch_timed("layout", 0, k_layout, 1, kHT, 0, s, work, L.recs, L.rec0, L.R, out, cap, offs,
                 base, err);
  if (emit_blocks)
    launch_timed("emit", L.values * 6ull, k_emit, emit_blocks, kThreads, 0, s, L.arrs, work,
                 L.recs, L.rec0, fold, pre_fixed, L.fixed_blocks, pre_copy, NA, X.chunk_words,
                 X.stage, slot32, slot64, out, cap, offs, base, err,
                 fused ? X.hist_part : nullptr, fused ? X.hist_max : nullptr);
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
                   int chunk_log2, int lut_log2, uint64_t bytes, uint32_t* lut, uint32_t* err,
                   hipStream_t s) {
  if (A == 0) return;
  k_lut<<<A, kHT, 0, s>>>(arrs_dev, lut, err);
  if (lut_log2 < 1) lut_log2 = 1;
  if (lut_log2 > kMaxLen) lut_log2 = kMaxLen;
  const size_t shm = (size_t)kThreads / kWave * kStageWords * 4 +
                     ((((size_t)1 << lut_log2) + 3) & ~(size_t)3) * 2 +
                     (lut_log2 <= kWinLog2Max ? (size_t)8 << kMW : 0);
  if (huff_blocks)
    launch_timed("decode_huff", bytes, k_decode_huff, huff_blocks, kThreads, shm, s, arrs_dev,
                 huff_prefix_dev, A, chunk_log2, lut, lut_log2, err);
  if (fixed_blocks)
    launch_timed("decode_fixed", bytes, k_decode_fixed, fixed_blocks, kThreads, 0, s,
               arrs_dev, fixed_prefix_dev, A, err);
}

}  // namespace lcp
