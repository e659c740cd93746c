// kernels_core.hip -- LCP-S / LCP-T data-parallel steps on gfx950:
//   extent pass (min/max per field, the min(D.x) of Eq. 5),
//   quantisation + block key (Eq. 5, Eq. 6),
//   stable LSD radix sort of (block key, input index) -> block order (Sec. 6.2.1),
//   device-wide scans, run detection (non-empty blocks), symbol arrays with delta
//   coding (Sec. 6.2.2), temporal residuals (Sec. 7.1), and the decode-side block
//   expansion and FP32 reconstruction.
#include <string.h>

#include <type_traits>

#include "lcp_internal.h"

namespace lcp {

namespace {

constexpr int kThreads = 256;

inline uint32_t grid_for(uint64_t n, uint64_t per_block, uint32_t cap = 1u << 20) {
  uint64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

// Every frame of a batch gets whole workgroups; a workgroup finds its frame by
// binary search in a prefix table of per-frame workgroup counts (R + 1 entries).
__device__ inline int seg_of_block(const uint32_t* pre, int R, uint32_t b) {
  int lo = 0, hi = R - 1;  // largest r with pre[r] <= b
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ radix sort
// Stable LSD radix sort of (key, value) pairs within each frame of a batch
// (segments [off, off + n) of the SegDev table), 8-bit digits.  Tiles of
// kRsTile elements never cross a frame.  The digit counts are laid out frame
// by frame, then digit by digit, then tile by tile, so one exclusive scan gives
// every (tile, digit) its output position inside its own frame.  The scatter
// ranks a tile stably in LDS (ballots over the digit bits), places it there in
// digit order, and writes each digit's run out contiguously.
constexpr int kRsItems = 16;
constexpr int kRsTile = kThreads * kRsItems;  // 4096 keys per tile
static_assert(kRsTile == (int)kSortTile, "sort tile");

// K: the key type, u32 when the block ids fit 32 bits (half the sort's key
// traffic), else u64.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const K* keys, const SegDev* S,
                                                         const uint32_t* pre, int R, int shift,
                                                         uint32_t* hist) {
  __shared__ uint32_t cnt[kThreads / kWave][256];
  const int t = threadIdx.x, w = wave_id();
  const int r = seg_of_block(pre, R, blockIdx.x);
  const uint32_t lt = blockIdx.x - pre[r], nt = pre[r + 1] - pre[r];
  const uint64_t base = S[r].off + (uint64_t)lt * kRsTile;
  const uint64_t end = S[r].off + S[r].n;
  for (int j = 0; j < 4; j++) cnt[j][t] = 0;
  __syncthreads();
#pragma unroll 4
  for (int j = 0; j < kRsItems; j++) {
    uint64_t i = base + (uint64_t)j * kThreads + t;
    if (i < end) atomicAdd(&cnt[w][(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)pre[r] * 256 + (uint64_t)t * nt + lt] = cnt[0][t] + cnt[1][t] + cnt[2][t] + cnt[3][t];
}

template <typename K>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const K* kin,
                                                            const uint32_t* vin, K* kout,
                                                            uint32_t* vout, const SegDev* S,
                                                            const uint32_t* pre, int R, int shift,
                                                            const uint32_t* offs,
                                                            uint64_t entries, uint64_t ntot) {
  __shared__ K sk[kRsTile];
  __shared__ uint32_t sv[kRsTile];
  __shared__ uint32_t gbase[256], lstart[256], run[256];
  __shared__ uint32_t wcnt[kThreads / kWave][256];
  __shared__ uint32_t sm[kThreads / kWave + 1];
  const int t = threadIdx.x, w = wave_id();
  const int r = seg_of_block(pre, R, blockIdx.x);
  const uint32_t lt = blockIdx.x - pre[r], nt = pre[r + 1] - pre[r];
  const uint64_t tile0 = S[r].off + (uint64_t)lt * kRsTile;
  const uint64_t rem = S[r].n - (uint64_t)lt * kRsTile;
  const uint32_t cnt = rem < (uint64_t)kRsTile ? (uint32_t)rem : (uint32_t)kRsTile;
  // this tile's output start and element count for digit t
  const uint64_t e = (uint64_t)pre[r] * 256 + (uint64_t)t * nt + lt;
  const uint32_t g = offs[e];
  const uint32_t c = (uint32_t)((e + 1 < entries ? (uint64_t)offs[e + 1] : ntot) - g);
  uint32_t tot;
  const uint32_t ls = block_incl_scan(c, sm, &tot) - c;
  gbase[t] = g;
  lstart[t] = ls;
  run[t] = 0;
  __syncthreads();
  const uint64_t lmask = lanemask_lt();
  for (int rd = 0; rd < kRsItems; rd++) {
    const uint32_t li = (uint32_t)rd * kThreads + t;
    const bool valid = li < cnt;
    const K key = valid ? kin[tile0 + li] : (K)0;
    const uint32_t val = valid ? vin[tile0 + li] : 0;
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
#pragma unroll
    for (int j = 0; j < kThreads / kWave; j++) wcnt[j][t] = 0;
    __syncthreads();
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lmask);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = lstart[d] + run[d] + rank;
      for (int j = 0; j < w; j++) pos += wcnt[j][d];
      sk[pos] = key;
      sv[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int j = 0; j < kThreads / kWave; j++) add += wcnt[j][t];
    run[t] += add;
    __syncthreads();
  }
  // the tile in digit order: consecutive slots of one digit go to consecutive
  // output positions
  for (uint32_t i = t; i < cnt; i += kThreads) {
    const K key = sk[i];
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    const uint64_t pos = (uint64_t)gbase[d] + (i - lstart[d]);
    kout[pos] = key;
    vout[pos] = sv[i];
  }
}

// ------------------------------------------------------------------ scans
constexpr int kScanItems = 8;
constexpr int kScanTile = kThreads * kScanItems;  // 2048

// Sum of tile blockIdx.x of in[0, nn) into partials[blockIdx.x].
template <typename T>
__device__ inline void scan_reduce_tile(const T* in, uint64_t nn, T* partials) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  T s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
    if (i < nn) s += in[i];
  }
  s = wave_sum(s);
  __shared__ T sm[kThreads / kWave];
  if (lane_id() == 0) sm[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    T tot = 0;
    for (int j = 0; j < kThreads / kWave; j++) tot += sm[j];
    partials[blockIdx.x] = tot;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(const T* in, uint64_t n,
                                                          const uint32_t* n_dev, T* partials) {
  scan_reduce_tile<T>(in, n_dev ? min((uint64_t)*n_dev, n) : n, partials);
}

// Scan of tile blockIdx.x of data[0, nn), plus prefix[blockIdx.x] when given:
// striped load through LDS, blocked per-thread scan.
template <typename T>
__device__ inline void scan_apply_tile(T* data, uint64_t nn, const T* prefix, int exclusive) {
  __shared__ T tile[kScanTile];
  __shared__ T sm[kThreads / kWave + 1];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
    tile[j * kThreads + threadIdx.x] = i < nn ? data[i] : (T)0;
  }
  __syncthreads();
  T v[kScanItems];
  T local = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    v[j] = tile[threadIdx.x * kScanItems + j];
    local += v[j];
  }
  T total;
  T incl = block_incl_scan(local, sm, &total);
  T run = incl - local + (prefix ? prefix[blockIdx.x] : (T)0);
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    if (exclusive) {
      tile[threadIdx.x * kScanItems + j] = run;
      run += v[j];
    } else {
      run += v[j];
      tile[threadIdx.x * kScanItems + j] = run;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
    if (i < nn) data[i] = tile[j * kThreads + threadIdx.x];
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_apply(T* data, uint64_t n,
                                                         const uint32_t* n_dev,
                                                         const T* prefix, int exclusive) {
  scan_apply_tile<T>(data, n_dev ? min((uint64_t)*n_dev, n) : n, prefix, exclusive);
}

// Up to four u32 arrays of one length scanned side by side, blockIdx.y picking
// the array (its tile sums at partials + y * tiles): one set of launches
// rather than one per array.
struct ScanSet {
  uint32_t* p[4];
};

__global__ __launch_bounds__(kThreads) void k_scan_reduce4(ScanSet a, uint64_t n,
                                                           uint32_t* partials, uint32_t tiles) {
  scan_reduce_tile<uint32_t>(a.p[blockIdx.y], n, partials + (uint64_t)blockIdx.y * tiles);
}

__global__ __launch_bounds__(kThreads) void k_scan_apply4(ScanSet a, uint64_t n,
                                                          const uint32_t* prefix, uint32_t tiles,
                                                          int exclusive) {
  scan_apply_tile<uint32_t>(a.p[blockIdx.y], n,
                            prefix ? prefix + (uint64_t)blockIdx.y * tiles : nullptr, exclusive);
}

// LCP-T: the frame's codes on the reference grid, in the reference's slot order,
// minus the reference codes (zigzag); the new codes become the next reference.
// The frame must stay inside the grid's float32 margin (|x| + 2 eb < 2^E,
// evaluated in double: since that sum grows with |x|, it holds exactly for
// |x| <= xmax, the largest float for which it holds, found on the host) and
// code range (|2q+1| < 2^24); a particle outside it flags the frame.  int32
// grids have no margin to keep: their reconstructions are exact integers.
// is_int: the grid's type, a constant where the caller is specialised for it.
// The checks are selects, not branches.
__device__ inline void t_code_as(float xv, int is_int, const GridDev& g, int f, uint32_t* bad,
                                 int32_t* qo) {
  const double xd = word_value(xv, is_int);
  const bool finite = is_int || __builtin_isfinite(xv);
  const bool inside = is_int || fabsf(xv) <= g.xmax[f];
  *bad |= (finite ? 0u : (uint32_t)kErrNonFinite) | (finite && !inside ? (uint32_t)kErrRange : 0u);
  int32_t q = quantise(xd, g.md[f], g.inv[f]);
  if (q < -kQLimit || q >= kQLimit) {
    *bad |= kErrRange;
    q = 0;
  }
  *qo = q;
}
__device__ inline void t_code(float xv, const GridDev& g, int f, uint32_t* bad, int32_t* qo) {
  t_code_as(xv, g.dtype, g, f, bad, qo);
}

// Sec. 7.1 with the anchor scale of Sec. 7.4.2: a temporal frame's code on its
// reference grid moves from the reference's code by a multiple of the grid's
// step s, the multiple nearest the frame's own code q (within (s - 1) / 2 of
// it, s odd); the residual is that multiple over s.  With s = 1 the code is q
// itself.  A code outside the code range flags the frame.
// Codes and references lie within +-2^23 here, so every quantity fits 32 bits.
__device__ inline int32_t t_step(int32_t q, int32_t ref, int32_t s, uint32_t* bad, int32_t* qn) {
  if (s == 1) {
    *qn = q;
    return q - ref;
  }
  const int32_t num = q - ref + (s - 1) / 2;
  const int32_t r = num >= 0 ? num / s : -((-num + s - 1) / s);
  int32_t c = ref + s * r;
  if (c < -kQLimit || c >= kQLimit) {
    *bad |= kErrRange;
    c = 0;
  }
  *qn = c;
  return r;
}

// Per-wave private bins of the fused residual histogram (symbols below this).
constexpr int kResPriv = 256;

__global__ __launch_bounds__(kThreads) void k_t_resid(FieldPtrs x, int F, uint64_t n, GridDev g,
                                                      const uint32_t* perm_ref,
                                                      const int32_t* q_ref, uint8_t* v8,
                                                      uint32_t* v_res, int32_t* q_new,
                                                      uint32_t* err, int vec,
                                                      uint32_t* hist_part,
                                                      unsigned long long* hist_max,
                                                      ArrWork* zw) {
  // per field and wave kResPriv private bins, sized by F at launch so that
  // LDS does not cap the workgroups resident per CU
  extern __shared__ uint32_t bins_lds[];
  __shared__ uint32_t smax[kMaxF][kThreads / kWave];
  auto bins = [&](int f, int w) { return bins_lds + ((uint32_t)f * (kThreads / kWave) + w) * kResPriv; };
  for (int j = threadIdx.x; j < F * (kThreads / kWave) * kResPriv; j += kThreads) bins_lds[j] = 0;
  // the coder's word totals start from zero (the frame before was emitted)
  if (zw && blockIdx.x == 0 && threadIdx.x < (uint32_t)(F * kWordParts))
    zw[threadIdx.x / kWordParts].huff_words[threadIdx.x % kWordParts] = 0;
  __syncthreads();
  const int copy = blockIdx.x % kHistCopies;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t bad = 0;
  uint32_t rmax[kMaxF];
#pragma unroll
  for (int f = 0; f < kMaxF; f++) rmax[f] = 0;
  auto count = [&](int f, HotCounts& h, uint32_t r) {
    uint32_t* shared = hist_part + ((uint64_t)f * kHistCopies + copy) * kAlphabet;
    hist_add_hot(h, shared, bins(f, wave_id()), kResPriv, r, true);
  };
  if (vec) {  // n % 4 == 0 and 16-byte aligned arrays: 4 slots per thread
    for (uint64_t s4 = gid; s4 < n / 4; s4 += stride) {
      const uint4 iv = reinterpret_cast<const uint4*>(perm_ref)[s4];
      const uint32_t idx[4] = {iv.x, iv.y, iv.z, iv.w};
      // four consecutive inputs: one 16-byte load per field (see float4_a4)
      const bool seq4 = idx[1] == idx[0] + 1 && idx[2] == idx[0] + 2 && idx[3] == idx[0] + 3;
      for (int f = 0; f < F; f++) {
        float xv[4];
        if (seq4 && ((uintptr_t)x.p[f] & 3) == 0) {
          const float4_a4 v4 = *reinterpret_cast<const float4_a4*>(x.p[f] + idx[0]);
          xv[0] = v4.x;
          xv[1] = v4.y;
          xv[2] = v4.z;
          xv[3] = v4.w;
        } else {
#pragma unroll
          for (int j = 0; j < 4; j++) xv[j] = x.p[f][idx[j]];
        }
        const int4 qr = reinterpret_cast<const int4*>(q_ref + (uint64_t)f * n)[s4];
        const int32_t qrv[4] = {qr.x, qr.y, qr.z, qr.w};
        uint32_t rv[4];
        int32_t qv[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
          int32_t q, qn;
          t_code(xv[j], g, f, &bad, &q);
          rv[j] = (uint32_t)zigzag32(t_step(q, qrv[j], g.scale, &bad, &qn));
          qv[j] = (int32_t)qn;
          rmax[f] = max(rmax[f], rv[j]);
        }
        if (v8) {
          uint32_t bytes = 0;
#pragma unroll
          for (int j = 0; j < 4; j++) bytes |= min(rv[j], 255u) << (8 * j);
          reinterpret_cast<uint32_t*>(v8 + (uint64_t)f * n)[s4] = bytes;
#pragma unroll
          for (int j = 0; j < 4; j++)
            if (rv[j] >= 255u) v_res[(uint64_t)f * n + 4 * s4 + j] = rv[j];
        } else {
          reinterpret_cast<uint4*>(v_res + (uint64_t)f * n)[s4] = make_uint4(rv[0], rv[1], rv[2], rv[3]);
        }
        reinterpret_cast<int4*>(q_new + (uint64_t)f * n)[s4] = make_int4(qv[0], qv[1], qv[2], qv[3]);
        HotCounts h{0u, 0u, 0u};
#pragma unroll
        for (int j = 0; j < 4; j++) count(f, h, rv[j]);
        hist_flush_hot(h, bins(f, wave_id()), 4u * (uint32_t)__popcll(__ballot(1)));
      }
    }
  } else {
    for (uint64_t s = gid; s < n; s += stride) {
      uint32_t i = perm_ref[s];
      for (int f = 0; f < F; f++) {
        int32_t q0, q;
        t_code(x.p[f][i], g, f, &bad, &q0);
        const uint32_t r =
            (uint32_t)zigzag32(t_step(q0, q_ref[(uint64_t)f * n + s], g.scale, &bad, &q));
        if (v8) {
          v8[(uint64_t)f * n + s] = (uint8_t)min(r, 255u);
          if (r >= 255u) v_res[(uint64_t)f * n + s] = r;
        } else {
          v_res[(uint64_t)f * n + s] = r;
        }
        q_new[(uint64_t)f * n + s] = (int32_t)q;
        rmax[f] = max(rmax[f], r);
        HotCounts h{0u, 0u, 0u};
        count(f, h, r);
        hist_flush_hot(h, bins(f, wave_id()), (uint32_t)__popcll(__ballot(1)));
      }
    }
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) bad |= (uint32_t)__shfl_xor((int)bad, d, kWave);
  if (lane_id() == 0 && bad) atomicOr(err, bad);
  for (int f = 0; f < F; f++) {
    uint32_t m = rmax[f];
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, kWave));
    if (lane_id() == 0) smax[f][wave_id()] = m;
  }
  __syncthreads();
  // merge the waves' bins into the array's spread copy (non-zero bins only)
  for (int f = 0; f < F; f++) {
    uint32_t* shared = hist_part + ((uint64_t)f * kHistCopies + copy) * kAlphabet;
    for (int j = threadIdx.x; j < kResPriv; j += kThreads) {
      uint32_t t = 0;
      for (int w = 0; w < kThreads / kWave; w++) t += bins(f, w)[j];
      if (t) atomicAdd(&shared[j], t);
    }
    if (threadIdx.x == 0) {
      uint32_t m = 0;
      for (int w = 0; w < kThreads / kWave; w++) m = max(m, smax[f][w]);
      if (m) atomicMax(&hist_max[(uint64_t)f * kHistCopies + copy], (unsigned long long)m);
    }
  }
}

// A run of J temporal frames that share one reference grid and slot order, each
// coded against the frame before it (the first against q_ref), in one launch:
// every thread owns fixed slots (four consecutive ones on the vector path, one
// otherwise), keeps their codes in registers from frame to frame, and per frame
// gathers the values through the permutation, quantises them on the grid,
// writes the zigzag residuals as bytes (255: the value is in the escape array)
// and counts them.  The workgroup keeps every frame's counts of symbols below
// kRunPriv in LDS (larger symbols go straight to the spread copy), so the
// frames follow one another without a barrier; the counts are merged into each
// array's spread copy once at the end.  Only the last frame's codes are stored.
// Array (frame j, field f) of the run is a = (a0 + j) F + f: its bytes at
// v8 + a * astride, escapes at vesc + a * astride, histogram copies
// [a copies, (a + 1) copies), work record zw[a]; frame j's error word at
// err + j * err_stride.
constexpr int kRunPriv = 64;
template <int F, int DT>
__global__ __launch_bounds__(kThreads) void k_t_resid_run(RunFrames fr, int J, uint64_t n,
                                                          GridDev g, const uint32_t* perm,
                                                          const int32_t* q_ref, int32_t* q_last,
                                                          uint8_t* v8, uint32_t* vesc,
                                                          uint64_t astride, int a0,
                                                          uint32_t* hist_part,
                                                          unsigned long long* hist_max,
                                                          int copies, ArrWork* zw, uint32_t* err,
                                                          int err_stride, int vec) {
  extern __shared__ uint32_t bins_lds[];  // [J][F][kRunPriv]
  __shared__ uint32_t smax[kRunMax][F];
  const int nbins = J * F * kRunPriv;
  for (int j = threadIdx.x; j < nbins; j += kThreads) bins_lds[j] = 0;
  if (threadIdx.x < (uint32_t)(kRunMax * F)) (&smax[0][0])[threadIdx.x] = 0;
  // the coder's word totals of every array of the run start from zero
  if (zw && blockIdx.x == 0)
    for (int t = threadIdx.x; t < J * F * kWordParts; t += kThreads)
      zw[(uint64_t)a0 * F + t / kWordParts].huff_words[t % kWordParts] = 0;
  const int copy = blockIdx.x % copies;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t items = vec ? n / 4 : n;
  const bool mine = gid < items;
  // the thread's slots, their input indices and their running codes
  uint32_t idx[4] = {0, 0, 0, 0};
  int32_t q[F][4];
  if (mine) {
    if (vec) {
      const uint4 iv = reinterpret_cast<const uint4*>(perm)[gid];
      idx[0] = iv.x;
      idx[1] = iv.y;
      idx[2] = iv.z;
      idx[3] = iv.w;
    } else {
      idx[0] = perm[gid];
    }
  }
  // four slots whose inputs are four consecutive values (a slot order that
  // keeps runs of the input order, as a trajectory's does) are read with one
  // 16-byte load per field instead of four gathers, wherever the run starts
  // (see float4_a4)
  const bool seq4 = vec && mine && idx[1] == idx[0] + 1 && idx[2] == idx[0] + 2 &&
                    idx[3] == idx[0] + 3;
#pragma unroll
  for (int f = 0; f < F; f++) {
    q[f][0] = q[f][1] = q[f][2] = q[f][3] = 0;
    if (mine) {
      if (vec) {
        const int4 qr = reinterpret_cast<const int4*>(q_ref + (uint64_t)f * n)[gid];
        q[f][0] = qr.x;
        q[f][1] = qr.y;
        q[f][2] = qr.z;
        q[f][3] = qr.w;
      } else {
        q[f][0] = q_ref[(uint64_t)f * n + gid];
      }
    }
  }
  // vector path: the next frame's values are requested while this frame is
  // coded (software pipelining: twice the loads in flight per wave).  A lane
  // without slots keeps zeros: it codes them like the others, and nothing of
  // it is stored or counted
  float xn[F][4];
#pragma unroll
  for (int f = 0; f < F; f++) xn[f][0] = xn[f][1] = xn[f][2] = xn[f][3] = 0.0f;
  // the values each array of a frame counts: four per lane with slots (one on
  // the scalar path)
  const uint32_t n_valid = (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(mine)) * (vec ? 4u : 1u);
  auto load_frame = [&](int j) {
#pragma unroll
    for (int f = 0; f < F; f++) {
      const float* x = fr.x[j][f];
      if (seq4 && ((uintptr_t)x & 3) == 0) {
        const float4_a4 v4 = *reinterpret_cast<const float4_a4*>(x + idx[0]);
        xn[f][0] = v4.x;
        xn[f][1] = v4.y;
        xn[f][2] = v4.z;
        xn[f][3] = v4.w;
      } else if (mine) {
#pragma unroll
        for (int u = 0; u < 4; u++) xn[f][u] = x[idx[u]];
      }
    }
  };
  if (vec) load_frame(0);
  __syncthreads();
  for (int j = 0; j < J; j++) {
    uint32_t bad = 0;
    float xc[F][4];
#pragma unroll
    for (int f = 0; f < F; f++)
#pragma unroll
      for (int u = 0; u < 4; u++) xc[f][u] = xn[f][u];
    if (vec && j + 1 < J) load_frame(j + 1);
#pragma unroll
    for (int f = 0; f < F; f++) {
      const uint64_t a = (uint64_t)(a0 + j) * F + f;
      uint32_t* shared = hist_part + (a * copies + copy) * kAlphabet;
      uint32_t* bins = bins_lds + (j * F + f) * kRunPriv;
      const float* x = fr.x[j][f];
      uint8_t* out8 = v8 + a * astride;
      uint32_t* oesc = vesc + a * astride;
      uint32_t rmax = 0;  // the lane's largest residual of this array
      HotCounts h{0u, 0u, 0u};
      if (vec) {
        const float* xv = xc[f];
        uint32_t rv[4], fl = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
          int32_t qc, qn;
          t_code_as(xv[u], DT, g, f, &fl, &qc);
          rv[u] = (uint32_t)zigzag32(t_step(qc, q[f][u], g.scale, &fl, &qn));
          q[f][u] = (int32_t)qn;
        }
        bad |= mine ? fl : 0u;
        if (mine) {
          rmax = max(max(rv[0], rv[1]), max(rv[2], rv[3]));
          uint32_t bytes = 0;
#pragma unroll
          for (int u = 0; u < 4; u++) bytes |= min(rv[u], 255u) << (8 * u);
          reinterpret_cast<uint32_t*>(out8)[gid] = bytes;
          if (rmax >= 255u) {
#pragma unroll
            for (int u = 0; u < 4; u++)
              if (rv[u] >= 255u) oesc[4 * gid + u] = rv[u];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; u++) hist_add_hot(h, shared, bins, kRunPriv, rv[u], mine);
      } else {
        uint32_t r = 0;
        if (mine) {
          int32_t qc, qn;
          t_code_as(x[idx[0]], DT, g, f, &bad, &qc);
          r = (uint32_t)zigzag32(t_step(qc, q[f][0], g.scale, &bad, &qn));
          q[f][0] = (int32_t)qn;
          out8[gid] = (uint8_t)min(r, 255u);
          if (r >= 255u) oesc[gid] = r;
          rmax = r;
        }
        hist_add_hot(h, shared, bins, kRunPriv, r, mine);
      }
      hist_flush_hot(h, bins, n_valid);
      const uint32_t wmax = wave_max_hot(h, rmax);
      if (lane_id() == 0 && wmax) atomicMax(&smax[j][f], wmax);
    }
    // the frame's error flags: each flagged lane reports its own (rare)
    if (bad) atomicOr(err + (uint64_t)j * err_stride, bad);
  }
  if (mine && q_last) {
#pragma unroll
    for (int f = 0; f < F; f++) {
      if (vec) reinterpret_cast<int4*>(q_last + (uint64_t)f * n)[gid] = make_int4(q[f][0], q[f][1], q[f][2], q[f][3]);
      else q_last[(uint64_t)f * n + gid] = q[f][0];
    }
  }
  __syncthreads();
  // every frame's counts into its arrays' spread copies (non-zero bins)
  for (int t = threadIdx.x; t < nbins; t += kThreads) {
    const uint32_t c = bins_lds[t];
    if (c) {
      const uint64_t a = (uint64_t)a0 * F + t / kRunPriv;  // t / kRunPriv = j F + f
      atomicAdd(&hist_part[(a * copies + copy) * kAlphabet + t % kRunPriv], c);
    }
  }
  if (threadIdx.x < (uint32_t)(J * F)) {
    const uint32_t m = (&smax[0][0])[threadIdx.x];
    if (m) atomicMax(&hist_max[((uint64_t)a0 * F + threadIdx.x) * copies + copy], (unsigned long long)m);
  }
}

// Temporal frames of several streams in one launch.  The launch's tiles of 256
// items (four slots each on a frame's vector path, one otherwise), counted
// frame after frame by the prefix table, are split into contiguous ranges, one
// per workgroup (a persistent grid of at most kMultiGrid workgroups); a
// workgroup codes its tiles exactly as k_t_resid codes a frame and keeps the
// counts of the frame it is in in its LDS bins, merging them into that frame's
// arrays' spread copies when it moves to the next frame and at the end (so a
// frame costs one merge per workgroup that touches it, not one per tile).
constexpr uint32_t kMultiGrid = 2048;
__global__ __launch_bounds__(kThreads) void k_t_resid_multi(const TFrameDev* T, const uint32_t* pre,
                                                            int R, int F, uint32_t tiles,
                                                            uint32_t* hist_part,
                                                            unsigned long long* hist_max,
                                                            int copies, ArrWork* zw) {
  extern __shared__ uint32_t bins_lds[];
  __shared__ uint32_t smax[kMaxF][kThreads / kWave];
  auto bins = [&](int f, int w) { return bins_lds + ((uint32_t)f * (kThreads / kWave) + w) * kResPriv; };
  for (int j = threadIdx.x; j < F * (kThreads / kWave) * kResPriv; j += kThreads) bins_lds[j] = 0;
  const int copy = blockIdx.x % copies;
  const uint32_t t0 = (uint32_t)((uint64_t)tiles * blockIdx.x / gridDim.x);
  const uint32_t t1 = (uint32_t)((uint64_t)tiles * (blockIdx.x + 1) / gridDim.x);
  uint32_t bad = 0;
  uint32_t rmax[kMaxF];
#pragma unroll
  for (int f = 0; f < kMaxF; f++) rmax[f] = 0;
  __syncthreads();
  // the counts, largest value and error bits gathered for frame r so far go
  // to its arrays; the bins start again from zero
  auto flush = [&](int r) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) bad |= (uint32_t)__shfl_xor((int)bad, d, kWave);
    if (lane_id() == 0 && bad) atomicOr(T[r].err, bad);
    for (int f = 0; f < F; f++) {
      uint32_t m = rmax[f];
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, kWave));
      if (lane_id() == 0) smax[f][wave_id()] = m;
    }
    __syncthreads();
    for (int f = 0; f < F; f++) {
      const uint64_t a = (uint64_t)r * F + f;
      uint32_t* shared = hist_part + (a * copies + copy) * kAlphabet;
      for (int j = threadIdx.x; j < kResPriv; j += kThreads) {
        uint32_t t = 0;
        for (int w = 0; w < kThreads / kWave; w++) {
          t += bins(f, w)[j];
          bins(f, w)[j] = 0;
        }
        if (t) atomicAdd(&shared[j], t);
      }
      if (threadIdx.x == 0) {
        uint32_t m = 0;
        for (int w = 0; w < kThreads / kWave; w++) m = max(m, smax[f][w]);
        if (m) atomicMax(&hist_max[a * copies + copy], (unsigned long long)m);
      }
    }
    __syncthreads();
    bad = 0;
#pragma unroll
    for (int f = 0; f < kMaxF; f++) rmax[f] = 0;
  };
  int cur = -1;
  for (uint32_t t = t0; t < t1; t++) {
    const int r = seg_of_block(pre, R, t);
    if (r != cur) {
      if (cur >= 0) flush(cur);
      cur = r;
    }
    const TFrameDev& fr = T[r];
    const uint32_t lb = t - pre[r];
    if (zw && lb == 0 && threadIdx.x < (uint32_t)(F * kWordParts))
      zw[(uint64_t)r * F + threadIdx.x / kWordParts].huff_words[threadIdx.x % kWordParts] = 0;
    const uint64_t n = fr.n;
    const uint64_t item = (uint64_t)lb * kThreads + threadIdx.x;
    const bool mine = item < (fr.vec ? n / 4 : n);
    uint32_t idx[4] = {0, 0, 0, 0};
    if (mine) {
      if (fr.vec) {
        const uint4 iv = reinterpret_cast<const uint4*>(fr.perm)[item];
        idx[0] = iv.x;
        idx[1] = iv.y;
        idx[2] = iv.z;
        idx[3] = iv.w;
      } else {
        idx[0] = fr.perm[item];
      }
    }
    // four consecutive inputs: one 16-byte load per field (see float4_a4)
    const bool seq4 = fr.vec && mine && idx[1] == idx[0] + 1 && idx[2] == idx[0] + 2 &&
                      idx[3] == idx[0] + 3;
    for (int f = 0; f < F; f++) {
      uint32_t* shared = hist_part + (((uint64_t)r * F + f) * copies + copy) * kAlphabet;
      uint32_t rv[4] = {0, 0, 0, 0};
      if (mine && fr.vec) {
        const float* x = fr.x[f];
        float xv[4];
        if (seq4 && ((uintptr_t)x & 3) == 0) {
          const float4_a4 v4 = *reinterpret_cast<const float4_a4*>(x + idx[0]);
          xv[0] = v4.x;
          xv[1] = v4.y;
          xv[2] = v4.z;
          xv[3] = v4.w;
        } else {
#pragma unroll
          for (int u = 0; u < 4; u++) xv[u] = x[idx[u]];
        }
        const int4 qr = reinterpret_cast<const int4*>(fr.q_ref + (uint64_t)f * n)[item];
        const int32_t qrv[4] = {qr.x, qr.y, qr.z, qr.w};
        int32_t qv[4];
        uint32_t bytes = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
          int32_t qc, q;
          t_code(xv[u], fr.g, f, &bad, &qc);
          rv[u] = (uint32_t)zigzag32(t_step(qc, qrv[u], fr.g.scale, &bad, &q));
          qv[u] = (int32_t)q;
          bytes |= min(rv[u], 255u) << (8 * u);
          rmax[f] = max(rmax[f], rv[u]);
        }
        reinterpret_cast<int4*>(fr.q_new + (uint64_t)f * n)[item] = make_int4(qv[0], qv[1], qv[2], qv[3]);
        reinterpret_cast<uint32_t*>(fr.v8 + (uint64_t)f * n)[item] = bytes;
#pragma unroll
        for (int u = 0; u < 4; u++)
          if (rv[u] >= 255u) fr.esc[(uint64_t)f * n + 4 * item + u] = rv[u];
      } else if (mine) {
        int32_t qc, q;
        t_code(fr.x[f][idx[0]], fr.g, f, &bad, &qc);
        rv[0] = (uint32_t)zigzag32(t_step(qc, fr.q_ref[(uint64_t)f * n + item], fr.g.scale, &bad, &q));
        fr.q_new[(uint64_t)f * n + item] = (int32_t)q;
        fr.v8[(uint64_t)f * n + item] = (uint8_t)min(rv[0], 255u);
        if (rv[0] >= 255u) fr.esc[(uint64_t)f * n + item] = rv[0];
        rmax[f] = max(rmax[f], rv[0]);
      }
      const int cnt = fr.vec ? 4 : 1;
      HotCounts h{0u, 0u, 0u};
      for (int u = 0; u < 4; u++)
        hist_add_hot(h, shared, bins(f, wave_id()), kResPriv, rv[u], mine && u < cnt);
      hist_flush_hot(h, bins(f, wave_id()),
                     (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(mine)) * (uint32_t)cnt);
    }
  }
  if (cur >= 0) flush(cur);
}

// Temporal frames of several streams reconstructed in one launch: workgroup b
// takes 1024 slots of the frame the prefix table gives it.
__global__ __launch_bounds__(kThreads) void k_t_recon_multi(const TReconDev* T, const uint32_t* pre,
                                                            int R, int F, uint32_t* err) {
  const int r = seg_of_block(pre, R, blockIdx.x);
  const TReconDev& fr = T[r];
  const uint64_t n = fr.n;
  const uint64_t s0 = (uint64_t)(blockIdx.x - pre[r]) * kSeg1k;
  uint32_t bad = 0;
  for (int f = 0; f < F; f++) {
    for (uint32_t j = threadIdx.x; j < kSeg1k; j += kThreads) {
      const uint64_t s = s0 + j;
      if (s >= n) break;
      int32_t rr = fr.r8[(uint64_t)f * n + s];
      if (rr == -128) rr = reinterpret_cast<const int32_t*>(fr.out[f])[s];
      int64_t q = (int64_t)fr.q_ref[(uint64_t)f * n + s] + (int64_t)fr.scale * rr;
      if (q < -(int64_t)kQLimit || q >= (int64_t)kQLimit) {
        bad = 1;
        q = 0;
      }
      fr.out[f][s] = reconstruct((int32_t)q, fr.eb_q[f], fr.m[f], fr.dtype);
      fr.q_new[(uint64_t)f * n + s] = (int32_t)q;
    }
  }
  if (bad) atomicOr(err, kErrCorrupt);
}

// The codes a temporal frame leaves as the next frame's reference: the frame's
// Eq. 5 codes on its reference grid, in the reference's slot order, moved in
// steps of the grid's scale from the reference's codes.  With step 1 they
// depend on the last frame alone; with a larger step the chain of J frames is
// followed from the codes q_ref of their first reference.  Either way they can
// be rebuilt when their slot was reused.
__global__ __launch_bounds__(kThreads) void k_t_codes(RunFrames fr, int J, int F, uint64_t n,
                                                      GridDev g, const uint32_t* perm_ref,
                                                      const int32_t* q_ref, int32_t* q_new,
                                                      uint32_t* err) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t bad = 0;
  const int j0 = g.scale == 1 ? J - 1 : 0;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
    const uint32_t i = perm_ref[s];
    for (int f = 0; f < F; f++) {
      int32_t c = g.scale == 1 ? 0 : q_ref[(uint64_t)f * n + s];
      for (int j = j0; j < J; j++) {
        int32_t q;
        t_code(fr.x[j][f][i], g, f, &bad, &q);
        t_step(q, c, g.scale, &bad, &c);
      }
      q_new[(uint64_t)f * n + s] = (int32_t)c;
    }
  }
  if (bad) atomicOr(err, bad);
}

// ------------------------------------------------------------------ spatial batch

__global__ __launch_bounds__(kThreads) void k_extent_b(const SegDev* S, const uint32_t* pre, int R,
                                                       uint32_t* part, uint32_t* err) {
  __shared__ uint32_t smn[kThreads / kWave], smx[kThreads / kWave];
  const int r = seg_of_block(pre, R, blockIdx.x);
  const uint32_t lb = blockIdx.x - pre[r], nb = pre[r + 1] - pre[r];
  const int f = blockIdx.y;
  const float* p = S[r].x[f];
  const uint64_t n = S[r].n;
  // order-preserving keys: float32 (float_key) or int32 (sign bit flipped)
  const int is_int = S[r].dtype;
  auto key_of = [&](float v) {
    return is_int ? __float_as_uint(v) ^ 0x80000000u : float_key(v);
  };
  uint32_t mn = 0xFFFFFFFFu, mx = 0u, bad = 0u;
  const uint64_t stride = (uint64_t)nb * blockDim.x;
  const uint64_t t0 = (uint64_t)lb * blockDim.x + threadIdx.x;
  // float4 body over the 16-byte aligned part, scalar head/tail
  uint64_t head = (uint64_t)((16 - ((uintptr_t)p & 15)) & 15) / 4;
  if (head > n) head = n;
  const uint64_t nv = (n - head) / 4;
  const float4* p4 = reinterpret_cast<const float4*>(p + head);
  for (uint64_t i = t0; i < nv; i += stride) {
    float4 v = p4[i];
    float a[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; j++) {
      uint32_t key = key_of(a[j]);
      mn = min(mn, key);
      mx = max(mx, key);
      bad |= !is_int && !__builtin_isfinite(a[j]);
    }
  }
  for (uint64_t i = t0; i < head + (n - head) % 4; i += stride) {
    uint64_t idx = i < head ? i : head + 4 * nv + (i - head);
    float v = p[idx];
    uint32_t key = key_of(v);
    mn = min(mn, key);
    mx = max(mx, key);
    bad |= !is_int && !__builtin_isfinite(v);
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor((int)mn, d, kWave));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, kWave));
    bad |= (uint32_t)__shfl_xor((int)bad, d, kWave);
  }
  if (lane_id() == 0) {
    smn[wave_id()] = mn;
    smx[wave_id()] = mx;
    if (bad) atomicOr(err, kErrNonFinite);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / kWave; w++) {
      mn = min(mn, smn[w]);
      mx = max(mx, smx[w]);
    }
    part[2 * ((uint64_t)f * gridDim.x + blockIdx.x)] = mn;
    part[2 * ((uint64_t)f * gridDim.x + blockIdx.x) + 1] = mx;
  }
}

// Workgroup (r, f): reduces frame r's partials of field f.
__global__ __launch_bounds__(kThreads) void k_extent_final_b(const uint32_t* part, const uint32_t* pre,
                                                             int R, int F, uint32_t total,
                                                             uint32_t* ext) {
  const int r = blockIdx.x, f = blockIdx.y;
  uint32_t mn = 0xFFFFFFFFu, mx = 0u;
  for (uint32_t b = pre[r] + threadIdx.x; b < pre[r + 1]; b += kThreads) {
    mn = min(mn, part[2 * ((uint64_t)f * total + b)]);
    mx = max(mx, part[2 * ((uint64_t)f * total + b) + 1]);
  }
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    mn = min(mn, (uint32_t)__shfl_xor((int)mn, d, kWave));
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, kWave));
  }
  __shared__ uint32_t smn[kThreads / kWave], smx[kThreads / kWave];
  if (lane_id() == 0) {
    smn[wave_id()] = mn;
    smx[wave_id()] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / kWave; w++) {
      mn = min(mn, smn[w]);
      mx = max(mx, smx[w]);
    }
    ext[(uint64_t)r * 2 * F + 2 * f] = mn;
    ext[(uint64_t)r * 2 * F + 2 * f + 1] = mx;
  }
}

// Eq. 5 and Eq. 6 per particle over the frame's D spatial axes (an axis the
// data does not have counts block 0).  vals = index within the frame.  rec
// holds, per particle in input order, what the slot pass needs of it in one
// padded record of rw words: the D offsets inside its block (k <= 16 bits each,
// 16 bits apart: word 0 for up to two axes, words 0-1 for three) and then the
// codes of the supplementary fields, so the slot pass gathers one record per
// slot instead of separate values.
// Persistent over the batch's tiles of `tile` slots (tile t of frame r at
// prefix pre[r]); every element-wise batch kernel below walks its tiles so.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_quant_key_b(const SegDev* S, const uint32_t* pre,
                                                          int R, int F, uint32_t tile,
                                                          uint32_t tiles, K* keys,
                                                          uint32_t* vals, uint32_t* rec, int rw) {
  for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
  const int r = seg_of_block(pre, R, t);
  const SegDev& g = S[r];
  const uint64_t n = g.n;
  const uint64_t i0 = (uint64_t)(t - pre[r]) * tile;
  const int k = g.k;
  const uint64_t pm = (1ull << k) - 1ull;
  for (uint32_t j = threadIdx.x; j < tile; j += kThreads) {
    const uint64_t i = i0 + j;
    if (i < n) {
      const int D = g.D;
      const uint64_t q0 = (uint64_t)quantise(word_value(g.x[0][i], g.dtype), g.md[0], g.inv[0]);
      const uint64_t q1 = D > 1 ? (uint64_t)quantise(word_value(g.x[1][i], g.dtype), g.md[1], g.inv[1]) : 0;
      const uint64_t q2 = D > 2 ? (uint64_t)quantise(word_value(g.x[2][i], g.dtype), g.md[2], g.inv[2]) : 0;
      const uint64_t b0 = q0 >> k, b1 = q1 >> k, b2 = q2 >> k;
      keys[g.off + i] = (K)(b0 + g.bn0 * (b1 + g.bn1 * b2));  // Eq. 6, x fastest
      vals[g.off + i] = (uint32_t)i;
      const uint64_t pr = (q0 & pm) | ((q1 & pm) << 16) | ((q2 & pm) << 32);
      uint32_t w[8] = {(uint32_t)pr, (uint32_t)(pr >> 32), 0, 0, 0, 0, 0, 0};
      // supplementary field f = D + j goes to word 2 + j with three axes, else
      // to word 1 + j (the offsets then fit word 0); constant word indices
      if (D == 3) {
#pragma unroll
        for (int j = 0; j < kMaxF - 3; j++)
          if (3 + j < F) w[2 + j] = (uint32_t)quantise(word_value(g.x[3 + j][i], g.dtype), g.md[3 + j], g.inv[3 + j]);
      } else {
#pragma unroll
        for (int j = 0; j < kMaxF - 1; j++)
          if (D + j < F) w[1 + j] = (uint32_t)quantise(word_value(g.x[D + j][i], g.dtype), g.md[D + j], g.inv[D + j]);
      }
      uint32_t* d = rec + (g.off + i) * (uint64_t)rw;
      if (rw == 2) {
        *reinterpret_cast<uint2*>(d) = make_uint2(w[0], w[1]);
      } else {
        *reinterpret_cast<uint4*>(d) = make_uint4(w[0], w[1], w[2], w[3]);
        if (rw == 8) *reinterpret_cast<uint4*>(d + 4) = make_uint4(w[4], w[5], w[6], w[7]);
      }
    }
  }
  }
}

// A slot starts a non-empty block when it is its frame's first slot or its key
// differs from the previous slot's.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_run_flags_b(const K* keys, const SegDev* S,
                                                          const uint32_t* pre, int R,
                                                          uint32_t tile, uint32_t tiles,
                                                          uint32_t* flags) {
  for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int r = seg_of_block(pre, R, t);
    const uint64_t n = S[r].n, off = S[r].off;
    const uint64_t i0 = (uint64_t)(t - pre[r]) * tile;
    for (uint32_t j = threadIdx.x; j < tile; j += kThreads) {
      const uint64_t i = i0 + j;
      if (i < n) flags[off + i] = (i == 0 || keys[off + i] != keys[off + i - 1]) ? 1u : 0u;
    }
  }
}

template <typename K>
__global__ __launch_bounds__(kThreads) void k_runs_write_b(const K* keys,
                                                           const uint32_t* scan, const SegDev* S,
                                                           const uint32_t* pre, int R,
                                                           uint32_t tile, uint32_t tiles,
                                                           uint64_t* ids, uint32_t* starts,
                                                           uint32_t* rstart, uint32_t* Bs) {
  for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
  const int r = seg_of_block(pre, R, t);
  const uint64_t n = S[r].n, off = S[r].off;
  const uint64_t i0 = (uint64_t)(t - pre[r]) * tile;
  for (uint32_t j = threadIdx.x; j < tile; j += kThreads) {
    const uint64_t i = i0 + j;
    if (i >= n) continue;
    const uint64_t g = off + i;
    if (i == 0 || keys[g] != keys[g - 1]) {
      const uint32_t b = scan[g] - 1;
      ids[b] = keys[g];
      starts[b] = (uint32_t)g;
      if (i == 0) rstart[r] = b;
    }
    if (i == n - 1) {
      Bs[r] = scan[g] - (off ? scan[off - 1] : 0u);
      if (r == R - 1) rstart[R] = scan[g];
    }
  }
  }
}

// Delta coding of block ids and counts (Sec. 6.2.2) per frame: id deltas,
// zigzag of count deltas; both restart at each frame's first block.
__global__ __launch_bounds__(kThreads) void k_block_syms_b(const uint64_t* ids,
                                                           const uint32_t* starts,
                                                           const uint32_t* rstart, int R,
                                                           const SegDev* S, uint64_t ntot,
                                                           uint64_t* v_id, uint64_t* v_cnt) {
  __shared__ uint32_t rs[kMaxBatch + 1];
  for (int j = threadIdx.x; j <= R; j += kThreads) rs[j] = rstart[j];
  __syncthreads();
  const uint64_t B = rs[R];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < B; b += stride) {
    int lo = 0, hi = R - 1;  // frame of block b: largest r with rs[r] <= b
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (rs[mid] <= b) lo = mid;
      else hi = mid - 1;
    }
    const bool first = b == rs[lo];
    const uint64_t dst = S[lo].off + (b - rs[lo]);
    v_id[dst] = ids[b] - (first ? 0 : ids[b - 1]);
    const int64_t c = (int64_t)((b + 1 < B ? (uint64_t)starts[b + 1] : ntot) - starts[b]);
    const int64_t cp = first ? 0 : (int64_t)(starts[b] - starts[b - 1]);
    v_cnt[dst] = zigzag64(c - cp);
  }
}

// Slot-order symbols, 256 slots per workgroup: each slot gathers its
// particle's record (offsets inside the block, supplementary codes); thread 0
// also reads the offsets of the slot before the workgroup's first, so that
// every relative position has its predecessor for the delta (mod p), which
// restarts at each frame's first slot.  q_slot (nullable) receives the codes in
// slot order: corner of the slot's block (from its sorted key) plus offset for
// x, y, z, the record's codes for the other fields.
__device__ inline void load_rec(const uint32_t* rec, uint64_t i, int rw, uint32_t* w) {
  const uint32_t* p = rec + i * (uint64_t)rw;
  if (rw == 2) {
    const uint2 a = *reinterpret_cast<const uint2*>(p);
    w[0] = a.x;
    w[1] = a.y;
  } else {
    const uint4 a = *reinterpret_cast<const uint4*>(p);
    w[0] = a.x;
    w[1] = a.y;
    w[2] = a.z;
    w[3] = a.w;
    if (rw == 8) {
      const uint4 b = *reinterpret_cast<const uint4*>(p + 4);
      w[4] = b.x;
      w[5] = b.y;
      w[6] = b.z;
      w[7] = b.w;
    }
  }
}

// RW: record words, a template parameter so that the record stays in registers
template <typename K, int RW>
__global__ __launch_bounds__(kThreads) void k_slot_syms_b(const SegDev* S, const uint32_t* pre,
                                                          int R, int F, const uint32_t* perm,
                                                          const K* keys,
                                                          const uint32_t* rec,
                                                          uint64_t ntot, uint32_t* v_rel,
                                                          uint32_t* v_sup, int32_t* q_slot,
                                                          uint32_t tiles) {
  __shared__ uint32_t rel[3][kThreads + 1];
  for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
  const int r = seg_of_block(pre, R, t);
  const SegDev& g = S[r];
  const uint64_t n = g.n, off = g.off;
  const uint64_t s0 = (uint64_t)(t - pre[r]) * kSeg256;
  const uint64_t s = s0 + threadIdx.x;
  const bool valid = s < n;
  if (valid) {
    const uint32_t i = perm[off + s];
    uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    load_rec(rec, off + i, RW, w);
    const int D = g.D;
    const uint64_t pr = (uint64_t)w[0] | (D == 3 ? (uint64_t)w[1] << 32 : 0ull);
    for (int d = 0; d < 3; d++) rel[d][threadIdx.x + 1] = (uint32_t)(pr >> (16 * d)) & 0xFFFFu;
    // supplementary codes in words w0.. (constant indices in each branch)
    uint32_t sup[kMaxF - 1];
    if (D == 3) {
#pragma unroll
      for (int j = 0; j < kMaxF - 1; j++) sup[j] = j < kMaxF - 2 ? w[2 + (j < kMaxF - 2 ? j : 0)] : 0u;
    } else {
#pragma unroll
      for (int j = 0; j < kMaxF - 1; j++) sup[j] = w[1 + j];
    }
#pragma unroll
    for (int j = 0; j < kMaxF - 1; j++)
      if (D + j < F) v_sup[(uint64_t)j * ntot + off + s] = sup[j];
    if (q_slot) {
      uint64_t b3[3];
      if constexpr (sizeof(K) == 4) {
        // 32-bit keys: the block counts per dimension are below 2^32 too, so
        // the block's coordinates come from 32-bit divisions
        const uint32_t key = keys[off + s], n0 = (uint32_t)g.bn0, n1 = (uint32_t)g.bn1;
        const uint32_t rest = key / n0;
        b3[0] = key - rest * n0;
        b3[1] = rest % n1;
        b3[2] = rest / n1;
      } else {
        const uint64_t key = (uint64_t)keys[off + s];
        const uint64_t rest = key / g.bn0;
        b3[0] = key % g.bn0;
        b3[1] = rest % g.bn1;
        b3[2] = rest / g.bn1;
      }
#pragma unroll
      for (int d = 0; d < 3; d++)
        if (d < D)
          q_slot[(uint64_t)d * ntot + off + s] = (int32_t)((b3[d] << g.k) + rel[d][threadIdx.x + 1]);
#pragma unroll
      for (int j = 0; j < kMaxF - 1; j++)
        if (D + j < F) q_slot[(uint64_t)(D + j) * ntot + off + s] = (int32_t)sup[j];
    }
  }
  if (threadIdx.x == 0) {
    if (s0 == 0) {
      rel[0][0] = rel[1][0] = rel[2][0] = 0;
    } else {
      const uint64_t j = off + perm[off + s0 - 1];
      const uint64_t pr = (uint64_t)rec[j * RW] | (g.D == 3 ? (uint64_t)rec[j * RW + 1] << 32 : 0ull);
      for (int d = 0; d < 3; d++) rel[d][0] = (uint32_t)(pr >> (16 * d)) & 0xFFFFu;
    }
  }
  const uint32_t pm = (1u << g.k) - 1u;
  __syncthreads();
  if (valid)
    for (int d = 0; d < g.D; d++)
      v_rel[(uint64_t)d * ntot + off + s] = (rel[d][threadIdx.x + 1] - rel[d][threadIdx.x]) & pm;
  __syncthreads();  // the next tile reuses rel
  }
}

__global__ __launch_bounds__(kThreads) void k_copy_perm_b(const uint32_t* perm, const SegDev* S,
                                                          const uint32_t* pre, int R,
                                                          uint32_t tile, uint32_t tiles,
                                                          uint32_t* const* dst) {
  for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int r = seg_of_block(pre, R, t);
    uint32_t* d = dst[r];
    if (!d) continue;
    const uint64_t n = S[r].n, off = S[r].off;
    const uint64_t i0 = (uint64_t)(t - pre[r]) * tile;
    for (uint32_t j = threadIdx.x; j < tile; j += kThreads) {
      const uint64_t i = i0 + j;
      if (i < n) d[i] = perm[off + i];
    }
  }
}

// ------------------------------------------------------------------ spatial batch decode
// Frames of a decode batch are concatenated like an encode batch: frame r owns
// slots [off, off + n) and blocks [boff, boff + B).  Per-frame inclusive scans
// are a batch-wide scan minus the scan value just before the frame.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_seg_bases(const T* X, uint64_t stride,
                                                        const DSegDev* D, int R, int by_block,
                                                        T* bases) {
  const int r = blockIdx.x * kThreads + threadIdx.x;
  const int d = blockIdx.y;
  if (r >= R) return;
  const uint64_t start = by_block ? D[r].boff : D[r].off;
  bases[(uint64_t)d * R + r] = start ? X[(uint64_t)d * stride + start - 1] : (T)0;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_seg_rebase(T* X, uint64_t stride, const DSegDev* D,
                                                         const uint32_t* pre, int R, int by_block,
                                                         const T* bases) {
  const int r = seg_of_block(pre, R, blockIdx.x);
  const int d = blockIdx.y;
  const uint64_t start = by_block ? D[r].boff : D[r].off;
  const uint64_t len = by_block ? D[r].B : D[r].n;
  const T base = bases[(uint64_t)d * R + r];
  const uint64_t i0 = (uint64_t)(blockIdx.x - pre[r]) * kSeg1k;
#pragma unroll
  for (int j = 0; j < (int)(kSeg1k / kThreads); j++) {
    const uint64_t i = i0 + (uint64_t)j * kThreads + threadIdx.x;
    if (i < len) X[(uint64_t)d * stride + start + i] -= base;
  }
}

// Per block: validate id / count, corner of the block in quantisation bins, and
// a start mark for the slot -> block expansion (every block but the batch's
// first).  ids and cnt hold per-frame inclusive scans of the decoded deltas;
// cum the batch-wide inclusive scan of the counts (slot ends).
__global__ __launch_bounds__(kThreads) void k_s_blocks_b(const uint64_t* ids, const uint64_t* cnt,
                                                         const uint64_t* cum, const DSegDev* D,
                                                         const uint32_t* pre, int R, uint64_t Btot,
                                                         uint64_t ntot, uint32_t* corner,
                                                         uint32_t* mark, uint32_t* err) {
  const int r = seg_of_block(pre, R, blockIdx.x);
  const DSegDev& g = D[r];
  const uint64_t j0 = (uint64_t)(blockIdx.x - pre[r]) * kSeg1k;
#pragma unroll
  for (int u = 0; u < (int)(kSeg1k / kThreads); u++) {
    const uint64_t jb = j0 + (uint64_t)u * kThreads + threadIdx.x;
    if (jb >= g.B) continue;
    const uint64_t j = g.boff + jb;
    const uint64_t id = ids[j];
    const uint64_t c = cnt[j];
    bool bad = id >= g.total_blocks || (jb > 0 && id <= ids[j - 1]) || c < 1 || c > g.n ||
               cum[j] > g.off + g.n;
    if (jb == g.B - 1 && cum[j] != g.off + g.n) bad = true;
    if (bad) {
      atomicOr(err, kErrCorrupt);
      continue;
    }
    const uint64_t start = cum[j] - c;
    const uint64_t bx = id % g.bn0, rest = id / g.bn0;
    const uint64_t by = rest % g.bn1, bz = rest / g.bn1;
    corner[j] = (uint32_t)(bx << g.k);
    corner[Btot + j] = (uint32_t)(by << g.k);
    corner[2 * Btot + j] = (uint32_t)(bz << g.k);
    if (j > 0 && start < ntot) mark[start] = 1u;
  }
}

// q = corner + relative position (fields 0-2) or the raw code (supplementary
// fields), then the float32 reconstruction into the frame's output arrays.
// blk holds the batch-wide block index of every slot, v the decoded slot
// symbols ([F][ntot]; relative positions already scanned per frame).
__global__ __launch_bounds__(kThreads) void k_s_recon_b(const uint32_t* blk, const uint32_t* corner,
                                                        const uint32_t* v, const DSegDev* D,
                                                        const uint32_t* pre, int R, int F,
                                                        uint64_t Btot, uint64_t ntot,
                                                        uint32_t* err) {
  const int r = seg_of_block(pre, R, blockIdx.x);
  const DSegDev& g = D[r];
  const uint32_t pm = (1u << g.k) - 1u;
  const uint64_t s0 = (uint64_t)(blockIdx.x - pre[r]) * kSeg1k;
  bool bad = false;
#pragma unroll
  for (int u = 0; u < (int)(kSeg1k / kThreads); u++) {
    const uint64_t s = s0 + (uint64_t)u * kThreads + threadIdx.x;
    if (s >= g.n) continue;
    const uint64_t gs = g.off + s;
    const uint64_t b = blk[gs];
    if (b < g.boff || b >= g.boff + g.B) {
      bad = true;
      continue;
    }
    for (int f = 0; f < F; f++) {
      uint64_t q = f < g.D ? (uint64_t)corner[(uint64_t)f * Btot + b] + (v[(uint64_t)f * ntot + gs] & pm)
                           : (uint64_t)v[(uint64_t)f * ntot + gs];
      if (q >= (uint64_t)kQLimit) {
        bad = true;
        q = 0;
      }
      g.out[f][s] = reconstruct((int32_t)q, g.eb_q[f], g.m[f], g.dtype);
    }
  }
  if (bad) atomicOr(err, kErrCorrupt);
}

// ------------------------------------------------------------------ decode side
// Per block: validate id / count, corner of the block in quantisation bins, and
// a start mark for the slot -> block expansion.  ids and cnt hold inclusive
// scans of the decoded deltas; cum is the inclusive scan of the counts.
__global__ __launch_bounds__(kThreads) void k_s_blocks(const uint64_t* ids,
                                                       const uint64_t* cnt,
                                                       const uint64_t* cum, uint64_t B,
                                                       uint64_t n, uint64_t total_blocks,
                                                       uint32_t bn0, uint32_t bn1, int k,
                                                       uint32_t* corner, uint32_t* mark,
                                                       uint32_t* err) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < B; b += stride) {
    uint64_t id = ids[b];
    uint64_t c = cnt[b];
    bool bad = id >= total_blocks || (b > 0 && id <= ids[b - 1]) || c < 1 || c > n;
    if (b == B - 1 && cum[b] != n) bad = true;
    uint64_t start = cum[b] - c;
    if (bad) {
      atomicOr(err, kErrCorrupt);
      continue;
    }
    uint64_t bx = id % bn0, rest = id / bn0;
    uint64_t by = rest % bn1, bz = rest / bn1;
    corner[b] = (uint32_t)(bx << k);
    corner[B + b] = (uint32_t)(by << k);
    corner[2 * B + b] = (uint32_t)(bz << k);
    if (b > 0 && start < n) mark[start] = 1u;
  }
}

__global__ __launch_bounds__(kThreads) void k_s_recon(const uint32_t* blk, const uint32_t* corner,
                                                      uint64_t B, int F, int D, uint64_t n, int k,
                                                      GridDev g, OutPtrs out, int32_t* q_slot,
                                                      uint32_t* err) {
  const uint32_t pm = (1u << k) - 1u;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += stride) {
    uint64_t b = blk[s];
    if (b >= B) {
      atomicOr(err, kErrCorrupt);
      continue;
    }
    for (int f = 0; f < F; f++) {
      uint32_t* cell = reinterpret_cast<uint32_t*>(out.p[f]) + s;
      uint64_t q;
      if (f < D) q = (uint64_t)corner[(uint64_t)f * B + b] + (*cell & pm);
      else q = *cell;
      if (q >= (uint64_t)kQLimit) {
        atomicOr(err, kErrCorrupt);
        q = 0;
      }
      out.p[f][s] = reconstruct((int32_t)q, g.eb_q[f], g.m[f], g.dtype);
      if (q_slot) q_slot[(uint64_t)f * n + s] = (int32_t)q;
    }
  }
}

// LCP-T decode: q = q_ref + residual (residuals decoded as int32 in place).
__global__ __launch_bounds__(kThreads) void k_t_recon(const int32_t* q_ref, int F, uint64_t n,
                                                      GridDev g, OutPtrs out, int32_t* q_slot,
                                                      uint32_t* err, int vec) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t bad = 0;
  if (vec) {
    for (uint64_t s4 = gid; s4 < n / 4; s4 += stride) {
      for (int f = 0; f < F; f++) {
        const int4 r = reinterpret_cast<const int4*>(out.p[f])[s4];
        const int4 qr = reinterpret_cast<const int4*>(q_ref + (uint64_t)f * n)[s4];
        const int64_t sc = g.scale;
        int64_t q[4] = {(int64_t)qr.x + sc * r.x, (int64_t)qr.y + sc * r.y,
                        (int64_t)qr.z + sc * r.z, (int64_t)qr.w + sc * r.w};
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
          if (q[j] < -(int64_t)kQLimit || q[j] >= (int64_t)kQLimit) {
            bad = 1;
            q[j] = 0;
          }
          o[j] = reconstruct((int32_t)q[j], g.eb_q[f], g.m[f], g.dtype);
        }
        reinterpret_cast<float4*>(out.p[f])[s4] = make_float4(o[0], o[1], o[2], o[3]);
        if (q_slot)
          reinterpret_cast<int4*>(q_slot + (uint64_t)f * n)[s4] =
              make_int4((int)q[0], (int)q[1], (int)q[2], (int)q[3]);
      }
    }
  } else {
    for (uint64_t s = gid; s < n; s += stride) {
      for (int f = 0; f < F; f++) {
        const int32_t r = reinterpret_cast<const int32_t*>(out.p[f])[s];
        int64_t q = (int64_t)q_ref[(uint64_t)f * n + s] + (int64_t)g.scale * r;
        if (q < -(int64_t)kQLimit || q >= (int64_t)kQLimit) {
          bad = 1;
          q = 0;
        }
        out.p[f][s] = reconstruct((int32_t)q, g.eb_q[f], g.m[f], g.dtype);
        if (q_slot) q_slot[(uint64_t)f * n + s] = (int32_t)q;
      }
    }
  }
  if (bad) atomicOr(err, kErrCorrupt);
}

// A chain of J temporal frames, each coded against the one before it (the
// first against q_ref): per slot the codes stay in registers while each
// frame's residuals (int32, decoded in place in its output arrays) are added
// and its float32 values written; only the last frame's codes are stored.
constexpr int kChainGroup = 8;  // frames of a chain whose residuals load together
typedef float F4 __attribute__((ext_vector_type(4)));

// A residual read as an int32 word (an escape, or a frame without byte
// residuals) outside +-2^25 cannot come from a valid record (codes and steps
// keep |s r| below 2^24): it is flagged and taken as 0, so the 32-bit code
// arithmetic below cannot overflow.
__device__ inline int32_t checked_residual(int32_t r, uint32_t* bad) {
  if ((uint32_t)(r + (1 << 25)) >= (1u << 26)) {
    *bad = 1;
    return 0;
  }
  return r;
}

template <int DT>
__global__ __launch_bounds__(kThreads) void k_t_recon_chain(const int32_t* q_ref, int F,
                                                            uint64_t n, GridDev g, ChainOut out,
                                                            int J, int32_t* q_last, uint32_t* err,
                                                            int vec) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t bad = 0;
  if (vec) {
    for (uint64_t s4 = gid; s4 < n / 4; s4 += stride) {
      for (int f = 0; f < F; f++) {
        const int4 qr = reinterpret_cast<const int4*>(q_ref + (uint64_t)f * n)[s4];
        int32_t q[4] = {qr.x, qr.y, qr.z, qr.w};
        // one frame of the chain: rr holds its four residuals (|rr| < 2^25)
        auto step = [&](int j, const int32_t* rr) {
          float v[4];
#pragma unroll
          for (int u = 0; u < 4; u++) {
            q[u] += g.scale * rr[u];
            if (q[u] < -kQLimit || q[u] >= kQLimit) {
              bad = 1;
              q[u] = 0;
            }
            v[u] = reconstruct(q[u], g.eb_q[f], g.m[f], DT);
          }
          // written once and not read again here: a streaming (non-temporal) store
          const F4 vv = {v[0], v[1], v[2], v[3]};
          __builtin_nontemporal_store(vv, reinterpret_cast<F4*>(out.p[j][f]) + s4);
        };
        for (int j0 = 0; j0 < J; j0 += kChainGroup) {
          const int G = min(kChainGroup, J - j0);
          bool bytes = true;
          for (int k = 0; k < G; k++) bytes = bytes && out.r8[j0 + k][f] != nullptr;
          uint32_t bw[kChainGroup];
          uint32_t esc = 0;
          if (bytes) {
            // the group's residual words are requested together (a store to
            // one frame's output could alias the next frame's residuals, so
            // loads issued frame by frame would each wait for memory in turn)
#pragma unroll
            for (int k = 0; k < kChainGroup; k++)
              bw[k] = reinterpret_cast<const uint32_t*>(out.r8[j0 + min(k, G - 1)][f])[s4];
#pragma unroll
            for (int k = 0; k < kChainGroup; k++) {
              const uint32_t x = bw[k] ^ 0x80808080u;  // a zero byte: an escape (-128)
              if (k < G) esc |= (x - 0x01010101u) & ~x & 0x80808080u;
            }
          }
          if (bytes && __ballot(esc != 0) == 0) {
            // no escapes in the wave: no loads between the stores
#pragma unroll
            for (int k = 0; k < kChainGroup; k++) {
              if (k >= G) break;
              int32_t rr[4];
#pragma unroll
              for (int u = 0; u < 4; u++) rr[u] = (int32_t)(int8_t)(uint8_t)(bw[k] >> (8 * u));
              step(j0 + k, rr);
            }
          } else {
            for (int k = 0; k < G; k++) {
              const int j = j0 + k;
              const int32_t* o = reinterpret_cast<const int32_t*>(out.p[j][f]) + 4 * s4;
              int32_t rr[4];
              if (out.r8[j][f]) {
                const uint32_t b = reinterpret_cast<const uint32_t*>(out.r8[j][f])[s4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                  rr[u] = (int32_t)(int8_t)(uint8_t)(b >> (8 * u));
                  if (rr[u] == -128) rr[u] = checked_residual(o[u], &bad);  // escaped: the int32 residual
                }
              } else {
                const int4 r = *reinterpret_cast<const int4*>(o);
                rr[0] = checked_residual(r.x, &bad);
                rr[1] = checked_residual(r.y, &bad);
                rr[2] = checked_residual(r.z, &bad);
                rr[3] = checked_residual(r.w, &bad);
              }
              step(j, rr);
            }
          }
        }
        if (q_last)
          reinterpret_cast<int4*>(q_last + (uint64_t)f * n)[s4] = make_int4(q[0], q[1], q[2], q[3]);
      }
    }
  } else {
    for (uint64_t s = gid; s < n; s += stride) {
      for (int f = 0; f < F; f++) {
        int32_t q = q_ref[(uint64_t)f * n + s];
        for (int j = 0; j < J; j++) {
          int32_t r;
          if (out.r8[j][f]) {
            r = out.r8[j][f][s];
            if (r == -128) r = checked_residual(reinterpret_cast<const int32_t*>(out.p[j][f])[s], &bad);
          } else {
            r = checked_residual(reinterpret_cast<const int32_t*>(out.p[j][f])[s], &bad);
          }
          q += g.scale * r;
          if (q < -kQLimit || q >= kQLimit) {
            bad = 1;
            q = 0;
          }
          out.p[j][f][s] = reconstruct(q, g.eb_q[f], g.m[f], DT);
        }
        if (q_last) q_last[(uint64_t)f * n + s] = q;
      }
    }
  }
  if (bad) atomicOr(err, kErrCorrupt);
}

// Record r of a merged launch (bytes [offs[r], offs[r+1]) of src) to its own
// destination tab[2r] when it fits the capacity tab[2r + 1]; blockIdx.y
// strides over its words.
__global__ void k_scatter_records(const unsigned long long* offs, const uint8_t* src,
                                  const uint64_t* tab, int R) {
  const int r = blockIdx.x;
  const uint64_t lo = offs[r], size = offs[r + 1] - lo;
  if (size > tab[2 * r + 1]) return;
  uint32_t* d = reinterpret_cast<uint32_t*>((uintptr_t)tab[2 * r]);
  const uint32_t* s = reinterpret_cast<const uint32_t*>(src + lo);
  const uint64_t words = size / 4, stride = (uint64_t)gridDim.y * blockDim.x;
  for (uint64_t w = (uint64_t)blockIdx.y * blockDim.x + threadIdx.x; w < words; w += stride) d[w] = s[w];
}

// Copies the first min(size, stage) bytes (whole words) of every record into a
// staging array, one workgroup per record.
__global__ void k_gather_headers(const uint64_t* tab, int stage, uint8_t* dst) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>((uintptr_t)tab[2 * blockIdx.x]);
  const uint64_t size = tab[2 * blockIdx.x + 1];
  const uint64_t words = (size < (uint64_t)stage ? size : (uint64_t)stage) / 4;
  uint32_t* d = reinterpret_cast<uint32_t*>(dst + (uint64_t)stage * blockIdx.x);
  for (uint64_t w = threadIdx.x; w < words; w += blockDim.x) d[w] = src[w];
}

// Small host tables travel as a kernel argument: no copy-engine round trip.
struct InstallArg {
  uint32_t w[kInstallWords];
};
__global__ void k_install(InstallArg a, uint32_t* dst, uint32_t words) {
  for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) dst[i] = a.w[i];
}

// System-scope loads: what the host wrote before the launch is what is read,
// whatever the GPU's caches hold of the pinned pages from an earlier fetch.
__global__ void k_fetch_host(const uint32_t* src, uint32_t* dst, uint32_t words) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_copy_u32(const uint32_t* src, uint32_t* dst, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

}  // namespace

// ------------------------------------------------------------------ launchers
uint32_t seg_ext_blocks(uint64_t n) { return grid_for(n / 4 + 1, kThreads * 4, kSegExtCap); }

void launch_extent_b(const SegDev* S, const uint32_t* pre_ext, uint32_t ext_blocks, int R, int F,
                     uint32_t* ext, uint32_t* part, uint32_t* err, uint64_t bytes, hipStream_t s) {
  launch_timed("extent", bytes, k_extent_b, dim3(ext_blocks, F), kThreads, 0, s,
               S, pre_ext, R, part, err);
  k_extent_final_b<<<dim3(R, F), kThreads, 0, s>>>(part, pre_ext, R, F, ext_blocks, ext);
}

// Frames one run launch takes at F fields: its LDS counts (J F kRunPriv words)
// stay within 48 KiB.
int run_launch_frames(int F) {
  const int j = (48 << 10) / (F * kRunPriv * 4);
  return j < kRunMax ? j : kRunMax;
}

int slot_rec_words(int F, int D) {
  const int w = (D == 3 ? 2 : 1) + (F - D);  // offsets, then supplementary codes
  return w <= 2 ? 2 : (w <= 4 ? 4 : 8);
}

inline uint32_t persistent_grid(uint32_t tiles, uint32_t grid) {
  return grid && grid < tiles ? grid : (tiles ? tiles : 1);
}

void launch_quant_key_b(const SegDev* S, const uint32_t* pre_tile, const TileShape& ts, int R,
                        int F, int D, uint64_t* keys, uint32_t* vals, uint32_t* rec, uint64_t ntot,
                        bool key32, hipStream_t s) {
  const int rw = slot_rec_words(F, D);
  const uint64_t bytes = ntot * (4ull * F + (key32 ? 8 : 12) + 4ull * rw);
  const uint32_t g = persistent_grid(ts.tiles, ts.grid);
  if (key32)
    launch_timed("quant_key", bytes, k_quant_key_b<uint32_t>, g, kThreads, 0, s, S, pre_tile, R,
                 F, ts.tile, ts.tiles, reinterpret_cast<uint32_t*>(keys), vals, rec, rw);
  else
    launch_timed("quant_key", bytes, k_quant_key_b<uint64_t>, g, kThreads, 0, s, S, pre_tile, R,
                 F, ts.tile, ts.tiles, keys, vals, rec, rw);
}

void launch_runs_b(const uint64_t* keys, const SegDev* S, const uint32_t* pre_tile,
                   const TileShape& ts, int R, uint64_t ntot, uint32_t* flags_scan, uint64_t* ids,
                   uint32_t* starts, uint32_t* rstart, uint32_t* Bs, uint32_t* tmp32,
                   bool key32, hipStream_t s) {
  const uint32_t g = persistent_grid(ts.tiles, ts.grid);
  const uint32_t* k32 = reinterpret_cast<const uint32_t*>(keys);
  if (key32)
    k_run_flags_b<uint32_t><<<g, kThreads, 0, s>>>(k32, S, pre_tile, R, ts.tile, ts.tiles, flags_scan);
  else
    k_run_flags_b<uint64_t><<<g, kThreads, 0, s>>>(keys, S, pre_tile, R, ts.tile, ts.tiles, flags_scan);
  scan_device<uint32_t>(flags_scan, ntot, nullptr, false, tmp32, s);
  if (key32)
    k_runs_write_b<uint32_t><<<g, kThreads, 0, s>>>(k32, flags_scan, S, pre_tile, R, ts.tile,
                                                    ts.tiles, ids, starts, rstart, Bs);
  else
    k_runs_write_b<uint64_t><<<g, kThreads, 0, s>>>(keys, flags_scan, S, pre_tile, R, ts.tile,
                                                    ts.tiles, ids, starts, rstart, Bs);
}

void launch_block_syms_b(const uint64_t* ids, const uint32_t* starts, const uint32_t* rstart,
                         int R, const SegDev* S, uint64_t ntot, uint64_t* v_id, uint64_t* v_cnt,
                         hipStream_t s) {
  k_block_syms_b<<<grid_for(ntot, kThreads * 4, 1u << 16), kThreads, 0, s>>>(
      ids, starts, rstart, R, S, ntot, v_id, v_cnt);
}

void launch_slot_syms_b(const SegDev* S, const uint32_t* pre_256, uint32_t tiles, uint32_t grid,
                        int R, int F, int D, const uint32_t* perm, const uint64_t* keys,
                        const uint32_t* rec, uint64_t ntot, uint32_t* v_rel, uint32_t* v_sup,
                        int32_t* q_slot, bool key32, hipStream_t s) {
  const int rw = slot_rec_words(F, D);
  uint64_t bytes = ntot * (4 + 4ull * rw + 4ull * F + (q_slot ? (key32 ? 4 : 8) + 4ull * F : 0));
  const uint32_t g = persistent_grid(tiles, grid);
  // one instance per key width and record width (2, 4 or 8 words)
  auto pick = [&](auto kt) {
    using K = typename decltype(kt)::type;
    auto* k = k_slot_syms_b<K, 2>;
    if (rw == 4) k = k_slot_syms_b<K, 4>;
    else if (rw == 8) k = k_slot_syms_b<K, 8>;
    return k;
  };
  if (key32)
    launch_timed("slot_syms", bytes, pick(std::common_type<uint32_t>()), g, kThreads, 0, s, S,
                 pre_256, R, F, perm, reinterpret_cast<const uint32_t*>(keys), rec, ntot, v_rel,
                 v_sup, q_slot, tiles);
  else
    launch_timed("slot_syms", bytes, pick(std::common_type<uint64_t>()), g, kThreads, 0, s, S,
                 pre_256, R, F, perm, keys, rec, ntot, v_rel, v_sup, q_slot, tiles);
}

void launch_copy_perm_b(const uint32_t* perm, const SegDev* S, const uint32_t* pre_tile,
                        const TileShape& ts, int R, uint32_t* const* dst, hipStream_t s) {
  k_copy_perm_b<<<persistent_grid(ts.tiles, ts.grid), kThreads, 0, s>>>(perm, S, pre_tile, R,
                                                                          ts.tile, ts.tiles, dst);
}

int radix_result(int bits) { return ((bits + 7) / 8) & 1; }

template <typename K>
int radix_sort_k(K* k0, uint32_t* v0, K* k1, uint32_t* v1, const SegDev* S,
                 const uint32_t* pre_tile, uint32_t ntiles, int R, uint64_t ntot, int bits,
                 uint32_t* hist, uint32_t* tmp32, hipStream_t s) {
  const uint64_t entries = (uint64_t)ntiles * 256;
  int cur = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    K* kin = cur ? k1 : k0;
    uint32_t* vin = cur ? v1 : v0;
    K* kout = cur ? k0 : k1;
    uint32_t* vout = cur ? v0 : v1;
    k_radix_hist<K><<<ntiles, kThreads, 0, s>>>(kin, S, pre_tile, R, shift, hist);
    scan_device<uint32_t>(hist, entries, nullptr, true, tmp32, s);
    launch_timed("radix_scatter", ntot * (2 * sizeof(K) + 8), k_radix_scatter<K>, ntiles, kThreads,
                 0, s, kin, vin, kout, vout, S, pre_tile, R, shift, hist, entries, ntot);
    cur ^= 1;
  }
  return cur;
}

int radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, const SegDev* S,
               const uint32_t* pre_tile, uint32_t ntiles, int R, uint64_t ntot, int bits,
               uint32_t* hist, uint32_t* tmp32, bool key32, hipStream_t s) {
  if (key32)
    return radix_sort_k<uint32_t>(reinterpret_cast<uint32_t*>(k0), v0,
                                  reinterpret_cast<uint32_t*>(k1), v1, S, pre_tile, ntiles, R, ntot,
                                  bits, hist, tmp32, s);
  return radix_sort_k<uint64_t>(k0, v0, k1, v1, S, pre_tile, ntiles, R, ntot, bits, hist, tmp32, s);
}

size_t scan_tmp_elems(uint64_t n) {
  size_t t = 0;
  uint64_t m = n;
  while (m > (uint64_t)kScanTile) {
    m = (m + kScanTile - 1) / kScanTile;
    t += m;
  }
  // four arrays side by side (scan_device4) need four sets of tile sums
  return 4 * t + 16;
}

template <typename T>
void scan_device(T* data, uint64_t n, const uint32_t* n_dev, bool exclusive, T* tmp,
                 hipStream_t s) {
  if (n == 0) return;
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    k_scan_apply<T><<<1, kThreads, 0, s>>>(data, n, n_dev, nullptr, exclusive ? 1 : 0);
    return;
  }
  k_scan_reduce<T><<<(uint32_t)tiles, kThreads, 0, s>>>(data, n, n_dev, tmp);
  scan_device<T>(tmp, tiles, nullptr, true, tmp + tiles, s);
  k_scan_apply<T><<<(uint32_t)tiles, kThreads, 0, s>>>(data, n, n_dev, tmp, exclusive ? 1 : 0);
}
template void scan_device<uint32_t>(uint32_t*, uint64_t, const uint32_t*, bool, uint32_t*,
                                    hipStream_t);

void scan_device4(uint32_t* const* arrs, int nd, uint64_t n, uint32_t* tmp, hipStream_t s) {
  if (n == 0 || nd <= 0) return;
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (nd > 4 || tiles > (uint64_t)kScanTile) {  // tile sums past one tile: one array at a time
    for (int d = 0; d < nd; d++) scan_device<uint32_t>(arrs[d], n, nullptr, false, tmp, s);
    return;
  }
  ScanSet a;
  memset(&a, 0, sizeof(a));
  for (int d = 0; d < nd; d++) a.p[d] = arrs[d];
  if (tiles == 1) {
    k_scan_apply4<<<dim3(1, nd), kThreads, 0, s>>>(a, n, nullptr, 0, 0);
    return;
  }
  ScanSet t;
  memset(&t, 0, sizeof(t));
  for (int d = 0; d < nd; d++) t.p[d] = tmp + (uint64_t)d * tiles;
  k_scan_reduce4<<<dim3((uint32_t)tiles, nd), kThreads, 0, s>>>(a, n, tmp, (uint32_t)tiles);
  k_scan_apply4<<<dim3(1, nd), kThreads, 0, s>>>(t, tiles, nullptr, 0, 1);
  k_scan_apply4<<<dim3((uint32_t)tiles, nd), kThreads, 0, s>>>(a, n, tmp, (uint32_t)tiles, 0);
}
template void scan_device<uint64_t>(uint64_t*, uint64_t, const uint32_t*, bool, uint64_t*,
                                    hipStream_t);

template <typename T>
void seg_rebase(T* X, uint64_t stride, int nd, const DSegDev* D, const uint32_t* pre,
                uint32_t blocks, int R, bool by_block, T* bases, hipStream_t s) {
  if (R == 1) return;  // a lone frame starts the batch: its base is zero
  k_seg_bases<T><<<dim3((R + kThreads - 1) / kThreads, nd), kThreads, 0, s>>>(X, stride, D, R,
                                                                            by_block, bases);
  k_seg_rebase<T><<<dim3(blocks, nd), kThreads, 0, s>>>(X, stride, D, pre, R, by_block, bases);
}
template void seg_rebase<uint32_t>(uint32_t*, uint64_t, int, const DSegDev*, const uint32_t*,
                                   uint32_t, int, bool, uint32_t*, hipStream_t);
template void seg_rebase<uint64_t>(uint64_t*, uint64_t, int, const DSegDev*, const uint32_t*,
                                   uint32_t, int, bool, uint64_t*, hipStream_t);

void launch_s_blocks_b(const uint64_t* ids, const uint64_t* cnt, const uint64_t* cum,
                       const DSegDev* D, const uint32_t* pre_blk, uint32_t blocks, int R,
                       uint64_t Btot, uint64_t ntot, uint32_t* corner, uint32_t* mark,
                       uint32_t* err, hipStream_t s) {
  k_s_blocks_b<<<blocks, kThreads, 0, s>>>(ids, cnt, cum, D, pre_blk, R, Btot, ntot, corner, mark,
                                           err);
}

void launch_s_recon_b(const uint32_t* blk, const uint32_t* corner, const uint32_t* v,
                      const DSegDev* D, const uint32_t* pre_slot, uint32_t blocks, int R, int F,
                      uint64_t Btot, uint64_t ntot, uint32_t* err, hipStream_t s) {
  launch_timed("s_recon", ntot * (4 + 12 + 8ull * F), k_s_recon_b, blocks, kThreads, 0, s,
               blk, corner, v, D, pre_slot, R, F, Btot, ntot, err);
}

inline bool al16(const void* p) { return ((uintptr_t)p & 15) == 0; }

void launch_t_resid(const FieldPtrs& x, int F, uint64_t n, const GridDev& g,
                    const uint32_t* perm_ref, const int32_t* q_ref, uint8_t* v8, uint32_t* v_res,
                    int32_t* q_new, uint32_t* err, uint32_t* hist_part,
                    unsigned long long* hist_max, ArrWork* zero_words, hipStream_t s) {
  const int vec = (n % 4 == 0) && al16(perm_ref) && al16(q_ref) && al16(v_res) && al16(q_new) &&
                  (!v8 || al16(v8));
  // algorithmic bytes: this kernel's share of what LCP-T compression must move
  // per particle -- the frame (4F), the reference codes (4F) and the slot
  // permutation (4) read, the new reference codes (4F) written; the residual
  // symbols it hands to the coder are an intermediate, not counted.  One item
  // per thread up to 4096 workgroups (a 4,194,304-particle frame in one pass):
  // two items per thread on half the workgroups measured 3-4% slower.
  launch_timed("t_resid", n * (4 + 12ull * F), k_t_resid, grid_for(vec ? n / 4 : n, kThreads, 4096), kThreads, (size_t)F * (kThreads / kWave) * kResPriv * 4, s,
               x, F, n, g, perm_ref, q_ref, v8, v_res, q_new, err, vec, hist_part, hist_max,
               zero_words);
}

void launch_t_resid_run(const RunFrames& fr, int J, int F, uint64_t n, const GridDev& g,
                        const uint32_t* perm, const int32_t* q_ref, int32_t* q_last, uint8_t* v8,
                        uint32_t* vesc, uint64_t astride, int a0, uint32_t* hist_part,
                        unsigned long long* hist_max, int copies, ArrWork* zero_words,
                        uint32_t* err, int err_stride, hipStream_t s) {
  if (J < 1 || n == 0) return;
  int vec = (n % 4 == 0) && al16(perm) && al16(q_ref) && (!q_last || al16(q_last)) &&
            (astride % 16 == 0) && al16(v8);
  const uint64_t items = vec ? n / 4 : n;
  // algorithmic bytes: the per-frame figure of LCP-T compression (a frame, its
  // reference codes and the permutation read, its codes written: 4 + 12F per
  // particle) for each of the J frames.  The kernel itself moves less -- J
  // frames read and their residual bytes written, the permutation and the first
  // reference codes read and the last codes written once -- since the codes
  // stay in registers from frame to frame
  // one instance per field count and element type
  auto pick = [&](auto dt) {
    constexpr int D = decltype(dt)::value;
    auto* k = k_t_resid_run<3, D>;
    switch (F) {
      case 1: k = k_t_resid_run<1, D>; break;
      case 2: k = k_t_resid_run<2, D>; break;
      case 4: k = k_t_resid_run<4, D>; break;
      case 5: k = k_t_resid_run<5, D>; break;
      case 6: k = k_t_resid_run<6, D>; break;
      case 7: k = k_t_resid_run<7, D>; break;
      case 8: k = k_t_resid_run<8, D>; break;
      default: break;
    }
    return k;
  };
  auto* kernel = g.dtype == kDtypeI32 ? pick(std::integral_constant<int, kDtypeI32>())
                                      : pick(std::integral_constant<int, kDtypeF32>());
  launch_timed("t_resid_run", n * (uint64_t)J * (4 + 12ull * F), kernel,
               grid_for(items, kThreads, 1u << 24), kThreads,
               (size_t)J * F * kRunPriv * 4, s, fr, J, n, g, perm, q_ref,
               q_last, v8, vesc, astride, a0, hist_part, hist_max, copies, zero_words, err,
               err_stride, vec);
}

uint32_t t_multi_blocks(uint64_t n, int vec) {
  const uint64_t items = vec ? n / 4 : n;
  return (uint32_t)((items + kThreads - 1) / kThreads);
}

void launch_t_resid_multi(const TFrameDev* frames, const uint32_t* pre, uint32_t blocks, int R,
                          int F, uint32_t* hist_part, unsigned long long* hist_max, int copies,
                          ArrWork* zero_words, uint64_t bytes, hipStream_t s) {
  if (!blocks) return;
  const uint32_t grid = blocks < kMultiGrid ? blocks : kMultiGrid;
  launch_timed("t_resid", bytes, k_t_resid_multi, grid, kThreads,
               (size_t)F * (kThreads / kWave) * kResPriv * 4, s, frames, pre, R, F, blocks,
               hist_part, hist_max, copies, zero_words);
}

void launch_t_recon_multi(const TReconDev* frames, const uint32_t* pre, uint32_t blocks, int R,
                          int F, uint32_t* err, uint64_t bytes, hipStream_t s) {
  if (!blocks) return;
  launch_timed("t_recon", bytes, k_t_recon_multi, blocks, kThreads, 0, s, frames, pre, R, F, err);
}

void launch_t_codes(const RunFrames& fr, int J, int F, uint64_t n, const GridDev& g,
                    const uint32_t* perm_ref, const int32_t* q_ref, int32_t* q_new,
                    uint32_t* err, hipStream_t s) {
  k_t_codes<<<grid_for(n, kThreads * 4, 1u << 16), kThreads, 0, s>>>(fr, J, F, n, g, perm_ref,
                                                                      q_ref, q_new, err);
}

void launch_s_blocks(const uint64_t* ids, const uint64_t* cnt, uint64_t* cum, uint64_t B,
                     uint64_t n, uint64_t total_blocks, const uint32_t* bn, int k,
                     uint32_t* corner, uint32_t* mark, uint32_t* err, hipStream_t s) {
  k_s_blocks<<<grid_for(B, kThreads * 4, 1u << 16), kThreads, 0, s>>>(
      ids, cnt, cum, B, n, total_blocks, bn[0], bn[1], k, corner, mark, err);
}

void launch_s_recon(const uint32_t* blk, const uint32_t* corner, uint64_t B, int F, int D, uint64_t n,
                    int k, const GridDev& g, const OutPtrs& out, int32_t* q_slot, uint32_t* err,
                    hipStream_t s) {
  launch_timed("s_recon", n * (4 + 12 + 8ull * F + (q_slot ? 4ull * F : 0)), k_s_recon, grid_for(n, kThreads * 4, 1u << 16), kThreads, 0, s,
               blk, corner, B, F, D, n, k, g, out, q_slot, err);
}

void launch_t_recon(const int32_t* q_ref, int F, uint64_t n, const GridDev& g,
                    const OutPtrs& out, int32_t* q_slot, uint32_t* err, hipStream_t s) {
  int vec = (n % 4 == 0) && al16(q_ref) && (!q_slot || al16(q_slot));
  for (int f = 0; f < F; f++) vec = vec && al16(out.p[f]);
  launch_timed("t_recon", n * (12ull * F + (q_slot ? 4ull * F : 0)), k_t_recon, grid_for(vec ? n / 4 : n, kThreads * 2, 1u << 16), kThreads, 0, s,
               q_ref, F, n, g, out, q_slot, err, vec);
}

void launch_t_recon_chain(const int32_t* q_ref, int F, uint64_t n, const GridDev& g,
                          const ChainOut& out, int J, int32_t* q_last, uint32_t* err,
                          hipStream_t s) {
  int vec = (n % 4 == 0) && al16(q_ref) && (!q_last || al16(q_last));
  uint64_t per = 0;  // bytes per slot: residuals read and values written
  for (int j = 0; j < J; j++)
    for (int f = 0; f < F; f++) {
      vec = vec && al16(out.p[j][f]) && (reinterpret_cast<uintptr_t>(out.r8[j][f]) & 3) == 0;
      per += out.r8[j][f] ? 5 : 8;
    }
  auto* kernel = g.dtype == kDtypeI32 ? k_t_recon_chain<kDtypeI32> : k_t_recon_chain<kDtypeF32>;
  launch_timed("t_recon", n * (per + 4ull * F + (q_last ? 4ull * F : 0)), kernel,
               grid_for(vec ? n / 4 : n, kThreads * 2, 1u << 16), kThreads, 0, s, q_ref, F, n, g,
               out, J, q_last, err, vec);
}

void launch_scatter_records(const unsigned long long* offs, const uint8_t* src, const uint64_t* tab,
                            int R, hipStream_t s) {
  if (R > 0) k_scatter_records<<<dim3(R, 16), kThreads, 0, s>>>(offs, src, tab, R);
}

void launch_gather_headers(const uint64_t* tab, int nrec, int stage, uint8_t* dst, hipStream_t s) {
  if (nrec) k_gather_headers<<<nrec, 128, 0, s>>>(tab, stage, dst);
}

void launch_install(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const uint8_t* sp = static_cast<const uint8_t*>(src);
  uint8_t* dp = static_cast<uint8_t*>(dst);
  while (bytes) {
    const size_t chunk = bytes < (size_t)kInstallWords * 4 ? bytes : (size_t)kInstallWords * 4;
    InstallArg a;
    memcpy(a.w, sp, chunk);
    k_install<<<1, 256, 0, s>>>(a, reinterpret_cast<uint32_t*>(dp), (uint32_t)(chunk / 4));
    sp += chunk;
    dp += chunk;
    bytes -= chunk;
  }
}

void launch_fetch_host(const void* host_src, void* dst, size_t bytes, hipStream_t s) {
  const uint32_t words = (uint32_t)(bytes / 4);
  if (words)
    k_fetch_host<<<(words + 255) / 256, 256, 0, s>>>(static_cast<const uint32_t*>(host_src),
                                                      static_cast<uint32_t*>(dst), words);
}

void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n) k_fill_u32<<<grid_for(n, kThreads * 4, 1u << 16), kThreads, 0, s>>>(p, n, v);
}

void launch_copy_perm(const uint32_t* src, uint32_t* dst, uint64_t n, hipStream_t s) {
  if (n) k_copy_u32<<<grid_for(n, kThreads * 4, 1u << 16), kThreads, 0, s>>>(src, dst, n);
}

}  // namespace lcp
