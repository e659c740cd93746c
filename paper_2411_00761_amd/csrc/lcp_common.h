// lcp_common.h -- format constants and wave64 device primitives shared by the
// LCP HIP kernels (gfx950, 64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lcp {

// ---- frame record layout (little-endian) ----
constexpr uint32_t kMagic = 0x3150434Cu;  // bytes "LCP1"
constexpr int kVersion = 1;
constexpr int kHdrBytes = 80;
constexpr int kDirBytes = 32;
constexpr int kMaxF = 8;
constexpr int kMaxArrays = kMaxF + 2;  // spatial record: ID, CNT, REL x/y/z, F-3 supplementary

// ---- entropy coder ----
// Values below kDirect are Huffman symbols themselves; a value v >= kDirect is
// the symbol kDirect + bitwidth(v) - kFirstClassBits followed by its
// bitwidth(v) - 1 low bits (the leading one is implied).
constexpr int kDirect = 4096;
constexpr int kFirstClassBits = 13;
constexpr int kAlphabet = kDirect + 64 - kFirstClassBits + 1;  // 4148
constexpr int kMaxLen = 13;                                     // longest Huffman code
constexpr int kQLimit = 1 << 23;  // |2q+1| < 2^24: (float)(2q+1) is exact

constexpr int kWave = 64;

__host__ __device__ inline int bitwidth64(uint64_t v) {
#ifdef __HIP_DEVICE_COMPILE__
  return v ? 64 - __clzll((long long)v) : 0;
#else
  return v ? 64 - __builtin_clzll(v) : 0;
#endif
}

__host__ __device__ inline uint64_t zigzag64(int64_t d) {
  return d >= 0 ? (uint64_t)d << 1 : (((uint64_t)(-(d + 1))) << 1) | 1u;
}
__host__ __device__ inline uint32_t zigzag32(int32_t d) {
  return ((uint32_t)d << 1) ^ (uint32_t)(d >> 31);
}
__host__ __device__ inline int64_t unzigzag64(uint64_t z) {
  return (z & 1) ? -(int64_t)(z >> 1) - 1 : (int64_t)(z >> 1);
}

// Huffman symbol of a value and the count of raw bits that follow its code.
__device__ inline int symbol_of(uint64_t v, int* extra) {
  if (v < (uint64_t)kDirect) {
    *extra = 0;
    return (int)v;
  }
  int b = bitwidth64(v);
  *extra = b - 1;
  return kDirect + b - kFirstClassBits;
}

// Element types of the input fields: every field of a plan is float32, or
// every field is int32 (a 4-byte word either way; kernels load the word as a
// float and reinterpret it for int32 plans).
constexpr int kDtypeF32 = 0, kDtypeI32 = 1;

// Four floats read with one 16-byte load from any 4-byte aligned address: CDNA
// global loads of four dwords need dword alignment only (the compiler emits
// global_load_dwordx4 for this type), so a run of four consecutive inputs is
// one load wherever it starts.
typedef float float4_a4 __attribute__((ext_vector_type(4), aligned(4)));

// Value of an input word, exact in double for both types.
__device__ inline double word_value(float w, int is_int) {
  return is_int ? (double)__float_as_int(w) : (double)w;
}

// Eq. 5 on the device: floor((x - md) * inv), IEEE double, no contraction (the
// build passes -ffp-contract=off).  float32 grids: md = m, inv = 1 / (2 eb_q).
// int32 grids: md = m - 1/2 and inv = 1 / w (rounded) for bins of w integers;
// then (x - md) = d + 1/2 with d = x - m an integer below 2^33 in magnitude,
// and (d + 1/2) / w lies at least 1 / (2w) from every integer while the two
// roundings move it by at most 2^-52 (d + 1/2) / w < 2^-19 / w, so the floor
// is floor(d / w) exactly.
// The codes in use lie within +-2^23: a value beyond the int32 range is held
// at its ends (NaN gives 0), where every caller's range check (or its
// finiteness test) rejects it, so one saturating 32-bit conversion serves
// instead of a 64-bit one.  The instruction saturates by itself; it is named
// directly because the language leaves an out-of-range conversion undefined.
__device__ inline int32_t cvt_i32_sat(double t) {
  int32_t r;
  asm("v_cvt_i32_f64 %0, %1" : "=v"(r) : "v"(t));
  return r;
}
__device__ inline int32_t quantise(double x, double md, double inv) {
  return cvt_i32_sat(floor((x - md) * inv));
}

// Reconstruction as a 4-byte output word from a code within +-2^23 (every
// caller range-checks it first, so 2q+1 is exact in 32 bits and converts to
// float in one instruction).  float32: (2q+1) eb_q + m, one rounding.  int32
// (m and eb_q then hold the bits of the origin and of the half width hb):
// m + q (2 hb + 1) + hb, held to the int32 range, which only moves a value
// toward its input.
__device__ inline float reconstruct(int32_t q, float eb_q, float m, int is_int) {
  if (is_int) {
    const int64_t hb = (int64_t)__float_as_uint(eb_q);
    int64_t v = (int64_t)__float_as_int(m) + (int64_t)q * (2 * hb + 1) + hb;
    v = v > (int64_t)INT32_MAX ? (int64_t)INT32_MAX : v;
    v = v < (int64_t)INT32_MIN ? (int64_t)INT32_MIN : v;
    return __int_as_float((int32_t)v);
  }
  return __builtin_fmaf((float)(2 * q + 1), eb_q, m);
}

__device__ inline int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ inline int wave_id() { return (int)(threadIdx.x / kWave); }
__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Inclusive prefix sums across the 64 lanes of a wave.
template <typename T>
__device__ inline T wave_incl_scan(T v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(v, d, kWave);
    if (lane_id() >= d) v += o;
  }
  return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Inclusive block-wide scan; `sm` holds at least blockDim.x / 64 + 1 values.
// Returns the inclusive prefix; *total receives the block total.
template <typename T>
__device__ inline T block_incl_scan(T v, T* sm, T* total) {
  const int nw = (int)(blockDim.x / kWave);
  T x = wave_incl_scan(v);
  if (lane_id() == kWave - 1) sm[wave_id()] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int w = 0; w < nw; w++) {
      T t = sm[w];
      sm[w] = run;
      run += t;
    }
    sm[nw] = run;
  }
  __syncthreads();
  T r = x + sm[wave_id()];
  *total = sm[nw];
  __syncthreads();
  return r;
}

// Adds the symbols of the active lanes of a wave to a histogram.  The first
// active lane's symbol is broadcast and its peers found with one ballot; one
// lane adds that group's size (a wave of identical symbols, e.g. zero
// residuals, costs one update) and every other lane adds 1 with an LDS atomic.
// Symbols below n_priv go to the wave-private bins `priv`, the rest to
// `shared`.
__device__ inline void wave_hist_add(uint32_t* shared, uint32_t* priv, int n_priv, uint32_t sym,
                                     bool valid) {
  const uint64_t todo = __builtin_amdgcn_ballot_w64(valid);
  if (!todo) return;
  const int l = __ffsll((long long)todo) - 1;
  const uint32_t s0 = (uint32_t)__builtin_amdgcn_readlane((int)sym, l);
  const uint64_t m = __builtin_amdgcn_ballot_w64(valid && sym == s0);
  uint32_t* bins = sym < (uint32_t)n_priv ? priv : shared;
  if (lane_id() == l) atomicAdd(&bins[sym], (uint32_t)__popcll(m));
  else if (valid && sym != s0) atomicAdd(&bins[sym], 1u);
}

// A temporally coded frame's residuals are nearly all 0, 1 and 2 after zigzag
// (0, -1 and +1), values that are their own symbols.  The wave counts 1, 2 and
// the rest with one ballot each into wave-uniform counters, which stay in
// scalar registers; the zeros are what remains of the values the caller knows
// it counted, and all three reach the bins once per array and frame
// (hist_flush_hot).  Only when some lane holds a value above 2 is its symbol
// formed and counted through wave_hist_add.  The private bins must hold
// symbols 0..2.
struct HotCounts {
  uint32_t c1, c2, rest;
};
__device__ inline void hist_add_hot(HotCounts& h, uint32_t* shared, uint32_t* priv, int n_priv,
                                    uint32_t v, bool valid) {
  // the bool ballot takes the compare mask as it is (no 0/1 round trip)
  h.c1 += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(valid && v == 1u));
  h.c2 += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(valid && v == 2u));
  const bool rest = valid && v > 2u;
  const uint64_t rm = __builtin_amdgcn_ballot_w64(rest);
  if (rm) {
    h.rest += (uint32_t)__popcll(rm);
    int e;
    wave_hist_add(shared, priv, n_priv, (uint32_t)symbol_of(v, &e), rest);
  }
}
// The largest value a wave counted, given each lane's own largest (0 for a lane
// without values): read off the hot counts unless some lane holds a value
// above 2, which alone costs a butterfly reduction.  Every lane of the wave
// must be active.
__device__ inline uint32_t wave_max_hot(const HotCounts& h, uint32_t m_lane) {
  if (__builtin_amdgcn_ballot_w64(m_lane > 2u)) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) m_lane = max(m_lane, (uint32_t)__shfl_xor((int)m_lane, d, kWave));
    return m_lane;
  }
  return h.c2 ? 2u : (h.c1 ? 1u : 0u);
}
// n_valid: the values the wave passed as valid since the counters started.
__device__ inline void hist_flush_hot(const HotCounts& h, uint32_t* priv, uint32_t n_valid) {
  const uint32_t c0 = n_valid - h.c1 - h.c2 - h.rest;
  // one lane adds them: the first active one (a grid-stride loop's last
  // iteration may have left out the low lanes)
  if (lane_id() == __ffsll((long long)__ballot(1)) - 1) {
    if (c0) atomicAdd(&priv[0], c0);
    if (h.c1) atomicAdd(&priv[1], h.c1);
    if (h.c2) atomicAdd(&priv[2], h.c2);
  }
}

// Sortable unsigned image of a float (monotone: a < b  <=>  key(a) < key(b)).
__host__ __device__ inline uint32_t float_key(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float key_float(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

}  // namespace lcp
