/*
 * lcp_oracle.c -- plain, slow, single-threaded CPU oracle of LCP-S / LCP-T.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the benchmark's
 * CPU-baseline leg to check the GPU library.  Shares no code with it.
 *
 * Each function follows one passage of the paper (arXiv 2411.00761):
 *   quantisation .............. Sec. 6.1, Eq. 5
 *   block id / size ........... Sec. 6.2.1, Eq. 6 (over the spatial dimensions, 1 to 3;
 *                               Sec. 4 allows data of other dimensions)
 *   block triples ............. Sec. 6.2.1 (non-empty blocks: id, count, relative
 *                               position to the block's (0,0,0) corner)
 *   delta coding .............. Sec. 6.2.2 (D_i - D_{i-1} on each array)
 *   Huffman / fixed selection . Sec. 6.2.2, Tab. 3 (expected length incl. table)
 *   LCP-T ..................... Sec. 7.1 (difference against the previous frame)
 *   LCP-FSM ................... Sec. 7.2 (S estimated by last S size; T tested with
 *                               a back-off S1X -> S2X -> S4X ...)
 *   anchor frames ............. Sec. 7.3, Alg. 1
 *   anchor error-bound scale .. Sec. 7.4.2 (anchors at eb / 5 while frames are
 *                               temporally correlated)
 *   block-size search ......... Sec. 7.4.1 (candidates 2^k, 0<=k<=16, on a sample)
 * The readings taken where the paper is silent (rounding margin, modular deltas,
 * escape classes, length limit, chunking, record layout, FSM details) are each
 * stated where they are used below.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.  No contraction,
 * so every double/float operation is one IEEE operation in round-to-nearest.
 */
#include "lcp_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAGIC 0x3150434Cu /* bytes "LCP1" */
#define VERSION 1
#define HDR_BYTES 80
#define DIR_BYTES 32
#define DIRECT_SYMBOLS 4096 /* values below this are Huffman symbols themselves */
#define FIRST_CLASS_BITS 13 /* smallest bit width of a value >= 4096 */
#define ALPHABET (DIRECT_SYMBOLS + 64 - FIRST_CLASS_BITS + 1) /* 4148 */
#define MAX_CODE_LEN 13
#define Q_LIMIT (1 << 23) /* |2q+1| < 2^24 keeps (float)(2q+1) exact */

/* ------------------------------------------------------------------ */
/* little-endian byte helpers                                          */
/* ------------------------------------------------------------------ */
static void put_u8(uint8_t* p, unsigned v) { p[0] = (uint8_t)v; }
static void put_u16(uint8_t* p, unsigned v) {
  p[0] = (uint8_t)v;
  p[1] = (uint8_t)(v >> 8);
}
static void put_u32(uint8_t* p, uint32_t v) {
  for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i));
}
static void put_u64(uint8_t* p, uint64_t v) {
  for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i));
}
static void put_f32(uint8_t* p, float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  put_u32(p, u);
}
static uint32_t get_u32(const uint8_t* p) {
  uint32_t v = 0;
  for (int i = 0; i < 4; i++) v |= (uint32_t)p[i] << (8 * i);
  return v;
}
static uint64_t get_u64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 0; i < 8; i++) v |= (uint64_t)p[i] << (8 * i);
  return v;
}
static float get_f32(const uint8_t* p) {
  uint32_t u = get_u32(p);
  float f;
  memcpy(&f, &u, 4);
  return f;
}

static int bitwidth(uint64_t v) {
  int b = 0;
  while (v) {
    b++;
    v >>= 1;
  }
  return b;
}
static uint64_t zigzag(int64_t d) { return d >= 0 ? (uint64_t)d * 2 : (uint64_t)(-(d + 1)) * 2 + 1; }
static int64_t unzigzag(uint64_t z) { return (z & 1) ? -(int64_t)(z >> 1) - 1 : (int64_t)(z >> 1); }

/* ------------------------------------------------------------------ */
/* a1: extent and error bound                                          */
/* ------------------------------------------------------------------ */
int lco_extent(const void* const* x, int F, uint64_t n, int dtype, double* lo, double* hi) {
  if (F < 1 || F > LCO_MAX_F || n == 0) return LCO_ERR_ARG;
  if (dtype != LCO_DTYPE_F32 && dtype != LCO_DTYPE_I32) return LCO_ERR_ARG;
  for (int f = 0; f < F; f++) {
    if (dtype == LCO_DTYPE_I32) {
      const int32_t* v = (const int32_t*)x[f];
      int32_t a = v[0], b = v[0];
      for (uint64_t i = 0; i < n; i++) {
        if (v[i] < a) a = v[i];
        if (v[i] > b) b = v[i];
      }
      lo[f] = (double)a;
      hi[f] = (double)b;
      continue;
    }
    const float* v = (const float*)x[f];
    float a = v[0], b = v[0];
    for (uint64_t i = 0; i < n; i++) {
      if (!isfinite(v[i])) return LCO_ERR_ARG;
      if (v[i] < a) a = v[i];
      if (v[i] > b) b = v[i];
    }
    /* -0 and +0 compare equal; the extent is taken as +0 so that the origin
     * written to the record does not depend on which zero came first */
    lo[f] = a == 0.0f ? 0.0 : (double)a;
    hi[f] = b == 0.0f ? 0.0 : (double)b;
  }
  return LCO_OK;
}

/* Value range of D is max(D) - min(D) (Sec. 4, PSNR definition).  The global
 * relative mode takes it over all fields; the per-field mode per field. */
int lco_field_eb(int eb_mode, double eb, int F, const double* lo, const double* hi, int dtype,
                 double* eb_f) {
  if (!(eb > 0) || !isfinite(eb)) return LCO_ERR_ARG;
  if (eb_mode == LCO_EB_ABS) {
    for (int f = 0; f < F; f++) eb_f[f] = eb;
  } else if (eb_mode == LCO_EB_REL_GLOBAL) {
    double a = lo[0], b = hi[0];
    for (int f = 1; f < F; f++) {
      if (lo[f] < a) a = lo[f];
      if (hi[f] > b) b = hi[f];
    }
    double r = b - a;
    for (int f = 0; f < F; f++) eb_f[f] = eb * r;
  } else if (eb_mode == LCO_EB_REL_PER_FIELD) {
    for (int f = 0; f < F; f++) eb_f[f] = eb * (hi[f] - lo[f]);
  } else {
    return LCO_ERR_ARG;
  }
  /* integers can always be kept exactly: a bound of 0 codes them losslessly */
  for (int f = 0; f < F; f++)
    if (dtype == LCO_DTYPE_I32 ? !(eb_f[f] >= 0) : !(eb_f[f] > 0)) return LCO_ERR_EB_TOO_SMALL;
  return LCO_OK;
}

/* Eq. 5 with the FP32 output in mind.  The exact reconstruction (2q+1)eb_q + m is
 * within eb_q of x; rounding it to float adds at most half an ulp of the top
 * binade 2^E.  Taking eb_q <= eb - 2^(E-24) therefore keeps |x - x'| <= eb. */
int lco_make_grid(float lo, float hi, double eb_f, lco_grid* g) {
  if (!isfinite(lo) || !isfinite(hi) || !(eb_f > 0) || !isfinite(eb_f)) return LCO_ERR_ARG;
  double a = fabs((double)lo), b = fabs((double)hi);
  double M = (a > b ? a : b) + 2.0 * eb_f;
  if (!isfinite(M)) return LCO_ERR_RANGE; /* the bound overflows the double range */
  int E;
  frexp(M, &E); /* M < 2^E */
  if (E < -100) E = -100;
  double delta = ldexp(1.0, E - 24);
  if (!(eb_f >= 2.0 * delta)) return LCO_ERR_EB_TOO_SMALL;
  double t = eb_f - delta;
  float e = (float)t;
  if ((double)e > t) e = nextafterf(e, 0.0f); /* round down */
  if (!(e > 0.0f)) return LCO_ERR_EB_TOO_SMALL;
  memset(g, 0, sizeof(*g));
  g->dtype = LCO_DTYPE_F32;
  g->m = lo;
  g->eb_q = e;
  g->inv = 1.0 / (2.0 * (double)e);
  g->eb = eb_f;
  g->E = E;
  return LCO_OK;
}

/* q = floor((x - m) / (2 eb_q)), evaluated as ((double)x - (double)m) * inv. */
int64_t lco_quant(float x, const lco_grid* g) {
  double t = ((double)x - (double)g->m) * g->inv;
  return (int64_t)floor(t);
}

/* x' = (2q+1) eb_q + m, one rounding to float (fused multiply-add). */
float lco_recon(int64_t q, const lco_grid* g) {
  return fmaf((float)(2 * q + 1), g->eb_q, g->m);
}

/* Integer fields (Sec. 3 allows them).  Eq. 5's bins of width 2 eb become runs
 * of w = 2 hb + 1 consecutive integers from the origin mi, and a value is
 * reconstructed as the integer at the centre of its run: within hb <= eb of
 * it, exactly, with no rounding margin.  hb = floor(eb) is the widest such run.
 * For an anchor whose chained temporal frames move by s bins (Sec. 7.4.2, s
 * odd) the error of those frames is up to (s w - 1) / 2, so w is the largest
 * odd integer with s w <= 2 floor(eb) + 1. */
int lco_make_grid_i(int32_t lo, double eb_f, int s, lco_grid* g) {
  if (!(eb_f >= 0) || s < 1 || s % 2 == 0) return LCO_ERR_ARG;
  /* a run of 2^32 - 1 integers covers any int32 field; wider bounds change nothing */
  int64_t b = eb_f >= 2147483647.0 ? 2147483647 : (int64_t)floor(eb_f);
  int64_t w = (2 * b + 1) / s;
  if (w % 2 == 0) w -= 1;
  if (w < 1) return LCO_ERR_EB_TOO_SMALL;
  memset(g, 0, sizeof(*g));
  g->dtype = LCO_DTYPE_I32;
  g->mi = lo;
  g->hb = (w - 1) / 2;
  g->eb = eb_f;
  return LCO_OK;
}

/* q = floor((x - mi) / w), exact integer division rounded down. */
int64_t lco_quant_i(int32_t x, const lco_grid* g) {
  int64_t d = (int64_t)x - (int64_t)g->mi, w = 2 * g->hb + 1;
  int64_t q = d / w; /* C rounds toward zero */
  if (d % w != 0 && d < 0) q -= 1;
  return q;
}

/* x' = mi + q w + hb, held to the int32 range: x lies in [INT32_MIN, INT32_MAX],
 * so a centre outside it moves toward x when clamped and stays within hb. */
int32_t lco_recon_i(int64_t q, const lco_grid* g) {
  int64_t v = (int64_t)g->mi + q * (2 * g->hb + 1) + g->hb;
  if (v > INT32_MAX) v = INT32_MAX;
  if (v < INT32_MIN) v = INT32_MIN;
  return (int32_t)v;
}

/* Code of x[f][i] or of an extent value v on the field's grid, either type. */
static int64_t quant_at(const void* const* x, int f, uint64_t i, const lco_grid* g) {
  if (g->dtype == LCO_DTYPE_I32) return lco_quant_i(((const int32_t*)x[f])[i], g);
  return lco_quant(((const float*)x[f])[i], g);
}
static int64_t quant_val(double v, const lco_grid* g) {
  return g->dtype == LCO_DTYPE_I32 ? lco_quant_i((int32_t)v, g) : lco_quant((float)v, g);
}

void lco_quantize(const float* x, uint64_t n, const lco_grid* g, int64_t* q) {
  for (uint64_t i = 0; i < n; i++) q[i] = lco_quant(x[i], g);
}

void lco_reconstruct(const int64_t* q, uint64_t n, const lco_grid* g, float* out) {
  for (uint64_t i = 0; i < n; i++) out[i] = lco_recon(q[i], g);
}

/* ------------------------------------------------------------------ */
/* a6: Huffman code lengths                                            */
/* ------------------------------------------------------------------ */
typedef struct {
  uint64_t w;
  int sym;
} leaf_t;

static int leaf_cmp(const void* a, const void* b) {
  const leaf_t* x = (const leaf_t*)a;
  const leaf_t* y = (const leaf_t*)b;
  if (x->w != y->w) return x->w < y->w ? -1 : 1;
  return x->sym < y->sym ? -1 : (x->sym > y->sym);
}

/* One Huffman build: leaves sorted by (count, symbol); internal nodes kept in
 * creation order (a FIFO, their weights never decrease); each step takes the
 * lighter head, the leaf on a tie.  Returns the longest code length. */
static int huffman_once(const uint64_t* counts, int K, uint8_t* len) {
  int U = 0;
  for (int s = 0; s < K; s++) len[s] = 0;
  for (int s = 0; s < K; s++) U += counts[s] > 0;
  if (U == 0) return 0;
  leaf_t* lv = (leaf_t*)malloc(sizeof(leaf_t) * U);
  int j = 0;
  for (int s = 0; s < K; s++)
    if (counts[s]) {
      lv[j].w = counts[s];
      lv[j].sym = s;
      j++;
    }
  qsort(lv, U, sizeof(leaf_t), leaf_cmp);
  if (U == 1) {
    len[lv[0].sym] = 1;
    free(lv);
    return 1;
  }
  int nodes = 2 * U - 1;
  uint64_t* w = (uint64_t*)malloc(sizeof(uint64_t) * nodes);
  int* parent = (int*)malloc(sizeof(int) * nodes);
  int* depth = (int*)malloc(sizeof(int) * nodes);
  for (int i = 0; i < U; i++) w[i] = lv[i].w;
  int li = 0, ii = U, next = U; /* leaf head, internal head, next internal */
  while (next < nodes) {
    int pick[2];
    for (int t = 0; t < 2; t++) {
      int take_leaf;
      if (li >= U) take_leaf = 0;
      else if (ii >= next) take_leaf = 1;
      else take_leaf = w[li] <= w[ii];
      pick[t] = take_leaf ? li++ : ii++;
    }
    w[next] = w[pick[0]] + w[pick[1]];
    parent[pick[0]] = next;
    parent[pick[1]] = next;
    next++;
  }
  depth[nodes - 1] = 0;
  for (int i = nodes - 2; i >= 0; i--) depth[i] = depth[parent[i]] + 1;
  int mx = 0;
  for (int i = 0; i < U; i++) {
    len[lv[i].sym] = (uint8_t)depth[i];
    if (depth[i] > mx) mx = depth[i];
  }
  free(lv);
  free(w);
  free(parent);
  free(depth);
  return mx;
}

/* Length-limited lengths: while the longest code exceeds 13 bits, every count
 * becomes ceil(count/2) and the code is rebuilt. */
int lco_huffman_lengths(const uint64_t* counts, int K, uint8_t* len) {
  uint64_t* c = (uint64_t*)malloc(sizeof(uint64_t) * (K > 0 ? K : 1));
  memcpy(c, counts, sizeof(uint64_t) * K);
  int mx;
  for (;;) {
    mx = huffman_once(c, K, len);
    if (mx <= MAX_CODE_LEN) break;
    for (int s = 0; s < K; s++)
      if (c[s]) c[s] = (c[s] + 1) / 2;
  }
  free(c);
  return mx;
}

/* Canonical codes (shorter first, then by symbol; RFC 1951 Sec. 3.2.2). */
static void canonical_codes(const uint8_t* len, int K, uint32_t* code) {
  int bl_count[MAX_CODE_LEN + 2] = {0};
  uint32_t next_code[MAX_CODE_LEN + 2] = {0};
  for (int s = 0; s < K; s++)
    if (len[s]) bl_count[len[s]]++;
  uint32_t c = 0;
  for (int l = 1; l <= MAX_CODE_LEN; l++) {
    c = (c + (uint32_t)bl_count[l - 1]) << 1;
    next_code[l] = c;
  }
  for (int s = 0; s < K; s++) code[s] = len[s] ? next_code[len[s]]++ : 0;
}

/* Values >= 4096 are written as a length class (symbol 4096 + bitwidth - 13)
 * followed by the value's bits below its leading one. */
static int sym_of(uint64_t v, int* extra_bits) {
  if (v < DIRECT_SYMBOLS) {
    *extra_bits = 0;
    return (int)v;
  }
  int b = bitwidth(v);
  *extra_bits = b - 1;
  return DIRECT_SYMBOLS + b - FIRST_CLASS_BITS;
}

/* ------------------------------------------------------------------ */
/* MSB-first bit writer / reader over little-endian u32 words          */
/* ------------------------------------------------------------------ */
typedef struct {
  uint8_t* base; /* NULL: only count */
  uint64_t bit;  /* bits written */
} bitw_t;

static void put_bits(bitw_t* w, uint64_t v, int nbits) {
  for (int i = nbits - 1; i >= 0; i--) {
    unsigned b = (unsigned)((v >> i) & 1);
    if (w->base && b) {
      uint64_t word = w->bit >> 5;
      int pos = 31 - (int)(w->bit & 31);
      uint32_t cur = get_u32(w->base + 4 * word);
      put_u32(w->base + 4 * word, cur | (1u << pos));
    }
    w->bit++;
  }
}

typedef struct {
  const uint8_t* base;
  uint64_t bit, end; /* end: bit limit */
} bitr_t;

static int get_bit(bitr_t* r, unsigned* b) {
  if (r->bit >= r->end) return 0;
  uint64_t word = r->bit >> 5;
  int pos = 31 - (int)(r->bit & 31);
  *b = (get_u32(r->base + 4 * word) >> pos) & 1u;
  r->bit++;
  return 1;
}
static int get_bits(bitr_t* r, int nbits, uint64_t* v) {
  uint64_t x = 0;
  for (int i = 0; i < nbits; i++) {
    unsigned b;
    if (!get_bit(r, &b)) return 0;
    x = (x << 1) | b;
  }
  *v = x;
  return 1;
}

/* ------------------------------------------------------------------ */
/* a6-a7: one coded array (fixed or Huffman, the shorter; tie -> fixed) */
/* ------------------------------------------------------------------ */
static uint64_t words_for_bits(uint64_t bits) { return (bits + 31) / 32; }

int lco_encode_array(const uint64_t* v, uint64_t n, int chunk_log2, uint8_t* out,
                     uint64_t cap, uint64_t* nbytes, int* coder, int* param,
                     uint32_t* used) {
  if (chunk_log2 < 5 || chunk_log2 > 16) return LCO_ERR_ARG;
  /* fixed-length size */
  uint64_t mx = 0;
  for (uint64_t i = 0; i < n; i++)
    if (v[i] > mx) mx = v[i];
  int w = bitwidth(mx);
  uint64_t fixed_bytes = 4 * words_for_bits(n * (uint64_t)w);

  /* Huffman size: table 4U + chunk offsets 4*nchunks + padded chunk payloads */
  uint64_t* counts = (uint64_t*)calloc(ALPHABET, sizeof(uint64_t));
  for (uint64_t i = 0; i < n; i++) {
    int e;
    counts[sym_of(v[i], &e)]++;
  }
  uint8_t len[ALPHABET];
  uint32_t code[ALPHABET];
  int L = lco_huffman_lengths(counts, ALPHABET, len);
  canonical_codes(len, ALPHABET, code);
  uint32_t U = 0;
  for (int s = 0; s < ALPHABET; s++) U += len[s] != 0;
  uint64_t C = (uint64_t)1 << chunk_log2;
  uint64_t nchunks = (n + C - 1) / C;
  uint64_t payload_words = 0;
  for (uint64_t c = 0; c < nchunks; c++) {
    uint64_t bits = 0;
    for (uint64_t i = c * C; i < n && i < (c + 1) * C; i++) {
      int e;
      int s = sym_of(v[i], &e);
      bits += (uint64_t)len[s] + (uint64_t)e;
    }
    payload_words += words_for_bits(bits);
  }
  uint64_t huff_bytes = 4 * (uint64_t)U + 4 * nchunks + 4 * payload_words;

  int use_huff = huff_bytes < fixed_bytes;
  uint64_t nb = use_huff ? huff_bytes : fixed_bytes;
  *nbytes = nb;
  *coder = use_huff;
  *param = use_huff ? L : w;
  *used = use_huff ? U : 0;
  if (!out) {
    free(counts);
    return LCO_OK;
  }
  if (nb > cap) {
    free(counts);
    return LCO_ERR_CAPACITY;
  }
  memset(out, 0, nb);
  if (!use_huff) {
    bitw_t bw = {out, 0};
    for (uint64_t i = 0; i < n; i++) put_bits(&bw, v[i], w);
  } else {
    uint8_t* p = out;
    for (int s = 0; s < ALPHABET; s++)
      if (len[s]) {
        put_u32(p, (uint32_t)s | ((uint32_t)len[s] << 16));
        p += 4;
      }
    uint8_t* offs = p;
    uint8_t* payload = p + 4 * nchunks;
    uint64_t word = 0;
    for (uint64_t c = 0; c < nchunks; c++) {
      bitw_t bw = {payload + 4 * word, 0};
      for (uint64_t i = c * C; i < n && i < (c + 1) * C; i++) {
        int e;
        int s = sym_of(v[i], &e);
        put_bits(&bw, code[s], len[s]);
        if (e) put_bits(&bw, v[i] - ((uint64_t)1 << e), e);
      }
      word += words_for_bits(bw.bit);
      put_u32(offs + 4 * c, (uint32_t)word);
    }
  }
  free(counts);
  return LCO_OK;
}

/* Textbook canonical decode: read one bit at a time until the code read so far
 * is one of the codes of that length. */
int lco_decode_array(const uint8_t* data, uint64_t nbytes, uint64_t n, int coder,
                     int param, uint32_t used, int chunk_log2, uint64_t* v) {
  if (coder == 0) {
    int w = param;
    if (w < 0 || w > 64) return LCO_ERR_CORRUPT;
    if (used != 0 || nbytes != 4 * words_for_bits(n * (uint64_t)w)) return LCO_ERR_CORRUPT;
    bitr_t r = {data, 0, nbytes * 8};
    for (uint64_t i = 0; i < n; i++)
      if (!get_bits(&r, w, &v[i])) return LCO_ERR_CORRUPT;
    return LCO_OK;
  }
  if (coder != 1 || chunk_log2 < 5 || chunk_log2 > 16) return LCO_ERR_CORRUPT;
  uint64_t C = (uint64_t)1 << chunk_log2;
  uint64_t nchunks = (n + C - 1) / C;
  if (used == 0 || used > ALPHABET) return n == 0 ? LCO_OK : LCO_ERR_CORRUPT;
  if (nbytes < 4 * (uint64_t)used + 4 * nchunks) return LCO_ERR_CORRUPT;
  uint8_t len[ALPHABET];
  uint32_t code[ALPHABET];
  memset(len, 0, sizeof(len));
  int prev = -1, L = 0;
  for (uint32_t j = 0; j < used; j++) {
    uint32_t e = get_u32(data + 4 * j);
    int s = (int)(e & 0xFFFF), l = (int)((e >> 16) & 0xFF);
    if ((e >> 24) != 0 || s >= ALPHABET || s <= prev || l < 1 || l > MAX_CODE_LEN)
      return LCO_ERR_CORRUPT;
    len[s] = (uint8_t)l;
    prev = s;
    if (l > L) L = l;
  }
  if (L != param) return LCO_ERR_CORRUPT;
  /* canonical decode tables: per length, the first code and the symbols of that
   * length in ascending order (codes of one length are consecutive) */
  int count[MAX_CODE_LEN + 1] = {0};
  int first_idx[MAX_CODE_LEN + 2] = {0};
  uint32_t first_code[MAX_CODE_LEN + 1] = {0};
  int sorted[ALPHABET];
  for (int s = 0; s < ALPHABET; s++)
    if (len[s]) count[len[s]]++;
  {
    uint32_t c = 0;
    for (int l = 1; l <= MAX_CODE_LEN; l++) {
      c = (c + (uint32_t)count[l - 1]) << 1;
      first_code[l] = c;
      first_idx[l + 1] = first_idx[l] + count[l];
    }
    int fill[MAX_CODE_LEN + 2];
    memcpy(fill, first_idx, sizeof(fill));
    for (int s = 0; s < ALPHABET; s++)
      if (len[s]) sorted[fill[len[s]]++] = s;
  }
  (void)code;
  const uint8_t* offs = data + 4 * (uint64_t)used;
  const uint8_t* payload = offs + 4 * nchunks;
  uint64_t payload_words = (nbytes - 4 * (uint64_t)used - 4 * nchunks) / 4;
  uint64_t start = 0;
  for (uint64_t c = 0; c < nchunks; c++) {
    uint64_t end = get_u32(offs + 4 * c);
    if (end < start || end > payload_words) return LCO_ERR_CORRUPT;
    bitr_t r = {payload, start * 32, end * 32};
    for (uint64_t i = c * C; i < n && i < (c + 1) * C; i++) {
      uint32_t cw = 0;
      int l = 0, s = -1;
      while (s < 0) {
        unsigned b;
        if (l >= MAX_CODE_LEN || !get_bit(&r, &b)) return LCO_ERR_CORRUPT;
        cw = (cw << 1) | b;
        l++;
        if (cw >= first_code[l] && cw - first_code[l] < (uint32_t)count[l])
          s = sorted[first_idx[l] + (int)(cw - first_code[l])];
      }
      if (s < DIRECT_SYMBOLS) {
        v[i] = (uint64_t)s;
      } else {
        int e = s - DIRECT_SYMBOLS + FIRST_CLASS_BITS - 1;
        uint64_t x;
        if (!get_bits(&r, e, &x)) return LCO_ERR_CORRUPT;
        v[i] = ((uint64_t)1 << e) + x;
      }
    }
    start = end;
  }
  if (start != payload_words) return LCO_ERR_CORRUPT;
  return LCO_OK;
}

/* ------------------------------------------------------------------ */
/* record assembly                                                     */
/* ------------------------------------------------------------------ */
typedef struct {
  const uint64_t* v;
  uint64_t n;
} arr_in;

uint64_t lco_bound(int F, uint64_t n, int chunk_log2) {
  (void)chunk_log2;
  /* fixed coding is never exceeded: ID <= 63 bits, CNT <= 33, REL <= 16,
   * supplementary codes <= 23, temporal residuals <= 25 bits per value. */
  uint64_t b = HDR_BYTES + 8 * (uint64_t)F + DIR_BYTES * (uint64_t)(F + 2);
  b += 4 * words_for_bits(n * 63) + 4 * words_for_bits(n * 33);
  b += (uint64_t)F * 4 * words_for_bits(n * 25);
  return b;
}

static int write_record(int mode, int scale, int dims, int F, uint64_t n, uint64_t B, int k,
                        int chunk_log2, const uint32_t* bn, uint64_t seq, uint64_t ref_seq,
                        const lco_grid* grids, const arr_in* arrs, int A, uint8_t* out,
                        uint64_t cap, uint64_t* size) {
  uint64_t hdr = HDR_BYTES + 8 * (uint64_t)F + DIR_BYTES * (uint64_t)A;
  uint64_t nb[LCO_MAX_F + 2];
  int coder[LCO_MAX_F + 2], param[LCO_MAX_F + 2];
  uint32_t used[LCO_MAX_F + 2];
  uint64_t total = hdr;
  for (int a = 0; a < A; a++) {
    int st = lco_encode_array(arrs[a].v, arrs[a].n, chunk_log2, NULL, 0, &nb[a], &coder[a],
                              &param[a], &used[a]);
    if (st) return st;
    total += nb[a];
  }
  *size = total;
  if (!out) return LCO_OK;
  if (total > cap) return LCO_ERR_CAPACITY;
  memset(out, 0, hdr);
  put_u32(out + 0, MAGIC);
  put_u16(out + 4, VERSION);
  put_u8(out + 6, (unsigned)mode);
  put_u8(out + 7, (unsigned)F);
  put_u8(out + 8, (unsigned)k);
  put_u8(out + 9, (unsigned)chunk_log2);
  put_u8(out + 10, (unsigned)A);
  put_u8(out + 11, scale > 1 ? (unsigned)scale : 0u); /* T residual step; 0 means 1 */
  put_u32(out + 12, (uint32_t)hdr);
  put_u64(out + 16, n);
  put_u64(out + 24, B);
  put_u64(out + 32, total);
  for (int d = 0; d < 3; d++) put_u32(out + 40 + 4 * d, bn ? bn[d] : 0);
  put_u8(out + 52, dims == 3 ? 0u : (unsigned)dims); /* spatial dimensions; 0 means 3 */
  put_u8(out + 53, (unsigned)grids[0].dtype);         /* element type of every field */
  put_u64(out + 56, seq);
  put_u64(out + 64, ref_seq);
  for (int f = 0; f < F; f++) {
    if (grids[f].dtype == LCO_DTYPE_I32) {
      put_u32(out + HDR_BYTES + 8 * f, (uint32_t)grids[f].mi);
      put_u32(out + HDR_BYTES + 8 * f + 4, (uint32_t)grids[f].hb);
    } else {
      put_f32(out + HDR_BYTES + 8 * f, grids[f].m);
      put_f32(out + HDR_BYTES + 8 * f + 4, grids[f].eb_q);
    }
  }
  uint64_t off = hdr;
  for (int a = 0; a < A; a++) {
    uint8_t* d = out + HDR_BYTES + 8 * F + DIR_BYTES * a;
    put_u8(d + 0, (unsigned)coder[a]);
    put_u8(d + 1, (unsigned)param[a]);
    put_u32(d + 4, used[a]);
    put_u64(d + 8, arrs[a].n);
    put_u64(d + 16, off);
    put_u64(d + 24, nb[a]);
    uint64_t got;
    int c2, p2;
    uint32_t u2;
    int st = lco_encode_array(arrs[a].v, arrs[a].n, chunk_log2, out + off, nb[a], &got, &c2,
                              &p2, &u2);
    if (st) return st;
    off += nb[a];
  }
  return LCO_OK;
}

/* ------------------------------------------------------------------ */
/* a2-a5, a13: LCP-S                                                   */
/* ------------------------------------------------------------------ */
typedef struct {
  uint64_t key;
  uint32_t idx;
} keyidx_t;

static int keyidx_cmp(const void* a, const void* b) {
  const keyidx_t* x = (const keyidx_t*)a;
  const keyidx_t* y = (const keyidx_t*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* bn_d = (qmax_d >> k) + 1 over the D spatial dimensions (1 for the others);
 * the block-id space must stay below 2^63. */
static int block_counts(const lco_grid* grids, const double* hi, int k, int D, uint32_t* bn) {
  unsigned __int128 tot = 1;
  for (int d = 0; d < 3; d++) bn[d] = 1;
  for (int d = 0; d < D; d++) {
    int64_t qm = quant_val(hi[d], &grids[d]);
    if (qm < 0 || qm >= Q_LIMIT) return LCO_ERR_RANGE;
    bn[d] = (uint32_t)((qm >> k) + 1);
    tot *= bn[d];
  }
  if (tot >= ((unsigned __int128)1 << 63)) return LCO_ERR_RANGE;
  return LCO_OK;
}

int lco_compress_s(const void* const* x, int F, int D, uint64_t n, const lco_grid* grids,
                   int k, int chunk_log2, uint64_t seq, uint8_t* out, uint64_t cap,
                   uint64_t* size, uint32_t* perm_out, int32_t* q_slot) {
  if (D < 1 || D > 3 || F < D || F > LCO_MAX_F || n == 0 || n > ((uint64_t)1 << 31) || k < 0 ||
      k > 16)
    return LCO_ERR_ARG;
  for (int f = 1; f < F; f++)
    if (grids[f].dtype != grids[0].dtype) return LCO_ERR_ARG;
  double lo[LCO_MAX_F], hi[LCO_MAX_F];
  int st = lco_extent(x, F, n, grids[0].dtype, lo, hi);
  if (st) return st;
  for (int f = 0; f < F; f++) {
    if (quant_val(lo[f], &grids[f]) < 0) return LCO_ERR_ARG; /* grid not from this frame */
    if (quant_val(hi[f], &grids[f]) >= Q_LIMIT) return LCO_ERR_RANGE;
  }
  uint32_t bn[3];
  st = block_counts(grids, hi, k, D, bn);
  if (st) return st;
  uint64_t p = (uint64_t)1 << k;

  /* Eq. 5 then Eq. 6: quantise, block id from q / p, row-major with x fastest
   * (a dimension the data does not have contributes block 0) */
  keyidx_t* ki = (keyidx_t*)malloc(sizeof(keyidx_t) * n);
  for (uint64_t i = 0; i < n; i++) {
    uint64_t b[3] = {0, 0, 0};
    for (int d = 0; d < D; d++) b[d] = (uint64_t)quant_at(x, d, i, &grids[d]) >> k;
    ki[i].key = b[0] + (uint64_t)bn[0] * (b[1] + (uint64_t)bn[1] * b[2]);
    ki[i].idx = (uint32_t)i;
  }
  /* particles stored block by block: stable order of (block id, input index) */
  qsort(ki, n, sizeof(keyidx_t), keyidx_cmp);

  /* non-empty blocks: ids and counts */
  uint64_t B = 0;
  for (uint64_t s = 0; s < n; s++)
    if (s == 0 || ki[s].key != ki[s - 1].key) B++;
  uint64_t* ids = (uint64_t*)malloc(sizeof(uint64_t) * B);
  uint64_t* cnt = (uint64_t*)malloc(sizeof(uint64_t) * B);
  uint64_t b = 0;
  for (uint64_t s = 0; s < n; s++) {
    if (s == 0 || ki[s].key != ki[s - 1].key) {
      ids[b] = ki[s].key;
      cnt[b] = 0;
      b++;
    }
    cnt[b - 1]++;
  }
  /* delta coding of the three arrays (Sec. 6.2.2) */
  uint64_t* v_id = (uint64_t*)malloc(sizeof(uint64_t) * B);
  uint64_t* v_cnt = (uint64_t*)malloc(sizeof(uint64_t) * B);
  for (uint64_t j = 0; j < B; j++) {
    v_id[j] = ids[j] - (j ? ids[j - 1] : 0);
    v_cnt[j] = zigzag((int64_t)cnt[j] - (int64_t)(j ? cnt[j - 1] : 0));
  }
  uint64_t* v_rel[3];
  uint64_t* v_sup[LCO_MAX_F];
  for (int d = 0; d < D; d++) {
    v_rel[d] = (uint64_t*)malloc(sizeof(uint64_t) * n);
    uint64_t prev = 0;
    for (uint64_t s = 0; s < n; s++) {
      uint64_t q = (uint64_t)quant_at(x, d, ki[s].idx, &grids[d]);
      uint64_t rel = q & (p - 1); /* offset from the block's (0,0,0) corner */
      v_rel[d][s] = (rel - prev) & (p - 1);
      prev = rel;
    }
  }
  for (int f = D; f < F; f++) {
    v_sup[f] = (uint64_t*)malloc(sizeof(uint64_t) * n);
    for (uint64_t s = 0; s < n; s++)
      v_sup[f][s] = (uint64_t)quant_at(x, f, ki[s].idx, &grids[f]);
  }
  arr_in arrs[LCO_MAX_F + 2];
  arrs[0].v = v_id;
  arrs[0].n = B;
  arrs[1].v = v_cnt;
  arrs[1].n = B;
  for (int d = 0; d < D; d++) {
    arrs[2 + d].v = v_rel[d];
    arrs[2 + d].n = n;
  }
  for (int f = D; f < F; f++) {
    arrs[2 + f].v = v_sup[f];
    arrs[2 + f].n = n;
  }
  st = write_record(0, 1, D, F, n, B, k, chunk_log2, bn, seq, UINT64_MAX, grids, arrs, F + 2,
                    out, cap, size);
  if (st == LCO_OK && perm_out)
    for (uint64_t s = 0; s < n; s++) perm_out[s] = ki[s].idx;
  if (st == LCO_OK && q_slot)
    for (int f = 0; f < F; f++)
      for (uint64_t s = 0; s < n; s++)
        q_slot[(uint64_t)f * n + s] = (int32_t)quant_at(x, f, ki[s].idx, &grids[f]);
  for (int d = 0; d < D; d++) free(v_rel[d]);
  for (int f = D; f < F; f++) free(v_sup[f]);
  free(v_id);
  free(v_cnt);
  free(ids);
  free(cnt);
  free(ki);
  return st;
}

/* ------------------------------------------------------------------ */
/* a9: LCP-T -- codes on the reference's grid, in its slot order,      */
/* minus the reference's codes                                         */
/* ------------------------------------------------------------------ */
int lco_compress_t(const void* const* x, int F, uint64_t n, const lco_grid* grids,
                   const uint32_t* ref_perm, const int32_t* ref_q, uint64_t ref_seq,
                   int scale, int chunk_log2, uint64_t seq, uint8_t* out, uint64_t cap,
                   uint64_t* size, int32_t* q_slot) {
  if (F < 1 || F > LCO_MAX_F || n == 0 || n > ((uint64_t)1 << 31)) return LCO_ERR_ARG;
  if (scale < 1 || scale > 15 || scale % 2 == 0) return LCO_ERR_ARG;
  if (!ref_perm || !ref_q) return LCO_ERR_NO_REFERENCE;
  for (int f = 1; f < F; f++)
    if (grids[f].dtype != grids[0].dtype) return LCO_ERR_ARG;
  const int is_int = grids[0].dtype == LCO_DTYPE_I32;
  double lo[LCO_MAX_F], hi[LCO_MAX_F];
  int st = lco_extent(x, F, n, grids[0].dtype, lo, hi);
  if (st) return st;
  for (int f = 0; f < F; f++) {
    /* the rounding margin of the inherited grid must still cover this frame
     * (float32 output; integer reconstructions are exact) */
    double a = fabs(lo[f]), b = fabs(hi[f]);
    double M = (a > b ? a : b) + 2.0 * grids[f].eb;
    if (!is_int && !(M < ldexp(1.0, grids[f].E))) return LCO_ERR_RANGE;
    if (quant_val(lo[f], &grids[f]) < -Q_LIMIT) return LCO_ERR_RANGE;
    if (quant_val(hi[f], &grids[f]) >= Q_LIMIT) return LCO_ERR_RANGE;
  }
  /* Sec. 7.1: quantise the frame, subtract the reference.  With an anchor grid
   * made at eb / s (Sec. 7.4.2) the frame is coded at eb on that finer grid: its
   * code moves from the reference's by a multiple of s, the one nearest to the
   * frame's own code (within (s - 1) / 2 of it, so the reconstruction is within
   * s bins' half width, i.e. eb).  The residual is that multiple divided by s. */
  const int64_t h = (scale - 1) / 2;
  uint64_t* v[LCO_MAX_F];
  arr_in arrs[LCO_MAX_F];
  for (int f = 0; f < F; f++) {
    v[f] = (uint64_t*)malloc(sizeof(uint64_t) * n);
    arrs[f].v = v[f];
    arrs[f].n = n;
  }
  for (int f = 0; f < F && st == LCO_OK; f++) {
    for (uint64_t s = 0; s < n; s++) {
      int64_t q = quant_at(x, f, ref_perm[s], &grids[f]);
      int64_t ref = (int64_t)ref_q[(uint64_t)f * n + s];
      int64_t num = q - ref + h;
      /* floor division, exact for negative numerators too */
      int64_t r = num >= 0 ? num / scale : -((-num + scale - 1) / scale);
      int64_t qn = ref + (int64_t)scale * r;
      if (qn < -Q_LIMIT || qn >= Q_LIMIT) {
        st = LCO_ERR_RANGE;
        break;
      }
      v[f][s] = zigzag(r);
      if (q_slot) q_slot[(uint64_t)f * n + s] = (int32_t)qn;
    }
  }
  if (st == LCO_OK)
    st = write_record(1, scale, 3, F, n, 0, 0, chunk_log2, NULL, seq, ref_seq, grids, arrs, F,
                      out, cap, size);
  for (int f = 0; f < F; f++) free(v[f]);
  return st;
}

/* ------------------------------------------------------------------ */
/* a8, a10: decompression                                              */
/* ------------------------------------------------------------------ */
int lco_record_info(const uint8_t* rec, uint64_t size, lco_info* info) {
  memset(info, 0, sizeof(*info));
  if (size < HDR_BYTES) return LCO_ERR_CORRUPT;
  if (get_u32(rec) != MAGIC || (rec[4] | (rec[5] << 8)) != VERSION) return LCO_ERR_CORRUPT;
  info->mode = rec[6];
  info->F = rec[7];
  info->k = rec[8];
  info->chunk_log2 = rec[9];
  info->n_arrays = rec[10];
  info->scale = rec[11] ? rec[11] : 1;
  info->dims = rec[52] ? rec[52] : 3;
  if (rec[52] > 2 || (info->mode == 1 && rec[52] != 0)) return LCO_ERR_CORRUPT;
  info->dtype = rec[53];
  if (info->dtype != LCO_DTYPE_F32 && info->dtype != LCO_DTYPE_I32) return LCO_ERR_CORRUPT;
  if ((info->mode == 0 && rec[11] != 0) || info->scale > 15 || info->scale % 2 == 0)
    return LCO_ERR_CORRUPT;
  if (info->mode > 1 || info->F < (info->mode == 0 ? info->dims : 1) || info->F > LCO_MAX_F ||
      info->k > 16 ||
      info->chunk_log2 < 5 || info->chunk_log2 > 16)
    return LCO_ERR_CORRUPT;
  int A = info->mode == 0 ? info->F + 2 : info->F;
  uint64_t hdr = HDR_BYTES + 8 * (uint64_t)info->F + DIR_BYTES * (uint64_t)A;
  if (info->n_arrays != A || get_u32(rec + 12) != hdr || size < hdr) return LCO_ERR_CORRUPT;
  info->n = get_u64(rec + 16);
  info->B = get_u64(rec + 24);
  info->total_bytes = get_u64(rec + 32);
  for (int d = 0; d < 3; d++) info->bn[d] = get_u32(rec + 40 + 4 * d);
  info->seq = get_u64(rec + 56);
  info->ref_seq = get_u64(rec + 64);
  if (info->total_bytes > size || info->n == 0 || info->n > ((uint64_t)1 << 31))
    return LCO_ERR_CORRUPT;
  if (info->mode == 0 && (info->B == 0 || info->B > info->n)) return LCO_ERR_CORRUPT;
  for (int f = 0; f < info->F; f++) {
    if (info->dtype == LCO_DTYPE_I32) {
      /* origin, then the half width of the integer bins (below 2^31) */
      info->mi[f] = (int32_t)get_u32(rec + HDR_BYTES + 8 * f);
      info->hb[f] = get_u32(rec + HDR_BYTES + 8 * f + 4);
      if (info->hb[f] > INT32_MAX) return LCO_ERR_CORRUPT;
      continue;
    }
    info->m[f] = get_f32(rec + HDR_BYTES + 8 * f);
    info->eb_q[f] = get_f32(rec + HDR_BYTES + 8 * f + 4);
    if (!isfinite(info->m[f]) || !(info->eb_q[f] > 0) || !isfinite(info->eb_q[f]))
      return LCO_ERR_CORRUPT;
  }
  uint64_t off = hdr;
  for (int a = 0; a < A; a++) {
    const uint8_t* d = rec + HDR_BYTES + 8 * info->F + DIR_BYTES * a;
    info->coder[a] = d[0];
    info->param[a] = d[1];
    info->used[a] = get_u32(d + 4);
    info->arr_n[a] = get_u64(d + 8);
    info->arr_off[a] = get_u64(d + 16);
    info->arr_bytes[a] = get_u64(d + 24);
    uint64_t expect_n = (info->mode == 0 && a < 2) ? info->B : info->n;
    if (info->arr_n[a] != expect_n || info->arr_off[a] != off ||
        info->arr_bytes[a] > info->total_bytes - off || info->coder[a] > 1)
      return LCO_ERR_CORRUPT;
    off += info->arr_bytes[a];
  }
  if (off != info->total_bytes) return LCO_ERR_CORRUPT;
  return LCO_OK;
}

static float recon_f(int64_t q, float eb_q, float m) {
  return fmaf((float)(2 * q + 1), eb_q, m);
}

int lco_decompress(const uint8_t* rec, uint64_t size, const int32_t* ref_q,
                   uint64_t ref_seq, uint64_t ref_n, void* const* out, uint64_t cap_n,
                   uint64_t* n_out, int32_t* q_slot) {
  lco_info I;
  int st = lco_record_info(rec, size, &I);
  if (st) return st;
  uint64_t n = I.n;
  *n_out = n;
  if (n > cap_n) return LCO_ERR_CAPACITY;
  int A = I.n_arrays;
  uint64_t* v[LCO_MAX_F + 2];
  for (int a = 0; a < A; a++) {
    v[a] = (uint64_t*)malloc(sizeof(uint64_t) * (I.arr_n[a] ? I.arr_n[a] : 1));
    if (st == LCO_OK)
      st = lco_decode_array(rec + I.arr_off[a], I.arr_bytes[a], I.arr_n[a], I.coder[a],
                            I.param[a], I.used[a], I.chunk_log2, v[a]);
  }
  int32_t* q = (int32_t*)malloc(sizeof(int32_t) * n * I.F);
  if (st == LCO_OK && I.mode == 0) {
    uint64_t B = I.B, p = (uint64_t)1 << I.k;
    unsigned __int128 tot = (unsigned __int128)I.bn[0] * I.bn[1] * I.bn[2];
    uint64_t id = 0, s = 0;
    int64_t c = 0;
    uint64_t rel[3] = {0, 0, 0};
    for (uint64_t b = 0; b < B && st == LCO_OK; b++) {
      /* inverse delta: running sums of ids and counts */
      /* an id delta is at least 1 after the first block and below the id space,
       * so the running id cannot wrap */
      if ((b > 0 && v[0][b] == 0) || (unsigned __int128)v[0][b] >= tot) {
        st = LCO_ERR_CORRUPT;
        break;
      }
      id += v[0][b];
      c = (int64_t)((uint64_t)c + (uint64_t)unzigzag(v[1][b]));
      if ((unsigned __int128)id >= tot || c < 1 || (uint64_t)c > n - s) {
        st = LCO_ERR_CORRUPT;
        break;
      }
      uint64_t bx = id % I.bn[0], by = (id / I.bn[0]) % I.bn[1],
               bz = id / ((uint64_t)I.bn[0] * I.bn[1]);
      uint64_t corner[3] = {bx << I.k, by << I.k, bz << I.k};
      for (int64_t j = 0; j < c; j++, s++) {
        for (int d = 0; d < I.dims; d++) {
          rel[d] = (rel[d] + v[2 + d][s]) & (p - 1);
          uint64_t qq = corner[d] + rel[d];
          if (v[2 + d][s] >= p || qq >= Q_LIMIT) st = LCO_ERR_CORRUPT;
          q[(uint64_t)d * n + s] = (int32_t)qq;
        }
      }
    }
    if (st == LCO_OK && s != n) st = LCO_ERR_CORRUPT;
    for (int f = I.dims; f < I.F && st == LCO_OK; f++)
      for (uint64_t t = 0; t < n; t++) {
        if (v[2 + f][t] >= Q_LIMIT) st = LCO_ERR_CORRUPT;
        q[(uint64_t)f * n + t] = (int32_t)v[2 + f][t];
      }
  } else if (st == LCO_OK) {
    if (!ref_q || ref_seq != I.ref_seq || ref_n != n) st = LCO_ERR_NO_REFERENCE;
    for (int f = 0; f < I.F && st == LCO_OK; f++)
      for (uint64_t t = 0; t < n; t++) {
        /* residuals of a valid record are below 2^26; a larger one is corrupt
         * (and would overflow the scaled sum) */
        int64_t d = v[f][t] < ((uint64_t)1 << 40) ? unzigzag(v[f][t]) : ((int64_t)1 << 40);
        int64_t qq = (int64_t)ref_q[(uint64_t)f * n + t] + (int64_t)I.scale * d;
        if (qq < -Q_LIMIT || qq >= Q_LIMIT) {
          st = LCO_ERR_CORRUPT;
          break;
        }
        q[(uint64_t)f * n + t] = (int32_t)qq;
      }
  }
  if (st == LCO_OK) {
    for (int f = 0; f < I.F; f++) {
      if (I.dtype == LCO_DTYPE_I32) {
        lco_grid g;
        memset(&g, 0, sizeof(g));
        g.dtype = LCO_DTYPE_I32;
        g.mi = I.mi[f];
        g.hb = I.hb[f];
        for (uint64_t t = 0; t < n; t++)
          ((int32_t*)out[f])[t] = lco_recon_i(q[(uint64_t)f * n + t], &g);
      } else {
        for (uint64_t t = 0; t < n; t++)
          ((float*)out[f])[t] = recon_f(q[(uint64_t)f * n + t], I.eb_q[f], I.m[f]);
      }
    }
    if (q_slot) memcpy(q_slot, q, sizeof(int32_t) * n * I.F);
  }
  free(q);
  for (int a = 0; a < A; a++) free(v[a]);
  return st;
}

/* ------------------------------------------------------------------ */
/* a11: Alg. 1 references and LCP-FSM                                  */
/* ------------------------------------------------------------------ */
typedef struct {
  int valid;
  int scale; /* the grid's step relative to the stream's bound: 1, or an anchor's scale */
  uint64_t seq, n;
  lco_grid grid[LCO_MAX_F];
  uint32_t* perm;
  int32_t* q;
} ref_t;

struct lco_stream {
  lco_params p;
  uint64_t max_n;
  int have_eb;
  double eb_f[LCO_MAX_F];
  /* compress side */
  uint64_t seq;
  ref_t prev, anchor;
  int fsm_t;     /* 0: S state, 1: T state */
  int interval;  /* S state: compare once every `interval` frames */
  int countdown; /* S frames left before the next comparison */
  uint64_t last_s;
  /* frames coded since the last anchor, and how many of them by LCP-T */
  uint64_t n_since_anchor, t_since_anchor;
  /* decompress side */
  uint64_t dseq;
  ref_t dprev, danchor;
};

static void ref_alloc(ref_t* r, uint64_t max_n, int F) {
  r->valid = 0;
  r->perm = (uint32_t*)malloc(sizeof(uint32_t) * max_n);
  r->q = (int32_t*)malloc(sizeof(int32_t) * max_n * F);
}
static void ref_free(ref_t* r) {
  free(r->perm);
  free(r->q);
}
static void ref_copy(ref_t* dst, const ref_t* src, int F) {
  dst->valid = src->valid;
  dst->scale = src->scale;
  dst->seq = src->seq;
  dst->n = src->n;
  memcpy(dst->grid, src->grid, sizeof(src->grid));
  if (src->valid) {
    memcpy(dst->perm, src->perm, sizeof(uint32_t) * src->n);
    memcpy(dst->q, src->q, sizeof(int32_t) * src->n * F);
  }
}

lco_stream* lco_stream_create(const lco_params* p, uint64_t max_n) {
  if (!p || p->n_fields < 1 || p->n_fields > LCO_MAX_F || p->block_log2 < 0 || p->n_dims < 0 ||
      p->n_dims > 3 || p->n_fields < (p->n_dims ? p->n_dims : 3) ||
      p->block_log2 > 16 || p->chunk_log2 < 5 || p->chunk_log2 > 16 || p->batch_size < 0 ||
      max_n == 0 || p->anchor_scale < 0 || p->anchor_scale > 15 ||
      (p->anchor_scale > 1 && p->anchor_scale % 2 == 0) ||
      (p->dtype != LCO_DTYPE_F32 && p->dtype != LCO_DTYPE_I32))
    return NULL;
  lco_stream* s = (lco_stream*)calloc(1, sizeof(lco_stream));
  s->p = *p;
  s->max_n = max_n;
  s->interval = 1;
  ref_alloc(&s->prev, max_n, p->n_fields);
  ref_alloc(&s->anchor, max_n, p->n_fields);
  ref_alloc(&s->dprev, max_n, p->n_fields);
  ref_alloc(&s->danchor, max_n, p->n_fields);
  return s;
}

void lco_stream_destroy(lco_stream* s) {
  if (!s) return;
  ref_free(&s->prev);
  ref_free(&s->anchor);
  ref_free(&s->dprev);
  ref_free(&s->danchor);
  free(s);
}

static int first_in_batch(const lco_params* p, uint64_t seq) {
  return p->batch_size == 0 ? seq == 0 : seq % (uint64_t)p->batch_size == 0;
}

static const ref_t* reference_for(const lco_params* p, uint64_t seq, const ref_t* prev,
                                  const ref_t* anchor) {
  const ref_t* r = first_in_batch(p, seq) ? anchor : prev;
  return r->valid ? r : NULL;
}

/* LCP-FSM (Sec. 7.2; the state diagram itself is not in the text).  States:
 * S with a test interval (S1X, S2X, S4X, ... S16X) and a countdown of untested S
 * frames, or T.  In S, a comparison runs both compressors; S winning doubles the
 * interval (the first frame, which has no reference, counts as such a win).  In
 * T, T runs and is kept while it is no larger than the last S size (the paper's
 * estimate of S); otherwise S runs too and the smaller wins, S returning the
 * machine to S1X. */
static int fsm_decide(const lco_stream* s, int have_ref) {
  if (!s->p.multi_frame || !have_ref) return LCO_DECIDE_S;
  if (s->fsm_t) return LCO_DECIDE_T;
  return s->countdown > 0 ? LCO_DECIDE_S : LCO_DECIDE_COMPARE;
}

static void fsm_s_win(lco_stream* s) {
  s->interval = s->interval * 2 > 16 ? 16 : s->interval * 2;
  s->countdown = s->interval - 1;
}

static void fsm_update(lco_stream* s, int decision, int have_ref, int chose_t) {
  if (!have_ref) { /* forced S: no reference frame */
    if (s->fsm_t) {
      s->fsm_t = 0;
      s->interval = 1;
    }
    fsm_s_win(s);
  } else if (decision == LCO_DECIDE_S) {
    s->countdown--;
  } else if (decision == LCO_DECIDE_COMPARE) {
    if (chose_t) s->fsm_t = 1;
    else fsm_s_win(s);
  } else if (!chose_t) { /* T state, S won */
    s->fsm_t = 0;
    s->interval = 1;
    s->countdown = 0;
  }
}

int lco_stream_select(const lco_stream* s, int* decision) {
  const ref_t* r = reference_for(&s->p, s->seq, &s->prev, &s->anchor);
  *decision = fsm_decide(s, r != NULL);
  return LCO_OK;
}

int lco_stream_compress(lco_stream* s, const void* const* x, uint64_t n, int method,
                        uint8_t* out, uint64_t cap, uint64_t* size, int* method_used,
                        uint32_t* perm_out) {
  int F = s->p.n_fields;
  if (n == 0 || n > s->max_n || method < 0 || method > 2) return LCO_ERR_ARG;
  const int is_int = s->p.dtype == LCO_DTYPE_I32;
  double lo[LCO_MAX_F], hi[LCO_MAX_F];
  int st = lco_extent(x, F, n, s->p.dtype, lo, hi);
  if (st) return st;
  double eb_f[LCO_MAX_F];
  if (s->p.multi_frame && s->have_eb) {
    memcpy(eb_f, s->eb_f, sizeof(eb_f));
  } else {
    st = lco_field_eb(s->p.eb_mode, s->p.eb, F, lo, hi, s->p.dtype, eb_f);
    if (st) return st;
  }
  lco_grid sg[LCO_MAX_F]; /* made only when LCP-S runs: a T frame needs no grid of its own */
  const ref_t* ref = s->p.multi_frame ? reference_for(&s->p, s->seq, &s->prev, &s->anchor)
                                      : NULL;
  if (ref && ref->n != n) ref = NULL;
  int decision;
  if (method == LCO_METHOD_S) decision = LCO_DECIDE_S;
  else if (method == LCO_METHOD_T) decision = LCO_DECIDE_T;
  else decision = fsm_decide(s, ref != NULL);
  if (decision != LCO_DECIDE_S && !ref) return LCO_ERR_NO_REFERENCE; /* forced T only */

  uint64_t bound = lco_bound(F, n, s->p.chunk_log2);
  uint8_t *bs = NULL, *bt = NULL;
  uint32_t* perm_s = NULL;
  int32_t *q_s = NULL, *q_t = NULL;
  uint64_t size_s = 0, size_tt = 0;
  int have_s = 0, have_t = 0;

  if (decision != LCO_DECIDE_S) {
    bt = (uint8_t*)malloc(bound);
    q_t = (int32_t*)malloc(sizeof(int32_t) * n * F);
    int st2 = lco_compress_t(x, F, n, ref->grid, ref->perm, ref->q, ref->seq, ref->scale,
                             s->p.chunk_log2, s->seq, bt, bound, &size_tt, q_t);
    if (st2 == LCO_OK) have_t = 1;
    else if (st2 != LCO_ERR_RANGE || method == LCO_METHOD_T) st = st2; /* RANGE: T infeasible */
  }
  int need_s = decision != LCO_DECIDE_T || !have_t ||
               (method == LCO_METHOD_AUTO && size_tt > s->last_s);
  /* Sec. 7.4.2: a frame that would become an anchor (first in its batch, coded
   * by S) is coded at eb / s while the stream's frames are temporally
   * correlated, read as: no frame coded since the last anchor yet (the stream's
   * start), or at least half of those frames coded by LCP-T. */
  int s_scale = 1;
  if (s->p.multi_frame && s->p.anchor_scale > 1 && first_in_batch(&s->p, s->seq) &&
      (s->n_since_anchor == 0 || 2 * s->t_since_anchor >= s->n_since_anchor))
    s_scale = s->p.anchor_scale;
  /* an integer bin holds at least one integer: when some field's unscaled bin
   * has fewer than s integers, no finer anchor grid exists and the anchor is
   * coded at the stream's bound */
  for (int f = 0; f < F && is_int && s_scale > 1; f++)
    if (2 * (eb_f[f] >= 2147483647.0 ? 2147483647 : (int64_t)floor(eb_f[f])) + 1 < s_scale)
      s_scale = 1;
  for (int f = 0; f < F && st == LCO_OK && need_s; f++)
    st = is_int ? lco_make_grid_i((int32_t)lo[f], eb_f[f], s_scale, &sg[f])
                : lco_make_grid((float)lo[f], (float)hi[f], eb_f[f] / (double)s_scale, &sg[f]);
  if (st == LCO_OK && need_s) {
    bs = (uint8_t*)malloc(bound);
    perm_s = (uint32_t*)malloc(sizeof(uint32_t) * n);
    q_s = (int32_t*)malloc(sizeof(int32_t) * n * F);
    st = lco_compress_s(x, F, s->p.n_dims ? s->p.n_dims : 3, n, sg, s->p.block_log2,
                        s->p.chunk_log2, s->seq, bs, bound,
                        &size_s, perm_s, q_s);
    if (st == LCO_OK) have_s = 1;
  }
  int chose_t = have_t && (!have_s || size_tt < size_s); /* ties -> S */
  uint64_t chosen = chose_t ? size_tt : size_s;
  if (st == LCO_OK && chosen > cap) {
    *size = chosen;
    st = LCO_ERR_CAPACITY;
  }
  if (st == LCO_OK) {
    memcpy(out, chose_t ? bt : bs, chosen);
    *size = chosen;
    if (method_used) *method_used = chose_t ? LCO_METHOD_T : LCO_METHOD_S;
    /* the estimate of S is an S record at the stream's bound; an anchor coded
     * at eb / s stands in only until there is one */
    if (have_s && (s_scale == 1 || s->last_s == 0)) s->last_s = size_s;
    if (s->p.multi_frame && method == LCO_METHOD_AUTO) fsm_update(s, decision, ref != NULL, chose_t);
    /* Alg. 1 bookkeeping: the previous frame; anchors are first-in-batch S frames */
    if (!chose_t) {
      s->prev.valid = 1;
      s->prev.scale = s_scale;
      s->prev.seq = s->seq;
      s->prev.n = n;
      memcpy(s->prev.grid, sg, sizeof(sg));
      memcpy(s->prev.perm, perm_s, sizeof(uint32_t) * n);
      memcpy(s->prev.q, q_s, sizeof(int32_t) * n * F);
      if (first_in_batch(&s->p, s->seq)) ref_copy(&s->anchor, &s->prev, F);
    } else {
      /* a T frame keeps its reference's grid and slot order */
      if (ref != &s->prev) {
        memcpy(s->prev.grid, ref->grid, sizeof(ref->grid));
        memcpy(s->prev.perm, ref->perm, sizeof(uint32_t) * n);
      }
      s->prev.scale = ref->scale;
      s->prev.valid = 1;
      s->prev.seq = s->seq;
      s->prev.n = n;
      memcpy(s->prev.q, q_t, sizeof(int32_t) * n * F);
    }
    if (perm_out) memcpy(perm_out, s->prev.perm, sizeof(uint32_t) * n);
    if (!chose_t && first_in_batch(&s->p, s->seq)) {
      s->n_since_anchor = 0;
      s->t_since_anchor = 0;
    } else {
      s->n_since_anchor++;
      s->t_since_anchor += chose_t ? 1 : 0;
    }
    if (s->p.multi_frame && !s->have_eb) {
      memcpy(s->eb_f, eb_f, sizeof(eb_f));
      s->have_eb = 1;
    }
    s->seq++;
  }
  free(bs);
  free(bt);
  free(perm_s);
  free(q_s);
  free(q_t);
  return st;
}

int lco_stream_decompress(lco_stream* s, const uint8_t* rec, uint64_t size,
                          void* const* out, uint64_t cap_n, uint64_t* n_out) {
  int F = s->p.n_fields;
  lco_info I;
  int st = lco_record_info(rec, size, &I);
  if (st) return st;
  if (I.F != F || I.n > s->max_n || I.dtype != s->p.dtype) return LCO_ERR_ARG;
  const ref_t* ref = NULL;
  if (I.mode == 1) {
    if (s->dprev.valid && s->dprev.seq == I.ref_seq) ref = &s->dprev;
    else if (s->danchor.valid && s->danchor.seq == I.ref_seq) ref = &s->danchor;
    if (!ref) return LCO_ERR_NO_REFERENCE;
  }
  int32_t* q = (int32_t*)malloc(sizeof(int32_t) * I.n * F);
  st = lco_decompress(rec, size, ref ? ref->q : NULL, ref ? ref->seq : 0, ref ? ref->n : 0,
                      out, cap_n, n_out, q);
  if (st == LCO_OK) {
    int fib = first_in_batch(&s->p, I.seq);
    s->dprev.valid = 1;
    s->dprev.seq = I.seq;
    s->dprev.n = I.n;
    memcpy(s->dprev.q, q, sizeof(int32_t) * I.n * F);
    if (I.mode == 0 && fib) ref_copy(&s->danchor, &s->dprev, F);
    s->dseq = I.seq + 1;
  }
  free(q);
  return st;
}

/* ------------------------------------------------------------------ */
/* multi-frame container: Sec. 7.3 stores the anchor frames (first in    */
/* their batch, coded by LCP-S) in an array of their own and retrieves a */
/* frame by locating it in its batch or the anchor array, decoding its   */
/* reference first when it is temporal                                  */
/* ------------------------------------------------------------------ */
#define CMAGIC 0x4350434Cu /* bytes "LCPC" */

int lco_container_pack(const uint8_t* const* recs, const uint64_t* sizes, uint64_t n,
                       int batch_size, uint8_t* out, uint64_t cap, uint64_t* size) {
  if (n == 0 || batch_size < 0 || !recs || !sizes) return LCO_ERR_ARG;
  lco_info* I = (lco_info*)malloc(sizeof(lco_info) * n);
  int st = LCO_OK;
  for (uint64_t j = 0; j < n && st == LCO_OK; j++) {
    st = lco_record_info(recs[j], sizes[j], &I[j]);
    /* one stream from its start: record j is frame j, references go back */
    if (st == LCO_OK && (I[j].seq != j || I[j].total_bytes != sizes[j] || I[j].F != I[0].F ||
                         (I[j].mode == 1 && I[j].ref_seq >= j)))
      st = LCO_ERR_ARG;
  }
  if (st) {
    free(I);
    return st;
  }
  /* where each record goes: batch arrays first, the anchor array last */
  uint64_t off = LCO_CONTAINER_HDR + LCO_CONTAINER_ENTRY * n, anchors = 0;
  uint64_t* where = (uint64_t*)malloc(sizeof(uint64_t) * n);
  int* is_anchor = (int*)malloc(sizeof(int) * n);
  for (uint64_t j = 0; j < n; j++) {
    int first = batch_size == 0 ? j == 0 : j % (uint64_t)batch_size == 0;
    is_anchor[j] = first && I[j].mode == 0;
    anchors += is_anchor[j];
    if (!is_anchor[j]) {
      where[j] = off;
      off += sizes[j];
    }
  }
  uint64_t anchor_off = off;
  for (uint64_t j = 0; j < n; j++)
    if (is_anchor[j]) {
      where[j] = off;
      off += sizes[j];
    }
  *size = off;
  if (out) {
    if (off > cap) {
      st = LCO_ERR_CAPACITY;
    } else {
      memset(out, 0, LCO_CONTAINER_HDR + LCO_CONTAINER_ENTRY * n);
      put_u32(out + 0, CMAGIC);
      put_u16(out + 4, 1);
      put_u32(out + 8, (uint32_t)batch_size);
      put_u32(out + 12, (uint32_t)I[0].F);
      put_u64(out + 16, n);
      put_u64(out + 24, anchors);
      put_u64(out + 32, LCO_CONTAINER_HDR);
      put_u64(out + 40, anchor_off);
      put_u64(out + 48, off);
      for (uint64_t j = 0; j < n; j++) {
        uint8_t* e = out + LCO_CONTAINER_HDR + LCO_CONTAINER_ENTRY * j;
        put_u64(e + 0, where[j]);
        put_u64(e + 8, sizes[j]);
        put_u64(e + 16, I[j].mode == 1 ? I[j].ref_seq : UINT64_MAX);
        put_u32(e + 24, (uint32_t)I[j].n);
        put_u8(e + 28, (unsigned)I[j].mode);
        put_u8(e + 29, (unsigned)is_anchor[j]);
        memcpy(out + where[j], recs[j], sizes[j]);
      }
    }
  }
  free(where);
  free(is_anchor);
  free(I);
  return st;
}

int lco_container_closure(const uint8_t* cont, uint64_t size, uint64_t k, uint64_t* frames,
                          uint64_t cap, uint64_t* count) {
  if (size < LCO_CONTAINER_HDR || get_u32(cont) != CMAGIC) return LCO_ERR_CORRUPT;
  uint64_t n = get_u64(cont + 16);
  if (n > (size - LCO_CONTAINER_HDR) / LCO_CONTAINER_ENTRY) return LCO_ERR_CORRUPT;
  if (k >= n) return LCO_ERR_ARG;
  /* walk the references back to a spatial frame, then list them in order */
  uint64_t c = 0, j = k;
  for (;;) {
    if (c >= cap) return LCO_ERR_CAPACITY;
    frames[c++] = j;
    const uint8_t* e = cont + LCO_CONTAINER_HDR + LCO_CONTAINER_ENTRY * j;
    if (e[28] == 0) break;
    uint64_t r = get_u64(e + 16);
    if (r >= j) return LCO_ERR_CORRUPT;
    j = r;
  }
  for (uint64_t a = 0, b = c - 1; a < b; a++, b--) {
    uint64_t t = frames[a];
    frames[a] = frames[b];
    frames[b] = t;
  }
  *count = c;
  return LCO_OK;
}

/* ------------------------------------------------------------------ */
/* a12: block-size search on a stride sample                           */
/* ------------------------------------------------------------------ */
int lco_search_k(const void* const* x, int F, uint64_t n, const lco_params* p, int* k_out,
                 uint64_t* sizes) {
  const int D = p->n_dims ? p->n_dims : 3;
  if (D < 1 || D > 3 || F < D || F > LCO_MAX_F || n == 0) return LCO_ERR_ARG;
  uint64_t stride = n >> 20;
  if (stride < 1) stride = 1;
  uint64_t ns = (n + stride - 1) / stride;
  /* every stride-th value (a 4-byte word of either type) */
  uint32_t* smp[LCO_MAX_F];
  for (int f = 0; f < F; f++) {
    smp[f] = (uint32_t*)malloc(sizeof(uint32_t) * ns);
    for (uint64_t j = 0; j < ns; j++) smp[f][j] = ((const uint32_t*)x[f])[j * stride];
  }
  const int is_int = p->dtype == LCO_DTYPE_I32;
  double lo[LCO_MAX_F], hi[LCO_MAX_F];
  double eb_f[LCO_MAX_F];
  lco_grid g[LCO_MAX_F];
  int st = lco_extent((const void* const*)smp, F, ns, p->dtype, lo, hi);
  if (!st) st = lco_field_eb(p->eb_mode, p->eb, F, lo, hi, p->dtype, eb_f);
  for (int f = 0; f < F && !st; f++)
    st = is_int ? lco_make_grid_i((int32_t)lo[f], eb_f[f], 1, &g[f])
                : lco_make_grid((float)lo[f], (float)hi[f], eb_f[f], &g[f]);
  int best = -1;
  uint64_t best_size = 0;
  for (int k = 0; k <= 16 && !st; k++) {
    uint64_t sz = 0;
    int s2 = lco_compress_s((const void* const*)smp, F, D, ns, g, k, p->chunk_log2, 0, NULL, 0,
                            &sz, NULL, NULL);
    if (sizes) sizes[k] = s2 == LCO_OK ? sz : 0;
    if (s2 == LCO_OK && (best < 0 || sz < best_size)) {
      best = k;
      best_size = sz;
    }
  }
  for (int f = 0; f < F; f++) free(smp[f]);
  if (st) return st;
  if (best < 0) return LCO_ERR_RANGE;
  *k_out = best;
  return LCO_OK;
}

/* ------------------------------------------------------------------------
 * Dictionary stage: order-0 rANS over bytes in blocks of 64 interleaved
 * lanes (see lcp_oracle.h for the stream).  Plain sequential code: one block
 * after the other, one lane after the other, one byte at a time.
 * ------------------------------------------------------------------------ */
#define DICT_M (1u << LCO_DICT_SCALE)
#define DICT_L (1u << 23)
#define DICT_W 64
#define DICT_HDR (4 + 4 + 8 + 2 * 256)

static uint64_t dict_blocks(uint64_t n, int block_log2) {
  return (n + (1ull << block_log2) - 1) >> block_log2;
}

uint64_t lco_dict_bound(uint64_t n, int block_log2) {
  if (block_log2 < 12 || block_log2 > 20) return 0;
  const uint64_t nb = dict_blocks(n, block_log2);
  /* a byte costs at most 12 bits (frequency 1 of 4096); a lane adds its state
     and a byte of rounding, a block its table of lane sizes */
  return DICT_HDR + 4 * nb + n + n / 2 + nb * (2 * DICT_W + 8 * DICT_W);
}

int lco_dict_normalise(const uint64_t* counts, uint16_t* freq) {
  uint64_t n = 0;
  for (int s = 0; s < 256; s++) n += counts[s];
  for (int s = 0; s < 256; s++) freq[s] = 0;
  if (n == 0) return LCO_OK;
  uint32_t f[256];
  int64_t sum = 0;
  for (int s = 0; s < 256; s++) {
    f[s] = 0;
    if (counts[s]) {
      const uint64_t q = (uint64_t)(((unsigned __int128)counts[s] * DICT_M) / n);
      f[s] = q < 1 ? 1u : (uint32_t)q;
      sum += f[s];
    }
  }
  if (sum < (int64_t)DICT_M) {
    int best = -1;
    for (int s = 0; s < 256; s++)
      if (counts[s] && (best < 0 || counts[s] > counts[best])) best = s;
    f[best] += (uint32_t)((int64_t)DICT_M - sum);
  }
  int64_t excess = sum - (int64_t)DICT_M;
  while (excess > 0) {
    int best = -1;
    for (int s = 0; s < 256; s++)
      if (f[s] > 1 && (best < 0 || f[s] > f[best])) best = s;
    if (best < 0) return LCO_ERR_CORRUPT; /* not reachable: 256 values < 4096 */
    const uint32_t d = (uint32_t)((int64_t)(f[best] - 1) < excess ? f[best] - 1 : excess);
    f[best] -= d;
    excess -= d;
  }
  for (int s = 0; s < 256; s++) freq[s] = (uint16_t)f[s];
  return LCO_OK;
}

static void put32(uint8_t* p, uint32_t v) {
  for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i));
}
static uint32_t get32(const uint8_t* p) {
  return (uint32_t)p[0] | (uint32_t)p[1] << 8 | (uint32_t)p[2] << 16 | (uint32_t)p[3] << 24;
}

int lco_dict_encode(const uint8_t* in, uint64_t n, int block_log2, uint8_t* out, uint64_t cap,
                    uint64_t* size) {
  if ((n && !in) || !out || !size || block_log2 < 12 || block_log2 > 20) return LCO_ERR_ARG;
  const uint64_t B = 1ull << block_log2, nb = dict_blocks(n, block_log2);
  *size = lco_dict_bound(n, block_log2);
  if (cap < DICT_HDR + 4 * nb) return LCO_ERR_CAPACITY;
  uint64_t counts[256] = {0};
  for (uint64_t i = 0; i < n; i++) counts[in[i]]++;
  uint16_t freq[256];
  int st = lco_dict_normalise(counts, freq);
  if (st) return st;
  uint32_t cum[257];
  cum[0] = 0;
  for (int s = 0; s < 256; s++) cum[s + 1] = cum[s] + freq[s];
  put32(out, LCO_DICT_MAGIC);
  put32(out + 4, (uint32_t)block_log2);
  put32(out + 8, (uint32_t)n);
  put32(out + 12, (uint32_t)(n >> 32));
  for (int s = 0; s < 256; s++) {
    out[16 + 2 * s] = (uint8_t)freq[s];
    out[17 + 2 * s] = (uint8_t)(freq[s] >> 8);
  }
  uint8_t* sizes = out + DICT_HDR;
  uint64_t pos = DICT_HDR + 4 * nb;
  /* a lane codes into a scratch buffer from its end, then is copied */
  const uint64_t lane_cap = (B / DICT_W) + (B / DICT_W) / 2 + 8;
  uint8_t* tmp = (uint8_t*)malloc(lane_cap);
  if (!tmp) return LCO_ERR_BUDGET;
  for (uint64_t b = 0; b < nb; b++) {
    const uint64_t i0 = b * B, len = n - i0 < B ? n - i0 : B;
    const uint64_t bpos = pos;
    if (pos + 2 * DICT_W > cap) {
      free(tmp);
      return LCO_ERR_CAPACITY;
    }
    pos += 2 * DICT_W; /* the lanes' sizes, u16 each */
    for (int k = 0; k < DICT_W; k++) {
      uint8_t* end = tmp + lane_cap;
      uint8_t* p = end;
      uint32_t x = DICT_L;
      /* lane k: bytes k, k + 64, ... of the block, from the last */
      const uint64_t cnt = (uint64_t)k < len ? (len - (uint64_t)k + DICT_W - 1) / DICT_W : 0;
      for (uint64_t m = cnt; m-- > 0;) {
        const uint32_t s = in[i0 + (uint64_t)k + DICT_W * m], f = freq[s];
        const uint32_t x_max = ((DICT_L >> LCO_DICT_SCALE) << 8) * f;
        while (x >= x_max) {
          *--p = (uint8_t)(x & 0xFF);
          x >>= 8;
        }
        x = (x / f) * DICT_M + x % f + cum[s];
      }
      p -= 4;
      put32(p, x);
      const uint64_t lsize = (uint64_t)(end - p);
      out[bpos + 2 * k] = (uint8_t)lsize;
      out[bpos + 2 * k + 1] = (uint8_t)(lsize >> 8);
      if (pos + lsize > cap) {
        free(tmp);
        *size = pos + lsize;
        return LCO_ERR_CAPACITY;
      }
      memcpy(out + pos, p, lsize);
      pos += lsize;
    }
    put32(sizes + 4 * b, (uint32_t)(pos - bpos));
  }
  free(tmp);
  *size = pos;
  return LCO_OK;
}

int lco_dict_decode(const uint8_t* in, uint64_t size, uint8_t* out, uint64_t cap, uint64_t* n_out) {
  if (!in || !n_out || size < DICT_HDR) return LCO_ERR_ARG;
  if (get32(in) != LCO_DICT_MAGIC) return LCO_ERR_CORRUPT;
  const int block_log2 = (int)get32(in + 4);
  if (block_log2 < 12 || block_log2 > 20) return LCO_ERR_CORRUPT;
  const uint64_t n = (uint64_t)get32(in + 8) | (uint64_t)get32(in + 12) << 32;
  *n_out = n;
  const uint64_t B = 1ull << block_log2, nb = dict_blocks(n, block_log2);
  if (nb > (size - DICT_HDR) / 4) return LCO_ERR_CORRUPT;
  if (n > cap || (n && !out)) return LCO_ERR_CAPACITY;
  uint16_t freq[256];
  uint32_t cum[257];
  cum[0] = 0;
  for (int s = 0; s < 256; s++) {
    freq[s] = (uint16_t)(in[16 + 2 * s] | in[17 + 2 * s] << 8);
    cum[s + 1] = cum[s] + freq[s];
  }
  if (n && cum[256] != DICT_M) return LCO_ERR_CORRUPT;
  uint64_t pos = DICT_HDR + 4 * nb;
  for (uint64_t b = 0; b < nb; b++) {
    const uint64_t bsize = get32(in + DICT_HDR + 4 * b);
    const uint64_t i0 = b * B, len = n - i0 < B ? n - i0 : B;
    if (bsize < 2 * DICT_W || pos + bsize > size) return LCO_ERR_CORRUPT;
    uint64_t lpos = pos + 2 * DICT_W;
    for (int k = 0; k < DICT_W; k++) {
      const uint64_t lsize = (uint64_t)in[pos + 2 * k] | (uint64_t)in[pos + 2 * k + 1] << 8;
      if (lsize < 4 || lpos + lsize > pos + bsize) return LCO_ERR_CORRUPT;
      const uint8_t* p = in + lpos;
      uint32_t x = get32(p);
      uint64_t r = 4;
      const uint64_t cnt = (uint64_t)k < len ? (len - (uint64_t)k + DICT_W - 1) / DICT_W : 0;
      for (uint64_t m = 0; m < cnt; m++) {
        const uint32_t slot = x & (DICT_M - 1);
        int s = 0;
        while (cum[s + 1] <= slot) s++; /* the byte whose interval holds the slot */
        x = freq[s] * (x >> LCO_DICT_SCALE) + slot - cum[s];
        while (x < DICT_L) {
          if (r >= lsize) return LCO_ERR_CORRUPT;
          x = (x << 8) | p[r++];
        }
        out[i0 + (uint64_t)k + DICT_W * m] = (uint8_t)s;
      }
      if (x != DICT_L || r != lsize) return LCO_ERR_CORRUPT;
      lpos += lsize;
    }
    if (lpos != pos + bsize) return LCO_ERR_CORRUPT;
    pos += bsize;
  }
  if (pos != size) return LCO_ERR_CORRUPT;
  return LCO_OK;
}
