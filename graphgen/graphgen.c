/*
 * graphgen.c - seeded synthetic input graphs (edge lists) for the triangle
 * counting library, its tests and its benchmark.
 *
 * This module only produces inputs. It holds none of the counting method's
 * arithmetic (no deduplication, ordering, orientation or intersection): the
 * edge lists it writes may contain duplicates, both orientations and self loops,
 * exactly as a raw generator would.
 *
 * Randomness is counter based. Every draw is the output function of SplitMix64
 * (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014) applied to stream_state + (i + 1) * golden_gamma, i.e. the i-th
 * output of a SplitMix64 generator seeded with stream_state. The i-th draw of a
 * stream therefore needs no sequential state, and the generated graph does not
 * depend on the number of host threads.
 *
 * Generators:
 *   gg_rmat  - recursive-matrix graph (Chakrabarti, Zhan and Faloutsos, SDM 2004):
 *              every edge descends `scale` levels of the adjacency matrix,
 *              choosing quadrant (0,0),(0,1),(1,0),(1,1) with probabilities
 *              a, b, c, 1-a-b-c by comparing one 32-bit draw per level against
 *              integer thresholds floor(p * 2^32). No per-level noise. Vertex
 *              ids are then scrambled by a seeded bijection of [0, 2^scale);
 *              when n is not a power of two an edge with an endpoint >= n is
 *              drawn again (next attempt counter), so ids lie in [0, n).
 *   gg_er    - Erdos-Renyi G(n, m): m distinct unordered non-loop pairs, drawn
 *              uniformly by rejection; each pair is emitted in the orientation
 *              it was drawn.
 *   gg_batch_spec - the per-graph (kind, n, parameter, seed) list of a batch of
 *              uneven graphs: n log-uniform in [nmin, nmax], even index ER with
 *              average degree U[dlo, dhi], odd index RMAT with edge factor
 *              U[elo, ehi].
 *   gg_uniform - a vector of U[0,1) doubles from one stream (used for arrival
 *              traces).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* i-th output (0-based) of a SplitMix64 generator whose state starts at `st`. */
static inline uint64_t gg_draw(uint64_t st, uint64_t i) {
  return gg_mix64(st + (i + 1) * GG_GAMMA);
}

/* Independent stream for (seed, purpose). */
static inline uint64_t gg_stream(uint64_t seed, uint64_t purpose) {
  return gg_mix64(gg_mix64(seed) ^ gg_mix64(purpose * GG_GAMMA + 0x632BE59BD9B4E019ULL));
}

/* U[0,1) with 53 random bits. */
static inline double gg_unit(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

enum { GG_P_RMAT = 1, GG_P_PERM = 2, GG_P_ER = 3, GG_P_BATCH = 4, GG_P_UNIFORM = 5 };

/* ---- seeded bijection of [0, 2^bits) ---------------------------------- */
typedef struct {
  int bits;
  uint64_t mask, m[3], c[3];
  int sh[3];
} gg_perm;

static void gg_perm_init(gg_perm* p, int bits, uint64_t seed) {
  uint64_t st = gg_stream(seed, GG_P_PERM);
  p->bits = bits;
  p->mask = bits >= 64 ? ~0ULL : ((1ULL << bits) - 1);
  for (int r = 0; r < 3; ++r) {
    p->m[r] = (gg_draw(st, 2 * r) | 1ULL) & p->mask; /* odd multiplier: bijective mod 2^bits */
    if (p->mask) p->m[r] |= 1ULL;
    p->c[r] = gg_draw(st, 2 * r + 1) & p->mask;
    p->sh[r] = bits > 1 ? (bits + r + 1) / (r + 2) : 1; /* xorshift by >= 1 bit is bijective */
    if (p->sh[r] < 1) p->sh[r] = 1;
  }
}

static inline uint64_t gg_perm_apply(const gg_perm* p, uint64_t x) {
  for (int r = 0; r < 3; ++r) {
    x = (x * p->m[r] + p->c[r]) & p->mask;
    x ^= x >> p->sh[r];
  }
  return x;
}

/* ---- RMAT ---------------------------------------------------------------- */
/* Returns 0 on success, -1 on bad arguments. src/dst have room for m entries. */
int gg_rmat(int scale, int64_t n, int64_t m, uint64_t seed, double a, double b, double c,
            int permute, int32_t* src, int32_t* dst, int nthreads) {
  if (scale < 1 || scale > 30 || m < 0 || n < 1 || n > (1LL << scale) || n <= (1LL << (scale - 1)) && scale > 1)
    return -1;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
  const uint64_t tA = (uint64_t)(a * 4294967296.0);
  const uint64_t tAB = (uint64_t)((a + b) * 4294967296.0);
  const uint64_t tABC = (uint64_t)((a + b + c) * 4294967296.0);
  const uint64_t st = gg_stream(seed, GG_P_RMAT);
  const int words = (scale + 1) / 2; /* two 32-bit level draws per 64-bit word */
  gg_perm perm;
  gg_perm_init(&perm, scale, seed);
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t e = 0; e < m; ++e) {
    for (uint64_t att = 0;; ++att) {
      uint64_t base = ((uint64_t)e * 64ULL + (att & 63ULL) + (att >> 6) * (uint64_t)m * 64ULL) * (uint64_t)words;
      uint64_t u = 0, v = 0, w = 0;
      for (int l = 0; l < scale; ++l) {
        if ((l & 1) == 0) w = gg_draw(st, base + (uint64_t)(l >> 1));
        uint64_t r = (l & 1) ? (w >> 32) : (w & 0xFFFFFFFFULL);
        uint64_t ub, vb;
        if (r < tA) { ub = 0; vb = 0; }
        else if (r < tAB) { ub = 0; vb = 1; }
        else if (r < tABC) { ub = 1; vb = 0; }
        else { ub = 1; vb = 1; }
        u = (u << 1) | ub;
        v = (v << 1) | vb;
      }
      if (permute) {
        u = gg_perm_apply(&perm, u);
        v = gg_perm_apply(&perm, v);
      }
      if ((int64_t)u < n && (int64_t)v < n) {
        src[e] = (int32_t)u;
        dst[e] = (int32_t)v;
        break;
      }
    }
  }
  return 0;
}

/* ---- Erdos-Renyi G(n, m) -------------------------------------------------- */
/* Returns 0 on success, -1 if m exceeds the number of unordered pairs. */
int gg_er(int64_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 1 || m < 0) return -1;
  if ((double)m > (double)n * (double)(n - 1) / 2.0) return -1;
  if (m == 0) return 0;
  uint64_t cap = 1;
  while (cap < (uint64_t)m * 2 + 16) cap <<= 1;
  uint64_t* set = (uint64_t*)calloc(cap, sizeof(uint64_t)); /* 0 = empty, key + 1 stored */
  if (!set) return -1;
  const uint64_t st = gg_stream(seed, GG_P_ER);
  int64_t out = 0;
  for (uint64_t i = 0; out < m; ++i) {
    uint64_t w = gg_draw(st, i);
    uint64_t u = ((w & 0xFFFFFFFFULL) * (uint64_t)n) >> 32;
    uint64_t v = ((w >> 32) * (uint64_t)n) >> 32;
    if (u == v) continue;
    uint64_t lo = u < v ? u : v, hi = u < v ? v : u;
    uint64_t key = lo * (uint64_t)n + hi + 1;
    uint64_t h = gg_mix64(key) & (cap - 1);
    int fresh = 1;
    while (set[h]) {
      if (set[h] == key) { fresh = 0; break; }
      h = (h + 1) & (cap - 1);
    }
    if (!fresh) continue;
    set[h] = key;
    src[out] = (int32_t)u;
    dst[out] = (int32_t)v;
    ++out;
  }
  free(set);
  return 0;
}

/* ---- batch of uneven graphs ---------------------------------------------- */
/* kind[g] = 0 (ER) or 1 (RMAT); n[g]; m[g] = number of generated edges
 * (ER: distinct pairs = round(n * avgdeg / 2); RMAT: round(n * edgefactor));
 * param[g] = avg degree or edge factor; gseed[g] = seed_base + g. */
void gg_batch_spec(int32_t count, uint64_t seed, int64_t nmin, int64_t nmax, double dlo, double dhi,
                   double elo, double ehi, uint64_t seed_base, int32_t* kind, int64_t* n, int64_t* m,
                   double* param, uint64_t* gseed) {
  const uint64_t st = gg_stream(seed, GG_P_BATCH);
  const double l0 = log((double)nmin), l1 = log((double)nmax);
  for (int32_t g = 0; g < count; ++g) {
    double u0 = gg_unit(gg_draw(st, 2 * (uint64_t)g));
    double u1 = gg_unit(gg_draw(st, 2 * (uint64_t)g + 1));
    int64_t nn = (int64_t)floor(exp(l0 + u0 * (l1 - l0)));
    if (nn < nmin) nn = nmin;
    if (nn > nmax) nn = nmax;
    n[g] = nn;
    gseed[g] = seed_base + (uint64_t)g;
    if ((g & 1) == 0) {
      double d = dlo + u1 * (dhi - dlo);
      int64_t mm = llround((double)nn * d / 2.0);
      int64_t maxp = nn * (nn - 1) / 2;
      kind[g] = 0;
      param[g] = d;
      m[g] = mm > maxp ? maxp : mm;
    } else {
      double ef = elo + u1 * (ehi - elo);
      kind[g] = 1;
      param[g] = ef;
      m[g] = llround((double)nn * ef);
    }
  }
}

/* ---- uniform stream -------------------------------------------------------- */
void gg_uniform(uint64_t seed, uint64_t purpose, int64_t count, double* out) {
  const uint64_t st = gg_stream(seed, GG_P_UNIFORM * 1000003ULL + purpose);
  for (int64_t i = 0; i < count; ++i) out[i] = gg_unit(gg_draw(st, (uint64_t)i));
}

/* smallest s with 2^s >= n (n >= 1); at least 1 */
int gg_scale_for(int64_t n) {
  int s = 1;
  while ((1LL << s) < n) ++s;
  return s;
}
