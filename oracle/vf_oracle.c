/*
 * vf_oracle.c -- plain, slow, obviously-correct CPU oracle for the
 * epsilon-cost sharded VFunc / VFilter construction and query of
 * S. Vigna, "epsilon-Cost Sharding: Scaling Hypergraph-Based Static
 * Functions and Filters to Trillions of Keys" (arXiv 2503.18397).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark call this code.  It shares nothing with
 * the HIP library: no header, helper, table or constant generator.
 *
 * The paper leaves several choices open (hash function, bit fields of the
 * signature, which of the many solutions of the 2-core system is stored,
 * per-shard seeds).  The readings taken here are, in order of use:
 *
 *  R1 signatures: two 64-bit words, each the SplitMix64 finalizer of the key
 *     xored with a seed word; the seed words are the first three outputs of
 *     SplitMix64 started at the user seed (section 4.3 hashes keys once to
 *     signatures and derives everything from them).
 *  R2 shard = the h highest bits of the first word (section 4, "higher bits").
 *  R3 segment = fixed-point inversion of 32 bits F: g = (F * ell) >> 32
 *     (section 4.5), F = the 32 bits right below the shard bits for local
 *     seed t = 0 (so the segment is monotone in the signature) and the high
 *     32 bits of L_t (R4) for t > 0.
 *  R4 in-segment offsets = three disjoint sigma-bit fields of L_t: the
 *     second word for t = 0, SplitMix64's finalizer of (second word +
 *     t * golden gamma) for t > 0.  Shard and fingerprint never depend on
 *     t; every retry of a shard draws a new graph (segments too, as a
 *     rehash with a local seed does in HEM, section 3.2): a fuse graph
 *     whose segments are overloaded (more equations than vertices in a
 *     stretch of segments) would otherwise stay unsolvable under every
 *     local seed.
 *  R5 fingerprint = top b bits of the finalizer of (hi ^ lo ^ third seed
 *     word); it is derived from the signature (section 4.5), so keys with
 *     equal signatures have equal fingerprints.
 *  R6 geometry: c = 1.105 and lg s from eq. (nln) for shards of at least
 *     800 000 keys, c = 1.125 and lg s from eq. (ln) for a single unsharded
 *     graph of at least 800 000 keys (Graf and Lemire's estimate, which
 *     section 4.2 says the paper partly adopts).  Below 800 000 keys section
 *     4.2 keeps c = 1.12 and solves what does not peel by Gaussian
 *     elimination, but fixes no segment size; section 4 leaves sizing to
 *     simulation where no bound is known.  Simulated with this oracle (one
 *     graph per size, 40 key sets, up to 64 local seeds): c = 1.12 builds
 *     whenever the middle segments carry at most about 0.93 equations per
 *     vertex, m / (ell s) <= 0.93, and the segments hold at least 2^8
 *     vertices; smaller segments fail for every local seed at any size
 *     (their local overloads do not move with the seed: the segment of a
 *     key never depends on it), and denser middle segments fail at 2 000 to
 *     8 000 keys.  Hence, for m keys with 64 <= m < 2^16:
 *       sigma = min(8, floor(lg m) - 2),
 *     and for 2^16 <= m < 800 000, sigma = 9, which keeps the expected
 *     duplicate edges of a shard, m / (2 c s^2) (section 4.2), at 0.11 for
 *     2^16 keys (0.45 with s = 2^8: a duplicate edge costs a retry);
 *       c = max(1.12, 1.075 + 2 s / m), rounded up to thousandths,
 *     which is c = 1.12 from 11 378 keys up and otherwise the smallest
 *     factor that keeps the middle density at 1 / 1.075 = 0.93.  The cap
 *     sigma <= 9 is a capacity parameter of the GPU elimination (the
 *     window of rows it keeps in LDS spans three segments), not a reading
 *     of the paper.
 *     Graphs of fewer than 64 keys are one block of three segments
 *     (ell = 1) with s = 2^ceil(lg((m + 1) / 2)), a random 3-partite
 *     hypergraph with 1.5 to 3 vertices per key; c is then reported as
 *     3 s / m.  ell = max(1, ceil(c M / s) - 2), V = (ell + 2) s.
 *  R11 MWHC (section 4.1): a 3-partite 3-hypergraph with three parts of
 *     ceil(c M / 3) vertices, c = 1.23 (the section's example); vertex i of
 *     an edge is i * part + ((f_i * part) >> 21) with f_i the i-th 21-bit
 *     field of L_t (R4).  The construction is peel-only, as in the paper:
 *     an attempt that leaves any edge unpeeled fails (kind 2) and the shard
 *     moves to its next local seed.  The paper bounds the shard count by
 *     eq. (dupmwhc) because it restarts globally on a duplicate edge; with
 *     local seeds a duplicate costs one shard's retry, so h comes from
 *     eq. (logballsbins) alone.
 *  R7 peeling is round-synchronous: in round r every live edge that has a
 *     vertex of degree one (degrees as they stand when the round starts) is
 *     removed; its hinge is the first such vertex in edge order (its
 *     "side", section 4.3).  The result does not depend on key order.
 *  R8 the unpeeled 2-core is solved by Gaussian elimination over GF(2) with
 *     every pivot the highest-numbered variable of its row and free
 *     variables set to zero.  This is the lexicographically smallest
 *     solution (vertex 0 most significant) of the core system, hence
 *     independent of equation order and of the elimination method.
 *  R9 values are assigned in reverse peel order: w[hinge] = rhs xor the
 *     other two vertices (section 4.3); unassigned vertices stay 0.
 *  R10 a shard whose core system is inconsistent is rebuilt with the next
 *     local seed t (HEM keeps a local seed per shard, section 3.2); the
 *     first successful t is stored, the failed attempts are recorded.
 */
#include "vf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN_GAMMA 0x9e3779b97f4a7c15ULL

/* ---------------------------------------------------------------- hashing */

/* SplitMix64 output function (Steele, Lea, Flood 2014; constants of
 * Stafford's "Mix13"): a bijection of 64-bit words. */
uint64_t orc_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* R1: the first three outputs of SplitMix64 started at `seed`. */
void orc_seed_words(uint64_t seed, uint64_t out[3]) {
  uint64_t state = seed;
  for (int i = 0; i < 3; i++) {
    state += GOLDEN_GAMMA;
    out[i] = orc_mix64(state);
  }
}

/* R1: key -> (hi, lo) signature. */
void orc_signature(uint64_t key, const uint64_t sw[3], uint64_t *hi,
                   uint64_t *lo) {
  *hi = orc_mix64(key ^ sw[0]);
  *lo = orc_mix64(key ^ sw[1]);
}

/* R5: b-bit filter fingerprint (Problem 2 via a static function to a
 * b-bit hash, section 3.1). */
uint64_t orc_fingerprint(uint64_t hi, uint64_t lo, const uint64_t sw[3],
                         int32_t b) {
  uint64_t f = orc_mix64(hi ^ lo ^ sw[2]);
  return b >= 64 ? f : f >> (64 - b);
}

/* R2: the shard of a signature is given by its h highest bits. */
uint32_t orc_shard_of(uint64_t hi, int32_t h) {
  return h == 0 ? 0u : (uint32_t)(hi >> (64 - h));
}

/* R3, R4: the fuse 3-graph edge of a signature in a shard of geometry
 * (ell, sigma) -- one vertex in each of the segments g, g+1, g+2
 * (section 4.2, definition of fuse graphs). */
void orc_edge(uint64_t hi, uint64_t lo, int32_t h, uint32_t l, int32_t sigma,
              uint32_t t, uint32_t v[3]) {
  uint64_t L = t == 0 ? lo : orc_mix64(lo + (uint64_t)t * GOLDEN_GAMMA);
  /* t = 0: the 32 bits right below the shard bits; t > 0: the top of L_t */
  uint64_t F = t == 0 ? (hi << h) >> 32 : L >> 32;
  uint64_t g = (F * (uint64_t)l) >> 32;
  uint64_t s = 1ULL << sigma;
  for (int i = 0; i < 3; i++)
    v[i] = (uint32_t)((g + (uint64_t)i) * s + ((L >> (i * sigma)) & (s - 1)));
}

/* R11: the MWHC edge of a signature (section 4.1, the 3-partite
 * construction): vertex i lies in part i of `part` vertices, at the
 * fixed-point image of the i-th 21-bit field of L_t (R4).  Shard bits and
 * segments play no role. */
void orc_edge_mwhc(uint64_t lo, uint32_t part, uint32_t t, uint32_t v[3]) {
  uint64_t L = t == 0 ? lo : orc_mix64(lo + (uint64_t)t * GOLDEN_GAMMA);
  for (int i = 0; i < 3; i++) {
    uint64_t f = (L >> (21 * i)) & ((1ULL << 21) - 1);
    v[i] = (uint32_t)((uint64_t)i * part + ((f * part) >> 21));
  }
}

/* --------------------------------------------------------- parameter math */

/* Principal branch of Lambert's W by Halley iteration (Corless, Gonnet,
 * Hare, Jeffrey, Knuth, "On the Lambert W function", 1996).  Section 4.2
 * asks for an accurate W, not the ln x - ln ln x approximation. */
double orc_lambert_w0(double x) {
  const double e = 2.718281828459045;
  if (x < -1.0 / e) return NAN;
  if (x == 0.0) return 0.0;
  double w;
  if (x < -0.3) { /* series at the branch point -1/e */
    double p = sqrt(2.0 * (e * x + 1.0));
    w = -1.0 + p - p * p / 3.0 + 11.0 / 72.0 * p * p * p;
  } else if (x < 3.0) {
    w = log1p(x) * 0.75;
  } else {
    double lx = log(x);
    w = lx - log(lx);
  }
  for (int it = 0; it < 200; it++) {
    double ew = exp(w);
    double f = w * ew - x;
    double wp1 = w + 1.0;
    if (wp1 == 0.0) break;
    double d = f / (ew * wp1 - (w + 2.0) * f / (2.0 * wp1));
    w -= d;
    if (fabs(d) <= 1e-16 * (1.0 + fabs(w))) break;
  }
  return w;
}

/* eq. (logballsbins): the number of shard bits that keeps the largest shard
 * within (1 + eps) of the mean (Raab-Steger bound with constant alpha). */
int32_t orc_shard_bits_eps(double n, double eps, double alpha) {
  double x = n * eps * eps / (2.0 * alpha * alpha);
  if (!(x > 2.718281828459045)) return 0;
  double hb = floor(log2(x) - log2(log(x)));
  if (hb < 0) hb = 0;
  if (hb > 32) hb = 32;
  return (int32_t)hb;
}

/* eq. (ballsbins) with the exact W: lg of the largest admissible shard
 * count, as a real number. */
double orc_shard_bits_exact(double n, double eps, double alpha) {
  double x = n * eps * eps / (2.0 * alpha * alpha);
  return orc_lambert_w0(x) / log(2.0);
}

/* eq. (dupmwhc): the number of shard bits for which a random 3-partite
 * hypergraph has no duplicate edge in any shard with probability >= 1-eta. */
int32_t orc_dupmwhc_bits(double n, double c, double eta) {
  double r = c / 3.0;
  double S = sqrt(-2.0 * n * r * r * r * log1p(-eta));
  return (int32_t)floor(log2(S));
}

/* The argument shared by eq. (dupfuse) and eq. (logdupfuse). */
static double dupfuse_arg(double n, double c, double eta, double alpha,
                          double beta) {
  return (log2(-n / (2.0 * c * log1p(-eta))) - 2.0 * beta) / (2.0 * alpha);
}

/* eq. (logdupfuse): right-hand side, as printed, of the bound on h. */
double orc_logdupfuse(double n, double c, double eta, double alpha,
                      double beta) {
  double A = dupfuse_arg(n, c, eta, alpha, beta);
  return log2(n) - A / (log(2.0) * orc_lambert_w0(A));
}

/* eq. (dupfuse): right-hand side, as printed, of the bound on S. */
double orc_dupfuse(double n, double c, double eta, double alpha, double beta) {
  double A = dupfuse_arg(n, c, eta, alpha, beta);
  return n * exp(-A / orc_lambert_w0(A));
}

/* R6: expansion factor, segment size and vertex count of every shard. */
void orc_geometry(uint32_t M, int32_t h, uint32_t c_num, uint32_t c_den,
                  int32_t sigma_override, orc_geom *g) {
  int large = M >= 800000u;
  int32_t sigma = -1;
  if (sigma_override >= 0) sigma = sigma_override;
  else if (large && h > 0) { /* eq. (nln) read as lg of the segment size */
    double lm = log((double)M);
    sigma = (int32_t)floor(0.41 * lm * log(lm) - 3.0);
  } else if (large) { /* eq. (ln), Graf and Lemire's segment size */
    sigma = (int32_t)floor(log((double)M) / log(3.33) + 2.25);
  } else if (M < 64u) { /* one block of three segments, s >= (M + 1) / 2 */
    sigma = 0;
    while ((2ULL << sigma) < (uint64_t)M + 1) sigma++;
  } else if (M >= 65536u) { /* 2^9 from 2^16 keys */
    sigma = 9;
  } else { /* floor(lg M) - 2, at most 8 */
    int32_t lg = 0;
    while ((2ULL << lg) <= M) lg++;
    sigma = lg - 2 < 8 ? lg - 2 : 8;
  }
  if (sigma < 0) sigma = 0;
  if (sigma > 20) sigma = 20;
  if (c_num == 0 || c_den == 0) {
    if (large && h > 0) { c_num = 1105; c_den = 1000; }  /* 1.105 */
    else if (large) { c_num = 1125; c_den = 1000; }      /* 1.125 */
    else if (M < 64u) { /* ell = 1 with the block's own segment size */
      int32_t st = 0;
      while ((2ULL << st) < (uint64_t)M + 1) st++;
      c_num = 3u << st;
      c_den = M ? M : 1u;
    } else { /* max(1.12, 1.075 + 2 s / M) in thousandths, rounded up */
      uint64_t x = 1075 + (2000ULL * (1ULL << sigma) + M - 1) / M;
      c_num = x > 1120 ? (uint32_t)x : 1120u;
      c_den = 1000;
    }
  }
  uint64_t num = (uint64_t)c_num * M;
  uint64_t den = (uint64_t)c_den << sigma;
  uint64_t q = (num + den - 1) / den; /* ceil(c M / s) */
  uint32_t l = q > 3 ? (uint32_t)(q - 2) : 1u;
  g->M = M;
  g->h = h;
  g->c_num = c_num;
  g->c_den = c_den;
  g->sigma = sigma;
  g->l = l;
  g->V = ((uint64_t)l + 2) << sigma;
  g->mwhc = 0;
  g->part = 0;
}

/* R11: MWHC geometry: c = 1.23 (section 4.1's example) unless given, three
 * parts of ceil(c M / 3) vertices. */
void orc_geometry_mwhc(uint32_t M, int32_t h, uint32_t c_num, uint32_t c_den,
                       orc_geom *g) {
  if (c_num == 0 || c_den == 0) {
    c_num = 123;
    c_den = 100;
  }
  uint64_t den = 3ULL * c_den;
  uint64_t part = ((uint64_t)c_num * M + den - 1) / den;
  if (part == 0) part = 1;
  g->M = M;
  g->h = h;
  g->c_num = c_num;
  g->c_den = c_den;
  g->sigma = 0;
  g->l = 1;
  g->V = 3 * part;
  g->mwhc = 1;
  g->part = (uint32_t)part;
}

/* --------------------------------------------------------------- solvers */

/* R7: round-synchronous peeling.  round[i] = round in which edge i was
 * peeled (-1: in the 2-core), side[i] = position of its hinge in the edge.
 * Returns the number of rounds that peeled at least one edge. */
int32_t orc_peel(uint64_t nv, uint32_t m, const uint32_t *e, int32_t *round,
                 int8_t *side) {
  uint32_t *deg = (uint32_t *)calloc(nv ? nv : 1, sizeof(uint32_t));
  uint32_t *now = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
  for (uint32_t i = 0; i < m; i++) {
    round[i] = -1;
    side[i] = -1;
    for (int k = 0; k < 3; k++) deg[e[3 * i + k]]++;
  }
  int32_t r = 0;
  for (;;) {
    uint32_t np = 0;
    /* select with the degrees of the start of the round */
    for (uint32_t i = 0; i < m; i++) {
      if (round[i] >= 0) continue;
      int k;
      for (k = 0; k < 3; k++)
        if (deg[e[3 * i + k]] == 1) break;
      if (k < 3) {
        round[i] = r;
        side[i] = (int8_t)k;
        now[np++] = i;
      }
    }
    if (np == 0) break;
    for (uint32_t j = 0; j < np; j++)
      for (int k = 0; k < 3; k++) deg[e[3 * now[j] + k]]--;
    r++;
  }
  free(now);
  free(deg);
  return r;
}

/* A row of the core system: sorted distinct variables and a right side. */
typedef struct {
  uint32_t *v;
  uint32_t n;
  uint64_t rhs;
} row_t;

/* Symmetric difference of two sorted variable lists (GF(2) row sum). */
static row_t row_xor(row_t a, row_t b) {
  row_t c;
  c.v = (uint32_t *)malloc(((size_t)a.n + b.n + 1) * sizeof(uint32_t));
  c.n = 0;
  c.rhs = a.rhs ^ b.rhs;
  uint32_t i = 0, j = 0;
  while (i < a.n || j < b.n) {
    if (j == b.n || (i < a.n && a.v[i] < b.v[j])) c.v[c.n++] = a.v[i++];
    else if (i == a.n || b.v[j] < a.v[i]) c.v[c.n++] = b.v[j++];
    else { i++; j++; }
  }
  return c;
}

/* A core row keyed by its highest variable, for sorting (no shared state:
 * the oracle may run on several threads at once). */
typedef struct {
  uint32_t top, row;
} top_row;

static int by_top_desc(const void *pa, const void *pb) {
  const top_row *a = (const top_row *)pa, *b = (const top_row *)pb;
  if (a->top != b->top) return a->top > b->top ? -1 : 1;
  return a->row < b->row ? -1 : (a->row > b->row);
}

/* R8: lexicographically smallest solution of the k equations
 * x[r0] ^ x[r1] ^ x[r2] = rhs (variables below nv).  Gaussian elimination
 * with the highest-numbered variable of each row as its pivot; equations are
 * inserted from the highest variable down (any order gives the same pivots
 * and the same solution), free variables are 0, and back-substitution runs
 * from the lowest pivot up.  x must be zero on entry; only pivot variables
 * are written.  Returns 0, or 1 if the system is inconsistent. */
int32_t orc_core_lexmin(uint64_t nv, uint32_t k, const uint32_t *rows3,
                        const uint64_t *rhs, uint64_t *x) {
  int64_t *piv = (int64_t *)malloc((nv ? nv : 1) * sizeof(int64_t));
  for (uint64_t v = 0; v < nv; v++) piv[v] = -1;
  row_t *store = (row_t *)malloc((k ? k : 1) * sizeof(row_t));
  uint32_t nstore = 0;
  top_row *order = (top_row *)malloc((k ? k : 1) * sizeof(top_row));
  for (uint32_t i = 0; i < k; i++) {
    uint32_t t = rows3[3 * i];
    if (rows3[3 * i + 1] > t) t = rows3[3 * i + 1];
    if (rows3[3 * i + 2] > t) t = rows3[3 * i + 2];
    order[i].top = t;
    order[i].row = i;
  }
  qsort(order, k, sizeof(top_row), by_top_desc);
  int32_t bad = 0;
  for (uint32_t oi = 0; oi < k && !bad; oi++) {
    uint32_t i = order[oi].row;
    /* sort the three variables; a variable twice in a row cancels */
    uint32_t a[3] = {rows3[3 * i], rows3[3 * i + 1], rows3[3 * i + 2]};
    for (int p = 0; p < 3; p++)
      for (int q = p + 1; q < 3; q++)
        if (a[q] < a[p]) { uint32_t tmp = a[p]; a[p] = a[q]; a[q] = tmp; }
    row_t r;
    r.v = (uint32_t *)malloc(3 * sizeof(uint32_t));
    r.n = 0;
    r.rhs = rhs[i];
    for (int p = 0; p < 3; p++) {
      if (r.n > 0 && r.v[r.n - 1] == a[p]) r.n--;
      else r.v[r.n++] = a[p];
    }
    for (;;) {
      if (r.n == 0) {
        if (r.rhs != 0) bad = 1;
        free(r.v);
        break;
      }
      uint32_t p = r.v[r.n - 1];
      if (piv[p] < 0) {
        piv[p] = nstore;
        store[nstore++] = r;
        break;
      }
      row_t nr = row_xor(r, store[piv[p]]);
      free(r.v);
      r = nr;
    }
  }
  if (!bad) {
    for (uint64_t p = 0; p < nv; p++) {
      if (piv[p] < 0) continue;
      row_t r = store[piv[p]];
      uint64_t val = r.rhs;
      for (uint32_t j = 0; j + 1 < r.n; j++) val ^= x[r.v[j]];
      x[p] = val;
    }
  }
  for (uint32_t i = 0; i < nstore; i++) free(store[i].v);
  free(store);
  free(order);
  free(piv);
  return bad;
}

/* R7-R9 on one hypergraph: peel, solve the 2-core, assign in reverse peel
 * order.  w (nv words) is overwritten.  Returns 0, or 1 if the core system
 * is inconsistent (w is then all zero). */
int32_t orc_solve(uint64_t nv, uint32_t m, const uint32_t *e,
                  const uint64_t *rhs, uint64_t *w, uint32_t *core_edges) {
  int32_t *round = (int32_t *)malloc((m ? m : 1) * sizeof(int32_t));
  int8_t *side = (int8_t *)malloc(m ? m : 1);
  int32_t nr = orc_peel(nv, m, e, round, side);
  uint32_t k = 0;
  for (uint32_t i = 0; i < m; i++) k += round[i] < 0;
  uint32_t *rows3 = (uint32_t *)malloc((3 * (size_t)k + 1) * sizeof(uint32_t));
  uint64_t *crhs = (uint64_t *)malloc((k + 1) * sizeof(uint64_t));
  k = 0;
  for (uint32_t i = 0; i < m; i++) {
    if (round[i] >= 0) continue;
    for (int q = 0; q < 3; q++) rows3[3 * k + q] = e[3 * i + q];
    crhs[k++] = rhs[i];
  }
  if (core_edges) *core_edges = k;
  memset(w, 0, nv * sizeof(uint64_t));
  int32_t bad = orc_core_lexmin(nv, k, rows3, crhs, w);
  if (bad) {
    memset(w, 0, nv * sizeof(uint64_t));
  } else {
    /* edges of round r, for r from the last round down to 0 */
    uint32_t *cnt = (uint32_t *)calloc((size_t)nr + 1, sizeof(uint32_t));
    for (uint32_t i = 0; i < m; i++)
      if (round[i] >= 0) cnt[round[i] + 1]++;
    for (int32_t r = 0; r < nr; r++) cnt[r + 1] += cnt[r];
    uint32_t *byr = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t *fill = (uint32_t *)malloc(((size_t)nr + 1) * sizeof(uint32_t));
    memcpy(fill, cnt, ((size_t)nr + 1) * sizeof(uint32_t));
    for (uint32_t i = 0; i < m; i++)
      if (round[i] >= 0) byr[fill[round[i]]++] = i;
    for (int32_t r = nr - 1; r >= 0; r--) {
      for (uint32_t j = cnt[r]; j < cnt[r + 1]; j++) {
        uint32_t i = byr[j];
        int hs = side[i];
        uint64_t val = rhs[i];
        for (int q = 0; q < 3; q++)
          if (q != hs) val ^= w[e[3 * i + q]];
        w[e[3 * i + hs]] = val;
      }
    }
    free(fill);
    free(byr);
    free(cnt);
  }
  free(crhs);
  free(rows3);
  free(side);
  free(round);
  return bad;
}

/* ------------------------------------------------- construction and query */

/* Count keys per shard and derive the common geometry (section 4: every
 * shard is sized by the largest one).  counts has 2^h entries. */
int32_t orc_plan(const uint64_t *keys, uint64_t n, int32_t h, uint64_t seed,
                 uint32_t c_num, uint32_t c_den, int32_t sigma_override,
                 orc_geom *g, uint32_t *counts) {
  if (h < 0 || h > 32) return -1;
  uint64_t S = 1ULL << h;
  uint64_t sw[3];
  orc_seed_words(seed, sw);
  memset(counts, 0, S * sizeof(uint32_t));
  for (uint64_t i = 0; i < n; i++) {
    uint64_t hi, lo;
    orc_signature(keys[i], sw, &hi, &lo);
    counts[orc_shard_of(hi, h)]++;
  }
  uint32_t M = 0;
  for (uint64_t j = 0; j < S; j++)
    if (counts[j] > M) M = counts[j];
  orc_geometry(M, h, c_num, c_den, sigma_override, g);
  return 0;
}

/* R2 for a whole key array: out[i] = shard of keys[i]. */
void orc_shard_ids(const uint64_t *keys, uint64_t n, int32_t h, uint64_t seed,
                   uint32_t *out) {
  uint64_t sw[3];
  orc_seed_words(seed, sw);
  for (uint64_t i = 0; i < n; i++) {
    uint64_t hi, lo;
    orc_signature(keys[i], sw, &hi, &lo);
    out[i] = orc_shard_of(hi, h);
  }
}

/* Build the listed shards (all shards if shards == NULL).  w_out holds V
 * words per listed shard, in list order; t_out holds the local seed of every
 * listed shard (tmax if every attempt failed).  Returns 0, or 1 if some
 * listed shard failed all tmax attempts. */
int32_t orc_build(const uint64_t *keys, const uint64_t *values, uint64_t n,
                  int32_t b, int32_t is_filter, uint64_t seed, uint32_t tmax,
                  const orc_geom *g, const uint32_t *shards, uint32_t nshards,
                  uint32_t *t_out, uint64_t *w_out, orc_fail *rec,
                  uint32_t rec_cap, uint32_t *nrec) {
  uint64_t S = 1ULL << g->h;
  uint64_t sw[3];
  orc_seed_words(seed, sw);
  uint64_t mask = b >= 64 ? ~0ULL : ((1ULL << b) - 1);
  uint64_t *hi = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
  uint64_t *lo = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
  uint32_t *sh = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
  uint64_t *start = (uint64_t *)calloc(S + 1, sizeof(uint64_t));
  for (uint64_t i = 0; i < n; i++) {
    orc_signature(keys[i], sw, &hi[i], &lo[i]);
    sh[i] = orc_shard_of(hi[i], g->h);
    start[sh[i] + 1]++;
  }
  for (uint64_t j = 0; j < S; j++) start[j + 1] += start[j];
  /* keys of each shard, in input order */
  uint64_t *idx = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
  uint64_t *fill = (uint64_t *)malloc((S + 1) * sizeof(uint64_t));
  memcpy(fill, start, (S + 1) * sizeof(uint64_t));
  for (uint64_t i = 0; i < n; i++) idx[fill[sh[i]]++] = i;
  free(fill);

  uint32_t M = g->M;
  uint64_t *shi = (uint64_t *)malloc((M ? M : 1) * sizeof(uint64_t));
  uint64_t *slo = (uint64_t *)malloc((M ? M : 1) * sizeof(uint64_t));
  uint64_t *srhs = (uint64_t *)malloc((M ? M : 1) * sizeof(uint64_t));
  uint32_t *e = (uint32_t *)malloc((3 * (size_t)M + 1) * sizeof(uint32_t));
  int32_t *prd = (int32_t *)malloc(((size_t)M + 1) * sizeof(int32_t));
  int8_t *psd = (int8_t *)malloc((size_t)M + 1);
  int32_t status = 0;
  *nrec = 0;
  uint32_t count = shards ? nshards : (uint32_t)S;
  for (uint32_t q = 0; q < count; q++) {
    uint32_t j = shards ? shards[q] : q;
    uint64_t *w = w_out + (uint64_t)q * g->V;
    uint32_t m = (uint32_t)(start[j + 1] - start[j]);
    for (uint32_t i = 0; i < m; i++) {
      uint64_t k = idx[start[j] + i];
      shi[i] = hi[k];
      slo[i] = lo[k];
      srhs[i] = is_filter ? orc_fingerprint(hi[k], lo[k], sw, b)
                          : (values[k] & mask);
    }
    uint32_t t;
    for (t = 0; t < tmax; t++) {
      for (uint32_t i = 0; i < m; i++) {
        if (g->mwhc) orc_edge_mwhc(slo[i], g->part, t, &e[3 * i]);
        else orc_edge(shi[i], slo[i], g->h, g->l, g->sigma, t, &e[3 * i]);
      }
      uint32_t core = 0;
      int32_t st;
      if (g->mwhc) {
        /* MWHC is peel-only (R11): any unpeeled edge fails the attempt */
        orc_peel(g->V, m, e, prd, psd);
        for (uint32_t i = 0; i < m; i++) core += prd[i] < 0;
        st = core > 0;
        if (!st) st = orc_solve(g->V, m, e, srhs, w, &core);
      } else {
        st = orc_solve(g->V, m, e, srhs, w, &core);
      }
      if (st == 0) break;
      if (*nrec < rec_cap) {
        rec[*nrec].shard = j;
        rec[*nrec].attempt = t;
        rec[*nrec].kind = g->mwhc ? 2 : 1;
        rec[*nrec].core_edges = core;
      }
      (*nrec)++;
    }
    t_out[q] = t;
    if (t == tmax) status = 1;
  }
  free(psd);
  free(prd);
  free(e);
  free(srhs);
  free(slo);
  free(shi);
  free(idx);
  free(start);
  free(sh);
  free(lo);
  free(hi);
  return status;
}

/* Bit-array storage of b-bit values (section 5): cell i occupies bits
 * [i b, i b + b) of a string of little-endian 64-bit words, bit k of the
 * cell at bit i b + k.  out (ceil(count b / 64) words) must be zero. */
void orc_pack(const uint64_t *w, uint64_t count, int32_t b, uint64_t *out) {
  for (uint64_t i = 0; i < count; i++)
    for (int32_t k = 0; k < b; k++)
      if ((w[i] >> k) & 1u) {
        uint64_t bit = i * (uint64_t)b + (uint64_t)k;
        out[bit / 64] |= 1ULL << (bit % 64);
      }
}

/* The b-bit cell i of a packed string. */
uint64_t orc_unpack(const uint64_t *words, uint64_t i, int32_t b) {
  uint64_t v = 0;
  for (int32_t k = 0; k < b; k++) {
    uint64_t bit = i * (uint64_t)b + (uint64_t)k;
    v |= ((words[bit / 64] >> (bit % 64)) & 1u) << k;
  }
  return v;
}

/* Query (eq. (MWHC) with k = 3): the xor of the three cells of the key's
 * edge in its shard; a filter compares it with the key's fingerprint.
 * slot_of_shard maps a shard to its block of V words in w (NULL: identity;
 * negative: not built, the answer is all ones). */
void orc_query(const uint64_t *keys, uint64_t n, uint64_t seed, int32_t b,
               int32_t is_filter, const orc_geom *g, const uint32_t *t_of_shard,
               const int32_t *slot_of_shard, const uint64_t *w, uint64_t *out) {
  uint64_t sw[3];
  orc_seed_words(seed, sw);
  for (uint64_t i = 0; i < n; i++) {
    uint64_t hi, lo;
    orc_signature(keys[i], sw, &hi, &lo);
    uint32_t j = orc_shard_of(hi, g->h);
    int64_t slot = slot_of_shard ? slot_of_shard[j] : (int64_t)j;
    if (slot < 0) {
      out[i] = ~0ULL;
      continue;
    }
    uint32_t v[3];
    if (g->mwhc) orc_edge_mwhc(lo, g->part, t_of_shard[j], v);
    else orc_edge(hi, lo, g->h, g->l, g->sigma, t_of_shard[j], v);
    const uint64_t *ws = w + (uint64_t)slot * g->V;
    uint64_t val = ws[v[0]] ^ ws[v[1]] ^ ws[v[2]];
    if (is_filter) out[i] = val == orc_fingerprint(hi, lo, sw, b);
    else out[i] = val;
  }
}
