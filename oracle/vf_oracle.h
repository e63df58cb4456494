/*
 * vf_oracle.h -- interface of the plain CPU oracle for epsilon-cost sharded
 * static functions (VFunc) and static filters (VFilter), after S. Vigna,
 * "epsilon-Cost Sharding: Scaling Hypergraph-Based Static Functions and
 * Filters to Trillions of Keys" (arXiv 2503.18397).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may call anything declared here.  The
 * product path (the HIP library) shares no code, header, table or helper
 * with this file and must never call it.
 *
 * Every value is a plain integer; vertices of a shard are numbered
 * 0 .. V-1, and the structure of shard j occupies cells j*V .. j*V+V-1.
 */
#ifndef VF_ORACLE_H
#define VF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Geometry of every shard (epsilon-cost sharding sizes all shards by the
 * largest one, section 4). */
typedef struct {
  uint32_t M;      /* keys in the largest shard */
  int32_t h;       /* shard bits, S = 2^h */
  uint32_t c_num;  /* expansion factor c = c_num / c_den */
  uint32_t c_den;
  int32_t sigma;   /* segment size s = 2^sigma */
  uint32_t l;      /* number of start segments (ell) */
  uint64_t V;      /* vertices per shard = (ell + 2) * s, or 3 * part */
  uint32_t mwhc;   /* 1: MWHC 3-partite hypergraph (section 4.1) */
  uint32_t part;   /* MWHC: vertices per part, ceil(c M / 3) */
} orc_geom;

/* One failed construction attempt of one shard. */
typedef struct {
  uint32_t shard;
  uint32_t attempt;    /* local seed t of the attempt */
  uint32_t kind;       /* 1 = inconsistent 2-core system, 2 = MWHC graph
                          not peelable */
  uint32_t core_edges; /* edges left unpeeled in that attempt */
} orc_fail;

/* hashing */
uint64_t orc_mix64(uint64_t z);
void orc_seed_words(uint64_t seed, uint64_t out[3]);
void orc_signature(uint64_t key, const uint64_t sw[3], uint64_t *hi, uint64_t *lo);
uint64_t orc_fingerprint(uint64_t hi, uint64_t lo, const uint64_t sw[3], int32_t b);
uint32_t orc_shard_of(uint64_t hi, int32_t h);
void orc_edge(uint64_t hi, uint64_t lo, int32_t h, uint32_t l, int32_t sigma,
              uint32_t t, uint32_t v[3]);
void orc_edge_mwhc(uint64_t lo, uint32_t part, uint32_t t, uint32_t v[3]);

/* parameter math */
double orc_lambert_w0(double x);
int32_t orc_shard_bits_eps(double n, double eps, double alpha);
double orc_shard_bits_exact(double n, double eps, double alpha);
int32_t orc_dupmwhc_bits(double n, double c, double eta);
double orc_logdupfuse(double n, double c, double eta, double alpha, double beta);
double orc_dupfuse(double n, double c, double eta, double alpha, double beta);
void orc_geometry(uint32_t M, int32_t h, uint32_t c_num, uint32_t c_den,
                  int32_t sigma_override, orc_geom *g);
void orc_geometry_mwhc(uint32_t M, int32_t h, uint32_t c_num, uint32_t c_den,
                       orc_geom *g);

/* solvers on an explicit 3-hypergraph (edges e[3*i+0..2]) */
int32_t orc_peel(uint64_t nv, uint32_t m, const uint32_t *e, int32_t *round,
                 int8_t *side);
int32_t orc_core_lexmin(uint64_t nv, uint32_t k, const uint32_t *rows3,
                        const uint64_t *rhs, uint64_t *x);
int32_t orc_solve(uint64_t nv, uint32_t m, const uint32_t *e,
                  const uint64_t *rhs, uint64_t *w, uint32_t *core_edges);

/* whole construction and query */
int32_t orc_plan(const uint64_t *keys, uint64_t n, int32_t h, uint64_t seed,
                 uint32_t c_num, uint32_t c_den, int32_t sigma_override,
                 orc_geom *g, uint32_t *counts);
void orc_shard_ids(const uint64_t *keys, uint64_t n, int32_t h, uint64_t seed,
                   uint32_t *out);
int32_t orc_build(const uint64_t *keys, const uint64_t *values, uint64_t n,
                  int32_t b, int32_t is_filter, uint64_t seed, uint32_t tmax,
                  const orc_geom *g, const uint32_t *shards, uint32_t nshards,
                  uint32_t *t_out, uint64_t *w_out, orc_fail *rec,
                  uint32_t rec_cap, uint32_t *nrec);
void orc_pack(const uint64_t *w, uint64_t count, int32_t b, uint64_t *out);
uint64_t orc_unpack(const uint64_t *words, uint64_t i, int32_t b);
void orc_query(const uint64_t *keys, uint64_t n, uint64_t seed, int32_t b,
               int32_t is_filter, const orc_geom *g, const uint32_t *t_of_shard,
               const int32_t *slot_of_shard, const uint64_t *w, uint64_t *out);

#ifdef __cplusplus
}
#endif
#endif
