/*
 * vf.h -- C ABI of the MI355X (gfx950) library for epsilon-cost sharded
 * static functions (VFunc) and static filters (VFilter), after S. Vigna,
 * "epsilon-Cost Sharding: Scaling Hypergraph-Based Static Functions and
 * Filters to Trillions of Keys" (arXiv 2503.18397).
 *
 * Problems solved (section 3):
 *   Problem 1 (static function): given n keys and a b-bit value per key,
 *     store a structure that returns the value of every key; any value may
 *     be returned for other keys.
 *   Problem 2 (static filter): store a structure that answers "is x in the
 *     set" with no false negatives and false-positive rate 2^-b; it is a
 *     static function from each key to a b-bit fingerprint derived from its
 *     signature (sections 3.1 and 4.5).
 *
 * Method (section 4): keys are hashed once to a signature; the h highest
 * signature bits pick one of S = 2^h shards; every shard is a fuse
 * 3-hypergraph sized by the largest shard (no offsets), is peeled, the
 * unpeeled 2-core is solved by Gaussian elimination over GF(2), and values
 * are assigned in reverse peel order.  A query xors three cells.
 *
 * Conventions shared by every entry point:
 *   - Return value: VF_OK (0) or a negative VF_E* code.  Nothing is thrown
 *     across the ABI.  On error, outputs are left untouched unless stated.
 *   - Keys are uint64 words in DEVICE memory (HBM).  Values, workspace,
 *     structure and query outputs are DEVICE buffers too, allocated and
 *     owned by the caller; the library only borrows them.
 *   - All device work is enqueued on the caller's HIP stream `stream`.
 *     vf_build/vfilter_build synchronize that stream twice (after shard
 *     counting, and at the end to collect the failure record); queries do
 *     not synchronize.
 *   - Keys must be distinct for a VFunc unless equal keys carry equal
 *     values; a filter accepts duplicate keys.
 *   - A handle is a small host object that records pointers into the
 *     caller's structure buffer: keep that buffer alive and unmodified for
 *     as long as the handle is used.
 */
#ifndef VF_H
#define VF_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VF_OK 0
#define VF_EINVAL (-1)    /* bad argument (null pointer, b, eps, sizes)   */
#define VF_ENOSPC (-2)    /* workspace or structure buffer too small      */
#define VF_EFAIL (-3)     /* some shard failed every local seed           */
#define VF_EHIP (-4)      /* a HIP runtime call failed, or a build kernel
                             gave up on an internal wait (a bug)           */
#define VF_ECAPACITY (-5) /* a shard exceeded a fixed on-chip capacity of
                             this implementation (elimination window or
                             pivot log); the method itself did not fail    */
#define VF_ENOMEM (-6)    /* a host-side allocation of the library failed  */

/* Options.  vf_default_opts() fills the paper's defaults. */
typedef struct vf_opts {
  int32_t h;          /* shard bits; -1: from eps by eq. (logballsbins)   */
  int32_t sigma;      /* lg of the segment size; -1: by the size rule     */
  uint32_t c_num;     /* expansion factor c = c_num / c_den; 0: by rule   */
  uint32_t c_den;
  uint32_t tmax;      /* local seeds tried per shard, 1..255 (default 255) */
  double alpha;       /* Raab-Steger constant of eq. (ballsbins) (1.0)    */
  int32_t mwhc;       /* 1: MWHC 3-partite hypergraphs (section 4.1): three
                         parts of ceil(c M / 3) cells, c = 1.23 by default,
                         peel-only (an attempt that does not peel fails, kind
                         2); keys must be distinct.  0: fuse graphs. */
  uint32_t max_window; /* rows of the elimination window a build workgroup
                         keeps (rounded down to a multiple of 8, at least
                         8); a shard whose window would grow beyond it is
                         rebuilt by the second launch, which has a whole
                         CU's LDS.  0 (default): as many as the workgroup's
                         share of LDS holds.  The result never depends on
                         it. */
  uint32_t packed;    /* 1: store the cells as one bit string of b-bit fields
                         (cell i of the structure, or of an instance of a
                         batch, at bits [i b, i b + b) of little-endian
                         64-bit words), the bit-array storage of values of
                         any width (section 5); the build assembles byte
                         cells in the workspace and packs them at the end.
                         Queries read the packed fields; grouped queries
                         use the plain gathers.  0 (default): cells of 1, 2,
                         4 or 8 bytes. */
  int32_t small;      /* batches: 0 (default) the kernel vf_batch_tuning
                         chose for each size class, 1 the one-wavefront
                         kernel for every instance it fits, 2 never it;
                         the cells are the same either way. */
  uint32_t ring_cols; /* test option: columns the back-substitution keeps in
                         its LDS ring, a power of two from 64 to 2048, for
                         every shard with cells of at most 4 bytes whatever
                         its segment size (so that vertices beyond the ring
                         and batches wider than half of it occur); 0
                         (default): 2048, for segment sizes s with
                         3 s + 64 <= 2048.  The result never depends on it;
                         other values are VF_EINVAL. */
} vf_opts;

/* Sizes returned by vf_plan (upper bounds: the largest shard is known only
 * after hashing). */
typedef struct vf_sizes {
  uint64_t structure_bytes; /* cells + per-shard seeds + header padding */
  uint64_t workspace_bytes; /* scratch used only during the build       */
  int32_t h;                /* shard bits that will be used             */
  uint32_t shard_cap;       /* largest shard the sizes allow            */
} vf_sizes;

/* Read-only description of a built structure. */
typedef struct vf_info_t {
  int32_t is_filter, b, h;
  uint32_t S;             /* shards                                      */
  uint32_t M;             /* keys of the largest shard                   */
  uint32_t c_num, c_den;  /* expansion factor                            */
  int32_t sigma;          /* segment size 2^sigma                        */
  uint32_t l;             /* start segments per shard                    */
  uint64_t V;             /* vertices (cells) per shard = (l + 2) 2^sigma */
  uint64_t n;             /* keys                                         */
  uint64_t seed;
  uint32_t cell_bytes;    /* bytes per cell in device memory: 1, 2, 4, 8 */
  uint32_t failed_shards; /* shards with no successful local seed        */
  uint32_t n_failures;    /* failed attempts recorded                    */
  uint64_t space_bits;    /* S * V * b: the information the method stores */
  const void *cells;      /* device: S * V cells of cell_bytes           */
  const uint8_t *local_seeds; /* device: S bytes, 255 = shard failed     */
  /* Durations of the build's device phases, measured with HIP events on
   * the build stream: shard counting + scan, grouping keys by shard, and
   * the per-shard construction kernel. */
  float ms_count, ms_scatter, ms_build;
  /* Shards whose elimination window outgrew a build workgroup's share of a
   * CU's LDS and were rebuilt by a second launch with a whole CU's LDS
   * (same result, slower). */
  uint32_t relaunched_shards;
  int32_t mwhc;           /* 1: MWHC hypergraphs (sigma 0, l 1, V = 3 parts) */
  uint32_t packed;        /* 1: cells is a bit string of b-bit fields      */
} vf_info_t;

/* One failed construction attempt of one shard. */
typedef struct vf_failure {
  uint32_t shard;
  uint32_t attempt;    /* local seed t */
  uint32_t kind;       /* 1 = the 2-core system was inconsistent,
                          2 = an MWHC hypergraph did not peel        */
  uint32_t core_edges; /* edges left by peeling in that attempt  */
} vf_failure;

typedef struct vf_handle vf_handle;

/* A description of the calling thread's last VF_EHIP (the failing HIP
 * call and its error), or an empty string.  The text stays valid until the
 * thread's next failing call. */
const char *vf_last_error(void);

/* Paper defaults: h from eps with alpha = 1 (section 4), c and the segment
 * size by the size rule (section 4.2), tmax = 255. */
void vf_default_opts(vf_opts *o);

/* Sizes of the caller-allocated buffers for n keys of b bits (section 4:
 * S * V cells, V from the largest shard, bounded here by the Raab-Steger
 * maximum load with a safety margin).  Pure host; o may be NULL.
 * Errors: VF_EINVAL for b outside 1..64, eps <= 0 with o->h < 0, out NULL. */
int vf_plan(uint64_t n, int32_t b, double eps, int32_t is_filter,
            const vf_opts *o, vf_sizes *out);

/* Build a static function (Problem 1).
 *   keys      device, n uint64 keys
 *   values    device, n uint64 words of b bits (Problem 1): a value with a
 *             bit at or above b makes the call return VF_EINVAL before the
 *             structure is written (checked on the device, read at the
 *             call's first synchronization)
 *   b         1..64 value bits; cells are 1, 2, 4 or 8 bytes wide
 *   eps, o    sharding as in vf_plan; seed selects the hash functions
 *   workspace device scratch of at least vf_plan().workspace_bytes
 *   structure device buffer of at least vf_plan().structure_bytes
 *   handle    receives a new handle (also on VF_EFAIL, for vf_failures)
 * Errors: VF_EINVAL, VF_ENOSPC (buffers too small for the actual largest
 * shard), VF_EFAIL, VF_ECAPACITY, VF_ENOMEM, VF_EHIP. */
int vf_build(const uint64_t *keys, const uint64_t *values, uint64_t n,
             int32_t b, double eps, uint64_t seed, const vf_opts *o,
             void *workspace, uint64_t workspace_bytes, void *structure,
             uint64_t structure_bytes, hipStream_t stream, vf_handle **handle);

/* Query a static function (eq. (MWHC) with k = 3): out[i] = xor of the
 * three cells of keys[i]'s edge; out has cell_bytes per key (device).
 * Errors: VF_EINVAL (null handle/pointers, or a filter handle). */
int vf_query(const vf_handle *h, const uint64_t *keys, uint64_t n, void *out,
             hipStream_t stream);

/* Build a static filter (Problem 2) with b-bit fingerprints; arguments as
 * vf_build without values. */
int vfilter_build(const uint64_t *keys, uint64_t n, int32_t b, double eps,
                  uint64_t seed, const vf_opts *o, void *workspace,
                  uint64_t workspace_bytes, void *structure,
                  uint64_t structure_bytes, hipStream_t stream,
                  vf_handle **handle);

/* Build a static filter from keys in host memory (pinned memory gives the
 * full PCIe rate), as vfilter_build would from the same keys on the device.
 * The keys are copied in chunks of `chunk` keys (0: one copy) on a stream
 * of the library's that overlaps each copy with the shard counting of the
 * previous chunks (section 4: one pass assigns keys to shards by their
 * signatures); the device copy lives in the workspace, which must hold
 * vf_plan().workspace_bytes plus 8 n bytes rounded up to 256.  The call
 * returns once every chunk has been copied (keys may then be reused).
 * Errors: as vfilter_build. */
int vfilter_build_host(const uint64_t *keys, uint64_t n, int32_t b, double eps,
                       uint64_t seed, const vf_opts *o, uint64_t chunk,
                       void *workspace, uint64_t workspace_bytes,
                       void *structure, uint64_t structure_bytes,
                       hipStream_t stream, vf_handle **handle);

/* The sharded build in three calls, so that its device work can be
 * captured into a HIP graph and replayed (for instance on new keys written
 * into the same buffers).  Every shard is sized for a bound on the largest
 * shard fixed in advance (max_shard; 0: the bound vf_plan sizes buffers
 * for, which a larger max_shard may not exceed) instead of the measured
 * largest shard (section 4 sizes every shard
 * by the largest one; a bound at least as large gives every shard room, at
 * the cost of the gap), so no step waits for the host.  The cells, seeds
 * and failure record are those vf_build / vfilter_build give for the same
 * keys when their largest shard is max_shard.
 *   vf_build_prepare  host only: plans layout and geometry, sets kernel
 *                     attributes; *handle answers no query until a
 *                     vf_build_finish reports a built structure.  Errors:
 *                     VF_EINVAL (as vf_build, or n = 0), VF_ENOSPC,
 *                     VF_ECAPACITY, VF_ENOMEM, VF_EHIP.
 *   vf_build_launch   enqueues counting, grouping, checks and the build on
 *                     stream: kernels only (no allocation, copy from the
 *                     host or wait), so it may run under stream capture.
 *                     keys (and values for a function, is_filter = 0) are
 *                     n device words read when the work runs.  A value with
 *                     a bit at or above b, or a shard above the bound, makes
 *                     every build kernel return at once (the structure
 *                     keeps what it held).  Errors: VF_EINVAL, VF_EHIP.
 *   vf_build_finish   once stream has run the launch (or a graph holding
 *                     it): reads the checks, the failure record and the
 *                     local seeds into the handle (synchronizes stream).
 *                     VF_EINVAL: a value was too wide; VF_ENOSPC: a shard
 *                     exceeded the bound (vf_last_error gives both sizes);
 *                     the handle is unchanged in both cases.  Otherwise as
 *                     vf_build (VF_OK, VF_EFAIL, VF_ECAPACITY, VF_EHIP).
 * workspace and structure (vf_plan sizes, caller-owned) stay with the
 * handle; launches of one handle that overlap on the device race. */
int vf_build_prepare(uint64_t n, uint32_t max_shard, int32_t b, double eps,
                     int32_t is_filter, uint64_t seed, const vf_opts *o,
                     void *workspace, uint64_t workspace_bytes,
                     void *structure, uint64_t structure_bytes,
                     vf_handle **handle);
int vf_build_launch(vf_handle *h, const uint64_t *keys, const uint64_t *values,
                    hipStream_t stream);
int vf_build_finish(vf_handle *h, hipStream_t stream);

/* One request of vf_query_multi: n keys (device) asked of structure h, the
 * answers written to out (device) exactly as vf_query (a function) or
 * vfilter_contains (a filter) would write them. */
typedef struct vf_query_req {
  const vf_handle *h;
  const uint64_t *keys;
  uint64_t n;
  void *out;
} vf_query_req;

/* Answers count query requests, each against its own structure (functions
 * and filters of any geometry, byte or packed cells, not batches), with one
 * kernel launch per VF_QUERY_MULTI_MAX requests: the per-key work of
 * vf_query and vfilter_contains (eq. (MWHC) per shard, sections 3 and 4.5)
 * over the concatenation of the requests' keys, without copying them.
 * Serving loops merge concurrent small query batches this way.  reqs is a
 * host array; no allocation, no wait, no copy from the host (the requests
 * travel as kernel arguments).  Errors: VF_EINVAL (reqs NULL with count >
 * 0, a NULL or batch handle, NULL keys or out with n > 0), VF_EHIP. */
#define VF_QUERY_MULTI_MAX 16
int vf_query_multi(const vf_query_req *reqs, uint32_t count, hipStream_t stream);

/* Filter query: out[i] = 1 if keys[i] may be in the set, 0 if it is not
 * (sections 3.1 and 4.5).  out is n bytes of device memory.
 * Errors: VF_EINVAL (null handle/pointers, or a function handle). */
int vfilter_contains(const vf_handle *h, const uint64_t *keys, uint64_t n,
                     uint8_t *out, hipStream_t stream);

/* ---- Queries grouped by shard --------------------------------------
 * The same answers as vf_query / vfilter_contains, computed another way: a
 * key's shard is a function of its signature alone (section 4, no offsets
 * are stored), so the queries can first be grouped by shard with a
 * counting sort, and each shard's queries answered together while its
 * cells sit on chip.  The three probes of a query then cost no memory
 * traffic; the grouping costs streaming passes over the keys.  Queries are
 * taken in chunks of up to 2^26 keys; each chunk is counted, scattered
 * into the workspace grouped by shard (each key hashed once, and stored as
 * its edge, fingerprint and position where these fit a word, else as the
 * key and its index) and answered, and the answers are moved to the keys'
 * own positions in out.  A
 * structure whose shards' cells do not fit in LDS (more than about 160 KB
 * per shard) is answered by the plain gathers of vf_query instead.
 * Grouping pays when a chunk holds many queries per shard (thousands at
 * 2^16-key shards); with very many shards the plain query is faster. */

/* Workspace that answers n keys of handle h in one chunk: per-shard
 * counters, offsets and per-segment tables, plus 12 bytes and one answer
 * (cell_bytes, 1 for a filter) per key of a chunk (up to 2^26 keys).
 * Errors: VF_EINVAL (null or batch handle, bytes NULL). */
int vf_query_grouped_bytes(const vf_handle *h, uint64_t n, uint64_t *bytes);

/* vf_query with the queries grouped by shard.
 *   keys       device, n uint64 keys (read only)
 *   out        device, n answers of cell_bytes each, as vf_query writes them
 *   workspace  device scratch of workspace_bytes, 8-byte aligned (keys
 *              too); any size from the per-shard part plus one key works
 *              (smaller chunks are slower), vf_query_grouped_bytes(h, n)
 *              gives a single chunk.
 *              Its contents are dead once the stream passes the call; two
 *              calls in flight at once need two workspaces.
 * Errors: VF_EINVAL (null handle/pointers, a filter or batch handle, keys
 * or workspace not 8-byte aligned), VF_ENOSPC (workspace below the
 * per-shard part plus one key), VF_EHIP. */
int vf_query_grouped(const vf_handle *h, const uint64_t *keys, uint64_t n, void *out,
                     void *workspace, uint64_t workspace_bytes, hipStream_t stream);

/* vfilter_contains with the queries grouped by shard; arguments and errors
 * as vf_query_grouped, out is n bytes (1 = may be in the set). */
int vfilter_contains_grouped(const vf_handle *h, const uint64_t *keys, uint64_t n, uint8_t *out,
                             void *workspace, uint64_t workspace_bytes, hipStream_t stream);

/* vfilter_contains_grouped for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same answers, with the workspace taken from a static
 * 64 MiB device array of the library instead of an argument.  No device or
 * host memory is allocated by the call (the array's address is looked up
 * once per device, on the first call with that device current).
 *   keys, n, out, stream  as vfilter_contains_grouped; any n (queries are
 *                         taken in chunks that fit the array)
 * Every call on one GPU shares that GPU's array: calls in flight on the
 * same GPU at the same time (other streams, other threads) race and give
 * wrong answers; serialize them.  Nothing must start at zero in the array
 * (each call initializes what it reads).
 * Errors: VF_EINVAL (null handle/pointers, a function or batch handle,
 * keys not 8-byte aligned), VF_ENOSPC (the structure's per-shard tables
 * alone exceed the array: more than about 2^21 shards), VF_EHIP. */
int vfilter_contains_grouped_noalloc(const vf_handle *h, const uint64_t *keys, uint64_t n,
                                     uint8_t *out, hipStream_t stream);

/* Describe a handle.  Errors: VF_EINVAL. */
int vf_info(const vf_handle *h, vf_info_t *out);

/* Copy up to cap failure records, sorted by (shard, attempt), into out
 * (host memory); *count receives the total number recorded.  The record of
 * the local seeds tried per shard (section 3.2: HEM keeps a local seed per
 * shard; here every failed attempt is listed).  Errors: VF_EINVAL. */
int vf_failures(const vf_handle *h, vf_failure *out, uint32_t cap,
                uint32_t *count);

/* ---- Batches of independent static functions -------------------------
 * Many unsharded functions (Problem 1, h = 0) of uneven sizes and value
 * widths built by one persistent launch per cell width (1, 2, 4, 8 bytes)
 * instead of one build per function.  Instance i is exactly the structure
 * vf_build would give for its keys, values, b_i and the batch seed with
 * h = 0: geometry by the size rule of section 4.2 for M = n_i, local seed,
 * failure record (shard field = instance index) and cells. */

/* One instance of a batch (host copy). */
typedef struct vf_batch_item_t {
  uint64_t n;             /* keys                                        */
  int32_t b;              /* value bits                                  */
  uint32_t c_num, c_den;  /* expansion factor                            */
  int32_t sigma;          /* segment size 2^sigma                        */
  uint32_t l;             /* start segments                              */
  uint64_t V;             /* cells = (l + 2) 2^sigma                     */
  uint32_t cell_bytes;    /* 1, 2, 4 or 8                                */
  uint32_t local_seed;    /* successful local seed, 255 = failed         */
  const void *cells;      /* device: V cells of cell_bytes, or with packed
                             a bit string of V b-bit fields              */
  uint32_t packed;        /* 1: packed cells                             */
} vf_batch_item_t;

/* Buffer sizes for a batch of count instances with n[i] keys of b[i] bits
 * (host arrays).  out->h is 0, out->shard_cap the largest n[i].
 * Errors: VF_EINVAL (count 0, null arrays, b outside 1..64), VF_ECAPACITY
 * (an instance too large for one graph of 2^21 cells). */
int vf_batch_plan(uint64_t count, const uint64_t *n, const int32_t *b,
                  const vf_opts *o, vf_sizes *out);

/* Build a batch.
 *   keys, values device; the keys (and values) of instance i follow those
 *                of instance i - 1 (n[0] + ... + n[count-1] words each);
 *                a value of instance i has b[i] bits: a higher bit makes
 *                the call return VF_EINVAL before the structure is written
 *   count, n, b  instances and their sizes and value bits (host arrays)
 *   seed, o      hash seed shared by all instances; o->h is ignored
 *   workspace, structure  device buffers of at least vf_batch_plan() bytes
 *   handle       receives a batch handle (also on VF_EFAIL)
 * The keys are used in place (no grouping pass); every launch is enqueued
 * on stream; the call synchronizes once after checking the values and once
 * at the end to read the failure record.  Errors: VF_EINVAL, VF_ENOSPC,
 * VF_EFAIL (an instance failed all local seeds), VF_ECAPACITY, VF_ENOMEM,
 * VF_EHIP. */
int vf_batch_build(const uint64_t *keys, const uint64_t *values, uint64_t count,
                   const uint64_t *n, const int32_t *b, uint64_t seed,
                   const vf_opts *o, void *workspace, uint64_t workspace_bytes,
                   void *structure, uint64_t structure_bytes,
                   hipStream_t stream, vf_handle **handle);

/* The same build in three calls, so that its device work can be captured
 * into a HIP graph and replayed (for instance on new keys written into the
 * same buffers).  The cells, seeds and failure record are those
 * vf_batch_build gives for the same input.
 *   vf_batch_prepare  plans the batch on the host and copies its instance
 *                     descriptors and launch lists into workspace and
 *                     structure (synchronizes stream once).  *handle
 *                     receives a batch handle that answers no query until
 *                     a vf_batch_finish has reported a built structure.
 *                     Uses the device's kernel choice as vf_batch_tuning
 *                     describes it at that moment (it does not tune).
 *   vf_batch_launch   enqueues the build on stream and nothing else: no
 *                     allocation, no copy from the host, no wait, so it may
 *                     run under stream capture.  The values are checked
 *                     on the device first; a value with a bit at or above
 *                     its b makes every build kernel return at once, and
 *                     the structure keeps what it held.
 *   vf_batch_finish   once stream has run the launch (or a graph holding
 *                     it): reads the check, the failure record and the
 *                     local seeds into the handle (synchronizes stream).
 *                     VF_EINVAL: a value was too wide (handle unchanged);
 *                     otherwise what vf_batch_build returns.
 * The handle refers to workspace and structure (caller-owned, kept for the
 * handle's life); keys and values are read when the launched work runs.
 * Launches of one handle that overlap on the device race on its buffers.
 * Errors of prepare as vf_batch_build's before any device work; of launch:
 * VF_EINVAL (not a prepared handle, null keys or values), VF_EHIP. */
int vf_batch_prepare(uint64_t count, const uint64_t *n, const int32_t *b,
                     uint64_t seed, const vf_opts *o, void *workspace,
                     uint64_t workspace_bytes, void *structure,
                     uint64_t structure_bytes, hipStream_t stream,
                     vf_handle **handle);
int vf_batch_launch(vf_handle *h, const uint64_t *keys, const uint64_t *values,
                    hipStream_t stream);
int vf_batch_finish(vf_handle *h, hipStream_t stream);

/* Query a batch: out[i] = value of keys[i] in instance inst[i] (eq. (MWHC)
 * in that instance), as a uint64 word.  inst, keys and out are device
 * arrays of nq entries; an instance index >= count gives all ones.
 * Errors: VF_EINVAL (null pointers, or a handle that is not a batch). */
int vf_batch_query(const vf_handle *h, const uint32_t *inst, const uint64_t *keys,
                   uint64_t nq, uint64_t *out, hipStream_t stream);

/* How batches are built on the current device.  Instances of at most 128
 * keys and 256 cells can be built by a one-wavefront kernel that keeps the
 * whole instance on chip (edges in registers, peeling and values in LDS, a
 * dense elimination of the 2-core in registers; section 4.2 solves small
 * sizes by Gaussian elimination) instead of the peel + band kernel; both
 * give the same cells.  The first vf_batch_build on a device that has at
 * least 256 such instances (one-byte cells) in a size class times both
 * kernels on up to 2048 of them per class and keeps the faster, and tunes
 * the grid of the one-wavefront kernel; until then the one-wavefront
 * kernel builds every instance that fits it.  Errors: VF_EINVAL. */
typedef struct vf_batch_tuning_t {
  int32_t tuned;            /* 1 once the classes have been measured       */
  uint32_t max_keys[4];     /* size classes: up to 16, 32, 64, 128 keys    */
  int32_t use_small[4];     /* 1: the one-wavefront kernel builds the class */
  float ms_small[4];        /* time of the sampled instances, each kernel  */
  float ms_band[4];
  uint32_t sampled[4];      /* instances timed per class                   */
  uint32_t small_groups_per_cu; /* workgroups per CU of the small kernel   */
} vf_batch_tuning_t;
int vf_batch_tuning(vf_batch_tuning_t *out);

/* Describe instance i of a batch.  Errors: VF_EINVAL (not a batch handle,
 * i out of range, out NULL). */
int vf_batch_item(const vf_handle *h, uint64_t i, vf_batch_item_t *out);

/* Stage clocks of the shard build kernel, for profiling.  With reset != 0
 * the counters are cleared; otherwise VF_STAGE_CLOCK_WORDS counters are
 * copied to out (host, at least that many words): for each of the first
 * 4096 build workgroups 32 counters of 100 MHz wall-clock ticks and counts
 * (the peeling wavefront per item, the elimination of a 2-core, the
 * assignment, the workgroup's first item and whole run, and per 32-column
 * word the phases of the searching and of an emitting wavefront).  Only a
 * library built with stage clocks keeps them (build.py --stage-clocks
 * writes libvf_stages.so); the plain library returns VF_EINVAL.
 * Errors: VF_EINVAL (no stage clocks, out NULL or too small), VF_EHIP. */
#define VF_STAGE_CLOCK_WORDS (4096 * 32)
int vf_stage_clocks(uint64_t *out, uint64_t words, int32_t reset);

/* Free the host-side handle only; the caller still owns every buffer. */
void vf_free(vf_handle *h);

#ifdef __cplusplus
}
#endif
#endif
