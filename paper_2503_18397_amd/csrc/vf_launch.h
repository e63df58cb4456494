// Internal interface between the host orchestration (vf_api.cpp) and the
// gfx950 kernels (vf_device.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vfk {

// Per-structure constants every kernel needs.
struct Geo {
  uint64_t khi, klo, kfp;  // seed words of the two signature halves and fingerprint
  uint64_t V;              // cells per shard
  uint64_t vmask;          // low-b-bit mask of values and fingerprints
  uint32_t h;              // shard bits
  uint32_t S;              // shards
  uint32_t l;              // start segments per shard
  uint32_t sigma;          // lg segment size
  uint32_t b;              // value / fingerprint bits
  uint32_t is_filter;
  uint32_t mwhc;           // 1: MWHC 3-partite hypergraph (peel-only)
  uint32_t part;           // MWHC: vertices per part
};

// One instance of a batch: an unsharded structure with its own keys,
// geometry and cells (cell_off bytes into the batch's cell area).
struct BatchItem {
  uint64_t key_off;   // first key (and value) of the instance
  uint64_t cell_off;  // byte offset of its cells
  uint64_t V;         // cells
  uint64_t vmask;     // low-b-bit mask
  uint32_t n;         // keys
  uint32_t l, sigma, b;
  uint32_t cell_bytes;
  uint32_t c_num, c_den;
  uint32_t pad;
};
static_assert(sizeof(BatchItem) == 64, "BatchItem layout");

struct FailRec {
  uint32_t shard, attempt, kind, core_edges;
};

// Counters shared by all build workgroups.
enum : uint32_t {
  kWorkNext = 0,       // next work item
  kWorkFails = 1,      // failure records written
  kWorkStatus = 2,     // kStatus* bits
  kWorkCap = 3,        // items appended to the overflow list by this launch
  kWorkRelaunch = 4,   // items appended to overflow lists by all launches
  kWorkWords = 5
};
enum : uint32_t {
  kStatusCapacity = 1u,  // a shard outgrew a fixed on-chip capacity
  kStatusStalled = 2u    // a wait inside a build workgroup ran out (internal error)
};

struct BuildArgs {
  Geo G;
  const uint64_t *bkeys;    // keys grouped by shard
  const uint64_t *bvals;    // values grouped by shard (function only)
  const uint64_t *offsets;  // S + 1 shard starts
  void *cells;              // S * V cells of cell_bytes
  uint8_t *tseed;           // S local seeds (255: failed)
  uint8_t *scratch;         // per-workgroup scratch, scratch_stride bytes each
  uint64_t scratch_stride;
  uint32_t *work;           // kWorkWords counters
  FailRec *fails;
  uint32_t fail_cap;
  uint32_t M;               // keys in the largest shard
  uint32_t tmax;            // local seeds per shard
  uint32_t wmax;            // elimination window slots
  uint32_t logcap;          // pivot log words per workgroup
  uint32_t lds_bytes;       // dynamic LDS of the launch
  uint32_t cell_bytes;      // 1, 2, 4 or 8
  // Shards to build: all (list == nullptr, taken in order) or the nlist
  // (shard, first local seed) pairs of list.
  const uint32_t *list;
  uint32_t nlist;
  const uint32_t *nlist_dev;  // if set, the list length is read from here
  // Shards whose elimination window outgrew the LDS of this launch are
  // appended here as (shard, local seed) pairs for a launch with more LDS;
  // nullptr: such shards fail with kStatusCapacity.
  uint32_t *overflow;
  // Batch mode: work item j is instance j of items (G then only supplies
  // the seed words and the function/filter kind); nullptr: item j is shard
  // j of one sharded structure.
  const BatchItem *items;
  // Largest cells and segment count over all items (scratch layout).
  uint64_t scr_V;
  uint32_t scr_l;
  // Test builds: columns of the back-substitution's ring (0: kRingCols).
  uint32_t ring_cols;
  // If set and nonzero when the kernel starts (a failed value check earlier
  // on the stream), the kernel returns without writing anything.
  const uint32_t *abort;
};

constexpr uint32_t kLdsBudget = 160 * 1024;  // LDS of one CU
// Bytes at the end of a build workgroup's dynamic LDS that hold the control
// blocks shared by its wavefronts and the back-substitution columns.
constexpr uint32_t kLdsTail = 2048;
// Columns of the back-substitution's LDS ring (cells of at most 4 bytes).
constexpr uint32_t kRingCols = 2048;
// Threads of a build workgroup: three wavefronts eliminate (one searches
// the pivots, two emit the pivot rows), one peels the next item and one
// assigns the cells of solved items.
constexpr uint32_t kBuildThreads = 320;

uint64_t build_scratch_bytes(uint32_t M, uint64_t V, uint32_t l, uint32_t logcap);
uint32_t window_slots(uint32_t sigma, uint32_t lds_bytes);

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
// Packs count cells of cell_bytes each (b bits used) into a little-endian
// bit string of 64-bit words (cell i at bits [i b, i b + b)).
hipError_t launch_pack(const void *in, uint32_t cell_bytes, uint64_t count, uint32_t b,
                       uint64_t *out, hipStream_t s);
// The same, returning at once if abort is set and nonzero.
hipError_t launch_pack_checked(const void *in, uint32_t cell_bytes, uint64_t count, uint32_t b,
                               uint64_t *out, const uint32_t *abort, hipStream_t s);
// Sets bit 1 of meta[1] if meta[0] (the largest shard) exceeds cap.
hipError_t launch_check_bound(uint32_t *meta, uint32_t cap, hipStream_t s);
// The same per instance of a batch: src offsets into in, dst into out.
hipError_t launch_pack_batch(const BatchItem *src, const BatchItem *dst, uint64_t count,
                             const uint8_t *in, uint8_t *out, const uint32_t *abort,
                             hipStream_t s);
// Sets bit 0 of *flag if a value has a bit at or above b (per instance for a
// batch); the flag must be cleared beforehand.
hipError_t launch_check_values(const uint64_t *vals, uint64_t n, uint32_t b, uint32_t *flag,
                              hipStream_t s);
hipError_t launch_check_batch_values(const BatchItem *items, uint64_t count, const uint64_t *vals,
                                    uint32_t *flag, hipStream_t s);
hipError_t launch_count(const uint64_t *keys, uint64_t n, uint64_t khi, uint32_t h,
                        uint32_t S, uint32_t *counts, int ncu, hipStream_t s);
hipError_t launch_scan(const uint32_t *counts, uint32_t S, uint64_t *offsets,
                       uint64_t *cursor, uint32_t *max_out, hipStream_t s,
                       uint32_t *clear = nullptr);
hipError_t launch_order(const uint32_t *counts, uint32_t S, uint32_t M, uint32_t *list,
                        hipStream_t s);
hipError_t launch_scatter(const uint64_t *keys, const uint64_t *vals, uint64_t n,
                          uint64_t khi, uint32_t h, uint32_t S, uint64_t *cursor,
                          uint64_t *bkeys, uint64_t *bvals, uint32_t *bidx, int ncu,
                          hipStream_t s);
hipError_t launch_build(const BuildArgs &a, int nwg, hipStream_t s);
// Wavefronts (instances in flight) per workgroup of the one-wavefront kernel.
constexpr uint32_t kSmallWavesPerGroup = 4;
// Instances small enough for the one-wavefront kernel (batches only).
bool small_instance(uint64_t n, uint64_t V);
// The one-wavefront build of the (instance, first local seed) pairs of
// a.list (a.items, a.cells, a.tseed, a.fails, a.work as for launch_build).
hipError_t launch_small(const BuildArgs &a, int nwg, hipStream_t s);

// Stage clocks of k_build (a build with -DVF_STAGE_CLOCKS): kClkSlots
// counters per workgroup for the first kClkWGs workgroups.
constexpr uint32_t kClkWGs = 4096, kClkSlots = 32;
enum : uint32_t {
  kClkPeel = 0,     // ticks, calls: peeling wavefront, per item's attempts
  kClkBand = 2,     // ticks, calls: elimination of a 2-core
  kClkAssign = 4,   // ticks, calls: back-substitution and assignment
  kClkFirst = 6,    // ticks: the workgroup's first item (all wavefronts)
  kClkTotal = 7,    // ticks: the whole workgroup
  kClkSearch = 8,   // 7 slots, per 32-column word of the searching wavefront:
                    // returned slots + entering rows, compaction, pivot
                    // search, row updates, flags, barrier; words
  kClkBackSub = 15, // ticks: back-substitutions (within kClkAssign)
  kClkEmit = 16,    // the same 7 slots for emitting wavefront 1 (emission,
                    // wait for the batch + row updates in slots 1 and 2)
  kClkElimEnd = 23, // ticks from the start to the end of the last elimination
  kClkPeelPhases = 24  // 8 slots, per attempt's peel: edges + cleared state,
                       // incidence, first frontier, rounds, 2-core grouping,
                       // duplicate-row check; attempts; rounds
};
// Copies kClkWGs * kClkSlots counters to out (host), or clears them;
// hipErrorNotSupported without -DVF_STAGE_CLOCKS.
hipError_t stage_clocks(uint64_t *out, int reset);
// Sets the kernel attributes launch_build needs for a's shape on the
// current device (launch_build sets them too when they are missing).
hipError_t prepare_build(const BuildArgs &a);
// The allocation-free grouped query's workspace: a device array of
// kNoAllocScratchBytes per device; *ptr receives its address on the current
// device (looked up once per device).
constexpr uint64_t kNoAllocScratchBytes = 64ull << 20;
hipError_t noalloc_scratch(void **ptr, uint64_t *bytes);

// Build workgroups that can be resident on one CU at once (registers and
// LDS); 0 if the runtime cannot tell.
int build_blocks_per_cu(uint32_t cell_bytes, uint32_t wmax, uint32_t lds_bytes);
// Requests of one combined query launch: request r answers the keys of
// combined indices [start[r], start[r + 1]) against its own structure.
struct MultiReq {
  Geo G;
  const void *cells;
  const uint8_t *tseed;
  const uint64_t *keys;
  void *out;
  uint32_t cell_bytes;  // answer width of a function (1, 2, 4, 8)
  uint32_t packed;      // cells are a bit string of b-bit fields
};
constexpr uint32_t kMultiMax = 16;  // a power of two
struct MultiArgs {
  uint64_t start[kMultiMax + 1];
  MultiReq req[kMultiMax];
  uint32_t count;
};
hipError_t launch_query_multi(const MultiArgs &a, int ncu, hipStream_t s);
hipError_t launch_query_batch(const Geo &G, const BatchItem *items, uint64_t count,
                              const uint8_t *cells, const uint8_t *tseed, const uint32_t *inst,
                              const uint64_t *keys, uint64_t n, uint64_t *out, int ncu,
                              hipStream_t s,
                              bool packed);
hipError_t launch_query(const Geo &G, const void *cells, uint32_t cell_bytes,
                        const uint8_t *tseed, const uint64_t *keys, uint64_t n,
                        void *out, int ncu, hipStream_t s, bool packed = false);
// Keys of a query chunk (n < 2^32) grouped by shard, one reservation per
// shard and segment (S <= 4096): rows is scratch of group_rows_words(S)
// words, totals (zero on entry, zero again on return) and cursor of S
// words, meta of 4; offsets gets S + 1 shard starts, bkeys / bidx the keys
// and their indices.
bool group_rows_fit(uint32_t S);
uint64_t group_rows_words(uint32_t S);
// The two passes of launch_group_rows on their own (a build scans in
// between and reads the largest shard); bidx and starts may be null.
hipError_t launch_count_rows(const uint64_t *keys, uint64_t n, uint64_t khi, uint32_t h,
                             uint32_t S, uint32_t *rows, uint32_t *totals, hipStream_t s);
hipError_t launch_scatter_rows(const uint64_t *keys, uint64_t n, uint64_t khi, uint32_t h,
                               uint32_t S, const uint32_t *rows, uint64_t *cursor,
                               uint64_t *bkeys, uint32_t *bidx, uint32_t *starts, hipStream_t s,
                               int mode = 0, const Geo *G = nullptr,
                               const uint8_t *tseed = nullptr, uint32_t vb = 0);
// Whether the queries of a structure of geometry G and S shards can be
// grouped hashed (mode 1: three vertices of vb bits and the fingerprint in a
// word; mode 2, chunks of n keys: segment, offsets, fingerprint and the
// position in a word, *vb bits for the segment; see k_scatter_rows).
bool pack_fits(const Geo &G, uint32_t S, uint32_t *vb);
bool pack_compact_fits(const Geo &G, uint32_t S, uint64_t n, uint32_t *vb);
hipError_t launch_group_rows(const uint64_t *keys, uint64_t n, uint64_t khi, uint32_t h,
                             uint32_t S, uint32_t *rows, uint32_t *totals, uint64_t *offsets,
                             uint64_t *cursor, uint32_t *meta, uint64_t *bkeys, uint32_t *bidx,
                             uint32_t *starts, hipStream_t s, int mode = 0,
                             const Geo *G = nullptr, const uint8_t *tseed = nullptr,
                             uint32_t vb = 0);
// Answers of a chunk of n keys in grouped order (ans, ob bytes each) moved
// to out[bidx] (or, with bwords, to the positions in the grouped words of
// mode 2): rows and starts (group_rows_words(S) words each) from
// launch_group_rows.  place_fits tells whether a segment's window fits LDS.
bool place_fits(uint32_t S, uint64_t n, uint32_t ob);
hipError_t launch_place_rows(const uint32_t *rows, const uint32_t *starts, uint32_t S,
                             uint64_t n, uint32_t ob, const void *ans, const uint32_t *bidx,
                             const uint64_t *bwords, void *out, hipStream_t s);
// Grouped query: off (S + 1 offsets), bkeys and bidx from launch_scatter or
// launch_group_rows (bkeys holding hashed queries in mode 1 or 2, see
// k_scatter_rows); answers go to out[bidx], or with ans to ans in grouped
// order (then bidx is not read; mode 2 needs ans).
// LDS bytes of one shard's cells, 0 when they do not fit (or are not
// 16-byte aligned): then the grouped query is not launched.
uint32_t query_grouped_lds_bytes(const Geo &G, const void *cells, uint32_t cell_bytes);
hipError_t launch_query_grouped(const Geo &G, const void *cells, uint32_t cell_bytes,
                                const uint8_t *tseed, const uint64_t *off, const uint64_t *bkeys,
                                const uint32_t *bidx, void *out, void *ans, uint32_t vb,
                                int mode, int ncu, hipStream_t s);

}  // namespace vfk
