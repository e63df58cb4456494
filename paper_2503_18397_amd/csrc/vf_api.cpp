// Host orchestration behind the C ABI of include/vf.h: parameter math
// (section 4: eq. (logballsbins) for the shard bits; section 4.2 for the
// expansion factor and segment size), buffer carving, kernel launches and
// the failure record.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "vf.h"
#include "vf_launch.h"

namespace {

constexpr uint32_t kMagic = 0x56465531u;  // "VFU1"
constexpr uint64_t kGoldenGamma = 0x9e3779b97f4a7c15ull;
constexpr uint32_t kMaxShardBits = 24;
constexpr uint64_t kMaxCells = (1ull << 21) - 1;  // packed edges hold 21-bit vertices

uint64_t splitmix_finalize(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// The three seed words: consecutive SplitMix64 outputs from the user seed.
void seed_words(uint64_t seed, uint64_t w[3]) {
  uint64_t st = seed;
  for (int i = 0; i < 3; i++) {
    st += kGoldenGamma;
    w[i] = splitmix_finalize(st);
  }
}

// eq. (logballsbins): floor(lg x - lg ln x), x = n eps^2 / (2 alpha^2); no
// sharding when x <= e.
int32_t shard_bits_from_eps(uint64_t n, double eps, double alpha) {
  double x = (double)n * eps * eps / (2.0 * alpha * alpha);
  if (!(x > 2.718281828459045)) return 0;
  double hb = std::floor(std::log2(x) - std::log2(std::log(x)));
  if (hb < 0) hb = 0;
  if (hb > kMaxShardBits) hb = kMaxShardBits;
  return (int32_t)hb;
}

struct Geometry {
  uint32_t M, c_num, c_den, l;
  int32_t sigma;
  uint64_t V;
  uint32_t mwhc = 0, part = 0;  // MWHC: 3 parts of `part` vertices
};

// Section 4.1: MWHC 3-partite hypergraphs, c = 1.23 unless given, three
// parts of ceil(c M / 3) vertices (sigma 0 and l 1 are placeholders).
Geometry geometry_mwhc(uint32_t M, uint32_t cn, uint32_t cd) {
  if (cn == 0 || cd == 0) {
    cn = 123;
    cd = 100;
  }
  const uint64_t den = 3ull * cd;
  uint64_t part = ((uint64_t)cn * M + den - 1) / den;
  if (part == 0) part = 1;
  Geometry g;
  g.M = M;
  g.c_num = cn;
  g.c_den = cd;
  g.l = 1;
  g.sigma = 0;
  g.V = 3 * part;
  g.mwhc = 1;
  g.part = (uint32_t)std::min<uint64_t>(part, 0xFFFFFFFFull);
  return g;
}

// Section 4.2: c = 1.105 with lg s from eq. (nln) for shards of at least
// 800 000 keys, c = 1.125 with lg s from eq. (ln) for a single large
// unsharded graph.  Below 800 000 keys the paper keeps c = 1.12 and solves
// the unpeeled part by Gaussian elimination without fixing a segment size;
// sized by simulation (section 4), c = 1.12 builds while the middle segments
// carry at most about 0.93 equations per vertex and hold at least 2^8
// vertices, so a shard of m keys takes lg s = min(8, floor(lg m) - 2) for
// 64 <= m < 2^16 and lg s = 9 for 2^16 <= m < 800 000 (expected duplicate
// edges m / (2 c s^2) of 0.11 at 2^16 keys instead of 0.45), and
// c = max(1.12, 1.075 + 2 s / m) in thousandths rounded up (1.12 from
// 11 378 keys up).  lg s <= 9 is a capacity of the elimination (its LDS
// window spans three segments).
// Graphs of fewer than 64 keys are one block of three segments with
// s = 2^ceil(lg((m + 1) / 2)), c = 3 s / m.
// ell = max(1, ceil(c M / s) - 2) start segments, V = (ell + 2) s cells.
Geometry geometry(uint32_t M, int32_t h, uint32_t cn, uint32_t cd, int32_t sigma_ovr) {
  const bool large = M >= 800000u;
  int32_t sg;
  if (sigma_ovr >= 0) {
    sg = sigma_ovr;
  } else if (large && h > 0) {
    const double lm = std::log((double)M);
    sg = (int32_t)std::floor(0.41 * lm * std::log(lm) - 3.0);
  } else if (large) {
    sg = (int32_t)std::floor(std::log((double)M) / std::log(3.33) + 2.25);
  } else if (M < 64u) {
    sg = 0;
    while ((2ull << sg) < (uint64_t)M + 1) sg++;
  } else if (M >= 65536u) {
    sg = 9;
  } else {
    const int32_t lg = 31 - __builtin_clz(M);
    sg = std::min(lg - 2, 8);
  }
  sg = std::min(std::max(sg, 0), 20);
  if (cn == 0 || cd == 0) {
    if (large && h > 0) { cn = 1105; cd = 1000; }
    else if (large) { cn = 1125; cd = 1000; }
    else if (M < 64u) {
      int32_t st = 0;
      while ((2ull << st) < (uint64_t)M + 1) st++;
      cn = 3u << st;
      cd = M ? M : 1u;
    } else {
      const uint64_t x = 1075 + ((2000ull << sg) + M - 1) / M;
      cn = (uint32_t)std::max<uint64_t>(x, 1120);
      cd = 1000;
    }
  }
  const uint64_t den = (uint64_t)cd << sg;
  const uint64_t q = ((uint64_t)cn * M + den - 1) / den;
  Geometry g;
  g.M = M;
  g.c_num = cn;
  g.c_den = cd;
  g.sigma = sg;
  g.l = q > 3 ? (uint32_t)(q - 2) : 1u;
  g.V = ((uint64_t)g.l + 2) << sg;
  return g;
}

uint32_t cell_bytes_for(int32_t b) { return b <= 8 ? 1 : b <= 16 ? 2 : b <= 32 ? 4 : 8; }

// Upper bound on the largest shard used to size buffers before hashing:
// mean + 1.5 * sqrt(2 mean ln S) + 64 (Raab-Steger maximum load, section 4).
uint32_t shard_cap(uint64_t n, uint32_t S) {
  if (S <= 1) return (uint32_t)std::min<uint64_t>(n, 0xFFFFFFFFull);
  const double mean = (double)n / S;
  double cap = std::ceil(mean + 1.5 * std::sqrt(2.0 * mean * std::log((double)S)) + 64.0);
  return (uint32_t)std::min<double>(std::min<double>(cap, (double)n), 4.0e9);
}

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// The last failure of this thread, for vf_last_error.
thread_local char g_last_error[160];

int hip_failed(hipError_t e, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "vf_api.cpp:%d: %s (%d)", line, hipGetErrorString(e),
           (int)e);
  return VF_EHIP;
}

// No C++ exception crosses the C ABI: a failed host allocation becomes
// VF_ENOMEM, anything else VF_EHIP.
template <class F>
int guarded(F &&f) {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    return VF_ENOMEM;
  } catch (...) {
    return VF_EHIP;
  }
}

// Elimination-window slots a shard needs: simulated and measured peaks of
// the window are about 0.55-0.75 s rows for fuse graphs at c = 1.12 (s =
// segment size); shards that outgrow their share are rebuilt by a second
// launch with a whole CU's LDS.
uint32_t window_target(int32_t sigma) {
  const uint32_t s = 1u << sigma;
  return std::min<uint32_t>(512u, s / 2 + s / 8 + 32);
}

// How many build workgroups share one CU's LDS, and the
// LDS each gets: as many as still leave every one a large enough window.
void build_occupancy(int32_t sigma, uint32_t *per_cu, uint32_t *lds_bytes) {
  const uint32_t want = window_target(sigma);
  uint32_t best = 1;
  for (uint32_t n = 2; n <= 8; n++)
    if (vfk::window_slots((uint32_t)sigma, (vfk::kLdsBudget / n) & ~255u) >= want) best = n;
  *per_cu = best;
  *lds_bytes = (vfk::kLdsBudget / best) & ~255u;
}

// Launch shape of a build: workgroups per CU bounded by both LDS (each
// keeps an elimination window of window_target slots) and registers, the
// LDS each gets once that count is known, and its window slots.
struct BuildShape {
  uint32_t per_cu, lds_bytes, wmax;
};
BuildShape build_shape(int32_t sigma, uint32_t cell_bytes) {
  BuildShape b{};
  build_occupancy(sigma, &b.per_cu, &b.lds_bytes);
  auto slots = [&] {
    uint32_t w = vfk::window_slots((uint32_t)sigma, b.lds_bytes);
    // at most six slot groups in registers when the target allows it (the
    // peaks of a window run well above the target for the larger graphs
    // of a segment size, and a window that outgrows its slots costs a
    // second launch)
    if (w > 384 && window_target(sigma) <= 384) w = 384;
    return w;
  };
  b.wmax = slots();
  const int occ = vfk::build_blocks_per_cu(cell_bytes, b.wmax, b.lds_bytes);
  if (occ > 0 && (uint32_t)occ < b.per_cu) {
    // registers allow fewer: give each resident workgroup more LDS
    b.per_cu = (uint32_t)occ;
    b.lds_bytes = (vfk::kLdsBudget / b.per_cu) & ~255u;
    b.wmax = slots();
  }
  return b;
}

int device_cus() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return ncu;
}

struct Layout {
  int32_t h;
  uint32_t S, cap;
  Geometry gcap;
  uint32_t cell_bytes;
  uint32_t nwg;
  uint32_t logcap;
  uint64_t scratch_stride;
  uint64_t ws_bytes, st_bytes;
  uint64_t cells_bytes;
  // workspace offsets
  uint64_t o_counts, o_offsets, o_cursor, o_meta, o_work, o_fails, o_overflow, o_order, o_bkeys,
      o_bvals, o_scratch, o_rows;
  bool rows;  // keys grouped by per-segment histograms (filters, S <= 4096)
  uint32_t fail_cap;
  bool packed;         // cells packed to b bits in the structure
  uint64_t o_tcells;   // packed: byte-aligned cells of the build (workspace)
  uint64_t tcells_bytes;
};

// The back-substitution ring's column count of a test build: 0, or a
// power of two the kernel's ring holds.
bool ring_cols_ok(uint32_t c) {
  return c == 0 || (c >= 64 && c <= vfk::kRingCols && (c & (c - 1)) == 0);
}

int make_layout(uint64_t n, int32_t b, double eps, int32_t is_filter, const vf_opts &o,
                int ncu, Layout *L, uint32_t cap_override = 0) {
  if (b < 1 || b > 64) return VF_EINVAL;
  int32_t h = o.h;
  if (h < 0) {
    if (!(eps > 0)) return VF_EINVAL;
    h = shard_bits_from_eps(n, eps, o.alpha > 0 ? o.alpha : 1.0);
  }
  if (h > (int32_t)kMaxShardBits) return VF_EINVAL;
  if (o.tmax < 1 || o.tmax > 255) return VF_EINVAL;
  if (!ring_cols_ok(o.ring_cols)) return VF_EINVAL;
  if ((o.c_num == 0) != (o.c_den == 0)) return VF_EINVAL;
  if (o.c_num && o.c_num < o.c_den) return VF_EINVAL;  // c >= 1
  if (o.sigma > 20) return VF_EINVAL;
  Layout l{};
  l.h = h;
  l.S = 1u << h;
  l.cap = shard_cap(n, l.S);
  if (cap_override) l.cap = std::min(l.cap, cap_override);
  if (o.mwhc) {
    l.gcap = geometry_mwhc(l.cap, o.c_num, o.c_den);
  } else {
    l.gcap = geometry(l.cap, h, o.c_num, o.c_den, o.sigma);
  // V is not monotone in the shard size (segments double at powers of two,
  // the factor changes at 800 000 keys): size buffers for the largest V,
  // segment and segment count any shard up to the cap may take
  {
    std::vector<uint32_t> probe;
    for (uint32_t k = 1; k <= 32 && (1ull << k) <= (uint64_t)l.cap; k++) {
      probe.push_back((1u << k) - 1);
      probe.push_back(1u << k);
    }
    if (l.cap > 799999u) probe.push_back(799999u);
    for (uint32_t m : probe) {
      Geometry gk = geometry(m, h, o.c_num, o.c_den, o.sigma);
      l.gcap.V = std::max(l.gcap.V, gk.V);
      l.gcap.l = std::max(l.gcap.l, gk.l);
      l.gcap.sigma = std::max(l.gcap.sigma, gk.sigma);
    }
  }
  l.gcap.V += 1ull << l.gcap.sigma;
  // smaller shards may use smaller segments and hence more of them: bound
  // the segment count over all sizes up to the cap
  for (uint32_t k = 1; k <= 64; k++) {
    Geometry gk = geometry((uint32_t)((uint64_t)l.cap * k / 64), h, o.c_num, o.c_den, o.sigma);
    if (gk.l > l.gcap.l) l.gcap.l = gk.l;
  }
  l.gcap.l += l.gcap.l / 8 + 8;
  }
  l.cell_bytes = cell_bytes_for(b);
  uint32_t per_cu, lds_bytes;
  build_occupancy(l.gcap.sigma, &per_cu, &lds_bytes);
  // registers let at most 4 build workgroups share a CU; scratch is sized
  // for that many (the launch takes as many as are resident at once)
  per_cu = 4;
  l.nwg = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>((uint64_t)per_cu * (ncu > 0 ? ncu : 256), l.S));
  // pivot log of the 2-core elimination (MWHC never eliminates)
  l.logcap = o.mwhc ? 4096u : 16u * l.cap + 4096u;
  // scratch is sized for the largest shard the buffers allow, with the
  // geometry of that size (the actual geometry is never larger)
  l.scratch_stride =
      align256(vfk::build_scratch_bytes(l.cap, l.gcap.V, l.gcap.l, l.logcap));
  l.fail_cap = 4u * l.S + 1024u;
  uint64_t o_ = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = o_;
    o_ += align256(bytes);
    return at;
  };
  l.o_counts = take(4ull * l.S);
  l.o_offsets = take(8ull * (l.S + 1));
  l.o_cursor = take(8ull * l.S);
  l.o_meta = take(16);
  l.o_work = take(4ull * vfk::kWorkWords);
  l.o_fails = take(sizeof(vfk::FailRec) * (uint64_t)l.fail_cap);
  l.o_overflow = take(8ull * l.S);
  l.o_order = take(8ull * l.S);
  l.o_bkeys = take(8ull * std::max<uint64_t>(n, 1));
  l.o_bvals = is_filter ? 0 : take(8ull * std::max<uint64_t>(n, 1));
  l.o_scratch = take(l.scratch_stride * l.nwg);
  l.rows = is_filter && vfk::group_rows_fit(l.S) && n >= 1 && n <= 0xFFFFFFFFull;
  l.o_rows = l.rows ? take(4 * vfk::group_rows_words(l.S)) : 0;
  l.packed = o.packed != 0;
  l.tcells_bytes = l.packed ? align256((uint64_t)l.S * l.gcap.V * l.cell_bytes) : 0;
  l.o_tcells = l.packed ? take(l.tcells_bytes) : 0;
  l.ws_bytes = o_;
  l.cells_bytes = l.packed ? align256(8 * (((uint64_t)l.S * l.gcap.V * b + 63) / 64))
                           : align256((uint64_t)l.S * l.gcap.V * l.cell_bytes);
  l.st_bytes = l.cells_bytes + align256(l.S);
  *L = l;
  return VF_OK;
}

// Size classes of small batch instances (up to 16, 32, 64, 128 keys) and
// the choice of kernel for each, measured once per device by the first
// batch build that has enough instances of a class (batch_build below).
constexpr uint32_t kClassKeys[4] = {16, 32, 64, 128};
int size_class(uint64_t n) {
  for (int c = 0; c < 4; c++)
    if (n && n <= kClassKeys[c]) return c;
  return -1;
}
struct BatchTuning {
  bool done = false;
  bool use_small[4] = {true, true, true, true};
  float ms_small[4] = {0, 0, 0, 0}, ms_band[4] = {0, 0, 0, 0};
  uint32_t sampled[4] = {0, 0, 0, 0};
  uint32_t small_groups_per_cu = 8;
};
constexpr int kTuneDevices = 64;
std::mutex g_tune_mu;
BatchTuning g_tune[kTuneDevices];
int current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kTuneDevices) return -1;
  return dev;
}
BatchTuning batch_tuning() {
  const int dev = current_device();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return dev < 0 ? BatchTuning{} : g_tune[dev];
}
void set_batch_tuning(const BatchTuning &t) {
  const int dev = current_device();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (dev >= 0) g_tune[dev] = t;
}
constexpr uint32_t kTuneSample = 2048;  // instances timed per class

// Buffers of a batch of unsharded functions.  Workspace: work counters,
// failure records, overflow list, per-class build orders, scratch; the
// structure: instance descriptors, local seeds, cells (8-byte aligned per
// instance).
struct BatchLayout {
  uint64_t count = 0, keys = 0;
  std::vector<vfk::BatchItem> items;
  uint32_t maxM = 0, maxl = 1;
  uint64_t maxV = 0;
  int32_t maxsigma = 0;
  uint32_t nwg = 0, logcap = 0, fail_cap = 0;
  uint64_t scratch_stride = 0;
  uint64_t o_work = 0, o_fails = 0, o_overflow = 0, o_order = 0, o_scratch = 0, ws_bytes = 0;
  uint64_t o_check = 0;  // instance descriptors and a flag for the value check
  uint64_t o_tune = 0;   // lists of the instances timed by the tuning
  bool packed = false;   // instance cells packed to b bits in the structure
  std::vector<vfk::BatchItem> pitems;  // packed: descriptors with structure offsets
  uint64_t o_tcells = 0, tcells_bytes = 0;  // packed: byte cells of the build
  uint64_t s_items = 0, s_seeds = 0, s_cells = 0, cells_bytes = 0, st_bytes = 0;
};

int make_batch_layout(uint64_t count, const uint64_t *n, const int32_t *b, const vf_opts &o,
                      int ncu, BatchLayout *L) {
  if (!count || !n || !b || count > 0xFFFFFFFFull) return VF_EINVAL;
  if (o.tmax < 1 || o.tmax > 255) return VF_EINVAL;
  if (!ring_cols_ok(o.ring_cols)) return VF_EINVAL;
  if ((o.c_num == 0) != (o.c_den == 0)) return VF_EINVAL;
  if (o.c_num && o.c_num < o.c_den) return VF_EINVAL;
  if (o.sigma > 20) return VF_EINVAL;
  BatchLayout l;
  l.count = count;
  l.items.resize(count);
  l.packed = o.packed != 0;
  if (l.packed) l.pitems.reserve(count);
  uint64_t cell_off = 0, packed_off = 0;
  for (uint64_t i = 0; i < count; i++) {
    if (b[i] < 1 || b[i] > 64 || n[i] > 0xFFFFFFFFull) return VF_EINVAL;
    const Geometry g = geometry((uint32_t)n[i], 0, o.c_num, o.c_den, o.sigma);
    if (g.V > kMaxCells) return VF_ECAPACITY;
    vfk::BatchItem &it = l.items[i];
    it.key_off = l.keys;
    it.cell_off = cell_off;
    it.V = g.V;
    it.vmask = b[i] >= 64 ? ~0ull : ((1ull << b[i]) - 1);
    it.n = (uint32_t)n[i];
    it.l = g.l;
    it.sigma = (uint32_t)g.sigma;
    it.b = (uint32_t)b[i];
    it.cell_bytes = cell_bytes_for(b[i]);
    it.c_num = g.c_num;
    it.c_den = g.c_den;
    it.pad = 0;
    l.keys += n[i];
    cell_off += (g.V * it.cell_bytes + 7) & ~7ull;
    if (o.packed) {
      vfk::BatchItem pit = it;
      pit.cell_off = packed_off;
      l.pitems.push_back(pit);
      packed_off += 8 * ((g.V * (uint64_t)b[i] + 63) / 64);
    }
    l.maxM = std::max(l.maxM, it.n);
    l.maxV = std::max(l.maxV, g.V);
    l.maxl = std::max(l.maxl, g.l);
    l.maxsigma = std::max(l.maxsigma, g.sigma);
  }
  uint32_t per_cu, lds_bytes;
  build_occupancy(l.maxsigma, &per_cu, &lds_bytes);
  l.nwg = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>((uint64_t)per_cu * (ncu > 0 ? ncu : 256), count));
  l.logcap = 16u * l.maxM + 4096u;
  l.scratch_stride = align256(vfk::build_scratch_bytes(l.maxM, l.maxV, l.maxl, l.logcap));
  l.fail_cap = (uint32_t)std::min<uint64_t>(4ull * count + 1024u, 0xFFFFFFF0ull);
  uint64_t o_ = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = o_;
    o_ += align256(bytes);
    return at;
  };
  l.o_work = take(4ull * vfk::kWorkWords);
  l.o_fails = take(sizeof(vfk::FailRec) * (uint64_t)l.fail_cap);
  l.o_overflow = take(8ull * count);
  l.o_order = take(8ull * count);
  l.o_scratch = take(l.scratch_stride * l.nwg);
  l.o_check = take(sizeof(vfk::BatchItem) * count + 256);
  l.o_tune = take(8ull * kTuneSample);
  l.tcells_bytes = l.packed ? align256(cell_off) : 0;
  l.o_tcells = l.packed ? take(l.tcells_bytes) : 0;
  l.ws_bytes = o_;
  o_ = 0;
  l.s_items = take(sizeof(vfk::BatchItem) * count);
  l.s_seeds = take(count);
  l.cells_bytes = align256(l.packed ? packed_off : cell_off);
  l.s_cells = take(l.cells_bytes);
  l.st_bytes = o_;
  *L = std::move(l);
  return VF_OK;
}

}  // namespace

struct BatchRun;
struct BuildRun;

struct vf_handle {
  uint32_t magic;
  int32_t is_filter, b, h;
  uint32_t S;
  Geometry g;
  uint64_t n, seed;
  uint32_t cell_bytes;
  vfk::Geo G;
  void *cells;
  uint8_t *tseed;
  std::vector<vf_failure> fails;
  uint32_t n_fail_total;
  uint32_t failed_shards;
  int ncu;
  float ms[3];
  uint32_t relaunched;
  uint32_t packed;  // cells are a bit string of b-bit fields
  // batches (kind 1): one descriptor and local seed per instance
  int32_t kind;
  uint64_t count;
  std::vector<vfk::BatchItem> items;
  std::vector<uint8_t> seeds;
  const vfk::BatchItem *items_dev;
  // a batch prepared by vf_batch_prepare (kind 2 until its first
  // vf_batch_finish reports a built structure, kind 1 after)
  std::shared_ptr<BatchRun> run;
  // a structure prepared by vf_build_prepare (kind 3 until its first
  // vf_build_finish reports a built structure, kind 0 after)
  std::shared_ptr<BuildRun> brun;
};

namespace {
// Events bracketing the device phases of one build (created per build).
struct PhaseEvents {
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool ok = true;
  PhaseEvents() {
    for (auto &e : ev) ok = ok && hipEventCreate(&e) == hipSuccess;
  }
  ~PhaseEvents() {
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void record(int i, hipStream_t s) {
    if (ok) ok = hipEventRecord(ev[i], s) == hipSuccess;
  }
  float between(int a, int b) const {
    float ms = 0.f;
    if (!ok || hipEventElapsedTime(&ms, ev[a], ev[b]) != hipSuccess) return -1.f;
    return ms;
  }
};
}  // namespace

extern "C" {

const char *vf_last_error(void) { return g_last_error; }

void vf_default_opts(vf_opts *o) {
  if (!o) return;
  o->h = -1;
  o->sigma = -1;
  o->c_num = 0;
  o->c_den = 0;
  o->tmax = 255;
  o->alpha = 1.0;
  o->mwhc = 0;
  o->max_window = 0;
  o->packed = 0;
  o->small = 0;
  o->ring_cols = 0;
}

int vf_plan(uint64_t n, int32_t b, double eps, int32_t is_filter, const vf_opts *o,
            vf_sizes *out) {
  if (!out) return VF_EINVAL;
  vf_opts d;
  vf_default_opts(&d);
  Layout L;
  int rc = guarded([&] { return make_layout(n, b, eps, is_filter, o ? *o : d, device_cus(), &L); });
  if (rc) return rc;
  out->structure_bytes = L.st_bytes;
  out->workspace_bytes = L.ws_bytes;
  out->h = L.h;
  out->shard_cap = L.cap;
  return VF_OK;
}

// Keys in host memory: copied into the workspace past the planned bytes in
// chunks on a copy stream of the library's, each chunk counted by shard as
// soon as it has arrived (the next chunk's copy overlaps the counting).
struct HostKeys {
  const uint64_t *keys = nullptr;  // host
  uint64_t chunk = 0;              // keys per copy
};

static int build_common(const uint64_t *keys, const uint64_t *values, uint64_t n, int32_t b,
                        double eps, uint64_t seed, const vf_opts *o, void *ws,
                        uint64_t ws_bytes, void *st, uint64_t st_bytes, hipStream_t stream,
                        vf_handle **handle, int32_t is_filter, const HostKeys *hk = nullptr) {
  if (hk) {
    if (!hk->keys && n) return VF_EINVAL;
    keys = hk->keys;
  }
  if (!handle || !ws || !st || (n && !keys) || (!is_filter && n && !values)) return VF_EINVAL;
  vf_opts d;
  vf_default_opts(&d);
  const vf_opts &op = o ? *o : d;
  const int ncu = device_cus();
  if (ncu <= 0) return VF_EHIP;
  Layout L;
  int rc = make_layout(n, b, eps, is_filter, op, ncu, &L);
  if (rc) return rc;
  const uint64_t ws_need = L.ws_bytes + (hk ? align256(8 * n) : 0);
  if (ws_bytes < ws_need || st_bytes < L.st_bytes) return VF_ENOSPC;

  uint8_t *W = (uint8_t *)ws;
  uint32_t *counts = (uint32_t *)(W + L.o_counts);
  uint64_t *offsets = (uint64_t *)(W + L.o_offsets);
  uint64_t *cursor = (uint64_t *)(W + L.o_cursor);
  uint32_t *meta = (uint32_t *)(W + L.o_meta);
  uint32_t *work = (uint32_t *)(W + L.o_work);
  vfk::FailRec *fails = (vfk::FailRec *)(W + L.o_fails);
  uint32_t *overflow = (uint32_t *)(W + L.o_overflow);
  uint32_t *order = (uint32_t *)(W + L.o_order);
  uint64_t *bkeys = (uint64_t *)(W + L.o_bkeys);
  uint64_t *bvals = is_filter ? nullptr : (uint64_t *)(W + L.o_bvals);
  uint8_t *scratch = W + L.o_scratch;
  // keys grouped through per-segment histograms (not for keys copied from
  // the host chunk by chunk)
  const bool rows = L.rows && !hk;
  uint32_t *row_counts = rows ? (uint32_t *)(W + L.o_rows) : nullptr;
  uint8_t *cells = (uint8_t *)st;
  uint8_t *tseed = cells + L.cells_bytes;

  uint64_t sw[3];
  seed_words(seed, sw);

#define HIPCHK(x)                                      \
  do {                                                 \
    const hipError_t e_ = (x);                         \
    if (e_ != hipSuccess) return hip_failed(e_, __LINE__); \
  } while (0)

  PhaseEvents pe;
  // 1. keys per shard, largest shard
  pe.record(0, stream);
  HIPCHK(vfk::launch_fill_u32(counts, L.S, 0, stream));
  HIPCHK(vfk::launch_fill_u32(meta, 4, 0, stream));
  if (hk && n) {
    uint64_t *dk = (uint64_t *)(W + L.ws_bytes);
    const uint64_t chunk = hk->chunk ? hk->chunk : n;
    hipStream_t cs = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool ok = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess;
    for (auto &e : ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    // the copy stream starts after the work already on the build stream
    ok = ok && hipEventRecord(ev[1], stream) == hipSuccess &&
         hipStreamWaitEvent(cs, ev[1], 0) == hipSuccess;
    for (uint64_t c0 = 0, i = 0; ok && c0 < n; c0 += chunk, i++) {
      const uint64_t cnt = std::min(chunk, n - c0);
      hipEvent_t e = ev[i & 1];
      ok = hipMemcpyAsync(dk + c0, hk->keys + c0, 8 * cnt, hipMemcpyHostToDevice, cs) ==
               hipSuccess &&
           hipEventRecord(e, cs) == hipSuccess && hipStreamWaitEvent(stream, e, 0) == hipSuccess &&
           vfk::launch_count(dk + c0, cnt, sw[0], (uint32_t)L.h, L.S, counts, ncu, stream) ==
               hipSuccess;
    }
    if (cs) ok = (hipStreamSynchronize(cs) == hipSuccess) && ok;
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
    if (cs) (void)hipStreamDestroy(cs);
    if (!ok) return VF_EHIP;
    keys = dk;
  } else if (rows) {
    HIPCHK(vfk::launch_count_rows(keys, n, sw[0], (uint32_t)L.h, L.S, row_counts, counts, stream));
  } else {
    HIPCHK(vfk::launch_count(keys, n, sw[0], (uint32_t)L.h, L.S, counts, ncu, stream));
  }
  HIPCHK(vfk::launch_scan(counts, L.S, offsets, cursor, meta, stream));
  // Problem 1 stores b-bit values: any higher bit makes the call fail
  // before the structure is written (meta[1])
  if (!is_filter) HIPCHK(vfk::launch_check_values(values, n, (uint32_t)b, meta + 1, stream));
  pe.record(1, stream);
  uint32_t hmeta[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(hmeta, meta, sizeof(hmeta), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  const uint32_t M = hmeta[0];
  if (hmeta[1]) return VF_EINVAL;
  if (M > L.cap) return VF_ENOSPC;
  const Geometry g =
      op.mwhc ? geometry_mwhc(M, op.c_num, op.c_den) : geometry(M, L.h, op.c_num, op.c_den, op.sigma);
  if (g.V > kMaxCells) return VF_ECAPACITY;
  const uint64_t need_cells = L.packed ? 8 * (((uint64_t)L.S * g.V * b + 63) / 64)
                                      : (uint64_t)L.S * g.V * L.cell_bytes;
  if (need_cells > L.cells_bytes ||
      (L.packed && (uint64_t)L.S * g.V * L.cell_bytes > L.tcells_bytes) ||
      vfk::build_scratch_bytes(M, g.V, g.l, L.logcap) > L.scratch_stride)
    return VF_ENOSPC;
  // packed structures are built on byte cells in the workspace
  uint8_t *const bcells = L.packed ? W + L.o_tcells : cells;

  // 2. group keys by shard; build order (largest shards first)
  HIPCHK(vfk::launch_order(counts, L.S, M, order, stream));
  if (rows)
    HIPCHK(vfk::launch_scatter_rows(keys, n, sw[0], (uint32_t)L.h, L.S, row_counts, cursor, bkeys,
                                    nullptr, nullptr, stream));
  else
    HIPCHK(vfk::launch_scatter(keys, values, n, sw[0], (uint32_t)L.h, L.S, cursor, bkeys, bvals,
                               nullptr, ncu, stream));
  pe.record(2, stream);

  // 3. build every shard
  vfk::BuildArgs A{};
  A.G.khi = sw[0];
  A.G.klo = sw[1];
  A.G.kfp = sw[2];
  A.G.V = g.V;
  A.G.vmask = b >= 64 ? ~0ull : ((1ull << b) - 1);
  A.G.h = (uint32_t)L.h;
  A.G.S = L.S;
  A.G.l = g.l;
  A.G.sigma = (uint32_t)g.sigma;
  A.G.b = (uint32_t)b;
  A.G.is_filter = (uint32_t)is_filter;
  A.G.mwhc = g.mwhc;
  A.G.part = g.part;
  A.bkeys = bkeys;
  A.bvals = bvals;
  A.offsets = offsets;
  A.cells = bcells;
  A.tseed = tseed;
  A.scratch = scratch;
  A.scratch_stride = L.scratch_stride;
  A.work = work;
  A.fails = fails;
  A.fail_cap = L.fail_cap;
  A.M = M;
  A.tmax = op.tmax;
  A.ring_cols = op.ring_cols;
  const BuildShape shape = build_shape(g.sigma, L.cell_bytes);
  A.lds_bytes = shape.lds_bytes;
  A.wmax = shape.wmax;
  if (op.max_window) A.wmax = std::min(A.wmax, std::max(8u, op.max_window & ~7u));
  const uint32_t per_cu = shape.per_cu;
  const uint32_t nwg = std::min<uint32_t>(L.nwg, per_cu * (uint32_t)ncu);
  A.logcap = L.logcap;
  A.cell_bytes = L.cell_bytes;
  A.list = order;
  A.nlist = L.S;
  A.overflow = overflow;
  A.items = nullptr;
  A.scr_V = g.V;
  A.scr_l = g.l;
  HIPCHK(vfk::launch_fill_u32(work, vfk::kWorkWords, 0, stream));
  HIPCHK(vfk::launch_build(A, (int)nwg, stream));
  uint32_t hwork[vfk::kWorkWords];
  HIPCHK(hipMemcpyAsync(hwork, work, sizeof(hwork), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (hwork[vfk::kWorkCap]) {
    // shards whose window outgrew their share of LDS: rebuild them from the
    // attempt they reached, one workgroup per CU with all of its LDS
    A.list = overflow;
    A.nlist = hwork[vfk::kWorkCap];
    A.overflow = nullptr;
    A.lds_bytes = (vfk::kLdsBudget - 256) & ~255u;
    A.wmax = vfk::window_slots((uint32_t)g.sigma, A.lds_bytes);
    HIPCHK(vfk::launch_fill_u32(work + vfk::kWorkNext, 1, 0, stream));
    HIPCHK(vfk::launch_build(A, (int)std::min<uint32_t>(nwg, (uint32_t)ncu), stream));
    HIPCHK(hipMemcpyAsync(hwork, work, sizeof(hwork), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
  }
  if (L.packed)
    HIPCHK(vfk::launch_pack(bcells, L.cell_bytes, (uint64_t)L.S * g.V, (uint32_t)b,
                            (uint64_t *)cells, stream));
  pe.record(3, stream);

  // 4. failure record
  const uint32_t nf = std::min(hwork[vfk::kWorkFails], L.fail_cap);
  std::vector<vfk::FailRec> fr(nf);
  if (nf)
    HIPCHK(hipMemcpyAsync(fr.data(), fails, nf * sizeof(vfk::FailRec), hipMemcpyDeviceToHost,
                          stream));
  std::vector<uint8_t> ts(L.S);
  HIPCHK(hipMemcpyAsync(ts.data(), tseed, L.S, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
#undef HIPCHK

  vf_handle *H = new (std::nothrow) vf_handle();
  if (!H) return VF_ENOMEM;
  H->magic = kMagic;
  H->is_filter = is_filter;
  H->b = b;
  H->h = L.h;
  H->S = L.S;
  H->g = g;
  H->n = n;
  H->seed = seed;
  H->cell_bytes = L.cell_bytes;
  H->G = A.G;
  H->cells = cells;
  H->packed = L.packed ? 1u : 0u;
  H->tseed = tseed;
  H->ncu = ncu;
  H->n_fail_total = hwork[vfk::kWorkFails];
  H->relaunched = hwork[vfk::kWorkCap];
  H->ms[0] = pe.between(0, 1);
  H->ms[1] = pe.between(1, 2);
  H->ms[2] = pe.between(2, 3);
  for (const auto &f : fr) H->fails.push_back(vf_failure{f.shard, f.attempt, f.kind, f.core_edges});
  std::sort(H->fails.begin(), H->fails.end(), [](const vf_failure &a, const vf_failure &c) {
    return a.shard != c.shard ? a.shard < c.shard : a.attempt < c.attempt;
  });
  H->failed_shards = (uint32_t)std::count(ts.begin(), ts.end(), (uint8_t)255);
  *handle = H;
  if (hwork[vfk::kWorkStatus] & vfk::kStatusStalled) {
    snprintf(g_last_error, sizeof(g_last_error), "a build workgroup gave up on a wait");
    return VF_EHIP;
  }
  if (hwork[vfk::kWorkStatus] & vfk::kStatusCapacity) return VF_ECAPACITY;
  if (H->failed_shards) return VF_EFAIL;
  return VF_OK;
}

// A sharded build whose geometry is fixed before the keys are seen (the
// largest shard is bounded by max_shard instead of measured), so that its
// device work needs no host read: vf_build_prepare / launch / finish.
struct BuildRun {
  Layout L;
  vf_opts op{};
  int ncu = 0;
  Geometry g{};
  int32_t b = 0, is_filter = 0;
  uint64_t n = 0, seed = 0;
  bool rows = false;
  uint32_t nwg = 0, relaunch_lds = 0, relaunch_wmax = 0;
  vfk::BuildArgs A{};  // keys, values and the abort flag are set per launch
  uint32_t *counts = nullptr, *meta = nullptr, *work = nullptr, *order = nullptr,
           *overflow = nullptr, *row_counts = nullptr;
  uint64_t *offsets = nullptr, *cursor = nullptr, *bkeys = nullptr, *bvals = nullptr;
  vfk::FailRec *fails = nullptr;
  uint8_t *cells = nullptr, *bcells = nullptr, *tseed = nullptr;
};

#define HIPCHK(x)                                          \
  do {                                                     \
    const hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) return hip_failed(e_, __LINE__); \
  } while (0)

static int build_prepare(uint64_t n, uint32_t max_shard, int32_t b, double eps, int32_t is_filter,
                         uint64_t seed, const vf_opts *o, void *ws, uint64_t ws_bytes, void *st,
                         uint64_t st_bytes, vf_handle **handle) {
  if (!handle || !ws || !st || !n) return VF_EINVAL;
  auto R = std::make_shared<BuildRun>();
  vf_default_opts(&R->op);
  if (o) R->op = *o;
  const vf_opts &op = R->op;
  R->ncu = device_cus();
  if (R->ncu <= 0) return VF_EHIP;
  Layout &L = R->L;
  int rc = make_layout(n, b, eps, is_filter, op, R->ncu, &L);
  if (rc) return rc;
  // buffers are sized for the plan's bound: a tighter bound only
  if (max_shard > L.cap) return VF_EINVAL;
  if (max_shard) {
    rc = make_layout(n, b, eps, is_filter, op, R->ncu, &L, max_shard);
    if (rc) return rc;
  }
  if (ws_bytes < L.ws_bytes || st_bytes < L.st_bytes) return VF_ENOSPC;
  const uint32_t M = L.cap;  // every shard is sized for the bound
  R->g = op.mwhc ? geometry_mwhc(M, op.c_num, op.c_den)
                 : geometry(M, L.h, op.c_num, op.c_den, op.sigma);
  const Geometry &g = R->g;
  if (g.V > kMaxCells) return VF_ECAPACITY;
  const uint64_t need_cells = L.packed ? 8 * (((uint64_t)L.S * g.V * b + 63) / 64)
                                      : (uint64_t)L.S * g.V * L.cell_bytes;
  if (need_cells > L.cells_bytes ||
      (L.packed && (uint64_t)L.S * g.V * L.cell_bytes > L.tcells_bytes) ||
      vfk::build_scratch_bytes(M, g.V, g.l, L.logcap) > L.scratch_stride)
    return VF_ENOSPC;
  R->b = b;
  R->is_filter = is_filter;
  R->n = n;
  R->seed = seed;
  R->rows = L.rows;
  uint8_t *W = (uint8_t *)ws;
  R->counts = (uint32_t *)(W + L.o_counts);
  R->offsets = (uint64_t *)(W + L.o_offsets);
  R->cursor = (uint64_t *)(W + L.o_cursor);
  R->meta = (uint32_t *)(W + L.o_meta);
  R->work = (uint32_t *)(W + L.o_work);
  R->fails = (vfk::FailRec *)(W + L.o_fails);
  R->overflow = (uint32_t *)(W + L.o_overflow);
  R->order = (uint32_t *)(W + L.o_order);
  R->bkeys = (uint64_t *)(W + L.o_bkeys);
  R->bvals = is_filter ? nullptr : (uint64_t *)(W + L.o_bvals);
  R->row_counts = R->rows ? (uint32_t *)(W + L.o_rows) : nullptr;
  R->cells = (uint8_t *)st;
  R->tseed = R->cells + L.cells_bytes;
  R->bcells = L.packed ? W + L.o_tcells : R->cells;
  uint64_t sw[3];
  seed_words(seed, sw);
  vfk::BuildArgs &A = R->A;
  A.G.khi = sw[0];
  A.G.klo = sw[1];
  A.G.kfp = sw[2];
  A.G.V = g.V;
  A.G.vmask = b >= 64 ? ~0ull : ((1ull << b) - 1);
  A.G.h = (uint32_t)L.h;
  A.G.S = L.S;
  A.G.l = g.l;
  A.G.sigma = (uint32_t)g.sigma;
  A.G.b = (uint32_t)b;
  A.G.is_filter = (uint32_t)is_filter;
  A.G.mwhc = g.mwhc;
  A.G.part = g.part;
  A.bkeys = R->bkeys;
  A.bvals = R->bvals;
  A.offsets = R->offsets;
  A.cells = R->bcells;
  A.tseed = R->tseed;
  A.scratch = W + L.o_scratch;
  A.scratch_stride = L.scratch_stride;
  A.work = R->work;
  A.fails = R->fails;
  A.fail_cap = L.fail_cap;
  A.M = M;
  A.tmax = op.tmax;
  A.ring_cols = op.ring_cols;
  const BuildShape shape = build_shape(g.sigma, L.cell_bytes);
  A.lds_bytes = shape.lds_bytes;
  A.wmax = shape.wmax;
  if (op.max_window) A.wmax = std::min(A.wmax, std::max(8u, op.max_window & ~7u));
  R->nwg = std::min<uint32_t>(L.nwg, shape.per_cu * (uint32_t)R->ncu);
  A.logcap = L.logcap;
  A.cell_bytes = L.cell_bytes;
  A.list = R->order;
  A.nlist = L.S;
  A.overflow = R->overflow;
  A.items = nullptr;
  A.scr_V = g.V;
  A.scr_l = g.l;
  R->relaunch_lds = (vfk::kLdsBudget - 256) & ~255u;
  R->relaunch_wmax = vfk::window_slots((uint32_t)g.sigma, R->relaunch_lds);
  // dynamic-LDS attributes now, so that a launch makes no such call
  HIPCHK(vfk::prepare_build(A));
  vfk::BuildArgs B = A;
  B.lds_bytes = R->relaunch_lds;
  B.wmax = R->relaunch_wmax;
  HIPCHK(vfk::prepare_build(B));
  vf_handle *H = new (std::nothrow) vf_handle();
  if (!H) return VF_ENOMEM;
  H->magic = kMagic;
  H->kind = 3;
  H->is_filter = is_filter;
  H->b = b;
  H->seed = seed;
  H->h = L.h;
  H->S = L.S;
  H->g = g;
  H->n = n;
  H->cell_bytes = L.cell_bytes;
  H->packed = L.packed ? 1u : 0u;
  H->brun = std::move(R);
  *handle = H;
  return VF_OK;
}

// Kernels only: count, scan, value and bound checks (either sets meta[1]
// and every later kernel of the build returns at once), order, scatter,
// build, rebuild of overflowing windows (list length read on the device),
// packing.
static int build_enqueue(const BuildRun &R, const uint64_t *keys, const uint64_t *values,
                         hipStream_t stream) {
  const Layout &L = R.L;
  const uint64_t n = R.n;
  const uint64_t khi = R.A.G.khi;
  HIPCHK(vfk::launch_fill_u32(R.counts, L.S, 0, stream));
  HIPCHK(vfk::launch_fill_u32(R.meta, 4, 0, stream));
  HIPCHK(vfk::launch_fill_u32(R.work, vfk::kWorkWords, 0, stream));
  if (R.rows)
    HIPCHK(vfk::launch_count_rows(keys, n, khi, (uint32_t)L.h, L.S, R.row_counts, R.counts,
                                  stream));
  else
    HIPCHK(vfk::launch_count(keys, n, khi, (uint32_t)L.h, L.S, R.counts, R.ncu, stream));
  HIPCHK(vfk::launch_scan(R.counts, L.S, R.offsets, R.cursor, R.meta, stream));
  if (!R.is_filter)
    HIPCHK(vfk::launch_check_values(values, n, (uint32_t)R.b, R.meta + 1, stream));
  HIPCHK(vfk::launch_check_bound(R.meta, L.cap, stream));
  HIPCHK(vfk::launch_order(R.counts, L.S, L.cap, R.order, stream));
  if (R.rows)
    HIPCHK(vfk::launch_scatter_rows(keys, n, khi, (uint32_t)L.h, L.S, R.row_counts, R.cursor,
                                    R.bkeys, nullptr, nullptr, stream));
  else
    HIPCHK(vfk::launch_scatter(keys, values, n, khi, (uint32_t)L.h, L.S, R.cursor, R.bkeys,
                               R.bvals, nullptr, R.ncu, stream));
  vfk::BuildArgs A = R.A;
  A.abort = R.meta + 1;
  HIPCHK(vfk::launch_build(A, (int)R.nwg, stream));
  vfk::BuildArgs B = A;
  B.list = R.overflow;
  B.nlist = 0;
  B.nlist_dev = R.work + vfk::kWorkCap;
  B.overflow = nullptr;
  B.lds_bytes = R.relaunch_lds;
  B.wmax = R.relaunch_wmax;
  HIPCHK(vfk::launch_fill_u32(R.work + vfk::kWorkNext, 1, 0, stream));
  HIPCHK(vfk::launch_build(B, (int)std::min<uint32_t>(R.nwg, (uint32_t)R.ncu), stream));
  if (L.packed)
    HIPCHK(vfk::launch_pack_checked(R.bcells, L.cell_bytes, (uint64_t)L.S * R.g.V,
                                    (uint32_t)R.b, (uint64_t *)R.cells, A.abort, stream));
  return VF_OK;
}

// After the launched work: the checks, counters, failure record and seeds
// into the handle (untouched when a check failed).
static int build_collect(const BuildRun &R, hipStream_t stream, vf_handle *H) {
  const Layout &L = R.L;
  uint32_t hmeta[4], hwork[vfk::kWorkWords];
  HIPCHK(hipMemcpyAsync(hmeta, R.meta, sizeof(hmeta), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(hwork, R.work, sizeof(hwork), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (hmeta[1] & 1u) return VF_EINVAL;
  if (hmeta[1] & 2u) {
    snprintf(g_last_error, sizeof(g_last_error), "largest shard %u above the bound %u", hmeta[0],
             L.cap);
    return VF_ENOSPC;
  }
  const uint32_t nf = std::min(hwork[vfk::kWorkFails], L.fail_cap);
  std::vector<vfk::FailRec> fr(nf);
  if (nf)
    HIPCHK(hipMemcpyAsync(fr.data(), R.fails, nf * sizeof(vfk::FailRec), hipMemcpyDeviceToHost,
                          stream));
  std::vector<uint8_t> ts(L.S);
  HIPCHK(hipMemcpyAsync(ts.data(), R.tseed, L.S, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  H->kind = 0;
  H->h = L.h;
  H->S = L.S;
  H->g = R.g;
  H->n = R.n;
  H->cell_bytes = L.cell_bytes;
  H->G = R.A.G;
  H->cells = R.cells;
  H->packed = L.packed ? 1u : 0u;
  H->tseed = R.tseed;
  H->ncu = R.ncu;
  H->n_fail_total = hwork[vfk::kWorkFails];
  H->relaunched = hwork[vfk::kWorkCap];
  H->ms[0] = H->ms[1] = H->ms[2] = 0.f;
  H->fails.clear();
  for (const auto &f : fr) H->fails.push_back(vf_failure{f.shard, f.attempt, f.kind, f.core_edges});
  std::sort(H->fails.begin(), H->fails.end(), [](const vf_failure &a, const vf_failure &c) {
    return a.shard != c.shard ? a.shard < c.shard : a.attempt < c.attempt;
  });
  H->failed_shards = (uint32_t)std::count(ts.begin(), ts.end(), (uint8_t)255);
  if (hwork[vfk::kWorkStatus] & vfk::kStatusStalled) {
    snprintf(g_last_error, sizeof(g_last_error), "a build workgroup gave up on a wait");
    return VF_EHIP;
  }
  if (hwork[vfk::kWorkStatus] & vfk::kStatusCapacity) return VF_ECAPACITY;
  if (H->failed_shards) return VF_EFAIL;
  return VF_OK;
}
#undef HIPCHK

int vf_build_prepare(uint64_t n, uint32_t max_shard, int32_t b, double eps, int32_t is_filter,
                     uint64_t seed, const vf_opts *o, void *workspace, uint64_t workspace_bytes,
                     void *structure, uint64_t structure_bytes, vf_handle **handle) {
  return guarded([&] {
    return build_prepare(n, max_shard, b, eps, is_filter ? 1 : 0, seed, o, workspace,
                         workspace_bytes, structure, structure_bytes, handle);
  });
}

int vf_build_launch(vf_handle *h, const uint64_t *keys, const uint64_t *values,
                    hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h || h->magic != kMagic || !h->brun || !keys) return VF_EINVAL;
    if (!h->brun->is_filter && !values) return VF_EINVAL;
    return build_enqueue(*h->brun, keys, values, stream);
  });
}

int vf_build_finish(vf_handle *h, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h || h->magic != kMagic || !h->brun) return VF_EINVAL;
    return build_collect(*h->brun, stream, h);
  });
}

int vf_build(const uint64_t *keys, const uint64_t *values, uint64_t n, int32_t b, double eps,
             uint64_t seed, const vf_opts *o, void *workspace, uint64_t workspace_bytes,
             void *structure, uint64_t structure_bytes, hipStream_t stream,
             vf_handle **handle) {
  return guarded([&] {
    return build_common(keys, values, n, b, eps, seed, o, workspace, workspace_bytes, structure,
                        structure_bytes, stream, handle, 0);
  });
}

int vfilter_build(const uint64_t *keys, uint64_t n, int32_t b, double eps, uint64_t seed,
                  const vf_opts *o, void *workspace, uint64_t workspace_bytes, void *structure,
                  uint64_t structure_bytes, hipStream_t stream, vf_handle **handle) {
  return guarded([&] {
    return build_common(keys, nullptr, n, b, eps, seed, o, workspace, workspace_bytes, structure,
                        structure_bytes, stream, handle, 1);
  });
}

int vfilter_build_host(const uint64_t *keys, uint64_t n, int32_t b, double eps, uint64_t seed,
                       const vf_opts *o, uint64_t chunk, void *workspace,
                       uint64_t workspace_bytes, void *structure, uint64_t structure_bytes,
                       hipStream_t stream, vf_handle **handle) {
  HostKeys hk;
  hk.keys = keys;
  hk.chunk = chunk;
  return guarded([&] {
    return build_common(nullptr, nullptr, n, b, eps, seed, o, workspace, workspace_bytes,
                        structure, structure_bytes, stream, handle, 1, &hk);
  });
}

static int query_common(const vf_handle *h, const uint64_t *keys, uint64_t n, void *out,
                        hipStream_t stream, int32_t want_filter) {
  if (!h || h->magic != kMagic || h->kind != 0 || h->is_filter != want_filter) return VF_EINVAL;
  if (n && (!keys || !out)) return VF_EINVAL;
  if (vfk::launch_query(h->G, h->cells, h->cell_bytes, h->tseed, keys, n, out, h->ncu, stream,
                        h->packed != 0) != hipSuccess)
    return VF_EHIP;
  return VF_OK;
}

int vf_query(const vf_handle *h, const uint64_t *keys, uint64_t n, void *out,
             hipStream_t stream) {
  return query_common(h, keys, n, out, stream, 0);
}

int vfilter_contains(const vf_handle *h, const uint64_t *keys, uint64_t n, uint8_t *out,
                     hipStream_t stream) {
  return query_common(h, keys, n, out, stream, 1);
}

static_assert(VF_QUERY_MULTI_MAX == vfk::kMultiMax, "combined query width");

int vf_query_multi(const vf_query_req *reqs, uint32_t count, hipStream_t stream) {
  return guarded([&]() -> int {
    if (count && !reqs) return VF_EINVAL;
    int ncu = 0;
    for (uint32_t r = 0; r < count; r++) {
      const vf_handle *h = reqs[r].h;
      if (!h || h->magic != kMagic || h->kind != 0) return VF_EINVAL;
      if (reqs[r].n && (!reqs[r].keys || !reqs[r].out)) return VF_EINVAL;
      ncu = std::max(ncu, h->ncu);
    }
    for (uint32_t r0 = 0; r0 < count; r0 += vfk::kMultiMax) {
      vfk::MultiArgs a{};
      a.count = std::min<uint32_t>(vfk::kMultiMax, count - r0);
      a.start[0] = 0;
      for (uint32_t i = 0; i < a.count; i++) {
        const vf_query_req &q = reqs[r0 + i];
        const vf_handle *h = q.h;
        vfk::MultiReq &m = a.req[i];
        m.G = h->G;
        m.cells = h->cells;
        m.tseed = h->tseed;
        m.keys = q.keys;
        m.out = q.out;
        m.cell_bytes = h->cell_bytes;
        m.packed = h->packed;
        a.start[i + 1] = a.start[i] + q.n;
      }
      for (uint32_t i = a.count; i < vfk::kMultiMax; i++) a.start[i + 1] = a.start[a.count];
      const hipError_t e = vfk::launch_query_multi(a, ncu, stream);
      if (e != hipSuccess) return hip_failed(e, __LINE__);
    }
    return VF_OK;
  });
}

// Grouped queries: workspace = shard totals, per-segment histograms and
// run starts, shard offsets and cursors, then for one chunk the keys grouped
// by shard, their indices and their answers in grouped order.
constexpr uint64_t kGroupChunkMax = 1ull << 26;

// one per-segment table (histogram rows, or run starts) of launch_group_rows
static uint64_t group_rows_bytes(uint32_t S) {
  return vfk::group_rows_fit(S) ? align256(4 * vfk::group_rows_words(S)) : 0;
}

// totals, rows, starts, offsets, cursor, meta; then per key of a chunk its
// key, index and answer (ob bytes)
static uint64_t group_fixed_bytes(uint32_t S) {
  return align256(4ull * S) + 2 * group_rows_bytes(S) + align256(8ull * (S + 1)) +
         align256(8ull * S) + 256;
}

static uint64_t group_bytes(uint32_t S, uint64_t chunk, uint32_t ob) {
  return group_fixed_bytes(S) + align256(8 * chunk) + align256(4 * chunk) + align256(ob * chunk);
}

int vf_query_grouped_bytes(const vf_handle *h, uint64_t n, uint64_t *bytes) {
  if (!h || h->magic != kMagic || h->kind != 0 || !bytes) return VF_EINVAL;
  *bytes = group_bytes(h->G.S, std::max<uint64_t>(1, std::min(n, kGroupChunkMax)),
                       h->is_filter ? 1 : h->cell_bytes);
  return VF_OK;
}

static int query_grouped_impl(const vf_handle *h, const uint64_t *keys, uint64_t n, void *out,
                                void *workspace, uint64_t workspace_bytes, hipStream_t stream,
                                int32_t want_filter) {
  if (!h || h->magic != kMagic || h->kind != 0 || h->is_filter != want_filter) return VF_EINVAL;
  if (n && (!keys || !out || !workspace)) return VF_EINVAL;
  if (!n) return VF_OK;
  if (((uintptr_t)keys | (uintptr_t)workspace) & 7) return VF_EINVAL;
  const uint32_t S = h->G.S;
  const uint32_t ob = want_filter ? 1 : h->cell_bytes;
  const uint64_t fixed = group_fixed_bytes(S);
  if (workspace_bytes < group_bytes(S, 1, ob)) return VF_ENOSPC;
  // a shard whose cells do not fit in LDS gains nothing from grouping: its
  // probes would miss the L2 as the plain gathers do
  if (h->packed || !vfk::query_grouped_lds_bytes(h->G, h->cells, h->cell_bytes))
    return vfk::launch_query(h->G, h->cells, h->cell_bytes, h->tseed, keys, n, out, h->ncu,
                             stream, h->packed != 0) == hipSuccess
               ? VF_OK
               : VF_EHIP;
  // the largest chunk the workspace holds (the alignment costs < 64 keys)
  uint64_t chunk = std::min((workspace_bytes - fixed) / (12 + ob), std::min(n, kGroupChunkMax));
  while (group_bytes(S, chunk, ob) > workspace_bytes) chunk--;
  uint8_t *W = (uint8_t *)workspace;
  uint32_t *counts = (uint32_t *)W;
  uint32_t *rows = (uint32_t *)(W + align256(4ull * S));
  uint32_t *starts = (uint32_t *)((uint8_t *)rows + group_rows_bytes(S));
  uint64_t *offsets = (uint64_t *)((uint8_t *)starts + group_rows_bytes(S));
  uint64_t *cursor = (uint64_t *)((uint8_t *)offsets + align256(8ull * (S + 1)));
  uint32_t *meta = (uint32_t *)((uint8_t *)cursor + align256(8ull * S));
  uint64_t *bkeys = (uint64_t *)((uint8_t *)meta + 256);
  uint32_t *bidx = (uint32_t *)((uint8_t *)bkeys + align256(8 * chunk));
  uint8_t *ans = (uint8_t *)bidx + align256(4 * chunk);
  // the per-chunk scan clears the shard totals for the next chunk
  if (vfk::group_rows_fit(S) && vfk::launch_fill_u32(counts, S, 0, stream) != hipSuccess)
    return VF_EHIP;
  // keys hashed once, while they are grouped: the grouped copy holds each
  // query's edge and fingerprint (and, in mode 2, its position) when they fit
  // a word
  uint32_t vb = 0, gb = 0;
  const bool pack = vfk::pack_fits(h->G, S, &vb);
  for (uint64_t c0 = 0; c0 < n; c0 += chunk) {
    const uint64_t cnt = std::min(chunk, n - c0);
    const uint64_t *k = keys + c0;
    uint8_t *o = (uint8_t *)out + c0 * ob;
    if (vfk::group_rows_fit(S)) {
      // answers in grouped order, then moved through LDS windows; or each
      // written straight to its position when a segment's window is too big
      const bool place = vfk::place_fits(S, cnt, ob);
      const int mode = place && vfk::pack_compact_fits(h->G, S, cnt, &gb) ? 2 : pack ? 1 : 0;
      const uint32_t w = mode == 2 ? gb : vb;
      if (vfk::launch_group_rows(k, cnt, h->G.khi, h->G.h, S, rows, counts, offsets, cursor,
                                 meta, bkeys, mode == 2 ? nullptr : bidx,
                                 place ? starts : nullptr, stream, mode, &h->G, h->tseed,
                                 w) != hipSuccess ||
          vfk::launch_query_grouped(h->G, h->cells, h->cell_bytes, h->tseed, offsets, bkeys,
                                    bidx, o, place ? ans : nullptr, w, mode, h->ncu,
                                    stream) != hipSuccess ||
          (place && vfk::launch_place_rows(rows, starts, S, cnt, ob, ans, bidx,
                                           mode == 2 ? bkeys : nullptr, o, stream) != hipSuccess))
        return VF_EHIP;
      continue;
    }
    if (vfk::launch_fill_u32(counts, S, 0, stream) != hipSuccess ||
        vfk::launch_count(k, cnt, h->G.khi, h->G.h, S, counts, h->ncu, stream) != hipSuccess ||
        vfk::launch_scan(counts, S, offsets, cursor, meta, stream) != hipSuccess ||
        vfk::launch_scatter(k, nullptr, cnt, h->G.khi, h->G.h, S, cursor, bkeys, nullptr, bidx,
                            h->ncu, stream) != hipSuccess ||
        vfk::launch_query_grouped(h->G, h->cells, h->cell_bytes, h->tseed, offsets, bkeys, bidx,
                                  o, nullptr, 0u, 0, h->ncu, stream) != hipSuccess)
      return VF_EHIP;
  }
  return VF_OK;
}

static int query_grouped_common(const vf_handle *h, const uint64_t *keys, uint64_t n, void *out,
                                void *workspace, uint64_t workspace_bytes, hipStream_t stream,
                                int32_t want_filter) {
  return guarded([&] {
    return query_grouped_impl(h, keys, n, out, workspace, workspace_bytes, stream, want_filter);
  });
}

int vf_query_grouped(const vf_handle *h, const uint64_t *keys, uint64_t n, void *out,
                     void *workspace, uint64_t workspace_bytes, hipStream_t stream) {
  return query_grouped_common(h, keys, n, out, workspace, workspace_bytes, stream, 0);
}

int vfilter_contains_grouped(const vf_handle *h, const uint64_t *keys, uint64_t n, uint8_t *out,
                             void *workspace, uint64_t workspace_bytes, hipStream_t stream) {
  return query_grouped_common(h, keys, n, out, workspace, workspace_bytes, stream, 1);
}

int vfilter_contains_grouped_noalloc(const vf_handle *h, const uint64_t *keys, uint64_t n,
                                     uint8_t *out, hipStream_t stream) {
  if (!h || h->magic != kMagic || h->kind != 0 || !h->is_filter) return VF_EINVAL;
  if (n && (!keys || !out)) return VF_EINVAL;
  void *ws = nullptr;
  uint64_t bytes = 0;
  if (vfk::noalloc_scratch(&ws, &bytes) != hipSuccess) return VF_EHIP;
  // the per-shard tables and one key must fit the static workspace
  if (bytes < group_bytes(h->G.S, 1, 1)) return VF_ENOSPC;
  return query_grouped_impl(h, keys, n, out, ws, bytes, stream, 1);
}

int vf_batch_plan(uint64_t count, const uint64_t *n, const int32_t *b, const vf_opts *o,
                  vf_sizes *out) {
  if (!out) return VF_EINVAL;
  vf_opts d;
  vf_default_opts(&d);
  BatchLayout L;
  const int rc = guarded([&] { return make_batch_layout(count, n, b, o ? *o : d, device_cus(), &L); });
  if (rc) return rc;
  out->structure_bytes = L.st_bytes;
  out->workspace_bytes = L.ws_bytes;
  out->h = 0;
  out->shard_cap = L.maxM;
  return VF_OK;
}

// Everything the host decides for one batch build: buffers, launch lists
// and launch shapes.  A prepared batch keeps it in its handle, so that the
// device work can be enqueued again and again (for instance as a captured
// graph) without host synchronization or allocation.
struct BatchRun {
  BatchLayout L;
  uint64_t count = 0;
  int ncu = 0;
  vf_opts op{};
  BatchTuning tune;
  std::vector<uint32_t> ord;
  uint64_t cls_begin[6] = {0, 0, 0, 0, 0, 0};
  struct Launch {
    uint32_t lds = 0, wmax = 0, nwg = 0;
    int32_t sigma = 0;
  } cls[4];
  uint32_t small_nwg = 0;
  vfk::BuildArgs A{};  // common arguments; keys and values are set per launch
  uint8_t *W = nullptr;
  uint32_t *work = nullptr, *overflow = nullptr, *order = nullptr, *flag = nullptr;
  vfk::FailRec *fails = nullptr;
  vfk::BatchItem *items = nullptr, *citems = nullptr;
  uint8_t *tseed = nullptr, *cells = nullptr;
};

static const uint32_t kClassBytes[4] = {1, 2, 4, 8};

// Launch lists: the instances the one-wavefront kernel takes (by the
// tuning, or by default), then those of each cell width for the peel + band
// kernel, largest first in each list; and the launch shape of each list.
static void batch_lists(BatchRun &R) {
  const uint64_t count = R.count;
  const BatchLayout &L = R.L;
  auto small = [&](uint32_t i) {
    const vfk::BatchItem &it = L.items[i];
    if (R.op.small == 2 || !vfk::small_instance(it.n, it.V)) return false;
    const int sc = size_class(it.n);
    return R.op.small == 1 || sc < 0 || !R.tune.done || R.tune.use_small[sc];
  };
  std::vector<uint32_t> idx(count);
  std::vector<int> c_of(count);
  for (uint64_t i = 0; i < count; i++) {
    idx[i] = (uint32_t)i;
    if (small((uint32_t)i)) {
      c_of[i] = 0;
    } else {
      const uint32_t cb = L.items[i].cell_bytes;
      c_of[i] = cb == 1 ? 1 : cb == 2 ? 2 : cb == 4 ? 3 : 4;
    }
  }
  std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t c) {
    return c_of[a] != c_of[c] ? c_of[a] < c_of[c] : L.items[a].n > L.items[c].n;
  });
  R.ord.assign(2 * count, 0);
  for (int c = 0; c < 6; c++) R.cls_begin[c] = 0;
  for (uint64_t i = 0; i < count; i++) {
    R.ord[2 * i] = idx[i];
    R.cls_begin[c_of[idx[i]] + 1] = i + 1;
  }
  for (int c = 1; c < 6; c++) R.cls_begin[c] = std::max(R.cls_begin[c], R.cls_begin[c - 1]);
  const uint64_t ns = R.cls_begin[1];
  R.small_nwg = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>((ns + vfk::kSmallWavesPerGroup - 1) / vfk::kSmallWavesPerGroup,
                            (uint64_t)R.ncu * (R.tune.done ? R.tune.small_groups_per_cu : 8)));
  for (int c = 0; c < 4; c++) {
    const uint64_t c0 = R.cls_begin[c + 1], c1 = R.cls_begin[c + 2];
    BatchRun::Launch &la = R.cls[c];
    la = BatchRun::Launch{};
    if (c1 == c0) continue;
    int32_t sg = 0;
    for (uint64_t i = c0; i < c1; i++) sg = std::max(sg, (int32_t)L.items[R.ord[2 * i]].sigma);
    const BuildShape shape = build_shape(sg, kClassBytes[c]);
    la.sigma = sg;
    la.lds = shape.lds_bytes;
    la.wmax = shape.wmax;
    if (R.op.max_window) la.wmax = std::min(la.wmax, std::max(8u, R.op.max_window & ~7u));
    la.nwg = (uint32_t)std::min<uint64_t>(
        std::min<uint64_t>(L.nwg, (uint64_t)shape.per_cu * R.ncu), c1 - c0);
  }
}

// Host-side plan of a batch (no device work).
static int batch_setup(BatchRun &R, uint64_t count, const uint64_t *n, const int32_t *b,
                       uint64_t seed, const vf_opts *o, void *ws, uint64_t ws_bytes, void *st,
                       uint64_t st_bytes) {
  if (!ws || !st) return VF_EINVAL;
  vf_default_opts(&R.op);
  if (o) R.op = *o;
  R.ncu = device_cus();
  if (R.ncu <= 0) return VF_EHIP;
  int rc = make_batch_layout(count, n, b, R.op, R.ncu, &R.L);
  if (rc) return rc;
  if (ws_bytes < R.L.ws_bytes || st_bytes < R.L.st_bytes) return VF_ENOSPC;
  R.count = count;
  R.tune = batch_tuning();
  const BatchLayout &L = R.L;
  R.W = (uint8_t *)ws;
  R.work = (uint32_t *)(R.W + L.o_work);
  R.fails = (vfk::FailRec *)(R.W + L.o_fails);
  R.overflow = (uint32_t *)(R.W + L.o_overflow);
  R.order = (uint32_t *)(R.W + L.o_order);
  R.citems = (vfk::BatchItem *)(R.W + L.o_check);
  R.flag = (uint32_t *)(R.W + L.o_check + sizeof(vfk::BatchItem) * count);
  uint8_t *S8 = (uint8_t *)st;
  R.items = (vfk::BatchItem *)(S8 + L.s_items);
  R.tseed = S8 + L.s_seeds;
  R.cells = S8 + L.s_cells;
  uint64_t sw[3];
  seed_words(seed, sw);
  vfk::BuildArgs &A = R.A;
  A = vfk::BuildArgs{};
  A.G.khi = sw[0];
  A.G.klo = sw[1];
  A.G.kfp = sw[2];
  A.G.h = 0;
  A.G.S = 1;
  A.G.is_filter = 0;
  A.offsets = nullptr;
  A.cells = L.packed ? R.W + L.o_tcells : R.cells;
  A.tseed = R.tseed;
  A.scratch = R.W + L.o_scratch;
  A.scratch_stride = L.scratch_stride;
  A.work = R.work;
  A.fails = R.fails;
  A.fail_cap = L.fail_cap;
  A.M = L.maxM;
  A.tmax = R.op.tmax;
  A.ring_cols = R.op.ring_cols;
  A.logcap = L.logcap;
  // the build reads the workspace descriptors (byte cells); queries read
  // the structure's (packed offsets when packed)
  A.items = R.citems;
  A.scr_V = L.maxV;
  A.scr_l = L.maxl;
  batch_lists(R);
  return VF_OK;
}

#define HIPCHK(x)                                          \
  do {                                                     \
    const hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) return hip_failed(e_, __LINE__); \
  } while (0)

// Descriptors and launch lists into the workspace; with structure, the
// descriptors queries read into the structure as well.
static int batch_upload(const BatchRun &R, hipStream_t stream, bool structure) {
  const uint64_t count = R.count;
  HIPCHK(hipMemcpyAsync(R.citems, R.L.items.data(), sizeof(vfk::BatchItem) * count,
                        hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(R.order, R.ord.data(), 8ull * count, hipMemcpyHostToDevice, stream));
  if (structure)
    HIPCHK(hipMemcpyAsync(R.items, (R.L.packed ? R.L.pitems : R.L.items).data(),
                          sizeof(vfk::BatchItem) * count, hipMemcpyHostToDevice, stream));
  return VF_OK;
}

// Kernel attributes a launch needs (dynamic LDS above the default), set
// ahead so that batch_enqueue makes no such call.
static int batch_prepare_kernels(const BatchRun &R) {
  for (int c = 0; c < 4; c++) {
    const BatchRun::Launch &la = R.cls[c];
    if (!la.nwg) continue;
    vfk::BuildArgs a = R.A;
    a.cell_bytes = kClassBytes[c];
    a.lds_bytes = la.lds;
    a.wmax = la.wmax;
    HIPCHK(vfk::prepare_build(a));
    a.lds_bytes = (vfk::kLdsBudget - 256) & ~255u;
    a.wmax = vfk::window_slots((uint32_t)la.sigma, a.lds_bytes);
    HIPCHK(vfk::prepare_build(a));
  }
  return VF_OK;
}

// The device work of a build: kernels only (no host wait, no allocation,
// no memset), so it can be captured into a graph.  With check, the values
// are checked first and a value wider than its b makes every build kernel
// end at once (the structure is not written; batch_collect reports it).
static int batch_enqueue(const BatchRun &R, const uint64_t *keys, const uint64_t *values,
                         hipStream_t stream, bool check) {
  vfk::BuildArgs A = R.A;
  A.bkeys = keys;
  A.bvals = values;
  A.abort = check ? R.flag : nullptr;
  HIPCHK(vfk::launch_fill_u32(R.flag, 1, 0, stream));
  if (check && R.L.keys)
    HIPCHK(vfk::launch_check_batch_values(R.citems, R.count, values, R.flag, stream));
  HIPCHK(vfk::launch_fill_u32(R.work, vfk::kWorkWords, 0, stream));
  if (R.cls_begin[1] > 0) {
    A.list = R.order;
    A.nlist = (uint32_t)R.cls_begin[1];
    A.nlist_dev = nullptr;
    A.overflow = nullptr;
    HIPCHK(vfk::launch_small(A, (int)R.small_nwg, stream));
  }
  for (int c = 0; c < 4; c++) {
    const BatchRun::Launch &la = R.cls[c];
    if (!la.nwg) continue;
    const uint64_t c0 = R.cls_begin[c + 1], c1 = R.cls_begin[c + 2];
    A.cell_bytes = kClassBytes[c];
    A.lds_bytes = la.lds;
    A.wmax = la.wmax;
    A.list = R.order + 2 * c0;
    A.nlist = (uint32_t)(c1 - c0);
    A.nlist_dev = nullptr;
    A.overflow = R.overflow;
    HIPCHK(vfk::launch_fill_u32(R.work + vfk::kWorkNext, 1, 0, stream));
    HIPCHK(vfk::launch_fill_u32(R.work + vfk::kWorkCap, 1, 0, stream));
    HIPCHK(vfk::launch_build(A, (int)la.nwg, stream));
    // instances whose window outgrew their share of LDS, again with a
    // whole CU's LDS; the list length is read on the device (no host wait)
    vfk::BuildArgs B = A;
    B.list = R.overflow;
    B.nlist = 0;
    B.nlist_dev = R.work + vfk::kWorkCap;
    B.overflow = nullptr;
    B.lds_bytes = (vfk::kLdsBudget - 256) & ~255u;
    B.wmax = vfk::window_slots((uint32_t)la.sigma, B.lds_bytes);
    HIPCHK(vfk::launch_fill_u32(R.work + vfk::kWorkNext, 1, 0, stream));
    HIPCHK(vfk::launch_build(B, (int)std::min<uint32_t>(la.nwg, (uint32_t)R.ncu), stream));
  }
  if (R.L.packed)
    HIPCHK(vfk::launch_pack_batch(R.citems, R.items, R.count, R.W + R.L.o_tcells, R.cells,
                                  A.abort, stream));
  return VF_OK;
}

// After the stream has passed batch_enqueue's work: the value check, the
// counters, failure record and local seeds.  Returns VF_EINVAL (failed value
// check) or a HIP error without touching *H; otherwise fills *H and returns
// the build's status.  take: move the descriptors into *H (the plan is not
// used again).
static int batch_collect(BatchRun &R, hipStream_t stream, vf_handle *H, bool take) {
  uint32_t hwork[vfk::kWorkWords];
  uint32_t hflag = 0;
  HIPCHK(hipMemcpyAsync(hwork, R.work, sizeof(hwork), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(&hflag, R.flag, 4, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (hflag) return VF_EINVAL;
  const uint32_t nf = std::min(hwork[vfk::kWorkFails], R.L.fail_cap);
  std::vector<vfk::FailRec> fr(nf);
  if (nf)
    HIPCHK(hipMemcpyAsync(fr.data(), R.fails, nf * sizeof(vfk::FailRec), hipMemcpyDeviceToHost,
                          stream));
  std::vector<uint8_t> ts(R.count);
  HIPCHK(hipMemcpyAsync(ts.data(), R.tseed, R.count, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  BatchLayout &L = R.L;
  H->magic = kMagic;
  H->kind = 1;
  H->packed = L.packed ? 1u : 0u;
  H->is_filter = 0;
  H->b = 0;
  H->h = 0;
  H->S = (uint32_t)R.count;
  H->g = Geometry{L.maxM, 0, 0, L.maxl, L.maxsigma, L.maxV};
  H->n = L.keys;
  H->cell_bytes = 0;
  H->G = R.A.G;
  H->cells = R.cells;
  H->tseed = R.tseed;
  H->ncu = R.ncu;
  H->n_fail_total = hwork[vfk::kWorkFails];
  H->relaunched = hwork[vfk::kWorkRelaunch];
  H->fails.clear();
  for (const auto &f : fr) H->fails.push_back(vf_failure{f.shard, f.attempt, f.kind, f.core_edges});
  std::sort(H->fails.begin(), H->fails.end(), [](const vf_failure &a, const vf_failure &c) {
    return a.shard != c.shard ? a.shard < c.shard : a.attempt < c.attempt;
  });
  H->failed_shards = (uint32_t)std::count(ts.begin(), ts.end(), (uint8_t)255);
  H->count = R.count;
  std::vector<vfk::BatchItem> &src = L.packed ? L.pitems : L.items;
  if (take)
    H->items = std::move(src);
  else
    H->items = src;
  H->seeds = std::move(ts);
  H->items_dev = R.items;
  if (hwork[vfk::kWorkStatus] & vfk::kStatusStalled) {
    snprintf(g_last_error, sizeof(g_last_error), "a build workgroup gave up on a wait");
    return VF_EHIP;
  }
  if (hwork[vfk::kWorkStatus] & vfk::kStatusCapacity) return VF_ECAPACITY;
  if (H->failed_shards) return VF_EFAIL;
  return VF_OK;
}

// Tuning (see vf_batch_tuning): for each size class with enough small
// instances of one-byte cells, the sampled instances are built by both
// kernels (the same cells either way) and timed; the faster builds the
// class from now on, on this device; the grid of the one-wavefront kernel
// is tuned on the largest sample.  Leaves counters and cells to be
// rebuilt.
static int batch_tune(BatchRun &R, const uint64_t *keys, const uint64_t *values,
                      hipStream_t stream) {
  const BatchLayout &L = R.L;
  BatchTuning nt;
  uint32_t *const tl = (uint32_t *)(R.W + L.o_tune);
  PhaseEvents te;
  int biggest = -1;
  uint32_t biggest_n = 0;
  std::vector<uint32_t> lists[4];
  for (uint64_t i = 0; i < R.count; i++) {
    const vfk::BatchItem &it = L.items[i];
    const int sc = size_class(it.n);
    if (sc >= 0 && it.cell_bytes == 1 && vfk::small_instance(it.n, it.V) &&
        lists[sc].size() < 2 * kTuneSample) {
      lists[sc].push_back((uint32_t)i);
      lists[sc].push_back(0);
    }
  }
  vfk::BuildArgs T = R.A;
  T.bkeys = keys;
  T.bvals = values;
  T.abort = nullptr;
  T.nlist_dev = nullptr;
  T.overflow = R.overflow;
  T.cell_bytes = 1;
  T.list = tl;
  HIPCHK(vfk::launch_fill_u32(R.work, vfk::kWorkWords, 0, stream));
  bool any = false;
  for (int sc = 0; sc < 4; sc++) {
    const uint32_t ns = (uint32_t)(lists[sc].size() / 2);
    nt.sampled[sc] = ns;
    if (ns < 256) continue;
    any = true;
    HIPCHK(hipMemcpyAsync(tl, lists[sc].data(), 8ull * ns, hipMemcpyHostToDevice, stream));
    T.nlist = ns;
    const uint64_t snwg = std::max<uint64_t>(1, std::min<uint64_t>(
        (ns + vfk::kSmallWavesPerGroup - 1) / vfk::kSmallWavesPerGroup,
        (uint64_t)R.ncu * nt.small_groups_per_cu));
    te.record(0, stream);
    HIPCHK(vfk::launch_small(T, (int)snwg, stream));
    te.record(1, stream);
    HIPCHK(hipStreamSynchronize(stream));
    nt.ms_small[sc] = te.between(0, 1);
    int32_t sg = 0;
    for (uint32_t k = 0; k < ns; k++) sg = std::max(sg, (int32_t)L.items[lists[sc][2 * k]].sigma);
    const BuildShape shape = build_shape(sg, 1);
    T.lds_bytes = shape.lds_bytes;
    T.wmax = shape.wmax;
    HIPCHK(vfk::launch_fill_u32(R.work + vfk::kWorkNext, 1, 0, stream));
    te.record(2, stream);
    HIPCHK(vfk::launch_build(T, (int)std::min<uint64_t>(ns, (uint64_t)shape.per_cu * R.ncu),
                             stream));
    te.record(3, stream);
    HIPCHK(hipStreamSynchronize(stream));
    nt.ms_band[sc] = te.between(2, 3);
    nt.use_small[sc] = nt.ms_small[sc] >= 0 && nt.ms_small[sc] <= nt.ms_band[sc];
    if (ns > biggest_n) {
      biggest_n = ns;
      biggest = sc;
    }
  }
  if (!any) return VF_OK;
  // the grid of the one-wavefront kernel, on the largest sample
  HIPCHK(hipMemcpyAsync(tl, lists[biggest].data(), 8ull * biggest_n, hipMemcpyHostToDevice,
                        stream));
  T.nlist = biggest_n;
  float best = -1.f;
  for (uint32_t per_cu : {2u, 4u, 8u, 16u}) {
    const uint64_t nwg = std::max<uint64_t>(1, std::min<uint64_t>(
        (biggest_n + vfk::kSmallWavesPerGroup - 1) / vfk::kSmallWavesPerGroup,
        (uint64_t)R.ncu * per_cu));
    te.record(0, stream);
    HIPCHK(vfk::launch_small(T, (int)nwg, stream));
    te.record(1, stream);
    HIPCHK(hipStreamSynchronize(stream));
    const float ms = te.between(0, 1);
    if (best < 0 || ms < best) {
      best = ms;
      nt.small_groups_per_cu = per_cu;
    }
  }
  nt.done = true;
  set_batch_tuning(nt);
  R.tune = nt;
  batch_lists(R);
  HIPCHK(hipMemcpyAsync(R.order, R.ord.data(), 8ull * R.count, hipMemcpyHostToDevice, stream));
  return VF_OK;
}

static int batch_build(const uint64_t *keys, const uint64_t *values, uint64_t count,
                       const uint64_t *n, const int32_t *b, uint64_t seed, const vf_opts *o,
                       void *ws, uint64_t ws_bytes, void *st, uint64_t st_bytes,
                       hipStream_t stream, vf_handle **handle) {
  if (!handle) return VF_EINVAL;
  BatchRun R;
  int rc = batch_setup(R, count, n, b, seed, o, ws, ws_bytes, st, st_bytes);
  if (rc) return rc;
  if (R.L.keys && (!keys || !values)) return VF_EINVAL;
  PhaseEvents pe;
  pe.record(0, stream);
  rc = batch_upload(R, stream, false);
  if (rc) return rc;
  // Problem 1 stores b-bit values: a value with a higher bit fails the
  // call before the structure is written
  if (R.L.keys) {
    uint32_t hflag = 0;
    HIPCHK(vfk::launch_fill_u32(R.flag, 1, 0, stream));
    HIPCHK(vfk::launch_check_batch_values(R.citems, count, values, R.flag, stream));
    HIPCHK(hipMemcpyAsync(&hflag, R.flag, 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (hflag) return VF_EINVAL;
  }
  HIPCHK(hipMemcpyAsync(R.items, (R.L.packed ? R.L.pitems : R.L.items).data(),
                        sizeof(vfk::BatchItem) * count, hipMemcpyHostToDevice, stream));
  pe.record(1, stream);
  if (!R.tune.done && R.op.small == 0) {
    rc = batch_tune(R, keys, values, stream);
    if (rc) return rc;
  }
  pe.record(2, stream);
  rc = batch_enqueue(R, keys, values, stream, false);
  if (rc) return rc;
  pe.record(3, stream);
  vf_handle *H = new (std::nothrow) vf_handle();
  if (!H) return VF_ENOMEM;
  H->seed = seed;
  rc = batch_collect(R, stream, H, true);
  if (H->magic != kMagic) {  // nothing was built
    delete H;
    return rc;
  }
  H->ms[0] = pe.between(0, 1);
  H->ms[1] = 0.f;
  H->ms[2] = pe.between(2, 3);
  *handle = H;
  return rc;
}
#undef HIPCHK

int vf_batch_build(const uint64_t *keys, const uint64_t *values, uint64_t count,
                   const uint64_t *n, const int32_t *b, uint64_t seed, const vf_opts *o,
                   void *ws, uint64_t ws_bytes, void *st, uint64_t st_bytes,
                   hipStream_t stream, vf_handle **handle) {
  return guarded([&] {
    return batch_build(keys, values, count, n, b, seed, o, ws, ws_bytes, st, st_bytes, stream,
                       handle);
  });
}

int vf_batch_prepare(uint64_t count, const uint64_t *n, const int32_t *b, uint64_t seed,
                     const vf_opts *o, void *ws, uint64_t ws_bytes, void *st, uint64_t st_bytes,
                     hipStream_t stream, vf_handle **handle) {
  return guarded([&]() -> int {
    if (!handle) return VF_EINVAL;
    auto R = std::make_shared<BatchRun>();
    int rc = batch_setup(*R, count, n, b, seed, o, ws, ws_bytes, st, st_bytes);
    if (rc) return rc;
    rc = batch_prepare_kernels(*R);
    if (rc) return rc;
    rc = batch_upload(*R, stream, true);
    if (rc) return rc;
    if (hipStreamSynchronize(stream) != hipSuccess) return VF_EHIP;
    vf_handle *H = new (std::nothrow) vf_handle();
    if (!H) return VF_ENOMEM;
    H->magic = kMagic;
    H->kind = 2;
    H->seed = seed;
    H->count = count;
    H->run = std::move(R);
    *handle = H;
    return VF_OK;
  });
}

int vf_batch_launch(vf_handle *h, const uint64_t *keys, const uint64_t *values,
                    hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h || h->magic != kMagic || !h->run) return VF_EINVAL;
    const BatchRun &R = *h->run;
    if (R.L.keys && (!keys || !values)) return VF_EINVAL;
    return batch_enqueue(R, keys, values, stream, true);
  });
}

int vf_batch_finish(vf_handle *h, hipStream_t stream) {
  return guarded([&]() -> int {
    if (!h || h->magic != kMagic || !h->run) return VF_EINVAL;
    return batch_collect(*h->run, stream, h, false);
  });
}

static_assert(VF_STAGE_CLOCK_WORDS == vfk::kClkWGs * vfk::kClkSlots, "stage clock layout");

int vf_stage_clocks(uint64_t *out, uint64_t words, int32_t reset) {
  if (!reset && (!out || words < VF_STAGE_CLOCK_WORDS)) return VF_EINVAL;
  const hipError_t e = vfk::stage_clocks(out, reset);
  if (e == hipErrorNotSupported) return VF_EINVAL;
  return e == hipSuccess ? VF_OK : hip_failed(e, __LINE__);
}

int vf_batch_tuning(vf_batch_tuning_t *out) {
  if (!out) return VF_EINVAL;
  const BatchTuning t = batch_tuning();
  out->tuned = t.done ? 1 : 0;
  for (int c = 0; c < 4; c++) {
    out->max_keys[c] = kClassKeys[c];
    out->use_small[c] = t.use_small[c] ? 1 : 0;
    out->ms_small[c] = t.ms_small[c];
    out->ms_band[c] = t.ms_band[c];
    out->sampled[c] = t.sampled[c];
  }
  out->small_groups_per_cu = t.small_groups_per_cu;
  return VF_OK;
}

int vf_batch_query(const vf_handle *h, const uint32_t *inst, const uint64_t *keys, uint64_t nq,
                   uint64_t *out, hipStream_t stream) {
  if (!h || h->magic != kMagic || h->kind != 1) return VF_EINVAL;
  if (nq && (!inst || !keys || !out)) return VF_EINVAL;
  if (vfk::launch_query_batch(h->G, h->items_dev, h->count, (const uint8_t *)h->cells, h->tseed,
                              inst, keys, nq, out, h->ncu, stream, h->packed != 0) != hipSuccess)
    return VF_EHIP;
  return VF_OK;
}

int vf_batch_item(const vf_handle *h, uint64_t i, vf_batch_item_t *out) {
  if (!h || h->magic != kMagic || h->kind != 1 || !out || i >= h->count) return VF_EINVAL;
  const vfk::BatchItem &it = h->items[i];
  out->n = it.n;
  out->b = (int32_t)it.b;
  out->c_num = it.c_num;
  out->c_den = it.c_den;
  out->sigma = (int32_t)it.sigma;
  out->l = it.l;
  out->V = it.V;
  out->cell_bytes = it.cell_bytes;
  out->local_seed = h->seeds[i];
  out->cells = (const uint8_t *)h->cells + it.cell_off;
  out->packed = h->packed;
  return VF_OK;
}

int vf_info(const vf_handle *h, vf_info_t *out) {
  if (!h || h->magic != kMagic || !out) return VF_EINVAL;
  out->is_filter = h->is_filter;
  out->b = h->b;
  out->h = h->h;
  out->S = h->S;
  out->M = h->g.M;
  out->c_num = h->g.c_num;
  out->c_den = h->g.c_den;
  out->sigma = h->g.sigma;
  out->l = h->g.l;
  out->V = h->g.V;
  out->n = h->n;
  out->seed = h->seed;
  out->cell_bytes = h->cell_bytes;
  out->failed_shards = h->failed_shards;
  out->n_failures = h->n_fail_total;
  out->space_bits = (uint64_t)h->S * h->g.V * (uint64_t)h->b;
  if (h->kind == 1) {
    out->space_bits = 0;
    for (const auto &it : h->items) out->space_bits += it.V * (uint64_t)it.b;
  }
  out->cells = h->cells;
  out->local_seeds = h->tseed;
  out->ms_count = h->ms[0];
  out->ms_scatter = h->ms[1];
  out->ms_build = h->ms[2];
  out->relaunched_shards = h->relaunched;
  out->mwhc = (int32_t)h->g.mwhc;
  out->packed = h->packed;
  return VF_OK;
}

int vf_failures(const vf_handle *h, vf_failure *out, uint32_t cap, uint32_t *count) {
  if (!h || h->magic != kMagic || !count || (cap && !out)) return VF_EINVAL;
  *count = h->n_fail_total;
  const uint32_t k = std::min<uint32_t>(cap, (uint32_t)h->fails.size());
  for (uint32_t i = 0; i < k; i++) out[i] = h->fails[i];
  return VF_OK;
}

void vf_free(vf_handle *h) {
  if (h && h->magic == kMagic) {
    h->magic = 0;
    delete h;
  }
}

}  // extern "C"
