// C-ABI layer of libpss: argument checks, launch planning, workspace layout
// and the launch sequence of the sort (see include/pss.h for the contract).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pss.h"
#include "pss_internal.hpp"

struct pss_prof_rec {
  const char *name;   // kernel family
  hipEvent_t begin, end;
  uint64_t bytes;     // algorithmic HBM bytes of this launch
};

struct pss_ctx {
  int device = 0;
  std::string last_error;
  bool profiling = false;
  std::string profile_only;  // kernel family timed while profiling ("" = all)
  pss_merge_method merge_method = PSS_MERGE_PAIRWISE;
  std::vector<pss_prof_rec> recs;
  std::vector<hipEvent_t> pool;  // events ready for reuse
};

namespace {

thread_local std::string g_thread_error;

pss_status fail(const pss_ctx *ctx, pss_status s, const std::string &msg) {
  if (ctx) const_cast<pss_ctx *>(ctx)->last_error = msg;
  g_thread_error = msg;
  return s;
}

pss_status hip_fail(const pss_ctx *ctx, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return fail(ctx, PSS_ERR_HIP, m);
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Largest table (rows x fan entries of uint32) the library allocates.
constexpr uint64_t kMaxTableEntries = (uint64_t)1 << 28;

// Merge passes that sort every segment of seg_len keys, starting from sorted
// tiles of `tile` keys: the number of doublings needed is split as evenly as
// possible over passes of at most 2^max_fan_log2 runs each, merged in
// partitions of `part` keys.
using PassList = pss::FixedVec<pss::RunGeom, pss::kMaxPlanPasses>;
using KeyBufs = pss::FixedVec<void *, pss::kMaxPlanPasses + 1>;
using ValBufs = pss::FixedVec<uint32_t *, pss::kMaxPlanPasses + 1>;

PassList plan_segment_passes(uint64_t n, uint64_t seg_len, uint32_t tile, uint32_t part,
                             int max_fan_log2) {
  PassList passes;
  if (n == 0 || seg_len == 0) return passes;
  const uint64_t tiles = ceil_div(seg_len, tile);
  int bits = 0;
  while (((uint64_t)1 << bits) < tiles) ++bits;
  if (bits == 0) return passes;
  const int npass = (bits + max_fan_log2 - 1) / max_fan_log2;
  const uint64_t nseg = ceil_div(n, seg_len);
  uint64_t run = tile;
  for (int q = 0; q < npass; ++q) {
    const int b = bits / npass + (q < bits % npass ? 1 : 0);
    pss::RunGeom g{};
    g.n = n;
    g.seg_len = seg_len;
    g.run_len = run;
    g.fan = 1u << b;
    g.group_len = std::min<uint64_t>((uint64_t)g.fan * run, seg_len);
    g.groups_per_seg = ceil_div(seg_len, g.group_len);
    g.n_groups = nseg * g.groups_per_seg;
    g.part_len = part;
    g.rows_per_group = (uint32_t)ceil_div(g.group_len, g.part_len) + 1;
    g.paper = 0;
    passes.push_back(g);
    run = std::min<uint64_t>((uint64_t)g.fan * run, seg_len);
  }
  return passes;
}

struct Plan {
  bool paper = false;
  bool kv = false;
  int kb = 8;
  uint64_t n = 0;
  uint32_t tile = pss::kTile;         // keys per tile of the tile sort
  uint32_t part = pss::kPart;         // keys per partition of the segment passes
  uint64_t seg_len = 0;               // segment sorted by tile sort + passes
  PassList passes;                    // merge passes inside each segment
  pss::RunGeom top{};                 // paper mode: the cross-block merge
  // paper mode with at most kMaxSampledFan blocks of at least 2^16 keys: the
  // last block pass leaves every kSample-th key of each block, and the
  // partition search starts from their merge (geometry top_gs)
  bool top_sampled = false;
  pss::RunGeom top_gs{};
  uint64_t table_entries = 0;
  // merged-sample index used by the splitter search of every segment pass
  uint64_t n_samples = 0, sample_table_entries = 0, prefix_entries = 0;
  // workspace layout (byte offsets)
  size_t off_keys0 = 0, off_keys1 = 0, off_vals0 = 0, off_vals1 = 0;
  size_t off_table = 0, off_sizes = 0, off_offsets = 0;
  size_t off_samples = 0, off_skeys = 0, off_sruns = 0, off_stable = 0, off_prefix = 0;
  size_t total = 0;
};

pss_status make_plan(pss_key_t key, pss_val_t val, uint64_t n, uint32_t n_blocks,
                     uint32_t n_parts, Plan *p, std::string *err) {
  p->kv = val == PSS_VAL_U32;
  p->kb = pss::key_bytes((int)key);
  p->n = n;
  p->paper = n_blocks > 0;
  p->tile = p->kv ? pss::kTileKV : pss::kTile;
  p->part = p->kv ? pss::kPartKV : pss::kPart;
  const int max_fan_log2 = p->kv ? pss::kMaxFanLog2KV : pss::kMaxFanLog2;
  if (!p->paper) {
    p->seg_len = n;
    p->passes = plan_segment_passes(n, n, p->tile, p->part, max_fan_log2);
  } else {
    const uint64_t L = n ? ceil_div(n, n_blocks) : 0;
    p->seg_len = L;
    p->passes = plan_segment_passes(n, L, p->tile, p->part, max_fan_log2);
    pss::RunGeom &t = p->top;
    t.n = n;
    t.seg_len = n;
    t.run_len = L ? L : 1;
    t.fan = n_blocks;
    t.group_len = n;
    t.groups_per_seg = 1;
    t.n_groups = 1;
    t.part_len = pss::kPart;
    t.paper = 1;
    t.n_parts = n_parts;
    t.sub_per_part = (uint32_t)std::max<uint64_t>(1, ceil_div(ceil_div(n, n_parts), pss::kPart));
    t.rows_per_group = 0;
    const uint64_t entries = t.total_rows() * (uint64_t)t.fan;
    if (entries > kMaxTableEntries) {
      *err = "n_blocks * n_parts too large for the library's split table";
      return PSS_ERR_UNSUPPORTED;
    }
    p->table_entries = entries;
    // (blocks shorter than 2^16 keys leave too few levels to skip to pay for
    // the two extra launches)
    if (!p->passes.empty() && n_blocks <= pss::kMaxSampledFan && L >= ((uint64_t)1 << 16)) {
      // blocks' samples as one group of n_blocks runs of L / kSample samples
      // (the last non-empty block's share is its own length / kSample)
      pss::RunGeom &gs = p->top_gs;
      const uint64_t rs = L >> pss::kSampleLog2;
      const uint64_t nonempty = ceil_div(n, L);
      const uint64_t last = n - (nonempty - 1) * L;
      gs.n = (nonempty - 1) * rs + (last >> pss::kSampleLog2);
      gs.seg_len = gs.n;
      gs.run_len = rs;
      gs.fan = n_blocks;
      gs.group_len = gs.n;
      gs.groups_per_seg = 1;
      gs.n_groups = 1;
      gs.part_len = pss::kPart;
      gs.rows_per_group = (uint32_t)ceil_div(gs.n, pss::kPart) + 1;
      gs.paper = 0;
      p->top_sampled = true;
      p->n_samples = std::max<uint64_t>(p->n_samples, gs.n);
      p->sample_table_entries = gs.total_rows() * (uint64_t)gs.fan;
      p->prefix_entries = gs.total_parts() * (uint64_t)(pss::kPart / pss::kChunk) * gs.fan;
    }
  }
  for (const auto &g : p->passes) {
    p->table_entries = std::max<uint64_t>(p->table_entries, g.total_rows() * (uint64_t)g.fan);
    const pss::RunGeom gs = pss::sample_geom(g);
    p->n_samples = std::max<uint64_t>(p->n_samples, gs.n);
    p->sample_table_entries =
        std::max<uint64_t>(p->sample_table_entries, gs.total_rows() * (uint64_t)gs.fan);
    p->prefix_entries = std::max<uint64_t>(
        p->prefix_entries, gs.total_parts() * (uint64_t)(pss::kPart / pss::kChunk) * gs.fan);
  }

  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  p->off_keys0 = take(n * (size_t)p->kb);
  p->off_keys1 = p->paper ? take(n * (size_t)p->kb) : 0;
  if (p->kv) {
    p->off_vals0 = take(n * sizeof(uint32_t));
    p->off_vals1 = p->paper ? take(n * sizeof(uint32_t)) : 0;
  }
  p->off_table = take(p->table_entries * sizeof(uint32_t));
  if (!p->passes.empty()) {
    p->off_samples = take(p->n_samples * (size_t)p->kb);
    p->off_skeys = take(p->n_samples * (size_t)p->kb);
    p->off_sruns = take(p->n_samples * sizeof(uint32_t));
    p->off_stable = take(p->sample_table_entries * sizeof(uint32_t));
    p->off_prefix = take(p->prefix_entries * sizeof(uint32_t));
  }
  if (p->paper) {
    p->off_sizes = take((size_t)n_parts * sizeof(uint64_t));
    p->off_offsets = take(((size_t)n_parts + 1) * sizeof(uint64_t));
  }
  p->total = off;
  return PSS_OK;
}

bool overlaps(const void *a, size_t alen, const void *b, size_t blen) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return alen && blen && x < y + blen && y < x + alen;
}

pss_status validate(const pss_ctx *ctx, pss_key_t key, pss_val_t val, const void *keys_in,
                    const void *keys_out, const void *vals_in, const void *vals_out, uint64_t n,
                    uint32_t n_blocks, uint32_t n_parts, size_t ws_bytes, Plan *plan) {
  if ((int)key < 0 || (int)key > 5) return fail(ctx, PSS_ERR_INVALID, "unknown key type");
  if ((int)val != PSS_VAL_NONE && (int)val != PSS_VAL_U32)
    return fail(ctx, PSS_ERR_INVALID, "unknown value type");
  if ((n_blocks == 0) != (n_parts == 0))
    return fail(ctx, PSS_ERR_INVALID, "n_blocks and n_parts must both be 0 (auto) or both > 0");
  if (n > PSS_MAX_KEYS) return fail(ctx, PSS_ERR_UNSUPPORTED, "n >= 2^31 is not supported");
  if (n_blocks > PSS_MAX_BLOCKS) return fail(ctx, PSS_ERR_UNSUPPORTED, "n_blocks > 2048");
  if (n_parts > PSS_MAX_PARTS) return fail(ctx, PSS_ERR_UNSUPPORTED, "n_parts > 4194304");
  const size_t kb = (size_t)pss::key_bytes((int)key);
  if (n > 0) {
    if (!keys_in || !keys_out) return fail(ctx, PSS_ERR_INVALID, "null key pointer");
    if (overlaps(keys_in, n * kb, keys_out, n * kb))
      return fail(ctx, PSS_ERR_INVALID, "keys_in and keys_out overlap (the sort is out of place)");
    if (val == PSS_VAL_U32) {
      if (!vals_in || !vals_out) return fail(ctx, PSS_ERR_INVALID, "null value pointer");
      if (overlaps(vals_in, n * 4, vals_out, n * 4))
        return fail(ctx, PSS_ERR_INVALID, "vals_in and vals_out overlap");
      if (overlaps(keys_out, n * kb, vals_out, n * 4) || overlaps(keys_in, n * kb, vals_out, n * 4) ||
          overlaps(vals_in, n * 4, keys_out, n * kb))
        return fail(ctx, PSS_ERR_INVALID, "key and value arrays overlap");
    }
  }
  std::string err;
  const pss_status ps = make_plan(key, val, n, n_blocks, n_parts, plan, &err);
  if (ps != PSS_OK) return fail(ctx, ps, err);
  if (ws_bytes != SIZE_MAX && ws_bytes < plan->total) {
    char m[160];
    snprintf(m, sizeof m, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
             plan->total);
    return fail(ctx, PSS_ERR_WORKSPACE, m);
  }
  return PSS_OK;
}

#define PSS_TRY(expr, what)                       \
  do {                                            \
    const hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

// Queued device work (kernel launches, async copies and fills): as PSS_TRY,
// and the operation pss_debug_inject armed fails instead of being queued.
#define PSS_LAUNCH(expr, what)                                                         \
  do {                                                                                 \
    if (pss::inject_fault(pss::kInjectLaunch))                                         \
      return fail(ctx, PSS_ERR_HIP, std::string(what) + ": injected fault (pss_debug_inject)"); \
    PSS_TRY(expr, what);                                                               \
  } while (0)

// Optional per-launch timing: when profiling is on, every kernel launch (or
// every launch of the family chosen by pss_profile_only) is bracketed by two
// events recorded on the launch stream.
hipEvent_t take_event(pss_ctx *ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct LaunchTimer {
  pss_ctx *ctx;
  hipStream_t s;
  pss_prof_rec rec{};
  bool on;
  LaunchTimer(pss_ctx *c, const char *name, uint64_t bytes, hipStream_t st)
      : ctx(c), s(st),
        on(c && c->profiling && (c->profile_only.empty() || c->profile_only == name)) {
    if (!on) return;
    rec.name = name;
    rec.bytes = bytes;
    rec.begin = take_event(ctx);
    rec.end = take_event(ctx);
    if (!rec.begin || !rec.end) {
      on = false;
      return;
    }
    hipEventRecord(rec.begin, s);
  }
  ~LaunchTimer() {
    if (!on) return;
    hipEventRecord(rec.end, s);
    ctx->recs.push_back(rec);
  }
};

// Tile sort plus the merge passes of every segment.  bufs[q] receives the
// output of pass q (bufs[0] the tile sort); values likewise.  Each pass first
// merges the regular samples its input runs left (a 1/kSample-size merge that
// records run ids and per-run prefix counts), then searches the exact
// splitters starting from those samples, then merges the data.
// last_samples: when set, the last pass also leaves every kSample-th key of
// each output run there (for a search over the sorted segments that follows).
pss_status run_segment_sort(pss_ctx *ctx, const Plan &p, int kt, const void *keys_in,
                            const uint32_t *vals_in, void *const *kbuf, uint32_t *const *vbuf,
                            int final_last, char *w, hipStream_t s,
                            void *last_samples = nullptr) {
  const size_t P = p.passes.size();
  const uint64_t sweep = 2 * p.n * ((uint64_t)p.kb + (p.kv ? 4 : 0));  // read + write all
  uint32_t *table = (uint32_t *)(w + p.off_table);
  void *samples = P ? (void *)(w + p.off_samples) : nullptr;
  void *skeys = w + p.off_skeys;
  uint32_t *sruns = (uint32_t *)(w + p.off_sruns);
  uint32_t *stable = (uint32_t *)(w + p.off_stable);
  uint32_t *prefix = (uint32_t *)(w + p.off_prefix);
  {
    LaunchTimer t(ctx, "tile_sort", sweep, s);
    PSS_LAUNCH(pss::launch_tile_sort(kt, p.kv, keys_in, vals_in, kbuf[0], vbuf[0], p.n, p.seg_len,
                                  p.tile, final_last && P == 0, samples, s),
            "tile sort launch");
  }
  for (size_t q = 1; q <= P; ++q) {
    const pss::RunGeom &g = p.passes[q - 1];
    const pss::RunGeom gs = pss::sample_geom(g);
    const uint64_t sbytes = gs.n * (uint64_t)p.kb;
    {
      LaunchTimer t(ctx, "sample_split_search", gs.total_rows() * gs.fan * 4, s);
      PSS_LAUNCH(pss::launch_corank(kt, samples, gs, stable, nullptr, nullptr, s),
              "sample split search launch");
    }
    {
      LaunchTimer t(ctx, "sample_merge", 2 * sbytes + gs.n * 4, s);
      PSS_LAUNCH(pss::launch_merge(kt, 2, samples, nullptr, skeys, sruns, gs, stable, nullptr, 0,
                                nullptr, prefix, s),
              "sample merge launch");
    }
    {
      LaunchTimer t(ctx, "split_search", g.total_rows() * g.fan * 4, s);
      PSS_LAUNCH(pss::launch_corank_sampled(kt, kbuf[q - 1], g, table, sruns, prefix, s),
              "split search launch");
    }
    {
      LaunchTimer t(ctx, "merge", sweep, s);
      PSS_LAUNCH(pss::launch_merge(kt, p.kv ? 1 : 0, kbuf[q - 1], vbuf[q - 1], kbuf[q], vbuf[q], g,
                                table, nullptr, final_last && q == P,
                                q < P ? samples : last_samples, nullptr, s),
              "merge launch");
    }
  }
  return PSS_OK;
}

// Step 1 of the paper's single level (the blocks sorted into kbuf[P], which
// the caller lays out), leaving the blocks' samples when the partition search
// will start from them.
pss_status run_paper_blocks(pss_ctx *ctx, const Plan &p, int kt, const void *keys_in,
                            const uint32_t *vals_in, void *const *kbuf, uint32_t *const *vbuf,
                            char *w, hipStream_t s) {
  return run_segment_sort(ctx, p, kt, keys_in, vals_in, kbuf, vbuf, 0, w, s,
                          p.top_sampled ? (void *)(w + p.off_samples) : nullptr);
}

// Steps 2-3 of the paper's single level: co-rank rows of geometry top (the
// paper's partitions, or data-dependent ones) over the sorted blocks.  With
// the blocks' samples the search starts at level kSampleLog2 from their merge
// (sample co-rank, sample merge with run ids and prefix counts); otherwise it
// runs every level.
pss_status paper_partition_search(pss_ctx *ctx, const Plan &p, int kt, const void *blocks,
                                  const pss::RunGeom &top, uint32_t *table, char *w,
                                  hipStream_t s) {
  if (!p.top_sampled) {
    LaunchTimer t(ctx, "partition_search", top.total_rows() * top.fan * 4, s);
    PSS_LAUNCH(pss::launch_corank(kt, blocks, top, table, nullptr, nullptr, s), "splitter launch");
    return PSS_OK;
  }
  const pss::RunGeom &gs = p.top_gs;
  void *samples = w + p.off_samples;
  void *skeys = w + p.off_skeys;
  uint32_t *sruns = (uint32_t *)(w + p.off_sruns);
  uint32_t *stable = (uint32_t *)(w + p.off_stable);
  uint32_t *prefix = (uint32_t *)(w + p.off_prefix);
  {
    LaunchTimer t(ctx, "partition_sample_search", gs.total_rows() * gs.fan * 4, s);
    PSS_LAUNCH(pss::launch_corank(kt, samples, gs, stable, nullptr, nullptr, s),
            "sample split search launch");
  }
  {
    LaunchTimer t(ctx, "partition_sample_merge", 2 * gs.n * (uint64_t)p.kb + gs.n * 4, s);
    PSS_LAUNCH(pss::launch_merge(kt, 2, samples, nullptr, skeys, sruns, gs, stable, nullptr, 0,
                              nullptr, prefix, s),
            "sample merge launch");
  }
  {
    LaunchTimer t(ctx, "partition_search", top.total_rows() * top.fan * 4, s);
    PSS_LAUNCH(pss::launch_corank_sampled(kt, blocks, top, table, sruns, prefix, s, nullptr, &gs),
            "splitter launch");
  }
  return PSS_OK;
}

// Automatic-plan sort of p.n keys (and values) from keys_in into keys_out:
// tile sort and merge passes alternate between keys_out and the workspace so
// that the last pass lands in keys_out.
pss_status run_auto_sort(pss_ctx *ctx, const Plan &p, int kt, const void *keys_in,
                         const uint32_t *vals_in, void *keys_out, uint32_t *vals_out, char *w,
                         hipStream_t s) {
  const size_t P = p.passes.size();
  KeyBufs kb;
  ValBufs vb;
  for (size_t q = 0; q <= P; ++q) {
    kb.push_back(nullptr);
    vb.push_back(nullptr);
  }
  for (size_t q = 0; q <= P; ++q) {
    const bool to_out = ((P - q) % 2) == 0;
    kb[q] = to_out ? keys_out : (void *)(w + p.off_keys0);
    if (p.kv) vb[q] = to_out ? vals_out : (uint32_t *)(w + p.off_vals0);
  }
  return run_segment_sort(ctx, p, kt, keys_in, vals_in, kb.data(), vb.data(), 1, w, s);
}

// Regular-sampling (PSRS) variant of the paper's single level: the same block
// sort, then n_P - 1 regular samples per block, their sort (an automatic-plan
// sort of the mapped keys as unsigned integers), pivots at regular intervals
// of the sorted samples and a value partition of every block, whose sizes
// follow the data.  Each partition is merged in chunks of at most kPart keys,
// cut by co-rank rows at the chunk boundaries.
constexpr uint64_t kMaxPsrsSamples = (uint64_t)1 << 27;

struct PsrsPlan {
  Plan base;           // paper-mode plan: block sort and workspace buffers
  Plan smp;            // automatic plan of the sample sort
  pss::RunGeom top{};  // merge geometry with data-dependent partitions
  uint64_t ns = 0;     // number of samples
  int skt = 0;         // key type the samples are sorted as
  size_t off_table = 0, off_samples = 0, off_ssorted = 0, off_sws = 0;
  size_t off_bounds = 0, off_chunks = 0, off_cprefix = 0, total = 0;
};

pss_status make_psrs_plan(pss_key_t key, pss_val_t val, uint64_t n, uint32_t n_blocks,
                          uint32_t n_parts, PsrsPlan *pp, std::string *err) {
  pss_status st = make_plan(key, val, n, n_blocks, n_parts, &pp->base, err);
  if (st != PSS_OK) return st;
  const uint64_t L = pp->base.seg_len;
  pp->ns = (n && n_parts > 1) ? ceil_div(n, L) * (uint64_t)(n_parts - 1) : 0;
  if (pp->ns > kMaxPsrsSamples) {
    *err = "more than 2^27 regular samples (non-empty blocks * (n_parts - 1))";
    return PSS_ERR_UNSUPPORTED;
  }
  pss::RunGeom &t = pp->top;
  t = pp->base.top;
  t.sub_per_part = 1;
  t.chunk_bound = ceil_div(n, pss::kPart) + n_parts;
  const uint64_t entries = (t.chunk_bound + 1) * (uint64_t)t.fan;
  if (entries > kMaxTableEntries) {
    *err = "n_blocks * (n / 8192 + n_parts) too large for the library's split table";
    return PSS_ERR_UNSUPPORTED;
  }
  pp->skt = pss::key_bytes((int)key) == 8 ? PSS_U64 : PSS_U32;
  if (pp->ns) {
    st = make_plan((pss_key_t)pp->skt, PSS_VAL_NONE, pp->ns, 0, 0, &pp->smp, err);
    if (st != PSS_OK) return st;
  }
  const size_t kb = (size_t)pss::key_bytes((int)key);
  size_t off = pp->base.total;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  pp->off_table = take(entries * sizeof(uint32_t));
  pp->off_samples = take(pp->ns * kb);
  pp->off_ssorted = take(pp->ns * kb);
  pp->off_sws = take(pp->ns ? pp->smp.total : 0);
  pp->off_bounds = take(((size_t)n_parts + 1) * sizeof(uint64_t));
  pp->off_chunks = take((size_t)n_parts * sizeof(uint64_t));
  pp->off_cprefix = take(((size_t)n_parts + 1) * sizeof(uint64_t));
  pp->total = off;
  return PSS_OK;
}

// Outputs of the PSRS steps (device pointers, each optional).
struct PsrsOut {
  void *sorted_blocks = nullptr;
  void *samples = nullptr;
  void *pivots = nullptr;
  uint64_t *split = nullptr;
  uint64_t *offsets = nullptr;
  uint64_t *sizes = nullptr;
};

// Steps 1-3 with regular-sampling pivots, then (merge = true) step 4 into
// keys_out / vals_out.
pss_status run_psrs(pss_ctx *ctx, const PsrsPlan &pp, int kt, const void *keys_in,
                    const uint32_t *vals_in, void *keys_out, uint32_t *vals_out,
                    const PsrsOut &o, bool merge, char *w, hipStream_t s) {
  const Plan &p = pp.base;
  const size_t P = p.passes.size();
  KeyBufs kbuf;
  ValBufs vbuf;
  for (size_t q = 0; q <= P; ++q) {
    kbuf.push_back(nullptr);
    vbuf.push_back(nullptr);
  }
  for (size_t q = 0; q <= P; ++q) {
    const bool even = ((P - q) % 2) == 0;
    kbuf[q] = even ? (void *)(w + p.off_keys0) : (void *)(w + p.off_keys1);
    if (p.kv) vbuf[q] = even ? (uint32_t *)(w + p.off_vals0) : (uint32_t *)(w + p.off_vals1);
  }
  pss_status st = run_paper_blocks(ctx, p, kt, keys_in, vals_in, kbuf.data(), vbuf.data(), w, s);
  if (st != PSS_OK) return st;
  const void *blocks = kbuf[P];
  const size_t kbytes = (size_t)p.kb;
  void *samples = w + pp.off_samples;
  void *ssorted = w + pp.off_ssorted;
  uint64_t *bounds = (uint64_t *)(w + pp.off_bounds);
  uint64_t *chunks = (uint64_t *)(w + pp.off_chunks);
  uint64_t *cprefix = (uint64_t *)(w + pp.off_cprefix);
  if (pp.ns) {
    {
      LaunchTimer t(ctx, "psrs_samples", pp.ns * kbytes * 2, s);
      PSS_LAUNCH(pss::launch_psrs_samples(kt, blocks, pp.top, samples, s), "sample launch");
    }
    {
      // one timing record for the whole sample sort
      LaunchTimer t(ctx, "psrs_sample_sort", pp.ns * kbytes * 2, s);
      const bool prof = ctx->profiling;
      ctx->profiling = false;
      st = run_auto_sort(ctx, pp.smp, pp.skt, samples, nullptr, ssorted, nullptr,
                         w + pp.off_sws, s);
      ctx->profiling = prof;
      if (st != PSS_OK) return st;
    }
    if (o.samples)
      PSS_LAUNCH(pss::launch_unmap_copy(kt, ssorted, o.samples, pp.ns, s), "sample copy");
  }
  {
    LaunchTimer t(ctx, "psrs_partition", (uint64_t)p.top.fan * (p.top.n_parts + 1) * 8, s);
    PSS_LAUNCH(pss::launch_psrs_partition(kt, blocks, pp.top, ssorted, pp.ns, bounds, o.pivots,
                                       o.split, s),
            "partition launch");
  }
  {
    LaunchTimer t(ctx, "psrs_chunks", (uint64_t)p.top.n_parts * 24, s);
    PSS_LAUNCH(pss::launch_psrs_chunks(pp.top, bounds, o.sizes, chunks, cprefix, s), "chunk launch");
  }
  if (o.offsets)
    PSS_LAUNCH(hipMemcpyAsync(o.offsets, bounds, ((size_t)p.top.n_parts + 1) * 8,
                           hipMemcpyDeviceToDevice, s),
            "offset copy");
  if (o.sorted_blocks)
    PSS_LAUNCH(pss::launch_unmap_copy(kt, blocks, o.sorted_blocks, p.n, s), "block copy");
  if (!merge) return PSS_OK;
  pss::RunGeom top = pp.top;
  top.bounds = bounds;
  top.chunk_prefix = cprefix;
  uint32_t *table = (uint32_t *)(w + pp.off_table);
  st = paper_partition_search(ctx, p, kt, blocks, top, table, w, s);
  if (st != PSS_OK) return st;
  {
    LaunchTimer t(ctx, "partition_merge", 2 * p.n * ((uint64_t)p.kb + (p.kv ? 4 : 0)), s);
    if (ctx->merge_method == PSS_MERGE_SORT)
      PSS_LAUNCH(pss::launch_sort_merge(kt, p.kv, blocks, vbuf[P], keys_out, vals_out, top, table,
                                     nullptr, 1, s),
              "merge launch");
    else
      PSS_LAUNCH(pss::launch_merge(kt, p.kv ? 1 : 0, blocks, vbuf[P], keys_out, vals_out, top, table,
                                nullptr, 1, nullptr, nullptr, s),
              "merge launch");
  }
  return PSS_OK;
}

// Argument checks shared by the two PSRS entry points; fills the plan.
pss_status psrs_prepare(pss_ctx *ctx, pss_key_t key, pss_val_t val, const void *keys_in,
                        const void *keys_out, const void *vals_in, const void *vals_out,
                        uint64_t n, uint32_t n_blocks, uint32_t n_parts, void *ws,
                        size_t ws_bytes, PsrsPlan *pp) {
  if (n_blocks == 0 || n_parts == 0)
    return fail(ctx, PSS_ERR_INVALID, "PSRS needs n_blocks > 0 and n_parts > 0");
  Plan p;
  pss_status st = validate(ctx, key, val, keys_in, keys_out, vals_in, vals_out, n, n_blocks,
                           n_parts, SIZE_MAX, &p);
  if (st != PSS_OK) return st;
  if (!ctx) return fail(nullptr, PSS_ERR_INVALID, "null context");
  std::string err;
  st = make_psrs_plan(key, val, n, n_blocks, n_parts, pp, &err);
  if (st != PSS_OK) return fail(ctx, st, err);
  if (n && ws_bytes < pp->total) {
    char m[160];
    snprintf(m, sizeof m, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
             pp->total);
    return fail(ctx, PSS_ERR_WORKSPACE, m);
  }
  if (n && !ws) return fail(ctx, PSS_ERR_WORKSPACE, "null workspace");
  return PSS_OK;
}

// Workspace of a record sort: keys, indices, sorted keys, permutation, then
// the key-value sort's own workspace.
struct RecordPlan {
  size_t off_keys = 0, off_idx = 0, off_skeys = 0, off_perm = 0, off_sort = 0, total = 0;
};

pss_status record_plan(const pss_ctx *ctx, pss_key_t key, uint64_t n, RecordPlan *rp) {
  if ((int)key < 0 || (int)key > 5) return fail(ctx, PSS_ERR_INVALID, "unknown key type");
  if (n > PSS_MAX_KEYS) return fail(ctx, PSS_ERR_UNSUPPORTED, "n >= 2^31 is not supported");
  Plan p;
  std::string err;
  const pss_status st = make_plan(key, PSS_VAL_U32, n, 0, 0, &p, &err);
  if (st != PSS_OK) return fail(ctx, st, err);
  const size_t kb = (size_t)pss::key_bytes((int)key);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  rp->off_keys = take(n * kb);
  rp->off_idx = take(n * 4);
  rp->off_skeys = take(n * kb);
  rp->off_perm = take(n * 4);
  rp->off_sort = take(p.total);
  rp->total = off;
  return PSS_OK;
}

}  // namespace

namespace pss {
RunGeom sample_geom(const RunGeom &g) {
  RunGeom s = g;
  const uint64_t nseg = (g.n + g.seg_len - 1) / g.seg_len;
  const uint64_t last = g.n - (nseg - 1) * g.seg_len;
  s.seg_len = g.seg_len >> kSampleLog2;
  s.n = (nseg - 1) * s.seg_len + (last >> kSampleLog2);
  s.run_len = g.run_len >> kSampleLog2;
  s.group_len = g.group_len >> kSampleLog2;
  s.part_len = kPart;
  s.rows_per_group = (uint32_t)((s.group_len + kPart - 1) / kPart) + 1;
  return s;
}

void set_thread_error(const char *msg) { g_thread_error = msg; }
int ctx_device(const pss_ctx *ctx) { return ctx->device; }
pss_status ctx_fail(const pss_ctx *ctx, pss_status s, const char *msg) { return fail(ctx, s, msg); }
bool ctx_set_profiling(pss_ctx *ctx, bool on) {
  const bool was = ctx->profiling;
  ctx->profiling = on;
  return was;
}
}  // namespace pss

namespace pss {

namespace {
// Operations of each kind still allowed before the armed one fails; -1 = not
// armed.  Index: kInjectLaunch, kInjectAlloc.
std::atomic<int64_t> g_inject[3] = {{-1}, {-1}, {-1}};
}  // namespace

bool inject_fault(int kind) {
  std::atomic<int64_t> &c = g_inject[kind];
  int64_t v = c.load(std::memory_order_relaxed);
  while (v >= 0) {
    if (c.compare_exchange_weak(v, v - 1, std::memory_order_acq_rel)) return v == 0;
  }
  return false;
}

}  // namespace pss

extern "C" {

pss_status pss_debug_inject(pss_inject_t what, int64_t after) {
  if (!pss::valid_enum(what, 2)) return fail(nullptr, PSS_ERR_INVALID, "unknown fault kind");
  if (what == PSS_INJECT_NONE) {
    pss::g_inject[pss::kInjectLaunch].store(-1);
    pss::g_inject[pss::kInjectAlloc].store(-1);
    return PSS_OK;
  }
  pss::g_inject[what == PSS_INJECT_LAUNCH ? pss::kInjectLaunch : pss::kInjectAlloc].store(
      after < 0 ? -1 : after);
  return PSS_OK;
}

pss_status pss_create(int device, pss_ctx **out) {
  if (!out) return fail(nullptr, PSS_ERR_INVALID, "null output handle");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
  if (device < 0 || device >= count) return fail(nullptr, PSS_ERR_HIP, "no such HIP device");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
  // the device address of pss_sort_noalloc's scratch array, looked up once
  // per device with the device current; a failed lookup is reported by that
  // entry point only
  (void)pss::scratch_setup(device);
  pss_ctx *c = new (std::nothrow) pss_ctx;
  if (!c) return fail(nullptr, PSS_ERR_OOM, "out of host memory");
  c->device = device;
  *out = c;
  return PSS_OK;
}

void pss_destroy(pss_ctx *ctx) {
  if (!ctx) return;
  for (auto &r : ctx->recs) {
    hipEventDestroy(r.begin);
    hipEventDestroy(r.end);
  }
  for (auto e : ctx->pool) hipEventDestroy(e);
  delete ctx;
}

pss_status pss_set_merge_method(pss_ctx *ctx, pss_merge_method method) {
  if (!ctx) return fail(nullptr, PSS_ERR_INVALID, "null context");
  if (!pss::valid_enum(method, 1)) return fail(ctx, PSS_ERR_INVALID, "unknown merge method");
  ctx->merge_method = method;
  return PSS_OK;
}

pss_status pss_profile_enable(pss_ctx *ctx, int on) {
  if (!ctx) return fail(nullptr, PSS_ERR_INVALID, "null context");
  ctx->profiling = on != 0;
  return PSS_OK;
}

pss_status pss_profile_only(pss_ctx *ctx, const char *family) {
  if (!ctx) return fail(nullptr, PSS_ERR_INVALID, "null context");
  if (family && strnlen(family, 64) > 63) return fail(ctx, PSS_ERR_INVALID, "family name too long");
  ctx->profile_only = family ? family : "";
  return PSS_OK;
}

pss_status pss_profile_read(pss_ctx *ctx, char *buf, size_t buf_len) {
  if (!ctx || !buf || buf_len == 0) return fail(ctx, PSS_ERR_INVALID, "null argument");
  struct Agg {
    std::string name;
    uint64_t launches = 0, bytes = 0;
    double ms = 0;
  };
  std::vector<Agg> agg;
  for (auto &r : ctx->recs) {
    PSS_TRY(hipEventSynchronize(r.end), "hipEventSynchronize");
    float ms = 0;
    PSS_TRY(hipEventElapsedTime(&ms, r.begin, r.end), "hipEventElapsedTime");
    auto it = std::find_if(agg.begin(), agg.end(), [&](const Agg &a) { return a.name == r.name; });
    if (it == agg.end()) {
      agg.push_back(Agg{r.name});
      it = agg.end() - 1;
    }
    it->launches++;
    it->bytes += r.bytes;
    it->ms += ms;
  }
  std::string j = "{";
  for (size_t i = 0; i < agg.size(); ++i) {
    char item[256];
    snprintf(item, sizeof item, "%s\"%s\": {\"launches\": %llu, \"ms\": %.6f, \"bytes\": %llu}",
             i ? ", " : "", agg[i].name.c_str(), (unsigned long long)agg[i].launches, agg[i].ms,
             (unsigned long long)agg[i].bytes);
    j += item;
  }
  j += "}";
  if (j.size() + 1 > buf_len) return fail(ctx, PSS_ERR_INVALID, "buffer too small");
  memcpy(buf, j.c_str(), j.size() + 1);
  for (auto &r : ctx->recs) {
    ctx->pool.push_back(r.begin);
    ctx->pool.push_back(r.end);
  }
  ctx->recs.clear();
  return PSS_OK;
}

const char *pss_status_string(pss_status s) {
  switch (s) {
    case PSS_OK: return "PSS_OK";
    case PSS_ERR_INVALID: return "PSS_ERR_INVALID";
    case PSS_ERR_UNSUPPORTED: return "PSS_ERR_UNSUPPORTED";
    case PSS_ERR_OOM: return "PSS_ERR_OOM";
    case PSS_ERR_HIP: return "PSS_ERR_HIP";
    case PSS_ERR_WORKSPACE: return "PSS_ERR_WORKSPACE";
    case PSS_ERR_BUDGET: return "PSS_ERR_BUDGET";
    case PSS_ERR_BUSY: return "PSS_ERR_BUSY";
    case PSS_ERR_CANCELLED: return "PSS_ERR_CANCELLED";
    default: return "PSS_ERR_UNKNOWN";
  }
}

const char *pss_last_error(const pss_ctx *ctx) {
  return ctx ? ctx->last_error.c_str() : g_thread_error.c_str();
}

pss_status pss_validate(pss_key_t key, pss_val_t val, const void *keys_in, const void *keys_out,
                        const void *vals_in, const void *vals_out, uint64_t n, uint32_t n_blocks,
                        uint32_t n_parts, size_t ws_bytes) {
  if (!pss::valid_enum(key, 5) || !pss::valid_enum(val, 1))
    return fail(nullptr, PSS_ERR_INVALID, "unknown key or value type");
  Plan p;
  return validate(nullptr, key, val, keys_in, keys_out, vals_in, vals_out, n, n_blocks, n_parts,
                  ws_bytes, &p);
}

pss_status pss_workspace_bytes(const pss_ctx *ctx, pss_key_t key, pss_val_t val, uint64_t n,
                               uint32_t n_blocks, uint32_t n_parts, size_t *bytes) {
  if (!pss::valid_enum(key, 5) || !pss::valid_enum(val, 1))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  if (!bytes) return fail(ctx, PSS_ERR_INVALID, "null output pointer");
  Plan p;
  // enum, mode and limit checks only (no arrays exist yet)
  const pss_status s = validate(ctx, key, val, nullptr, nullptr, nullptr, nullptr, 0, n_blocks,
                                n_parts, SIZE_MAX, &p);
  if (s != PSS_OK) return s;
  if (n > PSS_MAX_KEYS) return fail(ctx, PSS_ERR_UNSUPPORTED, "n >= 2^31 is not supported");
  std::string err;
  const pss_status ps = make_plan(key, val, n, n_blocks, n_parts, &p, &err);
  if (ps != PSS_OK) return fail(ctx, ps, err);
  *bytes = p.total;
  return PSS_OK;
}

pss_status pss_plan_describe(pss_key_t key, pss_val_t val, uint64_t n, uint32_t n_blocks,
                             uint32_t n_parts, char *buf, size_t buf_len) {
  if (!pss::valid_enum(key, 5) || !pss::valid_enum(val, 1))
    return fail(nullptr, PSS_ERR_INVALID, "unknown key or value type");
  if (!buf || buf_len == 0) return fail(nullptr, PSS_ERR_INVALID, "null buffer");
  size_t ws = 0;
  const pss_status s = pss_workspace_bytes(nullptr, key, val, n, n_blocks, n_parts, &ws);
  if (s != PSS_OK) return s;
  Plan p;
  std::string err;
  make_plan(key, val, n, n_blocks, n_parts, &p, &err);
  std::string j = "{\"mode\": \"";
  j += p.paper ? "paper" : "auto";
  j += "\", \"tile\": " + std::to_string(p.tile) + ", \"part\": " + std::to_string(p.part);
  std::string fans;
  for (size_t i = 0; i < p.passes.size(); ++i)
    fans += (i ? ", " : "") + std::to_string(p.passes[i].fan);
  if (p.paper) {
    j += ", \"passes\": [" + std::to_string(n_blocks) + "], \"block_passes\": [" + fans + "]";
  } else {
    j += ", \"passes\": [" + fans + "], \"block_passes\": []";
  }
  const size_t sweeps = (n ? 1 : 0) + p.passes.size() + (p.paper && n ? 1 : 0);
  j += ", \"n_blocks\": " + std::to_string(n_blocks) + ", \"n_parts\": " + std::to_string(n_parts);
  j += ", \"hbm_passes\": " + std::to_string(sweeps) + ", \"workspace_bytes\": " + std::to_string(ws) + "}";
  if (j.size() + 1 > buf_len) return fail(nullptr, PSS_ERR_INVALID, "buffer too small");
  memcpy(buf, j.c_str(), j.size() + 1);
  return PSS_OK;
}

pss_status pss_sort(pss_ctx *ctx, pss_key_t key, pss_val_t val, const void *keys_in,
                    void *keys_out, const uint32_t *vals_in, uint32_t *vals_out, uint64_t n,
                    uint32_t n_blocks, uint32_t n_parts, void *ws, size_t ws_bytes,
                    void *stream) {
  if (!pss::valid_enum(key, 5) || !pss::valid_enum(val, 1))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  Plan p;
  pss_status st = validate(ctx, key, val, keys_in, keys_out, vals_in, vals_out, n, n_blocks,
                           n_parts, ws_bytes, &p);
  if (st != PSS_OK) return st;
  if (!ctx) return fail(nullptr, PSS_ERR_INVALID, "null context");
  if (n == 0) return PSS_OK;
  if (!ws) return fail(ctx, PSS_ERR_WORKSPACE, "null workspace");
  PSS_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)ws;
  uint32_t *table = (uint32_t *)(w + p.off_table);
  const int kt = (int)key;
  const size_t P = p.passes.size();

  if (!p.paper) {
    st = run_auto_sort(ctx, p, kt, keys_in, vals_in, keys_out, vals_out, w, s);
    if (st != PSS_OK) return st;
  } else {
    // block sort ends in workspace buffer 0; the cross-block merge writes out
    KeyBufs kb;
    ValBufs vb;
    for (size_t q = 0; q <= P; ++q) {
      kb.push_back(nullptr);
      vb.push_back(nullptr);
    }
    for (size_t q = 0; q <= P; ++q) {
      const bool even = ((P - q) % 2) == 0;
      kb[q] = even ? (void *)(w + p.off_keys0) : (void *)(w + p.off_keys1);
      if (p.kv) vb[q] = even ? (uint32_t *)(w + p.off_vals0) : (uint32_t *)(w + p.off_vals1);
    }
    st = run_paper_blocks(ctx, p, kt, keys_in, vals_in, kb.data(), vb.data(), w, s);
    if (st != PSS_OK) return st;
    uint64_t *sizes = (uint64_t *)(w + p.off_sizes);
    uint64_t *offsets = (uint64_t *)(w + p.off_offsets);
    const uint64_t sweep = 2 * p.n * ((uint64_t)p.kb + (p.kv ? 4 : 0));
    st = paper_partition_search(ctx, p, kt, kb[P], p.top, table, w, s);
    if (st != PSS_OK) return st;
    {
      LaunchTimer t(ctx, "offset_scan", (uint64_t)p.top.n_parts * 16, s);
      PSS_LAUNCH(pss::launch_partition_offsets(p.top, table, sizes, offsets, s), "offset scan launch");
    }
    {
      LaunchTimer t(ctx, "partition_merge", sweep, s);
      if (ctx->merge_method == PSS_MERGE_SORT)
        PSS_LAUNCH(pss::launch_sort_merge(kt, p.kv, kb[P], vb[P], keys_out, vals_out, p.top, table,
                                       offsets, 1, s),
                "merge launch");
      else
        PSS_LAUNCH(pss::launch_merge(kt, p.kv ? 1 : 0, kb[P], vb[P], keys_out, vals_out, p.top,
                                  table, offsets, 1, nullptr, nullptr, s),
                "merge launch");
    }
  }
  return PSS_OK;
}

// ------------------------------------------------- batched segmented sort
namespace {

struct SegPlan {
  uint32_t max_passes = 0;
  uint32_t small0 = 2048, small1 = 4096;
  uint32_t fan_log2 = pss::kMaxFanLog2;  // runs merged per pass, log2
  // keys per tile of segments with merge passes, and per merge partition
  // (key-value batches: 4096, as in the automatic plan)
  uint32_t tile = pss::kTile, part = pss::kPart;
  std::vector<pss::RunGeom> g, gs;  // per pass: key level and sample level
  uint64_t ns = 0;                  // bound on samples
  size_t off_keys = 0, off_vals = 0, off_plan = 0, off_samples = 0, off_skeys = 0;
  size_t off_sruns = 0, off_table = 0, off_stable = 0, off_prefix = 0, total = 0;
};

uint32_t passes_for(uint64_t L, uint32_t fan_log2, uint32_t tile) {
  if (L <= (uint64_t)tile) return 0;
  const uint64_t tiles = ceil_div(L, tile);
  uint32_t bits = 0;
  while (((uint64_t)1 << bits) < tiles) ++bits;
  return (bits + fan_log2 - 1) / fan_log2;
}

pss_status make_seg_plan(const pss_ctx *ctx, pss_key_t key, pss_val_t val, uint64_t n,
                         uint32_t n_segs, const pss_tuning *tu, SegPlan *sp) {
  if ((int)key < 0 || (int)key > 5) return fail(ctx, PSS_ERR_INVALID, "unknown key type");
  if ((int)val != PSS_VAL_NONE && (int)val != PSS_VAL_U32)
    return fail(ctx, PSS_ERR_INVALID, "unknown value type");
  if (n > PSS_MAX_KEYS) return fail(ctx, PSS_ERR_UNSUPPORTED, "n >= 2^31 is not supported");
  if (n_segs > PSS_MAX_SEGMENTS) return fail(ctx, PSS_ERR_UNSUPPORTED, "too many segments");
  uint64_t max_len = n;
  if (tu) {
    if (tu->small_max_2k > 2048 || tu->small_max_4k > 4096 || tu->small_max_2k > tu->small_max_4k)
      return fail(ctx, PSS_ERR_INVALID, "tuning: need small_max_2k <= small_max_4k, <= 2048, <= 4096");
    sp->small0 = tu->small_max_2k;
    sp->small1 = tu->small_max_4k;
    if (tu->max_seg_len) max_len = std::min<uint64_t>(tu->max_seg_len, n);
    if (tu->fan_log2 != 0 && tu->fan_log2 != 5 && tu->fan_log2 != 6)
      return fail(ctx, PSS_ERR_INVALID, "tuning: fan_log2 must be 0, 5 or 6");
    if (tu->fan_log2) sp->fan_log2 = tu->fan_log2;
  }
  const uint32_t f = sp->fan_log2;
  const int kb = pss::key_bytes((int)key);
  const bool kv = val == PSS_VAL_U32;
  sp->tile = kv ? pss::kTileKV : pss::kTile;
  sp->part = kv ? pss::kPartKV : pss::kPart;
  sp->max_passes = passes_for(max_len, f, sp->tile);
  sp->ns = n >> pss::kSampleLog2;
  const uint64_t S = n_segs;
  uint64_t max_rows = 0, max_srows = 0, max_sparts = 0;
  for (uint32_t q = 1; q <= sp->max_passes; ++q) {
    pss::RunGeom g{};
    g.n = n;
    g.run_len = (uint64_t)sp->tile << (f * (q - 1));
    g.fan = 1u << f;
    g.group_len = g.run_len << f;
    g.part_len = sp->part;
    g.rows_per_group = (uint32_t)ceil_div(g.group_len, sp->part) + 1;
    const uint64_t groups = n / g.group_len + S + 1;
    g.part_bound = n / sp->part + groups + 1;
    g.row_bound = g.part_bound + groups + 1;
    g.seg_len = g.group_len;
    g.groups_per_seg = 1;
    g.n_groups = groups;
    pss::RunGeom gs = g;
    gs.part_len = pss::kPart;  // sample merges keep 8192-key partitions
    gs.n = sp->ns;
    gs.run_len = g.run_len >> pss::kSampleLog2;
    gs.group_len = g.group_len >> pss::kSampleLog2;
    // as the planning kernel counts them: a group of 32 runs of 4096 keys
    // leaves 4096 samples, one (short) sample partition
    gs.rows_per_group = (uint32_t)ceil_div(gs.group_len, pss::kPart) + 1;
    gs.part_bound = sp->ns / pss::kPart + groups + 1;
    gs.row_bound = gs.part_bound + groups + 1;
    max_rows = std::max(max_rows, g.row_bound);
    max_srows = std::max(max_srows, gs.row_bound);
    max_sparts = std::max(max_sparts, gs.part_bound);
    sp->g.push_back(g);
    sp->gs.push_back(gs);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  sp->off_keys = take(n * (size_t)kb);
  sp->off_vals = kv ? take(n * sizeof(uint32_t)) : 0;
  // 3 tile prefixes, sample offsets, 4 prefixes per pass, then npass
  sp->off_plan = take((4 + 4 * (size_t)pss::kMaxSegPasses) * (S + 1) * 8 + S * 4);
  if (sp->max_passes) {
    sp->off_samples = take(sp->ns * (size_t)kb);
    sp->off_skeys = take(sp->ns * (size_t)kb);
    sp->off_sruns = take(sp->ns * sizeof(uint32_t));
    sp->off_table = take(max_rows * (1u << f) * sizeof(uint32_t));
    sp->off_stable = take(max_srows * (1u << f) * sizeof(uint32_t));
    sp->off_prefix = take(max_sparts * (pss::kPart / pss::kChunk) * (1u << f) * sizeof(uint32_t));
  }
  sp->total = off;
  return PSS_OK;
}

pss::SegPlanPtrs seg_plan_ptrs(char *w, const SegPlan &sp, uint32_t n_segs) {
  pss::SegPlanPtrs pp{};
  uint64_t *a = (uint64_t *)(w + sp.off_plan);
  const size_t stride = (size_t)n_segs + 1;
  for (int c = 0; c < 3; ++c) pp.tiles[c] = a + c * stride;
  pp.soff = a + 3 * stride;
  for (uint32_t q = 0; q < pss::kMaxSegPasses; ++q) {
    pp.rows[q] = a + (4 + 4 * q + 0) * stride;
    pp.parts[q] = a + (4 + 4 * q + 1) * stride;
    pp.srows[q] = a + (4 + 4 * q + 2) * stride;
    pp.sparts[q] = a + (4 + 4 * q + 3) * stride;
  }
  pp.npass = (uint32_t *)(a + (4 + 4 * pss::kMaxSegPasses) * stride);
  return pp;
}

}  // namespace

pss_status pss_segmented_workspace_bytes(const pss_ctx *ctx, pss_key_t key, pss_val_t val,
                                         uint64_t n, uint32_t n_segs, const pss_tuning *tuning,
                                         size_t *bytes) {
  if (!pss::valid_enum(key, 5) || !pss::valid_enum(val, 1))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  if (!bytes) return fail(ctx, PSS_ERR_INVALID, "null output pointer");
  SegPlan sp;
  const pss_status st = make_seg_plan(ctx, key, val, n, n_segs, tuning, &sp);
  if (st != PSS_OK) return st;
  *bytes = sp.total;
  return PSS_OK;
}

pss_status pss_segmented_sort(pss_ctx *ctx, pss_key_t key, pss_val_t val, const void *keys_in,
                              void *keys_out, const uint32_t *vals_in, uint32_t *vals_out,
                              uint64_t n, const uint64_t *seg_offsets, uint32_t n_segs,
                              const pss_tuning *tuning, void *ws, size_t ws_bytes, void *stream) {
  if (!pss::valid_enum(key, 5) || !pss::valid_enum(val, 1))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  SegPlan sp;
  pss_status st = make_seg_plan(ctx, key, val, n, n_segs, tuning, &sp);
  if (st != PSS_OK) return st;
  const size_t kbytes = (size_t)pss::key_bytes((int)key);
  const bool kv = val == PSS_VAL_U32;
  if (n > 0) {
    if (!keys_in || !keys_out) return fail(ctx, PSS_ERR_INVALID, "null key pointer");
    if (overlaps(keys_in, n * kbytes, keys_out, n * kbytes))
      return fail(ctx, PSS_ERR_INVALID, "keys_in and keys_out overlap (the sort is out of place)");
    if (kv) {
      if (!vals_in || !vals_out) return fail(ctx, PSS_ERR_INVALID, "null value pointer");
      if (overlaps(vals_in, n * 4, vals_out, n * 4) || overlaps(keys_out, n * kbytes, vals_out, n * 4))
        return fail(ctx, PSS_ERR_INVALID, "value arrays overlap");
    }
    if (!seg_offsets || n_segs == 0) return fail(ctx, PSS_ERR_INVALID, "segment offsets missing");
  }
  if (ws_bytes < sp.total) {
    char m[160];
    snprintf(m, sizeof m, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, sp.total);
    return fail(ctx, PSS_ERR_WORKSPACE, m);
  }
  if (!ctx) return fail(nullptr, PSS_ERR_INVALID, "null context");
  if (n == 0) return PSS_OK;
  if (!ws) return fail(ctx, PSS_ERR_WORKSPACE, "null workspace");
  PSS_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int kt = (int)key;
  char *w = (char *)ws;
  const pss::SegPlanPtrs pp = seg_plan_ptrs(w, sp, n_segs);
  void *kws = w + sp.off_keys;
  uint32_t *vws = kv ? (uint32_t *)(w + sp.off_vals) : nullptr;
  void *samples = sp.max_passes ? (void *)(w + sp.off_samples) : nullptr;
  void *skeys = w + sp.off_skeys;
  uint32_t *sruns = (uint32_t *)(w + sp.off_sruns);
  uint32_t *table = (uint32_t *)(w + sp.off_table);
  uint32_t *stable = (uint32_t *)(w + sp.off_stable);
  uint32_t *prefix = (uint32_t *)(w + sp.off_prefix);
  const uint64_t sweep = 2 * n * (kbytes + (kv ? 4 : 0));
  {
    LaunchTimer t(ctx, "segment_plan", (uint64_t)n_segs * 16, s);
    PSS_LAUNCH(pss::launch_seg_plan(seg_offsets, n_segs, n, pp, sp.small0, sp.small1, sp.max_passes,
                                    sp.fan_log2, sp.tile, sp.part, s),
            "segment plan launch");
  }
  {
    LaunchTimer t(ctx, "tile_sort", sweep, s);
    PSS_LAUNCH(pss::launch_seg_tile_sorts(kt, kv, keys_in, vals_in, keys_out, kws, vals_out, vws,
                                       samples, seg_offsets, pp, n_segs, n, sp.tile, s),
            "tile sort launch");
  }
  for (uint32_t q = 1; q <= sp.max_passes; ++q) {
    pss::RunGeom g = sp.g[q - 1], gs = sp.gs[q - 1];
    g.seg = pss::SegTables{seg_offsets, pp.soff, pp.npass, pp.rows[q - 1], pp.parts[q - 1],
                           pp.sparts[q - 1], n_segs, q, 0};
    gs.seg = pss::SegTables{seg_offsets, pp.soff, pp.npass, pp.srows[q - 1], pp.sparts[q - 1],
                            pp.sparts[q - 1], n_segs, q, 1};
    {
      LaunchTimer t(ctx, "sample_split_search", gs.row_bound * gs.fan * 4, s);
      PSS_LAUNCH(pss::launch_corank(kt, samples, gs, stable, nullptr, nullptr, s),
              "sample split search launch");
    }
    {
      LaunchTimer t(ctx, "sample_merge", 2 * sp.ns * kbytes, s);
      PSS_LAUNCH(pss::launch_merge(kt, 2, samples, nullptr, skeys, sruns, gs, stable, nullptr, 0, nullptr,
                                prefix, s),
              "sample merge launch");
    }
    {
      LaunchTimer t(ctx, "split_search", g.row_bound * g.fan * 4, s);
      PSS_LAUNCH(pss::launch_corank_sampled(kt, keys_out, g, table, sruns, prefix, s, kws, &gs),
              "split search launch");
    }
    {
      LaunchTimer t(ctx, "merge", sweep, s);
      const pss::MergeAlt alt{kws, vws, kws, vws};
      PSS_LAUNCH(pss::launch_merge(kt, kv ? 1 : 0, keys_out, vals_out, keys_out, vals_out, g, table,
                                nullptr, 0, samples, nullptr, s, &alt),
              "merge launch");
    }
  }
  return PSS_OK;
}

struct pss_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

pss_status pss_segmented_graph_create(pss_ctx *ctx, pss_key_t key, pss_val_t val,
                                      const void *keys_in, void *keys_out,
                                      const uint32_t *vals_in, uint32_t *vals_out, uint64_t n,
                                      const uint64_t *seg_offsets, uint32_t n_segs,
                                      const pss_tuning *tuning, void *ws, size_t ws_bytes,
                                      pss_graph **out) {
  if (!pss::valid_enum(key, 5) || !pss::valid_enum(val, 1))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  if (!out) return fail(ctx, PSS_ERR_INVALID, "null output handle");
  *out = nullptr;
  if (!ctx) return fail(nullptr, PSS_ERR_INVALID, "null context");
  PSS_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t cs = nullptr;
  PSS_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
  const bool prof = ctx->profiling;
  ctx->profiling = false;  // no timing events inside a captured graph
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  pss_status st = PSS_OK;
  if (e == hipSuccess) {
    st = pss_segmented_sort(ctx, key, val, keys_in, keys_out, vals_in, vals_out, n, seg_offsets,
                            n_segs, tuning, ws, ws_bytes, cs);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (st == PSS_OK && e2 != hipSuccess) {
      ctx->profiling = prof;
      hipStreamDestroy(cs);
      return hip_fail(ctx, e2, "hipStreamEndCapture");
    }
    ctx->profiling = prof;
    if (st != PSS_OK) {
      if (g) hipGraphDestroy(g);
      hipStreamDestroy(cs);
      return st;
    }
    pss_graph *pg = new (std::nothrow) pss_graph;
    if (!pg) {
      hipGraphDestroy(g);
      hipStreamDestroy(cs);
      return fail(ctx, PSS_ERR_OOM, "out of host memory");
    }
    pg->graph = g;
    pg->device = ctx->device;
    e = hipGraphInstantiate(&pg->exec, g, nullptr, nullptr, 0);
    hipStreamDestroy(cs);
    if (e != hipSuccess) {
      hipGraphDestroy(g);
      delete pg;
      return hip_fail(ctx, e, "hipGraphInstantiate");
    }
    *out = pg;
    return PSS_OK;
  }
  ctx->profiling = prof;
  hipStreamDestroy(cs);
  return hip_fail(ctx, e, "hipStreamBeginCapture");
}

pss_status pss_graph_launch(pss_graph *g, void *stream) {
  if (!g || !g->exec) return fail(nullptr, PSS_ERR_INVALID, "null graph");
  hipError_t e = hipSetDevice(g->device);
  if (e == hipSuccess) e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGraphLaunch");
  return PSS_OK;
}

void pss_graph_destroy(pss_graph *g) {
  if (!g) return;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
}

pss_status pss_device_check(pss_ctx *ctx, uint32_t *code) {
  if (!ctx || !code) return fail(ctx, PSS_ERR_INVALID, "null argument");
  PSS_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  PSS_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  PSS_TRY(pss::read_device_error(code, true), "reading the device error word");
  return PSS_OK;
}

pss_status pss_splitters(pss_ctx *ctx, pss_key_t key, const void *keys_in, uint64_t n,
                         uint32_t n_blocks, uint32_t n_parts, void *sorted_blocks, void *pivots,
                         uint64_t *counts, uint64_t *split, uint64_t *offsets, void *ws,
                         size_t ws_bytes, void *stream) {
  if (!pss::valid_enum(key, 5))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  if (n_blocks == 0 || n_parts == 0)
    return fail(ctx, PSS_ERR_INVALID, "pss_splitters needs n_blocks > 0 and n_parts > 0");
  Plan p;
  // keys_out is not used here; validate the key input against a disjoint dummy
  const char dummy = 0;
  pss_status st = validate(ctx, key, PSS_VAL_NONE, keys_in, n ? &dummy : nullptr, nullptr, nullptr,
                           n, n_blocks, n_parts, ws_bytes, &p);
  if (st != PSS_OK) return st;
  if (!ctx) return fail(nullptr, PSS_ERR_INVALID, "null context");
  if (n > 0 && !ws) return fail(ctx, PSS_ERR_WORKSPACE, "null workspace");
  if (n_parts > 1 && (pivots != nullptr) != (counts != nullptr))
    return fail(ctx, PSS_ERR_INVALID, "pivots and counts must be given together");
  PSS_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int kt = (int)key;
  const int kbytes = pss::key_bytes(kt);
  if (n == 0) {
    if (counts && n_parts > 1)
      PSS_LAUNCH(hipMemsetAsync(counts, 0, (n_parts - 1) * sizeof(uint64_t), s), "memset");
    if (pivots && n_parts > 1)
      PSS_LAUNCH(hipMemsetAsync(pivots, 0, (size_t)(n_parts - 1) * kbytes, s), "memset");
    if (split) PSS_LAUNCH(hipMemsetAsync(split, 0, (size_t)n_blocks * (n_parts + 1) * 8, s), "memset");
    if (offsets) PSS_LAUNCH(hipMemsetAsync(offsets, 0, ((size_t)n_parts + 1) * 8, s), "memset");
    return PSS_OK;
  }
  char *w = (char *)ws;
  uint32_t *table = (uint32_t *)(w + p.off_table);
  const size_t P = p.passes.size();
  KeyBufs kb;
  ValBufs vb;
  for (size_t q = 0; q <= P; ++q) {
    kb.push_back(nullptr);
    vb.push_back(nullptr);
  }
  for (size_t q = 0; q <= P; ++q) {
    const bool even = ((P - q) % 2) == 0;
    kb[q] = even ? (void *)(w + p.off_keys0) : (void *)(w + p.off_keys1);
  }
  st = run_segment_sort(ctx, p, kt, keys_in, nullptr, kb.data(), vb.data(), 0, w, s);
  if (st != PSS_OK) return st;
  uint64_t *sizes = (uint64_t *)(w + p.off_sizes);
  uint64_t *offs = (uint64_t *)(w + p.off_offsets);
  // pivots and counts are written by the splitter search (both or neither)
  void *piv_dev = n_parts > 1 ? pivots : nullptr;
  uint64_t *cnt_dev = n_parts > 1 ? counts : nullptr;
  PSS_LAUNCH(pss::launch_corank(kt, kb[P], p.top, table, piv_dev, cnt_dev, s), "splitter launch");
  PSS_LAUNCH(pss::launch_partition_offsets(p.top, table, sizes, offs, s), "offset scan launch");
  if (offsets)
    PSS_LAUNCH(hipMemcpyAsync(offsets, offs, ((size_t)n_parts + 1) * 8, hipMemcpyDeviceToDevice, s),
            "offset copy");
  if (split) PSS_LAUNCH(pss::launch_split_table(p.top, table, split, s), "split table launch");
  if (sorted_blocks) PSS_LAUNCH(pss::launch_unmap_copy(kt, kb[P], sorted_blocks, n, s), "block copy");
  return PSS_OK;
}


pss_status pss_records_workspace_bytes(const pss_ctx *ctx, pss_key_t key, uint64_t n,
                                       size_t *bytes) {
  if (!pss::valid_enum(key, 5))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  if (!bytes) return fail(ctx, PSS_ERR_INVALID, "null output pointer");
  RecordPlan rp;
  const pss_status st = record_plan(ctx, key, n, &rp);
  if (st != PSS_OK) return st;
  *bytes = rp.total;
  return PSS_OK;
}

pss_status pss_sort_records(pss_ctx *ctx, pss_key_t key, const void *records_in,
                            void *records_out, uint64_t n, uint32_t record_bytes,
                            uint32_t key_offset, void *ws, size_t ws_bytes, void *stream) {
  if (!pss::valid_enum(key, 5))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  if (!ctx) return fail(nullptr, PSS_ERR_INVALID, "null context");
  RecordPlan rp;
  pss_status st = record_plan(ctx, key, n, &rp);
  if (st != PSS_OK) return st;
  const uint32_t kb = (uint32_t)pss::key_bytes((int)key);
  if (record_bytes < 4 || record_bytes > 4096 || record_bytes % 4 != 0 || record_bytes % kb != 0)
    return fail(ctx, PSS_ERR_INVALID,
                "record_bytes must be a multiple of 4 and of the key width, 4..4096");
  if (key_offset % kb != 0 || key_offset + kb > record_bytes)
    return fail(ctx, PSS_ERR_INVALID, "the key must lie aligned inside the record");
  if (n == 0) return PSS_OK;
  if (!records_in || !records_out) return fail(ctx, PSS_ERR_INVALID, "null record pointer");
  if (((uintptr_t)records_in | (uintptr_t)records_out) % kb != 0)
    return fail(ctx, PSS_ERR_INVALID, "record arrays must be aligned to the key width");
  if (overlaps(records_in, n * record_bytes, records_out, n * record_bytes))
    return fail(ctx, PSS_ERR_INVALID, "records_in and records_out overlap");
  if (!ws) return fail(ctx, PSS_ERR_WORKSPACE, "null workspace");
  if (ws_bytes < rp.total) {
    char m[160];
    snprintf(m, sizeof m, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
             rp.total);
    return fail(ctx, PSS_ERR_WORKSPACE, m);
  }
  PSS_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)ws;
  void *keys = w + rp.off_keys;
  uint32_t *idx = (uint32_t *)(w + rp.off_idx);
  uint32_t *perm = (uint32_t *)(w + rp.off_perm);
  {
    LaunchTimer t(ctx, "record_keys", n * ((uint64_t)record_bytes + kb + 4), s);
    PSS_LAUNCH(pss::launch_record_keys((int)key, records_in, n, record_bytes, key_offset, keys, idx,
                                    s),
            "record key launch");
  }
  st = pss_sort(ctx, key, PSS_VAL_U32, keys, w + rp.off_skeys, idx, perm, n, 0, 0,
                w + rp.off_sort, ws_bytes - rp.off_sort, stream);
  if (st != PSS_OK) return st;
  {
    LaunchTimer t(ctx, "record_gather", 2 * n * (uint64_t)record_bytes + 4 * n, s);
    PSS_LAUNCH(pss::launch_record_gather(records_in, records_out, perm, n, record_bytes, s),
            "record gather launch");
  }
  return PSS_OK;
}

pss_status pss_psrs_workspace_bytes(const pss_ctx *ctx, pss_key_t key, pss_val_t val, uint64_t n,
                                    uint32_t n_blocks, uint32_t n_parts, size_t *bytes) {
  if (!pss::valid_enum(key, 5) || !pss::valid_enum(val, 1))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  if (!bytes) return fail(ctx, PSS_ERR_INVALID, "null output pointer");
  if (n_blocks == 0 || n_parts == 0)
    return fail(ctx, PSS_ERR_INVALID, "PSRS needs n_blocks > 0 and n_parts > 0");
  Plan p;
  const pss_status s = validate(ctx, key, val, nullptr, nullptr, nullptr, nullptr, 0, n_blocks,
                                n_parts, SIZE_MAX, &p);
  if (s != PSS_OK) return s;
  if (n > PSS_MAX_KEYS) return fail(ctx, PSS_ERR_UNSUPPORTED, "n >= 2^31 is not supported");
  PsrsPlan pp;
  std::string err;
  const pss_status ps = make_psrs_plan(key, val, n, n_blocks, n_parts, &pp, &err);
  if (ps != PSS_OK) return fail(ctx, ps, err);
  *bytes = pp.total;
  return PSS_OK;
}


pss_status pss_psrs_sort(pss_ctx *ctx, pss_key_t key, pss_val_t val, const void *keys_in,
                         void *keys_out, const uint32_t *vals_in, uint32_t *vals_out, uint64_t n,
                         uint32_t n_blocks, uint32_t n_parts, uint64_t *part_sizes, void *ws,
                         size_t ws_bytes, void *stream) {
  if (!pss::valid_enum(key, 5) || !pss::valid_enum(val, 1))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  PsrsPlan pp;
  pss_status st = psrs_prepare(ctx, key, val, keys_in, keys_out, vals_in, vals_out, n, n_blocks,
                               n_parts, ws, ws_bytes, &pp);
  if (st != PSS_OK) return st;
  PSS_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) {
    if (part_sizes) PSS_LAUNCH(hipMemsetAsync(part_sizes, 0, (size_t)n_parts * 8, s), "memset");
    return PSS_OK;
  }
  PsrsOut o;
  o.sizes = part_sizes;
  return run_psrs(ctx, pp, (int)key, keys_in, vals_in, keys_out, vals_out, o, true, (char *)ws, s);
}

pss_status pss_psrs_splitters(pss_ctx *ctx, pss_key_t key, const void *keys_in, uint64_t n,
                              uint32_t n_blocks, uint32_t n_parts, void *sorted_blocks,
                              void *samples, void *pivots, uint64_t *split, uint64_t *offsets,
                              void *ws, size_t ws_bytes, void *stream) {
  if (!pss::valid_enum(key, 5))
    return fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  PsrsPlan pp;
  const char dummy = 0;  // no key output: validate keys_in against a disjoint dummy
  pss_status st = psrs_prepare(ctx, key, PSS_VAL_NONE, keys_in, n ? &dummy : nullptr, nullptr,
                               nullptr, n, n_blocks, n_parts, ws, ws_bytes, &pp);
  if (st != PSS_OK) return st;
  PSS_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int kt = (int)key;
  if (n == 0) {
    if (pivots && n_parts > 1)
      PSS_LAUNCH(hipMemsetAsync(pivots, 0, (size_t)(n_parts - 1) * pss::key_bytes(kt), s), "memset");
    if (split) PSS_LAUNCH(hipMemsetAsync(split, 0, (size_t)n_blocks * (n_parts + 1) * 8, s), "memset");
    if (offsets) PSS_LAUNCH(hipMemsetAsync(offsets, 0, ((size_t)n_parts + 1) * 8, s), "memset");
    return PSS_OK;
  }
  PsrsOut o;
  o.sorted_blocks = sorted_blocks;
  o.samples = samples;
  o.pivots = n_parts > 1 ? pivots : nullptr;
  o.split = split;
  o.offsets = offsets;
  return run_psrs(ctx, pp, kt, keys_in, nullptr, nullptr, nullptr, o, false, (char *)ws, s);
}

}  // extern "C"
