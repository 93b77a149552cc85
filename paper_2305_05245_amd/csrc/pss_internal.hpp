// Internal declarations shared by the C-ABI layer (pss_api.hip) and the HIP
// kernels (pss_kernels.hip).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>

#include "../../include/pss.h"

namespace pss {

// Step 1 tile sort: one workgroup sorts kTile keys held in LDS.
constexpr int kTileThreads = 512;
constexpr int kTileItems = 16;
constexpr int kTile = kTileThreads * kTileItems;  // 8192 keys

// Step 4 merge: one workgroup merges one partition of at most kPart keys.
constexpr int kMergeThreads = 512;
constexpr int kMergeItems = 16;
constexpr int kPart = kMergeThreads * kMergeItems;  // 8192 keys
// Outputs per thread and round of the LDS merge rounds: with at most 32 pairs
// per round, ceil-rounded chunks of 17 keys still fit in kMergeThreads
// ((8192 + 32 * 16) / 17 <= 512).
constexpr int kRoundItems = 17;
// Keys-only merges keep this many slots of the largest key after every run in
// LDS (at least kRoundItems), so their merge steps need no bound checks.
constexpr uint32_t kGap = kRoundItems + 1;

// Key-value sorts of the automatic plan hold 12 bytes a key in LDS.  Tiles of
// 8192 keys would leave one workgroup per CU, so they sort tiles of 4096 keys
// (256 threads; three workgroups per CU) and merge partitions of 4096 keys in
// chunks of 9 outputs per thread (two 1024-thread workgroups per CU), with up
// to 64 runs per pass so that 2^28 keys still take three passes.
constexpr int kTileKVThreads = 256;
constexpr int kTileKV = kTileKVThreads * kTileItems;  // 4096 keys
constexpr int kPartKV = 4096;
constexpr int kRoundItemsKV = 9;
constexpr int kMaxFanLog2KV = 6;

// Step 2 splitter search: one 64-lane workgroup per splitter.
constexpr int kCorankThreads = 64;
// Largest number of runs one splitter search handles (LDS-bound: the
// candidate set of one level is below 3 * runs).
constexpr uint32_t kMaxRuns = 2048;
// Runs merged by one pass of the automatic plan (powers of two); the
// segmented mode's default (its tuning may choose 6).
constexpr int kMaxFanLog2 = 5;

// Every sorted run also leaves a regular sample: the keys at run positions
// kSample*i + kSample-1.  A pass merges the samples first and reads the top
// levels of every splitter search off the merged samples.
constexpr int kSampleLog2 = 5;
constexpr uint32_t kSample = 1u << kSampleLog2;
// Merged samples carry per-run prefix counts every kChunk entries.
constexpr uint32_t kChunk = 64;
// Largest fan-in for which the sampled search is used (the automatic plan's
// passes merge at most 32 runs; the paper's single level up to 256 blocks).
constexpr uint32_t kMaxSampledFan = 256;

// Per-segment tables of the batched segmented sort (all device arrays, filled
// on the device by the planning kernel).  off == nullptr: not segmented.
struct SegTables {
  const uint64_t *off;    // key offsets of the segments [n_segs + 1]
  const uint64_t *soff;   // offsets of each segment's samples [n_segs + 1]
  const uint32_t *npass;  // merge passes each segment needs
  const uint64_t *rows;   // prefix over segments of this pass's table rows
  const uint64_t *parts;  // prefix over segments of this pass's partitions
  const uint64_t *sparts; // prefix over segments of this pass's sample partitions
  uint32_t n_segs;
  uint32_t pass;   // 1-based merge pass described by this geometry
  uint32_t level;  // 0 = keys, 1 = the sample array
};

// Geometry of one merge pass.  The array is cut into uniform segments of
// seg_len keys (the last one short); inside a segment, sorted runs of run_len
// keys are merged in groups of `fan` runs, each group's output cut into
// partitions of part_len keys.  In paper mode there is exactly one group (the
// whole array, runs = the paper's blocks) and partition boundaries are the
// paper's r_k = floor(k N / n_P), each paper partition further cut into
// sub_per_part chunks of at most part_len keys.
struct RunGeom {
  uint64_t n;
  uint64_t seg_len;
  uint64_t run_len;
  uint32_t fan;
  uint64_t group_len;       // min(fan * run_len, seg_len)
  uint64_t groups_per_seg;  // ceil(seg_len / group_len)
  uint64_t n_groups;        // n_segments * groups_per_seg
  uint32_t rows_per_group;  // partitions per full group + 1
  uint32_t part_len;
  int paper;
  uint32_t n_parts;       // paper mode: n_P
  uint32_t sub_per_part;  // paper mode: chunks per paper partition
  SegTables seg;          // segmented mode (seg.off != nullptr)
  uint64_t row_bound;     // segmented mode: grid upper bound for rows
  uint64_t part_bound;    // segmented mode: grid upper bound for partitions
  // Paper mode with partitions that follow the data (regular-sampling
  // pivots): device arrays of the partitions' first ranks [n_parts + 1] and
  // of the exclusive prefix over partitions of their chunk counts
  // ceil(size / part_len) [n_parts + 1].  Table rows are then the chunk
  // boundaries in order (at most chunk_bound chunks), not sub_per_part rows
  // per partition.
  const uint64_t *bounds;
  const uint64_t *chunk_prefix;
  uint64_t chunk_bound;
  uint64_t total_rows() const {
    if (seg.off) return row_bound;
    if (paper && bounds) return chunk_bound + 1;
    return paper ? (uint64_t)n_parts * sub_per_part + 1 : n_groups * rows_per_group;
  }
  uint64_t total_parts() const {
    if (seg.off) return part_bound;
    if (paper && bounds) return chunk_bound;
    return paper ? (uint64_t)n_parts * sub_per_part : n_groups * (rows_per_group - 1);
  }
};

// A vector of at most N elements held inline: the launch plans of a sort
// use it so that planning and launching a sort allocate no memory.
template <typename T, int N> class FixedVec {
 public:
  size_t size() const { return n_; }
  bool empty() const { return n_ == 0; }
  // false (and nothing stored) when full
  bool push_back(const T &v) {
    if (n_ >= (size_t)N) return false;
    a_[n_++] = v;
    return true;
  }
  T &operator[](size_t i) { return a_[i]; }
  const T &operator[](size_t i) const { return a_[i]; }
  T *data() { return a_; }
  const T *begin() const { return a_; }
  const T *end() const { return a_ + n_; }

 private:
  T a_[N] = {};
  size_t n_ = 0;
};

// Merge passes one plan may hold (n < 2^31 needs at most 7 at fan-in 32).
constexpr int kMaxPlanPasses = 8;

// Bits of the device error word (see read_device_error).
constexpr uint32_t kErrCandidates = 1u;  // splitter search: candidate set overflow
constexpr uint32_t kErrBracket = 2u;     // splitter search: target outside bracket
constexpr uint32_t kErrSplitRow = 4u;    // merge: split row not inside its run
constexpr uint32_t kErrPartSize = 8u;    // merge: segments do not add up to the partition
constexpr uint32_t kErrSegments = 16u;   // segmented sort: offsets invalid or too many passes

// Largest number of merge passes of one segment (n < 2^31: 2^18 tiles, 5
// doublings per pass).
constexpr uint32_t kMaxSegPasses = 4;

// Synchronous read (and optional clear) of the device error word.
hipError_t read_device_error(uint32_t *code, bool clear);
// Copy of the device error word into host memory (pinned, for the copy to
// be asynchronous) queued on stream s; the word is left as it is.
hipError_t read_device_error_async(uint32_t *host_code, hipStream_t s);

// Fault injection for tests (pss_debug_inject): kinds of operation that can be
// made to fail.  inject_fault(kind) is called before each such operation and
// returns true for the one operation armed to fail, which the caller then
// reports as a failure without performing it.  Process-wide, thread-safe.
constexpr int kInjectLaunch = 1;  // queued device work: launches, async copies
constexpr int kInjectAlloc = 2;   // device or pinned host allocations
bool inject_fault(int kind);

// Set the calling thread's error message (pss_last_error(NULL)).
void set_thread_error(const char *msg);

// HIP device a context is bound to.
int ctx_device(const pss_ctx *ctx);
// Record msg as the context's (and the calling thread's) last error.
pss_status ctx_fail(const pss_ctx *ctx, pss_status s, const char *msg);
// Turn a context's per-launch timing on or off; returns the previous setting.
bool ctx_set_profiling(pss_ctx *ctx, bool on);
// Look up, once per device and with that device current, the device address
// of the allocation-free entry point's scratch array (pss_create calls it).
hipError_t scratch_setup(int device);

// Whether an enum argument, which a C caller may have set to any int, holds
// one of 0..max.  Its bits are read as an int and never loaded as the C++
// enum, since loading a value outside the enumerators is undefined in C++.
template <typename E> inline bool valid_enum(const E &e, int max) {
  static_assert(sizeof(E) == sizeof(int), "enum held as int");
  int v;
  std::memcpy(&v, &e, sizeof v);
  return v >= 0 && v <= max;
}

// key-type codes (same numbering as pss_key_t)
inline int key_bytes(int kt) { return (kt == 0 || kt == 1 || kt == 4) ? 4 : 8; }

// Geometry of the sample array of the runs described by g (same groups).
RunGeom sample_geom(const RunGeom &g);

// Tile sizes of the segmented mode's small-segment classes.
constexpr int kSmallThreads0 = 128;  // 2048-key tiles
constexpr int kSmallThreads1 = 256;  // 4096-key tiles

// Device arrays of the segmented plan (see seg_plan_kernel).
struct SegPlanPtrs {
  uint64_t *tiles[3];
  uint64_t *soff;
  uint32_t *npass;
  uint64_t *rows[kMaxSegPasses], *parts[kMaxSegPasses];
  uint64_t *srows[kMaxSegPasses], *sparts[kMaxSegPasses];
};

// Second buffer set of a segmented merge (X_j not in the primary buffers).
struct MergeAlt {
  const void *src;
  const uint32_t *vsrc;
  void *dst;
  uint32_t *vdst;
};

// samples: optional output, every kSample-th key of each sorted tile.
// tile: kTile, or kTileKV (key-value sorts only).
hipError_t launch_tile_sort(int kt, bool kv, const void *in, const uint32_t *vin, void *out,
                            uint32_t *vout, uint64_t n, uint64_t seg_len, uint32_t tile,
                            int final_pass, void *samples, hipStream_t s);
hipError_t launch_seg_plan(const uint64_t *seg_off, uint32_t n_segs, uint64_t n,
                           const SegPlanPtrs &pp, uint32_t small0, uint32_t small1,
                           uint32_t max_passes, uint32_t fan_log2, uint32_t tile, uint32_t part,
                           hipStream_t s);
hipError_t launch_seg_tile_sorts(int kt, bool kv, const void *in, const uint32_t *vin, void *out,
                                 void *out_alt, uint32_t *vout, uint32_t *vout_alt, void *samples,
                                 const uint64_t *seg_off, const SegPlanPtrs &pp, uint32_t n_segs,
                                 uint64_t n, uint32_t tile, hipStream_t s);
// src_alt: segmented mode's second input buffer (nullptr = same as src).
hipError_t launch_corank(int kt, const void *src, const RunGeom &g, uint32_t *table,
                         void *pivots, uint64_t *counts, hipStream_t s,
                         const void *src_alt = nullptr);
// Splitter search that starts from the merged samples (see merge mode 2).
// gs: geometry of the sample array (nullptr = derived from g, uniform mode).
hipError_t launch_corank_sampled(int kt, const void *src, const RunGeom &g, uint32_t *table,
                                 const uint32_t *sample_runs, const uint32_t *sample_prefix,
                                 hipStream_t s, const void *src_alt = nullptr,
                                 const RunGeom *gs = nullptr);
// vmode 0: keys only; 1: keys + uint32 payload; 2: merge of a sample array,
// payload = source run index, per-run prefix counts written to `prefix`.
// samples: optional output, every kSample-th key of each output run.
hipError_t launch_merge(int kt, int vmode, const void *src, const uint32_t *vsrc, void *dst,
                        uint32_t *vdst, const RunGeom &g, const uint32_t *table,
                        const uint64_t *part_offsets, int final_pass, void *samples,
                        uint32_t *prefix, hipStream_t s, const MergeAlt *alt = nullptr);
hipError_t launch_partition_offsets(const RunGeom &g, const uint32_t *table, uint64_t *sizes,
                                    uint64_t *offsets, hipStream_t s);
hipError_t launch_split_table(const RunGeom &g, const uint32_t *table, uint64_t *split,
                              hipStream_t s);
hipError_t launch_unmap_copy(int kt, const void *src, void *dst, uint64_t n, hipStream_t s);

// Step 4 of the paper's single level by sorting each gathered chunk instead
// of merging its segments (paper-mode geometry only).
hipError_t launch_sort_merge(int kt, bool kv, const void *src, const uint32_t *vsrc, void *dst,
                             uint32_t *vdst, const RunGeom &g, const uint32_t *table,
                             const uint64_t *part_offsets, int final_pass, hipStream_t s);

// Records: their keys (raw, of type kt, at key_offset) and input indices;
// and the gather out[j] = in[perm[j]] of whole records (record_bytes a
// multiple of 4 and at most 4096).
hipError_t launch_record_keys(int kt, const void *records, uint64_t n, uint32_t record_bytes,
                              uint32_t key_offset, void *keys, uint32_t *idx, hipStream_t s);
hipError_t launch_record_gather(const void *in, void *out, const uint32_t *perm, uint64_t n,
                                uint32_t record_bytes, hipStream_t s);

// Regular-sampling (PSRS) pivots over the sorted blocks of g (paper mode;
// blocks hold mapped keys).  samples: n_P - 1 keys from each non-empty block.
hipError_t launch_psrs_samples(int kt, const void *blocks, const RunGeom &g, void *samples,
                               hipStream_t s);
// From the sorted samples (ns keys): the pivots P_k = S[floor(k ns / n_P)],
// the partition boundaries of every block (elements <= P_k), and the
// partitions' first ranks bounds[0..n_P].  pivots (unmapped) and split
// ([n_B][n_P + 1]) are optional outputs.
hipError_t launch_psrs_partition(int kt, const void *blocks, const RunGeom &g,
                                 const void *sorted_samples, uint64_t ns, uint64_t *bounds,
                                 void *pivots, uint64_t *split, hipStream_t s);
// Partition sizes (optional output) and the exclusive prefix of their chunk
// counts, from bounds.
hipError_t launch_psrs_chunks(const RunGeom &g, const uint64_t *bounds, uint64_t *sizes,
                              uint64_t *chunks, uint64_t *chunk_prefix, hipStream_t s);

}  // namespace pss
