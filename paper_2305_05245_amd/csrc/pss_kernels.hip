// HIP kernels for gfx950 (MI355X) implementing the hot path of parallel
// samplesort with exact splitting (PSES), arXiv 2305.05245, Section 2:
//
//   K0  order-preserving key map fused into the first load and the last store
//   K1  step 1 ("sorting each block"): LDS-resident tile sort
//   K2  step 2 (PSES pivot selection, Section 2.3, Eq. 1 and Eq. 2): exact
//       splitting by a bracketed bit-by-bit co-rank search over all sorted runs
//   K3  step 3 (partitioning): the split positions of every run, one table row
//       per splitter; a sorted run's partitions are contiguous, so no data moves
//   K4  offsets of the merged partitions: a device reduction and exclusive scan
//   K5  step 4 (multiway merging of partitions): one workgroup per partition
//       gathers the partition's segments from all runs into LDS and merges them
//       with rounds of stable merge-path merges, then stores coalesced.
//
// Keys are compared only as unsigned integers after the K0 map (signed ints:
// sign bit flipped; floats: IEEE totalOrder map), so every comparison is an
// integer comparison and the output is bit-exact.
#include "pss_internal.hpp"

#include <type_traits>

namespace pss {

// Set (bitwise or) by a kernel that finds one of its invariants broken; the
// kernel then stops before touching memory outside its own partition.
__device__ uint32_t g_device_error = 0;

namespace {

__device__ __forceinline__ void report(uint32_t code) { atomicOr(&g_device_error, code); }

// ------------------------------------------------------------------ K0 ----
template <int KT> struct Key;
template <> struct Key<0> {  // uint32
  using U = uint32_t;
  static __device__ __forceinline__ U map(U x) { return x; }
  static __device__ __forceinline__ U unmap(U x) { return x; }
};
template <> struct Key<1> {  // int32: flip the sign bit
  using U = uint32_t;
  static __device__ __forceinline__ U map(U x) { return x ^ 0x80000000u; }
  static __device__ __forceinline__ U unmap(U x) { return x ^ 0x80000000u; }
};
template <> struct Key<2> {  // uint64
  using U = uint64_t;
  static __device__ __forceinline__ U map(U x) { return x; }
  static __device__ __forceinline__ U unmap(U x) { return x; }
};
template <> struct Key<3> {  // int64
  using U = uint64_t;
  static __device__ __forceinline__ U map(U x) { return x ^ 0x8000000000000000ull; }
  static __device__ __forceinline__ U unmap(U x) { return x ^ 0x8000000000000000ull; }
};
template <> struct Key<4> {  // float32, IEEE totalOrder: negative -> all bits
  using U = uint32_t;        // inverted, otherwise the sign bit set
  static __device__ __forceinline__ U map(U x) {
    return (x & 0x80000000u) ? ~x : (x | 0x80000000u);
  }
  static __device__ __forceinline__ U unmap(U x) {
    return (x & 0x80000000u) ? (x & 0x7fffffffu) : ~x;
  }
};
template <> struct Key<5> {  // float64, IEEE totalOrder
  using U = uint64_t;
  static __device__ __forceinline__ U map(U x) {
    return (x & 0x8000000000000000ull) ? ~x : (x | 0x8000000000000000ull);
  }
  static __device__ __forceinline__ U unmap(U x) {
    return (x & 0x8000000000000000ull) ? (x & 0x7fffffffffffffffull) : ~x;
  }
};

template <typename U>
__device__ __forceinline__ U unmap_runtime(U x, int kt) {
  if constexpr (sizeof(U) == 4) {
    switch (kt) {
      case 1: return Key<1>::unmap(x);
      case 4: return Key<4>::unmap(x);
      default: return x;
    }
  } else {
    switch (kt) {
      case 3: return Key<3>::unmap(x);
      case 5: return Key<5>::unmap(x);
      default: return x;
    }
  }
}

template <typename U> __device__ __forceinline__ constexpr U key_max() { return ~U(0); }

// The same value, hidden from the optimiser (an empty asm that "changes" its
// register).  A compare-exchange written as two selects on one comparison
// would otherwise be rewritten as a minimum and a maximum, which the 64-bit
// lowering computes with one comparison each; selecting between opaque
// copies keeps one comparison for both selects.
template <typename U> __device__ __forceinline__ U opaque(U x) {
  asm("" : "+v"(x));
  return x;
}

// LDS index with one pad slot after every 16 keys, so that a thread reading or
// writing its 16 consecutive keys does not hit the same bank as its neighbours.
__device__ __forceinline__ uint32_t pad16(uint32_t i) { return i + (i >> 4); }

// Order LDS accesses within one wave: everything this wave wrote before is
// visible to everything it reads after (no other wave takes part).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ----------------------------------------------------- sorting networks ----
// Index pairs of Batcher's odd-even merge sort on N registers (unstable,
// keys only) and of odd-even transposition sort (stable: only neighbours are
// compared and equal keys are never swapped), generated at compile time.
template <int N> constexpr int batcher_pairs() {
  int c = 0;
  for (int p = 1; p < N; p <<= 1)
    for (int k = p; k >= 1; k >>= 1)
      for (int j = k % p; j + k < N; j += 2 * k)
        for (int i = 0; i < k && i + j + k < N; ++i)
          if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) ++c;
  return c;
}
template <int N> struct BatcherNet {
  int a[batcher_pairs<N>()];
  int b[batcher_pairs<N>()];
  constexpr BatcherNet() : a(), b() {
    int c = 0;
    for (int p = 1; p < N; p <<= 1)
      for (int k = p; k >= 1; k >>= 1)
        for (int j = k % p; j + k < N; j += 2 * k)
          for (int i = 0; i < k && i + j + k < N; ++i)
            if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) {
              a[c] = i + j;
              b[c] = i + j + k;
              ++c;
            }
  }
};
template <int N> constexpr int transposition_pairs() { return (N / 2) * ((N + 1) / 2) + ((N - 1) / 2) * (N / 2); }
template <int N> struct TranspositionNet {
  int a[transposition_pairs<N>()];
  constexpr TranspositionNet() : a() {
    int c = 0;
    for (int phase = 0; phase < N; ++phase)
      for (int i = phase & 1; i + 1 < N; i += 2) a[c++] = i;
  }
};

template <typename U, bool KV, int N>
__device__ __forceinline__ void register_sort(U (&k)[N], uint32_t (&v)[KV ? N : 1]) {
  if constexpr (!KV) {
    constexpr BatcherNet<N> net{};
#pragma unroll
    for (int c = 0; c < batcher_pairs<N>(); ++c) {
      const U x = k[net.a[c]], y = k[net.b[c]];
      const bool lt = x < y;
      const U ox = opaque(x), oy = opaque(y);
      k[net.a[c]] = lt ? ox : oy;
      k[net.b[c]] = lt ? oy : ox;
    }
  } else {
    constexpr TranspositionNet<N> net{};
#pragma unroll
    for (int c = 0; c < transposition_pairs<N>(); ++c) {
      const int i = net.a[c];
      const bool s = k[i + 1] < k[i];
      const U x = k[i], y = k[i + 1];
      const uint32_t vx = v[i], vy = v[i + 1];
      k[i] = s ? y : x;
      k[i + 1] = s ? x : y;
      v[i] = s ? vy : vx;
      v[i + 1] = s ? vx : vy;
    }
  }
}

// Largest s in [0, n_segs) with prefix[s] <= idx (prefix[0] = 0): the segment
// whose range of a prefix-summed count contains idx.
__device__ __forceinline__ uint32_t seg_find(const uint64_t *prefix, uint32_t n_segs, uint64_t idx) {
  uint32_t lo = 0, hi = n_segs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (prefix[mid] <= idx) lo = mid;
    else hi = mid;
  }
  return lo;
}

// LDS slot of index i: the padded layout (one spare slot after every 16, for
// phases where each thread reads or writes 16 consecutive slots) or flat.
template <bool PAD> __device__ __forceinline__ uint32_t lds_at(uint32_t i) {
  return PAD ? pad16(i) : i;
}

// One chunk of a stable pairwise merge in LDS: the CI outputs from `start` on
// of merging A = [A0, A1) and B = [A1, B1) (ties to A), into registers.  The
// merge-path search finds how many of the first start-A0 outputs come from A;
// then one output per step.  Outputs at or past B1 (only in a pair's last
// chunk) are meaningless and must not be stored; computing them reads at
// most CI slots past B1, which every LDS array using this leaves as slack.
template <typename U, bool KV, int CI, bool PAD>
__device__ __forceinline__ void merge_chunk(const U *sk, const uint32_t *sv, uint32_t A0,
                                            uint32_t A1, uint32_t B1, uint32_t start,
                                            U (&rk)[CI], uint32_t (&rv)[KV ? CI : 1]) {
  const uint32_t la = A1 - A0, lb = B1 - A1, d = start - A0;
  uint32_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sk[lds_at<PAD>(A0 + mid)] <= sk[lds_at<PAD>(A1 + d - 1 - mid)]) lo = mid + 1;
    else hi = mid;
  }
  uint32_t pa = A0 + lo, pb = A1 + (d - lo);
  U ka = sk[lds_at<PAD>(pa)], kb = sk[lds_at<PAD>(pb)];
  uint32_t va = 0, vb = 0;
  if constexpr (KV) {
    va = sv[lds_at<PAD>(pa)];
    vb = sv[lds_at<PAD>(pb)];
  }
#pragma unroll
  for (int i = 0; i < CI; ++i) {
    const bool takeA = pa < A1 && (pb >= B1 || ka <= kb);
    rk[i] = takeA ? ka : kb;
    if constexpr (KV) rv[i] = takeA ? va : vb;
    const uint32_t nxt = (takeA ? pa : pb) + 1;
    const U nk = sk[lds_at<PAD>(nxt)];
    ka = takeA ? nk : ka;
    kb = takeA ? kb : nk;
    if constexpr (KV) {
      const uint32_t nv = sv[lds_at<PAD>(nxt)];
      va = takeA ? nv : va;
      vb = takeA ? vb : nv;
    }
    pa += takeA ? 1u : 0u;
    pb += takeA ? 0u : 1u;
  }
}

// Keys-only chunk merge of two runs that are each followed in LDS by at least
// CI copies of the largest key: A = sk[a0, a0 + la), B = sk[b0, b0 + lb).  It
// produces outputs d .. d+CI-1 of their merged order.  After the merge-path
// search, every step outputs the smaller of the two heads and replaces it with
// the next key of its run.  Equal keys are bit-identical, so which run
// supplies a tie does not change the output; a used-up run shows the largest
// key from its gap, so no bound checks are needed, and a chunk reads at most
// CI slots past the end of a run.
template <typename U, int CI>
__device__ __forceinline__ void merge_chunk_keys(const U *sk, uint32_t a0, uint32_t la,
                                                 uint32_t b0, uint32_t lb, uint32_t d,
                                                 U (&rk)[CI]) {
  uint32_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (sk[a0 + mid] <= sk[b0 + d - 1 - mid]) lo = mid + 1;
    else hi = mid;
  }
  // positions as LDS byte offsets, so a step needs no index arithmetic
  const uint32_t pa = (a0 + lo) * (uint32_t)sizeof(U), pb = (b0 + (d - lo)) * (uint32_t)sizeof(U);
  const char *base = reinterpret_cast<const char *>(sk);
  const U ka = *reinterpret_cast<const U *>(base + pa);
  const U kb = *reinterpret_cast<const U *>(base + pb);
  const bool af = ka <= kb;
  U x = af ? ka : kb, y = af ? kb : ka;  // x: the next output, y: the other head
  uint32_t px = af ? pa : pb, py = af ? pb : pa;
#pragma unroll
  for (int i = 0; i < CI; ++i) {
    rk[i] = x;
    const uint32_t pn = px + (uint32_t)sizeof(U);
    const U nk = *reinterpret_cast<const U *>(base + pn);
    const bool keep = nk <= y;
    const U onk = opaque(nk), oy = opaque(y);
    const U nx = keep ? onk : oy, ny = keep ? oy : onk;
    const uint32_t npx = keep ? pn : py, npy = keep ? py : pn;
    x = nx;
    y = ny;
    px = npx;
    py = npy;
  }
}

// Keys only: merge the sorted 16-key runs held by single lanes into sorted
// 128-key runs held by groups of eight lanes (lane j of a group then holds the
// run's keys 16j..16j+15), with bitonic merge networks: a "flip" stage pairs
// key i of the lower run with key n-1-i of the upper one across lanes, then
// half-cleaners at falling distances, the last four inside each lane.  Lane
// exchanges use DPP moves (quad permutations and the half-row mirror).
template <typename U>
__device__ __forceinline__ void inlane_half_cleaners(U (&k)[kTileItems]) {
#pragma unroll
  for (int d = kTileItems / 2; d >= 1; d >>= 1) {
#pragma unroll
    for (int i = 0; i < kTileItems; ++i) {
      if ((i & d) == 0) {
        const U a = k[i], b = k[i + d];
        const bool sw = b < a;
        const U oa = opaque(a), ob = opaque(b);
        k[i] = sw ? ob : oa;
        k[i + d] = sw ? oa : ob;
      }
    }
  }
}

// x from the lane given by the DPP control CTRL (all lanes active)
template <int CTRL, typename U>
__device__ __forceinline__ U dpp_from(U x) {
  if constexpr (sizeof(U) == 8) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, 0xF, 0xF, false);
    return ((U)(uint32_t)hi << 32) | (U)(uint32_t)lo;
  } else {
    return (U)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
  }
}

constexpr int kDppXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kDppXor3 = 0x1B;  // quad_perm [3,2,1,0]
constexpr int kDppXor7 = 0x141; // row_half_mirror: lane i of 8 reads lane 7-i
constexpr int kDppRor8 = 0x128; // row_ror:8: lane i of 16 reads lane i xor 8

// x from lane (lane xor 16) within each half of the wave (swizzle unit)
template <typename T>
__device__ __forceinline__ T swizzle_xor16(T x) {
  constexpr int kPattern = (0x10 << 10) | 0x1F;  // bit mode: and 0x1f, or 0, xor 0x10
  if constexpr (sizeof(T) == 8) {
    const int lo = __builtin_amdgcn_ds_swizzle((int)(uint32_t)x, kPattern);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(uint32_t)((uint64_t)x >> 32), kPattern);
    return (T)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
  } else {
    return (T)__builtin_amdgcn_ds_swizzle((int)x, kPattern);
  }
}

// x from lane (lane xor D): DPP moves for D <= 8 (xor 4 is the half-row
// mirror followed by the quad reversal), the swizzle unit for 16, a full
// cross-lane permute beyond
template <int D, typename T>
__device__ __forceinline__ T shfl_xor_c(T x) {
  if constexpr (D == 1) return dpp_from<kDppXor1>(x);
  else if constexpr (D == 2) return dpp_from<kDppXor2>(x);
  else if constexpr (D == 4) return dpp_from<kDppXor3>(dpp_from<kDppXor7>(x));
  else if constexpr (D == 8) return dpp_from<kDppRor8>(x);
  else if constexpr (D == 16) return swizzle_xor16(x);
  else return __shfl_xor(x, D, 64);
}

template <int CTRL, bool FLIP, typename U>
__device__ __forceinline__ void cross_lane_stage(U (&k)[kTileItems], bool upper) {
  U o[kTileItems];
#pragma unroll
  for (int i = 0; i < kTileItems; ++i) o[i] = dpp_from<CTRL>(k[FLIP ? kTileItems - 1 - i : i]);
#pragma unroll
  for (int i = 0; i < kTileItems; ++i) {
    const bool lt = o[i] < k[i];
    k[i] = (lt != upper) ? o[i] : k[i];  // lower lane keeps the minimum, upper the maximum
  }
}

template <typename U>
__device__ __forceinline__ void lane_runs_to_128(U (&k)[kTileItems], uint32_t lane) {
  cross_lane_stage<kDppXor1, true>(k, (lane & 1) != 0);  // runs of 16 -> 32
  inlane_half_cleaners(k);
  cross_lane_stage<kDppXor3, true>(k, (lane & 2) != 0);  // runs of 32 -> 64
  cross_lane_stage<kDppXor1, false>(k, (lane & 1) != 0);
  inlane_half_cleaners(k);
  cross_lane_stage<kDppXor7, true>(k, (lane & 4) != 0);  // runs of 64 -> 128
  cross_lane_stage<kDppXor2, false>(k, (lane & 2) != 0);
  cross_lane_stage<kDppXor1, false>(k, (lane & 1) != 0);
  inlane_half_cleaners(k);
}

// --------------------------------------------------------------- K1 -------
// One workgroup sorts one tile of THREADS * 16 keys of one segment.  Keys
// are mapped on load (K0) and each thread sorts 16 of them in registers (the
// ones it loaded for keys only, 16 consecutive ones for key-value tiles); then
// runs are merged, across lanes and through LDS, up to the whole tile.  A
// short tile is padded with the largest key; pads sit after every real key
// (for key-value sorts the network and merges are stable, so pads stay last).
// Where one tile-sort workgroup reads and writes.  Uniform mode: tiles of
// kTile keys in uniform segments.  Segmented mode: `tiles` is the prefix over
// segments of the tiles of this launch's tile size (0 for segments another
// tile size handles); outputs go to the primary or alt buffer by the parity of
// the segment's merge passes, and only segments with merge passes leave
// samples.
template <typename U> struct TileArgs {
  uint64_t n, seg_len, tiles_per_seg;
  int final_pass;
  U *out, *out_alt;
  uint32_t *vout, *vout_alt;
  U *samples;
  const uint64_t *seg_off, *tiles, *soff;
  const uint32_t *npass;
  uint32_t n_segs;
};

template <int KT, bool KV, int THREADS>
__global__ __launch_bounds__(THREADS) void tile_sort_kernel(
    const typename Key<KT>::U *__restrict__ in, const uint32_t *__restrict__ vin,
    TileArgs<typename Key<KT>::U> ta) {
  using U = typename Key<KT>::U;
  constexpr uint32_t TILE = THREADS * kTileItems;
  // Key-value tiles: the padded layout of TILE slots.  Keys-only tiles: also
  // every wave's region of gapped runs (see below).  Both plus the slack a
  // merge chunk may read.
  constexpr uint32_t RW = 64 * kTileItems + (64 * kTileItems / 256) * kGap;
  constexpr uint32_t PADDED = TILE + TILE / 16;
  constexpr uint32_t GAPPED = (THREADS / 64) * RW;
  constexpr uint32_t P = (KV || PADDED > GAPPED ? PADDED : GAPPED) + 2 * kRoundItems + 2;
  // Padded layout (one spare slot per 16 keys).  Keys-only tiles place each
  // wave's 1024 keys at the start of that wave's region of RW slots, so the
  // wave later merges from the padded into the gapped layout on its own.
  auto tile_pad = [](uint32_t idx) -> uint32_t {
    return KV ? pad16(idx) : (idx >> 10) * RW + pad16(idx & 1023u);
  };
  __shared__ U sk[P];
  __shared__ uint32_t sv[KV ? P : 1];

  const uint32_t tid = threadIdx.x;
  const uint64_t t = blockIdx.x;
  uint64_t start, sbase = 0;
  uint32_t len;
  U *out = ta.out, *samples = ta.samples;
  uint32_t *vout = ta.vout;
  int final_pass = ta.final_pass;
  if (ta.seg_off) {
    if (t >= ta.tiles[ta.n_segs]) return;
    const uint32_t sg = seg_find(ta.tiles, ta.n_segs, t);
    const uint64_t j = t - ta.tiles[sg];
    const uint64_t slen = ta.seg_off[sg + 1] - ta.seg_off[sg];
    start = ta.seg_off[sg] + j * (uint64_t)TILE;
    len = (uint32_t)(slen - j * TILE < (uint64_t)TILE ? slen - j * TILE : TILE);
    const uint32_t np = ta.npass[sg];
    if (np & 1u) {  // X_0 is the output only after an even number of passes
      out = ta.out_alt;
      vout = ta.vout_alt;
    }
    final_pass = np == 0;
    if (np == 0) samples = nullptr;
    sbase = ta.soff[sg] + ((j * (uint64_t)TILE) >> kSampleLog2);
  } else {
    const uint64_t seg = t / ta.tiles_per_seg, j = t % ta.tiles_per_seg;
    const uint64_t seg_start = seg * ta.seg_len;
    if (seg_start >= ta.n) return;
    const uint64_t seg_end = seg_start + ta.seg_len < ta.n ? seg_start + ta.seg_len : ta.n;
    start = seg_start + j * (uint64_t)TILE;
    if (start >= seg_end) return;
    len = (uint32_t)(seg_end - start < (uint64_t)TILE ? seg_end - start : TILE);
    sbase = seg * (ta.seg_len >> kSampleLog2) + ((j * (uint64_t)TILE) >> kSampleLog2);
  }

  // All loads first (clamped into the tile, so none is conditional and all
  // are in flight together), then the key map and the padding of a short
  // tile with the largest key.
  U raw[kTileItems];
  uint32_t vraw[KV ? kTileItems : 1];
#pragma unroll
  for (int i = 0; i < kTileItems; ++i) {
    const uint32_t idx = i * THREADS + tid;
    const uint32_t j = idx < len ? idx : len - 1;  // len >= 1 for every tile launched
    raw[i] = __builtin_nontemporal_load(&in[start + j]);  // read once
    if constexpr (KV) vraw[i] = __builtin_nontemporal_load(&vin[start + j]);
  }
  U rk[kTileItems];
  uint32_t rv[KV ? kTileItems : 1];
  if constexpr (KV) {
    // A stable sort needs each thread's keys to be consecutive in the input:
    // through LDS, from the coalesced load order to 16 consecutive keys.
#pragma unroll
    for (int i = 0; i < kTileItems; ++i) {
      const uint32_t idx = i * THREADS + tid;
      sk[tile_pad(idx)] = idx < len ? Key<KT>::map(raw[i]) : key_max<U>();
      sv[pad16(idx)] = idx < len ? vraw[i] : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kTileItems; ++i) {
      const uint32_t idx = tid * kTileItems + i;
      rk[i] = sk[tile_pad(idx)];
      rv[i] = sv[pad16(idx)];
    }
  } else {
    // Keys only: which 16 keys of the tile a thread sorts does not matter,
    // so it sorts the ones it loaded (tile positions i * THREADS + tid).
#pragma unroll
    for (int i = 0; i < kTileItems; ++i) {
      const uint32_t idx = i * THREADS + tid;
      rk[i] = idx < len ? Key<KT>::map(raw[i]) : key_max<U>();
    }
  }
  register_sort<U, KV, kTileItems>(rk, rv);
  if constexpr (KV) {
    // every wave writes back the keys it read (its own 1024 positions)
    wave_sync();
  #pragma unroll
    for (int i = 0; i < kTileItems; ++i) {
      const uint32_t idx = tid * kTileItems + i;
      sk[pad16(idx)] = rk[i];
      if constexpr (KV) sv[pad16(idx)] = rv[i];
    }
    wave_sync();

    // Rounds of pairwise merges of runs of L keys.  Each pair's output is cut
    // into chunks of CI keys (never crossing into the next pair), one chunk per
    // thread: at most THREADS chunks per round.  The first round reads the
    // padded layout; every round writes the flat one (CI is odd, so the
    // threads' chunk stores do not collide in LDS banks).  While a pair fits in
    // the 1024 keys that one wave's threads sorted, each wave merges only its
    // own keys and, after the first round, synchronises only with itself.
    constexpr int CI = kRoundItems;
    constexpr uint32_t WKEYS = 64 * kTileItems;  // keys per wave
    U mk[CI];
    uint32_t mv[KV ? CI : 1];
    const uint32_t lane = tid & 63, wbase = (tid >> 6) * WKEYS;
    uint32_t L = kTileItems;
    for (; L < TILE && 2 * L <= WKEYS; L *= 2) {
      const uint32_t cpp = (2 * L + CI - 1) / CI;  // chunks per pair
      const uint32_t q = lane / cpp, c = lane - q * cpp;
      const bool active = q < WKEYS / (2 * L);
      const uint32_t A0 = wbase + q * 2 * L;
      const uint32_t cs = A0 + c * CI;  // this thread's first output
      const uint32_t count = active ? (A0 + 2 * L - cs < (uint32_t)CI ? A0 + 2 * L - cs : CI) : 0;
      if (active) {
        if (L == kTileItems)
          merge_chunk<U, KV, CI, true>(sk, sv, A0, A0 + L, A0 + 2 * L, cs, mk, mv);
        else
          merge_chunk<U, KV, CI, false>(sk, sv, A0, A0 + L, A0 + 2 * L, cs, mk, mv);
      }
      // The first round moves every wave's keys from the padded layout to the
      // flat one, whose slots overlap the previous wave's padded ones: all
      // waves must finish reading first.  Later rounds stay in the wave's own
      // flat slots.
      if (L == kTileItems) __syncthreads();
      else wave_sync();
  #pragma unroll
      for (int i = 0; i < CI; ++i) {
        if ((uint32_t)i < count) {
          sk[cs + i] = mk[i];
          if constexpr (KV) sv[cs + i] = mv[i];
        }
      }
      wave_sync();
    }
    __syncthreads();
    for (; L < TILE; L *= 2) {
      const uint32_t cpp = (2 * L + CI - 1) / CI;  // chunks per pair
      const uint32_t q = tid / cpp, c = tid - q * cpp;
      const uint32_t A0 = q * 2 * L;
      const bool active = A0 < TILE;
      const uint32_t cs = A0 + c * CI;  // this thread's first output
      const uint32_t count = active ? (A0 + 2 * L - cs < (uint32_t)CI ? A0 + 2 * L - cs : CI) : 0;
      if (active) merge_chunk<U, KV, CI, false>(sk, sv, A0, A0 + L, A0 + 2 * L, cs, mk, mv);
      __syncthreads();
  #pragma unroll
      for (int i = 0; i < CI; ++i) {
        if ((uint32_t)i < count) {
          sk[cs + i] = mk[i];
          if constexpr (KV) sv[cs + i] = mv[i];
        }
      }
      __syncthreads();
    }
  } else {
    // Keys only.  Runs of 128 are formed in registers (bitonic merges across
    // lanes), written to the padded layout of each thread's own 16 slots.
    lane_runs_to_128(rk, tid & 63);
    wave_sync();
#pragma unroll
    for (int i = 0; i < kTileItems; ++i) sk[tile_pad(tid * kTileItems + i)] = rk[i];
    wave_sync();
    // Then rounds of merge-path merges.  Round 128 reads the padded layout and
    // writes the gapped one, where every run is followed by kGap slots of the
    // largest key, so the later rounds use merge_chunk_keys (no bound
    // checks).  While a pair fits in one wave's 1024 keys, runs of length L
    // sit at q (L + G) in the wave's own region of RW slots and the wave
    // synchronises only with itself; larger rounds use runs at j (L + G)
    // across the tile.
    constexpr int CI = kRoundItems;
    constexpr uint32_t G = kGap, WKEYS = 64 * kTileItems;
    const uint32_t lane = tid & 63, wv = tid >> 6;
    U mk[CI];
    uint32_t dummy_v[1];
    uint32_t L = 128;
    for (; L < TILE && 2 * L <= WKEYS; L *= 2) {
      const uint32_t cpp = (2 * L + CI - 1) / CI;  // chunks per pair
      const uint32_t q = lane / cpp, c = lane - q * cpp;
      const bool active = q < WKEYS / (2 * L);
      const uint32_t o = c * CI;  // this chunk's first output within the pair
      const uint32_t count = active ? (2 * L - o < (uint32_t)CI ? 2 * L - o : CI) : 0u;
      const bool to_tile = 4 * L > WKEYS;  // the next round's pairs span waves
      const uint32_t dst = to_tile ? (wv * (WKEYS / (2 * L)) + q) * (2 * L + G)
                                   : wv * RW + q * (2 * L + G);
      if (active) {
        if (L == 128) {
          // padded layout of the wave's keys at the start of its region
          const uint32_t A0 = q * 2 * L;
          merge_chunk<U, false, CI, true>(sk + wv * RW, sv, A0, A0 + L, A0 + 2 * L, A0 + o, mk,
                                          dummy_v);
        } else {
          const uint32_t A0 = wv * RW + 2 * q * (L + G);
          merge_chunk_keys<U, CI>(sk, A0, L, A0 + L + G, L, o, mk);
        }
      }
      // a round writing tile-wide runs leaves the wave's region
      if (to_tile) __syncthreads();
      else wave_sync();
      // every active chunk stores all CI keys: a pair's last chunk spills
      // into the run's new gap, which it then fills with the largest key
      if (active) {
#pragma unroll
        for (int i = 0; i < CI; ++i) sk[dst + o + i] = mk[i];
        if (o + count == 2 * L)
          for (uint32_t j = 0; j < G; ++j) sk[dst + 2 * L + j] = key_max<U>();
      }
      if (to_tile) __syncthreads();
      else wave_sync();
    }
    for (; L < TILE; L *= 2) {
      const uint32_t cpp = (2 * L + CI - 1) / CI;  // chunks per pair
      const uint32_t q = tid / cpp, c = tid - q * cpp;
      const bool active = q < TILE / (2 * L);
      const uint32_t o = c * CI;
      const uint32_t count = active ? (2 * L - o < (uint32_t)CI ? 2 * L - o : CI) : 0u;
      const uint32_t A0 = 2 * q * (L + G), dst = q * (2 * L + G);
      if (active) merge_chunk_keys<U, CI>(sk, A0, L, A0 + L + G, L, o, mk);
      __syncthreads();
      if (active) {
#pragma unroll
        for (int i = 0; i < CI; ++i) sk[dst + o + i] = mk[i];
        if (o + count == 2 * L && 2 * L < TILE)
          for (uint32_t j = 0; j < G; ++j) sk[dst + 2 * L + j] = key_max<U>();
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < kTileItems; ++i) {
    const uint32_t idx = i * THREADS + tid;
    if (idx < len) {
      const U k = sk[idx];
      // written once and read a pass later: non-temporal, so that the
      // samples the next pass reads soon stay in L2
      __builtin_nontemporal_store(final_pass ? Key<KT>::unmap(k) : k, &out[start + idx]);
      if constexpr (KV) __builtin_nontemporal_store(sv[idx], &vout[start + idx]);
    }
  }
  // regular samples of the sorted tile (every kSample-th key, tile positions
  // kSample*i + kSample-1) for the next level's splitter search
  if (samples != nullptr) {
    for (uint32_t i = tid; i < (len >> kSampleLog2); i += THREADS)
      samples[sbase + i] = sk[(i << kSampleLog2) + kSample - 1];
  }
}

// ----------------------------------------------------- run geometry ------
struct GroupInfo {
  uint64_t start;  // first key of the group
  uint64_t len;    // keys in the group (0 = no such group)
  uint64_t gi;     // group index (table block index; uniform mode)
  uint32_t seg;    // segment (segmented mode)
  uint64_t gg;     // group within the segment (segmented mode)
};

__device__ __forceinline__ GroupInfo seg_group(const RunGeom &g, uint32_t s, uint64_t gg) {
  const uint64_t *base = g.seg.level ? g.seg.soff : g.seg.off;
  const uint64_t sstart = base[s], slen = base[s + 1] - base[s];
  const uint64_t goff = gg * g.group_len;
  GroupInfo r;
  r.start = sstart + goff;
  r.len = goff < slen ? (slen - goff < g.group_len ? slen - goff : g.group_len) : 0;
  r.gi = 0;
  r.seg = s;
  r.gg = gg;
  return r;
}

// Segmented mode: does buffer X_j of segment s (the output of its pass j;
// X_0 = tile sort) live in the primary (final output) buffer?  Passes
// alternate so that X_{npass} is the output.
__device__ __forceinline__ bool seg_primary(const RunGeom &g, uint32_t s, uint32_t j) {
  return ((g.seg.npass[s] - j) & 1u) == 0;
}

__device__ __forceinline__ GroupInfo group_of(const RunGeom &g, uint64_t gi) {
  GroupInfo r;
  r.gi = gi;
  r.seg = 0;
  r.gg = 0;
  const uint64_t seg = gi / g.groups_per_seg, gg = gi % g.groups_per_seg;
  const uint64_t seg_start = seg * g.seg_len;
  const uint64_t seg_len = seg_start < g.n ? (g.n - seg_start < g.seg_len ? g.n - seg_start : g.seg_len) : 0;
  const uint64_t goff = gg * g.group_len;
  r.start = seg_start + goff;
  r.len = goff < seg_len ? (seg_len - goff < g.group_len ? seg_len - goff : g.group_len) : 0;
  return r;
}

// r_k = floor(k N / n_P) (the paper's k N / n_P in exact integer arithmetic)
__device__ __forceinline__ uint64_t paper_rank(const RunGeom &g, uint64_t k) {
  return (uint64_t)(((unsigned __int128)k * g.n) / g.n_parts);
}

// Group and target rank of table row `row`: uniform partitions of part_len
// keys, or (paper mode) chunks of at most part_len keys inside each of the
// paper's partitions.
struct RowInfo {
  GroupInfo grp;
  uint64_t rank;
  uint32_t *out;
  bool valid;
};

// Paper partition holding chunk c (c < chunk_prefix[n_parts]): the largest p
// with chunk_prefix[p] <= c (an empty partition shares its prefix with the
// next one).
__device__ __forceinline__ uint32_t chunk_partition(const RunGeom &g, uint64_t c) {
  uint32_t lo = 0, hi = g.n_parts;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (g.chunk_prefix[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ RowInfo row_info(const RunGeom &g, uint64_t row, uint32_t *table) {
  RowInfo ri;
  ri.valid = true;
  if (g.seg.off) {
    ri.out = table + row * g.fan;
    if (row >= g.seg.rows[g.seg.n_segs]) {
      ri.valid = false;
      return ri;
    }
    const uint32_t sg = seg_find(g.seg.rows, g.seg.n_segs, row);
    const uint64_t local = row - g.seg.rows[sg];
    ri.grp = seg_group(g, sg, local / g.rows_per_group);
    const uint64_t r = (local % g.rows_per_group) * g.part_len;
    ri.rank = r < ri.grp.len ? r : ri.grp.len;
    return ri;
  }
  if (!g.paper) {
    const uint64_t gi = row / g.rows_per_group, k = row % g.rows_per_group;
    ri.grp = group_of(g, gi);
    const uint64_t r = k * g.part_len;
    ri.rank = r < ri.grp.len ? r : ri.grp.len;
  } else if (g.bounds) {
    ri.grp.gi = 0;
    ri.grp.start = 0;
    ri.grp.len = g.n;
    // rows are the chunk boundaries: chunk c starts at rank bounds[p] +
    // (c - chunk_prefix[p]) part_len; the last row is rank n
    const uint64_t C = g.chunk_prefix[g.n_parts];
    if (row > C) {
      ri.valid = false;
    } else if (row == C) {
      ri.rank = g.n;
    } else {
      const uint32_t p = chunk_partition(g, row);
      ri.rank = g.bounds[p] + (row - g.chunk_prefix[p]) * g.part_len;
    }
  } else {
    ri.grp.gi = 0;
    ri.grp.start = 0;
    ri.grp.len = g.n;
    const uint64_t last = (uint64_t)g.n_parts * g.sub_per_part;
    if (row >= last) {
      ri.rank = g.n;
    } else {
      const uint64_t p = row / g.sub_per_part, i = row % g.sub_per_part;
      const uint64_t rp = paper_rank(g, p), rp1 = paper_rank(g, p + 1);
      const uint64_t r = rp + i * g.part_len;
      ri.rank = r < rp1 ? r : rp1;
    }
  }
  ri.out = table + row * g.fan;
  return ri;
}

__device__ __forceinline__ uint32_t run_length(uint64_t group_len, uint64_t run_len, uint32_t b) {
  const uint64_t off = (uint64_t)b * run_len;
  if (off >= group_len) return 0;
  const uint64_t rem = group_len - off;
  return (uint32_t)(rem < run_len ? rem : run_len);
}

// ------------------------------------------------------- wave helpers ----
// Exclusive scan of a[0..n) in place, total into a[n]; one 64-lane workgroup.
__device__ void wave_exclusive_scan(uint32_t *a, uint32_t n) {
  const uint32_t lane = threadIdx.x;
  const uint32_t per = (n + 63) / 64;
  const uint32_t beg = lane * per < n ? lane * per : n;
  const uint32_t end = beg + per < n ? beg + per : n;
  uint32_t s = 0;
  for (uint32_t i = beg; i < end; ++i) s += a[i];
  uint32_t x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if ((int)lane >= d) x += y;
  }
  const uint32_t total = __shfl(x, 63, 64);
  uint32_t e = x - s;
  for (uint32_t i = beg; i < end; ++i) {
    const uint32_t v = a[i];
    a[i] = e;
    e += v;
  }
  if (lane == 0) a[n] = total;
}

// Exclusive scan of a[0..n) in place, total into a[n]; whole workgroup.
// `wsum` needs blockDim.x/64 + 1 entries.
__device__ void block_exclusive_scan(uint32_t *a, uint32_t n, uint32_t *wsum) {
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const uint32_t lane = tid & 63, wid = tid >> 6, nw = nthr >> 6;
  const uint32_t per = (n + nthr - 1) / nthr;
  const uint32_t beg = tid * per < n ? tid * per : n;
  const uint32_t end = beg + per < n ? beg + per : n;
  uint32_t s = 0;
  for (uint32_t i = beg; i < end; ++i) s += a[i];
  uint32_t x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if ((int)lane >= d) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      const uint32_t v = wsum[w];
      wsum[w] = run;
      run += v;
    }
    wsum[nw] = run;
  }
  __syncthreads();
  uint32_t e = x - s + wsum[wid];
  for (uint32_t i = beg; i < end; ++i) {
    const uint32_t v = a[i];
    a[i] = e;
    e += v;
  }
  if (tid == 0) a[n] = wsum[nw];
  __syncthreads();
}

// Compare-exchange of two (key, tie) slots, ascending when `up`.
template <typename U, int E>
__device__ __forceinline__ void cas(U &ka, uint32_t &ta, U &kb, uint32_t &tb, bool up) {
  const bool gt = ka > kb || (ka == kb && ta > tb);
  if (gt == up) {
    const U k = ka;
    ka = kb;
    kb = k;
    const uint32_t t = ta;
    ta = tb;
    tb = t;
  }
}

// One compare-exchange stage of the wave's bitonic sort at lane distance D
// (slot s = lane + 64 e; sort block k; ascending by (key, tie)).
template <int D, typename U, int E>
__device__ __forceinline__ void bitonic_lane_stage(U (&key)[E], uint32_t (&tie)[E], uint32_t lane,
                                                   uint32_t k, uint32_t Cp) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (64u * e < Cp) {
      const U ok = shfl_xor_c<D>(key[e]);
      const uint32_t ot = shfl_xor_c<D>(tie[e]);
      const uint32_t idx = lane + 64u * e;
      const bool lower = (lane & D) == 0;
      const bool up = (idx & k) == 0;
      const bool mine_gt = key[e] > ok || (key[e] == ok && tie[e] > ot);
      // the lower slot keeps the smaller when ascending
      const bool take_other = (lower == up) ? mine_gt : !mine_gt;
      key[e] = take_other ? ok : key[e];
      tie[e] = take_other ? ot : tie[e];
    }
  }
}

// Byte d (0 = least significant) of the composite (key, tie): the tie's four
// bytes below the key's.
template <typename U>
__device__ __forceinline__ uint32_t composite_digit(U key, uint32_t tie, int d) {
  return d < 4 ? (tie >> (8 * d)) & 0xFFu : (uint32_t)(key >> (8 * (d - 4))) & 0xFFu;
}

// The (key, tie) of rank k (0-based; k below the number of valid slots) among
// the valid slots s = lane + 64 e (bit e of `valid`) of one 64-lane
// workgroup, by radix selection: digits of 8 bits from the most significant
// (key first, then tie), a 256-bin histogram in LDS for each, the candidates
// narrowed to the bucket holding rank k, stopping once that bucket holds a
// single slot.  Composites are distinct (the tie holds run and position), so
// exactly one slot is left.  All lanes must call it.
template <typename U, int E>
__device__ __forceinline__ void select_rank(const U (&key)[E], const uint32_t (&tie)[E],
                                            uint32_t valid, uint32_t k, uint32_t lane,
                                            uint32_t *hist, U &out_key, uint32_t &out_tie) {
  constexpr int NDIG = (int)sizeof(U) + 4;
  uint32_t act = valid;
  for (int d = NDIG - 1; d >= 0; --d) {
    // a digit on which every active slot agrees narrows nothing: skip it
    uint32_t dmin = 0xFFu, dmax = 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if ((act >> e) & 1u) {
        const uint32_t dg = composite_digit<U>(key[e], tie[e], d);
        dmin = dg < dmin ? dg : dmin;
        dmax = dg > dmax ? dg : dmax;
      }
    }
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) {
      const uint32_t a = __shfl_xor(dmin, dd, 64), b = __shfl_xor(dmax, dd, 64);
      dmin = a < dmin ? a : dmin;
      dmax = b > dmax ? b : dmax;
    }
    if (dmin == dmax) continue;
    hist[lane] = 0;
    hist[lane + 64] = 0;
    hist[lane + 128] = 0;
    hist[lane + 192] = 0;
    __syncthreads();
    // equal digits in a row of a lane's slots go in with one atomic
    uint32_t run_d = 0u, run_c = 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if ((act >> e) & 1u) {
        const uint32_t dg = composite_digit<U>(key[e], tie[e], d);
        if (run_c && dg == run_d) {
          ++run_c;
        } else {
          if (run_c) atomicAdd(&hist[run_d], run_c);
          run_d = dg;
          run_c = 1u;
        }
      }
    }
    if (run_c) atomicAdd(&hist[run_d], run_c);
    __syncthreads();
    // lane l holds bins 4l..4l+3; the lane whose bins cover rank k picks one
    const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1];
    const uint32_t h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
    const uint32_t sum = h0 + h1 + h2 + h3;
    uint32_t incl = sum;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
      const uint32_t y = __shfl_up(incl, dd, 64);
      if ((int)lane >= dd) incl += y;
    }
    const uint32_t excl = incl - sum;
    const bool mine = k >= excl && k < incl;
    const int owner = __ffsll((unsigned long long)__ballot(mine)) - 1;
    uint32_t v = 0, before = 0, cnt = 0;
    if (mine) {
      if (k < excl + h0) {
        v = 4 * lane, before = excl, cnt = h0;
      } else if (k < excl + h0 + h1) {
        v = 4 * lane + 1, before = excl + h0, cnt = h1;
      } else if (k < excl + h0 + h1 + h2) {
        v = 4 * lane + 2, before = excl + h0 + h1, cnt = h2;
      } else {
        v = 4 * lane + 3, before = excl + h0 + h1 + h2, cnt = h3;
      }
    }
    v = __shfl(v, owner, 64);
    before = __shfl(before, owner, 64);
    cnt = __shfl(cnt, owner, 64);
    k -= before;
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (composite_digit<U>(key[e], tie[e], d) != v) act &= ~(1u << e);
    __syncthreads();  // the histogram is read before it is cleared again
    if (cnt == 1) break;
  }
  U kk = 0;
  uint32_t tt = 0;
#pragma unroll
  for (int e = 0; e < E; ++e)
    if ((act >> e) & 1u) {
      kk = key[e];
      tt = tie[e];
    }
  const int owner = __ffsll((unsigned long long)__ballot(act != 0u)) - 1;
  out_key = __shfl(kk, owner, 64);
  out_tie = __shfl(tt, owner, 64);
}

// Merged samples of one pass: the group's level-kSampleLog2 samples in
// (key, run, position) order as run ids, plus per-run prefix counts at every
// kChunk-th merged sample.  They give V_5(Q) for any Q without a search.
struct SampleIndex {
  const uint32_t *runs;  // run id of every merged sample
  const uint32_t *prefix; // [chunk][fan]: samples of each run before the chunk
  RunGeom gs;             // geometry of the sample array (groups align with data)
};

// --------------------------------------------------------------- K2/K3 ---
// Exact co-rank of one target rank r over the F sorted runs of one group:
// t_b = number of keys of run b among the r smallest keys of the group, where
// equal keys are ordered by run index, then position (lowest run first).
// This realises the paper's exact splitting: sum_b t_b = r exactly, all keys
// below the pivot go left, and of the keys equal to it exactly c_k go left,
// taken from the lowest-numbered run first.
//
// Search (our GPU design, not the paper's): positions are fixed one bit at a
// time from the most significant.  At level j the samples are the keys at
// positions i*2^j - 1.  The prefix of the Q smallest level-j samples, V_j(Q),
// is known to lie between V_j(Q_lo) and V_j(Q_hi) with
//   Q_lo(j) = max(0, floor((r - (2^j - 1)(F - 1)) / 2^j)),
//   Q_hi(j) = min(floor(r / 2^j), number of level-j samples),
// and V_j(Q)_b is within [2 V_{j+1}(Q_lo(j+1))_b, 2 V_{j+1}(Q_hi(j+1))_b + 1].
// So each level loads fewer than 3F candidate samples, sorts them in LDS and
// reads both prefixes off; at level 0, Q_lo = Q_hi = r and V_0(r) = t.
//
// E > 0: the candidates sit in registers, E slots per lane (slot s = lane +
// 64 e, at most 64 E of them; sTie holds each slot's run while they are
// loaded), and the two prefixes are found by selecting the candidates of rank
// rho_lo and rho_hi (radix selection) instead of sorting; E = 0: they are
// sorted in LDS (CMAX of them).
//
// SAMPLED: the search starts at level kSampleLog2 from the merged samples, as
// in corank_wave_kernel below, with per-run counts in LDS.
template <typename U, uint32_t MAXF, int E, bool SAMPLED = false>
__global__ __launch_bounds__(kCorankThreads) void corank_kernel(
    const U *__restrict__ src, RunGeom g, uint32_t *__restrict__ table,
    U *__restrict__ pivots, uint64_t *__restrict__ counts, int kt, SampleIndex si) {
  constexpr uint32_t CMAX = E > 0 ? 64 * E : (MAXF <= 64 ? 256 : (MAXF <= 512 ? 2048 : 8192));
  __shared__ U sKey[E > 0 ? 1 : CMAX];
  __shared__ uint32_t sTie[CMAX];
  __shared__ uint32_t sHist[E > 0 ? 256 : 1];
  __shared__ uint32_t sA[MAXF], sB[MAXF], sCnt[2 * MAXF], sOff[MAXF + 1];

  const uint32_t lane = threadIdx.x;
  const uint64_t row = blockIdx.x;
  const RowInfo ri = row_info(g, row, table);
  if (!ri.valid) return;  // whole workgroup: rows beyond a data-dependent row count
  const uint64_t glen = ri.grp.len, R = g.run_len, r = ri.rank;
  const uint32_t nruns = glen ? (uint32_t)((glen + R - 1) / R) : 0;
  const uint32_t F = g.fan;

  // trivial rows: nothing or everything taken
  const bool trivial = r == 0 || r >= glen;
  if (trivial) {
    for (uint32_t b = lane; b < nruns; b += 64) sA[b] = r == 0 ? 0u : run_length(glen, R, b);
    __syncthreads();
  }
  const uint32_t maxlen = trivial ? 1u : (uint32_t)(R < glen ? R : glen);
  const uint32_t lastlen = trivial ? 0u : run_length(glen, R, nruns - 1);
  const int J = trivial ? 0 : 32 - __clz(maxlen);
  if (!trivial) {
    for (uint32_t b = lane; b < nruns; b += 64) {
      sA[b] = 0;
      sB[b] = 0;
    }
    __syncthreads();
  }

  auto q_lo_at = [&](int j) -> uint64_t {
    const int64_t num = (int64_t)r - (int64_t)((((uint64_t)1 << j) - 1) * (uint64_t)(nruns - 1));
    return num > 0 ? ((uint64_t)num >> j) : 0;
  };

  int jtop = J;
  if constexpr (SAMPLED) {
    if (!trivial && J > kSampleLog2) {
      // V_kSampleLog2 at both bracket targets from the merged samples: the
      // prefix counts at the chunk plus the run ids of the remaining samples
      jtop = kSampleLog2;
      const GroupInfo sg = group_of(si.gs, ri.grp.gi);
      const uint64_t ns5 = sg.len, rs = si.gs.run_len;
      const uint32_t nruns_s = ns5 ? (uint32_t)((ns5 + rs - 1) / rs) : 0u;
      const uint64_t qs[2] = {q_lo_at(kSampleLog2),
                              (r >> kSampleLog2) < ns5 ? (r >> kSampleLog2) : ns5};
      const uint64_t prow0 = ri.grp.gi * (si.gs.rows_per_group - 1) * (kPart / kChunk);
      for (int t = 0; t < 2; ++t) {
        const uint64_t Q = qs[t];
        for (uint32_t b = lane; b < nruns; b += 64) sCnt[b] = 0;
        __syncthreads();
        const uint64_t C = Q / kChunk;
        if (Q < ns5) {
          const uint32_t rem = (uint32_t)(Q - C * kChunk);
          for (uint32_t i = lane; i < rem; i += 64)
            atomicAdd(&sCnt[si.runs[sg.start + C * kChunk + i]], 1u);
        }
        __syncthreads();
        for (uint32_t b = lane; b < nruns; b += 64) {
          uint32_t v;
          if (Q >= ns5) {
            v = run_length(glen, R, b) >> kSampleLog2;
          } else {
            v = (b < nruns_s ? si.prefix[(prow0 + C) * g.fan + b] : 0u) + sCnt[b];
          }
          if (t == 0) sA[b] = v;
          else sB[b] = v;
        }
        __syncthreads();
      }
    }
  }

  for (int j = jtop - 1; j >= 0; --j) {
    const uint64_t h = (uint64_t)1 << j;
    const uint64_t ns_total = (uint64_t)(nruns - 1) * (R >> j) + (lastlen >> j);
    const uint64_t q_lo = q_lo_at(j);
    const uint64_t q_hi = (r >> j) < ns_total ? (r >> j) : ns_total;
    const uint64_t base = 2 * q_lo_at(j + 1);

    for (uint32_t b = lane; b < nruns; b += 64) {
      const uint32_t ns = run_length(glen, R, b) >> j;
      const uint32_t lo_i = 2 * sA[b] + 1;
      const uint32_t hi_i = 2 * sB[b] + 1 < ns ? 2 * sB[b] + 1 : ns;
      sOff[b] = hi_i >= lo_i ? hi_i - lo_i + 1 : 0;
    }
    __syncthreads();
    wave_exclusive_scan(sOff, nruns);
    __syncthreads();
    uint32_t C = sOff[nruns];
    if (C > CMAX) {  // cannot happen while the bracket holds (C < 3 * runs)
      if (lane == 0) report(kErrCandidates);
      C = CMAX;
    }
    if constexpr (E > 0) {
      for (uint32_t b = lane; b < nruns; b += 64) {
        const uint32_t o = sOff[b], c = sOff[b + 1] - o;
        for (uint32_t x = 0; x < c; ++x)
          if (o + x < CMAX) sTie[o + x] = b;
      }
      for (uint32_t b = lane; b < 2 * nruns; b += 64) sCnt[b] = 0;
      __syncthreads();
      U key[E];
      uint32_t tie[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const uint32_t s = lane + 64u * e;
        key[e] = key_max<U>();
        tie[e] = 0xffffffffu;
        if (s < C) {
          const uint32_t b = sTie[s];
          const uint32_t x = s - sOff[b];
          key[e] = src[ri.grp.start + (uint64_t)b * R + (uint64_t)(2 * sA[b] + 1 + x) * h - 1];
          tie[e] = (b << 20) | x;
        }
      }
      uint64_t rho_lo = q_lo - base, rho_hi = q_hi - base;
      if (q_lo < base || q_hi < base || rho_hi > C || rho_lo > rho_hi) {  // bracket broken
        if (lane == 0) report(kErrBracket);
        rho_lo = rho_lo > C ? C : rho_lo;
        rho_hi = rho_hi > C ? C : rho_hi;
        rho_lo = rho_lo > rho_hi ? rho_hi : rho_lo;
      }
      uint32_t valid = 0;
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (lane + 64u * e < C) valid |= 1u << e;
      // a candidate is among the first rho iff it is below the one of rank rho
      U tk_lo = 0, tk_hi = 0;
      uint32_t tt_lo = 0, tt_hi = 0;
      if (rho_hi > 0 && rho_hi < C)
        select_rank<U, E>(key, tie, valid, (uint32_t)rho_hi, lane, sHist, tk_hi, tt_hi);
      if (rho_lo == rho_hi) {
        tk_lo = tk_hi;
        tt_lo = tt_hi;
      } else if (rho_lo > 0 && rho_lo < C) {
        select_rank<U, E>(key, tie, valid, (uint32_t)rho_lo, lane, sHist, tk_lo, tt_lo);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if ((valid >> e) & 1u) {
          const uint32_t b = tie[e] >> 20;
          const bool hi_in = rho_hi >= C ||
                             (rho_hi > 0 && (key[e] < tk_hi || (key[e] == tk_hi && tie[e] < tt_hi)));
          const bool lo_in = rho_lo >= C ||
                             (rho_lo > 0 && (key[e] < tk_lo || (key[e] == tk_lo && tie[e] < tt_lo)));
          if (hi_in) atomicAdd(&sCnt[2 * b + 1], 1u);
          if (lo_in) atomicAdd(&sCnt[2 * b], 1u);
        }
      }
      __syncthreads();
    } else {
      uint32_t Cp = 1;
      while (Cp < C) Cp <<= 1;

      // slot -> run in sTie first, then every lane loads slots lane, lane + 64,
      // ... with a batch of loads in flight (each slot is read and rewritten by
      // the one lane that owns it)
      for (uint32_t b = lane; b < nruns; b += 64) {
        const uint32_t o = sOff[b], c = sOff[b + 1] - o;
        for (uint32_t x = 0; x < c; ++x)
          if (o + x < CMAX) sTie[o + x] = b;
      }
      __syncthreads();
      constexpr uint32_t kBatch = 8;
      for (uint32_t s0 = 0; s0 < C; s0 += 64 * kBatch) {
        U v[kBatch];
        uint32_t t[kBatch];
  #pragma unroll
        for (uint32_t u = 0; u < kBatch; ++u) {
          const uint32_t s = s0 + u * 64 + lane;
          if (s < C) {
            const uint32_t b = sTie[s];
            const uint32_t x = s - sOff[b];
            v[u] = src[ri.grp.start + (uint64_t)b * R + (uint64_t)(2 * sA[b] + 1 + x) * h - 1];
            t[u] = (b << 20) | x;
          }
        }
  #pragma unroll
        for (uint32_t u = 0; u < kBatch; ++u) {
          const uint32_t s = s0 + u * 64 + lane;
          if (s < C) {
            sKey[s] = v[u];
            sTie[s] = t[u];
          }
        }
      }
      for (uint32_t s = C + lane; s < Cp && s < CMAX; s += 64) {
        sKey[s] = key_max<U>();
        sTie[s] = 0xffffffffu;
      }
      for (uint32_t b = lane; b < 2 * nruns; b += 64) sCnt[b] = 0;
      __syncthreads();

      // bitonic sort of (key, tie) pairs, ascending
      for (uint32_t k = 2; k <= Cp; k <<= 1) {
        for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
          for (uint32_t t = lane; t < Cp / 2; t += 64) {
            const uint32_t i = ((t & ~(jj - 1)) << 1) | (t & (jj - 1));
            const uint32_t l = i + jj;
            const U ki = sKey[i], kl = sKey[l];
            const uint32_t ti = sTie[i], tl = sTie[l];
            const bool gt = ki > kl || (ki == kl && ti > tl);
            const bool up = (i & k) == 0;
            if (gt == up) {
              sKey[i] = kl;
              sKey[l] = ki;
              sTie[i] = tl;
              sTie[l] = ti;
            }
          }
          __syncthreads();
        }
      }

      uint64_t rho_lo = q_lo - base, rho_hi = q_hi - base;
      if (q_lo < base || q_hi < base || rho_hi > C || rho_lo > rho_hi) {  // bracket broken
        if (lane == 0) report(kErrBracket);
        rho_lo = rho_lo > C ? C : rho_lo;
        rho_hi = rho_hi > C ? C : rho_hi;
        rho_lo = rho_lo > rho_hi ? rho_hi : rho_lo;
      }
      for (uint64_t s = lane; s < rho_hi; s += 64) {
        const uint32_t b = sTie[s] >> 20;
        atomicAdd(&sCnt[2 * b + 1], 1u);
        if (s < rho_lo) atomicAdd(&sCnt[2 * b], 1u);
      }
      __syncthreads();
    }
    for (uint32_t b = lane; b < nruns; b += 64) {
      const uint32_t a = sA[b];
      sA[b] = 2 * a + sCnt[2 * b];
      sB[b] = 2 * a + sCnt[2 * b + 1];
    }
    __syncthreads();
  }

  for (uint32_t b = lane; b < F; b += 64) ri.out[b] = b < nruns ? sA[b] : 0u;

  // Pivot P_k (the largest key taken, i.e. the key of rank r - 1) and c_k of
  // Eq. 2 (r minus the number of keys below P_k), for the paper's splitters.
  if (pivots != nullptr && g.paper) {
    const uint64_t p = row / g.sub_per_part;
    if (row % g.sub_per_part != 0 || p == 0 || p >= g.n_parts) return;
    if (r == 0) {  // empty prefix: c_k = 0, pivot unspecified (written as 0)
      if (lane == 0) {
        pivots[p - 1] = 0;
        counts[p - 1] = 0;
      }
      return;
    }
    U best = 0;
    for (uint32_t b = lane; b < nruns; b += 64) {
      const uint32_t t = sA[b];
      if (t > 0) {
        const U k = src[ri.grp.start + (uint64_t)b * R + t - 1];
        best = k > best ? k : best;
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const U o = __shfl_xor(best, d, 64);
      best = o > best ? o : best;
    }
    uint64_t lt = 0;
    for (uint32_t b = lane; b < nruns; b += 64) {
      const U *run = src + ri.grp.start + (uint64_t)b * R;
      uint32_t lo = 0, hi = run_length(glen, R, b);
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (run[mid] < best) lo = mid + 1;
        else hi = mid;
      }
      lt += lo;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) lt += __shfl_xor(lt, d, 64);
    if (lane == 0) {
      pivots[p - 1] = unmap_runtime<U>(best, kt);
      counts[p - 1] = r - lt;
    }
  }
}

// Same search for groups of at most 64 runs, one lane per run: the prefix
// bounds live in registers, each level's candidates are loaded one per slot
// by all lanes at once and sorted in registers by a bitonic network across the
// wave (slot s = lane + 64 e), and the two prefix counts are read off with LDS
// atomics.  E = largest number of slots per lane (3 * 64 candidates < 64 * 4).
template <typename U, int E, bool SAMPLED>
__global__ __launch_bounds__(kCorankThreads) void corank_wave_kernel(
    const U *__restrict__ src_primary, const U *__restrict__ src_alt, RunGeom g,
    uint32_t *__restrict__ table, U *__restrict__ pivots, uint64_t *__restrict__ counts, int kt,
    SampleIndex si) {
  __shared__ uint32_t slot_run[64 * E];
  __shared__ uint32_t cnt[2 * 64];

  const uint32_t lane = threadIdx.x;
  const uint64_t row = blockIdx.x;
  const RowInfo ri = row_info(g, row, table);
  if (!ri.valid) return;
  // segmented keys level: the input of pass q is the segment's X_{q-1}
  const U *src = (g.seg.off && g.seg.level == 0 && !seg_primary(g, ri.grp.seg, g.seg.pass - 1))
                     ? src_alt : src_primary;
  const uint64_t glen = ri.grp.len, R = g.run_len, r = ri.rank;
  const uint32_t nruns = glen ? (uint32_t)((glen + R - 1) / R) : 0;
  const uint32_t len = lane < nruns ? run_length(glen, R, lane) : 0u;
  const U *run = src + ri.grp.start + (uint64_t)lane * R;

  uint32_t A = 0, B = 0;
  if (r == 0 || r >= glen) {
    A = r == 0 ? 0u : len;
  } else {
    const uint32_t maxlen = (uint32_t)(R < glen ? R : glen);
    const uint32_t lastlen = run_length(glen, R, nruns - 1);
    const int J = 32 - __clz(maxlen);
    auto q_lo_at = [&](int j) -> uint64_t {
      const int64_t num = (int64_t)r - (int64_t)((((uint64_t)1 << j) - 1) * (uint64_t)(nruns - 1));
      return num > 0 ? ((uint64_t)num >> j) : 0;
    };
    int jtop = J;
    if constexpr (SAMPLED) {
      if (J > kSampleLog2) {
        // Start at level kSampleLog2: V_5 at both bracket targets is read
        // from the merged samples (prefix counts at the chunk + the run ids
        // of the remaining < kChunk merged samples).
        jtop = kSampleLog2;
        const GroupInfo sg = g.seg.off ? seg_group(si.gs, ri.grp.seg, ri.grp.gg)
                                       : group_of(si.gs, ri.grp.gi);
        const uint64_t ns5 = sg.len;
        // runs with at least one sample (a short last run may have none)
        const uint64_t rs = si.gs.run_len;
        const uint32_t nruns_s = ns5 ? (uint32_t)((ns5 + rs - 1) / rs) : 0u;
        const uint64_t qs[2] = {q_lo_at(kSampleLog2),
                                (r >> kSampleLog2) < ns5 ? (r >> kSampleLog2) : ns5};
        const uint64_t sppg = si.gs.rows_per_group - 1;  // sample partitions per full group
        const uint64_t prow0 =
            (g.seg.off ? si.gs.seg.parts[ri.grp.seg] + ri.grp.gg * sppg : ri.grp.gi * sppg) *
            (kPart / kChunk);
        uint32_t v[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const uint64_t Q = qs[t];
          cnt[lane] = 0;
          __syncthreads();
          uint32_t base_cnt = 0;
          if (Q >= ns5) {
            base_cnt = len >> kSampleLog2;
          } else {
            const uint64_t C = Q / kChunk;
            const uint32_t rem = (uint32_t)(Q - C * kChunk);
            if (lane < nruns_s) base_cnt = si.prefix[(prow0 + C) * g.fan + lane];
            if (lane < rem) atomicAdd(&cnt[si.runs[sg.start + C * kChunk + lane]], 1u);
          }
          __syncthreads();
          v[t] = base_cnt + (Q >= ns5 ? 0u : cnt[lane]);
          __syncthreads();
        }
        A = lane < nruns ? v[0] : 0u;
        B = lane < nruns ? v[1] : 0u;
      }
    }
    for (int j = jtop - 1; j >= 0; --j) {
      const uint64_t h = (uint64_t)1 << j;
      const uint64_t ns_total = (uint64_t)(nruns - 1) * (R >> j) + (lastlen >> j);
      const uint64_t q_lo = q_lo_at(j);
      const uint64_t q_hi = (r >> j) < ns_total ? (r >> j) : ns_total;
      const uint64_t base = 2 * q_lo_at(j + 1);

      const uint32_t ns = len >> j;
      const uint32_t lo_i = 2 * A + 1;
      const uint32_t hi_i = 2 * B + 1 < ns ? 2 * B + 1 : ns;
      const uint32_t c = hi_i >= lo_i ? hi_i - lo_i + 1 : 0u;
      uint32_t incl = c;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        if ((int)lane >= d) incl += y;
      }
      const uint32_t off = incl - c;
      uint32_t C = __shfl(incl, 63, 64);
      if (C > 64u * E) {
        if (lane == 0) report(kErrCandidates);
        C = 64u * E;
      }
      for (uint32_t x = 0; x < c; ++x)
        if (off + x < 64u * E) slot_run[off + x] = lane;
      cnt[lane] = 0;
      cnt[lane + 64] = 0;
      __syncthreads();

      uint32_t Cp = 64;
      while (Cp < C) Cp <<= 1;
      U key[E];
      uint32_t tie[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const uint32_t s = lane + 64 * e;
        // all lanes take part in the shuffles (no lane may be masked off)
        const uint32_t rb = s < C ? slot_run[s] : 0u;
        const uint32_t rb_off = __shfl(off, (int)rb, 64);
        const uint32_t rb_a = __shfl(A, (int)rb, 64);
        key[e] = key_max<U>();
        tie[e] = 0xffffffffu;
        if (s < C) {
          const uint32_t x = s - rb_off;
          key[e] = src[ri.grp.start + (uint64_t)rb * R + (uint64_t)(2 * rb_a + 1 + x) * h - 1];
          tie[e] = (rb << 20) | x;
        }
      }

      // bitonic sort of Cp slots, ascending by (key, tie): distances of 64
      // and more exchange slots inside a lane, smaller ones exchange lanes
      for (uint32_t k = 2; k <= Cp; k <<= 1) {
        for (uint32_t d = k >> 1; d >= 64; d >>= 1) {
          const uint32_t de = d >> 6;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if (E > 1 && ((uint32_t)e & de) == 0 && (e | (int)de) < E && 64u * (e | de) < Cp) {
              const bool up = ((lane + 64u * e) & k) == 0;
              if (de == 1) cas<U, E>(key[e], tie[e], key[e | 1], tie[e | 1], up);
              else if (de == 2) cas<U, E>(key[e], tie[e], key[(e | 2) & (E - 1)], tie[(e | 2) & (E - 1)], up);
            }
          }
        }
        if (k > 32) bitonic_lane_stage<32>(key, tie, lane, k, Cp);
        if (k > 16) bitonic_lane_stage<16>(key, tie, lane, k, Cp);
        if (k > 8) bitonic_lane_stage<8>(key, tie, lane, k, Cp);
        if (k > 4) bitonic_lane_stage<4>(key, tie, lane, k, Cp);
        if (k > 2) bitonic_lane_stage<2>(key, tie, lane, k, Cp);
        bitonic_lane_stage<1>(key, tie, lane, k, Cp);
      }

      uint64_t rho_lo = q_lo - base, rho_hi = q_hi - base;
      if (q_lo < base || q_hi < base || rho_hi > C || rho_lo > rho_hi) {
        if (lane == 0) report(kErrBracket);
        rho_lo = rho_lo > C ? C : rho_lo;
        rho_hi = rho_hi > C ? C : rho_hi;
        rho_lo = rho_lo > rho_hi ? rho_hi : rho_lo;
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const uint32_t s = lane + 64 * e;
        if (s < rho_hi) {
          const uint32_t rb = tie[e] >> 20;
          atomicAdd(&cnt[64 + rb], 1u);
          if (s < rho_lo) atomicAdd(&cnt[rb], 1u);
        }
      }
      __syncthreads();
      const uint32_t a = A;
      A = 2 * a + cnt[lane];
      B = 2 * a + cnt[64 + lane];
      __syncthreads();
    }
  }
  if (lane < g.fan) ri.out[lane] = lane < nruns ? A : 0u;

  if (pivots != nullptr && g.paper) {
    const uint64_t p = row / g.sub_per_part;
    if (row % g.sub_per_part != 0 || p == 0 || p >= g.n_parts) return;
    if (r == 0) {
      if (lane == 0) {
        pivots[p - 1] = 0;
        counts[p - 1] = 0;
      }
      return;
    }
    U best = 0;
    if (lane < nruns && A > 0) best = run[A - 1];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const U o = __shfl_xor(best, d, 64);
      best = o > best ? o : best;
    }
    uint64_t lt = 0;
    if (lane < nruns) {
      uint32_t lo = 0, hi = len;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (run[mid] < best) lo = mid + 1;
        else hi = mid;
      }
      lt = lo;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) lt += __shfl_xor(lt, d, 64);
    if (lane == 0) {
      pivots[p - 1] = unmap_runtime<U>(best, kt);
      counts[p - 1] = r - lt;
    }
  }
}

// --------------------------------------------------------------- K5 -------
struct PartInfo {
  bool valid;
  uint32_t size;  // keys in this partition
  uint64_t group_start, group_len, out_off;
  const uint32_t *lo_row, *hi_row;
  uint32_t seg;   // segmented mode: segment and group within it
  uint64_t gg;
};

__device__ __forceinline__ PartInfo part_info(const RunGeom &g, uint64_t pidx,
                                              const uint32_t *table, const uint64_t *part_off) {
  PartInfo pi;
  pi.valid = false;
  pi.seg = 0;
  pi.gg = 0;
  if (g.seg.off) {
    if (pidx >= g.seg.parts[g.seg.n_segs]) return pi;
    const uint32_t sg = seg_find(g.seg.parts, g.seg.n_segs, pidx);
    const uint64_t local = pidx - g.seg.parts[sg];
    const uint64_t ppg = g.rows_per_group - 1;
    const uint64_t gg = local / ppg, k = local % ppg;
    const GroupInfo grp = seg_group(g, sg, gg);
    const uint64_t rlo = k * g.part_len;
    if (rlo >= grp.len) return pi;
    const uint64_t rhi = rlo + g.part_len < grp.len ? rlo + g.part_len : grp.len;
    pi.size = (uint32_t)(rhi - rlo);
    pi.group_start = grp.start;
    pi.group_len = grp.len;
    pi.out_off = grp.start + rlo;
    pi.lo_row = table + (g.seg.rows[sg] + gg * g.rows_per_group + k) * g.fan;
    pi.hi_row = pi.lo_row + g.fan;
    pi.seg = sg;
    pi.gg = gg;
    pi.valid = true;
    return pi;
  }
  if (!g.paper) {
    const uint32_t ppg = g.rows_per_group - 1;
    const uint64_t gi = pidx / ppg, k = pidx % ppg;
    const GroupInfo grp = group_of(g, gi);
    const uint64_t rlo = k * g.part_len;
    if (rlo >= grp.len) return pi;
    const uint64_t rhi = rlo + g.part_len < grp.len ? rlo + g.part_len : grp.len;
    pi.size = (uint32_t)(rhi - rlo);
    pi.group_start = grp.start;
    pi.group_len = grp.len;
    pi.out_off = grp.start + rlo;
    pi.lo_row = table + (gi * g.rows_per_group + k) * g.fan;
    pi.hi_row = pi.lo_row + g.fan;
  } else if (g.bounds) {
    if (pidx >= g.chunk_prefix[g.n_parts]) return pi;
    const uint32_t p = chunk_partition(g, pidx);
    const uint64_t rp1 = g.bounds[p + 1];
    const uint64_t lo = g.bounds[p] + (pidx - g.chunk_prefix[p]) * g.part_len;
    const uint64_t hi = lo + g.part_len < rp1 ? lo + g.part_len : rp1;
    pi.size = (uint32_t)(hi - lo);
    pi.group_start = 0;
    pi.group_len = g.n;
    pi.out_off = lo;  // partitions follow each other: the output offset is the rank
    pi.lo_row = table + pidx * g.fan;
    pi.hi_row = pi.lo_row + g.fan;
  } else {
    const uint64_t p = pidx / g.sub_per_part, i = pidx % g.sub_per_part;
    const uint64_t rp = paper_rank(g, p), rp1 = paper_rank(g, p + 1);
    const uint64_t lo = rp + i * g.part_len;
    if (lo >= rp1) return pi;
    const uint64_t hi = lo + g.part_len < rp1 ? lo + g.part_len : rp1;
    pi.size = (uint32_t)(hi - lo);
    pi.group_start = 0;
    pi.group_len = g.n;
    pi.out_off = part_off[p] + (lo - rp);
    pi.lo_row = table + pidx * g.fan;
    pi.hi_row = pi.lo_row + g.fan;
  }
  pi.valid = true;
  return pi;
}

// Largest b in [0, F) with soff[b] <= pos (requires pos < soff[F]).
__device__ __forceinline__ uint32_t find_segment(const uint32_t *soff, uint32_t F, uint32_t pos) {
  uint32_t lo = 0, hi = F;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (soff[mid] <= pos) lo = mid;
    else hi = mid;
  }
  return lo;
}

// VMODE: 0 keys only, 1 keys + uint32 payload, 2 samples merge: the payload
// is the index of the run each key came from, and per-run prefix counts at
// every kChunk-th output are written to `prefix` (for the splitter search of
// the data pass).  samples != nullptr: write every kSample-th output key of
// each output run (run = this pass's group) for the next pass.
// Buffers of one merge launch.  Uniform and paper modes use the primary
// pointers only; the segmented mode picks, per segment, primary or alt by the
// parity of the segment's remaining passes.
template <typename U> struct MergeBufs {
  const U *src, *src_alt;
  const uint32_t *vsrc, *vsrc_alt;
  U *dst, *dst_alt;
  uint32_t *vdst, *vdst_alt;
};

template <int KT, int VMODE, uint32_t MAXF, uint32_t NT = kMergeThreads, uint32_t PART = kPart>
__global__ __launch_bounds__(NT, (VMODE != 2 && NT > kMergeThreads && (VMODE == 0 || PART < kPart)) ? 2 : 1)
void merge_kernel(
    MergeBufs<typename Key<KT>::U> bufs, RunGeom g, const uint32_t *__restrict__ table,
    const uint64_t *__restrict__ part_off, int final_pass,
    typename Key<KT>::U *__restrict__ samples, uint32_t *__restrict__ prefix) {
  using U = typename Key<KT>::U;
  constexpr bool KV = VMODE != 0;
  // NT threads, ITEMS keys each, partitions of at most PART keys; a merge
  // round gives each thread a chunk of CI outputs (odd, and small enough that
  // a round's chunks fit in NT).  On 8192-key partitions with 1024 threads,
  // chunks of ITEMS + 1 = 9 would keep more threads busy, but the 17-key
  // chunks measured faster (fewer chunk boundaries to search).  Key-value
  // merges of 4096-key partitions take chunks of 9: their registers then
  // allow two 1024-thread workgroups per CU.
  constexpr int ITEMS = PART / NT;
  constexpr int CI = (VMODE == 1 && PART < kPart) ? kRoundItemsKV : kRoundItems;
  constexpr int LP = PART / NT;  // positions each thread labels
  static_assert(NT * ITEMS == PART && CI % 2 == 1 && LP % 4 == 0, "merge geometry");
  static_assert(PART == kPart || (VMODE == 1 && MAXF <= 64), "short partitions: key-value only");
  // Keys-only merges of at most 32 runs leave kGap slots holding the largest
  // key after every segment in LDS (see merge_chunk_keys); others use the
  // flat layout.  Both add the slack a merge chunk may read past the end.
  constexpr bool GAPS = VMODE == 0 && MAXF <= 32;
  constexpr uint32_t G = GAPS ? kGap : 0;
  constexpr uint32_t P = PART + MAXF * G + 2 * kRoundItems + 2;
  __shared__ U sk[P];
  __shared__ uint32_t sv[KV ? P : 1];
  __shared__ uint32_t soff[MAXF + 1];
  // chunk prefixes over pairs, for each merge round (fan <= 64: 6 rounds)
  __shared__ uint32_t cpre[MAXF <= 64 ? 6 * 33 : 1];
  __shared__ uint64_t ssrc[MAXF];
  // segment of each position, one byte each (up to 256 segments)
  constexpr bool LABELS = MAXF <= 256;
  __shared__ uint32_t sseg[LABELS ? PART / 4 : 1];
  __shared__ uint32_t wsum[NT / 64 + 1];
  // per-run counts of a block of chunks (all chunks of a partition when
  // the fan is at most 64)
  constexpr uint32_t kHistWords = (kPart / kChunk) * 64;
  __shared__ uint32_t hist[VMODE == 2 ? kHistWords : 1];

  const uint32_t tid = threadIdx.x;
  const PartInfo pi = part_info(g, blockIdx.x, table, part_off);
  if (!pi.valid) return;
  const uint64_t R = g.run_len;
  const uint32_t F = (uint32_t)((pi.group_len + R - 1) / R);
  const U *src = bufs.src;
  const uint32_t *vsrc = bufs.vsrc;
  U *dst = bufs.dst;
  uint32_t *vdst = bufs.vdst;
  bool write_samples = samples != nullptr;
  if (g.seg.off && g.seg.level == 0) {
    const uint32_t q = g.seg.pass;
    if (!seg_primary(g, pi.seg, q - 1)) {
      src = bufs.src_alt;
      vsrc = bufs.vsrc_alt;
    }
    if (!seg_primary(g, pi.seg, q)) {
      dst = bufs.dst_alt;
      vdst = bufs.vdst_alt;
    }
    final_pass = g.seg.npass[pi.seg] == q;
    write_samples = write_samples && !final_pass;
  }

  if constexpr (MAXF <= 64) {
    // one wave: segment sizes and their exclusive scan
    if (tid < 64) {
      uint32_t c = 0;
      if (tid < F) {
        const uint32_t lo = pi.lo_row[tid], hi = pi.hi_row[tid];
        const uint32_t len = run_length(pi.group_len, R, tid);
        const bool ok = lo <= hi && hi <= len;
        if (!ok) report(kErrSplitRow);
        c = ok ? hi - lo : PART + 1;  // forces the size check below to fail
        ssrc[tid] = pi.group_start + (uint64_t)tid * R + lo;
      }
      uint32_t x = c;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if ((int)tid >= d) x += y;
      }
      const uint32_t e = x - c;  // soff[tid]; lanes at or past F hold the total
      const uint32_t total = __shfl(x, 63, 64);
      if (tid < F) soff[tid] = e;
      if (tid == 0) soff[F] = total;
    }
    __syncthreads();
  } else {
    for (uint32_t b = tid; b < F; b += NT) {
      const uint32_t lo = pi.lo_row[b], hi = pi.hi_row[b];
      const uint32_t len = run_length(pi.group_len, R, b);
      const bool ok = lo <= hi && hi <= len;
      if (!ok) report(kErrSplitRow);
      soff[b] = ok ? hi - lo : PART + 1;  // forces the size check below to fail
      ssrc[b] = pi.group_start + (uint64_t)b * R + lo;
    }
    __syncthreads();
    block_exclusive_scan(soff, F, wsum);
  }
  const uint32_t M = soff[F];
  if (M != pi.size) {  // split rows inconsistent with the partition: stop
    if (tid == 0) report(kErrPartSize);
    return;
  }

  // gather the partition's segments (coalesced within each segment): first
  // every source address, then all loads back to back, then the LDS stores
  {
    uint64_t addr[ITEMS];
    uint32_t runid[VMODE == 2 ? ITEMS : 1];
    uint32_t lpos[ITEMS];  // LDS slot of each item
    if constexpr (LABELS) {
      // Label every position with its segment (one byte each): thread t
      // labels positions 16t..16t+15, so each item below finds its segment
      // with one independent LDS read instead of a walk over the offsets.
      const uint32_t p0 = tid * LP;
      if (p0 < M) {
        uint32_t b = find_segment(soff, F, p0);
        uint32_t nxt = soff[b + 1];
        uint32_t wd[LP / 4];
#pragma unroll
        for (int j = 0; j < LP / 4; ++j) wd[j] = 0u;
#pragma unroll
        for (int j = 0; j < LP; ++j) {
          if (p0 + j < M) {
            while (p0 + j >= nxt) nxt = soff[++b + 1];
          }
          wd[j >> 2] |= b << (8 * (j & 3));
        }
#pragma unroll
        for (int j = 0; j < LP / 4; ++j) sseg[tid * (LP / 4) + j] = wd[j];
      }
      for (uint32_t b = tid; b < F; b += NT) ssrc[b] -= soff[b];
      __syncthreads();
      const uint8_t *seg_of = reinterpret_cast<const uint8_t *>(sseg);
      uint32_t bi[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = i * NT + tid;
        bi[i] = idx < M ? seg_of[idx] : 0u;
      }
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = i * NT + tid;
        addr[i] = ssrc[bi[i]] + idx;
        lpos[i] = idx + bi[i] * G;
        if constexpr (VMODE == 2) runid[i] = bi[i];
      }
    } else {
      uint32_t b = tid < M ? find_segment(soff, F, tid) : 0;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = i * NT + tid;
        addr[i] = 0;
        if (idx < M) {
          while (soff[b + 1] <= idx) ++b;
          addr[i] = ssrc[b] + (idx - soff[b]);
        }
        lpos[i] = idx;
        if constexpr (VMODE == 2) runid[i] = b;
      }
    }
    U kreg[ITEMS];
    uint32_t vreg[KV ? ITEMS : 1];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t idx = i * NT + tid;
      kreg[i] = idx < M ? __builtin_nontemporal_load(&src[addr[i]]) : U(0);  // read once
      if constexpr (VMODE == 1) vreg[i] = idx < M ? __builtin_nontemporal_load(&vsrc[addr[i]]) : 0u;
      if constexpr (VMODE == 2) vreg[i] = runid[i];
    }
    if constexpr (MAXF <= 64) {
      // While its loads are in flight, wave 0 computes the chunk prefix over
      // pairs of every merge round (published by the barrier below).
      if (tid < 64) {
        const uint32_t e = soff[tid < F ? tid : F];
        const uint32_t total = soff[F];
        auto off_at = [&](uint32_t j) {  // soff[j] for j <= F (all lanes take part)
          const uint32_t v = __shfl(e, (int)(j < 64 ? j : 63), 64);
          return j < 64 ? v : total;
        };
        uint32_t r = 0;
        for (uint32_t w = 1; w < F; w <<= 1, ++r) {
          const uint32_t np = (F + 2 * w - 1) / (2 * w);
          const uint32_t j0 = 2 * w * tid < F ? 2 * w * tid : F;
          const uint32_t j1 = 2 * w * tid + 2 * w < F ? 2 * w * tid + 2 * w : F;
          const uint32_t a0 = off_at(j0), b1 = off_at(j1);
          const uint32_t cc = tid < np ? (b1 - a0 + CI - 1) / CI : 0u;
          uint32_t xc = cc;
#pragma unroll
          for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(xc, d, 64);
            if ((int)tid >= d) xc += y;
          }
          if (tid < np) cpre[r * 33 + tid] = xc - cc;
          if (tid == np - 1) cpre[r * 33 + np] = xc;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t idx = i * NT + tid;
      if (idx < M) {
        sk[lpos[i]] = kreg[i];
        if constexpr (KV) sv[lpos[i]] = vreg[i];
      }
    }
    if constexpr (GAPS) {
      // the gap after segment b: slots soff[b+1] + b*G .. + G
      for (uint32_t t = tid; t < F * G; t += NT) {
        const uint32_t b = t / G;
        sk[soff[b + 1] + b * G + (t - b * G)] = key_max<U>();
      }
    }
  }
  __syncthreads();

  // rounds of pairwise stable merges: at width w, runs of w consecutive
  // segments are merged in pairs (the lower run wins ties)
  if constexpr (MAXF <= 64) {
    // Each pair's output is cut into chunks of CI that never cross into the
    // next pair; a chunk prefix over pairs maps threads to chunks.  With at
    // most 32 pairs, M <= PART keys fit in NT chunks.
    uint32_t round = 0;
    for (uint32_t w = 1; w < F; w <<= 1, ++round) {
      const uint32_t npairs = (F + 2 * w - 1) / (2 * w);
      const uint32_t *cp = cpre + round * 33;
      const uint32_t nchunks = cp[npairs];
      if (nchunks > NT && tid == 0) report(kErrPartSize);  // cannot happen for M <= PART
      U rk[CI];
      uint32_t rv[KV ? CI : 1];
      uint32_t start = 0, count = 0, gap_at = 0;
      bool last = false;
      if (GAPS && tid < nchunks) {
        uint32_t lo = 0, hi = npairs;  // pair q with cp[q] <= tid < cp[q+1]
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (cp[mid] <= tid) lo = mid;
          else hi = mid;
        }
        const uint32_t sa = 2 * w * lo;
        const uint32_t sb = sa + w < F ? sa + w : F;
        const uint32_t se = sa + 2 * w < F ? sa + 2 * w : F;
        const uint32_t la = soff[sb] - soff[sa], lb = soff[se] - soff[sb];
        const uint32_t a0 = soff[sa] + sa * G;
        const uint32_t b0 = sb < F ? soff[sb] + sb * G : a0 + la;  // no B: read A's gap
        const uint32_t o = (tid - cp[lo]) * CI;
        count = la + lb - o < (uint32_t)CI ? la + lb - o : (uint32_t)CI;
        start = a0 + o;
        last = o + count == la + lb;
        gap_at = a0 + la + lb;
        merge_chunk_keys<U, CI>(sk, a0, la, b0, lb, o, rk);
      } else if (!GAPS && tid < nchunks) {
        uint32_t lo = 0, hi = npairs;  // pair q with cp[q] <= tid < cp[q+1]
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (cp[mid] <= tid) lo = mid;
          else hi = mid;
        }
        const uint32_t s0 = 2 * w * lo;
        const uint32_t A0 = soff[s0];
        const uint32_t A1 = soff[s0 + w < F ? s0 + w : F];
        const uint32_t B1 = soff[s0 + 2 * w < F ? s0 + 2 * w : F];
        start = A0 + (tid - cp[lo]) * CI;
        count = B1 - start < (uint32_t)CI ? B1 - start : (uint32_t)CI;
        merge_chunk<U, KV, CI, false>(sk, sv, A0, A1, B1, start, rk, rv);
      }
      __syncthreads();
      if (GAPS) {
        // A pair's last chunk computes its outputs past the pair's end from
        // the gaps (the largest key) and stores them into the run's new gap,
        // which it then fills anyway: every active chunk stores all CI keys.
        if (count) {
#pragma unroll
          for (int i = 0; i < CI; ++i) sk[start + i] = rk[i];
          if (last)
            for (uint32_t j = 0; j < G; ++j) sk[gap_at + j] = key_max<U>();
        }
      } else {
#pragma unroll
        for (int i = 0; i < CI; ++i) {
          if ((uint32_t)i < count) {
            sk[start + i] = rk[i];
            if constexpr (KV) sv[start + i] = rv[i];
          }
        }
      }
      __syncthreads();
    }
  } else {
  const uint32_t p0 = tid * ITEMS;
  for (uint32_t w = 1; w < F; w <<= 1) {
    U rk[ITEMS];
    uint32_t rv[KV ? ITEMS : 1];
    if (p0 < M) {
      uint32_t A0 = 0, A1 = 0, B1 = 0, ai = 0, bi = 0, la = 0, lb = 0;
      U ka = 0, kb = 0;
      uint32_t va = 0, vb = 0;
      auto locate = [&](uint32_t pos) {
        const uint32_t seg = find_segment(soff, F, pos);
        const uint32_t s0 = (seg / (2 * w)) * (2 * w);
        A0 = soff[s0];
        A1 = soff[s0 + w < F ? s0 + w : F];
        B1 = soff[s0 + 2 * w < F ? s0 + 2 * w : F];
        la = A1 - A0;
        lb = B1 - A1;
        const uint32_t d = pos - A0;
        uint32_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (sk[A0 + mid] <= sk[A1 + d - 1 - mid]) lo = mid + 1;
          else hi = mid;
        }
        ai = lo;
        bi = d - lo;
        uint32_t ia = A0 + (ai < la ? ai : (la ? la - 1 : 0));
        uint32_t ib = A1 + (bi < lb ? bi : (lb ? lb - 1 : 0));
        ia = ia < M ? ia : M - 1;
        ib = ib < M ? ib : M - 1;
        ka = sk[ia];
        kb = sk[ib];
        if constexpr (KV) {
          va = sv[ia];
          vb = sv[ib];
        }
      };
      locate(p0);
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        if (p0 + i < M) {
          if (A0 + ai + bi == B1) locate(p0 + i);
          const bool takeA = ai < la && (bi >= lb || ka <= kb);
          rk[i] = takeA ? ka : kb;
          if constexpr (KV) rv[i] = takeA ? va : vb;
          uint32_t nxt = takeA ? A0 + ai + 1 : A1 + bi + 1;
          nxt = nxt < M ? nxt : M - 1;
          const U nk = sk[nxt];
          ka = takeA ? nk : ka;
          kb = takeA ? kb : nk;
          if constexpr (KV) {
            const uint32_t nv = sv[nxt];
            va = takeA ? nv : va;
            vb = takeA ? vb : nv;
          }
          ai += takeA ? 1u : 0u;
          bi += takeA ? 0u : 1u;
        }
      }
    }
    __syncthreads();
    if (p0 < M) {
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        if (p0 + i < M) {
          sk[p0 + i] = rk[i];
          if constexpr (KV) sv[p0 + i] = rv[i];
        }
      }
    }
    __syncthreads();
  }
  }

#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t idx = i * NT + tid;
    if (idx < M) {
      const U k = sk[idx];
      __builtin_nontemporal_store(final_pass ? Key<KT>::unmap(k) : k, &dst[pi.out_off + idx]);
      if constexpr (KV) __builtin_nontemporal_store(sv[idx], &vdst[pi.out_off + idx]);
    }
  }
  if (write_samples && !g.paper) {
    // this partition starts at group position rlo, a multiple of kSample
    const uint64_t rlo = pi.out_off - pi.group_start;
    uint64_t sbase;
    if (g.seg.off) {
      sbase = g.seg.soff[pi.seg] + ((pi.gg * g.group_len + rlo) >> kSampleLog2);
    } else {
      const uint64_t gi = blockIdx.x / (g.rows_per_group - 1);
      const uint64_t seg = gi / g.groups_per_seg, gg = gi % g.groups_per_seg;
      sbase = seg * (g.seg_len >> kSampleLog2) + ((gg * g.group_len + rlo) >> kSampleLog2);
    }
    for (uint32_t i = tid; i < (M >> kSampleLog2); i += NT)
      samples[sbase + i] = sk[(i << kSampleLog2) + kSample - 1];
  }
  if constexpr (VMODE == 2) {
    // per-run prefix counts at every kChunk-th output of this partition,
    // counted a block of CB chunks at a time (thread b carries run b's count)
    static_assert(MAXF <= NT, "one thread per run");
    constexpr uint32_t CB = kHistWords / MAXF;
    const uint32_t nch = (M + kChunk - 1) / kChunk;
    const uint64_t prow0 = (uint64_t)blockIdx.x * (kPart / kChunk);
    uint32_t run = tid < F ? pi.lo_row[tid] : 0u;
    for (uint32_t c0 = 0; c0 < nch; c0 += CB) {
      const uint32_t cb = nch - c0 < CB ? nch - c0 : CB;
      for (uint32_t i = tid; i < cb * F; i += NT) hist[i] = 0;
      __syncthreads();
      const uint32_t i1 = (c0 + cb) * kChunk < M ? (c0 + cb) * kChunk : M;
      for (uint32_t i = c0 * kChunk + tid; i < i1; i += NT)
        atomicAdd(&hist[(i / kChunk - c0) * F + sv[i]], 1u);
      __syncthreads();
      if (tid < F) {
        for (uint32_t c = 0; c < cb; ++c) {
          prefix[(prow0 + c0 + c) * g.fan + tid] = run;
          run += hist[c * F + tid];
        }
      }
      __syncthreads();
    }
  }
}

// --------------------------------------------------------------- K4 -------
// Size of each paper partition (sum over blocks of its split interval) and
// their exclusive scan: the offsets of the merged partitions in the output.
__global__ void partition_sizes_kernel(RunGeom g, const uint32_t *__restrict__ table,
                                       uint64_t *__restrict__ sizes) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.n_parts) return;
  const uint32_t *lo = table + p * g.sub_per_part * g.fan;
  const uint32_t *hi = table + (p + 1) * g.sub_per_part * g.fan;
  uint64_t m = 0;
  for (uint32_t b = 0; b < g.fan; ++b) m += hi[b] - lo[b];
  sizes[p] = m;
}

__global__ __launch_bounds__(1024) void exclusive_scan_u64_kernel(const uint64_t *__restrict__ in,
                                                                  uint64_t *__restrict__ out,
                                                                  uint64_t n) {
  __shared__ uint64_t wtot[16 + 1];
  __shared__ uint64_t carry;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (uint64_t base = 0; base < n; base += 1024) {
    const uint64_t i = base + tid;
    const uint64_t v = i < n ? in[i] : 0;
    uint64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(x, d, 64);
      if ((int)lane >= d) x += y;
    }
    if (lane == 63) wtot[wid] = x;
    __syncthreads();
    if (tid == 0) {
      uint64_t run = 0;
      for (int w = 0; w < 16; ++w) {
        const uint64_t t = wtot[w];
        wtot[w] = run;
        run += t;
      }
      wtot[16] = run;
    }
    __syncthreads();
    if (i < n) out[i] = carry + wtot[wid] + x - v;
    __syncthreads();
    if (tid == 0) carry += wtot[16];
    __syncthreads();
  }
  if (tid == 0) out[n] = carry;
}

// split[b][p] = t_b at the paper's rank r_p (p = 0..n_P), as 64-bit values.
__global__ void split_table_kernel(RunGeom g, const uint32_t *__restrict__ table,
                                   uint64_t *__restrict__ split) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t cols = (uint64_t)g.n_parts + 1;
  if (i >= (uint64_t)g.fan * cols) return;
  const uint64_t b = i / cols, p = i % cols;
  split[i] = table[p * g.sub_per_part * g.fan + b];
}

template <int KT>
__global__ void unmap_copy_kernel(const typename Key<KT>::U *__restrict__ src,
                                  typename Key<KT>::U *__restrict__ dst, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = Key<KT>::unmap(src[i]);
}

// ------------------------------------------------- step 4 by sorting ---
// Section 2.2's other way to merge: gather the n_B sorted segments of a
// partition and sort the whole.  One workgroup per chunk of at most kPart
// keys gathers its segments into LDS in run order, then sorts them with a
// bitonic network in LDS.  Key-value sorts order (key, LDS position): the
// position follows (run, position in run), so ties stay stable and the
// values are read through the sorted positions.
template <int KT, bool KV>
__global__ __launch_bounds__(kMergeThreads) void sort_merge_kernel(
    const typename Key<KT>::U *__restrict__ src, const uint32_t *__restrict__ vsrc,
    typename Key<KT>::U *__restrict__ dst, uint32_t *__restrict__ vdst, RunGeom g,
    const uint32_t *__restrict__ table, const uint64_t *__restrict__ part_off, int final_pass) {
  using U = typename Key<KT>::U;
  constexpr uint32_t NT = kMergeThreads;
  constexpr int ITEMS = kPart / NT;
  __shared__ U sk[kPart];
  __shared__ uint16_t spos[KV ? kPart : 1];
  __shared__ uint32_t sv[KV ? kPart : 1];
  __shared__ uint32_t soff[kMaxRuns + 1];
  __shared__ uint64_t ssrc[kMaxRuns];
  __shared__ uint32_t wsum[NT / 64 + 1];

  const uint32_t tid = threadIdx.x;
  const PartInfo pi = part_info(g, blockIdx.x, table, part_off);
  if (!pi.valid) return;
  const uint64_t R = g.run_len;
  const uint32_t F = (uint32_t)((pi.group_len + R - 1) / R);
  for (uint32_t b = tid; b < F; b += NT) {
    const uint32_t lo = pi.lo_row[b], hi = pi.hi_row[b];
    const uint32_t len = run_length(pi.group_len, R, b);
    const bool ok = lo <= hi && hi <= len;
    if (!ok) report(kErrSplitRow);
    soff[b] = ok ? hi - lo : (uint32_t)kPart + 1;  // forces the size check below to fail
    ssrc[b] = pi.group_start + (uint64_t)b * R + lo;
  }
  __syncthreads();
  block_exclusive_scan(soff, F, wsum);
  const uint32_t M = soff[F];
  if (M != pi.size) {
    if (tid == 0) report(kErrPartSize);
    return;
  }
  {
    uint64_t addr[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t idx = i * NT + tid;
      addr[i] = 0;
      if (idx < M) {
        const uint32_t b = find_segment(soff, F, idx);
        addr[i] = ssrc[b] + (idx - soff[b]);
      }
    }
    U kreg[ITEMS];
    uint32_t vreg[KV ? ITEMS : 1];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t idx = i * NT + tid;
      kreg[i] = idx < M ? src[addr[i]] : key_max<U>();
      if constexpr (KV) vreg[i] = idx < M ? vsrc[addr[i]] : 0u;
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint32_t idx = i * NT + tid;
      sk[idx] = kreg[i];
      if constexpr (KV) {
        spos[idx] = (uint16_t)idx;
        sv[idx] = vreg[i];
      }
    }
  }
  __syncthreads();
  // bitonic sort of all kPart slots (padding holds the largest key at
  // positions >= M, so it sorts after every real key)
  for (uint32_t k = 2; k <= (uint32_t)kPart; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t t = tid; t < (uint32_t)kPart / 2; t += NT) {
        const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const uint32_t l = i + j;
        const U a = sk[i], b = sk[l];
        bool gt = a > b;
        if constexpr (KV) gt = gt || (a == b && spos[i] > spos[l]);
        if (gt == ((i & k) == 0)) {
          sk[i] = b;
          sk[l] = a;
          if constexpr (KV) {
            const uint16_t pa = spos[i];
            spos[i] = spos[l];
            spos[l] = pa;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t idx = tid; idx < M; idx += NT) {
    const U k = sk[idx];
    dst[pi.out_off + idx] = final_pass ? Key<KT>::unmap(k) : k;
    if constexpr (KV) vdst[pi.out_off + idx] = sv[spos[idx]];
  }
}

// ------------------------------------------- regular-sampling pivots ---
// PSRS (Section 2.3): n_P - 1 samples at regular intervals of every sorted
// block, the samples sorted, n_P - 1 pivots at regular intervals of them, and
// every block cut by value (partition k: P_k < x <= P_{k+1}).  "Regular
// intervals" of a sorted sequence of length len are its positions
// floor(j len / n_P), j = 1..n_P-1; an empty block gives no samples.  Blocks
// hold mapped keys, so all comparisons are unsigned.

// One thread per sample: sample j of block b (only the first ceil(n / L)
// blocks are non-empty, and they come first).
template <typename U>
__global__ void psrs_sample_kernel(const U *__restrict__ blocks, RunGeom g, U *__restrict__ samples,
                                   uint64_t ns) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const uint64_t per = g.n_parts - 1;
  const uint64_t b = i / per, j = i % per + 1;
  const uint64_t L = g.run_len, start = b * L;
  const uint64_t len = g.n - start < L ? g.n - start : L;
  samples[i] = blocks[start + (j * len) / g.n_parts];
}

// One wave per boundary k = 0..n_P: lanes walk the blocks, each finds the
// number of elements <= P_k of its block by binary search; the wave sums them
// into bounds[k].  Boundaries 0 and n_P are the block ends.
template <int KT>
__global__ __launch_bounds__(256) void psrs_partition_kernel(
    const typename Key<KT>::U *__restrict__ blocks, RunGeom g,
    const typename Key<KT>::U *__restrict__ sorted_samples, uint64_t ns,
    uint64_t *__restrict__ bounds, typename Key<KT>::U *__restrict__ pivots,
    uint64_t *__restrict__ split) {
  using U = typename Key<KT>::U;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t k = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t P = g.n_parts;
  if (k > P) return;
  const uint64_t L = g.run_len;
  const bool inner = k > 0 && k < P && ns > 0;
  const U piv = inner ? sorted_samples[(k * ns) / P] : U(0);
  if (pivots && k > 0 && k < P && lane == 0) pivots[k - 1] = inner ? Key<KT>::unmap(piv) : U(0);
  uint64_t sum = 0;
  for (uint32_t b = lane; b < g.fan; b += 64) {
    const uint64_t start = (uint64_t)b * L;
    const uint64_t len = start >= g.n ? 0 : (g.n - start < L ? g.n - start : L);
    uint64_t c;
    if (k == 0 || (k < P && !inner)) {
      c = 0;
    } else if (k == P) {
      c = len;
    } else {
      uint64_t lo = 0, hi = len;
      while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (blocks[start + mid] <= piv) lo = mid + 1;
        else hi = mid;
      }
      c = lo;
    }
    if (split) split[(uint64_t)b * (P + 1) + k] = c;
    sum += c;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
  if (lane == 0) bounds[k] = sum;
}

// Partition sizes and their chunk counts ceil(size / part_len).
__global__ void psrs_chunks_kernel(RunGeom g, const uint64_t *__restrict__ bounds,
                                   uint64_t *__restrict__ sizes, uint64_t *__restrict__ chunks) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.n_parts) return;
  const uint64_t m = bounds[p + 1] - bounds[p];
  if (sizes) sizes[p] = m;
  chunks[p] = (m + g.part_len - 1) / g.part_len;
}

// ------------------------------------------------------------ records ---
// Fixed-size records sorted by a key field (Table 1's Pair and Particle):
// the keys and their input indices go through the key-value sort, then the
// whole records are gathered in the sorted order.

template <typename U>
__global__ void record_keys_kernel(const unsigned char *__restrict__ rec, uint64_t n, uint32_t rb,
                                   uint32_t koff, U *__restrict__ keys, uint32_t *__restrict__ idx) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[i] = *reinterpret_cast<const U *>(rec + i * rb + koff);
  idx[i] = (uint32_t)i;
}

// Each workgroup copies blockDim / words whole records, one W-sized word per
// thread: word w of output record j is word w of input record perm[j].
// Stores are contiguous across the workgroup; loads within a record.
template <typename W>
__global__ void record_gather_kernel(const W *__restrict__ in, W *__restrict__ out,
                                     const uint32_t *__restrict__ perm, uint64_t n,
                                     uint32_t words) {
  const uint32_t rpb = blockDim.x / words;
  const uint32_t r = threadIdx.x / words, w = threadIdx.x - r * words;
  const uint64_t j = (uint64_t)blockIdx.x * rpb + r;
  if (r >= rpb || j >= n) return;
  out[j * words + w] = in[(uint64_t)perm[j] * words + w];
}

// ------------------------------------------------- segmented planning ---
// One workgroup reads the segment offsets, checks them, and writes per
// segment: its tile class and tiles, merge passes, samples, and per pass the
// table rows and partitions at key and sample level; then turns every array
// into an exclusive prefix over segments.  Invalid offsets (not starting at
// 0, decreasing, or ending beyond n) give an empty plan and an error bit.
struct SegPlanArrays {
  uint64_t *tiles[3];
  uint64_t *soff;
  uint32_t *npass;
  uint64_t *rows[kMaxSegPasses], *parts[kMaxSegPasses];
  uint64_t *srows[kMaxSegPasses], *sparts[kMaxSegPasses];
};

__device__ void block_inclusive_scan_u64(uint64_t *a, uint32_t n, uint64_t *wsum) {
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const uint32_t lane = tid & 63, wid = tid >> 6, nw = nthr >> 6;
  const uint32_t per = (n + nthr - 1) / nthr;
  const uint32_t beg = tid * per < n ? tid * per : n;
  const uint32_t end = beg + per < n ? beg + per : n;
  uint64_t s = 0;
  for (uint32_t i = beg; i < end; ++i) s += a[i];
  uint64_t x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if ((int)lane >= d) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (tid == 0) {
    uint64_t run = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      const uint64_t v = wsum[w];
      wsum[w] = run;
      run += v;
    }
  }
  __syncthreads();
  uint64_t e = x - s + wsum[wid];
  for (uint32_t i = beg; i < end; ++i) {
    e += a[i];
    a[i] = e;
  }
  __syncthreads();
}

__global__ __launch_bounds__(1024) void seg_plan_kernel(const uint64_t *__restrict__ off,
                                                        uint32_t n_segs, uint64_t n,
                                                        SegPlanArrays pa, uint32_t small0,
                                                        uint32_t small1, uint32_t max_passes,
                                                        uint32_t fan_log2, uint32_t tile,
                                                        uint32_t part) {
  __shared__ uint64_t wsum[17];
  __shared__ uint32_t bad;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) bad = (off[0] != 0 || off[n_segs] > n) ? 1u : 0u;
  __syncthreads();
  for (uint32_t s = tid; s < n_segs; s += blockDim.x)
    if (off[s + 1] < off[s]) atomicOr(&bad, 1u);
  __syncthreads();
  const bool ok = bad == 0;
  if (tid == 0 && !ok) report(kErrSegments);
  for (uint32_t s = tid; s <= n_segs; s += blockDim.x) {
    // index s+1 holds segment s's count; index 0 stays 0 (exclusive prefix)
    if (s == 0) {
      for (int c = 0; c < 3; ++c) pa.tiles[c][0] = 0;
      pa.soff[0] = 0;
      for (uint32_t q = 0; q < max_passes; ++q) {
        pa.rows[q][0] = 0;
        pa.parts[q][0] = 0;
        pa.srows[q][0] = 0;
        pa.sparts[q][0] = 0;
      }
    }
    if (s == n_segs) continue;
    const uint64_t L = ok ? off[s + 1] - off[s] : 0;
    int cls = L == 0 ? -1 : (L <= small0 ? 0 : (L <= small1 ? 1 : 2));
    uint32_t np = 0;
    if (cls == 2 && L > (uint64_t)tile) {
      const uint64_t tiles = (L + tile - 1) / tile;
      uint32_t bits = 0;
      while (((uint64_t)1 << bits) < tiles) ++bits;
      np = (bits + fan_log2 - 1) / fan_log2;
    }
    if (np > max_passes) {  // the host bound on passes was too small
      atomicOr(&bad, 2u);
      np = 0;
      cls = -1;
    }
    for (int c = 0; c < 3; ++c)
      pa.tiles[c][s + 1] = c == cls ? (c == 2 ? (L + tile - 1) / tile : 1) : 0;
    pa.npass[s] = np;
    pa.soff[s + 1] = np ? (L >> kSampleLog2) : 0;
    const uint64_t Ls = L >> kSampleLog2;
    for (uint32_t q = 1; q <= max_passes; ++q) {
      uint64_t rows = 0, parts = 0, srows = 0, sparts = 0;
      if (q <= np) {
        const uint64_t R = (uint64_t)tile << (fan_log2 * (q - 1));
        const uint64_t G = R << fan_log2, Gs = G >> kSampleLog2;
        const uint64_t ng = (L + G - 1) / G;
        for (uint64_t gg = 0; gg < ng; ++gg) {
          const uint64_t glen = L - gg * G < G ? L - gg * G : G;
          const uint64_t gs = gg * Gs < Ls ? (Ls - gg * Gs < Gs ? Ls - gg * Gs : Gs) : 0;
          parts += (glen + part - 1) / part;
          rows += (glen + part - 1) / part + 1;
          sparts += (gs + kPart - 1) / kPart;
          srows += (gs + kPart - 1) / kPart + 1;
        }
      }
      pa.rows[q - 1][s + 1] = rows;
      pa.parts[q - 1][s + 1] = parts;
      pa.srows[q - 1][s + 1] = srows;
      pa.sparts[q - 1][s + 1] = sparts;
    }
  }
  __syncthreads();
  if (tid == 0 && (bad & 2u)) report(kErrSegments);
  for (int c = 0; c < 3; ++c) block_inclusive_scan_u64(pa.tiles[c] + 1, n_segs, wsum);
  block_inclusive_scan_u64(pa.soff + 1, n_segs, wsum);
  for (uint32_t q = 0; q < max_passes; ++q) {
    block_inclusive_scan_u64(pa.rows[q] + 1, n_segs, wsum);
    block_inclusive_scan_u64(pa.parts[q] + 1, n_segs, wsum);
    block_inclusive_scan_u64(pa.srows[q] + 1, n_segs, wsum);
    block_inclusive_scan_u64(pa.sparts[q] + 1, n_segs, wsum);
  }
}

template <typename F>
hipError_t dispatch_kt(int kt, F &&f) {
  switch (kt) {
    case 0: return f(std::integral_constant<int, 0>{});
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// ------------------------------------------------------------ launchers ---
namespace {
template <int KT, bool KV, int THREADS>
hipError_t go_tile(const void *in, const uint32_t *vin, const TileArgs<typename Key<KT>::U> &ta,
                   uint64_t grid, hipStream_t s) {
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((tile_sort_kernel<KT, KV, THREADS>), dim3((uint32_t)grid), dim3(THREADS), 0, s,
                     (const typename Key<KT>::U *)in, vin, ta);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_tile_sort(int kt, bool kv, const void *in, const uint32_t *vin, void *out,
                            uint32_t *vout, uint64_t n, uint64_t seg_len, uint32_t tile,
                            int final_pass, void *samples, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (tile != (uint32_t)kTile && !(kv && tile == (uint32_t)kTileKV)) return hipErrorInvalidValue;
  const uint64_t tps = (seg_len + tile - 1) / tile;
  const uint64_t nseg = (n + seg_len - 1) / seg_len;
  const uint64_t grid = nseg * tps;
  return dispatch_kt(kt, [&](auto ktc) {
    constexpr int KT = decltype(ktc)::value;
    using U = typename Key<KT>::U;
    TileArgs<U> ta{};
    ta.n = n;
    ta.seg_len = seg_len;
    ta.tiles_per_seg = tps;
    ta.final_pass = final_pass;
    ta.out = ta.out_alt = (U *)out;
    ta.vout = ta.vout_alt = vout;
    ta.samples = (U *)samples;
    if (kv && tile == (uint32_t)kTileKV) return go_tile<KT, true, kTileKVThreads>(in, vin, ta, grid, s);
    return kv ? go_tile<KT, true, kTileThreads>(in, vin, ta, grid, s)
              : go_tile<KT, false, kTileThreads>(in, vin, ta, grid, s);
  });
}

hipError_t launch_seg_plan(const uint64_t *seg_off, uint32_t n_segs, uint64_t n,
                           const SegPlanPtrs &pp, uint32_t small0, uint32_t small1,
                           uint32_t max_passes, uint32_t fan_log2, uint32_t tile, uint32_t part,
                           hipStream_t s) {
  SegPlanArrays pa{};
  for (int c = 0; c < 3; ++c) pa.tiles[c] = pp.tiles[c];
  pa.soff = pp.soff;
  pa.npass = pp.npass;
  for (uint32_t q = 0; q < kMaxSegPasses; ++q) {
    pa.rows[q] = pp.rows[q];
    pa.parts[q] = pp.parts[q];
    pa.srows[q] = pp.srows[q];
    pa.sparts[q] = pp.sparts[q];
  }
  hipLaunchKernelGGL(seg_plan_kernel, dim3(1), dim3(1024), 0, s, seg_off, n_segs, n, pa, small0,
                     small1, max_passes, fan_log2, tile, part);
  return hipGetLastError();
}

hipError_t launch_seg_tile_sorts(int kt, bool kv, const void *in, const uint32_t *vin, void *out,
                                 void *out_alt, uint32_t *vout, uint32_t *vout_alt, void *samples,
                                 const uint64_t *seg_off, const SegPlanPtrs &pp, uint32_t n_segs,
                                 uint64_t n, uint32_t tile, hipStream_t s) {
  if (tile != (uint32_t)kTile && !(kv && tile == (uint32_t)kTileKV)) return hipErrorInvalidValue;
  return dispatch_kt(kt, [&](auto ktc) {
    constexpr int KT = decltype(ktc)::value;
    using U = typename Key<KT>::U;
    TileArgs<U> ta{};
    ta.out = (U *)out;
    ta.out_alt = (U *)out_alt;
    ta.vout = vout;
    ta.vout_alt = vout_alt;
    ta.samples = (U *)samples;
    ta.seg_off = seg_off;
    ta.soff = pp.soff;
    ta.npass = pp.npass;
    ta.n_segs = n_segs;
    hipError_t e;
    // class 0: one 2048-key tile per segment; class 1: one 4096-key tile;
    // class 2: tiles of `tile` keys
    ta.tiles = pp.tiles[0];
    e = kv ? go_tile<KT, true, kSmallThreads0>(in, vin, ta, n_segs, s)
           : go_tile<KT, false, kSmallThreads0>(in, vin, ta, n_segs, s);
    if (e != hipSuccess) return e;
    ta.tiles = pp.tiles[1];
    e = kv ? go_tile<KT, true, kSmallThreads1>(in, vin, ta, n_segs, s)
           : go_tile<KT, false, kSmallThreads1>(in, vin, ta, n_segs, s);
    if (e != hipSuccess) return e;
    ta.tiles = pp.tiles[2];
    const uint64_t grid = (n + tile - 1) / tile + n_segs;
    if (kv && tile == (uint32_t)kTileKV) return go_tile<KT, true, kTileKVThreads>(in, vin, ta, grid, s);
    return kv ? go_tile<KT, true, kTileThreads>(in, vin, ta, grid, s)
              : go_tile<KT, false, kTileThreads>(in, vin, ta, grid, s);
  });
}

hipError_t launch_corank(int kt, const void *src, const RunGeom &g, uint32_t *table,
                         void *pivots, uint64_t *counts, hipStream_t s, const void *src_alt) {
  const uint64_t rows = g.total_rows();
  if (rows == 0) return hipSuccess;
  if (!src_alt) src_alt = src;
  // up to 512 runs the (fewer than 3 * fan) candidates are sorted in
  // registers, 64 * E slots; beyond, in LDS
  auto go = [&](auto u, auto maxf) -> hipError_t {
    using U = decltype(u);
    constexpr uint32_t MAXF = decltype(maxf)::value;
    constexpr int E = MAXF <= 512 ? (int)(MAXF / 16) : 0;
    const SampleIndex none{nullptr, nullptr, g};
    hipLaunchKernelGGL((corank_kernel<U, MAXF, E>), dim3((uint32_t)rows), dim3(kCorankThreads), 0,
                       s, (const U *)src, g, table, (U *)pivots, counts, kt, none);
    return hipGetLastError();
  };
  const bool wide = key_bytes(kt) == 8;
  if (g.fan <= 64) {
    const SampleIndex none{nullptr, nullptr, g};
    // fewer than 3 * fan candidates a level: two slots a lane up to 32 runs
    auto wave = [&](auto u, auto e) -> hipError_t {
      using U = decltype(u);
      hipLaunchKernelGGL((corank_wave_kernel<U, decltype(e)::value, false>), dim3((uint32_t)rows),
                         dim3(kCorankThreads), 0, s, (const U *)src, (const U *)src_alt, g, table,
                         (U *)pivots, counts, kt, none);
      return hipGetLastError();
    };
    using E2 = std::integral_constant<int, 2>;
    using E4 = std::integral_constant<int, 4>;
    if (g.fan <= 32) return wide ? wave(uint64_t{}, E2{}) : wave(uint32_t{}, E2{});
    return wide ? wave(uint64_t{}, E4{}) : wave(uint32_t{}, E4{});
  }
  if (g.seg.off) return hipErrorInvalidValue;
  if (g.fan <= 128)
    return wide ? go(uint64_t{}, std::integral_constant<uint32_t, 128>{})
                : go(uint32_t{}, std::integral_constant<uint32_t, 128>{});
  if (g.fan <= 256)
    return wide ? go(uint64_t{}, std::integral_constant<uint32_t, 256>{})
                : go(uint32_t{}, std::integral_constant<uint32_t, 256>{});
  if (g.fan <= 512)
    return wide ? go(uint64_t{}, std::integral_constant<uint32_t, 512>{})
                : go(uint32_t{}, std::integral_constant<uint32_t, 512>{});
  if (g.fan <= kMaxRuns)
    return wide ? go(uint64_t{}, std::integral_constant<uint32_t, kMaxRuns>{})
                : go(uint32_t{}, std::integral_constant<uint32_t, kMaxRuns>{});
  return hipErrorInvalidValue;
}

hipError_t launch_corank_sampled(int kt, const void *src, const RunGeom &g, uint32_t *table,
                                 const uint32_t *sample_runs, const uint32_t *sample_prefix,
                                 hipStream_t s, const void *src_alt, const RunGeom *gs_in) {
  const uint64_t rows = g.total_rows();
  if (rows == 0) return hipSuccess;
  if (g.fan > kMaxSampledFan) return hipErrorInvalidValue;
  // the paper's single level has no uniform sample geometry of its own
  if (g.paper && !gs_in) return hipErrorInvalidValue;
  if (!src_alt) src_alt = src;
  const SampleIndex si{sample_runs, sample_prefix, gs_in ? *gs_in : sample_geom(g)};
  // fewer than 3 * fan candidates a level: two slots a lane up to 32 runs
  auto wave = [&](auto u, auto e) -> hipError_t {
    using U = decltype(u);
    hipLaunchKernelGGL((corank_wave_kernel<U, decltype(e)::value, true>), dim3((uint32_t)rows),
                       dim3(kCorankThreads), 0, s, (const U *)src, (const U *)src_alt, g, table,
                       (U *)nullptr, (uint64_t *)nullptr, kt, si);
    return hipGetLastError();
  };
  using E2 = std::integral_constant<int, 2>;
  using E4 = std::integral_constant<int, 4>;
  const bool wide = key_bytes(kt) == 8;
  if (g.fan <= 32) return wide ? wave(uint64_t{}, E2{}) : wave(uint32_t{}, E2{});
  if (g.fan <= 64) return wide ? wave(uint64_t{}, E4{}) : wave(uint32_t{}, E4{});
  // 65-256 runs (the paper's single level only): per-run counts in LDS
  if (g.seg.off) return hipErrorInvalidValue;
  if (wide)
    hipLaunchKernelGGL((corank_kernel<uint64_t, 256, 16, true>), dim3((uint32_t)rows),
                       dim3(kCorankThreads), 0, s, (const uint64_t *)src, g, table,
                       (uint64_t *)nullptr, (uint64_t *)nullptr, kt, si);
  else
    hipLaunchKernelGGL((corank_kernel<uint32_t, 256, 16, true>), dim3((uint32_t)rows),
                       dim3(kCorankThreads), 0, s, (const uint32_t *)src, g, table,
                       (uint32_t *)nullptr, (uint64_t *)nullptr, kt, si);
  return hipGetLastError();
}

hipError_t launch_merge(int kt, int vmode, const void *src, const uint32_t *vsrc, void *dst,
                        uint32_t *vdst, const RunGeom &g, const uint32_t *table,
                        const uint64_t *part_offsets, int final_pass, void *samples,
                        uint32_t *prefix, hipStream_t s, const MergeAlt *alt) {
  const uint64_t parts = g.total_parts();
  if (parts == 0) return hipSuccess;
  if (vmode == 2) {
    // sample arrays hold mapped keys: merge them as plain unsigned integers
    if (g.fan > kMaxSampledFan || final_pass || samples) return hipErrorInvalidValue;
    auto go2 = [&](auto u) -> hipError_t {
      using U = decltype(u);
      constexpr int KTI = sizeof(U) == 8 ? 2 : 0;
      MergeBufs<U> b{(const U *)src, (const U *)src, vsrc, vsrc, (U *)dst, (U *)dst, vdst, vdst};
      if (g.fan <= 64)
        hipLaunchKernelGGL((merge_kernel<KTI, 2, 64, 2 * kMergeThreads>), dim3((uint32_t)parts),
                           dim3(2 * kMergeThreads), 0, s,
                           b, g, table, part_offsets, 0, (U *)nullptr, prefix);
      else
        hipLaunchKernelGGL((merge_kernel<KTI, 2, 256, kMergeThreads>), dim3((uint32_t)parts),
                           dim3(kMergeThreads), 0, s,
                           b, g, table, part_offsets, 0, (U *)nullptr, prefix);
      return hipGetLastError();
    };
    return key_bytes(kt) == 8 ? go2(uint64_t{}) : go2(uint32_t{});
  }
  return dispatch_kt(kt, [&](auto ktc) {
    constexpr int KT = decltype(ktc)::value;
    using U = typename Key<KT>::U;
    MergeBufs<U> b{(const U *)src, (const U *)src, vsrc, vsrc, (U *)dst, (U *)dst, vdst, vdst};
    if (alt) {
      b.src_alt = (const U *)alt->src;
      b.vsrc_alt = alt->vsrc;
      b.dst_alt = (U *)alt->dst;
      b.vdst_alt = alt->vdst;
    }
    auto go = [&](auto vm, auto maxf) -> hipError_t {
      constexpr int VM = decltype(vm)::value;
      constexpr uint32_t MAXF = decltype(maxf)::value;
      // key-value merges hold 12 bytes a key in LDS (one workgroup per CU):
      // twice the threads there hide more latency
      constexpr uint32_t NT = VM == 1 && MAXF <= 64 ? 2 * kMergeThreads : kMergeThreads;
      hipLaunchKernelGGL((merge_kernel<KT, VM, MAXF, NT>), dim3((uint32_t)parts), dim3(NT), 0, s,
                         b, g, table, part_offsets, final_pass, (U *)samples, (uint32_t *)nullptr);
      return hipGetLastError();
    };
    const bool kv = vmode == 1;
    if (g.part_len != (uint32_t)kPart) {
      // key-value passes of the automatic plan and segmented mode: 4096-key partitions
      if (!kv || g.part_len != (uint32_t)kPartKV || g.fan > 64 || g.paper)
        return hipErrorInvalidValue;
      constexpr uint32_t NT = 2 * kMergeThreads;
      hipLaunchKernelGGL((merge_kernel<KT, 1, 64, NT, kPartKV>), dim3((uint32_t)parts), dim3(NT), 0,
                         s, b, g, table, part_offsets, final_pass, (U *)samples, (uint32_t *)nullptr);
      return hipGetLastError();
    }
    if (!kv && g.fan <= 32) {
      constexpr uint32_t NT = 2 * kMergeThreads;
      hipLaunchKernelGGL((merge_kernel<KT, 0, 32, NT>), dim3((uint32_t)parts), dim3(NT), 0, s,
                         b, g, table, part_offsets, final_pass, (U *)samples, (uint32_t *)nullptr);
      return hipGetLastError();
    }
    if (g.fan <= 64)
      return kv ? go(std::integral_constant<int, 1>{}, std::integral_constant<uint32_t, 64>{})
                : go(std::integral_constant<int, 0>{}, std::integral_constant<uint32_t, 64>{});
    if (g.seg.off) return hipErrorInvalidValue;
    if (g.fan <= 256)
      return kv ? go(std::integral_constant<int, 1>{}, std::integral_constant<uint32_t, 256>{})
                : go(std::integral_constant<int, 0>{}, std::integral_constant<uint32_t, 256>{});
    if (g.fan <= kMaxRuns)
      return kv ? go(std::integral_constant<int, 1>{}, std::integral_constant<uint32_t, kMaxRuns>{})
                : go(std::integral_constant<int, 0>{}, std::integral_constant<uint32_t, kMaxRuns>{});
    return hipErrorInvalidValue;
  });
}

hipError_t launch_partition_offsets(const RunGeom &g, const uint32_t *table, uint64_t *sizes,
                                    uint64_t *offsets, hipStream_t s) {
  const uint32_t blocks = (uint32_t)((g.n_parts + 255) / 256);
  hipLaunchKernelGGL(partition_sizes_kernel, dim3(blocks), dim3(256), 0, s, g, table, sizes);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(exclusive_scan_u64_kernel, dim3(1), dim3(1024), 0, s, (const uint64_t *)sizes,
                     offsets, (uint64_t)g.n_parts);
  return hipGetLastError();
}

hipError_t launch_split_table(const RunGeom &g, const uint32_t *table, uint64_t *split,
                              hipStream_t s) {
  const uint64_t total = (uint64_t)g.fan * ((uint64_t)g.n_parts + 1);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(split_table_kernel, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, g,
                     table, split);
  return hipGetLastError();
}

hipError_t launch_psrs_samples(int kt, const void *blocks, const RunGeom &g, void *samples,
                               hipStream_t s) {
  if (g.n == 0 || g.n_parts < 2) return hipSuccess;
  const uint64_t nonempty = (g.n + g.run_len - 1) / g.run_len;
  const uint64_t ns = nonempty * (g.n_parts - 1);
  const uint32_t grid = (uint32_t)((ns + 255) / 256);
  if (key_bytes(kt) == 8)
    hipLaunchKernelGGL((psrs_sample_kernel<uint64_t>), dim3(grid), dim3(256), 0, s,
                       (const uint64_t *)blocks, g, (uint64_t *)samples, ns);
  else
    hipLaunchKernelGGL((psrs_sample_kernel<uint32_t>), dim3(grid), dim3(256), 0, s,
                       (const uint32_t *)blocks, g, (uint32_t *)samples, ns);
  return hipGetLastError();
}

hipError_t launch_psrs_partition(int kt, const void *blocks, const RunGeom &g,
                                 const void *sorted_samples, uint64_t ns, uint64_t *bounds,
                                 void *pivots, uint64_t *split, hipStream_t s) {
  const uint32_t grid = (uint32_t)(((uint64_t)g.n_parts + 1 + 3) / 4);
  return dispatch_kt(kt, [&](auto ktc) {
    constexpr int KT = decltype(ktc)::value;
    using U = typename Key<KT>::U;
    hipLaunchKernelGGL((psrs_partition_kernel<KT>), dim3(grid), dim3(256), 0, s,
                       (const U *)blocks, g, (const U *)sorted_samples, ns, bounds, (U *)pivots,
                       split);
    return hipGetLastError();
  });
}

hipError_t launch_psrs_chunks(const RunGeom &g, const uint64_t *bounds, uint64_t *sizes,
                              uint64_t *chunks, uint64_t *chunk_prefix, hipStream_t s) {
  hipLaunchKernelGGL(psrs_chunks_kernel, dim3((uint32_t)((g.n_parts + 255) / 256)), dim3(256), 0,
                     s, g, bounds, sizes, chunks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(exclusive_scan_u64_kernel, dim3(1), dim3(1024), 0, s, (const uint64_t *)chunks,
                     chunk_prefix, (uint64_t)g.n_parts);
  return hipGetLastError();
}

hipError_t launch_sort_merge(int kt, bool kv, const void *src, const uint32_t *vsrc, void *dst,
                             uint32_t *vdst, const RunGeom &g, const uint32_t *table,
                             const uint64_t *part_offsets, int final_pass, hipStream_t s) {
  const uint64_t parts = g.total_parts();
  if (parts == 0) return hipSuccess;
  if (!g.paper || g.fan > kMaxRuns) return hipErrorInvalidValue;
  return dispatch_kt(kt, [&](auto ktc) {
    constexpr int KT = decltype(ktc)::value;
    using U = typename Key<KT>::U;
    if (kv)
      hipLaunchKernelGGL((sort_merge_kernel<KT, true>), dim3((uint32_t)parts), dim3(kMergeThreads),
                         0, s, (const U *)src, vsrc, (U *)dst, vdst, g, table, part_offsets,
                         final_pass);
    else
      hipLaunchKernelGGL((sort_merge_kernel<KT, false>), dim3((uint32_t)parts), dim3(kMergeThreads),
                         0, s, (const U *)src, vsrc, (U *)dst, vdst, g, table, part_offsets,
                         final_pass);
    return hipGetLastError();
  });
}

hipError_t launch_record_keys(int kt, const void *records, uint64_t n, uint32_t record_bytes,
                              uint32_t key_offset, void *keys, uint32_t *idx, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)((n + 255) / 256);
  if (key_bytes(kt) == 8)
    hipLaunchKernelGGL((record_keys_kernel<uint64_t>), dim3(grid), dim3(256), 0, s,
                       (const unsigned char *)records, n, record_bytes, key_offset,
                       (uint64_t *)keys, idx);
  else
    hipLaunchKernelGGL((record_keys_kernel<uint32_t>), dim3(grid), dim3(256), 0, s,
                       (const unsigned char *)records, n, record_bytes, key_offset,
                       (uint32_t *)keys, idx);
  return hipGetLastError();
}

hipError_t launch_record_gather(const void *in, void *out, const uint32_t *perm, uint64_t n,
                                uint32_t record_bytes, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uintptr_t align = (uintptr_t)in | (uintptr_t)out | record_bytes;
  auto go = [&](auto w) -> hipError_t {
    using W = decltype(w);
    const uint32_t words = record_bytes / (uint32_t)sizeof(W);
    const uint32_t threads = words <= 256 ? 256 : 1024;
    if (words > threads) return hipErrorInvalidValue;
    const uint64_t rpb = threads / words;
    const uint64_t grid = (n + rpb - 1) / rpb;
    if (grid > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((record_gather_kernel<W>), dim3((uint32_t)grid), dim3(threads), 0, s,
                       (const W *)in, (W *)out, perm, n, words);
    return hipGetLastError();
  };
  if (align % 16 == 0) return go(uint4{});
  if (align % 8 == 0) return go(uint2{});
  if (align % 4 == 0) return go(uint32_t{});
  return hipErrorInvalidValue;
}

hipError_t read_device_error(uint32_t *code, bool clear) {
  hipError_t e = hipMemcpyFromSymbol(code, HIP_SYMBOL(g_device_error), sizeof(uint32_t), 0,
                                     hipMemcpyDeviceToHost);
  if (e != hipSuccess || !clear) return e;
  const uint32_t zero = 0;
  return hipMemcpyToSymbol(HIP_SYMBOL(g_device_error), &zero, sizeof(uint32_t), 0,
                           hipMemcpyHostToDevice);
}

hipError_t read_device_error_async(uint32_t *host_code, hipStream_t s) {
  return hipMemcpyFromSymbolAsync(host_code, HIP_SYMBOL(g_device_error), sizeof(uint32_t), 0,
                                  hipMemcpyDeviceToHost, s);
}

hipError_t launch_unmap_copy(int kt, const void *src, void *dst, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  return dispatch_kt(kt, [&](auto ktc) {
    constexpr int KT = decltype(ktc)::value;
    using U = typename Key<KT>::U;
    hipLaunchKernelGGL((unmap_copy_kernel<KT>), dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s,
                       (const U *)src, (U *)dst, n);
    return hipGetLastError();
  });
}

}  // namespace pss
