/*
 * pses_oracle.c -- TEST INFRASTRUCTURE ONLY (see pses_oracle.h).
 *
 * Sequential CPU reference of the paper's four-step parallel samplesort with
 * exact splitting (PSES), arXiv 2305.05245, Section 2:
 *   O0  key order (integer order, IEEE totalOrder for floats)
 *   O1  step 1: split A into n_B contiguous blocks of length ceil(N/n_B) and
 *       sort each block (Section 2, "sorting each block")
 *   O2  step 2: PSES pivots P_k and counts c_k (Section 2.3, Eq. 1, Eq. 2),
 *       found by binary search with per-block binary-search counting
 *   O3  step 3: partition each sorted block (Section 2 and Section 2.3: the
 *       k-th partition takes the elements between consecutive pivots plus c_k
 *       copies of a pivot value, Fig. 3b)
 *   O4  offsets of the merged partitions, computed sequentially (Section 2)
 *   O5  step 4: multiway merge of the k-th partition of every block with a
 *       selection tree (Section 2.2, tree selection after Knuth vol. 3)
 * and, for comparison, the same steps with PSRS pivots (regular sampling,
 * Section 2.3, first paragraph; oracle_psrs at the end of this file).
 * Everything is done one element at a time, in the order the paper states the
 * steps, with no blocking or fusion.  Slow on purpose.
 */
#include "pses_oracle.h"

#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---------------------------------------------------------------- O0 ---- */

static int key_bytes(int dtype) {
  switch (dtype) {
    case 0: case 1: case 4: return 4;
    case 2: case 3: case 5: return 8;
    default: return 0;
  }
}

static int cmp_u64(uint64_t a, uint64_t b) { return a < b ? -1 : (a > b ? 1 : 0); }
static int cmp_i64(int64_t a, int64_t b) { return a < b ? -1 : (a > b ? 1 : 0); }

/* IEEE 754-2019 totalOrder on raw bits of width `w` bits.  From the
 * definition: a negative-signed datum is below every positive-signed one;
 * between two positive-signed data the one with the larger magnitude field
 * (exponent and significand, read as an unsigned integer) is larger; between
 * two negative-signed data the one with the larger magnitude is smaller.  This
 * puts -NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN and orders NaNs of one
 * sign by payload.  Equal only when the bit patterns are equal. */
static int cmp_total_order(uint64_t a, uint64_t b, int w) {
  const uint64_t sign = (uint64_t)1 << (w - 1);
  const uint64_t mag_mask = sign - 1;
  const int sa = (a & sign) != 0, sb = (b & sign) != 0;
  const uint64_t ma = a & mag_mask, mb = b & mag_mask;
  if (sa != sb) return sa ? -1 : 1;
  if (!sa) return cmp_u64(ma, mb);
  return cmp_u64(mb, ma);
}

int oracle_compare(int dtype, uint64_t a, uint64_t b) {
  switch (dtype) {
    case 0: return cmp_u64(a & 0xffffffffu, b & 0xffffffffu);
    case 1: return cmp_i64((int32_t)(uint32_t)a, (int32_t)(uint32_t)b);
    case 2: return cmp_u64(a, b);
    case 3: return cmp_i64((int64_t)a, (int64_t)b);
    case 4: return cmp_total_order(a & 0xffffffffu, b & 0xffffffffu, 32);
    case 5: return cmp_total_order(a, b, 64);
    default: return 0;
  }
}

static uint64_t load_bits(const void *base, uint64_t i, int kb) {
  if (kb == 4) {
    uint32_t v;
    memcpy(&v, (const unsigned char *)base + i * 4, 4);
    return v;
  }
  uint64_t v;
  memcpy(&v, (const unsigned char *)base + i * 8, 8);
  return v;
}

static void store_bits(void *base, uint64_t i, int kb, uint64_t bits) {
  if (kb == 4) {
    uint32_t v = (uint32_t)bits;
    memcpy((unsigned char *)base + i * 4, &v, 4);
  } else {
    memcpy((unsigned char *)base + i * 8, &bits, 8);
  }
}

/* One element as the oracle carries it: key bits and its payload.  The input
 * index is kept so that stability can be stated and checked. */
typedef struct {
  uint64_t bits;
  uint64_t idx;
  uint32_t val;
} elem_t;

/* ---------------------------------------------------------------- O1 ---- */

/* Stable bottom-up merge sort of e[0..len) (any sequential sort is allowed by
 * Section 2.1; a stable one keeps key-value ties in input order). */
static int merge_sort_stable(int dtype, elem_t *e, uint64_t len) {
  if (len < 2) return ORACLE_OK;
  elem_t *tmp = (elem_t *)malloc(len * sizeof(elem_t));
  if (!tmp) return ORACLE_ERR_NOMEM;
  elem_t *src = e, *dst = tmp;
  for (uint64_t width = 1; width < len; width *= 2) {
    for (uint64_t lo = 0; lo < len; lo += 2 * width) {
      uint64_t mid = lo + width < len ? lo + width : len;
      uint64_t hi = lo + 2 * width < len ? lo + 2 * width : len;
      uint64_t i = lo, j = mid, o = lo;
      while (i < mid && j < hi) {
        /* take the left element on ties: stable */
        if (oracle_compare(dtype, src[i].bits, src[j].bits) <= 0) dst[o++] = src[i++];
        else dst[o++] = src[j++];
      }
      while (i < mid) dst[o++] = src[i++];
      while (j < hi) dst[o++] = src[j++];
    }
    elem_t *t = src; src = dst; dst = t;
  }
  if (src != e) memcpy(e, src, len * sizeof(elem_t));
  free(tmp);
  return ORACLE_OK;
}

/* Block b of N elements split into n_B blocks of length L = ceil(N/n_B):
 * [min(bL, N), min((b+1)L, N)).  Trailing blocks may be short or empty. */
static void block_range(uint64_t n, uint32_t n_b, uint32_t b, uint64_t *lo, uint64_t *hi) {
  uint64_t L = n / n_b + (n % n_b != 0);
  u128 l = (u128)L * b, h = (u128)L * (b + 1);
  *lo = l < n ? (uint64_t)l : n;
  *hi = h < n ? (uint64_t)h : n;
}

/* ---------------------------------------------------------- counting ---- */

/* In a sorted block: number of elements < v (lower bound) and <= v (upper
 * bound), each by binary search, as Section 2.3 describes the per-block count. */
static uint64_t count_less(int dtype, const elem_t *blk, uint64_t len, uint64_t v) {
  uint64_t lo = 0, hi = len;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (oracle_compare(dtype, blk[mid].bits, v) < 0) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

static uint64_t count_less_equal(int dtype, const elem_t *blk, uint64_t len, uint64_t v) {
  uint64_t lo = 0, hi = len;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (oracle_compare(dtype, blk[mid].bits, v) <= 0) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

/* |{x in A : x <= v}| summed over all sorted blocks. */
static uint64_t global_count_le(int dtype, elem_t *const *blk, const uint64_t *len,
                                uint32_t n_b, uint64_t v) {
  uint64_t s = 0;
  for (uint32_t b = 0; b < n_b; ++b) s += count_less_equal(dtype, blk[b], len[b], v);
  return s;
}

static uint64_t global_count_lt(int dtype, elem_t *const *blk, const uint64_t *len,
                                uint32_t n_b, uint64_t v) {
  uint64_t s = 0;
  for (uint32_t b = 0; b < n_b; ++b) s += count_less(dtype, blk[b], len[b], v);
  return s;
}

/* ---------------------------------------------------------------- O5 ---- */

/* Selection (tournament) tree over the heads of n_B runs (Section 2.2): the
 * leaves hold run ids, every internal node the winner of its two children;
 * the winner is the smaller head, ties going to the lower run id (stable).
 * Exhausted runs lose to everything. */
typedef struct {
  int dtype;
  uint32_t m;           /* number of leaves, a power of two >= number of runs */
  uint32_t *node;       /* node[1..2m): run id, or UINT32_MAX for "none"       */
  const elem_t *const *seg;
  const uint64_t *seg_len;
  uint64_t *pos;        /* next unread position in each run                  */
  uint32_t n_runs;
} seltree_t;

static int run_beats(const seltree_t *t, uint32_t a, uint32_t b) {
  if (a == UINT32_MAX) return 0;
  if (b == UINT32_MAX) return 1;
  int c = oracle_compare(t->dtype, t->seg[a][t->pos[a]].bits, t->seg[b][t->pos[b]].bits);
  if (c != 0) return c < 0;
  return a < b;
}

static uint32_t leaf_value(const seltree_t *t, uint32_t r) {
  if (r >= t->n_runs || t->pos[r] >= t->seg_len[r]) return UINT32_MAX;
  return r;
}

static void seltree_replay(seltree_t *t, uint32_t node) {
  for (node >>= 1; node >= 1; node >>= 1) {
    uint32_t l = t->node[2 * node], r = t->node[2 * node + 1];
    t->node[node] = run_beats(t, r, l) ? r : l;
  }
}

static int merge_selection_tree(int dtype, const elem_t *const *seg, const uint64_t *seg_len,
                                uint32_t n_runs, elem_t *out) {
  seltree_t t;
  t.dtype = dtype;
  t.m = 1;
  while (t.m < n_runs) t.m *= 2;
  t.node = (uint32_t *)malloc(2 * (size_t)t.m * sizeof(uint32_t));
  t.pos = (uint64_t *)calloc(n_runs ? n_runs : 1, sizeof(uint64_t));
  if (!t.node || !t.pos) { free(t.node); free(t.pos); return ORACLE_ERR_NOMEM; }
  t.seg = seg;
  t.seg_len = seg_len;
  t.n_runs = n_runs;
  for (uint32_t r = 0; r < t.m; ++r) t.node[t.m + r] = leaf_value(&t, r);
  for (uint32_t node = t.m - 1; node >= 1; --node) {
    uint32_t l = t.node[2 * node], r = t.node[2 * node + 1];
    t.node[node] = run_beats(&t, r, l) ? r : l;
  }
  uint64_t o = 0;
  while (t.node[1] != UINT32_MAX) {
    uint32_t w = t.node[1];
    out[o++] = seg[w][t.pos[w]];
    t.pos[w]++;
    t.node[t.m + w] = leaf_value(&t, w);
    seltree_replay(&t, t.m + w);
  }
  free(t.node);
  free(t.pos);
  return ORACLE_OK;
}

/* The same merge by a linear scan of all run heads per output element. */
static int merge_linear_heads(int dtype, const elem_t *const *seg, const uint64_t *seg_len,
                              uint32_t n_runs, elem_t *out) {
  uint64_t *pos = (uint64_t *)calloc(n_runs ? n_runs : 1, sizeof(uint64_t));
  if (!pos) return ORACLE_ERR_NOMEM;
  uint64_t o = 0;
  for (;;) {
    uint32_t best = UINT32_MAX;
    for (uint32_t r = 0; r < n_runs; ++r) {
      if (pos[r] >= seg_len[r]) continue;
      if (best == UINT32_MAX ||
          oracle_compare(dtype, seg[r][pos[r]].bits, seg[best][pos[best]].bits) < 0)
        best = r;
    }
    if (best == UINT32_MAX) break;
    out[o++] = seg[best][pos[best]++];
  }
  free(pos);
  return ORACLE_OK;
}

/* ------------------------------------------------------- the method ---- */

int oracle_pses(int dtype, uint64_t n, const void *keys, const uint32_t *vals,
                uint32_t n_b, uint32_t n_p, void *keys_out, uint32_t *vals_out,
                void *blocks_out, void *pivots, uint64_t *counts, uint64_t *split,
                uint64_t *offsets, int merge_kind) {
  const int kb = key_bytes(dtype);
  if (!kb || n_b == 0 || n_p == 0 || (n && (!keys || !keys_out))) return ORACLE_ERR_ARGS;
  if (vals && n && !vals_out) return ORACLE_ERR_ARGS;

  int rc = ORACLE_OK;
  elem_t *all = (elem_t *)malloc((n ? n : 1) * sizeof(elem_t));
  elem_t **blk = (elem_t **)malloc(n_b * sizeof(elem_t *));
  uint64_t *blen = (uint64_t *)malloc(n_b * sizeof(uint64_t));
  uint64_t *s = (uint64_t *)malloc((size_t)n_b * (n_p + 1) * sizeof(uint64_t));
  uint64_t *piv = (uint64_t *)calloc(n_p, sizeof(uint64_t));
  uint64_t *ck = (uint64_t *)calloc(n_p, sizeof(uint64_t));
  uint64_t *off = (uint64_t *)malloc((n_p + 1) * sizeof(uint64_t));
  const elem_t **seg = (const elem_t **)malloc(n_b * sizeof(elem_t *));
  uint64_t *seg_len = (uint64_t *)malloc(n_b * sizeof(uint64_t));
  elem_t *merged = (elem_t *)malloc((n ? n : 1) * sizeof(elem_t));
  if (!all || !blk || !blen || !s || !piv || !ck || !off || !seg || !seg_len || !merged) {
    rc = ORACLE_ERR_NOMEM;
    goto done;
  }

  /* O1: blocks, each copied and sorted on its own. */
  for (uint64_t i = 0; i < n; ++i) {
    all[i].bits = load_bits(keys, i, kb);
    all[i].idx = i;
    all[i].val = vals ? vals[i] : 0;
  }
  for (uint32_t b = 0; b < n_b; ++b) {
    uint64_t lo, hi;
    block_range(n, n_b, b, &lo, &hi);
    blk[b] = all + lo;
    blen[b] = hi - lo;
    rc = merge_sort_stable(dtype, blk[b], blen[b]);
    if (rc) goto done;
  }
  if (blocks_out)
    for (uint64_t i = 0; i < n; ++i) store_bits(blocks_out, i, kb, all[i].bits);

  /* O2: pivots.  r_k = floor(k N / n_P) stands for k N / n_P in Eq. 1 and
   * Eq. 2 (exact integer arithmetic; partition sizes then differ by <= 1).
   * P_k is found by a binary search inside each block for the first element
   * whose global count |{x <= element}| (a per-block binary search in every
   * block) reaches r_k; the smallest such element over all blocks is the
   * element of rank r_k - 1, which satisfies Eq. 1.  c_k follows from Eq. 2. */
  for (uint32_t k = 1; k < n_p; ++k) {
    const uint64_t r = (uint64_t)(((u128)k * n) / n_p);
    if (r == 0) { piv[k] = 0; ck[k] = 0; continue; }
    int have = 0;
    uint64_t best = 0;
    for (uint32_t b = 0; b < n_b; ++b) {
      uint64_t lo = 0, hi = blen[b];
      while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (global_count_le(dtype, blk, blen, n_b, blk[b][mid].bits) >= r) hi = mid;
        else lo = mid + 1;
      }
      if (lo < blen[b]) {
        uint64_t cand = blk[b][lo].bits;
        if (!have || oracle_compare(dtype, cand, best) < 0) best = cand;
        have = 1;
      }
    }
    if (!have) { rc = ORACLE_ERR_NO_PIVOT; goto done; }
    const uint64_t lt = global_count_lt(dtype, blk, blen, n_b, best);
    const uint64_t le = global_count_le(dtype, blk, blen, n_b, best);
    if (!(lt <= r && r <= le)) { rc = ORACLE_ERR_EQ1; goto done; }   /* Eq. 1 */
    piv[k] = best;
    ck[k] = r - lt;                                                   /* Eq. 2 */
    if (ck[k] < 1 || ck[k] > le - lt) { rc = ORACLE_ERR_CK; goto done; }
  }

  /* O3: partition boundaries in each sorted block.  All elements below P_k go
   * left of boundary k; of the elements equal to P_k, c_k go left, taken from
   * the lowest-numbered block first (Fig. 3b). */
  for (uint32_t b = 0; b < n_b; ++b) {
    s[(size_t)b * (n_p + 1) + 0] = 0;
    s[(size_t)b * (n_p + 1) + n_p] = blen[b];
  }
  for (uint32_t k = 1; k < n_p; ++k) {
    const uint64_t r = (uint64_t)(((u128)k * n) / n_p);
    uint64_t remaining = ck[k], total = 0;
    for (uint32_t b = 0; b < n_b; ++b) {
      uint64_t v;
      if (r == 0) {
        v = 0;
      } else {
        const uint64_t lt_b = count_less(dtype, blk[b], blen[b], piv[k]);
        const uint64_t eq_b = count_less_equal(dtype, blk[b], blen[b], piv[k]) - lt_b;
        const uint64_t take = eq_b < remaining ? eq_b : remaining;
        remaining -= take;
        v = lt_b + take;
      }
      s[(size_t)b * (n_p + 1) + k] = v;
      total += v;
    }
    if (total != r) { rc = ORACLE_ERR_SPLIT_SUM; goto done; }
  }
  for (uint32_t b = 0; b < n_b; ++b)
    for (uint32_t k = 0; k < n_p; ++k)
      if (s[(size_t)b * (n_p + 1) + k] > s[(size_t)b * (n_p + 1) + k + 1]) {
        rc = ORACLE_ERR_SPLIT_MONO;
        goto done;
      }

  /* O4: offsets of the merged partitions, one after another. */
  off[0] = 0;
  for (uint32_t k = 0; k < n_p; ++k) {
    uint64_t m = 0;
    for (uint32_t b = 0; b < n_b; ++b)
      m += s[(size_t)b * (n_p + 1) + k + 1] - s[(size_t)b * (n_p + 1) + k];
    const uint64_t fl = n / n_p, cl = fl + (n % n_p != 0);
    if (m != fl && m != cl) { rc = ORACLE_ERR_PART_SIZE; goto done; }
    off[k + 1] = off[k] + m;
  }
  for (uint32_t k = 0; k <= n_p; ++k)
    if (off[k] != (uint64_t)(((u128)k * n) / n_p)) { rc = ORACLE_ERR_OFFSET; goto done; }

  /* O5: merge partition k of every block into merged[O_k ...]. */
  for (uint32_t k = 0; k < n_p; ++k) {
    for (uint32_t b = 0; b < n_b; ++b) {
      const uint64_t a = s[(size_t)b * (n_p + 1) + k], e = s[(size_t)b * (n_p + 1) + k + 1];
      seg[b] = blk[b] + a;
      seg_len[b] = e - a;
    }
    rc = merge_kind == 1 ? merge_linear_heads(dtype, seg, seg_len, n_b, merged + off[k])
                         : merge_selection_tree(dtype, seg, seg_len, n_b, merged + off[k]);
    if (rc) goto done;
  }

  for (uint64_t i = 0; i < n; ++i) {
    store_bits(keys_out, i, kb, merged[i].bits);
    if (vals) vals_out[i] = merged[i].val;
  }
  if (pivots)
    for (uint32_t k = 1; k < n_p; ++k) store_bits(pivots, k - 1, kb, piv[k]);
  if (counts)
    for (uint32_t k = 1; k < n_p; ++k) counts[k - 1] = ck[k];
  if (split) memcpy(split, s, (size_t)n_b * (n_p + 1) * sizeof(uint64_t));
  if (offsets) memcpy(offsets, off, (n_p + 1) * sizeof(uint64_t));

done:
  free(all); free(blk); free(blen); free(s); free(piv); free(ck); free(off);
  free(seg); free(seg_len); free(merged);
  return rc;
}

void oracle_rank_counts(int dtype, uint64_t n, const void *keys, uint64_t v,
                        uint64_t *lt, uint64_t *le) {
  const int kb = key_bytes(dtype);
  uint64_t a = 0, b = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const int c = oracle_compare(dtype, load_bits(keys, i, kb), v);
    a += c < 0;
    b += c <= 0;
  }
  *lt = a;
  *le = b;
}

/* ------------------------------------------ PSRS pivots (Section 2.3) ---- */

/* The same four steps with the pivots of parallel sorting by regular sampling
 * (Section 2.3, first paragraph): n_P - 1 samples are taken at regular
 * intervals from every sorted block, all samples are sorted, n_P - 1 pivots
 * are taken at regular intervals from the sorted samples, and every block is
 * partitioned by value alone (partition k: P_k < x <= P_{k+1}, Section 2), so
 * partition sizes follow the data.  Regular intervals are read as the
 * positions floor(j len / n_P), j = 1..n_P-1, of a sorted sequence of length
 * len, both inside a block and in the sorted samples (P_k = S[floor(k |S| /
 * n_P)]); an empty block gives no samples. */
int oracle_psrs(int dtype, uint64_t n, const void *keys, const uint32_t *vals,
                uint32_t n_b, uint32_t n_p, void *keys_out, uint32_t *vals_out,
                void *blocks_out, void *samples_out, uint64_t *n_samples,
                void *pivots, uint64_t *split, uint64_t *offsets) {
  const int kb = key_bytes(dtype);
  if (!kb || n_b == 0 || n_p == 0 || (n && (!keys || !keys_out))) return ORACLE_ERR_ARGS;
  if (vals && n && !vals_out) return ORACLE_ERR_ARGS;

  int rc = ORACLE_OK;
  const uint64_t per = n_p - 1;
  elem_t *all = (elem_t *)malloc((n ? n : 1) * sizeof(elem_t));
  elem_t **blk = (elem_t **)malloc(n_b * sizeof(elem_t *));
  uint64_t *blen = (uint64_t *)malloc(n_b * sizeof(uint64_t));
  elem_t *smp = (elem_t *)malloc(((size_t)n_b * per + 1) * sizeof(elem_t));
  uint64_t *piv = (uint64_t *)calloc(n_p, sizeof(uint64_t));
  uint64_t *s = (uint64_t *)malloc((size_t)n_b * (n_p + 1) * sizeof(uint64_t));
  uint64_t *off = (uint64_t *)malloc((n_p + 1) * sizeof(uint64_t));
  const elem_t **seg = (const elem_t **)malloc(n_b * sizeof(elem_t *));
  uint64_t *seg_len = (uint64_t *)malloc(n_b * sizeof(uint64_t));
  elem_t *merged = (elem_t *)malloc((n ? n : 1) * sizeof(elem_t));
  uint64_t ns = 0;
  if (!all || !blk || !blen || !smp || !piv || !s || !off || !seg || !seg_len || !merged) {
    rc = ORACLE_ERR_NOMEM;
    goto done;
  }

  /* Step 1: blocks of ceil(N/n_B) elements, each sorted on its own. */
  for (uint64_t i = 0; i < n; ++i) {
    all[i].bits = load_bits(keys, i, kb);
    all[i].idx = i;
    all[i].val = vals ? vals[i] : 0;
  }
  for (uint32_t b = 0; b < n_b; ++b) {
    uint64_t lo, hi;
    block_range(n, n_b, b, &lo, &hi);
    blk[b] = all + lo;
    blen[b] = hi - lo;
    rc = merge_sort_stable(dtype, blk[b], blen[b]);
    if (rc) goto done;
  }
  if (blocks_out)
    for (uint64_t i = 0; i < n; ++i) store_bits(blocks_out, i, kb, all[i].bits);

  /* Step 2: regular samples of every non-empty block, sorted; pivots at
   * regular intervals of the sorted samples. */
  for (uint32_t b = 0; b < n_b; ++b) {
    if (blen[b] == 0) continue;
    for (uint64_t j = 1; j <= per; ++j) smp[ns++] = blk[b][(uint64_t)(((u128)j * blen[b]) / n_p)];
  }
  rc = merge_sort_stable(dtype, smp, ns);
  if (rc) goto done;
  for (uint32_t k = 1; k < n_p; ++k)
    piv[k] = ns ? smp[(uint64_t)(((u128)k * ns) / n_p)].bits : 0;

  /* Step 3: boundary k of block b after every element <= P_k. */
  for (uint32_t b = 0; b < n_b; ++b) {
    s[(size_t)b * (n_p + 1) + 0] = 0;
    s[(size_t)b * (n_p + 1) + n_p] = blen[b];
    for (uint32_t k = 1; k < n_p; ++k)
      s[(size_t)b * (n_p + 1) + k] = ns ? count_less_equal(dtype, blk[b], blen[b], piv[k]) : 0;
    for (uint32_t k = 0; k < n_p; ++k)
      if (s[(size_t)b * (n_p + 1) + k] > s[(size_t)b * (n_p + 1) + k + 1]) {
        rc = ORACLE_ERR_SPLIT_MONO;
        goto done;
      }
  }

  /* Offsets of the merged partitions, one after another; each boundary is the
   * number of elements <= P_k. */
  off[0] = 0;
  for (uint32_t k = 0; k < n_p; ++k) {
    uint64_t m = 0;
    for (uint32_t b = 0; b < n_b; ++b)
      m += s[(size_t)b * (n_p + 1) + k + 1] - s[(size_t)b * (n_p + 1) + k];
    off[k + 1] = off[k] + m;
  }
  for (uint32_t k = 1; k < n_p; ++k)
    if (ns && off[k] != global_count_le(dtype, blk, blen, n_b, piv[k])) {
      rc = ORACLE_ERR_SPLIT_SUM;
      goto done;
    }

  /* Step 4: merge partition k of every block into merged[O_k ...]. */
  for (uint32_t k = 0; k < n_p; ++k) {
    for (uint32_t b = 0; b < n_b; ++b) {
      const uint64_t a = s[(size_t)b * (n_p + 1) + k], e = s[(size_t)b * (n_p + 1) + k + 1];
      seg[b] = blk[b] + a;
      seg_len[b] = e - a;
    }
    rc = merge_selection_tree(dtype, seg, seg_len, n_b, merged + off[k]);
    if (rc) goto done;
  }

  for (uint64_t i = 0; i < n; ++i) {
    store_bits(keys_out, i, kb, merged[i].bits);
    if (vals) vals_out[i] = merged[i].val;
  }
  if (samples_out)
    for (uint64_t i = 0; i < ns; ++i) store_bits(samples_out, i, kb, smp[i].bits);
  if (n_samples) *n_samples = ns;
  if (pivots)
    for (uint32_t k = 1; k < n_p; ++k) store_bits(pivots, k - 1, kb, piv[k]);
  if (split) memcpy(split, s, (size_t)n_b * (n_p + 1) * sizeof(uint64_t));
  if (offsets) memcpy(offsets, off, (n_p + 1) * sizeof(uint64_t));

done:
  free(all); free(blk); free(blen); free(smp); free(piv); free(s); free(off);
  free(seg); free(seg_len); free(merged);
  return rc;
}

/* ------------------------------------- records sorted by a key field ---- */

/* Fixed-size records (Table 1: Pair, 16 bytes, and Particle, 96 bytes, each
 * sorted by a uint64 key): every record's key is read from key_offset, the
 * keys are sorted with their input index as payload by the four steps above
 * (stable: equal keys keep their input order), and the records are copied in
 * that order. */
int oracle_sort_records(int dtype, uint64_t n, const void *records, uint32_t record_bytes,
                        uint32_t key_offset, uint32_t n_b, uint32_t n_p, void *records_out) {
  const int kb = key_bytes(dtype);
  if (!kb || record_bytes == 0 || key_offset + (uint32_t)kb > record_bytes || n_b == 0 ||
      n_p == 0 || n > 0xffffffffull || (n && (!records || !records_out)))
    return ORACLE_ERR_ARGS;
  int rc = ORACLE_OK;
  unsigned char *keys = (unsigned char *)malloc((n ? n : 1) * (size_t)kb);
  unsigned char *keys_sorted = (unsigned char *)malloc((n ? n : 1) * (size_t)kb);
  uint32_t *idx = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
  uint32_t *perm = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
  if (!keys || !keys_sorted || !idx || !perm) {
    rc = ORACLE_ERR_NOMEM;
    goto done;
  }
  idx[0] = 0;
  for (uint64_t i = 0; i < n; ++i) {
    memcpy(keys + i * kb, (const unsigned char *)records + i * record_bytes + key_offset, kb);
    idx[i] = (uint32_t)i;
  }
  rc = oracle_pses(dtype, n, keys, idx, n_b, n_p, keys_sorted, perm, NULL, NULL, NULL, NULL,
                   NULL, 0);
  if (rc) goto done;
  /* the payload must come back as a permutation of 0..n-1 */
  memset(idx, 0, (n ? n : 1) * sizeof(uint32_t));
  for (uint64_t j = 0; j < n; ++j) {
    if (perm[j] >= n || idx[perm[j]]) {
      rc = ORACLE_ERR_PERM;
      goto done;
    }
    idx[perm[j]] = 1;
  }
  for (uint64_t j = 0; j < n; ++j)
    memcpy((unsigned char *)records_out + j * record_bytes,
           (const unsigned char *)records + (uint64_t)perm[j] * record_bytes, record_bytes);

done:
  free(keys); free(keys_sorted); free(idx); free(perm);
  return rc;
}
