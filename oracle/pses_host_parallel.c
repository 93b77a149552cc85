/*
 * pses_host_parallel.c -- TEST AND MEASUREMENT INFRASTRUCTURE ONLY.
 *
 * The host baseline of the benchmark: the oracle's own steps (pses_oracle.c,
 * included below so that every helper is the oracle's) run by T host
 * threads with OpenMP, in the paper's setting n_B = n_P = T (Section 3):
 *   step 1   one block per loop iteration (Section 2: blocks are sorted
 *            independently)
 *   step 2   one pivot per iteration (each P_k, c_k is found on its own)
 *   step 3   one pivot column of the split table per iteration
 *   offsets  sequentially, as Section 2 states
 *   step 4   one partition per iteration, merged by the oracle's selection
 *            tree into its own output range
 * Keys only.  The arithmetic is the oracle's; only the loops over blocks,
 * pivots and partitions are shared out among threads.  Never used by the
 * GPU library.
 */
#include "pses_oracle.c"

#include <omp.h>

int host_parallel_threads(void) { return omp_get_max_threads(); }

int host_parallel_pses(int dtype, uint64_t n, const void *keys, uint32_t n_b, uint32_t n_p,
                       void *keys_out) {
  const int kb = key_bytes(dtype);
  if (!kb || n_b == 0 || n_p == 0 || (n && (!keys || !keys_out))) return ORACLE_ERR_ARGS;
  int rc = ORACLE_OK;
  elem_t *all = (elem_t *)malloc((n ? n : 1) * sizeof(elem_t));
  elem_t **blk = (elem_t **)malloc(n_b * sizeof(elem_t *));
  uint64_t *blen = (uint64_t *)malloc(n_b * sizeof(uint64_t));
  uint64_t *s = (uint64_t *)malloc((size_t)n_b * (n_p + 1) * sizeof(uint64_t));
  uint64_t *piv = (uint64_t *)calloc(n_p, sizeof(uint64_t));
  uint64_t *ck = (uint64_t *)calloc(n_p, sizeof(uint64_t));
  uint64_t *off = (uint64_t *)malloc((n_p + 1) * sizeof(uint64_t));
  elem_t *merged = (elem_t *)malloc((n ? n : 1) * sizeof(elem_t));
  if (!all || !blk || !blen || !s || !piv || !ck || !off || !merged) {
    rc = ORACLE_ERR_NOMEM;
    goto done;
  }

#pragma omp parallel for schedule(static)
  for (uint64_t i = 0; i < n; ++i) {
    all[i].bits = load_bits(keys, i, kb);
    all[i].idx = i;
    all[i].val = 0;
  }
  /* step 1 */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc)
  for (uint32_t b = 0; b < n_b; ++b) {
    uint64_t lo, hi;
    block_range(n, n_b, b, &lo, &hi);
    blk[b] = all + lo;
    blen[b] = hi - lo;
    rc |= merge_sort_stable(dtype, blk[b], blen[b]);
  }
  if (rc) goto done;

  /* step 2: P_k and c_k exactly as the oracle finds them */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc)
  for (uint32_t k = 1; k < n_p; ++k) {
    const uint64_t r = (uint64_t)(((u128)k * n) / n_p);
    if (r == 0) continue;
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
    if (!have) { rc |= ORACLE_ERR_NO_PIVOT; continue; }
    const uint64_t lt = global_count_lt(dtype, blk, blen, n_b, best);
    const uint64_t le = global_count_le(dtype, blk, blen, n_b, best);
    if (!(lt <= r && r <= le)) { rc |= ORACLE_ERR_EQ1; continue; }
    piv[k] = best;
    ck[k] = r - lt;
  }
  if (rc) goto done;

  /* step 3: one pivot column per iteration, lowest block first among equals */
  for (uint32_t b = 0; b < n_b; ++b) {
    s[(size_t)b * (n_p + 1) + 0] = 0;
    s[(size_t)b * (n_p + 1) + n_p] = blen[b];
  }
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc)
  for (uint32_t k = 1; k < n_p; ++k) {
    const uint64_t r = (uint64_t)(((u128)k * n) / n_p);
    uint64_t remaining = ck[k], total = 0;
    for (uint32_t b = 0; b < n_b; ++b) {
      uint64_t v = 0;
      if (r != 0) {
        const uint64_t lt_b = count_less(dtype, blk[b], blen[b], piv[k]);
        const uint64_t eq_b = count_less_equal(dtype, blk[b], blen[b], piv[k]) - lt_b;
        const uint64_t take = eq_b < remaining ? eq_b : remaining;
        remaining -= take;
        v = lt_b + take;
      }
      s[(size_t)b * (n_p + 1) + k] = v;
      total += v;
    }
    if (total != r) rc |= ORACLE_ERR_SPLIT_SUM;
  }
  if (rc) goto done;

  /* offsets, sequentially */
  off[0] = 0;
  for (uint32_t k = 0; k < n_p; ++k) {
    uint64_t m = 0;
    for (uint32_t b = 0; b < n_b; ++b)
      m += s[(size_t)b * (n_p + 1) + k + 1] - s[(size_t)b * (n_p + 1) + k];
    off[k + 1] = off[k] + m;
  }
  if (off[n_p] != n) { rc = ORACLE_ERR_OFFSET; goto done; }

  /* step 4: one partition per iteration */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc)
  for (uint32_t k = 0; k < n_p; ++k) {
    const elem_t **seg = (const elem_t **)malloc(n_b * sizeof(elem_t *));
    uint64_t *seg_len = (uint64_t *)malloc(n_b * sizeof(uint64_t));
    if (!seg || !seg_len) {
      rc |= ORACLE_ERR_NOMEM;
    } else {
      for (uint32_t b = 0; b < n_b; ++b) {
        const uint64_t a = s[(size_t)b * (n_p + 1) + k], e = s[(size_t)b * (n_p + 1) + k + 1];
        seg[b] = blk[b] + a;
        seg_len[b] = e - a;
      }
      rc |= merge_selection_tree(dtype, seg, seg_len, n_b, merged + off[k]);
    }
    free(seg);
    free(seg_len);
  }
  if (rc) goto done;

#pragma omp parallel for schedule(static)
  for (uint64_t i = 0; i < n; ++i) store_bits(keys_out, i, kb, merged[i].bits);

done:
  free(all); free(blk); free(blen); free(s); free(piv); free(ck); free(off); free(merged);
  return rc;
}
