/*
 * pses_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, deliberately slow CPU reference of parallel samplesort
 * with exact splitting (PSES), and of its regular-sampling variant (PSRS),
 * Tokuue & Ishiyama, "Performance Evaluation of
 * Parallel Sortings on the Supercomputer Fugaku" (arXiv 2305.05245).
 * It exists so that tests, the smoke check and the benchmark's CPU-baseline leg
 * can check the GPU library against an independent implementation.  The GPU
 * product path never includes, links or calls anything in this directory.
 *
 * Key-type codes are this file's own (they happen to use the same numbering as
 * the public library so tests can pass one integer to both):
 *   0 uint32, 1 int32, 2 uint64, 3 int64, 4 float32, 5 float64.
 * Floats are ordered by IEEE 754-2019 totalOrder, written out from its
 * definition on raw bits (no floating-point compare anywhere).
 */
#ifndef PSES_ORACLE_H
#define PSES_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORACLE_OK = 0,
  ORACLE_ERR_ARGS = 1,
  ORACLE_ERR_NOMEM = 2,
  /* invariant violations (never expected; each names the check that failed) */
  ORACLE_ERR_EQ1 = 10,        /* Eq. 1 does not hold for the pivot found        */
  ORACLE_ERR_CK = 11,         /* c_k outside [1, |{x = P_k}|]                   */
  ORACLE_ERR_SPLIT_SUM = 12,  /* sum_b s[b][k] != r_k                           */
  ORACLE_ERR_SPLIT_MONO = 13, /* s[b][k] > s[b][k+1]                            */
  ORACLE_ERR_OFFSET = 14,     /* O_k != r_k                                     */
  ORACLE_ERR_PART_SIZE = 15,  /* |partition k| not floor or ceil of N/n_P       */
  ORACLE_ERR_NO_PIVOT = 16,   /* r_k > 0 but no block produced a candidate      */
  ORACLE_ERR_PERM = 17        /* sorted indices are not a permutation of 0..n-1 */
};

/* Step O0: three-way comparison of two keys of the given type, given as raw
 * bits (zero-extended to 64 bits for 4-byte types).  Returns -1, 0 or +1. */
int oracle_compare(int dtype, uint64_t a_bits, uint64_t b_bits);

/*
 * The whole method, steps 1-4 of the paper's four-step parallel samplesort
 * (Section 2), with PSES pivot selection (Section 2.3, Eq. 1 and Eq. 2).
 *
 *   dtype, n, keys      input keys (n elements of 4 or 8 bytes), never written
 *   vals                optional uint32 payload (NULL = keys only); ties in the
 *                       output are broken by input index (stable)
 *   n_blocks, n_parts   n_B >= 1 and n_P >= 1
 *   keys_out, vals_out  sorted output (n elements); vals_out only if vals
 *   blocks_out          optional: concatenation of the sorted blocks (step 1)
 *   pivots              optional: n_P-1 keys, canonical P_k (the value of the
 *                       element of rank r_k - 1); 0 when r_k = 0
 *   counts              optional: n_P-1 values c_k of Eq. 2 (0 when r_k = 0)
 *   split               optional: n_B*(n_P+1) values, row-major [b][k]:
 *                       partition k of block b is [split[b][k], split[b][k+1])
 *   offsets             optional: n_P+1 values, O_k (O_{n_P} = n)
 *   merge_kind          0 = selection tree (Knuth), 1 = linear scan of the run
 *                       heads (cross-check of the former on small inputs)
 * Returns ORACLE_OK or an ORACLE_ERR_* code.
 */
int oracle_pses(int dtype, uint64_t n, const void *keys, const uint32_t *vals,
                uint32_t n_blocks, uint32_t n_parts, void *keys_out,
                uint32_t *vals_out, void *blocks_out, void *pivots,
                uint64_t *counts, uint64_t *split, uint64_t *offsets,
                int merge_kind);

/*
 * The same four steps with the pivots of parallel sorting by regular sampling
 * (PSRS, Section 2.3, first paragraph): n_P - 1 samples from every non-empty
 * sorted block at positions floor(j len_b / n_P) (j = 1..n_P-1), the samples
 * sorted, P_k = S[floor(k |S| / n_P)], and every block cut by value alone
 * (partition k holds P_k < x <= P_{k+1}), so the sizes follow the data.
 *
 *   samples_out         optional: the sorted samples S (up to n_B*(n_P-1)
 *                       keys; their number is written to *n_samples)
 *   pivots              optional: n_P-1 keys P_k (0 when there are no samples)
 *   split, offsets      as for oracle_pses; offsets[k] = |{x <= P_k}|
 * Other arguments as for oracle_pses (the merge is the selection tree).
 */
int oracle_psrs(int dtype, uint64_t n, const void *keys, const uint32_t *vals,
                uint32_t n_blocks, uint32_t n_parts, void *keys_out,
                uint32_t *vals_out, void *blocks_out, void *samples_out,
                uint64_t *n_samples, void *pivots, uint64_t *split,
                uint64_t *offsets);

/*
 * Fixed-size records (Table 1's Pair and Particle) sorted by the key of type
 * dtype at byte offset key_offset of each record_bytes-byte record: the keys
 * with their input index go through oracle_pses (n_blocks, n_parts), and the
 * records are copied in the resulting stable order.  n < 2^32.
 */
int oracle_sort_records(int dtype, uint64_t n, const void *records, uint32_t record_bytes,
                        uint32_t key_offset, uint32_t n_blocks, uint32_t n_parts,
                        void *records_out);

/* Plain counts |{x in keys : x < v}| and |{x in keys : x <= v}| by one linear
 * pass: the definition used by Eq. 1, for checks at sizes where the full
 * oracle would be too slow. */
void oracle_rank_counts(int dtype, uint64_t n, const void *keys, uint64_t v_bits,
                        uint64_t *lt, uint64_t *le);

#ifdef __cplusplus
}
#endif
#endif
