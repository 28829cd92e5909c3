/*
 * nf_serial.h -- C ABI of libnf_serial.so: the paper's serial CPU algorithms
 * for the Nussinov table (Section 3), for running the paper's serial
 * comparisons (Section 6) on a host.  Host code only; it is not part of the
 * GPU library libnf.so, which never calls it.
 *
 * Variants (Section 3.1 and Section 3.2):
 *   NF_SERIAL_PLAIN       Eq. 1 cell by cell, every split point one by one
 *                         (the "Nussinov" column of the paper's tables).
 *   NF_SERIAL_TWO_VECTOR  Algorithm 1: R is built for every pair of vectors
 *                         before the fill; each q-group of split points of a
 *                         cell is one lookup (Eq. 3), the residual split
 *                         points at both ends one by one.
 *   NF_SERIAL_PARTIAL_MEMO  as two-vector, but the row of R for a horizontal
 *                         vector is built when that vector first appears in
 *                         the table (against every vertical vector).
 *   NF_SERIAL_FULL_MEMO   as two-vector, but each entry of R is built the
 *                         first time its pair of vectors meets in a lookup.
 *   NF_SERIAL_FG          Frid-Gusfield: for every finished row group, the
 *                         group's base plus the best prefix total against
 *                         every vertical vector is tabled for that group
 *                         (row, group, vector); a lookup reads it and adds
 *                         the column base.
 *
 * Fill order: column by column, each column bottom-up (Algorithm 1), when
 * threads = 1.  With threads > 1 (NF_SERIAL_PLAIN and NF_SERIAL_TWO_VECTOR
 * only) the cells of one anti-diagonal, which are independent (Section 4),
 * are shared among threads, diagonal after diagonal.  Every variant and order
 * fills the table of Eq. 1 exactly.
 *
 * Groups (Section 3.1): split point k of cell (i, j) pairs D(i, k-1) with
 * D(k, j); the k of group K are Kq+1 .. Kq+q (row cells D(i, Kq .. Kq+q-1),
 * column cells D(Kq+1 .. Kq+q, j)).  A group is looked up when all its k lie
 * in i+1 .. j; the rest are residual split points.
 *
 * Conventions as in nf.h: sequences of A, C, G, U (lower case accepted),
 * pairs A-U, U-A, C-G, G-C, 0 <= n <= NF_SERIAL_MAX_N, table layout
 * S_out[i*n + j] = D(i+1, j+1) for i <= j and 0 below (caller-owned, may be
 * NULL).  Returns D(1, n) >= 0, or NF_SERIAL_E_INVAL (bad argument or base),
 * NF_SERIAL_E_NOMEM (host memory).  Thread-safe: no state between calls.
 */
#ifndef NF_SERIAL_H
#define NF_SERIAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NF_SERIAL_MAX_N 65534
#define NF_SERIAL_Q_MAX 12
#define NF_SERIAL_E_INVAL (-1)
#define NF_SERIAL_E_NOMEM (-2)

enum {
    NF_SERIAL_PLAIN = 0,
    NF_SERIAL_TWO_VECTOR = 1,
    NF_SERIAL_PARTIAL_MEMO = 2,
    NF_SERIAL_FULL_MEMO = 3,
    NF_SERIAL_FG = 4
};

/* Work counted during one fold (exact counts, for checking and reporting):
 * lookups   Four-Russians steps (one per looked-up group of a cell);
 * splits    split points evaluated one by one (plain: all; else residual);
 * r_entries entries of R (or of the FG tables) computed, q-1 steps each;
 * vectors   row and column difference vectors stored. */
typedef struct {
    int64_t lookups, splits, r_entries, vectors;
} nf_serial_stats_t;

/* q in 1..NF_SERIAL_Q_MAX (ignored by NF_SERIAL_PLAIN); threads >= 1
 * (NF_SERIAL_E_INVAL above 1 for the memoized and FG variants); stats may be
 * NULL. */
int nf_serial_fold(const char* seq, int n, int q, int variant, int threads, int16_t* S_out,
                   nf_serial_stats_t* stats);

#ifdef __cplusplus
}
#endif
#endif /* NF_SERIAL_H */
