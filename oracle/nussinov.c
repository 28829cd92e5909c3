/*
 * Plain CPU oracle for the Nussinov base-pair maximisation table.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  The GPU product
 * path never calls it and shares no code with it.
 *
 * What it computes (Section 2, Eq. 1): for a sequence S_1..S_n over A,C,G,U,
 *     D(i, i-1) = D(i, i) = 0
 *     D(i, j)   = max{ b(S_i, S_j) + D(i+1, j-1),
 *                      max_{i+1 <= k <= j} D(i, k-1) + D(k, j) }      (i < j)
 * with b = 1 for the complementary pairs A-U, U-A, C-G, G-C and 0 otherwise
 * (G-U is not a pair).  The optimum is D(1, n).
 *
 * The table is filled along diagonals d = j - i = 1, 2, ..., n-1, one of the
 * fill orders Section 2 names.  Cells of one diagonal depend only on shorter
 * diagonals, so they are computed by independent OpenMP threads (the
 * observation Section 4 starts from).  A transposed copy Dt(j, k) = D(k, j) is
 * kept so that the split loop reads both operands contiguously; it holds the
 * same numbers as D.
 *
 * Output layout: out[(i-1)*n + (j-1)] = D(i, j) for i <= j, 0 for i > j.
 * Return value: D(1, n) >= 0, or -1 for a character outside A,C,G,U (either
 * case), or -2 for n < 0, or -3 if memory could not be obtained.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int upper(char c) { return (c >= 'a' && c <= 'z') ? c - 'a' + 'A' : c; }

/* b(x, y) of Eq. 1: Watson-Crick complementary bases. */
static int complementary(char x, char y)
{
    x = (char)upper(x);
    y = (char)upper(y);
    return (x == 'A' && y == 'U') || (x == 'U' && y == 'A') ||
           (x == 'C' && y == 'G') || (x == 'G' && y == 'C');
}

static int valid_base(char c)
{
    c = (char)upper(c);
    return c == 'A' || c == 'C' || c == 'G' || c == 'U';
}

/* nthreads <= 0 keeps the OpenMP default. */
long long nfo_fold(const char* seq, int n, int32_t* out, int nthreads)
{
    if (n < 0) return -2;
    for (int i = 0; i < n; ++i)
        if (!valid_base(seq[i])) return -1;
    if (out) memset(out, 0, (size_t)n * (size_t)n * sizeof(int32_t));
    if (n <= 1) return 0;

    /* 1-based indices 1..n plus the sentinel row n+1 / column 0. */
    const size_t ld = (size_t)n + 2;
    int32_t* D = (int32_t*)calloc(ld * ld, sizeof(int32_t));
    int32_t* Dt = (int32_t*)calloc(ld * ld, sizeof(int32_t));
    if (!D || !Dt) { free(D); free(Dt); return -3; }
    const char* S = seq - 1; /* S[1..n] */

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

    for (int d = 1; d < n; ++d) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 1; i <= n - d; ++i) {
            const int j = i + d;
            /* pairing term: b(S_i, S_j) + D(i+1, j-1); D(i+1, i) = 0 when d = 1 */
            int32_t best = complementary(S[i], S[j]) + D[(size_t)(i + 1) * ld + (size_t)(j - 1)];
            /* splitting term: max over i+1 <= k <= j of D(i, k-1) + D(k, j) */
            const int32_t* row = D + (size_t)i * ld;   /* row[k-1] = D(i, k-1) */
            const int32_t* col = Dt + (size_t)j * ld;  /* col[k]   = D(k, j)   */
            for (int k = i + 1; k <= j; ++k) {
                const int32_t v = row[k - 1] + col[k];
                best = v > best ? v : best;
            }
            D[(size_t)i * ld + (size_t)j] = best;
            Dt[(size_t)j * ld + (size_t)i] = best;
        }
    }

    const long long score = D[1 * ld + (size_t)n];
    if (out) {
        for (int i = 1; i <= n; ++i)
            for (int j = i; j <= n; ++j)
                out[(size_t)(i - 1) * (size_t)n + (size_t)(j - 1)] = D[(size_t)i * ld + (size_t)j];
    }
    free(D);
    free(Dt);
    return score;
}

/* Number of OpenMP threads a parallel region would use (for reporting). */
int nfo_max_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) return nthreads;
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}
