/*
 * nf_test.h -- test hooks of libnf.so, outside the folding ABI of nf.h.
 * nf_test_schedule and nf_test_set_perturb are host-only;
 * nf_test_packed_state runs a fold on the GPU.
 */
#ifndef NF_TEST_H
#define NF_TEST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* nf_test_schedule
 * Build the wavefront schedule (Section 4: tiles of one anti-diagonal are
 * independent) for `count` folds of NTs[f] >= 1 tiles per side with at most
 * about `target` between-group chunks per step, and check its invariants:
 * every tile finished once at the stage of its diagonal, after the main
 * diagonal; the between-group work of tile (A, B) covering each group tile C,
 * A+1 < C < B-1, exactly once in the stage before its finish, in one
 * accumulator slot (combined atomically when split) that the finish then
 * reads; no two tiles of a stage sharing a slot; slot halves alternating by
 * stage.  For a single fold (count = 1) it also checks that the closed form
 * of the schedule that the allocation-free entry point evaluates on the
 * device gives the same items, in the same order and slots.  Under a
 * perturbation seed (nf_test_set_perturb) the schedule is shuffled as plans
 * shuffle theirs before it is checked, and the closed form is not compared
 * (its order is the unperturbed one).  Returns 0 when
 * they hold, 1 with the first violation written to msg (cap bytes,
 * NUL-terminated), NF_E_INVAL for bad arguments. */
int nf_test_schedule(const int* NTs, int count, int target, char* msg, int cap);

/* nf_test_set_perturb
 * Race detection by schedule perturbation.  With seed != 0, every plan made
 * afterwards (single folds and batches; not the serving engine) runs the
 * items of each wavefront step, and the main-diagonal tiles, in an order
 * shuffled from the seed (so other workgroups, CUs and XCDs take them), and
 * its staged steps put a delay of 0 to about 17 us, drawn per step from the
 * seed, before the finish launch and before the between launch, so that the
 * finishes of one diagonal and the between chunks of the next overlap
 * differently.  Section 4's independence of a diagonal's tiles means no
 * result may change.  seed = 0 turns it off.  Plans are cached per seed;
 * nf_shutdown drops them.  Returns NF_OK. */
int nf_test_set_perturb(unsigned seed);

/* nf_test_packed_state
 * Fold seq[0..n) as nf_fold does (q in 1..9, explicit; n >= 2) and copy out
 * the fold's packed state: the row blocks to rs_out and the column blocks to
 * cs_out, tile_count(NT) * (64 / q) * 64 words each, numbered and laid out as
 * the kernels keep them.  Tiles are diagonal-major, tile (A, A+d) at
 * d*NT - d(d-1)/2 + A; a tile's block is [group k][64 rows or columns]; the
 * row word of row a and group k of tile (A, B) holds the base F(a, BT+kq) in
 * bits 15..0 and, above it, h << (q-1) with bit p-1 of h the difference
 * F(a, BT+kq+p) - F(a, BT+kq+p-1) (Lemma 1: 0 or 1), p = 1..q-1; the column
 * word of column b holds F(AT+kq, b) in bits 15..0 and in bits 31..16 c, bit
 * p-1 of c = F(AT+kq+p-1, b) - F(AT+kq+p, b).  Here F(a, b) = D(a+1, b) over
 * posts 0..NT*T-1, T = (64/q)*q, with the sequence padded by 'A' to
 * NT*T - 1 bases; rows and columns >= T are zero words.  The blocks of
 * main-diagonal tiles (d = 0) are not kept and not copied (left as the
 * caller had them).  *nt_out (if not NULL) receives NT.  Returns the score,
 * or NF_E_INVAL when cap_words is below the block size (with *nt_out set),
 * or another NF_E_* code. */
int nf_test_packed_state(const char* seq, int n, int q, uint32_t* rs_out, uint32_t* cs_out, size_t cap_words,
                         int* nt_out);

#ifdef __cplusplus
}
#endif

#endif
