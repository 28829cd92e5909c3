/*
 * nf_test.h -- test hooks of libnf.so, outside the folding ABI of nf.h.
 * Host-only: none of these touches the GPU.
 */
#ifndef NF_TEST_H
#define NF_TEST_H

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
 * device gives the same items, in the same order and slots.  Returns 0 when
 * they hold, 1 with the first violation written to msg (cap bytes,
 * NUL-terminated), NF_E_INVAL for bad arguments. */
int nf_test_schedule(const int* NTs, int count, int target, char* msg, int cap);

#ifdef __cplusplus
}
#endif

#endif
