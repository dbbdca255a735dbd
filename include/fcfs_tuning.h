/*
 * fcfs_tuning.h -- tuning and profiling hooks of the FCFS library (see
 * fcfs.h for the transform, the conventions and the error codes).  They serve
 * the autotuner, the tests that compare tile variants, and benchmarks; an
 * application needs none of them.
 */
#ifndef FCFS_TUNING_H_
#define FCFS_TUNING_H_

#include "fcfs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Batch autotuner.  The batch takes its contraction tile variant and corners
 * per work item per K bucket of a clip (bucket of max(K, L): 0 up to 63, 1 up
 * to 127, 2 up to 255, 3 up to 511, 4 above; clips whose buckets share a
 * variant share one persistent launch).  fcfs_autotune_batch builds and times
 * a plan of the clips c[0..n) for each candidate (variant, corners per item),
 * first alike for every bucket, then, when the clips span several buckets,
 * per bucket on that bucket's clips; the per-bucket choices are kept only if
 * the whole batch runs faster with them, and a candidate replaces the
 * built-in choice only when more than 3% faster.  The choices hold on h for
 * later fcfs_batch_workspace_size / fcfs_forward_batch calls of precision p.
 * Overwrites the clips' outputs.  effort 0..2 sets the timed repetitions
 * (2, 3, 5).  Allocates and frees a workspace per candidate and synchronises
 * the handle's stream.  fcfs_batch_choice reports the current choice of K
 * bucket kbucket (0..FCFS_BATCH_KBUCKETS-1). */
#define FCFS_BATCH_KBUCKETS 5
fcfs_status fcfs_autotune_batch(fcfs_handle *h, const fcfs_clip *c, int32_t n, fcfs_precision p,
                                int effort);
fcfs_status fcfs_batch_choice(fcfs_handle *h, fcfs_precision p, int32_t kbucket, int32_t *tile,
                              int64_t *chunk);

/* Contraction tile variants.  fcfs_tile_variants fills wk[i], wl[i]
 * (frequencies per wave in k and l of variant i, for i < cap) and returns the
 * number of variants.  fcfs_set_tile forces variant `variant` on every later
 * call of this handle (-1 restores the automatic choice).
 * fcfs_workspace_size_tile is fcfs_workspace_size (forward) for a given
 * variant. */
int32_t fcfs_tile_variants(int32_t *wk, int32_t *wl, int32_t cap);
fcfs_status fcfs_set_tile(fcfs_handle *h, int32_t variant);
fcfs_status fcfs_workspace_size_tile(const fcfs_clip *c, fcfs_precision p, int32_t tile,
                                     size_t *bytes);

/* Per-kernel timing with hipEvents on the stream each kernel runs on.  After
 * fcfs_profile_begin every launch of a kind whose bit is set in `kinds` (0:
 * every kind) is bracketed by two events; fcfs_profile_end waits for them and
 * writes, for kind i < nkinds, the summed milliseconds ms[i] and the launch
 * count count[i], then stops recording.  Kinds: 0 pre-pass, 1 side-stream
 * work (histograms, guard region, axis DFTs), 2 contraction, 3 epilogue,
 * 4 adjoint kernels, 5 batched graph, 6 lattice form, 7 Haar quadtree walk
 * (the Haar transform's clear-and-plan launches count as pre-pass, its
 * scaling pass as epilogue), 8 pupil loss, 9 direct form of small problems,
 * 10 replay of a captured optimisation step, 11 the adjoint's main-term GEMM
 * alone (also counted in kind 4).  Each bracketed launch adds two event
 * records to its stream. */
fcfs_status fcfs_profile_begin(fcfs_handle *h, uint32_t kinds);
fcfs_status fcfs_profile_end(fcfs_handle *h, double *ms, int64_t *count, int32_t nkinds);

#ifdef __cplusplus
}
#endif

#endif /* FCFS_TUNING_H_ */
