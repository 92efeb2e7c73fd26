/*
 * jk_tune.h -- plan autotuning of the J/K engine (jk.h).
 *
 * A build's plan has choices that do not change what is computed, only how
 * fast: the tile shape of the FP64 half-transform and the Q-chunk budget
 * (slabs per launch, hence launch count, workspace use and exchange
 * splits).  jk_autotune times the candidate plans of one problem on the
 * device and records the fastest for the problem's shape class; jk_build,
 * jk_fock, jk_laplace_build and jk_build_batched then use the recorded plan
 * for every problem of that class.  The table lives in the process and can
 * be saved to and loaded from JSON.
 *
 * Shape class: (ceil(nao / 64), ceil(ndens * rank / 64), precision, packed).
 *
 * Results: every plan computes the same J and K to rounding; with a fixed
 * table, results are bit-identical run to run.  A tile-shape choice alone
 * leaves the results bit-identical; a chunk choice changes the summation
 * order of K (and the half-transforms' inner products are unchanged).
 * Workspace: every candidate fits the workspace jk_workspace_bytes reports
 * (chunks up to 4 GiB; the derivative's chunks take 4 GiB as well).
 */
#ifndef JK_GFX950_TUNE_H
#define JK_GFX950_TUNE_H

#include "jk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t ht_tile;    /* FP64 half-transform tile.  On the 4x4x4 matrix instruction:
                           0 = 128 x 64 of four 64 x 32 wave tiles, 1 = 64 x 64, 2 = 128 x 64
                           of eight 64 x 16 wave tiles.  On the 16x16x4 instruction, over
                           the chunk's slabs stacked as one matrix: 3 = 128 x 128, 4 =
                           128 x 64.  Packed B and JK_MIXED use their own kernels;
                           jk_build_batched runs 2 as 0 and 3 as 4 */
    int32_t chunk_mb;   /* Q-chunk budget in MiB, 64 .. 4096 (jk_build_batched caps its
                           members at 256)                                             */
} jk_tuning;

/* Times every candidate plan for problem *p (each: one untimed build, then
 * `reps` timed builds bracketed by HIP events on the stream; reps 0 means 2),
 * records the fastest for p's shape class and writes it to *chosen (may be
 * NULL).  Arguments and workspace as jk_build; J and K end with the result of
 * one more build under the chosen plan.  Synchronizes the stream.  Not for
 * use under stream capture. */
jk_status jk_autotune(const jk_problem *p, const double *B, const double *CL, const double *CR,
                      double *J, double *K, void *ws, size_t ws_bytes, void *stream,
                      int32_t reps, jk_tuning *chosen);

/* The plan jk_build would use for *p: the recorded one, or the default
 * {4, 1024}.  Returns JK_EINVAL for an invalid problem. */
jk_status jk_tuning_get(const jk_problem *p, jk_tuning *t);

/* Records *t for p's shape class (JK_EINVAL if a field is out of range). */
jk_status jk_tuning_set(const jk_problem *p, const jk_tuning *t);

/* What a plan does with problem *p (host only, enqueues nothing).  With
 * t == NULL the plan jk_build would use (jk_tuning_get), else the plan *t. */
typedef struct {
    int32_t chunk_slabs;    /* slabs per Q-chunk                                         */
    int32_t nsplit;         /* exchange splits of a chunk, general densities             */
    int32_t nsplit_sym;     /* exchange splits of a chunk, C_L = C_R                     */
    int32_t int_depth;      /* JK_MIXED: the most inner indices any int32 slice-level
                               sum of the build takes (half-transform: the padded nao;
                               exchange: one split of a chunk's slab-rank index); 0 for
                               JK_FP64                                                    */
    int32_t int_depth_cap;  /* JK_MIXED: the depth up to which those sums are exact,
                               32767 (4 digit pairs of at most 2^14 per index stay
                               below 2^31); 0 for JK_FP64.  Every plan keeps
                               int_depth <= int_depth_cap by splitting the exchange.   */
    int32_t reserved;
} jk_plan_info;

/* Fills *out for problem *p under plan t (or the current plan).  Returns
 * JK_EINVAL for an invalid problem, plan or NULL out. */
jk_status jk_plan_describe(const jk_problem *p, const jk_tuning *t, jk_plan_info *out);

/* Forgets every recorded plan. */
void jk_tuning_clear(void);

/* Writes the table as JSON into buf (NUL-terminated when cap allows) and
 * returns the number of bytes the full text needs, NUL included; buf may be
 * NULL with cap 0 to query the size. */
size_t jk_tuning_save(char *buf, size_t cap);

/* Merges the entries of a JSON text written by jk_tuning_save.  Returns
 * JK_EINVAL (and records nothing) if the text does not parse or a value is
 * out of range. */
jk_status jk_tuning_load(const char *json);

#ifdef __cplusplus
}
#endif

#endif
