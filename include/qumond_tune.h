/*
 * qumond_tune.h -- launch-shape autotuning of the gfx950 smoother.
 *
 * The red-black smoother (the multigrid's dominant kernel, Sec. 2 of Angus et
 * al., arXiv:1201.3185) can be launched with several column-tile shapes and
 * z-march depths.  The library keeps one shape per level size (n = 2^J + 1)
 * and precision.  qumond_autotune times every candidate shape on synthetic
 * grids of each size from 33 up to n_max with hipEvents on the given stream
 * (median of `reps` launches after one warm-up), installs the fastest, and
 * optionally writes the table as JSON; qumond_tune_load installs a table a
 * previous run wrote.  Shapes change only speed, never results (every shape
 * computes the same red-black sweep).  Tuning allocates its own scratch grids
 * and synchronises the stream.
 */
#ifndef QUMOND_TUNE_H
#define QUMOND_TUNE_H

#include <stdint.h>
#include "qumond.h"

#ifdef __cplusplus
extern "C" {
#endif

/* variant: z-march over 0 = 32x8, 1 = 64x4, 2 = 64x8, 3 = 128x4, 4 = 32x16
 * columns per workgroup, 5 = 8^3 bricks held whole in LDS (small levels), or
 * z-march over 6 = 64x8, 7 = 64x16, 8 = 128x8 columns with one thread per
 * x-pair of nodes (half the threads per tile), 9 = 4^3, 10 = 6^3 bricks, or
 * 11 = 32x16, 12 = 32x8 pair columns, or 13 = 64x16, 14 = 128x8, 15 = 64x32
 * pair columns whose loads run two march steps ahead (plain sweeps; a sweep
 * that also applies the coarse-grid correction uses the pair kernel of the
 * same tile); all give identical results;
 * kchunk: z planes per workgroup (0 = all; ignored by bricks).  fp32 selects
 * the table of the single-precision smoother. */
qumond_status qumond_tune_set(int32_t n, int32_t fp32, int32_t variant, int32_t kchunk);
qumond_status qumond_tune_get(int32_t n, int32_t fp32, int32_t *variant, int32_t *kchunk);

/* Shape of the single sweep that also applies the coarse-grid correction
 * (the first post-smoothing sweep of a level when the correction is folded
 * into it), from the same variants and chunks as qumond_tune_set; variant -1
 * (the default) takes the level's plain-sweep shape.  The autotuner times
 * every shape with the correction applied; results are identical in every
 * shape.  Errors: n not 2^J + 1 in 5..1025, variant outside -1..15 or
 * kchunk < 0 -> QUMOND_ERR_INVALID. */
qumond_status qumond_tune_set_corr(int32_t n, int32_t fp32, int32_t variant, int32_t kchunk);
qumond_status qumond_tune_get_corr(int32_t n, int32_t fp32, int32_t *variant, int32_t *kchunk);

/* The same for the fused two-sweep smoother (variant 0 = 32x8, 1 = 64x4
 * z-march, 2 = 8^3, 3 = 4^3, 4 = 6^3 bricks, 5 = 64x16, 6 = 64x8, 7 = 32x16
 * z-march with one thread per pair of tile nodes and loads two steps
 * ahead, 8 = 64x16 and 9 = 32x8 whole-column marches with the four
 * half-sweeps skewed two planes apart, which apply the coarse-grid correction
 * in the same launch from coarse planes staged in LDS; 8 and 9 take no
 * z-chunk). */
qumond_status qumond_tune_set_fused(int32_t n, int32_t fp32, int32_t variant, int32_t kchunk);
qumond_status qumond_tune_get_fused(int32_t n, int32_t fp32, int32_t *variant, int32_t *kchunk);

/* Residual restriction kernel for a fine level of n points: variant 0 = one
 * thread per coarse node gathering its 27 fine residuals, 1 = LDS tile of the
 * fine block, 2, 3, 4 = z-march over chunks of 4, 8, 16 coarse planes forming
 * each fine residual once, 5 = 4x4x4, 6 = 4x4x2 coarse LDS tiles, 7, 8 = z-march
 * over the whole column of 32x8, 64x4 coarse columns (tiles from coarse column
 * 1, 512 threads, loads two steps ahead), 9 = 32x8 columns over 64-plane chunks,
 * 10, 11 = 32x8 whole columns loading three, four steps ahead (identical
 * results; the autotuner picks the fastest).  Errors: variant outside 0..11 ->
 * QUMOND_ERR_INVALID. */
qumond_status qumond_tune_set_rr(int32_t n, int32_t fp32, int32_t variant);
qumond_status qumond_tune_get_rr(int32_t n, int32_t fp32, int32_t *variant);

/* Coarse-grid correction of a level of n points (the u += P uc step of a
 * V-cycle before post-smoothing): split = 0 applies it inside the first
 * post-smoothing launch as each plane of u is loaded, split = 1 runs it as its
 * own prolong-add launch first (identical results; the autotuner times both in
 * the level's smoother form and keeps the faster).  Errors: n not 2^J + 1 in
 * 5..1025 or split outside {0, 1} -> QUMOND_ERR_INVALID. */
qumond_status qumond_tune_set_split(int32_t n, int32_t fp32, int32_t split);

/* Last pre-smoothing sweep of a level of n points and the residual restriction
 * that follows it (the u_l, f_{l-1} steps of a V-cycle): fused = 1 runs them as
 * one launch, each workgroup marching a whole z column and repeating its
 * neighbours' updates on a four-node ring so that it can form the residuals
 * at its edges; fused = 0 (default) as a sweep launch and a restriction launch
 * (identical results; the autotuner times both and keeps the faster).  Used
 * where the level sweeps one sweep per launch.  Errors: n not 2^J + 1 in
 * 5..1025 or fused outside {0, 1} -> QUMOND_ERR_INVALID. */
qumond_status qumond_tune_set_sweep_restrict(int32_t n, int32_t fp32, int32_t fused);
qumond_status qumond_tune_get_sweep_restrict(int32_t n, int32_t fp32, int32_t *fused);
qumond_status qumond_tune_get_split(int32_t n, int32_t fp32, int32_t *split);

/* One smoother sweep with an explicit shape (see qumond_k_rbgs_sweep); with
 * uc != NULL (device, ((n+1)/2)^3 doubles) the correction u += P uc is applied
 * to u_in's interior first, in the same launch.  u_in == NULL stands for a zero
 * iterate (boundary included), read from nowhere. */
qumond_status qumond_k_rbgs_sweep_shape(int32_t n, double h, const double *f, const double *u_in, double *u_out,
                                        int32_t variant, int32_t kchunk, const double *uc, void *stream);

/* One sweep of nb problems stored back to back (problem p's n^3 grid at
 * offset p n^3 of f, u_in and u_out, device doubles), all in one launch with
 * an explicit shape, as the batched runner sweeps a level of a size class.
 * u_in == NULL stands for a zero iterate of every problem.  Errors: n not
 * 2^J + 1 in 5..1025, nb outside 1..4096, h <= 0, a NULL f or u_out,
 * u_in == u_out, or a variant outside the table -> QUMOND_ERR_INVALID. */
qumond_status qumond_k_rbgs_sweep_stacked(int32_t n, int32_t nb, double h, const double *f, const double *u_in,
                                          double *u_out, int32_t variant, int32_t kchunk, void *stream);

/* Time all shapes of both smoother kernels for n = 33, 65, ..., n_max (and
 * both precisions if both != 0), install the fastest; json_path (host
 * string, optional) receives the table.  best_us (host, optional, 11 entries)
 * gets the FP64 time of one fused two-sweep launch indexed by log2(n-1).
 * For each size it also records whether the multigrid should use the fused
 * launch (faster than two single sweeps) or single sweeps, the fastest
 * residual-restriction kernel, and whether the coarse-grid correction runs as
 * its own launch (timed with two post-smoothing sweeps). */
qumond_status qumond_autotune(int32_t n_max, int32_t both, int32_t reps, const char *json_path, double *best_us,
                              void *stream);
qumond_status qumond_tune_load(const char *json_path);

#ifdef __cplusplus
}
#endif
#endif /* QUMOND_TUNE_H */
