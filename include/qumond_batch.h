/* Batched QUMOND solves of many independent single-box disks (the ensembles of
 * a rotation-curve fit, Sec. 3.4-3.5 of Angus et al.: every parameter set
 * (distance, mass-to-light ratio, stellar and gas scale heights) is one disk,
 * and each needs the Sec. 2 pipeline and its Eq. 4 circular speeds).
 *
 * Each problem is one box of side box_side centred on the origin with n_p
 * points per side (n_p = 2^J + 1; problems may differ in n_p), outer Dirichlet
 * values from the monopole of the problem's total mass, and the pipeline
 *   deposit -> Newtonian solve -> Eq. 2 source -> QUMOND solve -> Eq. 4 curve,
 * solved in mixed precision: an FP32 FMG (ncycle_fmg V-cycles per level)
 * seeds the FP64 iterate, then refine_iters FP64 residual-correction steps,
 * each one FP32 V-cycle on the residual scaled by its RMS, the 3^3 solve in
 * FP64 (the scheme of QUMOND_MIXED in qumond.h, with a fixed step count).
 *
 * Problems of the same n_p form a class whose grids lie back to back in HBM,
 * so every kernel launch covers the whole class; the classes run on streams
 * of their own.  The whole batch is one captured hipGraph: per-problem inputs
 * (particle pointers, counts, masses) live in device memory that the kernels
 * read, so new inputs do not need a new capture.  After the graph, the host
 * reads every problem's residual history (a tail check) and gives problems
 * above tol_rel extra refinement steps eagerly; a problem whose Newtonian
 * solve needed them has its source, QUMOND solve and curve redone.
 *
 * Results are bit-identical to the single-problem context of qumond.h
 * (one box, QUMOND_MIXED, the same ncycle_fmg, max_vcycles = refine_iters and
 * a tolerance that no residual meets), since both run the same kernels with
 * the same arithmetic.
 *
 * Pointers are device pointers unless marked host.  Calls return a status;
 * qumond_last_error() (qumond.h) gives the message.  A batch is not
 * thread-safe; distinct batches are independent.
 */
#ifndef QUMOND_BATCH_H
#define QUMOND_BATCH_H

#include <stdint.h>

#include "qumond.h"

#ifdef __cplusplus
extern "C" {
#endif

#define QUMOND_BATCH_MAX 1024

typedef struct qumond_batch qumond_batch;

typedef struct {
    int32_t nprob;        /* problems, 1..QUMOND_BATCH_MAX */
    double box_side;      /* kpc, the same for every problem */
    double G, a0;         /* as in qumond_config */
    int32_t npre, npost;  /* smoothing sweeps, default 2, 2 */
    int32_t ncycle_fmg;   /* FP32 FMG V-cycles per level, default 2 */
    int32_t refine_iters; /* FP64 refinement steps inside the graph, default 4 */
    int32_t max_extra;    /* tail: extra steps per solve at most, default 20 */
    double tol_rel;       /* tail target ||f - A u||_2 / ||f||_2, default 1e-6 */
    double gather_frac;   /* box choice of Eq. 4 points, default 0.2 (as qumond_config) */
    int32_t naz;          /* azimuths per radius of the curve, default 16 */
    int32_t autotune;     /* 1: time smoother shapes on the batch's own grids at the first run */
    double nu_n;          /* interpolating function, as qumond_config.nu_n (default 1: Eq. 2's nu) */
} qumond_batch_config;

typedef struct {
    double relres_newton;   /* relative residual after the Newtonian solve (tail included) */
    double relres_mond;     /* ... after the QUMOND solve */
    int32_t steps_newton;   /* refinement steps used (graph + tail) */
    int32_t steps_mond;
    int32_t converged;      /* both residuals <= tol_rel */
    int32_t redone;         /* 1 if the QUMOND part was redone after a Newtonian tail */
    int64_t n_inside;       /* particles deposited (inside the box) */
} qumond_batch_problem_info;

void qumond_batch_default_config(qumond_batch_config *cfg);

/* Checks the config, n_per_problem[nprob] (host; each 2^J + 1 with 17 <= n <= 1025)
 * and the radii (host R[nR], 0 < nR <= 4096, each finite and >= 0) without any
 * HIP call: QUMOND_ERR_INVALID on failure. */
qumond_status qumond_batch_validate(const qumond_batch_config *cfg, const int32_t *n_per_problem, const double *R,
                                    int32_t nR);

/* Allocates every grid (HBM use: about 48 bytes per grid point plus 4 MB
 * per problem of deposit scratch) on the current device; calls are enqueued on
 * `stream` (hipStream_t, NULL = default stream). */
qumond_status qumond_batch_create(const qumond_batch_config *cfg, const int32_t *n_per_problem, const double *R,
                                  int32_t nR, void *stream, qumond_batch **out);
qumond_status qumond_batch_destroy(qumond_batch *b);

/* Particles of problem p: device arrays of np doubles (SoA, kpc and Msun),
 * caller-owned, which must stay valid and unchanged until the run that reads
 * them has returned; total_mass (Msun, > 0) sets the outer values and the
 * deposit's fixed-point scale as in qumond_deposit.  Every problem needs
 * particles before the first run. */
qumond_status qumond_batch_set_particles(qumond_batch *b, int32_t p, const double *x, const double *y,
                                         const double *z, const double *m, int64_t np, double total_mass);

/* Runs the batch: with use_graph = 1 it replays the captured graph (capturing
 * it on first use), with 0 it enqueues the same launches directly; then the
 * tail check.  Synchronises the stream.  info: host array [nprob] or NULL.
 * QUMOND_ERR_NOT_CONVERGED if a problem stays above tol_rel after max_extra
 * steps (results kept, info filled). */
qumond_status qumond_batch_run(qumond_batch *b, int32_t use_graph, qumond_batch_problem_info *info);

/* vc2[p * nR + r] = v_c^2 (km/s)^2 of problem p at radius R[r] (Eq. 4, from the
 * QUMOND potential with mond = 1, from the Newtonian one with mond = 0):
 * device array of nprob * nR doubles.  Valid after a run. */
qumond_status qumond_batch_rotation_curves(qumond_batch *b, int32_t mond, double *vc2);

/* Copy of one field of problem p (QUMOND_FIELD_RHS, _PHI_N, _SOURCE, _PHI of
 * qumond.h) into dst, n_p^3 doubles, x fastest. */
qumond_status qumond_batch_get_field(qumond_batch *b, int32_t p, int32_t field, double *dst);

/* JSON text (host buffer of cap bytes) describing the classes: n, problems,
 * smoother shapes, graph nodes and the timings of the last autotune. */
qumond_status qumond_batch_describe(qumond_batch *b, char *buf, int64_t cap);

/* Device bytes held by the batch. */
int64_t qumond_batch_device_bytes(const qumond_batch *b);

#ifdef __cplusplus
}
#endif

#endif
