/*
 * qumond_kernels.h -- single-grid entry points of the gfx950 kernels behind
 * qumond.h, for callers that drive the multigrid pieces themselves (and for
 * step-by-step comparisons).  Every array is a DEVICE pointer to an n^3 (or
 * nc^3) x-fastest grid of doubles as described in qumond.h; stream is a
 * hipStream_t (NULL = default).  All calls are asynchronous except
 * qumond_k_fmg, which synchronises for its stopping test.  Sizes are checked
 * before any HIP call (QUMOND_ERR_INVALID).  The method steps are those of
 * Sec. 2 of Angus et al. (arXiv:1201.3185).
 */
#ifndef QUMOND_KERNELS_H
#define QUMOND_KERNELS_H

#include <stdint.h>
#include "qumond.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One red-black Gauss-Seidel sweep for (sum of 6 neighbours - 6u)/h^2 = f:
 * colour (i+j+k) even first, then odd, each interior node set to
 * (sum of 6 neighbours - h^2 f)/6.  Reads u_in, writes the interior of u_out
 * (u_out's boundary nodes must already hold the Dirichlet values; u_in and
 * u_out must not alias). */
qumond_status qumond_k_rbgs_sweep(int32_t n, double h, const double *f, const double *u_in, double *u_out,
                                  void *stream);

/* The sweep of qumond_k_rbgs_sweep from a zero iterate with zero boundary
 * values, without an input array: writes the interior of u_out (n^3 doubles,
 * device; its boundary nodes must already hold zeros) -- bit for bit the
 * result of qumond_k_rbgs_sweep on a zero-filled u_in, with red nodes at
 * (0 - h^2 f)/6.  The first smoothing sweep of a correction V-cycle (Sec. 2's
 * multigrid, in this build's mixed-precision refinement).  Errors: n not
 * 2^J + 1 in 5..1025, h <= 0 or a NULL pointer -> QUMOND_ERR_INVALID. */
qumond_status qumond_k_rbgs_sweep_from_zero(int32_t n, double h, const double *f, double *u_out, void *stream);

/* Two sweeps in one launch (same result, bit for bit, as two calls of
 * qumond_k_rbgs_sweep).  uc (optional): a coarse grid of (n+1)/2 points per side
 * whose trilinear prolongation is added to u_in's interior first, as the
 * coarse-grid correction of a V-cycle (qumond_k_prolong_add) does.  u_in NULL
 * (with uc NULL): a zero iterate, read from nowhere, as in
 * qumond_k_rbgs_sweep_from_zero; u_out's boundary must then hold zeros. */
qumond_status qumond_k_rbgs_double_sweep(int32_t n, double h, const double *f, const double *u_in, double *u_out,
                                         const double *uc, void *stream);

/* Coarse rhs fc = full-weighting restriction of r = f - A_h u (27-point,
 * weights (1/4,1/2,1/4) per axis; 0 on the coarse boundary), and the coarse
 * correction zeroed: uc0 entirely, uc1 (optional) on its boundary nodes.
 * nf = 2 nc - 1. */
qumond_status qumond_k_residual_restrict(int32_t nf, double h, const double *f, const double *u, double *fc,
                                         double *uc0, double *uc1, void *stream);

/* One red-black sweep u_in -> u_out (as qumond_k_rbgs_sweep, u_in != u_out)
 * and the residual restriction of u_out (as qumond_k_residual_restrict) in one
 * launch: the last pre-smoothing sweep of a V-cycle and the coarse right-hand
 * side it produces (Sec. 2, the multigrid solves of Eq. 1 and Eq. 2).  Same
 * values as the two separate calls.  n = 2^J + 1 with 9 <= n <= 1025;
 * u_in, u_out, f: n^3 doubles; fc, uc0 (and uc1, optional): nc^3 doubles,
 * nc = (n + 1) / 2.  Errors: bad sizes or NULL arrays -> QUMOND_ERR_INVALID. */
qumond_status qumond_k_rbgs_sweep_restrict(int32_t n, double h, const double *f, const double *u_in, double *u_out,
                                           double *fc, double *uc0, double *uc1, void *stream);

/* dst = full-weighting restriction of src (interior of the coarse grid; 0 on
 * its boundary). */
qumond_status qumond_k_restrict(int32_t nf, const double *src, double *dst, void *stream);

/* Trilinear prolongation of the coarse correction added to the fine interior:
 * uf += P uc.  nf = 2 nc - 1. */
qumond_status qumond_k_prolong_add(int32_t nc, const double *uc, double *uf, void *stream);

/* FMG interpolation: fine interior set to P uc (boundary untouched). */
qumond_status qumond_k_interp(int32_t nc, const double *uc, double *uf, void *stream);

/* Eq. 2 face-flux source S from Phi_N (see qumond_mond_source). */
qumond_status qumond_k_mond_source(int32_t n, double h, double a0, const double *phin, double *S, void *stream);

/* Boundary nodes of a box of half the side from the coarser box's field
 * (trilinear; nodes of the inner box lie on coarse node planes or halfway). */
qumond_status qumond_k_bc_from_coarse(int32_t n, const double *uc, double *uf, void *stream);

/* out3[0] = sum over interior nodes of (f - A_h u)^2, out3[1] = sum of f^2,
 * out3[2] = sum of (sum of the node's boundary neighbours / h^2)^2, in a fixed
 * reduction order (bitwise reproducible). */
qumond_status qumond_k_resid_norms(int32_t n, double h, const double *f, const double *u, double *out3,
                                   void *stream);

/* qumond_k_resid_norms without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and bits as
 * qumond_k_resid_norms.  The partial sums live in a fixed 48 KiB workspace
 * that the library holds on each device for the life of the process (its
 * address is looked up on the first call on a device); it covers every
 * n = 2^J + 1 up to 1025, and a larger n returns QUMOND_ERR_INVALID.  All
 * calls on one device share that workspace: calls that overlap in time on
 * one device (on different streams, or from different threads) race and must
 * be serialised by the caller; calls in order on one stream are safe. */
qumond_status qumond_k_resid_norms_noalloc(int32_t n, double h, const double *f, const double *u, double *out3,
                                           void *stream);

/* FMG solve of one box in place on u (boundary = Dirichlet values), as
 * qumond_solve_newton does per box.  relres, extra (host, optional). */
qumond_status qumond_k_fmg(int32_t n, double L, const double *f, double *u, int32_t npre, int32_t npost,
                           int32_t ncycle, int32_t max_extra, double tol, double *relres, int32_t *extra,
                           void *stream);

/* ncyc V(npre,npost) cycles on the finest level from the given u. */
qumond_status qumond_k_vcycles(int32_t n, double L, const double *f, double *u, int32_t npre, int32_t npost,
                               int32_t ncyc, double *relres, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* QUMOND_KERNELS_H */
