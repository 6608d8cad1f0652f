/*
 * qumond.h -- C ABI of the MI355X (gfx950) particle-mesh QUMOND solver.
 *
 * The calls follow the problem statement of Angus et al., "A QUMOND galactic
 * N-body code I: Poisson solver and rotation curve fitting" (arXiv:1201.3185),
 * Sec. 2, which lists the four per-cell quantities of the method:
 *   step 1  baryonic density on the grid by cloud-in-cell     -> qumond_deposit
 *   step 2  Newtonian potential, Eq. 1, by full multigrid     -> qumond_solve_newton
 *   step 3  the right-hand side of Eq. 2, div[nu grad Phi_N]  -> qumond_mond_source
 *   step 4  QUMOND potential, Eq. 2, by the same multigrid     -> qumond_solve_mond
 * followed by finite-difference gravity interpolated back to points with the
 * same cloud-in-cell kernel                                   -> qumond_gather_forces
 * and the circular speed of Eq. 4                             -> qumond_rotation_curve.
 *
 * Units: kpc, solar masses, km/s (potential in (km/s)^2, acceleration in
 * (km/s)^2/kpc).  Defaults: G = 4.300917270e-6 kpc (km/s)^2 / Msun and
 * a0 = 3.6 (km/s)^2/pc = 3600 (km/s)^2/kpc (Eq. 2).
 *
 * Grids.  Every box is a cube of side L centred on the origin holding n^3
 * vertex-centred nodes, n = 2^J + 1 (Sec. 2: 65, 129 or 257 points per side,
 * coarsened down to a 3^3 grid).  Node (i,j,k) sits at
 * (-L/2 + i h, -L/2 + j h, -L/2 + k h), h = L/(n-1), and every n^3 array
 * crossing this ABI is x-fastest: element i + n (j + n k).  Nested boxes
 * (Sec. 2, nested refinement) are given outermost first, each exactly half
 * the side of the previous one, all with the same n.
 *
 * Memory.  Every array pointer is a DEVICE pointer (for example a torch
 * tensor's data_ptr()) owned by the caller, unless marked "host".  The
 * library owns every grid it allocates inside a context.  All work is
 * enqueued on the HIP stream given to qumond_create; calls that return data
 * to the host (the solves, for their stopping test, and n_outside) synchronise
 * that stream, every other call is asynchronous.
 *
 * Errors.  Every call returns a status code; nothing aborts or throws across
 * the ABI.  Configuration and argument checks run before any HIP call, so
 * they behave identically on a machine without a GPU.  HIP failures map to
 * QUMOND_ERR_HIP; qumond_last_error() gives the text of the last failure in
 * the calling thread.  A context is not thread-safe; distinct contexts are
 * independent.
 */
#ifndef QUMOND_H
#define QUMOND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QUMOND_MAX_BOX 16

typedef enum {
    QUMOND_OK = 0,
    QUMOND_ERR_INVALID = 1,        /* bad configuration or argument */
    QUMOND_ERR_STATE = 2,          /* call out of the deposit->newton->source->mond order */
    QUMOND_ERR_OOM = 3,            /* device allocation failed */
    QUMOND_ERR_HIP = 4,            /* a HIP runtime call failed */
    QUMOND_ERR_NOT_CONVERGED = 5,  /* tolerance not met within max_vcycles; fields hold the last iterate */
    QUMOND_ERR_RANGE = 6           /* value out of the representable range (e.g. fixed-point overflow) */
} qumond_status;

/* QUMOND_MIXED: each solve starts from an FP32 FMG (FP32 smoothing,
 * restriction and prolongation; the 3^3 solve in FP64) and then repeats FP64
 * residual correction: r = f - A u in FP64, scaled by its RMS s, one FP32
 * V-cycle for A e = r/s with zero boundary values, u += s e in FP64, until the
 * FP64 relative residual meets tol_rel (max_vcycles refinements at most).
 * The Eq. 2 source stays FP64. */
typedef enum { QUMOND_FP64 = 0, QUMOND_MIXED = 1 } qumond_precision;
typedef enum { QUMOND_BC_ZERO = 0, QUMOND_BC_MONOPOLE = 1 } qumond_outer_bc;

typedef enum {
    QUMOND_FIELD_RHO_FIXED = 0,  /* int64 fixed-point mass per node, q = rint(w m 2^s) summed */
    QUMOND_FIELD_RHS = 1,        /* double, 4 pi G rho (Eq. 1 right-hand side) */
    QUMOND_FIELD_PHI_N = 2,      /* double, Newtonian potential (step 2) */
    QUMOND_FIELD_SOURCE = 3,     /* double, div[nu grad Phi_N] (step 3) */
    QUMOND_FIELD_PHI = 4         /* double, QUMOND potential (step 4) */
} qumond_field;

typedef enum { QUMOND_GUESS_NONE = 0, QUMOND_GUESS_F64 = 1, QUMOND_GUESS_F32 = 2, QUMOND_GUESS_BF16 = 3 } qumond_guess_kind;
/* Field choice ("which") of qumond_gather_forces, qumond_rotation_curve and
 * qumond_sigma_z. */
enum {
    QUMOND_WHICH_NEWTON = 0,     /* -grad Phi_N (Eq. 1) */
    QUMOND_WHICH_QUMOND = 1,     /* -grad Phi (Eq. 2) */
    QUMOND_WHICH_ALGEBRAIC = 2   /* Eq. 3: nu(|g_N| / a0) g_N at the point, g_N from Phi_N */
};

/* OR-ed into guess_kind: never fall back to FMG (for measuring plain V-cycles
 * from a given start); the solve then stops after ncycle_fmg + max_vcycles
 * cycles at the latest. */
#define QUMOND_GUESS_NO_FALLBACK 16

typedef struct qumond_config {
    int32_t n;                          /* points per side, 2^J + 1, 5 <= n <= 1025 */
    int32_t nbox;                       /* number of nested boxes, 1..16 */
    double box_side[QUMOND_MAX_BOX];    /* kpc, outermost first, box_side[b] = box_side[b-1] / 2 */
    double G;                           /* gravitational constant, > 0 */
    double a0;                          /* MOND acceleration constant, >= 0 (0 gives nu = 1) */
    int32_t npre, npost;                /* RB-GS sweeps before/after the coarse-grid correction, 0..8, sum >= 1 */
    int32_t ncycle_fmg;                 /* V-cycles per FMG level, 1..64 (the paper uses 6) */
    int32_t max_vcycles;                /* extra finest-level V-cycles allowed after FMG, 0..10000 */
    double tol_rel;                     /* stop when ||f - A u||_2 / ||f||_2 <= tol_rel; 0 = fixed schedule */
    int32_t precision;                  /* qumond_precision */
    int32_t outer_bc;                   /* qumond_outer_bc, Dirichlet value on the outermost box */
    double gather_frac;                 /* box choice: finest box with R, |z| < gather_frac * L_b, in (0, 0.5) */
    int32_t fixed_shift;                /* deposit scale exponent s (q = rint(w m 2^s)); 0 = from total mass */
    int32_t use_graphs;                 /* 1: FP64 solves without a guess replay the FMG schedule and each
                                           extra finest V-cycle (with its residual norms) from HIP graphs
                                           captured on first use per box and chain (on a context created with
                                           a non-NULL stream); results are identical */
    double nu_n;                        /* interpolating function (Sec. 2 allows other forms of nu): 1 = Eq. 2's
                                           nu(y) = 1/2 + 1/2 sqrt(1 + 4/y) (default); otherwise, 1 < nu_n <= 10,
                                           the n-family nu_n(y) = [(1 + sqrt(1 + 4 y^-n)) / 2]^(1/n) (2: the
                                           "standard" nu), used by the Eq. 2 source, the QUMOND monopole
                                           boundary and force, and Eq. 3 */
} qumond_config;

typedef struct qumond_solve_info {
    int32_t nbox;
    int32_t vcycles[QUMOND_MAX_BOX];    /* finest-level V-cycles run after the FMG schedule (or from the guess) */
    int32_t converged[QUMOND_MAX_BOX];  /* 1 if relres <= tol_rel (or fixed schedule) */
    int32_t refine_iters[QUMOND_MAX_BOX]; /* mixed precision: FP64 refinement iterations */
    double relres0[QUMOND_MAX_BOX];     /* relative residual after FMG (or of the guess) */
    double relres[QUMOND_MAX_BOX];      /* final relative residual */
    int32_t used_fallback;              /* 1 if a supplied guess was rejected and FMG from zero was run */
} qumond_solve_info;

typedef struct qumond_ctx qumond_ctx;

/* Fill *cfg with the paper's defaults for a single box of side 100 kpc and
 * n = 65: 2+2 sweeps and 6 V-cycles per FMG level (Sec. 2, Sec. 3.2),
 * monopole outer boundary, tol_rel 1e-10, gather_frac 0.2 (Sec. 3.1), Eq. 2's
 * nu (nu_n = 1). */
void qumond_default_config(qumond_config *cfg);

/* Check a configuration without touching the GPU.  Returns QUMOND_OK or
 * QUMOND_ERR_INVALID with the reason in qumond_last_error(). */
qumond_status qumond_validate_config(const qumond_config *cfg);

/* Validate cfg, allocate every grid of every box and bind the context to
 * hip_stream (a hipStream_t; NULL = the default stream) on the current
 * device.  *out is NULL on failure. */
qumond_status qumond_create(const qumond_config *cfg, void *hip_stream, qumond_ctx **out);
qumond_status qumond_destroy(qumond_ctx *ctx);

/* Step 1 (Sec. 2): cloud-in-cell assignment of np particles (x, y, z, m:
 * device arrays of doubles) into every box that contains them.  A particle is
 * in box b iff 0 <= u_d < n-1 on all axes, u_d = (x_d + L_b/2) (n-1)/L_b; its
 * 8 corner weights are products of 1-f_d or f_d (f_d the fractional part of
 * u_d) and each corner receives rint(w m 2^s) in a 64-bit integer grid, so the
 * result is independent of particle order.  s = 62 - ceil(log2 total_mass) - 1
 * unless fixed_shift is set.  Then rhs = 4 pi G q 2^-s / h^3.  total_mass is
 * the mass of all particles (also those outside every box): it sets the
 * monopole boundary value.  n_outside (host, optional; synchronises) receives
 * the number of particles outside the outermost box.  np = 0 is valid. */
qumond_status qumond_deposit(qumond_ctx *ctx, const double *x, const double *y, const double *z,
                             const double *m, int64_t np, double total_mass, int64_t *n_outside);

/* Step 2 (Eq. 1, Sec. 2): full-multigrid solve of A_h Phi_N = rhs box by box,
 * outermost first.  The outer box takes the configured Dirichlet value (zero,
 * or the Newtonian monopole -G M / r of total_mass); every inner box takes its
 * boundary by trilinear interpolation of the next coarser box's converged
 * Phi_N.  FMG: rhs restricted by full weighting to 3^3, boundary values
 * injected, exact 3^3 solve, trilinear interpolation level by level with
 * ncycle_fmg V(npre,npost) cycles of red-black Gauss-Seidel ((i+j+k) even
 * first) on each, then extra finest-level cycles until
 * ||rhs - A_h Phi_N||_2 / ||rhs||_2 <= tol_rel over the interior (a box with
 * no source is measured against the norm of its boundary-value contribution,
 * sum of boundary neighbours / h^2).  info (host,
 * optional) receives cycle counts and residuals.  Synchronises the stream.
 * Returns QUMOND_ERR_NOT_CONVERGED if any box missed tol_rel. */
qumond_status qumond_solve_newton(qumond_ctx *ctx, qumond_solve_info *info);

/* Step 3 (Eq. 2): S = div[nu(|grad Phi_N|/a0) grad Phi_N] on every box by a
 * conservative face-flux difference: on the face between nodes p and p+e_d the
 * normal gradient is (Phi_N(p+e_d) - Phi_N(p))/h, the two transverse ones the
 * average of the central differences on both sides, the flux
 * nu(|g|/a0) g_normal with nu(y) = 1/2 + 1/2 sqrt(1 + 4/y) (0 where |g| = 0),
 * and S(p) = sum_d (F(p+e_d/2) - F(p-e_d/2)) / h at interior nodes.  FP64. */
qumond_status qumond_mond_source(qumond_ctx *ctx);

/* Step 4 (Eq. 2): the same multigrid solve A_h Phi = S, outer box from the
 * configured Dirichlet value (zero, or the QUMOND monopole of total_mass),
 * inner boxes from the next coarser box's converged Phi.  guess (device,
 * optional): nbox * n^3 values of type guess_kind, box after box, whose
 * interior seeds the finest level instead of FMG, followed by V-cycles (with
 * QUMOND_MIXED: FP64 refinement steps, each one FP32 V-cycle, as after the
 * FP32 FMG); the guess is rejected in favour of FMG from zero
 * (info->used_fallback = 1) when it is not finite, when the relative
 * residual after its first cycle exceeds 1, or when it needs more than
 * ncycle_fmg + max_vcycles cycles.  Synchronises. */
qumond_status qumond_solve_mond(qumond_ctx *ctx, const void *guess, int32_t guess_kind, qumond_solve_info *info);

/* Steps 2-4 in one call with the two chains overlapped: the Newtonian solve
 * of box b+1 runs concurrently with the source and QUMOND solve of box b (the
 * QUMOND chain needs only box b's Phi_N and its own coarser box).  The
 * Newtonian chain runs on the context's stream, the QUMOND chain on a second
 * stream of default priority that the context creates on first use, driven by
 * a worker thread.  Results equal qumond_solve_newton + qumond_mond_source +
 * qumond_solve_mond bit for bit; on return the context's stream is ordered
 * after all of it.  Either info (host) may be NULL.  Synchronises. */
qumond_status qumond_solve(qumond_ctx *ctx, qumond_solve_info *info_newton, qumond_solve_info *info_mond);

/* Accelerations at np points: -grad Phi_N (which = QUMOND_WHICH_NEWTON),
 * -grad Phi (QUMOND_WHICH_QUMOND) or the algebraic MOND field of Eq. 3
 * (QUMOND_WHICH_ALGEBRAIC: the Newtonian acceleration g_N at the point times
 * nu(|g_N| / a0), the relation Sec. 1 compares QUMOND with).  Gravity
 * at nodes by central differences (one-sided second order on box faces),
 * weighted to the point with the cloud-in-cell weights.  Box choice (Sec. 3.1):
 * the finest box with sqrt(x^2+y^2) < gather_frac L_b and |z| < gather_frac L_b;
 * otherwise the outermost box that contains the point; otherwise the monopole
 * of total_mass (Newtonian, or QUMOND with nu(g_N/a0) for the other two).
 * box_used (device, optional) receives the box index, 255 for the monopole.
 * QUMOND_ERR_STATE before the solve the field needs. */
qumond_status qumond_gather_forces(qumond_ctx *ctx, const double *x, const double *y, const double *z,
                                   int64_t np, int32_t which, double *ax, double *ay, double *az,
                                   uint8_t *box_used);

/* Eq. 4: v_c^2(R) = R dPhi/dR at z = 0, averaged over naz azimuths
 * phi_k = 2 pi k / naz, for the nR radii R (device) into vc2 (device).
 * which as for qumond_gather_forces (QUMOND_WHICH_ALGEBRAIC gives the
 * algebraic MOND curve of Eq. 3).  1 <= naz <= 1024. */
qumond_status qumond_rotation_curve(qumond_ctx *ctx, const double *R, int32_t nR, int32_t naz, int32_t which,
                                    double *vc2);

/* Eq. 5 (Sec. 5), the vertical velocity dispersion of an isothermal stellar
 * disk, sigma_z^2 = -(dPhi/dz) rho_* / (d rho_* / dz), for stars whose density
 * falls off as sech^2(z / z0) at every radius (the vertical profile of the
 * disk models, scale height z0 > 0), so rho_* / (d rho_* / dz) =
 * -z0 / (2 tanh(z / z0)) and sigma_z^2 = -a_z z0 / (2 tanh(z / z0)).  a_z is
 * the gathered vertical acceleration of field `which` (as for
 * qumond_gather_forces) at height z > 0 (kpc) above and below the plane;
 * sig2[r] (device, (km/s)^2) is the mean over the 2 naz points
 * (R[r] cos phi_k, R[r] sin phi_k, +-z), phi_k = 2 pi k / naz, 1 <= naz <= 1024.
 * R (device) holds nR >= 0 radii.  Asynchronous on the context's stream. */
qumond_status qumond_sigma_z(qumond_ctx *ctx, const double *R, int32_t nR, int32_t naz, double z, double z0,
                             int32_t which, double *sig2);

/* Copy one n^3 field of box b to dst (device; int64 for RHO_FIXED, double
 * otherwise).  Asynchronous. */
qumond_status qumond_get_field(qumond_ctx *ctx, int32_t box, int32_t field, void *dst);

/* Overwrite one n^3 field of box b from src (device) and move the call-order
 * state to the step that produces it (RHS: after deposit; PHI_N: after the
 * Newtonian solve; SOURCE: after the source; PHI: after the QUMOND solve).
 * Lets a caller run any step on inputs it supplies.  Asynchronous. */
qumond_status qumond_set_field(qumond_ctx *ctx, int32_t box, int32_t field, const void *src);

/* Timing of the red-black smoother, the solve's dominant kernel: when
 * enabled, every smoother launch of the context's FP64 solves is bracketed by
 * two hipEvents on the stream it runs on.  on = 0 disables, on = 1 records
 * every level, on = n (2^J + 1 >= 5) records only the plain launches on
 * levels of n points per side (n = the box's n: the finest level), leaving out
 * the sweeps that also apply the coarse-grid correction as they load u, and of
 * the plain launches only the kind the level smooths pairs of sweeps with: the
 * two-sweep launches where its launch table fuses pairs, single sweeps
 * otherwise; any other value returns QUMOND_ERR_INVALID.  The first sweep of a
 * correction from a zero iterate is not recorded.  qumond_profile_read
 * synchronises, returns the number of launches, their summed duration, their
 * summed algorithmic traffic (read u, read f, write u: 3 values per node of
 * the level, per launch of one or two sweeps) and the sweeps per launch, and
 * clears the record. */
typedef struct qumond_kernel_stats {
    int64_t launches;
    double total_ms;
    double alg_bytes;
    int32_t sweeps_per_launch; /* 2 where the profiled level runs its sweeps in pairs, else 1 (0: none timed) */
} qumond_kernel_stats;
qumond_status qumond_profile_enable(qumond_ctx *ctx, int32_t on);
qumond_status qumond_profile_read(qumond_ctx *ctx, qumond_kernel_stats *out);

/* Device bytes held by the context. */
int64_t qumond_device_bytes(const qumond_ctx *ctx);

const char *qumond_status_string(qumond_status s);
const char *qumond_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QUMOND_H */
