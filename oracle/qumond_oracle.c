/*
 * Plain, slow, single-threaded FP64 CPU oracle for the particle-mesh QUMOND
 * solve of Angus et al., "A QUMOND galactic N-body code I: Poisson solver and
 * rotation curve fitting" (arXiv:1201.3185).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent judge of the HIP
 * library: it shares no code, header, table or constant generator with it,
 * and only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  The product path never calls into it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no FMA
 * contraction, so the CIC weights are the same IEEE products the paper's
 * recipe defines).
 *
 * Threads.  One thread unless orc_set_threads says otherwise.  Only loops
 * whose iterations write distinct nodes and read nothing another iteration
 * writes are split over threads (a colour pass of red-black Gauss-Seidel,
 * the residual, restriction, prolongation, interpolation, the Eq. 2 source
 * and the per-point gather), so every result is the same bit for bit at any
 * thread count; the deposit and every sum stay serial in their fixed order.
 *
 * What each routine follows:
 *   cic_*            Sec. 2, "cloud-in-cell technique" for the density (step 1),
 *                    in a 64-bit fixed-point form so a second implementation
 *                    can be compared bit for bit.
 *   rbgs/residual/restrict/prolong/interp/vcycle/fmg
 *                    Sec. 2, the full multigrid method of Numerical Recipes
 *                    extended to 3D with red-black Gauss-Seidel, V-cycles,
 *                    2 pre- and 2 post-smoothing sweeps, trilinear transfer,
 *                    and the FMG bootstrap from a 3x3x3 grid whose single
 *                    interior node is solved exactly.
 *   bc_*             Sec. 2, nested refinement: the outermost box carries a
 *                    Dirichlet value (zero, or a monopole), each inner box
 *                    takes its boundary by interpolating the coarser box.
 *   mond_source      Eq. 2: the right-hand side div[nu(|grad Phi_N|/a0) grad Phi_N]
 *                    by a conservative face-flux difference, nu from Eq. 2.
 *   gather           Sec. 2: finite-difference gravity on the grid, CIC
 *                    interpolation to a point, and the per-radius box choice
 *                    of Sec. 3.1.
 *
 * Grids are vertex-centred, n = 2^J + 1 nodes per side, node (i,j,k) of a box
 * of side L centred on the origin sits at (-L/2 + i h, -L/2 + j h, -L/2 + k h)
 * with h = L/(n-1); arrays are x-fastest: index i + n (j + n k).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ID3(n, i, j, k) ((size_t)(i) + (size_t)(n) * ((size_t)(j) + (size_t)(n) * (size_t)(k)))

/* Threads of the node-parallel loops (see the header note). */
static int orc_threads = 1;
void orc_set_threads(int t) { orc_threads = t < 1 ? 1 : t; }
int orc_get_threads(void) { return orc_threads; }
#define ORC_PAR _Pragma("omp parallel for num_threads(orc_threads) schedule(static)")

/* ------------------------------------------------------------------ nu */

/* Eq. 2: nu(y) = 1/2 + 1/2 sqrt(1 + 4/y), y = |grad Phi_N| / a0. */
double orc_nu(double y) { return 0.5 + 0.5 * sqrt(1.0 + 4.0 / y); }

/* Other forms of nu (Sec. 2 notes that nu could take another form): the
 * n-family nu_n(y) = [(1 + sqrt(1 + 4 y^-n)) / 2]^(1/n), whose n = 1 member
 * is Eq. 2's nu (evaluated by orc_nu) and n = 2 the "standard" function. */
double orc_nu_n(double y, double nn)
{
    if (nn == 1.0) return orc_nu(y);
    return pow(0.5 * (1.0 + sqrt(1.0 + 4.0 * pow(y, -nn))), 1.0 / nn);
}

/* --------------------------------------------------------------- deposit */

/* Fixed-point scale exponent s such that the integer grid can hold the total
 * mass times 2^s with a bit to spare: s = 62 - ceil(log2(M)) - 1. */
int orc_fixed_shift(double total_mass)
{
    int e;
    double mant = frexp(total_mass, &e); /* M = mant * 2^e, mant in [0.5, 1) */
    int ceil_log2 = (mant == 0.5) ? e - 1 : e;
    return 62 - ceil_log2 - 1;
}

/* Sec. 2 step 1: cloud-in-cell mass assignment into one box.  A particle is
 * assigned iff 0 <= u_d < n-1 on all three axes, u_d = (x_d + L/2) (n-1)/L;
 * its 8 corner weights are products of (1 - f_d) or f_d with f_d the
 * fractional part of u_d, and each corner receives rint(w m 2^s) (round half
 * to even) in a 64-bit integer grid.  Returns the number of assigned
 * particles. */
int64_t orc_cic_deposit(int n, double L, int64_t np, const double *x, const double *y,
                        const double *z, const double *m, int shift, int64_t *q)
{
    const double xmin = -0.5 * L;
    const double inv_h = (double)(n - 1) / L;
    const double scale = ldexp(1.0, shift);
    int64_t inside = 0;
    for (int64_t p = 0; p < np; p++) {
        double u[3];
        u[0] = (x[p] - xmin) * inv_h;
        u[1] = (y[p] - xmin) * inv_h;
        u[2] = (z[p] - xmin) * inv_h;
        int ok = 1;
        for (int d = 0; d < 3; d++)
            if (!(u[d] >= 0.0 && u[d] < (double)(n - 1))) ok = 0;
        if (!ok) continue;
        inside++;
        int ic[3];
        double w[3][2];
        for (int d = 0; d < 3; d++) {
            double fl = floor(u[d]);
            ic[d] = (int)fl;
            double fr = u[d] - fl;
            w[d][0] = 1.0 - fr;
            w[d][1] = fr;
        }
        for (int c = 0; c < 2; c++)
            for (int b = 0; b < 2; b++)
                for (int a = 0; a < 2; a++) {
                    double wt = (w[0][a] * w[1][b]) * w[2][c];
                    long long qv = llrint((wt * m[p]) * scale);
                    q[ID3(n, ic[0] + a, ic[1] + b, ic[2] + c)] += (int64_t)qv;
                }
    }
    return inside;
}

/* Eq. 1 right-hand side from the fixed-point mass grid:
 * rho = q 2^-s / h^3, f = 4 pi G rho. */
void orc_rhs_from_q(int n, double L, double G, int shift, const int64_t *q, double *f)
{
    const double h = L / (double)(n - 1);
    const double h3 = h * h * h;
    const double four_pi_G = 4.0 * M_PI * G;
    const size_t N = (size_t)n * n * n;
    for (size_t t = 0; t < N; t++) {
        double rho = ldexp((double)q[t], -shift) / h3;
        f[t] = four_pi_G * rho;
    }
}

/* --------------------------------------------------- boundary conditions */

static int on_boundary(int n, int i, int j, int k)
{
    return i == 0 || j == 0 || k == 0 || i == n - 1 || j == n - 1 || k == n - 1;
}

/* Newtonian potential of a point mass M at the origin. */
double orc_phi_point_newton(double r, double G, double M) { return -G * M / r; }

/* QUMOND potential of a point mass M at the origin: the radial integral of
 * g = nu(g_N/a0) g_N with g_N = GM/r^2, fixed so that it tends to -GM/r as
 * r -> 0.  (Derived in closed form; it reduces to -GM/r for a0 = 0.) */
double orc_phi_point_mond(double r, double G, double M, double a0)
{
    const double GM = G * M;
    return -GM / (2.0 * r) - sqrt(GM) * sqrt(GM + 4.0 * a0 * r * r) / (2.0 * r)
           + sqrt(GM * a0) * asinh(2.0 * r * sqrt(a0 / GM));
}

/* Outermost-box Dirichlet values (Sec. 2, nested refinement).  mode 0: zero
 * (the paper's box 2^10 times the galaxy); mode 1: Newtonian monopole of the
 * total mass; mode 2: QUMOND monopole.  Only boundary nodes are written. */
void orc_bc_outer(int n, double L, int mode, double G, double a0, double M, double *u)
{
    const double h = L / (double)(n - 1);
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                if (!on_boundary(n, i, j, k)) continue;
                double x = -0.5 * L + i * h, y = -0.5 * L + j * h, z = -0.5 * L + k * h;
                double r = sqrt(x * x + y * y + z * z);
                double v = 0.0;
                if (mode == 1) v = orc_phi_point_newton(r, G, M);
                if (mode == 2) v = orc_phi_point_mond(r, G, M, a0);
                u[ID3(n, i, j, k)] = v;
            }
}

/* Trilinear interpolation of a coarse-box field at a physical point. */
static double trilinear_at(int n, double L, const double *u, double x, double y, double z)
{
    const double h = L / (double)(n - 1);
    double p[3] = {(x + 0.5 * L) / h, (y + 0.5 * L) / h, (z + 0.5 * L) / h};
    int i0[3];
    double t[3];
    for (int d = 0; d < 3; d++) {
        double fl = floor(p[d]);
        int ii = (int)fl;
        if (ii > n - 2) ii = n - 2;
        if (ii < 0) ii = 0;
        i0[d] = ii;
        t[d] = p[d] - ii;
    }
    double s = 0.0;
    for (int c = 0; c < 2; c++)
        for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++) {
                double w = (a ? t[0] : 1.0 - t[0]) * (b ? t[1] : 1.0 - t[1]) * (c ? t[2] : 1.0 - t[2]);
                s += w * u[ID3(n, i0[0] + a, i0[1] + b, i0[2] + c)];
            }
    return s;
}

/* Sec. 2 nested refinement: the boundary of the inner box (side Lf) is the
 * coarse box's (side Lc) field interpolated through at each boundary node. */
void orc_bc_from_coarse(int n, double Lc, const double *uc, double Lf, double *uf)
{
    const double hf = Lf / (double)(n - 1);
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                if (!on_boundary(n, i, j, k)) continue;
                double x = -0.5 * Lf + i * hf, y = -0.5 * Lf + j * hf, z = -0.5 * Lf + k * hf;
                uf[ID3(n, i, j, k)] = trilinear_at(n, Lc, uc, x, y, z);
            }
}

/* ------------------------------------------------------------ multigrid */

/* One colour pass of red-black Gauss-Seidel for the 7-point Laplacian
 * (sum of 6 neighbours - 6u)/h^2 = f: every interior node with
 * (i+j+k) mod 2 == colour is set to (sum of 6 neighbours - h^2 f)/6. */
void orc_rbgs_colour(int n, double h, const double *f, double *u, int colour)
{
    const double h2 = h * h;
    ORC_PAR
    for (int k = 1; k < n - 1; k++)
        for (int j = 1; j < n - 1; j++)
            for (int i = 1; i < n - 1; i++) {
                if (((i + j + k) & 1) != colour) continue;
                double s = u[ID3(n, i - 1, j, k)] + u[ID3(n, i + 1, j, k)] + u[ID3(n, i, j - 1, k)]
                           + u[ID3(n, i, j + 1, k)] + u[ID3(n, i, j, k - 1)] + u[ID3(n, i, j, k + 1)];
                u[ID3(n, i, j, k)] = (s - h2 * f[ID3(n, i, j, k)]) / 6.0;
            }
}

/* One full sweep: colour 0 ((i+j+k) even) first, then colour 1. */
void orc_rbgs_sweep(int n, double h, const double *f, double *u)
{
    orc_rbgs_colour(n, h, f, u, 0);
    orc_rbgs_colour(n, h, f, u, 1);
}

/* r = f - A_h u at interior nodes, 0 on the boundary. */
void orc_residual(int n, double h, const double *f, const double *u, double *r)
{
    const double ih2 = 1.0 / (h * h);
    ORC_PAR
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                size_t c = ID3(n, i, j, k);
                if (on_boundary(n, i, j, k)) { r[c] = 0.0; continue; }
                double s = u[ID3(n, i - 1, j, k)] + u[ID3(n, i + 1, j, k)] + u[ID3(n, i, j - 1, k)]
                           + u[ID3(n, i, j + 1, k)] + u[ID3(n, i, j, k - 1)] + u[ID3(n, i, j, k + 1)];
                r[c] = f[c] - (s - 6.0 * u[c]) * ih2;
            }
}

/* Sum of squares of an array over interior nodes. */
double orc_interior_sumsq(int n, const double *a)
{
    double s = 0.0;
    for (int k = 1; k < n - 1; k++)
        for (int j = 1; j < n - 1; j++)
            for (int i = 1; i < n - 1; i++) {
                double v = a[ID3(n, i, j, k)];
                s += v * v;
            }
    return s;
}

/* Full-weighting restriction: coarse interior node I takes
 * sum over a,b,c in {-1,0,1} of w_a w_b w_c r(2I + (a,b,c)), w = (1/4,1/2,1/4);
 * coarse boundary nodes are 0.  nf = 2 nc - 1. */
void orc_restrict_fw(int nf, const double *rf, double *fc)
{
    const int nc = (nf + 1) / 2;
    static const double w[3] = {0.25, 0.5, 0.25};
    ORC_PAR
    for (int K = 0; K < nc; K++)
        for (int J = 0; J < nc; J++)
            for (int I = 0; I < nc; I++) {
                size_t C = ID3(nc, I, J, K);
                if (on_boundary(nc, I, J, K)) { fc[C] = 0.0; continue; }
                double s = 0.0;
                for (int c = -1; c <= 1; c++)
                    for (int b = -1; b <= 1; b++)
                        for (int a = -1; a <= 1; a++)
                            s += w[a + 1] * w[b + 1] * w[c + 1] * rf[ID3(nf, 2 * I + a, 2 * J + b, 2 * K + c)];
                fc[C] = s;
            }
}

/* Trilinear value of a coarse field at fine node (i,j,k): along each axis an
 * even fine index sits on coarse node i/2, an odd one halfway between
 * (i-1)/2 and (i+1)/2. */
static double prolong_value(int nc, const double *uc, int i, int j, int k)
{
    int lo[3], hi[3];
    double wl[3], wh[3];
    int idx[3] = {i, j, k};
    for (int d = 0; d < 3; d++) {
        if ((idx[d] & 1) == 0) { lo[d] = hi[d] = idx[d] / 2; wl[d] = 1.0; wh[d] = 0.0; }
        else { lo[d] = (idx[d] - 1) / 2; hi[d] = (idx[d] + 1) / 2; wl[d] = 0.5; wh[d] = 0.5; }
    }
    double s = 0.0;
    for (int c = 0; c < 2; c++)
        for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++) {
                double w = (a ? wh[0] : wl[0]) * (b ? wh[1] : wl[1]) * (c ? wh[2] : wl[2]);
                if (w == 0.0) continue;
                s += w * uc[ID3(nc, a ? hi[0] : lo[0], b ? hi[1] : lo[1], c ? hi[2] : lo[2])];
            }
    return s;
}

/* Coarse-grid correction: u_f += P u_c at fine interior nodes. */
void orc_prolong_add(int nc, const double *uc, double *uf)
{
    const int nf = 2 * nc - 1;
    ORC_PAR
    for (int k = 1; k < nf - 1; k++)
        for (int j = 1; j < nf - 1; j++)
            for (int i = 1; i < nf - 1; i++) uf[ID3(nf, i, j, k)] += prolong_value(nc, uc, i, j, k);
}

/* FMG interpolation: u_f = P u_c at fine interior nodes (boundary kept). */
void orc_interp(int nc, const double *uc, double *uf)
{
    const int nf = 2 * nc - 1;
    ORC_PAR
    for (int k = 1; k < nf - 1; k++)
        for (int j = 1; j < nf - 1; j++)
            for (int i = 1; i < nf - 1; i++) uf[ID3(nf, i, j, k)] = prolong_value(nc, uc, i, j, k);
}

typedef struct {
    int J;          /* finest level index, n = 2^J + 1 */
    double L;
    double **u, **f; /* per level 1..J; level l has 2^l + 1 nodes per side */
    double *r;      /* scratch of the finest size */
    int npre, npost;
} mg_t;

static int lvl_n(int l) { return (1 << l) + 1; }

static void vcycle(mg_t *mg, int l)
{
    const int n = lvl_n(l);
    const double h = mg->L / (double)(n - 1);
    if (l == 1) { /* 3x3x3: one interior node, one Gauss-Seidel update is exact */
        orc_rbgs_sweep(n, h, mg->f[l], mg->u[l]);
        return;
    }
    for (int s = 0; s < mg->npre; s++) orc_rbgs_sweep(n, h, mg->f[l], mg->u[l]);
    orc_residual(n, h, mg->f[l], mg->u[l], mg->r);
    orc_restrict_fw(n, mg->r, mg->f[l - 1]);
    const int nc = lvl_n(l - 1);
    memset(mg->u[l - 1], 0, sizeof(double) * (size_t)nc * nc * nc);
    vcycle(mg, l - 1);
    orc_prolong_add(nc, mg->u[l - 1], mg->u[l]);
    for (int s = 0; s < mg->npost; s++) orc_rbgs_sweep(n, h, mg->f[l], mg->u[l]);
}

static int log2_exact(int m)
{
    int J = 0;
    while ((1 << J) < m) J++;
    return ((1 << J) == m) ? J : -1;
}

/* Sum over interior nodes of (sum of the node's boundary neighbours / h^2)^2:
 * the norm of the right-hand side the Dirichlet values alone contribute. */
double orc_boundary_coupling_sumsq(int n, double h, const double *u)
{
    const double ih2 = 1.0 / (h * h);
    double s = 0.0;
    for (int k = 1; k < n - 1; k++)
        for (int j = 1; j < n - 1; j++)
            for (int i = 1; i < n - 1; i++) {
                double b = 0.0;
                if (i == 1) b += u[ID3(n, 0, j, k)];
                if (i == n - 2) b += u[ID3(n, n - 1, j, k)];
                if (j == 1) b += u[ID3(n, i, 0, k)];
                if (j == n - 2) b += u[ID3(n, i, n - 1, k)];
                if (k == 1) b += u[ID3(n, i, j, 0)];
                if (k == n - 2) b += u[ID3(n, i, j, n - 1)];
                b *= ih2;
                s += b * b;
            }
    return s;
}

/* Relative residual of the stopping test: ||f - A_h u||_2 / ||f||_2 over the
 * interior; for a source-free problem (||f|| = 0) the denominator is the norm
 * of the boundary-value contribution, and if that is 0 too the test is on the
 * absolute residual. */
static double relres_of(mg_t *mg, double fnorm)
{
    const int n = lvl_n(mg->J);
    const double h = mg->L / (double)(n - 1);
    orc_residual(n, h, mg->f[mg->J], mg->u[mg->J], mg->r);
    double rn = sqrt(orc_interior_sumsq(n, mg->r));
    double den = fnorm > 0.0 ? fnorm : sqrt(orc_boundary_coupling_sumsq(n, h, mg->u[mg->J]));
    return den > 0.0 ? rn / den : rn;
}

static int mg_alloc(mg_t *mg, int n, double L, const double *f, double *u, int npre, int npost)
{
    int J = log2_exact(n - 1);
    if (J < 1) return -1;
    mg->J = J;
    mg->L = L;
    mg->npre = npre;
    mg->npost = npost;
    mg->u = (double **)calloc((size_t)J + 1, sizeof(double *));
    mg->f = (double **)calloc((size_t)J + 1, sizeof(double *));
    mg->r = (double *)calloc((size_t)n * n * n, sizeof(double));
    for (int l = 1; l < J; l++) {
        size_t N = (size_t)lvl_n(l) * lvl_n(l) * lvl_n(l);
        mg->u[l] = (double *)calloc(N, sizeof(double));
        mg->f[l] = (double *)calloc(N, sizeof(double));
    }
    mg->u[J] = u;
    mg->f[J] = (double *)f;
    return 0;
}

static void mg_free(mg_t *mg)
{
    for (int l = 1; l < mg->J; l++) { free(mg->u[l]); free(mg->f[l]); }
    free(mg->u);
    free(mg->f);
    free(mg->r);
}

/* Full multigrid solve of A_h u = f on one box (Sec. 2).  On entry the
 * boundary nodes of u hold the Dirichlet values; interior values are ignored.
 *  1. f is restricted by full weighting down to the 3^3 level;
 *  2. every coarse level takes the boundary values of the finest level at
 *     coinciding nodes;
 *  3. the single interior node of the 3^3 level is solved exactly;
 *  4. for each finer level: trilinear interpolation of the coarser solution
 *     into the interior, then ncycle V-cycles (npre/npost RB-GS sweeps, zero
 *     Dirichlet corrections on coarser levels);
 *  5. then further finest-level V-cycles while
 *     ||f - A_h u||_2 / ||f||_2 (interior) > tol, at most max_extra of them
 *     (tol = 0: fixed schedule); see relres_of for a source-free box.
 * Returns 0 when converged (or fixed schedule), 1 when max_extra was hit,
 * -1 on a bad size.  *relres_out gets the final relative residual and
 * *extra_out the number of extra cycles. */
int orc_fmg(int n, double L, const double *f, double *u, int npre, int npost, int ncycle,
            int max_extra, double tol, double *relres_out, int *extra_out)
{
    mg_t mg;
    if (mg_alloc(&mg, n, L, f, u, npre, npost) != 0) return -1;
    const int J = mg.J;
    for (int l = J - 1; l >= 1; l--) orc_restrict_fw(lvl_n(l + 1), mg.f[l + 1], mg.f[l]);
    for (int l = 1; l < J; l++) {
        const int nl = lvl_n(l), stride = 1 << (J - l);
        for (int k = 0; k < nl; k++)
            for (int j = 0; j < nl; j++)
                for (int i = 0; i < nl; i++)
                    if (on_boundary(nl, i, j, k))
                        mg.u[l][ID3(nl, i, j, k)] = u[ID3(n, i * stride, j * stride, k * stride)];
    }
    {
        const int n1 = lvl_n(1);
        orc_rbgs_sweep(n1, L / (double)(n1 - 1), mg.f[1], mg.u[1]);
    }
    for (int l = 2; l <= J; l++) {
        orc_interp(lvl_n(l - 1), mg.u[l - 1], mg.u[l]);
        for (int c = 0; c < ncycle; c++) vcycle(&mg, l);
    }
    const double fnorm = sqrt(orc_interior_sumsq(n, f));
    double rr = relres_of(&mg, fnorm);
    int extra = 0;
    while (tol > 0.0 && rr > tol && extra < max_extra) {
        vcycle(&mg, J);
        extra++;
        rr = relres_of(&mg, fnorm);
    }
    if (relres_out) *relres_out = rr;
    if (extra_out) *extra_out = extra;
    mg_free(&mg);
    return (tol > 0.0 && rr > tol) ? 1 : 0;
}

/* ncyc V-cycles on the finest level starting from the given u (boundary
 * holds the Dirichlet values).  Returns the final relative residual. */
double orc_vcycles(int n, double L, const double *f, double *u, int npre, int npost, int ncyc)
{
    mg_t mg;
    if (mg_alloc(&mg, n, L, f, u, npre, npost) != 0) return -1.0;
    for (int c = 0; c < ncyc; c++) vcycle(&mg, mg.J);
    double rr = relres_of(&mg, sqrt(orc_interior_sumsq(n, f)));
    mg_free(&mg);
    return rr;
}

/* ------------------------------------------------------------ nu-source */

/* Flux through the face between node p and q = p + e_d (d = 0,1,2):
 * normal gradient (Phi_q - Phi_p)/h, transverse components averaged over the
 * four nodes beside the face, F = nu(|g|/a0) g_n, and F = 0 where |g| = 0
 * (the limit of nu(|g|/a0) g as |g| -> 0). */
static double face_flux(int n, double h, double a0, double nn, const double *P, int i, int j, int k, int d)
{
    int e[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    int qi = i + e[d][0], qj = j + e[d][1], qk = k + e[d][2];
    double gn = (P[ID3(n, qi, qj, qk)] - P[ID3(n, i, j, k)]) / h;
    double g2 = gn * gn;
    for (int t = 0; t < 3; t++) {
        if (t == d) continue;
        double gt = (P[ID3(n, i + e[t][0], j + e[t][1], k + e[t][2])]
                     + P[ID3(n, qi + e[t][0], qj + e[t][1], qk + e[t][2])]
                     - P[ID3(n, i - e[t][0], j - e[t][1], k - e[t][2])]
                     - P[ID3(n, qi - e[t][0], qj - e[t][1], qk - e[t][2])]) / (4.0 * h);
        g2 += gt * gt;
    }
    double g = sqrt(g2);
    if (g == 0.0) return 0.0;
    if (nn != 1.0) return gn * orc_nu_n(g / a0, nn);
    return 0.5 * gn * (1.0 + sqrt(1.0 + 4.0 * a0 / g));
}

/* Eq. 2 source: S_p = sum_d (F_{p+e_d/2} - F_{p-e_d/2}) / h at interior
 * nodes, 0 on the boundary; nu from the n-family (nn = 1: Eq. 2's nu). */
void orc_mond_source_nu(int n, double L, double a0, double nn, const double *phin, double *S)
{
    const double h = L / (double)(n - 1);
    ORC_PAR
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                size_t c = ID3(n, i, j, k);
                if (on_boundary(n, i, j, k)) { S[c] = 0.0; continue; }
                double s = 0.0;
                s += face_flux(n, h, a0, nn, phin, i, j, k, 0) - face_flux(n, h, a0, nn, phin, i - 1, j, k, 0);
                s += face_flux(n, h, a0, nn, phin, i, j, k, 1) - face_flux(n, h, a0, nn, phin, i, j - 1, k, 1);
                s += face_flux(n, h, a0, nn, phin, i, j, k, 2) - face_flux(n, h, a0, nn, phin, i, j, k - 1, 2);
                S[c] = s / h;
            }
}

void orc_mond_source(int n, double L, double a0, const double *phin, double *S)
{
    orc_mond_source_nu(n, L, a0, 1.0, phin, S);
}

/* ---------------------------------------------------------------- gather */

/* Gravity g = -grad Phi at a node: central difference inside, one-sided
 * second-order difference on the box faces. */
static double node_grad(int n, double h, const double *P, int i, int j, int k, int d)
{
    int idx[3] = {i, j, k};
    int a[3] = {i, j, k}, b[3] = {i, j, k}, c[3] = {i, j, k};
    double v;
    if (idx[d] > 0 && idx[d] < n - 1) {
        a[d] = idx[d] + 1;
        b[d] = idx[d] - 1;
        v = (P[ID3(n, a[0], a[1], a[2])] - P[ID3(n, b[0], b[1], b[2])]) / (2.0 * h);
    } else if (idx[d] == 0) {
        a[d] = 1;
        b[d] = 2;
        v = (-3.0 * P[ID3(n, i, j, k)] + 4.0 * P[ID3(n, a[0], a[1], a[2])] - P[ID3(n, b[0], b[1], b[2])]) / (2.0 * h);
    } else {
        a[d] = n - 2;
        b[d] = n - 3;
        v = (3.0 * P[ID3(n, i, j, k)] - 4.0 * P[ID3(n, a[0], a[1], a[2])] + P[ID3(n, b[0], b[1], b[2])]) / (2.0 * h);
    }
    (void)c;
    return -v;
}

/* Sec. 2 / Sec. 3.1: accelerations at arbitrary points.  Box choice: the
 * finest box b with R < frac L_b and |z| < frac L_b; failing that the
 * outermost box that contains the point (0 <= u_d < n-1); failing that the
 * monopole of mass M (Newtonian for mond == 0, QUMOND otherwise).  Inside the
 * chosen box the node gravities of the 8 CIC corners are weighted with the
 * CIC weights.  box_used gets the box index, 255 for the monopole. */
void orc_gather_nu(int nbox, int n, const double *Ls, const double *const *phis, int64_t np,
                   const double *x, const double *y, const double *z, double frac, double G,
                   double a0, double M, int mond, double nn, double *ax, double *ay, double *az,
                   uint8_t *box_used)
{
    ORC_PAR
    for (int64_t p = 0; p < np; p++) {
        double R = sqrt(x[p] * x[p] + y[p] * y[p]);
        double az_abs = fabs(z[p]);
        int sel = -1;
        for (int b = nbox - 1; b >= 0; b--)
            if (R < frac * Ls[b] && az_abs < frac * Ls[b]) { sel = b; break; }
        if (sel < 0) {
            for (int b = 0; b < nbox; b++) {
                double inv_h = (double)(n - 1) / Ls[b];
                double ux = (x[p] + 0.5 * Ls[b]) * inv_h, uy = (y[p] + 0.5 * Ls[b]) * inv_h,
                       uz = (z[p] + 0.5 * Ls[b]) * inv_h;
                if (ux >= 0 && ux < n - 1 && uy >= 0 && uy < n - 1 && uz >= 0 && uz < n - 1) { sel = b; break; }
            }
        }
        if (box_used) box_used[p] = (uint8_t)(sel < 0 ? 255 : sel);
        if (sel < 0) {
            double r = sqrt(x[p] * x[p] + y[p] * y[p] + z[p] * z[p]);
            double g = 0.0;
            if (r > 0.0) {
                double gN = G * M / (r * r);
                g = (mond && a0 > 0.0) ? orc_nu_n(gN / a0, nn) * gN : gN;
                g /= r;
            }
            ax[p] = -g * x[p];
            ay[p] = -g * y[p];
            az[p] = -g * z[p];
            continue;
        }
        const double L = Ls[sel];
        const double h = L / (double)(n - 1);
        const double inv_h = (double)(n - 1) / L;
        double u[3] = {(x[p] + 0.5 * L) * inv_h, (y[p] + 0.5 * L) * inv_h, (z[p] + 0.5 * L) * inv_h};
        int ic[3];
        double w[3][2];
        for (int d = 0; d < 3; d++) {
            double fl = floor(u[d]);
            ic[d] = (int)fl;
            double fr = u[d] - fl;
            w[d][0] = 1.0 - fr;
            w[d][1] = fr;
        }
        double acc[3] = {0.0, 0.0, 0.0};
        const double *P = phis[sel];
        for (int c = 0; c < 2; c++)
            for (int b = 0; b < 2; b++)
                for (int a = 0; a < 2; a++) {
                    double wt = (w[0][a] * w[1][b]) * w[2][c];
                    for (int d = 0; d < 3; d++)
                        acc[d] += wt * node_grad(n, h, P, ic[0] + a, ic[1] + b, ic[2] + c, d);
                }
        ax[p] = acc[0];
        ay[p] = acc[1];
        az[p] = acc[2];
    }
}

void orc_gather(int nbox, int n, const double *Ls, const double *const *phis, int64_t np,
                const double *x, const double *y, const double *z, double frac, double G,
                double a0, double M, int mond, double *ax, double *ay, double *az,
                uint8_t *box_used)
{
    orc_gather_nu(nbox, n, Ls, phis, np, x, y, z, frac, G, a0, M, mond, 1.0, ax, ay, az, box_used);
}
