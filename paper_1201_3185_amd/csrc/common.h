// Internal declarations of the gfx950 QUMOND library: grid indexing, the
// per-box descriptors handed to particle kernels by value, and the host
// launchers each kernel file exports to the multigrid driver and the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qm {

constexpr int kMaxBox = 16;

__host__ __device__ __forceinline__ size_t id3(int n, int i, int j, int k)
{
    return (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
}

// Workgroups are dispatched to the 8 XCDs round robin (hardware id w runs on
// XCD w mod 8), and each XCD has its own L2.  xcd_tile gives hardware id w the
// tile (w mod 8) * (nblk / 8) + w / 8, so that each XCD works through one
// contiguous range of tiles and neighbouring tiles share their halos in one
// L2; ids beyond the last multiple of 8 keep their own tile.
__device__ __forceinline__ unsigned xcd_tile(unsigned w, unsigned nblk)
{
    const unsigned full = nblk & ~7u;
    return w < full ? (w & 7u) * (full >> 3) + (w >> 3) : w;
}

// ------------------------------------------------------------ nu
// The interpolating function.  n == 1 is Eq. 2's nu(y) = 1/2 + 1/2 sqrt(1 + 4/y),
// evaluated by the closed expressions in each kernel; any other n is the
// n-family nu_n(y) = [(1 + sqrt(1 + 4 y^-n)) / 2]^(1/n) (n = 2: the "standard"
// function).  The point-mass QUMOND potential for n != 1 is
// -GM/r + sqrt(G M a0) I(r / r_M), r_M = sqrt(G M / a0), with the universal
// I(t) = int_0^t (nu_n(1/s^2) - 1) / s^2 ds tabulated at u = ln t on a uniform
// grid (values and exact slopes dI/du, cubic Hermite in between).
constexpr int kNuTab = 10241;
constexpr double kNuU0 = -20.0, kNuDu = 1.0 / 256.0;

struct NuFn {
    double n = 1.0;
    const double *tab = nullptr;  // device, [kNuTab][2] = {I, dI/du}; only for n != 1
};

__host__ __device__ inline double nu_family(double y, double n)
{
    return pow(0.5 * (1.0 + sqrt(1.0 + 4.0 * pow(y, -n))), 1.0 / n);
}

// I(t) from the table; below the table the leading term t^(2n-1) / (n (2n-1)),
// above it the end slope continued (I grows like ln t there).
__device__ inline double nu_point_integral(const NuFn &nu, double t)
{
#pragma clang fp contract(off)
    const double u = log(t);
    const double n = nu.n;
    if (u <= kNuU0) return pow(t, 2.0 * n - 1.0) / (n * (2.0 * n - 1.0));
    const double x = (u - kNuU0) / kNuDu;
    int k = (int)x;
    if (k >= kNuTab - 1) {
        const double *e = nu.tab + 2 * (kNuTab - 1);
        return e[0] + e[1] * (u - (kNuU0 + (kNuTab - 1) * kNuDu));
    }
    const double s = x - (double)k;
    const double *a = nu.tab + 2 * k;
    const double s2 = s * s, s3 = s2 * s;
    return (2.0 * s3 - 3.0 * s2 + 1.0) * a[0] + (s3 - 2.0 * s2 + s) * kNuDu * a[1] + (3.0 * s2 - 2.0 * s3) * a[2] +
           (s3 - s2) * kNuDu * a[3];
}

// Host: fills tab[kNuTab][2] for the n-family member n (n >= 1).
void build_nu_table(double n, double *tab);

// Geometry of one box as the particle kernels see it.
struct BoxGeom {
    double L;       // side, kpc
    double xmin;    // -L/2
    double inv_h;   // (n-1)/L
    double h;       // L/(n-1)
};

// LDS window of the deposit: every workgroup accumulates the corners that fall
// in a kWinX x kWinY x kWinZ block of nodes around each box's centre (where a
// galaxy's mass concentrates) in LDS, and writes it to its own scratch slab.
constexpr int kWinX = 48, kWinY = 48, kWinZ = 8, kWin = kWinX * kWinY * kWinZ;
constexpr int kDepositThreads = 1024;
constexpr int kDepositMaxBlocks = 256;

struct DepositArgs {
    int nbox, n;
    BoxGeom box[kMaxBox];
    unsigned long long *q[kMaxBox];
    int w0[kMaxBox][3];              // window origin node per box and axis
    unsigned long long *scratch;     // [blocks][nbox][kWin]
    double scale;                    // 2^s
};

struct GatherArgs {
    int nbox, n;
    BoxGeom box[kMaxBox];
    const double *phi[kMaxBox];
    double frac, GM, a0;
    int mond;  // monopole of points outside every box: 0 Newtonian, 1 QUMOND
    int alg;   // 1: Eq. 3 applied to the gathered (Newtonian) field
    double nun;  // interpolating function (NuFn::n)
};

// One problem of a batch as its kernels read it from device memory, so that a
// captured graph stays valid when the inputs change: particle arrays (device,
// caller-owned), count, total mass and the fixed-point scale 2^shift.
struct BatchProblem {
    const double *x, *y, *z, *m;
    long long np;
    double mass;
    double scale;
    int shift;
    int pad;
};
constexpr int kBatchDepositBlocks = 64;   // deposit workgroups per problem

// ---- grid_kernels.hip (templated on the storage type: double or float)
// Smoother launch shape: tile variant (z-march over 0: 32x8, 1: 64x4, 2: 64x8,
// 3: 128x4, 4: 32x16 columns; 5: 8^3 bricks; 6: 64x8, 7: 64x16, 8: 128x8
// columns with one thread per x-pair of nodes; 9: 4^3, 10: 6^3 bricks; 11: 32x16,
// 12: 32x8 pair columns; 13: 64x16, 14: 128x8, 15: 64x32 pair columns with
// loads two march steps ahead) and the number of z planes one workgroup
// marches through (ignored by bricks).
struct SmootherShape {
    int variant;
    int kchunk;
};
constexpr int kSmootherVariants = 16;
constexpr int kRrVariants = 12;   // residual restriction: gather, 8x8x4 LDS tile, z-march with 4/8/16-plane
                                  // chunks, 4x4x4 and 4x4x2 LDS tiles, whole-column z-march of 32x8 / 64x4
                                  // columns (512 threads), 32x8 columns over 64-plane chunks, 32x8 whole
                                  // columns loading three / four steps ahead
// bricks hold their whole block in LDS and take no z-chunk
inline bool is_brick_variant(int v, bool fused) { return fused ? (v >= 2 && v <= 4) : (v == 5 || v == 9 || v == 10); }
constexpr int kFusedVariants = 10;  // two sweeps: 0: 32x8, 1: 64x4 z-march, 2: 8^3, 3: 4^3, 4: 6^3 bricks,
                                    // 5: 64x16, 6: 64x8, 7: 32x16 pair z-march with loads two steps ahead,
                                    // 8: 64x16, 9: 32x8 whole columns with the four half-sweeps skewed
                                    // (rbgs2_skew.hip)
constexpr int kSkewVariant = 8, kSkew32Variant = 9;
// shapes that take no z-chunk: the bricks, and the skewed two-sweep marches (whole columns)
inline bool takes_no_chunk(int v, bool fused)
{
    return is_brick_variant(v, fused) || (fused && (v == kSkewVariant || v == kSkew32Variant));
}
// Every grid launcher takes nb, the number of problems stored back to back
// (problem p of a level with n points per side at offset p n^3); nb = 1 is the
// single-problem case.
// One sweep; with uc != NULL the correction u += P uc (uc on the next coarser
// level) is applied first, in the same launch.  A null uin stands for a zero
// iterate (boundary included) in the single-sweep kernels (z-march, pair
// z-march, brick), which then read no iterate at all.
template <typename T> void launch_rbgs(int n, double h, const T *f, const T *uin, T *uout, hipStream_t s, int nb = 1,
                                      const T *uc = nullptr);
template <typename T> void launch_rbgs_shape(int n, double h, const T *f, const T *uin, T *uout, SmootherShape sh,
                                            hipStream_t s, int nb = 1, const T *uc = nullptr);
template <typename T> SmootherShape &rbgs_shape(int n);   // the table entry used for n
// Shape of a single sweep that also applies the coarse-grid correction; a
// variant below 0 (the default) means the level's plain-sweep shape.
template <typename T> SmootherShape &rbgs_corr_shape(int n);
template <typename T> SmootherShape rbgs_corr_effective(int n);
// Two sweeps in one launch (variants 0: 32x8, 1: 64x4 z-march, 2: 8^3 bricks);
// with uc != NULL the correction u += P uc (uc on the next coarser level) is
// applied first.
template <typename T> void launch_rbgs2(int n, double h, const T *f, const T *uin, T *uout, const T *uc,
                                       hipStream_t s, int nb = 1);
template <typename T> void launch_rbgs2_shape(int n, double h, const T *f, const T *uin, T *uout, const T *uc,
                                             SmootherShape sh, hipStream_t s, int nb = 1);
template <typename T> SmootherShape &rbgs2_shape(int n);
// ---- rbgs2_skew.hip
// Two sweeps uin -> uout in one whole-column march with the four half-sweeps
// skewed two planes apart (same bits as two single sweeps); uin null is a zero
// iterate; with uc != NULL the correction u += P uc (uc on the next coarser
// level) is applied first, in the same launch (same bits as a prolong-add).
// tile 0: 64x16 columns (1024 threads), 1: 32x8 columns (320 threads).
template <typename T> void launch_rbgs2_skew(int n, double h, const T *f, const T *uin, T *uout, hipStream_t s, int nb,
                                            const T *uc = nullptr, int tile = 0);
// Whether the multigrid uses the fused kernel on a level of n points per side
// (set by the autotuner from measured times; n <= 65 by default).
template <typename T> int &use_fused(int n);
// Whether the coarse-grid correction of a level of n points is its own
// prolong-add launch (1) or is folded into the first post-smoothing launch (0);
// identical results, chosen by the autotuner from measured times.
template <typename T> int &split_prolong(int n);
// zero_u = false leaves the interior of uc0 unwritten (its boundary is still
// zeroed): for a caller whose next use of the coarse correction takes it as
// zero without reading it.
template <typename T> void launch_residual_restrict(int nf, double h, const T *f, const T *u, T *fc, T *uc0, T *uc1,
                                                   hipStream_t s, int nb = 1, bool zero_u = true);
// The implementations of the residual restriction (per-node gather, LDS tiles,
// z-march; identical results) and the table entry that selects one per fine
// level size (set by the autotuner).
template <typename T> void launch_residual_restrict_variant(int nf, double h, const T *f, const T *u, T *fc, T *uc0,
                                                           T *uc1, int variant, hipStream_t s, int nb = 1,
                                                           bool zero_u = true);
template <typename T> int &rr_variant(int nf);
template <typename T> void launch_restrict(int nf, const T *src, T *dst, hipStream_t s, int nb = 1);
// ---- sweep_restrict.hip
// One smoother sweep uin -> uout fused with the residual restriction of uout
// (fc = FW(f - A_h uout) on the next coarser level, uc0 = 0, uc1 = 0 on its
// boundary): the same values as launch_rbgs then launch_residual_restrict.
// Each workgroup marches a whole z column, so the grid needs n >= 9.
template <typename T> bool rbgs_restrict_fits(int n);
template <typename T> void launch_rbgs_restrict(int n, double h, const T *f, const T *uin, T *uout, T *fc, T *uc0, T *uc1,
                                               hipStream_t s, int nb = 1, bool zero_u = true);
// Whether the last pre-smoothing sweep of a level of n points runs fused with
// its residual restriction (1) or as a sweep launch and a restriction launch
// (0, the default); identical results, chosen by the autotuner.
template <typename T> int &sweep_restrict(int n);
template <typename T> void launch_prolong_add(int nc, const T *uc, T *uf, hipStream_t s, int nb = 1);
template <typename T> void launch_interp(int nc, const T *uc, T *uf, hipStream_t s, int nb = 1);
template <typename T> void launch_inject_boundary(int nfine, const T *ufine, int nl, T *u0, T *u1, hipStream_t s,
                                                 int nb = 1);
template <typename T> void launch_fill(T *p, size_t count, T v, hipStream_t s);
template <typename T> void launch_boundary_copy(int n, const T *src, T *dst, hipStream_t s);
// Coarse tail: all levels with n <= 17 inside one workgroup's LDS (one
// workgroup per problem).  mode 0: one V-cycle of the top level (correction,
// zero boundary); mode 2: the same from an iterate that is zero everywhere,
// which is then not read; mode 1: FMG from 3^3 up to the top level with ncycle
// V-cycles per level (boundary of u = Dirichlet values).
template <typename T> void launch_coarse_tail(int ltop, double L, const T *f, T *u, int npre, int npost, int ncycle,
                                             int mode, int nrep, hipStream_t s, int nb = 1);
// Sums over interior nodes of (f - A_h u)^2, f^2 and of the squared boundary-value
// contribution: per-block partials (3 per block, up to kNormBlocks blocks per
// problem), then one block per problem in fixed order, into out[3p..3p+2]
// (device doubles).
// hout (optional): device-mapped pinned host memory that also receives the sums.
template <typename T> void launch_resid_norms(int n, double h, const T *f, const T *u, double *partial, double *out,
                                             hipStream_t s, int nb = 1, double *hout = nullptr);
constexpr int kNormBlocks = 2048;

// mixed precision (FP64 refinement around FP32 multigrid); sc holds s and 1/s
// per problem, written by launch_mixed_scale from the residual norms.
void launch_narrow(const double *src, float *dst, size_t count, hipStream_t s);
void launch_narrow_boundary(int n, const double *src, float *d0, float *d1, hipStream_t s, int nb = 1);
void launch_widen_interior(int n, const float *src, double *dst, hipStream_t s, int nb = 1);
void launch_mixed_scale(int n, const double *norms, double *sc, hipStream_t s, int nb = 1);
// The residual norms (as launch_resid_norms) and, in the same pass, the
// residual times 1/s (sc per problem) rounded to FP32 at interior nodes.
void launch_resid_norms_r32(int n, double h, const double *f, const double *u, double *partial, double *out,
                            const double *sc, float *r32, hipStream_t s, int nb = 1, double *hout = nullptr);
void launch_resid_to_f32(int n, double h, const double *sc, const double *f, const double *u, float *r, hipStream_t s,
                         int nb = 1);
void launch_correct(int n, const double *sc, const float *e, double *u, hipStream_t s, int nb = 1);

// interior of u from an initial guess (kind 1: double, 2: float, 3: bf16)
void launch_guess_interior(int n, const void *g, int kind, double *u, hipStream_t s);

// ---- bc_kernels.hip
// mode 0 zero, 1 Newtonian monopole -GM/r, 2 QUMOND monopole.
void launch_bc_outer(int n, double L, int mode, double GM, double a0, double *u0, double *u1, hipStream_t s,
                     const NuFn &nu = NuFn());
// Mode 1 or 2 at every node with r -> sqrt(r^2 + soft^2) (n^3 doubles).
void launch_monopole_field(int n, double L, int mode, double GM, double a0, double soft, double *out, hipStream_t s);
// The same for nb problems (back to back), GM = G * prob[p].mass.
void launch_bc_outer_batch(int n, double L, int mode, double G, double a0, const BatchProblem *prob, double *u0,
                           int nb, hipStream_t s, const NuFn &nu = NuFn());
void launch_bc_from_coarse(int n, const double *uc, double *u0, double *u1, hipStream_t s);

// ---- particle_kernels.hip
// a.q must be zeroed; a.scratch must hold deposit_scratch_bytes(a.nbox) bytes.
size_t deposit_scratch_bytes(int nbox);
void launch_deposit(const DepositArgs &a, const double *x, const double *y, const double *z, const double *m,
                    int64_t np, unsigned long long *inside_count, hipStream_t s);
void launch_rhs_from_q(int n, double h, double four_pi_G, int shift, const long long *q, double *f, hipStream_t s);
void launch_gather(const GatherArgs &a, const double *x, const double *y, const double *z, int64_t np, double *ax,
                   double *ay, double *az, uint8_t *box_used, hipStream_t s);
void launch_rotation_curve(const GatherArgs &a, const double *R, int nR, int naz, double *vc2, hipStream_t s);
void launch_sigma_z(const GatherArgs &a, const double *R, int nR, int naz, double z, double z0, double *sig2,
                    hipStream_t s);
// Batches of single-box problems (one box of side L, n points per side):
// q must be zeroed; scratch holds deposit_batch_scratch_bytes(nb) bytes;
// inside[p] counts the particles of problem p deposited (must be zeroed).
size_t deposit_batch_scratch_bytes(int nb);
void launch_deposit_batch(int n, double L, const BatchProblem *prob, long long maxnp, unsigned long long *q,
                          unsigned long long *scratch, unsigned long long *inside, int nb, hipStream_t s);
void launch_rhs_batch(int n, double h, double four_pi_G, const BatchProblem *prob, const long long *q, double *f, int nb,
                      hipStream_t s);
// vc2[p nR + r]: Eq. 4 at radius R[r] from the potential of problem p (monopole
// force G prob[p].mass beyond the box; mond selects the QUMOND monopole).
void launch_rotation_curve_batch(int n, double L, double frac, double G, double a0, int mond,
                                 const BatchProblem *prob, const double *phi, const double *R, int nR, int naz,
                                 double *vc2, int nb, hipStream_t s, double nun = 1.0);

// ---- source_kernel.hip
void launch_mond_source(int n, double h, double a0, const double *phin, double *S, hipStream_t s, int nb = 1,
                        double nun = 1.0);

}  // namespace qm
