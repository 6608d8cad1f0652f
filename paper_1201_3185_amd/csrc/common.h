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
constexpr int kWinX = 32, kWinY = 32, kWinZ = 8, kWin = kWinX * kWinY * kWinZ;
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
    int mond;
};

// ---- grid_kernels.hip (templated on the storage type: double or float)
// Smoother launch shape: tile variant (0: 32x8, 1: 64x4, 2: 64x8, 3: 128x4,
// 4: 32x16 columns) and the number of z planes one workgroup marches through.
struct SmootherShape {
    int variant;
    int kchunk;
};
constexpr int kSmootherVariants = 5;
template <typename T> void launch_rbgs(int n, double h, const T *f, const T *uin, T *uout, hipStream_t s);
template <typename T> void launch_rbgs_shape(int n, double h, const T *f, const T *uin, T *uout, SmootherShape sh,
                                            hipStream_t s);
template <typename T> SmootherShape &rbgs_shape(int n);   // the table entry used for n
// Two sweeps in one launch (variants 0: 32x8, 1: 64x4); with uc != NULL the
// correction u += P uc (uc on the next coarser level) is applied first.
template <typename T> void launch_rbgs2(int n, double h, const T *f, const T *uin, T *uout, const T *uc,
                                       hipStream_t s);
template <typename T> SmootherShape &rbgs2_shape(int n);
// Whether the multigrid uses the fused kernel on a level of n points per side
// (set by the autotuner from measured times; n <= 65 by default).
template <typename T> int &use_fused(int n);
template <typename T> void launch_residual_restrict(int nf, double h, const T *f, const T *u, T *fc, T *uc0, T *uc1,
                                                   hipStream_t s);
template <typename T> void launch_restrict(int nf, const T *src, T *dst, hipStream_t s);
template <typename T> void launch_prolong_add(int nc, const T *uc, T *uf, hipStream_t s);
template <typename T> void launch_interp(int nc, const T *uc, T *uf, hipStream_t s);
template <typename T> void launch_inject_boundary(int nfine, const T *ufine, int nl, T *u0, T *u1, hipStream_t s);
template <typename T> void launch_fill(T *p, size_t count, T v, hipStream_t s);
template <typename T> void launch_boundary_copy(int n, const T *src, T *dst, hipStream_t s);
// Coarse tail: all levels with n <= 17 inside one workgroup's LDS.  mode 0: one
// V-cycle of the top level (correction, zero boundary); mode 1: FMG from 3^3 up to
// the top level with ncycle V-cycles per level (boundary of u = Dirichlet values).
template <typename T> void launch_coarse_tail(int ltop, double L, const T *f, T *u, int npre, int npost, int ncycle,
                                             int mode, int nrep, hipStream_t s);
// Sums over interior nodes of (f - A_h u)^2, f^2 and of the squared boundary-value
// contribution: per-block partials (3 per block), then one block in fixed order,
// into out[0..2] (device doubles).
template <typename T> void launch_resid_norms(int n, double h, const T *f, const T *u, double *partial, double *out,
                                             hipStream_t s);
constexpr int kNormBlocks = 512;

// mixed precision (FP64 refinement around FP32 multigrid)
void launch_narrow(const double *src, float *dst, size_t count, hipStream_t s);
void launch_narrow_boundary(int n, const double *src, float *d0, float *d1, hipStream_t s);
void launch_widen_interior(int n, const float *src, double *dst, hipStream_t s);
void launch_resid_to_f32(int n, double h, double inv_s, const double *f, const double *u, float *r, hipStream_t s);
void launch_correct(int n, double scale, const float *e, double *u, hipStream_t s);

// interior of u from an initial guess (kind 1: double, 2: float, 3: bf16)
void launch_guess_interior(int n, const void *g, int kind, double *u, hipStream_t s);

// ---- bc_kernels.hip
// mode 0 zero, 1 Newtonian monopole -GM/r, 2 QUMOND monopole.
void launch_bc_outer(int n, double L, int mode, double GM, double a0, double *u0, double *u1, hipStream_t s);
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

// ---- source_kernel.hip
void launch_mond_source(int n, double h, double a0, const double *phin, double *S, hipStream_t s);

}  // namespace qm
