// Particle <-> mesh kernels (Sec. 2 of Angus et al.): cloud-in-cell mass
// assignment in 64-bit fixed point (step 1), the Eq. 1 right-hand side, and
// the force gather with the same cloud-in-cell weights, plus the circular
// speed of Eq. 4.
//
// The deposit's weights are plain IEEE products (no fused multiply-add) and
// each corner receives rint(w m 2^s) as a 64-bit integer, so the integer grid
// does not depend on the order in which atomics land.
#include "common.h"

namespace qm {

// ------------------------------------------------------------------ deposit
//
// Workgroup g takes a contiguous share of the particles.  For each box it
// clears an LDS window of kWin nodes around the box centre, adds every corner
// of the particles whose whole cloud lies in the window with LDS 64-bit
// atomics, sends the other particles' corners to the grid with global 64-bit
// atomics, and writes the window to its scratch slab.  A second kernel sums
// the slabs of all workgroups into the grid.  Integer addition makes the
// result independent of the order of every add.

__device__ __forceinline__ bool cic_cell(const BoxGeom &g, int n, double px, double py, double pz, int ic[3],
                                         double w[3][2])
{
#pragma clang fp contract(off)
    const double top = (double)(n - 1);
    const double ux = (px - g.xmin) * g.inv_h;
    const double uy = (py - g.xmin) * g.inv_h;
    const double uz = (pz - g.xmin) * g.inv_h;
    if (!(ux >= 0.0 && ux < top && uy >= 0.0 && uy < top && uz >= 0.0 && uz < top)) return false;
    const double fx0 = floor(ux), fy0 = floor(uy), fz0 = floor(uz);
    ic[0] = (int)fx0;
    ic[1] = (int)fy0;
    ic[2] = (int)fz0;
    const double fx = ux - fx0, fy = uy - fy0, fz = uz - fz0;
    w[0][0] = 1.0 - fx;
    w[0][1] = fx;
    w[1][0] = 1.0 - fy;
    w[1][1] = fy;
    w[2][0] = 1.0 - fz;
    w[2][1] = fz;
    return true;
}

__global__ void __launch_bounds__(kDepositThreads)
deposit_window_k(DepositArgs A, const double *__restrict__ x, const double *__restrict__ y,
                 const double *__restrict__ z, const double *__restrict__ m, int64_t np, int64_t per_block,
                 unsigned long long *__restrict__ inside_count)
{
#pragma clang fp contract(off)
    __shared__ unsigned long long W[kWin];
    __shared__ unsigned int cnt_sh;
    const int64_t p0 = (int64_t)blockIdx.x * per_block;
    const int64_t p1 = min(np, p0 + per_block);
    if (threadIdx.x == 0) cnt_sh = 0;
    unsigned int in0 = 0;
    for (int b = 0; b < A.nbox; ++b) {
        for (int e = threadIdx.x; e < kWin; e += kDepositThreads) W[e] = 0ULL;
        __syncthreads();
        const BoxGeom g = A.box[b];
        const int wx = A.w0[b][0], wy = A.w0[b][1], wz = A.w0[b][2];
        unsigned long long *q = A.q[b];
        for (int64_t p = p0 + threadIdx.x; p < p1; p += kDepositThreads) {
            int ic[3];
            double w[3][2];
            if (!cic_cell(g, A.n, x[p], y[p], z[p], ic, w)) continue;
            if (b == 0) ++in0;
            const double pm = m[p];
            const int lx = ic[0] - wx, ly = ic[1] - wy, lz = ic[2] - wz;
            const bool inwin = lx >= 0 && lx < kWinX - 1 && ly >= 0 && ly < kWinY - 1 && lz >= 0 && lz < kWinZ - 1;
            for (int c = 0; c < 2; ++c)
                for (int bb = 0; bb < 2; ++bb)
                    for (int a = 0; a < 2; ++a) {
                        const double wt = (w[0][a] * w[1][bb]) * w[2][c];
                        const unsigned long long qv = (unsigned long long)__double2ll_rn((wt * pm) * A.scale);
                        if (inwin) atomicAdd(&W[(lx + a) + kWinX * ((ly + bb) + kWinY * (lz + c))], qv);
                        else atomicAdd(q + id3(A.n, ic[0] + a, ic[1] + bb, ic[2] + c), qv);
                    }
        }
        __syncthreads();
        unsigned long long *slab = A.scratch + ((size_t)blockIdx.x * A.nbox + b) * kWin;
        for (int e = threadIdx.x; e < kWin; e += kDepositThreads) slab[e] = W[e];
        __syncthreads();
    }
    // particles inside the outermost box: one LDS and one global add per workgroup
    atomicAdd(&cnt_sh, in0);
    __syncthreads();
    if (threadIdx.x == 0 && cnt_sh) atomicAdd(inside_count, (unsigned long long)cnt_sh);
}

__global__ void __launch_bounds__(256)
deposit_reduce_k(DepositArgs A, int nblocks)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (e >= kWin) return;
    const int li = e % kWinX, lj = (e / kWinX) % kWinY, lk = e / (kWinX * kWinY);
    const int i = A.w0[b][0] + li, j = A.w0[b][1] + lj, k = A.w0[b][2] + lk;
    if (i >= A.n || j >= A.n || k >= A.n) return;
    // four independent integer sums keep four slab loads in flight (any order gives the same sum)
    unsigned long long s0 = 0ULL, s1 = 0ULL, s2 = 0ULL, s3 = 0ULL;
    const size_t st = (size_t)A.nbox * kWin;
    const unsigned long long *src = A.scratch + (size_t)b * kWin + e;
    int g = 0;
    for (; g + 4 <= nblocks; g += 4) {
        s0 += src[(size_t)g * st];
        s1 += src[(size_t)(g + 1) * st];
        s2 += src[(size_t)(g + 2) * st];
        s3 += src[(size_t)(g + 3) * st];
    }
    for (; g < nblocks; ++g) s0 += src[(size_t)g * st];
    const unsigned long long s = (s0 + s1) + (s2 + s3);
    if (s) A.q[b][id3(A.n, i, j, k)] += s;
}

size_t deposit_scratch_bytes(int nbox) { return (size_t)kDepositMaxBlocks * nbox * kWin * sizeof(unsigned long long); }

void launch_deposit(const DepositArgs &a, const double *x, const double *y, const double *z, const double *m,
                    int64_t np, unsigned long long *inside_count, hipStream_t s)
{
    if (np <= 0) return;
    int64_t blocks = (np + kDepositThreads - 1) / kDepositThreads;
    if (blocks > kDepositMaxBlocks) blocks = kDepositMaxBlocks;
    const int64_t per_block = (np + blocks - 1) / blocks;
    hipLaunchKernelGGL(deposit_window_k, dim3((unsigned)blocks), dim3(kDepositThreads), 0, s, a, x, y, z, m, np,
                       per_block, inside_count);
    hipLaunchKernelGGL(deposit_reduce_k, dim3((kWin + 255) / 256, a.nbox), dim3(256), 0, s, a, (int)blocks);
}

// Batched single-box deposit: workgroup (g, p) takes a contiguous share of
// problem p's particles, with the same LDS window, scratch slabs and integer
// adds as above; problem p's grid starts at q + p n^3.
__global__ void __launch_bounds__(kDepositThreads)
deposit_batch_k(int n, BoxGeom g, int wx, int wy, int wz, const BatchProblem *__restrict__ prob,
                unsigned long long *__restrict__ qall, unsigned long long *__restrict__ scratch,
                unsigned long long *__restrict__ inside)
{
#pragma clang fp contract(off)
    __shared__ unsigned long long W[kWin];
    __shared__ unsigned int cnt_sh;
    const int pb = blockIdx.y;
    const BatchProblem P = prob[pb];
    const int64_t per_block = (P.np + kBatchDepositBlocks - 1) / kBatchDepositBlocks;
    const int64_t p0 = (int64_t)blockIdx.x * per_block;
    const int64_t p1 = min((int64_t)P.np, p0 + per_block);
    unsigned long long *q = qall + (size_t)pb * n * n * n;
    if (threadIdx.x == 0) cnt_sh = 0;
    for (int e = threadIdx.x; e < kWin; e += kDepositThreads) W[e] = 0ULL;
    __syncthreads();
    unsigned int in0 = 0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += kDepositThreads) {
        int ic[3];
        double w[3][2];
        if (!cic_cell(g, n, P.x[p], P.y[p], P.z[p], ic, w)) continue;
        ++in0;
        const double pm = P.m[p];
        const int lx = ic[0] - wx, ly = ic[1] - wy, lz = ic[2] - wz;
        const bool inwin = lx >= 0 && lx < kWinX - 1 && ly >= 0 && ly < kWinY - 1 && lz >= 0 && lz < kWinZ - 1;
        for (int c = 0; c < 2; ++c)
            for (int bb = 0; bb < 2; ++bb)
                for (int a = 0; a < 2; ++a) {
                    const double wt = (w[0][a] * w[1][bb]) * w[2][c];
                    const unsigned long long qv = (unsigned long long)__double2ll_rn((wt * pm) * P.scale);
                    if (inwin) atomicAdd(&W[(lx + a) + kWinX * ((ly + bb) + kWinY * (lz + c))], qv);
                    else atomicAdd(q + id3(n, ic[0] + a, ic[1] + bb, ic[2] + c), qv);
                }
    }
    __syncthreads();
    unsigned long long *slab = scratch + ((size_t)pb * kBatchDepositBlocks + blockIdx.x) * kWin;
    for (int e = threadIdx.x; e < kWin; e += kDepositThreads) slab[e] = W[e];
    atomicAdd(&cnt_sh, in0);
    __syncthreads();
    if (threadIdx.x == 0 && cnt_sh) atomicAdd(inside + pb, (unsigned long long)cnt_sh);
}

__global__ void __launch_bounds__(256)
deposit_batch_reduce_k(int n, int wx, int wy, int wz, unsigned long long *__restrict__ qall,
                       const unsigned long long *__restrict__ scratch)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int pb = blockIdx.y;
    if (e >= kWin) return;
    const int li = e % kWinX, lj = (e / kWinX) % kWinY, lk = e / (kWinX * kWinY);
    const int i = wx + li, j = wy + lj, k = wz + lk;
    if (i >= n || j >= n || k >= n) return;
    unsigned long long s = 0ULL;
    for (int g = 0; g < kBatchDepositBlocks; ++g) s += scratch[((size_t)pb * kBatchDepositBlocks + g) * kWin + e];
    if (s) qall[(size_t)pb * n * n * n + id3(n, i, j, k)] += s;
}

size_t deposit_batch_scratch_bytes(int nb)
{
    return (size_t)nb * kBatchDepositBlocks * kWin * sizeof(unsigned long long);
}

void launch_deposit_batch(int n, double L, const BatchProblem *prob, long long maxnp, unsigned long long *q,
                          unsigned long long *scratch, unsigned long long *inside, int nb, hipStream_t s)
{
    (void)maxnp;
    BoxGeom g;
    g.L = L;
    g.xmin = -0.5 * L;
    g.inv_h = (double)(n - 1) / L;
    g.h = L / (double)(n - 1);
    const int win[3] = {kWinX, kWinY, kWinZ};
    int w0[3];
    for (int d = 0; d < 3; ++d) {
        const int o = (n - 1) / 2 - win[d] / 2;
        w0[d] = o < 0 ? 0 : o;
    }
    hipLaunchKernelGGL(deposit_batch_k, dim3(kBatchDepositBlocks, nb), dim3(kDepositThreads), 0, s, n, g, w0[0], w0[1],
                       w0[2], prob, q, scratch, inside);
    hipLaunchKernelGGL(deposit_batch_reduce_k, dim3((kWin + 255) / 256, nb), dim3(256), 0, s, n, w0[0], w0[1], w0[2], q,
                       scratch);
}

__global__ void rhs_from_q_k(size_t count, double inv_h3, double four_pi_G, int shift, const long long *__restrict__ q,
                             double *__restrict__ f)
{
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x) {
        const double rho = ldexp((double)q[t], -shift) * inv_h3;
        f[t] = four_pi_G * rho;
    }
}

void launch_rhs_from_q(int n, double h, double four_pi_G, int shift, const long long *q, double *f, hipStream_t s)
{
    const size_t count = (size_t)n * n * n;
    size_t blocks = (count + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(rhs_from_q_k, dim3((unsigned)blocks), dim3(256), 0, s, count, 1.0 / (h * h * h), four_pi_G,
                       shift, q, f);
}

// Problem blockIdx.y; q and f may alias (each element is read before it is written).
__global__ void rhs_batch_k(size_t count, double inv_h3, double four_pi_G, const BatchProblem *__restrict__ prob,
                            const long long *q, double *f)
{
    const int shift = prob[blockIdx.y].shift;
    q += blockIdx.y * count;
    f += blockIdx.y * count;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x) {
        const double rho = ldexp((double)q[t], -shift) * inv_h3;
        f[t] = four_pi_G * rho;
    }
}

void launch_rhs_batch(int n, double h, double four_pi_G, const BatchProblem *prob, const long long *q, double *f, int nb,
                      hipStream_t s)
{
    const size_t count = (size_t)n * n * n;
    size_t blocks = (count + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(rhs_batch_k, dim3((unsigned)blocks, nb), dim3(256), 0, s, count, 1.0 / (h * h * h), four_pi_G,
                       prob, q, f);
}

// ------------------------------------------------------------------- gather
//
// The gather arithmetic is written out with contraction off, so that every
// kernel that inlines it (forces, curves, batched curves) rounds the same way.

// -d Phi / d x_d at node (i,j,k): central difference inside, one-sided second
// order on the faces.
__device__ __forceinline__ double node_accel(const double *__restrict__ P, int n, double inv2h, int i, int j, int k, int d)
{
#pragma clang fp contract(off)
    const size_t st = d == 0 ? 1 : (d == 1 ? (size_t)n : (size_t)n * n);
    const int c = d == 0 ? i : (d == 1 ? j : k);
    const size_t p = id3(n, i, j, k);
    double g;
    if (c > 0 && c < n - 1) g = P[p + st] - P[p - st];
    else if (c == 0) g = -3.0 * P[p] + 4.0 * P[p + st] - P[p + 2 * st];
    else g = 3.0 * P[p] - 4.0 * P[p - st] + P[p - 2 * st];
    return -g * inv2h;
}

// nu(y) with y = g / a0 (g > 0, a0 > 0): Eq. 2's function for nun == 1, else the n-family.
__device__ __forceinline__ double nu_of_g(double g, double a0, double nun)
{
#pragma clang fp contract(off)
    return nun == 1.0 ? 0.5 + 0.5 * sqrt(1.0 + 4.0 * a0 / g) : nu_family(g / a0, nun);
}

// Point-mass force (QUMOND: nu(g_N/a0) g_N) for points outside every box.
__device__ __forceinline__ void monopole_accel(double GM, double a0, int mond, double nun, double px, double py,
                                               double pz, double acc[3])
{
#pragma clang fp contract(off)
    const double r = sqrt(px * px + py * py + pz * pz);
    double g = 0.0;
    if (r > 0.0) {
        const double gN = GM / (r * r);
        g = (mond && a0 > 0.0 && gN > 0.0) ? nu_of_g(gN, a0, nun) * gN : gN;
        g /= r;
    }
    acc[0] = -g * px;
    acc[1] = -g * py;
    acc[2] = -g * pz;
}

__device__ __forceinline__ bool in_box(const BoxGeom &G, int n, double px, double py, double pz)
{
    const double top = (double)(n - 1);
    const double ux = (px - G.xmin) * G.inv_h, uy = (py - G.xmin) * G.inv_h, uz = (pz - G.xmin) * G.inv_h;
    return ux >= 0.0 && ux < top && uy >= 0.0 && uy < top && uz >= 0.0 && uz < top;
}

// Cloud-in-cell interpolation of the nodal accelerations of box G.
__device__ void box_accel(const BoxGeom &G, int n, const double *__restrict__ P, double px, double py, double pz,
                          double acc[3])
{
#pragma clang fp contract(off)
    const double u[3] = {(px - G.xmin) * G.inv_h, (py - G.xmin) * G.inv_h, (pz - G.xmin) * G.inv_h};
    int ic[3];
    double w[3][2];
    for (int d = 0; d < 3; ++d) {
        const double fl = floor(u[d]);
        ic[d] = (int)fl;
        const double fr = u[d] - fl;
        w[d][0] = 1.0 - fr;
        w[d][1] = fr;
    }
    const double inv2h = 0.5 * G.inv_h;
    acc[0] = acc[1] = acc[2] = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const double wt = (w[0][a] * w[1][b]) * w[2][c];
                for (int d = 0; d < 3; ++d) acc[d] += wt * node_accel(P, n, inv2h, ic[0] + a, ic[1] + b, ic[2] + c, d);
            }
}

// Eq. 3, the algebraic MOND relation: g = nu(|g_N| / a0) g_N at the point.
__device__ __forceinline__ void algebraic_mond(double a0, double nun, double acc[3])
{
#pragma clang fp contract(off)
    const double g = sqrt(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]);
    if (g > 0.0 && a0 > 0.0) {
        const double k = nu_of_g(g, a0, nun);
        acc[0] *= k;
        acc[1] *= k;
        acc[2] *= k;
    }
}

__device__ int gather_point(const GatherArgs &A, double px, double py, double pz, double acc[3])
{
#pragma clang fp contract(off)
    const double R = sqrt(px * px + py * py), az = fabs(pz);
    int sel = -1;
    for (int b = A.nbox - 1; b >= 0; --b)
        if (R < A.frac * A.box[b].L && az < A.frac * A.box[b].L) { sel = b; break; }
    if (sel < 0) {
        for (int b = 0; b < A.nbox; ++b)
            if (in_box(A.box[b], A.n, px, py, pz)) { sel = b; break; }
    }
    if (sel < 0) monopole_accel(A.GM, A.a0, A.mond, A.nun, px, py, pz, acc);
    else box_accel(A.box[sel], A.n, A.phi[sel], px, py, pz, acc);
    if (A.alg) algebraic_mond(A.a0, A.nun, acc);
    return sel < 0 ? 255 : sel;
}

__global__ void __launch_bounds__(256)
gather_k(GatherArgs A, const double *__restrict__ x, const double *__restrict__ y, const double *__restrict__ z,
         int64_t np, double *__restrict__ ax, double *__restrict__ ay, double *__restrict__ az, uint8_t *__restrict__ used)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= np) return;
    double acc[3];
    const int sel = gather_point(A, x[p], y[p], z[p], acc);
    ax[p] = acc[0];
    ay[p] = acc[1];
    az[p] = acc[2];
    if (used) used[p] = (uint8_t)sel;
}

void launch_gather(const GatherArgs &a, const double *x, const double *y, const double *z, int64_t np, double *ax,
                   double *ay, double *az, uint8_t *box_used, hipStream_t s)
{
    if (np <= 0) return;
    const int64_t blocks = (np + 255) / 256;
    hipLaunchKernelGGL(gather_k, dim3((unsigned)blocks), dim3(256), 0, s, a, x, y, z, np, ax, ay, az, box_used);
}

// Eq. 4 on the midplane: one workgroup per radius, azimuths phi_k = 2 pi k / naz,
// v_c^2 = -(x a_x + y a_y) averaged in a fixed order.
__global__ void __launch_bounds__(256)
rotation_curve_k(GatherArgs A, const double *__restrict__ R, int naz, double *__restrict__ vc2)
{
#pragma clang fp contract(off)
    __shared__ double sh[256];
    const double r = R[blockIdx.x];
    double s = 0.0;
    for (int k = threadIdx.x; k < naz; k += 256) {
        const double phi = 2.0 * M_PI * (double)k / (double)naz;
        const double px = r * cos(phi), py = r * sin(phi);
        double acc[3];
        gather_point(A, px, py, 0.0, acc);
        s += -(px * acc[0] + py * acc[1]);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) vc2[blockIdx.x] = sh[0] / (double)naz;
}

void launch_rotation_curve(const GatherArgs &a, const double *R, int nR, int naz, double *vc2, hipStream_t s)
{
    if (nR <= 0) return;
    hipLaunchKernelGGL(rotation_curve_k, dim3(nR), dim3(256), 0, s, a, R, naz, vc2);
}

// Eq. 5 for stars with a sech^2(z / z0) vertical profile at every radius:
// rho / d_z rho = -z0 / (2 tanh(z / z0)), so sigma_z^2 = -a_z z0 / (2 tanh(z / z0)).
// One workgroup per radius; samples k < naz at (R cos phi_k, R sin phi_k, +z),
// k >= naz at the same azimuths and -z, averaged in a fixed order.
__global__ void __launch_bounds__(256)
sigma_z_k(GatherArgs A, const double *__restrict__ R, int naz, double z, double z0, double *__restrict__ sig2)
{
#pragma clang fp contract(off)
    __shared__ double sh[256];
    const double r = R[blockIdx.x];
    const double c = z0 / (2.0 * tanh(z / z0));
    double s = 0.0;
    for (int k = threadIdx.x; k < 2 * naz; k += 256) {
        const bool up = k < naz;
        const int ka = up ? k : k - naz;
        const double phi = 2.0 * M_PI * (double)ka / (double)naz;
        const double px = r * cos(phi), py = r * sin(phi);
        double acc[3];
        gather_point(A, px, py, up ? z : -z, acc);
        s += up ? -acc[2] * c : acc[2] * c;  // tanh is odd
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sig2[blockIdx.x] = sh[0] / (double)(2 * naz);
}

void launch_sigma_z(const GatherArgs &a, const double *R, int nR, int naz, double z, double z0, double *sig2,
                    hipStream_t s)
{
    if (nR <= 0) return;
    hipLaunchKernelGGL(sigma_z_k, dim3(nR), dim3(256), 0, s, a, R, naz, z, z0, sig2);
}

// Batched single-box curves: workgroup (r, p), same sampling and order as rotation_curve_k.
__global__ void __launch_bounds__(256)
rotation_curve_batch_k(int n, BoxGeom G, double frac, double Gc, double a0, int mond, double nun,
                       const BatchProblem *__restrict__ prob, const double *__restrict__ phi, const double *__restrict__ R,
                       int nR, int naz, double *__restrict__ vc2)
{
#pragma clang fp contract(off)
    __shared__ double sh[256];
    const int pb = blockIdx.y;
    const double *P = phi + (size_t)pb * n * n * n;
    const double GM = Gc * prob[pb].mass;
    const double r = R[blockIdx.x];
    double s = 0.0;
    for (int k = threadIdx.x; k < naz; k += 256) {
        const double ph = 2.0 * M_PI * (double)k / (double)naz;
        const double px = r * cos(ph), py = r * sin(ph);
        double acc[3];
        // the box-choice rule of gather_point with one box
        const double Rp = sqrt(px * px + py * py);
        if ((Rp < frac * G.L && 0.0 < frac * G.L) || in_box(G, n, px, py, 0.0)) box_accel(G, n, P, px, py, 0.0, acc);
        else monopole_accel(GM, a0, mond, nun, px, py, 0.0, acc);
        s += -(px * acc[0] + py * acc[1]);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) vc2[(size_t)pb * nR + blockIdx.x] = sh[0] / (double)naz;
}

void launch_rotation_curve_batch(int n, double L, double frac, double G, double a0, int mond,
                                 const BatchProblem *prob, const double *phi, const double *R, int nR, int naz,
                                 double *vc2, int nb, hipStream_t s, double nun)
{
    if (nR <= 0 || nb <= 0) return;
    BoxGeom g;
    g.L = L;
    g.xmin = -0.5 * L;
    g.inv_h = (double)(n - 1) / L;
    g.h = L / (double)(n - 1);
    hipLaunchKernelGGL(rotation_curve_batch_k, dim3(nR, nb), dim3(256), 0, s, n, g, frac, G, a0, mond, nun, prob, phi,
                       R, nR, naz, vc2);
}

}  // namespace qm
