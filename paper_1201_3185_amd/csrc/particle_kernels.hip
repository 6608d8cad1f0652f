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
    unsigned long long s = 0ULL;
    for (int g = 0; g < nblocks; ++g) s += A.scratch[((size_t)g * A.nbox + b) * kWin + e];
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

// ------------------------------------------------------------------- gather

// -d Phi / d x_d at node (i,j,k): central difference inside, one-sided second
// order on the faces.
__device__ __forceinline__ double node_accel(const double *__restrict__ P, int n, double inv2h, int i, int j, int k, int d)
{
    const size_t st = d == 0 ? 1 : (d == 1 ? (size_t)n : (size_t)n * n);
    const int c = d == 0 ? i : (d == 1 ? j : k);
    const size_t p = id3(n, i, j, k);
    double g;
    if (c > 0 && c < n - 1) g = P[p + st] - P[p - st];
    else if (c == 0) g = -3.0 * P[p] + 4.0 * P[p + st] - P[p + 2 * st];
    else g = 3.0 * P[p] - 4.0 * P[p - st] + P[p - 2 * st];
    return -g * inv2h;
}

__device__ int gather_point(const GatherArgs &A, double px, double py, double pz, double acc[3])
{
    const double R = sqrt(px * px + py * py), az = fabs(pz);
    int sel = -1;
    for (int b = A.nbox - 1; b >= 0; --b)
        if (R < A.frac * A.box[b].L && az < A.frac * A.box[b].L) { sel = b; break; }
    const double top = (double)(A.n - 1);
    if (sel < 0) {
        for (int b = 0; b < A.nbox; ++b) {
            const double ux = (px - A.box[b].xmin) * A.box[b].inv_h, uy = (py - A.box[b].xmin) * A.box[b].inv_h,
                         uz = (pz - A.box[b].xmin) * A.box[b].inv_h;
            if (ux >= 0.0 && ux < top && uy >= 0.0 && uy < top && uz >= 0.0 && uz < top) { sel = b; break; }
        }
    }
    if (sel < 0) {
        const double r = sqrt(px * px + py * py + pz * pz);
        double g = 0.0;
        if (r > 0.0) {
            const double gN = A.GM / (r * r);
            g = (A.mond && A.a0 > 0.0) ? (0.5 + 0.5 * sqrt(1.0 + 4.0 * A.a0 / gN)) * gN : gN;
            g /= r;
        }
        acc[0] = -g * px;
        acc[1] = -g * py;
        acc[2] = -g * pz;
        return 255;
    }
    const BoxGeom G = A.box[sel];
    const int n = A.n;
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
    const double *P = A.phi[sel];
    acc[0] = acc[1] = acc[2] = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const double wt = (w[0][a] * w[1][b]) * w[2][c];
                for (int d = 0; d < 3; ++d) acc[d] += wt * node_accel(P, n, inv2h, ic[0] + a, ic[1] + b, ic[2] + c, d);
            }
    return sel;
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

}  // namespace qm
