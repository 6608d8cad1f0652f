// Dirichlet boundary values (Sec. 2, nested refinement of Angus et al.).
//
// The outermost box carries either zero (the paper's box 2^10 times the
// galaxy) or the monopole of the total mass: -G M / r for the Newtonian
// potential, and for the QUMOND potential the radial integral of
// nu(g_N/a0) g_N with g_N = G M / r^2,
//   -GM/(2r) - sqrt(GM) sqrt(GM + 4 a0 r^2)/(2r) + sqrt(GM a0) asinh(2 r sqrt(a0/GM)),
// which tends to -GM/r at small r and reduces to it for a0 = 0.  With another
// member of the n-family of interpolating functions the same integral is
// -GM/r + sqrt(GM a0) I(r / r_M), r_M = sqrt(GM / a0), I from the table of
// build_nu_table (below: composite Simpson in u = ln s on each table step).
// An inner box has half the side of the coarser one and the same n, so its
// node i lies at coarse coordinate (n-1)/4 + i/2: on a coarse node for even
// i, halfway between two for odd i; the boundary value is the trilinear
// interpolant of the coarser box's solution, with weights 1 or 1/2.
#include <cmath>

#include "common.h"

namespace qm {

__device__ __forceinline__ void bface_node(int n, int t, int &i, int &j, int &k)
{
    const int nn = n * n;
    const int face = t / nn, r = t - face * nn;
    const int a = r % n, b = r / n;
    switch (face) {
    case 0: i = 0; j = a; k = b; break;
    case 1: i = n - 1; j = a; k = b; break;
    case 2: j = 0; i = a; k = b; break;
    case 3: j = n - 1; i = a; k = b; break;
    case 4: k = 0; i = a; j = b; break;
    default: k = n - 1; i = a; j = b; break;
    }
}

// dI/du at u = ln s for the n-family member n: (nu_n(1/s^2) - 1) / s, with
// nu_n - 1 = expm1(log1p(q) / n), q = 2 w / (1 + sqrt(1 + 4 w)), w = s^(2n)
// (no cancellation at small s).
static double nu_point_slope(double u, double n)
{
    const double w = std::exp(2.0 * n * u);
    const double q = 2.0 * w / (1.0 + std::sqrt(1.0 + 4.0 * w));
    return std::expm1(std::log1p(q) / n) * std::exp(-u);
}

void build_nu_table(double n, double *tab)
{
    const double t0 = std::exp(kNuU0);
    double I = std::pow(t0, 2.0 * n - 1.0) / (n * (2.0 * n - 1.0));
    const int m = 32;  // Simpson sub-intervals per table step
    for (int k = 0; k < kNuTab; ++k) {
        const double u = kNuU0 + k * kNuDu;
        tab[2 * k] = I;
        tab[2 * k + 1] = nu_point_slope(u, n);
        if (k + 1 == kNuTab) break;
        const double d = kNuDu / m;
        double acc = nu_point_slope(u, n) + nu_point_slope(u + kNuDu, n);
        for (int j = 1; j < m; ++j) acc += (j & 1 ? 4.0 : 2.0) * nu_point_slope(u + j * d, n);
        I += acc * d / 3.0;
    }
}

__device__ __forceinline__ double monopole_value(int mode, double GM, double a0, double r, const NuFn &nu)
{
    double v = 0.0;
    if (mode == 1) {
        v = -GM / r;
    } else if (mode == 2 && nu.n != 1.0) {
        v = -GM / r;
        if (a0 > 0.0 && GM > 0.0) v += sqrt(GM * a0) * nu_point_integral(nu, r / sqrt(GM / a0));
    } else if (mode == 2) {
        v = -GM / (2.0 * r) - sqrt(GM) * sqrt(GM + 4.0 * a0 * r * r) / (2.0 * r) + sqrt(GM * a0) * asinh(2.0 * r * sqrt(a0 / GM));
    }
    return v;
}

__device__ __forceinline__ double bc_outer_value(int n, double L, int mode, double GM, double a0, int i, int j, int k,
                                                 const NuFn &nu)
{
    const double h = L / (double)(n - 1);
    const double x = -0.5 * L + i * h, y = -0.5 * L + j * h, z = -0.5 * L + k * h;
    return monopole_value(mode, GM, a0, sqrt(x * x + y * y + z * z), nu);
}

// The monopole potential at every node with r softened to sqrt(r^2 + soft^2)
// (finite at the centre); GM = 0 gives zero.
__global__ void monopole_field_k(int n, double L, int mode, double GM, double a0, double soft2, double *__restrict__ out)
{
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t N = (size_t)n * n * n;
    if (t >= N) return;
    const int i = (int)(t % n), j = (int)((t / n) % n), k = (int)(t / ((size_t)n * n));
    const double h = L / (double)(n - 1);
    const double x = -0.5 * L + i * h, y = -0.5 * L + j * h, z = -0.5 * L + k * h;
    out[t] = GM > 0.0 ? monopole_value(mode, GM, a0, sqrt(x * x + y * y + z * z + soft2), NuFn()) : 0.0;
}

void launch_monopole_field(int n, double L, int mode, double GM, double a0, double soft, double *out, hipStream_t s)
{
    const size_t N = (size_t)n * n * n;
    hipLaunchKernelGGL(monopole_field_k, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, n, L, mode, GM, a0,
                       soft * soft, out);
}

__global__ void bc_outer_k(int n, double L, int mode, double GM, double a0, NuFn nu, double *__restrict__ u0,
                           double *__restrict__ u1)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * n * n) return;
    int i, j, k;
    bface_node(n, t, i, j, k);
    const double v = bc_outer_value(n, L, mode, GM, a0, i, j, k, nu);
    const size_t p = id3(n, i, j, k);
    u0[p] = v;
    if (u1) u1[p] = v;
}

// problem blockIdx.y of a batch, GM = G M_p
__global__ void bc_outer_batch_k(int n, double L, int mode, double G, double a0, NuFn nu,
                                 const BatchProblem *__restrict__ prob, double *__restrict__ u0)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * n * n) return;
    int i, j, k;
    bface_node(n, t, i, j, k);
    const double GM = G * prob[blockIdx.y].mass;
    u0[id3(n, i, j, k) + blockIdx.y * (size_t)n * n * n] = bc_outer_value(n, L, mode, GM, a0, i, j, k, nu);
}

void launch_bc_outer(int n, double L, int mode, double GM, double a0, double *u0, double *u1, hipStream_t s,
                     const NuFn &nu)
{
    const int cnt = 6 * n * n;
    hipLaunchKernelGGL(bc_outer_k, dim3((cnt + 255) / 256), dim3(256), 0, s, n, L, mode, GM, a0, nu, u0, u1);
}

void launch_bc_outer_batch(int n, double L, int mode, double G, double a0, const BatchProblem *prob, double *u0,
                           int nb, hipStream_t s, const NuFn &nu)
{
    const int cnt = 6 * n * n;
    hipLaunchKernelGGL(bc_outer_batch_k, dim3((cnt + 255) / 256, nb), dim3(256), 0, s, n, L, mode, G, a0, nu, prob,
                       u0);
}

__global__ void bc_from_coarse_k(int n, const double *__restrict__ uc, double *__restrict__ u0, double *__restrict__ u1)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * n * n) return;
    int i, j, k;
    bface_node(n, t, i, j, k);
    const int off = (n - 1) / 4;
    const int ia = off + (i >> 1), ib = off + ((i + 1) >> 1);
    const int ja = off + (j >> 1), jb = off + ((j + 1) >> 1);
    const int ka = off + (k >> 1), kb = off + ((k + 1) >> 1);
    const double wia = (i & 1) ? 0.5 : 1.0, wib = (i & 1) ? 0.5 : 0.0;
    const double wja = (j & 1) ? 0.5 : 1.0, wjb = (j & 1) ? 0.5 : 0.0;
    const double wka = (k & 1) ? 0.5 : 1.0, wkb = (k & 1) ? 0.5 : 0.0;
    const double xa = wia * uc[id3(n, ia, ja, ka)] + wib * uc[id3(n, ib, ja, ka)];
    const double xb = wia * uc[id3(n, ia, jb, ka)] + wib * uc[id3(n, ib, jb, ka)];
    const double xc = wia * uc[id3(n, ia, ja, kb)] + wib * uc[id3(n, ib, ja, kb)];
    const double xd = wia * uc[id3(n, ia, jb, kb)] + wib * uc[id3(n, ib, jb, kb)];
    const double v = wka * (wja * xa + wjb * xb) + wkb * (wja * xc + wjb * xd);
    const size_t p = id3(n, i, j, k);
    u0[p] = v;
    if (u1) u1[p] = v;
}

void launch_bc_from_coarse(int n, const double *uc, double *u0, double *u1, hipStream_t s)
{
    const int cnt = 6 * n * n;
    hipLaunchKernelGGL(bc_from_coarse_k, dim3((cnt + 255) / 256), dim3(256), 0, s, n, uc, u0, u1);
}

}  // namespace qm
