// Right-hand side of Eq. 2 (Angus et al., Sec. 2, step 3):
// S = div[nu(|grad Phi_N|/a0) grad Phi_N], nu(y) = 1/2 + 1/2 sqrt(1 + 4/y),
// by a conservative face-flux difference in FP64.  On the face between node
// p and q = p + e_d: normal gradient (Phi_q - Phi_p)/h, each transverse
// component the mean of the central differences at p and q, flux
// F = nu(|g|/a0) g_n = g_n (1 + sqrt(1 + 4 a0/|g|)) / 2 (0 where |g| = 0, the
// limit of nu g), and S(p) = sum_d (F(p + e_d/2) - F(p - e_d/2)) / h.
// Batches of problems stored back to back are covered by the z block index.
// With another member of the n-family of interpolating functions (nun != 1)
// the flux is nu_n(|g|/a0) g_n.
#include "common.h"

namespace qm {

__device__ __forceinline__ double face_flux(const double *__restrict__ P, size_t p, size_t sd, size_t s1, size_t s2,
                                            double ih, double a0, double nun)
{
    const size_t q = p + sd;
    const double gn = (P[q] - P[p]) * ih;
    const double g1 = (P[p + s1] + P[q + s1] - P[p - s1] - P[q - s1]) * (0.25 * ih);
    const double g2 = (P[p + s2] + P[q + s2] - P[p - s2] - P[q - s2]) * (0.25 * ih);
    const double g = sqrt(gn * gn + g1 * g1 + g2 * g2);
    if (!(g > 0.0)) return 0.0;
    if (nun == 1.0) return 0.5 * gn * (1.0 + sqrt(1.0 + 4.0 * a0 / g));
    return gn * nu_family(g / a0, nun);
}

__global__ void __launch_bounds__(256)
mond_source_k(int n, double ih, double a0, double nun, const double *__restrict__ P, double *__restrict__ S, int zb)
{
    const int pb = blockIdx.z / zb;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = (blockIdx.z - pb * zb) * blockDim.z + threadIdx.z;
    if (i >= n || j >= n || k >= n) return;
    P += pb * (size_t)n * n * n;
    S += pb * (size_t)n * n * n;
    const size_t p = id3(n, i, j, k);
    if (i == 0 || j == 0 || k == 0 || i == n - 1 || j == n - 1 || k == n - 1) {
        S[p] = 0.0;
        return;
    }
    const size_t sx = 1, sy = (size_t)n, sz = (size_t)n * n;
    double s = face_flux(P, p, sx, sy, sz, ih, a0, nun) - face_flux(P, p - sx, sx, sy, sz, ih, a0, nun);
    s += face_flux(P, p, sy, sx, sz, ih, a0, nun) - face_flux(P, p - sy, sy, sx, sz, ih, a0, nun);
    s += face_flux(P, p, sz, sx, sy, ih, a0, nun) - face_flux(P, p - sz, sz, sx, sy, ih, a0, nun);
    S[p] = s * ih;
}

void launch_mond_source(int n, double h, double a0, const double *phin, double *S, hipStream_t s, int nb, double nun)
{
    dim3 blk(64, 2, 2);
    const int zb = (n + 1) / 2;
    dim3 grid((n + 63) / 64, (n + 1) / 2, zb * nb);
    hipLaunchKernelGGL(mond_source_k, grid, blk, 0, s, n, 1.0 / h, a0, nun, phin, S, zb);
}

}  // namespace qm
