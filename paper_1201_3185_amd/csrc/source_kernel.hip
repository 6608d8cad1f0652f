// Right-hand side of Eq. 2 (Angus et al., Sec. 2, step 3):
// S = div[nu(|grad Phi_N|/a0) grad Phi_N], nu(y) = 1/2 + 1/2 sqrt(1 + 4/y),
// by a conservative face-flux difference in FP64.  On the face between node
// p and q = p + e_d: normal gradient (Phi_q - Phi_p)/h, each transverse
// component the mean of the central differences at p and q, flux
// F = nu(|g|/a0) g_n = g_n (1 + sqrt(1 + 4 a0/|g|)) / 2 (0 where |g| = 0, the
// limit of nu g), and S(p) = sum_d (F(p + e_d/2) - F(p - e_d/2)) / h.
// With another member of the n-family of interpolating functions (nun != 1)
// the flux is nu_n(|g|/a0) g_n.
//
// Kernel design.  The face fluxes are the work: each needs |g| and
// sqrt(1 + 4 a0/|g|), formed from the hardware reciprocal square root refined
// by Newton-Raphson steps (a few ulp, no correctly rounded square root or
// division), and each face borders two nodes, so the kernel computes each
// flux once.  A
// workgroup owns a TX x TY column tile of interior nodes and marches up a
// chunk of z planes, holding three planes of Phi_N (k-1, k, k+1; tile plus a
// one-node ring) in LDS.  On plane k every lane forms the +x, +y and +z face
// fluxes of its node; the first wavefront also forms the -x faces of the
// tile's first column and the -y faces of its first row.  The x and y fluxes
// go through LDS to the neighbour that needs them as its minus face, the +z
// flux stays in the lane's registers as the -z flux of the next plane.  The
// next plane is loaded into registers while a plane is computed.  Every
// flux is the expression of the single-node formula above, so a face's flux
// is the same number whichever node's difference uses it.  Boundary nodes of
// S are set to 0 by a separate launch over the six faces.  Batches of
// problems stored back to back are covered by the slowest part of the block
// index.
#include "common.h"

namespace qm {

namespace {

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton-Raphson
// steps for f(y) = 1/y^2 - x, y <- y + y (1 - x y^2) / 2 (each step squares
// the relative error, so two steps take any estimate within 1e-4 to a few
// units in the last place).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-(x * y), y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

template <bool FAMILY>
__device__ __forceinline__ double face_flux(double pp, double pq, double t1, double t2, double ih, double a0,
                                            double nun)
{
    // pp, pq: Phi_N at the face's two nodes; t1, t2: the transverse sums
    // Phi(p+e) + Phi(q+e) - Phi(p-e) - Phi(q-e) along the two other axes.
    // Contraction off: every inlined copy rounds alike, so the two nodes of a
    // face see the same flux.
#pragma clang fp contract(off)
    const double gn = (pq - pp) * ih;
    const double g1 = t1 * (0.25 * ih);
    const double g2 = t2 * (0.25 * ih);
    const double G2 = gn * gn + g1 * g1 + g2 * g2;
    if (!(G2 > 0.0)) return 0.0;
    if (!FAMILY) {
        // nu g_n = g_n (1 + sqrt(1 + 4 a0 / |g|)) / 2 with 1/|g| = 1/sqrt(G2)
        // and sqrt(x) = x / sqrt(x) plus one Newton correction (x >= 1 here)
        const double x = 1.0 + 4.0 * a0 * rsqrt_nr(G2);
        const double y = rsqrt_nr(x);
        double r = x * y;
        r = fma(0.5 * y, fma(-r, r, x), r);
        return 0.5 * gn * (1.0 + r);
    }
    return gn * nu_family(sqrt(G2) / a0, nun);
}

constexpr int kSrcTX = 32, kSrcTY = 8;
static_assert(kSrcTX + kSrcTY <= 64, "the ring faces fit in the first wavefront");

template <int TX, int TY, bool FAMILY>
__global__ void __launch_bounds__(TX *TY)
mond_source_zmarch(int n, double ih, double a0, double nun, const double *__restrict__ P, double *__restrict__ S,
                   int kchunk, int nzc)
{
    constexpr int PX = TX + 2, PY = TY + 2, PL = PX * PY, NT = TX * TY;
    constexpr int NL = (PL + NT - 1) / NT;   // plane values loaded per lane
    __shared__ double pl[3][PL];
    __shared__ double fx[TY][TX + 1];        // x faces: fx[b][a] between tile columns a-1 and a
    __shared__ double fy[TY + 1][TX];        // y faces: fy[b][a] between tile rows b-1 and b
    const int tid = threadIdx.x;
    const unsigned tl = xcd_tile(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
    const int bx = tl % gridDim.x, by = (tl / gridDim.x) % gridDim.y, bzz = tl / (gridDim.x * gridDim.y);
    const int i0 = 1 + bx * TX, j0 = 1 + by * TY;
    const int pb = bzz / nzc;
    const int kb = 1 + (bzz - pb * nzc) * kchunk;
    if (kb > n - 2) return;
    const int ke = min(kb + kchunk - 1, n - 2);
    const size_t nn = (size_t)n * n;
    P += (size_t)pb * nn * n;
    S += (size_t)pb * nn * n;

    // this lane's share of a plane (tile + one-node ring), offsets in the plane
    int goff[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int t = tid + r * NT;
        const int i = i0 - 1 + t % PX, j = j0 - 1 + t / PX;
        goff[r] = (t < PL && i < n && j < n) ? i + n * j : -1;
    }
    double v[NL];
    auto fetch = [&](int k) {   // plane k into registers (0 outside the grid)
        const double *src = P + (size_t)k * nn;
#pragma unroll
        for (int r = 0; r < NL; ++r) v[r] = goff[r] >= 0 ? src[goff[r]] : 0.0;
    };
    auto commit = [&](int k) {   // registers into the plane's LDS slot
        double *D = pl[k % 3];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t < PL) D[t] = v[r];
        }
    };

    // this lane's node (tile column a, row b) and, in the first wavefront, a ring face
    const int a = tid % TX, b = tid / TX;
    const int i = i0 + a, j = j0 + b;
    const bool own = i <= n - 2 && j <= n - 2;
    const int c = (b + 1) * PX + (a + 1);
    // lanes 0..TY-1: the -x face of tile row tid (between ring column 0 and
    // tile column 0); lanes TY..TY+TX-1: the -y face of tile column tid-TY;
    // cr is the face's minus node in the plane
    const bool ring_x = tid < TY && j0 + tid <= n - 2;
    const bool ring_y = tid >= TY && tid < TY + TX && i0 + (tid - TY) <= n - 2;
    const int cr = tid < TY ? (tid + 1) * PX : (tid - TY + 1);

    auto flux_x = [&](const double *M, const double *Z, const double *Q, int q) {   // face q -> q + 1
        return face_flux<FAMILY>(Z[q], Z[q + 1], Z[q + PX] + Z[q + 1 + PX] - Z[q - PX] - Z[q + 1 - PX],
                         Q[q] + Q[q + 1] - M[q] - M[q + 1], ih, a0, nun);
    };
    auto flux_y = [&](const double *M, const double *Z, const double *Q, int q) {   // face q -> q + PX
        return face_flux<FAMILY>(Z[q], Z[q + PX], Z[q + 1] + Z[q + PX + 1] - Z[q - 1] - Z[q + PX - 1],
                         Q[q] + Q[q + PX] - M[q] - M[q + PX], ih, a0, nun);
    };
    auto flux_z = [&](const double *Z, const double *Q, int q) {   // face plane Z -> plane Q
        return face_flux<FAMILY>(Z[q], Q[q], Z[q + 1] + Q[q + 1] - Z[q - 1] - Q[q - 1],
                         Z[q + PX] + Q[q + PX] - Z[q - PX] - Q[q - PX], ih, a0, nun);
    };

    // warm-up: planes kb-1, kb, kb+1 (all loads in flight before the first
    // LDS store), the -z flux of plane kb, plane kb+2 in flight
    {
        double w[3][NL];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double *src = P + (size_t)(kb - 1 + q) * nn;
#pragma unroll
            for (int r = 0; r < NL; ++r) w[q][r] = goff[r] >= 0 ? src[goff[r]] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double *D = pl[(kb - 1 + q) % 3];
#pragma unroll
            for (int r = 0; r < NL; ++r) {
                const int t = tid + r * NT;
                if (t < PL) D[t] = w[q][r];
            }
        }
    }
    __syncthreads();
    double fz_lo = own ? flux_z(pl[(kb - 1) % 3], pl[kb % 3], c) : 0.0;
    if (kb + 2 <= ke + 1) fetch(kb + 2);

    for (int k = kb; k <= ke; ++k) {
        const double *M = pl[(k - 1) % 3], *Z = pl[k % 3], *Q = pl[(k + 1) % 3];
        double fz_hi = 0.0;
        if (own) {
            fx[b][a + 1] = flux_x(M, Z, Q, c);
            fy[b + 1][a] = flux_y(M, Z, Q, c);
            fz_hi = flux_z(Z, Q, c);
        }
        if (ring_x) fx[tid][0] = flux_x(M, Z, Q, cr);
        if (ring_y) fy[0][tid - TY] = flux_y(M, Z, Q, cr);
        __syncthreads();
        if (own) {
            double s = fx[b][a + 1] - fx[b][a];
            s += fy[b + 1][a] - fy[b][a];
            s += fz_hi - fz_lo;
            S[(size_t)k * nn + i + (size_t)n * j] = s * ih;
        }
        fz_lo = fz_hi;
        if (k + 2 <= ke + 1) {   // plane k+2 replaces plane k-1, whose readers are past the barrier
            commit(k + 2);
            if (k + 3 <= ke + 1) fetch(k + 3);
        }
        __syncthreads();
    }
}

// S = 0 on the six faces of every problem's grid.
__global__ void __launch_bounds__(256) zero_faces_k(int n, double *__restrict__ S)
{
    const size_t nn = (size_t)n * n;
    S += (size_t)blockIdx.y * nn * n;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;   // index over 6 n^2 face nodes
    if (t >= 6 * n * n) return;
    const int f = t / (n * n), r = t % (n * n), u = r % n, w = r / n;
    const int e = (f & 1) ? n - 1 : 0;
    size_t p;
    if (f < 2) p = id3(n, e, u, w);
    else if (f < 4) p = id3(n, u, e, w);
    else p = id3(n, u, w, e);
    S[p] = 0.0;
}

}  // namespace

void launch_mond_source(int n, double h, double a0, const double *phin, double *S, hipStream_t s, int nb, double nun)
{
    const int m = n - 2;
    const int kchunk = n >= 513 ? 32 : (n >= 257 ? 16 : (n >= 129 ? 8 : 4));
    const int nzc = (m + kchunk - 1) / kchunk;
    dim3 grid((m + kSrcTX - 1) / kSrcTX, (m + kSrcTY - 1) / kSrcTY, nzc * nb);
    if (nun == 1.0)
        hipLaunchKernelGGL((mond_source_zmarch<kSrcTX, kSrcTY, false>), grid, dim3(kSrcTX * kSrcTY), 0, s, n, 1.0 / h,
                           a0, nun, phin, S, kchunk, nzc);
    else
        hipLaunchKernelGGL((mond_source_zmarch<kSrcTX, kSrcTY, true>), grid, dim3(kSrcTX * kSrcTY), 0, s, n, 1.0 / h,
                           a0, nun, phin, S, kchunk, nzc);
    hipLaunchKernelGGL(zero_faces_k, dim3((6 * n * n + 255) / 256, nb), dim3(256), 0, s, n, S);
}

}  // namespace qm
