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
// by one Newton-Raphson step (relative error about 4e-15, no correctly
// rounded square root or division), with the constant factors of g and of the
// difference folded into one scale applied to S, and each face borders two
// nodes, so the kernel computes each flux once.  A
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

// 1/sqrt(x) for x > 0: the hardware estimate (v_rsq_f64, measured within
// 5.3e-8 relative on gfx950) refined by one Newton-Raphson step for
// f(y) = 1/y^2 - x, y <- y + y (1 - x y^2) / 2, which squares the relative
// error: about 1.5 (5.3e-8)^2 = 4e-15 (the same holds for the Newton step of
// the square root below).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(0.5 * y, e, y);
}

// The flux through one face scaled by 2h (F' = 2 h F), so that
// S(p) = (ih^2 / 2) sum_d (F'(p + e_d/2) - F'(p - e_d/2)).  With
// d = Phi_q - Phi_p and t1, t2 the transverse sums
// (Phi(p+e) - Phi(p-e)) + (Phi(q+e) - Phi(q-e)) along the two other axes,
// g = ih (d, t1/4, t2/4), so |g| = ih sqrt(A) / 4 with A = 16 d^2 + t1^2 + t2^2
// and 4 a0 / |g| = c16 / sqrt(A) with c16 = 16 a0 h; then
// F' = 2 nu g_n / ih = d (1 + sqrt(1 + c16 / sqrt(A))).  A = 0 only where
// d = t1 = t2 = 0, where the flux is 0 (the limit of nu g): DBL_MIN is added
// to A, which leaves every A above 2^53 DBL_MIN unchanged after rounding,
// keeps every step finite at A = 0 and gives 0 * finite there.
// Contraction off: every inlined copy rounds alike, so a face computed by two
// workgroups (a tile's ring face) has the same flux in both.
template <bool FAMILY>
__device__ __forceinline__ double face_flux(double pp, double pq, double t1, double t2, double h, double c16,
                                            double a0, double nun)
{
#pragma clang fp contract(off)
    const double d = pq - pp;
    const double d4 = 4.0 * d;
    if (!FAMILY) {
        const double A = fma(t2, t2, fma(t1, t1, fma(d4, d4, 2.2250738585072014e-308)));
        const double x = fma(c16, rsqrt_nr(A), 1.0);   // x >= 1
        // sqrt(x): r0 = x rsq(x), then one Newton step for r^2 = x,
        // r <- r0 + (x - r0^2) rsq(x) / 2 (relative error about 4e-15)
        const double y = __builtin_amdgcn_rsq(x);
        const double r0 = x * y;
        const double r = fma(0.5 * y, fma(-r0, r0, x), r0);
        return fma(d, r, d);
    }
    const double A = fma(t2, t2, fma(t1, t1, d4 * d4));
    if (!(A > 0.0)) return 0.0;
    return 2.0 * d * nu_family(sqrt(A) / (4.0 * h * a0), nun);
}

constexpr int kSrcTX = 32, kSrcTY = 16;
static_assert(kSrcTX + kSrcTY <= 64, "the ring faces fit in the first wavefront");

template <int TX, int TY, bool FAMILY>
__global__ void __launch_bounds__(TX *TY)
mond_source_zmarch(int n, double h, double a0, double nun, const double *__restrict__ P, double *__restrict__ S,
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
    const double ih = 1.0 / h, c16 = 16.0 * a0 * h, sscale = 0.5 * ih * ih;
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
    // tile column 0); lanes TY..TY+TX-1: the -y face of tile column tid-TY.
    // cr is the face's minus node in the plane, (rn, rt) its normal and
    // in-plane transverse strides, rdst where its flux goes; both kinds take
    // one pass of the same code.
    const bool ring = (tid < TY && j0 + tid <= n - 2) || (tid >= TY && tid < TY + TX && i0 + (tid - TY) <= n - 2);
    const int cr = tid < TY ? (tid + 1) * PX : (tid - TY + 1);
    const int rn = tid < TY ? 1 : PX, rt = tid < TY ? PX : 1;
    double *rdst = tid < TY ? &fx[tid][0] : &fy[0][min(max(tid - TY, 0), TX - 1)];

    // The transverse sums are sums of central differences at the face's two
    // nodes, each a difference of two plane values; a lane forms those of its
    // node once per plane and carries the x and y differences of plane k+1
    // to the next plane.  The ring faces form the same differences in the
    // same order, so they round alike.
    // flux through the face q -> q + sn of plane Z, st the other in-plane stride
    auto flux_xy = [&](const double *M, const double *Z, const double *Q, int q, int sn, int st) {
        return face_flux<FAMILY>(Z[q], Z[q + sn], (Z[q + st] - Z[q - st]) + (Z[q + sn + st] - Z[q + sn - st]),
                                 (Q[q] - M[q]) + (Q[q + sn] - M[q + sn]), h, c16, a0, nun);
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
    // x and y central differences of this lane's node on plane kb, and the
    // -z flux of plane kb (the face from plane kb-1)
    double cx = 0.0, cy = 0.0, fz_lo = 0.0;
    if (own) {
        const double *M = pl[(kb - 1) % 3], *Z = pl[kb % 3];
        cx = Z[c + 1] - Z[c - 1];
        cy = Z[c + PX] - Z[c - PX];
        fz_lo = face_flux<FAMILY>(M[c], Z[c], (M[c + 1] - M[c - 1]) + cx, (M[c + PX] - M[c - PX]) + cy, h, c16,
                                  a0, nun);
    }
    if (kb + 2 <= ke + 1) fetch(kb + 2);

    for (int k = kb; k <= ke; ++k) {
        const double *M = pl[(k - 1) % 3], *Z = pl[k % 3], *Q = pl[(k + 1) % 3];
        double fx_hi = 0.0, fy_hi = 0.0, fz_hi = 0.0;
        if (own) {
            const double cz = Q[c] - M[c];
            fx_hi = face_flux<FAMILY>(Z[c], Z[c + 1], cy + (Z[c + 1 + PX] - Z[c + 1 - PX]),
                                      cz + (Q[c + 1] - M[c + 1]), h, c16, a0, nun);
            fy_hi = face_flux<FAMILY>(Z[c], Z[c + PX], cx + (Z[c + PX + 1] - Z[c + PX - 1]),
                                      cz + (Q[c + PX] - M[c + PX]), h, c16, a0, nun);
            const double qx = Q[c + 1] - Q[c - 1], qy = Q[c + PX] - Q[c - PX];
            fz_hi = face_flux<FAMILY>(Z[c], Q[c], cx + qx, cy + qy, h, c16, a0, nun);
            cx = qx;
            cy = qy;
            fx[b][a + 1] = fx_hi;
            fy[b + 1][a] = fy_hi;
        }
        if (ring) *rdst = flux_xy(M, Z, Q, cr, rn, rt);
        __syncthreads();
        if (own) {
            double s = fx_hi - fx[b][a];
            s += fy_hi - fy[b][a];
            s += fz_hi - fz_lo;
            S[(size_t)k * nn + i + (size_t)n * j] = s * sscale;
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
        hipLaunchKernelGGL((mond_source_zmarch<kSrcTX, kSrcTY, false>), grid, dim3(kSrcTX * kSrcTY), 0, s, n, h,
                           a0, nun, phin, S, kchunk, nzc);
    else
        hipLaunchKernelGGL((mond_source_zmarch<kSrcTX, kSrcTY, true>), grid, dim3(kSrcTX * kSrcTY), 0, s, n, h,
                           a0, nun, phin, S, kchunk, nzc);
    hipLaunchKernelGGL(zero_faces_k, dim3((6 * n * n + 255) / 256, nb), dim3(256), 0, s, n, S);
}

}  // namespace qm
