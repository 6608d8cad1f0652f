// One red-black Gauss-Seidel sweep fused with the residual restriction that
// follows it in a V-cycle (Sec. 2: the multigrid solves of Eq. 1 and Eq. 2):
// u_out = sweep(u_in), then fc = FW(f - A_h u_out) on the next coarser level
// and uc0 = 0 there, in one pass over u and f instead of two.
//
// A workgroup owns a TX x TY column tile and marches the whole z column, one
// plane per step, with six planes of u in LDS (the tile plus a four-node
// ring).  It repeats the work of its neighbours on the ring so that it can
// form residuals there: red nodes are updated on the tile plus a three-node
// ring, black nodes on the tile plus a two-node ring, and the residual of the
// swept u on the tile plus a one-node ring.  Every node update and residual
// is the expression of the separate kernels (rbgs_zmarch_pair_deep and
// residual_restrict_k) on the same inputs, so the ring values equal the
// neighbours' and the results equal the two-kernel path bit for bit.  Step k
// stores plane k+3 of u into LDS, updates black nodes of plane k and writes
// the tile of plane k (phase 1), then updates red nodes of plane k+2 and forms
// the residual of plane k-1 into a ring of three residual planes (phase 2);
// coarse plane K is restricted in phase 1 of step 2K+3, once the residuals of
// fine planes 2K-1..2K+1 are in LDS.  Loads run two steps ahead: step k
// requests plane k+5 of u and the f values of the red nodes of plane k+4, the
// black nodes of plane k+2 and the residual nodes of plane k+1.
//
// Coarse node ownership: the tile whose fine columns i0..i0+TX-1 hold 2I - 1
// restricts column I (I = 0 and I = nc - 1 go to the first and the last
// tile), and likewise in y, so every coarse node is written by one workgroup.
// Red nodes are those with i + j + k even.
#include "common.h"

namespace qm {

namespace {

template <typename T, int TX, int TY>
__global__ void __launch_bounds__(TX *TY / 2)
rbgs_restrict_k(const T *__restrict__ uin, T *__restrict__ uout, const T *__restrict__ f, int n, T h2, T ih2,
                T *__restrict__ fc, T *__restrict__ uc0, T *__restrict__ uc1, int zu)
{
#pragma clang fp contract(off)
    constexpr int NT = TX * TY / 2;
    constexpr int PX = TX + 8, PY = TY + 8, PL = PX * PY, NS = 6;   // u planes: tile + 4-ring
    constexpr int NL = (PL + NT - 1) / NT;
    // red region (tile + 3-ring): local a, b in 1 .. P-2; black (tile + 2-ring): 2 .. P-3
    constexpr int R3W = PX - 2, R3H = PY - 2, R3S = (R3W + 1) / 2, NR3 = R3S * R3H, RI3 = (NR3 + NT - 1) / NT;
    constexpr int R2W = PX - 4, R2H = PY - 4, R2S = (R2W + 1) / 2, NR2 = R2S * R2H, RI2 = (NR2 + NT - 1) / NT;
    // residual region (tile + 1-ring): local 3 .. P-4, stored as its own RXxRY planes
    constexpr int RX = PX - 6, RY = PY - 6, RP = RX * RY, RI1 = (RP + NT - 1) / NT;
    // coarse columns a workgroup may own
    constexpr int CXO = TX / 2 + 1, CYO = TY / 2 + 1;
    static_assert(CXO * CYO <= NT, "one owned coarse column per thread");
    static_assert(TX % 2 == 0 && TY % 2 == 0, "even tiles");
    __shared__ T pl[NS][PL];
    __shared__ T rs[3][RP];
    const T sixth = T(1) / T(6);
    const int tid = threadIdx.x;
    const int gx = gridDim.x, gy = gridDim.y;
    const unsigned tl = xcd_tile(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    const int bx = tl % gx, by = (tl / gx) % gy, pb = tl / (gx * gy);
    const int i0 = 1 + bx * TX, j0 = 1 + by * TY;
    const int nc = (n + 1) / 2;
    const size_t nn = (size_t)n * n, Nc = (size_t)nc * nc * nc;
    uin += (size_t)pb * nn * n;
    uout += (size_t)pb * nn * n;
    f += (size_t)pb * nn * n;
    fc += (size_t)pb * Nc;
    uc0 += (size_t)pb * Nc;
    if (uc1) uc1 += (size_t)pb * Nc;
    const int ia = i0 - 4, ja = j0 - 4;   // grid position of local (0, 0)

    // this lane's share of a u plane
    int goff[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int t = tid + r * NT;
        const int i = ia + t % PX, j = ja + t / PX;
        goff[r] = (t < PL && i >= 0 && i < n && j >= 0 && j < n) ? i + n * j : -1;
    }
    // red slots: row b = 1 + e / R3S, slot q = e % R3S, column a = 1 + 2q (+1 by parity)
    int rb3[RI3], rq3[RI3];
#pragma unroll
    for (int r = 0; r < RI3; ++r) {
        const int e = tid + r * NT;
        rb3[r] = e < NR3 ? 1 + e / R3S : -1;
        rq3[r] = e % R3S;
    }
    int bb2[RI2], bq2[RI2];
#pragma unroll
    for (int r = 0; r < RI2; ++r) {
        const int e = tid + r * NT;
        bb2[r] = e < NR2 ? 2 + e / R2S : -1;
        bq2[r] = e % R2S;
    }
    // residual nodes: local (3 + t % RX, 3 + t / RX), interior of the grid only
    int rsl[RI1];
#pragma unroll
    for (int r = 0; r < RI1; ++r) {
        const int t = tid + r * NT;
        const int a = 3 + t % RX, b = 3 + t / RX;
        const int i = ia + a, j = ja + b;
        rsl[r] = (t < RP && i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) ? a + PX * b : -1;
    }
    // column (local a) of the red slot of row b on plane k, and of the black one
    auto red_col = [&](int a0, int b, int k) { return a0 + (((ia + a0) + (ja + b) + k) & 1); };
    auto interior = [&](int a, int b) {
        const int i = ia + a, j = ja + b;
        return i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2;
    };

    // owned coarse column of this lane
    const int cI0 = bx == 0 ? 0 : (i0 + 1) / 2, cJ0 = by == 0 ? 0 : (j0 + 1) / 2;
    const int cI1 = bx == gx - 1 ? nc - 1 : (i0 + TX - 1) / 2, cJ1 = by == gy - 1 ? nc - 1 : (j0 + TY - 1) / 2;
    const int oI = cI0 + tid % CXO, oJ = cJ0 + tid / CXO;
    const bool owner = tid < CXO * CYO && oI <= cI1 && oJ <= cJ1;
    const bool c_bnd = oI == 0 || oJ == 0 || oI == nc - 1 || oJ == nc - 1;
    // the fine residual (2I + a, 2J + b) sits at residual-plane offset (2I + a - ia - 3) + RX (2J + b - ja - 3)
    const int rbase = (2 * oI - ia - 3) + RX * (2 * oJ - ja - 3);
    auto zero_node = [&](int K) {
        const size_t C = (size_t)oI + (size_t)nc * ((size_t)oJ + (size_t)nc * K);
        uc0[C] = T(0);
        if (uc1) uc1[C] = T(0);
        fc[C] = T(0);
    };
    auto restrict_plane = [&](int K) {   // coarse plane K from residual planes 2K-1 .. 2K+1
        if (!owner) return;
        if (c_bnd) {
            zero_node(K);
            return;
        }
        const T w[3] = {T(0.25), T(0.5), T(0.25)};
        T acc = T(0);
        for (int c = -1; c <= 1; ++c) {
            const T *R = rs[(2 * K + c) % 3];
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a) acc += (w[a + 1] * w[b + 1] * w[c + 1]) * R[rbase + a + RX * b];
        }
        const size_t C = (size_t)oI + (size_t)nc * ((size_t)oJ + (size_t)nc * K);
        if (zu) uc0[C] = T(0);
        fc[C] = acc;
    };

    auto fetch = [&](int k, T *vv) {
        const T *src = uin + (size_t)k * nn;
#pragma unroll
        for (int r = 0; r < NL; ++r) vv[r] = goff[r] >= 0 ? src[goff[r]] : T(0);
    };
    auto commit = [&](int k, const T *vv) {
        T *P = pl[k % NS];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t < PL) P[t] = vv[r];
        }
    };
    auto f_red = [&](int k, T *fr) {
#pragma unroll
        for (int r = 0; r < RI3; ++r) {
            fr[r] = T(0);
            if (rb3[r] < 0) continue;
            const int a = red_col(1 + 2 * rq3[r], rb3[r], k);
            if (a <= PX - 2 && interior(a, rb3[r]))
                fr[r] = f[(size_t)k * nn + (size_t)(ia + a) + (size_t)n * (ja + rb3[r])];
        }
    };
    auto f_black = [&](int k, T *fb) {
#pragma unroll
        for (int r = 0; r < RI2; ++r) {
            fb[r] = T(0);
            if (bb2[r] < 0) continue;
            const int a = 2 + 2 * bq2[r] + 1 - (((ia + 2 + 2 * bq2[r]) + (ja + bb2[r]) + k) & 1);
            if (a <= PX - 3 && interior(a, bb2[r]))
                fb[r] = f[(size_t)k * nn + (size_t)(ia + a) + (size_t)n * (ja + bb2[r])];
        }
    };
    auto f_res = [&](int k, T *fq) {
#pragma unroll
        for (int r = 0; r < RI1; ++r) {
            fq[r] = T(0);
            if (rsl[r] < 0) continue;
            const int a = rsl[r] % PX, b = rsl[r] / PX;
            fq[r] = f[(size_t)k * nn + (size_t)(ia + a) + (size_t)n * (ja + b)];
        }
    };
    auto update = [&](T *P, const T *Pm, const T *Pp, int c, T fv) {
        const T s = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
        return (s - h2 * fv) * sixth;
    };
    auto red = [&](int k, const T *fr) {   // red nodes of plane k on the tile + 3-ring
        T *P = pl[k % NS];
        const T *Pm = pl[(k - 1) % NS], *Pp = pl[(k + 1) % NS];
#pragma unroll
        for (int r = 0; r < RI3; ++r) {
            if (rb3[r] < 0) continue;
            const int b = rb3[r], a = red_col(1 + 2 * rq3[r], b, k);
            if (a > PX - 2 || !interior(a, b)) continue;
            const int c = a + PX * b;
            P[c] = update(P, Pm, Pp, c, fr[r]);
        }
    };
    auto black = [&](int k, const T *fb) {   // black nodes of plane k on the tile + 2-ring; the tile's to uout
        T *P = pl[k % NS];
        const T *Pm = pl[(k - 1) % NS], *Pp = pl[(k + 1) % NS];
        T *dst = uout + (size_t)k * nn;
#pragma unroll
        for (int r = 0; r < RI2; ++r) {
            if (bb2[r] < 0) continue;
            const int b = bb2[r];
            const int a = 2 + 2 * bq2[r] + 1 - (((ia + 2 + 2 * bq2[r]) + (ja + b) + k) & 1);
            if (a > PX - 3 || !interior(a, b)) continue;
            const int c = a + PX * b;
            const T v = update(P, Pm, Pp, c, fb[r]);
            P[c] = v;
            if (a >= 4 && a < 4 + TX && b >= 4 && b < 4 + TY) dst[(size_t)(ia + a) + (size_t)n * (ja + b)] = v;
        }
    };
    auto store_red = [&](int k) {   // the tile's red nodes of plane k (final since step k-2) to uout
        const T *P = pl[k % NS];
        T *dst = uout + (size_t)k * nn;
        for (int e = tid; e < TX * TY / 2; e += NT) {
            const int b = 4 + e / (TX / 2), a = red_col(4 + 2 * (e % (TX / 2)), b, k);
            if (interior(a, b)) dst[(size_t)(ia + a) + (size_t)n * (ja + b)] = P[a + PX * b];
        }
    };
    auto resid = [&](int k, const T *fq) {   // residual of the swept plane k on the tile + 1-ring
        const T *P = pl[k % NS];
        const T *Pm = pl[(k - 1) % NS], *Pp = pl[(k + 1) % NS];
        T *R = rs[k % 3];
#pragma unroll
        for (int r = 0; r < RI1; ++r) {
            if (rsl[r] < 0) continue;
            const int c = rsl[r];
            const T lap = (P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c] - T(6) * P[c]) * ih2;
            R[tid + r * NT] = fq[r] - lap;
        }
    };

    if (owner) zero_node(0);
    // warm-up: planes 0..3 in LDS (all loads in flight before the first store),
    // red nodes of planes 1 and 2
    {
        T w[4][NL];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T *src = uin + (size_t)min(q, n - 1) * nn;
#pragma unroll
            for (int r = 0; r < NL; ++r) w[q][r] = goff[r] >= 0 ? src[goff[r]] : T(0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q <= n - 1) commit(q, w[q]);
    }
    T fr1[RI3], fr2[RI3];
    f_red(1, fr1);
    if (2 <= n - 2) f_red(2, fr2);
    __syncthreads();
    red(1, fr1);
    if (2 <= n - 2) red(2, fr2);
    __syncthreads();

    // two register sets: set A serves odd steps, set B even ones
    T vA[NL], vB[NL], rA[RI3], rB[RI3], bA[RI2], bB[RI2], qA[RI1], qB[RI1];
    auto refill = [&](int k, T *vX, T *rX, T *bX, T *qX) {   // the loads step k's set needs
        if (k + 3 <= n - 1) fetch(k + 3, vX);
        if (k + 2 <= n - 2) f_red(k + 2, rX);
        f_black(k, bX);
        if (k - 1 >= 1) f_res(k - 1, qX);
    };
    refill(1, vA, rA, bA, qA);
    if (2 <= n - 2) refill(2, vB, rB, bB, qB);
    auto step = [&](int k, T *vX, T *rX, T *bX, T *qX) {
        // phase 1: plane k+3 into LDS, black nodes of plane k, the tile of plane k out, coarse plane (k-3)/2
        if (k + 3 <= n - 1) commit(k + 3, vX);
        T frc[RI3], fqc[RI1];
#pragma unroll
        for (int r = 0; r < RI3; ++r) frc[r] = rX[r];
#pragma unroll
        for (int r = 0; r < RI1; ++r) fqc[r] = qX[r];
        black(k, bX);
        if (k + 2 <= n - 2) refill(k + 2, vX, rX, bX, qX);   // set for step k+2, in flight meanwhile
        store_red(k);
        if ((k & 1) && k >= 5) restrict_plane((k - 3) / 2);
        __syncthreads();
        // phase 2: red nodes of plane k+2, residual of plane k-1
        if (k + 2 <= n - 2) red(k + 2, frc);
        if (k - 1 >= 1) resid(k - 1, fqc);
        __syncthreads();
    };
    for (int k = 1; k <= n - 2; k += 2) {
        step(k, vA, rA, bA, qA);
        if (k + 1 <= n - 2) step(k + 1, vB, rB, bB, qB);
    }
    // the residual of the last interior plane, then the last coarse planes
    {
        T fq[RI1];
        f_res(n - 2, fq);
        resid(n - 2, fq);
    }
    __syncthreads();
    restrict_plane(nc - 2);   // planes up to nc - 3 were restricted in the march (n - 2 is odd)
    if (owner) zero_node(nc - 1);
}

}  // namespace

template <typename T>
bool rbgs_restrict_fits(int n)
{
    return n >= 9;
}

static int g_sweep_restrict[2][11] = {{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};

template <typename T>
int &sweep_restrict(int n)
{
    int J = 0;
    while ((1 << J) < n - 1) ++J;
    return g_sweep_restrict[sizeof(T) == 4 ? 1 : 0][J > 10 ? 10 : J];
}

template <typename T>
void launch_rbgs_restrict(int n, double h, const T *f, const T *uin, T *uout, T *fc, T *uc0, T *uc1, hipStream_t s,
                          int nb, bool zero_u)
{
    constexpr int TX = 64, TY = 16;
    const int m = n - 2;
    dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, nb);
    hipLaunchKernelGGL((rbgs_restrict_k<T, TX, TY>), grid, dim3(TX * TY / 2), 0, s, uin, uout, f, n, T(h * h),
                       T(1.0 / (h * h)), fc, uc0, uc1, zero_u ? 1 : 0);
}

template int &sweep_restrict<double>(int);
template int &sweep_restrict<float>(int);
template bool rbgs_restrict_fits<double>(int);
template bool rbgs_restrict_fits<float>(int);
template void launch_rbgs_restrict<double>(int, double, const double *, const double *, double *, double *, double *,
                                           double *, hipStream_t, int, bool);
template void launch_rbgs_restrict<float>(int, double, const float *, const float *, float *, float *, float *, float *,
                                          hipStream_t, int, bool);

}  // namespace qm
