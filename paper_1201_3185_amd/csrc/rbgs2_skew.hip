// Two red-black Gauss-Seidel sweeps in one pass over u and f (Sec. 2: the
// smoother of the multigrid solves of Eq. 1 and Eq. 2), with the four
// half-sweeps of a z-march skewed two planes apart.
//
// Step s of the march updates the red nodes of plane s (first sweep), the
// black nodes of plane s - 2 (first sweep), the red nodes of plane s - 4
// (second sweep) and the black nodes of plane s - 6 (second sweep).  Each of
// these reads only nodes of the other colour on its plane and the two next to
// it, and none of those is written in the same step: the red updates of steps
// s - 1 and s - 5 and the black updates of step s - 1 are the newest values any
// of them needs, so the four stages run together between one pair of
// barriers, and every node update sees exactly the values it sees in two
// sequential sweeps.  In x and y each stage covers one ring fewer than the one
// before (the tile plus three, two, one and zero nodes), recomputing the
// neighbours' ring nodes from the same inputs, so the tile's values equal the
// sequential sweeps' bit for bit.  LDS holds ten planes (s - 7 .. s + 2) of
// the tile plus a four-node ring; a plane of u and the f values of a step are
// requested two steps before use.  A workgroup marches the whole column.
// Red nodes are those with i + j + k even.
#include <type_traits>

#include "common.h"

namespace qm {

namespace {

template <typename T, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT)
rbgs2_skew_k(const T *__restrict__ uin, T *__restrict__ uout, const T *__restrict__ f, int n, T h2)
{
#pragma clang fp contract(off)
    constexpr int RG = 4;                                  // ring of the region held in LDS
    constexpr int PX = TX + 2 * RG, PY = TY + 2 * RG, PL = PX * PY;
    constexpr int NS = 10;                                 // planes s - 7 .. s + 2
    constexpr int NL = (PL + NT - 1) / NT;
    constexpr int HX = TX / 2;
    // nodes of one colour on the tile plus a ring of width w, per thread
    constexpr int R3 = ((TX + 6) / 2 * (TY + 6) + NT - 1) / NT;
    constexpr int R2 = ((TX + 4) / 2 * (TY + 4) + NT - 1) / NT;
    constexpr int R1 = ((TX + 2) / 2 * (TY + 2) + NT - 1) / NT;
    constexpr int NF = R3 + R2 + R1 + 1;                   // f values of one step
    static_assert(TX % 2 == 0 && HX * TY <= NT, "at most one pair of tile nodes per thread");
    __shared__ T pl[NS][PL];
    const T sixth = T(1) / T(6);
    const int tid = threadIdx.x;
    const unsigned tl = xcd_tile(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
    const int bx = tl % gridDim.x, by = (tl / gridDim.x) % gridDim.y, pb = tl / (gridDim.x * gridDim.y);
    const int i0 = 1 + bx * TX, j0 = 1 + by * TY;
    const size_t nn = (size_t)n * n;
    if (uin) uin += (size_t)pb * nn * n;   // a null uin (zero iterate) stays null
    uout += (size_t)pb * nn * n;
    f += (size_t)pb * nn * n;

    int goff[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int t = tid + r * NT;
        const int i = i0 - RG + t % PX, j = j0 - RG + t / PX;
        goff[r] = (t < PL && i >= 0 && i < n && j >= 0 && j < n) ? i + n * j : -1;
    }
    auto fetch = [&](int k, T *vv) {
        const T *src = uin ? uin + (size_t)k * nn : nullptr;
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const T x = src ? src[max(goff[r], 0)] : T(0);
            vv[r] = goff[r] >= 0 ? x : T(0);
        }
    };
    auto commit = [&](int k, const T *vv) {
        T *P = pl[k % NS];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t < PL) P[t] = vv[r];
        }
    };

    // node r of this thread among the colour-c nodes of plane k on the tile plus
    // a ring of width W: LDS offset and grid column, or -1 if it is not an
    // interior node
    auto node = [&](auto wc, int r, int k, int c, int &cl, int &gi, int &gj) {
        constexpr int W = decltype(wc)::value;
        constexpr int HW = (TX + 2 * W) / 2, NW = HW * (TY + 2 * W);
        const int e = tid + r * NT;
        cl = -1;
        if (e >= NW) return;
        const int br = e / HW, q = e % HW;
        const int j = j0 - W + br;
        const int off = (c + i0 - W + j + k) & 1;
        const int i = i0 - W + 2 * q + off;
        if (i < 1 || i > n - 2 || j < 1 || j > n - 2) return;
        cl = (RG - W + br) * PX + (RG - W + 2 * q + off);
        gi = i;
        gj = j;
    };
    // the f values a stage on plane k will need, with its nodes' LDS offsets
    // (-1: none) and, for the tile's black node, its grid column: requested two
    // steps ahead, so the stage itself does no index arithmetic
    auto f_stage = [&](auto wc, int k, int c, T *fv, int *cv, int *gv) {
        constexpr int W = decltype(wc)::value;
        constexpr int RW = ((TX + 2 * W) / 2 * (TY + 2 * W) + NT - 1) / NT;
        const bool kin = k >= 1 && k <= n - 2;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            int cl, gi = 0, gj = 0;
            node(wc, r, k, c, cl, gi, gj);
            cv[r] = kin ? cl : -1;
            if (W == 0) *gv = gi;
            fv[r] = (kin && cl >= 0) ? f[(size_t)k * nn + gi + (size_t)n * gj] : T(0);
        }
    };
    auto stage = [&](auto wc, int k, const T *fv, const int *cv) {
        constexpr int W = decltype(wc)::value;
        constexpr int RW = ((TX + 2 * W) / 2 * (TY + 2 * W) + NT - 1) / NT;
        if (k < 1 || k > n - 2) return;
        T *P = pl[k % NS];
        const T *Pm = pl[(k - 1) % NS];
        const T *Pp = pl[(k + 1) % NS];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int cl = cv[r];
            if (cl < 0) continue;
            const T s = P[cl - 1] + P[cl + 1] + P[cl - PX] + P[cl + PX] + Pm[cl] + Pp[cl];
            P[cl] = (s - h2 * fv[r]) * sixth;
        }
    };
    using W0 = std::integral_constant<int, 0>;
    using W1 = std::integral_constant<int, 1>;
    using W2 = std::integral_constant<int, 2>;
    using W3 = std::integral_constant<int, 3>;
    // the f values of step s: red of plane s (ring 3), black of s - 2 (ring 2),
    // red of s - 4 (ring 1), black of s - 6 (the tile)
    auto f_step = [&](int s, T *fv, int *cv, int *gv) {
        f_stage(W3{}, s, 0, fv, cv, gv);
        f_stage(W2{}, s - 2, 1, fv + R3, cv + R3, gv);
        f_stage(W1{}, s - 4, 0, fv + R3 + R2, cv + R3 + R2, gv);
        f_stage(W0{}, s - 6, 1, fv + R3 + R2 + R1, cv + R3 + R2 + R1, gv);
    };
    // the last stage of plane k, then the tile's pair of nodes of row j0 + tid / HX
    // goes out: the black node just updated and the red node final since step k + 4
    auto stage_out = [&](int k, T fb, int cl, int gi) {
        if (k < 1 || k > n - 2) return;
        if (tid >= HX * TY) return;   // threads beyond the tile's pairs
        const int br = tid / HX, q = tid % HX;
        const int j = j0 + br;
        if (j > n - 2) return;
        T *P = pl[k % NS];
        T *dst = uout + (size_t)k * nn + (size_t)n * j;
        if (cl >= 0) {
            const T *Pm = pl[(k - 1) % NS];
            const T *Pp = pl[(k + 1) % NS];
            const T s = P[cl - 1] + P[cl + 1] + P[cl - PX] + P[cl + PX] + Pm[cl] + Pp[cl];
            const T v = (s - h2 * fb) * sixth;
            P[cl] = v;
            dst[gi] = v;
        }
        // the red node of the pair: column i0 + 2q or i0 + 2q + 1, whichever is not black
        const int offb = (1 + i0 + j + k) & 1;
        const int ir = i0 + 2 * q + (1 - offb);
        if (ir <= n - 2) dst[ir] = P[(RG + br) * PX + (RG + 2 * q + (1 - offb))];
    };

    // warm-up: planes 0, 1, 2 in LDS; planes 3, 4 and the f values of steps 1, 2 in flight
    {
        T w[3][NL];
#pragma unroll
        for (int q = 0; q < 3; ++q) fetch(q, w[q]);
#pragma unroll
        for (int q = 0; q < 3; ++q) commit(q, w[q]);
    }
    T vA[NL], vB[NL], fA[NF], fB[NF];
    int cA[NF], cB[NF], gA = 0, gB = 0;
#pragma unroll
    for (int r = 0; r < NL; ++r) vA[r] = vB[r] = T(0);
    if (3 <= n - 1) fetch(3, vA);
    if (4 <= n - 1) fetch(4, vB);
    f_step(1, fA, cA, &gA);
    f_step(2, fB, cB, &gB);
    __syncthreads();

    const int smax = n + 4;   // the last black update of the second sweep is plane n - 2
    auto step = [&](int s, T *vX, T *fX, int *cX, int &gX) {
        T fc[NF];
        int cc[NF];
#pragma unroll
        for (int r = 0; r < NF; ++r) {
            fc[r] = fX[r];
            cc[r] = cX[r];
        }
        const int gc = gX;
        if (s + 2 <= smax) f_step(s + 2, fX, cX, &gX);   // the set just emptied serves step s + 2
        if (s + 2 <= n - 1) {
            commit(s + 2, vX);   // into the slot of plane s - 8, last read in step s - 1
            if (s + 4 <= n - 1) fetch(s + 4, vX);
        }
        stage(W3{}, s, fc, cc);
        stage(W2{}, s - 2, fc + R3, cc + R3);
        stage(W1{}, s - 4, fc + R3 + R2, cc + R3 + R2);
        stage_out(s - 6, fc[R3 + R2 + R1], cc[R3 + R2 + R1], gc);
        __syncthreads();
    };
    for (int s = 1; s <= smax; s += 2) {
        step(s, vA, fA, cA, gA);
        if (s + 1 <= smax) step(s + 1, vB, fB, cB, gB);
    }
}

}  // namespace

template <typename T>
void launch_rbgs2_skew(int n, double h, const T *f, const T *uin, T *uout, hipStream_t s, int nb)
{
    constexpr int TX = 64, TY = 16, NT = 1024;   // two threads per pair of tile nodes
    const int m = n - 2;
    const dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, nb);
    hipLaunchKernelGGL((rbgs2_skew_k<T, TX, TY, NT>), grid, dim3(NT), 0, s, uin, uout, f, n, T(h * h));
}

template void launch_rbgs2_skew<double>(int, double, const double *, const double *, double *, hipStream_t, int);
template void launch_rbgs2_skew<float>(int, double, const float *, const float *, float *, hipStream_t, int);

}  // namespace qm
