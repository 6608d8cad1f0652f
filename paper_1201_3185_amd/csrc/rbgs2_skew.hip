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
#include "common.h"

namespace qm {

namespace {

// ZERO: the iterate is zero (uin is not read).  PROLONG: the coarse-grid
// correction u += P uc (uc on the grid of nc = (n + 1) / 2 points) is added to
// every interior node as its plane is stored to LDS, with the trilinear
// expression of the prolong-add kernel evaluated in the same order (along x,
// then y, then z) on coarse planes staged in LDS, so the result is that of a
// prolong-add launch followed by the two sweeps, bit for bit.
template <typename T, int TX, int TY, int NT, bool ZERO, bool PROLONG>
__global__ void __launch_bounds__(NT)
rbgs2_skew_k(const T *__restrict__ uin, T *__restrict__ uout, const T *__restrict__ f, int n, T h2,
             const T *__restrict__ uc, int nc)
{
#pragma clang fp contract(off)
    typedef T pair_t __attribute__((ext_vector_type(2), aligned(sizeof(T))));
    constexpr int RG = 4;                                  // ring of the region held in LDS
    constexpr int PX = TX + 2 * RG, PY = TY + 2 * RG, PL = PX * PY;
    constexpr int NS = 10;                                 // planes s - 7 .. s + 2
    constexpr int HPX = PX / 2, NPL = HPX * PY;            // x-pairs of nodes of an LDS plane
    constexpr int HP = PX / 2, NP = HP * (TY + 6);         // node pairs: four-node ring in x, three in y
    static_assert(TX % 2 == 0 && NP <= NT, "at most one pair of nodes per thread");
    // coarse rows of the LDS region (tile origins are odd): TY / 2 + 5; a coarse
    // plane is staged interpolated along x, on the region's fine columns
    constexpr int CPY = TY / 2 + 5, XPL = PX * CPY, NXL = (XPL + NT - 1) / NT;
    static_assert(NPL <= NT, "one pair of an LDS plane per thread");
    __shared__ T pl[NS][PL];
    __shared__ T cpl[PROLONG ? 3 : 1][PROLONG ? XPL : 1];   // coarse plane c, along x, in slot c % 3
    const T sixth = T(1) / T(6);
    const int tid = threadIdx.x;
    const unsigned tl = xcd_tile(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
    const int bx = tl % gridDim.x, by = (tl / gridDim.x) % gridDim.y, pb = tl / (gridDim.x * gridDim.y);
    const int i0 = 1 + bx * TX, j0 = 1 + by * TY;
    const size_t nn = (size_t)n * n;
    if (!ZERO) uin += (size_t)pb * nn * n;
    uout += (size_t)pb * nn * n;
    f += (size_t)pb * nn * n;
    if (PROLONG) uc += (size_t)pb * nc * nc * nc;

    // A plane of u arrives as one x-pair of nodes per thread (iq, iq + 1 of
    // row jq; LDS offset lq): one 16-byte load from a base clamped into the
    // grid's row (node iq + e sits at element e + sh of the load), requested
    // into registers as it is and masked where it is stored, two steps later,
    // so nothing waits for the load in between; a lane with nothing to load
    // reads the tile's corner pair (lanes of all workgroups meeting on one
    // cache line would queue on it).
    const int qa = tid % HPX, qb = tid / HPX;
    const int iq = i0 - RG + 2 * qa, jq = j0 - RG + qb, lq = qb * PX + 2 * qa;
    const bool qrow = tid < NPL && jq >= 0 && jq < n;
    const int sh = iq - min(max(iq, 0), n - 2);
    const bool in0 = qrow && iq >= 0 && iq <= n - 1, in1 = qrow && iq + 1 >= 0 && iq + 1 <= n - 1;
    const int idle = i0 + n * j0;
    const int qoff = qrow ? min(max(iq, 0), n - 2) + n * jq : idle;
    auto fetch = [&](int k, pair_t &vv) {
        if (ZERO) return;
        vv = *reinterpret_cast<const pair_t *>(uin + (size_t)k * nn + qoff);
    };
    // The correction's coarse data: per staged entry r of this thread (fine
    // column a = t % PX, coarse row cj0 + t / PX of the region), the two
    // coarse nodes its x-interpolation weighs (xo, or -1 where the column is
    // not interior or the row is outside the grid: a lane with nothing to load
    // reads the first of the region's coarse nodes) and the column's parity;
    // per node e of the thread's pair that is interior in x and y, the offset
    // of its column and lower coarse row in the staged plane with the parity
    // of j in bit 16 (else -1).
    const int cj0 = (j0 - RG) >> 1;
    int xo[NXL], cnb[2] = {-1, -1};
    bool xodd[NXL];
    const int cidle = max((i0 - RG) >> 1, 0) + nc * max(cj0, 0);
    if constexpr (PROLONG) {
#pragma unroll
        for (int r = 0; r < NXL; ++r) {
            const int t = tid + r * NT;
            const int i = i0 - RG + t % PX, J = cj0 + t / PX;
            xo[r] = (t < XPL && i >= 1 && i <= n - 2 && J >= 0 && J < nc) ? (i >> 1) + nc * J : -1;
            xodd[r] = i & 1;
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int a = 2 * qa + e, i = iq + e, j = jq;
            cnb[e] = (tid < NPL && i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2)
                         ? a + PX * ((j >> 1) - cj0) + ((j & 1) << 16)
                         : -1;
        }
    }
    T cv0[NXL], cv1[NXL];
    auto fetch_c = [&](int c) {   // the coarse nodes of plane c (clamped into the grid) into cv0, cv1
        if constexpr (PROLONG) {
            const T *C = uc + (size_t)min(c, nc - 1) * nc * nc;
#pragma unroll
            for (int r = 0; r < NXL; ++r) {
                const int o = xo[r] >= 0 ? xo[r] : cidle;
                cv0[r] = C[o];
                cv1[r] = C[xodd[r] && xo[r] >= 0 ? o + 1 : o];
            }
        }
    };
    // ... interpolated along x into its LDS slot (prolong_at's x step: weights 1, 0 at even columns, 1/2, 1/2 at odd)
    auto store_c = [&](int c) {
        if constexpr (PROLONG) {
            if (c > nc - 1) return;
#pragma unroll
            for (int r = 0; r < NXL; ++r) {
                const int t = tid + r * NT;
                if (t >= XPL) continue;
                const T wia = xodd[r] ? T(0.5) : T(1), wib = xodd[r] ? T(0.5) : T(0);
                cpl[c % 3][t] = xo[r] >= 0 ? wia * cv0[r] + wib * cv1[r] : T(0);
            }
        }
    };
    // the correction at a node of plane k (1 <= k <= n - 2) from its packed offset:
    // prolong_at's y and z steps on the staged planes
    auto corr = [&](int cw, int k) {
        const int o = cw & 0xffff, dj = (cw >> 16) & 1;
        const T wja = dj ? T(0.5) : T(1), wjb = dj ? T(0.5) : T(0);
        const T wka = (k & 1) ? T(0.5) : T(1), wkb = (k & 1) ? T(0.5) : T(0);
        const T *Xa = cpl[(k >> 1) % 3], *Xb = cpl[((k + 1) >> 1) % 3];
        const int oj = o + dj * PX;
        const T xa = Xa[o], xb = Xa[oj], xc = Xb[o], xd = Xb[oj];
        return wka * (wja * xa + wjb * xb) + wkb * (wja * xc + wjb * xd);
    };
    // With the correction only the black node of a pair takes it: a red
    // node's own value is replaced by the first sweep's red update before any
    // update reads it, and red nodes of the outer ring are not read at all.
    auto commit = [&](int k, const pair_t &vv) {
        if (tid >= NPL) return;
        T x0 = (!ZERO && in0) ? (sh == 0 ? vv.x : vv.y) : T(0);
        T x1 = (!ZERO && in1) ? (sh == 0 ? vv.y : vv.x) : T(0);
        if (PROLONG && k >= 1 && k <= n - 2) {
            const int eb = (iq + jq + k + 1) & 1;   // the pair's black node
            const int cw = eb ? cnb[1] : cnb[0];
            if (cw >= 0) {
                const T c = corr(cw, k);
                if (eb) x1 += c;
                else x0 += c;
            }
        }
        T *P = pl[k % NS] + lq;
        P[0] = x0;
        P[1] = x1;
    };

    // This thread's pair of nodes: grid columns il, il + 1 of row jp, LDS
    // offsets cb, cb + 1.  Bit 2w + e of ok says that node e of the pair is an
    // interior node on the tile plus a ring of width w (rings 3, 2, 1, 0 hold
    // the four stages' nodes).
    const int q = tid % HP, br = tid / HP;
    const int il = i0 - RG + 2 * q, jp = j0 - 3 + br;
    const int cb = (br + RG - 3) * PX + 2 * q;
    unsigned ok = 0;
    if (tid < NP && jp >= 1 && jp <= n - 2) {
#pragma unroll
        for (int w = 0; w < 4; ++w)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int a = 2 * q + e, b = br + RG - 3, i = il + e;
                if (a >= RG - w && a <= RG + TX - 1 + w && b >= RG - w && b <= RG + TY - 1 + w && i >= 1 && i <= n - 2)
                    ok |= 1u << (2 * w + e);
            }
    }
    // f of the pair on plane k (in range: both columns lie in the grid when
    // either is interior; else the tile's corner pair)
    const bool fok = (ok >> 6) != 0;
    const size_t frow = fok ? (size_t)il + (size_t)n * jp : (size_t)idle;
    auto f_pair = [&](int k) { return *reinterpret_cast<const pair_t *>(f + (size_t)k * nn + frow); };
    // node e of the pair on plane k takes its update from f value fv
    auto update = [&](int k, int e, T fv) {
        T *P = pl[k % NS];
        const T *Pm = pl[(k - 1) % NS];
        const T *Pp = pl[(k + 1) % NS];
        const int c = cb + e;
        const T s = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
        const T v = (s - h2 * fv) * sixth;
        P[c] = v;
        return v;
    };

    // warm-up: planes 0, 1, 2 in LDS (with the correction: coarse planes 0, 1, 2
    // first); planes 3, 4, the f pairs of planes 1, 2 and coarse plane 3 in flight
    {
        pair_t w[3] = {};
#pragma unroll
        for (int z = 0; z < 3; ++z) fetch(z, w[z]);
        if constexpr (PROLONG) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                fetch_c(c);
                store_c(c);
            }
            __syncthreads();
        }
#pragma unroll
        for (int z = 0; z < 3; ++z) commit(z, w[z]);
    }
    fetch_c(3);
    pair_t vA = {T(0), T(0)}, vB = {T(0), T(0)};
    if (3 <= n - 1) fetch(3, vA);
    if (4 <= n - 1) fetch(4, vB);
    pair_t pA = {T(0), T(0)}, pB = {T(0), T(0)};
    if (1 <= n - 2) pA = f_pair(1);
    if (2 <= n - 2) pB = f_pair(2);
    // f of the red node of planes s .. s - 4 and of the black node of planes s .. s - 6
    T fr[5], fb[7];
#pragma unroll
    for (int r = 0; r < 5; ++r) fr[r] = T(0);
#pragma unroll
    for (int r = 0; r < 7; ++r) fb[r] = T(0);
    __syncthreads();

    const int smax = n + 4;   // the last black update of the second sweep is plane n - 2
    // even: s is even (the loop's second step of a pair); with the correction,
    // an even step s stores coarse plane (s + 4) / 2, first read by the commit
    // of fine plane s + 3 in step s + 1, and requests plane (s + 6) / 2
    auto step = [&](int s, pair_t &vX, pair_t &pX, bool even) {
        const int er = (il + jp + s) & 1;   // the red node of the pair on planes s, s - 4
        const int eb = er ^ 1;              // the black one on planes s - 2, s - 6
#pragma unroll
        for (int r = 4; r > 0; --r) fr[r] = fr[r - 1];
#pragma unroll
        for (int r = 6; r > 0; --r) fb[r] = fb[r - 1];
        fr[0] = er ? pX.y : pX.x;
        fb[0] = er ? pX.x : pX.y;
        if (s + 2 <= n - 1) commit(s + 2, vX);   // into the slot of plane s - 8, last read in step s - 1
        if (PROLONG && even) {   // into the slot of coarse plane s / 2 - 1, last read in step s - 3
            store_c((s + 4) / 2);
            fetch_c((s + 6) / 2);
        }
        // the next requests, their planes clamped into the grid (what the last
        // steps fetch beyond plane n - 1, or n - 2 for f, is never used)
        fetch(min(s + 4, n - 1), vX);
        pX = f_pair(min(s + 2, n - 2));
        if (s <= n - 2 && ((ok >> (6 + er)) & 1)) update(s, er, fr[0]);
        if (s - 2 >= 1 && s - 2 <= n - 2 && ((ok >> (4 + eb)) & 1)) update(s - 2, eb, fb[2]);
        if (s - 4 >= 1 && s - 4 <= n - 2 && ((ok >> (2 + er)) & 1)) update(s - 4, er, fr[4]);
        // plane s - 6 is final after its black update: the pair's tile nodes go out
        const int k = s - 6;
        if (k >= 1 && k <= n - 2 && (ok & 3)) {
            T *dst = uout + (size_t)k * nn + (size_t)n * jp + il;
            if ((ok >> eb) & 1) dst[eb] = update(k, eb, fb[6]);
            if ((ok >> er) & 1) dst[er] = pl[k % NS][cb + er];
        }
        __syncthreads();
    };
    int s = 1;
    for (; s + 1 <= smax; s += 2) {   // whole pairs of steps: no branch inside the loop
        step(s, vA, pA, false);
        step(s + 1, vB, pB, true);
    }
    if (s <= smax) step(s, vA, pA, false);
}

}  // namespace

template <typename T, int TX, int TY, int NT>
static void skew_launch(int n, double h, const T *f, const T *uin, T *uout, hipStream_t s, int nb, const T *uc)
{
    const int m = n - 2;
    const dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, nb);
    const int nc = (n + 1) / 2;
    if (uc && uin)
        hipLaunchKernelGGL((rbgs2_skew_k<T, TX, TY, NT, false, true>), grid, dim3(NT), 0, s, uin, uout, f, n, T(h * h),
                           uc, nc);
    else if (uc)
        hipLaunchKernelGGL((rbgs2_skew_k<T, TX, TY, NT, true, true>), grid, dim3(NT), 0, s, uin, uout, f, n, T(h * h),
                           uc, nc);
    else if (uin)
        hipLaunchKernelGGL((rbgs2_skew_k<T, TX, TY, NT, false, false>), grid, dim3(NT), 0, s, uin, uout, f, n, T(h * h),
                           uc, nc);
    else
        hipLaunchKernelGGL((rbgs2_skew_k<T, TX, TY, NT, true, false>), grid, dim3(NT), 0, s, uin, uout, f, n, T(h * h),
                           uc, nc);
}

template <typename T>
void launch_rbgs2_skew(int n, double h, const T *f, const T *uin, T *uout, hipStream_t s, int nb, const T *uc, int tile)
{
    if (tile == 1) skew_launch<T, 32, 8, 320>(n, h, f, uin, uout, s, nb, uc);   // 55 KB of LDS: two workgroups per CU
    else skew_launch<T, 64, 16, 1024>(n, h, f, uin, uout, s, nb, uc);          // 146 KB: one per CU
}

template void launch_rbgs2_skew<double>(int, double, const double *, const double *, double *, hipStream_t, int,
                                        const double *, int);
template void launch_rbgs2_skew<float>(int, double, const float *, const float *, float *, hipStream_t, int,
                                       const float *, int);

}  // namespace qm
