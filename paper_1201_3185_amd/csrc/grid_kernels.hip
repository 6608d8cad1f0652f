// Multigrid kernels for gfx950 (Sec. 2 of Angus et al.: FMG with red-black
// Gauss-Seidel for the 7-point Laplacian on vertex-centred n = 2^J + 1 grids).
//
// Smoother design.  One launch performs a whole red-black sweep out of place
// (u_in -> u_out).  Each workgroup owns a TX x TY column tile and marches up a
// range of z planes, keeping five planes of the tile plus a two-node ring in
// LDS.  A plane first holds the old values; the red pass overwrites its red
// entries (red = (i+j+k) even, updated first) over the tile and a one-node
// ring, which only needs old black values, so the black pass on the tile then
// finds every new red neighbour in LDS.  Red values on the ring are recomputed
// by the neighbouring tiles from the same old values, so the result equals a
// plain red pass followed by a black pass, with u read once and written once
// (24 bytes per point in FP64).  Reading u_in and writing u_out avoids any
// race between tiles; the driver alternates two buffers.
//
// Rounding.  The stencil kernels evaluate every node update, residual and
// transfer with floating-point contraction off, so that the result does not
// depend on which kernel (tile shape, fused or single sweep, gather or tile
// restriction) computes it.
//
// Batches.  Every grid kernel can sweep the same level of nb independent
// problems stored back to back (problem p of a level with n points per side
// starts at p n^3): the problem index is the slowest part of the block index,
// so one launch covers the whole batch, and nb = 1 is the single-problem case.
#include <algorithm>

#include "common.h"

namespace qm {

// Trilinear value of the coarse field at fine node (i,j,k): an even fine index
// sits on coarse node i/2, an odd one halfway between (i-1)/2 and (i+1)/2.
template <typename T>
__device__ __forceinline__ T prolong_at(int nc, const T *__restrict__ uc, int i, int j, int k)
{
#pragma clang fp contract(off)
    const int ia = i >> 1, ib = (i + 1) >> 1, ja = j >> 1, jb = (j + 1) >> 1, ka = k >> 1, kb = (k + 1) >> 1;
    const T wia = (i & 1) ? T(0.5) : T(1), wib = (i & 1) ? T(0.5) : T(0);
    const T wja = (j & 1) ? T(0.5) : T(1), wjb = (j & 1) ? T(0.5) : T(0);
    const T wka = (k & 1) ? T(0.5) : T(1), wkb = (k & 1) ? T(0.5) : T(0);
    const T xa = wia * uc[id3(nc, ia, ja, ka)] + wib * uc[id3(nc, ib, ja, ka)];
    const T xb = wia * uc[id3(nc, ia, jb, ka)] + wib * uc[id3(nc, ib, jb, ka)];
    const T xc = wia * uc[id3(nc, ia, ja, kb)] + wib * uc[id3(nc, ib, ja, kb)];
    const T xd = wia * uc[id3(nc, ia, jb, kb)] + wib * uc[id3(nc, ib, jb, kb)];
    return wka * (wja * xa + wjb * xb) + wkb * (wja * xc + wjb * xd);
}

// ------------------------------------------------------------------ smoother

// With PROLONG the coarse-grid correction u += P uc is applied to every
// interior node as its plane is loaded (the first post-smoothing sweep of a
// V-cycle), with the same expression as prolong_k.
template <typename T, int TX, int TY, bool PROLONG>
__global__ void __launch_bounds__(TX *TY)
rbgs_zmarch(const T *__restrict__ uin, T *__restrict__ uout, const T *__restrict__ f, int n, T h2, int kchunk, int nzc,
            const T *__restrict__ uc, int nc)
{
#pragma clang fp contract(off)
    constexpr int PX = TX + 4, PY = TY + 4, NS = 5, NT = TX * TY;
    constexpr int PL = PX * PY;                  // values of one LDS plane (tile + two-node ring)
    constexpr int NL = (PL + NT - 1) / NT;       // plane values loaded per thread
    constexpr int HALF = (TX + 2) / 2;           // red nodes per row of tile + one-node ring
    static_assert(HALF * (TY + 2) <= NT, "one red node per thread");
    __shared__ T pl[NS][PL];
    const T sixth = T(1) / T(6);
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
    // a null uin (zero iterate) stays null: only a real array is offset
    if (uin) uin += (size_t)pb * nn * n;
    uout += (size_t)pb * nn * n;
    f += (size_t)pb * nn * n;
    if (PROLONG) uc += (size_t)pb * nc * nc * nc;

    // plane offsets of this thread's share of a plane load (and, for the
    // correction, whether the node is interior in x and y)
    int goff[NL], gij[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int t = tid + r * NT;
        const int a = t % PX, b = t / PX;
        const int i = i0 - 2 + a, j = j0 - 2 + b;
        goff[r] = (t < PL && i >= 0 && i < n && j >= 0 && j < n) ? i + n * j : -1;
        gij[r] = (goff[r] >= 0 && i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) ? (i | (j << 16)) : -1;
    }
    auto corrected = [&](T x, int r, int k) {
        if (PROLONG && k >= 1 && k <= n - 2 && gij[r] >= 0) x += prolong_at(nc, uc, gij[r] & 0xffff, gij[r] >> 16, k);
        return x;
    };
    // this thread's red node (tile + ring): row b_r, column depends on the plane's parity
    const int b_r = 1 + tid / HALF, j_r = j0 - 2 + b_r, q_r = tid % HALF;
    const bool red_thread = tid < HALF * (TY + 2) && j_r >= 1 && j_r <= n - 2;
    auto red_a = [&](int k) { return ((((i0 - 1) + j_r + k) & 1) ? 2 : 1) + 2 * q_r; };
    // this thread's tile node (black pass and store)
    const int a_b = 2 + tid % TX, b_b = 2 + tid / TX;
    const int i_b = i0 - 2 + a_b, j_b = j0 - 2 + b_b;
    const bool tile_thread = i_b <= n - 2 && j_b <= n - 2;

    // a null uin is a zero iterate (boundary included), read from nowhere
    auto load_now = [&](int k) {
        T *P = pl[k % NS];
        const T *src = uin ? uin + (size_t)k * nn : nullptr;
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t < PL) P[t] = goff[r] >= 0 ? corrected(src ? src[goff[r]] : T(0), r, k) : T(0);
        }
    };
    T v[NL];
    auto prefetch = [&](int k) {
        const T *src = uin ? uin + (size_t)k * nn : nullptr;
#pragma unroll
        for (int r = 0; r < NL; ++r) v[r] = goff[r] >= 0 ? corrected(src ? src[goff[r]] : T(0), r, k) : T(0);
    };
    auto commit = [&](int k) {
        T *P = pl[k % NS];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t < PL) P[t] = v[r];
        }
    };
    // f at this thread's red node of plane k (0 if it has none)
    auto f_red = [&](int k) {
        const int i = i0 - 2 + red_a(k);
        return (red_thread && i >= 1 && i <= n - 2) ? f[(size_t)k * nn + i + (size_t)n * j_r] : T(0);
    };
    auto f_black = [&](int k) {
        return (tile_thread && ((i_b + j_b + k) & 1)) ? f[(size_t)k * nn + i_b + (size_t)n * j_b] : T(0);
    };
    auto red = [&](int k, T fv) {
        const int a = red_a(k), i = i0 - 2 + a;
        if (!red_thread || i < 1 || i > n - 2) return;
        T *P = pl[k % NS];
        const T *Pm = pl[(k - 1) % NS];
        const T *Pp = pl[(k + 1) % NS];
        const int c = b_r * PX + a;
        const T s = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
        P[c] = (s - h2 * fv) * sixth;
    };
    auto black_store = [&](int k, T fv) {
        if (!tile_thread) return;
        const T *P = pl[k % NS];
        const int c = b_b * PX + a_b;
        T val;
        if (((i_b + j_b + k) & 1) == 0) {
            val = P[c];
        } else {
            const T *Pm = pl[(k - 1) % NS];
            const T *Pp = pl[(k + 1) % NS];
            const T s = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
            val = (s - h2 * fv) * sixth;
        }
        uout[(size_t)k * nn + i_b + (size_t)n * j_b] = val;
    };

    // warm-up: planes kb-2..kb+2 and red of kb-1..kb+1
    if (kb >= 2) load_now(kb - 2);
    load_now(kb - 1);
    load_now(kb);
    load_now(kb + 1);
    if (kb + 2 <= n - 1) load_now(kb + 2);
    const T fr0 = kb - 1 >= 1 ? f_red(kb - 1) : T(0);
    const T fr1 = f_red(kb);
    const T fr2 = kb + 1 <= n - 2 ? f_red(kb + 1) : T(0);
    __syncthreads();
    if (kb - 1 >= 1) red(kb - 1, fr0);
    red(kb, fr1);
    if (kb + 1 <= n - 2) red(kb + 1, fr2);
    __syncthreads();

    auto need_red = [&](int k) { return (k + 2 <= n - 2) && (k + 2 <= ke + 1); };  // red(k+2) in iteration k
    T fr_next = T(0), fb_next = f_black(kb);
    if (need_red(kb)) {
        prefetch(kb + 3);
        fr_next = f_red(kb + 2);
    }
    for (int k = kb; k <= ke; ++k) {
        const bool more = need_red(k);
        if (more) commit(k + 3);
        const T fb = fb_next, fr = fr_next;
        // prefetch for iteration k+1 while this one computes
        if (k + 1 <= ke) {
            fb_next = f_black(k + 1);
            if (need_red(k + 1)) {
                prefetch(k + 4);
                fr_next = f_red(k + 3);
            }
        }
        black_store(k, fb);
        __syncthreads();
        if (more) red(k + 2, fr);
        __syncthreads();
    }
}

// The same sweep with half the threads: each thread owns an x-pair of tile
// nodes (columns 2q and 2q + 1 of its row), one red and one black on every
// plane, so the black pass keeps every lane busy (rbgs_zmarch leaves the
// lanes on red tile nodes idle there) and a plane needs half the thread
// iterations per node between its two barriers.  The red pass covers the
// tile plus a one-node ring (up to two red nodes per thread).  Node updates,
// their order within a plane and the plane pipeline are those of
// rbgs_zmarch, so the results agree bit for bit.
// With PROLONG, the coarse planes the correction u += P uc reads are staged
// in an LDS ring of three (the tile's coarse footprint, (TX/2 + 3) x
// (TY/2 + 3) values, loaded one march step ahead), and every plane of the
// march takes its correction from there as it is stored to LDS: one coarse
// load per coarse node instead of eight per fine node.  The expression is
// prolong_at's, so the bits are those of a separate prolong-add launch.
template <typename T, int TX, int TY, bool PROLONG>
__global__ void __launch_bounds__(TX *TY / 2)
rbgs_zmarch_pair(const T *__restrict__ uin, T *__restrict__ uout, const T *__restrict__ f, int n, T h2, int kchunk,
                 int nzc, const T *__restrict__ uc, int nc)
{
#pragma clang fp contract(off)
    static_assert(TX % 2 == 0, "x-pairs");
    constexpr int PX = TX + 4, PY = TY + 4, NS = 5, NT = TX * TY / 2;
    constexpr int PL = PX * PY;
    constexpr int NL = (PL + NT - 1) / NT;
    constexpr int HALF = (TX + 2) / 2;            // red nodes per row of tile + one-node ring
    constexpr int NRED = HALF * (TY + 2);
    constexpr int RI = (NRED + NT - 1) / NT;      // red nodes per thread
    constexpr int HX = TX / 2;                    // pairs per tile row
    constexpr int CPX = TX / 2 + 3, CPY = TY / 2 + 3, CPL = CPX * CPY;   // coarse footprint of a plane
    constexpr int NCL = (CPL + NT - 1) / NT;
    __shared__ T pl[NS][PL];
    __shared__ T cpl[PROLONG ? 3 : 1][PROLONG ? CPL : 1];
    const T sixth = T(1) / T(6);
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
    // a null uin (zero iterate) stays null: only a real array is offset
    if (uin) uin += (size_t)pb * nn * n;
    uout += (size_t)pb * nn * n;
    f += (size_t)pb * nn * n;
    if (PROLONG) uc += (size_t)pb * nc * nc * nc;
    // coarse footprint: coarse nodes ci0 .. ci0 + CPX - 1 (and likewise in y)
    // cover the interpolation stencils of fine nodes i0 - 2 .. i0 + TX + 1
    const int ci0 = (i0 - 3) >> 1, cj0 = (j0 - 3) >> 1;
    int coff[NCL];
    T cv[NCL];
#pragma unroll
    for (int r = 0; r < NCL; ++r) {
        const int t = tid + r * NT;
        const int I = ci0 + t % CPX, J = cj0 + t / CPX;
        coff[r] = (PROLONG && t < CPL && I >= 0 && I < nc && J >= 0 && J < nc) ? I + nc * J : -1;
        cv[r] = T(0);
    }
    auto fetch_c = [&](int c) {   // coarse plane c into registers
#pragma unroll
        for (int r = 0; r < NCL; ++r) cv[r] = coff[r] >= 0 ? uc[(size_t)c * nc * nc + coff[r]] : T(0);
    };
    auto store_c = [&](int c) {   // ... and from there into its LDS slot
        if constexpr (PROLONG) {
            T *D = cpl[c % 3];
#pragma unroll
            for (int r = 0; r < NCL; ++r) {
                const int t = tid + r * NT;
                if (t < CPL) D[t] = cv[r];
            }
        }
    };
    // prolong_at's trilinear value from the staged coarse planes
    auto prolong_lds = [&](int i, int j, int k) {
        const int ia = (i >> 1) - ci0, ib = ((i + 1) >> 1) - ci0, ja = (j >> 1) - cj0, jb = ((j + 1) >> 1) - cj0;
        const T *Ca = cpl[(k >> 1) % 3];
        const T *Cb = cpl[((k + 1) >> 1) % 3];
        const T wia = (i & 1) ? T(0.5) : T(1), wib = (i & 1) ? T(0.5) : T(0);
        const T wja = (j & 1) ? T(0.5) : T(1), wjb = (j & 1) ? T(0.5) : T(0);
        const T wka = (k & 1) ? T(0.5) : T(1), wkb = (k & 1) ? T(0.5) : T(0);
        const T xa = wia * Ca[ia + CPX * ja] + wib * Ca[ib + CPX * ja];
        const T xb = wia * Ca[ia + CPX * jb] + wib * Ca[ib + CPX * jb];
        const T xc = wia * Cb[ia + CPX * ja] + wib * Cb[ib + CPX * ja];
        const T xd = wia * Cb[ia + CPX * jb] + wib * Cb[ib + CPX * jb];
        return wka * (wja * xa + wjb * xb) + wkb * (wja * xc + wjb * xd);
    };

    int goff[NL], gij[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int t = tid + r * NT;
        const int a = t % PX, b = t / PX;
        const int i = i0 - 2 + a, j = j0 - 2 + b;
        goff[r] = (t < PL && i >= 0 && i < n && j >= 0 && j < n) ? i + n * j : -1;
        gij[r] = (goff[r] >= 0 && i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) ? (i | (j << 16)) : -1;
    }
    auto corrected = [&](T x, int r, int k) {
        if (PROLONG && k >= 1 && k <= n - 2 && gij[r] >= 0) x += prolong_at(nc, uc, gij[r] & 0xffff, gij[r] >> 16, k);
        return x;
    };
    // this thread's red nodes (tile + ring): row br[r], column from the plane's parity
    int br[RI], jr[RI], qr[RI];
    bool rv[RI];
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int t = tid + r * NT;
        br[r] = 1 + t / HALF;
        jr[r] = j0 - 2 + br[r];
        qr[r] = t % HALF;
        rv[r] = t < NRED && jr[r] >= 1 && jr[r] <= n - 2;
    }
    auto red_a = [&](int r, int k) { return ((((i0 - 1) + jr[r] + k) & 1) ? 2 : 1) + 2 * qr[r]; };
    // this thread's pair of tile nodes: columns lo, lo + 1 of row bb
    const int bb = 2 + tid / HX, lo = 2 + 2 * (tid % HX);
    const int jb = j0 - 2 + bb, ilo = i0 - 2 + lo;
    const bool row_ok = jb <= n - 2;
    auto black_a = [&](int k) { return ((ilo + jb + k) & 1) ? lo : lo + 1; };

    // a null uin is a zero iterate (boundary included), read from nowhere
    auto load_now = [&](int k) {
        T *P = pl[k % NS];
        const T *src = uin ? uin + (size_t)k * nn : nullptr;
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t < PL) P[t] = goff[r] >= 0 ? corrected(src ? src[goff[r]] : T(0), r, k) : T(0);
        }
    };
    T v[NL];
    auto prefetch = [&](int k) {   // raw values; the correction is added from LDS at commit
        const T *src = uin ? uin + (size_t)k * nn : nullptr;
#pragma unroll
        for (int r = 0; r < NL; ++r) v[r] = goff[r] >= 0 ? (src ? src[goff[r]] : T(0)) : T(0);
    };
    auto commit = [&](int k) {
        T *P = pl[k % NS];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t >= PL) continue;
            T x = v[r];
            if (PROLONG && k >= 1 && k <= n - 2 && gij[r] >= 0) x += prolong_lds(gij[r] & 0xffff, gij[r] >> 16, k);
            P[t] = x;
        }
    };
    auto f_red = [&](int k, T *fr) {
#pragma unroll
        for (int r = 0; r < RI; ++r) {
            const int i = i0 - 2 + red_a(r, k);
            fr[r] = (rv[r] && i >= 1 && i <= n - 2) ? f[(size_t)k * nn + i + (size_t)n * jr[r]] : T(0);
        }
    };
    auto f_black = [&](int k) {
        const int i = i0 - 2 + black_a(k);
        return (row_ok && i <= n - 2) ? f[(size_t)k * nn + i + (size_t)n * jb] : T(0);
    };
    auto red = [&](int k, const T *fr) {
        T *P = pl[k % NS];
        const T *Pm = pl[(k - 1) % NS];
        const T *Pp = pl[(k + 1) % NS];
#pragma unroll
        for (int r = 0; r < RI; ++r) {
            const int a = red_a(r, k), i = i0 - 2 + a;
            if (!rv[r] || i < 1 || i > n - 2) continue;
            const int c = br[r] * PX + a;
            const T s = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
            P[c] = (s - h2 * fr[r]) * sixth;
        }
    };
    auto black_store = [&](int k, T fv) {
        if (!row_ok) return;
        const T *P = pl[k % NS];
        const T *Pm = pl[(k - 1) % NS];
        const T *Pp = pl[(k + 1) % NS];
        const int ab = black_a(k), ar = ab == lo ? lo + 1 : lo;
        const int ib = i0 - 2 + ab, ir = i0 - 2 + ar;
        T *dst = uout + (size_t)k * nn + (size_t)n * jb;
        if (ib <= n - 2) {
            const int c = bb * PX + ab;
            const T s = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
            dst[ib] = (s - h2 * fv) * sixth;
        }
        if (ir <= n - 2) dst[ir] = P[bb * PX + ar];
    };

    // warm-up: planes kb-2..kb+2 and red of kb-1..kb+1
    if constexpr (!PROLONG) {
        // all five planes' loads in flight before the first LDS store (plane and
        // in-plane offsets clamped into the grid; out-of-grid planes not stored)
        T w[5][NL];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const T *src = uin ? uin + (size_t)min(max(kb - 2 + q, 0), n - 1) * nn : nullptr;
#pragma unroll
            for (int r = 0; r < NL; ++r) {
                const T x = src ? src[max(goff[r], 0)] : T(0);
                w[q][r] = goff[r] >= 0 ? x : T(0);
            }
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int k = kb - 2 + q;
            if (k < 0 || k > n - 1) continue;
            T *P = pl[k % NS];
#pragma unroll
            for (int r = 0; r < NL; ++r) {
                const int t = tid + r * NT;
                if (t < PL) P[t] = w[q][r];
            }
        }
    } else {
        if (kb >= 2) load_now(kb - 2);
        load_now(kb - 1);
        load_now(kb);
        load_now(kb + 1);
        if (kb + 2 <= n - 1) load_now(kb + 2);
        // the coarse planes of the march's first stored plane (kb + 3), and the
        // one the first odd step stages
        const int ca = (kb + 3) >> 1, cb = (kb + 4) >> 1;
        if (ca <= nc - 1) {
            fetch_c(ca);
            store_c(ca);
        }
        if (cb != ca && cb <= nc - 1) {
            fetch_c(cb);
            store_c(cb);
        }
        const int c1 = ((kb | 1) + 5) / 2;
        if (c1 <= nc - 1) fetch_c(c1);
    }
    T fr0[RI], fr1[RI], fr2[RI];
#pragma unroll
    for (int r = 0; r < RI; ++r) fr0[r] = fr2[r] = T(0);
    if (kb - 1 >= 1) f_red(kb - 1, fr0);
    f_red(kb, fr1);
    if (kb + 1 <= n - 2) f_red(kb + 1, fr2);
    __syncthreads();
    if (kb - 1 >= 1) red(kb - 1, fr0);
    red(kb, fr1);
    if (kb + 1 <= n - 2) red(kb + 1, fr2);
    __syncthreads();

    auto need_red = [&](int k) { return (k + 2 <= n - 2) && (k + 2 <= ke + 1); };  // red(k+2) in iteration k
    T fr_next[RI], fr[RI];
#pragma unroll
    for (int r = 0; r < RI; ++r) fr_next[r] = T(0);
    T fb_next = f_black(kb);
    if (need_red(kb)) {
        prefetch(kb + 3);
        f_red(kb + 2, fr_next);
    }
    for (int k = kb; k <= ke; ++k) {
        const bool more = need_red(k);
        if (more) commit(k + 3);
        const T fb = fb_next;
#pragma unroll
        for (int r = 0; r < RI; ++r) fr[r] = fr_next[r];
        if (k + 1 <= ke) {
            fb_next = f_black(k + 1);
            if (need_red(k + 1)) {
                prefetch(k + 4);
                f_red(k + 3, fr_next);
            }
        }
        black_store(k, fb);
        __syncthreads();
        if (more) red(k + 2, fr);
        // an odd step stages coarse plane (k + 5) / 2, first read by the store
        // of fine plane k + 4 in the next step, into the slot of plane
        // (k - 1) / 2, last read three steps ago; then loads the next one
        if (PROLONG && (k & 1)) {
            if ((k + 5) / 2 <= nc - 1) store_c((k + 5) / 2);
            if ((k + 7) / 2 <= nc - 1) fetch_c((k + 7) / 2);
        }
        __syncthreads();
    }
}

// The pair sweep with its loads two march steps ahead: plane k+5 of u, the
// red f values of plane k+4 and the black ones of plane k+2 are requested in
// step k, so a load has two steps' time to arrive (the pair kernel gives it
// one).  Two register sets alternate between even and odd steps (the loop is
// unrolled by two).  The plane pipeline, LDS layout and node updates are the
// pair kernel's, so the bits are too.
// With PROLONG the coarse-grid correction u += P uc is added to every plane
// as it is stored to LDS, from staged data in the order of prolong_at's
// expression (x first, then y, then z): each coarse plane arrives in an LDS
// buffer (two alternate), is interpolated along x once for the tile's fine
// columns and coarse rows into a ring of three x-interpolated planes, and a
// node's correction then takes four LDS values and three weighted sums.  An
// odd step k stores coarse plane (k+7)/2, interpolates plane (k+5)/2 along x
// (first read by the store of fine plane k+4, in step k+1) and requests plane
// (k+9)/2.
template <typename T, int TX, int TY, bool PROLONG>
__global__ void __launch_bounds__(TX *TY / 2)
rbgs_zmarch_pair_deep(const T *__restrict__ uin, T *__restrict__ uout, const T *__restrict__ f, int n, T h2,
                      int kchunk, int nzc, const T *__restrict__ uc, int nc)
{
#pragma clang fp contract(off)
    static_assert(TX % 2 == 0, "x-pairs");
    constexpr int PX = TX + 4, PY = TY + 4, NS = 5, NT = TX * TY / 2;
    constexpr int PL = PX * PY;
    constexpr int NL = (PL + NT - 1) / NT;
    constexpr int HALF = (TX + 2) / 2;
    constexpr int NRED = HALF * (TY + 2);
    constexpr int RI = (NRED + NT - 1) / NT;
    constexpr int HX = TX / 2;
    constexpr int CPX = TX / 2 + 3, CPY = TY / 2 + 3, CPL = CPX * CPY;   // coarse footprint of a plane
    constexpr int XPL = PX * CPY;                                         // x-interpolated plane
    constexpr int NCL = (CPL + NT - 1) / NT, NXL = (XPL + NT - 1) / NT;
    __shared__ T pl[NS][PL];
    __shared__ T craw[PROLONG ? 2 : 1][PROLONG ? CPL : 1];
    __shared__ T xip[PROLONG ? 3 : 1][PROLONG ? XPL : 1];
    const T sixth = T(1) / T(6);
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
    if (uin) uin += (size_t)pb * nn * n;   // a null uin (zero iterate) stays null
    uout += (size_t)pb * nn * n;
    f += (size_t)pb * nn * n;
    if (PROLONG) uc += (size_t)pb * nc * nc * nc;

    // coarse footprint: coarse nodes ci0 .. ci0 + CPX - 1 (and likewise in y)
    // cover the interpolation stencils of fine nodes i0 - 2 .. i0 + TX + 1
    const int ci0 = (i0 - 3) >> 1, cj0 = (j0 - 3) >> 1;
    int coff[NCL];
    T cv[NCL];
#pragma unroll
    for (int r = 0; r < NCL; ++r) {
        const int t = tid + r * NT;
        const int I = ci0 + t % CPX, J = cj0 + t / CPX;
        coff[r] = (PROLONG && t < CPL && I >= 0 && I < nc && J >= 0 && J < nc) ? I + nc * J : -1;
        cv[r] = T(0);
    }
    auto fetch_c = [&](int c) {   // coarse plane c into registers
#pragma unroll
        for (int r = 0; r < NCL; ++r) cv[r] = coff[r] >= 0 ? uc[(size_t)c * nc * nc + coff[r]] : T(0);
    };
    auto store_c = [&](int c) {   // ... into its raw LDS buffer
        if constexpr (PROLONG) {
            T *D = craw[c & 1];
#pragma unroll
            for (int r = 0; r < NCL; ++r) {
                const int t = tid + r * NT;
                if (t < CPL) D[t] = cv[r];
            }
        }
    };
    auto interp_x = [&](int c) {   // raw coarse plane c -> x-interpolated plane (fine columns, coarse rows)
        if constexpr (PROLONG) {
            const T *C = craw[c & 1];
            T *D = xip[c % 3];
#pragma unroll
            for (int r = 0; r < NXL; ++r) {
                const int t = tid + r * NT;
                if (t >= XPL) continue;
                const int a = t % PX, jj = t / PX;
                const int i = i0 - 2 + a;
                const int ia = (i >> 1) - ci0, ib = ((i + 1) >> 1) - ci0;
                const T wia = (i & 1) ? T(0.5) : T(1), wib = (i & 1) ? T(0.5) : T(0);
                D[t] = wia * C[ia + CPX * jj] + wib * C[ib + CPX * jj];
            }
        }
    };
    // the correction at fine node (column a of the plane, row j, plane k):
    // prolong_at's y and z sums over the x-interpolated planes
    auto corr_at = [&](int a, int j, int k) {
        const int ja = (j >> 1) - cj0, jb = ((j + 1) >> 1) - cj0;
        const T *Xa = xip[(k >> 1) % 3];
        const T *Xb = xip[((k + 1) >> 1) % 3];
        const T wja = (j & 1) ? T(0.5) : T(1), wjb = (j & 1) ? T(0.5) : T(0);
        const T wka = (k & 1) ? T(0.5) : T(1), wkb = (k & 1) ? T(0.5) : T(0);
        const T xa = Xa[a + PX * ja], xb = Xa[a + PX * jb], xc = Xb[a + PX * ja], xd = Xb[a + PX * jb];
        return wka * (wja * xa + wjb * xb) + wkb * (wja * xc + wjb * xd);
    };

    int goff[NL], gaj[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int t = tid + r * NT;
        const int a = t % PX, b = t / PX;
        const int i = i0 - 2 + a, j = j0 - 2 + b;
        goff[r] = (t < PL && i >= 0 && i < n && j >= 0 && j < n) ? i + n * j : -1;
        // plane column and grid row of a node interior in x and y (it takes the correction), else -1
        gaj[r] = (goff[r] >= 0 && i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) ? (a | (j << 16)) : -1;
    }
    int br[RI], jr[RI], qr[RI];
    bool rv[RI];
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int t = tid + r * NT;
        br[r] = 1 + t / HALF;
        jr[r] = j0 - 2 + br[r];
        qr[r] = t % HALF;
        rv[r] = t < NRED && jr[r] >= 1 && jr[r] <= n - 2;
    }
    auto red_a = [&](int r, int k) { return ((((i0 - 1) + jr[r] + k) & 1) ? 2 : 1) + 2 * qr[r]; };
    const int bb = 2 + tid / HX, lo = 2 + 2 * (tid % HX);
    const int jb = j0 - 2 + bb, ilo = i0 - 2 + lo;
    const bool row_ok = jb <= n - 2;
    auto black_a = [&](int k) { return ((ilo + jb + k) & 1) ? lo : lo + 1; };

    auto fetch = [&](int k, T *vv) {
        const T *src = uin ? uin + (size_t)k * nn : nullptr;
#pragma unroll
        for (int r = 0; r < NL; ++r) vv[r] = goff[r] >= 0 ? (src ? src[goff[r]] : T(0)) : T(0);
    };
    auto commit = [&](int k, const T *vv) {
        T *P = pl[k % NS];
        const bool kin = k >= 1 && k <= n - 2;
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t >= PL) continue;
            T x = vv[r];
            if (PROLONG && kin && gaj[r] >= 0) x += corr_at(gaj[r] & 0xffff, gaj[r] >> 16, k);
            P[t] = x;
        }
    };
    auto f_red = [&](int k, T *fr) {
#pragma unroll
        for (int r = 0; r < RI; ++r) {
            const int i = i0 - 2 + red_a(r, k);
            fr[r] = (rv[r] && i >= 1 && i <= n - 2) ? f[(size_t)k * nn + i + (size_t)n * jr[r]] : T(0);
        }
    };
    auto f_black = [&](int k) {
        const int i = i0 - 2 + black_a(k);
        return (row_ok && i <= n - 2) ? f[(size_t)k * nn + i + (size_t)n * jb] : T(0);
    };
    auto red = [&](int k, const T *fr) {
        T *P = pl[k % NS];
        const T *Pm = pl[(k - 1) % NS];
        const T *Pp = pl[(k + 1) % NS];
#pragma unroll
        for (int r = 0; r < RI; ++r) {
            const int a = red_a(r, k), i = i0 - 2 + a;
            if (!rv[r] || i < 1 || i > n - 2) continue;
            const int c = br[r] * PX + a;
            const T s = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
            P[c] = (s - h2 * fr[r]) * sixth;
        }
    };
    auto black_store = [&](int k, T fv) {
        if (!row_ok) return;
        const T *P = pl[k % NS];
        const T *Pm = pl[(k - 1) % NS];
        const T *Pp = pl[(k + 1) % NS];
        const int ab = black_a(k), ar = ab == lo ? lo + 1 : lo;
        const int ib = i0 - 2 + ab, ir = i0 - 2 + ar;
        T *dst = uout + (size_t)k * nn + (size_t)n * jb;
        // with the correction, both nodes of the pair as one two-element store (aligned to one element; measured:
        // faster there, slower in the plain sweep's whole-column march)
        if (PROLONG && ilo + 1 <= n - 2) {
            typedef T pair_t __attribute__((ext_vector_type(2), aligned(sizeof(T))));
            const int c = bb * PX + ab;
            const T s = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
            const T vb = (s - h2 * fv) * sixth, vr = P[bb * PX + ar];
            pair_t o;
            o.x = ab == lo ? vb : vr;
            o.y = ab == lo ? vr : vb;
            *reinterpret_cast<pair_t *>(dst + ilo) = o;
            return;
        }
        if (ib <= n - 2) {
            const int c = bb * PX + ab;
            const T s = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
            dst[ib] = (s - h2 * fv) * sixth;
        }
        if (ir <= n - 2) dst[ir] = P[bb * PX + ar];
    };

    // warm-up: planes kb-2..kb+2 (all loads in flight before the first LDS
    // store, offsets clamped into the grid; with PROLONG the correction of
    // these five planes is prolong_at from global memory) and red of
    // kb-1..kb+1
    {
        T w[5][NL];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const T *src = uin ? uin + (size_t)min(max(kb - 2 + q, 0), n - 1) * nn : nullptr;
#pragma unroll
            for (int r = 0; r < NL; ++r) {
                const T x = src ? src[max(goff[r], 0)] : T(0);
                w[q][r] = goff[r] >= 0 ? x : T(0);
            }
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int k = kb - 2 + q;
            if (k < 0 || k > n - 1) continue;
            T *P = pl[k % NS];
#pragma unroll
            for (int r = 0; r < NL; ++r) {
                const int t = tid + r * NT;
                if (t >= PL) continue;
                T x = w[q][r];
                if (PROLONG && k >= 1 && k <= n - 2 && gaj[r] >= 0)
                    x += prolong_at(nc, uc, i0 - 2 + (gaj[r] & 0xffff), gaj[r] >> 16, k);
                P[t] = x;
            }
        }
    }
    if constexpr (PROLONG) {
        // x-interpolated coarse planes read by the stores of the steps before the
        // first odd step k1, then the raw plane k1 interpolates and the one it stores
        const int k1 = kb | 1;
        for (int c = (kb + 3) >> 1; c <= ((k1 + 4) >> 1) && c <= nc - 1; ++c) {
            fetch_c(c);
            store_c(c);
            __syncthreads();
            interp_x(c);
            __syncthreads();
        }
        if ((k1 + 5) / 2 <= nc - 1) {
            fetch_c((k1 + 5) / 2);
            store_c((k1 + 5) / 2);
        }
        if ((k1 + 7) / 2 <= nc - 1) fetch_c((k1 + 7) / 2);
    }
    T fr0[RI], fr1[RI], fr2[RI];
#pragma unroll
    for (int r = 0; r < RI; ++r) fr0[r] = fr2[r] = T(0);
    if (kb - 1 >= 1) f_red(kb - 1, fr0);
    f_red(kb, fr1);
    if (kb + 1 <= n - 2) f_red(kb + 1, fr2);
    __syncthreads();
    if (kb - 1 >= 1) red(kb - 1, fr0);
    red(kb, fr1);
    if (kb + 1 <= n - 2) red(kb + 1, fr2);
    __syncthreads();

    auto need_red = [&](int k) { return (k + 2 <= n - 2) && (k + 2 <= ke + 1); };  // red(k+2) in step k
    // two register sets: set A serves the steps of kb's parity, set B the others
    T vA[NL], vB[NL], rA[RI], rB[RI];
    T bA = T(0), bB = T(0);
#pragma unroll
    for (int r = 0; r < RI; ++r) rA[r] = rB[r] = T(0);
    bA = f_black(kb);
    if (need_red(kb)) {
        fetch(kb + 3, vA);
        f_red(kb + 2, rA);
    }
    if (kb + 1 <= ke) {
        bB = f_black(kb + 1);
        if (need_red(kb + 1)) {
            fetch(kb + 4, vB);
            f_red(kb + 3, rB);
        }
    }
    auto step = [&](int k, T *vX, T *rX, T &bX) {
        const bool more = need_red(k);
        if (more) commit(k + 3, vX);
        const T fb = bX;
        T frc[RI];
#pragma unroll
        for (int r = 0; r < RI; ++r) frc[r] = rX[r];
        if (k + 2 <= ke) {   // refill the set for step k + 2
            bX = f_black(k + 2);
            if (need_red(k + 2)) {
                fetch(k + 5, vX);
                f_red(k + 4, rX);
            }
        }
        black_store(k, fb);
        __syncthreads();
        if (more) red(k + 2, frc);
        if (PROLONG && (k & 1)) {
            if ((k + 7) / 2 <= nc - 1) store_c((k + 7) / 2);   // raw buffer of plane (k+3)/2, interpolated two steps ago
            if ((k + 5) / 2 <= nc - 1) interp_x((k + 5) / 2);  // into the slot of plane (k-1)/2, last read in step k-3
            if ((k + 9) / 2 <= nc - 1) fetch_c((k + 9) / 2);
        }
        __syncthreads();
    };
    for (int k = kb; k <= ke; k += 2) {
        step(k, vA, rA, bA);
        if (k + 1 <= ke) step(k + 1, vB, rB, bB);
    }
}

template <typename T, int TX, int TY>
static void rbgs_pair_deep_launch(int n, double h, const T *f, const T *uin, T *uout, int kchunk, int nb, const T *uc,
                                  hipStream_t s)
{
    const int m = n - 2;
    const int nzc = (m + kchunk - 1) / kchunk;
    dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, nzc * nb);
    if (uc)
        hipLaunchKernelGGL((rbgs_zmarch_pair_deep<T, TX, TY, true>), grid, dim3(TX * TY / 2), 0, s, uin, uout, f, n,
                           T(h * h), kchunk, nzc, uc, (n + 1) / 2);
    else
        hipLaunchKernelGGL((rbgs_zmarch_pair_deep<T, TX, TY, false>), grid, dim3(TX * TY / 2), 0, s, uin, uout, f, n,
                           T(h * h), kchunk, nzc, uc, (n + 1) / 2);
}

template <typename T, int TX, int TY>
static void rbgs_pair_launch(int n, double h, const T *f, const T *uin, T *uout, int kchunk, int nb, const T *uc,
                             hipStream_t s)
{
    const int m = n - 2;
    const int nzc = (m + kchunk - 1) / kchunk;
    dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, nzc * nb);
    if (uc)
        hipLaunchKernelGGL((rbgs_zmarch_pair<T, TX, TY, true>), grid, dim3(TX * TY / 2), 0, s, uin, uout, f, n,
                           T(h * h), kchunk, nzc, uc, (n + 1) / 2);
    else
        hipLaunchKernelGGL((rbgs_zmarch_pair<T, TX, TY, false>), grid, dim3(TX * TY / 2), 0, s, uin, uout, f, n,
                           T(h * h), kchunk, nzc, uc, (n + 1) / 2);
}

template <typename T, int TX, int TY>
static void rbgs_launch(int n, double h, const T *f, const T *uin, T *uout, int kchunk, int nb, const T *uc,
                        hipStream_t s)
{
    const int m = n - 2;
    const int nzc = (m + kchunk - 1) / kchunk;
    dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, nzc * nb);
    if (uc)
        hipLaunchKernelGGL((rbgs_zmarch<T, TX, TY, true>), grid, dim3(TX * TY), 0, s, uin, uout, f, n, T(h * h), kchunk,
                           nzc, uc, (n + 1) / 2);
    else
        hipLaunchKernelGGL((rbgs_zmarch<T, TX, TY, false>), grid, dim3(TX * TY), 0, s, uin, uout, f, n, T(h * h),
                           kchunk, nzc, uc, (n + 1) / 2);
}

// ------------------------------------------------------ brick smoother
//
// For small levels, where a z-march spends most of its time filling its
// pipeline, each workgroup owns a B^3 brick of interior nodes, loads u on the
// brick plus a 2S-node ring (with the correction u += P uc added on load under
// PROLONG) and f on the brick plus a (2S-1)-node ring into LDS once, runs the
// 2S colour passes of S red-black sweeps on regions one node narrower each
// time, and stores the brick.  Ring values are recomputed by every brick that
// loads them, from the same inputs, so the stored brick equals S sequential
// sweeps; the node update is the same expression as in rbgs_zmarch, so the
// results agree bit for bit.
template <typename T, int B, int S, bool PROLONG>
__global__ void __launch_bounds__(256)
rbgs_brick(const T *__restrict__ uin, T *__restrict__ uout, const T *__restrict__ f, int n, T h2,
           const T *__restrict__ uc, int nc, int nbx)
{
#pragma clang fp contract(off)
    constexpr int R = 2 * S, E = B + 2 * R, FE = E - 2, NT = 256;
    __shared__ T U[E * E * E];
    __shared__ T F[FE * FE * FE];
    const T sixth = T(1) / T(6);
    const int tid = threadIdx.x;
    int bid = (int)xcd_tile(blockIdx.x, gridDim.x);
    const int bx = bid % nbx;
    bid /= nbx;
    const int by = bid % nbx;
    bid /= nbx;
    const int bz = bid % nbx;
    const int pb = bid / nbx;
    const size_t N = (size_t)n * n * n;
    if (uin) uin += pb * N;   // a null uin (zero iterate) stays null
    uout += pb * N;
    f += pb * N;
    if (PROLONG) uc += pb * (size_t)nc * nc * nc;
    const int i0 = 1 + bx * B - R, j0 = 1 + by * B - R, k0 = 1 + bz * B - R;   // global node of U[0]
    // Every lane issues all of its global loads before its first LDS store, so
    // their latencies overlap: addresses are clamped into the grid (always in
    // bounds) and nodes outside it are replaced by zero afterwards.
    constexpr int NU = (E * E * E + NT - 1) / NT, NF = (FE * FE * FE + NT - 1) / NT;
    T xu[NU], xf[NF];
#pragma unroll
    for (int r = 0; r < NU; ++r) {
        const int t = min(tid + r * NT, E * E * E - 1);
        const int a = t % E, b = (t / E) % E, c = t / (E * E);
        const int i = i0 + a, j = j0 + b, k = k0 + c;
        const bool in = i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n;
        const T x = uin ? uin[id3(n, min(max(i, 0), n - 1), min(max(j, 0), n - 1), min(max(k, 0), n - 1))]
                        : T(0);   // a null uin is a zero iterate
        xu[r] = in ? x : T(0);
    }
#pragma unroll
    for (int r = 0; r < NF; ++r) {
        const int t = min(tid + r * NT, FE * FE * FE - 1);
        const int a = t % FE, b = (t / FE) % FE, c = t / (FE * FE);
        const int i = i0 + 1 + a, j = j0 + 1 + b, k = k0 + 1 + c;
        const bool inner = i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2 && k >= 1 && k <= n - 2;
        const T x = f[id3(n, min(max(i, 1), n - 2), min(max(j, 1), n - 2), min(max(k, 1), n - 2))];
        xf[r] = inner ? x : T(0);
    }
#pragma unroll
    for (int r = 0; r < NU; ++r)
        if (tid + r * NT < E * E * E) U[tid + r * NT] = xu[r];
#pragma unroll
    for (int r = 0; r < NF; ++r)
        if (tid + r * NT < FE * FE * FE) F[tid + r * NT] = xf[r];
    if (PROLONG) {   // u += P uc on interior nodes: each lane updates the entries it stored
        for (int t = tid; t < E * E * E; t += NT) {
            const int a = t % E, b = (t / E) % E, c = t / (E * E);
            const int i = i0 + a, j = j0 + b, k = k0 + c;
            if (i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2 && k >= 1 && k <= n - 2)
                U[t] = U[t] + prolong_at(nc, uc, i, j, k);
        }
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < 2 * S; ++st) {
        const int colour = st & 1;           // red ((i+j+k) even) first
        const int r = R - 1 - st;            // ring of this pass
        const int W = B + 2 * r, o = R - r;  // region edge and its start in U
        const int hw = (W + 1) / 2;
        for (int t = tid; t < hw * W * W; t += NT) {
            const int q = t % hw, b = o + (t / hw) % W, c = o + t / (hw * W);
            const int j = j0 + b, k = k0 + c;
            const int ia = i0 + o;
            const int a = o + (((ia + j + k) & 1) == colour ? 0 : 1) + 2 * q;
            const int i = i0 + a;
            if (a >= o + W || i < 1 || i > n - 2 || j < 1 || j > n - 2 || k < 1 || k > n - 2) continue;
            const int p = a + E * (b + E * c);
            const T sum = U[p - 1] + U[p + 1] + U[p - E] + U[p + E] + U[p - E * E] + U[p + E * E];
            U[p] = (sum - h2 * F[(a - 1) + FE * ((b - 1) + FE * (c - 1))]) * sixth;
        }
        __syncthreads();
    }
    for (int t = tid; t < B * B * B; t += NT) {
        const int a = R + t % B, b = R + (t / B) % B, c = R + t / (B * B);
        const int i = i0 + a, j = j0 + b, k = k0 + c;
        if (i > n - 2 || j > n - 2 || k > n - 2) continue;
        uout[id3(n, i, j, k)] = U[a + E * (b + E * c)];
    }
}

template <typename T, int S, int B = 8>
static void brick_launch(int n, double h, const T *f, const T *uin, T *uout, const T *uc, int nb, hipStream_t s)
{
    const int nbx = (n - 2 + B - 1) / B;
    const dim3 grid((unsigned)((size_t)nbx * nbx * nbx * nb));
    if (uc)
        hipLaunchKernelGGL((rbgs_brick<T, B, S, true>), grid, dim3(256), 0, s, uin, uout, f, n, T(h * h), uc,
                           (n + 1) / 2, nbx);
    else
        hipLaunchKernelGGL((rbgs_brick<T, B, S, false>), grid, dim3(256), 0, s, uin, uout, f, n, T(h * h), uc,
                           (n + 1) / 2, nbx);
}

// ----------------------------------------------------- two fused sweeps
//
// Two red-black sweeps (A then B) in one pass: four stages one z plane
// apart run behind each other in the march, each on a ring one node narrower
// than the stage before (red A on the tile plus three nodes, black A plus two,
// red B plus one, black B on the tile), so every stage finds the values it
// needs in LDS.  A plane's LDS copy is updated in place: each stage writes one
// colour and reads only the other, whose newest values are the ones the
// sequential sweeps would read.  Each node update is the same expression as in
// rbgs_zmarch, so the result equals two separate sweeps bit for bit.  With
// PROLONG the coarse-grid correction u += P uc is applied to every interior
// node as its plane is loaded (the post-smoothing of a V-cycle).
template <typename T, int TX, int TY, bool PROLONG>
__global__ void __launch_bounds__(TX *TY)
rbgs2_zmarch(const T *__restrict__ uin, T *__restrict__ uout, const T *__restrict__ f, int n, T h2, int kchunk,
             const T *__restrict__ uc, int nc, int nzc)
{
#pragma clang fp contract(off)
    constexpr int R = 4;                         // ring of the LDS planes
    constexpr int PX = TX + 2 * R, PY = TY + 2 * R, NT = TX * TY;
    constexpr int PL = PX * PY;
    constexpr int FX = TX + 6, FY = TY + 6, FL = FX * FY;   // f on the ring-3 region
    constexpr int NS = 7, NF = 5;
    constexpr int NL = (PL + NT - 1) / NT, NFL = (FL + NT - 1) / NT;
    __shared__ T pl[NS][PL];
    __shared__ T fp[NF][FL];
    const T sixth = T(1) / T(6);
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
    // a null uin (zero iterate) stays null: only a real array is offset
    if (uin) uin += (size_t)pb * nn * n;
    uout += (size_t)pb * nn * n;
    f += (size_t)pb * nn * n;
    if (PROLONG) uc += (size_t)pb * nc * nc * nc;

    int goff[NL], gi[NL], gj[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int t = tid + r * NT;
        const int a = t % PX, b = t / PX;
        gi[r] = i0 - R + a;
        gj[r] = j0 - R + b;
        goff[r] = (t < PL && gi[r] >= 0 && gi[r] < n && gj[r] >= 0 && gj[r] < n) ? gi[r] + n * gj[r] : -1;
    }
    int foff[NFL];
#pragma unroll
    for (int r = 0; r < NFL; ++r) {
        const int t = tid + r * NT;
        const int a = t % FX, b = t / FX;
        const int i = i0 - 3 + a, j = j0 - 3 + b;
        foff[r] = (t < FL && i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) ? i + n * j : -1;
    }
    T v[NL], w[NFL];
    auto prefetch_u = [&](int k) {
        const T *src = uin ? uin + (size_t)k * nn : nullptr;   // null: a zero iterate, read from nowhere
        const bool inner_plane = k >= 1 && k <= n - 2;
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            T x = goff[r] >= 0 ? (src ? src[goff[r]] : T(0)) : T(0);
            if (PROLONG && inner_plane && goff[r] >= 0 && gi[r] >= 1 && gi[r] <= n - 2 && gj[r] >= 1 && gj[r] <= n - 2)
                x += prolong_at(nc, uc, gi[r], gj[r], k);
            v[r] = x;
        }
    };
    auto commit_u = [&](int k) {
        T *P = pl[k % NS];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t < PL) P[t] = v[r];
        }
    };
    auto prefetch_f = [&](int k) {
        const T *src = f + (size_t)k * nn;
#pragma unroll
        for (int r = 0; r < NFL; ++r) w[r] = foff[r] >= 0 ? src[foff[r]] : T(0);
    };
    auto commit_f = [&](int k) {
        T *F = fp[k % NF];
#pragma unroll
        for (int r = 0; r < NFL; ++r) {
            const int t = tid + r * NT;
            if (t < FL) F[t] = w[r];
        }
    };
    // one colour of plane k on the tile plus `ring` nodes
    auto stage = [&](int k, int ring, int colour) {
        T *P = pl[k % NS];
        const T *Pm = pl[(k + NS - 1) % NS];
        const T *Pp = pl[(k + 1) % NS];
        const T *F = fp[k % NF];
        const int hw = (TX + 2 * ring) / 2, rows = TY + 2 * ring, a0 = R - ring;
        for (int t = tid; t < hw * rows; t += NT) {
            const int b = a0 + t / hw;
            const int j = j0 - R + b;
            const int ia0 = i0 - R + a0;
            const int a = a0 + (((ia0 + j + k) & 1) == colour ? 0 : 1) + 2 * (t % hw);
            const int i = i0 - R + a;
            if (i < 1 || i > n - 2 || j < 1 || j > n - 2) continue;
            const int c = b * PX + a;
            const T s = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
            P[c] = (s - h2 * F[(b - 1) * FX + (a - 1)]) * sixth;
        }
    };
    auto store = [&](int k) {
        const T *P = pl[k % NS];
        for (int t = tid; t < TX * TY; t += NT) {
            const int a = R + t % TX, b = R + t / TX;
            const int i = i0 - R + a, j = j0 - R + b;
            if (i > n - 2 || j > n - 2) continue;
            uout[(size_t)k * nn + i + (size_t)n * j] = P[b * PX + a];
        }
    };
    auto in_u = [&](int k) { return k >= max(0, kb - 4) && k <= min(n - 1, ke + 4); };
    auto in_f = [&](int k) { return k >= max(1, kb - 3) && k <= min(n - 2, ke + 3); };
    auto in_stage = [&](int k, int lag) { return k >= max(1, kb - lag) && k <= min(n - 2, ke + lag); };

    if (in_u(kb - 4)) prefetch_u(kb - 4);
    if (in_f(kb - 5)) prefetch_f(kb - 5);
    for (int k = kb - 8; k <= ke; ++k) {
        if (in_u(k + 4)) commit_u(k + 4);
        if (in_f(k + 3)) commit_f(k + 3);
        if (in_u(k + 5)) prefetch_u(k + 5);
        if (in_f(k + 4)) prefetch_f(k + 4);
        __syncthreads();
        if (in_stage(k + 3, 3)) stage(k + 3, 3, 0);      // red, sweep A
        __syncthreads();
        if (in_stage(k + 2, 2)) stage(k + 2, 2, 1);      // black, sweep A
        __syncthreads();
        if (in_stage(k + 1, 1)) stage(k + 1, 1, 0);      // red, sweep B
        __syncthreads();
        if (k >= kb) {
            stage(k, 0, 1);                              // black, sweep B
            __syncthreads();
            store(k);
        }
    }
}

// The two-sweep march with one thread per pair of tile nodes and every load
// two steps ahead (u plane k+6 and f plane k+5 are requested in step k, two
// register sets alternating between even and odd steps), for large levels
// where the fused launch should move u and f once for two sweeps.  Six LDS
// planes of u (tile + four-node ring: step k reads planes k-1..k+4, and the
// store of plane k+4 at the start of step k takes the slot of plane k-2) and
// four of f (planes k..k+3 on the three-node ring).  The four stages, their
// regions and every node update are those of rbgs2_zmarch, so the bits are
// too; with PROLONG the correction u += P uc is prolong_at's, added as u is
// loaded.
template <typename T, int TX, int TY, bool PROLONG>
__global__ void __launch_bounds__(TX *TY / 2)
rbgs2_zmarch_deep(const T *__restrict__ uin, T *__restrict__ uout, const T *__restrict__ f, int n, T h2, int kchunk,
                  const T *__restrict__ uc, int nc, int nzc)
{
#pragma clang fp contract(off)
    constexpr int R = 4;
    constexpr int PX = TX + 2 * R, PY = TY + 2 * R, NT = TX * TY / 2;
    constexpr int PL = PX * PY;
    constexpr int FX = TX + 6, FY = TY + 6, FL = FX * FY;
    constexpr int NS = 6, NF = 4;
    constexpr int NL = (PL + NT - 1) / NT, NFL = (FL + NT - 1) / NT;
    __shared__ T pl[NS][PL];
    __shared__ T fp[NF][FL];
    const T sixth = T(1) / T(6);
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
    if (uin) uin += (size_t)pb * nn * n;   // a null uin (zero iterate) stays null
    uout += (size_t)pb * nn * n;
    f += (size_t)pb * nn * n;
    if (PROLONG) uc += (size_t)pb * nc * nc * nc;

    int goff[NL], gij[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int t = tid + r * NT;
        const int a = t % PX, b = t / PX;
        const int i = i0 - R + a, j = j0 - R + b;
        goff[r] = (t < PL && i >= 0 && i < n && j >= 0 && j < n) ? i + n * j : -1;
        gij[r] = (goff[r] >= 0 && i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) ? (i | (j << 16)) : -1;
    }
    int foff[NFL];
#pragma unroll
    for (int r = 0; r < NFL; ++r) {
        const int t = tid + r * NT;
        const int a = t % FX, b = t / FX;
        const int i = i0 - 3 + a, j = j0 - 3 + b;
        foff[r] = (t < FL && i >= 1 && i <= n - 2 && j >= 1 && j <= n - 2) ? i + n * j : -1;
    }
    auto fetch_u = [&](int k, T *vv) {
        const T *src = uin ? uin + (size_t)k * nn : nullptr;
        const bool inner_plane = k >= 1 && k <= n - 2;
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            T x = goff[r] >= 0 ? (src ? src[goff[r]] : T(0)) : T(0);
            if (PROLONG && inner_plane && gij[r] >= 0) x += prolong_at(nc, uc, gij[r] & 0xffff, gij[r] >> 16, k);
            vv[r] = x;
        }
    };
    auto commit_u = [&](int k, const T *vv) {
        T *P = pl[k % NS];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t < PL) P[t] = vv[r];
        }
    };
    auto fetch_f = [&](int k, T *ww) {
        const T *src = f + (size_t)k * nn;
#pragma unroll
        for (int r = 0; r < NFL; ++r) ww[r] = foff[r] >= 0 ? src[foff[r]] : T(0);
    };
    auto commit_f = [&](int k, const T *ww) {
        T *F = fp[k % NF];
#pragma unroll
        for (int r = 0; r < NFL; ++r) {
            const int t = tid + r * NT;
            if (t < FL) F[t] = ww[r];
        }
    };
    auto stage = [&](int k, int ring, int colour) {   // one colour of plane k on the tile plus `ring` nodes
        T *P = pl[k % NS];
        const T *Pm = pl[(k + NS - 1) % NS];
        const T *Pp = pl[(k + 1) % NS];
        const T *F = fp[k % NF];
        const int hw = (TX + 2 * ring) / 2, rows = TY + 2 * ring, a0 = R - ring;
        for (int t = tid; t < hw * rows; t += NT) {
            const int b = a0 + t / hw;
            const int j = j0 - R + b;
            const int ia0 = i0 - R + a0;
            const int a = a0 + (((ia0 + j + k) & 1) == colour ? 0 : 1) + 2 * (t % hw);
            const int i = i0 - R + a;
            if (i < 1 || i > n - 2 || j < 1 || j > n - 2) continue;
            const int c = b * PX + a;
            const T sum = P[c - 1] + P[c + 1] + P[c - PX] + P[c + PX] + Pm[c] + Pp[c];
            P[c] = (sum - h2 * F[(b - 1) * FX + (a - 1)]) * sixth;
        }
    };
    auto store = [&](int k) {
        const T *P = pl[k % NS];
        for (int t = tid; t < TX * TY; t += NT) {
            const int a = R + t % TX, b = R + t / TX;
            const int i = i0 - R + a, j = j0 - R + b;
            if (i > n - 2 || j > n - 2) continue;
            uout[(size_t)k * nn + i + (size_t)n * j] = P[b * PX + a];
        }
    };
    auto in_u = [&](int k) { return k >= max(0, kb - 4) && k <= min(n - 1, ke + 4); };
    auto in_f = [&](int k) { return k >= max(1, kb - 3) && k <= min(n - 2, ke + 3); };
    auto in_stage = [&](int k, int lag) { return k >= max(1, kb - lag) && k <= min(n - 2, ke + lag); };

    // step k stores u plane k+4 and f plane k+3 and requests u plane k+6 and
    // f plane k+5; set A serves the steps of kb's parity
    const int k0 = kb - 8;
    T uA[NL], uB[NL], fA[NFL], fB[NFL];
#pragma unroll
    for (int r = 0; r < NL; ++r) uA[r] = uB[r] = T(0);
#pragma unroll
    for (int r = 0; r < NFL; ++r) fA[r] = fB[r] = T(0);
    if (in_u(k0 + 4)) fetch_u(k0 + 4, uA);
    if (in_f(k0 + 3)) fetch_f(k0 + 3, fA);
    if (in_u(k0 + 5)) fetch_u(k0 + 5, uB);
    if (in_f(k0 + 4)) fetch_f(k0 + 4, fB);
    auto step = [&](int k, T *uX, T *fX) {
        if (in_u(k + 4)) commit_u(k + 4, uX);
        if (in_f(k + 3)) commit_f(k + 3, fX);
        if (in_u(k + 6)) fetch_u(k + 6, uX);
        if (in_f(k + 5)) fetch_f(k + 5, fX);
        __syncthreads();
        if (in_stage(k + 3, 3)) stage(k + 3, 3, 0);      // red, sweep A
        __syncthreads();
        if (in_stage(k + 2, 2)) stage(k + 2, 2, 1);      // black, sweep A
        __syncthreads();
        if (in_stage(k + 1, 1)) stage(k + 1, 1, 0);      // red, sweep B
        __syncthreads();
        if (k >= kb) {
            stage(k, 0, 1);                              // black, sweep B
            __syncthreads();
            store(k);
        }
    };
    for (int k = k0; k <= ke; k += 2) {
        step(k, uA, fA);
        if (k + 1 <= ke) step(k + 1, uB, fB);
    }
}

template <typename T, int TX, int TY>
static void rbgs2_deep_launch(int n, double h, const T *f, const T *uin, T *uout, int kchunk, const T *uc, int nb,
                              hipStream_t s)
{
    const int m = n - 2;
    const int nzc = (m + kchunk - 1) / kchunk;
    dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, nzc * nb);
    if (uc)
        hipLaunchKernelGGL((rbgs2_zmarch_deep<T, TX, TY, true>), grid, dim3(TX * TY / 2), 0, s, uin, uout, f, n,
                           T(h * h), kchunk, uc, (n + 1) / 2, nzc);
    else
        hipLaunchKernelGGL((rbgs2_zmarch_deep<T, TX, TY, false>), grid, dim3(TX * TY / 2), 0, s, uin, uout, f, n,
                           T(h * h), kchunk, uc, (n + 1) / 2, nzc);
}

template <typename T, int TX, int TY>
static void rbgs2_launch(int n, double h, const T *f, const T *uin, T *uout, int kchunk, const T *uc, int nb,
                         hipStream_t s)
{
    const int m = n - 2;
    const int nzc = (m + kchunk - 1) / kchunk;
    dim3 grid((m + TX - 1) / TX, (m + TY - 1) / TY, nzc * nb);
    if (uc)
        hipLaunchKernelGGL((rbgs2_zmarch<T, TX, TY, true>), grid, dim3(TX * TY), 0, s, uin, uout, f, n, T(h * h), kchunk,
                           uc, (n + 1) / 2, nzc);
    else
        hipLaunchKernelGGL((rbgs2_zmarch<T, TX, TY, false>), grid, dim3(TX * TY), 0, s, uin, uout, f, n, T(h * h),
                           kchunk, uc, (n + 1) / 2, nzc);
}

template <typename T>
void launch_rbgs2_shape(int n, double h, const T *f, const T *uin, T *uout, const T *uc, SmootherShape sh, hipStream_t s,
                        int nb)
{
    const int kc = sh.kchunk > 0 ? sh.kchunk : n;
    switch (sh.variant) {
    case 0: rbgs2_launch<T, 32, 8>(n, h, f, uin, uout, kc, uc, nb, s); break;
    case 2: brick_launch<T, 2>(n, h, f, uin, uout, uc, nb, s); break;
    case 3: brick_launch<T, 2, 4>(n, h, f, uin, uout, uc, nb, s); break;
    case 4: brick_launch<T, 2, 6>(n, h, f, uin, uout, uc, nb, s); break;
    case 5: rbgs2_deep_launch<T, 64, 16>(n, h, f, uin, uout, kc, uc, nb, s); break;
    case 6: rbgs2_deep_launch<T, 64, 8>(n, h, f, uin, uout, kc, uc, nb, s); break;
    case 7: rbgs2_deep_launch<T, 32, 16>(n, h, f, uin, uout, kc, uc, nb, s); break;
    case kSkewVariant: launch_rbgs2_skew<T>(n, h, f, uin, uout, s, nb, uc, 0); break;     // whole columns
    case kSkew32Variant: launch_rbgs2_skew<T>(n, h, f, uin, uout, s, nb, uc, 1); break;
    default: rbgs2_launch<T, 64, 4>(n, h, f, uin, uout, kc, uc, nb, s); break;
    }
}

template <typename T>
void launch_rbgs2(int n, double h, const T *f, const T *uin, T *uout, const T *uc, hipStream_t s, int nb)
{
    launch_rbgs2_shape<T>(n, h, f, uin, uout, uc, rbgs2_shape<T>(n), s, nb);
}

// Launch shapes of the smoother: tile variant and z-chunk per level size.
// Defaults below; the autotuner (tune.hip) overwrites entries after timing them.
static SmootherShape g_rbgs_shape[2][11];   // [fp32?][log2(n-1)]
static bool g_rbgs_init = false;

static void rbgs_defaults()
{
    for (int t = 0; t < 2; ++t)
        for (int J = 0; J <= 10; ++J) {
            SmootherShape &sh = g_rbgs_shape[t][J];
            if (J <= 5) sh = {0, 4};
            else if (J == 6) sh = {1, 8};
            else if (J == 7) sh = {1, 8};
            else if (J == 8) sh = {1, 32};
            else sh = {1, 64};
        }
    g_rbgs_init = true;
}

static SmootherShape g_rbgs2_shape[2][11];
static int g_use_fused[2][11] = {{1, 1, 1, 1, 1, 1, 1, 0, 0, 0, 0}, {1, 1, 1, 1, 1, 1, 1, 0, 0, 0, 0}};

template <typename T>
int &use_fused(int n)
{
    int J = 0;
    while ((1 << J) < n - 1) ++J;
    return g_use_fused[sizeof(T) == 4 ? 1 : 0][J > 10 ? 10 : J];
}

// Whether the coarse-grid correction of a level of n points runs as its own
// prolong-add launch before the post-smoothing (1) or is applied inside the
// first post-smoothing launch as planes are loaded (0, the default); both give
// the same values bit for bit.  Set by the autotuner per precision.
static int g_split_prolong[2][11] = {{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};

template <typename T>
int &split_prolong(int n)
{
    int J = 0;
    while ((1 << J) < n - 1) ++J;
    return g_split_prolong[sizeof(T) == 4 ? 1 : 0][J > 10 ? 10 : J];
}

// One flag for both precisions: the defaults of the whole table are written
// once, so an entry set for one precision is never reset by the first use of
// the other.
static bool g_rbgs2_init = false;

template <typename T>
SmootherShape &rbgs2_shape(int n)
{
    if (!g_rbgs2_init) {
        for (int t = 0; t < 2; ++t)
            for (int J = 0; J <= 10; ++J) {
                SmootherShape &sh = g_rbgs2_shape[t][J];
                if (J <= 5) sh = {0, 8};
                else if (J == 6) sh = {0, 16};
                else if (J == 7) sh = {1, 16};
                else sh = {1, 64};
            }
        g_rbgs2_init = true;
    }
    int J = 0;
    while ((1 << J) < n - 1) ++J;
    return g_rbgs2_shape[sizeof(T) == 4 ? 1 : 0][J > 10 ? 10 : J];
}

template <typename T>
SmootherShape &rbgs_shape(int n)
{
    if (!g_rbgs_init) rbgs_defaults();
    int J = 0;
    while ((1 << J) < n - 1) ++J;
    return g_rbgs_shape[sizeof(T) == 4 ? 1 : 0][J > 10 ? 10 : J];
}

// The correcting sweep's own shape per level and precision (the autotuner
// times it with the correction applied; -1: as the plain sweep).
static SmootherShape g_rbgs_corr_shape[2][11] = {
    {{-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}},
    {{-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}}};

template <typename T>
SmootherShape &rbgs_corr_shape(int n)
{
    int J = 0;
    while ((1 << J) < n - 1) ++J;
    return g_rbgs_corr_shape[sizeof(T) == 4 ? 1 : 0][J > 10 ? 10 : J];
}

template <typename T>
SmootherShape rbgs_corr_effective(int n)
{
    const SmootherShape c = rbgs_corr_shape<T>(n);
    return c.variant >= 0 ? c : rbgs_shape<T>(n);
}

template <typename T>
void launch_rbgs_shape(int n, double h, const T *f, const T *uin, T *uout, SmootherShape sh, hipStream_t s, int nb,
                       const T *uc)
{
    const int kc = sh.kchunk > 0 ? sh.kchunk : n;
    switch (sh.variant) {
    case 0: rbgs_launch<T, 32, 8>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 2: rbgs_launch<T, 64, 8>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 3: rbgs_launch<T, 128, 4>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 4: rbgs_launch<T, 32, 16>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 5: brick_launch<T, 1>(n, h, f, uin, uout, uc, nb, s); break;
    case 6: rbgs_pair_launch<T, 64, 8>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 7: rbgs_pair_launch<T, 64, 16>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 8: rbgs_pair_launch<T, 128, 8>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 9: brick_launch<T, 1, 4>(n, h, f, uin, uout, uc, nb, s); break;
    case 10: brick_launch<T, 1, 6>(n, h, f, uin, uout, uc, nb, s); break;
    case 11: rbgs_pair_launch<T, 32, 16>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 12: rbgs_pair_launch<T, 32, 8>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 13: rbgs_pair_deep_launch<T, 64, 16>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 14: rbgs_pair_deep_launch<T, 128, 8>(n, h, f, uin, uout, kc, nb, uc, s); break;
    case 15: rbgs_pair_deep_launch<T, 64, 32>(n, h, f, uin, uout, kc, nb, uc, s); break;
    default: rbgs_launch<T, 64, 4>(n, h, f, uin, uout, kc, nb, uc, s); break;
    }
}

template <typename T>
void launch_rbgs(int n, double h, const T *f, const T *uin, T *uout, hipStream_t s, int nb, const T *uc)
{
    launch_rbgs_shape<T>(n, h, f, uin, uout, uc ? rbgs_corr_effective<T>(n) : rbgs_shape<T>(n), s, nb, uc);
}

// ------------------------------------------------- residual and restriction

// Coarse node (I,J,K): fc = sum_{a,b,c} w_a w_b w_c r(2I+a, 2J+b, 2K+c) with
// r = f - A_h u, w = (1/4, 1/2, 1/4); coarse boundary 0.  Also zeroes the
// coarse correction (uc0 everywhere, uc1 on the boundary); with zu = 0 the
// interior of uc0 is left as it is, for a caller whose next use of the coarse
// correction takes it as zero without reading it (every residual-restriction
// kernel takes zu the same way).
template <typename T>
__global__ void residual_restrict_k(int nf, T ih2, const T *__restrict__ f, const T *__restrict__ u, T *__restrict__ fc,
                                    T *__restrict__ uc0, T *__restrict__ uc1, int zb, int zu)
{
#pragma clang fp contract(off)
    const int nc = (nf + 1) / 2;
    const int pb = blockIdx.z / zb;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = (blockIdx.z - pb * zb) * blockDim.z + threadIdx.z;
    if (I >= nc || J >= nc || K >= nc) return;
    const size_t Nf = (size_t)nf * nf * nf, Nc = (size_t)nc * nc * nc;
    f += pb * Nf;
    u += pb * Nf;
    fc += pb * Nc;
    uc0 += pb * Nc;
    if (uc1) uc1 += pb * Nc;
    const size_t C = id3(nc, I, J, K);
    const bool bnd = I == 0 || J == 0 || K == 0 || I == nc - 1 || J == nc - 1 || K == nc - 1;
    if (zu || bnd) uc0[C] = T(0);
    if (bnd) {
        if (uc1) uc1[C] = T(0);
        fc[C] = T(0);
        return;
    }
    const size_t sy = (size_t)nf, sz = (size_t)nf * nf;
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    T acc = T(0);
    for (int c = -1; c <= 1; ++c)
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) {
                const size_t p = id3(nf, 2 * I + a, 2 * J + b, 2 * K + c);
                const T lap = (u[p - 1] + u[p + 1] + u[p - sy] + u[p + sy] + u[p - sz] + u[p + sz] - T(6) * u[p]) * ih2;
                acc += (w[a + 1] * w[b + 1] * w[c + 1]) * (f[p] - lap);
            }
    fc[C] = acc;
}

template <typename T>
__global__ void restrict_k(int nf, const T *__restrict__ src, T *__restrict__ dst, int zb)
{
#pragma clang fp contract(off)
    const int nc = (nf + 1) / 2;
    const int pb = blockIdx.z / zb;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = (blockIdx.z - pb * zb) * blockDim.z + threadIdx.z;
    if (I >= nc || J >= nc || K >= nc) return;
    src += pb * (size_t)nf * nf * nf;
    dst += pb * (size_t)nc * nc * nc;
    const size_t C = id3(nc, I, J, K);
    if (I == 0 || J == 0 || K == 0 || I == nc - 1 || J == nc - 1 || K == nc - 1) {
        dst[C] = T(0);
        return;
    }
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    T acc = T(0);
    for (int c = -1; c <= 1; ++c)
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a)
                acc += (w[a + 1] * w[b + 1] * w[c + 1]) * src[id3(nf, 2 * I + a, 2 * J + b, 2 * K + c)];
    dst[C] = acc;
}

// Grid over an m^3 block of nodes for nb problems; zb = blocks per problem along z.
static dim3 grid3(int m, dim3 blk, int nb, int &zb)
{
    zb = (m + blk.z - 1) / blk.z;
    return dim3((m + blk.x - 1) / blk.x, (m + blk.y - 1) / blk.y, zb * nb);
}

// The same result with the fine block staged in LDS: a workgroup owns a
// CX x CY x CZ block of coarse nodes (8 x 8 x 4, or 4 x 4 x 4 and 4 x 4 x 2 for
// more workgroups on small levels), loads u on the fine nodes it needs plus a
// one-node ring and f on those nodes once, forms the fine residuals in LDS,
// and restricts them; each residual and each coarse sum is the same
// expression in the same order as in residual_restrict_k.
template <typename T, int CX, int CY, int CZ>
__global__ void __launch_bounds__(256)
residual_restrict_tile_k(int nf, T ih2, const T *__restrict__ f, const T *__restrict__ u, T *__restrict__ fc,
                         T *__restrict__ uc0, T *__restrict__ uc1, int tx, int ty, int tz, int zu)
{
#pragma clang fp contract(off)
    static_assert(CX * CY * CZ <= 256, "one coarse node per thread");
    constexpr int RX = 2 * CX + 1, RY = 2 * CY + 1, RZ = 2 * CZ + 1;   // fine residual region
    constexpr int UX = RX + 2, UY = RY + 2, UZ = RZ + 2;               // u region (one-node ring)
    __shared__ T Us[UX * UY * UZ];
    __shared__ T Rs[RX * RY * RZ];
    const int nc = (nf + 1) / 2;
    int bid = (int)xcd_tile(blockIdx.x, gridDim.x);
    const int bx = bid % tx;
    bid /= tx;
    const int by = bid % ty;
    bid /= ty;
    const int bz = bid % tz;
    const int pb = bid / tz;
    const size_t Nf = (size_t)nf * nf * nf, Nc = (size_t)nc * nc * nc;
    f += pb * Nf;
    u += pb * Nf;
    fc += pb * Nc;
    uc0 += pb * Nc;
    if (uc1) uc1 += pb * Nc;
    const int I0 = bx * CX, J0 = by * CY, K0 = bz * CZ;         // first coarse node of the block
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1, fk0 = 2 * K0 - 1;   // first fine node of the residual region
    // All of a lane's global loads go out before its first LDS store (clamped,
    // always in-bounds addresses; nodes outside the grid are zeroed after the load).
    constexpr int NU = (UX * UY * UZ + 255) / 256, NR = (RX * RY * RZ + 255) / 256;
    T xu[NU], xr[NR];
#pragma unroll
    for (int r = 0; r < NU; ++r) {
        const int t = min((int)threadIdx.x + r * 256, UX * UY * UZ - 1);
        const int a = t % UX, b = (t / UX) % UY, c = t / (UX * UY);
        const int i = fi0 - 1 + a, j = fj0 - 1 + b, k = fk0 - 1 + c;
        const bool in = i >= 0 && i < nf && j >= 0 && j < nf && k >= 0 && k < nf;
        const T x = u[id3(nf, min(max(i, 0), nf - 1), min(max(j, 0), nf - 1), min(max(k, 0), nf - 1))];
        xu[r] = in ? x : T(0);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int t = min((int)threadIdx.x + r * 256, RX * RY * RZ - 1);
        const int a = t % RX, b = (t / RX) % RY, c = t / (RX * RY);
        const int i = fi0 + a, j = fj0 + b, k = fk0 + c;
        const bool in = i >= 1 && i < nf - 1 && j >= 1 && j < nf - 1 && k >= 1 && k < nf - 1;
        const T x = f[id3(nf, min(max(i, 1), nf - 2), min(max(j, 1), nf - 2), min(max(k, 1), nf - 2))];
        xr[r] = in ? x : T(0);
    }
#pragma unroll
    for (int r = 0; r < NU; ++r)
        if ((int)threadIdx.x + r * 256 < UX * UY * UZ) Us[threadIdx.x + r * 256] = xu[r];
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if ((int)threadIdx.x + r * 256 < RX * RY * RZ) Rs[threadIdx.x + r * 256] = xr[r];
    __syncthreads();
    for (int t = threadIdx.x; t < RX * RY * RZ; t += 256) {
        const int a = t % RX, b = (t / RX) % RY, c = t / (RX * RY);
        const int i = fi0 + a, j = fj0 + b, k = fk0 + c;
        if (!(i >= 1 && i < nf - 1 && j >= 1 && j < nf - 1 && k >= 1 && k < nf - 1)) continue;
        const int q = (a + 1) + UX * ((b + 1) + UY * (c + 1));
        const T lap = (Us[q - 1] + Us[q + 1] + Us[q - UX] + Us[q + UX] + Us[q - UX * UY] + Us[q + UX * UY] -
                       T(6) * Us[q]) * ih2;
        Rs[t] = Rs[t] - lap;
    }
    __syncthreads();
    if ((int)threadIdx.x >= CX * CY * CZ) return;
    const int li = threadIdx.x % CX, lj = (threadIdx.x / CX) % CY, lk = threadIdx.x / (CX * CY);
    const int I = I0 + li, J = J0 + lj, K = K0 + lk;
    if (I >= nc || J >= nc || K >= nc) return;
    const size_t C = id3(nc, I, J, K);
    const bool bnd = I == 0 || J == 0 || K == 0 || I == nc - 1 || J == nc - 1 || K == nc - 1;
    if (zu || bnd) uc0[C] = T(0);
    if (bnd) {
        if (uc1) uc1[C] = T(0);
        fc[C] = T(0);
        return;
    }
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    T acc = T(0);
    for (int c = -1; c <= 1; ++c)
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a)
                acc += (w[a + 1] * w[b + 1] * w[c + 1]) * Rs[(2 * li + 1 + a) + RX * ((2 * lj + 1 + b) + RY * (2 * lk + 1 + c))];
    fc[C] = acc;
}

// Residual and restriction marching in z: a workgroup owns CX x CY coarse
// columns and a chunk of kc interior coarse planes.  For coarse plane K it
// loads u planes 2K+1 and 2K+2 into a ring of four LDS planes, forms the fine
// residuals of planes 2K and 2K+1 once each into a ring of three (plane 2K-1
// is kept from the step before), then restricts planes 2K-1..2K+1 to plane K.
// Every fine residual is formed once, with the expression and summation order
// of residual_restrict_k, so the two kernels give identical results.
// O1: tiles start at coarse column 1 rather than 0, so that 2^m interior-plus-
// one columns split into whole tiles (a 257^3 coarse grid into 8 x 32 tiles
// of 32 x 8, one workgroup per CU marching the whole column as the smoother
// does, neighbours on one XCD sharing their halos in L2); the owner of a
// column next to the low faces (I = 1 or J = 1) also zeroes the boundary
// column beyond it.  DEPTH 2, 3 or 4 fetches each step's planes that many
// steps ahead, into as many register sets used by the steps in turn.
template <typename T, int CX, int CY, int NT = 256, bool O1 = false, int DEPTH = 1>
__global__ void __launch_bounds__(NT)
residual_restrict_zmarch_k(int nf, T ih2, const T *__restrict__ f, const T *__restrict__ u, T *__restrict__ fc,
                           T *__restrict__ uc0, T *__restrict__ uc1, int tx, int ty, int tzc, int kc, int zu)
{
#pragma clang fp contract(off)
    constexpr int RX = 2 * CX + 1, RY = 2 * CY + 1, RP = RX * RY;   // fine residual region of a plane
    constexpr int UX = RX + 2, UY = RY + 2, UP = UX * UY;           // u region (one-node ring)
    constexpr int NU = (UP + NT - 1) / NT, NR = (RP + NT - 1) / NT;
    static_assert(CX * CY <= NT, "one coarse node per thread");
    __shared__ T Us[4][UP];
    __shared__ T Rs[3][RP];
    const int nc = (nf + 1) / 2;
    int bid = (int)xcd_tile(blockIdx.x, gridDim.x);
    const int bx = bid % tx;
    bid /= tx;
    const int by = bid % ty;
    bid /= ty;
    const int bz = bid % tzc;
    const int pb = bid / tzc;
    const size_t Nf = (size_t)nf * nf * nf, Nc = (size_t)nc * nc * nc;
    const size_t sy = (size_t)nf, sz = (size_t)nf * nf;
    f += pb * Nf;
    u += pb * Nf;
    fc += pb * Nc;
    uc0 += pb * Nc;
    if (uc1) uc1 += pb * Nc;
    const int tid = threadIdx.x;
    const int I0 = (O1 ? 1 : 0) + bx * CX, J0 = (O1 ? 1 : 0) + by * CY;
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1;   // origin of the fine residual region
    // this thread's share of a u plane and of a residual plane
    int uoff[NU], foff[NR], rq[NR];
#pragma unroll
    for (int r = 0; r < NU; ++r) {
        const int t = tid + r * NT;
        const int a = t % UX, b = t / UX;
        const int i = fi0 - 1 + a, j = fj0 - 1 + b;
        uoff[r] = (t < UP && i >= 0 && i < nf && j >= 0 && j < nf) ? i + nf * j : -1;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int t = tid + r * NT;
        const int a = t % RX, b = t / RX;
        const int i = fi0 + a, j = fj0 + b;
        foff[r] = (t < RP && i >= 1 && i <= nf - 2 && j >= 1 && j <= nf - 2) ? i + nf * j : -1;
        rq[r] = (a + 1) + UX * (b + 1);
    }
    // this thread's coarse node
    const int ci = tid % CX, cj = tid / CX;
    const int I = I0 + ci, J = J0 + cj;
    const bool c_thread = tid < CX * CY && I < nc && J < nc;
    const bool c_inner = c_thread && I >= 1 && I <= nc - 2 && J >= 1 && J <= nc - 2;
    const bool ex = O1 && c_thread && I == 1, ey = O1 && c_thread && J == 1;   // also own column 0 / row 0
    const int Kb = 1 + bz * kc, Ke = min(Kb + kc - 1, nc - 2);

    auto zero_at = [&](int Ix, int Jx, int K) {
        const size_t C = id3(nc, Ix, Jx, K);
        uc0[C] = T(0);
        if (uc1) uc1[C] = T(0);
        fc[C] = T(0);
    };
    auto zero_extra = [&](int K) {   // the boundary columns beyond this thread's (O1 tiles only)
        if (ex) zero_at(0, J, K);
        if (ey) zero_at(I, 0, K);
        if (ex && ey) zero_at(0, 0, K);
    };
    auto zero_node = [&](int K) {
        zero_at(I, J, K);
        zero_extra(K);
    };
    if (c_thread && bz == 0) zero_node(0);
    if (c_thread && bz == tzc - 1) zero_node(nc - 1);

    auto load_u = [&](int p) {
        T *U = Us[p & 3];
        const T *src = u + (size_t)p * sz;
#pragma unroll
        for (int r = 0; r < NU; ++r) {
            const int t = tid + r * NT;
            if (t < UP) U[t] = uoff[r] >= 0 ? src[uoff[r]] : T(0);
        }
    };
    auto load_f = [&](int p, T *fv) {
        const T *src = f + (size_t)p * sz;
#pragma unroll
        for (int r = 0; r < NR; ++r) fv[r] = foff[r] >= 0 ? src[foff[r]] : T(0);
    };
    auto resid = [&](int p, const T *fv) {
        const T *U = Us[p & 3];
        const T *Um = Us[(p - 1) & 3];
        const T *Up = Us[(p + 1) & 3];
        T *Rp = Rs[p % 3];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int t = tid + r * NT;
            if (t >= RP) continue;
            if (foff[r] < 0) {
                Rp[t] = T(0);
                continue;
            }
            const int q = rq[r];
            const T lap = (U[q - 1] + U[q + 1] + U[q - UX] + U[q + UX] + Um[q] + Up[q] - T(6) * U[q]) * ih2;
            Rp[t] = fv[r] - lap;
        }
    };
    auto restrict_plane = [&](int K) {
        if (!c_thread) return;
        if (!c_inner) {
            zero_node(K);
            return;
        }
        zero_extra(K);
        const T w[3] = {T(0.25), T(0.5), T(0.25)};
        T acc = T(0);
        for (int c = -1; c <= 1; ++c) {
            const T *Rp = Rs[(2 * K + c) % 3];
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a)
                    acc += (w[a + 1] * w[b + 1] * w[c + 1]) * Rp[(2 * ci + 1 + a) + RX * (2 * cj + 1 + b)];
        }
        const size_t C = id3(nc, I, J, K);
        if (zu) uc0[C] = T(0);
        fc[C] = acc;
    };

    // u planes 2K+1, 2K+2 and f planes 2K, 2K+1 of step K travel in registers
    // one step ahead: their loads are in flight while step K-1 computes
    T ua[NU], ub[NU], fa[NR], fb[NR];
    auto fetch_u = [&](int p, T *uv) {
        const T *src = u + (size_t)p * sz;
#pragma unroll
        for (int r = 0; r < NU; ++r) uv[r] = uoff[r] >= 0 ? src[uoff[r]] : T(0);
    };
    auto store_u = [&](int p, const T *uv) {
        T *U = Us[p & 3];
#pragma unroll
        for (int r = 0; r < NU; ++r) {
            const int t = tid + r * NT;
            if (t < UP) U[t] = uv[r];
        }
    };
    // warm-up: u planes 2Kb-2..2Kb and the residual of plane 2Kb-1
    load_u(2 * Kb - 2);
    load_u(2 * Kb - 1);
    load_u(2 * Kb);
    load_f(2 * Kb - 1, fa);
    __syncthreads();
    resid(2 * Kb - 1, fa);
    fetch_u(2 * Kb + 1, ua);
    fetch_u(2 * Kb + 2, ub);
    load_f(2 * Kb, fa);
    load_f(2 * Kb + 1, fb);
    __syncthreads();
    if constexpr (DEPTH == 1) {
        for (int K = Kb; K <= Ke; ++K) {
            store_u(2 * K + 1, ua);   // slots of planes 2K-3 and 2K-2, last read before the previous barrier
            store_u(2 * K + 2, ub);
            T fc0[NR], fc1[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                fc0[r] = fa[r];
                fc1[r] = fb[r];
            }
            if (K + 1 <= Ke) {   // the next step's planes, in flight during this one
                fetch_u(2 * K + 3, ua);
                fetch_u(2 * K + 4, ub);
                load_f(2 * K + 2, fa);
                load_f(2 * K + 3, fb);
            }
            __syncthreads();
            resid(2 * K, fc0);
            resid(2 * K + 1, fc1);
            __syncthreads();
            restrict_plane(K);
        }
    } else {
        // step K's planes sit in register set (K - Kb) mod DEPTH, fetched DEPTH steps ahead
        T ua2[NU], ub2[NU], fa2[NR], fb2[NR], ua3[NU], ub3[NU], fa3[NR], fb3[NR], ua4[NU], ub4[NU], fa4[NR], fb4[NR];
        auto fetch_step = [&](int K, T *xa, T *xb, T *ya, T *yb) {
            fetch_u(2 * K + 1, xa);
            fetch_u(2 * K + 2, xb);
            load_f(2 * K, ya);
            load_f(2 * K + 1, yb);
        };
        if (Kb + 1 <= Ke) fetch_step(Kb + 1, ua2, ub2, fa2, fb2);
        if (DEPTH >= 3 && Kb + 2 <= Ke) fetch_step(Kb + 2, ua3, ub3, fa3, fb3);
        if (DEPTH >= 4 && Kb + 3 <= Ke) fetch_step(Kb + 3, ua4, ub4, fa4, fb4);
        auto step = [&](int K, T *xa, T *xb, T *ya, T *yb) {
            store_u(2 * K + 1, xa);
            store_u(2 * K + 2, xb);
            T fc0[NR], fc1[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                fc0[r] = ya[r];
                fc1[r] = yb[r];
            }
            if (K + DEPTH <= Ke) fetch_step(K + DEPTH, xa, xb, ya, yb);   // into the set just emptied
            __syncthreads();
            resid(2 * K, fc0);
            resid(2 * K + 1, fc1);
            __syncthreads();
            restrict_plane(K);
        };
        for (int K = Kb; K <= Ke; K += DEPTH) {
            step(K, ua, ub, fa, fb);
            if (K + 1 <= Ke) step(K + 1, ua2, ub2, fa2, fb2);
            if (DEPTH >= 3 && K + 2 <= Ke) step(K + 2, ua3, ub3, fa3, fb3);
            if (DEPTH >= 4 && K + 3 <= Ke) step(K + 3, ua4, ub4, fa4, fb4);
        }
    }
}

// Which residual-restriction kernel a fine level of n points uses (0: per-node
// gather, 1: 8x8x4 LDS tile, 2/3/4: z-march over chunks of 4/8/16 coarse planes,
// 5: 4x4x4, 6: 4x4x2 LDS tiles, 7/8: whole-column z-march of 32x8 / 64x4
// columns with 512 threads loading two steps ahead, 9: 32x8 columns over
// 64-plane chunks, 10/11: 32x8 whole columns loading three / four steps
// ahead), per
// precision; set by the autotuner, gather by default.
static int g_rr_variant[2][11] = {{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};

template <typename T>
int &rr_variant(int nf)
{
    int J = 0;
    while ((1 << J) < nf - 1) ++J;
    return g_rr_variant[sizeof(T) == 4 ? 1 : 0][J > 10 ? 10 : J];
}

template <typename T>
void launch_residual_restrict_variant(int nf, double h, const T *f, const T *u, T *fc, T *uc0, T *uc1, int variant,
                                      hipStream_t s, int nb, bool zero_u)
{
    const int zu = zero_u ? 1 : 0;
    const int nc = (nf + 1) / 2;
    if (variant == 0) {
        dim3 blk(16, 4, 4);
        int zb;
        const dim3 g = grid3(nc, blk, nb, zb);
        hipLaunchKernelGGL(residual_restrict_k<T>, g, blk, 0, s, nf, T(1.0 / (h * h)), f, u, fc, uc0, uc1, zb, zu);
        return;
    }
    if (variant >= 2 && variant <= 4) {   // z-march with chunks of 4, 8 or 16 coarse planes
        constexpr int CX = 16, CY = 8;
        const int kc = variant == 2 ? 4 : (variant == 3 ? 8 : 16);
        const int tx = (nc + CX - 1) / CX, ty = (nc + CY - 1) / CY, tzc = (nc - 2 + kc - 1) / kc;
        const dim3 g((unsigned)((size_t)tx * ty * tzc * nb));
        hipLaunchKernelGGL((residual_restrict_zmarch_k<T, CX, CY>), g, dim3(256), 0, s, nf, T(1.0 / (h * h)), f, u, fc,
                           uc0, uc1, tx, ty, tzc, kc, zu);
        return;
    }
    if (variant >= 7 && variant <= 11) {   // tiles from coarse column 1 (see residual_restrict_zmarch_k)
        const T ih2 = T(1.0 / (h * h));
        if (variant == 8) {   // 64 x 4 columns, whole column, two steps ahead, 512 threads
            constexpr int CX = 64, CY = 4;
            const int tx = (nc - 1 + CX - 1) / CX, ty = (nc - 1 + CY - 1) / CY;
            const dim3 g((unsigned)((size_t)tx * ty * nb));
            hipLaunchKernelGGL((residual_restrict_zmarch_k<T, CX, CY, 512, true, 2>), g, dim3(512), 0, s, nf, ih2, f,
                               u, fc, uc0, uc1, tx, ty, 1, nc - 2, zu);
            return;
        }
        constexpr int CX = 32, CY = 8;
        const int tx = (nc - 1 + CX - 1) / CX, ty = (nc - 1 + CY - 1) / CY;
        if (variant == 7) {   // 32 x 8 columns, whole column, two steps ahead, 512 threads
            const dim3 g((unsigned)((size_t)tx * ty * nb));
            hipLaunchKernelGGL((residual_restrict_zmarch_k<T, CX, CY, 512, true, 2>), g, dim3(512), 0, s, nf, ih2, f,
                               u, fc, uc0, uc1, tx, ty, 1, nc - 2, zu);
            return;
        }
        if (variant == 10 || variant == 11) {   // 32 x 8 columns, whole column, three / four steps ahead
            const dim3 g((unsigned)((size_t)tx * ty * nb));
            if (variant == 10)
                hipLaunchKernelGGL((residual_restrict_zmarch_k<T, CX, CY, 512, true, 3>), g, dim3(512), 0, s, nf, ih2,
                                   f, u, fc, uc0, uc1, tx, ty, 1, nc - 2, zu);
            else
                hipLaunchKernelGGL((residual_restrict_zmarch_k<T, CX, CY, 512, true, 4>), g, dim3(512), 0, s, nf, ih2,
                                   f, u, fc, uc0, uc1, tx, ty, 1, nc - 2, zu);
            return;
        }
        const int kc = 64, tzc = (nc - 2 + kc - 1) / kc;   // 32 x 8 columns, 64-plane chunks, 256 threads
        const dim3 g((unsigned)((size_t)tx * ty * tzc * nb));
        hipLaunchKernelGGL((residual_restrict_zmarch_k<T, CX, CY, 256, true, 1>), g, dim3(256), 0, s, nf, ih2, f, u,
                           fc, uc0, uc1, tx, ty, tzc, kc, zu);
        return;
    }
    if (variant == 5) {   // 4 x 4 x 4 coarse tiles
        const int tx = (nc + 3) / 4, ty = (nc + 3) / 4, tz = (nc + 3) / 4;
        const dim3 g((unsigned)((size_t)tx * ty * tz * nb));
        hipLaunchKernelGGL((residual_restrict_tile_k<T, 4, 4, 4>), g, dim3(256), 0, s, nf, T(1.0 / (h * h)), f, u, fc,
                           uc0, uc1, tx, ty, tz, zu);
        return;
    }
    if (variant == 6) {   // 4 x 4 x 2 coarse tiles
        const int tx = (nc + 3) / 4, ty = (nc + 3) / 4, tz = (nc + 1) / 2;
        const dim3 g((unsigned)((size_t)tx * ty * tz * nb));
        hipLaunchKernelGGL((residual_restrict_tile_k<T, 4, 4, 2>), g, dim3(256), 0, s, nf, T(1.0 / (h * h)), f, u, fc,
                           uc0, uc1, tx, ty, tz, zu);
        return;
    }
    const int tx = (nc + 7) / 8, ty = (nc + 7) / 8, tz = (nc + 3) / 4;
    const dim3 g((unsigned)((size_t)tx * ty * tz * nb));
    hipLaunchKernelGGL((residual_restrict_tile_k<T, 8, 8, 4>), g, dim3(256), 0, s, nf, T(1.0 / (h * h)), f, u, fc, uc0,
                       uc1, tx, ty, tz, zu);
}

template <typename T>
void launch_residual_restrict(int nf, double h, const T *f, const T *u, T *fc, T *uc0, T *uc1, hipStream_t s, int nb,
                              bool zero_u)
{
    launch_residual_restrict_variant<T>(nf, h, f, u, fc, uc0, uc1, rr_variant<T>(nf), s, nb, zero_u);
}

template <typename T>
void launch_restrict(int nf, const T *src, T *dst, hipStream_t s, int nb)
{
    const int nc = (nf + 1) / 2;
    dim3 blk(16, 4, 4);
    int zb;
    const dim3 g = grid3(nc, blk, nb, zb);
    hipLaunchKernelGGL(restrict_k<T>, g, blk, 0, s, nf, src, dst, zb);
}

// ------------------------------------------------------------- prolongation

// One thread per pair of fine nodes along x, i = 2q + 1 (between coarse
// nodes q and q + 1) and i = 2q + 2 (on coarse node q + 1): both read the same
// two coarse values per (j, k) row, so a pair takes 8 coarse loads instead of
// 16.  Each fine value is the expression of prolong_at with its weights, in the
// same order, so the result equals prolong_at's bit for bit.
template <typename T, bool ADD>
__global__ void __launch_bounds__(256) prolong_k(int nc, const T *__restrict__ uc, T *__restrict__ uf, int zb)
{
#pragma clang fp contract(off)
    const int nf = 2 * nc - 1;
    const int pb = blockIdx.z / zb;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    const int k = 1 + (blockIdx.z - pb * zb) * blockDim.z + threadIdx.z;
    if (q > nc - 2 || j > nf - 2 || k > nf - 2) return;
    uc += pb * (size_t)nc * nc * nc;
    uf += pb * (size_t)nf * nf * nf;
    const int ja = j >> 1, jb = (j + 1) >> 1, ka = k >> 1, kb = (k + 1) >> 1;
    const T wja = (j & 1) ? T(0.5) : T(1), wjb = (j & 1) ? T(0.5) : T(0);
    const T wka = (k & 1) ? T(0.5) : T(1), wkb = (k & 1) ? T(0.5) : T(0);
    const T a0 = uc[id3(nc, q, ja, ka)], a1 = uc[id3(nc, q + 1, ja, ka)];
    const T b0 = uc[id3(nc, q, jb, ka)], b1 = uc[id3(nc, q + 1, jb, ka)];
    const T c0 = uc[id3(nc, q, ja, kb)], c1 = uc[id3(nc, q + 1, ja, kb)];
    const T d0 = uc[id3(nc, q, jb, kb)], d1 = uc[id3(nc, q + 1, jb, kb)];
    const T h = T(0.5), one = T(1), zero = T(0);
    const size_t p = id3(nf, 2 * q + 1, j, k);
    T vo, ve = T(0);
    {   // odd i: weights 1/2, 1/2 between coarse q and q + 1
        const T xa = h * a0 + h * a1, xb = h * b0 + h * b1, xc = h * c0 + h * c1, xd = h * d0 + h * d1;
        vo = wka * (wja * xa + wjb * xb) + wkb * (wja * xc + wjb * xd);
    }
    const bool even = 2 * q + 2 <= nf - 2;
    if (even) {   // even i: coarse q + 1 with weights 1, 0
        const T xa = one * a1 + zero * a1, xb = one * b1 + zero * b1, xc = one * c1 + zero * c1,
                xd = one * d1 + zero * d1;
        ve = wka * (wja * xa + wjb * xb) + wkb * (wja * xc + wjb * xd);
    }
    // the pair is adjacent in memory: one two-element access (aligned to one
    // element only) instead of two half-filled strided ones
    typedef T pair_t __attribute__((ext_vector_type(2), aligned(sizeof(T))));
    if (even) {
        pair_t *dst = reinterpret_cast<pair_t *>(uf + p);
        pair_t o;
        if (ADD) {
            o = *dst;
            o.x += vo;
            o.y += ve;
        } else {
            o.x = vo;
            o.y = ve;
        }
        *dst = o;
    } else if (ADD) {
        uf[p] += vo;
    } else {
        uf[p] = vo;
    }
}

template <typename T, bool ADD>
static void launch_prolong(int nc, const T *uc, T *uf, hipStream_t s, int nb)
{
    const int nf = 2 * nc - 1;
    const dim3 blk(64, 2, 2);
    const int zb = (nf - 2 + 1) / 2;
    const dim3 g((unsigned)((nc - 1 + 63) / 64), (unsigned)((nf - 2 + 1) / 2), (unsigned)(zb * nb));
    hipLaunchKernelGGL((prolong_k<T, ADD>), g, blk, 0, s, nc, uc, uf, zb);
}

template <typename T>
void launch_prolong_add(int nc, const T *uc, T *uf, hipStream_t s, int nb)
{
    launch_prolong<T, true>(nc, uc, uf, s, nb);
}

template <typename T>
void launch_interp(int nc, const T *uc, T *uf, hipStream_t s, int nb)
{
    launch_prolong<T, false>(nc, uc, uf, s, nb);
}

// ------------------------------------------------------- boundary helpers

// Boundary node number t in [0, 6 n^2) -> (i,j,k); edges are visited more
// than once, always with the same value.
__device__ __forceinline__ void face_node(int n, int t, int &i, int &j, int &k)
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

template <typename T>
__global__ void inject_boundary_k(int nfine, const T *__restrict__ ufine, int nl, T *__restrict__ u0, T *__restrict__ u1)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * nl * nl) return;
    const size_t Nl = (size_t)nl * nl * nl;
    ufine += blockIdx.y * (size_t)nfine * nfine * nfine;
    u0 += blockIdx.y * Nl;
    if (u1) u1 += blockIdx.y * Nl;
    int i, j, k;
    face_node(nl, t, i, j, k);
    const int st = (nfine - 1) / (nl - 1);
    const T v = ufine[id3(nfine, i * st, j * st, k * st)];
    u0[id3(nl, i, j, k)] = v;
    if (u1) u1[id3(nl, i, j, k)] = v;
}

template <typename T>
void launch_inject_boundary(int nfine, const T *ufine, int nl, T *u0, T *u1, hipStream_t s, int nb)
{
    const int cnt = 6 * nl * nl;
    hipLaunchKernelGGL(inject_boundary_k<T>, dim3((cnt + 255) / 256, nb), dim3(256), 0, s, nfine, ufine, nl, u0, u1);
}

template <typename T>
__global__ void boundary_copy_k(int n, const T *__restrict__ src, T *__restrict__ dst)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * n * n) return;
    int i, j, k;
    face_node(n, t, i, j, k);
    dst[id3(n, i, j, k)] = src[id3(n, i, j, k)];
}

template <typename T>
void launch_boundary_copy(int n, const T *src, T *dst, hipStream_t s)
{
    const int cnt = 6 * n * n;
    hipLaunchKernelGGL(boundary_copy_k<T>, dim3((cnt + 255) / 256), dim3(256), 0, s, n, src, dst);
}

template <typename T>
__global__ void fill_k(T *p, size_t count, T v)
{
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x)
        p[t] = v;
}

template <typename T>
void launch_fill(T *p, size_t count, T v, hipStream_t s)
{
    size_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) return;
    hipLaunchKernelGGL(fill_k<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
}

// ------------------------------------------------------------- coarse tail
//
// Every level with at most 17 points per side lives in the LDS of a single
// workgroup (u and f of 17^3, 9^3, 5^3, 3^3: 5794 values each), so a V-cycle
// or a whole FMG over these levels is one launch.  Level l has 2^l + 1 points.

constexpr int kTailTop = 4;              // 17^3
constexpr int kTailThreads = 1024;
__host__ __device__ constexpr int tail_off(int l)
{
    return l <= 1 ? 0 : tail_off(l - 1) + ((1 << (l - 1)) + 1) * ((1 << (l - 1)) + 1) * ((1 << (l - 1)) + 1);
}
constexpr int kTailSize = tail_off(kTailTop + 1);
constexpr int kTailTopN = (1 << kTailTop) + 1;

// Lanes of the 1024-thread workgroup cover a 16 x 16 x 4 brick of nodes (i, j
// from the lane, k strided by 4); colour passes use 8 x 16 x 8 with two nodes of
// one colour per row pair.  Every level is a compile-time template argument, so
// all node indexing folds to constants.
template <typename T>
struct TailLDS {
    T *U, *F, *R;
    T L;
    int npre, npost;
    T *h2, *ih2;   // in LDS: h^2 and 1/h^2 per level, h = L / (n - 1)

    __device__ void init_h() const   // by one thread, before the first barrier
    {
        for (int l = 1; l <= kTailTop; ++l) {
            const T h = L / T((1 << l));
            h2[l] = h * h;
            ih2[l] = T(1) / (h * h);
        }
    }
    template <int LV> __device__ T *u() const { return U + tail_off(LV); }
    template <int LV> __device__ T *fr() const { return F + tail_off(LV); }

    template <int LV>
    __device__ void gs(int colour) const
    {
#pragma clang fp contract(off)
        constexpr int n = (1 << LV) + 1, m = n - 2;
        const T hh = h2[LV], sixth = T(1) / T(6);
        T *uu = u<LV>();
        const T *ff = fr<LV>();
        const int tx = threadIdx.x & 7, ty = (threadIdx.x >> 3) & 15, tz = threadIdx.x >> 7;
        const int j = 1 + ty;
        if (j <= m) {
#pragma unroll
            for (int k = 1 + tz; k <= m; k += 8) {
                const int i = 1 + 2 * tx + ((colour + 1 + j + k) & 1);
                if (i > m) continue;
                const int p = i + n * (j + n * k);
                const T s = uu[p - 1] + uu[p + 1] + uu[p - n] + uu[p + n] + uu[p - n * n] + uu[p + n * n];
                uu[p] = (s - hh * ff[p]) * sixth;
            }
        }
        __syncthreads();
    }
    template <int LV>
    __device__ void sweeps(int ns) const
    {
        for (int s = 0; s < ns; ++s) {
            gs<LV>(0);
            gs<LV>(1);
        }
    }
    // exact solve of the single interior node of the 3^3 level, in FP64
    __device__ void exact() const
    {
#pragma clang fp contract(off)
        if (threadIdx.x == 0) {
            T *uu = u<1>();
            const T *ff = fr<1>();
            const double h = double(L) / 2.0;
            const int p = 13;
            const double s = double(uu[p - 1]) + double(uu[p + 1]) + double(uu[p - 3]) + double(uu[p + 3]) +
                             double(uu[p - 9]) + double(uu[p + 9]);
            uu[p] = T((s - h * h * double(ff[p])) / 6.0);
        }
        __syncthreads();
    }
    // fc = FW(f - A u) on level LV-1 and uc = 0: the residual of level LV is staged in R
    template <int LV>
    __device__ void resid_restrict() const
    {
#pragma clang fp contract(off)
        constexpr int n = (1 << LV) + 1, m = n - 2, nc = (1 << (LV - 1)) + 1;
        const T ih = ih2[LV];
        const T *uu = u<LV>();
        const T *ff = fr<LV>();
        const int li = threadIdx.x & 15, lj = (threadIdx.x >> 4) & 15, lk = threadIdx.x >> 8;
        if (li < m && lj < m) {
            const int i = 1 + li, j = 1 + lj;
            for (int k = 1 + lk; k <= m; k += 4) {
                const int p = i + n * (j + n * k);
                R[p] = ff[p] - (uu[p - 1] + uu[p + 1] + uu[p - n] + uu[p + n] + uu[p - n * n] + uu[p + n * n] -
                                T(6) * uu[p]) * ih;
            }
        }
        __syncthreads();
        T *fc = fr<LV - 1>();
        T *uc = u<LV - 1>();
        const T w[3] = {T(0.25), T(0.5), T(0.25)};
        if (li < nc && lj < nc) {
            for (int K = lk; K < nc; K += 4) {
                const int C = li + nc * (lj + nc * K);
                uc[C] = T(0);
                if (li == 0 || lj == 0 || K == 0 || li == nc - 1 || lj == nc - 1 || K == nc - 1) {
                    fc[C] = T(0);
                    continue;
                }
                T acc = T(0);
                for (int c = -1; c <= 1; ++c)
                    for (int b = -1; b <= 1; ++b)
                        for (int a = -1; a <= 1; ++a)
                            acc += (w[a + 1] * w[b + 1] * w[c + 1]) * R[(2 * li + a) + n * ((2 * lj + b) + n * (2 * K + c))];
                fc[C] = acc;
            }
        }
        __syncthreads();
    }
    template <int LV>
    __device__ void restrict_f() const   // f_{LV-1} = FW(f_LV)
    {
#pragma clang fp contract(off)
        constexpr int n = (1 << LV) + 1, nc = (1 << (LV - 1)) + 1;
        const T *ff = fr<LV>();
        T *fc = fr<LV - 1>();
        const T w[3] = {T(0.25), T(0.5), T(0.25)};
        const int li = threadIdx.x & 15, lj = (threadIdx.x >> 4) & 15, lk = threadIdx.x >> 8;
        if (li < nc && lj < nc) {
            for (int K = lk; K < nc; K += 4) {
                const int C = li + nc * (lj + nc * K);
                if (li == 0 || lj == 0 || K == 0 || li == nc - 1 || lj == nc - 1 || K == nc - 1) {
                    fc[C] = T(0);
                    continue;
                }
                T acc = T(0);
                for (int c = -1; c <= 1; ++c)
                    for (int b = -1; b <= 1; ++b)
                        for (int a = -1; a <= 1; ++a)
                            acc += (w[a + 1] * w[b + 1] * w[c + 1]) * ff[(2 * li + a) + n * ((2 * lj + b) + n * (2 * K + c))];
                fc[C] = acc;
            }
        }
        __syncthreads();
    }
    template <int LC>
    __device__ void prolong(bool add) const   // level LC -> LC+1 interior
    {
        constexpr int nc = (1 << LC) + 1, n = (1 << (LC + 1)) + 1, m = n - 2;
        const T *uc = u<LC>();
        T *uf = u<LC + 1>();
        const int li = threadIdx.x & 15, lj = (threadIdx.x >> 4) & 15, lk = threadIdx.x >> 8;
        if (li < m && lj < m) {
            const int i = 1 + li, j = 1 + lj;
            for (int k = 1 + lk; k <= m; k += 4) {
                const T v = prolong_at(nc, uc, i, j, k);
                const int p = i + n * (j + n * k);
                uf[p] = add ? uf[p] + v : v;
            }
        }
        __syncthreads();
    }
    template <int LV, int TOP>
    __device__ void inject() const   // boundary of level LV from level TOP, interior 0
    {
        constexpr int n = (1 << LV) + 1, nt = (1 << TOP) + 1, st = (nt - 1) / (n - 1);
        T *uu = u<LV>();
        const T *ut = u<TOP>();
        const int li = threadIdx.x & 15, lj = (threadIdx.x >> 4) & 15, lk = threadIdx.x >> 8;
        if (li < n && lj < n) {
            for (int k = lk; k < n; k += 4) {
                const bool bnd = li == 0 || lj == 0 || k == 0 || li == n - 1 || lj == n - 1 || k == n - 1;
                uu[li + n * (lj + n * k)] = bnd ? ut[(li * st) + nt * ((lj * st) + nt * (k * st))] : T(0);
            }
        }
        __syncthreads();
    }
    template <int LV>
    __device__ void down() const
    {
        if constexpr (LV >= 2) {
            sweeps<LV>(npre);
            resid_restrict<LV>();
            down<LV - 1>();
        }
    }
    template <int LV, int TOP>
    __device__ void up() const
    {
        if constexpr (LV <= TOP) {
            prolong<LV - 1>(true);
            sweeps<LV>(npost);
            up<LV + 1, TOP>();
        }
    }
    template <int TOP>
    __device__ void vcycle() const
    {
        down<TOP>();
        exact();
        up<2, TOP>();
    }
    template <int LV, int TOP>
    __device__ void restrict_all() const   // f of TOP-1 .. 1 from TOP
    {
        if constexpr (LV >= 2) {
            restrict_f<LV>();
            restrict_all<LV - 1, TOP>();
        }
    }
    template <int LV, int TOP>
    __device__ void inject_all() const
    {
        if constexpr (LV < TOP) {
            inject<LV, TOP>();
            inject_all<LV + 1, TOP>();
        }
    }
    template <int LV, int TOP>
    __device__ void fmg_up(int ncycle) const
    {
        if constexpr (LV <= TOP) {
            prolong<LV - 1>(false);
            for (int c = 0; c < ncycle; ++c) vcycle<LV>();
            fmg_up<LV + 1, TOP>(ncycle);
        }
    }
    template <int TOP>
    __device__ void run(int mode, int ncycle, int nrep) const
    {
        if (mode == 1) {
            restrict_all<TOP, TOP>();
            inject_all<1, TOP>();
            exact();
            fmg_up<2, TOP>(ncycle);
        } else {
            for (int r = 0; r < nrep; ++r) vcycle<TOP>();
        }
    }
};

template <typename T>
__global__ void __launch_bounds__(kTailThreads)
coarse_tail_k(int top, T L, const T *__restrict__ fg, T *__restrict__ ug, int npre, int npost, int ncycle, int mode,
              int nrep)
{
    __shared__ T U[kTailSize];
    __shared__ T F[kTailSize];
    __shared__ T Rs[kTailTopN * kTailTopN * kTailTopN];
    __shared__ T hs[2][kTailTop + 1];
    TailLDS<T> t{U, F, Rs, L, npre, npost, hs[0], hs[1]};
    if (threadIdx.x == 0) t.init_h();
    const int n = (1 << top) + 1, cnt = n * n * n;
    fg += (size_t)blockIdx.x * cnt;
    ug += (size_t)blockIdx.x * cnt;
    T *utop = U + tail_off(top), *ftop = F + tail_off(top);
    const bool uzero = mode == 2;   // a correction V-cycle whose iterate is known to be zero: not read
    // all global loads of a lane first, then its LDS stores (overlapped latency)
    constexpr int NL = (kTailTopN * kTailTopN * kTailTopN + kTailThreads - 1) / kTailThreads;
    T xu[NL], xf[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int p = min((int)threadIdx.x + r * kTailThreads, cnt - 1);
        xu[r] = uzero ? T(0) : ug[p];
        xf[r] = fg[p];
    }
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int p = threadIdx.x + r * kTailThreads;
        if (p < cnt) {
            utop[p] = xu[r];
            ftop[p] = xf[r];
        }
    }
    __syncthreads();
    const int md = mode == 1 ? 1 : 0;
    switch (top) {
    case 1: t.template run<1>(md, ncycle, nrep); break;
    case 2: t.template run<2>(md, ncycle, nrep); break;
    case 3: t.template run<3>(md, ncycle, nrep); break;
    default: t.template run<4>(md, ncycle, nrep); break;
    }
    for (int p = threadIdx.x; p < cnt; p += blockDim.x) ug[p] = utop[p];
}

template <typename T>
void launch_coarse_tail(int ltop, double L, const T *f, T *u, int npre, int npost, int ncycle, int mode, int nrep,
                        hipStream_t s, int nb)
{
    hipLaunchKernelGGL(coarse_tail_k<T>, dim3(nb), dim3(kTailThreads), 0, s, ltop, T(L), f, u, npre, npost, ncycle,
                       mode, nrep);
}

// ------------------------------------------------------------------ norms

template <int NT>
__device__ __forceinline__ void block_sum3(double *sh, double &a, double &b, double &c)
{
    sh[threadIdx.x] = a;
    sh[NT + threadIdx.x] = b;
    sh[2 * NT + threadIdx.x] = c;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[threadIdx.x] += sh[threadIdx.x + w];
            sh[NT + threadIdx.x] += sh[NT + threadIdx.x + w];
            sh[2 * NT + threadIdx.x] += sh[2 * NT + threadIdx.x + w];
        }
        __syncthreads();
    }
    a = sh[0];
    b = sh[NT];
    c = sh[2 * NT];
}

// Per-block partial sums over interior nodes of (f - A_h u)^2, f^2 and the
// squared boundary-value contribution (sum of boundary neighbours / h^2),
// which scales the stopping test of a source-free box.  A workgroup is 4 rows
// of 64 lanes: each lane row walks x along one interior (j, k) row (coalesced),
// the workgroups stride over the rows; the summation order depends only on n
// and the block count, so the norms are reproducible bit for bit.  With R32
// the pass also writes the residual times 1/s (sc[2p + 1]) rounded to FP32 at
// every interior node, the right-hand side of the next refinement step of a
// mixed solve (the value resid_to_f32_k forms, saving that pass).
template <typename T, bool R32>
__global__ void __launch_bounds__(256)
resid_norms_partial_k(int n, double ih2, const T *__restrict__ f, const T *__restrict__ u, double *__restrict__ partial,
                      const double *__restrict__ sc, float *__restrict__ r32)
{
    __shared__ double sh[768];
    const int m = n - 2;
    const unsigned rows = (unsigned)m * (unsigned)m;
    const size_t sy = (size_t)n, sz = (size_t)n * n;
    f += blockIdx.y * sz * n;
    u += blockIdx.y * sz * n;
    partial += blockIdx.y * 3 * (size_t)gridDim.x;
    double inv_s = 0.0;
    if (R32) {
        r32 += blockIdx.y * sz * n;
        inv_s = sc[2 * blockIdx.y + 1];
    }
    const int lane = threadIdx.x & 63, ty = threadIdx.x >> 6;
    double sr = 0.0, sf = 0.0, sb = 0.0;
    for (unsigned r = blockIdx.x * 4u + (unsigned)ty; r < rows; r += gridDim.x * 4u) {
        const unsigned kq = r / (unsigned)m;              // one division per row
        const int j = 1 + (int)(r - kq * (unsigned)m), k = 1 + (int)kq;
        const bool jk_edge = j == 1 || k == 1 || j == n - 2 || k == n - 2;
        const size_t row = id3(n, 0, j, k);
        for (int i = 1 + lane; i <= n - 2; i += 64) {
            const size_t p = row + (size_t)i;
            const double um = u[p - 1], up = u[p + 1], vm = u[p - sy], vp = u[p + sy], wm = u[p - sz], wp = u[p + sz];
            const double lap = (um + up + vm + vp + wm + wp - 6.0 * (double)u[p]) * ih2;
            const double fv = (double)f[p];
            const double res = fv - lap;
            if (R32) r32[p] = (float)(res * inv_s);
            sr += res * res;
            sf += fv * fv;
            if (jk_edge || i == 1 || i == n - 2) {
                const double b = ((i == 1 ? um : 0.0) + (i == n - 2 ? up : 0.0) + (j == 1 ? vm : 0.0) +
                                  (j == n - 2 ? vp : 0.0) + (k == 1 ? wm : 0.0) + (k == n - 2 ? wp : 0.0)) * ih2;
                sb += b * b;
            }
        }
    }
    block_sum3<256>(sh, sr, sf, sb);
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x] = sr;
        partial[3 * blockIdx.x + 1] = sf;
        partial[3 * blockIdx.x + 2] = sb;
    }
}

// The same partial sums from a z-march: a workgroup owns a 64 x 4 column tile
// of interior nodes and a chunk of z planes, holds three planes of u (tile
// plus a one-node ring) in LDS and loads each plane once, with the next plane
// and the next f values in flight while a plane is summed, so u and f are
// read from HBM about once (the row form reads the +-z neighbour rows again,
// from other workgroups at other times).  Each lane sums its own column; the
// order depends only on n and the launch shape, which the launcher fixes from
// n, so the sums are reproducible bit for bit.  Same residual expression, same
// FP32 residual with R32.
constexpr int kNzTX = 64, kNzTY = 4;

template <typename T, bool R32>
__global__ void __launch_bounds__(kNzTX *kNzTY)
resid_norms_zmarch_k(int n, double ih2, const T *__restrict__ f, const T *__restrict__ u,
                     double *__restrict__ partial, const double *__restrict__ sc, float *__restrict__ r32, int kchunk,
                     int gx, int gy)
{
    constexpr int TX = kNzTX, TY = kNzTY, PX = TX + 2, PY = TY + 2, PL = PX * PY, NT = TX * TY;
    constexpr int NL = (PL + NT - 1) / NT;
    __shared__ double pl[3][PL];
    __shared__ double sh[3 * NT];
    const size_t nn = (size_t)n * n;
    f += blockIdx.y * nn * n;
    u += blockIdx.y * nn * n;
    partial += blockIdx.y * 3 * (size_t)gridDim.x;
    double inv_s = 0.0;
    if (R32) {
        r32 += blockIdx.y * nn * n;
        inv_s = sc[2 * blockIdx.y + 1];
    }
    const int tid = threadIdx.x;
    const int b = blockIdx.x, bx = b % gx, by = (b / gx) % gy, bz = b / (gx * gy);
    const int i0 = 1 + bx * TX, j0 = 1 + by * TY;
    const int kb = 1 + bz * kchunk, ke = min(kb + kchunk - 1, n - 2);
    int goff[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const int t = tid + r * NT;
        const int i = i0 - 1 + t % PX, j = j0 - 1 + t / PX;
        goff[r] = (t < PL && i < n && j < n) ? i + n * j : -1;
    }
    double v[NL];
    auto fetch = [&](int k) {
        const T *src = u + (size_t)k * nn;
#pragma unroll
        for (int r = 0; r < NL; ++r) v[r] = goff[r] >= 0 ? (double)src[goff[r]] : 0.0;
    };
    auto commit = [&](int k) {
        double *D = pl[k % 3];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = tid + r * NT;
            if (t < PL) D[t] = v[r];
        }
    };
    const int a = tid % TX, bq = tid / TX;
    const int i = i0 + a, j = j0 + bq;
    const bool own = i <= n - 2 && j <= n - 2 && kb <= ke;
    const int c = (bq + 1) * PX + (a + 1);
    const size_t col = (size_t)i + (size_t)n * j;
    const bool ij_edge = i == 1 || j == 1 || i == n - 2 || j == n - 2;
    double sr = 0.0, sf = 0.0, sb = 0.0;
    if (kb <= ke) {
        {   // planes kb-1, kb, kb+1: all loads in flight before the first store
            double w[3][NL];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const T *src = u + (size_t)(kb - 1 + q) * nn;
#pragma unroll
                for (int r = 0; r < NL; ++r) w[q][r] = goff[r] >= 0 ? (double)src[goff[r]] : 0.0;
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
        if (kb + 2 <= ke + 1) fetch(kb + 2);
        double fv = own ? (double)f[(size_t)kb * nn + col] : 0.0;
        __syncthreads();
        for (int k = kb; k <= ke; ++k) {
            const double fn = (own && k + 1 <= ke) ? (double)f[(size_t)(k + 1) * nn + col] : 0.0;
            if (own) {
                const double *M = pl[(k - 1) % 3], *Z = pl[k % 3], *Q = pl[(k + 1) % 3];
                const double um = Z[c - 1], up = Z[c + 1], vm = Z[c - PX], vp = Z[c + PX], wm = M[c], wp = Q[c];
                const double lap = (um + up + vm + vp + wm + wp - 6.0 * Z[c]) * ih2;
                const double res = fv - lap;
                if (R32) r32[(size_t)k * nn + col] = (float)(res * inv_s);
                sr += res * res;
                sf += fv * fv;
                if (ij_edge || k == 1 || k == n - 2) {
                    const double bv = ((i == 1 ? um : 0.0) + (i == n - 2 ? up : 0.0) + (j == 1 ? vm : 0.0) +
                                       (j == n - 2 ? vp : 0.0) + (k == 1 ? wm : 0.0) + (k == n - 2 ? wp : 0.0)) * ih2;
                    sb += bv * bv;
                }
            }
            fv = fn;
            __syncthreads();
            if (k + 2 <= ke + 1) {   // plane k+2 replaces plane k-1, whose readers are past the barrier
                commit(k + 2);
                if (k + 3 <= ke + 1) fetch(k + 3);
            }
            __syncthreads();
        }
    }
    block_sum3<NT>(sh, sr, sf, sb);
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x] = sr;
        partial[3 * blockIdx.x + 1] = sf;
        partial[3 * blockIdx.x + 2] = sb;
    }
}

// Launch shape of the z-march norms for n: tiles of 64 x 4 columns and the
// z-chunk that keeps the block count at most kNormBlocks (and the chunks at
// least 8 planes); 0 blocks when the tiles alone exceed kNormBlocks (the row
// form serves then).
struct NormsShape {
    int gx, gy, kchunk, nzc, blocks;
};
static NormsShape norms_shape(int n)
{
    NormsShape sh;
    const int m = n - 2;
    sh.gx = (m + kNzTX - 1) / kNzTX;
    sh.gy = (m + kNzTY - 1) / kNzTY;
    const int tiles = sh.gx * sh.gy;
    if (tiles > kNormBlocks) {
        sh.kchunk = sh.nzc = sh.blocks = 0;
        return sh;
    }
    const int q = kNormBlocks / tiles;
    sh.kchunk = std::max(8, (m + q - 1) / q);
    sh.nzc = (m + sh.kchunk - 1) / sh.kchunk;
    sh.blocks = tiles * sh.nzc;
    return sh;
}

// hout (optional): the same three sums per problem, written straight into
// pinned host memory (its device-mapped address), so no copy launch follows.
__global__ void __launch_bounds__(256) norms_final_k(const double *__restrict__ partial, int nb, double *__restrict__ out,
                                                     double *__restrict__ hout)
{
    __shared__ double sh[768];
    partial += blockIdx.x * 3 * (size_t)nb;
    out += 3 * blockIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int t = threadIdx.x; t < nb; t += 256) {
        a += partial[3 * t];
        b += partial[3 * t + 1];
        c += partial[3 * t + 2];
    }
    block_sum3<256>(sh, a, b, c);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
        out[2] = c;
        if (hout) {
            hout += 3 * blockIdx.x;
            hout[0] = a;
            hout[1] = b;
            hout[2] = c;
            __threadfence_system();
        }
    }
}

template <typename T>
void launch_resid_norms(int n, double h, const T *f, const T *u, double *partial, double *out, hipStream_t s, int nb,
                        double *hout)
{
    const NormsShape zs = norms_shape(n);
    if (zs.blocks > 0) {
        hipLaunchKernelGGL((resid_norms_zmarch_k<T, false>), dim3(zs.blocks, nb), dim3(kNzTX * kNzTY), 0, s, n,
                           1.0 / (h * h), f, u, partial, nullptr, nullptr, zs.kchunk, zs.gx, zs.gy);
        hipLaunchKernelGGL(norms_final_k, dim3(nb), dim3(256), 0, s, partial, zs.blocks, out, hout);
        return;
    }
    // about 8 four-row groups per workgroup, at most kNormBlocks workgroups per problem
    const long long rows = (long long)(n - 2) * (n - 2);
    const int blocks = (int)std::min<long long>(kNormBlocks, std::max<long long>(1, (rows + 31) / 32));
    hipLaunchKernelGGL((resid_norms_partial_k<T, false>), dim3(blocks, nb), dim3(256), 0, s, n, 1.0 / (h * h), f, u,
                       partial, nullptr, nullptr);
    hipLaunchKernelGGL(norms_final_k, dim3(nb), dim3(256), 0, s, partial, blocks, out, hout);
}

void launch_resid_norms_r32(int n, double h, const double *f, const double *u, double *partial, double *out,
                            const double *sc, float *r32, hipStream_t s, int nb, double *hout)
{
    const NormsShape zs = norms_shape(n);
    if (zs.blocks > 0) {
        hipLaunchKernelGGL((resid_norms_zmarch_k<double, true>), dim3(zs.blocks, nb), dim3(kNzTX * kNzTY), 0, s, n,
                           1.0 / (h * h), f, u, partial, sc, r32, zs.kchunk, zs.gx, zs.gy);
        hipLaunchKernelGGL(norms_final_k, dim3(nb), dim3(256), 0, s, partial, zs.blocks, out, hout);
        return;
    }
    const long long rows = (long long)(n - 2) * (n - 2);
    const int blocks = (int)std::min<long long>(kNormBlocks, std::max<long long>(1, (rows + 31) / 32));
    hipLaunchKernelGGL((resid_norms_partial_k<double, true>), dim3(blocks, nb), dim3(256), 0, s, n, 1.0 / (h * h), f,
                       u, partial, sc, r32);
    hipLaunchKernelGGL(norms_final_k, dim3(nb), dim3(256), 0, s, partial, blocks, out, hout);
}

// ------------------------------------------------- mixed-precision helpers
//
// FP64 residual-correction refinement around FP32 multigrid: the FP64 iterate
// is corrected by s e where e solves A e = r / s in FP32 (zero Dirichlet
// values) and s is the power of two at or below the RMS of the FP64 residual
// r = f - A u over the interior (1 if that is 0 or not finite).  Scaling by a
// power of two is exact, and every FP32 multigrid operation commutes with it,
// so the corrected iterate does not depend on which power of two scales a
// step (values far from the FP32 subnormal range): a step may take its scale
// from the norms before the previous correction, which lets the norms pass
// of one step write the next step's scaled residual.  s and 1/s are computed
// on the device from the residual norms, so no host round trip sits between
// the steps.

__global__ void narrow_k(const double *__restrict__ src, float *__restrict__ dst, size_t count)
{
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x)
        dst[t] = (float)src[t];
}

__global__ void narrow_boundary_k(int n, const double *__restrict__ src, float *__restrict__ d0, float *__restrict__ d1)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * n * n) return;
    int i, j, k;
    face_node(n, t, i, j, k);
    const size_t p = id3(n, i, j, k) + blockIdx.y * (size_t)n * n * n;
    const float v = (float)src[p];
    d0[p] = v;
    if (d1) d1[p] = v;
}

// u64 interior = (double) u32
__global__ void widen_interior_k(int n, const float *__restrict__ src, double *__restrict__ dst, int zb)
{
    const int pb = blockIdx.z / zb;
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    const int k = 1 + (blockIdx.z - pb * zb) * blockDim.z + threadIdx.z;
    if (i > n - 2 || j > n - 2 || k > n - 2) return;
    const size_t p = id3(n, i, j, k) + pb * (size_t)n * n * n;
    dst[p] = (double)src[p];
}

// sc[2p] = s, sc[2p+1] = 1/s for problem p from its residual norms (3 per problem)
__global__ void mixed_scale_k(int n, int nb, const double *__restrict__ norms, double *__restrict__ sc)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nb) return;
    const double nint = (double)(n - 2) * (double)(n - 2) * (double)(n - 2);
    const double rms = sqrt(norms[3 * p] / nint);
    const int e = (rms > 0.0 && isfinite(rms)) ? ilogb(rms) : 0;
    sc[2 * p] = ldexp(1.0, e);
    sc[2 * p + 1] = ldexp(1.0, -e);
}

// r32 = (f - A_h u) / s in FP64, rounded to FP32, at interior nodes; 0 on the boundary
__global__ void resid_to_f32_k(int n, double ih2, const double *__restrict__ sc, const double *__restrict__ f,
                               const double *__restrict__ u, float *__restrict__ r, int zb)
{
    const int pb = blockIdx.z / zb;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = (blockIdx.z - pb * zb) * blockDim.z + threadIdx.z;
    if (i >= n || j >= n || k >= n) return;
    const double inv_s = sc[2 * pb + 1];
    const size_t p = id3(n, i, j, k) + pb * (size_t)n * n * n;
    if (i == 0 || j == 0 || k == 0 || i == n - 1 || j == n - 1 || k == n - 1) {
        r[p] = 0.0f;
        return;
    }
    const size_t sy = (size_t)n, sz = (size_t)n * n;
    const double lap = (u[p - 1] + u[p + 1] + u[p - sy] + u[p + sy] + u[p - sz] + u[p + sz] - 6.0 * u[p]) * ih2;
    r[p] = (float)((f[p] - lap) * inv_s);
}

// u64 += s e32 at interior nodes
__global__ void correct_k(int n, const double *__restrict__ sc, const float *__restrict__ e, double *__restrict__ u, int zb)
{
    const int pb = blockIdx.z / zb;
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    const int k = 1 + (blockIdx.z - pb * zb) * blockDim.z + threadIdx.z;
    if (i > n - 2 || j > n - 2 || k > n - 2) return;
    const size_t p = id3(n, i, j, k) + pb * (size_t)n * n * n;
    u[p] += sc[2 * pb] * (double)e[p];
}

void launch_narrow(const double *src, float *dst, size_t count, hipStream_t s)
{
    size_t blocks = (count + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(narrow_k, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, count);
}

void launch_narrow_boundary(int n, const double *src, float *d0, float *d1, hipStream_t s, int nb)
{
    const int cnt = 6 * n * n;
    hipLaunchKernelGGL(narrow_boundary_k, dim3((cnt + 255) / 256, nb), dim3(256), 0, s, n, src, d0, d1);
}

void launch_widen_interior(int n, const float *src, double *dst, hipStream_t s, int nb)
{
    dim3 blk(64, 2, 2);
    int zb;
    const dim3 g = grid3(n - 2, blk, nb, zb);
    hipLaunchKernelGGL(widen_interior_k, g, blk, 0, s, n, src, dst, zb);
}

void launch_mixed_scale(int n, const double *norms, double *sc, hipStream_t s, int nb)
{
    hipLaunchKernelGGL(mixed_scale_k, dim3((nb + 63) / 64), dim3(64), 0, s, n, nb, norms, sc);
}

void launch_resid_to_f32(int n, double h, const double *sc, const double *f, const double *u, float *r, hipStream_t s,
                         int nb)
{
    dim3 blk(64, 2, 2);
    int zb;
    const dim3 g = grid3(n, blk, nb, zb);
    hipLaunchKernelGGL(resid_to_f32_k, g, blk, 0, s, n, 1.0 / (h * h), sc, f, u, r, zb);
}

void launch_correct(int n, const double *sc, const float *e, double *u, hipStream_t s, int nb)
{
    dim3 blk(64, 2, 2);
    int zb;
    const dim3 g = grid3(n - 2, blk, nb, zb);
    hipLaunchKernelGGL(correct_k, g, blk, 0, s, n, sc, e, u, zb);
}

// Interior of u (FP64) from an initial guess of storage type T (boundary kept).
template <typename T>
__global__ void guess_interior_k(int n, const T *__restrict__ g, double *__restrict__ u)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    const int k = 1 + blockIdx.z * blockDim.z + threadIdx.z;
    if (i > n - 2 || j > n - 2 || k > n - 2) return;
    const size_t p = id3(n, i, j, k);
    u[p] = (double)(float)g[p];
}

template <>
__global__ void guess_interior_k<double>(int n, const double *__restrict__ g, double *__restrict__ u)
{
    const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = 1 + blockIdx.y * blockDim.y + threadIdx.y;
    const int k = 1 + blockIdx.z * blockDim.z + threadIdx.z;
    if (i > n - 2 || j > n - 2 || k > n - 2) return;
    const size_t p = id3(n, i, j, k);
    u[p] = g[p];
}

void launch_guess_interior(int n, const void *g, int kind, double *u, hipStream_t s)
{
    dim3 blk(64, 2, 2);
    int zb;
    const dim3 gr = grid3(n - 2, blk, 1, zb);
    if (kind == 1) hipLaunchKernelGGL(guess_interior_k<double>, gr, blk, 0, s, n, (const double *)g, u);
    else if (kind == 2) hipLaunchKernelGGL(guess_interior_k<float>, gr, blk, 0, s, n, (const float *)g, u);
    else hipLaunchKernelGGL(guess_interior_k<__bf16>, gr, blk, 0, s, n, (const __bf16 *)g, u);
}

// -------------------------------------------------------- instantiations
#define QM_INST(T)                                                                                              \
    template void launch_rbgs<T>(int, double, const T *, const T *, T *, hipStream_t, int, const T *);         \
    template SmootherShape &rbgs_corr_shape<T>(int);                                                            \
    template SmootherShape rbgs_corr_effective<T>(int);                                                         \
    template void launch_rbgs_shape<T>(int, double, const T *, const T *, T *, SmootherShape, hipStream_t, int,  \
                                       const T *);                                                              \
    template SmootherShape &rbgs_shape<T>(int);                                                                 \
    template SmootherShape &rbgs2_shape<T>(int);                                                                \
    template int &use_fused<T>(int);                                                                            \
    template int &split_prolong<T>(int);                                                                        \
    template void launch_rbgs2<T>(int, double, const T *, const T *, T *, const T *, hipStream_t, int);        \
    template void launch_rbgs2_shape<T>(int, double, const T *, const T *, T *, const T *, SmootherShape,        \
                                        hipStream_t, int);                                                      \
    template void launch_residual_restrict<T>(int, double, const T *, const T *, T *, T *, T *, hipStream_t,    \
                                              int, bool);                                                       \
    template void launch_residual_restrict_variant<T>(int, double, const T *, const T *, T *, T *, T *, int,     \
                                                      hipStream_t, int, bool);                                  \
    template int &rr_variant<T>(int);                                                                           \
    template void launch_restrict<T>(int, const T *, T *, hipStream_t, int);                                   \
    template void launch_prolong_add<T>(int, const T *, T *, hipStream_t, int);                                \
    template void launch_interp<T>(int, const T *, T *, hipStream_t, int);                                     \
    template void launch_inject_boundary<T>(int, const T *, int, T *, T *, hipStream_t, int);                  \
    template void launch_fill<T>(T *, size_t, T, hipStream_t);                                                 \
    template void launch_boundary_copy<T>(int, const T *, T *, hipStream_t);                                   \
    template void launch_coarse_tail<T>(int, double, const T *, T *, int, int, int, int, int, hipStream_t, int);\
    template void launch_resid_norms<T>(int, double, const T *, const T *, double *, double *, hipStream_t, int,    \
                                        double *);
QM_INST(double)
QM_INST(float)
#undef QM_INST
template void launch_fill<long long>(long long *, size_t, long long, hipStream_t);
template void launch_fill<unsigned long long>(unsigned long long *, size_t, unsigned long long, hipStream_t);

}  // namespace qm
