// Kernels of the 3D U-Net that predicts the QUMOND potential from (Phi_N,
// source) as an initial guess for the second multigrid solve.
//
// Tensors are channel-last BF16 on vertex-centred n^3 grids: element (v, c)
// of a tensor with slot width `cs` sits at v * cs + c (v = i + n (j + n k)), so
// a tensor can be a channel slice of a wider one (skip connections are
// written straight into the concatenated input of the decoder convolution).
// Slot widths and channel offsets are multiples of 8 (16-byte fragments).
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation: rows = 16 output voxels, columns = 16 output channels,
// K = 27 taps x input channels (padded to a multiple of 32).  With the lane
// layout of that instruction, lane l supplies row/column l % 16 and the
// eight consecutive K indices 8 (l / 16) .. 8 (l / 16) + 7, which are eight
// consecutive channels of one tap: one 16-byte load.  The 4 accumulators of
// lane l are column l % 16, rows 4 (l / 16) + r.
#include "common.h"
#include "unet.h"

namespace qm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ void decode3(int v, int n, int &i, int &j, int &k)
{
    i = v % n;
    const int t = v / n;
    j = t % n;
    k = t / n;
}

// ------------------------------------------------------------ convolution

// y[v, co] = act(bias[co] + sum_{tap, ci} x[s v + d(tap), ci] W[co, tap cin + ci])
//
// Each wave computes RB blocks of 16 consecutive output voxels for all cout
// = 16 NB channels: per K-chunk it loads RB activation fragments and NB weight
// fragments and issues RB x NB MFMAs, and it loads the next chunk's fragments
// before the current chunk's MFMAs.  Every output is accumulated over the
// K-chunks in the same order whatever RB is.
template <int NB, int RB>
__global__ void __launch_bounds__(256)
conv3d_fwd_k(Tensor x, int cin, const __bf16 *__restrict__ wt, int kpad, const float *__restrict__ bias, Tensor y,
             int stride, int relu)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nout = y.n, nin = x.n;
    const int Nout = nout * nout * nout;
    const int v0 = (blockIdx.x * 4 + wave) * 16 * RB;
    if (v0 >= Nout) return;
    const int g = lane >> 4, r16 = lane & 15;
    int bi[RB], bj[RB], bk[RB];
    bool ok[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int va = v0 + 16 * rb + r16;
        int io = 0, jo = 0, ko = 0;
        ok[rb] = va < Nout;
        if (ok[rb]) decode3(va, nout, io, jo, ko);
        bi[rb] = stride * io;
        bj[rb] = stride * jo;
        bk[rb] = stride * ko;
    }
    const int kreal = 27 * cin;
    const size_t xcs = (size_t)x.cs;
    // K index of this lane's fragment in the current chunk, as (tap, channel)
    int kk0 = 8 * g, tap = kk0 / cin, c0 = kk0 - tap * cin;
    auto load = [&](bf16x8 *a, bf16x8 *w) {
        const bool live = kk0 < kreal;
        const int di = tap % 3 - 1, dj = (tap / 3) % 3 - 1, dk = tap / 9 - 1;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            bf16x8 t = {};
            const int i = bi[rb] + di, j = bj[rb] + dj, k = bk[rb] + dk;
            if (live && ok[rb] && i >= 0 && i < nin && j >= 0 && j < nin && k >= 0 && k < nin)
                t = *reinterpret_cast<const bf16x8 *>(x.p + (size_t)(i + nin * (j + nin * k)) * xcs + c0);
            a[rb] = t;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b)
            w[b] = *reinterpret_cast<const bf16x8 *>(wt + (size_t)(b * 16 + r16) * kpad + kk0);
        kk0 += 32;
        c0 += 32;
        while (c0 >= cin) {
            c0 -= cin;
            ++tap;
        }
    };
    f32x4 acc[RB][NB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[rb][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 a[RB], w[NB];
    load(a, w);
    for (int kc = 0; kc < kpad; kc += 32) {
        bf16x8 an[RB], wn[NB];
        if (kc + 32 < kpad) load(an, wn);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[rb][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb], w[b], acc[rb][b], 0, 0, 0);
        if (kc + 32 < kpad) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) a[rb] = an[rb];
#pragma unroll
            for (int b = 0; b < NB; ++b) w[b] = wn[b];
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int co = b * 16 + r16;
        const float bb = bias ? bias[co] : 0.f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int v = v0 + 16 * rb + 4 * g + r;
                if (v >= Nout) continue;
                float val = acc[rb][b][r] + bb;
                if (relu) val = val > 0.f ? val : 0.f;
                y.p[(size_t)v * y.cs + co] = (__bf16)val;
            }
    }
}

// Stride-1 convolution with the input tile in LDS: a workgroup computes a
// 16 x 4 x 4 block of output voxels (each wave 4 x-rows of 16 voxels, one
// MFMA row block each) for all cout = 16 NB channels.  The input channels are
// taken in chunks of up to 32; for each chunk the 18 x 6 x 6 input voxels
// (block plus a one-voxel ring) are staged in LDS once and every one of the
// 27 taps reads its activation fragments from there.  Within a chunk of cc
// channels the K-steps of 32 cover 32 / cc taps at a time (cc = 8, 16 or 32),
// in the same (tap, channel) order as conv3d_fwd_k.
constexpr int kTileX = 16, kTileY = 4, kTileZ = 4;
constexpr int kInX = kTileX + 2, kInY = kTileY + 2, kInZ = kTileZ + 2, kInV = kInX * kInY * kInZ;
constexpr int kChunk = 32, kPitch = kChunk + 8;   // bf16 per staged voxel (padded against bank conflicts)

template <int NB>
__global__ void __launch_bounds__(256)
conv3d_fwd_lds_k(Tensor x, int cin, const __bf16 *__restrict__ wt, int kpad, const float *__restrict__ bias, Tensor y,
                 int relu, int tx, int ty)
{
    constexpr int RB = 4;
    __shared__ __bf16 tile[kInV * kPitch];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int n = y.n;   // = x.n (stride 1)
    int bid = blockIdx.x;
    const int bx = bid % tx;
    bid /= tx;
    const int by = bid % ty;
    const int bz = bid / ty;
    const int X0 = bx * kTileX, Y0 = by * kTileY, Z0 = bz * kTileZ;
    const size_t xcs = (size_t)x.cs;
    f32x4 acc[RB][NB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[rb][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    // this lane's rows: wave w, row block rb -> output row (y, z) = (rb, w) of the block, x = r16
    for (int cb = 0; cb < cin; cb += kChunk) {
        const int cc = min(kChunk, cin - cb);     // 8, 16 or 32 (cin is a multiple of 8; chunks of 32 then the rest)
        const int g8 = cc / 8;
        __syncthreads();
        for (int t = threadIdx.x; t < kInV * g8; t += 256) {
            const int v = t / g8, q = t - v * g8;
            const int a = v % kInX, b = (v / kInX) % kInY, c = v / (kInX * kInY);
            const int i = X0 - 1 + a, j = Y0 - 1 + b, k = Z0 - 1 + c;
            bf16x8 val = {};
            if (i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n)
                val = *reinterpret_cast<const bf16x8 *>(x.p + (size_t)(i + n * (j + n * k)) * xcs + cb + 8 * q);
            *reinterpret_cast<bf16x8 *>(tile + v * kPitch + 8 * q) = val;
        }
        __syncthreads();
        const int steps = (27 * cc + 31) / 32;
        // fragments of K-step st (activations from the tile, weights from global)
        auto frags = [&](int st, bf16x8 *a, bf16x8 *w) {
            const int kl = 32 * st + 8 * g;        // local K index of this lane's fragment
            const int tap = kl / cc, cl = kl - tap * cc;
            const bool live = tap < 27;
            const int dx = tap % 3, dy = (tap / 3) % 3, dz = tap / 9;   // offsets + 1
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int v = (r16 + dx) + kInX * ((rb + dy) + kInY * (wave + dz));
                a[rb] = live ? *reinterpret_cast<const bf16x8 *>(tile + v * kPitch + cl) : bf16x8{};
            }
            const int kw = live ? tap * cin + cb + cl : 0;
#pragma unroll
            for (int b = 0; b < NB; ++b)
                w[b] = live ? *reinterpret_cast<const bf16x8 *>(wt + (size_t)(b * 16 + r16) * kpad + kw) : bf16x8{};
        };
        bf16x8 a[RB], w[NB];
        frags(0, a, w);
        for (int st = 0; st < steps; ++st) {
            bf16x8 an[RB], wn[NB];
            if (st + 1 < steps) frags(st + 1, an, wn);   // in flight during this step's MFMAs
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[rb][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb], w[b], acc[rb][b], 0, 0, 0);
            if (st + 1 < steps) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) a[rb] = an[rb];
#pragma unroll
                for (int b = 0; b < NB; ++b) w[b] = wn[b];
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int co = b * 16 + r16;
        const float bb = bias ? bias[co] : 0.f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int j = Y0 + rb, k = Z0 + wave;
            if (j >= n || k >= n) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = X0 + 4 * g + r;
                if (i >= n) continue;
                float val = acc[rb][b][r] + bb;
                if (relu) val = val > 0.f ? val : 0.f;
                y.p[(size_t)(i + n * (j + n * k)) * y.cs + co] = (__bf16)val;
            }
        }
    }
}

template <int NB>
static void conv_fwd_nb(Tensor x, int cin, const __bf16 *wt, int kpad, const float *bias, Tensor y, int stride,
                        int relu, hipStream_t s)
{
    const int Nout = y.n * y.n * y.n;
    if (stride == 1 && NB <= 4 && (cin % 32 == 0 || cin == 8 || cin == 16 || cin == 48)) {
        const int tx = (y.n + kTileX - 1) / kTileX, ty = (y.n + kTileY - 1) / kTileY, tz = (y.n + kTileZ - 1) / kTileZ;
        hipLaunchKernelGGL((conv3d_fwd_lds_k<NB <= 4 ? NB : 4>), dim3((unsigned)(tx * ty * tz)), dim3(256), 0, s, x,
                           cin, wt, kpad, bias, y, relu, tx, ty);
        return;
    }
    // RB row blocks per wave while the grid keeps at least ~1024 workgroups
    if (Nout >= 1024 * 256 && NB <= 4) {
        hipLaunchKernelGGL((conv3d_fwd_k<NB, 4>), dim3((Nout + 255) / 256), dim3(256), 0, s, x, cin, wt, kpad, bias, y,
                           stride, relu);
    } else if (Nout >= 1024 * 128) {
        hipLaunchKernelGGL((conv3d_fwd_k<NB, 2>), dim3((Nout + 127) / 128), dim3(256), 0, s, x, cin, wt, kpad, bias, y,
                           stride, relu);
    } else {
        hipLaunchKernelGGL((conv3d_fwd_k<NB, 1>), dim3((Nout + 63) / 64), dim3(256), 0, s, x, cin, wt, kpad, bias, y,
                           stride, relu);
    }
}

void launch_conv3d_fwd(Tensor x, int cin, const __bf16 *wt, int kpad, int cout, const float *bias, Tensor y,
                       int stride, int relu, hipStream_t s)
{
    switch (cout / 16) {
    case 1: conv_fwd_nb<1>(x, cin, wt, kpad, bias, y, stride, relu, s); break;
    case 2: conv_fwd_nb<2>(x, cin, wt, kpad, bias, y, stride, relu, s); break;
    case 3: conv_fwd_nb<3>(x, cin, wt, kpad, bias, y, stride, relu, s); break;
    case 4: conv_fwd_nb<4>(x, cin, wt, kpad, bias, y, stride, relu, s); break;
    case 6: conv_fwd_nb<6>(x, cin, wt, kpad, bias, y, stride, relu, s); break;
    case 8: conv_fwd_nb<8>(x, cin, wt, kpad, bias, y, stride, relu, s); break;
    default: break;   // rejected by the caller
    }
}

// Weights for the input gradient: W'[ci, tap' cout + co] = W[co, tap cin + ci],
// tap' = 26 - tap (the mirrored offset), so dx = conv(dy, W') with stride 1.
__global__ void dgrad_weights_k(const __bf16 *__restrict__ wt, int cin, int cout, int kpad, __bf16 *__restrict__ wd,
                                int kpad_d)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cin * kpad_d) return;
    const int ci = t / kpad_d, kk = t - ci * kpad_d;
    __bf16 v = (__bf16)0.f;
    if (kk < 27 * cout) {
        const int tapd = kk / cout, co = kk - tapd * cout;
        v = wt[(size_t)co * kpad + (26 - tapd) * cin + ci];
    }
    wd[t] = v;
}

void launch_dgrad_weights(const __bf16 *wt, int cin, int cout, int kpad, __bf16 *wd, int kpad_d, hipStream_t s)
{
    const int cnt = cin * kpad_d;
    hipLaunchKernelGGL(dgrad_weights_k, dim3((cnt + 255) / 256), dim3(256), 0, s, wt, cin, cout, kpad, wd, kpad_d);
}

// Zero-insertion of a stride-2 output gradient onto the input grid; one
// thread per (voxel, group of 8 channels), 16-byte accesses.
__global__ void dilate_k(Tensor src, Tensor dst, int c)
{
    const int g8 = c / 8;
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const int nf = dst.n;
    const size_t N = (size_t)nf * nf * nf;
    if (t >= N * g8) return;
    const int v = (int)(t / g8), grp = (int)(t - (size_t)v * g8);
    int i, j, k;
    decode3(v, nf, i, j, k);
    const bool even = !((i | j | k) & 1);
    const int nc = src.n;
    bf16x8 val = {};
    if (even) {
        const size_t vc = (size_t)((i >> 1) + nc * ((j >> 1) + nc * (k >> 1)));
        val = *reinterpret_cast<const bf16x8 *>(src.p + vc * src.cs + 8 * grp);
    }
    *reinterpret_cast<bf16x8 *>(dst.p + (size_t)v * dst.cs + 8 * grp) = val;
}

void launch_dilate(Tensor src, Tensor dst, int c, hipStream_t s)
{
    const size_t cnt = (size_t)dst.n * dst.n * dst.n * (c / 8);
    hipLaunchKernelGGL(dilate_k, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, src, dst, c);
}

// Weight gradient: partial[split, co, kk] = sum over the split's output voxels
// o of dy[o, co] X[o, kk], X[o, tap cin + ci] = x[s o + d(tap), ci].  One wave
// per (16 co x 16 kk) tile and split; rows = co, columns = kk, K = voxels.
__global__ void __launch_bounds__(256)
wgrad_k(Tensor x, int cin, Tensor dy, int cout, int kpad, int stride, int nsplit, int per_split,
        float *__restrict__ partial)
{
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int nct = cout / 16, nkt = kpad / 16;
    const int ntile = nct * nkt;
    if (gw >= ntile * nsplit) return;
    const int split = gw / ntile, tile = gw - split * ntile;
    const int ct = tile / nkt, kt = tile - ct * nkt;
    const int g = lane >> 4, r16 = lane & 15;
    const int co = ct * 16 + r16, kk = kt * 16 + r16;
    const int nout = dy.n, nin = x.n, Nout = nout * nout * nout;
    const bool kvalid = kk < 27 * cin;
    const int tap = kvalid ? kk / cin : 0, ci = kvalid ? kk - tap * cin : 0;
    const int dxo = tap % 3 - 1, dyo = (tap / 3) % 3 - 1, dzo = tap / 9 - 1;
    const int ob = split * per_split, oe = min(Nout, ob + per_split);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int o0 = ob; o0 < oe; o0 += 32) {
        bf16x8 a, b;
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const int o = o0 + 8 * g + jj;
            __bf16 av = (__bf16)0.f, bv = (__bf16)0.f;
            if (o < oe) {
                av = dy.p[(size_t)o * dy.cs + co];
                if (kvalid) {
                    int i, j, k;
                    decode3(o, nout, i, j, k);
                    i = stride * i + dxo;
                    j = stride * j + dyo;
                    k = stride * k + dzo;
                    if (i >= 0 && i < nin && j >= 0 && j < nin && k >= 0 && k < nin)
                        bv = x.p[(size_t)(i + nin * (j + nin * k)) * x.cs + ci];
                }
            }
            a[jj] = av;
            b[jj] = bv;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    float *P = partial + (size_t)split * cout * kpad;
#pragma unroll
    for (int r = 0; r < 4; ++r) P[(size_t)(ct * 16 + 4 * g + r) * kpad + kk] = acc[r];
}

// out[t] = sum_s partial[s, t] in fixed order
__global__ void split_reduce_k(const float *__restrict__ partial, int nsplit, int count, float *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    float s = 0.f;
    for (int q = 0; q < nsplit; ++q) s += partial[(size_t)q * count + t];
    out[t] = s;
}

int wgrad_splits(int cout, int kpad, int nout)
{
    const int ntile = (cout / 16) * (kpad / 16);
    const int Nout = nout * nout * nout;
    int ns = 4096 / ntile;
    if (ns < 1) ns = 1;
    const int maxs = (Nout + 1023) / 1024;
    if (ns > maxs) ns = maxs;
    if (ns > kMaxSplit) ns = kMaxSplit;
    return ns;
}

void launch_wgrad(Tensor x, int cin, Tensor dy, int cout, int kpad, int stride, float *partial, float *dw, hipStream_t s)
{
    const int nsplit = wgrad_splits(cout, kpad, dy.n);
    const int Nout = dy.n * dy.n * dy.n;
    int per = (Nout + nsplit - 1) / nsplit;
    per = (per + 31) / 32 * 32;
    const int waves = (cout / 16) * (kpad / 16) * nsplit;
    hipLaunchKernelGGL(wgrad_k, dim3((waves + 3) / 4), dim3(256), 0, s, x, cin, dy, cout, kpad, stride, nsplit, per,
                       partial);
    const int cnt = cout * kpad;
    hipLaunchKernelGGL(split_reduce_k, dim3((cnt + 255) / 256), dim3(256), 0, s, partial, nsplit, cnt, dw);
}

// Splits of a voxel range for the fixed-order reductions below: at most
// kMaxSplit workgroups, each over a contiguous range.
static int reduce_splits(int N)
{
    int ns = (N + 2047) / 2048;
    return ns < 1 ? 1 : (ns > kMaxSplit ? kMaxSplit : ns);
}

// bias gradient: partial[split, c] = sum over the split's voxels of dy[v, c].
// Workgroup = split; thread t sums channel t % c over voxels t / c + q (256 / c)
// (c divides 256), then the c sums are combined in a fixed order.
__global__ void __launch_bounds__(256) bgrad_k(Tensor dy, int c, int per, float *__restrict__ partial)
{
    __shared__ float sh[256];
    const int N = dy.n * dy.n * dy.n;
    const int vb = blockIdx.x * per, ve = min(N, vb + per);
    const int ch = threadIdx.x % c, lanes = 256 / c, l = threadIdx.x / c;
    float s = 0.f;
    for (int v = vb + l; v < ve; v += lanes) s += (float)dy.p[(size_t)v * dy.cs + ch];
    sh[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < c) {
        float t = 0.f;
        for (int q = 0; q < lanes; ++q) t += sh[q * c + threadIdx.x];
        partial[(size_t)blockIdx.x * c + threadIdx.x] = t;
    }
}

void launch_bgrad(Tensor dy, int c, float *partial, float *db, hipStream_t s)
{
    const int N = dy.n * dy.n * dy.n;
    const int nsplit = reduce_splits(N);
    const int per = (N + nsplit - 1) / nsplit;
    hipLaunchKernelGGL(bgrad_k, dim3(nsplit), dim3(256), 0, s, dy, c, per, partial);
    hipLaunchKernelGGL(split_reduce_k, dim3((c + 255) / 256), dim3(256), 0, s, partial, nsplit, c, db);
}

// ---------------------------------------------------------- elementwise

// g[v, c] = 0 where the ReLU output y[v, c] is 0
__global__ void relu_bwd_k(Tensor g, Tensor y, int c)
{
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t N = (size_t)g.n * g.n * g.n;
    if (t >= N * c) return;
    const size_t v = t / c, ch = t - v * c;
    if (!((float)y.p[v * y.cs + ch] > 0.f)) g.p[v * g.cs + ch] = (__bf16)0.f;
}

void launch_relu_bwd(Tensor g, Tensor y, int c, hipStream_t s)
{
    const size_t cnt = (size_t)g.n * g.n * g.n * c;
    hipLaunchKernelGGL(relu_bwd_k, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, g, y, c);
}

// dst[v, c] += src[v, c] (rounded once to BF16)
__global__ void add_k(Tensor dst, Tensor src, int c)
{
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t N = (size_t)dst.n * dst.n * dst.n;
    if (t >= N * c) return;
    const size_t v = t / c, ch = t - v * c;
    __bf16 *d = dst.p + v * dst.cs + ch;
    *d = (__bf16)((float)*d + (float)src.p[v * src.cs + ch]);
}

void launch_add(Tensor dst, Tensor src, int c, hipStream_t s)
{
    const size_t cnt = (size_t)dst.n * dst.n * dst.n * c;
    hipLaunchKernelGGL(add_k, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, dst, src, c);
}

// Trilinear 2x up-sampling of vertex-centred grids (n_fine = 2 n_coarse - 1);
// one thread per (fine voxel, group of 8 channels).
__global__ void upsample_k(Tensor src, Tensor dst, int c)
{
    const int g8 = c / 8;
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const int nf = dst.n, nc = src.n;
    const size_t N = (size_t)nf * nf * nf;
    if (t >= N * g8) return;
    const int v = (int)(t / g8), grp = (int)(t - (size_t)v * g8);
    int i, j, k;
    decode3(v, nf, i, j, k);
    const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
    const float wi = (i & 1) ? 0.5f : 1.f, wj = (j & 1) ? 0.5f : 1.f, wk = (k & 1) ? 0.5f : 1.f;
    const float wi1 = (i & 1) ? 0.5f : 0.f, wj1 = (j & 1) ? 0.5f : 0.f, wk1 = (k & 1) ? 0.5f : 0.f;
    auto at = [&](int a, int b, int cc) {
        return *reinterpret_cast<const bf16x8 *>(src.p + (size_t)(a + nc * (b + nc * cc)) * src.cs + 8 * grp);
    };
    const bf16x8 a000 = at(i0, j0, k0), a100 = at(i1, j0, k0), a010 = at(i0, j1, k0), a110 = at(i1, j1, k0);
    const bf16x8 a001 = at(i0, j0, k1), a101 = at(i1, j0, k1), a011 = at(i0, j1, k1), a111 = at(i1, j1, k1);
    bf16x8 out;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float x00 = wi * (float)a000[e] + wi1 * (float)a100[e];
        const float x10 = wi * (float)a010[e] + wi1 * (float)a110[e];
        const float x01 = wi * (float)a001[e] + wi1 * (float)a101[e];
        const float x11 = wi * (float)a011[e] + wi1 * (float)a111[e];
        out[e] = (__bf16)(wk * (wj * x00 + wj1 * x10) + wk1 * (wj * x01 + wj1 * x11));
    }
    *reinterpret_cast<bf16x8 *>(dst.p + (size_t)v * dst.cs + 8 * grp) = out;
}

void launch_upsample(Tensor src, Tensor dst, int c, hipStream_t s)
{
    const size_t cnt = (size_t)dst.n * dst.n * dst.n * (c / 8);
    hipLaunchKernelGGL(upsample_k, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, src, dst, c);
}

// Adjoint of upsample_k: coarse node I gathers w g(2I + d) over d in {-1,0,1}^3,
// w = product over axes of (1 if d = 0 else 1/2).
// one thread per (coarse voxel, group of 8 channels)
__global__ void upsample_adj_k(Tensor gf, Tensor gc, int c)
{
    const int g8 = c / 8;
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const int nc = gc.n, nf = gf.n;
    const size_t N = (size_t)nc * nc * nc;
    if (t >= N * g8) return;
    const int v = (int)(t / g8), grp = (int)(t - (size_t)v * g8);
    int I, J, K;
    decode3(v, nc, I, J, K);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int dz = -1; dz <= 1; ++dz) {
        const int k = 2 * K + dz;
        if (k < 0 || k >= nf) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int j = 2 * J + dy;
            if (j < 0 || j >= nf) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                const int i = 2 * I + dx;
                if (i < 0 || i >= nf) continue;
                const float w = (dx ? 0.5f : 1.f) * (dy ? 0.5f : 1.f) * (dz ? 0.5f : 1.f);
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(gf.p + (size_t)(i + nf * (j + nf * k)) * gf.cs + 8 * grp);
#pragma unroll
                for (int e = 0; e < 8; ++e) s[e] += w * (float)a[e];
            }
        }
    }
    bf16x8 out;
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = (__bf16)s[e];
    *reinterpret_cast<bf16x8 *>(gc.p + (size_t)v * gc.cs + 8 * grp) = out;
}

void launch_upsample_adj(Tensor gf, Tensor gc, int c, hipStream_t s)
{
    const size_t cnt = (size_t)gc.n * gc.n * gc.n * (c / 8);
    hipLaunchKernelGGL(upsample_adj_k, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, gf, gc, c);
}

// ------------------------------------------------------------- head, loss

// yhat[v] = b + sum_c w[c] x[v, c] (c a multiple of 8; 16-byte loads, same order)
__global__ void head_fwd_k(Tensor x, int c, const float *__restrict__ w, const float *__restrict__ b, float *__restrict__ yh)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = x.n * x.n * x.n;
    if (v >= N) return;
    float s = b[0];
    for (int c8 = 0; c8 < c; c8 += 8) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(x.p + (size_t)v * x.cs + c8);
#pragma unroll
        for (int e = 0; e < 8; ++e) s += w[c8 + e] * (float)a[e];
    }
    yh[v] = s;
}

void launch_head_fwd(Tensor x, int c, const float *w, const float *b, float *yh, hipStream_t s)
{
    const int N = x.n * x.n * x.n;
    hipLaunchKernelGGL(head_fwd_k, dim3((N + 255) / 256), dim3(256), 0, s, x, c, w, b, yh);
}

// dx[v, c] = dy[v] w[c] (c a multiple of 8; 16-byte stores)
__global__ void head_bwd_x_k(const float *__restrict__ dyh, int c, const float *__restrict__ w, Tensor dx)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = dx.n * dx.n * dx.n;
    if (v >= N) return;
    const float d = dyh[v];
    for (int c8 = 0; c8 < c; c8 += 8) {
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = (__bf16)(d * w[c8 + e]);
        *reinterpret_cast<bf16x8 *>(dx.p + (size_t)v * dx.cs + c8) = o;
    }
}

// partial[split, c] = sum dy[v] x[v, c] (c < C), partial[split, C] = sum dy[v];
// workgroup = split, fixed-order combination as in bgrad_k (C divides 256).
__global__ void __launch_bounds__(256)
head_bwd_w_k(const float *__restrict__ dyh, Tensor x, int c, int per, float *__restrict__ partial)
{
    __shared__ float sh[256], sb[256];
    const int N = x.n * x.n * x.n;
    const int vb = blockIdx.x * per, ve = min(N, vb + per);
    const int ch = threadIdx.x % c, lanes = 256 / c, l = threadIdx.x / c;
    float s = 0.f, sbias = 0.f;
    for (int v = vb + l; v < ve; v += lanes) {
        const float d = dyh[v];
        s += d * (float)x.p[(size_t)v * x.cs + ch];
        sbias += d;
    }
    sh[threadIdx.x] = s;
    sb[threadIdx.x] = sbias;
    __syncthreads();
    if ((int)threadIdx.x < c) {
        float t = 0.f;
        for (int q = 0; q < lanes; ++q) t += sh[q * c + threadIdx.x];
        partial[(size_t)blockIdx.x * (c + 1) + threadIdx.x] = t;
    } else if ((int)threadIdx.x == c) {
        float t = 0.f;
        for (int q = 0; q < lanes; ++q) t += sb[q * c];   // channel-0 threads saw every voxel once
        partial[(size_t)blockIdx.x * (c + 1) + c] = t;
    }
}

void launch_head_bwd(const float *dyh, Tensor x, int c, const float *w, Tensor dx, float *partial, float *dwb,
                     hipStream_t s)
{
    const int N = x.n * x.n * x.n;
    hipLaunchKernelGGL(head_bwd_x_k, dim3((N + 255) / 256), dim3(256), 0, s, dyh, c, w, dx);
    const int nsplit = reduce_splits(N);
    const int per = (N + nsplit - 1) / nsplit;
    hipLaunchKernelGGL(head_bwd_w_k, dim3(nsplit), dim3(256), 0, s, dyh, x, c, per, partial);
    hipLaunchKernelGGL(split_reduce_k, dim3(1), dim3(256), 0, s, partial, nsplit, c + 1, dwb);
}

// Mean squared error over interior nodes; dy = 2 (yhat - t) / N_int there, 0 on
// the boundary.  partial[b] per block, then one block.
__global__ void __launch_bounds__(256)
mse_k(const float *__restrict__ yh, const float *__restrict__ tg, int n, float *__restrict__ dy, double *__restrict__ partial)
{
    __shared__ double sh[256];
    const int N = n * n * n;
    const double nint = (double)(n - 2) * (n - 2) * (n - 2);
    double s = 0.0;
    for (int v = blockIdx.x * 256 + threadIdx.x; v < N; v += gridDim.x * 256) {
        int i, j, k;
        decode3(v, n, i, j, k);
        const bool in = i > 0 && j > 0 && k > 0 && i < n - 1 && j < n - 1 && k < n - 1;
        const float d = in ? yh[v] - tg[v] : 0.f;
        dy[v] = (float)(2.0 * d / nint);
        s += (double)d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] / nint;
}

__global__ void sum_k(const double *__restrict__ partial, int nb, double *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += partial[b];
        out[0] = s;
    }
}

void launch_mse(const float *yh, const float *tg, int n, float *dy, double *partial, double *loss, hipStream_t s)
{
    hipLaunchKernelGGL(mse_k, dim3(kLossBlocks), dim3(256), 0, s, yh, tg, n, dy, partial);
    hipLaunchKernelGGL(sum_k, dim3(1), dim3(64), 0, s, partial, kLossBlocks, loss);
}

// Adam on FP32 master weights; the BF16 copy (if any) is refreshed.
__global__ void adam_k(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v, const float *__restrict__ g,
                       int count, float lr, float b1, float b2, float eps, float c1, float c2, __bf16 *__restrict__ wb)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    const float wt = w[t] - lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    w[t] = wt;
    if (wb) wb[t] = (__bf16)wt;
}

void launch_adam(float *w, float *m, float *v, const float *g, int count, float lr, int step, __bf16 *wb, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_k, dim3((count + 255) / 256), dim3(256), 0, s, w, m, v, g, count, lr, b1, b2, eps, c1, c2, wb);
}

__global__ void to_bf16_k(const float *__restrict__ src, __bf16 *__restrict__ dst, int count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) dst[t] = (__bf16)src[t];
}

void launch_to_bf16(const float *src, __bf16 *dst, int count, hipStream_t s)
{
    hipLaunchKernelGGL(to_bf16_k, dim3((count + 255) / 256), dim3(256), 0, s, src, dst, count);
}

// --------------------------------------------------------- inputs, outputs

// Network input: channel 0 = Phi_N / cn, channel 1 = h^2 S / cs, further channels
// of the slot (if any) = 0.
__global__ void prep_input_k(int n, const double *__restrict__ phin, const double *__restrict__ base,
                             const double *__restrict__ S, double inv_cn, double h2_cs, Tensor x)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n * n * n) return;
    __bf16 *p = x.p + (size_t)v * x.cs;
    p[0] = (__bf16)(float)((phin[v] - base[v]) * inv_cn);
    p[1] = (__bf16)(float)(S[v] * h2_cs);
    for (int c = 2; c < x.cs; ++c) p[c] = (__bf16)0.f;
}

// Two-channel compact sample -> the network's 8-channel input slot.
__global__ void expand_input_k(const __bf16 *__restrict__ xc, Tensor x)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= x.n * x.n * x.n) return;
    __bf16 *p = x.p + (size_t)v * x.cs;
    p[0] = xc[2 * (size_t)v];
    p[1] = xc[2 * (size_t)v + 1];
    for (int c = 2; c < x.cs; ++c) p[c] = (__bf16)0.f;
}

void launch_expand_input(const __bf16 *xc, Tensor x, hipStream_t s)
{
    const int N = x.n * x.n * x.n;
    hipLaunchKernelGGL(expand_input_k, dim3((N + 255) / 256), dim3(256), 0, s, xc, x);
}

void launch_prep_input(int n, const double *phin, const double *base, const double *S, double inv_cn, double h2_cs,
                       Tensor x, hipStream_t s)
{
    const int N = n * n * n;
    hipLaunchKernelGGL(prep_input_k, dim3((N + 255) / 256), dim3(256), 0, s, n, phin, base, S, inv_cn, h2_cs, x);
}

// out[v] = a * in[v] + base[v] (FP32 -> FP64)
__global__ void scale_out_k(const float *__restrict__ in, int count, double a, const double *__restrict__ base,
                            double *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) out[t] = a * (double)in[t] + base[t];
}

void launch_scale_out(const float *in, int count, double a, const double *base, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(scale_out_k, dim3((count + 255) / 256), dim3(256), 0, s, in, count, a, base, out);
}

// out[v] = (float)(a * (in[v] - base[v])) (FP64 -> FP32 target)
__global__ void scale_in_k(const double *__restrict__ in, const double *__restrict__ base, int count, double a,
                           float *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) out[t] = (float)(a * (in[t] - base[t]));
}

void launch_scale_in(const double *in, const double *base, int count, double a, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(scale_in_k, dim3((count + 255) / 256), dim3(256), 0, s, in, base, count, a, out);
}

}  // namespace qm
