// The U-Net of the learned initial guess: layers, buffers, forward, backward
// and Adam, behind qumond_unet.h.
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/qumond_unet.h"
#include "common.h"
#include "mg.h"
#include "unet.h"

void qm_set_last_error(const char *msg);

namespace {

using qm::Tensor;

qumond_status ufail(qumond_status s, const std::string &m)
{
    qm_set_last_error(m.c_str());
    return s;
}

struct Conv {
    int cin = 0, cout = 0, stride = 1, kpad = 0, kpad_d = 0, fan_in = 0;
    float *w = nullptr, *b = nullptr, *gw = nullptr, *gb = nullptr;
    float *mw = nullptr, *vw = nullptr, *mb = nullptr, *vb = nullptr;
    __bf16 *wb = nullptr, *wd = nullptr;
};

}  // namespace

struct qumond_unet {
    hipStream_t s = nullptr;
    int n[4] = {0, 0, 0, 0};
    Conv L[11];
    // head (1x1x1, 16 -> 1)
    float *hw = nullptr, *hgw = nullptr, *hm = nullptr, *hv = nullptr;   // 17 values: 16 weights + bias
    // activations
    Tensor x0, a0, c0, s0, d0, a1, c1, s1, d1, a2, c2, s2, d2, a3, b3;
    // gradients
    Tensor gd0, gc0, gd1, gc1, gd2, gc2, gb3, ga3, gs2, ga2, gs1, ga1, gs0, ga0, dil;
    float *yhat = nullptr, *dyhat = nullptr, *partial = nullptr;
    double *lpartial = nullptr, *loss = nullptr, *host_loss = nullptr;
    double *base_n = nullptr, *base_q = nullptr;   // point-mass baselines (n^3 each)
    int step = 0;
    std::vector<void *> owned;
    hipError_t err = hipSuccess;

    void *alloc(size_t bytes)
    {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            err = e;
            return nullptr;
        }
        owned.push_back(p);
        return p;
    }
    Tensor tensor(int nn, int cs)
    {
        Tensor t;
        t.n = nn;
        t.cs = cs;
        t.p = (__bf16 *)alloc((size_t)nn * nn * nn * cs * sizeof(__bf16));
        return t;
    }
};

namespace {

Tensor slice(Tensor t, int off)
{
    Tensor r = t;
    r.p = t.p + off;
    return r;
}

// Layer table: (cin storage, cout, stride, fan-in channels)
const int kLayer[11][4] = {
    {8, 16, 1, 2},      // 0  L0a  x0 -> a0
    {16, 16, 1, 16},    // 1  L0b  a0 -> s0
    {16, 32, 2, 16},    // 2  L1a  s0 -> a1
    {32, 32, 1, 32},    // 3  L1b  a1 -> s1
    {32, 64, 2, 32},    // 4  L2a  s1 -> a2
    {64, 64, 1, 64},    // 5  L2b  a2 -> s2
    {64, 64, 2, 64},    // 6  L3a  s2 -> a3
    {64, 64, 1, 64},    // 7  L3b  a3 -> b3
    {128, 64, 1, 128},  // 8  L2u  c2 -> d2
    {96, 32, 1, 96},    // 9  L1u  c1 -> d1
    {48, 16, 1, 48},    // 10 L0u  c0 -> d0
};

void conv_fwd(qumond_unet *u, int l, Tensor in, Tensor out)
{
    const Conv &c = u->L[l];
    qm::launch_conv3d_fwd(in, c.cin, c.wb, c.kpad, c.cout, c.b, out, c.stride, 1, u->s);
}

// Backward through layer l whose input was `in` and ReLU output `out`: g is
// the gradient of out (overwritten by the pre-activation gradient); gin (may
// have p == nullptr) receives the gradient of the input.
void conv_bwd(qumond_unet *u, int l, Tensor in, Tensor out, Tensor g, Tensor gin)
{
    Conv &c = u->L[l];
    qm::launch_relu_bwd(g, out, c.cout, u->s);
    qm::launch_wgrad(in, c.cin, g, c.cout, c.kpad, c.stride, u->partial, c.gw, u->s);
    qm::launch_bgrad(g, c.cout, u->partial, c.gb, u->s);
    if (!gin.p) return;
    qm::launch_dgrad_weights(c.wb, c.cin, c.cout, c.kpad, c.wd, c.kpad_d, u->s);
    if (c.stride == 2) {
        Tensor d = u->dil;
        d.n = in.n;
        d.cs = c.cout;
        qm::launch_dilate(g, d, c.cout, u->s);
        qm::launch_conv3d_fwd(d, c.cout, c.wd, c.kpad_d, c.cin, nullptr, gin, 1, 0, u->s);
    } else {
        qm::launch_conv3d_fwd(g, c.cout, c.wd, c.kpad_d, c.cin, nullptr, gin, 1, 0, u->s);
    }
}

void forward(qumond_unet *u)
{
    conv_fwd(u, 0, u->x0, u->a0);
    conv_fwd(u, 1, u->a0, u->s0);
    conv_fwd(u, 2, u->s0, u->a1);
    conv_fwd(u, 3, u->a1, u->s1);
    conv_fwd(u, 4, u->s1, u->a2);
    conv_fwd(u, 5, u->a2, u->s2);
    conv_fwd(u, 6, u->s2, u->a3);
    conv_fwd(u, 7, u->a3, u->b3);
    qm::launch_upsample(u->b3, slice(u->c2, 0), 64, u->s);
    conv_fwd(u, 8, u->c2, u->d2);
    qm::launch_upsample(u->d2, slice(u->c1, 0), 64, u->s);
    conv_fwd(u, 9, u->c1, u->d1);
    qm::launch_upsample(u->d1, slice(u->c0, 0), 32, u->s);
    conv_fwd(u, 10, u->c0, u->d0);
    qm::launch_head_fwd(u->d0, 16, u->hw, u->hw + 16, u->yhat, u->s);
}

void backward(qumond_unet *u)
{
    Tensor none;
    none.p = nullptr;
    none.n = 0;
    none.cs = 0;
    qm::launch_head_bwd(u->dyhat, u->d0, 16, u->hw, u->gd0, u->partial, u->hgw, u->s);
    conv_bwd(u, 10, u->c0, u->d0, u->gd0, u->gc0);
    qm::launch_upsample_adj(slice(u->gc0, 0), u->gd1, 32, u->s);
    conv_bwd(u, 9, u->c1, u->d1, u->gd1, u->gc1);
    qm::launch_upsample_adj(slice(u->gc1, 0), u->gd2, 64, u->s);
    conv_bwd(u, 8, u->c2, u->d2, u->gd2, u->gc2);
    qm::launch_upsample_adj(slice(u->gc2, 0), u->gb3, 64, u->s);
    conv_bwd(u, 7, u->a3, u->b3, u->gb3, u->ga3);
    conv_bwd(u, 6, u->s2, u->a3, u->ga3, u->gs2);
    qm::launch_add(u->gs2, slice(u->gc2, 64), 64, u->s);
    conv_bwd(u, 5, u->a2, u->s2, u->gs2, u->ga2);
    conv_bwd(u, 4, u->s1, u->a2, u->ga2, u->gs1);
    qm::launch_add(u->gs1, slice(u->gc1, 64), 32, u->s);
    conv_bwd(u, 3, u->a1, u->s1, u->gs1, u->ga1);
    conv_bwd(u, 2, u->s0, u->a1, u->ga1, u->gs0);
    qm::launch_add(u->gs0, slice(u->gc0, 32), 16, u->s);
    conv_bwd(u, 1, u->a0, u->s0, u->gs0, u->ga0);
    conv_bwd(u, 0, u->x0, u->a0, u->ga0, none);
}

void adam(qumond_unet *u, float lr)
{
    ++u->step;
    for (int l = 0; l < 11; ++l) {
        Conv &c = u->L[l];
        qm::launch_adam(c.w, c.mw, c.vw, c.gw, c.cout * c.kpad, lr, u->step, c.wb, u->s);
        qm::launch_adam(c.b, c.mb, c.vb, c.gb, c.cout, lr, u->step, nullptr, u->s);
    }
    qm::launch_adam(u->hw, u->hm, u->hv, u->hgw, 17, lr, u->step, nullptr, u->s);
}

bool good_n(int n) { return n >= 17 && n <= 513 && qm::log2_exact(n - 1) >= 4; }

qumond_status check_hip(const char *where)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ufail(QUMOND_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
    return QUMOND_OK;
}

}  // namespace

extern "C" {

qumond_status qumond_unet_destroy(qumond_unet *u)
{
    if (!u) return ufail(QUMOND_ERR_INVALID, "net is NULL");
    (void)hipStreamSynchronize(u->s);
    for (void *p : u->owned) (void)hipFree(p);
    if (u->host_loss) (void)hipHostFree(u->host_loss);
    delete u;
    return QUMOND_OK;
}

qumond_status qumond_unet_create(int32_t n, uint64_t seed, void *hip_stream, qumond_unet **out)
{
    if (!out) return ufail(QUMOND_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!good_n(n)) return ufail(QUMOND_ERR_INVALID, "n must be 2^J + 1 with J >= 4 and n <= 513");
    qumond_unet *u = new (std::nothrow) qumond_unet();
    if (!u) return ufail(QUMOND_ERR_OOM, "host allocation failed");
    u->s = (hipStream_t)hip_stream;
    u->n[0] = n;
    for (int l = 1; l < 4; ++l) u->n[l] = (u->n[l - 1] + 1) / 2;
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.f, 1.f);
    std::vector<float> hbuf;
    for (int l = 0; l < 11; ++l) {
        Conv &c = u->L[l];
        c.cin = kLayer[l][0];
        c.cout = kLayer[l][1];
        c.stride = kLayer[l][2];
        c.fan_in = kLayer[l][3];
        c.kpad = qm::kpad_of(c.cin);
        c.kpad_d = qm::kpad_of(c.cout);
        const size_t nw = (size_t)c.cout * c.kpad;
        c.w = (float *)u->alloc(nw * 4);
        c.gw = (float *)u->alloc(nw * 4);
        c.mw = (float *)u->alloc(nw * 4);
        c.vw = (float *)u->alloc(nw * 4);
        c.wb = (__bf16 *)u->alloc(nw * 2);
        c.wd = (__bf16 *)u->alloc((size_t)c.cin * c.kpad_d * 2);
        c.b = (float *)u->alloc(c.cout * 4);
        c.gb = (float *)u->alloc(c.cout * 4);
        c.mb = (float *)u->alloc(c.cout * 4);
        c.vb = (float *)u->alloc(c.cout * 4);
        if (u->err != hipSuccess) break;
        hbuf.assign(nw, 0.f);
        const float sd = std::sqrt(2.f / (27.f * c.fan_in));
        for (int co = 0; co < c.cout; ++co)
            for (int tap = 0; tap < 27; ++tap)
                for (int ci = 0; ci < c.fan_in; ++ci) hbuf[(size_t)co * c.kpad + tap * c.cin + ci] = sd * nd(rng);
        (void)hipMemcpy(c.w, hbuf.data(), nw * 4, hipMemcpyHostToDevice);
        (void)hipMemset(c.mw, 0, nw * 4);
        (void)hipMemset(c.vw, 0, nw * 4);
        (void)hipMemset(c.b, 0, c.cout * 4);
        (void)hipMemset(c.mb, 0, c.cout * 4);
        (void)hipMemset(c.vb, 0, c.cout * 4);
        qm::launch_to_bf16(c.w, c.wb, (int)nw, u->s);
    }
    u->hw = (float *)u->alloc(17 * 4);
    u->hgw = (float *)u->alloc(17 * 4);
    u->hm = (float *)u->alloc(17 * 4);
    u->hv = (float *)u->alloc(17 * 4);
    if (u->err == hipSuccess) {
        float hh[17];
        const float sd = std::sqrt(1.f / 16.f);
        for (int c = 0; c < 16; ++c) hh[c] = sd * nd(rng);
        hh[16] = 0.f;
        (void)hipMemcpy(u->hw, hh, sizeof hh, hipMemcpyHostToDevice);
        (void)hipMemset(u->hm, 0, 17 * 4);
        (void)hipMemset(u->hv, 0, 17 * 4);
    }
    const int n0 = u->n[0], n1 = u->n[1], n2 = u->n[2], n3 = u->n[3];
    u->x0 = u->tensor(n0, 8);
    u->a0 = u->tensor(n0, 16);
    u->c0 = u->tensor(n0, 48);
    u->s0 = slice(u->c0, 32);
    u->d0 = u->tensor(n0, 16);
    u->a1 = u->tensor(n1, 32);
    u->c1 = u->tensor(n1, 96);
    u->s1 = slice(u->c1, 64);
    u->d1 = u->tensor(n1, 32);
    u->a2 = u->tensor(n2, 64);
    u->c2 = u->tensor(n2, 128);
    u->s2 = slice(u->c2, 64);
    u->d2 = u->tensor(n2, 64);
    u->a3 = u->tensor(n3, 64);
    u->b3 = u->tensor(n3, 64);
    u->gd0 = u->tensor(n0, 16);
    u->gc0 = u->tensor(n0, 48);
    u->gd1 = u->tensor(n1, 32);
    u->gc1 = u->tensor(n1, 96);
    u->gd2 = u->tensor(n2, 64);
    u->gc2 = u->tensor(n2, 128);
    u->gb3 = u->tensor(n3, 64);
    u->ga3 = u->tensor(n3, 64);
    u->gs2 = u->tensor(n2, 64);
    u->ga2 = u->tensor(n2, 64);
    u->gs1 = u->tensor(n1, 32);
    u->ga1 = u->tensor(n1, 32);
    u->gs0 = u->tensor(n0, 16);
    u->ga0 = u->tensor(n0, 16);
    u->dil = u->tensor(n0, 32);
    const size_t N0 = (size_t)n0 * n0 * n0;
    u->yhat = (float *)u->alloc(N0 * 4);
    u->base_n = (double *)u->alloc(N0 * 8);
    u->base_q = (double *)u->alloc(N0 * 8);
    u->dyhat = (float *)u->alloc(N0 * 4);
    // wgrad partials: nsplit x cout x kpad <= max(4096 tiles x 256, cout x kpad); bias/head partials are smaller
    u->partial = (float *)u->alloc((size_t)2 * 1024 * 1024 * 4);
    u->lpartial = (double *)u->alloc(qm::kLossBlocks * 8);
    u->loss = (double *)u->alloc(8);
    if (u->err == hipSuccess && hipHostMalloc((void **)&u->host_loss, 8, hipHostMallocDefault) != hipSuccess)
        u->err = hipErrorOutOfMemory;
    if (u->err != hipSuccess) {
        const hipError_t e = u->err;
        qumond_unet_destroy(u);
        return ufail(e == hipErrorOutOfMemory ? QUMOND_ERR_OOM : QUMOND_ERR_HIP,
                     std::string("qumond_unet_create: ") + hipGetErrorString(e));
    }
    qumond_status st = check_hip("qumond_unet_create");
    if (st != QUMOND_OK) {
        qumond_unet_destroy(u);
        return st;
    }
    *out = u;
    return QUMOND_OK;
}

qumond_status qumond_unet_get_grads(qumond_unet *u, float *host)
{
    if (!u || !host) return ufail(QUMOND_ERR_INVALID, "NULL argument");
    if (hipStreamSynchronize(u->s) != hipSuccess) return check_hip("qumond_unet_get_grads");
    size_t off = 0;
    for (int l = 0; l < 11; ++l) {
        const Conv &c = u->L[l];
        (void)hipMemcpy(host + off, c.gw, (size_t)c.cout * c.kpad * 4, hipMemcpyDeviceToHost);
        off += (size_t)c.cout * c.kpad;
        (void)hipMemcpy(host + off, c.gb, (size_t)c.cout * 4, hipMemcpyDeviceToHost);
        off += c.cout;
    }
    (void)hipMemcpy(host + off, u->hgw, 17 * 4, hipMemcpyDeviceToHost);
    return check_hip("qumond_unet_get_grads");
}

int64_t qumond_unet_param_count(const qumond_unet *u)
{
    if (!u) return 0;
    int64_t c = 17;
    for (int l = 0; l < 11; ++l) c += (int64_t)u->L[l].cout * u->L[l].kpad + u->L[l].cout;
    return c;
}

qumond_status qumond_unet_get_params(qumond_unet *u, float *host)
{
    if (!u || !host) return ufail(QUMOND_ERR_INVALID, "NULL argument");
    if (hipStreamSynchronize(u->s) != hipSuccess) return check_hip("qumond_unet_get_params");
    size_t off = 0;
    for (int l = 0; l < 11; ++l) {
        const Conv &c = u->L[l];
        (void)hipMemcpy(host + off, c.w, (size_t)c.cout * c.kpad * 4, hipMemcpyDeviceToHost);
        off += (size_t)c.cout * c.kpad;
        (void)hipMemcpy(host + off, c.b, (size_t)c.cout * 4, hipMemcpyDeviceToHost);
        off += c.cout;
    }
    (void)hipMemcpy(host + off, u->hw, 17 * 4, hipMemcpyDeviceToHost);
    return check_hip("qumond_unet_get_params");
}

qumond_status qumond_unet_set_params(qumond_unet *u, const float *host)
{
    if (!u || !host) return ufail(QUMOND_ERR_INVALID, "NULL argument");
    if (hipStreamSynchronize(u->s) != hipSuccess) return check_hip("qumond_unet_set_params");
    size_t off = 0;
    for (int l = 0; l < 11; ++l) {
        Conv &c = u->L[l];
        const size_t nw = (size_t)c.cout * c.kpad;
        (void)hipMemcpy(c.w, host + off, nw * 4, hipMemcpyHostToDevice);
        off += nw;
        (void)hipMemcpy(c.b, host + off, (size_t)c.cout * 4, hipMemcpyHostToDevice);
        off += c.cout;
        (void)hipMemset(c.mw, 0, nw * 4);
        (void)hipMemset(c.vw, 0, nw * 4);
        (void)hipMemset(c.mb, 0, c.cout * 4);
        (void)hipMemset(c.vb, 0, c.cout * 4);
        qm::launch_to_bf16(c.w, c.wb, (int)nw, u->s);
    }
    (void)hipMemcpy(u->hw, host + off, 17 * 4, hipMemcpyHostToDevice);
    (void)hipMemset(u->hm, 0, 17 * 4);
    (void)hipMemset(u->hv, 0, 17 * 4);
    u->step = 0;
    return check_hip("qumond_unet_set_params");
}

static bool baseline_ok(double GM, double a0, double soft)
{
    return GM >= 0.0 && std::isfinite(GM) && a0 >= 0.0 && std::isfinite(a0) && soft > 0.0 && std::isfinite(soft);
}

static void baselines(qumond_unet *u, double h, double GM, double a0, double soft)
{
    const int n = u->n[0];
    const double L = h * (double)(n - 1);
    qm::launch_monopole_field(n, L, 1, GM, a0, soft, u->base_n, u->s);
    qm::launch_monopole_field(n, L, 2, GM, a0, soft, u->base_q, u->s);
}

qumond_status qumond_unet_prepare_sample(qumond_unet *u, const double *phin, const double *S, const double *phi,
                                         double h, double c_phin, double c_out, double GM, double a0, double soft,
                                         void *x, float *target)
{
    if (!u || !phin || !S || !phi || !x || !target || !(h > 0) || !(c_phin > 0) || !(c_out > 0) ||
        !baseline_ok(GM, a0, soft))
        return ufail(QUMOND_ERR_INVALID, "qumond_unet_prepare_sample: bad argument");
    const int n = u->n[0];
    Tensor t;
    t.p = (__bf16 *)x;
    t.n = n;
    t.cs = 2;
    baselines(u, h, GM, a0, soft);
    qm::launch_prep_input(n, phin, u->base_n, S, 1.0 / c_phin, h * h / c_out, t, u->s);
    qm::launch_scale_in(phi, u->base_q, n * n * n, 1.0 / c_out, target, u->s);
    return check_hip("qumond_unet_prepare_sample");
}

qumond_status qumond_unet_train_step(qumond_unet *u, const void *x, const float *target, float lr, double *loss)
{
    if (!u || !x || !target || !(lr > 0.f)) return ufail(QUMOND_ERR_INVALID, "qumond_unet_train_step: bad argument");
    const int n = u->n[0];
    qm::launch_expand_input((const __bf16 *)x, u->x0, u->s);
    forward(u);
    qm::launch_mse(u->yhat, target, n, u->dyhat, u->lpartial, u->loss, u->s);
    backward(u);
    adam(u, lr);
    if (loss) {
        (void)hipMemcpyAsync(u->host_loss, u->loss, 8, hipMemcpyDeviceToHost, u->s);
        if (hipStreamSynchronize(u->s) != hipSuccess) return check_hip("qumond_unet_train_step");
        *loss = *u->host_loss;
    }
    return check_hip("qumond_unet_train_step");
}

qumond_status qumond_unet_infer(qumond_unet *u, const double *phin, const double *S, double h, double c_phin,
                                double c_out, double GM, double a0, double soft, double *guess)
{
    if (!u || !phin || !S || !guess || !(h > 0) || !(c_phin > 0) || !(c_out > 0) || !baseline_ok(GM, a0, soft))
        return ufail(QUMOND_ERR_INVALID, "qumond_unet_infer: bad argument");
    const int n = u->n[0];
    baselines(u, h, GM, a0, soft);
    qm::launch_prep_input(n, phin, u->base_n, S, 1.0 / c_phin, h * h / c_out, u->x0, u->s);
    forward(u);
    qm::launch_scale_out(u->yhat, n * n * n, c_out, u->base_q, guess, u->s);
    return check_hip("qumond_unet_infer");
}

// ------------------------------------------------ single-layer entry points

static bool conv_shape_ok(int n_in, int cin, int cout, int stride)
{
    return n_in >= 3 && n_in <= 1025 && (n_in & 1) && cin >= 8 && cin % 8 == 0 && cin <= 256 && cout >= 16 &&
           cout % 16 == 0 && (cout / 16 <= 4 || cout == 96 || cout == 128) && (stride == 1 || stride == 2);
}

qumond_status qumond_k_conv3d_fwd(int32_t n_in, int32_t cin, const void *x, int32_t cout, const void *w,
                                  const float *bias, int32_t stride, int32_t relu, void *y, void *stream)
{
    if (!conv_shape_ok(n_in, cin, cout, stride) || !x || !w || !y) return ufail(QUMOND_ERR_INVALID, "qumond_k_conv3d_fwd: bad argument");
    Tensor tx{(__bf16 *)x, n_in, cin};
    Tensor ty{(__bf16 *)y, stride == 2 ? (n_in + 1) / 2 : n_in, cout};
    qm::launch_conv3d_fwd(tx, cin, (const __bf16 *)w, qm::kpad_of(cin), cout, bias, ty, stride, relu ? 1 : 0,
                          (hipStream_t)stream);
    return check_hip("qumond_k_conv3d_fwd");
}

qumond_status qumond_k_conv3d_dgrad(int32_t n_in, int32_t cin, int32_t cout, const void *w, int32_t stride,
                                    const void *dy, void *dx, void *stream)
{
    if (!conv_shape_ok(n_in, cin, cout, stride) || cin % 16 || !(cin / 16 <= 4 || cin == 96 || cin == 128) || !w ||
        !dy || !dx)
        return ufail(QUMOND_ERR_INVALID, "qumond_k_conv3d_dgrad: bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int kpad = qm::kpad_of(cin), kpad_d = qm::kpad_of(cout);
    const int n_out = stride == 2 ? (n_in + 1) / 2 : n_in;
    __bf16 *wd = nullptr, *dil = nullptr;
    if (hipMalloc((void **)&wd, (size_t)cin * kpad_d * 2) != hipSuccess) return ufail(QUMOND_ERR_OOM, "allocation");
    qm::launch_dgrad_weights((const __bf16 *)w, cin, cout, kpad, wd, kpad_d, s);
    Tensor tdy{(__bf16 *)dy, n_out, cout};
    Tensor tdx{(__bf16 *)dx, n_in, cin};
    if (stride == 2) {
        if (hipMalloc((void **)&dil, (size_t)n_in * n_in * n_in * cout * 2) != hipSuccess) {
            (void)hipFree(wd);
            return ufail(QUMOND_ERR_OOM, "allocation");
        }
        Tensor td{dil, n_in, cout};
        qm::launch_dilate(tdy, td, cout, s);
        qm::launch_conv3d_fwd(td, cout, wd, kpad_d, cin, nullptr, tdx, 1, 0, s);
    } else {
        qm::launch_conv3d_fwd(tdy, cout, wd, kpad_d, cin, nullptr, tdx, 1, 0, s);
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(wd);
    if (dil) (void)hipFree(dil);
    return check_hip("qumond_k_conv3d_dgrad");
}

qumond_status qumond_k_conv3d_wgrad(int32_t n_in, int32_t cin, const void *x, int32_t cout, const void *dy,
                                    int32_t stride, float *dw, void *stream)
{
    if (!conv_shape_ok(n_in, cin, cout, stride) || !x || !dy || !dw) return ufail(QUMOND_ERR_INVALID, "qumond_k_conv3d_wgrad: bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int kpad = qm::kpad_of(cin);
    const int n_out = stride == 2 ? (n_in + 1) / 2 : n_in;
    float *partial = nullptr;
    const int ns = qm::wgrad_splits(cout, kpad, n_out);
    if (hipMalloc((void **)&partial, (size_t)ns * cout * kpad * 4) != hipSuccess) return ufail(QUMOND_ERR_OOM, "allocation");
    Tensor tx{(__bf16 *)x, n_in, cin};
    Tensor tdy{(__bf16 *)dy, n_out, cout};
    qm::launch_wgrad(tx, cin, tdy, cout, kpad, stride, partial, dw, s);
    (void)hipStreamSynchronize(s);
    (void)hipFree(partial);
    return check_hip("qumond_k_conv3d_wgrad");
}

}  // extern "C"
