// C ABI of the QUMOND particle-mesh solver: configuration checks, the
// per-context grids of every nested box, the call-order state machine, and the
// box-by-box chaining of Sec. 2 (outer Dirichlet value, then each inner box's
// boundary interpolated from the coarser box's converged solution).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/qumond.h"
#include "common.h"
#include "mg.h"

namespace {

thread_local std::string g_last_error;

qumond_status fail(qumond_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

qumond_status hip_fail(hipError_t e, const char *where)
{
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? QUMOND_ERR_OOM : QUMOND_ERR_HIP;
}

enum Stage { ST_CREATED = 0, ST_DEPOSITED = 1, ST_NEWTON = 2, ST_SOURCE = 3, ST_MOND = 4 };

// FP32 multigrid of the mixed-precision solve: hierarchy, the finest level's
// two buffers (initial FMG iterate, then corrections) and its right-hand side
// (FP32 rhs for the FMG, then the scaled FP64 residual).
struct Mixed {
    qm::Multigrid<float> mg;
    float *a[2] = {nullptr, nullptr};
    float *r = nullptr;
    double *sc = nullptr;   // two slots of the refinement scale s and 1/s (device)
    int cur = 0;            // slot of the scale r was formed with
    bool fresh = false;     // r holds the scaled residual of the current iterate
};

struct Box {
    double L = 0, h = 0;
    long long *q = nullptr;
    double *f = nullptr, *phin = nullptr, *S = nullptr, *phi = nullptr;
};

}  // namespace

void qm_set_last_error(const char *msg) { g_last_error = msg; }

struct qumond_ctx {
    qumond_config cfg;
    hipStream_t s = nullptr;
    int n = 0;
    size_t N = 0;
    Box box[QUMOND_MAX_BOX];
    double *scratch = nullptr;           // finest-size ping-pong partner
    qm::Multigrid<double> mg;
    Mixed mix, mix2;   // FP32 hierarchies of the two chains (mixed precision only)
    double total_mass = 0.0;
    int shift = 0;
    int stage = ST_CREATED;
    unsigned long long *d_count = nullptr;
    unsigned long long *h_count = nullptr;  // pinned
    unsigned long long *dep_scratch = nullptr;
    // second solve chain (QUMOND potential) for qumond_solve, created on first use
    bool chain2 = false;
    hipStream_t s2 = nullptr;
    qm::Multigrid<double> mg2;
    double *scratch2 = nullptr;
    hipEvent_t ev_newton[QUMOND_MAX_BOX] = {};
    hipEvent_t ev_done = nullptr;
    qm::NuFn nu;                         // interpolating function (+ device table for nu_n != 1)
    std::vector<void *> owned;
    int64_t bytes = 0;

    hipError_t alloc(void **p, size_t b)
    {
        hipError_t e = hipMalloc(p, b);
        if (e == hipSuccess) {
            owned.push_back(*p);
            bytes += (int64_t)b;
        }
        return e;
    }
};

// The point-mass integral table of the n-family member cfg.nu_n (none for 1).
static hipError_t qm_make_nu(double nu_n, qm::NuFn &nu, const std::function<hipError_t(void **, size_t)> &alloc)
{
    nu.n = nu_n;
    nu.tab = nullptr;
    if (nu_n == 1.0) return hipSuccess;
    std::vector<double> tab(2 * (size_t)qm::kNuTab);
    qm::build_nu_table(nu_n, tab.data());
    double *d = nullptr;
    hipError_t e = alloc((void **)&d, tab.size() * sizeof(double));
    if (e != hipSuccess) return e;
    if ((e = hipMemcpy(d, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess) return e;
    nu.tab = d;
    return hipSuccess;
}

// Deposit scale 2^s with s = 62 - ceil(log2 M) - 1, so that the integer sum of
// all corner shares stays below 2^62 (also used by the batched solver).
int qm_fixed_shift_for(double total_mass)
{
    int e;
    const double mant = std::frexp(total_mass, &e);
    const int ceil_log2 = (mant == 0.5) ? e - 1 : e;
    return 62 - ceil_log2 - 1;
}

extern "C" {

void qumond_default_config(qumond_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n = 65;
    cfg->nbox = 1;
    cfg->box_side[0] = 100.0;
    cfg->G = 4.300917270e-6;
    cfg->a0 = 3600.0;
    cfg->npre = 2;
    cfg->npost = 2;
    cfg->ncycle_fmg = 6;
    cfg->max_vcycles = 50;
    cfg->tol_rel = 1e-10;
    cfg->precision = QUMOND_FP64;
    cfg->outer_bc = QUMOND_BC_MONOPOLE;
    cfg->gather_frac = 0.2;
    cfg->fixed_shift = 0;
    cfg->use_graphs = 0;
    cfg->nu_n = 1.0;
}

qumond_status qumond_validate_config(const qumond_config *c)
{
    if (!c) return fail(QUMOND_ERR_INVALID, "config is NULL");
    if (c->n < 5 || c->n > 1025 || qm::log2_exact(c->n - 1) < 2)
        return fail(QUMOND_ERR_INVALID, "n must be 2^J + 1 with 5 <= n <= 1025");
    if (c->nbox < 1 || c->nbox > QUMOND_MAX_BOX) return fail(QUMOND_ERR_INVALID, "nbox must be in 1..16");
    for (int b = 0; b < c->nbox; ++b) {
        if (!(c->box_side[b] > 0.0) || !std::isfinite(c->box_side[b]))
            return fail(QUMOND_ERR_INVALID, "box_side must be finite and positive");
        if (b > 0 && std::fabs(c->box_side[b] - 0.5 * c->box_side[b - 1]) > 1e-12 * c->box_side[b - 1])
            return fail(QUMOND_ERR_INVALID, "each box_side must be half the previous one");
    }
    if (!(c->G > 0.0) || !std::isfinite(c->G)) return fail(QUMOND_ERR_INVALID, "G must be finite and positive");
    if (!(c->a0 >= 0.0) || !std::isfinite(c->a0)) return fail(QUMOND_ERR_INVALID, "a0 must be finite and >= 0");
    if (c->npre < 0 || c->npre > 8 || c->npost < 0 || c->npost > 8 || c->npre + c->npost < 1)
        return fail(QUMOND_ERR_INVALID, "npre, npost must be in 0..8 with npre + npost >= 1");
    if (c->ncycle_fmg < 1 || c->ncycle_fmg > 64) return fail(QUMOND_ERR_INVALID, "ncycle_fmg must be in 1..64");
    if (c->max_vcycles < 0 || c->max_vcycles > 10000) return fail(QUMOND_ERR_INVALID, "max_vcycles must be in 0..10000");
    if (!(c->tol_rel >= 0.0) || !std::isfinite(c->tol_rel)) return fail(QUMOND_ERR_INVALID, "tol_rel must be >= 0");
    if (c->precision != QUMOND_FP64 && c->precision != QUMOND_MIXED)
        return fail(QUMOND_ERR_INVALID, "precision must be QUMOND_FP64 or QUMOND_MIXED");
    if (c->outer_bc != QUMOND_BC_ZERO && c->outer_bc != QUMOND_BC_MONOPOLE)
        return fail(QUMOND_ERR_INVALID, "outer_bc must be QUMOND_BC_ZERO or QUMOND_BC_MONOPOLE");
    if (!(c->gather_frac > 0.0 && c->gather_frac < 0.5))
        return fail(QUMOND_ERR_INVALID, "gather_frac must be in (0, 0.5)");
    if (c->fixed_shift < 0 || c->fixed_shift > 120) return fail(QUMOND_ERR_INVALID, "fixed_shift must be in 0..120");
    if (!(c->nu_n >= 1.0 && c->nu_n <= 10.0)) return fail(QUMOND_ERR_INVALID, "nu_n must be in [1, 10]");
    return QUMOND_OK;
}

const char *qumond_status_string(qumond_status s)
{
    switch (s) {
    case QUMOND_OK: return "ok";
    case QUMOND_ERR_INVALID: return "invalid argument";
    case QUMOND_ERR_STATE: return "call out of order";
    case QUMOND_ERR_OOM: return "device out of memory";
    case QUMOND_ERR_HIP: return "HIP runtime error";
    case QUMOND_ERR_NOT_CONVERGED: return "not converged";
    case QUMOND_ERR_RANGE: return "value out of range";
    }
    return "unknown status";
}

const char *qumond_last_error(void) { return g_last_error.c_str(); }

qumond_status qumond_destroy(qumond_ctx *ctx)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    (void)hipStreamSynchronize(ctx->s);
    if (ctx->chain2) {
        (void)hipStreamSynchronize(ctx->s2);
        ctx->mg2.release();
        for (hipEvent_t e : ctx->ev_newton)
            if (e) (void)hipEventDestroy(e);
        if (ctx->ev_done) (void)hipEventDestroy(ctx->ev_done);
        (void)hipStreamDestroy(ctx->s2);
    }
    ctx->mg.release();
    ctx->mix.mg.release();
    ctx->mix2.mg.release();
    for (void *p : ctx->owned) (void)hipFree(p);
    if (ctx->h_count) (void)hipHostFree(ctx->h_count);
    delete ctx;
    return QUMOND_OK;
}

qumond_status qumond_create(const qumond_config *cfg, void *hip_stream, qumond_ctx **out)
{
    if (!out) return fail(QUMOND_ERR_INVALID, "out is NULL");
    *out = nullptr;
    qumond_status st = qumond_validate_config(cfg);
    if (st != QUMOND_OK) return st;
    qumond_ctx *c = new (std::nothrow) qumond_ctx();
    if (!c) return fail(QUMOND_ERR_OOM, "host allocation failed");
    c->cfg = *cfg;
    c->s = (hipStream_t)hip_stream;
    c->n = cfg->n;
    c->N = (size_t)c->n * c->n * c->n;
    hipError_t e;
    for (int b = 0; b < cfg->nbox; ++b) {
        Box &B = c->box[b];
        B.L = cfg->box_side[b];
        B.h = B.L / (double)(c->n - 1);
        if ((e = c->alloc((void **)&B.q, c->N * sizeof(long long))) != hipSuccess ||
            (e = c->alloc((void **)&B.f, c->N * sizeof(double))) != hipSuccess ||
            (e = c->alloc((void **)&B.phin, c->N * sizeof(double))) != hipSuccess ||
            (e = c->alloc((void **)&B.S, c->N * sizeof(double))) != hipSuccess ||
            (e = c->alloc((void **)&B.phi, c->N * sizeof(double))) != hipSuccess) {
            qumond_status r = hip_fail(e, "qumond_create: hipMalloc");
            qumond_destroy(c);
            return r;
        }
    }
    if ((e = c->alloc((void **)&c->scratch, c->N * sizeof(double))) != hipSuccess ||
        (e = c->alloc((void **)&c->dep_scratch, qm::deposit_scratch_bytes(cfg->nbox))) != hipSuccess ||
        (e = c->alloc((void **)&c->d_count, sizeof(unsigned long long))) != hipSuccess ||
        (e = hipHostMalloc((void **)&c->h_count, sizeof(unsigned long long), hipHostMallocDefault)) != hipSuccess ||
        (e = c->mg.init(c->n, cfg->npre, cfg->npost, c->s)) != hipSuccess ||
        (cfg->precision == QUMOND_MIXED &&
         ((e = c->mix.mg.init(c->n, cfg->npre, cfg->npost, c->s)) != hipSuccess ||
          (e = c->alloc((void **)&c->mix.a[0], c->N * sizeof(float))) != hipSuccess ||
          (e = c->alloc((void **)&c->mix.a[1], c->N * sizeof(float))) != hipSuccess ||
          (e = c->alloc((void **)&c->mix.r, c->N * sizeof(float))) != hipSuccess ||
          (e = c->alloc((void **)&c->mix.sc, 4 * sizeof(double))) != hipSuccess))) {
        qumond_status r = hip_fail(e, "qumond_create: allocation");
        qumond_destroy(c);
        return r;
    }
    if ((e = qm_make_nu(cfg->nu_n, c->nu, [c](void **p, size_t b) { return c->alloc(p, b); })) != hipSuccess) {
        qumond_status r = hip_fail(e, "qumond_create: nu table");
        qumond_destroy(c);
        return r;
    }
    for (int b = 0; b < cfg->nbox; ++b) {
        qm::launch_fill<long long>(c->box[b].q, c->N, 0LL, c->s);
        qm::launch_fill<double>(c->box[b].f, c->N, 0.0, c->s);
        qm::launch_fill<double>(c->box[b].phin, c->N, 0.0, c->s);
        qm::launch_fill<double>(c->box[b].S, c->N, 0.0, c->s);
        qm::launch_fill<double>(c->box[b].phi, c->N, 0.0, c->s);
    }
    if ((e = hipGetLastError()) != hipSuccess) {
        qumond_status r = hip_fail(e, "qumond_create: launch");
        qumond_destroy(c);
        return r;
    }
    *out = c;
    return QUMOND_OK;
}

qumond_status qumond_profile_enable(qumond_ctx *ctx, int32_t on)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (on < 0 || (on > 1 && (on < 5 || qm::log2_exact(on - 1) < 2)))
        return fail(QUMOND_ERR_INVALID, "qumond_profile_enable: on must be 0, 1 or a level size 2^J + 1 >= 5");
    for (qm::SmootherProfile *p : {&ctx->mg.prof, &ctx->mg2.prof}) {
        p->on = on != 0;
        p->only_n = on > 1 ? on : 0;
    }
    return QUMOND_OK;
}

qumond_status qumond_profile_read(qumond_ctx *ctx, qumond_kernel_stats *out)
{
    if (!ctx || !out) return fail(QUMOND_ERR_INVALID, "NULL argument");
    hipError_t e = hipStreamSynchronize(ctx->s);
    if (e != hipSuccess) return hip_fail(e, "qumond_profile_read");
    if (ctx->chain2 && (e = hipStreamSynchronize(ctx->s2)) != hipSuccess) return hip_fail(e, "qumond_profile_read");
    out->launches = 0;
    out->total_ms = 0.0;
    out->alg_bytes = 0.0;
    out->sweeps_per_launch = 0;
    for (qm::SmootherProfile *p : {&ctx->mg.prof, &ctx->mg2.prof}) {
        out->launches += (int64_t)p->used;
        if (p->used) out->sweeps_per_launch = std::max(out->sweeps_per_launch, (int32_t)p->sweeps);
        for (size_t i = 0; i < p->used; ++i) {
            float ms = 0.0f;
            if ((e = hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1])) != hipSuccess)
                return hip_fail(e, "qumond_profile_read: elapsed");
            out->total_ms += ms;
            out->alg_bytes += p->bytes[i];
        }
        p->used = 0;
        p->bytes.clear();
    }
    return QUMOND_OK;
}

int64_t qumond_device_bytes(const qumond_ctx *ctx)
{
    return ctx ? ctx->bytes + (int64_t)ctx->mg.bytes + (int64_t)ctx->mg2.bytes + (int64_t)ctx->mix.mg.bytes +
                     (int64_t)ctx->mix2.mg.bytes
               : 0;
}


qumond_status qumond_deposit(qumond_ctx *ctx, const double *x, const double *y, const double *z, const double *m,
                             int64_t np, double total_mass, int64_t *n_outside)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (np < 0) return fail(QUMOND_ERR_INVALID, "np must be >= 0");
    if (np > 0 && (!x || !y || !z || !m)) return fail(QUMOND_ERR_INVALID, "particle arrays must not be NULL");
    if (!(total_mass > 0.0) || !std::isfinite(total_mass))
        return fail(QUMOND_ERR_INVALID, "total_mass must be finite and positive");
    const int shift = ctx->cfg.fixed_shift ? ctx->cfg.fixed_shift : qm_fixed_shift_for(total_mass);
    if (std::ldexp(total_mass, shift) >= 9.2e18) return fail(QUMOND_ERR_RANGE, "fixed_shift overflows 64 bits");
    ctx->shift = shift;
    ctx->total_mass = total_mass;
    qm::DepositArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nbox = ctx->cfg.nbox;
    a.n = ctx->n;
    a.scale = std::ldexp(1.0, shift);
    a.scratch = ctx->dep_scratch;
    const int win[3] = {qm::kWinX, qm::kWinY, qm::kWinZ};
    for (int b = 0; b < a.nbox; ++b) {
        for (int d = 0; d < 3; ++d) {
            const int o = (ctx->n - 1) / 2 - win[d] / 2;
            a.w0[b][d] = o < 0 ? 0 : o;
        }
        const Box &B = ctx->box[b];
        a.box[b].L = B.L;
        a.box[b].xmin = -0.5 * B.L;
        a.box[b].inv_h = (double)(ctx->n - 1) / B.L;
        a.box[b].h = B.h;
        a.q[b] = (unsigned long long *)B.q;
        qm::launch_fill<long long>(B.q, ctx->N, 0LL, ctx->s);
    }
    qm::launch_fill<unsigned long long>(ctx->d_count, 1, 0ULL, ctx->s);
    qm::launch_deposit(a, x, y, z, m, np, ctx->d_count, ctx->s);
    const double four_pi_G = 4.0 * M_PI * ctx->cfg.G;
    for (int b = 0; b < a.nbox; ++b)
        qm::launch_rhs_from_q(ctx->n, ctx->box[b].h, four_pi_G, shift, ctx->box[b].q, ctx->box[b].f, ctx->s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "qumond_deposit: launch");
    if (n_outside) {
        if ((e = hipMemcpyAsync(ctx->h_count, ctx->d_count, sizeof(unsigned long long), hipMemcpyDeviceToHost, ctx->s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(ctx->s)) != hipSuccess)
            return hip_fail(e, "qumond_deposit: count");
        *n_outside = np - (int64_t)*ctx->h_count;
    }
    ctx->stage = ST_DEPOSITED;
    return QUMOND_OK;
}

// The solve resources of one chain: hierarchy, stream and ping-pong partner.
struct Chain {
    qm::Multigrid<double> *mg;
    hipStream_t s;
    double *scratch;
    Mixed *mix;
};

static void info_clear(qumond_solve_info *info, int nbox)
{
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->nbox = nbox;
}

// One box of one potential: Dirichlet values (outer value for box 0, the
// coarser box's solution otherwise), FMG, then V-cycles under the stopping test.
static qumond_status solve_box(qumond_ctx *ctx, const Chain &ch, bool mond, int b, qumond_solve_info *info, bool &ok,
                               const void *guess = nullptr, int guess_kind = 0)
{
    const qumond_config &c = ctx->cfg;
    const double GM = c.G * ctx->total_mass;
    Box &B = ctx->box[b];
    double *u = mond ? B.phi : B.phin;
    double *f = mond ? B.S : B.f;
    if (b == 0) {
        const int mode = c.outer_bc == QUMOND_BC_ZERO ? 0 : (mond ? 2 : 1);
        qm::launch_bc_outer(ctx->n, B.L, mode, GM, c.a0, u, ch.scratch, ch.s, ctx->nu);
    } else {
        const double *uc = mond ? ctx->box[b - 1].phi : ctx->box[b - 1].phin;
        qm::launch_bc_from_coarse(ctx->n, uc, u, ch.scratch, ch.s);
    }
    ch.mg->bind(B.L, u, ch.scratch, f);
    ch.mg->set_r32(nullptr, nullptr);
    ch.mix->fresh = false;
    double rr = 0.0, rr0 = 0.0;
    int extra = 0;
    hipError_t e;
    // One FP64 residual-correction step of the mixed solve: the FP64 residual
    // scaled by its RMS (from the norms of the last relres), one FP32 V-cycle
    // on it with zero boundary values, the scaled correction added in FP64.
    // The norms pass that follows a step (the relres() of the loop) also forms
    // the next step's right-hand side, scaled by the power of two from the
    // norms before the step's correction (any power of two gives the same
    // corrected iterate), so only the first step forms it separately.
    auto refine_step = [&]() {
        Mixed &X = *ch.mix;
        double *sc = X.sc + 2 * X.cur;
        if (!X.fresh) {
            qm::launch_mixed_scale(ctx->n, ch.mg->norms, sc, ch.s);
            qm::launch_resid_to_f32(ctx->n, B.h, sc, f, u, X.r, ch.s);
        }
        // zero correction iterate: the buffers are cleared on the first step of
        // a solve; later steps' first sweeps read no iterate
        X.mg.bind(B.L, X.a[0], X.a[1], X.r);
        if (!X.fresh || !X.mg.zero_start_ok()) {
            qm::launch_fill<float>(X.a[0], ctx->N, 0.0f, ch.s);
            qm::launch_fill<float>(X.a[1], ctx->N, 0.0f, ch.s);
        }
        X.mg.zero_start = X.mg.zero_start_ok();
        X.mg.finest_cycle();
        qm::launch_correct(ctx->n, sc, X.mg.result(), u, ch.s);
        X.cur ^= 1;
        qm::launch_mixed_scale(ctx->n, ch.mg->norms, X.sc + 2 * X.cur, ch.s);
        ch.mg->set_r32(X.sc + 2 * X.cur, X.r);
        X.fresh = true;
    };
    const bool mixed = c.precision == QUMOND_MIXED;
    if (guess) {
        // Seeded solve: V-cycles from the guess's interior (in mixed precision,
        // refinement steps with FP32 V-cycles).  The guess is rejected (FMG
        // from zero instead) if it is not finite, if the relative residual
        // after its first V-cycle exceeds 1 (the first smoothing removes the
        // guess's high-frequency error, so the raw residual of the guess says
        // little), or if it needs more cycles than FMG plus max_vcycles.
        const bool no_fallback = (guess_kind & QUMOND_GUESS_NO_FALLBACK) != 0;
        const int kind = guess_kind & 3;
        const size_t esz = kind == QUMOND_GUESS_F64 ? 8 : (kind == QUMOND_GUESS_F32 ? 4 : 2);
        qm::launch_guess_interior(ctx->n, (const char *)guess + (size_t)b * ctx->N * esz, kind, u, ch.s);
        if ((e = ch.mg->relres(rr)) != hipSuccess) return hip_fail(e, "solve: guess");
        rr0 = rr;
        bool accept = no_fallback || std::isfinite(rr);
        const int budget = c.ncycle_fmg + c.max_vcycles;
        while (accept && c.tol_rel > 0.0 && rr > c.tol_rel && extra < budget) {
            if (mixed) refine_step();
            else ch.mg->finest_cycle();
            ++extra;
            if ((e = ch.mg->relres(rr)) != hipSuccess) return hip_fail(e, "solve: V-cycle");
            if (!no_fallback && (!std::isfinite(rr) || (extra == 1 && rr > 1.0))) accept = false;
        }
        if (no_fallback || (accept && !(c.tol_rel > 0.0 && rr > c.tol_rel))) {
            ch.mg->finish();
            ok = !(c.tol_rel > 0.0 && !(rr <= c.tol_rel));
            if (info) {
                if (mixed) info->refine_iters[b] = extra;
                info->vcycles[b] = extra;
                info->relres0[b] = rr0;
                info->relres[b] = rr;
                info->converged[b] = ok ? 1 : 0;
            }
            if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "solve: launch");
            return QUMOND_OK;
        }
        // fallback: FMG from zero with the same Dirichlet values
        ch.mg->finish();
        if (info) info->used_fallback = 1;
        qm::launch_fill<double>(u, ctx->N, 0.0, ch.s);
        if (b == 0) {
            const int mode = c.outer_bc == QUMOND_BC_ZERO ? 0 : (mond ? 2 : 1);
            qm::launch_bc_outer(ctx->n, B.L, mode, GM, c.a0, u, ch.scratch, ch.s, ctx->nu);
        } else {
            const double *uc = mond ? ctx->box[b - 1].phi : ctx->box[b - 1].phin;
            qm::launch_bc_from_coarse(ctx->n, uc, u, ch.scratch, ch.s);
        }
        ch.mg->bind(B.L, u, ch.scratch, f);
        extra = 0;
    }
    if (mixed) {
        // FP32 FMG seeds the FP64 iterate ...
        Mixed &X = *ch.mix;
        qm::launch_narrow(f, X.r, ctx->N, ch.s);
        qm::launch_narrow_boundary(ctx->n, u, X.a[0], X.a[1], ch.s);
        X.mg.bind(B.L, X.a[0], X.a[1], X.r);
        X.mg.fmg(c.ncycle_fmg);
        qm::launch_widen_interior(ctx->n, X.mg.result(), u, ch.s);
        if ((e = ch.mg->relres(rr)) != hipSuccess) return hip_fail(e, "solve: FP32 FMG");
        rr0 = rr;
        // ... then FP64 residual correction with FP32 V-cycles (zero boundary
        // values); the scale comes from the residual norms already on the device.
        while (c.tol_rel > 0.0 && rr > c.tol_rel && extra < c.max_vcycles) {
            refine_step();
            ++extra;
            if ((e = ch.mg->relres(rr)) != hipSuccess) return hip_fail(e, "solve: refinement");
        }
        if (info) info->refine_iters[b] = extra;
    } else {
        // the fixed schedules run from captured graphs when cfg.use_graphs is set
        ch.mg->use_graphs = c.use_graphs != 0;
        if ((e = ch.mg->fmg_norms(c.ncycle_fmg)) != hipSuccess || (e = ch.mg->relres_read(rr)) != hipSuccess)
            return hip_fail(e, "solve: FMG");
        rr0 = rr;
        while (c.tol_rel > 0.0 && rr > c.tol_rel && extra < c.max_vcycles) {
            ++extra;
            if ((e = ch.mg->cycle_norms()) != hipSuccess || (e = ch.mg->relres_read(rr)) != hipSuccess)
                return hip_fail(e, "solve: V-cycle");
        }
        ch.mg->finish();
    }
    ok = !(c.tol_rel > 0.0 && !(rr <= c.tol_rel));
    if (info) {
        info->vcycles[b] = extra;
        info->relres0[b] = rr0;
        info->relres[b] = rr;
        info->converged[b] = ok ? 1 : 0;
    }
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "solve: launch");
    return QUMOND_OK;
}

// FMG chain over the boxes for one of the two potentials.
static qumond_status solve_chain(qumond_ctx *ctx, bool mond, qumond_solve_info *info, const void *guess = nullptr,
                                 int guess_kind = 0)
{
    info_clear(info, ctx->cfg.nbox);
    const Chain ch{&ctx->mg, ctx->s, ctx->scratch, &ctx->mix};
    bool all_ok = true;
    for (int b = 0; b < ctx->cfg.nbox; ++b) {
        bool ok = true;
        qumond_status st = solve_box(ctx, ch, mond, b, info, ok, guess, guess_kind);
        if (st != QUMOND_OK) return st;
        all_ok = all_ok && ok;
    }
    if (!all_ok) return fail(QUMOND_ERR_NOT_CONVERGED, "relative residual above tol_rel after max_vcycles");
    return QUMOND_OK;
}

qumond_status qumond_solve_newton(qumond_ctx *ctx, qumond_solve_info *info)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (ctx->stage < ST_DEPOSITED) return fail(QUMOND_ERR_STATE, "qumond_solve_newton before qumond_deposit");
    qumond_status st = solve_chain(ctx, false, info);
    if (st == QUMOND_OK || st == QUMOND_ERR_NOT_CONVERGED) ctx->stage = ST_NEWTON;
    return st;
}

qumond_status qumond_mond_source(qumond_ctx *ctx)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (ctx->stage < ST_NEWTON) return fail(QUMOND_ERR_STATE, "qumond_mond_source before qumond_solve_newton");
    for (int b = 0; b < ctx->cfg.nbox; ++b)
        qm::launch_mond_source(ctx->n, ctx->box[b].h, ctx->cfg.a0, ctx->box[b].phin, ctx->box[b].S, ctx->s, 1,
                              ctx->cfg.nu_n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "qumond_mond_source: launch");
    ctx->stage = ST_SOURCE;
    return QUMOND_OK;
}

qumond_status qumond_solve_mond(qumond_ctx *ctx, const void *guess, int32_t guess_kind, qumond_solve_info *info)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (ctx->stage < ST_SOURCE) return fail(QUMOND_ERR_STATE, "qumond_solve_mond before qumond_mond_source");
    const int kind = guess_kind & ~QUMOND_GUESS_NO_FALLBACK;
    if (kind < QUMOND_GUESS_NONE || kind > QUMOND_GUESS_BF16 || (guess_kind & ~(QUMOND_GUESS_NO_FALLBACK | 3)))
        return fail(QUMOND_ERR_INVALID, "unknown guess_kind");
    if (kind != QUMOND_GUESS_NONE && !guess) return fail(QUMOND_ERR_INVALID, "guess is NULL");
    qumond_status st = solve_chain(ctx, true, info, kind == QUMOND_GUESS_NONE ? nullptr : guess, guess_kind);
    if (st == QUMOND_OK || st == QUMOND_ERR_NOT_CONVERGED) ctx->stage = ST_MOND;
    return st;
}

// Steps 2-4 with the two chains overlapped: the Newtonian chain runs on the
// context's stream in the calling thread; the QUMOND chain runs on a second
// stream in a worker thread, box b starting (source, then solve) as soon as the
// Newtonian solve of box b has completed on the device.  Same kernels, same
// schedules: the fields equal those of the three separate calls bit for bit.
static qumond_status ensure_chain2(qumond_ctx *ctx)
{
    if (ctx->chain2) return QUMOND_OK;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&ctx->s2, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "qumond_solve: stream");
    if ((e = ctx->mg2.init(ctx->n, ctx->cfg.npre, ctx->cfg.npost, ctx->s2)) != hipSuccess ||
        (e = ctx->alloc((void **)&ctx->scratch2, ctx->N * sizeof(double))) != hipSuccess)
        return hip_fail(e, "qumond_solve: allocation");
    if (ctx->cfg.precision == QUMOND_MIXED &&
        ((e = ctx->mix2.mg.init(ctx->n, ctx->cfg.npre, ctx->cfg.npost, ctx->s2)) != hipSuccess ||
         (e = ctx->alloc((void **)&ctx->mix2.a[0], ctx->N * sizeof(float))) != hipSuccess ||
         (e = ctx->alloc((void **)&ctx->mix2.a[1], ctx->N * sizeof(float))) != hipSuccess ||
         (e = ctx->alloc((void **)&ctx->mix2.r, ctx->N * sizeof(float))) != hipSuccess ||
         (e = ctx->alloc((void **)&ctx->mix2.sc, 4 * sizeof(double))) != hipSuccess))
        return hip_fail(e, "qumond_solve: allocation");
    for (int b = 0; b < ctx->cfg.nbox; ++b)
        if ((e = hipEventCreateWithFlags(&ctx->ev_newton[b], hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "qumond_solve: event");
    if ((e = hipEventCreateWithFlags(&ctx->ev_done, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "qumond_solve: event");
    ctx->mg2.prof.on = ctx->mg.prof.on;
    ctx->chain2 = true;
    return QUMOND_OK;
}

qumond_status qumond_solve(qumond_ctx *ctx, qumond_solve_info *info_newton, qumond_solve_info *info_mond)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (ctx->stage < ST_DEPOSITED) return fail(QUMOND_ERR_STATE, "qumond_solve before qumond_deposit");
    qumond_status st = ensure_chain2(ctx);
    if (st != QUMOND_OK) return st;
    const int nbox = ctx->cfg.nbox;
    info_clear(info_newton, nbox);
    info_clear(info_mond, nbox);
    hipError_t e;
    // the second stream must see everything already queued on the first (the deposit)
    if ((e = hipEventRecord(ctx->ev_done, ctx->s)) != hipSuccess || (e = hipStreamWaitEvent(ctx->s2, ctx->ev_done, 0)) != hipSuccess)
        return hip_fail(e, "qumond_solve: order");
    std::mutex mu;
    std::condition_variable cv;
    int newton_done = 0;
    int mond_waited = 0;        // boxes whose Newtonian event the QUMOND stream already waits on
    bool worker_exited = false;
    bool abort = false;
    qumond_status st_m = QUMOND_OK;
    std::string err_m;
    bool ok_m = true;
    // With graph capture, a stream may not wait on an event of a stream that is
    // capturing: the Newtonian chain starts its next box (and capture) only after
    // the QUMOND stream has enqueued its wait on the previous box's event.
    const bool handshake = ctx->cfg.use_graphs != 0;
    std::thread worker([&]() {
        struct Exit {
            std::mutex &mu;
            std::condition_variable &cv;
            bool &flag;
            ~Exit()
            {
                std::lock_guard<std::mutex> lk(mu);
                flag = true;
                cv.notify_all();
            }
        } on_exit{mu, cv, worker_exited};
        const Chain ch{&ctx->mg2, ctx->s2, ctx->scratch2, &ctx->mix2};
        for (int b = 0; b < nbox; ++b) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return newton_done > b || abort; });
                if (newton_done <= b) return;   // the Newtonian chain failed
            }
            hipError_t we = hipStreamWaitEvent(ctx->s2, ctx->ev_newton[b], 0);
            {
                std::lock_guard<std::mutex> lk(mu);
                mond_waited = b + 1;
                cv.notify_all();
            }
            if (we != hipSuccess) {
                st_m = hip_fail(we, "qumond_solve: wait");
                err_m = g_last_error;
                return;
            }
            qm::launch_mond_source(ctx->n, ctx->box[b].h, ctx->cfg.a0, ctx->box[b].phin, ctx->box[b].S, ctx->s2, 1,
                                  ctx->cfg.nu_n);
            bool ok = true;
            st_m = solve_box(ctx, ch, true, b, info_mond, ok);
            if (st_m != QUMOND_OK) {
                err_m = g_last_error;
                return;
            }
            ok_m = ok_m && ok;
        }
    });
    const Chain ch{&ctx->mg, ctx->s, ctx->scratch, &ctx->mix};
    bool ok_n = true;
    qumond_status st_n = QUMOND_OK;
    for (int b = 0; b < nbox; ++b) {
        bool ok = true;
        st_n = solve_box(ctx, ch, false, b, info_newton, ok);
        if (st_n == QUMOND_OK && (e = hipEventRecord(ctx->ev_newton[b], ctx->s)) != hipSuccess)
            st_n = hip_fail(e, "qumond_solve: record");
        if (st_n != QUMOND_OK) break;
        ok_n = ok_n && ok;
        std::unique_lock<std::mutex> lk(mu);
        newton_done = b + 1;
        cv.notify_all();
        if (handshake && b + 1 < nbox) cv.wait(lk, [&] { return mond_waited > b || worker_exited; });
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        if (st_n != QUMOND_OK) abort = true;
        cv.notify_all();
    }
    worker.join();
    if (st_n != QUMOND_OK) return st_n;
    if (st_m != QUMOND_OK) return fail(st_m, err_m);
    // later work on the context's stream (the gather) must see the QUMOND chain
    if ((e = hipEventRecord(ctx->ev_done, ctx->s2)) != hipSuccess || (e = hipStreamWaitEvent(ctx->s, ctx->ev_done, 0)) != hipSuccess)
        return hip_fail(e, "qumond_solve: join");
    ctx->stage = ST_MOND;
    if (!ok_n || !ok_m) return fail(QUMOND_ERR_NOT_CONVERGED, "relative residual above tol_rel after max_vcycles");
    return QUMOND_OK;
}

static qm::GatherArgs gather_args(const qumond_ctx *ctx, int which)
{
    qm::GatherArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nbox = ctx->cfg.nbox;
    a.n = ctx->n;
    for (int b = 0; b < a.nbox; ++b) {
        const Box &B = ctx->box[b];
        a.box[b].L = B.L;
        a.box[b].xmin = -0.5 * B.L;
        a.box[b].inv_h = (double)(ctx->n - 1) / B.L;
        a.box[b].h = B.h;
        a.phi[b] = which == QUMOND_WHICH_QUMOND ? B.phi : B.phin;
    }
    a.frac = ctx->cfg.gather_frac;
    a.GM = ctx->cfg.G * ctx->total_mass;
    a.a0 = ctx->cfg.a0;
    a.mond = which == QUMOND_WHICH_QUMOND;
    a.alg = which == QUMOND_WHICH_ALGEBRAIC;
    a.nun = ctx->cfg.nu_n;
    return a;
}

// The field choice of the gather-type calls and the stage it needs.
static qumond_status check_which(const qumond_ctx *ctx, int which)
{
    if (which != QUMOND_WHICH_NEWTON && which != QUMOND_WHICH_QUMOND && which != QUMOND_WHICH_ALGEBRAIC)
        return fail(QUMOND_ERR_INVALID, "which must be 0 (Newton), 1 (QUMOND) or 2 (algebraic MOND)");
    if (ctx->stage < (which == QUMOND_WHICH_QUMOND ? ST_MOND : ST_NEWTON))
        return fail(QUMOND_ERR_STATE, "potential not solved yet");
    return QUMOND_OK;
}

qumond_status qumond_gather_forces(qumond_ctx *ctx, const double *x, const double *y, const double *z, int64_t np,
                                   int32_t which, double *ax, double *ay, double *az, uint8_t *box_used)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (np < 0) return fail(QUMOND_ERR_INVALID, "np must be >= 0");
    if (np > 0 && (!x || !y || !z || !ax || !ay || !az)) return fail(QUMOND_ERR_INVALID, "array is NULL");
    qumond_status st = check_which(ctx, which);
    if (st != QUMOND_OK) return st;
    qm::launch_gather(gather_args(ctx, which), x, y, z, np, ax, ay, az, box_used, ctx->s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "qumond_gather_forces: launch");
    return QUMOND_OK;
}

qumond_status qumond_rotation_curve(qumond_ctx *ctx, const double *R, int32_t nR, int32_t naz, int32_t which,
                                    double *vc2)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (nR < 0 || naz < 1 || naz > 1024) return fail(QUMOND_ERR_INVALID, "need nR >= 0 and 1 <= naz <= 1024");
    if (nR > 0 && (!R || !vc2)) return fail(QUMOND_ERR_INVALID, "array is NULL");
    qumond_status st = check_which(ctx, which);
    if (st != QUMOND_OK) return st;
    qm::launch_rotation_curve(gather_args(ctx, which), R, nR, naz, vc2, ctx->s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "qumond_rotation_curve: launch");
    return QUMOND_OK;
}

qumond_status qumond_sigma_z(qumond_ctx *ctx, const double *R, int32_t nR, int32_t naz, double z, double z0,
                             int32_t which, double *sig2)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (nR < 0 || naz < 1 || naz > 1024) return fail(QUMOND_ERR_INVALID, "need nR >= 0 and 1 <= naz <= 1024");
    if (!(z > 0.0) || !(z0 > 0.0) || !std::isfinite(z) || !std::isfinite(z0))
        return fail(QUMOND_ERR_INVALID, "need finite z > 0 and z0 > 0");
    if (nR > 0 && (!R || !sig2)) return fail(QUMOND_ERR_INVALID, "array is NULL");
    qumond_status st = check_which(ctx, which);
    if (st != QUMOND_OK) return st;
    qm::launch_sigma_z(gather_args(ctx, which), R, nR, naz, z, z0, sig2, ctx->s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "qumond_sigma_z: launch");
    return QUMOND_OK;
}

static void *field_ptr(qumond_ctx *ctx, int box, int field)
{
    Box &B = ctx->box[box];
    switch (field) {
    case QUMOND_FIELD_RHO_FIXED: return B.q;
    case QUMOND_FIELD_RHS: return B.f;
    case QUMOND_FIELD_PHI_N: return B.phin;
    case QUMOND_FIELD_SOURCE: return B.S;
    case QUMOND_FIELD_PHI: return B.phi;
    }
    return nullptr;
}

qumond_status qumond_get_field(qumond_ctx *ctx, int32_t box, int32_t field, void *dst)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (box < 0 || box >= ctx->cfg.nbox) return fail(QUMOND_ERR_INVALID, "box out of range");
    if (field < QUMOND_FIELD_RHO_FIXED || field > QUMOND_FIELD_PHI) return fail(QUMOND_ERR_INVALID, "unknown field");
    if (!dst) return fail(QUMOND_ERR_INVALID, "dst is NULL");
    hipError_t e = hipMemcpyAsync(dst, field_ptr(ctx, box, field), ctx->N * 8, hipMemcpyDeviceToDevice, ctx->s);
    if (e != hipSuccess) return hip_fail(e, "qumond_get_field");
    return QUMOND_OK;
}

qumond_status qumond_set_field(qumond_ctx *ctx, int32_t box, int32_t field, const void *src)
{
    if (!ctx) return fail(QUMOND_ERR_INVALID, "ctx is NULL");
    if (box < 0 || box >= ctx->cfg.nbox) return fail(QUMOND_ERR_INVALID, "box out of range");
    if (field < QUMOND_FIELD_RHS || field > QUMOND_FIELD_PHI)
        return fail(QUMOND_ERR_INVALID, "settable fields: RHS, PHI_N, SOURCE, PHI");
    if (!src) return fail(QUMOND_ERR_INVALID, "src is NULL");
    hipError_t e = hipMemcpyAsync(field_ptr(ctx, box, field), src, ctx->N * 8, hipMemcpyDeviceToDevice, ctx->s);
    if (e != hipSuccess) return hip_fail(e, "qumond_set_field");
    static const int stage_of[] = {ST_DEPOSITED, ST_DEPOSITED, ST_NEWTON, ST_SOURCE, ST_MOND};
    ctx->stage = stage_of[field];
    return QUMOND_OK;
}

}  // extern "C"
