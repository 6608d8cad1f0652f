// Batched single-box QUMOND solves (qumond_batch.h): many independent disks of
// a rotation-curve fit, grouped by grid size into classes whose grids lie back
// to back, so that each launch of the Sec. 2 pipeline covers a whole class.
// The classes run on streams of their own; the whole batch is captured once
// as a hipGraph (fork/join over the class streams) and replayed.  Per-problem
// inputs sit in a device table, so a replay picks up new particles without a
// new capture.  After each run the host reads the residual history of every
// problem and gives the few above tolerance extra refinement steps.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qumond_batch.h"
#include "common.h"
#include "mg.h"

void qm_set_last_error(const char *msg);
int qm_fixed_shift_for(double total_mass);

namespace {

qumond_status bfail(qumond_status s, const std::string &m)
{
    qm_set_last_error(m.c_str());
    return s;
}

qumond_status bhip(hipError_t e, const char *where)
{
    const std::string m = std::string(where) + ": " + hipGetErrorString(e);
    qm_set_last_error(m.c_str());
    return e == hipErrorOutOfMemory ? QUMOND_ERR_OOM : QUMOND_ERR_HIP;
}

// One class: every problem with the same n, stored back to back.
struct Class {
    int n = 0, J = 0, P = 0;
    size_t N = 0;
    double h = 0.0;
    std::vector<int> ids;                 // batch index of each slot
    hipStream_t s = nullptr;
    hipEvent_t join = nullptr;
    qm::BatchProblem *prob = nullptr;     // device table [P]
    qm::BatchProblem *hprob = nullptr;    // pinned staging of the table
    double *f = nullptr, *phin = nullptr, *S = nullptr, *phi = nullptr;   // [P][N] FP64
    long long *q = nullptr;               // fixed-point mass, aliases S (dead once f is formed)
    float *a[2] = {nullptr, nullptr}, *r = nullptr;                       // [P][N] FP32 finest level
    qm::Multigrid<float> mg;              // FP32 coarse levels, nb = P
    qm::LevelShapes shapes;
    double *partial = nullptr;            // norm partials [P][3][kNormBlocks]
    double *hist = nullptr;               // norms [2 solves][K+1 steps][P][3]
    double *hhist = nullptr;              // pinned copy
    double *sc = nullptr;                 // refinement scale [P][2]
    unsigned long long *dep = nullptr;    // deposit slabs
    unsigned long long *inside = nullptr; // [P]
    unsigned long long *hinside = nullptr;
    double *vc2[2] = {nullptr, nullptr};  // [P][nR] Newton, QUMOND
    // single-problem tail resources
    double *norms1 = nullptr, *sc1 = nullptr, *hnorms1 = nullptr;
    std::string tune_json;
};

double relres_of(const double *nm)
{
    const double rn = std::sqrt(nm[0]), fn = std::sqrt(nm[1]), bn = std::sqrt(nm[2]);
    const double den = fn > 0.0 ? fn : bn;
    return den > 0.0 ? rn / den : rn;
}

bool good_batch_n(int n) { return n >= 17 && n <= 1025 && qm::log2_exact(n - 1) >= 4; }

}  // namespace

struct qumond_batch {
    qumond_batch_config cfg;
    hipStream_t user = nullptr;   // caller's stream
    hipStream_t main = nullptr;   // capture stream
    hipEvent_t ev_in = nullptr, fork = nullptr;
    std::vector<int> n_of, cls_of, slot_of;
    std::vector<std::unique_ptr<Class>> cls;
    std::vector<int> has_particles;
    double *R = nullptr;
    int nR = 0;
    qm::NuFn nu;                  // interpolating function (+ device table for nu_n != 1)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t graph_nodes = 0;
    bool tuned = false;
    std::vector<void *> owned, owned_host;
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
    hipError_t alloc_host(void **p, size_t b)
    {
        hipError_t e = hipHostMalloc(p, b, hipHostMallocDefault);
        if (e == hipSuccess) owned_host.push_back(*p);
        return e;
    }
};

namespace {

int K_of(const qumond_batch *B) { return B->cfg.refine_iters; }

double *hist_slot(const qumond_batch *B, Class &C, bool mond, int step, int slot)
{
    const int K = K_of(B);
    return C.hist + (((size_t)(mond ? 1 : 0) * (K + 1) + step) * C.P + slot) * 3;
}

// A view of the class hierarchy for a single problem (its first slice of each
// level; the levels only hold temporaries).
qm::Multigrid<float> single_view(const Class &C)
{
    qm::Multigrid<float> v;
    v.J = C.mg.J;
    v.lt = C.mg.lt;
    v.L = C.mg.L;
    v.npre = C.mg.npre;
    v.npost = C.mg.npost;
    v.lv = C.mg.lv;
    v.s = C.mg.s;
    v.nb = 1;
    v.shapes = C.mg.shapes;
    return v;
}

// One potential's mixed-precision solve for slots [p0, p0 + nb) of class C:
// outer values, FP32 FMG seed, FP64 norms, then K refinement steps, each
// followed by the FP64 norms that scale the next step.
void enqueue_solve(const qumond_batch *B, Class &C, qm::Multigrid<float> &mg, bool mond, int p0, int nb, int K,
                   hipStream_t s)
{
    const qumond_batch_config &c = B->cfg;
    double *u = (mond ? C.phi : C.phin) + (size_t)p0 * C.N;
    const double *f = (mond ? C.S : C.f) + (size_t)p0 * C.N;
    const size_t cnt = (size_t)nb * C.N;
    qm::launch_bc_outer_batch(C.n, c.box_side, mond ? 2 : 1, c.G, c.a0, C.prob + p0, u, nb, s, B->nu);
    qm::launch_narrow(f, C.r, cnt, s);
    qm::launch_narrow_boundary(C.n, u, C.a[0], C.a[1], s, nb);
    mg.bind(c.box_side, C.a[0], C.a[1], C.r);
    mg.fmg(c.ncycle_fmg);
    qm::launch_widen_interior(C.n, mg.result(), u, s, nb);
    qm::launch_resid_norms<double>(C.n, C.h, f, u, C.partial, hist_slot(B, C, mond, 0, p0), s, nb);
    // Scales in two slots of 2 nb doubles: step k corrects with the scale its
    // right-hand side was formed with, and its norms pass forms the next
    // right-hand side with the power of two from the norms before its correction.
    double *const scs[2] = {C.sc, C.sc + 2 * (size_t)C.P};
    for (int k = 1; k <= K; ++k) {
        double *cur = scs[(k - 1) & 1], *next = scs[k & 1];
        if (k == 1) {
            qm::launch_mixed_scale(C.n, hist_slot(B, C, mond, 0, p0), cur, s, nb);
            qm::launch_resid_to_f32(C.n, C.h, cur, f, u, C.r, s, nb);
        }
        // zero correction iterate: the buffers (boundaries left by the FMG) are
        // cleared once; later steps' first sweeps read no iterate
        mg.bind(c.box_side, C.a[0], C.a[1], C.r);
        if (k == 1 || !mg.zero_start_ok()) {
            qm::launch_fill<float>(C.a[0], cnt, 0.0f, s);
            qm::launch_fill<float>(C.a[1], cnt, 0.0f, s);
        }
        mg.zero_start = mg.zero_start_ok();
        mg.finest_cycle();
        qm::launch_correct(C.n, cur, mg.result(), u, s, nb);
        qm::launch_mixed_scale(C.n, hist_slot(B, C, mond, k - 1, p0), next, s, nb);
        qm::launch_resid_norms_r32(C.n, C.h, f, u, C.partial, hist_slot(B, C, mond, k, p0), next, C.r, s, nb);
    }
}

void enqueue_curves(const qumond_batch *B, Class &C, int p0, int nb, int which, hipStream_t s)
{
    const qumond_batch_config &c = B->cfg;
    for (int w = 0; w < 2; ++w) {
        if (which >= 0 && w != which) continue;
        qm::launch_rotation_curve_batch(C.n, c.box_side, c.gather_frac, c.G, c.a0, w, C.prob + p0,
                                        (w ? C.phi : C.phin) + (size_t)p0 * C.N, B->R, B->nR, c.naz,
                                        C.vc2[w] + (size_t)p0 * B->nR, nb, s, c.nu_n);
    }
}

// The whole pipeline of one class on stream s.
void enqueue_class(const qumond_batch *B, Class &C, hipStream_t s)
{
    const qumond_batch_config &c = B->cfg;
    qm::launch_fill<long long>(C.q, (size_t)C.P * C.N, 0LL, s);
    qm::launch_fill<unsigned long long>(C.inside, (size_t)C.P, 0ULL, s);
    qm::launch_deposit_batch(C.n, c.box_side, C.prob, 0, (unsigned long long *)C.q, C.dep, C.inside, C.P, s);
    qm::launch_rhs_batch(C.n, C.h, 4.0 * M_PI * c.G, C.prob, C.q, C.f, C.P, s);
    enqueue_solve(B, C, C.mg, false, 0, C.P, K_of(B), s);
    qm::launch_mond_source(C.n, C.h, c.a0, C.phin, C.S, s, C.P, c.nu_n);
    enqueue_solve(B, C, C.mg, true, 0, C.P, K_of(B), s);
    enqueue_curves(B, C, 0, C.P, -1, s);
    (void)hipMemcpyAsync(C.hinside, C.inside, (size_t)C.P * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(C.hhist, C.hist, (size_t)2 * (K_of(B) + 1) * C.P * 3 * sizeof(double),
                         hipMemcpyDeviceToHost, s);
}

hipError_t enqueue_all(qumond_batch *B)
{
    hipError_t e;
    if ((e = hipEventRecord(B->fork, B->main)) != hipSuccess) return e;
    for (auto &cp : B->cls) {
        Class &C = *cp;
        if ((e = hipStreamWaitEvent(C.s, B->fork, 0)) != hipSuccess) return e;
        enqueue_class(B, C, C.s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipEventRecord(C.join, C.s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(B->main, C.join, 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Extra refinement steps for slot p (single problem) until tol or max_extra;
// starts from the norms at `last` (device, 3 doubles).  Returns the steps
// taken and the final relative residual.
hipError_t tail_steps(qumond_batch *B, Class &C, bool mond, int p, const double *last, int &steps, double &rr)
{
    const qumond_batch_config &c = B->cfg;
    qm::Multigrid<float> mg = single_view(C);
    double *u = (mond ? C.phi : C.phin) + (size_t)p * C.N;
    const double *f = (mond ? C.S : C.f) + (size_t)p * C.N;
    hipStream_t s = C.s;
    steps = 0;
    hipError_t e;
    while (rr > c.tol_rel && steps < c.max_extra) {
        qm::launch_mixed_scale(C.n, last, C.sc1, s, 1);
        qm::launch_resid_to_f32(C.n, C.h, C.sc1, f, u, C.r, s, 1);
        mg.bind(c.box_side, C.a[0], C.a[1], C.r);
        if (steps == 0 || !mg.zero_start_ok()) {
            qm::launch_fill<float>(C.a[0], C.N, 0.0f, s);
            qm::launch_fill<float>(C.a[1], C.N, 0.0f, s);
        }
        mg.zero_start = mg.zero_start_ok();
        mg.finest_cycle();
        qm::launch_correct(C.n, C.sc1, mg.result(), u, s, 1);
        qm::launch_resid_norms<double>(C.n, C.h, f, u, C.partial, C.norms1, s, 1);
        if ((e = hipMemcpyAsync(C.hnorms1, C.norms1, 3 * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return e;
        rr = relres_of(C.hnorms1);
        last = C.norms1;
        ++steps;
        if (!std::isfinite(rr)) break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ autotuner

const int kTuneChunks[] = {2, 4, 8, 16, 32, 64, 0};

hipError_t tune_class(qumond_batch *B, Class &C, int reps)
{
    hipStream_t s = C.s;
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
    std::string js = "[";
    bool first = true;
    const int zmax = 65535 / C.P;
    for (int l = C.mg.lt + 1; l <= C.J; ++l) {
        const int n = (1 << l) + 1;
        const size_t cnt = (size_t)n * n * n * C.P;
        float *u0 = l == C.J ? C.a[0] : C.mg.lv[l].u[0];
        float *u1 = l == C.J ? C.a[1] : C.mg.lv[l].u[1];
        float *f = l == C.J ? C.r : C.mg.lv[l].f;
        qm::launch_fill<float>(u0, cnt, 0.5f, s);
        qm::launch_fill<float>(u1, cnt, 0.5f, s);
        qm::launch_fill<float>(f, cnt, 1.0f, s);
        const double h = B->cfg.box_side / (double)(n - 1);
        double best[2] = {1e30, 1e30};
        for (int fz = 0; fz < 2; ++fz) {
            const int nvar = fz ? qm::kFusedVariants : qm::kSmootherVariants;
            for (int v = 0; v < nvar; ++v)
                for (int kc : kTuneChunks) {
                    if (kc != 0 && kc >= n - 2) continue;
                    if (qm::takes_no_chunk(v, fz != 0) && kc != 0) continue;
                    if (fz && kc != 0 && kc < 4) continue;   // the two-sweep march needs 4-plane chunks
                    const int nzc = kc ? (n - 2 + kc - 1) / kc : 1;
                    if (nzc > zmax) continue;
                    const qm::SmootherShape sh{v, kc};
                    auto run = [&](int r) {
                        const float *a = (r & 1) ? u1 : u0;
                        float *b = (r & 1) ? u0 : u1;
                        if (fz) qm::launch_rbgs2_shape<float>(n, h, f, a, b, nullptr, sh, s, C.P);
                        else qm::launch_rbgs_shape<float>(n, h, f, a, b, sh, s, C.P);
                    };
                    run(0);
                    std::vector<float> t;
                    for (int r = 0; r < reps; ++r) {
                        (void)hipEventRecord(e0, s);
                        run(r);
                        (void)hipEventRecord(e1, s);
                        if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
                        float ms = 0.f;
                        (void)hipEventElapsedTime(&ms, e0, e1);
                        t.push_back(ms);
                    }
                    std::sort(t.begin(), t.end());
                    const double us = 1e3 * t[t.size() / 2];
                    if (us < best[fz]) {
                        best[fz] = us;
                        (fz ? C.shapes.fused[l] : C.shapes.single[l]) = sh;
                    }
                }
        }
        C.shapes.use_fused[l] = best[1] < 2.0 * best[0] ? 1 : 0;
        // the single sweep that also applies the coarse-grid correction: its own shape, timed with a correction
        const int ncl = (n + 1) / 2;
        float *ucr = C.mg.lv[l - 1].u[0];
        qm::launch_fill<float>(ucr, (size_t)ncl * ncl * ncl * C.P, 0.001f, s);
        double best_corr = 1e30;
        for (int v = 0; v < qm::kSmootherVariants; ++v)
            for (int kc : kTuneChunks) {
                if (kc != 0 && kc >= n - 2) continue;
                if (qm::is_brick_variant(v, false) && kc != 0) continue;
                const int nzc = kc ? (n - 2 + kc - 1) / kc : 1;
                if (nzc > zmax) continue;
                const qm::SmootherShape sh{v, kc};
                auto run = [&](int r) {
                    const float *a = (r & 1) ? u1 : u0;
                    float *b = (r & 1) ? u0 : u1;
                    qm::launch_rbgs_shape<float>(n, h, f, a, b, sh, s, C.P, ucr);
                };
                run(0);
                std::vector<float> t;
                for (int r = 0; r < reps; ++r) {
                    (void)hipEventRecord(e0, s);
                    run(r);
                    (void)hipEventRecord(e1, s);
                    if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    t.push_back(ms);
                }
                std::sort(t.begin(), t.end());
                const double us = 1e3 * t[t.size() / 2];
                if (us < best_corr) {
                    best_corr = us;
                    C.shapes.corr[l] = sh;
                }
            }
        // residual restriction from this level: both kernels on the batch's own grids
        double rr_us[qm::kRrVariants] = {};
        {
            // levels lt..J-1 are allocated and l - 1 >= lt here
            float *fc = C.mg.lv[l - 1].f, *c0 = C.mg.lv[l - 1].u[0], *c1 = C.mg.lv[l - 1].u[1];
            {
                for (int v = 0; v < qm::kRrVariants; ++v) {
                    qm::launch_residual_restrict_variant<float>(n, h, f, u0, fc, c0, c1, v, s, C.P);
                    std::vector<float> t;
                    for (int r = 0; r < reps; ++r) {
                        (void)hipEventRecord(e0, s);
                        qm::launch_residual_restrict_variant<float>(n, h, f, u0, fc, c0, c1, v, s, C.P);
                        (void)hipEventRecord(e1, s);
                        if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
                        float ms = 0.f;
                        (void)hipEventElapsedTime(&ms, e0, e1);
                        t.push_back(ms);
                    }
                    std::sort(t.begin(), t.end());
                    rr_us[v] = 1e3 * t[t.size() / 2];
                }
                int best = 0;
                for (int v = 1; v < qm::kRrVariants; ++v)
                    if (rr_us[v] < rr_us[best]) best = v;
                C.shapes.rr[l] = best;
            }
        }
        // the first post-smoothing launch with the coarse-grid correction inside
        // it, against a prolong-add launch and the same launch without it
        double sp_us[2] = {};
        {
            const int nc = (n + 1) / 2;
            const float *uc = C.mg.lv[l - 1].u[0];
            const bool fz = C.shapes.use_fused[l] != 0 && C.mg.npost >= 2;
            for (int sp = 0; sp < 2; ++sp) {
                auto run = [&](int r) {
                    float *a = (r & 1) ? u1 : u0, *b = (r & 1) ? u0 : u1;
                    const float *c = uc;
                    if (sp) {
                        qm::launch_prolong_add<float>(nc, uc, a, s, C.P);
                        c = nullptr;
                    }
                    if (fz) {
                        qm::launch_rbgs2_shape<float>(n, h, f, a, b, c, C.shapes.fused[l], s, C.P);
                    } else {
                        qm::launch_rbgs_shape<float>(n, h, f, a, b, c ? C.shapes.corr[l] : C.shapes.single[l], s, C.P, c);
                    }
                };
                run(0);
                std::vector<float> t;
                for (int r = 0; r < reps; ++r) {
                    (void)hipEventRecord(e0, s);
                    run(r);
                    (void)hipEventRecord(e1, s);
                    if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    t.push_back(ms);
                }
                std::sort(t.begin(), t.end());
                sp_us[sp] = 1e3 * t[t.size() / 2];
            }
            C.shapes.split[l] = sp_us[1] < sp_us[0] ? 1 : 0;
        }
        char buf[400];
        std::snprintf(buf, sizeof buf,
                      "%s{\"n\": %d, \"single\": [%d, %d, %.2f], \"corr\": [%d, %d, %.2f], \"fused\": [%d, %d, %.2f], "
                      "\"use_fused\": %d, \"rr\": [%d",
                      first ? "" : ", ", n, C.shapes.single[l].variant, C.shapes.single[l].kchunk, best[0],
                      C.shapes.corr[l].variant, C.shapes.corr[l].kchunk, best_corr, C.shapes.fused[l].variant,
                      C.shapes.fused[l].kchunk, best[1], C.shapes.use_fused[l], C.shapes.rr[l]);
        js += buf;
        for (int v = 0; v < qm::kRrVariants; ++v) {
            std::snprintf(buf, sizeof buf, ", %.2f", rr_us[v]);
            js += buf;
        }
        std::snprintf(buf, sizeof buf, "], \"split_prolong\": [%d, %.2f, %.2f]}", C.shapes.split[l], sp_us[0], sp_us[1]);
        js += buf;
        first = false;
    }
    js += "]";
    C.tune_json = js;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return hipGetLastError();
}

void release(qumond_batch *B)
{
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    for (auto &cp : B->cls) {
        cp->mg.release();
        if (cp->join) (void)hipEventDestroy(cp->join);
        if (cp->s) (void)hipStreamDestroy(cp->s);
    }
    for (void *p : B->owned) (void)hipFree(p);
    for (void *p : B->owned_host) (void)hipHostFree(p);
    if (B->fork) (void)hipEventDestroy(B->fork);
    if (B->ev_in) (void)hipEventDestroy(B->ev_in);
    if (B->main) (void)hipStreamDestroy(B->main);
}

}  // namespace

extern "C" {

void qumond_batch_default_config(qumond_batch_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->nprob = 1;
    cfg->box_side = 120.0;
    cfg->G = 4.300917270e-6;
    cfg->a0 = 3600.0;
    cfg->npre = 2;
    cfg->npost = 2;
    cfg->ncycle_fmg = 2;
    cfg->refine_iters = 4;
    cfg->max_extra = 20;
    cfg->tol_rel = 1e-6;
    cfg->gather_frac = 0.2;
    cfg->naz = 16;
    cfg->autotune = 0;
    cfg->nu_n = 1.0;
}

qumond_status qumond_batch_validate(const qumond_batch_config *c, const int32_t *n_per_problem, const double *R,
                                    int32_t nR)
{
    if (!c) return bfail(QUMOND_ERR_INVALID, "config is NULL");
    if (c->nprob < 1 || c->nprob > QUMOND_BATCH_MAX) return bfail(QUMOND_ERR_INVALID, "nprob must be in 1..1024");
    if (!n_per_problem) return bfail(QUMOND_ERR_INVALID, "n_per_problem is NULL");
    if (!(c->box_side > 0.0) || !std::isfinite(c->box_side))
        return bfail(QUMOND_ERR_INVALID, "box_side must be finite and positive");
    if (!(c->G > 0.0) || !std::isfinite(c->G)) return bfail(QUMOND_ERR_INVALID, "G must be finite and positive");
    if (!(c->a0 >= 0.0) || !std::isfinite(c->a0)) return bfail(QUMOND_ERR_INVALID, "a0 must be finite and >= 0");
    if (c->npre < 0 || c->npre > 8 || c->npost < 0 || c->npost > 8 || c->npre + c->npost < 1)
        return bfail(QUMOND_ERR_INVALID, "npre, npost must be in 0..8 with npre + npost >= 1");
    if (c->ncycle_fmg < 1 || c->ncycle_fmg > 64) return bfail(QUMOND_ERR_INVALID, "ncycle_fmg must be in 1..64");
    if (c->refine_iters < 0 || c->refine_iters > 64) return bfail(QUMOND_ERR_INVALID, "refine_iters must be in 0..64");
    if (c->max_extra < 0 || c->max_extra > 1000) return bfail(QUMOND_ERR_INVALID, "max_extra must be in 0..1000");
    if (!(c->tol_rel >= 0.0) || !std::isfinite(c->tol_rel)) return bfail(QUMOND_ERR_INVALID, "tol_rel must be >= 0");
    if (!(c->gather_frac > 0.0 && c->gather_frac < 0.5))
        return bfail(QUMOND_ERR_INVALID, "gather_frac must be in (0, 0.5)");
    if (c->naz < 1 || c->naz > 1024) return bfail(QUMOND_ERR_INVALID, "naz must be in 1..1024");
    if (c->autotune != 0 && c->autotune != 1) return bfail(QUMOND_ERR_INVALID, "autotune must be 0 or 1");
    if (!(c->nu_n >= 1.0 && c->nu_n <= 10.0)) return bfail(QUMOND_ERR_INVALID, "nu_n must be in [1, 10]");
    if (nR < 1 || nR > 4096 || !R) return bfail(QUMOND_ERR_INVALID, "need 1 <= nR <= 4096 radii");
    for (int i = 0; i < nR; ++i)
        if (!(R[i] >= 0.0) || !std::isfinite(R[i])) return bfail(QUMOND_ERR_INVALID, "radii must be finite and >= 0");
    std::vector<int> count(11, 0);
    for (int p = 0; p < c->nprob; ++p) {
        if (!good_batch_n(n_per_problem[p]))
            return bfail(QUMOND_ERR_INVALID, "each n must be 2^J + 1 with 17 <= n <= 1025");
        ++count[qm::log2_exact(n_per_problem[p] - 1)];
    }
    // a launch's z blocks (about (n+1)/2 per problem) must fit the 65535 limit
    for (int J = 4; J <= 10; ++J)
        if (count[J] && (size_t)count[J] * (((1 << J) + 2) / 2) > 65535)
            return bfail(QUMOND_ERR_INVALID, "too many problems of one grid size for one launch");
    return QUMOND_OK;
}

qumond_status qumond_batch_create(const qumond_batch_config *cfg, const int32_t *n_per_problem, const double *R,
                                  int32_t nR, void *stream, qumond_batch **out)
{
    if (!out) return bfail(QUMOND_ERR_INVALID, "out is NULL");
    *out = nullptr;
    qumond_status st = qumond_batch_validate(cfg, n_per_problem, R, nR);
    if (st != QUMOND_OK) return st;
    qumond_batch *B = new (std::nothrow) qumond_batch();
    if (!B) return bfail(QUMOND_ERR_OOM, "qumond_batch_create: host allocation");
    B->cfg = *cfg;
    B->user = (hipStream_t)stream;
    B->nR = nR;
    const int np = cfg->nprob, K = cfg->refine_iters;
    B->n_of.assign(n_per_problem, n_per_problem + np);
    B->cls_of.assign(np, -1);
    B->slot_of.assign(np, -1);
    B->has_particles.assign(np, 0);
    // classes in increasing n, slots in problem order
    for (int J = 4; J <= 10; ++J) {
        const int n = (1 << J) + 1;
        std::unique_ptr<Class> C(new Class());
        for (int p = 0; p < np; ++p)
            if (n_per_problem[p] == n) {
                B->cls_of[p] = (int)B->cls.size();
                B->slot_of[p] = (int)C->ids.size();
                C->ids.push_back(p);
            }
        if (C->ids.empty()) continue;
        C->n = n;
        C->J = J;
        C->P = (int)C->ids.size();
        C->N = (size_t)n * n * n;
        C->h = cfg->box_side / (double)(n - 1);
        B->cls.push_back(std::move(C));
    }
    hipError_t e;
#define BCHK(x)                                                    \
    if ((e = (x)) != hipSuccess) {                                 \
        st = bhip(e, "qumond_batch_create");                       \
        release(B);                                                \
        delete B;                                                  \
        return st;                                                 \
    }
    BCHK(hipStreamCreateWithFlags(&B->main, hipStreamNonBlocking));
    BCHK(hipEventCreateWithFlags(&B->fork, hipEventDisableTiming));
    BCHK(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
    BCHK(B->alloc((void **)&B->R, (size_t)nR * sizeof(double)));
    BCHK(hipMemcpy(B->R, R, (size_t)nR * sizeof(double), hipMemcpyHostToDevice));
    B->nu.n = cfg->nu_n;
    if (cfg->nu_n != 1.0) {
        std::vector<double> tab(2 * (size_t)qm::kNuTab);
        qm::build_nu_table(cfg->nu_n, tab.data());
        double *d = nullptr;
        BCHK(B->alloc((void **)&d, tab.size() * sizeof(double)));
        BCHK(hipMemcpy(d, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
        B->nu.tab = d;
    }
    for (auto &cp : B->cls) {
        Class &C = *cp;
        const size_t PN = (size_t)C.P * C.N;
        BCHK(hipStreamCreateWithFlags(&C.s, hipStreamNonBlocking));
        BCHK(hipEventCreateWithFlags(&C.join, hipEventDisableTiming));
        BCHK(B->alloc((void **)&C.prob, (size_t)C.P * sizeof(qm::BatchProblem)));
        BCHK(B->alloc_host((void **)&C.hprob, (size_t)C.P * sizeof(qm::BatchProblem)));
        std::memset(C.hprob, 0, (size_t)C.P * sizeof(qm::BatchProblem));
        BCHK(B->alloc((void **)&C.f, PN * sizeof(double)));
        BCHK(B->alloc((void **)&C.phin, PN * sizeof(double)));
        BCHK(B->alloc((void **)&C.S, PN * sizeof(double)));
        BCHK(B->alloc((void **)&C.phi, PN * sizeof(double)));
        C.q = (long long *)C.S;
        BCHK(B->alloc((void **)&C.a[0], PN * sizeof(float)));
        BCHK(B->alloc((void **)&C.a[1], PN * sizeof(float)));
        BCHK(B->alloc((void **)&C.r, PN * sizeof(float)));
        BCHK(C.mg.init(C.n, cfg->npre, cfg->npost, C.s, C.P));
        BCHK(B->alloc((void **)&C.partial, (size_t)C.P * 3 * qm::kNormBlocks * sizeof(double)));
        const size_t nh = (size_t)2 * (K + 1) * C.P * 3;
        BCHK(B->alloc((void **)&C.hist, nh * sizeof(double)));
        BCHK(B->alloc_host((void **)&C.hhist, nh * sizeof(double)));
        BCHK(B->alloc((void **)&C.sc, (size_t)C.P * 4 * sizeof(double)));
        BCHK(B->alloc((void **)&C.dep, qm::deposit_batch_scratch_bytes(C.P)));
        BCHK(B->alloc((void **)&C.inside, (size_t)C.P * sizeof(unsigned long long)));
        BCHK(B->alloc_host((void **)&C.hinside, (size_t)C.P * sizeof(unsigned long long)));
        BCHK(B->alloc((void **)&C.vc2[0], (size_t)C.P * nR * sizeof(double)));
        BCHK(B->alloc((void **)&C.vc2[1], (size_t)C.P * nR * sizeof(double)));
        BCHK(B->alloc((void **)&C.norms1, 3 * sizeof(double)));
        BCHK(B->alloc((void **)&C.sc1, 2 * sizeof(double)));
        BCHK(B->alloc_host((void **)&C.hnorms1, 3 * sizeof(double)));
        // library-wide FP32 shapes until the autotuner replaces them
        for (int l = 0; l <= 10 && l <= C.J; ++l) {
            const int nl = (1 << l) + 1;
            C.shapes.single[l] = qm::rbgs_shape<float>(nl < 5 ? 5 : nl);
            C.shapes.corr[l] = qm::SmootherShape{-1, 0};   // until tuned: the correcting sweep as the single sweep
            C.shapes.sr[l] = 0;                              // sweep and residual restriction as two launches
            C.shapes.fused[l] = qm::rbgs2_shape<float>(nl < 5 ? 5 : nl);
            C.shapes.use_fused[l] = qm::use_fused<float>(nl < 5 ? 5 : nl);
            C.shapes.rr[l] = qm::rr_variant<float>(nl < 5 ? 5 : nl);
            C.shapes.split[l] = qm::split_prolong<float>(nl < 5 ? 5 : nl);
        }
        C.mg.shapes = &C.shapes;
        // the solver's buffers start defined (a solve reads only what it wrote)
        qm::launch_fill<double>(C.phin, PN, 0.0, C.s);
        qm::launch_fill<double>(C.phi, PN, 0.0, C.s);
        BCHK(hipGetLastError());
        BCHK(hipStreamSynchronize(C.s));
    }
#undef BCHK
    *out = B;
    return QUMOND_OK;
}

qumond_status qumond_batch_destroy(qumond_batch *b)
{
    if (!b) return QUMOND_OK;
    for (auto &cp : b->cls)
        if (cp->s) (void)hipStreamSynchronize(cp->s);
    if (b->main) (void)hipStreamSynchronize(b->main);
    release(b);
    delete b;
    return QUMOND_OK;
}

qumond_status qumond_batch_set_particles(qumond_batch *b, int32_t p, const double *x, const double *y,
                                         const double *z, const double *m, int64_t np, double total_mass)
{
    if (!b) return bfail(QUMOND_ERR_INVALID, "batch is NULL");
    if (p < 0 || p >= b->cfg.nprob) return bfail(QUMOND_ERR_INVALID, "problem index out of range");
    if (np < 0) return bfail(QUMOND_ERR_INVALID, "np must be >= 0");
    if (np > 0 && (!x || !y || !z || !m)) return bfail(QUMOND_ERR_INVALID, "particle arrays must not be NULL");
    if (!(total_mass > 0.0) || !std::isfinite(total_mass))
        return bfail(QUMOND_ERR_INVALID, "total_mass must be finite and positive");
    const int shift = qm_fixed_shift_for(total_mass);
    if (std::ldexp(total_mass, shift) >= 9.2e18) return bfail(QUMOND_ERR_RANGE, "fixed_shift overflows 64 bits");
    Class &C = *b->cls[b->cls_of[p]];
    qm::BatchProblem &P = C.hprob[b->slot_of[p]];
    P.x = x;
    P.y = y;
    P.z = z;
    P.m = m;
    P.np = np;
    P.mass = total_mass;
    P.shift = shift;
    P.scale = std::ldexp(1.0, shift);
    P.pad = 0;
    b->has_particles[p] = 1;
    return QUMOND_OK;
}

qumond_status qumond_batch_run(qumond_batch *b, int32_t use_graph, qumond_batch_problem_info *info)
{
    if (!b) return bfail(QUMOND_ERR_INVALID, "batch is NULL");
    if (use_graph != 0 && use_graph != 1) return bfail(QUMOND_ERR_INVALID, "use_graph must be 0 or 1");
    for (int p = 0; p < b->cfg.nprob; ++p)
        if (!b->has_particles[p]) return bfail(QUMOND_ERR_STATE, "every problem needs particles before a run");
    hipError_t e;
    // order after the caller's work, then the input tables (outside the graph)
    if ((e = hipEventRecord(b->ev_in, b->user)) != hipSuccess || (e = hipStreamWaitEvent(b->main, b->ev_in, 0)) != hipSuccess)
        return bhip(e, "qumond_batch_run: order");
    for (auto &cp : b->cls)
        if ((e = hipMemcpyAsync(cp->prob, cp->hprob, (size_t)cp->P * sizeof(qm::BatchProblem), hipMemcpyHostToDevice,
                                b->main)) != hipSuccess)
            return bhip(e, "qumond_batch_run: inputs");
    if (b->cfg.autotune && !b->tuned) {
        if ((e = hipStreamSynchronize(b->main)) != hipSuccess) return bhip(e, "qumond_batch_run: sync");
        for (auto &cp : b->cls)
            if ((e = tune_class(b, *cp, 3)) != hipSuccess) return bhip(e, "qumond_batch_run: autotune");
        b->tuned = true;
    }
    if (use_graph) {
        if (!b->exec) {
            if ((e = hipStreamSynchronize(b->main)) != hipSuccess) return bhip(e, "qumond_batch_run: sync");
            if ((e = hipStreamBeginCapture(b->main, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return bhip(e, "qumond_batch_run: begin capture");
            hipError_t ee = enqueue_all(b);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(b->main, &g);
            if (ee != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return bhip(ee, "qumond_batch_run: capture");
            }
            if (e != hipSuccess) return bhip(e, "qumond_batch_run: end capture");
            b->graph = g;
            if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
                b->exec = nullptr;
                return bhip(e, "qumond_batch_run: instantiate");
            }
            size_t nn = 0;
            (void)hipGraphGetNodes(g, nullptr, &nn);
            b->graph_nodes = nn;
            // the input tables again: synchronising above drained the earlier copy
            for (auto &cp : b->cls)
                if ((e = hipMemcpyAsync(cp->prob, cp->hprob, (size_t)cp->P * sizeof(qm::BatchProblem),
                                        hipMemcpyHostToDevice, b->main)) != hipSuccess)
                    return bhip(e, "qumond_batch_run: inputs");
        }
        if ((e = hipGraphLaunch(b->exec, b->main)) != hipSuccess) return bhip(e, "qumond_batch_run: graph launch");
    } else {
        if ((e = enqueue_all(b)) != hipSuccess) return bhip(e, "qumond_batch_run: launch");
    }
    if ((e = hipStreamSynchronize(b->main)) != hipSuccess) return bhip(e, "qumond_batch_run: sync");
    // tail check
    const int K = K_of(b);
    const double tol = b->cfg.tol_rel;
    bool all_ok = true;
    for (auto &cp : b->cls) {
        Class &C = *cp;
        for (int sl = 0; sl < C.P; ++sl) {
            const int p = C.ids[sl];
            double rn = relres_of(C.hhist + (((size_t)0 * (K + 1) + K) * C.P + sl) * 3);
            double rm = relres_of(C.hhist + (((size_t)1 * (K + 1) + K) * C.P + sl) * 3);
            int sn = 0, sm = 0, redone = 0;
            if (rn > tol && b->cfg.max_extra > 0) {
                if ((e = tail_steps(b, C, false, sl, hist_slot(b, C, false, K, sl), sn, rn)) != hipSuccess)
                    return bhip(e, "qumond_batch_run: tail");
                if (sn > 0) {
                    // the QUMOND part depends on Phi_N: redo it for this problem
                    qm::Multigrid<float> mg = single_view(C);
                    qm::launch_mond_source(C.n, C.h, b->cfg.a0, C.phin + (size_t)sl * C.N, C.S + (size_t)sl * C.N, C.s, 1,
                                           b->cfg.nu_n);
                    enqueue_solve(b, C, mg, true, sl, 1, K, C.s);
                    enqueue_curves(b, C, sl, 1, -1, C.s);
                    double *hm = C.hhist + (((size_t)1 * (K + 1) + K) * C.P + sl) * 3;
                    if ((e = hipMemcpyAsync(hm, hist_slot(b, C, true, K, sl), 3 * sizeof(double), hipMemcpyDeviceToHost,
                                            C.s)) != hipSuccess ||
                        (e = hipStreamSynchronize(C.s)) != hipSuccess)
                        return bhip(e, "qumond_batch_run: redo");
                    rm = relres_of(hm);
                    redone = 1;
                }
            }
            if (rm > tol && b->cfg.max_extra > 0) {
                if ((e = tail_steps(b, C, true, sl, hist_slot(b, C, true, K, sl), sm, rm)) != hipSuccess)
                    return bhip(e, "qumond_batch_run: tail");
                if (sm > 0) enqueue_curves(b, C, sl, 1, 1, C.s);
            }
            if (sn > 0 || sm > 0)
                if ((e = hipStreamSynchronize(C.s)) != hipSuccess) return bhip(e, "qumond_batch_run: tail sync");
            const bool ok = rn <= tol && rm <= tol;
            all_ok = all_ok && ok;
            if (info) {
                qumond_batch_problem_info &I = info[p];
                I.relres_newton = rn;
                I.relres_mond = rm;
                I.steps_newton = K + sn;
                I.steps_mond = K + sm;
                I.converged = ok ? 1 : 0;
                I.redone = redone;
                I.n_inside = (int64_t)C.hinside[sl];
            }
        }
    }
    // later work on the caller's stream sees the results
    if ((e = hipEventRecord(b->fork, b->main)) != hipSuccess || (e = hipStreamWaitEvent(b->user, b->fork, 0)) != hipSuccess)
        return bhip(e, "qumond_batch_run: join");
    if ((e = hipGetLastError()) != hipSuccess) return bhip(e, "qumond_batch_run");
    if (!all_ok) return bfail(QUMOND_ERR_NOT_CONVERGED, "a problem stayed above tol_rel after max_extra steps");
    return QUMOND_OK;
}

qumond_status qumond_batch_rotation_curves(qumond_batch *b, int32_t mond, double *vc2)
{
    if (!b) return bfail(QUMOND_ERR_INVALID, "batch is NULL");
    if (mond != 0 && mond != 1) return bfail(QUMOND_ERR_INVALID, "mond must be 0 or 1");
    if (!vc2) return bfail(QUMOND_ERR_INVALID, "vc2 is NULL");
    hipError_t e;
    for (auto &cp : b->cls)
        for (int sl = 0; sl < cp->P; ++sl)
            if ((e = hipMemcpyAsync(vc2 + (size_t)cp->ids[sl] * b->nR, cp->vc2[mond] + (size_t)sl * b->nR,
                                    (size_t)b->nR * sizeof(double), hipMemcpyDeviceToDevice, b->user)) != hipSuccess)
                return bhip(e, "qumond_batch_rotation_curves");
    return QUMOND_OK;
}

qumond_status qumond_batch_get_field(qumond_batch *b, int32_t p, int32_t field, double *dst)
{
    if (!b) return bfail(QUMOND_ERR_INVALID, "batch is NULL");
    if (p < 0 || p >= b->cfg.nprob) return bfail(QUMOND_ERR_INVALID, "problem index out of range");
    if (!dst) return bfail(QUMOND_ERR_INVALID, "dst is NULL");
    Class &C = *b->cls[b->cls_of[p]];
    const double *src = nullptr;
    switch (field) {
    case QUMOND_FIELD_RHS: src = C.f; break;
    case QUMOND_FIELD_PHI_N: src = C.phin; break;
    case QUMOND_FIELD_SOURCE: src = C.S; break;
    case QUMOND_FIELD_PHI: src = C.phi; break;
    default: return bfail(QUMOND_ERR_INVALID, "fields: RHS, PHI_N, SOURCE, PHI");
    }
    hipError_t e = hipMemcpyAsync(dst, src + (size_t)b->slot_of[p] * C.N, C.N * sizeof(double), hipMemcpyDeviceToDevice,
                                  b->user);
    if (e != hipSuccess) return bhip(e, "qumond_batch_get_field");
    return QUMOND_OK;
}

qumond_status qumond_batch_describe(qumond_batch *b, char *buf, int64_t cap)
{
    if (!b || !buf || cap < 1) return bfail(QUMOND_ERR_INVALID, "bad argument");
    std::string js = "{\"classes\": [";
    for (size_t c = 0; c < b->cls.size(); ++c) {
        const Class &C = *b->cls[c];
        char t[128];
        std::snprintf(t, sizeof t, "%s{\"n\": %d, \"problems\": %d, \"shapes\": ", c ? ", " : "", C.n, C.P);
        js += t;
        js += C.tune_json.empty() ? "null" : C.tune_json;
        js += "}";
    }
    char t[160];
    std::snprintf(t, sizeof t, "], \"graph_nodes\": %zu, \"tuned\": %d, \"device_bytes\": %lld}", b->graph_nodes,
                  b->tuned ? 1 : 0, (long long)qumond_batch_device_bytes(b));
    js += t;
    if ((int64_t)js.size() + 1 > cap) return bfail(QUMOND_ERR_RANGE, "buffer too small");
    std::memcpy(buf, js.c_str(), js.size() + 1);
    return QUMOND_OK;
}

int64_t qumond_batch_device_bytes(const qumond_batch *b)
{
    if (!b) return 0;
    int64_t t = b->bytes;
    for (auto &cp : b->cls) t += (int64_t)cp->mg.bytes;
    return t;
}

}  // extern "C"
