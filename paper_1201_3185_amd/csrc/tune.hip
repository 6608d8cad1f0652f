// Smoother launch-shape autotuner and its persisted table (qumond_tune.h).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qumond_tune.h"
#include "common.h"
#include "mg.h"

void qm_set_last_error(const char *msg);

namespace {

qumond_status tfail(const std::string &m)
{
    qm_set_last_error(m.c_str());
    return QUMOND_ERR_INVALID;
}

bool good_n(int n) { return n >= 5 && n <= 1025 && qm::log2_exact(n - 1) >= 2; }

const int kChunks[] = {2, 4, 8, 16, 32, 64, 128, 256, 0};

// Time every single-sweep shape (fused: every two-sweep shape; corr: every
// single-sweep shape applying a coarse-grid correction) on a level of n
// points and install the fastest.
template <typename T>
qumond_status tune_one(int n, int reps, hipStream_t s, double &best_us, bool fused, bool corr = false)
{
    const size_t N = (size_t)n * n * n;
    const int nc = (n + 1) / 2;
    const size_t Nc = (size_t)nc * nc * nc;
    T *f = nullptr, *u0 = nullptr, *u1 = nullptr, *uc = nullptr;
    if (hipMalloc((void **)&f, N * sizeof(T)) != hipSuccess || hipMalloc((void **)&u0, N * sizeof(T)) != hipSuccess ||
        hipMalloc((void **)&u1, N * sizeof(T)) != hipSuccess ||
        (corr && hipMalloc((void **)&uc, Nc * sizeof(T)) != hipSuccess)) {
        (void)hipFree(f);
        (void)hipFree(u0);
        (void)hipFree(u1);
        qm_set_last_error("qumond_autotune: allocation failed");
        return QUMOND_ERR_OOM;
    }
    qm::launch_fill<T>(f, N, T(1), s);
    qm::launch_fill<T>(u0, N, T(0.5), s);
    qm::launch_fill<T>(u1, N, T(0.5), s);
    if (corr) qm::launch_fill<T>(uc, Nc, T(0.001), s);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    qm::SmootherShape &slot = fused ? qm::rbgs2_shape<T>(n) : (corr ? qm::rbgs_corr_shape<T>(n) : qm::rbgs_shape<T>(n));
    qm::SmootherShape best = corr ? qm::rbgs_corr_effective<T>(n) : slot;
    best_us = 1e30;
    const double h = 1.0 / (n - 1);
    auto run = [&](const T *a, T *b, const qm::SmootherShape &sh) {
        if (fused) {
            slot = sh;
            qm::launch_rbgs2<T>(n, h, f, a, b, nullptr, s);
        } else {
            qm::launch_rbgs_shape<T>(n, h, f, a, b, sh, s, 1, uc);
        }
    };
    const int nvar = fused ? qm::kFusedVariants : qm::kSmootherVariants;
    for (int v = 0; v < nvar; ++v)
        for (int kc : kChunks) {
            if (kc != 0 && kc >= n - 2) continue;
            if (qm::takes_no_chunk(v, fused) && kc != 0) continue;   // bricks and whole-column marches
            if (fused && kc != 0 && kc < 4) continue;   // the two-sweep march needs 4-plane chunks
            const qm::SmootherShape sh{v, kc};
            std::vector<float> t;
            run(u0, u1, sh);   // warm-up
            for (int r = 0; r < reps; ++r) {
                (void)hipEventRecord(e0, s);
                run((r & 1) ? u1 : u0, (r & 1) ? u0 : u1, sh);
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                t.push_back(ms);
            }
            std::sort(t.begin(), t.end());
            const double us = 1e3 * t[t.size() / 2];
            if (us < best_us) {
                best_us = us;
                best = sh;
            }
        }
    slot = best;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(f);
    (void)hipFree(u0);
    (void)hipFree(u1);
    if (uc) (void)hipFree(uc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        qm_set_last_error(hipGetErrorString(e));
        return QUMOND_ERR_HIP;
    }
    return QUMOND_OK;
}

// Time both residual-restriction kernels on a fine level of n points and
// install the faster one.
template <typename T>
qumond_status tune_rr(int n, int reps, hipStream_t s, double us[qm::kRrVariants])
{
    const int nc = (n + 1) / 2;
    const size_t N = (size_t)n * n * n, Nc = (size_t)nc * nc * nc;
    T *f = nullptr, *u = nullptr, *fc = nullptr, *c0 = nullptr, *c1 = nullptr;
    if (hipMalloc((void **)&f, N * sizeof(T)) != hipSuccess || hipMalloc((void **)&u, N * sizeof(T)) != hipSuccess ||
        hipMalloc((void **)&fc, Nc * sizeof(T)) != hipSuccess || hipMalloc((void **)&c0, Nc * sizeof(T)) != hipSuccess ||
        hipMalloc((void **)&c1, Nc * sizeof(T)) != hipSuccess) {
        (void)hipFree(f);
        (void)hipFree(u);
        (void)hipFree(fc);
        (void)hipFree(c0);
        (void)hipFree(c1);
        qm_set_last_error("qumond_autotune: allocation failed");
        return QUMOND_ERR_OOM;
    }
    qm::launch_fill<T>(f, N, T(1), s);
    qm::launch_fill<T>(u, N, T(0.5), s);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const double h = 1.0 / (n - 1);
    for (int v = 0; v < qm::kRrVariants; ++v) {
        qm::launch_residual_restrict_variant<T>(n, h, f, u, fc, c0, c1, v, s);
        std::vector<float> t;
        for (int r = 0; r < reps; ++r) {
            (void)hipEventRecord(e0, s);
            qm::launch_residual_restrict_variant<T>(n, h, f, u, fc, c0, c1, v, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t.push_back(ms);
        }
        std::sort(t.begin(), t.end());
        us[v] = 1e3 * t[t.size() / 2];
    }
    int best = 0;
    for (int v = 1; v < qm::kRrVariants; ++v)
        if (us[v] < us[best]) best = v;
    qm::rr_variant<T>(n) = best;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(f);
    (void)hipFree(u);
    (void)hipFree(fc);
    (void)hipFree(c0);
    (void)hipFree(c1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        qm_set_last_error(hipGetErrorString(e));
        return QUMOND_ERR_HIP;
    }
    return QUMOND_OK;
}

// Time the last pre-smoothing sweep of a level of n points followed by its
// residual restriction (us[0], the level's own sweep shape and restriction
// kernel) against the fused sweep-and-restriction launch (us[1]), and install
// the faster.
template <typename T>
qumond_status tune_sweep_restrict(int n, int reps, hipStream_t s, double us[2])
{
    us[0] = us[1] = 0.0;
    if (!qm::rbgs_restrict_fits<T>(n)) return QUMOND_OK;
    const int nc = (n + 1) / 2;
    const size_t N = (size_t)n * n * n, Nc = (size_t)nc * nc * nc;
    T *f = nullptr, *u0 = nullptr, *u1 = nullptr, *fc = nullptr, *c0 = nullptr, *c1 = nullptr;
    if (hipMalloc((void **)&f, N * sizeof(T)) != hipSuccess || hipMalloc((void **)&u0, N * sizeof(T)) != hipSuccess ||
        hipMalloc((void **)&u1, N * sizeof(T)) != hipSuccess || hipMalloc((void **)&fc, Nc * sizeof(T)) != hipSuccess ||
        hipMalloc((void **)&c0, Nc * sizeof(T)) != hipSuccess || hipMalloc((void **)&c1, Nc * sizeof(T)) != hipSuccess) {
        for (T *p : {f, u0, u1, fc, c0, c1}) (void)hipFree(p);
        qm_set_last_error("qumond_autotune: allocation failed");
        return QUMOND_ERR_OOM;
    }
    qm::launch_fill<T>(f, N, T(1), s);
    qm::launch_fill<T>(u0, N, T(0.5), s);
    qm::launch_fill<T>(u1, N, T(0.5), s);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const double h = 1.0 / (n - 1);
    for (int fz = 0; fz < 2; ++fz) {
        auto run = [&](int r) {
            const T *a = (r & 1) ? u1 : u0;
            T *b = (r & 1) ? u0 : u1;
            if (fz) {
                qm::launch_rbgs_restrict<T>(n, h, f, a, b, fc, c0, c1, s);
            } else {
                qm::launch_rbgs<T>(n, h, f, a, b, s);
                qm::launch_residual_restrict<T>(n, h, f, b, fc, c0, c1, s);
            }
        };
        run(0);
        std::vector<float> t;
        for (int r = 0; r < reps; ++r) {
            (void)hipEventRecord(e0, s);
            run(r);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t.push_back(ms);
        }
        std::sort(t.begin(), t.end());
        us[fz] = 1e3 * t[t.size() / 2];
    }
    qm::sweep_restrict<T>(n) = us[1] < us[0] ? 1 : 0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (T *p : {f, u0, u1, fc, c0, c1}) (void)hipFree(p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        qm_set_last_error(hipGetErrorString(e));
        return QUMOND_ERR_HIP;
    }
    return QUMOND_OK;
}

// Time the first post-smoothing launch of a level of n points with the
// coarse-grid correction applied inside it (us[0]) against a prolong-add
// launch followed by the same smoother launch without it (us[1]), in the
// smoother form the tables choose for that level, and install the faster.
template <typename T>
qumond_status tune_split(int n, int reps, hipStream_t s, double us[2])
{
    const int nc = (n + 1) / 2;
    const size_t N = (size_t)n * n * n, Nc = (size_t)nc * nc * nc;
    T *f = nullptr, *u0 = nullptr, *u1 = nullptr, *uc = nullptr;
    if (hipMalloc((void **)&f, N * sizeof(T)) != hipSuccess || hipMalloc((void **)&u0, N * sizeof(T)) != hipSuccess ||
        hipMalloc((void **)&u1, N * sizeof(T)) != hipSuccess || hipMalloc((void **)&uc, Nc * sizeof(T)) != hipSuccess) {
        (void)hipFree(f);
        (void)hipFree(u0);
        (void)hipFree(u1);
        (void)hipFree(uc);
        qm_set_last_error("qumond_autotune: allocation failed");
        return QUMOND_ERR_OOM;
    }
    qm::launch_fill<T>(f, N, T(1), s);
    qm::launch_fill<T>(u0, N, T(0.5), s);
    qm::launch_fill<T>(u1, N, T(0.5), s);
    qm::launch_fill<T>(uc, Nc, T(0.001), s);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const double h = 1.0 / (n - 1);
    const bool fz = qm::use_fused<T>(n) != 0;
    for (int sp = 0; sp < 2; ++sp) {
        auto run = [&](int r) {
            T *a = (r & 1) ? u1 : u0, *b = (r & 1) ? u0 : u1;
            const T *c = uc;
            if (sp) {
                qm::launch_prolong_add<T>(nc, uc, a, s);
                c = nullptr;
            }
            if (fz) {
                qm::launch_rbgs2<T>(n, h, f, a, b, c, s);
            } else {
                qm::launch_rbgs<T>(n, h, f, a, b, s, 1, c);
            }
        };
        run(0);
        std::vector<float> t;
        for (int r = 0; r < reps; ++r) {
            (void)hipEventRecord(e0, s);
            run(r);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t.push_back(ms);
        }
        std::sort(t.begin(), t.end());
        us[sp] = 1e3 * t[t.size() / 2];
    }
    qm::split_prolong<T>(n) = us[1] < us[0] ? 1 : 0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(f);
    (void)hipFree(u0);
    (void)hipFree(u1);
    (void)hipFree(uc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        qm_set_last_error(hipGetErrorString(e));
        return QUMOND_ERR_HIP;
    }
    return QUMOND_OK;
}

}  // namespace

extern "C" {

qumond_status qumond_tune_set(int32_t n, int32_t fp32, int32_t variant, int32_t kchunk)
{
    if (!good_n(n) || variant < 0 || variant >= qm::kSmootherVariants || kchunk < 0)
        return tfail("qumond_tune_set: bad argument");
    qm::SmootherShape sh{variant, kchunk};
    if (fp32) qm::rbgs_shape<float>(n) = sh;
    else qm::rbgs_shape<double>(n) = sh;
    return QUMOND_OK;
}

qumond_status qumond_tune_get(int32_t n, int32_t fp32, int32_t *variant, int32_t *kchunk)
{
    if (!good_n(n) || !variant || !kchunk) return tfail("qumond_tune_get: bad argument");
    const qm::SmootherShape sh = fp32 ? qm::rbgs_shape<float>(n) : qm::rbgs_shape<double>(n);
    *variant = sh.variant;
    *kchunk = sh.kchunk;
    return QUMOND_OK;
}

qumond_status qumond_tune_set_corr(int32_t n, int32_t fp32, int32_t variant, int32_t kchunk)
{
    if (!good_n(n) || variant < -1 || variant >= qm::kSmootherVariants || kchunk < 0)
        return tfail("qumond_tune_set_corr: bad argument");
    const qm::SmootherShape sh{variant, variant < 0 ? 0 : kchunk};
    if (fp32) qm::rbgs_corr_shape<float>(n) = sh;
    else qm::rbgs_corr_shape<double>(n) = sh;
    return QUMOND_OK;
}

qumond_status qumond_tune_get_corr(int32_t n, int32_t fp32, int32_t *variant, int32_t *kchunk)
{
    if (!good_n(n) || !variant || !kchunk) return tfail("qumond_tune_get_corr: bad argument");
    const qm::SmootherShape sh = fp32 ? qm::rbgs_corr_shape<float>(n) : qm::rbgs_corr_shape<double>(n);
    *variant = sh.variant;
    *kchunk = sh.kchunk;
    return QUMOND_OK;
}

qumond_status qumond_tune_set_fused(int32_t n, int32_t fp32, int32_t variant, int32_t kchunk)
{
    if (!good_n(n) || variant < 0 || variant >= qm::kFusedVariants || kchunk < 0)
        return tfail("qumond_tune_set_fused: bad argument");
    qm::SmootherShape sh{variant, kchunk};
    if (fp32) qm::rbgs2_shape<float>(n) = sh;
    else qm::rbgs2_shape<double>(n) = sh;
    return QUMOND_OK;
}

qumond_status qumond_tune_get_fused(int32_t n, int32_t fp32, int32_t *variant, int32_t *kchunk)
{
    if (!good_n(n) || !variant || !kchunk) return tfail("qumond_tune_get_fused: bad argument");
    const qm::SmootherShape sh = fp32 ? qm::rbgs2_shape<float>(n) : qm::rbgs2_shape<double>(n);
    *variant = sh.variant;
    *kchunk = sh.kchunk;
    return QUMOND_OK;
}

qumond_status qumond_tune_set_rr(int32_t n, int32_t fp32, int32_t variant)
{
    if (!good_n(n) || variant < 0 || variant >= qm::kRrVariants) return tfail("qumond_tune_set_rr: bad argument");
    if (fp32) qm::rr_variant<float>(n) = variant;
    else qm::rr_variant<double>(n) = variant;
    return QUMOND_OK;
}

qumond_status qumond_tune_get_rr(int32_t n, int32_t fp32, int32_t *variant)
{
    if (!good_n(n) || !variant) return tfail("qumond_tune_get_rr: bad argument");
    *variant = fp32 ? qm::rr_variant<float>(n) : qm::rr_variant<double>(n);
    return QUMOND_OK;
}

qumond_status qumond_tune_set_sweep_restrict(int32_t n, int32_t fp32, int32_t fused)
{
    if (!good_n(n) || fused < 0 || fused > 1) return tfail("qumond_tune_set_sweep_restrict: bad argument");
    if (fp32) qm::sweep_restrict<float>(n) = fused;
    else qm::sweep_restrict<double>(n) = fused;
    return QUMOND_OK;
}

qumond_status qumond_tune_get_sweep_restrict(int32_t n, int32_t fp32, int32_t *fused)
{
    if (!good_n(n) || !fused) return tfail("qumond_tune_get_sweep_restrict: bad argument");
    *fused = fp32 ? qm::sweep_restrict<float>(n) : qm::sweep_restrict<double>(n);
    return QUMOND_OK;
}

qumond_status qumond_tune_set_split(int32_t n, int32_t fp32, int32_t split)
{
    if (!good_n(n) || split < 0 || split > 1) return tfail("qumond_tune_set_split: bad argument");
    if (fp32) qm::split_prolong<float>(n) = split;
    else qm::split_prolong<double>(n) = split;
    return QUMOND_OK;
}

qumond_status qumond_tune_get_split(int32_t n, int32_t fp32, int32_t *split)
{
    if (!good_n(n) || !split) return tfail("qumond_tune_get_split: bad argument");
    *split = fp32 ? qm::split_prolong<float>(n) : qm::split_prolong<double>(n);
    return QUMOND_OK;
}

qumond_status qumond_k_rbgs_sweep_shape(int32_t n, double h, const double *f, const double *u_in, double *u_out,
                                        int32_t variant, int32_t kchunk, const double *uc, void *stream)
{
    if (!good_n(n) || !(h > 0.0) || !f || !u_out || u_in == u_out || variant < 0 ||
        variant >= qm::kSmootherVariants || kchunk < 0)
        return tfail("qumond_k_rbgs_sweep_shape: bad argument");
    qm::launch_rbgs_shape<double>(n, h, f, u_in, u_out, qm::SmootherShape{variant, kchunk}, (hipStream_t)stream, 1, uc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        qm_set_last_error(hipGetErrorString(e));
        return QUMOND_ERR_HIP;
    }
    return QUMOND_OK;
}

qumond_status qumond_k_rbgs_sweep_stacked(int32_t n, int32_t nb, double h, const double *f, const double *u_in,
                                          double *u_out, int32_t variant, int32_t kchunk, void *stream)
{
    if (!good_n(n) || nb < 1 || nb > 4096 || !(h > 0.0) || !f || !u_out || u_in == u_out || variant < 0 ||
        variant >= qm::kSmootherVariants || kchunk < 0)
        return tfail("qumond_k_rbgs_sweep_stacked: bad argument");
    qm::launch_rbgs_shape<double>(n, h, f, u_in, u_out, qm::SmootherShape{variant, kchunk}, (hipStream_t)stream, nb,
                                  nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        qm_set_last_error(hipGetErrorString(e));
        return QUMOND_ERR_HIP;
    }
    return QUMOND_OK;
}

qumond_status qumond_autotune(int32_t n_max, int32_t both, int32_t reps, const char *json_path, double *best_us,
                              void *stream)
{
    if (!good_n(n_max) || reps < 1 || reps > 1000) return tfail("qumond_autotune: bad argument");
    hipStream_t s = (hipStream_t)stream;
    std::string js = "{\"smoother\": [";
    bool first = true;
    for (int J = 5; (1 << J) + 1 <= n_max; ++J) {
        const int n = (1 << J) + 1;
        for (int prec = 0; prec < (both ? 2 : 1); ++prec) {
            double us_pair[2] = {0.0, 0.0};
            for (int fz = 0; fz < 2; ++fz) {
                double us = 0.0;
                qumond_status st =
                    prec ? tune_one<float>(n, reps, s, us, fz != 0) : tune_one<double>(n, reps, s, us, fz != 0);
                if (st != QUMOND_OK) return st;
                if (!prec && fz && best_us) best_us[J] = us;
                const qm::SmootherShape sh = fz ? (prec ? qm::rbgs2_shape<float>(n) : qm::rbgs2_shape<double>(n))
                                                : (prec ? qm::rbgs_shape<float>(n) : qm::rbgs_shape<double>(n));
                char buf[200];
                std::snprintf(buf, sizeof buf,
                              "%s{\"n\": %d, \"fp32\": %d, \"fused\": %d, \"variant\": %d, \"kchunk\": %d, \"us\": %.3f}",
                              first ? "" : ", ", n, prec, fz, sh.variant, sh.kchunk, us);
                js += buf;
                first = false;
                us_pair[fz] = us;
            }
            {   // the single sweep that applies the coarse-grid correction
                double us = 0.0;
                qumond_status st = prec ? tune_one<float>(n, reps, s, us, false, true)
                                        : tune_one<double>(n, reps, s, us, false, true);
                if (st != QUMOND_OK) return st;
                const qm::SmootherShape sh = prec ? qm::rbgs_corr_shape<float>(n) : qm::rbgs_corr_shape<double>(n);
                char buf[200];
                std::snprintf(buf, sizeof buf,
                              ", {\"n\": %d, \"fp32\": %d, \"corr_variant\": %d, \"corr_kchunk\": %d, \"us\": %.3f}", n,
                              prec, sh.variant, sh.kchunk, us);
                js += buf;
            }
            // fused launch (two sweeps) against two single sweeps
            const int fuse = us_pair[1] < 2.0 * us_pair[0] ? 1 : 0;
            if (prec) qm::use_fused<float>(n) = fuse;
            else qm::use_fused<double>(n) = fuse;
            double rr_us[qm::kRrVariants] = {};
            const qumond_status st = prec ? tune_rr<float>(n, reps, s, rr_us) : tune_rr<double>(n, reps, s, rr_us);
            if (st != QUMOND_OK) return st;
            const int rrv = prec ? qm::rr_variant<float>(n) : qm::rr_variant<double>(n);
            double sp_us[2] = {};
            const qumond_status st2 = prec ? tune_split<float>(n, reps, s, sp_us) : tune_split<double>(n, reps, s, sp_us);
            if (st2 != QUMOND_OK) return st2;
            const int spv = prec ? qm::split_prolong<float>(n) : qm::split_prolong<double>(n);
            double sr_us[2] = {};
            const qumond_status st3 =
                prec ? tune_sweep_restrict<float>(n, reps, s, sr_us) : tune_sweep_restrict<double>(n, reps, s, sr_us);
            if (st3 != QUMOND_OK) return st3;
            const int srv = prec ? qm::sweep_restrict<float>(n) : qm::sweep_restrict<double>(n);
            char buf[400];
            std::snprintf(buf, sizeof buf, ", {\"n\": %d, \"fp32\": %d, \"use_fused\": %d}, {\"n\": %d, \"fp32\": %d, \"rr\": %d, \"rr_us\": [",
                          n, prec, fuse, n, prec, rrv);
            js += buf;
            for (int v = 0; v < qm::kRrVariants; ++v) {
                std::snprintf(buf, sizeof buf, "%s%.3f", v ? ", " : "", rr_us[v]);
                js += buf;
            }
            std::snprintf(buf, sizeof buf, "]}, {\"n\": %d, \"fp32\": %d, \"split_prolong\": %d, \"us\": [%.3f, %.3f]}", n, prec,
                          spv, sp_us[0], sp_us[1]);
            js += buf;
            std::snprintf(buf, sizeof buf, ", {\"n\": %d, \"fp32\": %d, \"sweep_restrict\": %d, \"us\": [%.3f, %.3f]}", n,
                          prec, srv, sr_us[0], sr_us[1]);
            js += buf;
        }
    }
    js += "]}\n";
    if (json_path) {
        FILE *fp = std::fopen(json_path, "w");
        if (!fp) return tfail("qumond_autotune: cannot write the table");
        std::fputs(js.c_str(), fp);
        std::fclose(fp);
    }
    return QUMOND_OK;
}

qumond_status qumond_tune_load(const char *json_path)
{
    if (!json_path) return tfail("qumond_tune_load: path is NULL");
    FILE *fp = std::fopen(json_path, "r");
    if (!fp) return tfail("qumond_tune_load: cannot open the table");
    std::string txt;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, fp)) > 0) txt.append(buf, k);
    std::fclose(fp);
    size_t pos = 0;
    int loaded = 0;
    while ((pos = txt.find("{\"n\":", pos)) != std::string::npos) {
        int n = 0, fp32 = 0, fz = 0, variant = 0, kchunk = 0;
        if (std::sscanf(txt.c_str() + pos, "{\"n\": %d, \"fp32\": %d, \"fused\": %d, \"variant\": %d, \"kchunk\": %d",
                        &n, &fp32, &fz, &variant, &kchunk) == 5) {
            const qumond_status st = fz ? qumond_tune_set_fused(n, fp32, variant, kchunk)
                                        : qumond_tune_set(n, fp32, variant, kchunk);
            if (st != QUMOND_OK) return QUMOND_ERR_INVALID;
            ++loaded;
        }
        ++pos;
    }
    pos = 0;
    while ((pos = txt.find("{\"n\":", pos)) != std::string::npos) {
        int n = 0, fp32 = 0, variant = 0, kchunk = 0;
        if (std::sscanf(txt.c_str() + pos, "{\"n\": %d, \"fp32\": %d, \"corr_variant\": %d, \"corr_kchunk\": %d", &n,
                        &fp32, &variant, &kchunk) == 4) {
            if (qumond_tune_set_corr(n, fp32, variant, kchunk) != QUMOND_OK) return QUMOND_ERR_INVALID;
            ++loaded;
        }
        ++pos;
    }
    pos = 0;
    while ((pos = txt.find("{\"n\":", pos)) != std::string::npos) {
        int n = 0, fp32 = 0, srv = 0;
        if (std::sscanf(txt.c_str() + pos, "{\"n\": %d, \"fp32\": %d, \"sweep_restrict\": %d", &n, &fp32, &srv) == 3) {
            if (qumond_tune_set_sweep_restrict(n, fp32, srv) != QUMOND_OK) return QUMOND_ERR_INVALID;
            ++loaded;
        }
        ++pos;
    }
    pos = 0;
    while ((pos = txt.find("{\"n\":", pos)) != std::string::npos) {
        int n = 0, fp32 = 0, fuse = 0;
        if (std::sscanf(txt.c_str() + pos, "{\"n\": %d, \"fp32\": %d, \"use_fused\": %d", &n, &fp32, &fuse) == 3 &&
            good_n(n)) {
            if (fp32) qm::use_fused<float>(n) = fuse ? 1 : 0;
            else qm::use_fused<double>(n) = fuse ? 1 : 0;
        }
        ++pos;
    }
    pos = 0;
    while ((pos = txt.find("{\"n\":", pos)) != std::string::npos) {
        int n = 0, fp32 = 0, rrv = 0;
        if (std::sscanf(txt.c_str() + pos, "{\"n\": %d, \"fp32\": %d, \"rr\": %d", &n, &fp32, &rrv) == 3 && good_n(n)) {
            const int v = rrv >= 0 && rrv < qm::kRrVariants ? rrv : 0;
            if (fp32) qm::rr_variant<float>(n) = v;
            else qm::rr_variant<double>(n) = v;
        }
        ++pos;
    }
    pos = 0;
    while ((pos = txt.find("{\"n\":", pos)) != std::string::npos) {
        int n = 0, fp32 = 0, sp = 0;
        if (std::sscanf(txt.c_str() + pos, "{\"n\": %d, \"fp32\": %d, \"split_prolong\": %d", &n, &fp32, &sp) == 3 &&
            good_n(n)) {
            if (fp32) qm::split_prolong<float>(n) = sp ? 1 : 0;
            else qm::split_prolong<double>(n) = sp ? 1 : 0;
        }
        ++pos;
    }
    if (!loaded) return tfail("qumond_tune_load: no entries");
    return QUMOND_OK;
}

}  // extern "C"
