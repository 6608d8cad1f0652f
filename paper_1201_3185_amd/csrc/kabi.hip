// Single-grid entry points (qumond_kernels.h): each runs one kernel, or one
// FMG / V-cycle schedule, on caller-owned device grids.
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/qumond_kernels.h"
#include "common.h"
#include "mg.h"

void qm_set_last_error(const char *msg);  // defined with the main ABI

namespace {
qumond_status kfail(const char *msg)
{
    qm_set_last_error(msg);
    return QUMOND_ERR_INVALID;
}
qumond_status kcheck(const char *where)
{
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) return QUMOND_OK;
    qm_set_last_error((std::string(where) + ": " + hipGetErrorString(e)).c_str());
    return QUMOND_ERR_HIP;
}
bool good_n(int n) { return n >= 5 && n <= 1025 && qm::log2_exact(n - 1) >= 2; }
bool good_nc(int nc) { return nc >= 3 && nc <= 513 && qm::log2_exact(nc - 1) >= 1; }
}  // namespace

// Workspace of qumond_k_resid_norms_noalloc: the per-workgroup partial sums
// (three doubles per workgroup) of one problem.  The partial pass uses at most
// kNormBlocks workgroups for any n, so 48 KiB covers every grid up to the
// largest the library takes (n = 1025).  Each device holds its own copy for
// the life of the process.  Host code never uses this name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[3 * qm::kNormBlocks];

namespace {
constexpr int kScratchMaxN = 1025;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call made on that device.
qumond_status scratch_on_current_device(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        qm_set_last_error((std::string("qumond_k_resid_norms_noalloc: hipGetDevice: ") + hipGetErrorString(e)).c_str());
        return QUMOND_ERR_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        qm_set_last_error("qumond_k_resid_norms_noalloc: device index beyond the workspace table (64 devices)");
        return QUMOND_ERR_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            qm_set_last_error((std::string("qumond_k_resid_norms_noalloc: hipGetSymbolAddress: ") +
                               hipGetErrorString(e)).c_str());
            return QUMOND_ERR_HIP;
        }
        g_scratch_dev[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return QUMOND_OK;
}
}  // namespace

extern "C" {

qumond_status qumond_k_rbgs_sweep(int32_t n, double h, const double *f, const double *u_in, double *u_out, void *stream)
{
    if (!good_n(n) || !(h > 0.0) || !f || !u_in || !u_out || u_in == u_out) return kfail("qumond_k_rbgs_sweep: bad argument");
    qm::launch_rbgs<double>(n, h, f, u_in, u_out, (hipStream_t)stream);
    return kcheck("qumond_k_rbgs_sweep");
}

qumond_status qumond_k_rbgs_sweep_from_zero(int32_t n, double h, const double *f, double *u_out, void *stream)
{
    if (!good_n(n) || !(h > 0.0) || !f || !u_out) return kfail("qumond_k_rbgs_sweep_from_zero: bad argument");
    qm::launch_rbgs<double>(n, h, f, nullptr, u_out, (hipStream_t)stream);
    return kcheck("qumond_k_rbgs_sweep_from_zero");
}

qumond_status qumond_k_rbgs_double_sweep(int32_t n, double h, const double *f, const double *u_in, double *u_out,
                                         const double *uc, void *stream)
{
    if (!good_n(n) || !(h > 0.0) || !f || !u_out || u_in == u_out || (!u_in && uc))
        return kfail("qumond_k_rbgs_double_sweep: bad argument");
    qm::launch_rbgs2<double>(n, h, f, u_in, u_out, uc, (hipStream_t)stream);
    return kcheck("qumond_k_rbgs_double_sweep");
}

qumond_status qumond_k_residual_restrict(int32_t nf, double h, const double *f, const double *u, double *fc,
                                         double *uc0, double *uc1, void *stream)
{
    if (!good_n(nf) || !(h > 0.0) || !f || !u || !fc || !uc0) return kfail("qumond_k_residual_restrict: bad argument");
    qm::launch_residual_restrict<double>(nf, h, f, u, fc, uc0, uc1, (hipStream_t)stream);
    return kcheck("qumond_k_residual_restrict");
}

qumond_status qumond_k_rbgs_sweep_restrict(int32_t n, double h, const double *f, const double *u_in, double *u_out,
                                           double *fc, double *uc0, double *uc1, void *stream)
{
    if (!good_n(n) || !qm::rbgs_restrict_fits<double>(n) || !(h > 0.0) || !f || !u_in || !u_out || u_in == u_out ||
        !fc || !uc0)
        return kfail("qumond_k_rbgs_sweep_restrict: bad argument");
    qm::launch_rbgs_restrict<double>(n, h, f, u_in, u_out, fc, uc0, uc1, (hipStream_t)stream);
    return kcheck("qumond_k_rbgs_sweep_restrict");
}

qumond_status qumond_k_restrict(int32_t nf, const double *src, double *dst, void *stream)
{
    if (!good_n(nf) || !src || !dst) return kfail("qumond_k_restrict: bad argument");
    qm::launch_restrict<double>(nf, src, dst, (hipStream_t)stream);
    return kcheck("qumond_k_restrict");
}

qumond_status qumond_k_prolong_add(int32_t nc, const double *uc, double *uf, void *stream)
{
    if (!good_nc(nc) || !uc || !uf) return kfail("qumond_k_prolong_add: bad argument");
    qm::launch_prolong_add<double>(nc, uc, uf, (hipStream_t)stream);
    return kcheck("qumond_k_prolong_add");
}

qumond_status qumond_k_interp(int32_t nc, const double *uc, double *uf, void *stream)
{
    if (!good_nc(nc) || !uc || !uf) return kfail("qumond_k_interp: bad argument");
    qm::launch_interp<double>(nc, uc, uf, (hipStream_t)stream);
    return kcheck("qumond_k_interp");
}

qumond_status qumond_k_mond_source(int32_t n, double h, double a0, const double *phin, double *S, void *stream)
{
    if (!good_n(n) || !(h > 0.0) || !(a0 >= 0.0) || !phin || !S) return kfail("qumond_k_mond_source: bad argument");
    qm::launch_mond_source(n, h, a0, phin, S, (hipStream_t)stream);
    return kcheck("qumond_k_mond_source");
}

qumond_status qumond_k_bc_from_coarse(int32_t n, const double *uc, double *uf, void *stream)
{
    if (!good_n(n) || !uc || !uf) return kfail("qumond_k_bc_from_coarse: bad argument");
    qm::launch_bc_from_coarse(n, uc, uf, nullptr, (hipStream_t)stream);
    return kcheck("qumond_k_bc_from_coarse");
}

qumond_status qumond_k_resid_norms(int32_t n, double h, const double *f, const double *u, double *out2, void *stream)
{
    if (!good_n(n) || !(h > 0.0) || !f || !u || !out2) return kfail("qumond_k_resid_norms: bad argument");
    double *partial = nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (hipMallocAsync((void **)&partial, 3 * qm::kNormBlocks * sizeof(double), s) != hipSuccess)
        return kcheck("qumond_k_resid_norms: allocation");
    qm::launch_resid_norms<double>(n, h, f, u, partial, out2, s);
    (void)hipFreeAsync(partial, s);
    return kcheck("qumond_k_resid_norms");
}

qumond_status qumond_k_resid_norms_noalloc(int32_t n, double h, const double *f, const double *u, double *out3,
                                           void *stream)
{
    if (n > kScratchMaxN)
        return kfail("qumond_k_resid_norms_noalloc: n exceeds the workspace maximum (1025 points per side)");
    if (!good_n(n) || !(h > 0.0) || !f || !u || !out3) return kfail("qumond_k_resid_norms_noalloc: bad argument");
    static_assert(3 * qm::kNormBlocks * sizeof(double) == sizeof(scratch), "one problem's partial sums");
    double *partial = nullptr;
    const qumond_status st = scratch_on_current_device(&partial);
    if (st != QUMOND_OK) return st;
    qm::launch_resid_norms<double>(n, h, f, u, partial, out3, (hipStream_t)stream);
    return kcheck("qumond_k_resid_norms_noalloc");
}

static qumond_status run_schedule(int32_t n, double L, const double *f, double *u, int32_t npre, int32_t npost,
                                  int32_t ncycle, int32_t nextra, double tol, bool do_fmg, double *relres,
                                  int32_t *extra, void *stream)
{
    if (!good_n(n) || !(L > 0.0) || !f || !u || npre < 0 || npost < 0 || npre + npost < 1 || npre > 8 || npost > 8 ||
        ncycle < 0 || nextra < 0 || !(tol >= 0.0))
        return kfail("multigrid schedule: bad argument");
    hipStream_t s = (hipStream_t)stream;
    qm::Multigrid<double> mg;
    double *scratch = nullptr;
    const size_t N = (size_t)n * n * n;
    if (mg.init(n, npre, npost, s) != hipSuccess || hipMalloc((void **)&scratch, N * sizeof(double)) != hipSuccess) {
        mg.release();
        return kcheck("multigrid schedule: allocation");
    }
    qm::launch_boundary_copy<double>(n, u, scratch, s);
    mg.bind(L, u, scratch, const_cast<double *>(f));
    double rr = 0.0;
    int done = 0;
    if (do_fmg) {
        mg.fmg(ncycle);
        if (mg.relres(rr) != hipSuccess) goto out;
        while (tol > 0.0 && rr > tol && done < nextra) {
            mg.finest_cycle();
            ++done;
            if (mg.relres(rr) != hipSuccess) goto out;
        }
    } else {
        mg.finest_cycle(ncycle);
        if (mg.relres(rr) != hipSuccess) goto out;
    }
    mg.finish();
    (void)hipStreamSynchronize(s);
out:
    (void)hipFree(scratch);
    mg.release();
    if (relres) *relres = rr;
    if (extra) *extra = done;
    return kcheck("multigrid schedule");
}

qumond_status qumond_k_fmg(int32_t n, double L, const double *f, double *u, int32_t npre, int32_t npost, int32_t ncycle,
                           int32_t max_extra, double tol, double *relres, int32_t *extra, void *stream)
{
    if (ncycle < 1) return kfail("qumond_k_fmg: ncycle must be >= 1");
    return run_schedule(n, L, f, u, npre, npost, ncycle, max_extra, tol, true, relres, extra, stream);
}

qumond_status qumond_k_vcycles(int32_t n, double L, const double *f, double *u, int32_t npre, int32_t npost,
                               int32_t ncyc, double *relres, void *stream)
{
    return run_schedule(n, L, f, u, npre, npost, ncyc, 0, 0.0, false, relres, nullptr, stream);
}

}  // extern "C"
