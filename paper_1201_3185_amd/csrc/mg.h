// Host-side full-multigrid schedule (Sec. 2 of Angus et al., after the
// Numerical Recipes FMG cited there): rhs restricted to the coarse levels,
// boundary values injected, the levels with at most 17 points per side solved
// inside one workgroup (FMG bootstrap from the exact 3^3 solve), then for each
// finer level trilinear interpolation and ncycle V(npre,npost) cycles, then
// extra finest-level cycles under a relative-residual test.
//
// Every level keeps two buffers for u because the smoother works out of place;
// `cur` says which one holds the iterate.  Both buffers carry the level's
// boundary values (Dirichlet values on FMG levels, zero on correction levels).
//
// A hierarchy can hold nb problems of the same size back to back on every
// level; each launch then covers all of them.
//
// With graphs enabled, the FMG schedule and the finest-level cycle (each with
// the residual norms copied to pinned host memory at its end) are captured once
// per (finest buffers, ping-pong state, launch shapes) and replayed: the
// schedule has no host decisions, so a replay runs exactly the launches of an
// eager run.  The host-side ping-pong state after the capture is recorded and
// restored at every replay.
#pragma once
#include <cmath>
#include <vector>

#include "common.h"

namespace qm {

inline int log2_exact(int m)
{
    int J = 0;
    while ((1 << J) < m) ++J;
    return ((1 << J) == m) ? J : -1;
}

constexpr int kTailLevel = 4;  // 17^3: the coarse tail kernel's top level

template <typename T>
struct Level {
    int n = 0;
    double h = 0.0;
    T *u[2] = {nullptr, nullptr};
    T *f = nullptr;
    int cur = 0;
};

// Optional per-launch timing of the smoother (hipEvents on the solve stream)
// with its algorithmic traffic: read u, read f, write u = 3 values per node.
struct SmootherProfile {
    bool on = false;
    int only_n = 0;   // if > 0, only the plain launches (no folded correction) on levels of only_n points per side,
                      // and of those only the kind the level runs its pre-smoothing with: two-sweep launches
                      // where it fuses pairs of sweeps, single sweeps otherwise
    int sweeps = 0;   // sweeps per recorded launch (1 or 2; 0 before the first)
    std::vector<hipEvent_t> ev;
    std::vector<double> bytes;
    size_t used = 0;
    void record_pair(hipStream_t s, hipEvent_t *a, hipEvent_t *b)
    {
        if (ev.size() < 2 * (used + 1)) {
            hipEvent_t e0, e1;
            (void)hipEventCreate(&e0);
            (void)hipEventCreate(&e1);
            ev.push_back(e0);
            ev.push_back(e1);
        }
        *a = ev[2 * used];
        *b = ev[2 * used + 1];
        ++used;
        (void)s;
    }
    void release()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        ev.clear();
        bytes.clear();
        used = 0;
    }
};

// Smoother launch shapes chosen for one hierarchy (indexed by level), used in
// place of the library-wide tables when set.
struct LevelShapes {
    SmootherShape single[11];
    SmootherShape corr[11];   // single sweep with the correction applied (variant < 0: as single)
    SmootherShape fused[11];
    int use_fused[11];
    int rr[11];   // residual-restriction kernel of fine level l
    int split[11];   // coarse-grid correction of level l as its own launch
    int sr[11];   // last pre-smoothing sweep of level l fused with its residual restriction
};

template <typename T>
struct Multigrid {
    int J = 0, lt = 0;
    int nb = 1;                          // problems per level
    const LevelShapes *shapes = nullptr;
    double L = 0.0;
    int npre = 2, npost = 2;
    std::vector<Level<T>> lv;  // index = level, n = 2^l + 1
    double *partial = nullptr, *norms = nullptr;
    double *host_norms = nullptr;  // pinned, 3 doubles per problem
    double *host_norms_dev = nullptr;   // its device-mapped address (null: copied instead)
    hipStream_t s = nullptr;
    size_t bytes = 0;
    std::vector<void *> owned;
    SmootherProfile prof;
    bool fused = true;   // two sweeps per launch where possible
    double last_r2 = 0.0;  // sum of squared residuals of the last relres()
    bool use_graphs = false;   // replay fmg_norms / cycle_norms from captured graphs
    const double *r32_sc = nullptr;   // set_r32: the next norms pass also writes r32_out
    // set by a caller whose finest iterate is zero before a finest_cycle():
    // its first sweep reads no iterate (the smoother's null input), so the
    // caller need not fill the interiors again; both ping-pong buffers'
    // boundaries must hold zeros.  Valid where zero_start_ok().
    bool zero_start = false;
    bool zero_start_ok() const { return J > lt && npre > 0; }
    // Level l's coarse correction is zero on its interior but was not written
    // there by the restriction: its first pre-smoothing sweep reads no iterate.
    bool zin[11] = {};
    float *r32_out = nullptr;

    struct GraphEntry {
        int kind;                        // 0: FMG + norms, 1: finest cycle + norms
        const void *u0, *u1, *f;         // finest buffers the schedule was captured on
        unsigned cur_in, cur_out;        // ping-pong state before / after
        int ncycle;
        std::vector<int> sig;            // launch shapes in force at capture
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;

    hipError_t alloc(void **p, size_t b)
    {
        hipError_t e = hipMalloc(p, b);
        if (e == hipSuccess) {
            owned.push_back(*p);
            bytes += b;
        }
        return e;
    }

    // Allocate the coarse levels lt..J-1 for a finest grid of n points per side
    // (nb problems per level).
    hipError_t init(int n, int npre_, int npost_, hipStream_t stream, int nb_ = 1)
    {
        nb = nb_;
        J = log2_exact(n - 1);
        lt = J < kTailLevel ? J : kTailLevel;
        npre = npre_;
        npost = npost_;
        s = stream;
        lv.assign(J + 1, Level<T>());
        for (int l = 1; l <= J; ++l) lv[l].n = (1 << l) + 1;
        for (int l = lt; l < J; ++l) {
            const size_t N = (size_t)lv[l].n * lv[l].n * lv[l].n * nb;
            hipError_t e;
            if ((e = alloc((void **)&lv[l].u[0], N * sizeof(T))) != hipSuccess) return e;
            if ((e = alloc((void **)&lv[l].u[1], N * sizeof(T))) != hipSuccess) return e;
            if ((e = alloc((void **)&lv[l].f, N * sizeof(T))) != hipSuccess) return e;
        }
        hipError_t e;
        if ((e = alloc((void **)&partial, 3 * (size_t)kNormBlocks * nb * sizeof(double))) != hipSuccess) return e;
        if ((e = alloc((void **)&norms, 3 * (size_t)nb * sizeof(double))) != hipSuccess) return e;
        if ((e = hipHostMalloc((void **)&host_norms, 3 * (size_t)nb * sizeof(double), hipHostMallocDefault)) != hipSuccess)
            return e;
        // kernels write the norms into the pinned buffer directly where it is mapped
        if (hipHostGetDevicePointer((void **)&host_norms_dev, host_norms, 0) != hipSuccess) {
            host_norms_dev = nullptr;
            (void)hipGetLastError();   // not mapped: copy instead, and leave no error behind
        }
        return hipSuccess;
    }

    void release()
    {
        for (GraphEntry &g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
        prof.release();
        for (void *p : owned) (void)hipFree(p);
        owned.clear();
        if (host_norms) (void)hipHostFree(host_norms);
        host_norms = nullptr;
        host_norms_dev = nullptr;
        bytes = 0;
    }

    // Bind the finest level: u0 holds the iterate (and the result), u1 is the
    // ping-pong partner; both must already hold the boundary values.
    void bind(double box_side, T *u0, T *u1, T *f)
    {
        L = box_side;
        for (int l = 1; l <= J; ++l) lv[l].h = L / (double)(lv[l].n - 1);
        lv[J].u[0] = u0;
        lv[J].u[1] = u1;
        lv[J].f = f;
        for (int l = 1; l <= J; ++l) lv[l].cur = 0;
    }

    void time_begin(hipEvent_t *e0, hipEvent_t *e1, double bytes, int n, bool folds_correction, int sweeps,
                    bool level_fuses)
    {
        if (!prof.on || (prof.only_n > 0 && (prof.only_n != n || folds_correction || sweeps != (level_fuses ? 2 : 1))))
            return;
        prof.sweeps = sweeps;
        prof.record_pair(s, e0, e1);
        prof.bytes.push_back(bytes);
        (void)hipEventRecord(*e0, s);
    }
    void time_end(hipEvent_t e1)
    {
        if (prof.on && e1) (void)hipEventRecord(e1, s);
    }

    // The single-sweep shape of level l, with or without the correction.
    SmootherShape corr_shape(int l, bool with_corr) const
    {
        const int n = lv[l].n;
        if (!with_corr) return shapes ? shapes->single[l] : rbgs_shape<T>(n);
        if (shapes) return shapes->corr[l].variant >= 0 ? shapes->corr[l] : shapes->single[l];
        return rbgs_corr_effective<T>(n);
    }

    // ns red-black sweeps on level l; pairs of sweeps run as one fused launch.
    // With uc != NULL the correction u += P uc is applied before the first
    // sweep: inside its launch, or by a prolong-add launch of its own where
    // the level's table entry asks for that (or when ns == 0).
    void smooth(int l, int ns, const T *uc = nullptr)
    {
        Level<T> &v = lv[l];
        const double pts = (double)v.n * v.n * v.n;
        const bool fuse = fused && (shapes ? shapes->use_fused[l] != 0 : use_fused<T>(v.n) != 0);
        bool zs = false;   // the first fused launch reads no iterate
        if (zero_start && l == J && ns > 0 && !uc) {   // the iterate is zero: first sweep without reading it
            zero_start = false;
            if (fuse && ns >= 2) {
                zs = true;
            } else {
                const SmootherShape sh = shapes ? shapes->single[l] : rbgs_shape<T>(v.n);
                launch_rbgs_shape<T>(v.n, v.h, v.f, nullptr, v.u[1 - v.cur], sh, s, nb);
                v.cur ^= 1;
                --ns;
            }
        }
        if (uc && (ns == 0 || (shapes ? shapes->split[l] : split_prolong<T>(v.n)) != 0)) {
            launch_prolong_add<T>(lv[l - 1].n, uc, v.u[v.cur], s, nb);
            uc = nullptr;
        }
        // a zero iterate, or a zero correction the restriction left unwritten
        bool zi = (zin[l] || zs) && !uc && ns > 0;
        zin[l] = false;
        while (ns > 0) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            const SmootherShape shf = fuse ? (shapes ? shapes->fused[l] : rbgs2_shape<T>(v.n)) : SmootherShape{0, 0};
            const bool two = ns >= 2 && fuse;
            time_begin(&e0, &e1, (zi ? 2.0 : 3.0) * sizeof(T) * pts * nb, v.n, uc != nullptr, two ? 2 : 1, fuse);
            const T *uin = zi ? nullptr : v.u[v.cur];
            zi = false;
            if (two) {
                const SmootherShape sh = shf;
                launch_rbgs2_shape<T>(v.n, v.h, v.f, uin, v.u[1 - v.cur], uc, sh, s, nb);
                ns -= 2;
            } else {
                const SmootherShape sh = corr_shape(l, uc != nullptr);
                launch_rbgs_shape<T>(v.n, v.h, v.f, uin, v.u[1 - v.cur], sh, s, nb, uc);
                ns -= 1;
            }
            uc = nullptr;
            time_end(e1);
            v.cur ^= 1;
        }
    }

    // One V-cycle with top level l (l > lt), zero-boundary corrections below.
    void vcycle(int l)
    {
        Level<T> &v = lv[l];
        Level<T> &c = lv[l - 1];
        if (fuse_sweep_restrict(l)) {
            smooth(l, npre - 1);
            const bool zu = !coarse_reads_no_iterate(l - 1);
            launch_rbgs_restrict<T>(v.n, v.h, v.f, v.u[v.cur], v.u[1 - v.cur], c.f, c.u[c.cur], c.u[1 - c.cur], s, nb,
                                    zu);
            zin[l - 1] = !zu && l - 1 > lt;
            v.cur ^= 1;
        } else {
            smooth(l, npre);
            restrict_residual(l);
        }
        // the restriction zeroed the correction: the tail need not read it
        if (l - 1 == lt) launch_coarse_tail<T>(lt, L, c.f, c.u[c.cur], npre, npost, 1, 2, 1, s, nb);
        else vcycle(l - 1);
        smooth(l, npost, c.u[c.cur]);
    }

    // Whether level l's last pre-smoothing sweep runs fused with the residual
    // restriction: where the table asks for it, the level sweeps one sweep per
    // launch, and that sweep reads an iterate (not the zero-iterate first sweep).
    bool fuse_sweep_restrict(int l) const
    {
        const int n = lv[l].n;
        if (!(shapes ? shapes->sr[l] : sweep_restrict<T>(n)) || !rbgs_restrict_fits<T>(n) || npre < 1) return false;
        if (fused && (shapes ? shapes->use_fused[l] : use_fused<T>(n)) != 0 && npre >= 2) return false;
        return !(zero_start && l == J && npre == 1);
    }

    // Whether the V-cycle on coarse level c starts without reading its
    // (zero) correction: the coarse tail takes it as zero, and so does a first
    // pre-smoothing sweep of smooth(); a fused sweep-and-restriction reads it.
    bool coarse_reads_no_iterate(int c) const
    {
        if (c == lt) return true;
        if (npre < 1) return false;
        return !(npre == 1 && fuse_sweep_restrict(c));
    }

    void restrict_residual(int l)
    {
        Level<T> &v = lv[l];
        Level<T> &c = lv[l - 1];
        const bool zu = !coarse_reads_no_iterate(l - 1);
        if (shapes)
            launch_residual_restrict_variant<T>(v.n, v.h, v.f, v.u[v.cur], c.f, c.u[c.cur], c.u[1 - c.cur],
                                                shapes->rr[l], s, nb, zu);
        else
            launch_residual_restrict<T>(v.n, v.h, v.f, v.u[v.cur], c.f, c.u[c.cur], c.u[1 - c.cur], s, nb, zu);
        zin[l - 1] = !zu && l - 1 > lt;
    }

    // The finest-level cycle used after the FMG schedule.
    void finest_cycle(int nrep = 1)
    {
        if (J <= lt) {
            zero_start = false;
            launch_coarse_tail<T>(J, L, lv[J].f, lv[J].u[lv[J].cur], npre, npost, 1, 0, nrep, s, nb);
            return;
        }
        for (int r = 0; r < nrep; ++r) vcycle(J);
        zero_start = false;
    }

    // FMG with ncycle V-cycles per level.  The finest u's boundary holds the
    // Dirichlet values.
    void fmg(int ncycle)
    {
        Level<T> &F = lv[J];
        if (J <= lt) {
            launch_coarse_tail<T>(J, L, F.f, F.u[F.cur], npre, npost, ncycle, 1, 1, s, nb);
            return;
        }
        for (int l = J - 1; l >= lt; --l) launch_restrict<T>(lv[l + 1].n, lv[l + 1].f, lv[l].f, s, nb);
        for (int l = lt; l < J; ++l)
            launch_inject_boundary<T>(F.n, F.u[F.cur], lv[l].n, lv[l].u[0], lv[l].u[1], s, nb);
        Level<T> &t = lv[lt];
        launch_coarse_tail<T>(lt, L, t.f, t.u[t.cur], npre, npost, ncycle, 1, 1, s, nb);
        for (int l = lt + 1; l <= J; ++l) {
            Level<T> &c = lv[l - 1];
            launch_interp<T>(c.n, c.u[c.cur], lv[l].u[lv[l].cur], s, nb);
            for (int k = 0; k < ncycle; ++k) vcycle(l);
        }
    }

    // Residual norms of the finest level of every problem into norms (device);
    // after set_r32 the next norms pass (once) also writes the residual times
    // 1/s, rounded to FP32, to r32 (FP64 hierarchies only).
    void device_norms(double *hout = nullptr)
    {
        Level<T> &F = lv[J];
        if constexpr (sizeof(T) == 8) {
            if (r32_out) {
                launch_resid_norms_r32(F.n, F.h, F.f, F.u[F.cur], partial, norms, r32_sc, r32_out, s, nb, hout);
                r32_sc = nullptr;
                r32_out = nullptr;
                return;
            }
        }
        launch_resid_norms<T>(F.n, F.h, F.f, F.u[F.cur], partial, norms, s, nb, hout);
    }
    void set_r32(const double *sc, float *r)
    {
        r32_sc = sc;
        r32_out = r;
    }

    // Enqueue the residual norms of the finest level into host_norms (needs a
    // stream synchronisation before reading).
    void enqueue_norms()
    {
        if (host_norms_dev) {   // the norms kernel writes the pinned copy itself
            device_norms(host_norms_dev);
            return;
        }
        device_norms();
        (void)hipMemcpyAsync(host_norms, norms, 3 * (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, s);
    }

    unsigned cur_mask() const
    {
        unsigned m = 0;
        for (int l = 1; l <= J; ++l) m |= (unsigned)lv[l].cur << l;
        return m;
    }
    void set_cur(unsigned m)
    {
        for (int l = 1; l <= J; ++l) lv[l].cur = (int)((m >> l) & 1u);
    }

    // The launch shapes a schedule of this hierarchy uses.
    std::vector<int> shape_sig() const
    {
        std::vector<int> v;
        for (int l = lt; l <= J; ++l) {
            const int n = lv[l].n;
            const SmootherShape a = shapes ? shapes->single[l] : rbgs_shape<T>(n);
            const SmootherShape c = corr_shape(l, true);
            const SmootherShape b = shapes ? shapes->fused[l] : rbgs2_shape<T>(n);
            const int uf = shapes ? shapes->use_fused[l] : use_fused<T>(n);
            const int rr = shapes ? shapes->rr[l] : rr_variant<T>(n);
            const int sp = shapes ? shapes->split[l] : split_prolong<T>(n);
            const int sr = shapes ? shapes->sr[l] : sweep_restrict<T>(n);
            v.insert(v.end(), {a.variant, a.kchunk, c.variant, c.kchunk, b.variant, b.kchunk, uf, rr, sp, sr});
        }
        v.insert(v.end(), {fused ? 1 : 0, npre, npost});
        return v;
    }

    // Enqueue body() (kind 0: fmg(ncycle), 1: finest_cycle(), each followed by
    // enqueue_norms()), from a captured graph when graphs are on and the
    // smoother is not being timed.
    template <class Body>
    hipError_t enqueue_schedule(int kind, int ncycle, Body body)
    {
        if (!use_graphs || prof.on || s == nullptr) {   // the null stream cannot be captured
            body();
            enqueue_norms();
            return hipSuccess;
        }
        const unsigned cin = cur_mask();
        const std::vector<int> sig = shape_sig();
        for (size_t i = 0; i < graphs.size(); ++i) {
            GraphEntry &g = graphs[i];
            if (g.kind != kind || g.u0 != lv[J].u[0] || g.u1 != lv[J].u[1] || g.f != lv[J].f || g.cur_in != cin ||
                g.ncycle != ncycle)
                continue;
            if (g.sig != sig) {   // shapes changed since the capture
                (void)hipGraphExecDestroy(g.exec);
                graphs.erase(graphs.begin() + (long)i);
                break;
            }
            set_cur(g.cur_out);
            return hipGraphLaunch(g.exec, s);
        }
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        body();
        enqueue_norms();
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(s, &graph);
        if (e != hipSuccess) return e;
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        graphs.push_back(GraphEntry{kind, lv[J].u[0], lv[J].u[1], lv[J].f, cin, cur_mask(), ncycle, sig, exec});
        return hipGraphLaunch(exec, s);
    }

    // FMG then the residual norms, and one finest cycle then the norms; the
    // relative residual is read by relres_read().
    hipError_t fmg_norms(int ncycle)
    {
        return enqueue_schedule(0, ncycle, [&] { fmg(ncycle); });
    }
    hipError_t cycle_norms()
    {
        return enqueue_schedule(1, 0, [&] { finest_cycle(); });
    }

    // The relative residual from norms already enqueued (synchronises).
    hipError_t relres_read(double &out)
    {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        last_r2 = host_norms[0];
        const double rn = std::sqrt(host_norms[0]), fn = std::sqrt(host_norms[1]), bn = std::sqrt(host_norms[2]);
        const double den = fn > 0.0 ? fn : bn;
        out = den > 0.0 ? rn / den : rn;
        return hipSuccess;
    }

    hipError_t relres(double &out)
    {
        enqueue_norms();
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        // ||f - A u|| / ||f||; a source-free box is measured against the
        // boundary-value contribution instead, and if that is 0 the residual is absolute.
        last_r2 = host_norms[0];
        const double rn = std::sqrt(host_norms[0]), fn = std::sqrt(host_norms[1]), bn = std::sqrt(host_norms[2]);
        const double den = fn > 0.0 ? fn : bn;
        out = den > 0.0 ? rn / den : rn;
        return hipSuccess;
    }

    T *result() { return lv[J].u[lv[J].cur]; }

    // Leave the result in u[0] of the finest level.
    void finish()
    {
        Level<T> &F = lv[J];
        if (F.cur == 1) {
            (void)hipMemcpyAsync(F.u[0], F.u[1], (size_t)F.n * F.n * F.n * nb * sizeof(T), hipMemcpyDeviceToDevice, s);
            F.cur = 0;
        }
    }
};

}  // namespace qm
