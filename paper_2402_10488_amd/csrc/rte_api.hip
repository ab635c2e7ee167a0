// C ABI of the gfx950 RTE library: argument validation, workspace carving and the host-side
// iteration driver of Alg. 1 / Alg. 2.  Every arithmetic step runs in the kernels of
// sweep.hip, iterate.hip, dsa.hip and rom.hip.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "rte_internal.h"

using namespace rte;

namespace {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Carver {
    char *base;
    size_t off, cap;
    bool ok;
    explicit Carver(void *b, size_t c) : base((char *)b), off(0), cap(c), ok(true) {}
    template <typename T>
    T *take(size_t n) {
        const size_t bytes = align_up(n * sizeof(T));
        T *ptr = base ? (T *)(base + off) : nullptr;
        off += bytes;
        if (base && off > cap) ok = false;
        return ptr;
    }
};

// Everything the calls carve out of the caller's workspace, in one fixed order.
struct Layout {
    double *rho_star, *delta;
    void *src;
    double *partial;        // 2D sweep partials
    void *fscratch;         // 1D angular flux scratch
    IterState st;
    CGSpace cg;
    double *dsa1d;          // 1D DSA scratch
    RomSpace rom;
    int *rom_status;
    unsigned long long *cg_total;   // CG iterations summed over instances and calls
    int *cg_fail;           // [1] diffusion CG failures (graph mode reads it at the end)
    int *flag;
    int *mask;              // [B] instances selected by rte_sisa_admit
    GmresSpace gm;          // DSA-preconditioned GMRES (rte_pgmres_solve)
    // 2D material tables of the sweep (launch_materials): cell indices [B][ncell], flags and
    // counts [B], values [B][kMaxMat], coefficients [B][n_sorted][kMaxMat][8] T
    int *mat, *mat_ok, *nmat;
    double *mvals, *mcvals;
    void *mcoef;
    bool use_mat;           // host: this call's sweeps use them (prepared in this workspace)
    // host-side: the CG iteration after which the previous diffusion solve of this call was
    // first seen finished (0: none yet); where do_dsa first looks at the running count
    mutable int cg_look;
};

int nparts_for(const rte_problem *p) { return sweep_nparts(p); }

Layout carve(Carver &c, const rte_problem *p, rte_mode mode, const rte_rom *rom,
             rte_precision prec, int max_iter, int gm_m = 0) {
    Layout L;
    std::memset(&L, 0, sizeof(L));
    const size_t B = p->B, nd = p->ndof;
    const size_t ts = prec == RTE_MIXED ? 4 : 8;
    L.rho_star = c.take<double>(B * nd);
    L.delta = c.take<double>(B * nd);
    // sweep input block: 2D two diagonal layouts of (source, sigma_t); 1D natural source
    L.src = c.take<char>(p->dim == 2 ? B * (size_t)p->ncell * 10 * ts : B * nd * ts);
    if (p->dim == 2) L.partial = c.take<double>(B * (size_t)nparts_for(p) * nd);
    else L.fscratch = c.take<char>(B * (size_t)p->n_dir * nd * ts);
    L.st.maxd = c.take<unsigned long long>(B);
    L.st.maxr = c.take<unsigned long long>(B);
    L.st.active = c.take<int>(B);
    L.st.kind = c.take<int>(B);
    L.st.n_sweep = c.take<int>(B);
    L.st.status = c.take<int>(B);
    L.st.change = c.take<double>(B * (size_t)std::max(max_iter, 1));
    L.st.kinds = c.take<int>(B * (size_t)std::max(max_iter, 1));
    L.st.n_active = c.take<int>(3);
    L.cg_total = c.take<unsigned long long>(1);
    L.cg_fail = c.take<int>(1);
    L.flag = c.take<int>(1);
    L.mask = c.take<int>(B);
    if (p->dim == 2) {
        L.mat = c.take<int>(B * (size_t)p->ncell);
        L.mat_ok = c.take<int>(B);
        L.nmat = c.take<int>(B);
        L.mvals = c.take<double>(B * (size_t)kMaxMat);
        L.mcvals = c.take<double>(B * (size_t)mat_chunks(p) * (kMaxMat + 1));
        L.mcoef = c.take<char>(B * (size_t)p->n_sorted * kMaxMat * 8 * ts);
    }
    if (mode != RTE_SI) {
        if (p->dim == 2) {
            L.cg.nblk = (int)cg_blocks_per_instance(p);
            L.cg.precond[0] = L.cg.precond[1] = nullptr;
            L.cg.x = c.take<double>(B * nd);
            L.cg.r = c.take<double>(B * nd);
            L.cg.z = c.take<double>(B * nd);
            L.cg.p0 = c.take<double>(B * nd);
            L.cg.p1 = c.take<double>(B * nd);
            L.cg.q = c.take<double>(B * nd);
            L.cg.part = c.take<double>(B * 5 * (size_t)L.cg.nblk);
            L.cg.iters = c.take<int>(B);
            L.cg.state = c.take<int>(B);
            L.cg.fails = L.cg_fail;
            L.cg.n_running = c.take<int>(2);
            L.cg.tol2 = c.take<double>(1);
            L.cg.cf = c.take<double>(B * (size_t)p->ncell * 5);
            L.cg.binv = c.take<float>(B * (size_t)p->ncell * 10);
            int nvx[kMaxLevels], nvy[kMaxLevels];
            L.cg.mg.L = p->dsa_mg ? mg_levels(p->nx, p->ny, nvx, nvy) : 0;
            for (int l = 0; l < L.cg.mg.L; ++l) {
                MGLevel &g = L.cg.mg.lv[l];
                g.nvx = nvx[l];
                g.nvy = nvy[l];
                g.nv = (long long)nvx[l] * nvy[l];
                g.S = c.take<double>(B * (size_t)g.nv * kStencilPlanes);
                g.S32 = c.take<float>(B * (size_t)g.nv * kStencilPlanes);
                g.xa = c.take<double>(B * (size_t)g.nv);
                g.xb = c.take<double>(B * (size_t)g.nv);
                g.bv = c.take<double>(B * (size_t)g.nv);
                g.rv = c.take<double>(B * (size_t)g.nv);
            }
            L.cg.mg.cinv = nullptr;
            L.cg.zf32 = prec == RTE_MIXED && L.cg.mg.L > 0;
            L.cg.cf32 = L.cg.zf32 ? c.take<float>(B * (size_t)p->ncell * 5) : nullptr;
            if (L.cg.mg.L > 0) {
                L.cg.mg.t = c.take<double>(B * nd);
                L.cg.mg.e = c.take<double>(B * (size_t)L.cg.mg.lv[0].nv);
                const long long nc = L.cg.mg.lv[L.cg.mg.L - 1].nv;
                if (nc <= kDirectCoarse) L.cg.mg.cinv = c.take<double>(B * (size_t)(nc * nc));
            }
        } else {
            L.dsa1d = c.take<double>(B * (size_t)p->nx * 20);
            L.cg.iters = c.take<int>(B);
        }
    }
    if (rom) {
        L.rom.nsplit = (int)rom_split(p, rom);
        L.rom.ypart = c.take<double>(B * (size_t)L.rom.nsplit * rom->r);
        L.rom.dc = c.take<double>(B * (size_t)rom->r);
        L.rom.y = c.take<double>(B * (size_t)rom->r);
        L.rom.A = c.take<double>(B * (size_t)rom->r * rom->r);
        L.rom.n_fallback = L.st.n_active + 1;    // a singular system's instance takes DSA
        L.rom_status = c.take<int>(B);
    }
    if (gm_m > 0) {
        GmresSpace &g = L.gm;
        g.m = gm_m;
        g.nblk = gmres_blocks(p);
        g.nslot = gm_m + 2;
        g.normslot = gm_m + 1;
        g.V = c.take<double>((size_t)(gm_m + 1) * B * nd);
        g.w = c.take<double>(B * nd);
        g.t = c.take<double>(B * nd);
        g.u = c.take<double>(B * nd);
        g.bbar = c.take<double>(B * nd);
        g.lv = c.take<double>(B * nd);
        g.part = c.take<double>(B * (size_t)g.nslot * g.nblk);
        g.h = c.take<double>(B * (size_t)g.nslot);
        g.h2 = c.take<double>(B * (size_t)g.nslot);
        g.H = c.take<double>(B * (size_t)(gm_m + 1) * gm_m);
        g.cs = c.take<double>(B * (size_t)gm_m);
        g.sn = c.take<double>(B * (size_t)gm_m);
        g.y = c.take<double>(B * (size_t)gm_m);
        g.g = c.take<double>(B * (size_t)(gm_m + 1));
        g.nb = c.take<double>(B);
        g.est = c.take<double>(B);
        g.wn = c.take<double>(B);
        g.act = c.take<int>(B);
        g.cyc = c.take<int>(B);
        g.kused = c.take<int>(B);
        g.n_sweep = c.take<int>(B);
        g.n_iter = c.take<int>(B);
        g.count = c.take<int>(1);
    }
    return L;
}

// the last HIP error a call of this thread returned RTE_EDEVICE for (rte_last_device_error)
thread_local hipError_t g_last_hip = hipSuccess;

int device_error(hipError_t e) {
    g_last_hip = e;
    return RTE_EDEVICE;
}

#define HIPCHK(x)                                        \
    do {                                                 \
        hipError_t e_ = (x);                             \
        if (e_ != hipSuccess) return device_error(e_);   \
    } while (0)

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

void choose_tuning(rte_problem *p, int dg_req, int wpb_req, int bands_req) {
    int nqmax = 0;
    for (int q = 0; q < 4; ++q) nqmax = std::max(nqmax, p->quad.count[q]);
    auto wavefronts = [&](int d) {
        long long items = 0;
        for (int q = 0; q < 4; ++q) items += (long long)p->B * ((p->quad.count[q] + d - 1) / d);
        return items;
    };
    int dg = 1;
    if (dg_req > 0) {
        dg = dg_req;
    } else {
        // largest group that still gives >= 4096 wavefronts (16 per CU), at most 8 directions
        // per lane (the FP64 kernel spills beyond that)
        const int cand[4] = {8, 4, 2, 1};
        for (int i = 0; i < 4; ++i) {
            const int d = cand[i];
            if (d > nqmax) continue;
            if (wavefronts(d) >= 4096 || d == 1) { dg = d; break; }
        }
    }
    // wavefronts per workgroup: as many direction groups of a quadrant as fit (<= 4)
    int wpb = wpb_req > 0 ? wpb_req : 4;
    const int groups = (nqmax + dg - 1) / dg;
    if (wpb_req <= 0 && wpb > groups) wpb = groups < 1 ? 1 : groups;
    // LDS: partial-sum buffers 2*wpb*64*4 doubles + rings wpb*nx*dg*2 values of <= 8 bytes
    auto lds = [&](int w, int d) { return (size_t)2 * w * 64 * 4 * 8 + (size_t)w * p->nx * d * 2 * 8; };
    while (wpb > 1 && lds(wpb, dg) > 64 * 1024) wpb /= 2;
    while (dg > 1 && lds(wpb, dg) > 64 * 1024) dg /= 2;
    // mesh bands in flight per workgroup: a batch too small to fill the chip (fewer than 16
    // wavefronts per CU) runs two bands at once, one with fewer than 4 per CU runs four bands
    // of two-wavefront workgroups; the launch lowers the count to what the mesh and LDS allow
    int bands = 1;
    if (bands_req > 0) {
        bands = bands_req;
    } else if (p->dim == 2) {
        const long long wf = wavefronts(dg);
        if (wf < 1024) {
            bands = 4;
            if (wpb_req <= 0 && wpb > 2) wpb = 2;
        } else if (wf < 4096) {
            bands = 2;
        }
    }
    p->tune.dg = dg;
    p->tune.wpb = wpb;
    p->tune.bands = bands;
}

// Per-kernel timing with HIP events recorded on the launch stream (enabled by
// rte_profile_enable).  Events come from a pool that is reused across calls.
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t next = 0;
    std::vector<std::pair<size_t, size_t>> marks[RTE_PROF_NKERNELS];
    hipEvent_t get() {
        if (next == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[next++];
    }
};
Profiler g_prof;
// the profiler's pool and marks are shared by every host thread (rte_sisa_solve_multi runs
// solves in several); capture of an iteration graph switches timing off for its own thread only
std::mutex g_prof_mu;
thread_local bool t_prof_off = false;

struct ProfScope {
    hipEvent_t a = nullptr;
    int id;
    hipStream_t s;
    size_t ia = 0;
    ProfScope(int kid, hipStream_t st) : id(kid), s(st) {
        if (!g_prof.on || t_prof_off) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        ia = g_prof.next;
        a = g_prof.get();
        if (a) (void)hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (!g_prof.on || t_prof_off || !a) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        const size_t ib = g_prof.next;
        hipEvent_t b = g_prof.get();
        if (!b) return;
        (void)hipEventRecord(b, s);
        g_prof.marks[id].push_back({ia, ib});
    }
};

}  // namespace

// One outer iteration of rte_sisa_solve / rte_sisa_iterate captured as a HIP graph, kept by the
// problem handle for the workspace and arguments it was captured with (the graph's kernels hold
// their device pointers), with the stream it is captured on and the pinned words and events
// through which the host reads the active count.
struct rte_iter_graph {
    struct Exec {
        hipGraphExec_t exec = nullptr;
        int *h_active = nullptr;              // pinned host [2]: active counts of polled launches
        hipEvent_t ev[2] = {nullptr, nullptr};
        ~Exec() {
            if (exec) (void)hipGraphExecDestroy(exec);
            for (hipEvent_t e : ev)
                if (e) (void)hipEventDestroy(e);
            if (h_active) (void)hipHostFree(h_active);
        }
    };
    struct Key {
        const void *ws;
        size_t ws_bytes;
        int mode;
        unsigned long long rom;               // serial of the ROM (0: none)
        const double *psi;
        double *rho;
        void *f_out;
        double eps, eps_romsad, cg_rtol;
        int max_iter, relative, theta, precision, depth;
        bool operator==(const Key &o) const {
            return ws == o.ws && ws_bytes == o.ws_bytes && mode == o.mode && rom == o.rom &&
                   psi == o.psi && rho == o.rho && f_out == o.f_out && eps == o.eps &&
                   eps_romsad == o.eps_romsad && cg_rtol == o.cg_rtol && max_iter == o.max_iter &&
                   relative == o.relative && theta == o.theta && precision == o.precision &&
                   depth == o.depth;
        }
    };
    std::mutex mu;
    hipStream_t cs = nullptr;                 // capture stream
    Key key{};
    bool valid = false;
    std::shared_ptr<Exec> cur;
    ~rte_iter_graph() {
        cur.reset();
        if (cs) (void)hipStreamDestroy(cs);
    }
};

// The multigrid preconditioner's launches (one graph per parity slot of its (r, z) partial sums),
// kept by the problem handle for the workspace carve-up they were captured with: their kernels
// hold its device pointers, so a call with another workspace, mode, precision, iteration
// history, ROM or preconditioner choice captures again.  A call holds the graphs it uses by a
// shared pointer, so a capture for another call on the handle never frees them under it.
struct rte_precond_graphs {
    struct Exec {
        hipGraphExec_t g[2] = {nullptr, nullptr};
        ~Exec() {
            for (hipGraphExec_t &x : g)
                if (x) (void)hipGraphExecDestroy(x);
        }
    };
    struct Key {
        int caller;                           // 0 rte_sisa_solve, 1 rte_pgmres_solve
        const void *ws;
        size_t ws_bytes;
        int mode, precision, max_iter, mg;
        unsigned long long rom;
        const void *z, *t, *part;             // a check on the carve-up itself
        bool operator==(const Key &o) const {
            return caller == o.caller && ws == o.ws && ws_bytes == o.ws_bytes && mode == o.mode &&
                   precision == o.precision && max_iter == o.max_iter && mg == o.mg &&
                   rom == o.rom && z == o.z && t == o.t && part == o.part;
        }
    };
    std::mutex mu;
    Key key{};
    bool valid = false;
    std::shared_ptr<Exec> cur;
};

int rte_problem::nparts() const { return nparts_for(this); }

extern "C" {

int rte_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.on = on != 0;
    g_prof.next = 0;
    for (int k = 0; k < RTE_PROF_NKERNELS; ++k) g_prof.marks[k].clear();
    return RTE_OK;
}

int rte_profile_read(int kernel, double *total_ms, long long *count) {
    if (kernel < 0 || kernel >= RTE_PROF_NKERNELS || !total_ms || !count) return RTE_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double t = 0.0;
    for (const auto &m : g_prof.marks[kernel]) {
        if (hipEventSynchronize(g_prof.pool[m.second]) != hipSuccess) return RTE_EDEVICE;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, g_prof.pool[m.first], g_prof.pool[m.second]) != hipSuccess)
            return RTE_EDEVICE;
        t += ms;
    }
    *total_ms = t;
    *count = (long long)g_prof.marks[kernel].size();
    return RTE_OK;
}

const char *rte_strerror(int s) {
    switch (s) {
        case RTE_OK: return "ok";
        case RTE_EINVAL: return "invalid argument";
        case RTE_ENOCONV: return "iteration limit reached before the tolerance";
        case RTE_ESINGULAR: return "singular reduced system";
        case RTE_ECG: return "diffusion CG did not converge";
        case RTE_ENOMEM: return "workspace too small";
        case RTE_EDEVICE: return "HIP runtime error";
        case RTE_EUNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char *rte_last_device_error(void) {
    return g_last_hip == hipSuccess ? "" : hipGetErrorString(g_last_hip);
}

int rte_problem_create(const rte_problem_desc *d, rte_problem **out) {
    return rte_problem_create_sched(d, 0, 0, 0, out);
}

int rte_problem_create_tuned(const rte_problem_desc *d, int dg, int wpb, rte_problem **out) {
    return rte_problem_create_sched(d, dg, wpb, 0, out);
}

int rte_problem_create_sched(const rte_problem_desc *d, int dg, int wpb, int bands,
                             rte_problem **out) {
    if (!d || !out) return RTE_EINVAL;
    if (bands < 0 || bands > 16) return RTE_EINVAL;
    *out = nullptr;
    if (d->dim != 1 && d->dim != 2) return RTE_EINVAL;
    if (d->nx < 1 || d->ny < 1 || d->batch < 1 || d->n_dir < 1) return RTE_EINVAL;
    if (d->dim == 1 && d->ny != 1) return RTE_EINVAL;
    if (!d->dir_x || !d->weight) return RTE_EINVAL;
    if (d->dim == 2 && !d->dir_y) return RTE_EINVAL;
    if (d->dim == 1 && !d->widths) return RTE_EINVAL;
    if (!d->sigma_t || !d->sigma_s || !d->source || !d->inflow) return RTE_EINVAL;
    if (dg != 0 && dg != 1 && dg != 2 && dg != 4 && dg != 8) return RTE_EINVAL;
    if (wpb < 0 || wpb > 4) return RTE_EINVAL;
    if ((long long)d->nx * d->ny > (1ll << 31)) return RTE_EUNSUPPORTED;
    double wsum = 0.0;
    for (int j = 0; j < d->n_dir; ++j) {
        if (!finite_pos(d->weight[j]) || !std::isfinite(d->dir_x[j])) return RTE_EINVAL;
        if (d->dim == 2 && !std::isfinite(d->dir_y[j])) return RTE_EINVAL;
        if (d->dim == 2 && d->dir_x[j] == 0.0 && d->dir_y[j] == 0.0) return RTE_EINVAL;
        if (d->dim == 1 && d->dir_x[j] == 0.0) return RTE_EINVAL;
        wsum += d->weight[j];
    }
    if (std::fabs(wsum - 1.0) > 1e-12) return RTE_EINVAL;
    if (d->dim == 2 && (!finite_pos(d->lx) || !finite_pos(d->ly))) return RTE_EINVAL;
    if (d->dim == 1)
        for (int i = 0; i < d->nx; ++i)
            if (!finite_pos(d->widths[i])) return RTE_EINVAL;

    rte_problem *p = new (std::nothrow) rte_problem();
    if (!p) return RTE_ENOMEM;
    p->dim = d->dim;
    p->nx = d->nx;
    p->ny = d->ny;
    p->B = d->batch;
    p->n_dir = d->n_dir;
    p->K = d->dim == 2 ? 4 : 2;
    p->ncell = (long long)d->nx * d->ny;
    p->ndof = p->ncell * p->K;
    p->lx = d->lx;
    p->ly = d->ly;
    p->hx = d->dim == 2 ? d->lx / d->nx : 1.0;
    p->hy = d->dim == 2 ? d->ly / d->ny : 1.0;
    p->vx.assign(d->dir_x, d->dir_x + d->n_dir);
    p->w.assign(d->weight, d->weight + d->n_dir);
    if (d->dim == 2) p->vy.assign(d->dir_y, d->dir_y + d->n_dir);
    else p->vy.assign(d->n_dir, 0.0);
    if (d->dim == 1) p->widths.assign(d->widths, d->widths + d->nx);
    p->sigma_t = d->sigma_t;
    p->sigma_s = d->sigma_s;
    p->source = d->source;
    p->inflow = d->inflow;
    p->cxx = p->cyy = p->kmin_x = p->kmin_y = p->c1 = p->c2 = p->c3 = 0.0;
    for (int j = 0; j < d->n_dir; ++j) {
        const double vx = p->vx[j], vy = p->vy[j], w = p->w[j];
        p->cxx += w * vx * vx;
        p->cyy += w * vy * vy;
        if (vx > 0) p->kmin_x += w * vx;
        if (vy > 0) p->kmin_y += w * vy;
        if (vx > 0) { p->c1 += w * vx; p->c3 += w * vx * vx * vx; }
        p->c2 += w * vx * vx;
    }
    p->d_dirs = nullptr;
    p->d_mu = p->d_w = p->d_widths = nullptr;
    p->d_vxy = nullptr;
    p->dsa_mg = 1;
    {
        int dev = 0, ncu = 0, lds = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) {
            delete p;
            return device_error(e);
        }
        p->n_cu = ncu > 0 ? ncu : 1;
        p->lds_per_cu = lds > 0 ? lds : 64 * 1024;
    }
    // quadrant-sorted, padded direction table (2D)
    std::vector<DirEntry> table;
    for (int q = 0; q < 4; ++q) p->quad.count[q] = 0;
    if (d->dim == 2) {
        std::vector<int> idx[4];
        for (int j = 0; j < d->n_dir; ++j) {
            const int q = (p->vx[j] < 0 ? 1 : 0) | (p->vy[j] < 0 ? 2 : 0);
            idx[q].push_back(j);
        }
        for (int q = 0; q < 4; ++q) {
            p->quad.start[q] = (int)table.size();
            p->quad.count[q] = (int)idx[q].size();
            for (int j : idx[q]) {
                DirEntry e;
                e.alpha = std::fabs(p->vx[j]) / p->hx;
                e.beta = std::fabs(p->vy[j]) / p->hy;
                e.w = p->w[j];
                e.orig = j;
                e.pad = 0;
                table.push_back(e);
            }
            while (table.size() % kQuadPad) {
                DirEntry e;
                e.alpha = 1.0;
                e.beta = 1.0;
                e.w = 0.0;
                e.orig = -1;
                e.pad = 0;
                table.push_back(e);
            }
        }
    }
    p->n_sorted = (int)table.size();
    choose_tuning(p, dg, wpb, bands);
    // the sweep's table kernels need dynamic LDS past 64 KiB (set once, outside any capture)
    {
        static std::once_flag lds_once;
        const int lds_max = p->lds_per_cu;
        std::call_once(lds_once, [lds_max] { sweep_lds_limits(lds_max); });
    }
    hipError_t e = hipSuccess;
    auto upload = [&](auto **dst, const void *src, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc((void **)dst, bytes);
        if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    if (!table.empty()) upload(&p->d_dirs, table.data(), table.size() * sizeof(DirEntry));
    upload(&p->d_w, p->w.data(), sizeof(double) * p->n_dir);
    if (d->dim == 1) {
        upload(&p->d_mu, p->vx.data(), sizeof(double) * p->n_dir);
        upload(&p->d_widths, p->widths.data(), sizeof(double) * p->nx);
    }
    if (d->dim == 2) {
        std::vector<double> vxy(2 * (size_t)p->n_dir);
        for (int j = 0; j < p->n_dir; ++j) { vxy[j] = p->vx[j]; vxy[p->n_dir + j] = p->vy[j]; }
        upload(&p->d_vxy, vxy.data(), sizeof(double) * vxy.size());
    }
    if (e != hipSuccess) {
        rte_problem_destroy(p);
        return device_error(e);
    }
    *out = p;
    return RTE_OK;
}

void rte_problem_destroy(rte_problem *p) {
    if (!p) return;
    if (p->d_dirs) (void)hipFree(p->d_dirs);
    if (p->d_w) (void)hipFree(p->d_w);
    if (p->d_mu) (void)hipFree(p->d_mu);
    if (p->d_widths) (void)hipFree(p->d_widths);
    if (p->d_vxy) (void)hipFree(p->d_vxy);
    delete p->iter_graph;
    delete p->precond_graphs;
    delete p;
}

int rte_problem_dsa_multigrid(rte_problem *p, int on) {
    if (!p) return RTE_EINVAL;
    p->dsa_mg = on != 0;
    return RTE_OK;
}

int rte_problem_tuning(const rte_problem *p, int *dg, int *wpb, int *nparts) {
    if (!p) return RTE_EINVAL;
    if (dg) *dg = p->tune.dg;
    if (wpb) *wpb = p->tune.wpb;
    if (nparts) *nparts = p->dim == 2 ? nparts_for(p) : 0;
    return RTE_OK;
}

int rte_problem_bands(const rte_problem *p, int *bands) {
    if (!p || !bands) return RTE_EINVAL;
    *bands = sweep_bands(p);
    return RTE_OK;
}

int rte_workspace_size(const rte_problem *p, rte_mode mode, const rte_rom *rom,
                       rte_precision prec, int max_iter, size_t *bytes) {
    if (!p || !bytes || max_iter < 0) return RTE_EINVAL;
    if (mode != RTE_SI && mode != RTE_SI_DSA && mode != RTE_ROMSAD) return RTE_EINVAL;
    if (prec != RTE_FP64 && prec != RTE_MIXED) return RTE_EINVAL;
    Carver c(nullptr, 0);
    carve(c, p, mode, rom, prec, max_iter);
    *bytes = c.off;
    return RTE_OK;
}

int rte_pgmres_workspace_size(const rte_problem *p, int restart, size_t *bytes) {
    if (!p || !bytes || restart < 1 || restart > 200) return RTE_EINVAL;
    Carver c(nullptr, 0);
    carve(c, p, RTE_SI_DSA, nullptr, RTE_FP64, 1, restart);
    *bytes = c.off;
    return RTE_OK;
}

int rte_problem_check(const rte_problem *p, void *ws, size_t ws_bytes, rte_stream_t stream) {
    if (!p || !ws) return RTE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    Layout L = carve(c, p, RTE_SI, nullptr, RTE_FP64, 1);
    if (!c.ok) return RTE_ENOMEM;
    HIPCHK(launch_fill_int(L.flag, 1, 0, s));
    HIPCHK(launch_check_materials(p, L.flag, s));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, L.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return bad ? RTE_EINVAL : RTE_OK;
}

int rte_rom_create(const rte_problem *p, const rte_rom_desc *d, rte_rom **out) {
    if (!p || !d || !out) return RTE_EINVAL;
    *out = nullptr;
    if (d->r < 1 || d->r > 64 || d->m < 0) return RTE_EINVAL;
    if (!d->U_rho || !d->U_iso || !d->A0 || (d->m > 0 && !d->A)) return RTE_EINVAL;
    const size_t nu = (size_t)p->ndof * d->r;
    for (size_t i = 0; i < nu; ++i)
        if (!std::isfinite(d->U_rho[i]) || !std::isfinite(d->U_iso[i])) return RTE_EINVAL;
    rte_rom *r = new (std::nothrow) rte_rom();
    if (!r) return RTE_ENOMEM;
    r->r = d->r;
    r->m = d->m;
    r->ndof = p->ndof;
    r->eps_pod = d->eps_pod;
    r->eps_train = d->eps_train;
    static std::atomic<unsigned long long> rom_serial{0};
    r->serial = ++rom_serial;
    r->d_U_rho = r->d_U_iso = r->d_A0 = r->d_A = r->d_b_in = nullptr;
    r->d_U_rho_f = r->d_U_iso_f = nullptr;
    std::vector<float> tmp(nu);
    bool ok = true;
    ok = ok && hipMalloc(&r->d_U_rho, nu * 8) == hipSuccess;
    ok = ok && hipMalloc(&r->d_U_iso, nu * 8) == hipSuccess;
    ok = ok && hipMalloc(&r->d_U_rho_f, nu * 4) == hipSuccess;
    ok = ok && hipMalloc(&r->d_U_iso_f, nu * 4) == hipSuccess;
    ok = ok && hipMalloc(&r->d_A0, (size_t)d->r * d->r * 8) == hipSuccess;
    ok = ok && hipMalloc(&r->d_A, std::max<size_t>(1, (size_t)d->m * d->r * d->r) * 8) == hipSuccess;
    ok = ok && hipMalloc(&r->d_b_in, (size_t)4 * d->r * 8) == hipSuccess;
    {
        std::vector<double> bin((size_t)4 * d->r, 0.0);
        if (d->b_inflow)
            for (size_t i = 0; i < bin.size(); ++i) bin[i] = d->b_inflow[i];
        ok = ok && hipMemcpy(r->d_b_in, bin.data(), bin.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
    }
    ok = ok && hipMemcpy(r->d_U_rho, d->U_rho, nu * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(r->d_U_iso, d->U_iso, nu * 8, hipMemcpyHostToDevice) == hipSuccess;
    for (size_t i = 0; ok && i < nu; ++i) tmp[i] = (float)d->U_rho[i];
    ok = ok && hipMemcpy(r->d_U_rho_f, tmp.data(), nu * 4, hipMemcpyHostToDevice) == hipSuccess;
    for (size_t i = 0; ok && i < nu; ++i) tmp[i] = (float)d->U_iso[i];
    ok = ok && hipMemcpy(r->d_U_iso_f, tmp.data(), nu * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(r->d_A0, d->A0, (size_t)d->r * d->r * 8, hipMemcpyHostToDevice) == hipSuccess;
    if (d->m > 0)
        ok = ok && hipMemcpy(r->d_A, d->A, (size_t)d->m * d->r * d->r * 8, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        rte_rom_destroy(r);
        return RTE_EDEVICE;
    }
    *out = r;
    return RTE_OK;
}

void rte_rom_destroy(rte_rom *r) {
    if (!r) return;
    if (r->d_U_rho) (void)hipFree(r->d_U_rho);
    if (r->d_U_iso) (void)hipFree(r->d_U_iso);
    if (r->d_b_in) (void)hipFree(r->d_b_in);
    if (r->d_U_rho_f) (void)hipFree(r->d_U_rho_f);
    if (r->d_U_iso_f) (void)hipFree(r->d_U_iso_f);
    if (r->d_A0) (void)hipFree(r->d_A0);
    if (r->d_A) (void)hipFree(r->d_A);
    delete r;
}

}  // extern "C"

namespace {

// one sweep of every active instance: src -> rho_star (+ change maxima against rho_prev)
// The material tables of the selected instances (all if mask is null) for this call's sweeps
bool mat_usable(const rte_problem *p, const Layout &L, int fp32) {
    return p->dim == 2 && L.mat && sweep_mat_fits(p, fp32 ? sizeof(float) : sizeof(double));
}

int prepare_materials(const rte_problem *p, Layout &L, const int *mask, int fp32, hipStream_t s) {
    L.use_mat = false;
    if (!mat_usable(p, L, fp32)) return RTE_OK;
    HIPCHK(launch_materials(p, mask, L.mat, L.mat_ok, L.nmat, L.mvals, L.mcvals, L.mcoef, fp32,
                            s));
    L.use_mat = true;
    return RTE_OK;
}

int do_sweep(const rte_problem *p, const Layout &L, const void *src, void *f_out,
             double *rho_star, const double *rho_prev, const int *active, int zero_inflow,
             int fp32, hipStream_t s) {
    if (p->dim == 2) {
        // the f stores address one direction's array with 32-bit byte offsets
        if (f_out && p->ncell >= (1LL << 26)) return RTE_EUNSUPPORTED;
        SweepLaunch a;
        a.p = p;
        a.src = src;
        a.partial = rho_star ? L.partial : nullptr;
        a.f_out = f_out;
        a.active = active;
        a.zero_inflow = zero_inflow;
        a.fp32 = fp32;
        if (L.use_mat) {
            a.mat_ok = L.mat_ok;
            a.mat_coef = L.mcoef;
        }
        {
            ProfScope ps(RTE_PROF_SWEEP2D, s);
            HIPCHK(launch_sweep2d(a, s));
        }
        ProfScope ps(RTE_PROF_REDUCE, s);
        if (rho_star)
            HIPCHK(launch_reduce_parts(p, L.partial, nparts_for(p), rho_star, rho_prev,
                                       rho_prev ? L.st.maxd : nullptr,
                                       rho_prev ? L.st.maxr : nullptr, active, s));
    } else {
        void *f = f_out ? f_out : L.fscratch;
        {
            ProfScope ps(RTE_PROF_SWEEP1D, s);
            HIPCHK(launch_sweep1d(p, src, f, active, zero_inflow, fp32, s));
        }
        if (rho_star)
            HIPCHK(launch_scalar_flux(p, f, rho_star, fp32, rho_prev,
                                      rho_prev ? L.st.maxd : nullptr,
                                      rho_prev ? L.st.maxr : nullptr, active, s));
    }
    return RTE_OK;
}

// diffusion correction for the instances whose kind equals `want` (all if kind == nullptr)
// guess (nullable): each instance's previous correction, the warm-start direction of the CG
int do_dsa(const rte_problem *p, const Layout &L, const double *rho_star, const double *rho_prev,
           double *delta, const int *kind, int want, double rtol, int maxit, int *iters_out,
           int *failed, const double *guess, hipStream_t s) {
    ProfScope ps(RTE_PROF_DSA, s);
    if (p->dim == 1) {
        HIPCHK(launch_dsa1d(p, rho_star, rho_prev, delta, kind, want, L.dsa1d, s));
        return RTE_OK;
    }
    // the CG iterates in the output itself (the call's last kernel then only gathers its
    // statistics), unless the output is one of the inputs
    CGSpace cg = L.cg;
    if (delta != rho_star && delta != rho_prev) cg.x = delta;
    // the multigrid hierarchy depends only on the materials: built by the caller once
    HIPCHK(launch_cg_setup(p, cg, rho_star, rho_prev, kind, want, guess, rtol, s));
    // A look at the number of running instances drains the queue, and an iteration launched
    // after every instance stopped still costs its launches (its kernels return at once).  So
    // the host first looks after the iteration at which the previous solve of this call was seen
    // finished (after iteration 8 for the first), then after every iteration.  When the first look
    // already finds every instance stopped, the next solve looks one iteration earlier, so the
    // look follows iteration counts that shrink as well as grow.
    const int first = L.cg_look > 0 ? L.cg_look : 8;
    int counts[2] = {1, 0};       // running, failed
    for (int it = 1; it <= maxit + 1; ++it) {
        HIPCHK(launch_cg_iteration(p, cg, it, rtol, maxit, s));
        if (it >= first || it == maxit + 1) {
            HIPCHK(hipMemcpyAsync(counts, L.cg.n_running, sizeof(counts), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (counts[0] == 0) {
                L.cg_look = it == first ? std::max(2, it - 1) : it;
                break;
            }
        }
    }
    // iteration maxit + 1 stops every instance still running and counts it as failed
    if (failed) *failed = counts[0] != 0 || counts[1] != 0;
    HIPCHK(launch_cg_finish(p, cg, delta, iters_out, L.cg_total, s));
    return RTE_OK;
}


// The multigrid preconditioner as graphs for one long call: the handle's cached capture for this
// carve-up, or a new one (kept for the next call).  The graphs stay alive while the call holds
// them; the kernels run one by one when capture is off or fails.
struct PrecondGraphs {
    CGSpace &c;
    std::shared_ptr<rte_precond_graphs::Exec> ex;
    PrecondGraphs(const rte_problem *p, CGSpace &cg, bool on,
                  const rte_precond_graphs::Key &k) : c(cg) {
        c.precond[0] = c.precond[1] = nullptr;
        if (!on || c.mg.L == 0) return;
        if (!p->precond_graphs) {
            p->precond_graphs = new (std::nothrow) rte_precond_graphs();
            if (!p->precond_graphs) return;
        }
        rte_precond_graphs &G = *p->precond_graphs;
        std::lock_guard<std::mutex> lock(G.mu);
        if (!(G.valid && G.key == k)) {
            G.valid = false;
            G.cur.reset();
            CGSpace tmp = c;
            mg_precond_capture(p, tmp);
            if (!tmp.precond[0] || !tmp.precond[1]) {
                mg_precond_release(tmp);
                return;
            }
            auto e = std::make_shared<rte_precond_graphs::Exec>();
            e->g[0] = tmp.precond[0];
            e->g[1] = tmp.precond[1];
            G.cur = e;
            G.key = k;
            G.valid = true;
        }
        ex = G.cur;
        c.precond[0] = ex->g[0];
        c.precond[1] = ex->g[1];
    }
    ~PrecondGraphs() { c.precond[0] = c.precond[1] = nullptr; }
};

rte_precond_graphs::Key precond_key(int caller, const rte_problem *p, const Layout &L,
                                    const void *ws, size_t ws_bytes, int mode, int precision,
                                    int max_iter, const rte_rom *rom) {
    rte_precond_graphs::Key k{};
    k.caller = caller;
    k.ws = ws;
    k.ws_bytes = ws_bytes;
    k.mode = mode;
    k.precision = precision;
    k.max_iter = max_iter;
    k.mg = p->dsa_mg;
    k.rom = rom ? rom->serial : 0ull;
    k.z = L.cg.z;
    k.t = L.cg.mg.t;
    k.part = L.cg.part;
    return k;
}

// psi is checked only where the ROM correction runs (need_psi)
int check_solve_args(const rte_problem *p, rte_mode mode, const rte_rom *rom, const double *psi,
                     bool need_psi, const rte_solve_opts *o) {
    if (!p || !o) return RTE_EINVAL;
    if (mode != RTE_SI && mode != RTE_SI_DSA && mode != RTE_ROMSAD) return RTE_EINVAL;
    if (mode == RTE_ROMSAD && (!rom || rom->ndof != p->ndof)) return RTE_EINVAL;
    if (mode == RTE_ROMSAD && need_psi && rom->m > 0 && !psi) return RTE_EINVAL;
    if (!(o->eps >= 0.0) || o->max_iter < 1 || o->theta < 0) return RTE_EINVAL;
    if (o->precision != RTE_FP64 && o->precision != RTE_MIXED) return RTE_EINVAL;
    if (mode != RTE_SI && p->dim == 2 && (!(o->cg_rtol > 0.0) || o->cg_maxit < 1)) return RTE_EINVAL;
    return RTE_OK;
}

// One outer iteration of Alg. 1 (Alg. 2 for ROMSAD) for every active instance, enqueued with no
// host read: the sweep and its reduction, the stop test and choice of correction, ROMSA for the
// instances that chose it (a singular reduced system turns its instance into a DSA one on the
// device), the diffusion correction for the DSA instances, and the update.  The 2D diffusion CG
// runs `depth` iterations (an instance that converges stops inside and its kernels return at
// once); iteration depth + 1 stops any instance still running and counts it as failed.
int enqueue_iteration(const rte_problem *p, const Layout &L, rte_mode mode, const rte_rom *rom,
                      const double *psi, const rte_solve_opts *o, double eps_romsad, double *rho,
                      void *f_out, int depth, hipStream_t s) {
    const int fp32 = o->precision == RTE_MIXED;
    const bool corrected = mode != RTE_SI;
    int rc = do_sweep(p, L, L.src, f_out, L.rho_star, rho, L.st.active, 0, fp32, s);
    if (rc) return rc;
    HIPCHK(launch_decide(p, L.st, o->max_iter, o->eps, o->relative, (int)mode, o->theta,
                         eps_romsad, s));
    if (mode == RTE_ROMSAD)
        HIPCHK(launch_rom_correct(p, rom, psi, L.rho_star, rho, L.delta, L.rom_status, L.st.kind,
                                  2, L.rom, fp32, s));
    if (corrected) {
        if (p->dim == 1) {
            HIPCHK(launch_dsa1d(p, L.rho_star, rho, L.delta, L.st.kind, 1, L.dsa1d, s));
        } else {
            CGSpace cg = L.cg;
            cg.x = L.delta;                       // the CG iterates in the correction itself
            HIPCHK(launch_cg_setup(p, cg, L.rho_star, rho, L.st.kind, 1, L.delta, o->cg_rtol, s));
            for (int it = 1; it <= depth + 1; ++it)
                HIPCHK(launch_cg_iteration(p, cg, it, o->cg_rtol, depth, s));
            HIPCHK(launch_cg_finish(p, cg, L.delta, L.cg.iters, L.cg_total, s));
        }
    }
    HIPCHK(launch_update(p, L.st, L.rho_star, corrected ? L.delta : nullptr, rho, L.src, fp32, s));
    return RTE_OK;
}

// The handle's outer-iteration graph for these arguments: the cached one, or a new capture of
// enqueue_iteration on the handle's capture stream.
int iteration_graph(const rte_problem *p, const Layout &L, rte_mode mode, const rte_rom *rom,
                    const double *psi, const rte_solve_opts *o, double eps_romsad, double *rho,
                    void *f_out, const void *ws, size_t ws_bytes,
                    std::shared_ptr<rte_iter_graph::Exec> *out) {
    if (!p->iter_graph) {
        p->iter_graph = new (std::nothrow) rte_iter_graph();
        if (!p->iter_graph) return RTE_ENOMEM;
    }
    rte_iter_graph &G = *p->iter_graph;
    const int depth = mode != RTE_SI && p->dim == 2 ? std::min(o->cg_maxit, o->graph_cg_iters) : 0;
    rte_iter_graph::Key k{ws, ws_bytes, (int)mode, rom ? rom->serial : 0ull, psi, rho, f_out,
                          o->eps, eps_romsad, mode != RTE_SI ? o->cg_rtol : 0.0, o->max_iter,
                          o->relative, o->theta, (int)o->precision, depth};
    std::lock_guard<std::mutex> lock(G.mu);
    if (G.valid && G.key == k) {
        *out = G.cur;
        return RTE_OK;
    }
    G.valid = false;
    G.cur.reset();
    if (!G.cs) HIPCHK(hipStreamCreateWithFlags(&G.cs, hipStreamNonBlocking));
    auto ex = std::make_shared<rte_iter_graph::Exec>();
    HIPCHK(hipHostMalloc((void **)&ex->h_active, 2 * sizeof(int), hipHostMallocDefault));
    for (hipEvent_t &e : ex->ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // the library's per-kernel event timing stays out of the graph
    const bool prof_off = t_prof_off;
    t_prof_off = true;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(G.cs, hipStreamCaptureModeThreadLocal);
    int rc = RTE_OK;
    if (e == hipSuccess) {
        rc = enqueue_iteration(p, L, mode, rom, psi, o, eps_romsad, rho, f_out, depth, G.cs);
        const hipError_t ee = hipStreamEndCapture(G.cs, &g);
        if (ee != hipSuccess && rc == RTE_OK) rc = device_error(ee);
    } else {
        rc = device_error(e);
    }
    t_prof_off = prof_off;
    if (rc == RTE_OK && g) {
        e = hipGraphInstantiate(&ex->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = device_error(e);
    } else if (rc == RTE_OK) {
        rc = RTE_EDEVICE;
    }
    if (g) (void)hipGraphDestroy(g);
    if (rc) return rc;
    G.key = k;
    G.cur = ex;
    G.valid = true;
    *out = ex;
    return RTE_OK;
}

// Graph mode of run_iterations: one graph launch per outer iteration.  After every poll_every-th
// launch the active count is copied to pinned host memory behind an event; the host waits for
// that event only after it has queued the next launch, so the device never idles on the read.
// Launches after every instance stopped change nothing (every kernel is predicated on the
// instance's state).
int run_graph_iterations(const rte_problem *p, const Layout &L, rte_mode mode, const rte_rom *rom,
                         const double *psi, const rte_solve_opts *o, double eps_romsad,
                         double *rho, void *f_out, int n_max, const void *ws, size_t ws_bytes,
                         hipStream_t s, int *iterations, bool *cg_failed) {
    std::shared_ptr<rte_iter_graph::Exec> ex;
    int rc = iteration_graph(p, L, mode, rom, psi, o, eps_romsad, rho, f_out, ws, ws_bytes, &ex);
    if (rc) return rc;
    const int poll = o->poll_every > 0 ? o->poll_every : 1;
    int pending = -1;                       // slot of the last poll not yet read
    for (int l = 1; l <= n_max; ++l) {
        HIPCHK(hipGraphLaunch(ex->exec, s));
        *iterations = l;
        if (l % poll != 0 && l != n_max) continue;
        const int slot = l & 1;
        HIPCHK(hipMemcpyAsync(ex->h_active + slot, L.st.n_active, sizeof(int),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(ex->ev[slot], s));
        if (pending >= 0) {
            HIPCHK(hipEventSynchronize(ex->ev[pending]));
            if (ex->h_active[pending] == 0) break;
        }
        pending = slot;
    }
    int fails = 0;
    HIPCHK(hipMemcpyAsync(&fails, L.cg_fail, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *cg_failed = *cg_failed || fails > 0;
    return RTE_OK;
}

// Up to n_max outer iterations (Alg. 1; Alg. 2 for ROMSAD) of every active instance; returns
// early once no instance is active.  SI looks at the active count every poll_every iterations.
// The modes with a diffusion solve wait on the device inside every iteration anyway, so they
// read the decision's counts at once: a correction no instance takes is not launched, and the
// loop ends with the iteration in which the last instance stopped.
int run_iterations(const rte_problem *p, const Layout &L, rte_mode mode, const rte_rom *rom,
                   const double *psi, const rte_solve_opts *o, double *rho, void *f_out, int n_max,
                   const void *ws, size_t ws_bytes, hipStream_t s, int *iterations,
                   bool *cg_failed) {
    const int fp32 = o->precision == RTE_MIXED;
    double eps_romsad = o->eps_romsad;
    if (mode == RTE_ROMSAD && eps_romsad < 0.0)
        eps_romsad = 0.1 * std::max(rom->eps_train, rom->eps_pod);   // eq. (romsad_parameters)
    HIPCHK(launch_fill_int(L.cg_fail, 1, 0, s));
    if (o->graph_cg_iters > 0)
        return run_graph_iterations(p, L, mode, rom, psi, o, eps_romsad, rho, f_out, n_max, ws,
                                    ws_bytes, s, iterations, cg_failed);
    const int poll = o->poll_every > 0 ? o->poll_every : 1;
    const bool corrected = mode != RTE_SI;
    int counts[3] = {1, 1, 1};                // active, taking DSA, taking ROMSA
    for (int l = 1; l <= n_max; ++l) {
        int rc = do_sweep(p, L, L.src, f_out, L.rho_star, rho, L.st.active, 0, fp32, s);
        if (rc) return rc;
        HIPCHK(launch_decide(p, L.st, o->max_iter, o->eps, o->relative, (int)mode, o->theta,
                             eps_romsad, s));
        if (corrected) {
            HIPCHK(hipMemcpyAsync(counts, L.st.n_active, sizeof(counts), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        // L.delta holds every instance's previous correction (zero before its first)
        const double *delta = corrected ? L.delta : nullptr;
        // a singular reduced system sends its instance to DSA (kind 1) and adds it to the DSA
        // count on the device; when the decision sent none there, the count is read again
        bool need_dsa = corrected && counts[1] > 0;
        if (mode == RTE_ROMSAD && counts[2] > 0) {
            {
                ProfScope ps(RTE_PROF_ROM, s);
                HIPCHK(launch_rom_correct(p, rom, psi, L.rho_star, rho, L.delta, L.rom_status,
                                          L.st.kind, 2, L.rom, fp32, s));
            }
            if (!need_dsa) {
                int n_dsa = 0;
                HIPCHK(hipMemcpyAsync(&n_dsa, L.st.n_active + 1, sizeof(int),
                                      hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                need_dsa = n_dsa > 0;
            }
        }
        if (need_dsa) {
            int failed = 0;
            rc = do_dsa(p, L, L.rho_star, rho, L.delta, L.st.kind, 1, o->cg_rtol, o->cg_maxit,
                        L.cg.iters, &failed, L.delta, s);
            if (rc) return rc;
            *cg_failed = *cg_failed || failed;
        }
        HIPCHK(launch_update(p, L.st, L.rho_star, delta, rho, L.src, fp32, s));
        *iterations = l;
        if (corrected) {
            if (counts[0] == 0) break;
        } else if (l % poll == 0 || l == n_max) {
            int n_active = 0;
            HIPCHK(hipMemcpyAsync(&n_active, L.st.n_active, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (n_active == 0) break;
        }
    }
    return RTE_OK;
}

// host-visible results, copied on the solve's stream only (other streams keep running)
int finish_stats(const rte_problem *p, const Layout &L, int max_iter, int iterations,
                 bool cg_failed, int *active_out, rte_solve_stats *stats, hipStream_t s) {
    std::vector<int> status(p->B);
    const auto d2h = hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(status.data(), L.st.status, sizeof(int) * p->B, d2h, s));
    if (active_out) HIPCHK(hipMemcpyAsync(active_out, L.st.active, sizeof(int) * p->B, d2h, s));
    if (stats) {
        if (stats->n_sweep)
            HIPCHK(hipMemcpyAsync(stats->n_sweep, L.st.n_sweep, sizeof(int) * p->B, d2h, s));
        if (stats->change)
            HIPCHK(hipMemcpyAsync(stats->change, L.st.change, sizeof(double) * p->B * max_iter, d2h, s));
        if (stats->kind)
            HIPCHK(hipMemcpyAsync(stats->kind, L.st.kinds, sizeof(int) * p->B * max_iter, d2h, s));
    }
    unsigned long long cg_total = 0;
    HIPCHK(hipMemcpyAsync(&cg_total, L.cg_total, sizeof(cg_total), d2h, s));
    HIPCHK(hipStreamSynchronize(s));
    int rc = RTE_OK;
    for (int b = 0; b < p->B; ++b)
        if (status[b] != RTE_OK) rc = RTE_ENOCONV;
    if (stats) {
        if (stats->status) std::memcpy(stats->status, status.data(), sizeof(int) * p->B);
        stats->cg_iterations = (long long)cg_total;
        stats->iterations = iterations;
    }
    if (cg_failed) rc = RTE_ECG;      // an inexact correction outranks an iteration limit
    return rc;
}

}  // namespace

// One sweep of rte_sweep.  prepare: form the material tables first (else the ones an earlier
// call formed in this workspace are used).
int sweep_call(const rte_problem *p, const double *rho_in, void *f_out, double *rho_star_out,
               int zero_inflow, rte_precision prec, void *ws, size_t ws_bytes, hipStream_t s,
               bool prepare) {
    Carver c(ws, ws_bytes);
    Layout L = carve(c, p, RTE_SI, nullptr, prec, 1);
    if (!c.ok) return RTE_ENOMEM;
    const int fp32 = prec == RTE_MIXED;
    if (prepare) {
        const int rc = prepare_materials(p, L, nullptr, fp32, s);
        if (rc) return rc;
    } else {
        L.use_mat = mat_usable(p, L, fp32);
    }
    HIPCHK(launch_source(p, rho_in, L.src, nullptr, fp32, s, true, L.use_mat ? L.mat : nullptr,
                         L.mat_ok));
    return do_sweep(p, L, L.src, f_out, rho_star_out, nullptr, nullptr, zero_inflow, fp32, s);
}

extern "C" {

int rte_sweep(const rte_problem *p, const double *rho_in, void *f_out, double *rho_star_out,
              int zero_inflow, rte_precision prec, void *ws, size_t ws_bytes, rte_stream_t stream) {
    if (!p || !rho_in || (!f_out && !rho_star_out) || !ws) return RTE_EINVAL;
    if (prec != RTE_FP64 && prec != RTE_MIXED) return RTE_EINVAL;
    return sweep_call(p, rho_in, f_out, rho_star_out, zero_inflow, prec, ws, ws_bytes,
                      (hipStream_t)stream, true);
}

}  // extern "C"

namespace {

// Device memory of rte_sweep_noalloc: the sweep's input block, partial densities and material
// tables live here instead of in a caller workspace.  Each device that loads the library holds its own copy for
// the life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name on the host is a stand-in, not
// a device address).  Nothing in it has to start at zero: the material kernels write every
// table value they or the sweep read, the source kernel writes the whole input block, and every
// partial slot is written in full by the sweep before it is reduced.
static __device__ __align__(256) unsigned char scratch[RTE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
struct ScratchAddr {
    std::once_flag once;
    void *ptr = nullptr;
    hipError_t err = hipSuccess;
};
ScratchAddr g_scratch_addr[kMaxScratchDevices];

// the current device's address of `scratch`, looked up once per device with that device current
int scratch_address(void **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return RTE_EUNSUPPORTED;
    ScratchAddr &a = g_scratch_addr[dev];
    std::call_once(a.once, [&a] {
        void *ptr = nullptr;
        a.err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (a.err == hipSuccess) a.ptr = ptr;
    });
    if (a.err != hipSuccess) return device_error(a.err);
    if (!a.ptr) return RTE_EDEVICE;
    *out = a.ptr;
    return RTE_OK;
}

}  // namespace

extern "C" {

int rte_sweep_noalloc(const rte_problem *p, const double *rho_in, void *f_out, double *rho_star_out,
                      int zero_inflow, rte_precision prec, rte_stream_t stream) {
    if (!p || !rho_in || (!f_out && !rho_star_out)) return RTE_EINVAL;
    if (prec != RTE_FP64 && prec != RTE_MIXED) return RTE_EINVAL;
    size_t need = 0;
    {
        Carver sizing(nullptr, 0);
        carve(sizing, p, RTE_SI, nullptr, prec, 1);
        need = sizing.off;
    }
    if (need > (size_t)RTE_NOALLOC_SCRATCH_BYTES) return RTE_ENOMEM;
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    // rte_sweep's kernels, material tables included (the material kernels write every value
    // they or the sweep read, so nothing left by an earlier call matters)
    return sweep_call(p, rho_in, f_out, rho_star_out, zero_inflow, prec, ws,
                      (size_t)RTE_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream, true);
}

int rte_tune_sweep(const rte_problem_desc *desc, rte_precision prec, int n_cand, const int *dg,
                   const int *wpb, const int *bands, const double *rho_in, void *f_out,
                   int warmup, int reps, double *ms_out, rte_stream_t stream) {
    if (!desc || !dg || !wpb || !rho_in || !ms_out || n_cand < 1 || warmup < 0 || reps < 1)
        return RTE_EINVAL;
    if (prec != RTE_FP64 && prec != RTE_MIXED) return RTE_EINVAL;
    if (desc->dim != 2) return RTE_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < n_cand; ++i) ms_out[i] = -1.0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (hipEvent_t &e : ev) HIPCHK(hipEventCreate(&e));
    int rc = RTE_OK;
    for (int i = 0; i < n_cand && rc == RTE_OK; ++i) {
        if (dg[i] < 1 || wpb[i] < 1 || (bands && bands[i] < 1)) continue;
        rte_problem *p = nullptr;
        const int cr = rte_problem_create_sched(desc, dg[i], wpb[i], bands ? bands[i] : 1, &p);
        if (cr == RTE_EINVAL) continue;                       // not a schedule the sweep has
        if (cr != RTE_OK) { rc = cr; break; }
        // a schedule the LDS budget would change is not this candidate
        if (p->tune.dg != dg[i] || p->tune.wpb != wpb[i] ||
            (bands && sweep_bands_used(p, prec) != bands[i])) {
            rte_problem_destroy(p);
            continue;
        }
        size_t bytes = 0;
        rte_workspace_size(p, RTE_SI, nullptr, prec, 1, &bytes);
        void *ws = nullptr;
        double *rs = nullptr;
        hipError_t e = hipMalloc(&ws, bytes);
        if (e == hipSuccess) e = hipMalloc((void **)&rs, sizeof(double) * (size_t)p->B * p->ndof);
        if (e != hipSuccess) rc = device_error(e);
        // the material tables once, as a solve forms them once; then the timed sweeps
        if (rc == RTE_OK) rc = sweep_call(p, rho_in, f_out, rs, 0, prec, ws, bytes, s, true);
        for (int k = 0; k < warmup && rc == RTE_OK; ++k)
            rc = sweep_call(p, rho_in, f_out, rs, 0, prec, ws, bytes, s, false);
        if (rc == RTE_OK) rc = hipEventRecord(ev[0], s) == hipSuccess ? RTE_OK : RTE_EDEVICE;
        for (int k = 0; k < reps && rc == RTE_OK; ++k)
            rc = sweep_call(p, rho_in, f_out, rs, 0, prec, ws, bytes, s, false);
        if (rc == RTE_OK) {
            e = hipEventRecord(ev[1], s);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (e == hipSuccess) ms_out[i] = (double)ms / reps;
            else rc = device_error(e);
        }
        (void)hipStreamSynchronize(s);
        if (rs) (void)hipFree(rs);
        if (ws) (void)hipFree(ws);
        rte_problem_destroy(p);
    }
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    return rc;
}

int rte_scalar_flux(const rte_problem *p, const void *f, double *rho_out, rte_precision prec,
                    rte_stream_t stream) {
    if (!p || !f || !rho_out) return RTE_EINVAL;
    if (prec != RTE_FP64 && prec != RTE_MIXED) return RTE_EINVAL;
    HIPCHK(launch_scalar_flux(p, f, rho_out, prec == RTE_MIXED, nullptr, nullptr, nullptr, nullptr,
                              (hipStream_t)stream));
    return RTE_OK;
}

int rte_dsa_correct(const rte_problem *p, const double *rho_star, const double *rho_prev,
                    double *delta_rho, double cg_rtol, int cg_maxit, int *cg_iters_out, void *ws,
                    size_t ws_bytes, rte_stream_t stream) {
    if (!p || !rho_star || !rho_prev || !delta_rho || !ws) return RTE_EINVAL;
    if (p->dim == 2 && (!(cg_rtol > 0.0) || cg_maxit < 1)) return RTE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    Layout L = carve(c, p, RTE_SI_DSA, nullptr, RTE_FP64, 1);
    if (!c.ok) return RTE_ENOMEM;
    int failed = 0;
    if (p->dim == 2) HIPCHK(launch_dsa_build(p, L.cg, nullptr, s));
    int rc = do_dsa(p, L, rho_star, rho_prev, delta_rho, nullptr, 0, cg_rtol, cg_maxit,
                    cg_iters_out, &failed, nullptr, s);
    if (rc) return rc;
    return failed ? RTE_ECG : RTE_OK;
}

int rte_rom_initial_guess(const rte_problem *p, const rte_rom *rom, const double *psi,
                          double *rho_out, int *status_out, void *ws, size_t ws_bytes,
                          rte_stream_t stream) {
    if (!p || !rom || !rho_out || !ws) return RTE_EINVAL;
    if (rom->m > 0 && !psi) return RTE_EINVAL;
    if (rom->ndof != p->ndof) return RTE_EINVAL;
    if (p->dim != 2) return RTE_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    Layout L = carve(c, p, RTE_ROMSAD, rom, RTE_FP64, 1);
    if (!c.ok) return RTE_ENOMEM;
    HIPCHK(launch_rom_initial_guess(p, rom, psi, rho_out, status_out ? status_out : L.rom_status,
                                    L.rom, s));
    return RTE_OK;
}

int rte_rom_correct(const rte_problem *p, const rte_rom *rom, const double *psi,
                    const double *rho_star, const double *rho_prev, double *delta_rho,
                    int *status_out, rte_precision prec, void *ws, size_t ws_bytes,
                    rte_stream_t stream) {
    if (!p || !rom || !rho_star || !rho_prev || !delta_rho || !ws) return RTE_EINVAL;
    if (rom->m > 0 && !psi) return RTE_EINVAL;
    if (rom->ndof != p->ndof) return RTE_EINVAL;
    if (prec != RTE_FP64 && prec != RTE_MIXED) return RTE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    Layout L = carve(c, p, RTE_ROMSAD, rom, prec, 1);
    if (!c.ok) return RTE_ENOMEM;
    HIPCHK(launch_rom_correct(p, rom, psi, rho_star, rho_prev, delta_rho,
                              status_out ? status_out : L.rom_status, nullptr, 0, L.rom,
                              prec == RTE_MIXED, s));
    return RTE_OK;
}

int rte_sisa_solve(const rte_problem *p, rte_mode mode, const rte_rom *rom, const double *psi,
                   const rte_solve_opts *o, double *rho, void *f_out, rte_solve_stats *stats,
                   void *ws, size_t ws_bytes, rte_stream_t stream) {
    if (!rho || !ws) return RTE_EINVAL;
    int rc = check_solve_args(p, mode, rom, psi, true, o);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    Layout L = carve(c, p, mode, mode == RTE_ROMSAD ? rom : nullptr, o->precision, o->max_iter);
    if (!c.ok) return RTE_ENOMEM;
    HIPCHK(launch_init_state(p, L.st, o->max_iter, nullptr, 1, s));
    HIPCHK(launch_zero_rows(L.delta, p->B, p->ndof, nullptr, s));
    HIPCHK(launch_zero_u64(L.cg_total, 1, s));
    if (mode != RTE_SI && p->dim == 2) HIPCHK(launch_dsa_build(p, L.cg, nullptr, s));
    PrecondGraphs graphs(p, L.cg, mode != RTE_SI && p->dim == 2 && o->graph_cg_iters <= 0,
                         precond_key(0, p, L, ws, ws_bytes, (int)mode, (int)o->precision,
                                     o->max_iter, mode == RTE_ROMSAD ? rom : nullptr));
    if ((rc = prepare_materials(p, L, nullptr, o->precision == RTE_MIXED, s))) return rc;
    HIPCHK(launch_source(p, rho, L.src, nullptr, o->precision == RTE_MIXED, s, true,
                         L.use_mat ? L.mat : nullptr, L.mat_ok));
    int iterations = 0;
    bool cg_failed = false;
    rc = run_iterations(p, L, mode, rom, psi, o, rho, f_out, o->max_iter, ws, ws_bytes, s,
                        &iterations, &cg_failed);
    if (rc) return rc;
    return finish_stats(p, L, o->max_iter, iterations, cg_failed, nullptr, stats, s);
}

int rte_sisa_solve_multi(int n, const rte_problem *const *probs, rte_mode mode,
                         const rte_rom *const *roms, const double *const *psi,
                         const rte_solve_opts *opts, double *const *rho, void *const *f_out,
                         rte_solve_stats *stats, void *const *ws, const size_t *ws_bytes,
                         const rte_stream_t *streams, int *status) {
    if (n < 1 || n > RTE_MULTI_MAX || !probs || !opts || !rho || !ws || !ws_bytes || !streams)
        return RTE_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!probs[i] || !rho[i] || !ws[i]) return RTE_EINVAL;
        for (int k = 0; k < i; ++k) {
            const char *a0 = (const char *)ws[i], *b0 = (const char *)ws[k];
            const bool overlap = a0 < b0 + ws_bytes[k] && b0 < a0 + ws_bytes[i];
            if (probs[i] == probs[k] || rho[i] == rho[k] || overlap) return RTE_EINVAL;
        }
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::vector<int> rc(n, RTE_OK);
    auto run = [&](int i) {
        if (hipSetDevice(dev) != hipSuccess) { rc[i] = RTE_EDEVICE; return; }
        rc[i] = rte_sisa_solve(probs[i], mode, roms ? roms[i] : nullptr, psi ? psi[i] : nullptr,
                               opts, rho[i], f_out ? f_out[i] : nullptr,
                               stats ? &stats[i] : nullptr, ws[i], ws_bytes[i], streams[i]);
    };
    std::vector<std::thread> th;
    th.reserve(n - 1);
    try {
        for (int i = 1; i < n; ++i) th.emplace_back(run, i);
    } catch (...) {
        for (auto &t : th) t.join();
        return RTE_ENOMEM;
    }
    run(0);
    for (auto &t : th) t.join();
    if (status)
        for (int i = 0; i < n; ++i) status[i] = rc[i];
    // an argument or device error first, then a CG failure, then non-convergence
    for (int i = 0; i < n; ++i)
        if (rc[i] != RTE_OK && rc[i] != RTE_ECG && rc[i] != RTE_ENOCONV) return rc[i];
    for (int i = 0; i < n; ++i)
        if (rc[i] == RTE_ECG) return RTE_ECG;
    for (int i = 0; i < n; ++i)
        if (rc[i] == RTE_ENOCONV) return RTE_ENOCONV;
    return RTE_OK;
}

int rte_pgmres_solve(const rte_problem *p, const rte_krylov_opts *o, double *rho,
                     rte_krylov_stats *stats, void *ws, size_t ws_bytes, rte_stream_t stream) {
    if (!p || !o || !rho || !ws) return RTE_EINVAL;
    if (!(o->tol > 0.0) || o->restart < 1 || o->restart > 200 || o->max_cycles < 1) return RTE_EINVAL;
    if (o->precondition && p->dim == 2 && (!(o->cg_rtol > 0.0) || o->cg_maxit < 1)) return RTE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    Layout L = carve(c, p, RTE_SI_DSA, nullptr, RTE_FP64, 1, o->restart);
    if (!c.ok) return RTE_ENOMEM;
    const GmresSpace &G = L.gm;
    const int m = o->restart;
    const size_t vstride = (size_t)p->B * p->ndof;
    bool cg_failed = false;
    // M^-1 in = in + C Sigma_s in (DSA correction of the residual in), for the flagged instances
    auto minv = [&](const double *in, double *out, const int *flag) -> int {
        if (!o->precondition) {
            HIPCHK(gm_lincomb(p, in, nullptr, 0.0, nullptr, 0.0, out, flag, s));
            return RTE_OK;
        }
        int failed = 0;
        int rc = do_dsa(p, L, in, nullptr, L.delta, flag, 1, o->cg_rtol, o->cg_maxit, nullptr,
                        &failed, nullptr, s);
        if (rc) return rc;
        cg_failed = cg_failed || failed;
        HIPCHK(gm_lincomb(p, in, L.delta, 1.0, nullptr, 0.0, out, flag, s));
        return RTE_OK;
    };
    // density of one sweep: with_G and vacuum/physical inflow per `homogeneous`
    auto sweep = [&](const double *in, double *out, const int *flag, bool homogeneous) -> int {
        HIPCHK(launch_source(p, in, L.src, flag, 0, s, !homogeneous));
        int rc = do_sweep(p, L, L.src, nullptr, out, nullptr, flag, homogeneous ? 1 : 0, 0, s);
        if (rc) return rc;
        HIPCHK(gm_count_sweep(p, G, flag, s));
        return RTE_OK;
    };
    auto read_count = [&](int *v) -> int {
        HIPCHK(hipMemcpyAsync(v, G.count, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return RTE_OK;
    };
    int rc;
    HIPCHK(launch_fill_int(G.act, p->B, 1, s));
    HIPCHK(launch_fill_int(G.n_sweep, p->B, 0, s));
    HIPCHK(launch_fill_int(G.n_iter, p->B, 0, s));
    if (o->precondition && p->dim == 2) HIPCHK(launch_dsa_build(p, L.cg, nullptr, s));
    PrecondGraphs graphs(p, L.cg, o->precondition && p->dim == 2,
                         precond_key(1, p, L, ws, ws_bytes, (int)RTE_SI_DSA, (int)RTE_FP64,
                                     o->restart, nullptr));
    // b_bar: one sweep from zero with the source and the inflow; |M^-1 b_bar|
    HIPCHK(launch_zero_rows(G.u, p->B, p->ndof, nullptr, s));
    if ((rc = sweep(G.u, G.bbar, G.act, false))) return rc;
    if ((rc = minv(G.bbar, G.w, G.act))) return rc;
    HIPCHK(gm_norm(p, G, G.w, G.act, s));
    HIPCHK(gm_sqrt_norm(p, G, G.act, G.nb, s));
    int cycles = 0;
    for (int cyc = 0; cyc < o->max_cycles; ++cyc) {
        // (re)start: r = M^-1 (b_bar - x + L x)
        if ((rc = sweep(rho, G.lv, G.act, true))) return rc;
        HIPCHK(gm_lincomb(p, G.bbar, rho, -1.0, G.lv, 1.0, G.t, G.act, s));
        if ((rc = minv(G.t, G.w, G.act))) return rc;
        HIPCHK(gm_norm(p, G, G.w, G.act, s));
        HIPCHK(launch_fill_int(G.count, 1, 0, s));
        HIPCHK(gm_cycle_start(p, G, o->tol, s));
        HIPCHK(gm_scale(p, G, G.w, G.g, m + 1, 0, G.V, G.cyc, s));
        int running = 0;
        if ((rc = read_count(&running))) return rc;
        if (running == 0) break;
        ++cycles;
        for (int i = 0; i < m; ++i) {
            double *Vi = G.V + (size_t)i * vstride;
            // w = M^-1 (V_i - L V_i)
            if ((rc = sweep(Vi, G.lv, G.cyc, true))) return rc;
            HIPCHK(gm_lincomb(p, Vi, G.lv, -1.0, nullptr, 0.0, G.u, G.cyc, s));
            if ((rc = minv(G.u, G.w, G.cyc))) return rc;
            // classical Gram-Schmidt, twice: h = V^T w, w -= V h (coefficients summed over passes)
            HIPCHK(gm_dots(p, G, i + 1, G.V, G.w, G.cyc, G.h, 0, s));
            HIPCHK(gm_axpy(p, G, i + 1, G.V, G.h, G.nslot, -1.0, G.w, G.cyc, false, s));
            HIPCHK(gm_dots(p, G, i + 1, G.V, G.w, G.cyc, G.h2, 0, s));
            HIPCHK(gm_resum(p, G, i + 1, G.cyc, G.h, 1, s));
            HIPCHK(gm_axpy(p, G, i + 1, G.V, G.h2, G.nslot, -1.0, G.w, G.cyc, true, s));
            HIPCHK(launch_fill_int(G.count, 1, 0, s));
            HIPCHK(gm_givens(p, G, i, o->tol, s));
            HIPCHK(gm_scale(p, G, G.w, G.wn, 1, 0, G.V + (size_t)(i + 1) * vstride, G.cyc, s));
            if ((rc = read_count(&running))) return rc;
            if (running == 0) break;
        }
        // x += V y for every running instance (the minimizer over its cycle's steps)
        HIPCHK(gm_solve(p, G, s));
        HIPCHK(gm_axpy(p, G, m, G.V, G.y, m, 1.0, rho, G.act, false, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int> act(p->B);
    HIPCHK(hipMemcpy(act.data(), G.act, sizeof(int) * p->B, hipMemcpyDeviceToHost));
    int status = RTE_OK;
    for (int b = 0; b < p->B; ++b)
        if (act[b]) status = RTE_ENOCONV;
    if (stats) {
        if (stats->n_sweep)
            HIPCHK(hipMemcpy(stats->n_sweep, G.n_sweep, sizeof(int) * p->B, hipMemcpyDeviceToHost));
        if (stats->iterations)
            HIPCHK(hipMemcpy(stats->iterations, G.n_iter, sizeof(int) * p->B, hipMemcpyDeviceToHost));
        if (stats->residual)
            HIPCHK(hipMemcpy(stats->residual, G.est, sizeof(double) * p->B, hipMemcpyDeviceToHost));
        if (stats->status)
            for (int b = 0; b < p->B; ++b) stats->status[b] = act[b] ? RTE_ENOCONV : RTE_OK;
        stats->cycles = cycles;
    }
    if (cg_failed && status == RTE_OK) status = RTE_ECG;
    return status;
}

int rte_sisa_begin(const rte_problem *p, rte_mode mode, const rte_rom *rom, const rte_solve_opts *o,
                   void *ws, size_t ws_bytes, rte_stream_t stream) {
    if (!ws) return RTE_EINVAL;
    int rc = check_solve_args(p, mode, rom, nullptr, false, o);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    Layout L = carve(c, p, mode, mode == RTE_ROMSAD ? rom : nullptr, o->precision, o->max_iter);
    if (!c.ok) return RTE_ENOMEM;
    HIPCHK(launch_init_state(p, L.st, o->max_iter, nullptr, 0, s));
    HIPCHK(launch_zero_u64(L.cg_total, 1, s));
    if (L.mat_ok) HIPCHK(launch_fill_int(L.mat_ok, p->B, 0, s));   // no slot has a table yet
    return RTE_OK;
}

int rte_sisa_admit(const rte_problem *p, rte_mode mode, const rte_rom *rom, const rte_solve_opts *o,
                   const int *slots, int n_slots, const double *rho, void *ws, size_t ws_bytes,
                   rte_stream_t stream) {
    if (!ws || !rho || n_slots < 0 || (n_slots > 0 && !slots)) return RTE_EINVAL;
    int rc = check_solve_args(p, mode, rom, nullptr, false, o);
    if (rc) return rc;
    std::vector<int> mask(p->B, 0);
    for (int k = 0; k < n_slots; ++k) {
        if (slots[k] < 0 || slots[k] >= p->B) return RTE_EINVAL;
        mask[slots[k]] = 1;
    }
    if (n_slots == 0) return RTE_OK;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    Layout L = carve(c, p, mode, mode == RTE_ROMSAD ? rom : nullptr, o->precision, o->max_iter);
    if (!c.ok) return RTE_ENOMEM;
    HIPCHK(hipMemcpyAsync(L.mask, mask.data(), sizeof(int) * p->B, hipMemcpyHostToDevice, s));
    HIPCHK(launch_init_state(p, L.st, o->max_iter, L.mask, 1, s));
    HIPCHK(launch_zero_rows(L.delta, p->B, p->ndof, L.mask, s));
    if (mode != RTE_SI && p->dim == 2) HIPCHK(launch_dsa_build(p, L.cg, L.mask, s));
    if ((rc = prepare_materials(p, L, L.mask, o->precision == RTE_MIXED, s))) return rc;
    HIPCHK(launch_source(p, rho, L.src, L.mask, o->precision == RTE_MIXED, s, true,
                         L.use_mat ? L.mat : nullptr, L.mat_ok));
    // the host mask must outlive the copy
    HIPCHK(hipStreamSynchronize(s));
    return RTE_OK;
}

int rte_sisa_iterate(const rte_problem *p, rte_mode mode, const rte_rom *rom, const double *psi,
                     const rte_solve_opts *o, double *rho, int n_iter, int *active_out,
                     rte_solve_stats *stats, void *ws, size_t ws_bytes, rte_stream_t stream) {
    if (!ws || !rho || n_iter < 1) return RTE_EINVAL;
    int rc = check_solve_args(p, mode, rom, psi, true, o);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    Layout L = carve(c, p, mode, mode == RTE_ROMSAD ? rom : nullptr, o->precision, o->max_iter);
    if (!c.ok) return RTE_ENOMEM;
    L.use_mat = mat_usable(p, L, o->precision == RTE_MIXED);   // prepared by rte_sisa_admit
    int iterations = 0;
    bool cg_failed = false;
    rc = run_iterations(p, L, mode, rom, psi, o, rho, nullptr, n_iter, ws, ws_bytes, s,
                        &iterations, &cg_failed);
    if (rc) return rc;
    rc = finish_stats(p, L, o->max_iter, iterations, cg_failed, active_out, stats, s);
    return rc == RTE_ENOCONV ? RTE_OK : rc;     // slots still running are not an error here
}

}  // extern "C"
