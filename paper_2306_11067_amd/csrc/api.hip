// C-ABI of the library (include/rls.h): problem setup, weight updates and
// the batched lambda sweep.  Host code here only allocates, validates and
// sequences kernels; every arithmetic step runs on the GPU.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "outer.h"
#include "rls_internal.h"

using namespace rls;

namespace {

thread_local std::string g_last_error;

rls_status fail(rls_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define RLS_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess)                                                \
            return fail(e_ == hipErrorOutOfMemory ? RLS_E_OOM : RLS_E_HIP,   \
                        std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define RLS_TRY(expr)                      \
    do {                                   \
        rls_status s_ = (expr);            \
        if (s_ != RLS_OK) return s_;       \
    } while (0)

// A device allocation owned by the library.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

rls_status dalloc(DBuf& b, size_t bytes) {
    if (b.p && b.bytes >= bytes) return RLS_OK;
    b.release();
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return fail(e == hipErrorOutOfMemory ? RLS_E_OOM : RLS_E_HIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    b.bytes = bytes;
    return RLS_OK;
}

struct Band {
    int n = 0, bw = 0, map = MAP_ZERO, uniform = 0;
    size_t taps_off = 0;     // offset (in values) of the uniform row in table
    DBuf table, diag, rowabs;
    DBuf table32, diag32;    // FP32 copies (FP32 V-cycle)
    std::vector<double> htaps;   // host copy of the uniform row
    std::vector<float> htaps32;
    BandDev dev() const {
        BandDev b;
        b.n = n;
        b.bw = bw;
        b.map = map;
        b.uniform = uniform;
        b.table = table.as<double>();
        b.taps = table.as<double>() + taps_off;
        b.diag = diag.as<double>();
        b.rowabs = rowabs.as<double>();
        b.htaps = htaps.empty() ? nullptr : htaps.data();
        return b;
    }
    BandDevT<float> dev32() const {
        BandDevT<float> b;
        b.n = n;
        b.bw = bw;
        b.map = map;
        b.uniform = uniform;
        b.table = table32.as<float>();
        b.taps = table32.as<float>() + taps_off;
        b.diag = diag32.as<float>();
        b.htaps = htaps32.empty() ? nullptr : htaps32.data();
        return b;
    }
};

// Sparse A_k of a tomography level (values FP64, FP32 copies for the FP32
// V-cycle) and pointers to the shared application workspace.
struct CtLevel {
    int on = 0;
    int64_t m = 0, nnz = 0;
    DBuf rp, ci, va, rpt, cit, vat, va32, vat32, diag, diag32, rowabs;
    double *v = nullptr, *y = nullptr, *t = nullptr, *res = nullptr;
    float *v32 = nullptr, *y32 = nullptr, *t32 = nullptr, *res32 = nullptr;
    CsrDevT<double> dev() const {
        CsrDevT<double> c;
        if (!on) return c;
        c.on = 1;
        c.m = m;
        c.rp = rp.as<int64_t>();
        c.ci = ci.as<int>();
        c.va = va.as<double>();
        c.rpt = rpt.as<int64_t>();
        c.cit = cit.as<int>();
        c.vat = vat.as<double>();
        c.diag = diag.as<double>();
        c.rowabs = rowabs.as<double>();
        c.v = v;
        c.y = y;
        c.t = t;
        c.res = res;
        return c;
    }
    CsrDevT<float> dev32() const {
        CsrDevT<float> c;
        if (!on) return c;
        c.on = 1;
        c.m = m;
        c.rp = rp.as<int64_t>();
        c.ci = ci.as<int>();
        c.va = va32.as<float>();
        c.rpt = rpt.as<int64_t>();
        c.cit = cit.as<int>();
        c.vat = vat32.as<float>();
        c.diag = diag32.as<float>();
        c.rowabs = rowabs.as<double>();
        c.v = v32;
        c.y = y32;
        c.t = t32;
        c.res = res32;
        return c;
    }
};

struct Level {
    int nv = 0, nh = 0;
    Band gv, gh;
    CtLevel ct;
    DBuf planes, srowabs;
    int nine = 0;
    int periodic = 0;
    int64_t n() const { return (int64_t)nv * nh; }
    DBuf planes32;           // FP32 copy of the five stencil planes
    LevelGeom geom() const {
        LevelGeom g;
        g.nv = nv;
        g.nh = nh;
        g.gv = gv.dev();
        g.gh = gh.dev();
        const double* pl = planes.as<double>();
        const int64_t m = n();
        g.S.c = pl;
        g.S.cn = pl + m;
        g.S.ce = pl + 2 * m;
        g.S.cne = pl + 3 * m;
        g.S.cse = pl + 4 * m;
        g.S.rowabs = srowabs.as<double>();
        g.S.nine = nine;
        g.S.periodic = periodic;
        g.ct = ct.dev();
        return g;
    }
    LevelGeomT<float> geom32() const {
        LevelGeomT<float> g;
        g.nv = nv;
        g.nh = nh;
        g.gv = gv.dev32();
        g.gh = gh.dev32();
        const float* pl = planes32.as<float>();
        const int64_t m = n();
        g.S.c = pl;
        g.S.cn = pl + m;
        g.S.ce = pl + 2 * m;
        g.S.cne = pl + 3 * m;
        g.S.cse = pl + 4 * m;
        g.S.nine = nine;
        g.S.periodic = periodic;
        g.ct = ct.dev32();
        return g;
    }
    template <class R> LevelGeomT<R> geom_t() const;
};
template <> LevelGeomT<double> Level::geom_t<double>() const { return geom(); }
template <> LevelGeomT<float> Level::geom_t<float>() const { return geom32(); }

// Per-sweep workspace, grown on demand.
struct Work {
    int cap = 0;                 // slots allocated
    DBuf lam2, zero_lam2, st, active, beta, part, rho, cheb, kc, winv, info;
    DBuf f;                      // A^T b (n)
    DBuf fpart, rrpart, outv, slots;
    DBuf part_pq, part_rr, part_rz;    // PCG partial sums per slot
    DBuf part_zq;                      // flexible beta: partials of z . q
    // reduced-precision V-cycle (FP32 or BF16 elements): fine rhs, result
    DBuf rlo, zlo;
    DBuf ctv, cty, ctt, ctres, ctv32, cty32, ctt32, ctres32;  // sparse levels
    std::vector<DBuf> lxlo, lxblo, ldlo, lflo;   // its level vectors
    int* h_active = nullptr;     // pinned host mirrors
    int* h_slots = nullptr;
    ~Work() {
        if (h_active) hipHostFree(h_active);
        if (h_slots) hipHostFree(h_slots);
    }
    DBuf r, z, p0, p1, q, y;     // fine vectors (cap * n)
    std::vector<DBuf> lx, lxb, ld, lt, lf;   // per level (cap * n_k)
};

}  // namespace

struct rls_problem {
    int device = 0;
    int nv = 0, nh = 0, levels = 0, bc = 0, lbc = 0;
    int prec = RLS_PREC_FP64;    // V-cycle arithmetic
    int is_ct = 0;               // sparse (tomography) forward operator
    int64_t ct_m = 0;            // its rows
    DBuf ct_gram;                // dense A_c^T A_c of the coarsest level
    std::vector<int> nu;         // Chebyshev steps per level
    std::vector<double> ratio;   // Chebyshev interval ratio per level
    int nu_max = 2;
    int periodic = 0;            // multigrid / gradient periodicity
    // RLS_FINE_KERNEL=generic at set-up: the finest-level Chebyshev step
    // always takes the general level-operator kernel
    int fine_generic = 0;
    // measured workgroup size of the tiled finest-level Chebyshev kernel
    // per slot count (0: not measured), for the FP64 and for the reduced-
    // precision V-cycle
    std::vector<int> fine_nt64 = std::vector<int>(FINE_ZMAX + 1, 0);
    std::vector<int> fine_ntlo = std::vector<int>(FINE_ZMAX + 1, 0);
    int r_v = 0, r_h = 0;
    std::vector<double> taps_v, taps_h;
    std::vector<Level> lev;
    Band av, ah, atv, ath;       // A and A^T bands (fine)
    DBuf weights;                // 2n, or empty for D = I
    int unit_weights = 1;
    Work w;
    hipStream_t cstream = nullptr;   // capture stream for iteration graphs
    hipStream_t bstream = nullptr;   // this problem's stream in a batch
    // Host copy of the device slot list w.slots while a sweep launches
    // iterations over it (copied into the kernel arguments when short).
    const int* hslots = nullptr;
    int hslots_n = 0;
    // live timing of the finest-level Chebyshev-step kernel
    bool timer_on = false;
    bool fine_tiled = false;     // the last FP64 finest-level step was tiled
    struct TimedRun {
        hipEvent_t a = nullptr, b = nullptr;
        int launches = 0;
    };
    std::vector<TimedRun> run_pool;      // free event pairs
    std::vector<TimedRun> run_pending;   // recorded, not yet read
    TimedRun run_cur;
    long long timer_launches = 0;
    double timer_seconds = 0.0, timer_bytes = 0.0;
    int kt = 0;                      // first level handled by the tail kernel
    int64_t n() const { return (int64_t)nv * nh; }
    ~rls_problem() {
        for (auto* v : {&run_pool, &run_pending})
            for (auto& e : *v) { hipEventDestroy(e.a); hipEventDestroy(e.b); }
        if (cstream) hipStreamDestroy(cstream);
        if (bstream) hipStreamDestroy(bstream);
    }
};

namespace {

int max_part_slots(const rls_problem* P) {
    int m = vec_blocks(P->n());
    if (P->is_ct) m = std::max(m, vec_blocks(P->ct_m));
    for (const Level& L : P->lev) m = std::max(m, apply_tiles(L.geom()));
    return m;
}

rls_status check_launch(const char* where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(RLS_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
    return RLS_OK;
}

// Finest-level Chebyshev steps come in runs of consecutive launches (the
// pre- and the post-smoothing steps of a V-cycle).  With the kernel timer
// on (direct launches only), each run is bracketed by one pair of HIP
// events on the launch stream, so the event time is that of the kernels
// back to back and not of the dispatch of each one.
void run_begin(rls_problem* P, hipStream_t s) {
    if (!P->timer_on) return;
    if (P->run_pool.empty()) {
        rls_problem::TimedRun r;
        hipEventCreate(&r.a);
        hipEventCreate(&r.b);
        P->run_pool.push_back(r);
    }
    P->run_cur = P->run_pool.back();
    P->run_pool.pop_back();
    P->run_cur.launches = 0;
    hipEventRecord(P->run_cur.a, s);
}

// The level operator of either operator kind.
template <class R, class V>
void level_apply(int pro, int epi, const ApplyArgsT<R, V>& a, hipStream_t s) {
    if constexpr (std::is_same<V, bf16>::value) {
        launch_apply(pro, epi, a, s);   // sparse operators have no BF16 path
    } else {
        if (a.g.ct.on) launch_ct_apply(pro, epi, a, s);
        else launch_apply(pro, epi, a, s);
    }
}

// The launch arguments with the measured workgroup size for this slot count.
template <class R, class V>
ApplyArgsT<R, V> with_fine_nt(const std::vector<int>& tab,
                              const ApplyArgsT<R, V>& a) {
    ApplyArgsT<R, V> b = a;
    if (a.nslot >= 1 && a.nslot <= FINE_ZMAX) b.fine_nt = tab[a.nslot];
    return b;
}

void smooth_fine(rls_problem* P, const ApplyArgs& a, hipStream_t s) {
    if (a.g.ct.on) {
        launch_ct_apply(PRO_PLAIN, EPI_CHEB, a, s);
        return;
    }
    if (P->fine_generic) {
        launch_apply(PRO_PLAIN, EPI_CHEB, a, s);
        P->fine_tiled = false;
    } else {
        P->fine_tiled = launch_smooth_fine_tiled(with_fine_nt(P->fine_nt64, a), s);
        if (!P->fine_tiled) launch_apply(PRO_PLAIN, EPI_CHEB, a, s);
    }
    if (P->timer_on) P->run_cur.launches += 1;
}
// FP32 and BF16 V-cycles: not timed (the kernel timer covers the FP64
// step).
void smooth_fine(rls_problem* P, const ApplyArgsT<float>& a, hipStream_t s) {
    if (a.g.ct.on) launch_ct_apply(PRO_PLAIN, EPI_CHEB, a, s);
    else if (P->fine_generic) launch_apply(PRO_PLAIN, EPI_CHEB, a, s);
    else launch_smooth_fine(with_fine_nt(P->fine_ntlo, a), s);
}
void smooth_fine(rls_problem* P, const ApplyArgsT<float, bf16>& a,
                 hipStream_t s) {
    if (P->fine_generic) launch_apply(PRO_PLAIN, EPI_CHEB, a, s);
    else launch_smooth_fine(with_fine_nt(P->fine_ntlo, a), s);
}

void run_end(rls_problem* P, hipStream_t s) {
    if (!P->timer_on) return;
    hipEventRecord(P->run_cur.b, s);
    P->run_pending.push_back(P->run_cur);
}

// After a stream synchronization: fold the timed runs into the totals.
void drain_timer(rls_problem* P) {
    for (auto& r : P->run_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            P->timer_seconds += 1e-3 * ms;
            P->timer_launches += r.launches;
        } else {
            (void)hipGetLastError();   // not a launch error: do not keep it
        }
        P->run_pool.push_back(r);
    }
    P->run_pending.clear();
}

rls_status ensure_work(rls_problem* P, int nslot) {
    Work& w = P->w;
    if (w.cap >= nslot) return RLS_OK;
    const int cap = std::max(nslot, w.cap * 2);
    const int64_t n = P->n();
    const int L = P->levels;
    RLS_TRY(dalloc(w.lam2, sizeof(double) * cap));
    RLS_TRY(dalloc(w.zero_lam2, sizeof(double) * cap));
    RLS_HIP(hipMemset(w.zero_lam2.p, 0, sizeof(double) * cap));
    RLS_TRY(dalloc(w.st, sizeof(SlotState) * cap));
    RLS_TRY(dalloc(w.active, sizeof(int) * cap));
    RLS_TRY(dalloc(w.beta, sizeof(double) * cap));
    RLS_TRY(dalloc(w.part, sizeof(double) * (size_t)cap * max_part_slots(P)));
    RLS_TRY(dalloc(w.rho, sizeof(double) * (size_t)cap * L));
    RLS_TRY(dalloc(w.cheb, sizeof(double) * (size_t)cap * L * 2 * P->nu_max));
    const int64_t nc = P->lev.back().n();
    RLS_TRY(dalloc(w.kc, sizeof(double) * (size_t)cap * nc * nc));
    RLS_TRY(dalloc(w.winv, sizeof(double) * (size_t)cap * 2 * nc * nc));
    RLS_TRY(dalloc(w.info, sizeof(int) * cap));
    RLS_TRY(dalloc(w.f, sizeof(double) * n));
    RLS_TRY(dalloc(w.fpart, sizeof(double) * vec_blocks(n)));
    RLS_TRY(dalloc(w.rrpart, sizeof(double) * (size_t)cap * vec_blocks(n)));
    RLS_TRY(dalloc(w.outv, sizeof(double) * 3 * cap));
    RLS_TRY(dalloc(w.slots, sizeof(int) * cap));
    {
        const int t0 = apply_tiles(P->lev[0].geom());
        RLS_TRY(dalloc(w.part_pq, sizeof(double) * (size_t)cap * t0));
        RLS_TRY(dalloc(w.part_rz, sizeof(double) * (size_t)cap * t0));
        RLS_TRY(dalloc(w.part_zq, sizeof(double) * (size_t)cap * t0));
        RLS_TRY(dalloc(w.part_rr, sizeof(double) * (size_t)cap * vec_blocks(n)));
    }
    if (w.h_active) hipHostFree(w.h_active);
    if (w.h_slots) hipHostFree(w.h_slots);
    w.h_active = w.h_slots = nullptr;
    RLS_HIP(hipHostMalloc((void**)&w.h_active, sizeof(int) * cap, hipHostMallocDefault));
    RLS_HIP(hipHostMalloc((void**)&w.h_slots, sizeof(int) * cap, hipHostMallocDefault));
    for (DBuf* b : {&w.r, &w.z, &w.p0, &w.p1, &w.q, &w.y})
        RLS_TRY(dalloc(*b, sizeof(double) * (size_t)cap * n));
    w.lx.resize(L);
    w.lxb.resize(L);
    w.ld.resize(L);
    w.lt.resize(L);
    w.lf.resize(L);
    for (int k = 0; k < L; ++k) {
        const size_t bytes = sizeof(double) * (size_t)cap * P->lev[k].n();
        RLS_TRY(dalloc(w.lxb[k], bytes));
        RLS_TRY(dalloc(w.ld[k], bytes));
        RLS_TRY(dalloc(w.lt[k], bytes));
        if (k > 0) {
            RLS_TRY(dalloc(w.lx[k], bytes));
            RLS_TRY(dalloc(w.lf[k], bytes));
        }
    }
    if (P->is_ct) {
        const size_t cn = (size_t)cap * n, cm = (size_t)cap * P->ct_m;
        RLS_TRY(dalloc(w.ctv, sizeof(double) * cn));
        RLS_TRY(dalloc(w.cty, sizeof(double) * cm));
        RLS_TRY(dalloc(w.ctt, sizeof(double) * cn));
        RLS_TRY(dalloc(w.ctres, sizeof(double) * cn));
        RLS_TRY(dalloc(w.ctv32, sizeof(float) * cn));
        RLS_TRY(dalloc(w.cty32, sizeof(float) * cm));
        RLS_TRY(dalloc(w.ctt32, sizeof(float) * cn));
        RLS_TRY(dalloc(w.ctres32, sizeof(float) * cn));
        for (Level& Lv : P->lev) {
            Lv.ct.v = w.ctv.as<double>();
            Lv.ct.y = w.cty.as<double>();
            Lv.ct.t = w.ctt.as<double>();
            Lv.ct.res = w.ctres.as<double>();
            Lv.ct.v32 = w.ctv32.as<float>();
            Lv.ct.y32 = w.cty32.as<float>();
            Lv.ct.t32 = w.ctt32.as<float>();
            Lv.ct.res32 = w.ctres32.as<float>();
        }
    }
    if (P->prec != RLS_PREC_FP64) {
        const size_t esz = P->prec == RLS_PREC_MIXED_BF16 ? sizeof(bf16)
                                                          : sizeof(float);
        RLS_TRY(dalloc(w.rlo, esz * (size_t)cap * n));
        RLS_TRY(dalloc(w.zlo, esz * (size_t)cap * n));
        for (auto* v : {&w.lxlo, &w.lxblo, &w.ldlo, &w.lflo}) v->resize(L);
        for (int k = 0; k < L; ++k) {
            const size_t bytes = esz * (size_t)cap * P->lev[k].n();
            RLS_TRY(dalloc(w.lxblo[k], bytes));
            RLS_TRY(dalloc(w.ldlo[k], bytes));
            if (k > 0) {
                RLS_TRY(dalloc(w.lxlo[k], bytes));
                RLS_TRY(dalloc(w.lflo[k], bytes));
            }
        }
    }
    w.cap = cap;
    return RLS_OK;
}

// Build the 1D Gram band hierarchy of one direction.
rls_status build_direction(rls_problem* P, const std::vector<double>& taps,
                           int r, int dir, hipStream_t s) {
    const int n0 = dir == 0 ? P->nv : P->nh;
    const int blur_periodic = P->bc == RLS_BC_PERIODIC;
    DBuf dtaps;
    RLS_TRY(dalloc(dtaps, sizeof(double) * taps.size()));
    RLS_HIP(hipMemcpyAsync(dtaps.p, taps.data(), sizeof(double) * taps.size(),
                           hipMemcpyHostToDevice, s));
    Band& A = dir == 0 ? P->av : P->ah;
    Band& At = dir == 0 ? P->atv : P->ath;
    A.n = At.n = n0;
    A.bw = At.bw = r;
    A.map = At.map = blur_periodic ? MAP_WRAP : MAP_ZERO;
    A.uniform = At.uniform = 0;
    RLS_TRY(dalloc(A.table, sizeof(double) * n0 * (2 * r + 1)));
    RLS_TRY(dalloc(At.table, sizeof(double) * n0 * (2 * r + 1)));
    for (Band* b : {&A, &At}) {
        RLS_TRY(dalloc(b->diag, sizeof(double) * n0));
        RLS_TRY(dalloc(b->rowabs, sizeof(double) * n0));
    }
    launch_blur_band(dtaps.as<double>(), r, n0, P->bc, A.table.as<double>(), s);
    launch_transpose_band(A.table.as<double>(), n0, r, blur_periodic,
                          At.table.as<double>(), s);
    launch_band_stats(A.table.as<double>(), n0, r, A.diag.as<double>(),
                      A.rowabs.as<double>(), s);
    launch_band_stats(At.table.as<double>(), n0, r, At.diag.as<double>(),
                      At.rowabs.as<double>(), s);
    // level Gram bands
    int bw = 2 * r;
    for (int k = 0; k < P->levels; ++k) {
        Level& L = P->lev[k];
        Band& G = dir == 0 ? L.gv : L.gh;
        const int nk = dir == 0 ? L.nv : L.nh;
        G.n = nk;
        G.bw = bw;
        if (nk < 2 * bw + 1)
            return fail(RLS_E_UNSUPPORTED,
                        "level " + std::to_string(k) +
                            " is narrower than its Gram band (" +
                            std::to_string(nk) + " < " +
                            std::to_string(2 * bw + 1) + "); use fewer levels "
                            "or a smaller blur radius");
        RLS_TRY(dalloc(G.table, sizeof(double) * nk * (2 * bw + 1)));
        RLS_TRY(dalloc(G.diag, sizeof(double) * nk));
        RLS_TRY(dalloc(G.rowabs, sizeof(double) * nk));
        if (k == 0) {
            launch_gram_band(A.table.as<double>(), nk, r, blur_periodic,
                             G.table.as<double>(), bw, s);
        } else {
            Band& Gf = dir == 0 ? P->lev[k - 1].gv : P->lev[k - 1].gh;
            launch_galerkin_band(Gf.table.as<double>(), Gf.n, Gf.bw,
                                 P->periodic, G.table.as<double>(), bw, s);
        }
        launch_band_stats(G.table.as<double>(), nk, bw, G.diag.as<double>(),
                          G.rowabs.as<double>(), s);
        // Uniform fast path: periodic levels are circulant (every row equals
        // row 0); the fine reflective Gram of a symmetric PSF equals the
        // half-sample reflective convolution with its interior row.
        G.taps_off = 0;
        if (P->periodic) {
            G.uniform = 1;
            G.map = MAP_WRAP;
        } else if (k == 0 && P->bc == RLS_BC_REFLECTIVE) {
            bool sym = true;
            for (int t = 0; t <= r; ++t)
                if (taps[t] != taps[2 * r - t]) sym = false;
            G.uniform = sym ? 1 : 0;
            G.map = sym ? MAP_REFLECT : MAP_ZERO;
            G.taps_off = sym ? (size_t)(nk / 2) * (2 * bw + 1) : 0;
        } else {
            G.uniform = 0;
            G.map = MAP_ZERO;
        }
        if (G.uniform) {
            G.htaps.resize(2 * bw + 1);
            RLS_HIP(hipMemcpyAsync(G.htaps.data(), G.table.as<double>() + G.taps_off,
                                   sizeof(double) * (2 * bw + 1),
                                   hipMemcpyDeviceToHost, s));
            RLS_HIP(hipStreamSynchronize(s));
            G.htaps32.assign(G.htaps.begin(), G.htaps.end());
        }
        if (P->prec != RLS_PREC_FP64) {   // FP32 copies for the V-cycle
            const size_t tn = (size_t)nk * (2 * bw + 1);
            RLS_TRY(dalloc(G.table32, sizeof(float) * tn));
            RLS_TRY(dalloc(G.diag32, sizeof(float) * nk));
            launch_to_f32(G.table.as<double>(), (int64_t)tn, 1, nullptr,
                          G.table32.as<float>(), s);
            launch_to_f32(G.diag.as<double>(), nk, 1, nullptr,
                          G.diag32.as<float>(), s);
        }
        bw = (bw + 2) / 2;
    }
    RLS_TRY(check_launch("build_direction"));
    RLS_HIP(hipStreamSynchronize(s));   // dtaps goes out of scope
    return RLS_OK;
}

// Sparse operator hierarchy (paper Section 3.2, one-sided): A_0 = A, then
// A_{k+1} = A_k P row by row, A_k^T by a deterministic transpose, column
// statistics diag(A_k^T A_k) and A_k^T A_k 1, and the dense A_c^T A_c of
// the coarsest level.  All on the GPU; the host only reads the sizes.
rls_status build_ct(rls_problem* P, const rls_op_desc* A, hipStream_t s) {
    const int64_t m = A->m;
    DBuf err;
    RLS_TRY(dalloc(err, sizeof(int)));
    RLS_HIP(hipMemsetAsync(err.p, 0, sizeof(int), s));
    {
        CtLevel& c = P->lev[0].ct;
        c.on = 1;
        c.m = m;
        c.nnz = A->nnz;
        RLS_TRY(dalloc(c.rp, sizeof(int64_t) * (m + 1)));
        RLS_TRY(dalloc(c.ci, sizeof(int) * c.nnz));
        RLS_TRY(dalloc(c.va, sizeof(double) * c.nnz));
        RLS_TRY(dalloc(c.va32, sizeof(float) * c.nnz));
        RLS_HIP(hipMemcpyAsync(c.rp.p, A->rowptr, sizeof(int64_t) * (m + 1),
                               hipMemcpyHostToDevice, s));
        RLS_HIP(hipMemcpyAsync(c.ci.p, A->col, sizeof(int) * c.nnz,
                               hipMemcpyHostToDevice, s));
        RLS_HIP(hipMemcpyAsync(c.va32.p, A->val, sizeof(float) * c.nnz,
                               hipMemcpyHostToDevice, s));
        launch_f64_from_f32(c.va32.as<float>(), c.nnz, c.va.as<double>(), s);
    }
    DBuf cnt, ones_y;
    RLS_TRY(dalloc(cnt, sizeof(int64_t) * (std::max<int64_t>(m, P->n()) + 1)));
    RLS_TRY(dalloc(ones_y, sizeof(double) * m));
    for (int k = 0; k < P->levels; ++k) {
        Level& Lk = P->lev[k];
        CtLevel& c = Lk.ct;
        const int64_t nk = Lk.n();
        if (k > 0) {
            const Level& Lf = P->lev[k - 1];
            const CtLevel& f = Lf.ct;
            c.on = 1;
            c.m = m;
            RLS_TRY(dalloc(c.rp, sizeof(int64_t) * (m + 1)));
            launch_csr_coarsen(f.rp.as<int64_t>(), f.ci.as<int>(),
                               f.va.as<double>(), m, Lf.nv, Lf.nh, P->periodic,
                               0, cnt.as<int64_t>(), nullptr, nullptr, nullptr,
                               err.as<int>(), s);
            launch_scan_excl(cnt.as<int64_t>(), m, c.rp.as<int64_t>(), s);
            int64_t nnz = 0;
            RLS_HIP(hipMemcpyAsync(&nnz, c.rp.as<int64_t>() + m, sizeof(int64_t),
                                   hipMemcpyDeviceToHost, s));
            RLS_HIP(hipStreamSynchronize(s));
            c.nnz = nnz;
            RLS_TRY(dalloc(c.ci, sizeof(int) * std::max<int64_t>(nnz, 1)));
            RLS_TRY(dalloc(c.va, sizeof(double) * std::max<int64_t>(nnz, 1)));
            launch_csr_coarsen(f.rp.as<int64_t>(), f.ci.as<int>(),
                               f.va.as<double>(), m, Lf.nv, Lf.nh, P->periodic,
                               1, nullptr, c.rp.as<int64_t>(), c.ci.as<int>(),
                               c.va.as<double>(), err.as<int>(), s);
            RLS_TRY(dalloc(c.va32, sizeof(float) * std::max<int64_t>(nnz, 1)));
            launch_to_f32(c.va.as<double>(), nnz, 1, nullptr, c.va32.as<float>(), s);
        }
        // transpose
        RLS_TRY(dalloc(c.rpt, sizeof(int64_t) * (nk + 1)));
        RLS_TRY(dalloc(c.cit, sizeof(int) * std::max<int64_t>(c.nnz, 1)));
        RLS_TRY(dalloc(c.vat, sizeof(double) * std::max<int64_t>(c.nnz, 1)));
        RLS_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int64_t) * (nk + 1), s));
        launch_csr_transpose_count(c.ci.as<int>(), c.nnz,
                                   cnt.as<unsigned long long>(), s);
        launch_scan_excl(cnt.as<int64_t>(), nk, c.rpt.as<int64_t>(), s);
        RLS_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int64_t) * (nk + 1), s));
        launch_csr_transpose_fill(c.rp.as<int64_t>(), c.ci.as<int>(),
                                  c.va.as<double>(), m, nk, c.rpt.as<int64_t>(),
                                  cnt.as<unsigned long long>(), c.cit.as<int>(),
                                  c.vat.as<double>(), err.as<int>(), s);
        RLS_TRY(dalloc(c.vat32, sizeof(float) * std::max<int64_t>(c.nnz, 1)));
        launch_to_f32(c.vat.as<double>(), c.nnz, 1, nullptr, c.vat32.as<float>(), s);
        // diag(A_k^T A_k) and A_k^T (A_k 1)
        RLS_TRY(dalloc(c.diag, sizeof(double) * nk));
        RLS_TRY(dalloc(c.diag32, sizeof(float) * nk));
        RLS_TRY(dalloc(c.rowabs, sizeof(double) * nk));
        launch_row_sumsq(c.rpt.as<int64_t>(), c.vat.as<double>(), nk,
                         c.diag.as<double>(), s);
        launch_to_f32(c.diag.as<double>(), nk, 1, nullptr, c.diag32.as<float>(), s);
        launch_spmv<double, double, double>(c.rp.as<int64_t>(), c.ci.as<int>(),
                                            c.va.as<double>(), m, nk, nullptr, 1,
                                            m, ones_y.as<double>(), 1, nullptr,
                                            nullptr, s);
        launch_spmv<double, double, double>(c.rpt.as<int64_t>(), c.cit.as<int>(),
                                            c.vat.as<double>(), nk, m,
                                            ones_y.as<double>(), 1, nk,
                                            c.rowabs.as<double>(), 1, nullptr,
                                            nullptr, s);
    }
    {
        const Level& C = P->lev[P->levels - 1];
        const int nc = (int)C.n();
        RLS_TRY(dalloc(P->ct_gram, sizeof(double) * (size_t)nc * nc));
        launch_dense_gram(C.ct.rpt.as<int64_t>(), C.ct.cit.as<int>(),
                          C.ct.vat.as<double>(), nc, P->ct_gram.as<double>(), s);
    }
    RLS_TRY(check_launch("build_ct"));
    int herr = 0;
    RLS_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
    RLS_HIP(hipStreamSynchronize(s));
    if (herr)
        return fail(RLS_E_UNSUPPORTED,
                    "sparse operator rows or columns too long for the on-GPU "
                    "hierarchy build (row: 512 nonzeros, column: 4096)");
    return RLS_OK;
}

rls_status install_weights(rls_problem* P, const double* d, hipStream_t s) {
    const int64_t n = P->n();
    if (d) {
        // validate the caller's weights before replacing the current ones
        DBuf bad;
        RLS_TRY(dalloc(bad, sizeof(int)));
        RLS_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
        launch_check_weights(d, 2 * n, bad.as<int>(), s);
        int hbad = 0;
        RLS_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost,
                               s));
        RLS_HIP(hipStreamSynchronize(s));
        if (hbad) return fail(RLS_E_ARG, "weights must be finite and >= 0");
        RLS_TRY(dalloc(P->weights, sizeof(double) * 2 * n));
        RLS_HIP(hipMemcpyAsync(P->weights.p, d, sizeof(double) * 2 * n,
                               hipMemcpyDeviceToDevice, s));
        P->unit_weights = 0;
    } else {
        P->weights.release();
        P->unit_weights = 1;
    }
    for (int k = 0; k < P->levels; ++k) {
        Level& L = P->lev[k];
        const int64_t m = L.n();
        RLS_TRY(dalloc(L.planes, sizeof(double) * 5 * m));
        RLS_TRY(dalloc(L.srowabs, sizeof(double) * m));
        L.periodic = P->periodic;
        L.nine = k > 0;
        if (k == 0)
            launch_fine_stencil(P->unit_weights ? nullptr : P->weights.as<double>(),
                                L.nv, L.nh, P->periodic, L.planes.as<double>(), s);
        else
            launch_galerkin_stencil(P->lev[k - 1].planes.as<double>(),
                                    P->lev[k - 1].nv, P->lev[k - 1].nh,
                                    P->periodic, L.planes.as<double>(), s);
        launch_stencil_rowabs(L.planes.as<double>(), L.nv, L.nh, P->periodic,
                              L.srowabs.as<double>(), s);
        if (P->prec != RLS_PREC_FP64) {   // FP32 copies for the V-cycle
            RLS_TRY(dalloc(L.planes32, sizeof(float) * 5 * m));
            launch_to_f32(L.planes.as<double>(), 5 * m, 1, nullptr,
                          L.planes32.as<float>(), s);
        }
    }
    RLS_TRY(check_launch("install_weights"));
    return RLS_OK;
}

// Band-only geometry (stencil scaled by a zero lambda) for A or A^T.
LevelGeom blur_geom(const rls_problem* P, int transpose) {
    LevelGeom g = P->lev[0].geom();
    g.gv = (transpose ? P->atv : P->av).dev();
    g.gh = (transpose ? P->ath : P->ah).dev();
    return g;
}

rls_status upload_lam(rls_problem* P, const double* lam, int nlam,
                      hipStream_t s) {
    std::vector<double> l2(nlam);
    for (int i = 0; i < nlam; ++i) {
        if (!(lam[i] > 0.0) || !std::isfinite(lam[i]))
            return fail(RLS_E_ARG, "lambda values must be finite and > 0");
        l2[i] = lam[i] * lam[i];
    }
    RLS_HIP(hipMemcpyAsync(P->w.lam2.p, l2.data(), sizeof(double) * nlam,
                           hipMemcpyHostToDevice, s));
    return RLS_OK;
}

// Per-sweep, lambda-dependent preconditioner data: Gershgorin bounds and
// Chebyshev coefficients per level, coarsest factorization per slot.
rls_status prepare_sweep(rls_problem* P, int nslot, hipStream_t s) {
    Work& w = P->w;
    const int L = P->levels;
    const int cs = 2 * P->nu_max;
    for (int k = 0; k + 1 < L; ++k) {
        double* rho = w.rho.as<double>() + (size_t)k * w.cap;
        if (P->is_ct)
            launch_gershgorin_ct(P->lev[k].geom(), w.lam2.as<double>(), nslot,
                                 rho, s);
        else
            launch_gershgorin(P->lev[k].geom(), w.lam2.as<double>(), nslot,
                              rho, s);
        launch_cheb_coeffs(rho, nslot, P->ratio[k], P->nu[k], cs,
                           w.cheb.as<double>() + (size_t)k * w.cap * cs, s);
    }
    const Level& C = P->lev[L - 1];
    const int nc = (int)C.n();
    if (P->is_ct)
        launch_coarse_assemble_ct(C.geom(), P->ct_gram.as<double>(),
                                  w.lam2.as<double>(), nslot,
                                  w.kc.as<double>(), s);
    else
        launch_coarse_assemble(C.geom(), w.lam2.as<double>(), nslot,
                               w.kc.as<double>(), s);
    launch_cholesky_inverse(w.kc.as<double>(), nc, nslot, w.winv.as<double>(),
                            w.info.as<int>(), s);
    RLS_TRY(check_launch("prepare_sweep"));
    std::vector<int> info(nslot);
    RLS_HIP(hipMemcpyAsync(info.data(), w.info.p, sizeof(int) * nslot,
                           hipMemcpyDeviceToHost, s));
    RLS_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nslot; ++i)
        if (info[i])
            return fail(RLS_E_NOT_SPD,
                        "coarsest matrix not positive definite (slot " +
                            std::to_string(i) + ", pivot " +
                            std::to_string(info[i]) + ")");
    return RLS_OK;
}

// PCG control folded into the level-0 kernels of a V-cycle: a convergence
// test in the first kernel, partial sums of r . z in the last.
struct CycleCtl {
    int gate = 0;
    SlotState* st = nullptr;
    int* active_w = nullptr;
    const double* part_rr = nullptr;
    int nrr = 0;
    double* dot_part = nullptr;
    int dot_stride = 0;
};

// Put the slot list in the kernel arguments when it is the sweep's list
// and short enough.
template <class R, class V>
static void inline_slots(const rls_problem* P, ApplyArgsT<R, V>& a) {
    a.zn = 0;
    if (!a.slots || a.slots != P->w.slots.as<int>() || !P->hslots ||
        P->hslots_n != a.nslot || a.nslot > ZINLINE)
        return;
    for (int i = 0; i < a.nslot; ++i) a.zslot[i] = P->hslots[i];
    a.zn = a.nslot;
}

// z = V-cycle(f) on level k (Algorithm 1, gamma = 1, V(nu, nu)), for the
// nslot slots listed in `slots` (null: slots 0..nslot-1).
template <class V>
V* lvec(std::vector<DBuf>& v64, std::vector<DBuf>& vlo, int k);
template <>
double* lvec<double>(std::vector<DBuf>& v64, std::vector<DBuf>&, int k) {
    return v64[k].as<double>();
}
template <>
float* lvec<float>(std::vector<DBuf>&, std::vector<DBuf>& vlo, int k) {
    return vlo[k].as<float>();
}
template <>
bf16* lvec<bf16>(std::vector<DBuf>&, std::vector<DBuf>& vlo, int k) {
    return vlo[k].as<bf16>();
}

// V is the V-cycle's vector type (double, or float or bf16 under flexible
// PCG), R its arithmetic type (double, float for both reduced types); the
// coarse tail always computes in FP64.
template <class V>
void vcycle(rls_problem* P, int k, int nslot, const int* slots,
            const int* active, const V* f, V* z, const CycleCtl& ctl,
            hipStream_t s) {
    using R = typename CompOf<V>::T;
    Work& w = P->w;
    const int L = P->levels;
    const int cs = 2 * P->nu_max;
    const int nu = P->nu[k];
    const bool top = k == 0;
    if (k >= P->kt) {
        TailArgsT<V> t;
        t.nlev = L - k;
        for (int i = 0; i < t.nlev; ++i) {
            const LevelGeom g = P->lev[k + i].geom();
            t.lev[i].nv = g.nv;
            t.lev[i].nh = g.nh;
            t.lev[i].gv = g.gv;
            t.lev[i].gh = g.gh;
            t.lev[i].S = g.S;
            t.lev[i].cheb = w.cheb.as<double>() + (size_t)(k + i) * w.cap * cs;
            t.lev[i].nu = P->nu[k + i];
        }
        t.cheb_stride = cs;
        t.periodic = P->periodic;
        t.lam2 = w.lam2.as<double>();
        t.slots = slots;
        t.active = active;
        t.f = f;
        t.z = z;
        t.W = w.winv.as<double>();
        if (top) {
            t.gate = ctl.gate;
            t.st = ctl.st;
            t.active_w = ctl.active_w;
            t.part_rr = ctl.part_rr;
            t.nrr = ctl.nrr;
            t.dot = ctl.dot_part != nullptr;
            t.part = ctl.dot_part;
            t.part_stride = ctl.dot_stride;
        }
        launch_tail(t, nslot, s);
        return;
    }
    // the kernel timer covers the FP64 finest-level step only
    constexpr bool TIMED = std::is_same<R, double>::value;
    const LevelGeomT<R> g = P->lev[k].template geom_t<R>();
    const double* cheb = w.cheb.as<double>() + (size_t)k * w.cap * cs;
    V* d = lvec<V>(w.ld, w.ldlo, k);
    ApplyArgsT<R, V> a;
    a.g = g;
    a.nslot = nslot;
    a.slots = slots;
    a.lam2 = w.lam2.as<double>();
    a.active = active;
    a.f = f;
    a.d = d;
    a.cheb_stride = cs;
    a.cheb_first = cheb;
    inline_slots(P, a);
    auto gate_first = [&](ApplyArgsT<R, V>& aa) {
        if (top && ctl.gate) {
            aa.gate = 1;
            aa.st = ctl.st;
            aa.active_w = ctl.active_w;
            aa.part_rr = ctl.part_rr;
            aa.nrr = ctl.nrr;
        }
    };
    V* fc = lvec<V>(w.lf, w.lflo, k + 1);
    V* zc = lvec<V>(w.lx, w.lxlo, k + 1);
    if (nu == 1) {
        // x1 = c f / diag never leaves the tiles: the restriction kernel
        // forms it on the fly, the correction kernel forms it again.
        ApplyArgsT<R, V> r = a;
        gate_first(r);
        r.fc = fc;
        level_apply(PRO_JACOBI, EPI_RESTRICT, r, s);
        vcycle(P, k + 1, nslot, slots, active, (const V*)fc, zc, CycleCtl(), s);
        ApplyArgsT<R, V> c = a;
        c.ec = zc;
        c.out = z;
        c.cheb = cheb;
        if (top && ctl.dot_part) {
            c.dot = 1;
            c.part = ctl.dot_part;
            c.part_stride = ctl.dot_stride;
        }
        level_apply(PRO_PROLONG_JAC, EPI_CHEB, c, s);
        return;
    }
    // nu >= 2.  Buffer writes: the first pre-smoothing step writes buffer 0,
    // nu - 2 more pre steps and nu post steps each swap; choose buffer 0 so
    // that the result lands in z.
    const int swaps = (nu - 2) + nu;
    V* bufs[2];
    bufs[swaps % 2 == 0 ? 0 : 1] = z;
    bufs[swaps % 2 == 0 ? 1 : 0] = lvec<V>(w.lxb, w.lxblo, k);
    int cur = 0;
    {
        ApplyArgsT<R, V> j = a;
        gate_first(j);
        j.out = bufs[cur];
        j.cheb = cheb + 2;
        level_apply(PRO_JACOBI, EPI_CHEB, j, s);   // x1 = c f / diag, step 2
    }
    if (TIMED && top && nu > 2) run_begin(P, s);
    for (int st = 2; st < nu; ++st) {
        ApplyArgsT<R, V> c = a;
        c.in = bufs[cur];
        c.out = bufs[1 - cur];
        c.cheb = cheb + 2 * st;
        c.fine_xstep = st - 2;
        if (top) smooth_fine(P, c, s);
        else level_apply(PRO_PLAIN, EPI_CHEB, c, s);
        cur = 1 - cur;
    }
    if (TIMED && top && nu > 2) run_end(P, s);
    {
        ApplyArgsT<R, V> r = a;                     // residual + restriction
        r.in = bufs[cur];
        r.fc = fc;
        level_apply(PRO_PLAIN, EPI_RESTRICT, r, s);
    }
    vcycle(P, k + 1, nslot, slots, active, (const V*)fc, zc, CycleCtl(), s);
    for (int st = 0; st < nu; ++st) {              // correction + smoothing
        ApplyArgsT<R, V> c = a;
        c.in = bufs[cur];
        c.out = bufs[1 - cur];
        c.cheb = cheb + 2 * st;
        c.ec = st == 0 ? zc : nullptr;
        if (top && ctl.dot_part && st == nu - 1) {
            c.dot = 1;
            c.part = ctl.dot_part;
            c.part_stride = ctl.dot_stride;
        }
        if (TIMED && top && st == 1) run_begin(P, s);
        c.fine_xstep = st - 1;
        if (top && st > 0) smooth_fine(P, c, s);
        else level_apply(st == 0 ? PRO_PROLONG : PRO_PLAIN, EPI_CHEB, c, s);
        if (TIMED && top && st > 0 && st == nu - 1) run_end(P, s);
        cur = 1 - cur;
    }
}

// Autotuning of the tiled finest-level Chebyshev kernel: for the slot
// counts a sweep can reach, in increasing order, time its 256- and
// 512-thread workgroups on the V-cycle's (zeroed) workspace vectors and keep
// the faster; once 256 threads have won at two consecutive counts, larger
// counts take 256 without timing (more slots only add workgroups per CU,
// which favours the smaller size).  The two sizes give bit-identical
// results, so the choice only affects speed.  It runs once per problem and
// slot count, at the start of a sweep, before any graph capture; problems
// the tiled kernel does not serve are skipped.
template <class V>
rls_status tune_fine_t(rls_problem* P, std::vector<int>& tab, int nmax,
                       hipStream_t s) {
    using R = typename CompOf<V>::T;
    Work& w = P->w;
    nmax = std::min(nmax, FINE_ZMAX);
    bool need = false;
    for (int z = 1; z <= nmax; ++z) need = need || tab[z] == 0;
    if (!need || P->fine_generic || P->is_ct) return RLS_OK;
    const size_t n = (size_t)P->n();
    V *in, *out, *d, *f;
    if constexpr (std::is_same<V, double>::value) {
        in = w.lxb[0].as<double>();
        out = w.lt[0].as<double>();
        d = w.ld[0].as<double>();
        f = w.r.as<double>();
    } else {
        in = w.lxblo[0].as<V>();
        out = w.zlo.as<V>();
        d = w.ldlo[0].as<V>();
        f = w.rlo.as<V>();
    }
    for (V* b : {in, out, d, f})
        RLS_HIP(hipMemsetAsync(b, 0, sizeof(V) * (size_t)nmax * n, s));
    ApplyArgsT<R, V> a;
    a.g = P->lev[0].template geom_t<R>();
    a.lam2 = w.lam2.as<double>();
    a.in = in;
    a.out = out;
    a.d = d;
    a.f = f;
    a.cheb = w.cheb.as<double>();      // level 0, any step's coefficients
    a.cheb_stride = 2 * P->nu_max;
    hipEvent_t ev[2];
    RLS_HIP(hipEventCreate(&ev[0]));
    RLS_HIP(hipEventCreate(&ev[1]));
    rls_status st = RLS_OK;
    int wins256 = 0;   // consecutive slot counts where 256 threads won
    for (int z = 1; z <= nmax && st == RLS_OK; ++z) {
        if (tab[z]) {
            wins256 = tab[z] == 256 ? wins256 + 1 : 0;
            continue;
        }
        if (wins256 >= 2) {   // larger launches only favour 256 threads more
            tab[z] = 256;
            continue;
        }
        a.nslot = z;
        float best[2] = {1e30f, 1e30f};
        for (int rep = 0; rep < 3 && st == RLS_OK; ++rep) {
            for (int v = 0; v < 2; ++v) {
                a.fine_nt = v ? 512 : 256;
                if (!launch_smooth_fine_tiled(a, s)) {   // not served
                    std::fill(tab.begin(), tab.end(), 256);
                    st = check_launch("tune_fine");
                    break;
                }
                hipEventRecord(ev[0], s);
                for (int k = 0; k < 4; ++k) launch_smooth_fine_tiled(a, s);
                hipEventRecord(ev[1], s);
                if (hipEventSynchronize(ev[1]) != hipSuccess) {
                    st = fail(RLS_E_HIP, "tune_fine: event");
                    break;
                }
                float ms = 0.f;
                hipEventElapsedTime(&ms, ev[0], ev[1]);
                best[v] = std::min(best[v], ms);
            }
            if (tab[z]) break;
        }
        if (st == RLS_OK && !tab[z]) tab[z] = best[1] < best[0] ? 512 : 256;
        wins256 = tab[z] == 256 ? wins256 + 1 : 0;
    }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (st != RLS_OK) return st;
    return check_launch("tune_fine");
}
rls_status tune_fine(rls_problem* P, int nmax, hipStream_t s) {
    if (P->prec == RLS_PREC_FP64) return tune_fine_t<double>(P, P->fine_nt64, nmax, s);
    if (P->prec == RLS_PREC_MIXED_BF16)
        return tune_fine_t<bf16>(P, P->fine_ntlo, nmax, s);
    return tune_fine_t<float>(P, P->fine_ntlo, nmax, s);
}

// z = M r through the reduced-precision V-cycle with vectors of type V:
// narrowing of r (after the convergence test when st is given), the
// V-cycle, widening of z with the partials of r . z (and z . q).
template <class V>
void vcycle_lo_t(rls_problem* p, int ns, const int* sl, int* active,
                 SlotState* st, const double* part_rr, int nrr, const double* r,
                 double* z, const double* q, double* part_rz, double* part_zq,
                 int npart, hipStream_t s) {
    Work& w = p->w;
    const int64_t n = p->n();
    V* rlo = w.rlo.as<V>();
    V* zlo = w.zlo.as<V>();
    launch_vc_enter<V>(st, active, sl, ns, part_rr, nrr, n, r, rlo, s);
    vcycle<V>(p, 0, ns, sl, active, (const V*)rlo, zlo, CycleCtl(), s);
    launch_vc_exit<V>(sl, active, ns, n, npart, zlo, z, r, q, part_rz, part_zq,
                      s);
}
void vcycle_lo(rls_problem* p, int ns, const int* sl, int* active,
               SlotState* st, const double* part_rr, int nrr, const double* r,
               double* z, const double* q, double* part_rz, double* part_zq,
               int npart, hipStream_t s) {
    if (p->prec == RLS_PREC_MIXED_BF16)
        vcycle_lo_t<bf16>(p, ns, sl, active, st, part_rr, nrr, r, z, q, part_rz,
                          part_zq, npart, s);
    else
        vcycle_lo_t<float>(p, ns, sl, active, st, part_rr, nrr, r, z, q,
                           part_rz, part_zq, npart, s);
}

rls_status validate_grid(const rls_grid_desc* g) {
    if (g->nv < 4 || g->nh < 4) return fail(RLS_E_ARG, "grid must be >= 4 x 4");
    if (g->levels < 1 || g->levels > 16) return fail(RLS_E_ARG, "levels in 1..16");
    if (g->nu < 1 || g->nu > 256) return fail(RLS_E_ARG, "nu in 1..256");
    if (g->nu_coarse < 0 || g->nu_coarse > 256)
        return fail(RLS_E_ARG, "nu_coarse in 0..256");
    if (!(g->cheb_ratio > 1.0) || !std::isfinite(g->cheb_ratio))
        return fail(RLS_E_ARG, "cheb_ratio must be > 1");
    if (g->cheb_ratio_coarse != 0.0 &&
        (!(g->cheb_ratio_coarse > 1.0) || !std::isfinite(g->cheb_ratio_coarse)))
        return fail(RLS_E_ARG, "cheb_ratio_coarse must be 0 or > 1");
    if (g->lbc != RLS_L_NEUMANN && g->lbc != RLS_L_PERIODIC)
        return fail(RLS_E_ARG, "unknown gradient boundary");
    for (int k = 0; k < g->levels; ++k) {
        const int v = g->nv >> k, h = g->nh >> k;
        if ((v << k) != g->nv || (h << k) != g->nh)
            return fail(RLS_E_ARG, "grid not divisible by 2^(levels-1)");
        if (v < 4 || h < 4)
            return fail(RLS_E_ARG, "every level must be at least 4 x 4");
    }
    const int64_t nc = (int64_t)(g->nv >> (g->levels - 1)) * (g->nh >> (g->levels - 1));
    if (nc > 1024)
        return fail(RLS_E_ARG, "coarsest level exceeds 1024 unknowns; add levels");
    if (g->precision != RLS_PREC_FP64 && g->precision != RLS_PREC_MIXED_FP32 &&
        g->precision != RLS_PREC_MIXED_BF16)
        return fail(RLS_E_UNSUPPORTED,
                    "precision must be RLS_PREC_FP64, RLS_PREC_MIXED_FP32 or "
                    "RLS_PREC_MIXED_BF16");
    return RLS_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char* rls_last_error(void) { return g_last_error.c_str(); }

rls_status rls_solve_batch(rls_sweep* sweeps, int nsweep, void* stream) {
    g_last_error.clear();
    if (!sweeps || nsweep < 1) return fail(RLS_E_ARG, "empty batch");
    for (int i = 0; i < nsweep; ++i) {
        if (!sweeps[i].prob) return fail(RLS_E_ARG, "null handle in batch");
        for (int j = 0; j < i; ++j)
            if (sweeps[j].prob == sweeps[i].prob)
                return fail(RLS_E_ARG, "a handle is listed twice in the batch");
    }
    hipStream_t s = (hipStream_t)stream;
    // order every problem's stream after the caller's work
    hipEvent_t ready = nullptr;
    RLS_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ready, s);
    for (int i = 0; i < nsweep && e == hipSuccess; ++i) {
        rls_problem* p = sweeps[i].prob;
        if (!p->bstream) e = hipStreamCreateWithFlags(&p->bstream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamWaitEvent(p->bstream, ready, 0);
    }
    if (e != hipSuccess) {
        (void)hipEventDestroy(ready);
        return fail(RLS_E_HIP, std::string("batch streams: ") + hipGetErrorString(e));
    }
    std::vector<std::string> msgs(nsweep);
    auto run = [&](int i) {
        rls_sweep& w = sweeps[i];
        (void)hipSetDevice(w.prob->device);
        w.status = rls_solve_sweep(w.prob, w.b, w.lam, w.nlam, w.tol, w.opts,
                                   w.x0, w.x, w.resnorm, w.seminorm, w.info,
                                   w.prob->bstream);
        if (w.status != RLS_OK) msgs[i] = rls_last_error();
    };
    std::vector<std::thread> pool;
    pool.reserve(nsweep);
    for (int i = 1; i < nsweep; ++i) pool.emplace_back(run, i);
    run(0);
    for (auto& th : pool) th.join();
    (void)hipEventDestroy(ready);
    // every sweep synchronized its stream before returning
    for (int i = 0; i < nsweep; ++i)
        if (sweeps[i].status != RLS_OK)
            return fail(sweeps[i].status, "sweep " + std::to_string(i) + ": " + msgs[i]);
    return RLS_OK;
}

void rls_destroy(rls_problem* p) { delete p; }

// rls_setup for a sparse (tomography) operator.
static rls_status setup_ct(rls_problem** out, const rls_op_desc* A,
                           const rls_grid_desc* g, const double* d,
                           void* stream) {
    if (g->precision != RLS_PREC_MIXED_FP32)
        return fail(RLS_E_UNSUPPORTED,
                    "sparse operators run with RLS_PREC_MIXED_FP32 (FP32 "
                    "V-cycle, FP64 PCG)");
    const int64_t n = (int64_t)g->nv * g->nh;
    if (n > (int64_t)1 << 28)
        return fail(RLS_E_UNSUPPORTED, "grids are limited to 2^28 points");
    if (A->m < 1 || A->nnz < 1 || !A->rowptr || !A->col || !A->val)
        return fail(RLS_E_ARG, "sparse operator: m, nnz >= 1 and host rowptr, "
                               "col, val required");
    if (A->rowptr[0] != 0 || A->rowptr[A->m] != A->nnz)
        return fail(RLS_E_ARG, "rowptr must start at 0 and end at nnz");
    for (int64_t i = 0; i < A->m; ++i) {
        if (A->rowptr[i + 1] < A->rowptr[i])
            return fail(RLS_E_ARG, "rowptr must be nondecreasing");
        if (A->rowptr[i + 1] - A->rowptr[i] > 512)
            return fail(RLS_E_UNSUPPORTED, "rows are limited to 512 nonzeros");
        for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e) {
            if (A->col[e] < 0 || A->col[e] >= n ||
                (e > A->rowptr[i] && A->col[e] <= A->col[e - 1]))
                return fail(RLS_E_ARG, "columns must be in [0, nv*nh) and "
                                       "strictly increasing within a row");
            if (!(A->val[e] >= 0.0f) || !std::isfinite(A->val[e]))
                return fail(RLS_E_ARG, "values must be finite and >= 0 (ray "
                                       "lengths)");
        }
    }
    std::unique_ptr<rls_problem> P(new rls_problem());
    RLS_HIP(hipGetDevice(&P->device));
    RLS_HIP(hipStreamCreateWithFlags(&P->cstream, hipStreamNonBlocking));
    configure_apply_kernels();
    P->nv = g->nv;
    P->nh = g->nh;
    P->levels = g->levels;
    P->prec = g->precision;
    P->is_ct = 1;
    P->ct_m = A->m;
    for (int k = 0; k < g->levels; ++k) {
        const bool fine = k == 0;
        P->nu.push_back(fine || g->nu_coarse == 0 ? g->nu : g->nu_coarse);
        P->ratio.push_back(fine || g->cheb_ratio_coarse == 0.0
                               ? g->cheb_ratio : g->cheb_ratio_coarse);
    }
    P->nu_max = *std::max_element(P->nu.begin(), P->nu.end());
    P->bc = -1;
    P->lbc = g->lbc;
    P->periodic = g->lbc == RLS_L_PERIODIC;
    P->lev.resize(P->levels);
    for (int k = 0; k < P->levels; ++k) {
        P->lev[k].nv = P->nv >> k;
        P->lev[k].nh = P->nh >> k;
    }
    P->kt = P->levels - 1;    // the tail kernel solves the coarsest level only
    hipStream_t s = (hipStream_t)stream;
    RLS_TRY(build_ct(P.get(), A, s));
    RLS_TRY(install_weights(P.get(), d, s));
    RLS_HIP(hipStreamSynchronize(s));
    *out = P.release();
    return RLS_OK;
}

rls_status rls_setup(rls_problem** out, const rls_op_desc* A,
                     const rls_grid_desc* g, const double* d, void* stream) {
    g_last_error.clear();
    if (!out || !A || !g) return fail(RLS_E_ARG, "null argument");
    *out = nullptr;
    RLS_TRY(validate_grid(g));
    if (A->kind == RLS_OP_CSR) return setup_ct(out, A, g, d, stream);
    if (A->kind != RLS_OP_BLUR_SEPARABLE) return fail(RLS_E_ARG, "unknown operator kind");
    if (!A->taps_v || !A->taps_h) return fail(RLS_E_ARG, "null taps");
    if (A->r_v < 0 || A->r_h < 0 || 2 * A->r_v + 1 > g->nv || 2 * A->r_h + 1 > g->nh)
        return fail(RLS_E_ARG, "blur radius must satisfy 2r+1 <= n");
    const int pair_ok = (A->bc == RLS_BC_PERIODIC && g->lbc == RLS_L_PERIODIC) ||
                        (A->bc == RLS_BC_REFLECTIVE && g->lbc == RLS_L_NEUMANN) ||
                        (A->bc == RLS_BC_ZERO && g->lbc == RLS_L_NEUMANN);
    if (A->bc < 0 || A->bc > 2) return fail(RLS_E_ARG, "unknown blur boundary");
    if (!pair_ok)
        return fail(RLS_E_UNSUPPORTED,
                    "supported (blur, gradient) boundary pairs: (periodic, "
                    "periodic), (reflective, neumann), (zero, neumann)");
    if ((int64_t)g->nv * g->nh > (int64_t)1 << 28)
        return fail(RLS_E_UNSUPPORTED, "grids are limited to 2^28 points");
    {
        // the finest level has the widest Gram bands (half-width 2r); its
        // restriction tile with per-row coefficients is the largest LDS user
        LevelGeom g0;
        g0.nv = g->nv;
        g0.nh = g->nh;
        g0.gv.bw = 2 * A->r_v;
        g0.gh.bw = 2 * A->r_h;
        const size_t need = apply_lds_bytes(g0, EPI_RESTRICT);
        const size_t have = 160 * 1024 - sizeof(double) * APPLY_THREADS;
        if (need > have)
            return fail(RLS_E_UNSUPPORTED,
                        "blur radius too large for the level-operator tile: "
                        "needs " + std::to_string(need) + " bytes of LDS, " +
                        std::to_string(have) + " available");
    }
    std::unique_ptr<rls_problem> P(new rls_problem());
    RLS_HIP(hipGetDevice(&P->device));
    RLS_HIP(hipStreamCreateWithFlags(&P->cstream, hipStreamNonBlocking));
    configure_apply_kernels();
    P->nv = g->nv;
    P->nh = g->nh;
    P->levels = g->levels;
    P->prec = g->precision;
    for (int k = 0; k < g->levels; ++k) {
        const bool fine = k == 0;
        P->nu.push_back(fine || g->nu_coarse == 0 ? g->nu : g->nu_coarse);
        P->ratio.push_back(fine || g->cheb_ratio_coarse == 0.0
                               ? g->cheb_ratio : g->cheb_ratio_coarse);
    }
    P->nu_max = *std::max_element(P->nu.begin(), P->nu.end());
    P->bc = A->bc;
    P->lbc = g->lbc;
    P->periodic = g->lbc == RLS_L_PERIODIC;
    {
        const char* e = std::getenv("RLS_FINE_KERNEL");
        P->fine_generic = e && std::strcmp(e, "generic") == 0;
    }
    P->r_v = A->r_v;
    P->r_h = A->r_h;
    P->taps_v.assign(A->taps_v, A->taps_v + 2 * A->r_v + 1);
    P->taps_h.assign(A->taps_h, A->taps_h + 2 * A->r_h + 1);
    for (double t : P->taps_v)
        if (!std::isfinite(t)) return fail(RLS_E_ARG, "non-finite tap");
    for (double t : P->taps_h)
        if (!std::isfinite(t)) return fail(RLS_E_ARG, "non-finite tap");
    P->lev.resize(P->levels);
    for (int k = 0; k < P->levels; ++k) {
        P->lev[k].nv = P->nv >> k;
        P->lev[k].nh = P->nh >> k;
    }
    P->kt = P->levels - 1;
    while (P->kt > 0 && P->lev[P->kt - 1].n() <= TAIL_MAX_POINTS &&
           P->levels - (P->kt - 1) <= TAIL_MAX_LEVELS)
        --P->kt;
    hipStream_t s = (hipStream_t)stream;
    RLS_TRY(build_direction(P.get(), P->taps_v, P->r_v, 0, s));
    RLS_TRY(build_direction(P.get(), P->taps_h, P->r_h, 1, s));
    RLS_TRY(install_weights(P.get(), d, s));
    RLS_HIP(hipStreamSynchronize(s));
    *out = P.release();
    return RLS_OK;
}

rls_status rls_set_weights(rls_problem* p, const double* d, void* stream) {
    g_last_error.clear();
    if (!p) return fail(RLS_E_STATE, "null handle");
    hipStream_t s = (hipStream_t)stream;
    RLS_TRY(install_weights(p, d, s));
    RLS_HIP(hipStreamSynchronize(s));
    return RLS_OK;
}

namespace {

// eq. (g) on the problem's own weights: D <- diag(1 - (|D L x| /
// ||D L x||_inf)^q) D, then the per-weighting set-up (stencils of every
// level) for the new D.
rls_status update_weights(rls_problem* P, const double* x, double q,
                          double* top_host, hipStream_t s) {
    const int64_t n = P->n();
    DBuf part, dnew, top;
    RLS_TRY(dalloc(part, sizeof(double) * weight_update_parts()));
    RLS_TRY(dalloc(dnew, sizeof(double) * 2 * n));
    RLS_TRY(dalloc(top, sizeof(double)));
    launch_weight_update(x, P->unit_weights ? nullptr : P->weights.as<double>(),
                         P->nv, P->nh, P->periodic, q, part.as<double>(),
                         dnew.as<double>(), top.as<double>(), s);
    RLS_TRY(check_launch("weight update"));
    RLS_TRY(install_weights(P, dnew.as<double>(), s));
    if (top_host)
        RLS_HIP(hipMemcpyAsync(top_host, top.p, sizeof(double),
                               hipMemcpyDeviceToHost, s));
    RLS_HIP(hipStreamSynchronize(s));
    return RLS_OK;
}

rls_status check_lcurve(const double* lam, const double* rho,
                        const double* eta, int m) {
    if (!lam || !rho || !eta) return fail(RLS_E_ARG, "null L-curve array");
    if (m < 3) return fail(RLS_E_ARG, "the L-curve needs at least 3 points");
    for (int i = 0; i < m; ++i) {
        if (!(std::isfinite(lam[i]) && lam[i] > 0 && std::isfinite(rho[i]) &&
              rho[i] > 0 && std::isfinite(eta[i]) && eta[i] > 0))
            return fail(RLS_E_ARG, "lambda, residual and seminorm must be "
                                   "positive and finite");
        if (i && !(lam[i] > lam[i - 1]))
            return fail(RLS_E_ARG, "lambdas must be strictly increasing");
    }
    return RLS_OK;
}

}  // namespace

rls_status rls_update_weights(rls_problem* p, const double* x, double q,
                              double* gmax, void* stream) {
    g_last_error.clear();
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (!x) return fail(RLS_E_ARG, "null x");
    if (!(std::isfinite(q) && q > 0)) return fail(RLS_E_ARG, "q must be > 0");
    return update_weights(p, x, q, gmax, (hipStream_t)stream);
}

rls_status rls_get_weights(const rls_problem* p, double* d, void* stream) {
    g_last_error.clear();
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (!d) return fail(RLS_E_ARG, "null d");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n2 = 2 * p->n();
    if (p->unit_weights) {
        std::vector<double> ones(n2, 1.0);
        RLS_HIP(hipMemcpyAsync(d, ones.data(), sizeof(double) * n2,
                               hipMemcpyHostToDevice, s));
    } else {
        RLS_HIP(hipMemcpyAsync(d, p->weights.p, sizeof(double) * n2,
                               hipMemcpyDeviceToDevice, s));
    }
    RLS_HIP(hipStreamSynchronize(s));
    return RLS_OK;
}

rls_status rls_lcurve_corner(const double* lam, const double* rho,
                             const double* eta, int m, int* index) {
    g_last_error.clear();
    if (!index) return fail(RLS_E_ARG, "null index");
    RLS_TRY(check_lcurve(lam, rho, eta, m));
    *index = lcurve_corner_host(lam, rho, eta, m);
    return RLS_OK;
}

rls_status rls_trim_window(int i_prev, int m, int* lo, int* hi) {
    g_last_error.clear();
    if (!lo || !hi) return fail(RLS_E_ARG, "null output");
    if (m < TRIM_SIZE) return fail(RLS_E_ARG, "pruning needs at least 10 lambdas");
    if (i_prev < 0 || i_prev >= m) return fail(RLS_E_ARG, "index out of range");
    trim_window_host(i_prev, m, lo, hi);
    return RLS_OK;
}

rls_status rls_regularize(rls_problem* p, const double* b, const double* lam,
                          int m, double q, double tol,
                          const rls_sweep_opts* opts, int maxouter,
                          int* chosen, double* x, rls_outer_info* info,
                          void* stream) {
    g_last_error.clear();
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (!b || !lam || !x || !chosen) return fail(RLS_E_ARG, "null argument");
    if (m < TRIM_SIZE) return fail(RLS_E_ARG, "Algorithm 2 needs at least 10 lambdas");
    if (maxouter < 1) return fail(RLS_E_ARG, "maxouter must be >= 1");
    if (!(std::isfinite(q) && q > 0)) return fail(RLS_E_ARG, "q must be > 0");
    for (int i = 0; i < m; ++i)
        if (!(std::isfinite(lam[i]) && lam[i] > 0) || (i && !(lam[i] > lam[i - 1])))
            return fail(RLS_E_ARG, "lambdas must be positive, finite and "
                                   "strictly increasing");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = p->n();
    // every lambda's latest solution: the warm start of its next solve
    DBuf xall;
    RLS_TRY(dalloc(xall, sizeof(double) * (size_t)m * n));
    RLS_HIP(hipMemsetAsync(xall.p, 0, sizeof(double) * (size_t)m * n, s));
    RLS_TRY(install_weights(p, nullptr, s));           // D = I
    std::vector<double> res(m), sem(m);
    std::vector<rls_solve_info> sinfo(m);
    rls_outer_info out{};
    int stopped = 0, ell = 0, pick = 0;
    for (; ell < maxouter && !stopped; ++ell) {
        int lo = 0, hi = m - 1;
        if (ell) trim_window_host(chosen[ell - 1], m, &lo, &hi);
        const int cnt = hi - lo + 1;
        double* xs = xall.as<double>() + (size_t)lo * n;
        RLS_TRY(rls_solve_sweep(p, b, lam + lo, cnt, tol, opts, xs, xs,
                                res.data(), sem.data(), sinfo.data(), stream));
        for (int i = 0; i < cnt; ++i) out.iters += sinfo[i].iters;
        for (int i = 0; i < cnt; ++i)
            if (!(res[i] > 0 && sem[i] > 0 && std::isfinite(res[i]) &&
                  std::isfinite(sem[i])))
                return fail(RLS_E_ARG, "a sweep returned a zero or non-finite "
                                       "L-curve point");
        pick = lo + lcurve_corner_host(lam + lo, res.data(), sem.data(), cnt);
        chosen[ell] = pick;
        stopped = ell >= 2 && chosen[ell - 2] == pick && chosen[ell - 1] == pick;
        if (!stopped && ell + 1 < maxouter)
            RLS_TRY(update_weights(p, xall.as<double>() + (size_t)pick * n, q,
                                   nullptr, s));
    }
    RLS_HIP(hipMemcpyAsync(x, xall.as<double>() + (size_t)pick * n,
                           sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    RLS_HIP(hipStreamSynchronize(s));
    out.outer = ell;
    out.stopped = stopped;
    out.chosen_index = pick;
    if (info) *info = out;
    return RLS_OK;
}

rls_status rls_level_shape(const rls_problem* p, int level, int* nv, int* nh) {
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (level < 0 || level >= p->levels) return fail(RLS_E_ARG, "level out of range");
    if (nv) *nv = p->lev[level].nv;
    if (nh) *nh = p->lev[level].nh;
    return RLS_OK;
}

rls_status rls_get_stencil(const rls_problem* p, int level, double* out) {
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (level < 0 || level >= p->levels || !out) return fail(RLS_E_ARG, "bad level/out");
    const Level& L = p->lev[level];
    RLS_HIP(hipMemcpy(out, L.planes.p, sizeof(double) * 5 * L.n(),
                      hipMemcpyDeviceToHost));
    return RLS_OK;
}

rls_status rls_get_gram_band(const rls_problem* p, int level, int dir, int* bw,
                             double* out) {
    if (p && p->is_ct)
        return fail(RLS_E_UNSUPPORTED, "sparse operators have no Gram bands");
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (level < 0 || level >= p->levels || dir < 0 || dir > 1)
        return fail(RLS_E_ARG, "bad level/direction");
    const Band& B = dir == 0 ? p->lev[level].gv : p->lev[level].gh;
    if (bw) *bw = B.bw;
    if (out)
        RLS_HIP(hipMemcpy(out, B.table.p, sizeof(double) * B.n * (2 * B.bw + 1),
                          hipMemcpyDeviceToHost));
    return RLS_OK;
}

rls_status rls_apply_normal(rls_problem* p, int level, const double* lam,
                            int nlam, const double* v, double* out,
                            void* stream) {
    g_last_error.clear();
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (level < 0 || level >= p->levels || nlam < 1 || !lam || !v || !out)
        return fail(RLS_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    RLS_TRY(ensure_work(p, nlam));
    RLS_TRY(upload_lam(p, lam, nlam, s));
    ApplyArgs a;
    a.g = p->lev[level].geom();
    a.nslot = nlam;
    a.lam2 = p->w.lam2.as<double>();
    a.in = v;
    a.out = out;
    level_apply(PRO_PLAIN, EPI_STORE, a, s);
    RLS_TRY(check_launch("rls_apply_normal"));
    RLS_HIP(hipStreamSynchronize(s));
    return RLS_OK;
}

rls_status rls_gershgorin(rls_problem* p, int level, const double* lam,
                          int nlam, double* rho, void* stream) {
    g_last_error.clear();
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (level < 0 || level >= p->levels || nlam < 1 || !lam || !rho)
        return fail(RLS_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    RLS_TRY(ensure_work(p, nlam));
    RLS_TRY(upload_lam(p, lam, nlam, s));
    if (p->is_ct)
        launch_gershgorin_ct(p->lev[level].geom(), p->w.lam2.as<double>(), nlam,
                             p->w.rho.as<double>(), s);
    else
        launch_gershgorin(p->lev[level].geom(), p->w.lam2.as<double>(), nlam,
                          p->w.rho.as<double>(), s);
    RLS_TRY(check_launch("rls_gershgorin"));
    RLS_HIP(hipMemcpyAsync(rho, p->w.rho.p, sizeof(double) * nlam,
                           hipMemcpyDeviceToHost, s));
    RLS_HIP(hipStreamSynchronize(s));
    return RLS_OK;
}

rls_status rls_vcycle(rls_problem* p, const double* lam, int nlam,
                      const double* r, double* z, void* stream) {
    g_last_error.clear();
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (nlam < 1 || !lam || !r || !z) return fail(RLS_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    RLS_TRY(ensure_work(p, nlam));
    RLS_TRY(upload_lam(p, lam, nlam, s));
    RLS_TRY(prepare_sweep(p, nlam, s));
    if (p->prec != RLS_PREC_FP64) {
        vcycle_lo(p, nlam, nullptr, nullptr, nullptr, nullptr, 0, r, z, nullptr,
                  p->w.part_rz.as<double>(), nullptr,
                  apply_tiles(p->lev[0].geom()), s);
    } else {
        vcycle(p, 0, nlam, nullptr, nullptr, r, z, CycleCtl(), s);
    }
    RLS_TRY(check_launch("rls_vcycle"));
    RLS_HIP(hipStreamSynchronize(s));
    return RLS_OK;
}

rls_status rls_kernel_timer(rls_problem* p, int enable) {
    if (!p) return fail(RLS_E_STATE, "null handle");
    p->timer_on = enable != 0;
    p->timer_launches = 0;
    p->timer_seconds = p->timer_bytes = 0.0;
    return RLS_OK;
}

rls_status rls_kernel_timer_read(const rls_problem* p, long long* launches,
                                 double* seconds, double* bytes) {
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (launches) *launches = p->timer_launches;
    if (seconds) *seconds = p->timer_seconds;
    if (bytes) *bytes = p->timer_bytes;
    return RLS_OK;
}

static rls_status apply_blur(rls_problem* p, int transpose, const double* x,
                             double* y, int nvec, hipStream_t s) {
    RLS_TRY(ensure_work(p, nvec));
    if (p->is_ct) {
        // y = A x (n -> m) or y = A^T x (m -> n), FP64
        const CtLevel& c = p->lev[0].ct;
        const int64_t n = p->n(), m = p->ct_m;
        if (!transpose)
            launch_spmv<double, double, double>(
                c.rp.as<int64_t>(), c.ci.as<int>(), c.va.as<double>(), m, n,
                x, 0, m, y, nvec, nullptr, nullptr, s);
        else
            launch_spmv<double, double, double>(
                c.rpt.as<int64_t>(), c.cit.as<int>(), c.vat.as<double>(), n, m,
                x, 0, n, y, nvec, nullptr, nullptr, s);
        return check_launch("apply_operator");
    }
    ApplyArgs a;
    a.g = blur_geom(p, transpose);
    a.nslot = nvec;
    a.lam2 = p->w.zero_lam2.as<double>();
    a.in = x;
    a.out = y;
    launch_apply(PRO_PLAIN, EPI_STORE, a, s);
    return check_launch("apply_blur");
}

rls_status rls_apply_forward(rls_problem* p, const double* x, double* y,
                             int nvec, void* stream) {
    g_last_error.clear();
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (!x || !y || nvec < 1) return fail(RLS_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    RLS_TRY(apply_blur(p, 0, x, y, nvec, s));
    RLS_HIP(hipStreamSynchronize(s));
    return RLS_OK;
}

rls_status rls_apply_adjoint(rls_problem* p, const double* y, double* x,
                             int nvec, void* stream) {
    g_last_error.clear();
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (!x || !y || nvec < 1) return fail(RLS_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    RLS_TRY(apply_blur(p, 1, y, x, nvec, s));
    RLS_HIP(hipStreamSynchronize(s));
    return RLS_OK;
}

rls_status rls_solve_sweep(rls_problem* p, const double* b, const double* lam,
                           int nlam, double tol, const rls_sweep_opts* opts,
                           const double* x0, double* x, double* resnorm,
                           double* seminorm, rls_solve_info* info,
                           void* stream) {
    g_last_error.clear();
    if (!p) return fail(RLS_E_STATE, "null handle");
    if (!b || !x || !lam || nlam < 1) return fail(RLS_E_ARG, "bad arguments");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(RLS_E_ARG, "tol must be > 0");
    rls_sweep_opts o{100000, RLS_TOL_RELATIVE, 32, 1};
    if (opts) o = *opts;
    if (o.maxit < 1 || o.poll_every < 1 ||
        (o.tol_mode != RLS_TOL_RELATIVE && o.tol_mode != RLS_TOL_ABSOLUTE))
        return fail(RLS_E_ARG, "bad sweep options");
    hipStream_t s = (hipStream_t)stream;
    const int ns = nlam;
    const int64_t n = p->n();
    RLS_TRY(ensure_work(p, ns));
    Work& w = p->w;
    RLS_TRY(upload_lam(p, lam, nlam, s));
    RLS_TRY(prepare_sweep(p, ns, s));
    RLS_TRY(tune_fine(p, ns, s));
    double* part = w.part.as<double>();
    const int vb = vec_blocks(n);
    const LevelGeom g0 = p->lev[0].geom();
    const int tiles0 = apply_tiles(g0);
    SlotState* st = w.st.as<SlotState>();
    int* active = w.active.as<int>();
    double* r = w.r.as<double>();
    double* z = w.z.as<double>();
    double* q = w.q.as<double>();
    double* pb[2] = {w.p0.as<double>(), w.p1.as<double>()};
    double* f = w.f.as<double>();
    double* fpart = w.fpart.as<double>();
    double* rrpart = w.rrpart.as<double>();
    // f = A^T b and partial sums of ||f||^2
    RLS_TRY(apply_blur(p, 1, b, f, 1, s));
    launch_sumsq_slots(f, n, 1, fpart, s);
    // x0 and the initial residual r0 = f - K x0
    ApplyArgs a;
    a.g = g0;
    a.nslot = ns;
    a.lam2 = w.lam2.as<double>();
    if (x0) {
        if (x0 != x)
            RLS_HIP(hipMemcpyAsync(x, x0, sizeof(double) * ns * n,
                                   hipMemcpyDeviceToDevice, s));
        a.in = x;
        a.out = r;
        a.f = f;
        a.f_shared = 1;
        level_apply(PRO_PLAIN, EPI_RESID, a, s);
    } else {
        RLS_HIP(hipMemsetAsync(x, 0, sizeof(double) * ns * n, s));
        launch_broadcast(f, n, ns, r, s);
    }
    launch_sumsq_slots(r, n, ns, rrpart, s);
    // z0 = M r0 with partial sums of r0 . z0 (consumed by the first
    // iteration, where beta = 0 makes p0 = z0)
    const bool mixed = p->prec != RLS_PREC_FP64;
    if (mixed) {
        vcycle_lo(p, ns, nullptr, nullptr, nullptr, nullptr, 0, r, z, nullptr,
                  w.part_rz.as<double>(), nullptr, tiles0, s);
    } else {
        CycleCtl c0;
        c0.dot_part = w.part_rz.as<double>();
        c0.dot_stride = tiles0;
        vcycle(p, 0, ns, nullptr, nullptr, (const double*)r, z, c0, s);
    }
    launch_pcg_init(st, ns, fpart, vb, rrpart, vb, tol,
                    o.tol_mode == RLS_TOL_ABSOLUTE, o.maxit, active, s);
    RLS_HIP(hipMemsetAsync(pb[0], 0, sizeof(double) * ns * n, s));
    RLS_TRY(check_launch("pcg init"));

    // One PCG iteration (parity `cur`) for the `nact` slots in w.slots:
    //   p = z + beta p, q = K p, partials of p . q      (beta folded in)
    //   x += alpha p, r -= alpha q, partials of ||r||^2 (alpha folded in)
    //   z = M r with the convergence test first and partials of r . z last
    auto iteration = [&](int nact, int cur, hipStream_t ss) {
        const int* sl = w.slots.as<int>();
        ApplyArgs ak;
        ak.g = g0;
        ak.nslot = nact;
        ak.slots = sl;
        inline_slots(p, ak);
        ak.lam2 = w.lam2.as<double>();
        ak.active = active;
        ak.in = z;
        ak.pold = pb[cur];
        ak.pnew = pb[1 - cur];
        ak.out = q;
        ak.part = w.part_pq.as<double>();
        ak.part_stride = tiles0;
        ak.st = st;
        ak.active_w = active;
        ak.part_rz = w.part_rz.as<double>();
        ak.nrz = tiles0;
        ak.parity = cur;
        if (mixed) {
            ak.flex = 1;
            ak.part_zq = w.part_zq.as<double>();
        }
        level_apply(PRO_PUPDATE, EPI_DOT, ak, ss);
        launch_update_xr(st, active, sl, n, nact, x, r, pb[1 - cur], q,
                         w.part_pq.as<double>(), tiles0, cur,
                         w.part_rr.as<double>(), ss);
        if (mixed) {
            // reduced-precision V-cycle: gate and narrowing, V-cycle,
            // widening with the partials of r . z and z . q for the
            // flexible beta
            vcycle_lo(p, nact, sl, active, st, w.part_rr.as<double>(), vb, r, z,
                      q, w.part_rz.as<double>(), w.part_zq.as<double>(), tiles0,
                      ss);
            return;
        }
        CycleCtl c;
        c.gate = 1;
        c.st = st;
        c.active_w = active;
        c.part_rr = w.part_rr.as<double>();
        c.nrr = vb;
        c.dot_part = w.part_rz.as<double>();
        c.dot_stride = tiles0;
        vcycle(p, 0, nact, sl, active, (const double*)r, z, c, ss);
    };

    // Iterate in chunks of `chunk` iterations (even, so that the p buffers
    // return to the same roles), polling the active flags between chunks.
    // With graphs, a chunk is captured once per active-slot count and
    // replayed.
    const int chunk = o.poll_every + (o.poll_every & 1);
    int* hact = w.h_active;
    int* hsl = w.h_slots;
    hipGraphExec_t exec = nullptr;
    int exec_nact = -1;
    rls_status status = RLS_OK;
    for (;;) {
        RLS_HIP(hipMemcpyAsync(hact, active, sizeof(int) * ns,
                               hipMemcpyDeviceToHost, s));
        RLS_HIP(hipStreamSynchronize(s));
        if (p->timer_on) drain_timer(p);
        int nact = 0;
        for (int i = 0; i < ns; ++i)
            if (hact[i]) hsl[nact++] = i;
        if (nact == 0) break;
        RLS_HIP(hipMemcpyAsync(w.slots.p, hsl, sizeof(int) * nact,
                               hipMemcpyHostToDevice, s));
        p->hslots = hsl;        // slots only ever leave the active set, so a
        p->hslots_n = nact;     // captured chunk's list is fixed by nact
        if (!o.graph || p->timer_on) {
            for (int k = 0; k < chunk; ++k) iteration(nact, k & 1, s);
            status = check_launch("pcg iteration");
            if (status != RLS_OK) break;
            continue;
        }
        if (nact != exec_nact) {
            if (exec) hipGraphExecDestroy(exec);
            exec = nullptr;
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(p->cstream,
                                                 hipStreamCaptureModeRelaxed);
            if (e == hipSuccess) {
                for (int k = 0; k < chunk; ++k) iteration(nact, k & 1, p->cstream);
                e = hipStreamEndCapture(p->cstream, &graph);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) hipGraphDestroy(graph);
            if (e != hipSuccess) {
                status = fail(RLS_E_HIP, std::string("graph capture: ") +
                                             hipGetErrorString(e));
                break;
            }
            exec_nact = nact;
        }
        hipError_t e = hipGraphLaunch(exec, s);
        if (e != hipSuccess) {
            status = fail(RLS_E_HIP, std::string("hipGraphLaunch: ") +
                                         hipGetErrorString(e));
            break;
        }
    }
    if (exec) hipGraphExecDestroy(exec);
    p->hslots = nullptr;
    p->hslots_n = 0;
    if (status != RLS_OK) return status;

    // true residual ||f - K x||, L-curve pair (||A x - b||, ||D L x||)
    a = ApplyArgs();
    a.g = g0;
    a.nslot = ns;
    a.lam2 = w.lam2.as<double>();
    a.in = x;
    a.out = q;
    a.f = f;
    a.f_shared = 1;
    level_apply(PRO_PLAIN, EPI_RESID, a, s);
    double* o_true = w.outv.as<double>();
    double* o_res = o_true + ns;
    double* o_sem = o_true + 2 * ns;
    launch_sumsq_slots(q, n, ns, part, s);
    launch_reduce_slots(part, vb, ns, o_true, s);
    {
        // ||A x - b|| over the data space (m values for a sparse operator)
        const int64_t md = p->is_ct ? p->ct_m : n;
        double* ax = p->is_ct ? w.cty.as<double>() : w.y.as<double>();
        RLS_TRY(apply_blur(p, 0, x, ax, ns, s));
        launch_sub_sumsq(ax, b, md, ns, part, s);
        launch_reduce_slots(part, vec_blocks(md), ns, o_res, s);
    }
    launch_weighted_grad_sq(x, p->unit_weights ? nullptr : p->weights.as<double>(),
                            p->nv, p->nh, p->periodic, ns, part, s);
    launch_reduce_slots(part, vb, ns, o_sem, s);
    RLS_TRY(check_launch("sweep outputs"));
    std::vector<double> h3(3 * ns);
    std::vector<SlotState> hst(ns);
    RLS_HIP(hipMemcpyAsync(h3.data(), o_true, sizeof(double) * 3 * ns,
                           hipMemcpyDeviceToHost, s));
    RLS_HIP(hipMemcpyAsync(hst.data(), st, sizeof(SlotState) * ns,
                           hipMemcpyDeviceToHost, s));
    RLS_HIP(hipStreamSynchronize(s));
    if (p->timer_on) {
        drain_timer(p);
        // Every V-cycle of a slot takes part in 2 nu - 3 finest-level
        // Chebyshev-step launches (32 bytes per pixel per slot in the
        // tiled kernel's three-term form: read x_k, x_{k-1} or d, f, write
        // x_{k+1}; 40 in the general kernel, which also writes d); a launch
        // with at least one active slot also reads the two shared stencil
        // coupling planes (16 bytes per pixel; the centre coefficient is
        // minus their sum on the finest level).
        const int nu0 = p->nu[0];
        const int per_cycle =
            (p->kt > 0 && nu0 >= 2 && p->prec == RLS_PREC_FP64) ? 2 * nu0 - 3 : 0;
        double slot_launches = 0.0;
        int max_cycles = 0;
        for (int i = 0; i < ns; ++i) {
            slot_launches += (double)hst[i].ncycle * per_cycle;
            max_cycles = std::max(max_cycles, hst[i].ncycle);
        }
        const double slot_bytes = p->fine_tiled ? 32.0 : 40.0;
        p->timer_bytes += (double)n * slot_bytes * slot_launches +
                          (double)n * 16.0 * (double)max_cycles * per_cycle;
    }
    for (int i = 0; i < ns; ++i) {
        if (resnorm) resnorm[i] = std::sqrt(h3[ns + i]);
        if (seminorm) seminorm[i] = std::sqrt(h3[2 * ns + i]);
        if (info) {
            const double fn = hst[i].fnorm > 0 ? hst[i].fnorm : 1.0;
            info[i].iters = hst[i].it;
            info[i].flags = hst[i].flags;
            info[i].relres = std::sqrt(hst[i].rr) / fn;
            info[i].relres_true = std::sqrt(h3[i]) / fn;
        }
    }
    return RLS_OK;
}

}  // extern "C"
