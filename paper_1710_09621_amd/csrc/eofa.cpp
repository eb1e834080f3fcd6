// Host runtime and C ABI of the gfx950 EOFA / optimal-DWF solver (see include/eofa.h).
//
// Solve path for H_T(m+, m-) x = b (the 5D systems inside Eq.(Hij) and Eqs.(m1m2_m1m4),
// (m1m2_m3m2)):  H_T = gamma_5 R5 D_T, so x = D_T^{-1} c with c = R5 gamma_5 b.  D_T is split
// into 4D parities,
//     D_T = [[A_T, -H_eo/2], [-H_oe/2, A_T]],   A_T = 4 - m0 + P_+ M_+ + P_- M_-  (site-local),
// and CG runs on the normal equations of the site-normalised Schur complement
//     Dhat = 1 - (1/4) A_T^{-1} H_oe A_T^{-1} H_eo          (odd sites).
// Every hop kernel carries its site-local operator as an epilogue, so one CG iteration is four
// fused hop launches and one BLAS launch, with alpha/beta/|r|^2 kept on the device.  The true
// residual ||c - D_T x|| is recomputed in FP64 at the end and the solve restarts on the defect
// if it is above tolerance.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/eofa.h"
#include "cnn.h"
#include "force.h"
#include "hmc.h"
#include "eofa_int.h"

using namespace eofa;

// ------------------------------------------------------------------ allocation-free scratch
// Device memory of eofa_apply_static, for callers that cannot allocate: the intermediate half fields, the
// site-operator tables and the reduction buffers of one operator application.  Every GPU the library runs on
// holds its own copy until the process ends; host code reaches it only through the per-device address that
// hipGetSymbolAddress returns (scratch_addr), never through the array's name.
constexpr size_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on device dev (which must be current); resolved once per device.
hipError_t scratch_addr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return hipSuccess;
}
}  // namespace

struct eofa_ctx {
    int L[4] = {0, 0, 0, 0};
    int dev = 0;
    void* scratch = nullptr;  // this device's address of the static scratch array
    std::string scratch_err;
    int Ns = 0;
    double m0 = 0;
    int tbc = -1;
    std::vector<double> omega;
    hipStream_t st = nullptr;
    Geom g{};
    size_t nh = 0;  // complex elements of one half field (Vh * 12 * Ns)
    cd* U[2] = {nullptr, nullptr};
    cpx<float>* Uf[2] = {nullptr, nullptr};
    bool gauge = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    double* partials = nullptr;
    double* scal = nullptr;   // [0, SC_N): single-system scalars; [SC_N, SC_N+128): coefficient vectors;
                              // [BATCH_OFF, BATCH_OFF + NRMAX*SC_N): multi-RHS scalars
    double* hscal = nullptr;  // pinned mirror of scal
    double* partials_mr = nullptr;
    int pstride = 0;
    std::map<std::tuple<int, double, double>, SiteOp*> tabs;
    double* md_F = nullptr;  // molecular dynamics: one force field, 4 V 8 doubles
    cd* md_U0 = nullptr;     // the links at the start of a trajectory (restored on rejection)
    std::vector<cd*> md_guess;  // chronological start vectors, two halves per action
    double* md_fn = nullptr;    // link-summed |F| of every fermion force evaluation of a trajectory
    size_t md_fn_len = 0;
    void* hb = nullptr;  // heat-bath: the 4D outputs of the shifted chiral actions
    size_t hb_bytes = 0;
    std::string err;
    // device time of the FP64 CG iteration's kernels (eofa_kernel_timing): HIP events around each launch
    bool timing = false;
    struct Ev {
        hipEvent_t a, b;
        int k;
    };
    std::vector<Ev> ev_pool;
    size_t ev_used = 0;
    double k_ms[EOFA_NKERN] = {};
    long k_n[EOFA_NKERN] = {};
    double k_bytes[EOFA_NKERN] = {};
    // learned preconditioner (see cnn.hip)
    struct Cnn {
        bool ready = false;
        int relu = 0;
        float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;  // CNN_NPARAM each
        unsigned short *Wb = nullptr, *Wt = nullptr;                    // bf16 forward / backward-data weights
        int rows = 0;
        unsigned short *X0 = nullptr, *A[3] = {nullptr, nullptr, nullptr}, *dYb = nullptr, *XT = nullptr, *dYT = nullptr;
        float *Y = nullptr, *T = nullptr, *dY = nullptr, *dA = nullptr, *part = nullptr;
        long step = 0;
    } cnn;
    double* dots = nullptr;  // FGCR dot products (device)
    // captured CG-iteration blocks (use_graph): key = every launch argument that can vary
    hipStream_t cap_st = nullptr;
    std::map<std::vector<uintptr_t>, hipGraphExec_t> graphs;
    long graph_replays = 0;
    // workgroup schedules of the hop kernels per storage (0: FP64, 1: FP32, 2: FP16 columns), set by the autotuner
    Sched sched[3] = {{0, 0, 1, 1, 1, 1, 0}, {0, 0, 1, 1, 1, 1, 0}, {0, 0, 1, 1, 1, 1, 0}};
    double tuned_ms[3] = {0, 0, 0};
};

namespace {

constexpr int BATCH_OFF = 256;
constexpr int SCAL_TOTAL = BATCH_OFF + NRMAX * SC_N;

struct Fail {
    eofa_status st;
};

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);                     \
            throw Fail{EOFA_EHIP};                                                            \
        }                                                                                     \
    } while (0)

#define REQUIRE(cond, code, msg)                                                              \
    do {                                                                                      \
        if (!(cond)) {                                                                        \
            ctx->err = (msg);                                                                 \
            throw Fail{code};                                                                 \
        }                                                                                     \
    } while (0)

template <typename F> eofa_status guarded(eofa_ctx* ctx, F&& f) {
    if (!ctx) return EOFA_EINVAL;
    try {
        ctx->err.clear();
        return f();
    } catch (const Fail& e) {
        return e.st;
    } catch (const std::exception& e) {
        ctx->err = e.what();
        return EOFA_EHIP;
    } catch (...) {
        ctx->err = "unknown error";
        return EOFA_EHIP;
    }
}

const SiteOp* site_tab(eofa_ctx* ctx, SiteKind kind, double mp, double mm) {
    auto key = std::make_tuple((int)kind, mp, mm);
    auto it = ctx->tabs.find(key);
    if (it != ctx->tabs.end()) return it->second;
    SiteOp h;
    build_site_op(h, kind, ctx->Ns, ctx->m0, ctx->omega.data(), mp, mm);
    SiteOp* d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(SiteOp)));
    HIPCHK(hipMemcpy(d, &h, sizeof(SiteOp), hipMemcpyHostToDevice));
    ctx->tabs[key] = d;
    return d;
}

Red red_of(eofa_ctx* ctx, int slot, int epi) { return Red{ctx->partials, ctx->scal, slot, epi}; }

void sync_scal(eofa_ctx* ctx) {
    HIPCHK(hipMemcpyAsync(ctx->hscal, ctx->scal, sizeof(double) * SC_N, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
}

// ------------------------------------------------------------------ workspace
struct Vec2 {
    cd* h[2];  // even, odd halves
};

struct Work64 {
    Vec2 c, x, res;
    cd *bh, *r, *p, *u, *w, *wt, *at, *xcg;
};

constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

size_t work64_bytes(const eofa_ctx* ctx) { return 14 * align_up(ctx->nh * sizeof(cd)); }
size_t work32_bytes(const eofa_ctx* ctx) { return 9 * align_up(ctx->nh * sizeof(cpx<float>)); }

// per system of a multi-RHS batch: FP64 solution accumulator and Schur source, then the Krylov
// vectors x, r (batch precision: FP64 or FP32) and p, u, w, wt, at (FP64, FP32 or FP16 columns)
size_t batch_vec_bytes(const eofa_ctx* ctx, const eofa_solve_params* p, bool xr) {
    const int prec = p ? p->prec : EOFA_FP64;
    if (prec == EOFA_FP64) return align_up(ctx->nh * sizeof(cd));
    if (prec == EOFA_MIXED_FP16 && !xr) return align_up(half_field_bytes_h(ctx->g, ctx->Ns));
    return align_up(ctx->nh * sizeof(cpx<float>));
}
size_t batch_sys_bytes(const eofa_ctx* ctx, const eofa_solve_params* p) {
    return 2 * align_up(ctx->nh * sizeof(cd)) + 2 * batch_vec_bytes(ctx, p, true) + 5 * batch_vec_bytes(ctx, p, false);
}

constexpr int FGCR_M = 8;  // directions kept by the truncated flexible GCR (a ring)

size_t fgcr_bytes(const eofa_ctx* ctx) { return (2 * FGCR_M + 1) * align_up(ctx->nh * sizeof(cd)); }

// workspace: FP64 set | FP32 set (mixed) | then either the FGCR directions or the batched systems
size_t base_bytes(const eofa_ctx* ctx, const eofa_solve_params* p) {
    return work64_bytes(ctx) + ((p && p->prec == EOFA_MIXED_FP32) ? work32_bytes(ctx) : 0);
}

// FP16 storage runs through the batch kernels, also for a single system
size_t needed_bytes(const eofa_ctx* ctx, const eofa_solve_params* p, int nrhs = 1) {
    size_t extra = 0;
    if (p && p->pc == EOFA_PC_LEARNED) extra = fgcr_bytes(ctx);
    const bool fp16 = p && p->prec == EOFA_MIXED_FP16;
    if ((nrhs > 1 || fp16) && ctx->Ns >= 8)
        extra = std::max(extra, (size_t)std::min(nrhs, NRMAX) * batch_sys_bytes(ctx, p));
    return base_bytes(ctx, p) + extra;
}

void ensure_ws(eofa_ctx* ctx, size_t need) {
    if (ctx->ws_bytes >= need) return;
    REQUIRE(ctx->ws == nullptr || ctx->ws_owned, EOFA_ENOMEM,
            "workspace too small: need " + std::to_string(need) + " bytes, have " + std::to_string(ctx->ws_bytes));
    if (ctx->ws) HIPCHK(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    hipError_t e = hipMalloc(&ctx->ws, need);
    REQUIRE(e == hipSuccess, EOFA_ENOMEM, "hipMalloc of " + std::to_string(need) + " workspace bytes failed");
    ctx->ws_bytes = need;
    ctx->ws_owned = true;
}

Work64 carve64(eofa_ctx* ctx) {
    char* p = ctx->ws;
    const size_t hb = align_up(ctx->nh * sizeof(cd));
    auto take = [&]() { cd* r = (cd*)p; p += hb; return r; };
    Work64 w;
    w.c.h[0] = take(); w.c.h[1] = take();
    w.x.h[0] = take(); w.x.h[1] = take();
    w.res.h[0] = take(); w.res.h[1] = take();
    w.bh = take(); w.r = take(); w.p = take(); w.u = take(); w.w = take(); w.wt = take(); w.at = take(); w.xcg = take();
    return w;
}

struct Work32 {
    cpx<float> *x, *r, *p, *u, *w, *wt, *at, *e0, *e1;
};

Work32 carve32(eofa_ctx* ctx) {
    char* p = ctx->ws + work64_bytes(ctx);
    const size_t hb = align_up(ctx->nh * sizeof(cpx<float>));
    auto take = [&]() { cpx<float>* r = (cpx<float>*)p; p += hb; return r; };
    Work32 w;
    w.x = take(); w.r = take(); w.p = take(); w.u = take(); w.w = take(); w.wt = take(); w.at = take();
    w.e0 = take(); w.e1 = take();
    return w;
}

// ------------------------------------------------------------------ hop launch helpers
template <typename R> HopArgs<R> hop_args(eofa_ctx* ctx, int par);
template <> HopArgs<double> hop_args<double>(eofa_ctx* ctx, int par) {
    HopArgs<double> a{};
    a.g = ctx->g;
    a.par = par;
    a.Uown = ctx->U[par];
    a.Uoth = ctx->U[1 - par];
    a.sc = ctx->sched[0];
    a.diag = 4.0 - ctx->m0;
    a.scal = ctx->scal;
    return a;
}
template <> HopArgs<float> hop_args<float>(eofa_ctx* ctx, int par) {
    HopArgs<float> a{};
    a.g = ctx->g;
    a.par = par;
    a.Uown = ctx->Uf[par];
    a.Uoth = ctx->Uf[1 - par];
    a.sc = ctx->sched[1];
    a.diag = (float)(4.0 - ctx->m0);
    a.scal = ctx->scal;
    return a;
}

// Algorithmic HBM bytes of one launch of CG-iteration kernel k in FP64: every spinor field the kernel reads or
// writes counted once (12 Ns complex per 4D site), the 8 links of each output site once.
double kernel_bytes(const eofa_ctx* ctx, int k) {
    const double col = 12.0 * ctx->Ns * sizeof(cd), links = 8.0 * 9 * sizeof(cd);
    const int fields[EOFA_NKERN] = {2, 4, 2, 4, 5};  // K1 in+out; K2 in, p, w, wt; K3; K4 in, w, r in/out; K5 x, p, r, x, p
    return (double)ctx->g.Vh * (fields[k] * col + (k < 4 ? links : 0.0));
}

// Runs launch() (kernel launches on ctx->st) and, while timing is on and k >= 0, records events around it
// for kernel class k.
template <typename F> void timed(eofa_ctx* ctx, int k, F&& launch) {
    if (k < 0 || !ctx->timing) { launch(); return; }
    if (ctx->ev_used == ctx->ev_pool.size()) {
        eofa_ctx::Ev e{nullptr, nullptr, 0};
        HIPCHK(hipEventCreate(&e.a));
        HIPCHK(hipEventCreate(&e.b));
        ctx->ev_pool.push_back(e);
    }
    eofa_ctx::Ev& e = ctx->ev_pool[ctx->ev_used++];
    e.k = k;
    HIPCHK(hipEventRecord(e.a, ctx->st));
    launch();
    HIPCHK(hipEventRecord(e.b, ctx->st));
    ctx->k_n[k]++;
    ctx->k_bytes[k] += kernel_bytes(ctx, k);
}

template <typename R> void hop(eofa_ctx* ctx, bool dag, int mode, bool red, const HopArgs<R>& a, int k = -1) {
    timed(ctx, k, [&] { HIPCHK(launch_hop<R>(ctx->Ns, dag, mode, red, a, ctx->st)); });
}

void collect_timing(eofa_ctx* ctx) {
    if (ctx->ev_used == 0) return;
    HIPCHK(hipStreamSynchronize(ctx->st));
    for (size_t i = 0; i < ctx->ev_used; i++) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev_pool[i].a, ctx->ev_pool[i].b));
        ctx->k_ms[ctx->ev_pool[i].k] += ms;
    }
    ctx->ev_used = 0;
}

// Launch the work of body() (kernel launches on ctx->st only: no host synchronisation, copies or
// memsets) as one replay of a captured graph.  The capture runs once per key on a private stream
// (the caller's stream may be the legacy default stream, which cannot be captured) and the
// instantiated graph is replayed on ctx->st.  Kernel arguments are captured by value, so the key
// holds every pointer and parameter the launches take.
template <typename F> void graph_run(eofa_ctx* ctx, std::vector<uintptr_t> key, F&& body) {
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if (ctx->graphs.size() >= 64) {
            for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
            ctx->graphs.clear();
        }
        if (!ctx->cap_st) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_st, hipStreamNonBlocking));
        hipStream_t user = ctx->st;
        const bool timing = ctx->timing;
        ctx->st = ctx->cap_st;
        ctx->timing = false;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(ctx->cap_st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            try {
                body();
            } catch (...) {
                (void)hipStreamEndCapture(ctx->cap_st, &g);
                if (g) (void)hipGraphDestroy(g);
                ctx->st = user;
                ctx->timing = timing;
                throw;
            }
            e = hipStreamEndCapture(ctx->cap_st, &g);
        }
        ctx->st = user;
        ctx->timing = timing;
        HIPCHK(e);
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
        it = ctx->graphs.emplace(std::move(key), ex).first;
    }
    HIPCHK(hipGraphLaunch(it->second, ctx->st));
    ctx->graph_replays++;
}

template <typename R> std::vector<uintptr_t> graph_key(const eofa_ctx* ctx, int kind, int n,
                                                       std::initializer_list<const void*> ptrs, bool half = false) {
    std::vector<uintptr_t> k{(uintptr_t)kind, (uintptr_t)n, sizeof(R), (uintptr_t)ctx->scal,
                             (uintptr_t)ctx->partials, (uintptr_t)ctx->partials_mr, (uintptr_t)ctx->pstride};
    const Sched& sc = ctx->sched[half ? 2 : (sizeof(R) == 8 ? 0 : 1)];
    for (int v : {sc.mode, sc.xcd, sc.ty, sc.tz, sc.tt, sc.nyb, sc.ord}) k.push_back((uintptr_t)v);
    for (const void* p : ptrs) k.push_back((uintptr_t)p);
    return k;
}

// One CG iteration on Dhat^dag Dhat in storage/arithmetic type R (the four fused hops + BLAS).  Once the
// device has flagged convergence (SC_DONE) every kernel of later iterations exits at once, and SC_ITERS
// counts the iterations that were applied, so blocks of iterations can run without host checks.  FP64
// iterations are timed per kernel (K1..K5) while kernel timing is on.
template <typename R>
void cg_iteration(eofa_ctx* ctx, cpx<R>* x, cpx<R>* r, cpx<R>* p, cpx<R>* u, cpx<R>* w, cpx<R>* wt, cpx<R>* at,
                  const SiteOp* Ai, const SiteOp* Ad) {
    const int k0 = sizeof(R) == 8 ? 0 : -EOFA_NKERN;  // kernel classes are timed in FP64 only
    const double* done = ctx->scal + SC_DONE;
    {
        auto a = hop_args<R>(ctx, 0);
        a.in = p; a.out = u; a.opA = Ai; a.cz = 1; a.caux = 0; a.done = done;
        hop<R>(ctx, false, HM_SITE, false, a, k0 + EOFA_K_HOP);
    }
    {
        auto a = hop_args<R>(ctx, 1);
        a.in = u; a.out = w; a.out2 = wt; a.aux = p; a.opA = Ai; a.opB = Ad; a.cz = (R)-0.25; a.caux = 1;
        a.red = red_of(ctx, 0, EPI_CG_W); a.done = done;
        hop<R>(ctx, false, HM_SCHUR_W, true, a, k0 + EOFA_K_SCHUR_W);
    }
    {
        auto a = hop_args<R>(ctx, 0);
        a.in = wt; a.out = at; a.opA = Ad; a.cz = 1; a.caux = 0; a.done = done;
        hop<R>(ctx, true, HM_SITE, false, a, k0 + EOFA_K_HOP_DAG);
    }
    {
        auto a = hop_args<R>(ctx, 1);
        a.in = at; a.out = r; a.aux = w; a.aux2 = r; a.cz = (R)-0.25; a.caux = 1;
        a.red = red_of(ctx, 0, EPI_CG_R); a.done = done;
        hop<R>(ctx, true, HM_SCHUR_Q, true, a, k0 + EOFA_K_SCHUR_Q);
    }
    timed(ctx, k0 + EOFA_K_XP, [&] { HIPCHK(launch_cg_xp<R>(x, p, r, ctx->scal, ctx->nh, ctx->st)); });
    HIPCHK(launch_sync_done(ctx->scal, 1, ctx->st));
}

// ------------------------------------------------------------------ FP64 CG on Dhat^dag Dhat
struct CgOut {
    int iters = 0;
    int applies = 0;
    bool converged = false;
};

// r = Dhat^dag bh, p = r, |r|^2 -> SC_RR, SC_RR0 (EPI_CG_INIT also clears SC_DONE unless r = 0, SC_DONEX and
// SC_ITERS); x = 0.  The stop threshold SC_TOL2 = tol2.
void cg64_init(eofa_ctx* ctx, const Work64& W, const SiteOp* Ad, double tol2) {
    const size_t nh = ctx->nh;
    HIPCHK(hipMemsetAsync(W.xcg, 0, nh * sizeof(cd), ctx->st));
    HIPCHK(launch_scal_set(ctx->scal, SC_TOL2, tol2, -1, 0, -1, 0, ctx->st));
    // r = Dhat^dag bh = bh - 1/4 g5 H_oe g5 A^{-dag} g5 H_eo g5 A^{-dag} bh ; p = r
    HIPCHK(launch_site<double>(ctx->Ns, true, W.bh, W.wt, Ad, ctx->g.Vh, ctx->st));
    {
        auto a = hop_args<double>(ctx, 0);
        a.in = W.wt; a.out = W.at; a.opA = Ad; a.cz = 1.0; a.caux = 0.0;
        hop<double>(ctx, true, HM_SITE, false, a);
    }
    {
        auto a = hop_args<double>(ctx, 1);
        a.in = W.at; a.out = W.r; a.aux = W.bh; a.caux = 1.0; a.cz = -0.25;
        a.red = red_of(ctx, 0, EPI_CG_INIT);
        hop<double>(ctx, true, HM_LIN, true, a);
    }
    HIPCHK(hipMemcpyAsync(W.p, W.r, nh * sizeof(cd), hipMemcpyDeviceToDevice, ctx->st));
}

// Solve Dhat x = bh (odd sites) to |r_normal| <= tol_n |r_normal,0|; x starts at zero.  The host looks at the
// device scalars every check_every iterations; iterations past convergence inside a block are skipped on the
// device, and the iteration count is the device's.  With graph, every full block is one graph replay.
CgOut cg64(eofa_ctx* ctx, const Work64& W, double mp, double mm, double tol_n, int maxit, int check_every,
           bool graph = false) {
    const SiteOp* Ai = site_tab(ctx, SK_AINV, mp, mm);
    const SiteOp* Ad = site_tab(ctx, SK_AINV_DAG, mp, mm);
    CgOut o;
    cg64_init(ctx, W, Ad, tol_n * tol_n);
    o.applies = 1;
    sync_scal(ctx);
    if (ctx->hscal[SC_DONE] != 0.0) { o.converged = true; return o; }
    if (check_every <= 0) check_every = 1;
    int launched = 0;
    while (launched < maxit) {
        // u = A^{-1} H_eo p ; w = Dhat p, wt = A^{-dag} w, |w|^2 -> alpha ; at = A^{-dag} g5 H_eo g5 wt ;
        // r -= alpha (w - g5 H_oe g5 at / 4), |r|^2 -> beta ; x += alpha p, p = r + beta p
        const int blk = std::min(check_every, maxit - launched);
        if (graph && blk == check_every) {
            graph_run(ctx, graph_key<double>(ctx, 1, blk, {W.xcg, W.r, W.p, W.u, W.w, W.wt, W.at, Ai, Ad}), [&] {
                for (int k = 0; k < blk; k++) cg_iteration<double>(ctx, W.xcg, W.r, W.p, W.u, W.w, W.wt, W.at, Ai, Ad);
            });
        } else {
            for (int k = 0; k < blk; k++) cg_iteration<double>(ctx, W.xcg, W.r, W.p, W.u, W.w, W.wt, W.at, Ai, Ad);
        }
        launched += blk;
        sync_scal(ctx);
        o.iters = (int)ctx->hscal[SC_ITERS];
        o.applies = 1 + 2 * o.iters;
        if (!std::isfinite(ctx->hscal[SC_RR]) || !std::isfinite(ctx->hscal[SC_ALPHA])) {
            ctx->err = "CG breakdown (non-finite scalar)";
            return o;
        }
        if (ctx->hscal[SC_DONE] != 0.0) { o.converged = true; break; }
    }
    return o;
}

void ensure_partials_mr(eofa_ctx* ctx) {
    // batch kernels: one partial per 256 sites x s; launch_mdot: up to 1024 blocks
    const int need = std::max((int)(((size_t)ctx->g.Vh * ctx->Ns + 255) / 256) + 1, 1024);
    if (ctx->partials_mr && ctx->pstride >= need) return;
    if (ctx->partials_mr) HIPCHK(hipFree(ctx->partials_mr));
    // rows: NRMAX systems of the batch kernels, or 2 x 9 (re, im) dot products of launch_mdot
    HIPCHK(hipMalloc(&ctx->partials_mr, sizeof(double) * (size_t)need * (NRMAX > 18 ? NRMAX : 18)));
    ctx->pstride = need;
}

double norm2_half(eofa_ctx* ctx, const cd* v) {
    HIPCHK(launch_norm2<double>(v, ctx->nh, red_of(ctx, SC_TMP + 9, EPI_STORE), ctx->st));
    sync_scal(ctx);
    return ctx->hscal[SC_TMP + 9];
}

// Iterations between host checks when the caller leaves it to the library.  Iterations past convergence
// inside a block exit at once on the device, so a block costs at most a few launches of waste; 16 keeps the
// host out of the loop and gives a captured graph 16 iterations at every volume.
constexpr int kAutoCheckEvery = 16;

// ------------------------------------------------------------------ mixed precision CG
// FP64 normal residual r = Dhat^dag (bh - Dhat x) into W.r; returns |r|^2 (host sync).
double normal_residual64(eofa_ctx* ctx, const Work64& W, const cd* x, const cd* bh, const SiteOp* Ai,
                         const SiteOp* Ad) {
    {
        auto a = hop_args<double>(ctx, 0);
        a.in = x; a.out = W.u; a.opA = Ai; a.cz = 1.0; a.caux = 0.0;
        hop<double>(ctx, false, HM_SITE, false, a);
    }
    {
        auto a = hop_args<double>(ctx, 1);
        a.in = W.u; a.out = W.w; a.out2 = W.wt; a.aux = x; a.opA = Ai; a.opB = Ad; a.cz = -0.25; a.caux = 1.0;
        a.red = red_of(ctx, SC_TMP + 10, EPI_STORE);
        hop<double>(ctx, false, HM_SCHUR_W, true, a);
    }
    // rho = bh - Dhat x ; r = Dhat^dag rho
    HIPCHK(launch_axpby<double>(1.0, bh, -1.0, W.w, ctx->nh, nullptr, ctx->st));
    HIPCHK(launch_site<double>(ctx->Ns, true, W.w, W.wt, Ad, ctx->g.Vh, ctx->st));
    {
        auto a = hop_args<double>(ctx, 0);
        a.in = W.wt; a.out = W.at; a.opA = Ad; a.cz = 1.0; a.caux = 0.0;
        hop<double>(ctx, true, HM_SITE, false, a);
    }
    {
        auto a = hop_args<double>(ctx, 1);
        a.in = W.at; a.out = W.r; a.aux = W.w; a.caux = 1.0; a.cz = -0.25;
        a.red = red_of(ctx, SC_TMP + 11, EPI_STORE);
        hop<double>(ctx, true, HM_LIN, true, a);
    }
    sync_scal(ctx);
    return ctx->hscal[SC_TMP + 11];
}

// A replacement cycle that runs this long without reaching its delta target is cut short: the FP64
// residual is recomputed anyway, so a reduced-precision recurrence that has stopped tracking the true
// residual is caught by the stagnation test instead of iterating to max_iter.
constexpr int kMaxCycle = 500;

// Reliable-update CG: FP32 storage and arithmetic for the Krylov iteration, FP64 solution
// accumulation and FP64 residual replacement whenever |r| has dropped by delta since the
// last replacement.  Solves Dhat W.xcg = W.bh to |r_normal| <= tol_n |r_normal,0|.
CgOut cg_mixed(eofa_ctx* ctx, const Work64& W, double mp, double mm, double tol_n, int maxit, int check_every,
               double delta, int* updates, bool graph = false) {
    const SiteOp* Ai = site_tab(ctx, SK_AINV, mp, mm);
    const SiteOp* Ad = site_tab(ctx, SK_AINV_DAG, mp, mm);
    const Work32 F = carve32(ctx);
    const size_t nh = ctx->nh;
    CgOut o;
    if (delta <= 0 || delta >= 1) delta = 0.1;
    if (check_every <= 0) check_every = 1;
    HIPCHK(hipMemsetAsync(W.xcg, 0, nh * sizeof(cd), ctx->st));
    double rr = normal_residual64(ctx, W, W.xcg, W.bh, Ai, Ad);
    o.applies = 2;
    const double rr0 = rr;
    if (rr0 == 0.0) { o.converged = true; return o; }
    HIPCHK(launch_convert_d2f(W.r, F.r, nh, ctx->st));
    HIPCHK(hipMemcpyAsync(F.p, F.r, nh * sizeof(cpx<float>), hipMemcpyDeviceToDevice, ctx->st));
    HIPCHK(hipMemsetAsync(F.x, 0, nh * sizeof(cpx<float>), ctx->st));
    int stall = 0;
    while (o.iters < maxit) {
        // inner FP32 iterations until |r|^2 <= max(delta^2, target) * rr (the last replaced residual)
        const double tol2 = std::max(delta * delta, tol_n * tol_n * rr0 / rr);
        HIPCHK(launch_scal_set(ctx->scal, SC_RR, rr, SC_RR0, rr, SC_TOL2, tol2, ctx->st));
        HIPCHK(launch_scal_set(ctx->scal, SC_DONE, 0.0, SC_DONEX, 0.0, SC_ITERS, 0.0, ctx->st));
        const int base = o.iters;
        int launched = 0;
        while (base + launched < maxit) {
            const int blk = std::min(check_every, maxit - base - launched);
            if (graph && blk == check_every) {
                graph_run(ctx, graph_key<float>(ctx, 2, blk, {F.x, F.r, F.p, F.u, F.w, F.wt, F.at, Ai, Ad}), [&] {
                    for (int k = 0; k < blk; k++) cg_iteration<float>(ctx, F.x, F.r, F.p, F.u, F.w, F.wt, F.at, Ai, Ad);
                });
            } else {
                for (int k = 0; k < blk; k++) cg_iteration<float>(ctx, F.x, F.r, F.p, F.u, F.w, F.wt, F.at, Ai, Ad);
            }
            launched += blk;
            sync_scal(ctx);
            const int inner = (int)ctx->hscal[SC_ITERS];
            o.iters = base + inner;
            if (!std::isfinite(ctx->hscal[SC_RR])) { ctx->err = "mixed CG breakdown"; return o; }
            if (ctx->hscal[SC_DONE] != 0.0 || inner >= kMaxCycle) break;
        }
        o.applies += 2 * (o.iters - base);
        // reliable update: x_hi += x_lo ; r = Dhat^dag (bh - Dhat x_hi) in FP64
        HIPCHK(launch_accum_f(W.xcg, F.x, nh, ctx->st));
        HIPCHK(hipMemsetAsync(F.x, 0, nh * sizeof(cpx<float>), ctx->st));
        const double rr_prev = rr;
        rr = normal_residual64(ctx, W, W.xcg, W.bh, Ai, Ad);
        o.applies += 2;
        if (updates) (*updates)++;
        if (!std::isfinite(rr)) { ctx->err = "mixed CG: non-finite residual"; return o; }
        if (rr <= tol_n * tol_n * rr0) { o.converged = true; return o; }
        // stagnation (less than 2x in norm over 8 replacements): hand back to the FP64 defect correction
        stall = (rr > 0.25 * rr_prev) ? stall + 1 : 0;
        if (stall >= 8) return o;
        HIPCHK(launch_convert_d2f(W.r, F.r, nh, ctx->st));
    }
    return o;
}

// ------------------------------------------------------------------ learned preconditioner (host side)
void cnn_alloc(eofa_ctx* ctx) {
    auto& c = ctx->cnn;
    const int rows = ctx->g.Vh * ctx->Ns;
    if (!c.P) {
        for (float** q : {&c.P, &c.G, &c.M, &c.V}) {
            HIPCHK(hipMalloc(q, sizeof(float) * CNN_NPARAM));
            HIPCHK(hipMemsetAsync(*q, 0, sizeof(float) * CNN_NPARAM, ctx->st));
        }
        HIPCHK(hipMalloc(&c.Wb, sizeof(unsigned short) * CNN_LAYERS * CNN_WSZ));
        HIPCHK(hipMalloc(&c.Wt, sizeof(unsigned short) * CNN_LAYERS * CNN_WSZ));
    }
    if (c.rows != rows) {
        for (void* q : {(void*)c.X0, (void*)c.A[0], (void*)c.A[1], (void*)c.A[2], (void*)c.dYb, (void*)c.XT,
                        (void*)c.dYT, (void*)c.Y, (void*)c.T, (void*)c.dY, (void*)c.dA, (void*)c.part})
            if (q) HIPCHK(hipFree(q));
        const size_t r32 = (size_t)rows * 32;
        for (unsigned short** q : {&c.X0, &c.A[0], &c.A[1], &c.A[2], &c.dYb, &c.XT, &c.dYT})
            HIPCHK(hipMalloc(q, sizeof(unsigned short) * r32));
        for (float** q : {&c.Y, &c.T, &c.dY, &c.dA}) HIPCHK(hipMalloc(q, sizeof(float) * r32));
        HIPCHK(hipMalloc(&c.part, sizeof(float) * (size_t)cnn_wgrad_chunks(rows) * 81 * 1024));
        c.rows = rows;
    }
}

// bf16 copies of the weights for the forward and backward-data convolutions
void cnn_refresh(eofa_ctx* ctx) {
    auto& c = ctx->cnn;
    for (int l = 0; l < CNN_LAYERS; l++) {
        HIPCHK(cnn_f32_to_bf16(c.P + (size_t)l * CNN_LSZ, c.Wb + (size_t)l * CNN_WSZ, CNN_WSZ, ctx->st));
        HIPCHK(cnn_w_transpose(c.P + (size_t)l * CNN_LSZ, c.Wt + (size_t)l * CNN_WSZ, ctx->st));
    }
}

// X0 -> Y through the four layers
void cnn_forward_rows(eofa_ctx* ctx) {
    auto& c = ctx->cnn;
    const unsigned short* in = c.X0;
    for (int l = 0; l < CNN_LAYERS; l++) {
        const bool last = (l == CNN_LAYERS - 1);
        void* out = last ? (void*)c.Y : (void*)c.A[l];
        HIPCHK(cnn_conv_fwd(in, c.Wb + (size_t)l * CNN_WSZ, c.P + (size_t)l * CNN_LSZ + CNN_WSZ, out, last, ctx->g,
                            ctx->Ns, last ? 0 : c.relu, ctx->st));
        if (!last) in = c.A[l];
    }
}

// out = |in| N(in / |in|) on odd half fields (FP64); slot SC_TMP+12 holds |in|^2
void cnn_apply_half(eofa_ctx* ctx, const cd* in, cd* out) {
    auto& c = ctx->cnn;
    double* n2 = ctx->scal + SC_TMP + 12;
    HIPCHK(launch_norm2<double>(in, ctx->nh, red_of(ctx, SC_TMP + 12, EPI_STORE), ctx->st));
    HIPCHK(cnn_half_to_rows(in, c.X0, ctx->g, ctx->Ns, n2, 1, ctx->st));
    cnn_forward_rows(ctx);
    HIPCHK(cnn_rows_to_half(c.Y, out, ctx->g, ctx->Ns, n2, ctx->st));
}

// Loss and gradient for one (rho, e) pair: input rho/|rho|, target e/|rho|, L = |N - T|^2 / |T|^2.
// Gradients go to c.G (dL/dparam scaled by |T|^2 / 2).  Returns L.
double cnn_grad(eofa_ctx* ctx, const cd* rho, const cd* e) {
    auto& c = ctx->cnn;
    const int rows = c.rows;
    const size_t r32 = (size_t)rows * 32;
    double* n2 = ctx->scal + SC_TMP + 12;
    HIPCHK(launch_norm2<double>(rho, ctx->nh, red_of(ctx, SC_TMP + 12, EPI_STORE), ctx->st));
    HIPCHK(cnn_half_to_rows(rho, c.X0, ctx->g, ctx->Ns, n2, 1, ctx->st));
    HIPCHK(cnn_half_to_rows_f32(e, c.T, ctx->g, ctx->Ns, n2, ctx->st));
    cnn_forward_rows(ctx);
    HIPCHK(cnn_mse(c.Y, c.T, c.dY, r32, 1.0f, red_of(ctx, SC_TMP + 13, EPI_STORE), ctx->st));
    HIPCHK(launch_norm2<float>((const cpx<float>*)c.T, r32 / 2, red_of(ctx, SC_TMP + 14, EPI_STORE), ctx->st));
    const float* dcur = c.dY;
    for (int l = CNN_LAYERS - 1; l >= 0; l--) {
        const unsigned short* in = (l == 0) ? c.X0 : c.A[l - 1];
        HIPCHK(cnn_to_chmajor(dcur, true, c.dYT, rows, ctx->st));
        HIPCHK(cnn_to_chmajor(in, false, c.XT, rows, ctx->st));
        HIPCHK(cnn_wgrad(c.dYT, c.XT, c.part, c.G + (size_t)l * CNN_LSZ, ctx->g, ctx->Ns, CNN_CIN[l], CNN_COUT[l], ctx->st));
        HIPCHK(cnn_bgrad(dcur, rows, c.G + (size_t)l * CNN_LSZ + CNN_WSZ, CNN_COUT[l], (double*)c.part, ctx->st));
        if (l > 0) {
            HIPCHK(cnn_f32_to_bf16(dcur, c.dYb, r32, ctx->st));
            HIPCHK(cnn_conv_fwd(c.dYb, c.Wt + (size_t)l * CNN_WSZ, nullptr, c.dA, true, ctx->g, ctx->Ns, 0, ctx->st));
            if (c.relu) HIPCHK(cnn_relu_bwd(c.dA, c.A[l - 1], r32, ctx->st));
            dcur = c.dA;
        }
    }
    sync_scal(ctx);
    const double t2 = ctx->hscal[SC_TMP + 14];
    return t2 > 0 ? ctx->hscal[SC_TMP + 13] / t2 : 0.0;
}

// out = Dhat^dag in (odd half fields); scratch W.wt, W.at
void schur_dag64(eofa_ctx* ctx, const Work64& W, const SiteOp* Ad, const cd* in, cd* out) {
    HIPCHK(launch_site<double>(ctx->Ns, true, in, W.wt, Ad, ctx->g.Vh, ctx->st));
    auto c = hop_args<double>(ctx, 0);
    c.in = W.wt; c.out = W.at; c.opA = Ad; c.cz = 1.0; c.caux = 0.0;
    hop<double>(ctx, true, HM_SITE, false, c);
    auto d = hop_args<double>(ctx, 1);
    d.in = W.at; d.out = out; d.aux = in; d.caux = 1.0; d.cz = -0.25;
    hop<double>(ctx, true, HM_LIN, false, d);
}

// out = Dhat in; also W.wt = A^{-dag} out (for a following Dhat^dag); scratch W.u
void schur64(eofa_ctx* ctx, const Work64& W, const SiteOp* Ai, const SiteOp* Ad, const cd* in, cd* out) {
    auto a = hop_args<double>(ctx, 0);
    a.in = in; a.out = W.u; a.opA = Ai; a.cz = 1.0; a.caux = 0.0;
    hop<double>(ctx, false, HM_SITE, false, a);
    auto b = hop_args<double>(ctx, 1);
    b.in = W.u; b.out = out; b.out2 = W.wt; b.aux = in; b.opA = Ai; b.opB = Ad; b.cz = -0.25; b.caux = 1.0;
    b.red = red_of(ctx, SC_TMP + 15, EPI_STORE);
    hop<double>(ctx, false, HM_SCHUR_W, true, b);
}

// ------------------------------------------------------------------ flexible GCR with the network
// Solves Dhat x = bh (odd sites) with the right preconditioner z = N(Dhat^dag r), the network N standing
// in for (Dhat^dag Dhat)^{-1}: Dhat itself is not positive-real (plain GCR on it stagnates), while
// Dhat N Dhat^dag is Hermitian positive definite for N = 1 and stays positive-real while N is close
// to a positive operator.  Truncated GCR keeps the last FGCR_M directions in a ring (each new
// q = Dhat z made orthogonal to the kept ones by classical Gram-Schmidt, the same combination applied
// to z).  Falls back to FP64 CG (cg64) on the remaining defect when the residual stops falling (less
// than 2x in norm over 20 iterations) or on breakdown.
CgOut fgcr(eofa_ctx* ctx, const Work64& W, double mp, double mm, double tol_n, int maxit, const eofa_solve_params& P,
           bool* fell_back) {
    const SiteOp* Ai = site_tab(ctx, SK_AINV, mp, mm);
    const SiteOp* Ad = site_tab(ctx, SK_AINV_DAG, mp, mm);
    const size_t nh = ctx->nh;
    const size_t hb = align_up(nh * sizeof(cd));
    char* q0 = ctx->ws + base_bytes(ctx, &P);
    cd* Z[FGCR_M];
    cd* Q[FGCR_M];
    for (int i = 0; i < FGCR_M; i++) { Z[i] = (cd*)(q0 + (2 * i) * hb); Q[i] = (cd*)(q0 + (2 * i + 1) * hb); }
    cd* rr = (cd*)(q0 + 2 * FGCR_M * hb);  // residual
    if (!ctx->dots) HIPCHK(hipMalloc(&ctx->dots, sizeof(double) * 32));
    ensure_partials_mr(ctx);
    double* dh = ctx->hscal + BATCH_OFF;  // host copies of the dots (batch area unused here)
    CgOut o;
    *fell_back = false;
    HIPCHK(hipMemsetAsync(W.xcg, 0, nh * sizeof(cd), ctx->st));
    HIPCHK(hipMemcpyAsync(rr, W.bh, nh * sizeof(cd), hipMemcpyDeviceToDevice, ctx->st));
    const double b2 = norm2_half(ctx, W.bh);
    if (b2 == 0.0) { o.converged = true; return o; }
    double r2 = b2, best = b2, mark = b2;
    double qq[FGCR_M];
    int since = 0;
    auto dots = [&](const cd* const* v, int nv, const cd* y) {
        HIPCHK(launch_mdot(v, nv, y, nh, ctx->partials_mr, ctx->pstride, ctx->dots, ctx->st));
        HIPCHK(hipMemcpyAsync(dh, ctx->dots, sizeof(double) * 2 * nv, hipMemcpyDeviceToHost, ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));
    };
    while (o.iters < maxit) {
        const int j = o.iters % FGCR_M;  // slot of the new direction (overwrites the oldest)
        // z = N(Dhat^dag r), q = Dhat z
        schur_dag64(ctx, W, Ad, rr, W.p);
        cnn_apply_half(ctx, W.p, Z[j]);
        schur64(ctx, W, Ai, Ad, Z[j], Q[j]);
        o.applies += 2;
        const cd* ko[FGCR_M];  // kept directions other than slot j
        const cd* kz[FGCR_M];
        int kept[FGCR_M], nk = 0;
        for (int i = 0; i < std::min(o.iters, FGCR_M); i++)
            if (i != j) { kept[nk] = i; ko[nk] = Q[i]; kz[nk] = Z[i]; nk++; }
        if (nk > 0) {  // q -= sum_i <q_i, q>/|q_i|^2 q_i, same combination on z
            dots(ko, nk, Q[j]);
            double cr[FGCR_M], ci[FGCR_M];
            for (int i = 0; i < nk; i++) { cr[i] = -dh[2 * i] / qq[kept[i]]; ci[i] = -dh[2 * i + 1] / qq[kept[i]]; }
            HIPCHK(launch_maxpy(ko, cr, ci, nk, Q[j], nh, ctx->st));
            HIPCHK(launch_maxpy(kz, cr, ci, nk, Z[j], nh, ctx->st));
        }
        const cd* qr[2] = {Q[j], Q[j]};
        const cd* qv[1] = {Q[j]};
        dots(qv, 1, Q[j]);
        qq[j] = dh[0];
        dots(qr, 1, rr);
        const double ar = dh[0] / qq[j], ai = dh[1] / qq[j];
        bool broke = !(qq[j] > 0) || !std::isfinite(ar) || !std::isfinite(ai);
        if (!broke) {
            const cd* zs[1] = {Z[j]};
            const cd* qs[1] = {Q[j]};
            double pr = ar, pi = ai, mr = -ar, mi = -ai;
            HIPCHK(launch_maxpy(zs, &pr, &pi, 1, W.xcg, nh, ctx->st));
            HIPCHK(launch_maxpy(qs, &mr, &mi, 1, rr, nh, ctx->st));
            r2 = norm2_half(ctx, rr);
            broke = !std::isfinite(r2);
        }
        o.iters++;
        since++;
        if (!broke && r2 <= tol_n * tol_n * b2) { o.converged = true; return o; }
        if (r2 < best) best = r2;
        if (since >= 20) {
            if (best > 0.25 * mark) broke = true;  // less than 2x in norm over 20 iterations
            mark = best;
            since = 0;
        }
        if (broke) break;
    }
    // fall back to CG on the remaining defect: Dhat d = r, x += d
    *fell_back = true;
    HIPCHK(hipMemcpyAsync(W.bh, rr, nh * sizeof(cd), hipMemcpyDeviceToDevice, ctx->st));
    HIPCHK(hipMemcpyAsync(Z[0], W.xcg, nh * sizeof(cd), hipMemcpyDeviceToDevice, ctx->st));
    const double rel = std::sqrt(std::max(r2, 1e-300) / b2);
    CgOut c = cg64(ctx, W, mp, mm, std::min(0.5, tol_n / rel), maxit - o.iters, kAutoCheckEvery);
    HIPCHK(launch_axpby<double>(1.0, Z[0], 1.0, W.xcg, nh, nullptr, ctx->st));
    o.iters += c.iters;
    o.applies += c.applies;
    o.converged = c.converged;
    return o;
}

// ------------------------------------------------------------------ 5D solve D_T x = c
struct SolveOut {
    int iters = 0, applies = 0, restarts = 0, updates = 0, fell_back = 0;
    double relres = 0;
    bool ok = false;
};

// true residual res = c - D_T x on both parities; returns |res|^2
double residual64(eofa_ctx* ctx, const Work64& W, double mp, double mm) {
    const SiteOp* M = site_tab(ctx, SK_M, mp, mm);
    for (int par = 0; par < 2; par++) {
        auto a = hop_args<double>(ctx, par);
        a.in = W.x.h[1 - par]; a.self = W.x.h[par]; a.aux = W.c.h[par]; a.out = W.res.h[par];
        a.opA = M; a.caux = 1.0; a.cz = -1.0;
        a.red = red_of(ctx, SC_TMP + par, EPI_STORE);
        hop<double>(ctx, false, HM_DT, true, a);
    }
    sync_scal(ctx);
    return ctx->hscal[SC_TMP] + ctx->hscal[SC_TMP + 1];
}

double norm2_64(eofa_ctx* ctx, const Vec2& v) {
    for (int par = 0; par < 2; par++) HIPCHK(launch_norm2<double>(v.h[par], ctx->nh, red_of(ctx, SC_TMP + 2 + par, EPI_STORE), ctx->st));
    sync_scal(ctx);
    return ctx->hscal[SC_TMP + 2] + ctx->hscal[SC_TMP + 3];
}

CgOut cg_single_fp16(eofa_ctx* ctx, const Work64& W, double mp, double mm, double tol_n, int maxit, int ce,
                     const eofa_solve_params& P, int* updates);

// Even-odd solve of D_T d = rhs (rhs = W.res), result added to W.x.
CgOut eo_correct64(eofa_ctx* ctx, const Work64& W, double mp, double mm, double tol_n, int maxit, int check_every,
                   const eofa_solve_params& P, int* updates, int* fell_back) {
    const SiteOp* Ai = site_tab(ctx, SK_AINV, mp, mm);
    // u_e = A^{-1} res_e ; bh = A^{-1} (res_o + 1/2 H_oe u_e)
    HIPCHK(launch_site<double>(ctx->Ns, false, W.res.h[0], W.u, Ai, ctx->g.Vh, ctx->st));
    {
        auto a = hop_args<double>(ctx, 1);
        a.in = W.u; a.out = W.bh; a.aux = W.res.h[1]; a.caux = 1.0; a.cz = 0.5; a.opA = Ai;
        hop<double>(ctx, false, HM_SITE, false, a);
    }
    CgOut o;
    if (P.pc == EOFA_PC_LEARNED) {
        bool fb = false;
        o = fgcr(ctx, W, mp, mm, tol_n, maxit, P, &fb);
        if (fb && fell_back) *fell_back = 1;
    } else if (P.prec == EOFA_FP64) {
        o = cg64(ctx, W, mp, mm, tol_n, maxit, check_every, P.use_graph != 0);
    } else if (P.prec == EOFA_MIXED_FP16) {
        o = cg_single_fp16(ctx, W, mp, mm, tol_n, maxit, check_every, P, updates);
    } else {
        o = cg_mixed(ctx, W, mp, mm, tol_n, maxit, check_every, P.reliable_delta, updates, P.use_graph != 0);
    }
    // d_e = A^{-1} (res_e + 1/2 H_eo d_o) -> u ; x += d
    {
        auto a = hop_args<double>(ctx, 0);
        a.in = W.xcg; a.out = W.u; a.aux = W.res.h[0]; a.caux = 1.0; a.cz = 0.5; a.opA = Ai;
        hop<double>(ctx, false, HM_SITE, false, a);
    }
    HIPCHK(launch_axpby<double>(1.0, W.u, 1.0, W.x.h[0], ctx->nh, nullptr, ctx->st));
    HIPCHK(launch_axpby<double>(1.0, W.xcg, 1.0, W.x.h[1], ctx->nh, nullptr, ctx->st));
    o.applies += 1;
    return o;
}

SolveOut solve_dt(eofa_ctx* ctx, const Work64& W, double mp, double mm, const eofa_solve_params& P,
                  bool guess = false);

int auto_check_every(const eofa_solve_params& P) { return P.check_every > 0 ? P.check_every : kAutoCheckEvery; }

// Defect correction on D_T x = c with W.x holding the current solution and W.res = c - D_T x:
// even-odd Krylov solves of the defect until ||c - D_T x|| / ||c|| <= tol.
void refine(eofa_ctx* ctx, const Work64& W, double mp, double mm, const eofa_solve_params& P, double cn2, double rel,
            SolveOut& so) {
    const int ce = auto_check_every(P);
    so.relres = rel;
    eofa_solve_params Q = P;  // switched to plain FP64 CG if a correction fails to halve the defect
    for (int attempt = 0; attempt < 20; attempt++) {
        if (rel <= P.tol) { so.ok = true; return; }
        if (so.iters >= P.max_iter) return;
        if (attempt > 0) so.restarts++;
        // inner target on the normal residual, relative to the current defect
        double tol_n = std::max(0.25 * P.tol / rel, 1e-15);
        CgOut o = eo_correct64(ctx, W, mp, mm, std::min(tol_n, 0.5), P.max_iter - so.iters, ce, Q, &so.updates,
                               &so.fell_back);
        so.iters += o.iters;
        so.applies += o.applies;
        double r2 = residual64(ctx, W, mp, mm);
        const double prev = rel;
        rel = std::sqrt(r2 / cn2);
        so.relres = rel;
        if (!std::isfinite(rel)) { ctx->err = "non-finite residual"; return; }
        if (rel > 0.5 * prev && (Q.prec != EOFA_FP64 || Q.pc != EOFA_PC_NONE)) {
            Q.prec = EOFA_FP64;
            Q.pc = EOFA_PC_NONE;
            so.fell_back = 1;
        }
    }
}

// guess: W.x holds a start vector (a previous solution); it is used when its residual is below |c|.
SolveOut solve_dt_fp64(eofa_ctx* ctx, const Work64& W, double mp, double mm, const eofa_solve_params& P,
                       bool guess = false) {
    SolveOut so;
    const double cn2 = norm2_64(ctx, W.c);
    REQUIRE(std::isfinite(cn2), EOFA_EINVAL, "source has non-finite entries");
    if (guess && cn2 > 0.0) {
        const double r2 = residual64(ctx, W, mp, mm);  // W.res = c - D_T x
        if (std::isfinite(r2) && r2 < cn2) {
            refine(ctx, W, mp, mm, P, cn2, std::sqrt(r2 / cn2), so);
            return so;
        }
    }
    for (int par = 0; par < 2; par++) {
        HIPCHK(hipMemsetAsync(W.x.h[par], 0, ctx->nh * sizeof(cd), ctx->st));
        HIPCHK(hipMemcpyAsync(W.res.h[par], W.c.h[par], ctx->nh * sizeof(cd), hipMemcpyDeviceToDevice, ctx->st));
    }
    if (cn2 == 0.0) { so.ok = true; return so; }
    refine(ctx, W, mp, mm, P, cn2, 1.0, so);
    return so;
}

// ------------------------------------------------------------------ multi-RHS batch
struct Sys {
    int cycle = 0;      // iterations since the last residual replacement
    int base = 0;       // iterations before the current cycle
    int stall = 0;      // consecutive reliable updates that failed to halve the residual norm
    double rr_last = 0; // |r|^2 at the last reliable update
    double mp = 0, mm = 0;
    const SiteOp* Ai = nullptr;
    const SiteOp* Ad = nullptr;
    cd* xhi = nullptr;  // FP64 solution accumulator (odd sites)
    cd* bh = nullptr;   // FP64 Schur right-hand side
    void *x, *r, *p, *u, *w, *wt, *at;  // Krylov vectors in the batch precision
    double rr0 = 0;
    bool conv = false;
    int iters = 0, updates = 0;
};

void carve_batch(eofa_ctx* ctx, const eofa_solve_params& P, std::vector<Sys>& sys) {
    char* q = ctx->ws + base_bytes(ctx, &P);
    const size_t h64 = align_up(ctx->nh * sizeof(cd));
    const size_t hxr = batch_vec_bytes(ctx, &P, true), hk = batch_vec_bytes(ctx, &P, false);
    for (Sys& y : sys) {
        y.xhi = (cd*)q; q += h64;
        y.bh = (cd*)q; q += h64;
        y.x = q; q += hxr;
        y.r = q; q += hxr;
        void** v[5] = {&y.p, &y.u, &y.w, &y.wt, &y.at};
        for (void** pp : v) { *pp = q; q += hk; }
    }
}


double* sys_scal(eofa_ctx* ctx, int r) { return ctx->scal + BATCH_OFF + r * SC_N; }

void sync_scal_batch(eofa_ctx* ctx, int nr) {
    HIPCHK(hipMemcpyAsync(ctx->hscal + BATCH_OFF, ctx->scal + BATCH_OFF, sizeof(double) * SC_N * nr,
                          hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
}

template <typename R> HopArgsMR<R> mr_args(eofa_ctx* ctx, int par, int nr, bool half = false) {
    HopArgsMR<R> a{};
    HopArgs<R> b = hop_args<R>(ctx, par);
    a.g = b.g; a.sc = half ? ctx->sched[2] : b.sc; a.par = par; a.nr = nr; a.Uown = b.Uown; a.Uoth = b.Uoth;
    a.scal = ctx->scal + BATCH_OFF;
    a.partials = ctx->partials_mr;
    a.pstride = ctx->pstride;
    return a;
}

// One batched CG iteration over the systems (converged ones are skipped on the device).  H: p, u, w,
// wt, at in FP16 columns (R = float).
template <typename R, bool H = false> void cg_iteration_mr(eofa_ctx* ctx, std::vector<Sys>& sys) {
    const int nr = (int)sys.size();
    auto V = [](void* p) { return (cpx<R>*)p; };
    {
        auto a = mr_args<R>(ctx, 0, nr, H);
        for (int r = 0; r < nr; r++) { a.in[r] = V(sys[r].p); a.out[r] = V(sys[r].u); a.opA[r] = sys[r].Ai; }
        a.cz = 1; a.caux = 0;
        HIPCHK(launch_hop_mr<R>(ctx->Ns, false, HM_SITE, a, ctx->st, H));
    }
    {
        auto a = mr_args<R>(ctx, 1, nr, H);
        for (int r = 0; r < nr; r++) {
            a.in[r] = V(sys[r].u); a.out[r] = V(sys[r].w); a.out2[r] = V(sys[r].wt); a.aux[r] = V(sys[r].p);
            a.opA[r] = sys[r].Ai; a.opB[r] = sys[r].Ad;
        }
        a.cz = (R)-0.25; a.caux = 1; a.epi = EPI_CG_W;
        HIPCHK(launch_hop_mr<R>(ctx->Ns, false, HM_SCHUR_W, a, ctx->st, H));
    }
    {
        auto a = mr_args<R>(ctx, 0, nr, H);
        for (int r = 0; r < nr; r++) { a.in[r] = V(sys[r].wt); a.out[r] = V(sys[r].at); a.opA[r] = sys[r].Ad; }
        a.cz = 1; a.caux = 0;
        HIPCHK(launch_hop_mr<R>(ctx->Ns, true, HM_SITE, a, ctx->st, H));
    }
    {
        auto a = mr_args<R>(ctx, 1, nr, H);
        for (int r = 0; r < nr; r++) {
            a.in[r] = V(sys[r].at); a.out[r] = V(sys[r].r); a.aux[r] = V(sys[r].w); a.aux2[r] = V(sys[r].r);
        }
        a.cz = (R)-0.25; a.caux = 1; a.epi = EPI_CG_R;
        HIPCHK(launch_hop_mr<R>(ctx->Ns, true, HM_SCHUR_Q, a, ctx->st, H));
    }
    cpx<R>* xs[NRMAX];
    cpx<R>* ps[NRMAX];
    cpx<R>* rs[NRMAX];
    for (int r = 0; r < nr; r++) { xs[r] = V(sys[r].x); ps[r] = V(sys[r].p); rs[r] = V(sys[r].r); }
    if constexpr (H) {
        void* ph[NRMAX];
        for (int r = 0; r < nr; r++) ph[r] = sys[r].p;
        HIPCHK(launch_cg_xp_mr_h(ctx->Ns, nr, (cpx<float>* const*)xs, ph, (cpx<float>* const*)rs, ctx->scal + BATCH_OFF,
                                 ctx->g.Vh, ctx->st));
    } else {
        HIPCHK(launch_cg_xp_mr<R>(nr, xs, ps, rs, ctx->scal + BATCH_OFF, ctx->nh, ctx->st));
    }
}

// Batched CG on the systems' Schur normal equations to |r_normal| <= tol_n |r_normal,0| each.  With R = float
// every system gets FP64 reliable updates (residual replacement) on its own schedule.
template <typename R, bool H = false>
void cg_batch(eofa_ctx* ctx, const Work64& W, std::vector<Sys>& sys, double tol_n, int maxit, int ce, double delta,
              bool graph = false) {
    const int nr = (int)sys.size();
    const bool mixed = sizeof(R) == 4;
    if (delta <= 0 || delta >= 1) delta = 0.1;
    if (ce <= 0) ce = 1;
    const size_t nb = ctx->nh * sizeof(cpx<R>);
    auto arm = [&](int r, double rr, double rr_ref) {
        const double tol2 = mixed ? std::max(delta * delta, tol_n * tol_n * sys[r].rr0 / rr) : tol_n * tol_n;
        double* S = sys_scal(ctx, r);
        HIPCHK(launch_scal_set(S, SC_RR, rr, SC_RR0, rr_ref, SC_TOL2, tol2, ctx->st));
        HIPCHK(launch_scal_set(S, SC_DONE, 0.0, SC_DONEX, 0.0, SC_ITERS, 0.0, ctx->st));
        sys[r].base = sys[r].iters;  // SC_ITERS counts this cycle's iterations
        sys[r].cycle = 0;
    };
    for (int r = 0; r < nr; r++) {
        Sys& y = sys[r];
        HIPCHK(hipMemsetAsync(y.xhi, 0, ctx->nh * sizeof(cd), ctx->st));
        HIPCHK(hipMemsetAsync(y.x, 0, nb, ctx->st));
        double rr = normal_residual64(ctx, W, y.xhi, y.bh, y.Ai, y.Ad);   // r = Dhat^dag bh in W.r
        y.rr0 = rr;
        if (rr == 0.0) {
            y.conv = true;
            HIPCHK(launch_scal_set(sys_scal(ctx, r), SC_DONE, 1.0, SC_DONEX, 1.0, -1, 0, ctx->st));
            continue;
        }
        if (mixed) HIPCHK(launch_convert_d2f(W.r, (cpx<float>*)y.r, ctx->nh, ctx->st));
        else HIPCHK(hipMemcpyAsync(y.r, W.r, nb, hipMemcpyDeviceToDevice, ctx->st));
        if constexpr (H) HIPCHK(launch_f2h(ctx->Ns, (const cpx<float>*)y.r, y.p, ctx->g.Vh, ctx->st));
        else HIPCHK(hipMemcpyAsync(y.p, y.r, nb, hipMemcpyDeviceToDevice, ctx->st));
        arm(r, rr, rr);
    }
    // blocks of ce iterations between host checks; each system counts its applied iterations on the device
    int it = 0;
    while (it < maxit) {
        bool all = true;
        for (const Sys& y : sys) all &= y.conv;
        if (all) break;
        const int blk = std::min(ce, maxit - it);
        if (graph && blk == ce) {
            std::vector<uintptr_t> key = graph_key<R>(ctx, H ? 4 : 3, ce, {}, H);
            for (const Sys& y : sys)
                for (const void* q : {(const void*)y.Ai, (const void*)y.Ad, (const void*)y.x, (const void*)y.r,
                                      (const void*)y.p, (const void*)y.u, (const void*)y.w, (const void*)y.wt,
                                      (const void*)y.at})
                    key.push_back((uintptr_t)q);
            graph_run(ctx, std::move(key), [&] {
                for (int k = 0; k < ce; k++) cg_iteration_mr<R, H>(ctx, sys);
            });
        } else {
            for (int k = 0; k < blk; k++) cg_iteration_mr<R, H>(ctx, sys);
        }
        it += blk;
        sync_scal_batch(ctx, nr);
        for (int r = 0; r < nr; r++) {
            Sys& y = sys[r];
            const double* hs = ctx->hscal + BATCH_OFF + r * SC_N;
            if (y.conv) continue;
            y.cycle = (int)hs[SC_ITERS];
            y.iters = y.base + y.cycle;
            if (hs[SC_DONE] == 0.0 && !(mixed && y.cycle >= kMaxCycle)) continue;
            if (!std::isfinite(hs[SC_RR])) { ctx->err = "batched CG breakdown"; y.conv = true; continue; }
            if (!mixed) { y.conv = true; HIPCHK(hipMemcpyAsync(y.xhi, y.x, nb, hipMemcpyDeviceToDevice, ctx->st)); continue; }
            // reliable update of system r (its delta target reached, or its cycle cut at kMaxCycle)
            HIPCHK(launch_accum_f(y.xhi, (const cpx<float>*)y.x, ctx->nh, ctx->st));
            HIPCHK(hipMemsetAsync(y.x, 0, nb, ctx->st));
            double rr = normal_residual64(ctx, W, y.xhi, y.bh, y.Ai, y.Ad);
            y.updates++;
            // stagnation: the reduced-precision iteration no longer reduces the FP64 residual (the
            // defect correction above the batch then continues in FP64)
            y.stall = (y.rr_last > 0 && rr > 0.25 * y.rr_last) ? y.stall + 1 : 0;
            y.rr_last = rr;
            if (rr <= tol_n * tol_n * y.rr0 || !std::isfinite(rr) || y.stall >= 8) {
                y.conv = true;
                HIPCHK(launch_scal_set(sys_scal(ctx, r), SC_DONE, 1.0, SC_DONEX, 1.0, -1, 0, ctx->st));
                continue;
            }
            HIPCHK(launch_convert_d2f(W.r, (cpx<float>*)y.r, ctx->nh, ctx->st));
            arm(r, rr, rr);
        }
    }
    if (!mixed)  // systems stopped by max_iter: keep their last iterate
        for (Sys& y : sys)
            if (!y.conv) HIPCHK(hipMemcpyAsync(y.xhi, y.x, nb, hipMemcpyDeviceToDevice, ctx->st));
    if (mixed)
        for (Sys& y : sys)
            if (!y.conv) HIPCHK(launch_accum_f(y.xhi, (const cpx<float>*)y.x, ctx->nh, ctx->st));
}

// Dhat W.xcg = W.bh with FP16-column Krylov vectors: a one-system batch (FP64 reliable updates)
CgOut cg_single_fp16(eofa_ctx* ctx, const Work64& W, double mp, double mm, double tol_n, int maxit, int ce,
                     const eofa_solve_params& P, int* updates) {
    std::vector<Sys> sys(1);
    carve_batch(ctx, P, sys);
    ensure_partials_mr(ctx);
    Sys& y = sys[0];
    y.mp = mp;
    y.mm = mm;
    y.Ai = site_tab(ctx, SK_AINV, mp, mm);
    y.Ad = site_tab(ctx, SK_AINV_DAG, mp, mm);
    y.bh = W.bh;
    cg_batch<float, true>(ctx, W, sys, tol_n, maxit, ce, P.reliable_delta, P.use_graph != 0);
    HIPCHK(hipMemcpyAsync(W.xcg, y.xhi, ctx->nh * sizeof(cd), hipMemcpyDeviceToDevice, ctx->st));
    CgOut o;
    o.iters = y.iters;
    o.applies = 2 * y.iters + 2 * y.updates + 2;
    o.converged = y.conv;
    if (updates) *updates += y.updates;
    return o;
}

void check_params(eofa_ctx* ctx, const eofa_solve_params* P) {
    REQUIRE(P != nullptr, EOFA_EINVAL, "params is NULL");
    REQUIRE(P->tol > 0 && P->tol < 1, EOFA_EINVAL, "tol must be in (0, 1)");
    REQUIRE(P->max_iter > 0, EOFA_EINVAL, "max_iter must be positive");
    REQUIRE(P->prec == EOFA_FP64 || P->prec == EOFA_MIXED_FP32 || P->prec == EOFA_MIXED_FP16, EOFA_EINVAL,
            "unknown precision");
    REQUIRE(P->pc == EOFA_PC_NONE || P->pc == EOFA_PC_LEARNED, EOFA_EINVAL, "unknown preconditioner");
    REQUIRE(ctx->gauge, EOFA_ESTATE, "no gauge field set");
}

SolveOut solve_dt(eofa_ctx* ctx, const Work64& W, double mp, double mm, const eofa_solve_params& P, bool guess) {
    if (P.prec == EOFA_MIXED_FP16)
        REQUIRE(ctx->Ns >= 8 && ctx->Ns % 8 == 0, EOFA_EINVAL, "EOFA_MIXED_FP16 needs Ns in {8, 16, 32}");
    if (P.pc == EOFA_PC_LEARNED) {
        REQUIRE(ctx->cnn.ready, EOFA_ESTATE, "learned preconditioner: no weights (eofa_cnn_init or eofa_set_precond)");
        REQUIRE(ctx->Ns % 8 == 0, EOFA_EINVAL, "learned preconditioner needs Ns % 8 == 0");
    }
    return solve_dt_fp64(ctx, W, mp, mm, P, guess);
}

void fill_info(eofa_solve_info* info, const SolveOut& so, double secs) {
    if (!info) return;
    info->iters = so.iters;
    info->op_applies = so.applies;
    info->reliable_updates = so.restarts + 1 + so.updates;
    info->fell_back = so.fell_back;
    info->true_rel_resid = so.relres;
    info->seconds = secs;
}

double kfac(double mj, double mi) { return 2.0 * (mj - mi) / ((1.0 + mj) * (1.0 + mi)); }

// Om_s = (-1)^s omega_s^{-1/2} (s = 1..Ns), the vector of Eq.(delta_ij) for this operator.
std::vector<double> omega_vec(const eofa_ctx* ctx) {
    std::vector<double> Om(ctx->Ns);
    for (int s = 0; s < ctx->Ns; s++) Om[s] = ((s % 2 == 0) ? -1.0 : 1.0) / std::sqrt(ctx->omega[s]);
    return Om;
}

// W.c = R5 gamma_5 (Om (x) P_chir phi), i.e. c_s = chir Om_{Ns+1-s} P_chir phi, on both parities.
void make_source(eofa_ctx* ctx, const Work64& W, int chir, const void* phi) {
    const int Ns = ctx->Ns;
    std::vector<double> Om = omega_vec(ctx), coef(Ns);
    for (int s = 0; s < Ns; s++) coef[s] = chir * Om[Ns - 1 - s];
    double* dcoef = ctx->scal + SC_N;
    HIPCHK(launch_set_vec(dcoef, Ns, coef.data(), ctx->st));
    for (int par = 0; par < 2; par++)
        HIPCHK(launch_source((const cd*)phi, W.c.h[par], ctx->g, par, Ns, chir, dcoef, ctx->st));
}

// bh = A^{-1} (c_o + H_oe A^{-1} c_e / 2), the Schur right-hand side of D_T x = c.
void prep_schur(eofa_ctx* ctx, const Work64& W, const SiteOp* Ai, cd* bh) {
    HIPCHK(launch_site<double>(ctx->Ns, false, W.c.h[0], W.u, Ai, ctx->g.Vh, ctx->st));
    auto a = hop_args<double>(ctx, 1);
    a.in = W.u; a.out = bh; a.aux = W.c.h[1]; a.caux = 1.0; a.cz = 0.5; a.opA = Ai;
    hop<double>(ctx, false, HM_SITE, false, a);
}

// W.x = (A^{-1} (c_e + H_eo xo / 2), xo)
void reconstruct(eofa_ctx* ctx, const Work64& W, const SiteOp* Ai, const cd* xo) {
    auto a = hop_args<double>(ctx, 0);
    a.in = xo; a.out = W.x.h[0]; a.aux = W.c.h[0]; a.caux = 1.0; a.cz = 0.5; a.opA = Ai;
    hop<double>(ctx, false, HM_SITE, false, a);
    HIPCHK(hipMemcpyAsync(W.x.h[1], xo, ctx->nh * sizeof(cd), hipMemcpyDeviceToDevice, ctx->st));
}

// out = P_chir phi + chir k Om^T P_chir x (written, or added with accumulate); returns Re phi^dag (this part).
double combine(eofa_ctx* ctx, const Work64& W, int chir, double k, const void* phi, void* out, int accumulate) {
    std::vector<double> Om = omega_vec(ctx);
    double* dOm = ctx->scal + SC_N + 64;
    HIPCHK(launch_set_vec(dOm, ctx->Ns, Om.data(), ctx->st));
    for (int par = 0; par < 2; par++)
        HIPCHK(launch_combine((const cd*)phi, W.x.h[par], (cd*)out, ctx->g, par, ctx->Ns, chir, chir * k, dOm, accumulate,
                              red_of(ctx, SC_TMP + 4 + par, EPI_STORE), ctx->st));
    sync_scal(ctx);
    return ctx->hscal[SC_TMP + 4] + ctx->hscal[SC_TMP + 5];
}

double action_k(int chir, double m3, double m4, double mo) { return (chir < 0) ? kfac(mo, m4) : kfac(mo, m3); }

void check_action(eofa_ctx* ctx, int chir, double m3, double m4, double mo, const void* phi, const void* out) {
    REQUIRE(chir == 1 || chir == -1, EOFA_EINVAL, "chir must be +1 or -1");
    REQUIRE(phi && out, EOFA_EINVAL, "null field pointer");
    REQUIRE(phi != out, EOFA_EINVAL, "phi and out may not alias");
    for (double m : {m3, m4, mo}) REQUIRE(m > 0 && m <= 1, EOFA_EINVAL, "masses must lie in (0, 1]");
}

// One chiral action; writes (accumulate = 0) or adds (accumulate = 1) its P_chir part into out.
// x0 (optional): the two internal halves of a start vector for the 5D solve.
eofa_status chiral_impl(eofa_ctx* ctx, int chir, double m3, double m4, double mo, const void* phi, void* out,
                        int accumulate, double* S, const eofa_solve_params* P, eofa_solve_info* info,
                        cd* const* x0 = nullptr) {
    check_params(ctx, P);
    check_action(ctx, chir, m3, m4, mo, phi, out);
    auto t0 = std::chrono::steady_clock::now();
    ensure_ws(ctx, needed_bytes(ctx, P));
    Work64 W = carve64(ctx);
    make_source(ctx, W, chir, phi);
    if (x0)
        for (int par = 0; par < 2; par++) HIPCHK(launch_copy(W.x.h[par], x0[par], ctx->nh * sizeof(cd), ctx->st));
    SolveOut so = solve_dt(ctx, W, m3, m4, *P, x0 != nullptr);
    const double s = combine(ctx, W, chir, action_k(chir, m3, m4, mo), phi, out, accumulate);
    if (S) *S = s;
    collect_timing(ctx);
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(info, so, secs);
    if (!so.ok) {
        if (ctx->err.empty()) ctx->err = "solve did not reach tol within max_iter";
        return EOFA_ENOCONV;
    }
    return EOFA_OK;
}

// n 5D systems D_T(mp[j], mm[j]) x_j = c_j through the multi-RHS path, in groups of up to NRMAX systems:
// fill_c(W, j) writes c_j into W.c; done(W, j, so) consumes the solution in W.x once the FP64 defect
// correction has brought it to tol.
template <typename FillC, typename Done>
eofa_status batch_solve(eofa_ctx* ctx, int n, const double* mp, const double* mm, const eofa_solve_params* P,
                        eofa_solve_info* info, FillC&& fill_c, Done&& done) {
    ensure_ws(ctx, needed_bytes(ctx, P, n));
    ensure_partials_mr(ctx);
    Work64 W = carve64(ctx);
    eofa_status worst = EOFA_OK;
    for (int g0 = 0; g0 < n; g0 += NRMAX) {
        const int nr = std::min(NRMAX, n - g0);
        auto t0 = std::chrono::steady_clock::now();
        std::vector<Sys> sys(nr);
        carve_batch(ctx, *P, sys);
        for (int r = 0; r < nr; r++) {
            const int j = g0 + r;
            Sys& y = sys[r];
            y.mp = mp[j];
            y.mm = mm[j];
            y.Ai = site_tab(ctx, SK_AINV, y.mp, y.mm);
            y.Ad = site_tab(ctx, SK_AINV_DAG, y.mp, y.mm);
            fill_c(W, j);
            REQUIRE(std::isfinite(norm2_64(ctx, W.c)), EOFA_EINVAL, "source has non-finite entries");
            prep_schur(ctx, W, y.Ai, y.bh);
        }
        const double tol_n = 0.25 * P->tol;
        const int ce = auto_check_every(*P);
        if (P->prec == EOFA_FP64) cg_batch<double>(ctx, W, sys, tol_n, P->max_iter, ce, P->reliable_delta, P->use_graph != 0);
        else if (P->prec == EOFA_MIXED_FP16)
            cg_batch<float, true>(ctx, W, sys, tol_n, P->max_iter, ce, P->reliable_delta, P->use_graph != 0);
        else cg_batch<float>(ctx, W, sys, tol_n, P->max_iter, ce, P->reliable_delta, P->use_graph != 0);
        HIPCHK(hipStreamSynchronize(ctx->st));
        const double tb = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() / nr;
        for (int r = 0; r < nr; r++) {
            const int j = g0 + r;
            Sys& y = sys[r];
            auto t1 = std::chrono::steady_clock::now();
            fill_c(W, j);
            const double cn2 = norm2_64(ctx, W.c);
            reconstruct(ctx, W, y.Ai, y.xhi);
            SolveOut so;
            so.iters = y.iters;
            so.updates = y.updates;
            so.applies = 2 * y.iters + 2 * y.updates + 2;
            const double rel = cn2 > 0 ? std::sqrt(residual64(ctx, W, y.mp, y.mm) / cn2) : 0.0;
            refine(ctx, W, y.mp, y.mm, *P, cn2 > 0 ? cn2 : 1.0, rel, so);
            done(W, j, so);
            const double te = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
            fill_info(info ? &info[j] : nullptr, so, tb + te);
            if (!so.ok) worst = EOFA_ENOCONV;
        }
    }
    collect_timing(ctx);
    if (worst != EOFA_OK && ctx->err.empty()) ctx->err = "a batched solve did not reach tol within max_iter";
    return worst;
}

// Whether n systems under P go through the multi-RHS kernels (else one by one).
bool use_batch(const eofa_ctx* ctx, int n, const eofa_solve_params* P) {
    return !((n <= 1 && P->prec != EOFA_MIXED_FP16) || ctx->Ns < 8 || P->pc != EOFA_PC_NONE);
}

// n chiral actions through the multi-RHS path, in groups of up to NRMAX systems.
eofa_status chiral_batch_impl(eofa_ctx* ctx, int n, const int* chir, const double* m3, const double* m4,
                              const double* mo, const void* const* phi, void* const* out, const int* accumulate,
                              double* S, const eofa_solve_params* P, eofa_solve_info* info) {
    check_params(ctx, P);
    for (int j = 0; j < n; j++) check_action(ctx, chir[j], m3[j], m4[j], mo[j], phi[j], out[j]);
    if (!use_batch(ctx, n, P)) {
        eofa_status worst = EOFA_OK;
        for (int j = 0; j < n; j++) {
            double sj = 0;
            eofa_status a = chiral_impl(ctx, chir[j], m3[j], m4[j], mo[j], phi[j], out[j], accumulate ? accumulate[j] : 0,
                                        &sj, P, info ? &info[j] : nullptr);
            if (S) S[j] = sj;
            if (a != EOFA_OK && a != EOFA_ENOCONV) return a;
            if (a != EOFA_OK) worst = a;
        }
        return worst;
    }
    return batch_solve(
        ctx, n, m3, m4, P, info, [&](const Work64& W, int j) { make_source(ctx, W, chir[j], phi[j]); },
        [&](const Work64& W, int j, const SolveOut&) {
            const double s = combine(ctx, W, chir[j], action_k(chir[j], m3[j], m4[j], mo[j]), phi[j], out[j],
                                     accumulate ? accumulate[j] : 0);
            if (S) S[j] = s;
        });
}

// H_T(mp, mm) x5 = b5 on canonical 5D fields: c = R5 gamma_5 b, D_T x = c.
eofa_status solve_ht_impl(eofa_ctx* ctx, double mp, double mm, const void* b5, void* x5, const eofa_solve_params* P,
                          eofa_solve_info* info) {
    check_params(ctx, P);
    REQUIRE(b5 && x5 && b5 != x5, EOFA_EINVAL, "bad field pointers");
    REQUIRE(mp > 0 && mp <= 1 && mm > 0 && mm <= 1, EOFA_EINVAL, "masses must lie in (0, 1]");
    auto t0 = std::chrono::steady_clock::now();
    ensure_ws(ctx, needed_bytes(ctx, P));
    Work64 W = carve64(ctx);
    for (int par = 0; par < 2; par++)
        HIPCHK(launch_pack5<double>((const cd*)b5, W.c.h[par], ctx->g, par, ctx->Ns, 1, ctx->st));
    SolveOut so = solve_dt(ctx, W, mp, mm, *P);
    for (int par = 0; par < 2; par++)
        HIPCHK(launch_unpack5<double>(W.x.h[par], (cd*)x5, ctx->g, par, ctx->Ns, 0, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    collect_timing(ctx);
    fill_info(info, so, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    if (!so.ok) {
        if (ctx->err.empty()) ctx->err = "solve did not reach tol within max_iter";
        return EOFA_ENOCONV;
    }
    return EOFA_OK;
}

// ------------------------------------------------------------------ heat-bath (Sec. I, Eq.(CG_gaussian))
// The pseudofermion of a chiral action S = phi^dag A phi is drawn as phi = A^{-1/2} P_c eta from Gaussian noise
// eta.  x^{-1/2} is replaced on the interval [lo, hi] that holds the spectrum of A by Zolotarev's optimal
// rational function in partial fractions, a0 + sum_l a_l / (x + b_l) (b_l > 0), so
//     phi = a0 P_c eta + sum_l a_l (A + b_l)^{-1} P_c eta.
// For the - action A = 1 - k Om^T H_T(m3, m4)^{-1} Om P_-, the Woodbury identity and the rank-one mass
// difference H_T(m3, m4') = H_T(m3, m4) - k(m4', m4) P_- Om Om^T give
//     (1 + b) (A + b)^{-1} eta = P_- [eta + c Om^T H_T(m3, m4')^{-1} Om P_- eta],  k(m4', m4) = c = k / (1 + b),
// which is the - chiral action (m3, m4') / (m3, m4) of eta; likewise the + action with m3' from
// k(m3', m3) = k / (1 + b) and the other mass m3.  The shifted masses lie between the action's two masses, and
// every pole's system goes through one multi-RHS launch sequence.

// complete elliptic integral of the first kind K(k) (modulus k < 1) by the arithmetic-geometric mean
double ellip_K(double k) {
    double a = 1.0, b = std::sqrt((1.0 - k) * (1.0 + k));
    for (int i = 0; i < 64 && std::fabs(a - b) > 1e-16 * a; i++) {
        const double an = 0.5 * (a + b);
        b = std::sqrt(a * b);
        a = an;
    }
    return M_PI / (2.0 * a);
}

// Jacobi elliptic sn(u, k) and cn(u, k) by the descending Landen (AGM) scheme
void ellip_sncn(double u, double k, double& sn, double& cn) {
    double a[64], c[64];
    double b = std::sqrt((1.0 - k) * (1.0 + k));
    a[0] = 1.0;
    c[0] = k;
    int n = 0;
    while (n < 62 && std::fabs(c[n]) > 1e-17) {
        a[n + 1] = 0.5 * (a[n] + b);
        c[n + 1] = 0.5 * (a[n] - b);
        b = std::sqrt(a[n] * b);
        n++;
    }
    double phi = std::ldexp(1.0, n) * a[n] * u;
    for (int i = n; i > 0; i--) phi = 0.5 * (phi + std::asin(c[i] * std::sin(phi) / a[i]));
    sn = std::sin(phi);
    cn = std::cos(phi);
}

struct RatInvSqrt {
    int n = 0;
    double a0 = 1.0, a[HB_MAXTERMS] = {}, b[HB_MAXTERMS] = {};
    double err = 0.0;  // max |sqrt(x) r(x) - 1| on [lo, hi] (dense geometric grid)
};

// Zolotarev's optimal relative approximation of x^{-1/2} on [lo, hi] with n poles: zeros and poles
// c_j = lo sn^2 / cn^2 (j K' / (2n + 1); k'), k' = sqrt(1 - lo / hi), K' = K(k'), poles at -c_{2l-1} and zeros
// at -c_{2l}; the overall factor makes sqrt(x) r(x) equioscillate about 1.
RatInvSqrt zolotarev_inv_sqrt(double lo, double hi, int n) {
    RatInvSqrt r;
    r.n = n;
    const double kp = std::sqrt(1.0 - lo / hi), K = ellip_K(kp);
    std::vector<double> c(2 * n + 1);
    for (int j = 1; j <= 2 * n; j++) {
        double sn, cn;
        ellip_sncn(j * K / (2 * n + 1), kp, sn, cn);
        c[j] = lo * sn * sn / (cn * cn);
    }
    double R[HB_MAXTERMS];
    for (int l = 0; l < n; l++) {  // residue of prod (x + z_j) / (x + p_j) at the pole -p_l
        const double pl = c[2 * l + 1];
        double num = 1.0, den = 1.0;
        for (int j = 0; j < n; j++) {
            num *= c[2 * j + 2] - pl;
            if (j != l) den *= c[2 * j + 1] - pl;
        }
        R[l] = num / den;
        r.b[l] = pl;
    }
    auto e = [&](double x) {
        double v = 1.0;
        for (int l = 0; l < n; l++) v += R[l] / (x + r.b[l]);
        return std::sqrt(x) * v;
    };
    const int G = 8001;
    double emax = 0, emin = 1e300;
    for (int i = 0; i < G; i++) {
        const double v = e(lo * std::pow(hi / lo, (double)i / (G - 1)));
        emax = std::max(emax, v);
        emin = std::min(emin, v);
    }
    const double D = 2.0 / (emax + emin);
    r.a0 = D;
    for (int l = 0; l < n; l++) r.a[l] = D * R[l];
    r.err = std::max(D * emax - 1.0, 1.0 - D * emin);
    return r;
}

// the fewest poles (<= HB_MAXTERMS) whose error on [lo, hi] is at most rel_err
RatInvSqrt choose_inv_sqrt(eofa_ctx* ctx, double lo, double hi, double rel_err) {
    RatInvSqrt r;
    for (int n = 1; n <= HB_MAXTERMS; n++) {
        r = zolotarev_inv_sqrt(lo, hi, n);
        if (r.err <= rel_err) return r;
    }
    REQUIRE(false, EOFA_EINVAL, "heat-bath: rel_err " + std::to_string(rel_err) + " needs more than " +
                                    std::to_string(HB_MAXTERMS) + " poles on [lo, hi]");
    return r;
}

// the mass m' with k(m', m) = c (between m and the mass whose k it divides)
double shifted_mass(double m, double c) { return (2.0 * m + c * (1.0 + m)) / (2.0 - c * (1.0 + m)); }

// phi (+)= A^{-1/2} P_chir eta for the chiral action (chir, m3, m4, mo)
eofa_status heatbath_impl(eofa_ctx* ctx, int chir, double m3, double m4, double mo, const void* eta, void* phi,
                          double lo, double hi, double rel_err, const eofa_solve_params* P, int accumulate,
                          int verify, eofa_heatbath_info* info) {
    check_params(ctx, P);
    check_action(ctx, chir, m3, m4, mo, eta, phi);
    REQUIRE(rel_err > 0 && rel_err < 1, EOFA_EINVAL, "rel_err must lie in (0, 1)");
    auto t0 = std::chrono::steady_clock::now();
    const double ma = std::min(chir < 0 ? m4 : m3, mo), mb = std::max(chir < 0 ? m4 : m3, mo);
    const double rr = (1.0 + ma) / (1.0 + mb);
    if (lo <= 0 && hi <= 0) { lo = 0.9 * rr; hi = 1.1 / rr; }
    REQUIRE(lo > 0 && hi > lo, EOFA_EINVAL, "heat-bath: need 0 < lo < hi (or both 0 for the default)");
    const double k = action_k(chir, m3, m4, mo);
    RatInvSqrt R;
    if (k != 0.0) R = choose_inv_sqrt(ctx, lo, hi, rel_err);  // k = 0: A = 1, phi = P_c eta exactly
    const size_t n4 = (size_t)ctx->g.Vh * 2 * 12;            // complex elements of a 4D field
    const size_t need = (size_t)(R.n + 1) * n4 * sizeof(cd);
    if (ctx->hb_bytes < need) {
        if (ctx->hb) HIPCHK(hipFree(ctx->hb));
        ctx->hb = nullptr;
        ctx->hb_bytes = 0;
        HIPCHK(hipMalloc(&ctx->hb, need));
        ctx->hb_bytes = need;
    }
    std::vector<int> ch(R.n, chir);
    std::vector<double> a3(R.n), a4(R.n), ao(R.n), Sj(R.n);
    std::vector<const void*> src(R.n, eta);
    std::vector<void*> dst(R.n);
    std::vector<eofa_solve_info> inf(R.n);
    HbTerms t{};
    t.a0 = R.a0;
    t.n = R.n;
    for (int l = 0; l < R.n; l++) {
        const double c = k / (1.0 + R.b[l]);
        if (chir < 0) { a3[l] = m3; a4[l] = shifted_mass(m4, c); ao[l] = m4; }
        else { a3[l] = shifted_mass(m3, c); a4[l] = m4; ao[l] = m3; }
        dst[l] = (void*)((cd*)ctx->hb + (size_t)l * n4);
        t.out[l] = (const cd*)dst[l];
        t.coef[l] = R.a[l] / (1.0 + R.b[l]);
    }
    eofa_status st = EOFA_OK;
    if (R.n > 0) {
        st = chiral_batch_impl(ctx, R.n, ch.data(), a3.data(), a4.data(), ao.data(), src.data(), dst.data(), nullptr,
                               Sj.data(), P, inf.data());
        if (st != EOFA_OK && st != EOFA_ENOCONV) return st;
    }
    HIPCHK(launch_hb_combine((const cd*)eta, (cd*)phi, t, n4, chir, accumulate, red_of(ctx, SC_TMP + 16, EPI_STORE),
                             ctx->st));
    sync_scal(ctx);
    const double eta2 = ctx->hscal[SC_TMP + 16];
    double check = 0.0;
    if (verify) {  // S(phi) = phi^dag A phi (the action reads the P_c half of phi only) against |P_c eta|^2
        double S = 0;
        eofa_solve_info vi{};
        const eofa_status s2 = chiral_impl(ctx, chir, m3, m4, mo, phi, (void*)((cd*)ctx->hb + (size_t)R.n * n4), 0, &S,
                                           P, &vi);
        if (s2 != EOFA_OK && s2 != EOFA_ENOCONV) return s2;
        check = eta2 > 0 ? S / eta2 - 1.0 : 0.0;
    }
    if (info) {
        info->npoles = R.n;
        info->approx_err = R.err;
        info->lo = lo;
        info->hi = hi;
        info->check = check;
        info->iters_max = 0;
        info->true_rel_resid_max = 0;
        for (const auto& i : inf) {
            info->iters_max = std::max(info->iters_max, i.iters);
            info->true_rel_resid_max = std::max(info->true_rel_resid_max, i.true_rel_resid);
        }
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

// nrep launches of the fused hop (A_T^{-1} epilogue) alternating parities on workspace buffers,
// under schedule sc; returns the average device ms per launch.
double time_hop(eofa_ctx* ctx, int prec, int nrep, const Sched& sc) {
    Work64 W = carve64(ctx);
    const SiteOp* Ai = site_tab(ctx, SK_AINV, 0.01, 0.01);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto run = [&](int n) {
        for (int i = 0; i < n; i++) {
            const int par = i & 1;
            if (prec == EOFA_FP64) {
                auto a = hop_args<double>(ctx, par);
                a.sc = sc;
                a.in = par ? W.u : W.p; a.out = par ? W.p : W.u; a.opA = Ai; a.cz = 1.0; a.caux = 0.0;
                HIPCHK(launch_hop<double>(ctx->Ns, false, HM_SITE, false, a, ctx->st));
            } else if (prec == EOFA_MIXED_FP32) {
                auto a = hop_args<float>(ctx, par);
                a.sc = sc;
                cpx<float>* pf = (cpx<float>*)W.p;
                cpx<float>* uf = (cpx<float>*)W.u;
                a.in = par ? uf : pf; a.out = par ? pf : uf; a.opA = Ai; a.cz = 1.0f; a.caux = 0.0f;
                HIPCHK(launch_hop<float>(ctx->Ns, false, HM_SITE, false, a, ctx->st));
            } else {  // FP16 columns through the batch kernel, one system
                auto a = mr_args<float>(ctx, par, 1, true);
                a.sc = sc;
                cpx<float>* pf = (cpx<float>*)W.p;
                cpx<float>* uf = (cpx<float>*)W.u;
                a.in[0] = par ? uf : pf; a.out[0] = par ? pf : uf; a.opA[0] = Ai; a.cz = 1.0f; a.caux = 0.0f;
                HIPCHK(launch_hop_mr<float>(ctx->Ns, false, HM_SITE, a, ctx->st, true));
            }
        }
    };
    run(2);
    HIPCHK(hipEventRecord(e0, ctx->st));
    run(nrep);
    HIPCHK(hipEventRecord(e1, ctx->st));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return t / nrep;
}

void fill_bench_buffers(eofa_ctx* ctx) {
    Work64 W = carve64(ctx);
    // finite, non-trivial contents (0x3F3F... is about 4.4e-4 as a double, 0.75 as a float)
    HIPCHK(hipMemsetAsync(W.p, 0x3F, ctx->nh * sizeof(cd), ctx->st));
    HIPCHK(hipMemsetAsync(W.u, 0x3F, ctx->nh * sizeof(cd), ctx->st));
}

std::vector<Sched> sched_candidates(const eofa_ctx* ctx, int prec) {
    std::vector<Sched> c;
    const Geom& g = ctx->g;
    const long lanes_line = (long)g.Lxh * g.Ly * ctx->Ns;  // lanes of one (z, t) line
    const int nyb = (lanes_line % 256 == 0) ? (int)(lanes_line / 256) : 0;
    for (int x = 0; x < 2; x++) c.push_back(Sched{0, x, 1, 1, 1, nyb > 0 ? nyb : 1, 0});
    if (nyb == 0) return c;
    const int opts[] = {1, 2, 4, 8, 16};
    for (int x = 0; x < 2; x++) {
        // small 3D tiles, yb fastest
        for (int ty : opts)
            for (int tz : opts)
                for (int tt : opts) {
                    if (nyb % ty || g.Lz % tz || g.Lt % tt) continue;
                    const int per = ty * tz * tt;
                    if (per < 16 || per > 128) continue;
                    c.push_back(Sched{1, x, ty, tz, tt, nyb, 0});
                }
        // long tiles through yb with a small (z, t) patch visited fastest: the yb-neighbour rows stay within
        // one patch of the L2 window, z/t neighbours inside the patch
        for (int ty : {nyb, nyb / 2, nyb / 4})
            for (int tz : opts)
                for (int tt : opts) {
                    if (ty < 1 || nyb % ty || g.Lz % tz || g.Lt % tt) continue;
                    const int pz = tz * tt;
                    if (pz < 4 || pz > 64) continue;
                    c.push_back(Sched{1, x, ty, tz, tt, nyb, 1});
                }
    }
    if (prec != EOFA_MIXED_FP16) {
        // t-walk (mode 3; mode 5 with the x neighbours from LDS): patches of 8 .. 64 segments per XCD,
        // chunks of 16 slabs or the whole t extent, with and without 48 KB of reserved LDS
        for (int ty : opts)
            for (int tz : opts)
                for (int tt : {16, g.Lt})
                    for (int pad : {0, 48})
                        for (int mode : {3, 5, 6}) {
                            // modes 5 and 6 already hold the whole LDS of a CU (one workgroup per CU): a reserve
                            // would be clamped to nothing and only duplicate the candidate
                            if (mode >= 5 && pad) continue;
                            const Sched s{mode, 1, ty, tz, tt, nyb, pad};
                            const int per = ty * tz;
                            if (per < 8 || per > 64 || tw_grid(g, ctx->Ns, s) == 0) continue;
                            bool dup = false;
                            for (const Sched& o : c)
                                dup |= (o.mode == mode && o.ty == ty && o.tz == tz && o.tt == tt && o.ord == pad);
                            if (!dup) c.push_back(s);
                        }
    }
    return c;
}

template <typename R> struct ApplyBufs {
    cpx<R>* in[2];
    cpx<R>* out[2];
    cpx<R> *u, *w, *wt, *at;
    const SiteOp* tab[SK_NKIND];  // site-operator tables by SiteKind for (mp, mm); a null entry is taken from site_tab
    double* partials;      // reduction buffers of the Schur kernels (null: the context's)
    double* scal;
};

// out = op(in) on canonical 5D fields, in storage/arithmetic type R.  Every step is a kernel launch on
// ctx->st (no memset or copy nodes, no allocation once the tables B.tab are given).
template <typename R>
void apply_op(eofa_ctx* ctx, int op, double mp, double mm, const cd* in, cd* out, const ApplyBufs<R>& B) {
    const int Ns = ctx->Ns;
    const size_t nh = ctx->nh;
    auto tab = [&](SiteKind k) { return B.tab[k] ? B.tab[k] : site_tab(ctx, k, mp, mm); };
    for (int par = 0; par < 2; par++) HIPCHK(launch_pack5<R>(in, B.in[par], ctx->g, par, Ns, 0, ctx->st));
    switch (op) {
    case EOFA_OP_DW:
    case EOFA_OP_HOP:
    case EOFA_OP_DT:
    case EOFA_OP_DT_DAG:
    case EOFA_OP_HT: {
        const bool dag = (op == EOFA_OP_DT_DAG);
        const SiteOp* M = tab(dag ? SK_M_DAG : SK_M);
        for (int par = 0; par < 2; par++) {
            auto a = hop_args<R>(ctx, par);
            a.in = B.in[1 - par]; a.self = B.in[par]; a.out = B.out[par]; a.opA = M; a.cz = 1; a.caux = 0;
            int mode = (op == EOFA_OP_DW) ? HM_DW : (op == EOFA_OP_HOP ? HM_LIN : HM_DT);
            hop<R>(ctx, dag, mode, false, a);
        }
        break;
    }
    case EOFA_OP_AT_INV: {
        const SiteOp* Ai = tab(SK_AINV);
        for (int par = 0; par < 2; par++) HIPCHK(launch_site<R>(Ns, false, B.in[par], B.out[par], Ai, ctx->g.Vh, ctx->st));
        break;
    }
    case EOFA_OP_DODWF: {  // D_odwf in = A in - (1/2) H omega (1 + L) in
        const SiteOp* A = tab(SK_A);
        const SiteOp* W = tab(SK_OM1L);
        cpx<R>* v[2] = {B.u, B.w};
        cpx<R>* a[2] = {B.wt, B.at};
        for (int par = 0; par < 2; par++) {
            HIPCHK(launch_site<R>(Ns, false, B.in[par], v[par], W, ctx->g.Vh, ctx->st));
            HIPCHK(launch_site<R>(Ns, false, B.in[par], a[par], A, ctx->g.Vh, ctx->st));
        }
        for (int par = 0; par < 2; par++) {
            auto h = hop_args<R>(ctx, par);
            h.in = v[1 - par]; h.out = B.out[par]; h.aux = a[par]; h.caux = 1; h.cz = (R)-0.5;
            hop<R>(ctx, false, HM_LIN, false, h);
        }
        break;
    }
    case EOFA_OP_DODWF_DAG: {  // D_odwf^dag in = A^dag in - (1/2) (1 + L)^dag omega gamma_5 H gamma_5 in
        const SiteOp* Ad = tab(SK_A_DAG);
        const SiteOp* Wd = tab(SK_OM1L_DAG);
        cpx<R>* t[2] = {B.u, B.w};
        for (int par = 0; par < 2; par++) {
            auto h = hop_args<R>(ctx, par);
            h.in = B.in[1 - par]; h.out = t[par]; h.opA = Wd; h.cz = (R)-0.5; h.caux = 0;
            hop<R>(ctx, true, HM_SITE, false, h);
        }
        for (int par = 0; par < 2; par++) {
            HIPCHK(launch_site<R>(Ns, true, B.in[par], B.out[par], Ad, ctx->g.Vh, ctx->st));
            HIPCHK(launch_axpby<R>((R)1, t[par], (R)1, B.out[par], nh, nullptr, ctx->st));
        }
        break;
    }
    case EOFA_OP_HOP_EO:
    case EOFA_OP_HOP_OE: {  // the hop into one parity from the other; the input's own parity is not read
        const int par = op == EOFA_OP_HOP_EO ? 0 : 1;
        auto h = hop_args<R>(ctx, par);
        h.in = B.in[1 - par]; h.out = B.out[par]; h.cz = 1; h.caux = 0;
        hop<R>(ctx, false, HM_LIN, false, h);
        HIPCHK(launch_fill0(B.out[1 - par], nh * sizeof(cpx<R>), ctx->st));
        break;
    }
    default: {  // SCHUR, SCHUR_DAG, SCHUR_NORMAL
        const SiteOp* Ai = tab(SK_AINV);
        const SiteOp* Ad = tab(SK_AINV_DAG);
        HIPCHK(launch_fill0(B.out[0], nh * sizeof(cpx<R>), ctx->st));
        const cpx<R>* src = B.in[1];
        if (op != EOFA_OP_SCHUR_DAG) {
            auto a = hop_args<R>(ctx, 0);
            a.in = src; a.out = B.u; a.opA = Ai; a.cz = 1; a.caux = 0;
            hop<R>(ctx, false, HM_SITE, false, a);
            auto b = hop_args<R>(ctx, 1);
            b.in = B.u; b.out = B.w; b.out2 = B.wt; b.aux = src; b.opA = Ai; b.opB = Ad; b.cz = (R)-0.25; b.caux = 1;
            b.red = red_of(ctx, SC_TMP + 7, EPI_STORE);
            if (B.partials) { b.red.partials = B.partials; b.red.scal = B.scal; }
            hop<R>(ctx, false, HM_SCHUR_W, true, b);
            if (op == EOFA_OP_SCHUR) {
                HIPCHK(launch_copy(B.out[1], B.w, nh * sizeof(cpx<R>), ctx->st));
                break;
            }
            src = B.w;
        } else {
            HIPCHK(launch_site<R>(Ns, true, src, B.wt, Ad, ctx->g.Vh, ctx->st));
        }
        auto c = hop_args<R>(ctx, 0);
        c.in = B.wt; c.out = B.at; c.opA = Ad; c.cz = 1; c.caux = 0;
        hop<R>(ctx, true, HM_SITE, false, c);
        auto d = hop_args<R>(ctx, 1);
        d.in = B.at; d.out = B.out[1]; d.aux = src; d.caux = 1; d.cz = (R)-0.25;
        hop<R>(ctx, true, HM_LIN, false, d);
    }
    }
    // H_T = gamma_5 R5 D_T reflects in s and flips the lower spins on the way out
    for (int par = 0; par < 2; par++)
        HIPCHK(launch_unpack5<R>(B.out[par], out, ctx->g, par, Ns, op == EOFA_OP_HT ? 1 : 0, ctx->st));
}

void check_apply(eofa_ctx* ctx, int op, const void* in, const void* out, int prec) {
    REQUIRE(ctx->gauge, EOFA_ESTATE, "no gauge field set");
    REQUIRE(in && out && in != out, EOFA_EINVAL, "bad field pointers");
    REQUIRE(prec == EOFA_FP64 || prec == EOFA_MIXED_FP32, EOFA_EINVAL, "prec must be EOFA_FP64 or EOFA_MIXED_FP32");
    REQUIRE(op >= EOFA_OP_DW && op <= EOFA_OP_HOP_OE, EOFA_EINVAL, "unknown op");
}

// the site-operator tables apply_op reads for op
std::vector<SiteKind> op_kinds(int op) {
    switch (op) {
    case EOFA_OP_DT_DAG: return {SK_M_DAG};
    case EOFA_OP_AT_INV: return {SK_AINV};
    case EOFA_OP_SCHUR: case EOFA_OP_SCHUR_DAG: case EOFA_OP_SCHUR_NORMAL: return {SK_AINV, SK_AINV_DAG};
    case EOFA_OP_DODWF: return {SK_A, SK_OM1L};
    case EOFA_OP_DODWF_DAG: return {SK_A_DAG, SK_OM1L_DAG};
    case EOFA_OP_HOP_EO: case EOFA_OP_HOP_OE: return {};
    default: return {SK_M};  // DW, HOP, DT, HT
    }
}

// Pack the canonical links U into the per-parity FP64 and FP32 hop layouts (stream-ordered, no sync).
void pack_gauge(eofa_ctx* ctx, const cd* U) {
    const size_t n = (size_t)ctx->g.Vh * 36;
    for (int par = 0; par < 2; par++) {
        if (!ctx->U[par]) HIPCHK(hipMalloc(&ctx->U[par], n * sizeof(cd)));
        if (!ctx->Uf[par]) HIPCHK(hipMalloc(&ctx->Uf[par], n * sizeof(cpx<float>)));
        HIPCHK(launch_pack_links<double>(U, ctx->U[par], ctx->g, par, (double)ctx->tbc, ctx->st));
        HIPCHK(launch_pack_links<float>(U, ctx->Uf[par], ctx->g, par, (double)ctx->tbc, ctx->st));
    }
    ctx->gauge = true;
}

// Solve and force of one chiral action into force[mu][site][8] (both parities' links).
// x0 (optional): start vector of the solve (internal halves); xsave (optional): receives the solution.
eofa_status chiral_force_impl(eofa_ctx* ctx, int chir, double m3, double m4, double mo, const void* phi,
                              double* force, double* S, const eofa_solve_params* params, eofa_solve_info* info,
                              cd* const* x0 = nullptr, cd* const* xsave = nullptr) {
    check_params(ctx, params);
    REQUIRE(ctx->gauge, EOFA_ESTATE, "no gauge field set");
    ensure_ws(ctx, needed_bytes(ctx, params));
    Work64 W = carve64(ctx);
    // the 4D output of the action is not needed: a workspace field (written after the solve) takes it
    eofa_status st = chiral_impl(ctx, chir, m3, m4, mo, phi, (void*)W.res.h[0], 0, S, params, info, x0);
    if (st != EOFA_OK && st != EOFA_ENOCONV) return st;
    const double kappa = chir * action_k(chir, m3, m4, mo);
    for (int par = 0; par < 2; par++)
        HIPCHK(launch_force(W.x.h[par], W.x.h[1 - par], ctx->U[par], ctx->g, par, ctx->Ns, kappa, force, ctx->st));
    if (xsave)
        for (int par = 0; par < 2; par++) HIPCHK(launch_copy(xsave[par], W.x.h[par], ctx->nh * sizeof(cd), ctx->st));
    return st;
}

// Doubles of a momentum or force field: 4 directions x V sites x 8 components (V = 2 Vh).
size_t md_len(const eofa_ctx* ctx) { return 4 * 8 * 2 * (size_t)ctx->g.Vh; }

// S_g = beta sum (1 - Re Tr U_P / 3) of the canonical links U.
double gauge_action_dev(eofa_ctx* ctx, const cd* U, double beta) {
    const Red red = red_of(ctx, SC_TMP + 17, EPI_STORE);
    HIPCHK(launch_plaquette(U, ctx->g, red, ctx->st));
    HIPCHK(launch_finish(red, (unsigned)((2 * (size_t)ctx->g.Vh + 255) / 256), ctx->st));
    sync_scal(ctx);
    return beta * ctx->hscal[SC_TMP + 17];
}

// 1/2 sum P^a P^a over the 32 V momentum components.
double kinetic_dev(eofa_ctx* ctx, const double* P) {
    HIPCHK(launch_norm2<double>((const cd*)P, md_len(ctx) / 2, red_of(ctx, SC_TMP + 18, EPI_STORE), ctx->st));
    sync_scal(ctx);
    return 0.5 * ctx->hscal[SC_TMP + 18];
}

// The nested Omelyan integration of the molecular dynamics (see eofa_md_trajectory).
struct MdRun {
    eofa_ctx* ctx;
    cd* U;
    double* P;
    int nact;
    const eofa_md_action* acts;
    const eofa_md_params* md;
    const eofa_solve_params* sp;
    eofa_md_info* info;
    eofa_status st = EOFA_OK;
    // Momentum updates are deferred until the links change: the kicks of one level between two link updates
    // see the same links, so their force is evaluated once with the summed step (pend[level]); kicks of
    // different levels commute.  Every level has a pending kick at the start and at the end of the trajectory,
    // so those two flushes also give every action's S (Sf_flush, with `all` set when each action was solved).
    double pend[4] = {0, 0, 0, 0};
    bool has[4] = {false, false, false, false};
    double Sf_flush = 0;
    bool all = false;
    bool sf0 = false;  // info->Sf0 was taken from the first flush
    // chronological start vectors: the last solution of each action in this trajectory (md->chrono)
    std::vector<bool> have;
    // force magnitudes: action i's k-th evaluation goes to md_fn[off[i] + k]
    std::vector<size_t> off;
    std::vector<int> nev;
};

constexpr double kOmelyanLambda = 0.1931833275037836;

void md_kick(MdRun& m, int level, double h) {
    m.pend[level] += h;
    m.has[level] = true;
}

// Apply every pending kick at the current links.  last: the flush at the end of the trajectory.
void md_flush(MdRun& m, bool last = false) {
    eofa_ctx* ctx = m.ctx;
    m.Sf_flush = 0;
    int solved = 0;
    // the first and the last evaluations also give the actions in H: they keep the solve's tolerance
    eofa_solve_params fp = *m.sp;
    if (m.md->force_tol > 0 && m.info->link_updates > 0 && !last) fp.tol = m.md->force_tol;
    for (int level = 0; level < m.md->nlevels; level++) {
        if (!m.has[level]) continue;
        const double h = m.pend[level];
        m.pend[level] = 0;
        m.has[level] = false;
        m.info->force_evals[level]++;
        if (level == 0) {
            HIPCHK(launch_gauge_force(m.U, ctx->g, m.md->beta, nullptr, m.P, h, 1, ctx->st));
            continue;
        }
        for (int i = 0; i < m.nact; i++) {
            const eofa_md_action& a = m.acts[i];
            if (a.level != level) continue;
            eofa_solve_info si{};
            double S = 0;
            cd* const* g = m.md->chrono ? &ctx->md_guess[2 * i] : nullptr;
            const eofa_status st = chiral_force_impl(ctx, a.chir, a.m3, a.m4, a.mo, a.phi, ctx->md_F, &S, &fp, &si,
                                                     g && m.have[i] ? g : nullptr, g);
            if (g) m.have[i] = true;
            m.info->cg_iters += si.iters;
            if (st != EOFA_OK) {
                m.st = st;
                throw Fail{st};
            }
            m.Sf_flush += S;
            solved++;
            if (i < (int)m.nev.size() && m.nev[i] < (int)(m.off[i + 1] - m.off[i])) {
                const Red red{ctx->partials, ctx->md_fn, (int)(m.off[i] + m.nev[i]++), EPI_STORE};
                const size_t nl = md_len(ctx) / 8;
                HIPCHK(launch_link_norms(ctx->md_F, nl, red, ctx->st));
                HIPCHK(launch_finish(red, (unsigned)((nl + 255) / 256), ctx->st));
            }
            HIPCHK(launch_kick(m.P, ctx->md_F, h, md_len(ctx), ctx->st));
        }
    }
    m.all = (solved == m.nact);
}

void md_links(MdRun& m, double h) {
    eofa_ctx* ctx = m.ctx;
    md_flush(m);
    if (m.info->link_updates == 0 && m.all) {  // the first flush: every action at U(0)
        m.info->Sf0 = m.Sf_flush;
        m.sf0 = true;
    }
    HIPCHK(launch_link_update(m.U, m.P, h, ctx->g, ctx->st));
    pack_gauge(ctx, m.U);
    m.info->link_updates++;
}

void md_integrate(MdRun& m, int level, double tau) {
    const int top = m.md->nlevels - 1;
    const int n = level == top ? m.md->steps[level] : m.md->steps[level] / (2 * m.md->steps[level + 1]);
    const double e = tau / n, lam = kOmelyanLambda;
    auto inner = [&](double h) {
        if (level == 0) md_links(m, h);
        else md_integrate(m, level - 1, h);
    };
    for (int k = 0; k < n; k++) {
        md_kick(m, level, lam * e);
        inner(e / 2);
        md_kick(m, level, (1 - 2 * lam) * e);
        inner(e / 2);
        md_kick(m, level, lam * e);
    }
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

eofa_status eofa_create(eofa_ctx** out, const int dims[4], int Ns, double m0, const double* omega_host, int t_bc,
                        void* hip_stream) {
    if (!out) return EOFA_EINVAL;
    *out = nullptr;
    eofa_ctx* ctx = new (std::nothrow) eofa_ctx();
    if (!ctx) return EOFA_ENOMEM;
    eofa_status st = guarded(ctx, [&]() -> eofa_status {
        REQUIRE(dims && omega_host, EOFA_EINVAL, "null dims or omega");
        long V = 1;
        for (int i = 0; i < 4; i++) {
            REQUIRE(dims[i] >= 2 && dims[i] % 2 == 0, EOFA_EINVAL, "every lattice extent must be even and >= 2");
            ctx->L[i] = dims[i];
            V *= dims[i];
        }
        REQUIRE(V / 2 < (1L << 31) / 64, EOFA_EINVAL, "lattice too large");
        REQUIRE(Ns == 4 || Ns == 8 || Ns == 16 || Ns == 32, EOFA_EINVAL, "Ns must be 4, 8, 16 or 32");
        REQUIRE(m0 > 0 && m0 < 2, EOFA_EINVAL, "m0 must be in (0, 2)");
        REQUIRE(t_bc == 1 || t_bc == -1, EOFA_EINVAL, "t_bc must be +1 or -1");
        for (int s = 0; s < Ns; s++) {
            REQUIRE(std::isfinite(omega_host[s]) && omega_host[s] > 0, EOFA_EINVAL, "omega_s must be positive");
            double o2 = omega_host[Ns - 1 - s];
            REQUIRE(std::fabs(omega_host[s] - o2) <= 1e-14 * std::fabs(omega_host[s]), EOFA_EINVAL,
                    "omega must be R5-symmetric");
        }
        ctx->Ns = Ns;
        ctx->m0 = m0;
        ctx->tbc = t_bc;
        ctx->omega.assign(omega_host, omega_host + Ns);
        ctx->st = (hipStream_t)hip_stream;
        HIPCHK(hipGetDevice(&ctx->dev));
        {   // the static scratch of eofa_apply_static; a failure here only disables that entry point
            const hipError_t e = scratch_addr(ctx->dev, &ctx->scratch);
            if (e != hipSuccess) {
                ctx->scratch = nullptr;
                ctx->scratch_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            }
        }
        ctx->g = Geom{dims[0], dims[1], dims[2], dims[3], dims[0] / 2, (int)(V / 2)};
        ctx->nh = (size_t)(V / 2) * 12 * Ns;
        // one partial per block: hop kernels use <= nh / 256 blocks, grid-stride reductions <= 4096
        const size_t maxblk = (ctx->nh + 255) / 256 + 4096;
        HIPCHK(hipMalloc(&ctx->partials, sizeof(double) * maxblk));
        HIPCHK(hipMalloc(&ctx->scal, sizeof(double) * SCAL_TOTAL));
        HIPCHK(hipMemset(ctx->scal, 0, sizeof(double) * SCAL_TOTAL));
        HIPCHK(hipHostMalloc(&ctx->hscal, sizeof(double) * SCAL_TOTAL, hipHostMallocDefault));
        return EOFA_OK;
    });
    if (st != EOFA_OK) {
        std::fprintf(stderr, "eofa_create: %s\n", ctx->err.c_str());
        eofa_destroy(ctx);
        return st;
    }
    *out = ctx;
    return EOFA_OK;
}

eofa_status eofa_workspace_size(const eofa_ctx* cctx, const eofa_solve_params* params, int nrhs, size_t* bytes) {
    if (!cctx || !bytes || nrhs < 1) return EOFA_EINVAL;
    *bytes = needed_bytes(cctx, params, nrhs);
    return EOFA_OK;
}

eofa_status eofa_set_workspace(eofa_ctx* ctx, void* dev_ptr, size_t bytes) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(((uintptr_t)dev_ptr % kAlign) == 0, EOFA_EINVAL, "workspace must be 256-byte aligned");
        if (ctx->ws && ctx->ws_owned) HIPCHK(hipFree(ctx->ws));
        ctx->ws = (char*)dev_ptr;
        ctx->ws_bytes = dev_ptr ? bytes : 0;
        ctx->ws_owned = false;
        return EOFA_OK;
    });
}

eofa_status eofa_set_gauge(eofa_ctx* ctx, const void* U) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(U != nullptr, EOFA_EINVAL, "U is NULL");
        pack_gauge(ctx, (const cd*)U);
        HIPCHK(hipStreamSynchronize(ctx->st));
        return EOFA_OK;
    });
}

eofa_status eofa_chiral_action(eofa_ctx* ctx, int chir, double m3, double m4, double mo, const void* phi, void* out,
                               double* S, const eofa_solve_params* params, eofa_solve_info* info) {
    return guarded(ctx, [&]() { return chiral_impl(ctx, chir, m3, m4, mo, phi, out, 0, S, params, info); });
}

eofa_status eofa_chiral_force(eofa_ctx* ctx, int chir, double m3, double m4, double mo, const void* phi, double* force,
                              double* S, const eofa_solve_params* params, eofa_solve_info* info) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(force, EOFA_EINVAL, "null force pointer");
        const eofa_status st = chiral_force_impl(ctx, chir, m3, m4, mo, phi, force, S, params, info);
        HIPCHK(hipStreamSynchronize(ctx->st));
        return st;
    });
}

eofa_status eofa_gauge_action(eofa_ctx* ctx, const void* U, double beta, double* S) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(U && S, EOFA_EINVAL, "null pointer");
        *S = gauge_action_dev(ctx, (const cd*)U, beta);
        return EOFA_OK;
    });
}

eofa_status eofa_gauge_force(eofa_ctx* ctx, const void* U, double beta, double* force) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(U && force, EOFA_EINVAL, "null pointer");
        HIPCHK(launch_gauge_force((const cd*)U, ctx->g, beta, force, nullptr, 0.0, 0, ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));
        return EOFA_OK;
    });
}

eofa_status eofa_md_trajectory(eofa_ctx* ctx, void* U, double* P, int nact, const eofa_md_action* acts,
                               const eofa_md_params* md, const eofa_solve_params* solve, eofa_md_info* info) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(U && P && md && solve && info, EOFA_EINVAL, "null pointer");
        REQUIRE(nact >= 0 && (nact == 0 || acts), EOFA_EINVAL, "bad action list");
        REQUIRE(md->nlevels >= 1 && md->nlevels <= 4, EOFA_EINVAL, "nlevels must be 1 .. 4");
        REQUIRE(md->tau > 0 && std::isfinite(md->tau) && std::isfinite(md->beta), EOFA_EINVAL, "bad tau or beta");
        REQUIRE(md->metropolis_u < 1.0, EOFA_EINVAL, "metropolis_u must be < 1");
        REQUIRE(md->force_tol >= 0 && md->force_tol < 1 && std::isfinite(md->force_tol), EOFA_EINVAL,
                "force_tol must lie in [0, 1)");
        for (int j = 0; j < md->nlevels; j++) REQUIRE(md->steps[j] >= 1, EOFA_EINVAL, "steps must be >= 1");
        for (int j = 1; j < md->nlevels; j++)
            REQUIRE(md->steps[j - 1] % (2 * md->steps[j]) == 0, EOFA_EINVAL,
                    "steps[j - 1] must be a multiple of 2 steps[j]");
        // every link update is a kernel plus a repack: bound the work of one call
        REQUIRE((long)md->steps[0] <= 100000, EOFA_EINVAL, "too many steps");
        for (int i = 0; i < nact; i++) {
            REQUIRE(acts[i].level >= 1 && acts[i].level < md->nlevels, EOFA_EINVAL, "action level out of range");
            REQUIRE(acts[i].phi, EOFA_EINVAL, "null phi");
        }
        check_params(ctx, solve);
        const auto t0 = std::chrono::steady_clock::now();
        *info = eofa_md_info{};
        info->accepted = -1;
        const size_t nU = 72 * (size_t)ctx->g.Vh;  // complex entries of the canonical links
        if (!ctx->md_F) HIPCHK(hipMalloc(&ctx->md_F, sizeof(double) * md_len(ctx)));
        if (!ctx->md_U0) HIPCHK(hipMalloc(&ctx->md_U0, sizeof(cd) * nU));
        if (md->chrono)
            while ((int)ctx->md_guess.size() < 2 * nact) {
                cd* q = nullptr;
                HIPCHK(hipMalloc(&q, ctx->nh * sizeof(cd)));
                ctx->md_guess.push_back(q);
            }
        MdRun m{ctx, (cd*)U, P, nact, acts, md, solve, info};
        m.have.assign(nact, false);
        {   // one slot per force evaluation of each reported action (2 steps[level] + 1 of them)
            const int nrep = nact < 8 ? nact : 8;
            m.off.assign(nrep + 1, 0);
            m.nev.assign(nrep, 0);
            for (int i = 0; i < nrep; i++) m.off[i + 1] = m.off[i] + 2 * (size_t)md->steps[acts[i].level] + 1;
            if (m.off[nrep] > ctx->md_fn_len) {
                if (ctx->md_fn) HIPCHK(hipFree(ctx->md_fn));
                ctx->md_fn = nullptr;
                ctx->md_fn_len = 0;
                HIPCHK(hipMalloc(&ctx->md_fn, sizeof(double) * m.off[nrep]));
                ctx->md_fn_len = m.off[nrep];
            }
        }
        HIPCHK(launch_copy(ctx->md_U0, U, sizeof(cd) * nU, ctx->st));
        pack_gauge(ctx, (const cd*)U);
        info->K0 = kinetic_dev(ctx, P);
        info->Sg0 = gauge_action_dev(ctx, (const cd*)U, md->beta);
        {   // the gauge force at the start, averaged over the links
            const size_t nl = md_len(ctx) / 8;
            const Red red = red_of(ctx, SC_TMP + 19, EPI_STORE);
            HIPCHK(launch_gauge_force((const cd*)U, ctx->g, md->beta, ctx->md_F, nullptr, 0.0, 0, ctx->st));
            HIPCHK(launch_link_norms(ctx->md_F, nl, red, ctx->st));
            HIPCHK(launch_finish(red, (unsigned)((nl + 255) / 256), ctx->st));
            sync_scal(ctx);
            info->gauge_force0 = ctx->hscal[SC_TMP + 19] / (double)nl;
        }
        try {
            md_integrate(m, md->nlevels - 1, md->tau);
            md_flush(m, true);  // the last kicks, at U(tau)
        } catch (const Fail&) {  // a solve failed: hand back the starting links (P holds the partial update)
            const std::string why = ctx->err;
            HIPCHK(launch_copy(U, ctx->md_U0, sizeof(cd) * nU, ctx->st));
            pack_gauge(ctx, (const cd*)U);
            HIPCHK(hipStreamSynchronize(ctx->st));
            ctx->err = why;
            throw;
        }
        // every level kicks before the first link update and after the last one, so both flushes solved every
        // action; anything else is a defect of the integrator
        REQUIRE(m.sf0 && m.all, EOFA_EHIP, "internal: the end flushes did not evaluate every action");
        info->Sf1 = m.Sf_flush;
        if (!m.nev.empty()) {
            std::vector<double> fn(m.off.back());
            HIPCHK(hipMemcpyAsync(fn.data(), ctx->md_fn, sizeof(double) * fn.size(), hipMemcpyDeviceToHost, ctx->st));
            HIPCHK(hipStreamSynchronize(ctx->st));
            const double nl = (double)(md_len(ctx) / 8);
            for (size_t i = 0; i < m.nev.size(); i++) {
                double mx = 0, sum = 0;
                for (int k = 0; k < m.nev[i]; k++) {
                    const double v = fn[m.off[i] + k] / nl;
                    mx = std::max(mx, v);
                    sum += v;
                }
                info->force_max[i] = mx;
                info->force_mean[i] = m.nev[i] ? sum / m.nev[i] : 0.0;
            }
        }
        info->K1 = kinetic_dev(ctx, P);
        info->Sg1 = gauge_action_dev(ctx, (const cd*)U, md->beta);
        info->H0 = info->K0 + info->Sg0 + info->Sf0;
        info->H1 = info->K1 + info->Sg1 + info->Sf1;
        info->dH = info->H1 - info->H0;
        if (md->metropolis_u >= 0) {
            info->accepted = (md->metropolis_u < std::exp(-info->dH)) ? 1 : 0;
            if (!info->accepted) {
                HIPCHK(launch_copy(U, ctx->md_U0, sizeof(cd) * nU, ctx->st));
                pack_gauge(ctx, (const cd*)U);
            }
        }
        HIPCHK(hipStreamSynchronize(ctx->st));
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return EOFA_OK;
    });
}

eofa_status eofa_hinv(eofa_ctx* ctx, double m_lo, double m_hi, const void* phi, void* out, double* S,
                      const eofa_solve_params* params, eofa_solve_info info[2]) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(m_lo > 0 && m_lo <= m_hi && m_hi <= 1, EOFA_EINVAL, "need 0 < m_lo <= m_hi <= 1");
        double s1 = 0, s2 = 0;
        eofa_status a = chiral_impl(ctx, -1, m_lo, m_lo, m_hi, phi, out, 0, &s1, params, info ? &info[0] : nullptr);
        if (a != EOFA_OK && a != EOFA_ENOCONV) return a;
        eofa_status b = chiral_impl(ctx, +1, m_lo, m_hi, m_hi, phi, out, 1, &s2, params, info ? &info[1] : nullptr);
        if (S) *S = s1 + s2;
        if (b != EOFA_OK) return b;
        return a;
    });
}

eofa_status eofa_chiral_action_batch(eofa_ctx* ctx, int n, const int* chir, const double* m3, const double* m4,
                                     const double* mo, const void* const* phi, void* const* out, double* S,
                                     const eofa_solve_params* params, eofa_solve_info* info) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(n >= 0 && chir && m3 && m4 && mo && phi && out, EOFA_EINVAL, "bad batch arguments");
        return chiral_batch_impl(ctx, n, chir, m3, m4, mo, phi, out, nullptr, S, params, info);
    });
}

eofa_status eofa_hinv_batch(eofa_ctx* ctx, int n, const double* m_lo, const double* m_hi, const void* const* phi,
                            void* const* out, double* S, const eofa_solve_params* params, eofa_solve_info* info) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(n >= 0 && m_lo && m_hi && phi && out, EOFA_EINVAL, "bad batch arguments");
        std::vector<int> chir(2 * n), acc(2 * n);
        std::vector<double> a3(2 * n), a4(2 * n), ao(2 * n), s2(2 * n);
        std::vector<const void*> f(2 * n);
        std::vector<void*> o(2 * n);
        for (int j = 0; j < n; j++) {
            REQUIRE(m_lo[j] > 0 && m_lo[j] <= m_hi[j] && m_hi[j] <= 1, EOFA_EINVAL, "need 0 < m_lo <= m_hi <= 1");
            // - action (m_lo,m_lo)/(m_lo,m_hi) writes out, then + action (m_lo,m_hi)/(m_hi,m_hi) adds to it
            chir[2 * j] = -1; a3[2 * j] = m_lo[j]; a4[2 * j] = m_lo[j]; ao[2 * j] = m_hi[j]; acc[2 * j] = 0;
            chir[2 * j + 1] = +1; a3[2 * j + 1] = m_lo[j]; a4[2 * j + 1] = m_hi[j]; ao[2 * j + 1] = m_hi[j]; acc[2 * j + 1] = 1;
            f[2 * j] = f[2 * j + 1] = phi[j];
            o[2 * j] = o[2 * j + 1] = out[j];
        }
        eofa_status st = chiral_batch_impl(ctx, 2 * n, chir.data(), a3.data(), a4.data(), ao.data(), f.data(), o.data(),
                                           acc.data(), s2.data(), params, info);
        if (S)
            for (int j = 0; j < n; j++) S[j] = s2[2 * j] + s2[2 * j + 1];
        return st;
    });
}

eofa_status eofa_solve_ht(eofa_ctx* ctx, double m_plus, double m_minus, const void* b5, void* x5,
                          const eofa_solve_params* params, eofa_solve_info* info) {
    return guarded(ctx, [&]() { return solve_ht_impl(ctx, m_plus, m_minus, b5, x5, params, info); });
}

eofa_status eofa_solve_ht_batch(eofa_ctx* ctx, int n, const double* m_plus, const double* m_minus,
                                const void* const* b5, void* const* x5, const eofa_solve_params* params,
                                eofa_solve_info* info) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(n >= 0 && m_plus && m_minus && b5 && x5, EOFA_EINVAL, "bad batch arguments");
        check_params(ctx, params);
        for (int j = 0; j < n; j++) {
            REQUIRE(b5[j] && x5[j] && b5[j] != x5[j], EOFA_EINVAL, "bad field pointers");
            REQUIRE(m_plus[j] > 0 && m_plus[j] <= 1 && m_minus[j] > 0 && m_minus[j] <= 1, EOFA_EINVAL,
                    "masses must lie in (0, 1]");
        }
        if (!use_batch(ctx, n, params)) {
            eofa_status worst = EOFA_OK;
            for (int j = 0; j < n; j++) {
                eofa_status a = solve_ht_impl(ctx, m_plus[j], m_minus[j], b5[j], x5[j], params, info ? &info[j] : nullptr);
                if (a != EOFA_OK && a != EOFA_ENOCONV) return a;
                if (a != EOFA_OK) worst = a;
            }
            return worst;
        }
        const eofa_status st = batch_solve(
            ctx, n, m_plus, m_minus, params, info,
            [&](const Work64& W, int j) {
                for (int par = 0; par < 2; par++)
                    HIPCHK(launch_pack5<double>((const cd*)b5[j], W.c.h[par], ctx->g, par, ctx->Ns, 1, ctx->st));
            },
            [&](const Work64& W, int j, const SolveOut&) {
                for (int par = 0; par < 2; par++)
                    HIPCHK(launch_unpack5<double>(W.x.h[par], (cd*)x5[j], ctx->g, par, ctx->Ns, 0, ctx->st));
            });
        HIPCHK(hipStreamSynchronize(ctx->st));
        return st;
    });
}

eofa_status eofa_apply(eofa_ctx* ctx, int op, double m_plus, double m_minus, const void* in, void* out,
                       eofa_precision prec) {
    return guarded(ctx, [&]() -> eofa_status {
        check_apply(ctx, op, in, out, prec);
        eofa_solve_params P{1e-10, 1, prec, EOFA_PC_NONE, 0, 0, 0};
        ensure_ws(ctx, needed_bytes(ctx, &P));
        if (prec == EOFA_FP64) {
            Work64 W = carve64(ctx);
            ApplyBufs<double> B{{W.x.h[0], W.x.h[1]}, {W.res.h[0], W.res.h[1]}, W.u, W.w, W.wt, W.at, {}, nullptr, nullptr};
            apply_op<double>(ctx, op, m_plus, m_minus, (const cd*)in, (cd*)out, B);
        } else {
            Work32 F = carve32(ctx);
            ApplyBufs<float> B{{F.x, F.r}, {F.e0, F.e1}, F.u, F.w, F.wt, F.at, {}, nullptr, nullptr};
            apply_op<float>(ctx, op, m_plus, m_minus, (const cd*)in, (cd*)out, B);
        }
        HIPCHK(hipStreamSynchronize(ctx->st));
        return EOFA_OK;
    });
}

eofa_status eofa_apply_static(eofa_ctx* ctx, int op, double m_plus, double m_minus, const void* in, void* out,
                              eofa_precision prec) {
    return guarded(ctx, [&]() -> eofa_status {
        check_apply(ctx, op, in, out, prec);
        REQUIRE(ctx->scratch != nullptr, EOFA_ESTATE, "static scratch unavailable on this device: " + ctx->scratch_err);
        const size_t rs = prec == EOFA_FP64 ? sizeof(cd) : sizeof(cpx<float>);
        const size_t hb = align_up(ctx->nh * rs);
        const size_t tb = align_up(sizeof(SiteOp));
        const size_t nblocks = (ctx->nh + 255) / 256 + 4096;  // as the context's partials: >= any hop grid
        const size_t pb = align_up(nblocks * sizeof(double)), sb = align_up(SC_N * sizeof(double));
        const size_t need = 8 * hb + 4 * tb + pb + sb;
        REQUIRE(need <= kStaticScratchBytes, EOFA_EINVAL,
                "eofa_apply_static: this lattice needs " + std::to_string(need) + " bytes of scratch, more than the "
                "static " + std::to_string(kStaticScratchBytes) + " (use eofa_apply)");
        char* q = (char*)ctx->scratch;
        auto take = [&](size_t n) { char* r = q; q += n; return r; };
        void* h[8];
        for (void*& v : h) v = take(hb);
        // the site-operator tables this op reads (at most 4), built on the host and written by kernels
        ApplyBufs<double> B64{};
        ApplyBufs<float> B32{};
        const std::vector<SiteKind> kinds = op_kinds(op);
        for (size_t i = 0; i < 4; i++) {
            double* d = (double*)take(tb);
            if (i >= kinds.size()) continue;
            SiteOp host;
            build_site_op(host, kinds[i], ctx->Ns, ctx->m0, ctx->omega.data(), m_plus, m_minus);
            HIPCHK(launch_set_block(d, sizeof(SiteOp) / sizeof(double), (const double*)&host, ctx->st));
            B64.tab[kinds[i]] = B32.tab[kinds[i]] = (const SiteOp*)d;
        }
        double* partials = (double*)take(pb);
        double* scal = (double*)take(sb);
        if (prec == EOFA_FP64) {
            ApplyBufs<double>& B = B64;
            B.in[0] = (cd*)h[0]; B.in[1] = (cd*)h[1]; B.out[0] = (cd*)h[2]; B.out[1] = (cd*)h[3];
            B.u = (cd*)h[4]; B.w = (cd*)h[5]; B.wt = (cd*)h[6]; B.at = (cd*)h[7];
            B.partials = partials; B.scal = scal;
            apply_op<double>(ctx, op, m_plus, m_minus, (const cd*)in, (cd*)out, B);
        } else {
            using cf = cpx<float>;
            ApplyBufs<float>& B = B32;
            B.in[0] = (cf*)h[0]; B.in[1] = (cf*)h[1]; B.out[0] = (cf*)h[2]; B.out[1] = (cf*)h[3];
            B.u = (cf*)h[4]; B.w = (cf*)h[5]; B.wt = (cf*)h[6]; B.at = (cf*)h[7];
            B.partials = partials; B.scal = scal;
            apply_op<float>(ctx, op, m_plus, m_minus, (const cd*)in, (cd*)out, B);
        }
        HIPCHK(hipGetLastError());
        return EOFA_OK;
    });
}

eofa_status eofa_chiral_heatbath(eofa_ctx* ctx, int chir, double m3, double m4, double mo, const void* eta, void* phi,
                                 double lo, double hi, double rel_err, int verify, const eofa_solve_params* params,
                                 eofa_heatbath_info* info) {
    return guarded(ctx, [&]() {
        return heatbath_impl(ctx, chir, m3, m4, mo, eta, phi, lo, hi, rel_err, params, 0, verify, info);
    });
}

eofa_status eofa_heatbath(eofa_ctx* ctx, double m_lo, double m_hi, const void* eta, void* phi, double rel_err,
                          int verify, const eofa_solve_params* params, eofa_heatbath_info info[2]) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(m_lo > 0 && m_lo <= m_hi && m_hi <= 1, EOFA_EINVAL, "need 0 < m_lo <= m_hi <= 1");
        eofa_status a = heatbath_impl(ctx, -1, m_lo, m_lo, m_hi, eta, phi, 0, 0, rel_err, params, 0, verify,
                                      info ? &info[0] : nullptr);
        if (a != EOFA_OK && a != EOFA_ENOCONV) return a;
        eofa_status b = heatbath_impl(ctx, +1, m_lo, m_hi, m_hi, eta, phi, 0, 0, rel_err, params, 1, verify,
                                      info ? &info[1] : nullptr);
        return b != EOFA_OK ? b : a;
    });
}

eofa_status eofa_inv_sqrt_rational(double lo, double hi, int n, double* a0, double* a, double* b, double* err) {
    if (!(lo > 0 && hi > lo) || n < 1 || n > HB_MAXTERMS || !a0 || !a || !b) return EOFA_EINVAL;
    const RatInvSqrt r = zolotarev_inv_sqrt(lo, hi, n);
    *a0 = r.a0;
    for (int l = 0; l < n; l++) { a[l] = r.a[l]; b[l] = r.b[l]; }
    if (err) *err = r.err;
    return EOFA_OK;
}

eofa_status eofa_graph_stats(eofa_ctx* ctx, long* replays, int* cached) {
    return guarded(ctx, [&]() -> eofa_status {
        if (replays) *replays = ctx->graph_replays;
        if (cached) *cached = (int)ctx->graphs.size();
        return EOFA_OK;
    });
}

eofa_status eofa_kernel_timing(eofa_ctx* ctx, int enable, int reset, eofa_kernel_stats* stats) {
    return guarded(ctx, [&]() -> eofa_status {
        collect_timing(ctx);
        if (reset)
            for (int k = 0; k < EOFA_NKERN; k++) { ctx->k_ms[k] = 0; ctx->k_n[k] = 0; ctx->k_bytes[k] = 0; }
        ctx->timing = enable != 0;
        if (stats)
            for (int k = 0; k < EOFA_NKERN; k++) {
                stats->ms[k] = ctx->k_ms[k];
                stats->launches[k] = ctx->k_n[k];
                stats->bytes[k] = ctx->k_bytes[k];
            }
        return EOFA_OK;
    });
}

eofa_status eofa_cg_block(eofa_ctx* ctx, int chir, double m3, double m4, const void* phi, int niter, double* rel) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(ctx->gauge, EOFA_ESTATE, "no gauge field set");
        REQUIRE(niter >= 1, EOFA_EINVAL, "niter must be >= 1");
        REQUIRE(chir == 1 || chir == -1, EOFA_EINVAL, "chir must be +1 or -1");
        REQUIRE(phi != nullptr, EOFA_EINVAL, "null field pointer");
        for (double m : {m3, m4}) REQUIRE(m > 0 && m <= 1, EOFA_EINVAL, "masses must lie in (0, 1]");
        eofa_solve_params P{1e-10, 1, EOFA_FP64, EOFA_PC_NONE, 0, 0, 0};
        ensure_ws(ctx, needed_bytes(ctx, &P));
        Work64 W = carve64(ctx);
        const SiteOp* Ai = site_tab(ctx, SK_AINV, m3, m4);
        const SiteOp* Ad = site_tab(ctx, SK_AINV_DAG, m3, m4);
        make_source(ctx, W, chir, phi);
        prep_schur(ctx, W, Ai, W.bh);
        cg64_init(ctx, W, Ad, 0.0);  // threshold 0: the device never flags convergence
        for (int k = 0; k < niter; k++) cg_iteration<double>(ctx, W.xcg, W.r, W.p, W.u, W.w, W.wt, W.at, Ai, Ad);
        sync_scal(ctx);
        collect_timing(ctx);
        const double rr = ctx->hscal[SC_RR], rr0 = ctx->hscal[SC_RR0];
        REQUIRE(std::isfinite(rr), EOFA_ENOCONV, "CG breakdown (non-finite residual)");
        if (rel) *rel = rr0 > 0 ? std::sqrt(rr / rr0) : 0.0;
        return EOFA_OK;
    });
}

eofa_status eofa_dslash_bench(eofa_ctx* ctx, int prec, int nrep, double* ms, double* alg_bytes) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(ctx->gauge, EOFA_ESTATE, "no gauge field set");
        REQUIRE(nrep > 0 && ms, EOFA_EINVAL, "bad arguments");
        REQUIRE(prec == EOFA_FP64 || prec == EOFA_MIXED_FP32 || (prec == EOFA_MIXED_FP16 && ctx->Ns >= 8),
                EOFA_EINVAL, "prec must be FP64, MIXED_FP32 or MIXED_FP16 (Ns >= 8)");
        eofa_solve_params P{1e-10, 1, (eofa_precision)prec, EOFA_PC_NONE, 0, 0, 0};
        ensure_ws(ctx, needed_bytes(ctx, &P));
        if (prec == EOFA_MIXED_FP16) ensure_partials_mr(ctx);
        fill_bench_buffers(ctx);
        *ms = time_hop(ctx, prec, nrep, ctx->sched[prec]);
        // in + out spinor columns and 8 links per 4D site (FP16 columns: 48 B + a 4-byte norm; FP32 links)
        const double col = (prec == EOFA_FP64) ? 12 * 16.0 : (prec == EOFA_MIXED_FP32 ? 12 * 8.0 : 12 * 4.0 + 4.0);
        const double lk = (prec == EOFA_FP64) ? 16.0 : 8.0;
        if (alg_bytes) *alg_bytes = (double)ctx->g.Vh * (2.0 * ctx->Ns * col + 8 * 9 * lk);
        return EOFA_OK;
    });
}

eofa_status eofa_autotune(eofa_ctx* ctx, int prec, int nrep, int sched_out[7], double* best_ms, double* base_ms) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(ctx->gauge, EOFA_ESTATE, "no gauge field set");
        REQUIRE(prec == EOFA_FP64 || prec == EOFA_MIXED_FP32 || (prec == EOFA_MIXED_FP16 && ctx->Ns >= 8),
                EOFA_EINVAL, "prec must be FP64, MIXED_FP32 or MIXED_FP16 (Ns >= 8)");
        if (nrep <= 0) nrep = 4;
        eofa_solve_params P{1e-10, 1, (eofa_precision)prec, EOFA_PC_NONE, 0, 0, 0};
        ensure_ws(ctx, needed_bytes(ctx, &P));
        if (prec == EOFA_MIXED_FP16) ensure_partials_mr(ctx);
        fill_bench_buffers(ctx);
        const int k = prec;
        std::vector<Sched> cand = sched_candidates(ctx, prec);
        double best = 1e30, base = 0;
        Sched bs = cand[0];
        for (size_t i = 0; i < cand.size(); i++) {
            double t = time_hop(ctx, prec, nrep, cand[i]);
            if (i == 0) base = t;
            if (t < best) { best = t; bs = cand[i]; }
        }
        ctx->sched[k] = bs;
        ctx->tuned_ms[k] = best;
        if (sched_out) {
            sched_out[0] = bs.mode; sched_out[1] = bs.xcd; sched_out[2] = bs.ty;
            sched_out[3] = bs.tz; sched_out[4] = bs.tt; sched_out[5] = bs.nyb; sched_out[6] = bs.ord;
        }
        if (best_ms) *best_ms = best;
        if (base_ms) *base_ms = base;
        return EOFA_OK;
    });
}

eofa_status eofa_set_schedule(eofa_ctx* ctx, int prec, const int sched_in[7]) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(sched_in, EOFA_EINVAL, "null schedule");
        REQUIRE(prec == EOFA_FP64 || prec == EOFA_MIXED_FP32 || prec == EOFA_MIXED_FP16, EOFA_EINVAL,
                "prec must be FP64, MIXED_FP32 or MIXED_FP16");
        Sched s{sched_in[0], sched_in[1], sched_in[2], sched_in[3], sched_in[4], sched_in[5], sched_in[6]};
        bool ok = false;
        for (const Sched& c : sched_candidates(ctx, prec))
            ok |= (c.mode == s.mode && c.xcd == s.xcd && c.ty == s.ty && c.tz == s.tz && c.tt == s.tt &&
                   c.nyb == s.nyb && c.ord == s.ord);
        REQUIRE(ok, EOFA_EINVAL, "schedule not valid for this lattice");
        ctx->sched[prec] = s;
        return EOFA_OK;
    });
}

eofa_status eofa_schedule_candidates(eofa_ctx* ctx, int prec, int max, int* sched_out, int* n) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(n && max >= 0 && (sched_out || max == 0), EOFA_EINVAL, "null count, or null rows with max > 0");
        REQUIRE(prec == EOFA_FP64 || prec == EOFA_MIXED_FP32 || prec == EOFA_MIXED_FP16, EOFA_EINVAL,
                "prec must be FP64, MIXED_FP32 or MIXED_FP16");
        const std::vector<Sched> c = sched_candidates(ctx, prec);
        for (int i = 0; i < max && i < (int)c.size(); i++) {
            int* r = sched_out + 7 * i;
            r[0] = c[i].mode; r[1] = c[i].xcd; r[2] = c[i].ty; r[3] = c[i].tz;
            r[4] = c[i].tt; r[5] = c[i].nyb; r[6] = c[i].ord;
        }
        *n = (int)c.size();
        return EOFA_OK;
    });
}

eofa_status eofa_set_precond(eofa_ctx* ctx, const float* params_host, size_t count, int relu) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(params_host && count == (size_t)CNN_NPARAM, EOFA_EINVAL,
                "eofa_set_precond expects " + std::to_string(CNN_NPARAM) + " FP32 parameters");
        REQUIRE(ctx->Ns % 8 == 0, EOFA_EINVAL, "learned preconditioner needs Ns % 8 == 0");
        for (size_t i = 0; i < count; i++) REQUIRE(std::isfinite(params_host[i]), EOFA_EINVAL, "non-finite parameter");
        cnn_alloc(ctx);
        ctx->cnn.relu = relu ? 1 : 0;
        HIPCHK(hipMemcpy(ctx->cnn.P, params_host, sizeof(float) * count, hipMemcpyHostToDevice));
        HIPCHK(hipMemset(ctx->cnn.M, 0, sizeof(float) * count));
        HIPCHK(hipMemset(ctx->cnn.V, 0, sizeof(float) * count));
        ctx->cnn.step = 0;
        cnn_refresh(ctx);
        HIPCHK(hipStreamSynchronize(ctx->st));
        ctx->cnn.ready = true;
        return EOFA_OK;
    });
}

eofa_status eofa_cnn_init(eofa_ctx* ctx, unsigned long long seed, int relu) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(ctx->Ns % 8 == 0, EOFA_EINVAL, "learned preconditioner needs Ns % 8 == 0");
        std::vector<float> h(CNN_NPARAM, 0.0f);
        uint64_t x = seed * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
        auto u01 = [&]() {  // xorshift64*, 53-bit uniform in (0, 1)
            x ^= x >> 12; x ^= x << 25; x ^= x >> 27;
            return ((double)((x * 0x2545F4914F6CDD1Dull) >> 11) + 0.5) / 9007199254740992.0;
        };
        for (int l = 0; l < CNN_LAYERS; l++) {
            const double sd = std::sqrt((relu ? 2.0 : 1.0) / (81.0 * CNN_CIN[l]));
            for (int tap = 0; tap < 81; tap++)
                for (int n = 0; n < CNN_COUT[l]; n++)
                    for (int k = 0; k < CNN_CIN[l]; k++) {
                        const double g = std::sqrt(-2.0 * std::log(u01())) * std::cos(6.283185307179586 * u01());
                        h[(size_t)l * CNN_LSZ + (size_t)tap * 1024 + n * 32 + k] = (float)(sd * g);
                    }
        }
        cnn_alloc(ctx);
        ctx->cnn.relu = relu ? 1 : 0;
        HIPCHK(hipMemcpy(ctx->cnn.P, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemset(ctx->cnn.M, 0, sizeof(float) * h.size()));
        HIPCHK(hipMemset(ctx->cnn.V, 0, sizeof(float) * h.size()));
        ctx->cnn.step = 0;
        cnn_refresh(ctx);
        HIPCHK(hipStreamSynchronize(ctx->st));
        ctx->cnn.ready = true;
        return EOFA_OK;
    });
}

eofa_status eofa_cnn_params(eofa_ctx* ctx, float* params_host, size_t count) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(ctx->cnn.ready, EOFA_ESTATE, "no network");
        REQUIRE(params_host && count == (size_t)CNN_NPARAM, EOFA_EINVAL, "bad parameter buffer");
        HIPCHK(hipStreamSynchronize(ctx->st));
        HIPCHK(hipMemcpy(params_host, ctx->cnn.P, sizeof(float) * count, hipMemcpyDeviceToHost));
        return EOFA_OK;
    });
}

eofa_status eofa_cnn_apply(eofa_ctx* ctx, const void* in5, void* out5) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(ctx->cnn.ready, EOFA_ESTATE, "no network");
        REQUIRE(in5 && out5 && in5 != out5, EOFA_EINVAL, "bad field pointers");
        eofa_solve_params P{1e-10, 1, EOFA_FP64, EOFA_PC_NONE, 0, 0, 0};
        ensure_ws(ctx, needed_bytes(ctx, &P));
        Work64 W = carve64(ctx);
        HIPCHK(launch_pack5<double>((const cd*)in5, W.r, ctx->g, 1, ctx->Ns, 0, ctx->st));
        cnn_apply_half(ctx, W.r, W.p);
        HIPCHK(hipMemsetAsync(W.u, 0, ctx->nh * sizeof(cd), ctx->st));
        HIPCHK(launch_unpack5<double>(W.u, (cd*)out5, ctx->g, 0, ctx->Ns, 0, ctx->st));
        HIPCHK(launch_unpack5<double>(W.p, (cd*)out5, ctx->g, 1, ctx->Ns, 0, ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));
        return EOFA_OK;
    });
}

// gradient (grad_host, may be NULL) and/or an Adam step (lr > 0) for one pair of canonical 5D fields
eofa_status eofa_cnn_train_step(eofa_ctx* ctx, const void* rho5, const void* e5, double lr, double* loss,
                                float* grad_host) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(ctx->cnn.ready, EOFA_ESTATE, "no network");
        REQUIRE(rho5 && e5, EOFA_EINVAL, "bad field pointers");
        eofa_solve_params P{1e-10, 1, EOFA_FP64, EOFA_PC_NONE, 0, 0, 0};
        ensure_ws(ctx, needed_bytes(ctx, &P));
        Work64 W = carve64(ctx);
        HIPCHK(launch_pack5<double>((const cd*)rho5, W.r, ctx->g, 1, ctx->Ns, 0, ctx->st));
        HIPCHK(launch_pack5<double>((const cd*)e5, W.p, ctx->g, 1, ctx->Ns, 0, ctx->st));
        const double L = cnn_grad(ctx, W.r, W.p);
        if (loss) *loss = L;
        auto& c = ctx->cnn;
        if (grad_host) {
            HIPCHK(hipStreamSynchronize(ctx->st));
            HIPCHK(hipMemcpy(grad_host, c.G, sizeof(float) * CNN_NPARAM, hipMemcpyDeviceToHost));
        }
        if (lr > 0) {
            c.step++;
            const float b1 = 0.9f, b2 = 0.999f;
            const float c1 = 1.0f - std::pow(b1, (float)c.step), c2 = 1.0f - std::pow(b2, (float)c.step);
            HIPCHK(cnn_adam(c.P, c.G, c.M, c.V, CNN_NPARAM, (float)lr, b1, b2, 1e-8f, c1, c2, 1.0f, ctx->st));
            cnn_refresh(ctx);
            HIPCHK(hipStreamSynchronize(ctx->st));
        }
        return EOFA_OK;
    });
}

// Training pairs from one CG solve of Dhat(mp, mm) x = b with a Gaussian b on the odd sites (seeded):
// snapshots x_k at k = 2, 4, 8, ...; after convergence e_k = x* - x_k and rho_k = Dhat^dag Dhat e_k,
// written as canonical 5D fields (odd sites; even sites zero).  *made = number of pairs written (<= n).
eofa_status eofa_training_pairs(eofa_ctx* ctx, double mp, double mm, unsigned long long seed, int n,
                                void* const* rho5, void* const* e5, int* made) {
    return guarded(ctx, [&]() -> eofa_status {
        REQUIRE(ctx->gauge, EOFA_ESTATE, "no gauge field set");
        REQUIRE(n >= 1 && n <= 16 && rho5 && e5 && made, EOFA_EINVAL, "bad arguments");
        eofa_solve_params P{1e-10, 1, EOFA_FP64, EOFA_PC_NONE, 0, 0, 0};
        ensure_ws(ctx, needed_bytes(ctx, &P));
        Work64 W = carve64(ctx);
        const size_t nh = ctx->nh;
        {   // Gaussian source on the odd sites
            std::vector<cd> h(nh);
            uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
            auto u01 = [&]() {
                x ^= x >> 12; x ^= x << 25; x ^= x >> 27;
                return ((double)((x * 0x2545F4914F6CDD1Dull) >> 11) + 0.5) / 9007199254740992.0;
            };
            for (size_t i = 0; i < nh; i++) {
                const double r = std::sqrt(-std::log(u01())), t = 6.283185307179586 * u01();
                h[i] = {r * std::cos(t), r * std::sin(t)};
            }
            HIPCHK(hipMemcpy(W.bh, h.data(), nh * sizeof(cd), hipMemcpyHostToDevice));
        }
        const SiteOp* Ai = site_tab(ctx, SK_AINV, mp, mm);
        const SiteOp* Ad = site_tab(ctx, SK_AINV_DAG, mp, mm);
        // CG as in cg64, with snapshots of x into the odd sites of e5[i]
        HIPCHK(hipMemsetAsync(W.xcg, 0, nh * sizeof(cd), ctx->st));
        HIPCHK(launch_scal_set(ctx->scal, SC_TOL2, 1e-24, -1, 0, -1, 0, ctx->st));
        double rr = normal_residual64(ctx, W, W.xcg, W.bh, Ai, Ad);
        HIPCHK(hipMemcpyAsync(W.p, W.r, nh * sizeof(cd), hipMemcpyDeviceToDevice, ctx->st));
        HIPCHK(launch_scal_set(ctx->scal, SC_RR, rr, SC_RR0, rr, SC_DONE, 0.0, ctx->st));
        HIPCHK(launch_scal_set(ctx->scal, SC_DONEX, 0.0, SC_ITERS, 0.0, -1, 0, ctx->st));
        int k = 0, snap = 0, next = 2;
        const int ce = kAutoCheckEvery;
        while (k < 100000) {
            cg_iteration<double>(ctx, W.xcg, W.r, W.p, W.u, W.w, W.wt, W.at, Ai, Ad);
            k++;
            if (k == next && snap < n) {
                sync_scal(ctx);  // no snapshot of an iterate the device has stopped updating
                if (ctx->hscal[SC_DONE] != 0.0) break;
                HIPCHK(hipMemsetAsync(W.res.h[0], 0, nh * sizeof(cd), ctx->st));
                HIPCHK(launch_unpack5<double>(W.res.h[0], (cd*)e5[snap], ctx->g, 0, ctx->Ns, 0, ctx->st));
                HIPCHK(launch_unpack5<double>(W.xcg, (cd*)e5[snap], ctx->g, 1, ctx->Ns, 0, ctx->st));
                snap++;
                next *= 2;
            }
            if (k % ce == 0) {
                sync_scal(ctx);
                if (ctx->hscal[SC_DONE] != 0.0 || !std::isfinite(ctx->hscal[SC_RR])) break;
            }
        }
        // e_i = x* - x_i ; rho_i = Dhat^dag Dhat e_i
        for (int i = 0; i < snap; i++) {
            HIPCHK(launch_pack5<double>((const cd*)e5[i], W.c.h[1], ctx->g, 1, ctx->Ns, 0, ctx->st));
            HIPCHK(launch_axpby<double>(1.0, W.xcg, -1.0, W.c.h[1], nh, nullptr, ctx->st));
            schur64(ctx, W, Ai, Ad, W.c.h[1], W.w);
            schur_dag64(ctx, W, Ad, W.w, W.p);
            HIPCHK(launch_unpack5<double>(W.c.h[1], (cd*)e5[i], ctx->g, 1, ctx->Ns, 0, ctx->st));
            HIPCHK(launch_unpack5<double>(W.res.h[0], (cd*)rho5[i], ctx->g, 0, ctx->Ns, 0, ctx->st));
            HIPCHK(launch_unpack5<double>(W.p, (cd*)rho5[i], ctx->g, 1, ctx->Ns, 0, ctx->st));
        }
        HIPCHK(hipStreamSynchronize(ctx->st));
        *made = snap;
        return EOFA_OK;
    });
}

const char* eofa_last_error(const eofa_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void eofa_destroy(eofa_ctx* ctx) {
    if (!ctx) return;
    for (auto& kv : ctx->tabs) (void)hipFree(kv.second);
    for (int p = 0; p < 2; p++) {
        if (ctx->U[p]) (void)hipFree(ctx->U[p]);
        if (ctx->Uf[p]) (void)hipFree(ctx->Uf[p]);
    }
    if (ctx->ws && ctx->ws_owned) (void)hipFree(ctx->ws);
    if (ctx->partials) (void)hipFree(ctx->partials);
    if (ctx->hb) (void)hipFree(ctx->hb);
    if (ctx->md_F) (void)hipFree(ctx->md_F);
    if (ctx->md_U0) (void)hipFree(ctx->md_U0);
    for (cd* q : ctx->md_guess) (void)hipFree(q);
    if (ctx->md_fn) (void)hipFree(ctx->md_fn);
    if (ctx->partials_mr) (void)hipFree(ctx->partials_mr);
    {
        auto& c = ctx->cnn;
        void* ptrs[] = {c.P, c.G, c.M, c.V, c.Wb, c.Wt, c.X0, c.A[0], c.A[1], c.A[2], c.dYb, c.XT, c.dYT,
                        c.Y, c.T, c.dY, c.dA, c.part, ctx->dots};
        for (void* q : ptrs)
            if (q) (void)hipFree(q);
    }
    for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    if (ctx->cap_st) (void)hipStreamDestroy(ctx->cap_st);
    if (ctx->scal) (void)hipFree(ctx->scal);
    if (ctx->hscal) (void)hipHostFree(ctx->hscal);
    for (auto& e : ctx->ev_pool) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    delete ctx;
}

}  // extern "C"
