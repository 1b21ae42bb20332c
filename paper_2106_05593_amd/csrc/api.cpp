// C-ABI of libmmc (include/mmc.h): contexts, device buffers and the order of
// kernel launches of a sweep.  All physics setup is FP64 on the host.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mmc_internal.h"

using namespace mmc;

namespace {
thread_local std::string g_err;

mmc_status fail(mmc_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCK(expr)                                                                                  \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            if (ctx) ctx->dead = true;                                                               \
            return fail(e_ == hipErrorOutOfMemory ? MMC_ERR_OOM : MMC_ERR_DEVICE, "%s: %s (%s:%d)", #expr, \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                  \
        }                                                                                            \
    } while (0)

int pad_pow2(int n, int minimum) {
    int p = 1;
    while (p < 2 * n - 1) p <<= 1;
    return std::max(p, minimum);
}
int ilog2i(int v) { int l = 0; while ((1 << l) < v) ++l; return l; }
}  // namespace

struct mmc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool dead = false;
    mmc_grid g{};
    mmc_cellsize cs{};
    mmc_material mat{};
    mmc_run run{};
    long long N = 0, Nc = 0;
    int hw = 0;
    double V = 0;
    // material classes (grains)
    int nclass = 1;
    bool has_classes = false;
    std::vector<double> ea, K1, K2, Tc;
    std::vector<double> Tg;      // per-grain temperatures (empty: every grain at run.T)
    // anisotropy form: uniaxial (ea, K1, K2 above) or cubic (ncub sets of axes and constants:
    // 1 for every class or one per class); kscale: temperature law of the constants
    bool cubic = false;
    bool kscale = false;
    int ncub = 0;
    std::vector<double> cax, cK1, cK2;
    double bscale = 1.0;
    std::vector<ClassCoef> ctab;
    ClassCoef* d_ctab = nullptr;
    uint32_t* d_cid = nullptr;
    // state
    float* d_m = nullptr;        // [2][3][Nc] colour-split
    float* d_h = nullptr;        // [2][3][Nc] colour-split demag field
    float* d_nat = nullptr;      // 3N natural staging
    DevState* d_st = nullptr;
    SweepAccum* d_acc = nullptr; // per-sweep statistics accumulators
    int fp_shift = 0;            // fixed-point scale of the accumulators
    double* d_epart = nullptr;
    int epart_n = 0;
    double* d_series = nullptr;
    int series_cap = 0;
    // demag
    bool demag = false;
    DemagPlan plan{};
    double xtune_us[6] = {0, 0, 0, 0, 0, 0};   // x-pass tuning: us per launch of each candidate
    int fuse = -1;               // colour-pass form: 0 separate, 1 fused, 2 half fused, -1 not decided (tuned)
    double fuse_us[3] = {0, 0, 0};  // tuning: us per colour of the separate, fused and half-fused forms
    float2* d_tw = nullptr;
    SweepArgs args{};
    unsigned long long host_sweep = 0;
    unsigned version = 0;        // bumps when kernel arguments change
    // mmc_sweep's graph of kSweepGraph sweeps, captured at `sg_version`
    hipGraph_t sg_graph = nullptr;
    hipGraphExec_t sg_exec = nullptr;
    unsigned sg_version = 0;
};

// Chains of one shape advance together: one launch per kernel serves all of
// them (chain = blockIdx.y).  Each group runs on a stream of its own.
struct BatchGroup {
    std::vector<int> idx;                 // chains of the group
    ChainDesc* d_list = nullptr;          // device copies of their descriptors
};

struct mmc_batch {
    std::vector<mmc_ctx*> ch;
    std::vector<BatchGroup> groups;
    std::vector<hipStream_t> streams;     // one per group
    std::vector<hipEvent_t> done;
    std::vector<hipEvent_t> chain_ev;     // per chain: orders its own stream against the batch launch
    hipEvent_t fork = nullptr;
    hipEvent_t joined = nullptr;          // recorded on the first chain's stream after a launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_n = -1;
    int graph_sched = -1;
    std::vector<unsigned> versions;
    // schedule: requested (MMC_SCHED_*) and in use; persistent plan
    int sched_req = MMC_SCHED_AUTO;
    int sched_used = MMC_SCHED_GROUPS;
    bool tuned = false;                   // the automatic choice was made for these chains
    double tune_ms[2] = {0.0, 0.0};       // measured time per trial for groups, persistent (0: not timed)
    PersistPlan pplan;
    bool pplan_ok = false;
};

// Automatic schedule choices by batch signature (process-wide).
static std::mutex g_sched_mu;
static std::map<std::string, int> g_sched_cache;

static void update_args(mmc_ctx* c) {
    SweepArgs& a = c->args;
    const double kT = kB * c->run.T;
    a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz; a.hw = c->hw; a.Nc = c->Nc;
    a.wx = (float)(c->V * c->mat.A0 / (c->cs.hx * c->cs.hx * kT));
    a.wy = (float)(c->V * c->mat.A0 / (c->cs.hy * c->cs.hy * kT));
    a.wz = (float)(c->V * c->mat.A0 / (c->cs.hz * c->cs.hz * kT));
    a.cdx = (float)(c->V * c->mat.D0 / (c->cs.hx * kT));
    a.cdy = (float)(c->V * c->mat.D0 / (c->cs.hy * kT));
    a.bx = (float)(c->V * c->mat.Ms0 * c->run.B[0] / kT);
    a.by = (float)(c->V * c->mat.Ms0 * c->run.B[1] / kT);
    a.bz = (float)(c->V * c->mat.Ms0 * c->run.B[2] / kT);
    a.cdm = (float)(kMu0 * c->V * c->mat.Ms0 * c->mat.Ms0 / kT);
    a.bscale = (float)c->bscale;
    a.k0 = (uint32_t)(c->run.seed & 0xFFFFFFFFull);
    a.k1 = (uint32_t)(c->run.seed >> 32);
    a.chain = c->run.chain_id;
    c->version++;
}

// The kernel-side view of one chain.
static ChainDesc make_desc(const mmc_ctx* ctx) {
    ChainDesc v{};
    v.a = ctx->args;
    v.ctab = ctx->d_ctab;
    v.cid = ctx->has_classes ? ctx->d_cid : nullptr;
    v.m = ctx->d_m;
    v.h = ctx->d_h;
    v.st = ctx->d_st;
    v.acc = ctx->d_acc;
    v.X = ctx->plan.X;
    return v;
}
static Chains single(const mmc_ctx* ctx) { return Chains{make_desc(ctx), nullptr, 1}; }

static mmc_status upload_classes(mmc_ctx* ctx) {
    ctx->ctab.resize(ctx->nclass);
    for (int k = 0; k < ctx->nclass; ++k) {
        const double T = ctx->Tg.empty() ? ctx->run.T : ctx->Tg[k];
        const int j = ctx->ncub == 1 ? 0 : k;
        ctx->ctab[k] = ctx->cubic
            ? class_coef(ctx->mat, T, ctx->run.T, ctx->V, ctx->cK1[j], ctx->cK2[j], &ctx->ea[3 * k], &ctx->cax[6 * j],
                         ctx->kscale, ctx->Tc[k], ctx->run.sigma_fixed)
            : class_coef(ctx->mat, T, ctx->run.T, ctx->V, ctx->K1[k], ctx->K2[k], &ctx->ea[3 * k], nullptr,
                         ctx->kscale, ctx->Tc[k], ctx->run.sigma_fixed);
    }
    if (ctx->d_ctab) { HIPCK(hipFree(ctx->d_ctab)); ctx->d_ctab = nullptr; }
    HIPCK(hipMalloc(&ctx->d_ctab, sizeof(ClassCoef) * ctx->nclass));
    ctx->version++;              // graphs captured before hold the old table's address
    HIPCK(hipMemcpyAsync(ctx->d_ctab, ctx->ctab.data(), sizeof(ClassCoef) * ctx->nclass, hipMemcpyHostToDevice,
                         ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MMC_OK;
}

static mmc_status init_state(mmc_ctx* ctx) {
    const double* d = ctx->run.init_dir;
    double n = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double u[3] = {0, 0, 1};
    if (n > 0) { u[0] = d[0] / n; u[1] = d[1] / n; u[2] = d[2] / n; }
    HIPCK(launch_init(ctx->args, ctx->d_ctab, ctx->d_cid, ctx->d_m, ctx->run.init, (float)u[0], (float)u[1],
                      (float)u[2], ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MMC_OK;
}

// Launch sequence of n sweeps.  With `prof`, HIP events bracket every launch
// (kinds: 0 demag x-forward, 1 demag y-pass, 2 demag x-inverse, 3 colour pass,
// 4 end of sweep, 5 fused x-inverse + colour pass (+ x-forward in the full form)).
struct LaunchProf {
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    size_t used = 0;
    int every = 1;    // instrument sweeps 0, every, 2*every, ...
};

// The fused colour passes serve chains of uniform material, nx % 8 == 0 and
// the field refreshed before each colour (the half form from a padded x
// length of 64 on); MMC_FUSE=0, 1 or 2 in the environment at mmc_create
// forces the separate kernels, the fused or the half-fused form.
static bool fuse_eligible(const mmc_ctx* c, int form) {
    return c->demag && c->run.refresh_per_sweep >= 2 && !c->cubic &&
           fused_ok(c->args, c->plan.L, c->has_classes, form == 1);
}
static int fused_form(const mmc_ctx* c) { return c->fuse >= 1 && fuse_eligible(c, c->fuse) ? c->fuse : 0; }

// n sweeps of the chains ch, all of c0's shape, on stream st.
static mmc_status enqueue_core(mmc_ctx* c0, const Chains& ch, int n, hipStream_t st, double* series,
                               unsigned long long rec_base, LaunchProf* prof) {
    mmc_ctx* ctx = c0;
    int sw = 0;
    auto mark = [&](int kind) -> hipError_t {
        if (!prof || sw % prof->every != 0) return hipSuccess;
        if (prof->used + 1 >= prof->ev.size()) return hipErrorInvalidValue;
        if (kind >= 0) prof->kind.push_back(kind);
        return hipEventRecord(prof->ev[prof->used++], st);
    };
    const bool exact = c0->run.lenmove == MMC_LEN_EXACT, dmi = c0->mat.D0 != 0.0;
    const int form = fused_form(c0);
    if (n > 0 && form == 2) {
        // per colour: x-spectrum of the current state, y pass, half-fused pass
        for (int s = 0; s < n; ++s) {
            sw = s;
            for (int c = 0; c < 2; ++c) {
                for (int stage = 0; stage < 2; ++stage) {
                    HIPCK(mark(-1));
                    HIPCK(launch_demag_stage(stage, c0->args, c0->plan, ch, 1 << c, c0->d_tw, st));
                    HIPCK(mark(stage));
                }
                HIPCK(mark(-1));
                HIPCK(launch_fused(c0->args, c0->plan, exact, dmi, ch, c, c0->fp_shift, c0->d_tw, st, false));
                HIPCK(mark(5));
            }
            HIPCK(mark(-1));
            HIPCK(launch_end_sweep(ch, c0->fp_shift, c0->N, series, rec_base, st));
            HIPCK(mark(4));
        }
        return MMC_OK;
    }
    if (n > 0 && form == 1) {
        // x-spectrum of the current state, then per colour: y pass, fused pass
        // (which leaves the updated state's x-spectrum for the next y pass)
        sw = 0;
        HIPCK(mark(-1));
        HIPCK(launch_demag_stage(0, c0->args, c0->plan, ch, 3, c0->d_tw, st));
        HIPCK(mark(0));
        for (int s = 0; s < n; ++s) {
            sw = s;
            for (int c = 0; c < 2; ++c) {
                HIPCK(mark(-1));
                HIPCK(launch_demag_stage(1, c0->args, c0->plan, ch, 1 << c, c0->d_tw, st));
                HIPCK(mark(1));
                HIPCK(mark(-1));
                HIPCK(launch_fused(c0->args, c0->plan, exact, dmi, ch, c, c0->fp_shift, c0->d_tw, st, true));
                HIPCK(mark(5));
            }
            HIPCK(mark(-1));
            HIPCK(launch_end_sweep(ch, c0->fp_shift, c0->N, series, rec_base, st));
            HIPCK(mark(4));
        }
        return MMC_OK;
    }
    for (int s = 0; s < n; ++s) {
        sw = s;
        for (int c = 0; c < 2; ++c) {
            const bool refresh = c0->demag && (c == 0 || c0->run.refresh_per_sweep >= 2);
            if (refresh) {
                const int mask = c0->run.refresh_per_sweep >= 2 ? (1 << c) : 3;
                for (int stage = 0; stage < 3; ++stage) {
                    HIPCK(mark(-1));
                    HIPCK(launch_demag_stage(stage, c0->args, c0->plan, ch, mask, c0->d_tw, st));
                    HIPCK(mark(stage));
                }
            }
            HIPCK(mark(-1));
            HIPCK(launch_pass(c0->args, c0->has_classes, c0->demag, exact, dmi, c0->cubic, ch, c, true, c0->fp_shift,
                              nullptr, st));
            HIPCK(mark(3));
        }
        HIPCK(mark(-1));
        HIPCK(launch_end_sweep(ch, c0->fp_shift, c0->N, series, rec_base, st));
        HIPCK(mark(4));
    }
    return MMC_OK;
}

static mmc_status enqueue_sweeps(mmc_ctx* ctx, int n, double* series, unsigned long long rec_base,
                                 LaunchProf* prof = nullptr) {
    mmc_status s = enqueue_core(ctx, single(ctx), n, ctx->stream, series, rec_base, prof);
    if (s != MMC_OK) return s;
    ctx->host_sweep += (unsigned long long)n;
    return MMC_OK;
}

// ---------------------------------------------------------------------
// Tile-shape tuner of the x passes: rows per thread 1, 2 or 4 (tiles of
// x_rows_conc(L) * rpt rows), timed for each direction on the chain's own
// buffers (the x passes write only the spectrum work buffer and the demag
// field, both recomputed before every use, and every choice gives the same
// bits), the fastest kept; the choice is cached per (x length, ny, nz).
// MMC_TUNE=0 in the environment keeps the untuned default.
// ---------------------------------------------------------------------
struct XTune {
    int f = 2, i = 2;
    double us[6] = {0, 0, 0, 0, 0, 0};   // forward rpt 1, 2, 4; inverse rpt 1, 2, 4 (us per launch)
};
static std::mutex g_xtune_mu;
static std::map<std::string, XTune> g_xtune;

static mmc_status tune_x(mmc_ctx* ctx) {
    DemagPlan& p = ctx->plan;
    std::fill(ctx->xtune_us, ctx->xtune_us + 6, 0.0);
    const char* env = getenv("MMC_TUNE");
    if (env && (env[0] == '0' || env[0] == '1' || env[0] == '2' || env[0] == '4') && env[1] == 0) {
        // 0: the untuned default; 1, 2, 4: that many rows per thread both ways
        p.rpt_f = p.rpt_i = env[0] == '0' ? x_rpt_default(p.L) : env[0] - '0';
        return MMC_OK;
    }
    char key[64];
    snprintf(key, sizeof key, "%d,%d,%d", p.L, ctx->g.ny, ctx->g.nz);
    {
        std::lock_guard<std::mutex> lk(g_xtune_mu);
        auto it = g_xtune.find(key);
        if (it != g_xtune.end()) {
            p.rpt_f = it->second.f;
            p.rpt_i = it->second.i;
            std::copy(it->second.us, it->second.us + 6, ctx->xtune_us);
            return MMC_OK;
        }
    }
    p.rpt_f = p.rpt_i = x_rpt_default(p.L);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(MMC_ERR_DEVICE, "event creation failed");
    }
    XTune t;
    const int rpts[3] = {1, 2, 4};
    constexpr int kWarm = 2, kTimed = 5;
    mmc_status st = MMC_OK;
    for (int d = 0; d < 2 && st == MMC_OK; ++d) {
        const int stage = d == 0 ? 0 : 2;
        double best = 1e30;
        for (int r = 0; r < 3 && st == MMC_OK; ++r) {
            // candidates whose blocks need more than 96 KiB of LDS (two per CU) are skipped
            if (rpts[r] != x_rpt_default(p.L) && x_pass_lds(p.L, rpts[r]) > 96 * 1024) continue;
            (d == 0 ? p.rpt_f : p.rpt_i) = rpts[r];
            hipError_t e = hipSuccess;
            for (int k = 0; k < kWarm + kTimed && e == hipSuccess; ++k) {
                if (k == kWarm) e = hipEventRecord(e0, ctx->stream);
                if (e == hipSuccess) e = launch_demag_stage(stage, ctx->args, p, single(ctx), 3, ctx->d_tw, ctx->stream);
            }
            if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { st = fail(MMC_ERR_DEVICE, "x-pass tuning: %s", hipGetErrorString(e)); break; }
            const double us = 1e3 * ms / kTimed;
            t.us[3 * d + r] = us;
            if (us < best) { best = us; (d == 0 ? t.f : t.i) = rpts[r]; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MMC_OK) return st;
    p.rpt_f = t.f;
    p.rpt_i = t.i;
    std::copy(t.us, t.us + 6, ctx->xtune_us);
    std::lock_guard<std::mutex> lk(g_xtune_mu);
    g_xtune[key] = t;
    return MMC_OK;
}

// Fused or separate colour passes: one colour of each eligible form (x-inverse,
// colour pass, x-forward; the fused kernel; the half-fused kernel and the
// x-forward) is timed from the same state, which is restored afterwards (m,
// run state and statistics accumulators; the spectrum and field buffers are
// recomputed before every use), and the fastest form is kept; the choice is
// cached per shape.  All forms give the same bits.
struct FuseChoice {
    int form;
    double us[3];
};
static std::mutex g_fuse_mu;
static std::map<std::string, FuseChoice> g_fuse;

static mmc_status tune_fuse(mmc_ctx* ctx) {
    if (!fuse_eligible(ctx, 1)) { ctx->fuse = 0; return MMC_OK; }
    char key[96];
    snprintf(key, sizeof key, "%d,%d,%d,%d,%d", ctx->g.nx, ctx->g.ny, ctx->g.nz, ctx->run.lenmove, ctx->mat.D0 != 0.0);
    {
        std::lock_guard<std::mutex> lk(g_fuse_mu);
        auto it = g_fuse.find(key);
        if (it != g_fuse.end()) {
            ctx->fuse = it->second.form;
            std::copy(it->second.us, it->second.us + 3, ctx->fuse_us);
            return MMC_OK;
        }
    }
    const size_t mb = sizeof(float) * 6 * (size_t)ctx->Nc;
    const size_t tot = mb + sizeof(DevState) + sizeof(SweepAccum);
    void* snap = nullptr;
    if (hipMalloc(&snap, tot) != hipSuccess) return fail(MMC_ERR_OOM, "tuning snapshot");
    char* p = (char*)snap;
    auto save = [&](bool restore) -> hipError_t {
        const hipMemcpyKind k = hipMemcpyDeviceToDevice;
        hipError_t e = restore ? hipMemcpyAsync(ctx->d_m, p, mb, k, ctx->stream) : hipMemcpyAsync(p, ctx->d_m, mb, k, ctx->stream);
        if (e == hipSuccess)
            e = restore ? hipMemcpyAsync(ctx->d_st, p + mb, sizeof(DevState), k, ctx->stream)
                        : hipMemcpyAsync(p + mb, ctx->d_st, sizeof(DevState), k, ctx->stream);
        if (e == hipSuccess)
            e = restore ? hipMemcpyAsync(ctx->d_acc, p + mb + sizeof(DevState), sizeof(SweepAccum), k, ctx->stream)
                        : hipMemcpyAsync(p + mb + sizeof(DevState), ctx->d_acc, sizeof(SweepAccum), k, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        return e;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = save(false);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const bool exact = ctx->run.lenmove == MMC_LEN_EXACT, dmi = ctx->mat.D0 != 0.0;
    const Chains one = single(ctx);
    double us[3] = {0, 0, 0};
    constexpr int kWarm = 1, kTimed = 3;
    const int nforms = fuse_eligible(ctx, 2) ? 3 : 2;
    for (int form = 0; form < nforms && e == hipSuccess; ++form) {
        for (int k = 0; k < kWarm + kTimed && e == hipSuccess; ++k) {
            if (k == kWarm) e = hipEventRecord(e0, ctx->stream);
            if (e != hipSuccess) break;
            if (form == 0) {
                e = launch_demag_stage(2, ctx->args, ctx->plan, one, 1, ctx->d_tw, ctx->stream);
                if (e == hipSuccess)
                    e = launch_pass(ctx->args, false, true, exact, dmi, false, one, 0, true, ctx->fp_shift, nullptr,
                                    ctx->stream);
                if (e == hipSuccess) e = launch_demag_stage(0, ctx->args, ctx->plan, one, 3, ctx->d_tw, ctx->stream);
            } else if (form == 1) {
                e = launch_fused(ctx->args, ctx->plan, exact, dmi, one, 0, ctx->fp_shift, ctx->d_tw, ctx->stream, true);
            } else {
                e = launch_fused(ctx->args, ctx->plan, exact, dmi, one, 0, ctx->fp_shift, ctx->d_tw, ctx->stream, false);
                if (e == hipSuccess) e = launch_demag_stage(0, ctx->args, ctx->plan, one, 3, ctx->d_tw, ctx->stream);
            }
        }
        if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        us[form] = 1e3 * ms / kTimed;
        if (e == hipSuccess) e = save(true);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(snap);
    if (e != hipSuccess) return fail(MMC_ERR_DEVICE, "fusion tuning: %s", hipGetErrorString(e));
    int best = 0;
    for (int f = 1; f < nforms; ++f)
        if (us[f] < us[best]) best = f;
    ctx->fuse = best;
    std::copy(us, us + 3, ctx->fuse_us);
    std::lock_guard<std::mutex> lk(g_fuse_mu);
    g_fuse[key] = {best, {us[0], us[1], us[2]}};
    return MMC_OK;
}

static mmc_status check_live(mmc_ctx* ctx) {
    if (!ctx) return fail(MMC_ERR_ARG, "NULL context");
    if (ctx->dead) return fail(MMC_ERR_STATE, "context had a device error; destroy it");
    HIPCK(hipSetDevice(ctx->device));
    return MMC_OK;
}

extern "C" {

const char* mmc_status_str(mmc_status s) {
    switch (s) {
        case MMC_OK: return "ok";
        case MMC_ERR_ARG: return "invalid argument";
        case MMC_ERR_DOMAIN: return "value outside the physical domain";
        case MMC_ERR_OOM: return "out of memory";
        case MMC_ERR_DEVICE: return "device error";
        case MMC_ERR_STATE: return "invalid state";
        case MMC_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* mmc_last_error(void) { return g_err.c_str(); }

void mmc_destroy(mmc_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    void* bufs[] = {ctx->d_ctab, ctx->d_cid, ctx->d_m, ctx->d_h, ctx->d_nat, ctx->d_st, ctx->d_acc,
                    ctx->d_epart, ctx->d_series, ctx->plan.X, ctx->plan.K, ctx->d_tw};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (ctx->sg_exec) (void)hipGraphExecDestroy(ctx->sg_exec);
    if (ctx->sg_graph) (void)hipGraphDestroy(ctx->sg_graph);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

mmc_status mmc_create(const mmc_grid* grid, const mmc_cellsize* cell, const mmc_material* mat, const mmc_run* run,
                      void* hip_stream, mmc_ctx** out) {
    mmc_ctx* ctx = nullptr;
    if (!grid || !cell || !mat || !run || !out) return fail(MMC_ERR_ARG, "NULL argument");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || grid->nx > 2048 || grid->ny > 2048 || grid->nz > 4096 ||
        (long long)grid->nx * grid->ny * grid->nz > (1LL << 28))
        return fail(MMC_ERR_ARG, "grid %d x %d x %d out of range", grid->nx, grid->ny, grid->nz);
    if (!(cell->hx > 0 && cell->hy > 0 && cell->hz > 0) || !std::isfinite(cell->hx * cell->hy * cell->hz))
        return fail(MMC_ERR_DOMAIN, "cell sizes must be positive");
    if (!(mat->Ms0 > 0) || !(mat->A0 >= 0) || !(mat->Tc > 0) || !(mat->mu_atomic > 0) || !std::isfinite(mat->D0) ||
        !std::isfinite(mat->K1) || !std::isfinite(mat->K2))
        return fail(MMC_ERR_DOMAIN, "invalid material constants");
    if (mat->mf != MMC_MF_LANGEVIN && mat->mf != MMC_MF_BRILLOUIN_HALF) return fail(MMC_ERR_ARG, "unknown mean-field model");
    const double ean = std::sqrt(mat->easy_axis[0] * mat->easy_axis[0] + mat->easy_axis[1] * mat->easy_axis[1] +
                                 mat->easy_axis[2] * mat->easy_axis[2]);
    if (!(ean > 0) || !std::isfinite(ean)) return fail(MMC_ERR_DOMAIN, "easy axis must be non-zero");
    if (!(run->T > 0) || !std::isfinite(run->T)) return fail(MMC_ERR_DOMAIN, "temperature must be > 0");
    if (run->cone_deg < 1 || run->cone_deg > 180) return fail(MMC_ERR_ARG, "cone_deg must be in [1, 180]");
    if (run->adapt_every < 0) return fail(MMC_ERR_ARG, "adapt_every must be >= 0");
    if (run->lenmove != MMC_LEN_PAPER && run->lenmove != MMC_LEN_EXACT) return fail(MMC_ERR_ARG, "unknown lenmove");
    if (run->demag < MMC_DEMAG_OFF || run->demag > MMC_DEMAG_SPLIT_FP16) return fail(MMC_ERR_ARG, "unknown demag mode");
    if (run->refresh_per_sweep != 1 && run->refresh_per_sweep != 2) return fail(MMC_ERR_ARG, "refresh_per_sweep must be 1 or 2");
    if (run->init != 0 && run->init != 1) return fail(MMC_ERR_ARG, "init must be 0 or 1");
    if (!(run->sigma_fixed < 1.0)) return fail(MMC_ERR_DOMAIN, "sigma_fixed must be < 1");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(run->B[k])) return fail(MMC_ERR_DOMAIN, "field must be finite");
    if (run->demag) {
        if (grid->nz > ystage_max_nz()) return fail(MMC_ERR_UNSUPPORTED, "demag needs nz <= %d", ystage_max_nz());
        const int Py = pad_pow2(grid->ny, 1);
        if (run->demag >= MMC_DEMAG_SPLIT_BF16 && !ypass_split_ok(grid->nz, Py))
            return fail(MMC_ERR_UNSUPPORTED,
                        "split-precision demag needs an even nz and a padded y length of 512, 1024 or 2048 "
                        "(nz = 2, 4) or 256 or 1024 (nz = 6, 8); got nz %d, padded y %d", grid->nz, Py);
    }

    ctx = new (std::nothrow) mmc_ctx();
    if (!ctx) return fail(MMC_ERR_OOM, "host allocation failed");
    mmc_status st = MMC_OK;
    do {
        ctx->g = *grid; ctx->cs = *cell; ctx->mat = *mat; ctx->run = *run;
        if (hipGetDevice(&ctx->device) != hipSuccess) { st = fail(MMC_ERR_DEVICE, "no HIP device"); break; }
        {
            const char* fe = getenv("MMC_FUSE");
            ctx->fuse = (fe && fe[0] >= '0' && fe[0] <= '2' && fe[1] == 0) ? fe[0] - '0' : -1;
        }
        // set-up of mmc_energy_noalloc's scratch on this device (once per device)
        {
            const hipError_t e = energy_scratch_init(ctx->device);
            if (e != hipSuccess) {
                st = fail(MMC_ERR_DEVICE, "energy scratch set-up on device %d: %s", ctx->device, hipGetErrorString(e));
                break;
            }
        }
        if (hip_stream) ctx->stream = (hipStream_t)hip_stream;
        else {
            if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
                st = fail(MMC_ERR_DEVICE, "stream creation failed");
                break;
            }
            ctx->own_stream = true;
        }
        ctx->N = (long long)grid->nx * grid->ny * grid->nz;
        ctx->hw = (grid->nx + 1) / 2;
        ctx->Nc = (long long)grid->nz * grid->ny * ctx->hw;
        ctx->V = cell->hx * cell->hy * cell->hz;
        ctx->nclass = 1;
        ctx->ea.assign(mat->easy_axis, mat->easy_axis + 3);
        ctx->K1.assign(1, mat->K1); ctx->K2.assign(1, mat->K2); ctx->Tc.assign(1, mat->Tc);
        ctx->demag = run->demag != MMC_DEMAG_OFF;
        update_args(ctx);
        st = upload_classes(ctx);
        if (st != MMC_OK) break;
        const size_t msz = sizeof(float) * 6 * (size_t)ctx->Nc;
        auto alloc = [&](void** p, size_t bytes) -> bool {
            hipError_t e = hipMalloc(p, bytes);
            if (e != hipSuccess) {
                st = fail(e == hipErrorOutOfMemory ? MMC_ERR_OOM : MMC_ERR_DEVICE, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
                return false;
            }
            return true;
        };
        if (!alloc((void**)&ctx->d_m, msz)) break;
        if (hipMemset(ctx->d_m, 0, msz) != hipSuccess) { st = fail(MMC_ERR_DEVICE, "memset"); break; }
        if (!alloc((void**)&ctx->d_h, msz)) break;
        if (hipMemset(ctx->d_h, 0, msz) != hipSuccess) { st = fail(MMC_ERR_DEVICE, "memset"); break; }
        if (!alloc((void**)&ctx->d_st, sizeof(DevState))) break;
        if (!alloc((void**)&ctx->d_acc, sizeof(SweepAccum))) break;
        if (hipMemset(ctx->d_acc, 0, sizeof(SweepAccum)) != hipSuccess) { st = fail(MMC_ERR_DEVICE, "memset"); break; }
        {   // fixed point with headroom for |m| <= 4 summed over N cells: N * 16 * 2^shift <= 2^60
            int lg = 0;
            while ((1LL << lg) < ctx->N) ++lg;
            ctx->fp_shift = 56 - lg;
        }
        DevState hs{};
        hs.cone_deg = run->cone_deg;
        hs.adapt_every = run->adapt_every;
        const double sh = std::sin(0.5 * run->cone_deg * kPi / 180.0);
        hs.omc = (float)(2.0 * sh * sh);
        if (hipMemcpy(ctx->d_st, &hs, sizeof hs, hipMemcpyHostToDevice) != hipSuccess) { st = fail(MMC_ERR_DEVICE, "copy"); break; }
        if (ctx->demag) {
            DemagPlan& p = ctx->plan;
            p.Px = pad_pow2(grid->nx, 2);
            p.Py = pad_pow2(grid->ny, 1);
            p.L = p.Px / 2;
            p.logL = ilog2i(p.L);
            p.logPy = ilog2i(p.Py);
            p.S = 3 * grid->nz;
            std::vector<float> K;
            tensor_spectrum(grid->nx, grid->ny, grid->nz, cell->hx, cell->hy, cell->hz, p.Px, p.Py, K);
            p.prec = run->demag == MMC_DEMAG_SPLIT_BF16 ? 1 : (run->demag == MMC_DEMAG_SPLIT_FP16 ? 2 : 0);
            p.kmax = 0.f;
            for (float kv : K) p.kmax = std::max(p.kmax, std::fabs(kv));
            if (!alloc((void**)&p.K, sizeof(float) * K.size())) break;
            if (hipMemcpy(p.K, K.data(), sizeof(float) * K.size(), hipMemcpyHostToDevice) != hipSuccess) { st = fail(MMC_ERR_DEVICE, "copy"); break; }
            // staged y pass (more than 8 layers, or a padded y too long for the
            // one-kernel pass's registers): its work buffer follows X
            const size_t xel = (size_t)(p.L + 1) * p.S * grid->ny;
            const size_t wel = ystage_needed(grid->nz, p.Py) ? (size_t)ystage_work_elems(p.L, p.S, p.Py) : 0;
            p.woff = wel ? (long long)xel : 0;
            if (!alloc((void**)&p.X, sizeof(float2) * (xel + wel))) break;
            std::vector<float2> tw(8192);
            for (int j = 0; j < 8192; ++j) tw[j] = make_float2((float)std::cos(-2.0 * kPi * j / 8192), (float)std::sin(-2.0 * kPi * j / 8192));
            if (!alloc((void**)&ctx->d_tw, sizeof(float2) * (8192 + 4096))) break;
            if (hipMemcpy(ctx->d_tw, tw.data(), sizeof(float2) * 8192, hipMemcpyHostToDevice) != hipSuccess) { st = fail(MMC_ERR_DEVICE, "copy"); break; }
            if (launch_x_twiddles(p, ctx->d_tw, ctx->stream) != hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess) { st = fail(MMC_ERR_DEVICE, "twiddle tables"); break; }
        }
        st = init_state(ctx);
        if (st == MMC_OK && ctx->demag) st = tune_x(ctx);
        if (st == MMC_OK && ctx->fuse < 0) st = tune_fuse(ctx);
    } while (false);
    if (st != MMC_OK) {
        mmc_destroy(ctx);
        return st;
    }
    *out = ctx;
    return MMC_OK;
}

mmc_status mmc_set_grains(mmc_ctx* ctx, const uint32_t* grain_of_cell, uint32_t n_grains, const double* easy_axis3,
                          const double* K1, const double* K2, const double* Tc, double boundary_exchange_scale) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!grain_of_cell || !easy_axis3 || !K1 || !K2 || !Tc || n_grains < 1) return fail(MMC_ERR_ARG, "NULL or empty grain data");
    if (!(boundary_exchange_scale >= 0) || !std::isfinite(boundary_exchange_scale)) return fail(MMC_ERR_DOMAIN, "bad boundary scale");
    for (uint32_t k = 0; k < n_grains; ++k) {
        const double* e = easy_axis3 + 3 * k;
        if (!(Tc[k] > 0) || !std::isfinite(K1[k]) || !std::isfinite(K2[k]) || !(e[0] * e[0] + e[1] * e[1] + e[2] * e[2] > 0))
            return fail(MMC_ERR_DOMAIN, "grain %u: invalid constants", k);
    }
    std::vector<uint32_t> split(2 * (size_t)ctx->Nc, 0u);
    for (long long p = 0; p < ctx->N; ++p) {
        const uint32_t k = grain_of_cell[p];
        if (k >= n_grains) return fail(MMC_ERR_ARG, "grain id %u of cell %lld >= n_grains", k, p);
        const int x = (int)(p % ctx->g.nx), y = (int)((p / ctx->g.nx) % ctx->g.ny), z = (int)(p / ((long long)ctx->g.nx * ctx->g.ny));
        const int c = (x + y + z) & 1;
        split[(size_t)c * ctx->Nc + ((size_t)z * ctx->g.ny + y) * ctx->hw + (x >> 1)] = k;
    }
    ctx->nclass = (int)n_grains;
    ctx->ea.assign(easy_axis3, easy_axis3 + 3 * (size_t)n_grains);
    ctx->K1.assign(K1, K1 + n_grains); ctx->K2.assign(K2, K2 + n_grains); ctx->Tc.assign(Tc, Tc + n_grains);
    ctx->bscale = boundary_exchange_scale;
    ctx->has_classes = true;
    ctx->Tg.clear();
    ctx->cubic = false;
    ctx->kscale = false;
    ctx->ncub = 0;
    if (!ctx->d_cid) HIPCK(hipMalloc(&ctx->d_cid, sizeof(uint32_t) * 2 * (size_t)ctx->Nc));
    HIPCK(hipMemcpy(ctx->d_cid, split.data(), sizeof(uint32_t) * split.size(), hipMemcpyHostToDevice));
    update_args(ctx);
    s = upload_classes(ctx);
    if (s != MMC_OK) return s;
    return init_state(ctx);
}

mmc_status mmc_set_field(mmc_ctx* ctx, const double mu0H_tesla[3]) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!mu0H_tesla) return fail(MMC_ERR_ARG, "NULL field");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(mu0H_tesla[k])) return fail(MMC_ERR_DOMAIN, "field must be finite");
    for (int k = 0; k < 3; ++k) ctx->run.B[k] = mu0H_tesla[k];
    update_args(ctx);
    return MMC_OK;
}

mmc_status mmc_set_temperature(mmc_ctx* ctx, double T) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!(T > 0) || !std::isfinite(T)) return fail(MMC_ERR_DOMAIN, "temperature must be > 0");
    HIPCK(hipStreamSynchronize(ctx->stream));
    ctx->run.T = T;
    ctx->Tg.clear();
    update_args(ctx);
    return upload_classes(ctx);
}

mmc_status mmc_set_grain_temperatures(mmc_ctx* ctx, const double* T_of_grain, uint32_t n_grains) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!ctx->has_classes) return fail(MMC_ERR_STATE, "no grains: call mmc_set_grains first");
    if (T_of_grain) {
        if ((int)n_grains != ctx->nclass) return fail(MMC_ERR_ARG, "%u temperatures for %d grains", n_grains, ctx->nclass);
        for (uint32_t k = 0; k < n_grains; ++k)
            if (!(T_of_grain[k] > 0) || !std::isfinite(T_of_grain[k]))
                return fail(MMC_ERR_DOMAIN, "grain %u: temperature must be > 0", k);
    }
    HIPCK(hipStreamSynchronize(ctx->stream));
    if (T_of_grain) ctx->Tg.assign(T_of_grain, T_of_grain + n_grains);
    else ctx->Tg.clear();
    update_args(ctx);
    return upload_classes(ctx);
}

mmc_status mmc_set_anisotropy(mmc_ctx* ctx, int32_t kind, const double* axes6, const double* K1, const double* K2,
                              uint32_t n, int32_t me_scaling) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (me_scaling != 0 && me_scaling != 1) return fail(MMC_ERR_ARG, "me_scaling must be 0 or 1");
    if (kind == MMC_ANIS_UNIAXIAL) {
        if (axes6 || K1 || K2 || n != 0) return fail(MMC_ERR_ARG, "uniaxial form takes no axes or constants");
    } else if (kind == MMC_ANIS_CUBIC) {
        if (!axes6 || !K1 || !K2) return fail(MMC_ERR_ARG, "NULL cubic axes or constants");
        if (n != 1 && (int64_t)n != (int64_t)ctx->nclass)
            return fail(MMC_ERR_ARG, "%u cubic sets: need 1 or one per grain (%d)", n, ctx->nclass);
        for (uint32_t k = 0; k < n; ++k) {
            const double* a = axes6 + 6 * (size_t)k;
            const double n1 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2], n2 = a[3] * a[3] + a[4] * a[4] + a[5] * a[5];
            const double cx = a[1] * a[5] - a[2] * a[4], cy = a[2] * a[3] - a[0] * a[5], cz = a[0] * a[4] - a[1] * a[3];
            bool fin = std::isfinite(K1[k]) && std::isfinite(K2[k]);
            for (int q = 0; q < 6; ++q) fin = fin && std::isfinite(a[q]);
            if (!fin) return fail(MMC_ERR_DOMAIN, "cubic set %u: constants and axes must be finite", k);
            if (!(n1 > 0) || !(n2 > 0) || !(cx * cx + cy * cy + cz * cz > 1e-12 * n1 * n2))
                return fail(MMC_ERR_ARG, "cubic set %u: axes zero or parallel", k);
        }
    } else {
        return fail(MMC_ERR_ARG, "unknown anisotropy kind %d", kind);
    }
    HIPCK(hipStreamSynchronize(ctx->stream));
    ctx->cubic = kind == MMC_ANIS_CUBIC;
    ctx->kscale = me_scaling != 0;
    ctx->ncub = ctx->cubic ? (int)n : 0;
    if (ctx->cubic) {
        ctx->cax.assign(axes6, axes6 + 6 * (size_t)n);
        ctx->cK1.assign(K1, K1 + n);
        ctx->cK2.assign(K2, K2 + n);
    } else {
        ctx->cax.clear(); ctx->cK1.clear(); ctx->cK2.clear();
    }
    ctx->version++;
    return upload_classes(ctx);
}

mmc_status mmc_set_m(mmc_ctx* ctx, const float* m, int on_device) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!m) return fail(MMC_ERR_ARG, "NULL state");
    std::vector<float> host;
    const float* hm = m;
    if (on_device) {
        host.resize(3 * (size_t)ctx->N);
        HIPCK(hipMemcpyAsync(host.data(), m, sizeof(float) * host.size(), hipMemcpyDeviceToHost, ctx->stream));
        HIPCK(hipStreamSynchronize(ctx->stream));
        hm = host.data();
    }
    for (long long p = 0; p < ctx->N; ++p) {
        const double a = hm[p], b = hm[ctx->N + p], c = hm[2 * ctx->N + p];
        const double q = a * a + b * b + c * c;
        if (!(q > 0) || !std::isfinite(q)) return fail(MMC_ERR_DOMAIN, "cell %lld: |m| must be finite and > 0", p);
    }
    if (!ctx->d_nat) HIPCK(hipMalloc(&ctx->d_nat, sizeof(float) * 3 * (size_t)ctx->N));
    HIPCK(hipMemcpyAsync(ctx->d_nat, m, sizeof(float) * 3 * (size_t)ctx->N,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
    HIPCK(launch_to_split(ctx->args, ctx->d_nat, ctx->d_m, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MMC_OK;
}

mmc_status mmc_get_m(mmc_ctx* ctx, float* out, int on_device) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!out) return fail(MMC_ERR_ARG, "NULL output");
    if (on_device) {
        HIPCK(launch_from_split(ctx->args, ctx->d_m, out, ctx->stream));
    } else {
        if (!ctx->d_nat) HIPCK(hipMalloc(&ctx->d_nat, sizeof(float) * 3 * (size_t)ctx->N));
        HIPCK(launch_from_split(ctx->args, ctx->d_m, ctx->d_nat, ctx->stream));
        HIPCK(hipMemcpyAsync(out, ctx->d_nat, sizeof(float) * 3 * (size_t)ctx->N, hipMemcpyDeviceToHost, ctx->stream));
    }
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MMC_OK;
}

// Sweep calls of at least kSweepGraph sweeps replay a HIP graph of
// kSweepGraph sweeps' launches (captured from the chain's stream once, and
// again after any change of kernel arguments), then enqueue the rest
// directly: the same kernels in the same order, so the same bits, without the
// host's per-launch cost, which bounds small chains (a sweep is five to nine
// launches).  MMC_SWEEP_GRAPH=0 in the environment at mmc_sweep keeps direct
// launches.
static constexpr int kSweepGraph = 16;

// *ready tells whether a current graph exists; a stream that refuses capture
// or a graph that does not instantiate leaves it false (the caller then
// launches directly), a failed launch during capture is an error.
static mmc_status sweep_graph_ready(mmc_ctx* ctx, bool* ready) {
    *ready = ctx->sg_exec && ctx->sg_version == ctx->version;
    if (*ready) return MMC_OK;
    if (ctx->sg_exec) { (void)hipGraphExecDestroy(ctx->sg_exec); ctx->sg_exec = nullptr; }
    if (ctx->sg_graph) { (void)hipGraphDestroy(ctx->sg_graph); ctx->sg_graph = nullptr; }
    if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return MMC_OK;
    }
    const mmc_status st = enqueue_core(ctx, single(ctx), kSweepGraph, ctx->stream, nullptr, 0, nullptr);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->stream, &gr);
    if (st != MMC_OK) { if (gr) (void)hipGraphDestroy(gr); return st; }
    if (e != hipSuccess || !gr) {
        (void)hipGetLastError();
        return MMC_OK;
    }
    ctx->sg_graph = gr;
    if (hipGraphInstantiate(&ctx->sg_exec, ctx->sg_graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        ctx->sg_exec = nullptr;
        return MMC_OK;
    }
    ctx->sg_version = ctx->version;
    *ready = true;
    return MMC_OK;
}

mmc_status mmc_sweep(mmc_ctx* ctx, int32_t n) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (n < 0) return fail(MMC_ERR_ARG, "negative sweep count");
    const char* env = getenv("MMC_SWEEP_GRAPH");
    if (n < kSweepGraph || (env && env[0] == '0')) return enqueue_sweeps(ctx, n, nullptr, 0);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCK(hipStreamIsCapturing(ctx->stream, &cap));
    if (cap != hipStreamCaptureStatusNone) return enqueue_sweeps(ctx, n, nullptr, 0);   // into the caller's capture
    bool ready = false;
    s = sweep_graph_ready(ctx, &ready);
    if (s != MMC_OK) return s;
    if (!ready) return enqueue_sweeps(ctx, n, nullptr, 0);
    const int reps = n / kSweepGraph;
    for (int r = 0; r < reps; ++r) HIPCK(hipGraphLaunch(ctx->sg_exec, ctx->stream));
    ctx->host_sweep += (unsigned long long)reps * kSweepGraph;
    return enqueue_sweeps(ctx, n - reps * kSweepGraph, nullptr, 0);
}

mmc_status mmc_sweep_timed(mmc_ctx* ctx, int32_t n, int32_t every, double ms_out[6], int32_t launches_out[6]) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (n < 0 || every < 1 || !ms_out || !launches_out) return fail(MMC_ERR_ARG, "bad count, sampling or NULL output");
    LaunchProf prof;
    prof.every = every;
    const size_t per_sweep = 2 * (ctx->demag ? 3 : 0) + 3;
    const size_t sampled = ((size_t)n + every - 1) / every;
    prof.ev.resize(2 * per_sweep * sampled + 2);
    mmc_status st = MMC_OK;
    size_t made = 0;
    for (; made < prof.ev.size(); ++made)
        if (hipEventCreate(&prof.ev[made]) != hipSuccess) { st = fail(MMC_ERR_DEVICE, "event creation failed"); break; }
    if (st == MMC_OK) st = enqueue_sweeps(ctx, n, nullptr, 0, &prof);
    if (st == MMC_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(MMC_ERR_DEVICE, "synchronize failed");
    for (int k = 0; k < 6; ++k) { ms_out[k] = 0.0; launches_out[k] = 0; }
    if (st == MMC_OK) {
        for (size_t i = 0; i < prof.kind.size(); ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, prof.ev[2 * i], prof.ev[2 * i + 1]) != hipSuccess) {
                st = fail(MMC_ERR_DEVICE, "event timing failed");
                break;
            }
            ms_out[prof.kind[i]] += ms;
            launches_out[prof.kind[i]] += 1;
        }
    }
    for (size_t i = 0; i < made; ++i) (void)hipEventDestroy(prof.ev[i]);
    return st;
}

mmc_status mmc_sweep_record(mmc_ctx* ctx, int32_t n, double* series) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (n < 0 || (n > 0 && !series)) return fail(MMC_ERR_ARG, "bad count or NULL series");
    if (n == 0) return MMC_OK;
    if (ctx->series_cap < n) {
        if (ctx->d_series) HIPCK(hipFree(ctx->d_series));
        ctx->d_series = nullptr;
        HIPCK(hipMalloc(&ctx->d_series, sizeof(double) * 5 * (size_t)n));
        ctx->series_cap = n;
    }
    // rows are indexed by the device's sweep counter minus its value now (read
    // back rather than tracked on the host: graphs the caller replays advance it)
    HIPCK(hipStreamSynchronize(ctx->stream));
    DevState hs{};
    HIPCK(hipMemcpy(&hs, ctx->d_st, sizeof hs, hipMemcpyDeviceToHost));
    ctx->host_sweep = hs.sweep;
    s = enqueue_sweeps(ctx, n, ctx->d_series, hs.sweep);
    if (s != MMC_OK) return s;
    HIPCK(hipMemcpyAsync(series, ctx->d_series, sizeof(double) * 5 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MMC_OK;
}

mmc_status mmc_demag_field(mmc_ctx* ctx, float* h_out, int on_device) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!h_out) return fail(MMC_ERR_ARG, "NULL output");
    if (!ctx->demag) return fail(MMC_ERR_STATE, "demag is off for this context");
    HIPCK(launch_demag(ctx->args, ctx->plan, single(ctx), 3, ctx->d_tw, ctx->stream));
    float* dst = on_device ? h_out : nullptr;
    if (!on_device) {
        if (!ctx->d_nat) HIPCK(hipMalloc(&ctx->d_nat, sizeof(float) * 3 * (size_t)ctx->N));
        dst = ctx->d_nat;
    }
    HIPCK(launch_from_split(ctx->args, ctx->d_h, dst, ctx->stream));
    if (!on_device)
        HIPCK(hipMemcpyAsync(h_out, dst, sizeof(float) * 3 * (size_t)ctx->N, hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MMC_OK;
}

mmc_status mmc_energy(mmc_ctx* ctx, double* E_total, double E_terms[6]) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!E_total && !E_terms) return fail(MMC_ERR_ARG, "NULL outputs");
    if (ctx->demag) HIPCK(launch_demag(ctx->args, ctx->plan, single(ctx), 3, ctx->d_tw, ctx->stream));
    const int blocks = (int)std::min<long long>((ctx->N + 255) / 256, 2048);
    if (ctx->epart_n < blocks) {
        if (ctx->d_epart) HIPCK(hipFree(ctx->d_epart));
        ctx->d_epart = nullptr;
        HIPCK(hipMalloc(&ctx->d_epart, sizeof(double) * 6 * blocks));
        ctx->epart_n = blocks;
    }
    int nb = 0;
    HIPCK(launch_energy(ctx->args, ctx->has_classes, ctx->cubic, ctx->d_ctab, ctx->d_cid, ctx->d_m, ctx->demag ? ctx->d_h : nullptr,
                        ctx->d_epart, ctx->stream, &nb));
    std::vector<double> part(6 * (size_t)nb);
    HIPCK(hipMemcpyAsync(part.data(), ctx->d_epart, sizeof(double) * part.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    const double kT = kB * ctx->run.T;
    double t[6] = {0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < 6; ++k) t[k] += part[6 * b + k];
    double tot = 0;
    for (int k = 0; k < 6; ++k) { t[k] *= kT; tot += t[k]; }
    if (E_terms) for (int k = 0; k < 6; ++k) E_terms[k] = t[k];
    if (E_total) *E_total = tot;
    return MMC_OK;
}

mmc_status mmc_energy_noalloc(mmc_ctx* ctx, double* out_device) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!out_device) return fail(MMC_ERR_ARG, "NULL output");
    double* part = energy_scratch(ctx->device);
    if (!part) return fail(MMC_ERR_STATE, "energy scratch of device %d is not set up", ctx->device);
    const long long blocks = std::min<long long>((ctx->N + 255) / 256, kEnergyMaxBlocks);
    if (blocks > kEnergyMaxBlocks)
        return fail(MMC_ERR_UNSUPPORTED, "energy needs %lld partial sums, the scratch holds %d", blocks, kEnergyMaxBlocks);
    if (ctx->demag) HIPCK(launch_demag(ctx->args, ctx->plan, single(ctx), 3, ctx->d_tw, ctx->stream));
    int nb = 0;
    HIPCK(launch_energy(ctx->args, ctx->has_classes, ctx->cubic, ctx->d_ctab, ctx->d_cid, ctx->d_m,
                        ctx->demag ? ctx->d_h : nullptr, part, ctx->stream, &nb));
    HIPCK(launch_energy_sum(part, nb, kB * ctx->run.T, out_device, ctx->stream));
    return MMC_OK;
}

mmc_status mmc_subsweep(mmc_ctx* ctx, int32_t colour, const float* h_in, uint8_t* acc_out) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (colour != 0 && colour != 1) return fail(MMC_ERR_ARG, "colour must be 0 or 1");
    if (!acc_out) return fail(MMC_ERR_ARG, "NULL decision output");
    HIPCK(hipMemsetAsync(acc_out, 255, (size_t)ctx->N, ctx->stream));
    if (h_in) HIPCK(launch_to_split(ctx->args, h_in, ctx->d_h, ctx->stream));
    HIPCK(launch_pass(ctx->args, ctx->has_classes, h_in != nullptr, ctx->run.lenmove == MMC_LEN_EXACT,
                      ctx->mat.D0 != 0.0, ctx->cubic, single(ctx), colour, false, ctx->fp_shift, acc_out, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MMC_OK;
}

mmc_status mmc_get_tuning(mmc_ctx* ctx, int32_t rows_per_thread[2], double us_per_launch[6], int32_t* fused,
                          double fuse_us[3]) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!rows_per_thread) return fail(MMC_ERR_ARG, "NULL output");
    if (!ctx->demag) return fail(MMC_ERR_STATE, "demag is off for this context");
    rows_per_thread[0] = ctx->plan.rpt_f;
    rows_per_thread[1] = ctx->plan.rpt_i;
    if (us_per_launch) std::copy(ctx->xtune_us, ctx->xtune_us + 6, us_per_launch);
    if (fused) *fused = fused_form(ctx);
    if (fuse_us) std::copy(ctx->fuse_us, ctx->fuse_us + 3, fuse_us);
    return MMC_OK;
}

mmc_status mmc_get_stats(mmc_ctx* ctx, mmc_stats* out) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!out) return fail(MMC_ERR_ARG, "NULL output");
    DevState hs{};
    HIPCK(hipMemcpyAsync(&hs, ctx->d_st, sizeof hs, hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    out->sweeps = hs.sweep;
    out->accepts_window = hs.window;
    out->cone_deg = hs.cone_deg;
    out->sigma = ctx->ctab[0].sigma;
    out->me = std::sqrt(ctx->ctab[0].me2);
    for (int k = 0; k < 3; ++k) out->m_mean[k] = hs.last[k];
    out->m2_mean = hs.last[3];
    out->accepts_last = hs.accepts_last;
    return MMC_OK;
}

mmc_status mmc_take_averages(mmc_ctx* ctx, double avg_out[4], uint64_t* n_out) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (!avg_out || !n_out) return fail(MMC_ERR_ARG, "NULL output");
    DevState hs{};
    HIPCK(hipMemcpyAsync(&hs, ctx->d_st, sizeof hs, hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 4; ++k) avg_out[k] = hs.avg_n ? hs.avg_sum[k] / (double)hs.avg_n : 0.0;
    *n_out = hs.avg_n;
    // reset only the accumulators (the rest of the state is left as the device has it)
    const double zsum[4] = {0.0, 0.0, 0.0, 0.0};
    const unsigned long long zn = 0;
    HIPCK(hipMemcpy((char*)ctx->d_st + offsetof(DevState, avg_sum), zsum, sizeof zsum, hipMemcpyHostToDevice));
    HIPCK(hipMemcpy((char*)ctx->d_st + offsetof(DevState, avg_n), &zn, sizeof zn, hipMemcpyHostToDevice));
    return MMC_OK;
}

mmc_status mmc_get_state(mmc_ctx* ctx, uint64_t* sweep, int32_t* cone_deg, uint64_t* accepts_window) {
    mmc_stats st{};
    mmc_status s = mmc_get_stats(ctx, &st);
    if (s != MMC_OK) return s;
    if (sweep) *sweep = st.sweeps;
    if (cone_deg) *cone_deg = st.cone_deg;
    if (accepts_window) *accepts_window = st.accepts_window;
    return MMC_OK;
}

mmc_status mmc_set_state(mmc_ctx* ctx, uint64_t sweep, int32_t cone_deg, uint64_t accepts_window) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    if (cone_deg < 1 || cone_deg > 180) return fail(MMC_ERR_ARG, "cone_deg must be in [1, 180]");
    HIPCK(hipStreamSynchronize(ctx->stream));
    DevState hs{};
    HIPCK(hipMemcpy(&hs, ctx->d_st, sizeof hs, hipMemcpyDeviceToHost));
    hs.sweep = sweep;
    hs.window = accepts_window;
    hs.cone_deg = cone_deg;
    const double sh = std::sin(0.5 * cone_deg * kPi / 180.0);
    hs.omc = (float)(2.0 * sh * sh);
    HIPCK(hipMemcpy(ctx->d_st, &hs, sizeof hs, hipMemcpyHostToDevice));
    ctx->host_sweep = sweep;
    return MMC_OK;
}

mmc_status mmc_sync(mmc_ctx* ctx) {
    mmc_status s = check_live(ctx);
    if (s != MMC_OK) return s;
    HIPCK(hipStreamSynchronize(ctx->stream));
    return MMC_OK;
}

// ---------------------------------------------------------------------
// Batches: chains are grouped by shape (grid, cell, material classes on/off,
// demag and its cadence, move kind, DMI on/off); each group advances in
// shared launches (chain = blockIdx.y) on a stream of its own, the groups
// forked from and joined back to the first chain's stream.  The sequence is
// captured once as a HIP graph and replayed.
// ---------------------------------------------------------------------
mmc_status mmc_batch_create(mmc_ctx* const* chains, int32_t n, mmc_batch** out) {
    mmc_ctx* ctx = nullptr;
    if (!chains || n < 1 || !out) return fail(MMC_ERR_ARG, "need at least one chain");
    for (int i = 0; i < n; ++i) {
        if (!chains[i]) return fail(MMC_ERR_ARG, "NULL chain %d", i);
        if (chains[i]->dead) return fail(MMC_ERR_STATE, "chain %d had a device error", i);
        if (chains[i]->device != chains[0]->device) return fail(MMC_ERR_ARG, "chains on different devices");
        for (int j = 0; j < i; ++j)
            if (chains[j] == chains[i]) return fail(MMC_ERR_ARG, "chain %d listed twice", i);
    }
    mmc_batch* b = new (std::nothrow) mmc_batch();
    if (!b) return fail(MMC_ERR_OOM, "host allocation failed");
    b->ch.assign(chains, chains + n);
    HIPCK(hipSetDevice(chains[0]->device));
    bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&b->joined, hipEventDisableTiming) == hipSuccess;
    b->chain_ev.assign(n, nullptr);
    for (int i = 0; ok && i < n; ++i) ok = hipEventCreateWithFlags(&b->chain_ev[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        mmc_batch_destroy(b);
        return fail(MMC_ERR_DEVICE, "event creation failed");
    }
    *out = b;
    return MMC_OK;
}

static void batch_drop_graph(mmc_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_n = -1;
    b->graph_sched = -1;
}

static bool same_shape(const mmc_ctx* a, const mmc_ctx* c) {
    return a->g.nx == c->g.nx && a->g.ny == c->g.ny && a->g.nz == c->g.nz && a->cs.hx == c->cs.hx &&
           a->cs.hy == c->cs.hy && a->cs.hz == c->cs.hz && a->has_classes == c->has_classes &&
           a->demag == c->demag && (!a->demag || a->run.refresh_per_sweep == c->run.refresh_per_sweep) &&
           a->run.demag == c->run.demag &&
           a->run.lenmove == c->run.lenmove && (a->mat.D0 != 0.0) == (c->mat.D0 != 0.0) && a->cubic == c->cubic;
}

// Regroups the chains and uploads each group's descriptors.
static mmc_status batch_regroup(mmc_batch* b) {
    mmc_ctx* ctx = nullptr;
    for (auto& g : b->groups)
        if (g.d_list) HIPCK(hipFree(g.d_list));
    b->groups.clear();
    for (int i = 0; i < (int)b->ch.size(); ++i) {
        bool placed = false;
        for (auto& g : b->groups)
            if (same_shape(b->ch[g.idx[0]], b->ch[i])) { g.idx.push_back(i); placed = true; break; }
        if (!placed) b->groups.push_back(BatchGroup{{i}, nullptr});
    }
    for (auto& g : b->groups) {
        std::vector<ChainDesc> h(g.idx.size());
        for (size_t k = 0; k < g.idx.size(); ++k) h[k] = make_desc(b->ch[g.idx[k]]);
        HIPCK(hipMalloc(&g.d_list, sizeof(ChainDesc) * h.size()));
        HIPCK(hipMemcpy(g.d_list, h.data(), sizeof(ChainDesc) * h.size(), hipMemcpyHostToDevice));
    }
    while (b->streams.size() < b->groups.size()) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        HIPCK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        b->streams.push_back(st);
        HIPCK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        b->done.push_back(ev);
    }
    return MMC_OK;
}

// The persistent schedule is switched off: its launches did not finish on
// the GPU and the cause is not found yet.  Requests for it are refused and the
// automatic choice is the grouped form.
static constexpr bool kPersistEnabled = false;

// The persistent kernel serves uniform materials without DMI, FP32 or no
// demag with 1 or 2 layers, and one length-move kind across the batch.
static bool batch_persist_ok(const mmc_batch* b) {
    if (!kPersistEnabled) return false;
    for (const mmc_ctx* c : b->ch) {
        if (c->has_classes || c->cubic || c->mat.D0 != 0.0) return false;
        if (c->run.demag != MMC_DEMAG_OFF && c->run.demag != MMC_DEMAG_FP32) return false;
        if (c->run.lenmove != b->ch[0]->run.lenmove) return false;
        if (!persist_shape_ok(c->g.nx, c->g.ny, c->g.nz, c->demag)) return false;
    }
    return true;
}

static std::string batch_signature(const mmc_batch* b) {
    std::vector<std::string> parts;
    char buf[160];
    for (const mmc_ctx* c : b->ch) {
        snprintf(buf, sizeof buf, "%d,%d,%d,%.6g,%.6g,%.6g,%d,%d,%d", c->g.nx, c->g.ny, c->g.nz, c->cs.hx, c->cs.hy,
                 c->cs.hz, c->run.demag, c->run.refresh_per_sweep, c->run.lenmove);
        parts.push_back(buf);
    }
    std::sort(parts.begin(), parts.end());
    std::string sig;
    for (auto& p : parts) sig += p + ";";
    return sig;
}

static mmc_status batch_build_persist(mmc_batch* b) {
    mmc_ctx* ctx = nullptr;
    if (b->pplan_ok) return MMC_OK;
    std::vector<PersistChain> pcs(b->ch.size());
    for (size_t i = 0; i < b->ch.size(); ++i) {
        const mmc_ctx* c = b->ch[i];
        PersistChain& q = pcs[i];
        q.cd = make_desc(c);
        q.K = c->plan.K;
        q.tw = c->d_tw;
        q.L = c->plan.L;
        q.Py = c->plan.Py;
        q.demag = c->demag;
        q.refresh_per_sweep = c->run.refresh_per_sweep;
        q.shift = c->fp_shift;
    }
    b->pplan.exact = b->ch[0]->run.lenmove == MMC_LEN_EXACT;
    const hipError_t e = persist_build(pcs.data(), (int)pcs.size(), &b->pplan);
    if (e != hipSuccess) {
        persist_free(&b->pplan);
        return fail(MMC_ERR_DEVICE, "persistent plan: %s", hipGetErrorString(e));
    }
    HIPCK(hipMemset(b->pplan.err, 0, sizeof(int)));
    b->pplan_ok = true;
    return MMC_OK;
}

// Time limit of one wait in the persistent kernel (s): far above any phase.
static constexpr double kPersistWaitLimit = 5.0;

// Captures n sweeps of every chain under schedule sched as one graph on the
// first chain's stream.
static mmc_status batch_capture(mmc_batch* b, int n, int sched) {
    mmc_ctx* ctx = nullptr;
    batch_drop_graph(b);
    // a chain's own stream may hold earlier work: order it before the graph
    for (auto* c : b->ch) HIPCK(hipStreamSynchronize(c->stream));
    mmc_status st = MMC_OK;
    if (sched == MMC_SCHED_PERSISTENT) {
        // descriptors change with T, field or grains: rebuild the plan
        if (b->pplan_ok) { persist_free(&b->pplan); b->pplan_ok = false; }
        st = batch_build_persist(b);
    } else {
        st = batch_regroup(b);
    }
    if (st != MMC_OK) return st;
    hipStream_t s0 = b->ch[0]->stream;
    HIPCK(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
    if (sched == MMC_SCHED_PERSISTENT) {
        const hipError_t e = persist_launch(b->pplan, n, kPersistWaitLimit, s0);
        if (e != hipSuccess) st = fail(MMC_ERR_DEVICE, "persistent launch: %s", hipGetErrorString(e));
    } else {
        HIPCK(hipEventRecord(b->fork, s0));
        for (size_t gi = 0; gi < b->groups.size() && st == MMC_OK; ++gi) {
            const BatchGroup& g = b->groups[gi];
            HIPCK(hipStreamWaitEvent(b->streams[gi], b->fork, 0));
            const mmc_ctx* c0 = b->ch[g.idx[0]];
            st = enqueue_core(b->ch[g.idx[0]], Chains{make_desc(c0), g.d_list, (int)g.idx.size()}, n,
                              b->streams[gi], nullptr, 0, nullptr);
            if (st != MMC_OK) break;
            HIPCK(hipEventRecord(b->done[gi], b->streams[gi]));
            HIPCK(hipStreamWaitEvent(s0, b->done[gi], 0));
        }
    }
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(s0, &gr);
    if (st != MMC_OK) { if (gr) (void)hipGraphDestroy(gr); return st; }
    HIPCK(e);
    b->graph = gr;
    HIPCK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_n = n;
    b->graph_sched = sched;
    b->versions.resize(b->ch.size());
    for (size_t i = 0; i < b->ch.size(); ++i) b->versions[i] = b->ch[i]->version;
    return MMC_OK;
}

// State of the chains (m, run state, statistics accumulators) for trial runs.
struct BatchSnapshot {
    std::vector<void*> buf;
};
static mmc_status batch_snapshot(mmc_batch* b, BatchSnapshot& sn, bool restore) {
    mmc_ctx* ctx = nullptr;
    if (!restore) sn.buf.assign(b->ch.size(), nullptr);
    for (size_t i = 0; i < b->ch.size(); ++i) {
        const mmc_ctx* c = b->ch[i];
        const size_t mb = sizeof(float) * 6 * (size_t)c->Nc;
        const size_t tot = mb + sizeof(DevState) + sizeof(SweepAccum);
        if (!restore) HIPCK(hipMalloc(&sn.buf[i], tot));
        char* p = (char*)sn.buf[i];
        const hipMemcpyKind k = hipMemcpyDeviceToDevice;
        if (restore) {
            HIPCK(hipMemcpy(c->d_m, p, mb, k));
            HIPCK(hipMemcpy(c->d_st, p + mb, sizeof(DevState), k));
            HIPCK(hipMemcpy(c->d_acc, p + mb + sizeof(DevState), sizeof(SweepAccum), k));
        } else {
            HIPCK(hipMemcpy(p, c->d_m, mb, k));
            HIPCK(hipMemcpy(p + mb, c->d_st, sizeof(DevState), k));
            HIPCK(hipMemcpy(p + mb + sizeof(DevState), c->d_acc, sizeof(SweepAccum), k));
        }
    }
    return MMC_OK;
}
static void batch_snapshot_free(BatchSnapshot& sn) {
    for (void* p : sn.buf) if (p) (void)hipFree(p);
    sn.buf.clear();
}

// Automatic schedule: times a few sweeps of each form from the same state
// (which is restored afterwards, so the chains continue bit for bit) and keeps
// the faster; the choice is cached per batch signature.
static mmc_status batch_tune(mmc_batch* b) {
    mmc_ctx* ctx = nullptr;
    const std::string sig = batch_signature(b);
    {
        std::lock_guard<std::mutex> lk(g_sched_mu);
        auto it = g_sched_cache.find(sig);
        if (it != g_sched_cache.end()) { b->sched_used = it->second; b->tuned = true; return MMC_OK; }
    }
    constexpr int kTrial = 3;
    for (auto* c : b->ch) HIPCK(hipStreamSynchronize(c->stream));
    BatchSnapshot sn;
    mmc_status st = batch_snapshot(b, sn, false);
    hipStream_t s0 = b->ch[0]->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == MMC_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(MMC_ERR_DEVICE, "event creation failed");
    for (int sched = MMC_SCHED_GROUPS; st == MMC_OK && sched <= MMC_SCHED_PERSISTENT; ++sched) {
        st = batch_capture(b, kTrial, sched);
        for (int rep = 0; st == MMC_OK && rep < 2; ++rep) {   // warm-up, then timed
            if (hipEventRecord(e0, s0) != hipSuccess || hipGraphLaunch(b->exec, s0) != hipSuccess ||
                hipEventRecord(e1, s0) != hipSuccess || hipStreamSynchronize(s0) != hipSuccess) {
                st = fail(MMC_ERR_DEVICE, "trial launch failed");
                break;
            }
            if (sched == MMC_SCHED_PERSISTENT) {
                int err = 0;
                if (hipMemcpy(&err, b->pplan.err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess || err)
                    st = fail(MMC_ERR_DEVICE, "persistent trial: a wait exceeded its time limit");
            }
            float ms = 0.f;
            if (st == MMC_OK) (void)hipEventElapsedTime(&ms, e0, e1);
            b->tune_ms[sched - 1] = ms;
            if (st == MMC_OK) st = batch_snapshot(b, sn, true);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    batch_snapshot_free(sn);
    batch_drop_graph(b);
    if (st != MMC_OK) {
        for (auto* c : b->ch) c->dead = true;
        return st;
    }
    b->sched_used = b->tune_ms[1] < b->tune_ms[0] ? MMC_SCHED_PERSISTENT : MMC_SCHED_GROUPS;
    b->tuned = true;
    std::lock_guard<std::mutex> lk(g_sched_mu);
    g_sched_cache[sig] = b->sched_used;
    return MMC_OK;
}

mmc_status mmc_batch_set_schedule(mmc_batch* b, int32_t sched) {
    mmc_ctx* ctx = nullptr;
    if (!b) return fail(MMC_ERR_ARG, "NULL batch");
    if (sched < MMC_SCHED_AUTO || sched > MMC_SCHED_PERSISTENT) return fail(MMC_ERR_ARG, "unknown schedule %d", sched);
    HIPCK(hipSetDevice(b->ch[0]->device));
    if (sched == MMC_SCHED_PERSISTENT && !kPersistEnabled)
        return fail(MMC_ERR_UNSUPPORTED, "the persistent schedule is switched off in this build");
    if (sched == MMC_SCHED_PERSISTENT && !batch_persist_ok(b))
        return fail(MMC_ERR_UNSUPPORTED,
                    "persistent schedule needs uniform materials without DMI, FP32 or no demag with nz 1 or 2, "
                    "x lengths 17..1024 and y lengths 17..512 with demag, and one length-move kind");
    b->sched_req = sched;
    b->tuned = false;
    if (sched != MMC_SCHED_AUTO) b->sched_used = sched;
    batch_drop_graph(b);
    return MMC_OK;
}

mmc_status mmc_batch_get_schedule(mmc_batch* b, int32_t* used, double trial_ms[2]) {
    mmc_ctx* ctx = nullptr;
    if (!b || !used) return fail(MMC_ERR_ARG, "NULL argument");
    *used = b->sched_used;
    if (trial_ms) { trial_ms[0] = b->tune_ms[0]; trial_ms[1] = b->tune_ms[1]; }
    return MMC_OK;
}

mmc_status mmc_batch_sweep(mmc_batch* b, int32_t n) {
    mmc_ctx* ctx = nullptr;
    if (!b) return fail(MMC_ERR_ARG, "NULL batch");
    if (n < 0) return fail(MMC_ERR_ARG, "negative sweep count");
    if (n == 0) return MMC_OK;
    for (auto* c : b->ch)
        if (c->dead) return fail(MMC_ERR_STATE, "a chain had a device error");
    HIPCK(hipSetDevice(b->ch[0]->device));
    // schedule: the requested one, or the tuned choice (groups when the
    // persistent kernel does not serve these chains)
    if (b->sched_req == MMC_SCHED_AUTO && !b->tuned) {
        if (batch_persist_ok(b)) {
            mmc_status st = batch_tune(b);
            if (st != MMC_OK) return st;
        } else {
            b->sched_used = MMC_SCHED_GROUPS;
            b->tuned = true;
        }
    }
    if (b->sched_used == MMC_SCHED_PERSISTENT && !batch_persist_ok(b)) {
        if (b->sched_req == MMC_SCHED_PERSISTENT)
            return fail(MMC_ERR_UNSUPPORTED, "the chains no longer suit the persistent schedule");
        b->sched_used = MMC_SCHED_GROUPS;
    }
    bool stale = b->graph_n != n || b->graph_sched != b->sched_used || b->versions.size() != b->ch.size();
    for (size_t i = 0; !stale && i < b->ch.size(); ++i) stale = b->versions[i] != b->ch[i]->version;
    hipStream_t s0 = b->ch[0]->stream;
    if (stale) {
        mmc_status st = batch_capture(b, n, b->sched_used);
        if (st != MMC_OK) return st;
    }
    // work queued earlier on a chain's own stream (mmc_sweep, setters) runs
    // before the graph, and later work on that stream (getters, sweeps) after it
    for (size_t i = 0; i < b->ch.size(); ++i) {
        if (b->ch[i]->stream == s0) continue;
        HIPCK(hipEventRecord(b->chain_ev[i], b->ch[i]->stream));
        HIPCK(hipStreamWaitEvent(s0, b->chain_ev[i], 0));
    }
    HIPCK(hipGraphLaunch(b->exec, s0));
    HIPCK(hipEventRecord(b->joined, s0));
    for (auto* c : b->ch)
        if (c->stream != s0) HIPCK(hipStreamWaitEvent(c->stream, b->joined, 0));
    for (auto* c : b->ch) c->host_sweep += (unsigned long long)n;
    return MMC_OK;
}

mmc_status mmc_batch_sync(mmc_batch* b) {
    mmc_ctx* ctx = nullptr;
    if (!b) return fail(MMC_ERR_ARG, "NULL batch");
    HIPCK(hipSetDevice(b->ch[0]->device));
    HIPCK(hipStreamSynchronize(b->ch[0]->stream));
    if (b->pplan_ok) {
        int err = 0;
        HIPCK(hipMemcpy(&err, b->pplan.err, sizeof(int), hipMemcpyDeviceToHost));
        if (err) {
            for (auto* c : b->ch) c->dead = true;
            return fail(MMC_ERR_DEVICE, "persistent batch: a wait exceeded its time limit; the chains are unusable");
        }
    }
    return MMC_OK;
}

void mmc_batch_destroy(mmc_batch* b) {
    if (!b) return;
    if (!b->ch.empty()) {
        (void)hipSetDevice(b->ch[0]->device);
        (void)hipStreamSynchronize(b->ch[0]->stream);
    }
    batch_drop_graph(b);
    if (b->pplan_ok) persist_free(&b->pplan);
    for (auto& g : b->groups) if (g.d_list) (void)hipFree(g.d_list);
    for (auto s : b->streams) if (s) (void)hipStreamDestroy(s);
    for (auto e : b->done) if (e) (void)hipEventDestroy(e);
    for (auto e : b->chain_ev) if (e) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->joined) (void)hipEventDestroy(b->joined);
    delete b;
}

}  // extern "C"
