// Persistent batched sweeps: one kernel launch advances every chain of a
// batch by n sweeps (paper Sec. II steps 1-4 with the Sec. III demag refresh,
// per chain exactly as the single-chain launch sequence).
//
// Work items are (sweep s, phase slot p, chain c, tile t), numbered sweep by
// sweep, within a sweep slot by slot, within a slot chain by chain.  The nine
// slots of a sweep are x-forward, y pass, x-inverse, colour pass 0, the same
// three demag stages again, colour pass 1 and the end-of-sweep reduction; a
// chain has no tiles in the slots it does not use (no demag, or one refresh
// per sweep).  Blocks take items from a global counter in that order.  Before
// its item a block waits until its chain has completed every item of its
// earlier slots (a per-chain count, released and acquired at device scope);
// those items have lower numbers and are held by blocks that are already
// running, so the waits always end.  A waiting block polls its count with
// relaxed loads and acquires once the count is reached (an acquire load in the
// poll loop would invalidate its XCD's L2 on every poll and starve the blocks
// doing work).  Each wait, and the whole launch, is also bounded in time: past
// a limit the block raises the error flag and every block leaves, which the
// host reports as a device error.
//
// The tiles are the blocks of the single-chain kernels, run by the same
// bodies, so a batch gives the same bits as its chains run alone.  y passes
// whose thread group is narrower than the 256-thread block run several kx per
// block, one group each, with their barriers kept uniform.
#include "demag_fft.h"
#include "sweep_kernels.h"

namespace mmc {

// slots of one sweep
enum { PS_XF0 = 0, PS_YP0, PS_XI0, PS_PASS0, PS_XF1, PS_YP1, PS_XI1, PS_PASS1, PS_END, PS_N };

struct PChain {
    ChainDesc cd;
    const float* K;        // tensor spectrum
    const float2* tw;      // twiddle tables
    long long N;
    int L, Py, nz, S;      // x half-length, padded y, layers, signals
    int xnt;               // x-pass row tiles per signal
    int vec4;              // colour pass with four cells per thread
    int dmg;               // demag on
    int mask0;             // x-inverse colour mask of the first refresh (1, or 3 for one refresh per sweep)
    int shift;             // fixed-point scale of the statistics
};

// tiles per slot for a chain (host and device)
__host__ __device__ inline int p_y_groups(int nz, int Py) {   // thread groups of the y pass per 256-thread block
    const int threads = (nz % 2 == 0 && Py / 8 >= 64 && Py / 8 <= 256) ? 2 * (Py / 8) : Py / 4;
    return 256 / threads;
}

template <int L>
__device__ __attribute__((noinline)) void p_xpass(const PChain& P, int inv, int mask, int t, int tid, float2* lds) {
    constexpr int RPT = x_RPT(L, 0);
    if (inv) xinv_body<L, RPT>(P.cd, P.S, P.xnt, mask, P.tw, t, tid, lds);
    else xfwd_body<L, RPT>(P.cd, P.S, P.xnt, P.tw, t, tid, lds);
}

template <int NZ, int PY>
__device__ __attribute__((noinline)) void p_ypass(const PChain& P, int t, int tid, float2* lds) {
    if constexpr (y2_use(NZ, PY)) {
        constexpr int TH = 2 * PY / y2_E(NZ), NSB = 256 / TH;
        const int sb = tid / TH;
        ypass2_body<NZ, PY, 0, true>(P.cd, P.K, P.tw, 0.f, t * NSB + sb, tid - sb * TH, P.L,
                                     lds + sb * (y2_lds_bytes<NZ, PY>(0) / (int)sizeof(float2)));
    } else {
        constexpr int TH = PY / y_E(NZ, PY), NSB = 256 / TH;
        const int sb = tid / TH;
        ypass_body<NZ, PY, true>(P.cd, P.K, P.tw, t * NSB + sb, tid - sb * TH, P.L, lds + sb * y1_lds(NZ, PY));
    }
}

template <int NZ>
__device__ __forceinline__ void p_ypass_nz(const PChain& P, int t, int tid, float2* lds) {
    switch (P.Py) {
        case 64: p_ypass<NZ, 64>(P, t, tid, lds); break;
        case 128: p_ypass<NZ, 128>(P, t, tid, lds); break;
        case 256: p_ypass<NZ, 256>(P, t, tid, lds); break;
        case 512: p_ypass<NZ, 512>(P, t, tid, lds); break;
        case 1024: p_ypass<NZ, 1024>(P, t, tid, lds); break;
        default: break;
    }
}

__device__ __forceinline__ void p_x(const PChain& P, int inv, int mask, int t, int tid, float2* lds) {
    switch (P.L) {
        case 32: p_xpass<32>(P, inv, mask, t, tid, lds); break;
        case 64: p_xpass<64>(P, inv, mask, t, tid, lds); break;
        case 128: p_xpass<128>(P, inv, mask, t, tid, lds); break;
        case 256: p_xpass<256>(P, inv, mask, t, tid, lds); break;
        case 512: p_xpass<512>(P, inv, mask, t, tid, lds); break;
        case 1024: p_xpass<1024>(P, inv, mask, t, tid, lds); break;
        default: break;
    }
}

template <bool EXACT>
__device__ __attribute__((noinline)) void p_pass(const PChain& P, int colour, int t, int tid) {
    if (P.vec4) {
        if (P.dmg) pass4_body<true, EXACT, false>(P.cd, colour, 1, P.shift, nullptr, t, tid);
        else pass4_body<false, EXACT, false>(P.cd, colour, 1, P.shift, nullptr, t, tid);
    } else {
        if (P.dmg) pass1_body<false, true, EXACT, false, false>(P.cd, colour, 1, P.shift, nullptr, t, tid);
        else pass1_body<false, false, EXACT, false, false>(P.cd, colour, 1, P.shift, nullptr, t, tid);
    }
}

__device__ __attribute__((noinline)) void p_end(const PChain& P, int tid) {
    end_sweep_body(P.cd, P.shift, P.N, nullptr, 0, tid);
}

// ctr[0]: next item; ctr[1 + c]: items completed by chain c.  off[k], k = p * nch
// + c: first item of (p, c) within a sweep (off[PS_N * nch] = W); pre[k]:
// items of chain c in slots before p; wc[c]: items of chain c per sweep.
template <bool EXACT>
__global__ __launch_bounds__(256, 2) void k_persist(const PChain* __restrict__ pc, const int* __restrict__ off,
                                                 const int* __restrict__ pre, const int* __restrict__ wc, int nch,
                                                 long long total, unsigned long long* ctr, int* err,
                                                 unsigned long long limit_ticks, unsigned long long deadline_ticks) {
    extern __shared__ float2 lds[];
    __shared__ long long s_item;
    __shared__ int s_go;
    const int tid = threadIdx.x;
    const int W = off[PS_N * nch];
    // s_memrealtime counts at 100 MHz
    const unsigned long long t_begin = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        if (tid == 0) {
            bool stop = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            if (!stop && __builtin_amdgcn_s_memrealtime() - t_begin > deadline_ticks) {
                __hip_atomic_store(err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                stop = true;
            }
            s_item = stop ? total : (long long)atomicAdd(&ctr[0], 1ull);
        }
        __syncthreads();
        const long long item = s_item;
        if (item >= total) break;
        const int s = (int)(item / W), r = (int)(item - (long long)s * W);
        int lo = 0, hi = PS_N * nch - 1;                  // largest k with off[k] <= r
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= r) lo = mid;
            else hi = mid - 1;
        }
        const int k = lo, p = k / nch, c = k - p * nch, t = r - off[k];
        if (tid == 0) {
            const unsigned long long need = (unsigned long long)s * (unsigned long long)wc[c] + (unsigned long long)pre[k];
            unsigned long long* done = &ctr[1 + c];
            int go = 1;
            if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
                while (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    __builtin_amdgcn_s_sleep(16);
                    const unsigned long long now = __builtin_amdgcn_s_memrealtime();
                    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        now - t0 > limit_ticks || now - t_begin > deadline_ticks) {
                        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        go = 0;
                        break;
                    }
                }
            }
            // the chain's earlier items are complete: see their writes
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_go = go;
        }
        __syncthreads();
        if (!s_go) break;
        const PChain& P = pc[c];
        switch (p) {
            case PS_XF0: case PS_XF1: p_x(P, 0, 0, t, tid, lds); break;
            case PS_XI0: p_x(P, 1, P.mask0, t, tid, lds); break;
            case PS_XI1: p_x(P, 1, 2, t, tid, lds); break;
            case PS_YP0: case PS_YP1:
                if (P.nz == 1) p_ypass_nz<1>(P, t, tid, lds);
                else p_ypass_nz<2>(P, t, tid, lds);
                break;
            case PS_PASS0: p_pass<EXACT>(P, 0, t, tid); break;
            case PS_PASS1: p_pass<EXACT>(P, 1, t, tid); break;
            default: p_end(P, tid); break;
        }
        __syncthreads();
        if (tid == 0)
            __hip_atomic_fetch_add(&ctr[1 + c], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// (the error flag is cleared only when the plan is built, so it stays raised
// across later launches until the host has seen it)
__global__ void k_persist_reset(unsigned long long* ctr, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) ctr[i] = 0ull;
}

// ---------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------
bool persist_shape_ok(int nx, int ny, int nz, bool demag) {
    if (!demag) return true;
    auto pad = [](int n) { int p = 1; while (p < 2 * n - 1) p *= 2; return p; };
    const int Px = std::max(pad(nx), 2), Py = pad(ny), L = Px / 2;
    return (nz == 1 || nz == 2) && L >= 32 && L <= 1024 && Py >= 64 && Py <= 1024 && L % p_y_groups(nz, Py) == 0;
}

// LDS bytes a chain's tiles need
static size_t persist_lds(const PChain& P) {
    if (!P.dmg) return 0;
    size_t xb = 0;
    switch (P.L) {
        case 32: xb = x_lds(32, x_RPT(32, 0)); break;
        case 64: xb = x_lds(64, x_RPT(64, 0)); break;
        case 128: xb = x_lds(128, x_RPT(128, 0)); break;
        case 256: xb = x_lds(256, x_RPT(256, 0)); break;
        case 512: xb = x_lds(512, x_RPT(512, 0)); break;
        default: xb = x_lds(1024, x_RPT(1024, 0)); break;
    }
    size_t yb = 0;
    const int g = p_y_groups(P.nz, P.Py);
    const bool two = P.nz % 2 == 0 && P.Py / 8 >= 64 && P.Py / 8 <= 256;
    if (two) yb = (size_t)g * (P.Py == 512 ? y2_lds_bytes<2, 512>(0) : y2_lds_bytes<2, 1024>(0));
    else {
        int one = 0;
        switch (P.Py) {
            case 64: one = P.nz == 1 ? y1_lds(1, 64) : y1_lds(2, 64); break;
            case 128: one = P.nz == 1 ? y1_lds(1, 128) : y1_lds(2, 128); break;
            case 256: one = P.nz == 1 ? y1_lds(1, 256) : y1_lds(2, 256); break;
            case 512: one = y1_lds(1, 512); break;
            default: one = y1_lds(1, 1024); break;
        }
        yb = (size_t)g * one * sizeof(float2);
    }
    return std::max(xb, yb);
}

hipError_t persist_build(const PersistChain* in, int n, PersistPlan* out) {
    out->nch = n;
    std::vector<PChain> pcs(n);
    std::vector<int> tiles((size_t)PS_N * n, 0);
    out->lds = 0;
    for (int c = 0; c < n; ++c) {
        const PersistChain& q = in[c];
        PChain& P = pcs[c];
        P.cd = q.cd;
        P.K = q.K;
        P.tw = q.tw;
        P.N = (long long)q.cd.a.nx * q.cd.a.ny * q.cd.a.nz;
        P.nz = q.cd.a.nz;
        P.dmg = q.demag ? 1 : 0;
        P.L = q.L;
        P.Py = q.Py;
        P.S = 3 * P.nz;
        P.vec4 = (q.cd.a.nx % 8 == 0) ? 1 : 0;
        P.shift = q.shift;
        P.mask0 = q.refresh_per_sweep >= 2 ? 1 : 3;
        const long long pthreads = (long long)q.cd.a.ny * q.cd.a.nz * (P.vec4 ? q.cd.a.hw / 4 : q.cd.a.hw);
        const int ptiles = (int)((pthreads + 255) / 256);
        int xt = 0, yt = 0;
        if (P.dmg) {
            int R = 0;
            switch (P.L) {
                case 32: R = x_rows_conc(32) * x_RPT(32, 0); break;
                case 64: R = x_rows_conc(64) * x_RPT(64, 0); break;
                case 128: R = x_rows_conc(128) * x_RPT(128, 0); break;
                case 256: R = x_rows_conc(256) * x_RPT(256, 0); break;
                case 512: R = x_rows_conc(512) * x_RPT(512, 0); break;
                default: R = x_rows_conc(1024) * x_RPT(1024, 0); break;
            }
            P.xnt = (q.cd.a.ny + R - 1) / R;
            xt = P.xnt * P.S;
            yt = P.L / p_y_groups(P.nz, P.Py);
        }
        int* tc = &tiles[0];
        const bool two = P.dmg && q.refresh_per_sweep >= 2;
        tc[PS_XF0 * n + c] = xt;
        tc[PS_YP0 * n + c] = yt;
        tc[PS_XI0 * n + c] = xt;
        tc[PS_PASS0 * n + c] = ptiles;
        tc[PS_XF1 * n + c] = two ? xt : 0;
        tc[PS_YP1 * n + c] = two ? yt : 0;
        tc[PS_XI1 * n + c] = two ? xt : 0;
        tc[PS_PASS1 * n + c] = ptiles;
        tc[PS_END * n + c] = 1;
        out->lds = std::max(out->lds, persist_lds(P));
    }
    std::vector<int> off((size_t)PS_N * n + 1), pre((size_t)PS_N * n), wc(n, 0);
    int acc = 0;
    for (int k = 0; k < PS_N * n; ++k) { off[k] = acc; acc += tiles[k]; }
    off[(size_t)PS_N * n] = acc;
    out->W = acc;
    for (int c = 0; c < n; ++c) {
        int a = 0;
        for (int p = 0; p < PS_N; ++p) { pre[p * n + c] = a; a += tiles[p * n + c]; }
        wc[c] = a;
    }
    out->host_off = off;
    out->host_pre = pre;
    out->host_wc = wc;
    const size_t bytes = sizeof(PChain) * n + sizeof(int) * (off.size() + pre.size() + wc.size()) +
                         sizeof(unsigned long long) * (n + 1) + 256;
    hipError_t e = hipMalloc(&out->mem, bytes + 64 * 5);
    if (e != hipSuccess) return e;
    char* base = (char*)out->mem;
    auto carve = [&](size_t b) { char* p = base; base += (b + 63) / 64 * 64; return (void*)p; };
    out->pc = carve(sizeof(PChain) * n);
    out->off = (int*)carve(sizeof(int) * off.size());
    out->pre = (int*)carve(sizeof(int) * pre.size());
    out->wc = (int*)carve(sizeof(int) * wc.size());
    out->ctr = (unsigned long long*)carve(sizeof(unsigned long long) * (n + 1));
    out->err = (int*)carve(sizeof(int));
    if ((e = hipMemcpy(out->pc, pcs.data(), sizeof(PChain) * n, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(out->off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(out->pre, pre.data(), sizeof(int) * pre.size(), hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(out->wc, wc.data(), sizeof(int) * wc.size(), hipMemcpyHostToDevice)) != hipSuccess) return e;
    int dev = 0, ncu = 0, per = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    const void* fn = out->exact ? (const void*)k_persist<true> : (const void*)k_persist<false>;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, out->lds)) != hipSuccess) return e;
    out->grid = std::max(1, per) * ncu;
    return hipSuccess;
}

hipError_t persist_launch(const PersistPlan& p, int nsweeps, double limit_s, hipStream_t s) {
    hipLaunchKernelGGL(k_persist_reset, dim3(1), dim3(64), 0, s, p.ctr, p.nch + 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long total = (long long)nsweeps * p.W;
    if (total <= 0) return hipSuccess;
    const unsigned long long ticks = (unsigned long long)(limit_s * 1e8);   // s_memrealtime runs at 100 MHz
    // the whole launch: 10 s plus 50 ms per sweep (a sweep of a batch takes about 1 ms)
    const unsigned long long deadline = (unsigned long long)((10.0 + 0.05 * nsweeps) * 1e8);
    const long long blocks = std::min<long long>(p.grid, total);
    if (p.exact)
        hipLaunchKernelGGL(k_persist<true>, dim3((unsigned)blocks), dim3(256), p.lds, s, (const PChain*)p.pc, p.off,
                           p.pre, p.wc, p.nch, total, p.ctr, p.err, ticks, deadline);
    else
        hipLaunchKernelGGL(k_persist<false>, dim3((unsigned)blocks), dim3(256), p.lds, s, (const PChain*)p.pc, p.off,
                           p.pre, p.wc, p.nch, total, p.ctr, p.err, ticks, deadline);
    return hipGetLastError();
}

void persist_free(PersistPlan* p) {
    if (p->mem) (void)hipFree(p->mem);
    *p = PersistPlan{};
}

}  // namespace mmc
