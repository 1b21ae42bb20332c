// Demag field h = -N * m by zero-padded FFT convolution (paper Sec. III,
// Eq. 14) for gfx950: FFT engine and kernel templates.
//
// Three launches per refresh:
//   x forward  rows of nx reals -> Px/2+1 complex bins (Px = padded length) via
//              a half-length complex FFT of z[n] = x[2n] + i x[2n+1]; with the
//              colour-split state x[2n] and x[2n+1] are slot n of the two
//              colour rows.  Output X[(k*S + s)*ny + y], S = 3*nz signals,
//              k < L; the bins k = 0 and k = L are real and travel packed as
//              X[0] + i X[L] in row 0.
//   y pass     one block per kx < L: FFT over padded y of all S signals,
//              direct mixing over layers with the tensor spectrum (all S
//              values of a bin sit in one thread's registers), inverse FFT,
//              crop.  Block 0 splits the packed pair into its two Hermitian
//              spectra before the mixing and packs the results after it.
//   x inverse  inverse of the first, writing h of the requested colours.
//
// FFT engine: mixed-radix Stockham, length N and E elements per thread fixed
// at compile time, data in registers in the strided layout x[j + T*m]
// (thread j < T = N/E, m < E).  Each pass is a radix-rho butterfly in
// registers; passes exchange through LDS; the last pass leaves the result in
// the same strided layout, so the layer mixing needs no exchange.  Twiddles
// come from tw[i] = exp(-2 pi i i / TW_N), computed in FP64 on the host.
#pragma once
#include "mmc_internal.h"

namespace mmc {

constexpr int TW_N = 8192;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) { return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }
// multiply by exp(-+ i pi/2): -i for the forward transform, +i for the inverse
template <bool INV> __device__ __forceinline__ float2 rot90(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// multiply by exp(-+ i theta) given (c, s) = (cos theta, sin theta)
template <bool INV> __device__ __forceinline__ float2 twc(float2 a, float c, float s) {
    return INV ? make_float2(a.x * c - a.y * s, a.x * s + a.y * c) : make_float2(a.x * c + a.y * s, a.y * c - a.x * s);
}

// LDS index with one slot of skew every 32 float2 (the 32 lanes that one
// 8-byte access serves per cycle cover the 64 banks once when their slots
// differ mod 32; one slot per 32 measured 3 % faster than one per 16 on the y
// pass, whose radix-8 first-pass writes it makes conflict-free); the
// per-signal stride is kept at 1 mod 32.  With power-of-two passes the
// outputs of a butterfly stay at lpad(base) + r*NSUB + (r*NSUB >> kSkew).
#ifndef MMC_LDS_SKEW
#define MMC_LDS_SKEW 5
#endif
constexpr int kSkew = MMC_LDS_SKEW, kSkewP = 1 << MMC_LDS_SKEW;   // one slot of skew per kSkewP slots
__device__ __forceinline__ int lpad(int i) { return i + (i >> kSkew); }
constexpr int lds_len(int n) {
    const int l = n - 1 + ((n - 1) >> kSkew) + 1;
    return l + ((kSkewP + 1 - l % kSkewP) % kSkewP);   // round up to 1 mod kSkewP
}

template <bool INV> __device__ __forceinline__ void dft2(float2* a) {
    const float2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
}
template <bool INV> __device__ __forceinline__ void dft4(float2* a) {
    const float2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    const float2 s13 = cadd(a[1], a[3]), d13 = rot90<INV>(csub(a[1], a[3]));
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, d13);
    a[3] = csub(d02, d13);
}
constexpr float kR2 = 0.70710678118654752440f;
constexpr float kC8 = 0.92387953251128675613f;   // cos(pi/8)
constexpr float kS8 = 0.38268343236508977173f;   // sin(pi/8)
template <bool INV> __device__ __forceinline__ void dft8(float2* a) {
    float2 e[4] = {a[0], a[2], a[4], a[6]}, o[4] = {a[1], a[3], a[5], a[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    o[1] = twc<INV>(o[1], kR2, kR2);
    o[2] = rot90<INV>(o[2]);
    o[3] = twc<INV>(o[3], -kR2, kR2);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = cadd(e[k], o[k]);
        a[k + 4] = csub(e[k], o[k]);
    }
}
template <bool INV> __device__ __forceinline__ void dft16(float2* a) {
    float2 e[8], o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) { e[k] = a[2 * k]; o[k] = a[2 * k + 1]; }
    dft8<INV>(e);
    dft8<INV>(o);
    o[1] = twc<INV>(o[1], kC8, kS8);
    o[2] = twc<INV>(o[2], kR2, kR2);
    o[3] = twc<INV>(o[3], kS8, kC8);
    o[4] = rot90<INV>(o[4]);
    o[5] = twc<INV>(o[5], -kS8, kC8);
    o[6] = twc<INV>(o[6], -kR2, kR2);
    o[7] = twc<INV>(o[7], -kC8, kS8);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = cadd(e[k], o[k]);
        a[k + 8] = csub(e[k], o[k]);
    }
}
template <int R, bool INV> __device__ __forceinline__ void dft(float2* a) {
    if constexpr (R == 2) dft2<INV>(a);
    else if constexpr (R == 4) dft4<INV>(a);
    else if constexpr (R == 8) dft8<INV>(a);
    else if constexpr (R == 16) dft16<INV>(a);
}

// Per-pass twiddle tables (kept in LDS): the pass with sub-size NSUB > 1 and
// radix RHO uses entry (r-1)*NSUB + k = exp(-2 pi i r k / (NSUB*RHO)),
// 1 <= r < RHO, k < NSUB, at offset tw_off(N, E, NSUB) of the table.
constexpr int tw_off(int N, int E, int nsub_target) {
    int off = 0, ns = 1;
    while (ns < N && ns != nsub_target) {
        const int rho = (N / ns) < E ? (N / ns) : E;
        if (ns > 1) off += ns * (rho - 1);
        ns *= rho;
    }
    return off;
}
constexpr int tw_len(int N, int E) { return tw_off(N, E, N); }

// Index into tw[] of table entry idx (passes searched at compile time).
template <int N, int E, int NS, int OFF>
__device__ __forceinline__ int tw_src(int idx) {
    constexpr int RHO = (N / NS) < E ? (N / NS) : E;
    if constexpr (NS == 1) {
        return tw_src<N, E, RHO, 0>(idx);
    } else {
        constexpr int CNT = NS * (RHO - 1);
        const int i = idx - OFF;
        const int src = (i / NS + 1) * (i % NS) * (TW_N / (NS * RHO));
        if constexpr (NS * RHO >= N) return src;
        else return idx < OFF + CNT ? src : tw_src<N, E, NS * RHO, OFF + CNT>(idx);
    }
}

// Fill the per-pass tables with NT threads; all loads are independent so
// they are in flight together.
template <int N, int E, int NT>
__device__ __forceinline__ void build_twiddles(float2* tab, const float2* __restrict__ tw, int tid) {
    constexpr int LEN = tw_len(N, E);
    if constexpr (LEN > 0) {
#pragma unroll
        for (int i = 0; i < (LEN + NT - 1) / NT; ++i) {
            // clamped: surplus threads rewrite the last entry with its own value
            const int idx = min(tid + NT * i, LEN - 1);
            tab[idx] = tw[tw_src<N, E, 1, 0>(idx)];
        }
    }
}

// One Stockham pass, sub-transform size NSUB -> NSUB*RHO, on NS signals
// v[S0..S0+NS).  Non-final passes write to LDS (signal s at lds + s*ls); the
// final pass leaves its outputs in registers.  With the skew-16 layout the
// RHO outputs of a butterfly land at lpad(base) + r*NSUB + (r*NSUB >> kSkew)
// for every power-of-two NSUB, so one address per butterfly suffices.  ptab: this
// pass's twiddle table, entry (r-1)*NSUB + k (unused when NSUB = 1).
template <int N, int E, int RHO, int NSUB, bool INV, bool LAST, int NS, int S0, int S>
__device__ __forceinline__ void st_pass(float2 (&v)[S][E], int j, const float2* ptab, float2* lds, int ls) {
    constexpr int T = N / E;
    constexpr int Q = E / RHO;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = j + q * T;
        const int k = b & (NSUB - 1);
        float2 w[RHO];
        if constexpr (NSUB > 1) {
            const float2* twk = ptab + k;
#pragma unroll
            for (int r = 1; r < RHO; ++r) w[r] = twk[(r - 1) * NSUB];
        }
        const int wb = lpad((b - k) * RHO + k);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            float2 a[RHO];
#pragma unroll
            for (int r = 0; r < RHO; ++r) {
                a[r] = v[S0 + s][q + r * Q];
                if constexpr (NSUB > 1) {
                    if (r > 0) a[r] = INV ? cmulc(a[r], w[r]) : cmul(a[r], w[r]);
                }
            }
            dft<RHO, INV>(a);
#pragma unroll
            for (int r = 0; r < RHO; ++r) {
                if constexpr (LAST) v[S0 + s][q + r * Q] = a[r];
                else lds[s * ls + wb + r * NSUB + ((r * NSUB) >> kSkew)] = a[r];
            }
        }
    }
}

template <int N, int E, int NSUB, bool INV, int NS, int S0, int S>
__device__ __forceinline__ void st_passes(float2 (&v)[S][E], int j, const float2* tab, float2* lds, int ls) {
    if constexpr (NSUB < N) {
        constexpr int T = N / E;
        constexpr int RHO = (N / NSUB) < E ? (N / NSUB) : E;
        constexpr bool LAST = NSUB * RHO >= N;
        if constexpr (!LAST) __syncthreads();   // earlier readers of lds are done
        st_pass<N, E, RHO, NSUB, INV, LAST, NS, S0, S>(v, j, tab + tw_off(N, E, NSUB), lds, ls);
        if constexpr (!LAST) {
            __syncthreads();
            const int rb = lpad(j);
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    if constexpr (T % kSkewP == 0) v[S0 + s][m] = lds[s * ls + rb + m * (T + T / kSkewP)];
                    else v[S0 + s][m] = lds[s * ls + lpad(j + T * m)];
                }
        }
        st_passes<N, E, NSUB * RHO, INV, NS, S0, S>(v, j, tab, lds, ls);
    }
}

// Full length-N transform (unnormalised) of signals v[S0..S0+NS); tab holds
// the per-pass twiddle tables built by build_twiddles<N, E>.
template <int N, int E, bool INV, int NS, int S0, int S>
__device__ __forceinline__ void st_fft(float2 (&v)[S][E], int j, const float2* tab, float2* lds, int ls) {
    st_passes<N, E, 1, INV, NS, S0, S>(v, j, tab, lds, ls);
}

// Blocks are dealt to the 8 XCDs round-robin; renumber them so that
// consecutive logical blocks (neighbouring rows) share an XCD and its L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7, xcd = b & 7, i = b >> 3;
    return xcd < rem ? xcd * (per + 1) + i : rem * (per + 1) + (xcd - rem) * per + i;
}

// ---------------------------------------------------------------------
// Compile-time launch geometry
// ---------------------------------------------------------------------
constexpr int x_E(int L) { return L < 8 ? L : (L / 8 > 256 ? L / 256 : 8); }
constexpr int x_T(int L) { return L / x_E(L); }
constexpr int x_rows_conc(int L) { return 256 / x_T(L); }
constexpr size_t x_lds(int L, int rpt) { return (size_t)x_rows_conc(L) * rpt * lds_len(L) * sizeof(float2); }
// rows per thread: as many (<= 4) as keep a block's LDS within 48 KB (three
// blocks per CU); at 1024x1024 that is 4 rows per block, which measured
// faster than 2 or 8 for both directions
constexpr int x_RPT_lds(int L, int kb) {
    return x_lds(L, 4) <= kb * 1024 ? 4 : (x_lds(L, 2) <= kb * 1024 ? 2 : 1);
}
constexpr int x_RPT(int L, int stage) { return (void)stage, x_RPT_lds(L, 48); }

// y-pass elements per thread: 4 (two waves per SIMD at 512 threads, which
// measured faster than 8 elements on 256 threads), more when PY needs it
constexpr int y_E(int nz, int Py) {
    (void)nz;
    int E = 4;
    if (E > Py) E = Py;
    while (Py / E > 512) E *= 2;
    return E;
}
// signals per LDS exchange group (divides 3*nz; 6 groups two layers when nz is even)
constexpr int y_NSG(int nz, int Py) { return (Py <= 2048 && nz % 2 == 0) ? 6 : 3; }

// ---------------------------------------------------------------------
// x forward: a block holds R consecutive rows of one signal s.
// ---------------------------------------------------------------------
// Rows y0 .. y0+R-1 of signal s (R = x_rows_conc(L) * RPT), thread tid < 256,
// LDS at lds (x_lds(L, RPT) bytes).
template <int L, int RPT>
__device__ __forceinline__ void xfwd_rows(const ChainDesc& cd, int S, int s, int y0, const float2* __restrict__ tw,
                                          int tid, float2* lds) {
    const SweepArgs a = cd.a;
    const float* __restrict__ m = cd.m;
    float2* __restrict__ X = cd.X;
    constexpr int E = x_E(L), T = x_T(L), RC = x_rows_conc(L), R = RC * RPT;
    constexpr int LS = lds_len(L);
    const int comp = s / a.nz, z = s - comp * a.nz;
    const int j = tid % T, rg = tid / T;
    // zero padding: hw <= L/2 (L >= 2), so slots n >= L/2 are zero
    constexpr int QH = E > 1 ? E / 2 : 1;
    float2 v[RPT][E];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int y = y0 + rg + RC * i;
        const int ce = (y + z) & 1;
        const long long ro = ((long long)z * a.ny + y) * a.hw;
        const float* me = m + ((long long)ce * 3 + comp) * a.Nc + ro;
        const float* mo = m + ((long long)(1 - ce) * 3 + comp) * a.Nc + ro;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int n = j + T * q;
            float2 t = make_float2(0.f, 0.f);
            if (q < QH && y < a.ny && n < a.hw) {
                if (2 * n < a.nx) t.x = me[n];
                if (2 * n + 1 < a.nx) t.y = mo[n];
            }
            v[i][q] = t;
        }
    }
    // row r = rg + RC*i lives at lds + r*LS; the per-pass twiddle tables
    // follow the base table in global memory (L1-resident)
    const float2* tab = tw + TW_N;
    float2* my = lds + rg * LS;
    st_fft<L, E, false, RPT, 0, RPT>(v, j, tab, my, RC * LS);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int q = 0; q < E; ++q) my[i * RC * LS + lpad(j + T * q)] = v[i][q];
    __syncthreads();
    // X[k] = A + W^k B, A = (Z[k] + conj Z[L-k])/2, B = (Z[k] - conj Z[L-k])/(2i), W = exp(-i pi/L).
    // The pair (k, L-k) shares A and B up to conjugation: X[L-k] = conj(A - W^k B),
    // so one thread forms both from one pair of LDS reads.  k = 0: X[0] = A + B
    // and X[L] = A - B are real (stored as X[0] + i X[L]); its partner is the
    // self-paired bin L/2, X[L/2] = conj Z[L/2].
    // (loop bodies are branch-free apart from the stores, so the unrolled
    // reads of several iterations are in flight together)
    constexpr int WSTEP = TW_N / (2 * L);
    constexpr int KH = L >= 2 ? L / 2 : 1;
    static_assert((R * KH) % 256 == 0, "x tile covers whole waves");
#pragma unroll 8
    for (int i = 0; i < R * KH / 256; ++i) {
        const int e = tid + 256 * i;
        const int k = e / R, r = e - k * R, y = y0 + r;
        const int kb = k == 0 ? KH : L - k;              // partner bin (L/2 for k = 0)
        const float2 Zk = lds[r * LS + lpad(k)];
        const float2 Zr = lds[r * LS + lpad(kb & (L - 1))];
        const float2 Zo = k == 0 ? Zk : Zr;              // Z[L-k]
        const float2 A = make_float2(0.5f * (Zk.x + Zo.x), 0.5f * (Zk.y - Zo.y));
        const float2 B = make_float2(0.5f * (Zk.y + Zo.y), -0.5f * (Zk.x - Zo.x));
        const float2 WB = cmul(tw[k * WSTEP], B);
        const float2 out = k == 0 ? make_float2(A.x + B.x, A.x - B.x) : make_float2(A.x + WB.x, A.y + WB.y);
        const float2 out2 = k == 0 ? make_float2(Zr.x, -Zr.y) : make_float2(A.x - WB.x, WB.y - A.y);
        if (y < a.ny) {
            X[((long long)k * S + s) * a.ny + y] = out;
            if (L >= 2) X[((long long)kb * S + s) * a.ny + y] = out2;
        }
    }
}
// Body of one x-forward block: logical block lb (tile of R rows of one
// signal), thread tid < 256, LDS at lds.
template <int L, int RPT>
__device__ __forceinline__ void xfwd_body(const ChainDesc& cd, int S, int ntiles, const float2* __restrict__ tw,
                                          int lb, int tid, float2* lds) {
    constexpr int R = x_rows_conc(L) * RPT;
    const int s = lb / ntiles;
    xfwd_rows<L, RPT>(cd, S, s, (lb - s * ntiles) * R, tw, tid, lds);
}

template <int L, int RPT, bool BAT>
__global__ __launch_bounds__(256) void k_xfwd(ChainDesc d0, const ChainDesc* __restrict__ dl, int S, int ntiles,
                                              const float2* __restrict__ tw) {
    extern __shared__ float2 lds[];
    xfwd_body<L, RPT>(chain_at<BAT>(d0, dl, blockIdx.y), S, ntiles, tw, xcd_block(blockIdx.x, gridDim.x), threadIdx.x,
                      lds);
}

// Per-pass twiddle tables of the x transforms (length L, x_E(L) per thread),
// written once per plan after the base table.
template <int L>
__global__ void k_x_twiddles(float2* __restrict__ out, const float2* __restrict__ tw) {
    build_twiddles<L, x_E(L), 256>(out, tw, threadIdx.x);
}

// x inverse, mirror of the forward, for rows y0 .. y0+R-1 of signal s: writes
// h of colour c when (mask >> c) & 1; TOL: instead writes the field of the
// cells of colour `mask` to hb[r * hw + n], r = y - y0, n the slot (rows past
// ny untouched).
template <int L, int RPT, bool TOL = false>
__device__ __forceinline__ void xinv_rows(const ChainDesc& cd, int S, int s, int y0, int mask,
                                          const float2* __restrict__ tw, int tid, float2* lds, float* hb = nullptr) {
    const SweepArgs a = cd.a;
    const float2* __restrict__ X = cd.X;
    float* __restrict__ h = cd.h;
    constexpr int E = x_E(L), T = x_T(L), RC = x_rows_conc(L), R = RC * RPT;
    constexpr int LS = lds_len(L);
    const int comp = s / a.nz, z = s - comp * a.nz;
    const int j = tid % T, rg = tid / T;
    constexpr int WSTEP = TW_N / (2 * L);
    // Z[k] = A + i B, A = X[k] + conj X[L-k], B = (X[k] - conj X[L-k]) W^-k; the
    // partner bin L-k gives Z[L-k] = conj A + i conj B, so one thread forms both
    // from one pair of loads.  Row 0 holds the real pair P = X[0] + i X[L]:
    // Z[0] = (P.x + P.y, P.x - P.y); its partner is the self-paired bin L/2,
    // Z[L/2] = 2 conj X[L/2].
    // (rows past ny read row ny-1 and store zero: no branch around the loads)
    constexpr int KH = L >= 2 ? L / 2 : 1;
    static_assert((R * KH) % 256 == 0, "x tile covers whole waves");
#pragma unroll 8
    for (int i = 0; i < R * KH / 256; ++i) {
        const int e = tid + 256 * i;
        const int k = e / R, r = e - k * R, y = y0 + r;
        const int yc = y < a.ny ? y : a.ny - 1;
        const int kb = k == 0 ? KH : L - k;              // partner bin (L/2 for k = 0)
        const float2 Xa = X[((long long)k * S + s) * a.ny + yc];
        const float2 Xb = X[((long long)(kb & (L - 1)) * S + s) * a.ny + yc];
        const float2 A = make_float2(Xa.x + Xb.x, Xa.y - Xb.y);
        const float2 D = make_float2(Xa.x - Xb.x, Xa.y + Xb.y);
        const float2 B = cmulc(D, tw[k * WSTEP]);
        const float2 z1 = k == 0 ? make_float2(Xa.x + Xa.y, Xa.x - Xa.y) : make_float2(A.x - B.y, A.y + B.x);
        const float2 z2 = k == 0 ? make_float2(2.f * Xb.x, -2.f * Xb.y) : make_float2(A.x + B.y, B.x - A.y);
        const bool in = y < a.ny;
        lds[r * LS + lpad(k)] = in ? z1 : make_float2(0.f, 0.f);
        if (L >= 2) lds[r * LS + lpad(kb)] = in ? z2 : make_float2(0.f, 0.f);
    }
    const float2* tab = tw + TW_N;
    __syncthreads();
    float2* my = lds + rg * LS;
    float2 v[RPT][E];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int q = 0; q < E; ++q) v[i][q] = my[i * RC * LS + lpad(j + T * q)];
    st_fft<L, E, true, RPT, 0, RPT>(v, j, tab, my, RC * LS);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int y = y0 + rg + RC * i;
        if (y >= a.ny) continue;
        const int ce = (y + z) & 1;
        constexpr int QH = E > 1 ? E / 2 : 1;   // slots n < hw <= L/2 only
        if constexpr (TOL) {
            // slot n of colour `mask`: x = 2n when the even cells have it, else 2n+1
            float* hr = hb + (rg + RC * i) * a.hw;
            const bool ev = ce == mask;
#pragma unroll
            for (int q = 0; q < QH; ++q) {
                const int n = j + T * q;
                if (n < a.hw && 2 * n + (ev ? 0 : 1) < a.nx) hr[n] = ev ? v[i][q].x : v[i][q].y;
            }
        } else {
            const long long ro = ((long long)z * a.ny + y) * a.hw;
            float* he = h + ((long long)ce * 3 + comp) * a.Nc + ro;
            float* ho = h + ((long long)(1 - ce) * 3 + comp) * a.Nc + ro;
            const bool we = (mask >> ce) & 1, wo = (mask >> (1 - ce)) & 1;
#pragma unroll
            for (int q = 0; q < QH; ++q) {
                const int n = j + T * q;
                if (n >= a.hw) continue;
                if (we && 2 * n < a.nx) he[n] = v[i][q].x;
                if (wo && 2 * n + 1 < a.nx) ho[n] = v[i][q].y;
            }
        }
    }
}
template <int L, int RPT>
__device__ __forceinline__ void xinv_body(const ChainDesc& cd, int S, int ntiles, int mask,
                                          const float2* __restrict__ tw, int lb, int tid, float2* lds) {
    constexpr int R = x_rows_conc(L) * RPT;
    const int s = lb / ntiles;
    xinv_rows<L, RPT>(cd, S, s, (lb - s * ntiles) * R, mask, tw, tid, lds);
}

template <int L, int RPT, bool BAT>
__global__ __launch_bounds__(256) void k_xinv(ChainDesc d0, const ChainDesc* __restrict__ dl, int S, int ntiles,
                                              int mask, const float2* __restrict__ tw) {
    extern __shared__ float2 lds[];
    xinv_body<L, RPT>(chain_at<BAT>(d0, dl, blockIdx.y), S, ntiles, mask, tw, xcd_block(blockIdx.x, gridDim.x),
                      threadIdx.x, lds);
}

// Forward or inverse FFT of all S signals in groups of NSG through LDS.
template <int PY, int E, bool INV, int NSG, int G, int S>
__device__ __forceinline__ void y_groups(float2 (&v)[S][E], int j, const float2* __restrict__ twl, float2* lds, int ls) {
    if constexpr (G < S) {
        st_fft<PY, E, INV, NSG, G, S>(v, j, twl, lds, ls);
        y_groups<PY, E, INV, NSG, G + NSG, S>(v, j, twl, lds, ls);
    }
}

// Inverse transforms of signals [G, S) in groups of NSG; after each group,
// its cropped outputs (bins y = j + T*q < ny, q < QH) go to dst0 + s*ny.
template <int PY, int E, int NSG, int G, int S, int QH>
__device__ __forceinline__ void y_inv_store(float2 (&v)[S][E], int j, const float2* __restrict__ twl, float2* lds,
                                            int ls, float2* __restrict__ dst0, int ny) {
    if constexpr (G < S) {
        constexpr int T = PY / E;
        st_fft<PY, E, true, NSG, G, S>(v, j, twl, lds, ls);
#pragma unroll
        for (int s = G; s < G + NSG; ++s) {
            float2* dst = dst0 + (long long)s * ny;
#pragma unroll
            for (int q = 0; q < QH; ++q) {
                const int y = j + T * q;
                if (y < ny) dst[y] = v[s][q];
            }
        }
        y_inv_store<PY, E, NSG, G + NSG, S, QH>(v, j, twl, lds, ls, dst0, ny);
    }
}

// Block 0 of the y pass carries Z = X0 + i XL, X0 and XL real along y, so
// their spectra are Hermitian: Y0[k] = (Z[k] + conj Z[-k])/2 and
// YL[k] = (Z[k] - conj Z[-k])/(2i).  SPLIT keeps Y0[k] in slot k and YL[k]
// in slot PY-k for 0 < k < PY/2 (slots 0 and PY/2 already hold the real pair
// (Y0, YL)); the merge maps the mixed (H0, HL) back to W = H0 + i HL over the
// full range.  Works on the signals in groups of NSG through LDS.
// (act = false: only the barriers, for thread groups that run other kx
// values in lockstep with the kx = 0 group)
template <int PY, int E, bool SPLIT, int NSG, int G, int S>
__device__ __forceinline__ void y_pair(float2 (&v)[S][E], int j, float2* lds, int ls, bool act = true) {
    if constexpr (G < S) {
        constexpr int T = PY / E;
        __syncthreads();
        if (act) {
#pragma unroll
            for (int s = 0; s < NSG; ++s)
#pragma unroll
                for (int q = 0; q < E; ++q) lds[s * ls + lpad(j + T * q)] = v[G + s][q];
        }
        __syncthreads();
        if (act) {
#pragma unroll
        for (int s = 0; s < NSG; ++s)
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int ky = j + T * q, kp = (PY - ky) & (PY - 1);
                if (ky == kp) continue;
                const float2 z = v[G + s][q], p = lds[s * ls + lpad(kp)];
                if (SPLIT) {
                    v[G + s][q] = ky < kp ? make_float2(0.5f * (z.x + p.x), 0.5f * (z.y - p.y))
                                          : make_float2(0.5f * (p.y + z.y), -0.5f * (p.x - z.x));
                } else {
                    v[G + s][q] = ky < kp ? make_float2(z.x - p.y, z.y + p.x) : make_float2(p.x + z.y, z.x - p.y);
                }
            }
        }
        y_pair<PY, E, SPLIT, NSG, G + NSG, S>(v, j, lds, ls, act);
    }
}

// Direct mixing of one bin over layers: H_i(z) = sum_z' sum_j K_ij(z - z') M_j(z').
// Kp: the 6*NZ tensor values of the bin, in registers (xx, yy, zz, xy real; xz, yz
// imaginary, stored as their imaginary parts), sy = -1 for bins past PY/2.
template <int NZ>
__device__ __forceinline__ void load_bin(float (&kv)[6 * NZ], const float* __restrict__ Kp) {
#pragma unroll
    for (int i = 0; i < 6 * NZ; ++i) kv[i] = Kp[i];
}
template <int NZ>
__device__ __forceinline__ void mix_layers(const float (&Kp)[6 * NZ], float sy, const float2 (&M)[3 * NZ],
                                           float2 (&H)[3 * NZ]) {
#pragma unroll
    for (int s = 0; s < 3 * NZ; ++s) H[s] = make_float2(0.f, 0.f);
#pragma unroll
    for (int zo = 0; zo < NZ; ++zo) {
#pragma unroll
        for (int zi = 0; zi < NZ; ++zi) {
            const int dz = zo - zi, adz = dz >= 0 ? dz : -dz;
            const float sz = dz >= 0 ? 1.0f : -1.0f;
            const float kxx = Kp[0 * NZ + adz], kyy = Kp[1 * NZ + adz], kzz = Kp[2 * NZ + adz];
            const float kxy = sy * Kp[3 * NZ + adz], kxz = sz * Kp[4 * NZ + adz], kyz = sy * sz * Kp[5 * NZ + adz];
            const float2 Mx = M[0 * NZ + zi], My = M[1 * NZ + zi], Mz = M[2 * NZ + zi];
            // xz, yz spectra are imaginary: (i k) M = (-k M.y, k M.x)
            H[0 * NZ + zo].x += kxx * Mx.x + kxy * My.x - kxz * Mz.y;
            H[0 * NZ + zo].y += kxx * Mx.y + kxy * My.y + kxz * Mz.x;
            H[1 * NZ + zo].x += kxy * Mx.x + kyy * My.x - kyz * Mz.y;
            H[1 * NZ + zo].y += kxy * Mx.y + kyy * My.y + kyz * Mz.x;
            H[2 * NZ + zo].x += -kxz * Mx.y - kyz * My.y + kzz * Mz.x;
            H[2 * NZ + zo].y += kxz * Mx.x + kyz * My.x + kzz * Mz.y;
        }
    }
}

// y pass: one group of T = PY/E threads per kx < L (the kx = 0 group also
// carries kx = L); thread j owns bins j + T*q.  nkx = L.  UNI: several groups
// share a block (each with its own LDS), so every group runs the kx = 0
// group's barriers too.
constexpr int y1_lds(int nz, int Py) { return y_NSG(nz, Py) * lds_len(Py) + tw_len(Py, y_E(nz, Py)); }
template <int NZ, int PY, bool UNI>
__device__ __forceinline__ void ypass_body(const ChainDesc& cd, const float* __restrict__ K,
                                           const float2* __restrict__ tw, int kx, int j, int nkx, float2* lds) {
    const SweepArgs a = cd.a;
    float2* __restrict__ X = cd.X;
    constexpr int S = 3 * NZ, E = y_E(NZ, PY), T = PY / E, NSG = y_NSG(NZ, PY);
    constexpr int LS = lds_len(PY);
    float2* twl = lds + NSG * LS;      // per-pass twiddle tables
    const int ny = a.ny;
    // zero padding: ny <= PY/2, so the upper half of each thread's strided
    // registers (y >= PY/2) is zero on input and not needed on output
    constexpr int QH = E > 1 ? E / 2 : 1;
    float2 v[S][E];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const float2* src = X + ((long long)kx * S + s) * ny;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int y = j + T * q;
            v[s][q] = (q < QH && y < ny) ? src[y] : make_float2(0.f, 0.f);
        }
    }
    build_twiddles<PY, E, T>(twl, tw, j);
    __syncthreads();
    y_groups<PY, E, false, NSG, 0, S>(v, j, twl, lds, LS);
    constexpr int HP = PY / 2;
    // (the pair split and merge of the kx = 0 group sit outside the branches,
    // so their barriers are reached by uniform control flow)
    if (UNI || kx == 0) y_pair<PY, E, true, NSG, 0, S>(v, j, lds, LS, kx == 0);
    if (kx != 0) {
        // the tensor values of bin q+1 are loaded while bin q is mixed
        auto bin = [&](int q) {
            const int ky = j + T * q;
            return K + ((long long)kx * (HP + 1) + (ky <= HP ? ky : PY - ky)) * 6 * NZ;
        };
        float kc[6 * NZ];
        load_bin<NZ>(kc, bin(0));
#pragma unroll
        for (int q = 0; q < E; ++q) {
            float kn[6 * NZ];
            if (q + 1 < E) load_bin<NZ>(kn, bin(q + 1));
            const int ky = j + T * q;
            float2 M[S], H[S];
#pragma unroll
            for (int s = 0; s < S; ++s) M[s] = v[s][q];
            mix_layers<NZ>(kc, ky <= HP ? 1.0f : -1.0f, M, H);
#pragma unroll
            for (int s = 0; s < S; ++s) v[s][q] = H[s];
            if (q + 1 < E) {
#pragma unroll
                for (int i = 0; i < 6 * NZ; ++i) kc[i] = kn[i];
            }
        }
    } else {
        // kx = 0 in slots k <= PY/2 and kx = L in slots PY-k (both at +k);
        // the self-paired slots 0 and PY/2 mix the real pair separately
        const float* K0 = K;
        const float* KL = K + (long long)nkx * (HP + 1) * 6 * NZ;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int ky = j + T * q;
            float2 M[S], H[S];
            float kv[6 * NZ];
            if (ky == 0 || ky == HP) {
                // real pair (Y0, YL): the xy, xz and yz spectra vanish on these
                // four bins (each is odd along x or along y), so the mixing is
                // the diagonal one, with the kx = 0 tensor on the real part and
                // the kx = L tensor on the imaginary part
                const float* k0 = K0 + (long long)ky * 6 * NZ;
                const float* kl = KL + (long long)ky * 6 * NZ;
#pragma unroll
                for (int i = 0; i < 3 * NZ; ++i) {
                    kv[i] = k0[i];
                    kv[3 * NZ + i] = kl[i];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int zo = 0; zo < NZ; ++zo) {
                        float hr = 0.f, hi = 0.f;
#pragma unroll
                        for (int zi = 0; zi < NZ; ++zi) {
                            const int adz = zo >= zi ? zo - zi : zi - zo;
                            hr += kv[c * NZ + adz] * v[c * NZ + zi][q].x;
                            hi += kv[3 * NZ + c * NZ + adz] * v[c * NZ + zi][q].y;
                        }
                        H[c * NZ + zo] = make_float2(hr, hi);
                    }
#pragma unroll
                for (int s = 0; s < S; ++s) v[s][q] = H[s];
            } else {
                load_bin<NZ>(kv, ky < HP ? K0 + (long long)ky * 6 * NZ : KL + (long long)(PY - ky) * 6 * NZ);
#pragma unroll
                for (int s = 0; s < S; ++s) M[s] = v[s][q];
                mix_layers<NZ>(kv, 1.0f, M, H);
#pragma unroll
                for (int s = 0; s < S; ++s) v[s][q] = H[s];
            }
        }
    }
    if (UNI || kx == 0) y_pair<PY, E, false, NSG, 0, S>(v, j, lds, LS, kx == 0);
    y_groups<PY, E, true, NSG, 0, S>(v, j, twl, lds, LS);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        float2* dst = X + ((long long)kx * S + s) * ny;
#pragma unroll
        for (int q = 0; q < QH; ++q) {
            const int y = j + T * q;
            if (y < ny) dst[y] = v[s][q];
        }
    }
}

template <int NZ, int PY, bool BAT>
__global__ __launch_bounds__(PY / y_E(NZ, PY)) void k_ypass(ChainDesc d0, const ChainDesc* __restrict__ dl,
                                                            const float* __restrict__ K,
                                                            const float2* __restrict__ tw) {
    extern __shared__ float2 lds[];
    ypass_body<NZ, PY, false>(chain_at<BAT>(d0, dl, blockIdx.y), K, tw, blockIdx.x, threadIdx.x, gridDim.x, lds);
}

// ---------------------------------------------------------------------
// Split-precision DFT stages on the matrix cores (y pass, MMC_DEMAG_SPLIT_*).
//
// A radix-16 Stockham pass is a product of the 16-point DFT matrix with a
// 16 x 16 block of butterflies: as real arithmetic, C[q][b] = sum_kk A[q][kk]
// B[kk][b] with kk = 2r + (0: real part, 1: imaginary part) of the r-th
// (twiddled) input of butterfly b, one product for the real outputs (A_re)
// and one for the imaginary outputs (A_im), v_mfma_f32_16x16x32 each.  Both
// operands are split into a high and a low 16-bit part (x = hi + lo), and
// each product sums hi*hi + hi*lo + lo*hi in FP32 (the lo*lo term is below
// the rounding of hi + lo).  BF16 parts keep 16 significant bits of each
// operand; FP16 parts keep 22 but have the range of FP16, so the FP16 form
// scales each pass's inputs by a power of two chosen from a bound on their
// magnitude (exact, undone on the outputs).
//
// Operand layouts of v_mfma_f32_16x16x32_{bf16,f16} (wave64): lane l holds
// A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16], e < 8, and
// C[4 (l / 16) + e][l % 16], e < 4.  So lane (c = l % 16, g = l / 16) loads
// inputs r = 4g .. 4g+3 of butterfly c of the block and writes outputs q =
// 4g .. 4g+3 of the same butterfly.
// ---------------------------------------------------------------------
typedef __bf16 mf_bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 mf_f16x8 __attribute__((ext_vector_type(8)));
typedef float mf_f32x4 __attribute__((ext_vector_type(4)));

// PREC: 0 FP32 transforms on the vector units, 1 split BF16, 2 split FP16.
template <int PREC> struct MfOps;
template <> struct MfOps<1> {
    typedef __bf16 S;
    typedef mf_bf16x8 V;
    static __device__ __forceinline__ mf_f32x4 mma(V a, V b, mf_f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct MfOps<2> {
    typedef _Float16 S;
    typedef mf_f16x8 V;
    static __device__ __forceinline__ mf_f32x4 mma(V a, V b, mf_f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// x*sc = hi + lo (sc: a power of two; 1 in the BF16 form).  BF16: hi is x
// truncated to its top 16 bits (exact as FP32, packed two per register by a
// byte permute), lo the exact remainder rounded to BF16.  FP16: hi = f16(x sc),
// lo = f16(x sc - hi), each one mixed-precision FMA.
template <int PREC>
__device__ __forceinline__ void mf_split8(const float (&x)[8], float sc, typename MfOps<PREC>::V& hi,
                                          typename MfOps<PREC>::V& lo) {
    if constexpr (PREC == 1) {
        typedef float f2v __attribute__((ext_vector_type(2)));
        typedef __bf16 b2v __attribute__((ext_vector_type(2)));
        uint32_t hw[4], lw[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const uint32_t u0 = __float_as_uint(x[2 * p]), u1 = __float_as_uint(x[2 * p + 1]);
            hw[p] = __builtin_amdgcn_perm(u1, u0, 0x07060302u);   // top halves of u0 (low), u1 (high)
            f2v r;
            r.x = x[2 * p] - __uint_as_float(u0 & 0xffff0000u);
            r.y = x[2 * p + 1] - __uint_as_float(u1 & 0xffff0000u);
            const b2v lb = __builtin_convertvector(r, b2v);
            lw[p] = __builtin_bit_cast(uint32_t, lb);
        }
        typedef uint32_t u4v __attribute__((ext_vector_type(4)));
        const u4v H = {hw[0], hw[1], hw[2], hw[3]}, Lo = {lw[0], lw[1], lw[2], lw[3]};
        hi = __builtin_bit_cast(typename MfOps<PREC>::V, H);
        lo = __builtin_bit_cast(typename MfOps<PREC>::V, Lo);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const _Float16 h = (_Float16)(x[e] * sc);
            hi[e] = h;
            lo[e] = (_Float16)fmaf(x[e], sc, -(float)h);
        }
    }
}

// The 16-point DFT matrix of one direction in the A layout, split, as two
// 16 x 32 halves: half h has rows i = 2 (q - 8h) + part for the outputs q of
// 8h .. 8h+7 (part 0 real, 1 imaginary), so the accumulator of lane (c, g)
// holds (re, im) of outputs 8h + 2g and 8h + 2g + 1 of butterfly c.
template <int PREC> struct MfDft {
    typename MfOps<PREC>::V h0, l0, h1, l1;
};
// tw: base table exp(-2 pi i t / TW_N); lane = thread index mod 64.
template <int PREC, bool INV>
__device__ __forceinline__ MfDft<PREC> mf_dft16(int lane, const float2* __restrict__ tw) {
    const int i = lane & 15, po = i & 1;
    float a0[8], a1[8];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = 8 * h + (i >> 1);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int kk = 8 * (lane >> 4) + e, r = kk >> 1, pi = kk & 1;
            const float2 w = tw[((r * q) & 15) * (TW_N / 16)];   // (cos t, -sin t), t = 2 pi r q / 16
            const float c = w.x, sn = -w.y;
            // forward, y = sum x e^{-it}: re = xr c + xi sn, im = xi c - xr sn;
            // inverse, y = sum x e^{+it}: re = xr c - xi sn, im = xi c + xr sn
            const float sg = INV ? -1.0f : 1.0f;
            const float val = po == 0 ? (pi == 0 ? c : sg * sn) : (pi == 0 ? -sg * sn : c);
            (h == 0 ? a0 : a1)[e] = val;
        }
    }
    MfDft<PREC> A;
    mf_split8<PREC>(a0, 1.0f, A.h0, A.l0);
    mf_split8<PREC>(a1, 1.0f, A.h1, A.l1);
    return A;
}

// Pass structure of a length-N transform with E elements per thread:
// forward: radix-E pass (vector units; its inputs past N/2 are the zero
// padding), mf_kf radix-16 passes on the matrix cores, then a radix-mf_rf pass
// on the vector units if mf_rf > 1; inverse: mf_ki radix-16 passes, then a
// radix-mf_ri pass (vector units, only the cropped outputs kept).
constexpr int mf_pow16(int k) { return k == 0 ? 1 : 16 * mf_pow16(k - 1); }
constexpr int mf_kf(int N, int E) { return (N / E) >= 256 ? 2 : ((N / E) >= 16 ? 1 : 0); }
constexpr int mf_rf(int N, int E) { return N / (E * mf_pow16(mf_kf(N, E))); }
constexpr int mf_ki(int N, int E) { return (N / E) > 16 ? 2 : 1; }
constexpr int mf_ri(int N, int E) { return N / mf_pow16(mf_ki(N, E)); }
// Twiddle tables of the split transforms (in LDS): radix-16 pass with
// sub-size NSUB: 16*NSUB entries, entry r*NSUB + k = exp(-2 pi i r k / (16 NSUB));
// vector pass of radix R and sub-size N/R: (R-1)*(N/R) entries, (r-1)*NSUB + k.
// Order: forward passes 1, 2, forward vector pass, inverse pass 2, inverse vector pass.
constexpr int mf_len_f1(int N, int E) { return mf_kf(N, E) >= 1 ? 16 * E : 0; }
constexpr int mf_len_f2(int N, int E) { return mf_kf(N, E) >= 2 ? 16 * 16 * E : 0; }
constexpr int mf_len_fl(int N, int E) { return mf_rf(N, E) > 1 ? (mf_rf(N, E) - 1) * (N / mf_rf(N, E)) : 0; }
constexpr int mf_len_i2(int N, int E) { return mf_ki(N, E) >= 2 ? 16 * 16 : 0; }
constexpr int mf_len_il(int N, int E) { return mf_ri(N, E) > 1 ? (mf_ri(N, E) - 1) * (N / mf_ri(N, E)) : 0; }
constexpr int mf_off_f2(int N, int E) { return mf_len_f1(N, E); }
constexpr int mf_off_fl(int N, int E) { return mf_off_f2(N, E) + mf_len_f2(N, E); }
constexpr int mf_off_i2(int N, int E) { return mf_off_fl(N, E) + mf_len_fl(N, E); }
constexpr int mf_off_il(int N, int E) { return mf_off_i2(N, E) + mf_len_i2(N, E); }
constexpr int mf_tw_len(int N, int E) { return mf_off_il(N, E) + mf_len_il(N, E); }

template <int NSUB, int RHO, bool ZERO_ROW>
__device__ __forceinline__ float2 mf_tw_entry(int i, const float2* __restrict__ tw) {
    // ZERO_ROW: entry r*NSUB + k (r from 0); else (r-1)*NSUB + k
    const int r = i / NSUB + (ZERO_ROW ? 0 : 1), k = i % NSUB;
    return tw[(r * k) * (TW_N / (NSUB * RHO))];
}
// (FP16 form: the tables of the second radix-16 pass of each direction are
// scaled by 1/16, which keeps that pass's inputs within the bound of the first)
template <int N, int E, int NT, int PREC>
__device__ __forceinline__ void mf_build_twiddles(float2* tab, const float2* __restrict__ tw, int tid) {
    constexpr int LEN = mf_tw_len(N, E);
    constexpr float S2 = PREC == 2 ? 0.0625f : 1.0f;
    for (int i = tid; i < LEN; i += NT) {
        float2 v;
        if (i < mf_off_f2(N, E)) v = mf_tw_entry<E, 16, true>(i, tw);
        else if (i < mf_off_fl(N, E)) {
            v = mf_tw_entry<16 * E, 16, true>(i - mf_off_f2(N, E), tw);
            v.x *= S2;
            v.y *= S2;
        }
        else if (i < mf_off_i2(N, E))
            v = mf_tw_entry<N / (mf_rf(N, E) > 1 ? mf_rf(N, E) : 1), (mf_rf(N, E) > 1 ? mf_rf(N, E) : 1), false>(
                i - mf_off_fl(N, E), tw);
        else if (i < mf_off_il(N, E)) {
            v = mf_tw_entry<16, 16, true>(i - mf_off_i2(N, E), tw);
            v.x *= S2;
            v.y *= S2;
        }
        else
            v = mf_tw_entry<N / (mf_ri(N, E) > 1 ? mf_ri(N, E) : 1), (mf_ri(N, E) > 1 ? mf_ri(N, E) : 1), false>(
                i - mf_off_il(N, E), tw);
        tab[i] = v;
    }
}

// One radix-16 Stockham pass on the matrix cores over the NSG signals of one
// thread set (T threads, signal s at lds + s*ls, slots lpad(i)), in place:
// every wave reads the inputs of its blocks of 16 butterflies, the block
// synchronises, then each block is twiddled, scaled by sc, split and
// multiplied, and its outputs (times isc) are written.  ptab: 16*NSUB
// twiddles, entry r*NSUB + k.
template <int N, int NSUB, bool INV, int PREC, int NSG, int T>
__device__ __forceinline__ void mf_pass(float2* lds, int ls, const float2* ptab, int jt, const MfDft<PREC>& A,
                                        float sc) {
    constexpr int NB = N / 16;           // butterflies per signal
    constexpr int GPS = NB / 16;         // blocks of 16 butterflies per signal
    constexpr int WV = T / 64;           // waves per set
    static_assert(GPS >= 1 && (NSG * GPS) % WV == 0, "whole blocks per wave");
    constexpr int NGW = NSG * GPS / WV;  // blocks per wave
    const int w = jt >> 6, l = jt & 63, c = l & 15, g = l >> 4;
    float2 in[NGW][4];
#pragma unroll
    for (int i = 0; i < NGW; ++i) {
        const int gi = w + WV * i, s = gi / GPS, b = 16 * (gi % GPS) + c;
#pragma unroll
        for (int t = 0; t < 4; ++t) in[i][t] = lds[s * ls + lpad(b + (4 * g + t) * NB)];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NGW; ++i) {
        const int gi = w + WV * i, s = gi / GPS, b = 16 * (gi % GPS) + c;
        const int k = b & (NSUB - 1);
        float x[8];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float2 a = in[i][t];
            if constexpr (NSUB > 1) {
                const float2 wv = ptab[(4 * g + t) * NSUB + k];
                a = INV ? cmulc(a, wv) : cmul(a, wv);
            }
            x[2 * t] = a.x;
            x[2 * t + 1] = a.y;
        }
        typename MfOps<PREC>::V bh, bl;
        mf_split8<PREC>(x, sc, bh, bl);
        mf_f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
        c0 = MfOps<PREC>::mma(A.l0, bh, c0);
        c0 = MfOps<PREC>::mma(A.h0, bl, c0);
        c0 = MfOps<PREC>::mma(A.h0, bh, c0);
        c1 = MfOps<PREC>::mma(A.l1, bh, c1);
        c1 = MfOps<PREC>::mma(A.h1, bl, c1);
        c1 = MfOps<PREC>::mma(A.h1, bh, c1);
        const int ob = (b - k) * 16 + k;
        float2* o = lds + s * ls;
        // outputs q = 2g, 2g+1 (c0) and 8+2g, 9+2g (c1)
        o[lpad(ob + (2 * g) * NSUB)] = make_float2(c0[0], c0[1]);
        o[lpad(ob + (2 * g + 1) * NSUB)] = make_float2(c0[2], c0[3]);
        o[lpad(ob + (2 * g + 8) * NSUB)] = make_float2(c1[0], c1[1]);
        o[lpad(ob + (2 * g + 9) * NSUB)] = make_float2(c1[2], c1[3]);
    }
}

// Scales of the FP16 form (powers of two): the bound b on the first
// radix-16 pass's inputs of a direction is mapped to at most 2^14; the second
// pass's inputs stay within it through its 1/16 twiddles.  The data keep the
// scale through the layer mixing (linear) and lose it at the store.
__device__ __forceinline__ float mf_scale(float b) {
    int ex;
    (void)frexpf(b, &ex);                 // b <= 2^ex
    return ldexpf(1.0f, 14 - ex);
}
struct MfScales {
    float f1;                             // forward pass 1 (the data are unscaled before it)
    float i1;                             // inverse pass 1, relative to the forward result's scale
    float out;                            // factor that unscales the inverse result
};

// Forward split transform of signals [G, G+NSG) of one set (registers in the
// strided layout, thread j holds points j + T*m), result in the same layout.
template <int N, int E, int PREC, int NSG, int G, int SH>
__device__ __forceinline__ void y_fwd_mf(float2 (&v)[SH][E], int j, const float2* tabs, float2* lds, int ls,
                                         const MfDft<PREC>& A, const MfScales& sc) {
    constexpr int T = N / E;
    constexpr int KF = mf_kf(N, E), RF = mf_rf(N, E);
    __syncthreads();                      // earlier readers of lds are done
    st_pass<N, E, E, 1, false, false, NSG, G, SH>(v, j, tabs, lds, ls);
    __syncthreads();
    if constexpr (KF >= 1) {
        mf_pass<N, E, false, PREC, NSG, T>(lds, ls, tabs, j, A, sc.f1);
        __syncthreads();
    }
    if constexpr (KF >= 2) {
        mf_pass<N, 16 * E, false, PREC, NSG, T>(lds, ls, tabs + mf_off_f2(N, E), j, A, 1.0f);
        __syncthreads();
    }
    const int rb = lpad(j);
#pragma unroll
    for (int s = 0; s < NSG; ++s)
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if constexpr (T % kSkewP == 0) v[G + s][m] = lds[s * ls + rb + m * (T + T / kSkewP)];
            else v[G + s][m] = lds[s * ls + lpad(j + T * m)];
        }
    if constexpr (RF > 1)
        st_pass<N, E, RF, N / RF, false, true, NSG, G, SH>(v, j, tabs + mf_off_fl(N, E), lds, ls);
}

// Inverse split transform of signals [G, G+NSG) of one set, then the cropped
// outputs (points y = j + T*q < ny, q < E/2) times osc go to dst0 + s*ny.
template <int N, int E, int PREC, int NSG, int G, int SH>
__device__ __forceinline__ void y_inv_mf_store(float2 (&v)[SH][E], int j, const float2* tabs, float2* lds, int ls,
                                               const MfDft<PREC>& A, const MfScales& sc, float2* __restrict__ dst0,
                                               int ny, float osc) {
    constexpr int T = N / E, QH = E / 2;
    constexpr int KI = mf_ki(N, E), RI = mf_ri(N, E);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NSG; ++s)
#pragma unroll
        for (int m = 0; m < E; ++m) lds[s * ls + lpad(j + T * m)] = v[G + s][m];
    __syncthreads();
    mf_pass<N, 1, true, PREC, NSG, T>(lds, ls, tabs, j, A, sc.i1);
    __syncthreads();
    if constexpr (KI >= 2) {
        mf_pass<N, 16, true, PREC, NSG, T>(lds, ls, tabs + mf_off_i2(N, E), j, A, 1.0f);
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < NSG; ++s)
#pragma unroll
        for (int m = 0; m < E; ++m) v[G + s][m] = lds[s * ls + lpad(j + T * m)];
    if constexpr (RI > 1)
        st_pass<N, E, RI, N / RI, true, true, NSG, G, SH>(v, j, tabs + mf_off_il(N, E), lds, ls);
#pragma unroll
    for (int s = G; s < G + NSG; ++s) {
        float2* dst = dst0 + (long long)s * ny;
#pragma unroll
        for (int q = 0; q < QH; ++q) {
            const int y = j + T * q;
            if (y < ny) {
                if constexpr (PREC == 2) dst[y] = make_float2(v[s][q].x * osc, v[s][q].y * osc);
                else dst[y] = v[s][q];
            }
        }
    }
}

template <int N, int E, int PREC, int NSG, int G, int SH>
__device__ __forceinline__ void y_fwd_mf_groups(float2 (&v)[SH][E], int j, const float2* tabs, float2* lds, int ls,
                                                const MfDft<PREC>& A, const MfScales& sc) {
    if constexpr (G < SH) {
        y_fwd_mf<N, E, PREC, NSG, G, SH>(v, j, tabs, lds, ls, A, sc);
        y_fwd_mf_groups<N, E, PREC, NSG, G + NSG, SH>(v, j, tabs, lds, ls, A, sc);
    }
}
template <int N, int E, int PREC, int NSG, int G, int SH>
__device__ __forceinline__ void y_inv_mf_groups(float2 (&v)[SH][E], int j, const float2* tabs, float2* lds, int ls,
                                                const MfDft<PREC>& A, const MfScales& sc, float2* __restrict__ dst0,
                                                int ny, float osc) {
    if constexpr (G < SH) {
        y_inv_mf_store<N, E, PREC, NSG, G, SH>(v, j, tabs, lds, ls, A, sc, dst0, ny, osc);
        y_inv_mf_groups<N, E, PREC, NSG, G + NSG, SH>(v, j, tabs, lds, ls, A, sc, dst0, ny, osc);
    }
}

// ---------------------------------------------------------------------
// y pass with two thread sets (even NZ, E = 8 for NZ <= 4 and 4 above, T =
// PY/E in [64, 256], 2T <= 512 threads): set g < 2 transforms signals
// [g*S/2, (g+1)*S/2), so a thread holds half the signals of its E bins; for
// the layer mixing the sets swap half of their bins through LDS, after which
// each thread holds all S signals of E/2 bins, j + T*(i + g*E/2), i < E/2.
// At E = 8 the radix-8 passes need three LDS exchanges per transform where
// radix 4 needs five.
// ---------------------------------------------------------------------
constexpr int y2_E(int nz) { return nz <= 4 ? 8 : 4; }
constexpr bool y2_use(int nz, int Py) {
    return nz % 2 == 0 && Py / y2_E(nz) >= 64 && Py / y2_E(nz) <= 256;
}
constexpr int y2_NSG(int nz) { return (3 * nz / 2) % 3 == 0 ? 3 : ((3 * nz / 2) % 2 == 0 ? 2 : 1); }

// Swap bins between the sets (HB = E/2): set 0 sends bins HB..E-1 of its
// signals and receives the other set's signals at bins 0..HB-1 into the same
// registers; set 1 sends bins 0..HB-1 and receives bins HB..E-1.  Signals in
// groups of NSG.
template <int E, int T, int NSG, int SH, int G>
__device__ __forceinline__ void y_swap(float2 (&v)[SH][E], int g, int j, float2* lds) {
    constexpr int HB = E / 2;
    if constexpr (G < SH) {
        // (selects rather than branches keep v in registers)
        const bool g0 = g == 0;
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NSG; ++s)
#pragma unroll
            for (int i = 0; i < HB; ++i) {
                // the empty asm pins both values in registers, so the select is
                // not folded into a load from a runtime-chosen array element
                float2 hi = v[G + s][i + HB], lo = v[G + s][i];
                asm volatile("" : "+v"(hi.x), "+v"(hi.y), "+v"(lo.x), "+v"(lo.y));
                lds[((g * NSG + s) * HB + i) * T + j] = g0 ? hi : lo;
            }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NSG; ++s)
#pragma unroll
            for (int i = 0; i < HB; ++i) {
                const float2 in = lds[(((1 - g) * NSG + s) * HB + i) * T + j];
                v[G + s][i + HB] = g0 ? in : v[G + s][i + HB];
                v[G + s][i] = g0 ? v[G + s][i] : in;
            }
        y_swap<E, T, NSG, SH, G + NSG>(v, g, j, lds);
    }
}

// Body: kx, thread tid < 2T, nkx = L, LDS at lds; UNI as for the one-set pass.
template <int NZ, int PY> constexpr int y2_lds_bytes(int prec) {
    return prec == 0 ? (int)sizeof(float2) * (2 * y2_NSG(NZ) * lds_len(PY) + tw_len(PY, y2_E(NZ)))
                     : (int)sizeof(float2) * (2 * y2_NSG(NZ) * lds_len(PY) + mf_tw_len(PY, y2_E(NZ))) +
                           (int)sizeof(float) * 16;
}
template <int NZ, int PY, int PREC, bool UNI>
__device__ __forceinline__ void ypass2_body(const ChainDesc& cd, const float* __restrict__ K,
                                            const float2* __restrict__ tw, float kmax, int kx, int tid, int nkx,
                                            float2* lds) {
    const SweepArgs a = cd.a;
    float2* __restrict__ X = cd.X;
    constexpr int S = 3 * NZ, SH = S / 2, E = y2_E(NZ), HB = E / 2, T = PY / E, NSG = y2_NSG(NZ);
    constexpr int LS = lds_len(PY), HP = PY / 2, QH = E / 2;
    float2* twl = lds + 2 * NSG * LS;
    const int g = tid / T, j = tid - g * T;
    const int ny = a.ny;
    float2 v[SH][E];
#pragma unroll
    for (int s = 0; s < SH; ++s) {
        const float2* src = X + ((long long)kx * S + g * SH + s) * ny;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int y = j + T * q;
            v[s][q] = (q < QH && y < ny) ? src[y] : make_float2(0.f, 0.f);
        }
    }
    float2* mine = lds + g * NSG * LS;
    [[maybe_unused]] MfScales msc{1.f, 1.f, 1.f};
    if constexpr (PREC == 0) {
        build_twiddles<PY, E, 2 * T>(twl, tw, tid);
        __syncthreads();
        y_groups<PY, E, false, NSG, 0, SH>(v, j, twl, mine, LS);
    } else {
        mf_build_twiddles<PY, E, 2 * T, PREC>(twl, tw, tid);
        if constexpr (PREC == 2) {
            // the block's largest input magnitude bounds every pass's inputs:
            // forward pass 1 (after the radix-E pass over E/2 nonzero points)
            // E/2 * xmax, pass 2 16 times that; inverse pass 1 the mixed
            // spectrum, |H| <= 3 NZ kmax * ny xmax (twice that for the paired
            // kx = 0 block), pass 2 16 times that
            float mx = 0.f;
#pragma unroll
            for (int s = 0; s < SH; ++s)
#pragma unroll
                for (int q = 0; q < QH; ++q) mx = fmaxf(mx, fmaxf(fabsf(v[s][q].x), fabsf(v[s][q].y)));
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
            float* red = (float*)(twl + mf_tw_len(PY, E));
            if ((tid & 63) == 0) red[tid >> 6] = mx;
            __syncthreads();
            mx = 0.f;
#pragma unroll
            for (int w = 0; w < 2 * T / 64; ++w) mx = fmaxf(mx, red[w]);
            const float bf = 0.5f * E * mx, bi = 2.0f * 3.0f * NZ * kmax * (float)ny * mx;
            constexpr float DF = mf_kf(PY, E) >= 2 ? 16.0f : 1.0f, DI = mf_ki(PY, E) >= 2 ? 16.0f : 1.0f;
            const float f1 = mf_scale(bf), i1 = mf_scale(bi);
            msc.f1 = f1;
            msc.i1 = i1 * DF / f1;        // forward result carries f1 / DF
            msc.out = DI / i1;            // inverse result carries i1 / DI
        } else {
            __syncthreads();
        }
        const MfDft<PREC> A = mf_dft16<PREC, false>(tid & 63, tw);
        y_fwd_mf_groups<PY, E, PREC, NSG, 0, SH>(v, j, twl, mine, LS, A, msc);
    }
    if (UNI || kx == 0) y_pair<PY, E, true, NSG, 0, SH>(v, j, mine, LS, kx == 0);
    y_swap<E, T, NSG, SH, 0>(v, g, j, lds);
    // signal s' of bin i: s' < SH ? v[s'][i] : v[s' - SH][i + HB]
    if (kx != 0) {
        auto bin = [&](int i) {
            const int ky = j + T * (i + HB * g);
            return K + ((long long)kx * (HP + 1) + (ky <= HP ? ky : PY - ky)) * 6 * NZ;
        };
        // (for NZ <= 4 the tensor values of bin i+1 are loaded while bin i is
        // mixed; at larger NZ the registers are not there for it)
        constexpr bool PF = NZ <= 4;
        float kc[6 * NZ];
        load_bin<NZ>(kc, bin(0));
#pragma unroll
        for (int i = 0; i < HB; ++i) {
            float kn[6 * NZ];
            if (PF && i + 1 < HB) load_bin<NZ>(kn, bin(i + 1));
            const int ky = j + T * (i + HB * g);
            float2 M[S], H[S];
#pragma unroll
            for (int s = 0; s < SH; ++s) {
                M[s] = v[s][i];
                M[SH + s] = v[s][i + HB];
            }
            mix_layers<NZ>(kc, ky <= HP ? 1.0f : -1.0f, M, H);
#pragma unroll
            for (int s = 0; s < SH; ++s) {
                v[s][i] = H[s];
                v[s][i + HB] = H[SH + s];
            }
            if (i + 1 < HB) {
                if constexpr (PF) {
#pragma unroll
                    for (int t = 0; t < 6 * NZ; ++t) kc[t] = kn[t];
                } else {
                    load_bin<NZ>(kc, bin(i + 1));
                }
            }
        }
    } else {
        // kx = 0 in slots k <= PY/2 and kx = L in slots PY-k (both at +k);
        // the self-paired slots 0 and PY/2 mix the real pair on the diagonal
        const float* K0 = K;
        const float* KL = K + (long long)nkx * (HP + 1) * 6 * NZ;
#pragma unroll
        for (int i = 0; i < HB; ++i) {
            const int ky = j + T * (i + HB * g);
            float2 M[S], H[S];
            float kv[6 * NZ];
#pragma unroll
            for (int s = 0; s < SH; ++s) {
                M[s] = v[s][i];
                M[SH + s] = v[s][i + HB];
            }
            if (ky == 0 || ky == HP) {
                const float* k0 = K0 + (long long)ky * 6 * NZ;
                const float* kl = KL + (long long)ky * 6 * NZ;
#pragma unroll
                for (int t = 0; t < 3 * NZ; ++t) {
                    kv[t] = k0[t];
                    kv[3 * NZ + t] = kl[t];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int zo = 0; zo < NZ; ++zo) {
                        float hr = 0.f, hi = 0.f;
#pragma unroll
                        for (int zi = 0; zi < NZ; ++zi) {
                            const int adz = zo >= zi ? zo - zi : zi - zo;
                            hr += kv[c * NZ + adz] * M[c * NZ + zi].x;
                            hi += kv[3 * NZ + c * NZ + adz] * M[c * NZ + zi].y;
                        }
                        H[c * NZ + zo] = make_float2(hr, hi);
                    }
            } else {
                load_bin<NZ>(kv, ky < HP ? K0 + (long long)ky * 6 * NZ : KL + (long long)(PY - ky) * 6 * NZ);
                mix_layers<NZ>(kv, 1.0f, M, H);
            }
#pragma unroll
            for (int s = 0; s < SH; ++s) {
                v[s][i] = H[s];
                v[s][i + HB] = H[SH + s];
            }
        }
    }
    y_swap<E, T, NSG, SH, 0>(v, g, j, lds);
    if (UNI || kx == 0) y_pair<PY, E, false, NSG, 0, SH>(v, j, mine, LS, kx == 0);
    // inverse transforms group by group, each group's outputs stored as soon
    // as they are final (the stores overlap the next group's transforms)
    if constexpr (PREC == 0) {
        y_inv_store<PY, E, NSG, 0, SH, QH>(v, j, twl, mine, LS, X + ((long long)kx * S + g * SH) * ny, ny);
    } else {
        const MfDft<PREC> Ai = mf_dft16<PREC, true>(tid & 63, tw);
        y_inv_mf_groups<PY, E, PREC, NSG, 0, SH>(v, j, twl, mine, LS, Ai, msc, X + ((long long)kx * S + g * SH) * ny,
                                                 ny, msc.out);
    }
}

// PREC 0: FP32 transforms on the vector units; 1, 2: split BF16 / FP16 radix-16
// stages on the matrix cores (kmax: largest magnitude in K, for the FP16 scales).
template <int NZ, int PY, bool BAT, int PREC>
__global__ __launch_bounds__(2 * PY / y2_E(NZ)) void k_ypass2(ChainDesc d0, const ChainDesc* __restrict__ dl,
                                                   const float* __restrict__ K,
                                                   const float2* __restrict__ tw, float kmax) {
    extern __shared__ float2 lds[];
    ypass2_body<NZ, PY, PREC, false>(chain_at<BAT>(d0, dl, blockIdx.y), K, tw, kmax, blockIdx.x, threadIdx.x,
                                     gridDim.x, lds);
}

// Shapes whose y pass can run split-precision stages: the two-set kernel
// with whole waves per set and at least one radix-16 stage each way.
constexpr bool ysplit_ok(int nz, int Py) {
    return y2_use(nz, Py) && Py / y2_E(nz) >= 64 && mf_kf(Py, y2_E(nz)) >= 1 && mf_rf(Py, y2_E(nz)) <= y2_E(nz) &&
           mf_ri(Py, y2_E(nz)) <= y2_E(nz);
}

template <int NZ, int PY, int PREC>
hipError_t launch_ypass2(const Chains& c, const DemagPlan& p, const float2* tw, hipStream_t s) {
    constexpr int E2 = y2_E(NZ);
    constexpr size_t sh = y2_lds_bytes<NZ, PY>(PREC);
    if (c.many)
        hipLaunchKernelGGL((k_ypass2<NZ, PY, true, PREC>), dim3(p.L, c.n), dim3(2 * PY / E2), sh, s, c.one, c.many,
                           (const float*)p.K, tw, p.kmax);
    else
        hipLaunchKernelGGL((k_ypass2<NZ, PY, false, PREC>), dim3(p.L), dim3(2 * PY / E2), sh, s, c.one, c.many,
                           (const float*)p.K, tw, p.kmax);
    return hipGetLastError();
}

// y-pass launcher for one layer count (instantiated per NZ in its own unit).
template <int NZ, int PY>
hipError_t launch_ypass_py(const Chains& c, const DemagPlan& p, const float2* tw, hipStream_t s) {
    constexpr int E = y_E(NZ, PY);
    if constexpr (y2_use(NZ, PY)) {
        if (p.prec != 0) {
            if constexpr (ysplit_ok(NZ, PY)) {
                if (p.prec == 1) return launch_ypass2<NZ, PY, 1>(c, p, tw, s);
                return launch_ypass2<NZ, PY, 2>(c, p, tw, s);
            } else {
                return hipErrorInvalidValue;   // rejected at context creation
            }
        }
        return launch_ypass2<NZ, PY, 0>(c, p, tw, s);
    } else if constexpr (3 * NZ * E <= 96) {
        if (p.prec != 0) return hipErrorInvalidValue;   // rejected at context creation
        constexpr size_t sh = sizeof(float2) * y1_lds(NZ, PY);
        if (c.many)
            hipLaunchKernelGGL((k_ypass<NZ, PY, true>), dim3(p.L, c.n), dim3(PY / E), sh, s, c.one, c.many,
                               (const float*)p.K, tw);
        else
            hipLaunchKernelGGL((k_ypass<NZ, PY, false>), dim3(p.L), dim3(PY / E), sh, s, c.one, c.many,
                               (const float*)p.K, tw);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;   // rejected at context creation
    }
}

template <int NZ>
hipError_t launch_ypass_nz(const Chains& c, const DemagPlan& p, const float2* tw, hipStream_t s) {
    switch (p.Py) {
        case 1: return launch_ypass_py<NZ, 1>(c, p, tw, s);
        case 2: return launch_ypass_py<NZ, 2>(c, p, tw, s);
        case 4: return launch_ypass_py<NZ, 4>(c, p, tw, s);
        case 8: return launch_ypass_py<NZ, 8>(c, p, tw, s);
        case 16: return launch_ypass_py<NZ, 16>(c, p, tw, s);
        case 32: return launch_ypass_py<NZ, 32>(c, p, tw, s);
        case 64: return launch_ypass_py<NZ, 64>(c, p, tw, s);
        case 128: return launch_ypass_py<NZ, 128>(c, p, tw, s);
        case 256: return launch_ypass_py<NZ, 256>(c, p, tw, s);
        case 512: return launch_ypass_py<NZ, 512>(c, p, tw, s);
        case 1024: return launch_ypass_py<NZ, 1024>(c, p, tw, s);
        case 2048: return launch_ypass_py<NZ, 2048>(c, p, tw, s);
        case 4096: return launch_ypass_py<NZ, 4096>(c, p, tw, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mmc
