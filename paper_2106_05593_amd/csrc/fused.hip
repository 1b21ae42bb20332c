// One colour pass with the demag stages on either side of it fused (paper
// Sec. II steps 1-4 with the Sec. III field refreshed before each colour):
// x-inverse of the field that the pass reads, the pass, and the x-forward of
// the state that the next refresh needs, for one tile of rows at a time.
//
// Unfused, each colour c runs y pass, x-inverse (spectrum -> field of colour
// c in HBM), colour pass (field read back) and x-forward of the next refresh
// (the whole state read again).  Here a block takes R = x_rows_conc(L)
// consecutive rows y0 .. y0+R-1 of one layer z:
//   1. for each field component, the inverse x transform of its R rows from
//      the spectrum (the y pass's output), keeping the field of the colour-c
//      cells in LDS;
//   2. the colour pass of those rows (four cells per thread; R * hw / 4 <= 256
//      tasks, one per thread), reading the field from LDS;
//   3. for each component, the forward x transform of the R updated rows
//      (read back through L2) into the spectrum, in place of the rows it read
//      in step 1, ready for the next y pass.
// Each row's transforms and each cell's move are the same arithmetic as in
// the separate kernels, so the state is the same bits; the statistics bins
// follow the tiles.  The spectrum holds the state's x-spectrum between calls
// only within one sweep call: a call starts with a separate x-forward.
//
// The half form (SPEC = false) stops after step 2, and the x-forward of the
// next refresh runs as its own kernel.  It keeps the gain in HBM traffic of
// steps 1-2 (the field never goes to HBM) without step 3's costs: tiles of
// R = x_rows_conc(L) * RPT rows with RPT = 2, so the separate x-forward and the
// x-inverse here both move whole 32-byte runs of 4 rows, and the register
// budget of a kernel without the forward transform.
#include "demag_fft.h"
#include "sweep_kernels.h"

namespace mmc {

// LDS: the x transforms' rows, then (16-byte aligned for the pass's float4
// reads) the field of the colour-c cells, 3 components x R rows x hw <= L/2 slots
template <int L, int RPT> constexpr size_t fused_hb_off() { return (x_lds(L, RPT) + 15) / 16 * 16; }
template <int L, int RPT> constexpr size_t fused_lds() {
    return fused_hb_off<L, RPT>() + sizeof(float) * 3 * x_rows_conc(L) * RPT * (L / 2 > 0 ? L / 2 : 1);
}

// The two transform phases are separate functions so that each gets its own
// register allocation (inlined, values of the transform phases were kept
// live across the colour pass, which then spilled); the pass stays in the
// kernel, where the chain's constants are scalar kernel arguments.
#ifndef MMC_FUSED_MINB
#define MMC_FUSED_MINB 2     // blocks per CU the register budget is sized for
#endif
#ifndef MMC_FUSED_HALF_MINB
#define MMC_FUSED_HALF_MINB 2   // the same for the half form (3 spills 32 bytes per lane and ran 1-2 % slower)
#endif
#ifndef MMC_FUSED_CALLS
#define MMC_FUSED_CALLS 0    // 1: the transform phases as separate functions
#endif
#if MMC_FUSED_CALLS
#define MMC_FUSED_PHASE __device__ __attribute__((noinline))
#else
#define MMC_FUSED_PHASE __device__ __forceinline__
#endif

template <int L, int RPT>
MMC_FUSED_PHASE void fused_field(const ChainDesc& cd, int colour, int z, int y0,
                                                      const float2* __restrict__ tw, int tid, float2* lds, float* hb) {
    constexpr int R = x_rows_conc(L) * RPT;
    const int S = 3 * cd.a.nz;
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        __syncthreads();                                    // earlier readers of lds are done
        xinv_rows<L, RPT, true>(cd, S, c * cd.a.nz + z, y0, colour, tw, tid, lds, hb + c * R * cd.a.hw);
    }
}

// the pass of the tile's R * hw / 4 four-cell tasks, 256 at a time
template <int L, int RPT, bool EXACT, bool DMI>
__device__ __forceinline__ void fused_pass(const ChainDesc& cd, int colour, int z, int y0, int shift,
                                                     int lb, int tid, const float* hb) {
    constexpr int R = x_rows_conc(L) * RPT;
    const SweepArgs& a = cd.a;
    const int hwc = a.hw >> 2;
    double sx = 0, sy = 0, sz = 0, sq = 0;
    unsigned long long nacc = 0;
    const DevState* __restrict__ st = cd.st;
#pragma unroll 1
    for (int task = tid; task < R * hwc; task += 256) {
        const int r = task / hwc, ic = task - r * hwc;
        if (y0 + r < a.ny)
            pass4_cells<true, EXACT, DMI>(a, cd.ctab[0], cd.m, colour, y0 + r, z, ic, hb + r * a.hw + ic * 4,
                                          (long long)R * a.hw, st->sweep, st->omc, nullptr, sx, sy, sz, sq, nacc);
    }
    block_stats(sx, sy, sz, sq, nacc, cd.acc, shift, lb, tid);
}

template <int L>
MMC_FUSED_PHASE void fused_spectrum(const ChainDesc& cd, int z, int y0,
                                                         const float2* __restrict__ tw, int tid, float2* lds) {
    const int S = 3 * cd.a.nz;
#pragma unroll 1
    for (int c = 0; c < 3; ++c) xfwd_rows<L, 1>(cd, S, c * cd.a.nz + z, y0, tw, tid, lds);
}

template <int L, int RPT, bool SPEC, bool EXACT, bool DMI, bool BAT>
__global__ __launch_bounds__(256, SPEC ? MMC_FUSED_MINB : MMC_FUSED_HALF_MINB) void k_fused(
        ChainDesc d0, const ChainDesc* __restrict__ dl, int colour, int shift, const float2* __restrict__ tw) {
    const ChainDesc& cd = chain_at<BAT>(d0, dl, blockIdx.y);
    constexpr int R = x_rows_conc(L) * RPT;
    extern __shared__ float2 lds[];
    float* hb = (float*)((char*)lds + fused_hb_off<L, RPT>());  // [3][R][hw] field of the colour-c cells
    const int tid = threadIdx.x;
    // tiles (y tile, z) with z fastest: the z neighbours of a tile's rows are
    // read by adjacent blocks (same XCD, same L2)
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int z = lb % cd.a.nz, y0 = (lb / cd.a.nz) * R;
    // 1. field of the colour-c cells of the tile's rows
    fused_field<L, RPT>(cd, colour, z, y0, tw, tid, lds, hb);
    __syncthreads();
    // 2. the colour pass of the tile
    fused_pass<L, RPT, EXACT, DMI>(cd, colour, z, y0, shift, lb, tid, hb);
    if constexpr (SPEC) {
        __syncthreads();                                    // the tile's rows are written
        // 3. the x-spectrum of the updated rows
        fused_spectrum<L>(cd, z, y0, tw, tid, lds);
    }
}

template <int L, int RPT, bool SPEC, bool EXACT, bool DMI>
static hipError_t launch_fused_t(const SweepArgs& a, const Chains& c, int colour, int shift, const float2* tw,
                                 hipStream_t s) {
    constexpr int R = x_rows_conc(L) * RPT;
    const dim3 grid(((a.ny + R - 1) / R) * a.nz, c.many ? c.n : 1);
    const size_t sh = fused_lds<L, RPT>();
    if (c.many)
        hipLaunchKernelGGL((k_fused<L, RPT, SPEC, EXACT, DMI, true>), grid, dim3(256), sh, s, c.one, c.many, colour,
                           shift, tw);
    else
        hipLaunchKernelGGL((k_fused<L, RPT, SPEC, EXACT, DMI, false>), grid, dim3(256), sh, s, c.one, c.many, colour,
                           shift, tw);
    return hipGetLastError();
}

template <int L, int RPT, bool SPEC>
static hipError_t launch_fused_f(const SweepArgs& a, bool exact, bool dmi, const Chains& c, int colour, int shift,
                                 const float2* tw, hipStream_t s) {
    if (exact) return dmi ? launch_fused_t<L, RPT, SPEC, true, true>(a, c, colour, shift, tw, s)
                          : launch_fused_t<L, RPT, SPEC, true, false>(a, c, colour, shift, tw, s);
    return dmi ? launch_fused_t<L, RPT, SPEC, false, true>(a, c, colour, shift, tw, s)
               : launch_fused_t<L, RPT, SPEC, false, false>(a, c, colour, shift, tw, s);
}

template <int L>
static hipError_t launch_fused_l(const SweepArgs& a, bool exact, bool dmi, const Chains& c, int colour, int shift,
                                 const float2* tw, hipStream_t s, bool spec) {
    if (spec) return launch_fused_f<L, 1, true>(a, exact, dmi, c, colour, shift, tw, s);
    if constexpr (L >= 32) return launch_fused_f<L, 2, false>(a, exact, dmi, c, colour, shift, tw, s);
    return hipErrorInvalidValue;
}

bool fused_ok(const SweepArgs& a, int L, bool classes, bool spec) {
    // four cells per thread (rows of a multiple of 4 slots), uniform material,
    // at least 4 cells of a row per thread task (hw >= 4); the half form's
    // tiles of 2 x x_rows_conc(L) rows fit the LDS from L = 32 on
    return !classes && a.nx % 8 == 0 && L >= (spec ? 8 : 32) && L <= 2048;
}

hipError_t launch_fused(const SweepArgs& a, const DemagPlan& p, bool exact, bool dmi, const Chains& c, int colour,
                        int shift, const float2* tw, hipStream_t s, bool spec) {
    switch (p.L) {
        case 8: return launch_fused_l<8>(a, exact, dmi, c, colour, shift, tw, s, spec);
        case 16: return launch_fused_l<16>(a, exact, dmi, c, colour, shift, tw, s, spec);
        case 32: return launch_fused_l<32>(a, exact, dmi, c, colour, shift, tw, s, spec);
        case 64: return launch_fused_l<64>(a, exact, dmi, c, colour, shift, tw, s, spec);
        case 128: return launch_fused_l<128>(a, exact, dmi, c, colour, shift, tw, s, spec);
        case 256: return launch_fused_l<256>(a, exact, dmi, c, colour, shift, tw, s, spec);
        case 512: return launch_fused_l<512>(a, exact, dmi, c, colour, shift, tw, s, spec);
        case 1024: return launch_fused_l<1024>(a, exact, dmi, c, colour, shift, tw, s, spec);
        case 2048: return launch_fused_l<2048>(a, exact, dmi, c, colour, shift, tw, s, spec);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mmc
