// Demag refresh launches: x-direction FFT kernels and the dispatcher of the
// three stages (kernels and FFT engine in demag_fft.h; the y pass of each
// layer count is compiled in its own unit, ypass.hip; shapes it cannot hold
// take the staged y pass of ystage.hip).
#include "demag_fft.h"

namespace mmc {

// y-pass launchers instantiated in ypass.hip (one unit per layer count)
extern template hipError_t launch_ypass_nz<1>(const Chains&, const DemagPlan&, const float2*, hipStream_t);
extern template hipError_t launch_ypass_nz<2>(const Chains&, const DemagPlan&, const float2*, hipStream_t);
extern template hipError_t launch_ypass_nz<3>(const Chains&, const DemagPlan&, const float2*, hipStream_t);
extern template hipError_t launch_ypass_nz<4>(const Chains&, const DemagPlan&, const float2*, hipStream_t);
extern template hipError_t launch_ypass_nz<5>(const Chains&, const DemagPlan&, const float2*, hipStream_t);
extern template hipError_t launch_ypass_nz<6>(const Chains&, const DemagPlan&, const float2*, hipStream_t);
extern template hipError_t launch_ypass_nz<7>(const Chains&, const DemagPlan&, const float2*, hipStream_t);
extern template hipError_t launch_ypass_nz<8>(const Chains&, const DemagPlan&, const float2*, hipStream_t);

int ypass_E(int nz, int Py) { return y_E(nz, Py); }
size_t x_pass_lds(int L, int rpt) {
    for (int l = 1; l <= 2048; l *= 2)
        if (l == L) return (size_t)x_rows_conc(l) * rpt * lds_len(l) * sizeof(float2);
    return 0;
}
int x_rpt_default(int L) {
    switch (L) {
        case 1: return x_RPT(1, 0); case 2: return x_RPT(2, 0); case 4: return x_RPT(4, 0);
        case 8: return x_RPT(8, 0); case 16: return x_RPT(16, 0); case 32: return x_RPT(32, 0);
        case 64: return x_RPT(64, 0); case 128: return x_RPT(128, 0); case 256: return x_RPT(256, 0);
        case 512: return x_RPT(512, 0); case 1024: return x_RPT(1024, 0); default: return x_RPT(2048, 0);
    }
}
bool ypass_split_ok(int nz, int Py) { return ysplit_ok(nz, Py); }

// x passes with R = x_rows_conc(L) * RPT rows per block; RPT (rows per thread)
// is the plan's tuned choice for each direction, 1, 2 or 4.
template <int L, int RPT>
static hipError_t launch_x_LR(int stage, const SweepArgs& a, const DemagPlan& p, const Chains& c, int mask,
                              const float2* tw, hipStream_t s) {
    constexpr int R = x_rows_conc(L) * RPT;
    const int gy = c.many ? c.n : 1;
    const dim3 grid(((a.ny + R - 1) / R) * p.S, gy);
    const int ntiles = (a.ny + R - 1) / R;
    if (stage == 0) {
        if (c.many)
            hipLaunchKernelGGL((k_xfwd<L, RPT, true>), grid, dim3(256), x_lds(L, RPT), s, c.one, c.many, p.S, ntiles, tw);
        else
            hipLaunchKernelGGL((k_xfwd<L, RPT, false>), grid, dim3(256), x_lds(L, RPT), s, c.one, c.many, p.S, ntiles, tw);
    } else {
        if (c.many)
            hipLaunchKernelGGL((k_xinv<L, RPT, true>), grid, dim3(256), x_lds(L, RPT), s, c.one, c.many, p.S, ntiles,
                               mask, tw);
        else
            hipLaunchKernelGGL((k_xinv<L, RPT, false>), grid, dim3(256), x_lds(L, RPT), s, c.one, c.many, p.S, ntiles,
                               mask, tw);
    }
    return hipGetLastError();
}

template <int L>
static hipError_t launch_x_L(int stage, const SweepArgs& a, const DemagPlan& p, const Chains& c, int mask,
                             const float2* tw, hipStream_t s) {
    const int rpt = stage == 0 ? p.rpt_f : p.rpt_i;
    if (rpt == 1) return launch_x_LR<L, 1>(stage, a, p, c, mask, tw, s);
    if (rpt == 4) return launch_x_LR<L, 4>(stage, a, p, c, mask, tw, s);
    return launch_x_LR<L, 2>(stage, a, p, c, mask, tw, s);
}

static hipError_t launch_x(int stage, const SweepArgs& a, const DemagPlan& p, const Chains& c, int mask,
                           const float2* tw, hipStream_t s) {
    switch (p.L) {
        case 1: return launch_x_L<1>(stage, a, p, c, mask, tw, s);
        case 2: return launch_x_L<2>(stage, a, p, c, mask, tw, s);
        case 4: return launch_x_L<4>(stage, a, p, c, mask, tw, s);
        case 8: return launch_x_L<8>(stage, a, p, c, mask, tw, s);
        case 16: return launch_x_L<16>(stage, a, p, c, mask, tw, s);
        case 32: return launch_x_L<32>(stage, a, p, c, mask, tw, s);
        case 64: return launch_x_L<64>(stage, a, p, c, mask, tw, s);
        case 128: return launch_x_L<128>(stage, a, p, c, mask, tw, s);
        case 256: return launch_x_L<256>(stage, a, p, c, mask, tw, s);
        case 512: return launch_x_L<512>(stage, a, p, c, mask, tw, s);
        case 1024: return launch_x_L<1024>(stage, a, p, c, mask, tw, s);
        case 2048: return launch_x_L<2048>(stage, a, p, c, mask, tw, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_demag_stage(int stage, const SweepArgs& a, const DemagPlan& p, const Chains& c, int colour_mask,
                              const float2* tw, hipStream_t s) {
    if (stage == 0 || stage == 2) return launch_x(stage, a, p, c, colour_mask, tw, s);
    if (p.woff > 0) return launch_ystage(c, p, a.nz, tw, s);
    switch (a.nz) {
        case 1: return launch_ypass_nz<1>(c, p, tw, s);
        case 2: return launch_ypass_nz<2>(c, p, tw, s);
        case 3: return launch_ypass_nz<3>(c, p, tw, s);
        case 4: return launch_ypass_nz<4>(c, p, tw, s);
        case 5: return launch_ypass_nz<5>(c, p, tw, s);
        case 6: return launch_ypass_nz<6>(c, p, tw, s);
        case 7: return launch_ypass_nz<7>(c, p, tw, s);
        case 8: return launch_ypass_nz<8>(c, p, tw, s);
        default: return hipErrorInvalidValue;
    }
}

template <int L>
static hipError_t launch_xtw_L(float2* tw, hipStream_t s) {
    hipLaunchKernelGGL(k_x_twiddles<L>, dim3(1), dim3(256), 0, s, tw + TW_N, (const float2*)tw);
    return hipGetLastError();
}

hipError_t launch_x_twiddles(const DemagPlan& p, float2* tw, hipStream_t s) {
    switch (p.L) {
        case 1: return launch_xtw_L<1>(tw, s);
        case 2: return launch_xtw_L<2>(tw, s);
        case 4: return launch_xtw_L<4>(tw, s);
        case 8: return launch_xtw_L<8>(tw, s);
        case 16: return launch_xtw_L<16>(tw, s);
        case 32: return launch_xtw_L<32>(tw, s);
        case 64: return launch_xtw_L<64>(tw, s);
        case 128: return launch_xtw_L<128>(tw, s);
        case 256: return launch_xtw_L<256>(tw, s);
        case 512: return launch_xtw_L<512>(tw, s);
        case 1024: return launch_xtw_L<1024>(tw, s);
        case 2048: return launch_xtw_L<2048>(tw, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_demag(const SweepArgs& a, const DemagPlan& p, const Chains& c, int colour_mask, const float2* tw,
                        hipStream_t s) {
    for (int st = 0; st < 3; ++st) {
        hipError_t e = launch_demag_stage(st, a, p, c, colour_mask, tw, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace mmc
