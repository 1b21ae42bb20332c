// Launchers of the colour pass and the end-of-sweep kernel (kernels and their
// bodies in sweep_kernels.h).
#include "sweep_kernels.h"

namespace mmc {

bool pass_vec4(const SweepArgs& a, bool classes) { return !classes && (a.nx % 8 == 0); }

int pass_blocks(const SweepArgs& a, bool classes) {
    const long long threads = (long long)a.ny * a.nz * (pass_vec4(a, classes) ? a.hw / 4 : a.hw);
    return (int)((threads + 255) / 256);
}

template <bool CLS, bool DMG, bool EXACT, bool DMI, bool CUB, bool B>
static void launch_pass_b(const SweepArgs& a, const Chains& c, int colour, int stats, int shift, uint8_t* dec,
                          hipStream_t s) {
    const dim3 grid(pass_blocks(a, CLS || CUB), B ? c.n : 1);
    if constexpr (!CLS && !CUB) {
        if (pass_vec4(a, false)) {
            hipLaunchKernelGGL((k_pass4<DMG, EXACT, DMI, B>), grid, dim3(256), 0, s, c.one, c.many, colour, stats,
                               shift, dec);
            return;
        }
    }
    hipLaunchKernelGGL((k_pass1<CLS, DMG, EXACT, DMI, CUB, B>), grid, dim3(256), 0, s, c.one, c.many, colour, stats,
                       shift, dec);
}

template <bool CLS, bool DMG, bool EXACT, bool DMI>
static void launch_pass_t(const SweepArgs& a, bool cubic, const Chains& c, int colour, int stats, int shift,
                          uint8_t* dec, hipStream_t s) {
    if (cubic) {
        if (c.many) launch_pass_b<CLS, DMG, EXACT, DMI, true, true>(a, c, colour, stats, shift, dec, s);
        else launch_pass_b<CLS, DMG, EXACT, DMI, true, false>(a, c, colour, stats, shift, dec, s);
    } else {
        if (c.many) launch_pass_b<CLS, DMG, EXACT, DMI, false, true>(a, c, colour, stats, shift, dec, s);
        else launch_pass_b<CLS, DMG, EXACT, DMI, false, false>(a, c, colour, stats, shift, dec, s);
    }
}

hipError_t launch_pass(const SweepArgs& a, bool classes, bool demag, bool exact, bool dmi, bool cubic,
                       const Chains& c, int colour, bool stats, int shift, uint8_t* dec, hipStream_t s) {
    const int key = (classes ? 8 : 0) | (demag ? 4 : 0) | (exact ? 2 : 0) | (dmi ? 1 : 0);
    const int st = stats ? 1 : 0;
#define MMC_PASS(K, A_, B_, C_, D_) \
    case K: launch_pass_t<A_, B_, C_, D_>(a, cubic, c, colour, st, shift, dec, s); break;
    switch (key) {
        MMC_PASS(0, false, false, false, false) MMC_PASS(1, false, false, false, true)
        MMC_PASS(2, false, false, true, false)  MMC_PASS(3, false, false, true, true)
        MMC_PASS(4, false, true, false, false)  MMC_PASS(5, false, true, false, true)
        MMC_PASS(6, false, true, true, false)   MMC_PASS(7, false, true, true, true)
        MMC_PASS(8, true, false, false, false)  MMC_PASS(9, true, false, false, true)
        MMC_PASS(10, true, false, true, false)  MMC_PASS(11, true, false, true, true)
        MMC_PASS(12, true, true, false, false)  MMC_PASS(13, true, true, false, true)
        MMC_PASS(14, true, true, true, false)   MMC_PASS(15, true, true, true, true)
    }
#undef MMC_PASS
    return hipGetLastError();
}

hipError_t launch_end_sweep(const Chains& c, int shift, long long N, double* series, unsigned long long rec_base,
                            hipStream_t s) {
    if (c.many)
        hipLaunchKernelGGL(k_end_sweep<true>, dim3(c.n), dim3(kAccBins), 0, s, c.one, c.many, shift, N, series,
                           rec_base);
    else
        hipLaunchKernelGGL(k_end_sweep<false>, dim3(1), dim3(kAccBins), 0, s, c.one, c.many, shift, N, series,
                           rec_base);
    return hipGetLastError();
}

}  // namespace mmc
