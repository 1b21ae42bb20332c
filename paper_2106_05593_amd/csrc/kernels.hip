// Device kernels of libmmc for gfx950 (CDNA4, wave64).
//
// Data layout in HBM ("colour-split SoA", FP32): the two checkerboard colours
// are stored apart, m[colour][component][z][y][x>>1], so a colour pass reads
// and writes its own cells with unit stride and reads the other colour (all of
// its neighbours) with unit stride too.  A row of one colour holds hw =
// ceil(nx/2) slots; cell (x,y,z) has colour (x+y+z)&1 and slot x>>1.
#include "rng.h"

#include <mutex>

namespace mmc {

// ---------------------------------------------------------------------
// Initial state: length m0 of the cell's class; direction uniform (dir) or
// random (Philox tag 1: cos(theta) = 2u0 - 1, phi = 2 pi u1).
// ---------------------------------------------------------------------
__global__ void k_init(SweepArgs a, const ClassCoef* __restrict__ ctab, const uint32_t* __restrict__ cid,
                       float* __restrict__ m, int kind, float dx, float dy, float dz) {
    const long long N = (long long)a.nx * a.ny * a.nz;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < N; p += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(p % a.nx), y = (int)((p / a.nx) % a.ny), z = (int)(p / ((long long)a.nx * a.ny));
        const int c = (x + y + z) & 1;
        const long long idx = ((long long)z * a.ny + y) * a.hw + (x >> 1);
        const uint32_t k = cid ? cid[(long long)c * a.Nc + idx] : 0u;
        const float L = ctab[k].m0;
        float ux = dx, uy = dy, uz = dz;
        if (kind == 1) {
            const uint4 r = philox4x32_10(make_uint4((uint32_t)p, 0u, a.chain, 2u), a.k0, a.k1);
            const float ct = 2.0f * u01(r.x) - 1.0f;
            const float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
            float sp, cp;
            sincospif(2.0f * u01(r.y), &sp, &cp);
            ux = st * cp; uy = st * sp; uz = ct;
        }
        float* o = m + (long long)c * 3 * a.Nc;
        o[idx] = L * ux;
        o[a.Nc + idx] = L * uy;
        o[2 * a.Nc + idx] = L * uz;
    }
}

__global__ void k_layout(SweepArgs a, const float* __restrict__ src, float* __restrict__ dst, int to_split) {
    const long long N = (long long)a.nx * a.ny * a.nz;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < N; p += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(p % a.nx), y = (int)((p / a.nx) % a.ny), z = (int)(p / ((long long)a.nx * a.ny));
        const int c = (x + y + z) & 1;
        const long long idx = ((long long)c * 3) * a.Nc + ((long long)z * a.ny + y) * a.hw + (x >> 1);
        for (int k = 0; k < 3; ++k) {
            if (to_split) dst[idx + k * a.Nc] = src[k * N + p];
            else dst[k * N + p] = src[idx + k * a.Nc];
        }
    }
}

__global__ void k_set_cone(DevState* st, int cone_deg) {
    st->cone_deg = cone_deg;
    const double sh = sin(0.5 * cone_deg * 3.14159265358979323846 / 180.0);
    st->omc = (float)(2.0 * sh * sh);
}

// ---------------------------------------------------------------------
// Total energy terms (kT units, FP64 per cell): bonds to +x/+y/+z, site terms.
// ---------------------------------------------------------------------
__device__ __forceinline__ void load_m(const SweepArgs& a, const float* m, int x, int y, int z, float& mx, float& my, float& mz) {
    const int c = (x + y + z) & 1;
    const long long idx = ((long long)c * 3) * a.Nc + ((long long)z * a.ny + y) * a.hw + (x >> 1);
    mx = m[idx]; my = m[idx + a.Nc]; mz = m[idx + 2 * a.Nc];
}

template <bool CLS>
__global__ __launch_bounds__(256) void k_energy(SweepArgs a, const ClassCoef* __restrict__ ctab, const uint32_t* __restrict__ cid,
                                                const float* __restrict__ m, const float* __restrict__ h,
                                                double* __restrict__ part, int cubic) {
    const long long N = (long long)a.nx * a.ny * a.nz;
    double e[6] = {0, 0, 0, 0, 0, 0};
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < N; p += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(p % a.nx), y = (int)((p / a.nx) % a.ny), z = (int)(p / ((long long)a.nx * a.ny));
        const int c = (x + y + z) & 1;
        const long long idx = ((long long)z * a.ny + y) * a.hw + (x >> 1);
        const uint32_t kp = CLS ? cid[(long long)c * a.Nc + idx] : 0u;
        const ClassCoef C = ctab[kp];
        float mx, my, mz;
        load_m(a, m, x, y, z, mx, my, mz);
        const int nb[3][3] = {{x + 1, y, z}, {x, y + 1, z}, {x, y, z + 1}};
        const bool has[3] = {x + 1 < a.nx, y + 1 < a.ny, z + 1 < a.nz};
        const float w[3] = {a.wx, a.wy, a.wz};
        for (int d = 0; d < 3; ++d) {
            if (!has[d]) continue;
            float qx, qy, qz;
            load_m(a, m, nb[d][0], nb[d][1], nb[d][2], qx, qy, qz);
            double ww = w[d];
            if (CLS) {
                const int cq = (nb[d][0] + nb[d][1] + nb[d][2]) & 1;
                const long long iq = ((long long)nb[d][2] * a.ny + nb[d][1]) * a.hw + (nb[d][0] >> 1);
                if (cid[(long long)cq * a.Nc + iq] != kp) ww *= a.bscale;
            }
            const double d0 = (double)mx - qx, d1 = (double)my - qy, d2 = (double)mz - qz;
            e[0] += ww * (d0 * d0 + d1 * d1 + d2 * d2);
            if (d == 0) e[1] += -(double)a.cdx * ((double)mz * qx - (double)mx * qz);
            if (d == 1) e[1] += -(double)a.cdy * ((double)mz * qy - (double)my * qz);
        }
        // (class terms are in units of the class's kT: 1/tsc converts to the chain's kT0)
        const double cs = CLS ? 1.0 / (double)C.tsc : 1.0;
        if (cubic) {   // Eq. 12 on the direction cosines of m along the crystal axes
            const double L = sqrt((double)mx * mx + (double)my * my + (double)mz * mz);
            if (L > 0.0) {
                const double p1 = ((double)mx * C.ex + (double)my * C.ey + (double)mz * C.ez) / L;
                const double p2 = ((double)mx * C.fx + (double)my * C.fy + (double)mz * C.fz) / L;
                const double p3 = ((double)mx * C.gx + (double)my * C.gy + (double)mz * C.gz) / L;
                const double s1 = p1 * p1, s2 = p2 * p2, s3 = p3 * p3;
                e[2] += cs * ((double)C.ka1 * (s1 * s2 + s1 * s3 + s2 * s3) + (double)C.ka2 * s1 * s2 * s3);
            }
        } else {       // Eq. 11, m non-unit
            const double dd = (double)mx * C.ex + (double)my * C.ey + (double)mz * C.ez;
            const double u = 1.0 - dd * dd;
            e[2] += cs * ((double)C.ka1 * u + (double)C.ka2 * u * u);
        }
        e[3] += -((double)a.bx * mx + (double)a.by * my + (double)a.bz * mz);
        const double q = (double)mx * mx + (double)my * my + (double)mz * mz;
        if (C.below != 0.0f) { const double dq = q - C.me2; e[4] += cs * (double)C.la * dq * dq; }
        else e[4] += cs * ((double)C.lb * q + (double)C.lbc * q * q);
        if (h) {
            const long long ih = ((long long)c * 3) * a.Nc + idx;
            e[5] += -0.5 * (double)a.cdm * ((double)mx * h[ih] + (double)my * h[ih + a.Nc] + (double)mz * h[ih + 2 * a.Nc]);
        }
    }
    __shared__ double red[4][6];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < 6; ++k) e[k] = wave_sum(e[k]);
    if (lane == 0) for (int k = 0; k < 6; ++k) red[wv][k] = e[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 6; ++k) {
            double t = 0;
            for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) t += red[w2][k];
            part[6 * blockIdx.x + k] = t;
        }
    }
}

// ---------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------

hipError_t launch_init(const SweepArgs& a, const ClassCoef* ctab, const uint32_t* cid, float* m, int kind,
                       float dx, float dy, float dz, hipStream_t s) {
    const long long N = (long long)a.nx * a.ny * a.nz;
    const int blocks = (int)std::min<long long>((N + 255) / 256, 65536);
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, s, a, ctab, cid, m, kind, dx, dy, dz);
    return hipGetLastError();
}

hipError_t launch_to_split(const SweepArgs& a, const float* nat, float* split, hipStream_t s) {
    const long long N = (long long)a.nx * a.ny * a.nz;
    const int blocks = (int)std::min<long long>((N + 255) / 256, 65536);
    hipLaunchKernelGGL(k_layout, dim3(blocks), dim3(256), 0, s, a, nat, split, 1);
    return hipGetLastError();
}

hipError_t launch_from_split(const SweepArgs& a, const float* split, float* nat, hipStream_t s) {
    const long long N = (long long)a.nx * a.ny * a.nz;
    const int blocks = (int)std::min<long long>((N + 255) / 256, 65536);
    hipLaunchKernelGGL(k_layout, dim3(blocks), dim3(256), 0, s, a, split, nat, 0);
    return hipGetLastError();
}

hipError_t launch_set_cone(DevState* st, int cone_deg, hipStream_t s) {
    hipLaunchKernelGGL(k_set_cone, dim3(1), dim3(1), 0, s, st, cone_deg);
    return hipGetLastError();
}

hipError_t launch_energy(const SweepArgs& a, bool classes, bool cubic, const ClassCoef* ctab, const uint32_t* cid,
                         const float* m, const float* h, double* part, hipStream_t s, int* nblk_out) {
    const long long N = (long long)a.nx * a.ny * a.nz;
    const int blocks = (int)std::min<long long>((N + 255) / 256, kEnergyMaxBlocks);
    *nblk_out = blocks;
    const int cb = cubic ? 1 : 0;
    if (classes) hipLaunchKernelGGL(k_energy<true>, dim3(blocks), dim3(256), 0, s, a, ctab, cid, m, h, part, cb);
    else hipLaunchKernelGGL(k_energy<false>, dim3(blocks), dim3(256), 0, s, a, ctab, cid, m, h, part, cb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Allocation-free energy: the per-block partial sums of k_energy live in a
// static device array instead of a buffer of the context.  Each GPU holds its
// own copy until the process ends, and every call on a GPU shares it, so
// calls that overlap on one GPU race.  Host code takes the array's device
// address from energy_scratch(), never from its name.
// ---------------------------------------------------------------------
static __device__ __align__(256) double scratch[6 * kEnergyMaxBlocks];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

hipError_t energy_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the device must be current
    double* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

double* energy_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

// Sum of the nb block partials per term in block order, times kT, and their
// total in term order: the same operations, in the same order, as the host
// sum of mmc_energy, so both give the same doubles.
__global__ void k_energy_sum(const double* __restrict__ part, int nb, double kT, double* __restrict__ out) {
#pragma clang fp contract(off)
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double t[6] = {0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < 6; ++k) t[k] += part[6 * b + k];
    double tot = 0;
    for (int k = 0; k < 6; ++k) {
        t[k] *= kT;
        tot += t[k];
        out[k] = t[k];
    }
    out[6] = tot;
}

hipError_t launch_energy_sum(const double* part, int nb, double kT, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_sum, dim3(1), dim3(64), 0, s, part, nb, kT, out);
    return hipGetLastError();
}

}  // namespace mmc
