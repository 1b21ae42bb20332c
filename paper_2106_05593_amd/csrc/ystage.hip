// Staged y pass of the demag refresh (paper Sec. III, Eq. 14), for shapes the
// one-kernel y pass cannot hold in registers: more than 8 layers, or a padded
// y length whose 3*nz signals per kx exceed its register budget.
//
// The one-kernel y pass keeps all 3*nz signals of one kx in registers so that
// the layer mixing needs no memory round trip.  Here the three steps are
// separate kernels that meet in a work buffer W (complex, [kx][s][PY], after
// the x-spectrum X in the same allocation):
//   1. k_ys_col<PY, false>: forward y transform of each (kx, s) column of X, zero-padded
//      from ny to PY, into W (3 signals per thread group; the kx = 0 group,
//      which carries the real pair kx = 0 and kx = L packed as X0 + i XL, also
//      splits the pair as the one-kernel pass does);
//   2. k_ys_mixn / k_ys_mix: one thread per (kx, ky) bin mixes the 3*nz
//      signals over layers, H_i(z) = sum_z' sum_j K_ij(z - z') M_j(z'), in
//      place in W: for 9..16 layers with nz fixed at compile time (everything
//      in registers), otherwise with nz a runtime value up to the template's
//      NZB (the bin's tensor values staged in LDS, its inputs in registers);
//   3. k_ys_col<PY, true>: inverse y transform of each column of W (merging the kx = 0
//      pair back first), cropped to ny, into X.
// The arithmetic of each step is the one-kernel pass's (same FFT engine, same
// mixing formulas and tensor layout); only the order of memory traffic
// differs.  W costs L * 3nz * PY * 8 bytes of HBM.
#include "demag_fft.h"

namespace mmc {

// thread groups of PY/E threads, NG of them per block (at least 256 threads)
constexpr int ys_E(int Py) { return y_E(0, Py); }
constexpr int ys_T(int Py) { return Py / ys_E(Py); }
constexpr int ys_NG(int Py) { return ys_T(Py) >= 256 ? 1 : 256 / ys_T(Py); }
constexpr int ys_NSG(int Py) { return Py >= 4096 ? 1 : 3; }   // signals per LDS exchange
template <int PY> constexpr size_t ys_lds() {
    return ((size_t)ys_NG(PY) * ys_NSG(PY) * lds_len(PY) + tw_len(PY, ys_E(PY))) * sizeof(float2);
}

// Forward (INV = false: X -> W) or inverse (INV = true: W -> X) y transforms of
// items (kx, sg): signals 3 sg .. 3 sg + 2 of kx; S3 = S / 3 items per kx.
template <int PY, bool INV, bool BAT>
__global__ __launch_bounds__(ys_NG(PY) * ys_T(PY)) void k_ys_col(ChainDesc d0, const ChainDesc* __restrict__ dl,
                                                                 int S, int L, long long woff,
                                                                 const float2* __restrict__ tw) {
    constexpr int E = ys_E(PY), T = ys_T(PY), NG = ys_NG(PY), NSG = ys_NSG(PY), LS = lds_len(PY);
    constexpr int QH = E > 1 ? E / 2 : 1;   // registers holding y < PY/2
    extern __shared__ float2 lds[];
    const ChainDesc& cd = chain_at<BAT>(d0, dl, blockIdx.y);
    const int ny = cd.a.ny;
    const int S3 = S / 3;
    const int g = threadIdx.x / T, j = threadIdx.x - g * T;
    const long long item = (long long)blockIdx.x * NG + g;
    const bool act = item < (long long)L * S3;
    const int kx = act ? (int)(item / S3) : 0, s0 = act ? 3 * (int)(item - (long long)kx * S3) : 0;
    // the block holds a kx = 0 item (block-uniform: items are numbered kx-major)
    const bool has0 = (long long)blockIdx.x * NG < S3;
    float2* glds = lds + g * NSG * LS;
    float2* twl = lds + NG * NSG * LS;
    float2* __restrict__ X = cd.X;
    float2* __restrict__ W = cd.X + woff;
    float2 v[3][E];
    if (!INV) {
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const float2* src = X + ((long long)kx * S + s0 + s) * ny;
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int y = j + T * q;
                v[s][q] = (act && q < QH && y < ny) ? src[y] : make_float2(0.f, 0.f);
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const float2* src = W + ((long long)kx * S + s0 + s) * PY;
#pragma unroll
            for (int q = 0; q < E; ++q) v[s][q] = act ? src[j + T * q] : make_float2(0.f, 0.f);
        }
    }
    build_twiddles<PY, E, NG * T>(twl, tw, threadIdx.x);
    __syncthreads();
    if (!INV) {
        y_groups<PY, E, false, NSG, 0, 3>(v, j, twl, glds, LS);
        if (has0) y_pair<PY, E, true, NSG, 0, 3>(v, j, glds, LS, act && kx == 0);
        if (act) {
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                float2* dst = W + ((long long)kx * S + s0 + s) * PY;
#pragma unroll
                for (int q = 0; q < E; ++q) dst[j + T * q] = v[s][q];
            }
        }
    } else {
        if (has0) y_pair<PY, E, false, NSG, 0, 3>(v, j, glds, LS, act && kx == 0);
        y_groups<PY, E, true, NSG, 0, 3>(v, j, twl, glds, LS);
        if (act) {
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                float2* dst = X + ((long long)kx * S + s0 + s) * ny;
#pragma unroll
                for (int q = 0; q < QH; ++q) {
                    const int y = j + T * q;
                    if (y < ny) dst[y] = v[s][q];
                }
            }
        }
    }
}

// Layer mixing of one bin per thread, nz <= NZB layers (runtime).  Bin b =
// kx * PY + ky; the tensor spectrum K[kx'][ky'][q][dz] holds (L+1) x (PY/2+1)
// bins of 6 nz values (xx, yy, zz, xy real; xz, yz imaginary, stored as their
// imaginary parts), ky' = ky or PY - ky with the xy and yz signs flipped past
// PY/2.  The kx = 0 slots hold kx = 0 at ky <= PY/2 and kx = L at PY - ky
// (both at +ky); the self-paired slots 0 and PY/2 hold the real pair (kx = 0
// in the real part, kx = L in the imaginary part), mixed by the diagonal
// components only (the others vanish on those bins).
constexpr int ys_BT(int nzb) { return nzb <= 16 ? 128 : 64; }
template <int NZB, bool BAT>
__global__ __launch_bounds__(ys_BT(NZB)) void k_ys_mix(ChainDesc d0, const ChainDesc* __restrict__ dl,
                                                       const float* __restrict__ K, int nz, int L, int PY,
                                                       long long woff) {
    constexpr int BT = ys_BT(NZB);
    extern __shared__ float kl[];   // [6 nz][BT]: this thread's tensor values at kl[i * BT + t]
    const ChainDesc& cd = chain_at<BAT>(d0, dl, blockIdx.y);
    const int t = threadIdx.x;
    const long long b = (long long)blockIdx.x * BT + t;
    const bool act = b < (long long)L * PY;
    const int kx = act ? (int)(b / PY) : 0, ky = act ? (int)(b - (long long)kx * PY) : 0;
    const int HP = PY / 2, S = 3 * nz;
    float2* __restrict__ W = cd.X + woff + (long long)kx * S * PY + ky;
    // which tensor bin, and its sign on the ky-odd components (xy, yz)
    const bool pair = kx == 0 && (ky == 0 || ky == HP);
    long long kb;
    float sy = 1.0f;
    if (kx != 0) {
        kb = (long long)kx * (HP + 1) + (ky <= HP ? ky : PY - ky);
        sy = ky <= HP ? 1.0f : -1.0f;
    } else {
        kb = ky <= HP ? ky : (long long)L * (HP + 1) + (PY - ky);
    }
    if (act) {
        if (!pair) {
            const float* Kp = K + kb * 6 * nz;
            for (int i = 0; i < 6 * nz; ++i) kl[i * BT + t] = Kp[i];
        } else {
            // diagonal components: kx = 0 bin in [0, 3 nz), kx = L bin in [3 nz, 6 nz)
            const float* K0 = K + (long long)ky * 6 * nz;
            const float* KL = K + ((long long)L * (HP + 1) + ky) * 6 * nz;
            for (int i = 0; i < 3 * nz; ++i) {
                kl[i * BT + t] = K0[i];
                kl[(3 * nz + i) * BT + t] = KL[i];
            }
        }
    }
    // (each thread reads only its own LDS column: no barrier needed)
    if (!act) return;
    float2 M[3 * NZB];
#pragma unroll
    for (int s = 0; s < 3 * NZB; ++s) {
        const int c = s / NZB, z = s - c * NZB;
        M[s] = z < nz ? W[(long long)(c * nz + z) * PY] : make_float2(0.f, 0.f);
    }
#pragma unroll 1
    for (int zo = 0; zo < nz; ++zo) {
        float2 hx = make_float2(0.f, 0.f), hy = hx, hz = hx;
        if (!pair) {
#pragma unroll
            for (int zi = 0; zi < NZB; ++zi) {
                if (zi < nz) {
                    const int dz = zo - zi, adz = dz >= 0 ? dz : -dz;
                    const float sz = dz >= 0 ? 1.0f : -1.0f;
                    const float kxx = kl[(0 * nz + adz) * BT + t], kyy = kl[(1 * nz + adz) * BT + t];
                    const float kzz = kl[(2 * nz + adz) * BT + t];
                    const float kxy = sy * kl[(3 * nz + adz) * BT + t], kxz = sz * kl[(4 * nz + adz) * BT + t];
                    const float kyz = sy * sz * kl[(5 * nz + adz) * BT + t];
                    const float2 Mx = M[0 * NZB + zi], My = M[1 * NZB + zi], Mz = M[2 * NZB + zi];
                    // xz, yz spectra are imaginary: (i k) M = (-k M.y, k M.x)
                    hx.x += kxx * Mx.x + kxy * My.x - kxz * Mz.y;
                    hx.y += kxx * Mx.y + kxy * My.y + kxz * Mz.x;
                    hy.x += kxy * Mx.x + kyy * My.x - kyz * Mz.y;
                    hy.y += kxy * Mx.y + kyy * My.y + kyz * Mz.x;
                    hz.x += -kxz * Mx.y - kyz * My.y + kzz * Mz.x;
                    hz.y += kxz * Mx.x + kyz * My.x + kzz * Mz.y;
                }
            }
        } else {
#pragma unroll
            for (int zi = 0; zi < NZB; ++zi) {
                if (zi < nz) {
                    const int adz = zo >= zi ? zo - zi : zi - zo;
                    hx.x += kl[(0 * nz + adz) * BT + t] * M[0 * NZB + zi].x;
                    hy.x += kl[(1 * nz + adz) * BT + t] * M[1 * NZB + zi].x;
                    hz.x += kl[(2 * nz + adz) * BT + t] * M[2 * NZB + zi].x;
                    hx.y += kl[(3 * nz + 0 * nz + adz) * BT + t] * M[0 * NZB + zi].y;
                    hy.y += kl[(3 * nz + 1 * nz + adz) * BT + t] * M[1 * NZB + zi].y;
                    hz.y += kl[(3 * nz + 2 * nz + adz) * BT + t] * M[2 * NZB + zi].y;
                }
            }
        }
        W[(long long)(0 * nz + zo) * PY] = hx;
        W[(long long)(1 * nz + zo) * PY] = hy;
        W[(long long)(2 * nz + zo) * PY] = hz;
    }
}

// The same mixing with the layer count NZ fixed at compile time (9 <= NZ <= 16):
// the bin's 6 NZ tensor values and 3 NZ inputs in registers, the pair loop
// unrolled (the mixing formulas of the one-kernel y pass), each output layer
// stored as soon as it is summed.  Up to 10 layers the register budget is set
// for two waves per SIMD (10 layers spill 28 bytes per lane and still run 7 %
// faster than at one wave); above, one wave (at two, 11 layers spill 164 bytes
// and more).
template <int NZ, bool BAT>
__global__ __launch_bounds__(128, NZ <= 10 ? 2 : 1) void k_ys_mixn(ChainDesc d0, const ChainDesc* __restrict__ dl,
                                                 const float* __restrict__ K, int L, int PY, long long woff) {
    const ChainDesc& cd = chain_at<BAT>(d0, dl, blockIdx.y);
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= (long long)L * PY) return;
    const int kx = (int)(b / PY), ky = (int)(b - (long long)kx * PY);
    constexpr int S = 3 * NZ;
    const int HP = PY / 2;
    float2* __restrict__ W = cd.X + woff + (long long)kx * S * PY + ky;
    float2 M[S];
#pragma unroll
    for (int s = 0; s < S; ++s) M[s] = W[(long long)s * PY];
    float kv[6 * NZ];
    if (kx == 0 && (ky == 0 || ky == HP)) {
        // the real pair: diagonal components, kx = 0 on the real part and kx = L on the imaginary part
        const float* k0 = K + (long long)ky * 6 * NZ;
        const float* kl = K + ((long long)L * (HP + 1) + ky) * 6 * NZ;
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
                W[(long long)(c * NZ + zo) * PY] = make_float2(hr, hi);
            }
        return;
    }
    long long kb;
    float sy = 1.0f;
    if (kx != 0) {
        kb = (long long)kx * (HP + 1) + (ky <= HP ? ky : PY - ky);
        sy = ky <= HP ? 1.0f : -1.0f;
    } else {
        kb = ky <= HP ? ky : (long long)L * (HP + 1) + (PY - ky);
    }
    load_bin<NZ>(kv, K + kb * 6 * NZ);
    // the ky-odd components (xy, yz) carry sy once; the z-odd ones (xz, yz)
    // take the sign of dz, known at compile time in the unrolled loops
#pragma unroll
    for (int i = 0; i < NZ; ++i) {
        kv[3 * NZ + i] *= sy;
        kv[5 * NZ + i] *= sy;
    }
#pragma unroll
    for (int zo = 0; zo < NZ; ++zo) {
        float2 hx = make_float2(0.f, 0.f), hy = hx, hz = hx;
#pragma unroll
        for (int zi = 0; zi < NZ; ++zi) {
            const int dz = zo - zi, adz = dz >= 0 ? dz : -dz;
            const float kxx = kv[0 * NZ + adz], kyy = kv[1 * NZ + adz], kzz = kv[2 * NZ + adz];
            const float kxy = kv[3 * NZ + adz];
            const float kxz = dz >= 0 ? kv[4 * NZ + adz] : -kv[4 * NZ + adz];
            const float kyz = dz >= 0 ? kv[5 * NZ + adz] : -kv[5 * NZ + adz];
            const float2 Mx = M[0 * NZ + zi], My = M[1 * NZ + zi], Mz = M[2 * NZ + zi];
            // xz, yz spectra are imaginary: (i k) M = (-k M.y, k M.x)
            hx.x += kxx * Mx.x + kxy * My.x - kxz * Mz.y;
            hx.y += kxx * Mx.y + kxy * My.y + kxz * Mz.x;
            hy.x += kxy * Mx.x + kyy * My.x - kyz * Mz.y;
            hy.y += kxy * Mx.y + kyy * My.y + kyz * Mz.x;
            hz.x += -kxz * Mx.y - kyz * My.y + kzz * Mz.x;
            hz.y += kxz * Mx.x + kyz * My.x + kzz * Mz.y;
        }
        W[(long long)(0 * NZ + zo) * PY] = hx;
        W[(long long)(1 * NZ + zo) * PY] = hy;
        W[(long long)(2 * NZ + zo) * PY] = hz;
    }
}

template <int NZ>
static hipError_t launch_mixn(const Chains& c, const DemagPlan& p, long long woff, hipStream_t s) {
    const long long bins = (long long)p.L * p.Py;
    const dim3 grid((unsigned)((bins + 127) / 128), c.many ? c.n : 1);
    if (c.many)
        hipLaunchKernelGGL((k_ys_mixn<NZ, true>), grid, dim3(128), 0, s, c.one, c.many, (const float*)p.K, p.L, p.Py,
                           woff);
    else
        hipLaunchKernelGGL((k_ys_mixn<NZ, false>), grid, dim3(128), 0, s, c.one, c.many, (const float*)p.K, p.L, p.Py,
                           woff);
    return hipGetLastError();
}

template <int PY>
static hipError_t launch_cols(bool inv, const Chains& c, const DemagPlan& p, long long woff, const float2* tw,
                              hipStream_t s) {
    constexpr int NT = ys_NG(PY) * ys_T(PY);
    const long long items = (long long)p.L * (p.S / 3);
    const dim3 grid((unsigned)((items + ys_NG(PY) - 1) / ys_NG(PY)), c.many ? c.n : 1);
    const size_t sh = ys_lds<PY>();
    if (inv) {
        if (c.many) hipLaunchKernelGGL((k_ys_col<PY, true, true>), grid, dim3(NT), sh, s, c.one, c.many, p.S, p.L, woff, tw);
        else hipLaunchKernelGGL((k_ys_col<PY, true, false>), grid, dim3(NT), sh, s, c.one, c.many, p.S, p.L, woff, tw);
    } else {
        if (c.many) hipLaunchKernelGGL((k_ys_col<PY, false, true>), grid, dim3(NT), sh, s, c.one, c.many, p.S, p.L, woff, tw);
        else hipLaunchKernelGGL((k_ys_col<PY, false, false>), grid, dim3(NT), sh, s, c.one, c.many, p.S, p.L, woff, tw);
    }
    return hipGetLastError();
}

static hipError_t launch_cols_py(bool inv, const Chains& c, const DemagPlan& p, long long woff, const float2* tw,
                                 hipStream_t s) {
    switch (p.Py) {
        case 1: return launch_cols<1>(inv, c, p, woff, tw, s);
        case 2: return launch_cols<2>(inv, c, p, woff, tw, s);
        case 4: return launch_cols<4>(inv, c, p, woff, tw, s);
        case 8: return launch_cols<8>(inv, c, p, woff, tw, s);
        case 16: return launch_cols<16>(inv, c, p, woff, tw, s);
        case 32: return launch_cols<32>(inv, c, p, woff, tw, s);
        case 64: return launch_cols<64>(inv, c, p, woff, tw, s);
        case 128: return launch_cols<128>(inv, c, p, woff, tw, s);
        case 256: return launch_cols<256>(inv, c, p, woff, tw, s);
        case 512: return launch_cols<512>(inv, c, p, woff, tw, s);
        case 1024: return launch_cols<1024>(inv, c, p, woff, tw, s);
        case 2048: return launch_cols<2048>(inv, c, p, woff, tw, s);
        case 4096: return launch_cols<4096>(inv, c, p, woff, tw, s);
        default: return hipErrorInvalidValue;
    }
}

template <int NZB>
static hipError_t launch_mix(const Chains& c, const DemagPlan& p, int nz, long long woff, hipStream_t s) {
    constexpr int BT = ys_BT(NZB);
    const long long bins = (long long)p.L * p.Py;
    const dim3 grid((unsigned)((bins + BT - 1) / BT), c.many ? c.n : 1);
    const size_t sh = sizeof(float) * 6 * nz * BT;
    if (c.many)
        hipLaunchKernelGGL((k_ys_mix<NZB, true>), grid, dim3(BT), sh, s, c.one, c.many, (const float*)p.K, nz, p.L,
                           p.Py, woff);
    else
        hipLaunchKernelGGL((k_ys_mix<NZB, false>), grid, dim3(BT), sh, s, c.one, c.many, (const float*)p.K, nz, p.L,
                           p.Py, woff);
    return hipGetLastError();
}

bool ystage_needed(int nz, int Py) { return nz > 8 || 3 * nz * y_E(nz, Py) > 96; }
int ystage_max_nz() { return 32; }
long long ystage_work_elems(int L, int S, int Py) { return (long long)L * S * Py; }

hipError_t launch_ystage(const Chains& c, const DemagPlan& p, int nz, const float2* tw, hipStream_t s) {
    if (p.woff <= 0 || p.S != 3 * nz || nz < 1 || nz > 32) return hipErrorInvalidValue;
    hipError_t e = launch_cols_py(false, c, p, p.woff, tw, s);
    if (e != hipSuccess) return e;
    switch (nz) {
        case 9: e = launch_mixn<9>(c, p, p.woff, s); break;
        case 10: e = launch_mixn<10>(c, p, p.woff, s); break;
        case 11: e = launch_mixn<11>(c, p, p.woff, s); break;
        case 12: e = launch_mixn<12>(c, p, p.woff, s); break;
        case 13: e = launch_mixn<13>(c, p, p.woff, s); break;
        case 14: e = launch_mixn<14>(c, p, p.woff, s); break;
        case 15: e = launch_mixn<15>(c, p, p.woff, s); break;
        case 16: e = launch_mixn<16>(c, p, p.woff, s); break;
        default: e = nz <= 8 ? launch_mix<8>(c, p, nz, p.woff, s) : launch_mix<32>(c, p, nz, p.woff, s);
    }
    if (e != hipSuccess) return e;
    return launch_cols_py(true, c, p, p.woff, tw, s);
}

}  // namespace mmc
