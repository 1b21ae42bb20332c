// Device kernels of libmmc for gfx950 (CDNA4, wave64).
//
// Data layout in HBM ("colour-split SoA", FP32): the two checkerboard colours
// are stored apart, m[colour][component][z][y][x>>1], so a colour pass reads
// and writes its own cells with unit stride and reads the other colour (all of
// its neighbours) with unit stride too.  A row of one colour holds hw =
// ceil(nx/2) slots; cell (x,y,z) has colour (x+y+z)&1 and slot x>>1.
#include "mmc_internal.h"

namespace mmc {

// ---------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter (4 words), key (2 words).
// ---------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        uint4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// (x >> 8) * 2^-24: exact in binary32.
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-8f; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

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

// ---------------------------------------------------------------------
// Colour pass: one compound trial move per cell of `colour` (paper Sec. II,
// steps 1-4).  One thread per cell; neighbours are the other colour, which
// this pass does not modify.
// ---------------------------------------------------------------------
template <bool CLS, bool DMG, bool EXACT, bool DMI>
__global__ __launch_bounds__(256) void k_subsweep(SweepArgs a, const ClassCoef* __restrict__ ctab,
                                                  const uint32_t* __restrict__ cid, float* __restrict__ m,
                                                  const float* __restrict__ h, int colour,
                                                  const DevState* __restrict__ st, double* __restrict__ part,
                                                  unsigned long long* __restrict__ pacc,
                                                  uint8_t* __restrict__ acc_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    const int par = (colour + y + z) & 1;
    const int x = 2 * i + par;
    const bool valid = (i < a.hw) && (y < a.ny) && (x < a.nx);
    const long long Nc = a.Nc;
    float* __restrict__ own = m + (long long)colour * 3 * Nc;
    const float* __restrict__ oth = m + (long long)(1 - colour) * 3 * Nc;

    double sx = 0.0, sy = 0.0, sz = 0.0, sq = 0.0;
    unsigned long long nacc = 0;
    if (valid) {
        const unsigned long long sweep = st->sweep;
        const float omc = st->omc;
        const long long row = ((long long)z * a.ny + y) * a.hw;
        const long long idx = row + i;
        const long long pnat = ((long long)z * a.ny + y) * a.nx + x;
        const uint32_t kp = CLS ? cid[(long long)colour * Nc + idx] : 0u;
        const ClassCoef C = ctab[kp];

        const float ax = own[idx], ay = own[Nc + idx], az = own[2 * Nc + idx];
        const double qAd = (double)ax * ax + (double)ay * ay + (double)az * az;
        const float qA = (float)qAd;
        const float len = sqrtf(qA);
        const float inv = 1.0f / len;
        const float nx_ = ax * inv, ny_ = ay * inv, nz_ = az * inv;

        const uint4 r = philox4x32_10(make_uint4((uint32_t)pnat, (uint32_t)sweep, a.chain, (uint32_t)colour), a.k0, a.k1);
        const float u0 = u01(r.x), u1 = u01(r.y), u2 = u01(r.z), u3 = u01(r.w);

        // 1) rotation uniform on the cap of half-angle theta_c
        const float t = u0 * omc;
        const float ct = 1.0f - t, stt = sqrtf(t * (2.0f - t));
        float sp, cp;
        sincospif(2.0f * u1, &sp, &cp);
        // orthonormal frame of n (Duff et al., JCGT 2017)
        const float sg = copysignf(1.0f, nz_);
        const float ia = -1.0f / (sg + nz_);
        const float ib = nx_ * ny_ * ia;
        const float e1x = 1.0f + sg * nx_ * nx_ * ia, e1y = sg * ib, e1z = -sg * nx_;
        const float e2x = ib, e2y = sg + ny_ * ny_ * ia, e2z = -ny_;
        const float dxr = cp * e1x + sp * e2x, dyr = cp * e1y + sp * e2y, dzr = cp * e1z + sp * e2z;
        const float nbx = ct * nx_ + stt * dxr, nby = ct * ny_ + stt * dyr, nbz = ct * nz_ + stt * dzr;

        // 2) length change
        float fm1, lnf;
        if (EXACT) { lnf = (2.0f * u2 - 1.0f) * C.ln1ps; fm1 = expm1f(lnf); }
        else { fm1 = C.sigma * (2.0f * u2 - 1.0f); lnf = log1pf(fm1); }
        const float Lb = (1.0f + fm1) * len;
        const float bx = Lb * nbx, by = Lb * nby, bz = Lb * nbz;
        const float Dx = bx - ax, Dy = by - ay, Dz = bz - az;
        const float Sx = bx + ax, Sy = by + ay, Sz = bz + az;

        // 3) free-energy change in units of kT
        float dF = 0.0f;
        // exchange: sum_j w_j D.(S - 2 m_j)
        float xmx = 0.f, xmy = 0.f, xmz = 0.f, xpx = 0.f, xpy = 0.f, xpz = 0.f;  // x-1, x+1 (0 if absent)
        float ymx = 0.f, ymy = 0.f, ymz = 0.f, ypx = 0.f, ypy = 0.f, ypz = 0.f;  // y-1, y+1
        float ex = 0.0f;
        auto bond = [&](long long j, float w, float& ox, float& oy, float& oz) {
            ox = oth[j]; oy = oth[Nc + j]; oz = oth[2 * Nc + j];
            float ww = w;
            if (CLS) { if (cid[(long long)(1 - colour) * Nc + j] != kp) ww *= a.bscale; }
            ex += ww * (Dx * (Sx - 2.0f * ox) + Dy * (Sy - 2.0f * oy) + Dz * (Sz - 2.0f * oz));
        };
        if (x > 0) bond(par ? idx : idx - 1, a.wx, xmx, xmy, xmz);
        if (x + 1 < a.nx) bond(par ? idx + 1 : idx, a.wx, xpx, xpy, xpz);
        if (y > 0) bond(idx - a.hw, a.wy, ymx, ymy, ymz);
        if (y + 1 < a.ny) bond(idx + a.hw, a.wy, ypx, ypy, ypz);
        {
            float t0, t1, t2;
            if (z > 0) bond(idx - (long long)a.ny * a.hw, a.wz, t0, t1, t2);
            if (z + 1 < a.nz) bond(idx + (long long)a.ny * a.hw, a.wz, t0, t1, t2);
        }
        dF += ex;
        // interfacial DMI (Eq. 15), central differences, missing neighbours = 0
        if (DMI) {
            dF -= a.cdx * (Dz * (xpx - xmx) - Dx * (xpz - xmz)) + a.cdy * (Dz * (ypy - ymy) - Dy * (ypz - ymz));
        }
        // uniaxial anisotropy (Eq. 11)
        {
            const float dA = ax * C.ex + ay * C.ey + az * C.ez;
            const float dB = bx * C.ex + by * C.ey + bz * C.ez;
            const float dd = Dx * C.ex + Dy * C.ey + Dz * C.ez;   // dB - dA
            const float pAmB = -dd * (dA + dB);                  // pA - pB
            const float pS = dA * dA + dB * dB;
            dF += pAmB * (C.ka1 + C.ka2 * (2.0f - pS));
        }
        // Zeeman
        dF -= a.bx * Dx + a.by * Dy + a.bz * Dz;
        // longitudinal (Eq. 7 exponent); qB - qA = ((1+fm1)^2 - 1) qA
        {
            const float dq = fm1 * (2.0f + fm1) * qA;
            if (C.below != 0.0f) {
                const float dA2 = (float)(qAd - C.me2);
                dF += C.la * dq * (2.0f * dA2 + dq);
            } else {
                dF += dq * (C.lb + C.lbc * (2.0f * qA + dq));
            }
        }
        // demag with the frozen field (Eq. 14)
        if (DMG) {
            const float* hc = h + (long long)colour * 3 * Nc;
            dF -= a.cdm * (Dx * hc[idx] + Dy * hc[Nc + idx] + Dz * hc[2 * Nc + idx]);
        }
        // 4) accept with min{1, (mB/mA)^k exp(-dF/kT)}
        const float k = EXACT ? 3.0f : 4.0f;
        const float margin = (k * lnf - dF) - logf(u3);
        const bool ok = margin > 0.0f;
        const float nxv = ok ? bx : ax, nyv = ok ? by : ay, nzv = ok ? bz : az;
        own[idx] = nxv;
        own[Nc + idx] = nyv;
        own[2 * Nc + idx] = nzv;
        if (acc_out) acc_out[pnat] = ok ? 1 : 0;
        nacc = ok ? 1ull : 0ull;
        sx = nxv; sy = nyv; sz = nzv;
        sq = (double)nxv * nxv + (double)nyv * nyv + (double)nzv * nzv;
    }
    // block partials: wave reduction, then fixed-order sum over waves
    __shared__ double red[4][4];
    __shared__ unsigned long long redc[4];
    const int lane = (threadIdx.y * blockDim.x + threadIdx.x) & 63;
    const int wv = (threadIdx.y * blockDim.x + threadIdx.x) >> 6;
    sx = wave_sum(sx); sy = wave_sum(sy); sz = wave_sum(sz); sq = wave_sum(sq);
    nacc = wave_sum_u64(nacc);
    if (lane == 0) { red[wv][0] = sx; red[wv][1] = sy; red[wv][2] = sz; red[wv][3] = sq; redc[wv] = nacc; }
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        const int nw = (blockDim.x * blockDim.y + 63) >> 6;
        double t0 = 0, t1 = 0, t2 = 0, t3 = 0;
        unsigned long long tc = 0;
        for (int w = 0; w < nw; ++w) { t0 += red[w][0]; t1 += red[w][1]; t2 += red[w][2]; t3 += red[w][3]; tc += redc[w]; }
        const long long blk = blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
        part[4 * blk + 0] = t0; part[4 * blk + 1] = t1; part[4 * blk + 2] = t2; part[4 * blk + 3] = t3;
        pacc[blk] = tc;
    }
}

// Ends a sweep: sums both colours' block partials in a fixed order, stores the
// statistics, advances the sweep counter and adapts the cone every
// adapt_every sweeps (rate > 0.55: +1 degree; < 0.45: -1 degree; [1, 180]).
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ part, const unsigned long long* __restrict__ pacc,
                                                  int nblk2, long long N, DevState* __restrict__ st,
                                                  double* __restrict__ series, unsigned long long rec_base) {
    double s[4] = {0, 0, 0, 0};
    unsigned long long c = 0;
    for (int b = threadIdx.x; b < nblk2; b += blockDim.x) {
        for (int k = 0; k < 4; ++k) s[k] += part[4 * b + k];
        c += pacc[b];
    }
    __shared__ double red[4][4];
    __shared__ unsigned long long redc[4];
    for (int k = 0; k < 4; ++k) s[k] = wave_sum(s[k]);
    c = wave_sum_u64(c);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { for (int k = 0; k < 4; ++k) red[wv][k] = s[k]; redc[wv] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[4] = {0, 0, 0, 0};
        unsigned long long tc = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { for (int k = 0; k < 4; ++k) t[k] += red[w][k]; tc += redc[w]; }
        const double inv = 1.0 / (double)N;
        for (int k = 0; k < 4; ++k) st->last[k] = t[k] * inv;
        st->accepts_last = tc;
        st->window += tc;
        const unsigned long long sw = st->sweep;
        if (series) {
            double* o = series + 5 * (sw - rec_base);
            o[0] = t[0] * inv; o[1] = t[1] * inv; o[2] = t[2] * inv; o[3] = t[3] * inv; o[4] = (double)tc;
        }
        if (st->adapt_every > 0 && (sw + 1) % (unsigned long long)st->adapt_every == 0) {
            const unsigned long long tot = (unsigned long long)st->adapt_every * (unsigned long long)N;
            int cd = st->cone_deg;
            if (100ull * st->window > 55ull * tot && cd < 180) cd += 1;
            else if (100ull * st->window < 45ull * tot && cd > 1) cd -= 1;
            st->cone_deg = cd;
            const double sh = sin(0.5 * cd * 3.14159265358979323846 / 180.0);
            st->omc = (float)(2.0 * sh * sh);
            st->window = 0;
        }
        st->sweep = sw + 1;
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
                                                double* __restrict__ part) {
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
        const double dd = (double)mx * C.ex + (double)my * C.ey + (double)mz * C.ez;
        const double u = 1.0 - dd * dd;
        e[2] += (double)C.ka1 * u + (double)C.ka2 * u * u;
        e[3] += -((double)a.bx * mx + (double)a.by * my + (double)a.bz * mz);
        const double q = (double)mx * mx + (double)my * my + (double)mz * mz;
        if (C.below != 0.0f) { const double dq = q - C.me2; e[4] += (double)C.la * dq * dq; }
        else e[4] += (double)C.lb * q + (double)C.lbc * q * q;
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
// Demag field h = -N * m by zero-padded FFT convolution (paper Sec. III).
//   x pass:  rows of nx reals -> Px/2+1 complex bins (Px = padded length),
//            as a half-length complex FFT of z[n] = x[2n] + i x[2n+1].
//            With the colour-split layout x[2n] and x[2n+1] are slot n of the
//            two colour rows.
//   y pass:  per kx column: FFT over padded y of every (component, layer),
//            direct mixing over layers with the tensor spectrum, inverse FFT.
//   x pass back: inverse of the first, writing h of the requested colours.
// LDS FFTs: radix-2 decimation in time, input loaded in bit-reversed order.
// Twiddles tw[j] = exp(-2 pi i j / TW_N), precomputed in FP64.
// ---------------------------------------------------------------------
constexpr int TW_N = 8192;

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) { return bits ? (__brev(v) >> (32 - bits)) : 0u; }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) { return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }  // a * conj(b)

// In-place radix-2 DIT over `nsig` signals of length n (bit-reversed input),
// stored at buf[s*stride + k]; sign < 0 forward, > 0 inverse (unnormalised).
__device__ __forceinline__ void lds_fft(float2* buf, int nsig, int stride, int n, int logn, const float2* __restrict__ tw,
                                        bool inverse) {
    const int half_n = n >> 1;
    for (int lg = 1; lg <= logn; ++lg) {
        const int len = 1 << lg, half = len >> 1;
        const int tstep = TW_N >> lg;
        for (int e = threadIdx.x; e < nsig * half_n; e += blockDim.x) {
            const int s = e / half_n, b = e - s * half_n;
            const int grp = b >> (lg - 1), k = b & (half - 1);
            const int i0 = s * stride + grp * len + k, i1 = i0 + half;
            const float2 w = tw[k * tstep];
            const float2 v = inverse ? cmulc(buf[i1], w) : cmul(buf[i1], w);
            const float2 u = buf[i0];
            buf[i0] = make_float2(u.x + v.x, u.y + v.y);
            buf[i1] = make_float2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

// x forward: grid (ceil(ny/R), S); X[(k*S + s)*ny + y], k in [0, L].
__global__ __launch_bounds__(256) void k_xfwd(SweepArgs a, int L, int logL, int R, int S, const float* __restrict__ m,
                                              float2* __restrict__ X, const float2* __restrict__ tw) {
    extern __shared__ float2 sbuf[];
    const int y0 = blockIdx.x * R, s = blockIdx.y;
    const int comp = s / a.nz, z = s - comp * a.nz;
    for (int e = threadIdx.x; e < R * L; e += blockDim.x) {
        const int r = e / L, n = e - r * L, y = y0 + r;
        float2 v = make_float2(0.f, 0.f);
        if (y < a.ny && n < a.hw) {
            const int ce = (y + z) & 1;
            const long long ro = ((long long)z * a.ny + y) * a.hw + n;
            if (2 * n < a.nx) v.x = m[((long long)ce * 3 + comp) * a.Nc + ro];
            if (2 * n + 1 < a.nx) v.y = m[((long long)(1 - ce) * 3 + comp) * a.Nc + ro];
        }
        sbuf[r * L + bitrev(n, logL)] = v;
    }
    __syncthreads();
    lds_fft(sbuf, R, L, L, logL, tw, false);
    const int wstep = TW_N / (2 * L);
    for (int e = threadIdx.x; e < R * (L + 1); e += blockDim.x) {
        const int k = e / R, r = e - k * R, y = y0 + r;
        if (y >= a.ny) continue;
        const float2 Zk = sbuf[r * L + (k & (L - 1))];
        const float2 Zr = sbuf[r * L + ((L - k) & (L - 1))];
        // A = (Zk + conj Zr)/2, B = (Zk - conj Zr)/(2i), X = A + W^k B
        const float2 A = make_float2(0.5f * (Zk.x + Zr.x), 0.5f * (Zk.y - Zr.y));
        const float2 B = make_float2(0.5f * (Zk.y + Zr.y), -0.5f * (Zk.x - Zr.x));
        const float2 W = tw[k * wstep];
        const float2 WB = cmul(W, B);
        X[((long long)k * S + s) * a.ny + y] = make_float2(A.x + WB.x, A.y + WB.y);
    }
}

// x inverse: grid (ceil(ny/R), S); writes h of colour c when (mask >> c) & 1.
__global__ __launch_bounds__(256) void k_xinv(SweepArgs a, int L, int logL, int R, int S, const float2* __restrict__ X,
                                              float* __restrict__ h, int mask, const float2* __restrict__ tw) {
    extern __shared__ float2 sbuf[];
    const int y0 = blockIdx.x * R, s = blockIdx.y;
    const int comp = s / a.nz, z = s - comp * a.nz;
    const int wstep = TW_N / (2 * L);
    for (int e = threadIdx.x; e < R * L; e += blockDim.x) {
        const int k = e / R, r = e - k * R, y = y0 + r;
        float2 Zv = make_float2(0.f, 0.f);
        if (y < a.ny) {
            const float2 Xa = X[((long long)k * S + s) * a.ny + y];
            const float2 Xb = X[((long long)(L - k) * S + s) * a.ny + y];
            // A = Xa + conj Xb, B = (Xa - conj Xb) W^-k, Z = A + i B
            const float2 A = make_float2(Xa.x + Xb.x, Xa.y - Xb.y);
            const float2 D = make_float2(Xa.x - Xb.x, Xa.y + Xb.y);
            const float2 B = cmulc(D, tw[k * wstep]);
            Zv = make_float2(A.x - B.y, A.y + B.x);
        }
        sbuf[r * L + bitrev(k, logL)] = Zv;
    }
    __syncthreads();
    lds_fft(sbuf, R, L, L, logL, tw, true);
    for (int e = threadIdx.x; e < R * L; e += blockDim.x) {
        const int r = e / L, n = e - r * L, y = y0 + r;
        if (y >= a.ny || n >= a.hw) continue;
        const float2 v = sbuf[r * L + n];
        const int ce = (y + z) & 1;
        const long long ro = ((long long)z * a.ny + y) * a.hw + n;
        if (((mask >> ce) & 1) && 2 * n < a.nx) h[((long long)ce * 3 + comp) * a.Nc + ro] = v.x;
        if (((mask >> (1 - ce)) & 1) && 2 * n + 1 < a.nx) h[((long long)(1 - ce) * 3 + comp) * a.Nc + ro] = v.y;
    }
}

// y pass: one block per kx; NT = Py/BINS threads; thread t owns bins b*NT + t.
template <int NZ, int BINS>
__global__ __launch_bounds__(256) void k_ypass(SweepArgs a, int Py, int logPy, float2* __restrict__ X,
                                               const float* __restrict__ K, const float2* __restrict__ tw) {
    constexpr int S = 3 * NZ;
    extern __shared__ float2 sbuf[];
    const int kx = blockIdx.x;
    const int NT = blockDim.x;
    const int ny = a.ny;
    float2 v[S][BINS];
    for (int s = 0; s < S; ++s) {
        const float2* src = X + ((long long)kx * S + s) * ny;
        for (int e = threadIdx.x; e < Py; e += NT) sbuf[bitrev(e, logPy)] = e < ny ? src[e] : make_float2(0.f, 0.f);
        __syncthreads();
        lds_fft(sbuf, 1, Py, Py, logPy, tw, false);
#pragma unroll
        for (int b = 0; b < BINS; ++b) v[s][b] = sbuf[b * NT + threadIdx.x];
        __syncthreads();
    }
    // direct mixing over layers: H_i(z) = sum_z' sum_j K_ij(z - z') M_j(z')
    const int hp = Py >> 1;
#pragma unroll
    for (int b = 0; b < BINS; ++b) {
        const int ky = b * NT + threadIdx.x;
        const int kyp = ky <= hp ? ky : Py - ky;
        const float sy = ky <= hp ? 1.0f : -1.0f;
        const float* Kp = K + ((long long)kx * (hp + 1) + kyp) * 6 * NZ;
        float2 H[S];
#pragma unroll
        for (int s = 0; s < S; ++s) H[s] = make_float2(0.f, 0.f);
#pragma unroll
        for (int zo = 0; zo < NZ; ++zo) {
#pragma unroll
            for (int zi = 0; zi < NZ; ++zi) {
                const int dz = zo - zi, adz = dz >= 0 ? dz : -dz;
                const float sz = dz >= 0 ? 1.0f : -1.0f;
                const float kxx = Kp[0 * NZ + adz], kyy = Kp[1 * NZ + adz], kzz = Kp[2 * NZ + adz];
                const float kxy = sy * Kp[3 * NZ + adz], kxz = sz * Kp[4 * NZ + adz], kyz = sy * sz * Kp[5 * NZ + adz];
                const float2 Mx = v[0 * NZ + zi][b], My = v[1 * NZ + zi][b], Mz = v[2 * NZ + zi][b];
                // xz, yz spectra are imaginary: (i k) M = (-k M.y, k M.x)
                H[0 * NZ + zo].x += kxx * Mx.x + kxy * My.x - kxz * Mz.y;
                H[0 * NZ + zo].y += kxx * Mx.y + kxy * My.y + kxz * Mz.x;
                H[1 * NZ + zo].x += kxy * Mx.x + kyy * My.x - kyz * Mz.y;
                H[1 * NZ + zo].y += kxy * Mx.y + kyy * My.y + kyz * Mz.x;
                H[2 * NZ + zo].x += -kxz * Mx.y - kyz * My.y + kzz * Mz.x;
                H[2 * NZ + zo].y += kxz * Mx.x + kyz * My.x + kzz * Mz.y;
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) v[s][b] = H[s];
    }
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int b = 0; b < BINS; ++b) sbuf[bitrev(b * NT + threadIdx.x, logPy)] = v[s][b];
        __syncthreads();
        lds_fft(sbuf, 1, Py, Py, logPy, tw, true);
        float2* dst = X + ((long long)kx * S + s) * ny;
        for (int e = threadIdx.x; e < ny; e += NT) dst[e] = sbuf[e];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------
static int ilog2(int v) { int l = 0; while ((1 << l) < v) ++l; return l; }

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

template <int NZ, int B>
static hipError_t ypass_launch(const SweepArgs& a, const DemagPlan& p, const float2* tw, hipStream_t s) {
    if constexpr (3 * NZ * B <= 96) {
        hipLaunchKernelGGL((k_ypass<NZ, B>), dim3(p.L + 1), dim3(p.Py / B), sizeof(float2) * p.Py, s, a, p.Py,
                           p.logPy, p.X, (const float*)p.K, tw);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;   // rejected at context creation
    }
}

template <int NZ>
static hipError_t launch_ypass_nz(const SweepArgs& a, const DemagPlan& p, const float2* tw, hipStream_t s) {
    const int bins = p.Py <= 256 ? 1 : p.Py / 256;
    switch (bins) {
        case 1: return ypass_launch<NZ, 1>(a, p, tw, s);
        case 2: return ypass_launch<NZ, 2>(a, p, tw, s);
        case 4: return ypass_launch<NZ, 4>(a, p, tw, s);
        case 8: return ypass_launch<NZ, 8>(a, p, tw, s);
        case 16: return ypass_launch<NZ, 16>(a, p, tw, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_demag_stage(int stage, const SweepArgs& a, const DemagPlan& p, const float* m, float* h,
                              int colour_mask, const float2* tw, hipStream_t s) {
    const size_t shx = sizeof(float2) * (size_t)p.R * p.L;
    const dim3 gx((a.ny + p.R - 1) / p.R, p.S);
    if (stage == 0) {
        hipLaunchKernelGGL(k_xfwd, gx, dim3(256), shx, s, a, p.L, p.logL, p.R, p.S, m, p.X, tw);
        return hipGetLastError();
    }
    if (stage == 2) {
        hipLaunchKernelGGL(k_xinv, gx, dim3(256), shx, s, a, p.L, p.logL, p.R, p.S, (const float2*)p.X, h, colour_mask, tw);
        return hipGetLastError();
    }
    switch (a.nz) {
        case 1: return launch_ypass_nz<1>(a, p, tw, s);
        case 2: return launch_ypass_nz<2>(a, p, tw, s);
        case 3: return launch_ypass_nz<3>(a, p, tw, s);
        case 4: return launch_ypass_nz<4>(a, p, tw, s);
        case 5: return launch_ypass_nz<5>(a, p, tw, s);
        case 6: return launch_ypass_nz<6>(a, p, tw, s);
        case 7: return launch_ypass_nz<7>(a, p, tw, s);
        case 8: return launch_ypass_nz<8>(a, p, tw, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_demag(const SweepArgs& a, const DemagPlan& p, const float* m, float* h, int colour_mask,
                        const float2* tw, hipStream_t s) {
    for (int st = 0; st < 3; ++st) {
        hipError_t e = launch_demag_stage(st, a, p, m, h, colour_mask, tw, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static void sweep_shape(const SweepArgs& a, dim3& grid, dim3& block) {
    int bx = 1;
    while (bx < a.hw && bx < 256) bx <<= 1;
    int by = 256 / bx;
    if (by > a.ny) { by = 1; while (by < a.ny) by <<= 1; }
    block = dim3(bx, by, 1);
    grid = dim3((a.hw + bx - 1) / bx, (a.ny + by - 1) / by, a.nz);
}

int subsweep_blocks(const SweepArgs& a) {
    dim3 g, b;
    sweep_shape(a, g, b);
    return (int)(g.x * g.y * g.z);
}

template <bool CLS, bool DMG, bool EXACT, bool DMI>
static void launch_sub_t(dim3 g, dim3 b, hipStream_t s, const SweepArgs& a, const ClassCoef* ctab, const uint32_t* cid,
                         float* m, const float* h, int colour, const DevState* st, double* part,
                         unsigned long long* pacc, uint8_t* acc) {
    hipLaunchKernelGGL((k_subsweep<CLS, DMG, EXACT, DMI>), g, b, 0, s, a, ctab, cid, m, h, colour, st, part, pacc, acc);
}

hipError_t launch_subsweep(const SweepArgs& a, bool classes, bool demag, bool exact, bool dmi,
                           const ClassCoef* ctab, const uint32_t* cid, float* m, const float* h, int colour,
                           const DevState* st, double* part, unsigned long long* pacc, uint8_t* acc_out,
                           hipStream_t s, int* nblk_out) {
    dim3 g, b;
    sweep_shape(a, g, b);
    if (nblk_out) *nblk_out = (int)(g.x * g.y * g.z);
    const int key = (classes ? 8 : 0) | (demag ? 4 : 0) | (exact ? 2 : 0) | (dmi ? 1 : 0);
#define MMC_SUB(K, A_, B_, C_, D_) case K: launch_sub_t<A_, B_, C_, D_>(g, b, s, a, ctab, cid, m, h, colour, st, part, pacc, acc_out); break;
    switch (key) {
        MMC_SUB(0, false, false, false, false) MMC_SUB(1, false, false, false, true)
        MMC_SUB(2, false, false, true, false)  MMC_SUB(3, false, false, true, true)
        MMC_SUB(4, false, true, false, false)  MMC_SUB(5, false, true, false, true)
        MMC_SUB(6, false, true, true, false)   MMC_SUB(7, false, true, true, true)
        MMC_SUB(8, true, false, false, false)  MMC_SUB(9, true, false, false, true)
        MMC_SUB(10, true, false, true, false)  MMC_SUB(11, true, false, true, true)
        MMC_SUB(12, true, true, false, false)  MMC_SUB(13, true, true, false, true)
        MMC_SUB(14, true, true, true, false)   MMC_SUB(15, true, true, true, true)
    }
#undef MMC_SUB
    return hipGetLastError();
}

hipError_t launch_finalize(const double* part, const unsigned long long* pacc, int nblk, long long N,
                           DevState* st, double* series, unsigned long long rec_base, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, part, pacc, 2 * nblk, N, st, series, rec_base);
    return hipGetLastError();
}

hipError_t launch_set_cone(DevState* st, int cone_deg, hipStream_t s) {
    hipLaunchKernelGGL(k_set_cone, dim3(1), dim3(1), 0, s, st, cone_deg);
    return hipGetLastError();
}

hipError_t launch_energy(const SweepArgs& a, bool classes, const ClassCoef* ctab, const uint32_t* cid,
                         const float* m, const float* h, double* part, hipStream_t s, int* nblk_out) {
    const long long N = (long long)a.nx * a.ny * a.nz;
    const int blocks = (int)std::min<long long>((N + 255) / 256, 2048);
    *nblk_out = blocks;
    if (classes) hipLaunchKernelGGL(k_energy<true>, dim3(blocks), dim3(256), 0, s, a, ctab, cid, m, h, part);
    else hipLaunchKernelGGL(k_energy<false>, dim3(blocks), dim3(256), 0, s, a, ctab, cid, m, h, part);
    return hipGetLastError();
}

}  // namespace mmc
