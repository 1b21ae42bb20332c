// Colour pass of the micromagnetic Monte Carlo sweep (paper Sec. II, steps
// 1-4, red-black decomposition) for gfx950.
//
// One thread handles C consecutive cells of one colour row (C = 4 with float4
// loads and stores when rows allow it, else 1).  Neighbours belong to the
// other colour, which this pass does not modify.  Statistics: each thread sums
// its cells' new m and |m|^2 in FP64, a block reduces them in a fixed order
// and adds them as fixed-point integers (scale 2^shift) with 64-bit atomics
// into one of kAccBins bins, so the totals do not depend on block scheduling;
// a one-block kernel ends the sweep (means, accept window, cone adaptation,
// sweep counter) and clears the bins.
#pragma once
#include "rng.h"

namespace mmc {

__device__ __forceinline__ int xcd_block_s(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7, xcd = b & 7, i = b >> 3;
    return xcd < rem ? xcd * (per + 1) + i : rem * (per + 1) + (xcd - rem) * per + i;
}

struct Nbr {          // one neighbour: value and exchange weight (0 when absent)
    float x, y, z, w;
};

// Proposal and acceptance of one cell.  Returns the decision, writes the new m.
// TS: per-class temperatures; the exchange, DMI, Zeeman and demag terms are
// formed in units of the chain's kT0 and scaled by C.tsc = T0/T of the class,
// so every term of dF is in units of the cell's own kT (local detailed balance).
// CUB: cubic anisotropy (Eq. 12) in place of the uniaxial form (Eq. 11).
template <bool EXACT, bool DMI, bool DMG, bool TS, bool CUB = false>
__device__ __forceinline__ bool cell_move(const SweepArgs& a, const ClassCoef& C, const uint4 r, const float omc,
                                          const float ax, const float ay, const float az, const Nbr (&nb)[6],
                                          const float hx, const float hy, const float hz,
                                          float& ox, float& oy, float& oz) {
    // nb: 0 x-1, 1 x+1, 2 y-1, 3 y+1, 4 z-1, 5 z+1 (absent: value 0, weight 0)
    const float u0 = u01(r.x), u1 = u01(r.y), u2 = u01(r.z), u3 = u01(r.w);
    const double qAd = (double)ax * ax + (double)ay * ay + (double)az * az;
    const float qA = (float)qAd;
    const float inv = __builtin_amdgcn_rsqf(qA);     // hardware 1/sqrt, ~1 ulp
    const float len = qA * inv;
    const float nx_ = ax * inv, ny_ = ay * inv, nz_ = az * inv;
    // 1) rotation uniform on the cap of half-angle theta_c
    const float t = u0 * omc;
    const float ct = 1.0f - t, stt = sqrtf(t * (2.0f - t));
    float sp, cp;
    sincospif(2.0f * u1, &sp, &cp);
    // orthonormal frame of the current direction (Duff et al., JCGT 2017)
    const float sg = copysignf(1.0f, nz_);
    const float ia = -__builtin_amdgcn_rcpf(sg + nz_);   // |sg + nz| >= 1
    const float ib = nx_ * ny_ * ia;
    const float e1x = 1.0f + sg * nx_ * nx_ * ia, e1y = sg * ib, e1z = -sg * nx_;
    const float e2x = ib, e2y = sg + ny_ * ny_ * ia, e2z = -ny_;
    const float dxr = cp * e1x + sp * e2x, dyr = cp * e1y + sp * e2y, dzr = cp * e1z + sp * e2z;
    const float nbx = ct * nx_ + stt * dxr, nby = ct * ny_ + stt * dyr, nbz = ct * nz_ + stt * dzr;
    // 2) length change (logarithms in base 2 with the hardware log2/exp2)
    float fm1, l2f;
    if (EXACT) { l2f = (2.0f * u2 - 1.0f) * C.ln1ps * 1.44269504088896341f; fm1 = __builtin_amdgcn_exp2f(l2f) - 1.0f; }
    else { fm1 = C.sigma * (2.0f * u2 - 1.0f); l2f = __builtin_amdgcn_logf(1.0f + fm1); }
    const float Lb = (1.0f + fm1) * len;
    const float bx = Lb * nbx, by = Lb * nby, bz = Lb * nbz;
    const float Dx = bx - ax, Dy = by - ay, Dz = bz - az;
    const float Sx = bx + ax, Sy = by + ay, Sz = bz + az;
    // 3) free-energy change / kT (with TS: the chain terms accumulate in dFc)
    float dF = 0.0f, dFc = 0.0f;
    float& dch = TS ? dFc : dF;
#pragma unroll
    for (int k = 0; k < 6; ++k)   // exchange: exact change of sum_bonds w |m_i - m_j|^2
        dch += nb[k].w * (Dx * (Sx - 2.0f * nb[k].x) + Dy * (Sy - 2.0f * nb[k].y) + Dz * (Sz - 2.0f * nb[k].z));
    if (DMI)   // interfacial DMI (Eq. 15), central differences
        dch -= a.cdx * (Dz * (nb[1].x - nb[0].x) - Dx * (nb[1].z - nb[0].z)) +
               a.cdy * (Dz * (nb[3].y - nb[2].y) - Dy * (nb[3].z - nb[2].z));
    if (CUB) {   // cubic anisotropy (Eq. 12): squared direction cosines along the crystal axes e, f, g
        const float a1 = nx_ * C.ex + ny_ * C.ey + nz_ * C.ez, a2 = nx_ * C.fx + ny_ * C.fy + nz_ * C.fz;
        const float a3 = nx_ * C.gx + ny_ * C.gy + nz_ * C.gz;
        const float b1 = nbx * C.ex + nby * C.ey + nbz * C.ez, b2 = nbx * C.fx + nby * C.fy + nbz * C.fz;
        const float b3 = nbx * C.gx + nby * C.gy + nbz * C.gz;
        const float pa = a1 * a1, qa = a2 * a2, ra = a3 * a3, pb = b1 * b1, qb = b2 * b2, rb = b3 * b3;
        dF += C.ka1 * ((pb * (qb + rb) + qb * rb) - (pa * (qa + ra) + qa * ra)) + C.ka2 * (pb * qb * rb - pa * qa * ra);
    } else {   // uniaxial anisotropy (Eq. 11)
        const float dA = ax * C.ex + ay * C.ey + az * C.ez;
        const float dB = bx * C.ex + by * C.ey + bz * C.ez;
        const float dd = Dx * C.ex + Dy * C.ey + Dz * C.ez;
        const float pAmB = -dd * (dA + dB);
        dF += pAmB * (C.ka1 + C.ka2 * (2.0f - (dA * dA + dB * dB)));
    }
    dch -= a.bx * Dx + a.by * Dy + a.bz * Dz;   // Zeeman
    {   // longitudinal (Eq. 7 exponent); qB - qA = ((1+fm1)^2 - 1) qA
        const float dq = fm1 * (2.0f + fm1) * qA;
        if (C.below != 0.0f) dF += C.la * dq * (2.0f * (float)(qAd - C.me2) + dq);
        else dF += dq * (C.lb + C.lbc * (2.0f * qA + dq));
    }
    if (DMG) dch -= a.cdm * (Dx * hx + Dy * hy + Dz * hz);   // frozen demag field (Eq. 14)
    if (TS) dF += C.tsc * dFc;
    // 4) accept with min{1, (mB/mA)^k exp(-dF/kT)} (Eq. 5): ln u3 < k ln f - dF
    const float kexp = EXACT ? 3.0f : 4.0f;
    const bool ok = (kexp * l2f - dF * 1.44269504088896341f) > __builtin_amdgcn_logf(u3);
    ox = ok ? bx : ax;
    oy = ok ? by : ay;
    oz = ok ? bz : az;
    return ok;
}

// Block statistics: fixed-order reduction inside the block, then fixed-point
// atomic adds into bin (logical block index mod kAccBins).
__device__ __forceinline__ void block_stats(double sx, double sy, double sz, double sq, unsigned long long nacc,
                                            SweepAccum* __restrict__ acc, int shift, int lb, int tid) {
    __shared__ double red[4][4];
    __shared__ unsigned long long redc[4];
    const int lane = tid & 63, wv = tid >> 6;
    sx = wave_sum(sx); sy = wave_sum(sy); sz = wave_sum(sz); sq = wave_sum(sq);
    nacc = wave_sum_u64(nacc);
    if (lane == 0) { red[wv][0] = sx; red[wv][1] = sy; red[wv][2] = sz; red[wv][3] = sq; redc[wv] = nacc; }
    __syncthreads();
    if (tid == 0) {
        double tt[4] = {0, 0, 0, 0};
        unsigned long long tc = 0;
        const int nw = 4;   // blocks of 256 threads
        for (int w = 0; w < nw; ++w) { for (int k = 0; k < 4; ++k) tt[k] += red[w][k]; tc += redc[w]; }
        const int b = lb & (kAccBins - 1);
        for (int k = 0; k < 4; ++k)
            atomicAdd((unsigned long long*)&acc->bin[b][k], (unsigned long long)__double2ll_rn(ldexp(tt[k], shift)));
        atomicAdd((unsigned long long*)&acc->bin[b][4], tc);
    }
}

// End of a sweep (one block of kAccBins threads): totals of the bins (exact
// integer sums), means, accept window, cone adaptation (rate > 0.55: +1
// degree, < 0.45: -1 degree, kept in [1, 180]), sweep counter; clears the bins.
// Block b serves chain b.
__device__ __forceinline__ void end_sweep_body(const ChainDesc& cd, int shift, long long N, double* __restrict__ series,
                                               unsigned long long rec_base, int tid) {
    SweepAccum* __restrict__ acc = cd.acc;
    DevState* __restrict__ st = cd.st;
    __shared__ long long fin[kAccBins / 64][5];
    const int lane = tid & 63, wv = tid >> 6;
    long long v[5];
    for (int k = 0; k < 5; ++k) {
        v[k] = acc->bin[tid][k];
        acc->bin[tid][k] = 0;
    }
    for (int k = 0; k < 5; ++k) v[k] = (long long)wave_sum_u64((unsigned long long)v[k]);
    if (lane == 0) for (int k = 0; k < 5; ++k) fin[wv][k] = v[k];
    __syncthreads();
    if (tid != 0) return;
    long long tot[5] = {0, 0, 0, 0, 0};
    for (int w = 0; w < kAccBins / 64; ++w)
        for (int k = 0; k < 5; ++k) tot[k] += fin[w][k];
    double t[4];
    for (int k = 0; k < 4; ++k) t[k] = ldexp((double)tot[k], -shift);
    const unsigned long long tc = (unsigned long long)tot[4];
    const double inv = 1.0 / (double)N;
    for (int k = 0; k < 4; ++k) {
#pragma clang fp contract(off)
        const double mk = t[k] * inv;   // the rounded mean (no fused multiply-add into the running sum)
        st->last[k] = mk;
        st->avg_sum[k] += mk;
    }
    st->avg_n += 1;
    st->accepts_last = tc;
    st->window += tc;
    const unsigned long long sw = st->sweep;
    if (series) {
        double* o = series + 5 * (sw - rec_base);
        o[0] = t[0] * inv; o[1] = t[1] * inv; o[2] = t[2] * inv; o[3] = t[3] * inv; o[4] = (double)tc;
    }
    if (st->adapt_every > 0 && (sw + 1) % (unsigned long long)st->adapt_every == 0) {
        const unsigned long long win_tot = (unsigned long long)st->adapt_every * (unsigned long long)N;
        int cd = st->cone_deg;
        if (100ull * st->window > 55ull * win_tot && cd < 180) cd += 1;
        else if (100ull * st->window < 45ull * win_tot && cd > 1) cd -= 1;
        st->cone_deg = cd;
        const double sh = sin(0.5 * cd * 3.14159265358979323846 / 180.0);
        st->omc = (float)(2.0 * sh * sh);
        st->window = 0;
    }
    st->sweep = sw + 1;
}
template <bool B>
__global__ __launch_bounds__(kAccBins) void k_end_sweep(ChainDesc d0, const ChainDesc* __restrict__ dl, int shift,
                                                        long long N, double* __restrict__ series,
                                                        unsigned long long rec_base) {
    end_sweep_body(chain_at<B>(d0, dl, blockIdx.x), shift, N, series, rec_base, threadIdx.x);
}

// C = 4: rows hold a multiple of 4 slots (nx % 8 == 0), uniform material.
// (single chain: at most 128 VGPRs for four waves per SIMD, measured faster
// than three; the batched form needs a few more registers for its chain view)
// Four consecutive cells of colour `colour` in row (y, z), slots 4 ic .. 4 ic + 3
// (rows hold a multiple of 4 slots).  hp: the frozen field of those slots,
// component c at hp + c * hcs (float4-aligned; DMG only).  Adds the new
// m, |m|^2 and accepted moves to the running sums.
template <bool DMG, bool EXACT, bool DMI>
__device__ __forceinline__ void pass4_cells(const SweepArgs& a, const ClassCoef& C, float* __restrict__ m, int colour,
                                            int y, int z, int ic, const float* hp, long long hcs,
                                            unsigned long long sweep, float omc, uint8_t* __restrict__ dec,
                                            double& sx, double& sy, double& sz, double& sq,
                                            unsigned long long& nacc) {
    const int row = z * a.ny + y;
    const int par = (colour + y + z) & 1;
    const int Nc = (int)a.Nc;
    const int i0 = ic * 4;
    const int o0 = row * a.hw + i0;
    float* own = m + colour * 3 * Nc;
    const float* oth = m + (1 - colour) * 3 * Nc;
    float4 A[3], O[3], YM[3], YP[3], ZM[3], ZP[3], H[3];
    float EL[3], ER[3];
    const bool hy_m = y > 0, hy_p = y + 1 < a.ny, hz_m = z > 0, hz_p = z + 1 < a.nz;
    const bool el = i0 > 0, er = i0 + 4 < a.hw;
    // neighbour rows/slots: load from a clamped (always valid) address, zero what is absent
    const int dym = hy_m ? -a.hw : 0, dyp = hy_p ? a.hw : 0;
    const int dzm = hz_m ? -a.ny * a.hw : 0, dzp = hz_p ? a.ny * a.hw : 0;
    const int del = el ? -1 : 0, der = er ? 4 : 3;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float* oc = oth + c * Nc + o0;
        A[c] = *(const float4*)(own + c * Nc + o0);
        O[c] = *(const float4*)oc;
        YM[c] = *(const float4*)(oc + dym);
        YP[c] = *(const float4*)(oc + dyp);
        ZM[c] = *(const float4*)(oc + dzm);
        ZP[c] = *(const float4*)(oc + dzp);
        EL[c] = oc[del];
        ER[c] = oc[der];
        if (DMG) H[c] = *(const float4*)(hp + c * hcs);
        if (!hy_m) YM[c] = zero4;
        if (!hy_p) YP[c] = zero4;
        if (!hz_m) ZM[c] = zero4;
        if (!hz_p) ZP[c] = zero4;
        if (!el) EL[c] = 0.f;
        if (!er) ER[c] = 0.f;
    }
    auto comp = [](const float4& v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w)); };
    float4 OUT[3];
    const int xbase = 2 * i0 + par;
    const unsigned pbase = (unsigned)((z * a.ny + y) * a.nx + xbase);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = xbase + 2 * k;
        Nbr nb[6];
        // x-1: other slot i0+k-1 (par 0) or i0+k (par 1); x+1: i0+k (par 0) or i0+k+1 (par 1)
        float lx, ly, lz, rx, ry, rz;
        if (par) {
            lx = comp(O[0], k); ly = comp(O[1], k); lz = comp(O[2], k);
            if (k < 3) { rx = comp(O[0], k + 1); ry = comp(O[1], k + 1); rz = comp(O[2], k + 1); }
            else { rx = ER[0]; ry = ER[1]; rz = ER[2]; }
        } else {
            if (k > 0) { lx = comp(O[0], k - 1); ly = comp(O[1], k - 1); lz = comp(O[2], k - 1); }
            else { lx = EL[0]; ly = EL[1]; lz = EL[2]; }
            rx = comp(O[0], k); ry = comp(O[1], k); rz = comp(O[2], k);
        }
        nb[0] = {lx, ly, lz, x > 0 ? a.wx : 0.f};
        nb[1] = {rx, ry, rz, x + 1 < a.nx ? a.wx : 0.f};
        nb[2] = {comp(YM[0], k), comp(YM[1], k), comp(YM[2], k), hy_m ? a.wy : 0.f};
        nb[3] = {comp(YP[0], k), comp(YP[1], k), comp(YP[2], k), hy_p ? a.wy : 0.f};
        nb[4] = {comp(ZM[0], k), comp(ZM[1], k), comp(ZM[2], k), hz_m ? a.wz : 0.f};
        nb[5] = {comp(ZP[0], k), comp(ZP[1], k), comp(ZP[2], k), hz_p ? a.wz : 0.f};
        const unsigned pnat = pbase + 2u * k;
        const uint4 r = philox4x32_10(make_uint4(pnat, (uint32_t)sweep, a.chain, (uint32_t)colour), a.k0, a.k1);
        float ox, oy, oz;
        const bool ok = cell_move<EXACT, DMI, DMG, false>(a, C, r, omc, comp(A[0], k), comp(A[1], k), comp(A[2], k), nb,
                                                   DMG ? comp(H[0], k) : 0.f, DMG ? comp(H[1], k) : 0.f,
                                                   DMG ? comp(H[2], k) : 0.f, ox, oy, oz);
        if (k == 0) { OUT[0].x = ox; OUT[1].x = oy; OUT[2].x = oz; }
        if (k == 1) { OUT[0].y = ox; OUT[1].y = oy; OUT[2].y = oz; }
        if (k == 2) { OUT[0].z = ox; OUT[1].z = oy; OUT[2].z = oz; }
        if (k == 3) { OUT[0].w = ox; OUT[1].w = oy; OUT[2].w = oz; }
        if (dec) dec[pnat] = ok ? 1 : 0;
        nacc += ok ? 1ull : 0ull;
        sx += ox; sy += oy; sz += oz;
        sq += (double)ox * ox + (double)oy * oy + (double)oz * oz;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) *(float4*)(own + c * Nc + o0) = OUT[c];
}

template <bool DMG, bool EXACT, bool DMI>
__device__ __forceinline__ void pass4_body(const ChainDesc& cd, int colour, int stats, int shift,
                                           uint8_t* __restrict__ dec, int lb, int tid) {
    const SweepArgs a = cd.a;
    const ClassCoef* __restrict__ ctab = cd.ctab;
    float* __restrict__ m = cd.m;
    const float* __restrict__ h = cd.h;
    const DevState* __restrict__ st = cd.st;
    SweepAccum* __restrict__ acc = stats ? cd.acc : nullptr;
    const int tflat = lb * 256 + tid;
    const int hwc = a.hw >> 2;
    // rows are taken y-major, z-minor: the nz layers of one y run in adjacent
    // blocks, so z neighbours are read through the same XCD's L2
    const int lr = tflat / hwc;
    const int ic = tflat - lr * hwc;
    double sx = 0, sy = 0, sz = 0, sq = 0;
    unsigned long long nacc = 0;
    if (lr < a.ny * a.nz) {
        const int y = lr / a.nz, z = lr - y * a.nz;
        const long long o0 = (long long)(z * a.ny + y) * a.hw + ic * 4;
        pass4_cells<DMG, EXACT, DMI>(a, ctab[0], m, colour, y, z, ic, h + colour * 3 * a.Nc + o0, a.Nc, st->sweep,
                                     st->omc, dec, sx, sy, sz, sq, nacc);
    }
    if (acc) block_stats(sx, sy, sz, sq, nacc, acc, shift, lb, tid);
}

template <bool DMG, bool EXACT, bool DMI, bool B>
__global__ __launch_bounds__(256, B ? 3 : 4) void k_pass4(ChainDesc d0, const ChainDesc* __restrict__ dl, int colour, int stats,
                                               int shift, uint8_t* __restrict__ dec) {
    pass4_body<DMG, EXACT, DMI>(chain_at<B>(d0, dl, blockIdx.y), colour, stats, shift, dec,
                                xcd_block_s(blockIdx.x, gridDim.x), threadIdx.x);
}

// C = 1: any grid, optional per-cell material classes (grains), uniaxial or
// cubic anisotropy (CUB).
template <bool CLS, bool DMG, bool EXACT, bool DMI, bool CUB>
__device__ __forceinline__ void pass1_body(const ChainDesc& cd, int colour, int stats, int shift,
                                           uint8_t* __restrict__ dec, int lb, int tid) {
    const SweepArgs a = cd.a;
    const ClassCoef* __restrict__ ctab = cd.ctab;
    const uint32_t* __restrict__ cid = cd.cid;
    float* __restrict__ m = cd.m;
    const float* __restrict__ h = cd.h;
    const DevState* __restrict__ st = cd.st;
    SweepAccum* __restrict__ acc = stats ? cd.acc : nullptr;
    const int tflat = lb * 256 + tid;
    const int lr = tflat / a.hw;          // y-major, z-minor row order
    const int i = tflat - lr * a.hw;
    double sx = 0, sy = 0, sz = 0, sq = 0;
    unsigned long long nacc = 0;
    if (lr < a.ny * a.nz) {
        const int y = lr / a.nz, z = lr - y * a.nz;
        const int row = z * a.ny + y;
        const int par = (colour + y + z) & 1;
        const int x = 2 * i + par;
        if (x < a.nx) {
            const int Nc = (int)a.Nc;
            const int idx = row * a.hw + i;
            float* own = m + colour * 3 * Nc;
            const float* oth = m + (1 - colour) * 3 * Nc;
            const unsigned long long sweep = st->sweep;
            const float omc = st->omc;
            const uint32_t kp = CLS ? cid[colour * Nc + idx] : 0u;
            const ClassCoef C = ctab[kp];
            const int nbi[6] = {par ? idx : idx - 1, par ? idx + 1 : idx, idx - a.hw, idx + a.hw,
                                idx - a.ny * a.hw, idx + a.ny * a.hw};
            const bool has[6] = {x > 0, x + 1 < a.nx, y > 0, y + 1 < a.ny, z > 0, z + 1 < a.nz};
            const float wv[6] = {a.wx, a.wx, a.wy, a.wy, a.wz, a.wz};
            Nbr nb[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                if (has[k]) {
                    const int j = nbi[k];
                    float w = wv[k];
                    if (CLS) { if (cid[(1 - colour) * Nc + j] != kp) w *= a.bscale; }
                    nb[k] = {oth[j], oth[Nc + j], oth[2 * Nc + j], w};
                } else {
                    nb[k] = {0.f, 0.f, 0.f, 0.f};
                }
            }
            float hx = 0.f, hy = 0.f, hz = 0.f;
            if (DMG) {
                const float* hc = h + colour * 3 * Nc;
                hx = hc[idx]; hy = hc[Nc + idx]; hz = hc[2 * Nc + idx];
            }
            const unsigned pnat = (unsigned)((z * a.ny + y) * a.nx + x);
            const uint4 r = philox4x32_10(make_uint4(pnat, (uint32_t)sweep, a.chain, (uint32_t)colour), a.k0, a.k1);
            float ox, oy, oz;
            const bool ok = cell_move<EXACT, DMI, DMG, CLS, CUB>(a, C, r, omc, own[idx], own[Nc + idx], own[2 * Nc + idx], nb,
                                                       hx, hy, hz, ox, oy, oz);
            own[idx] = ox;
            own[Nc + idx] = oy;
            own[2 * Nc + idx] = oz;
            if (dec) dec[pnat] = ok ? 1 : 0;
            nacc = ok ? 1ull : 0ull;
            sx = ox; sy = oy; sz = oz;
            sq = (double)ox * ox + (double)oy * oy + (double)oz * oz;
        }
    }
    if (acc) block_stats(sx, sy, sz, sq, nacc, acc, shift, lb, tid);
}
template <bool CLS, bool DMG, bool EXACT, bool DMI, bool CUB, bool B>
__global__ __launch_bounds__(256) void k_pass1(ChainDesc d0, const ChainDesc* __restrict__ dl, int colour, int stats,
                                               int shift, uint8_t* __restrict__ dec) {
    pass1_body<CLS, DMG, EXACT, DMI, CUB>(chain_at<B>(d0, dl, blockIdx.y), colour, stats, shift, dec,
                                          xcd_block_s(blockIdx.x, gridDim.x), threadIdx.x);
}

}  // namespace mmc
