/*
 * mmc_oracle.c -- plain FP64 CPU oracle of the micromagnetic Monte Carlo
 * method (arXiv 2106.05593).  TEST INFRASTRUCTURE ONLY: see mmc_oracle.h.
 *
 * Written for readability against the paper, not for speed: no blocking, no
 * fusion, no reordering beyond what the method states.  OpenMP only spreads
 * independent cells of one colour (and independent FFT lines) over threads;
 * every random number is counter based, so results do not depend on the
 * thread count.
 *
 * Parity status of each function (how it is pinned by the CPU tests):
 *   or_philox4x32_10   published known-answer vectors + rocRAND host engine
 *   or_meanfield       closed-form limits, fixed-point residual
 *   or_newell*         cube self term 1/3, trace 1, Aharoni prism factors,
 *                      point-dipole far field, mpmath high-precision values
 *   or_demag_*         FFT path == brute-force direct sum
 *   or_delta_F         equals E_total(after) - E_total(before) per term
 *   or_subsweep/or_run macrospin quadrature of the paper's Eq. 1 target
 *   or_serial_*        demag off: identical to the parallel sweep; kept field ==
 *                      direct sum; energy change == sum of accepted dF
 *   or_energy          isotropy + closed forms on uniform states (uniaxial and
 *                      the cubic <100>, <110>, <111> values), cubic symmetry
 */
#include "mmc_oracle.h"
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011): 10 rounds of the 4x32 S-box with a  */
/* Weyl key schedule.                                                     */
/* ------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double or_u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* ------------------------------------------------------------------ */
/* Mean field (paper Eqs. 8-9, at zero applied field)                      */
/* ------------------------------------------------------------------ */
static double langevin(double x) {
    double ax = fabs(x);
    if (ax < 0.05) {   /* series: sum 2^{2n} B_{2n} x^{2n-1} / (2n)! */
        double x2 = x * x;
        return x * (1.0 / 3.0 + x2 * (-1.0 / 45.0 + x2 * (2.0 / 945.0 + x2 * (-1.0 / 4725.0 + x2 * (2.0 / 93555.0)))));
    }
    return 1.0 / tanh(x) - 1.0 / x;
}
static double langevin_d(double x) {
    double ax = fabs(x);
    if (ax < 0.05) {
        double x2 = x * x;
        return 1.0 / 3.0 + x2 * (-3.0 / 45.0 + x2 * (10.0 / 945.0 + x2 * (-7.0 / 4725.0 + x2 * (18.0 / 93555.0))));
    }
    double s = sinh(x);
    return 1.0 / (x * x) - 1.0 / (s * s);
}

/* Mean-field magnetization m = B(k * m) with k = 3Tc/T (Langevin) or Tc/T (J=1/2). */
static double mf_B(int model, double x) { return model == 0 ? langevin(x) : tanh(x); }
static double mf_dB(int model, double x) {
    if (model == 0) return langevin_d(x);
    double c = cosh(x);
    return 1.0 / (c * c);
}
static double mf_k(int model, double T, double Tc) { return model == 0 ? 3.0 * Tc / T : Tc / T; }

void or_meanfield(int model, double T, double Tc, double mu, double* me, double* inv_chi) {
    double kT = OR_KB * T;
    if (T >= Tc) {
        /* me = 0; chi = (mu/kT) B'(0) / (1 - B'(0) k) */
        *me = 0.0;
        *inv_chi = (model == 0 ? 3.0 : 1.0) * OR_KB * (T - Tc) / mu;
        return;
    }
    double k = mf_k(model, T, Tc);
    /* bisection on g(m) = B(k m) - m, g(0+) > 0 > g(1) */
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double g = mf_B(model, k * mid) - mid;
        if (g > 0) lo = mid; else hi = mid;
    }
    double m = 0.5 * (lo + hi);
    *me = m;
    double d = mf_dB(model, k * m);
    double chi = (mu / kT) * d / (1.0 - d * k);   /* Eq. 8 */
    *inv_chi = 1.0 / chi;
}

/* <m^2> under f_l(m) ~ m^2 exp(-(lb m^2 + lbc m^4)) (Eq. 7, T >= Tc),
 * composite Simpson on [0, L] with L many widths out. */
static double above_tc_m2(double lb, double lbc) {
    double w = 1e300;
    if (lb > 0) w = 1.0 / sqrt(lb);
    if (lbc > 0) { double w4 = pow(lbc, -0.25); if (w4 < w) w = w4; }
    double L = 12.0 * w;
    int n = 20000;
    double hstep = L / n, s2 = 0.0, s4 = 0.0;
    for (int i = 0; i <= n; ++i) {
        double m = i * hstep, q = m * m;
        double wt = (i == 0 || i == n) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
        double e = exp(-(lb * q + lbc * q * q));
        s2 += wt * q * e;
        s4 += wt * q * q * e;
    }
    return s4 / s2;
}

/* Temperature of class c (non-uniform temperature profiles, paper Sec. IV). */
static double T_of(const or_sys* s, int c) { return s->Tcl ? s->Tcl[c] : s->T; }

void or_class_coeffs(const or_sys* s, or_class* out) {
    double V = s->hx * s->hy * s->hz;
    for (int c = 0; c < s->nclass; ++c) {
        or_class* o = &out[c];
        double Tc = s->Tc[c], T = T_of(s, c), kT = OR_KB * T;
        or_meanfield(s->mf, T, Tc, s->mu, &o->me, &o->inv_chi);
        if (T < Tc) {
            o->below = 1;
            /* Eq. 7, T < Tc: V Ms0 (m^2 - me^2)^2 / (8 chi me^2 kT) */
            o->la = V * s->Ms0 * o->inv_chi / (8.0 * o->me * o->me * kT);
            o->lb = o->lbc = 0.0;
            /* Eq. 13: sigma = 2 me sqrt(chi kT / (V Ms0)), capped at 0.03 */
            o->sigma = 2.0 * o->me * sqrt(kT / (V * s->Ms0 * o->inv_chi));
            if (o->sigma > 0.03) o->sigma = 0.03;
            o->m0 = o->me;
        } else {
            o->below = 0;
            o->la = 0.0;
            /* Eq. 7, T >= Tc: V Ms0 m^2 (1 + c Tc m^2/(T-Tc)) / (2 chi kT);
             * c = 3/10 for the Langevin model (as printed), 1/6 for J=1/2.
             * The quartic coefficient is written in its non-singular form. */
            o->lb = V * s->Ms0 * o->inv_chi / (2.0 * kT);
            if (s->mf == 0) o->lbc = 9.0 * V * s->Ms0 * Tc / (20.0 * s->mu * T);
            else            o->lbc = V * s->Ms0 * Tc / (12.0 * s->mu * T);
            o->sigma = 0.03;
            o->m0 = sqrt(above_tc_m2(o->lb, o->lbc));
        }
        if (s->sigma_fixed > 0) o->sigma = s->sigma_fixed;
    }
}

/* ------------------------------------------------------------------ */
/* Newell demag tensor                                                     */
/* ------------------------------------------------------------------ */
static double newell_f(double x, double y, double z) {
    x = fabs(x); y = fabs(y); z = fabs(z);
    double x2 = x * x, y2 = y * y, z2 = z * z;
    double R = sqrt(x2 + y2 + z2);
    if (R == 0.0) return 0.0;
    double t = 0.0;
    if (y > 0 && x2 + z2 > 0) t += 0.5 * y * (z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (z > 0 && x2 + y2 > 0) t += 0.5 * z * (y2 - x2) * asinh(z / sqrt(x2 + y2));
    if (x > 0 && y > 0 && z > 0) t -= x * y * z * atan(y * z / (x * R));
    t += (2.0 * x2 - y2 - z2) * R / 6.0;
    return t;
}

static double newell_g(double x, double y, double z) {
    double sg = 1.0;
    if (x < 0) { sg = -sg; x = -x; }
    if (y < 0) { sg = -sg; y = -y; }
    z = fabs(z);
    double x2 = x * x, y2 = y * y, z2 = z * z;
    double R = sqrt(x2 + y2 + z2);
    if (R == 0.0) return 0.0;
    double t = 0.0;
    if (z > 0 && x2 + y2 > 0) t += x * y * z * asinh(z / sqrt(x2 + y2));
    if (x > 0 && y2 + z2 > 0) t += y / 6.0 * (3.0 * z2 - y2) * asinh(x / sqrt(y2 + z2));
    if (y > 0 && x2 + z2 > 0) t += x / 6.0 * (3.0 * z2 - x2) * asinh(y / sqrt(x2 + z2));
    if (z > 0) t -= z2 * z / 6.0 * atan(x * y / (z * R));
    if (y > 0) t -= z * y2 / 2.0 * atan(x * z / (y * R));
    if (x > 0) t -= z * x2 / 2.0 * atan(y * z / (x * R));
    t -= x * y * R / 3.0;
    return sg * t;
}

/* Sum over the 27-point stencil of products of second differences
 * (weights 2 at the centre, -1 at +-h in each direction). */
static double newell_stencil(double (*fn)(double, double, double),
                             double X, double Y, double Z, double a, double b, double c) {
    static const double w[3] = {-1.0, 2.0, -1.0};
    double s = 0.0;
    for (int i = -1; i <= 1; ++i)
        for (int j = -1; j <= 1; ++j)
            for (int k = -1; k <= 1; ++k)
                s += w[i + 1] * w[j + 1] * w[k + 1] * fn(X + i * a, Y + j * b, Z + k * c);
    return s / (4.0 * M_PI * a * b * c);
}

void or_newell_exact(double X, double Y, double Z, double hx, double hy, double hz, double out[6]) {
    out[0] = newell_stencil(newell_f, X, Y, Z, hx, hy, hz);   /* xx */
    out[1] = newell_stencil(newell_f, Y, X, Z, hy, hx, hz);   /* yy */
    out[2] = newell_stencil(newell_f, Z, Y, X, hz, hy, hx);   /* zz */
    out[3] = newell_stencil(newell_g, X, Y, Z, hx, hy, hz);   /* xy */
    out[4] = newell_stencil(newell_g, X, Z, Y, hx, hz, hy);   /* xz */
    out[5] = newell_stencil(newell_g, Y, Z, X, hy, hz, hx);   /* yz */
}

static double dfact2(int n) { double r = 1.0; for (int k = n; k > 1; k -= 2) r *= k; return r; }
static double fact(int n) { double r = 1.0; for (int k = 2; k <= n; ++k) r *= k; return r; }
static double ipow(double x, int n) { double r = 1.0; for (int k = 0; k < n; ++k) r *= x; return r; }

/* Derivatives of 1/r: sum over pairings of the derivative indices; a pair of
 * equal axes contributes a Kronecker delta, unpaired indices a coordinate. */
double or_dinvr(int a, int b, int c, double x, double y, double z) {
    int n = a + b + c;
    double r2 = x * x + y * y + z * z, r = sqrt(r2);
    double s = 0.0;
    for (int mx = 0; 2 * mx <= a; ++mx)
        for (int my = 0; 2 * my <= b; ++my)
            for (int mz = 0; 2 * mz <= c; ++mz) {
                int m = mx + my + mz;
                double pa = fact(a) / (ipow(2.0, mx) * fact(mx) * fact(a - 2 * mx));
                double pb = fact(b) / (ipow(2.0, my) * fact(my) * fact(b - 2 * my));
                double pc = fact(c) / (ipow(2.0, mz) * fact(mz) * fact(c - 2 * mz));
                double sign = ((n - m) & 1) ? -1.0 : 1.0;
                double term = sign * dfact2(2 * n - 2 * m - 1) / ipow(r, 2 * n - 2 * m + 1);
                term *= pa * pb * pc * ipow(x, a - 2 * mx) * ipow(y, b - 2 * my) * ipow(z, c - 2 * mz);
                s += term;
            }
    return s;
}

/* Far field: N_ij(R) = -(V/4pi) <d_i d_j (1/r)> averaged over the offset
 * u - v of two points uniform in the two cells.  Per axis the average is the
 * operator (sinh(h d/2)/(h d/2))^2 = sum_n 2 (h d)^{2n} / (2n+2)!, expanded to
 * total order `order` in the cell sizes. */
void or_newell_far(double X, double Y, double Z, double hx, double hy, double hz, int order, double out[6]) {
    static const int comp[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    double h[3] = {hx, hy, hz};
    double V = hx * hy * hz;
    for (int q = 0; q < 6; ++q) {
        double s = 0.0;
        for (int px = 0; px <= order; px += 2)
            for (int py = 0; px + py <= order; py += 2)
                for (int pz = 0; px + py + pz <= order; pz += 2) {
                    int p[3] = {px, py, pz};
                    double coef = 1.0;
                    for (int k = 0; k < 3; ++k) coef *= 2.0 * ipow(h[k], p[k]) / fact(p[k] + 2);
                    int e[3] = {px, py, pz};
                    e[comp[q][0]] += 1;
                    e[comp[q][1]] += 1;
                    s += coef * or_dinvr(e[0], e[1], e[2], X, Y, Z);
                }
        out[q] = -V / (4.0 * M_PI) * s;
    }
}

/* Closed form for |R| < 12 h_max; beyond, the far-field series to an order
 * whose first omitted term is below ~1e-10 relative. */
void or_newell(double X, double Y, double Z, double hx, double hy, double hz, double out[6]) {
    double hm = hx > hy ? hx : hy;
    if (hz > hm) hm = hz;
    double rho = sqrt(X * X + Y * Y + Z * Z) / hm;
    if (rho < 12.0) { or_newell_exact(X, Y, Z, hx, hy, hz, out); return; }
    int order = 6;
    if (rho >= 32.0) order = 4;
    if (rho >= 320.0) order = 2;
    or_newell_far(X, Y, Z, hx, hy, hz, order, out);
}

/* ------------------------------------------------------------------ */
/* Demag field h = -N * m                                                  */
/* ------------------------------------------------------------------ */
static void apply_tensor(const double N[6], const double mj[3], double h[3]) {
    h[0] -= N[0] * mj[0] + N[3] * mj[1] + N[4] * mj[2];
    h[1] -= N[3] * mj[0] + N[1] * mj[1] + N[5] * mj[2];
    h[2] -= N[4] * mj[0] + N[5] * mj[1] + N[2] * mj[2];
}

void or_demag_direct(int nx, int ny, int nz, double hx, double hy, double hz, const double* m, double* h) {
    int64_t N = (int64_t)nx * ny * nz;
    int ox = 2 * nx - 1, oy = 2 * ny - 1, oz = 2 * nz - 1;
    double* tab = (double*)malloc(sizeof(double) * 6 * (size_t)ox * oy * oz);
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int k = 0; k < oz; ++k)
        for (int j = 0; j < oy; ++j)
            for (int i = 0; i < ox; ++i) {
                size_t o = ((size_t)k * oy + j) * ox + i;
                or_newell((i - (nx - 1)) * hx, (j - (ny - 1)) * hy, (k - (nz - 1)) * hz, hx, hy, hz, &tab[6 * o]);
            }
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((int64_t)nx * ny));
        double hp[3] = {0, 0, 0};
        for (int64_t q = 0; q < N; ++q) {
            int qx = (int)(q % nx), qy = (int)((q / nx) % ny), qz = (int)(q / ((int64_t)nx * ny));
            size_t o = ((size_t)(z - qz + nz - 1) * oy + (y - qy + ny - 1)) * ox + (x - qx + nx - 1);
            double mj[3] = {m[q], m[N + q], m[2 * N + q]};
            apply_tensor(&tab[6 * o], mj, hp);
        }
        h[p] = hp[0]; h[N + p] = hp[1]; h[2 * N + p] = hp[2];
    }
    free(tab);
}

void or_demag_direct_at(int nx, int ny, int nz, double hx, double hy, double hz, const double* m,
                        const int64_t* cells, int ncells, double* h_out) {
    int64_t N = (int64_t)nx * ny * nz;
    for (int s = 0; s < ncells; ++s) {
        int64_t p = cells[s];
        int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((int64_t)nx * ny));
        double hx_ = 0, hy_ = 0, hz_ = 0;
#pragma omp parallel for reduction(+ : hx_, hy_, hz_) schedule(static)
        for (int64_t q = 0; q < N; ++q) {
            int qx = (int)(q % nx), qy = (int)((q / nx) % ny), qz = (int)(q / ((int64_t)nx * ny));
            double Nt[6], hp[3] = {0, 0, 0};
            or_newell((x - qx) * hx, (y - qy) * hy, (z - qz) * hz, hx, hy, hz, Nt);
            double mj[3] = {m[q], m[N + q], m[2 * N + q]};
            apply_tensor(Nt, mj, hp);
            hx_ += hp[0]; hy_ += hp[1]; hz_ += hp[2];
        }
        h_out[3 * s] = hx_; h_out[3 * s + 1] = hy_; h_out[3 * s + 2] = hz_;
    }
}

/* Radix-2 complex FFT along one axis of a 3-D array (in place). */
static void fft_line(double complex* a, int n, int64_t stride, int inverse) {
    if (n <= 1) return;
    for (int i = 1, j = 0; i < n; ++i) {           /* bit reversal */
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { double complex t = a[i * stride]; a[i * stride] = a[j * stride]; a[j * stride] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < len / 2; ++k) {
                double ang = (inverse ? 2.0 : -2.0) * M_PI * k / len;
                double complex w = cos(ang) + I * sin(ang);
                double complex u = a[(i + k) * stride], v = a[(i + k + len / 2) * stride] * w;
                a[(i + k) * stride] = u + v;
                a[(i + k + len / 2) * stride] = u - v;
            }
    }
}

static void fft3(double complex* a, int Px, int Py, int Pz, int inverse) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < Pz; ++k)
        for (int j = 0; j < Py; ++j) fft_line(a + ((int64_t)k * Py + j) * Px, Px, 1, inverse);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < Pz; ++k)
        for (int i = 0; i < Px; ++i) fft_line(a + (int64_t)k * Py * Px + i, Py, Px, inverse);
#pragma omp parallel for collapse(2) schedule(static)
    for (int j = 0; j < Py; ++j)
        for (int i = 0; i < Px; ++i) fft_line(a + (int64_t)j * Px + i, Pz, (int64_t)Px * Py, inverse);
}

static int pad_pow2(int n) { int p = 1; while (p < 2 * n - 1) p <<= 1; return p; }

struct or_demag_plan {
    int nx, ny, nz, Px, Py, Pz;
    double complex* K[6];   /* tensor spectra */
    double complex* W[3];   /* work arrays */
};

or_demag_plan* or_demag_plan_create(int nx, int ny, int nz, double hx, double hy, double hz) {
    or_demag_plan* pl = (or_demag_plan*)calloc(1, sizeof(or_demag_plan));
    pl->nx = nx; pl->ny = ny; pl->nz = nz;
    pl->Px = pad_pow2(nx); pl->Py = pad_pow2(ny); pl->Pz = pad_pow2(nz);
    int64_t P = (int64_t)pl->Px * pl->Py * pl->Pz;
    for (int q = 0; q < 6; ++q) pl->K[q] = (double complex*)calloc(P, sizeof(double complex));
    for (int c = 0; c < 3; ++c) pl->W[c] = (double complex*)calloc(P, sizeof(double complex));
    /* tensor of offset (X,Y,Z) sits at index (X mod Px, Y mod Py, Z mod Pz) */
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int k = -(nz - 1); k <= nz - 1; ++k)
        for (int j = -(ny - 1); j <= ny - 1; ++j)
            for (int i = -(nx - 1); i <= nx - 1; ++i) {
                double Nt[6];
                or_newell(i * hx, j * hy, k * hz, hx, hy, hz, Nt);
                int ii = (i + pl->Px) % pl->Px, jj = (j + pl->Py) % pl->Py, kk = (k + pl->Pz) % pl->Pz;
                int64_t o = ((int64_t)kk * pl->Py + jj) * pl->Px + ii;
                for (int q = 0; q < 6; ++q) pl->K[q][o] = Nt[q];
            }
    for (int q = 0; q < 6; ++q) fft3(pl->K[q], pl->Px, pl->Py, pl->Pz, 0);
    return pl;
}

void or_demag_plan_apply(or_demag_plan* pl, const double* m, double* h) {
    int nx = pl->nx, ny = pl->ny, nz = pl->nz, Px = pl->Px, Py = pl->Py, Pz = pl->Pz;
    int64_t N = (int64_t)nx * ny * nz, P = (int64_t)Px * Py * Pz;
    for (int c = 0; c < 3; ++c) {
        memset(pl->W[c], 0, sizeof(double complex) * P);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    pl->W[c][((int64_t)z * Py + y) * Px + x] = m[c * N + ((int64_t)z * ny + y) * nx + x];
        fft3(pl->W[c], Px, Py, Pz, 0);
    }
    /* H~_i = - sum_j N~_ij M~_j */
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < P; ++o) {
        double complex mx = pl->W[0][o], my = pl->W[1][o], mz = pl->W[2][o];
        double complex hx_ = -(pl->K[0][o] * mx + pl->K[3][o] * my + pl->K[4][o] * mz);
        double complex hy_ = -(pl->K[3][o] * mx + pl->K[1][o] * my + pl->K[5][o] * mz);
        double complex hz_ = -(pl->K[4][o] * mx + pl->K[5][o] * my + pl->K[2][o] * mz);
        pl->W[0][o] = hx_; pl->W[1][o] = hy_; pl->W[2][o] = hz_;
    }
    for (int c = 0; c < 3; ++c) {
        fft3(pl->W[c], Px, Py, Pz, 1);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    h[c * N + ((int64_t)z * ny + y) * nx + x] = creal(pl->W[c][((int64_t)z * Py + y) * Px + x]) / (double)P;
    }
}

void or_demag_plan_destroy(or_demag_plan* pl) {
    if (!pl) return;
    for (int q = 0; q < 6; ++q) free(pl->K[q]);
    for (int c = 0; c < 3; ++c) free(pl->W[c]);
    free(pl);
}

/* ------------------------------------------------------------------ */
/* Free energy                                                             */
/* ------------------------------------------------------------------ */
static inline int cls_of(const or_sys* s, int64_t p) { return s->cls ? (int)s->cls[p] : 0; }

static double fl_kT(const or_class* c, double q) {   /* Eq. 7 exponent, q = m^2 */
    if (c->below) { double d = q - c->me * c->me; return c->la * d * d; }
    return c->lb * q + c->lbc * q * q;
}

/* Anisotropy constants of class c in J/m^3 as the free energy uses them.  With
 * kscale the temperature law of Sec. III applies: a term of order l scales as
 * me^{l(l+1)/2}.  Uniaxial (Eq. 11): K1 is of order 2, K2 of order 4; cubic
 * (Eq. 12): K1 of order 4, K2 of order 6. */
static void an_consts(const or_sys* s, const or_class* c, int cp, double* k1, double* k2) {
    *k1 = s->K1[cp];
    *k2 = s->K2[cp];
    if (s->kscale) {
        int l1 = s->anis ? 4 : 2, l2 = s->anis ? 6 : 4;
        *k1 *= pow(c->me, 0.5 * l1 * (l1 + 1));
        *k2 *= pow(c->me, 0.5 * l2 * (l2 + 1));
    }
}

/* Anisotropy energy density of one cell over its constants (J/m^3):
 * uniaxial (Eq. 11) k1 (1 - (m.e)^2) + k2 (1 - (m.e)^2)^2 with m non-unit;
 * cubic (Eq. 12) k1 (a^2 b^2 + a^2 g^2 + b^2 g^2) + k2 a^2 b^2 g^2 with a, b, g
 * the direction cosines of m (components of m/|m| along the crystal axes). */
static double an_density(const or_sys* s, int cp, double k1, double k2, const double mi[3]) {
    if (!s->anis) {
        const double* e = &s->ea[3 * cp];
        double dd = mi[0] * e[0] + mi[1] * e[1] + mi[2] * e[2];
        double u = 1.0 - dd * dd;
        return k1 * u + k2 * u * u;
    }
    double L = sqrt(mi[0] * mi[0] + mi[1] * mi[1] + mi[2] * mi[2]);
    if (L == 0.0) return 0.0;
    double dc[3];
    for (int a = 0; a < 3; ++a) {
        const double* ax = &s->cax[9 * cp + 3 * a];
        dc[a] = (mi[0] * ax[0] + mi[1] * ax[1] + mi[2] * ax[2]) / L;
    }
    double a2 = dc[0] * dc[0], b2 = dc[1] * dc[1], g2 = dc[2] * dc[2];
    return k1 * (a2 * b2 + a2 * g2 + b2 * g2) + k2 * a2 * b2 * g2;
}

void or_delta_F(const or_sys* s, const or_class* cc, const double* m, const double* h,
                int64_t p, const double mB[3], double out[6]) {
    int nx = s->nx, ny = s->ny, nz = s->nz;
    int64_t N = (int64_t)nx * ny * nz;
    int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((int64_t)nx * ny));
    int cp = cls_of(s, p);
    double V = s->hx * s->hy * s->hz, kT = OR_KB * T_of(s, cp);
    const or_class* c = &cc[cp];
    double mA[3] = {m[p], m[N + p], m[2 * N + p]};
    double D[3], S[3];
    for (int k = 0; k < 3; ++k) { D[k] = mB[k] - mA[k]; S[k] = mB[k] + mA[k]; }

    /* exchange: exact change of E_ex = sum_bonds s V A0 |m_i - m_j|^2 / h^2 */
    double ex = 0.0;
    int64_t nb[6]; double hb[6]; int nn = 0;
    if (x > 0)      { nb[nn] = p - 1;  hb[nn++] = s->hx; }
    if (x < nx - 1) { nb[nn] = p + 1;  hb[nn++] = s->hx; }
    if (y > 0)      { nb[nn] = p - nx; hb[nn++] = s->hy; }
    if (y < ny - 1) { nb[nn] = p + nx; hb[nn++] = s->hy; }
    if (z > 0)      { nb[nn] = p - (int64_t)nx * ny; hb[nn++] = s->hz; }
    if (z < nz - 1) { nb[nn] = p + (int64_t)nx * ny; hb[nn++] = s->hz; }
    for (int k = 0; k < nn; ++k) {
        int64_t q = nb[k];
        double w = V * s->A0 / (hb[k] * hb[k] * kT);
        if (cls_of(s, q) != cp) w *= s->bscale;
        double mj[3] = {m[q], m[N + q], m[2 * N + q]};
        ex += w * (D[0] * (S[0] - 2 * mj[0]) + D[1] * (S[1] - 2 * mj[1]) + D[2] * (S[2] - 2 * mj[2]));
    }
    out[0] = ex;

    /* interfacial DMI (Eq. 15): -(2 V D0/kT) D.G, G = z div m - grad m_z
     * by central differences, missing neighbours taken as zero */
    double dxmx = 0, dxmz = 0, dymy = 0, dymz = 0;
    if (x < nx - 1) { dxmx += m[p + 1];  dxmz += m[2 * N + p + 1]; }
    if (x > 0)      { dxmx -= m[p - 1];  dxmz -= m[2 * N + p - 1]; }
    if (y < ny - 1) { dymy += m[N + p + nx]; dymz += m[2 * N + p + nx]; }
    if (y > 0)      { dymy -= m[N + p - nx]; dymz -= m[2 * N + p - nx]; }
    dxmx /= 2 * s->hx; dxmz /= 2 * s->hx; dymy /= 2 * s->hy; dymz /= 2 * s->hy;
    double G[3] = {-dxmz, -dymz, dxmx + dymy};
    out[1] = -(2.0 * V * s->D0 / kT) * (D[0] * G[0] + D[1] * G[1] + D[2] * G[2]);

    /* anisotropy (Eq. 11 or 12), V on both terms */
    double k1, k2;
    an_consts(s, c, cp, &k1, &k2);
    out[2] = (V / kT) * (an_density(s, cp, k1, k2, mB) - an_density(s, cp, k1, k2, mA));

    /* Zeeman: -V Ms0 (mB - mA).B */
    out[3] = -(V * s->Ms0 / kT) * (D[0] * s->B[0] + D[1] * s->B[1] + D[2] * s->B[2]);

    /* longitudinal (Eq. 7 exponent) */
    double qA = mA[0] * mA[0] + mA[1] * mA[1] + mA[2] * mA[2];
    double qB = mB[0] * mB[0] + mB[1] * mB[1] + mB[2] * mB[2];
    out[4] = fl_kT(c, qB) - fl_kT(c, qA);

    /* demag with frozen field (Eq. 14): -V mu0 dM.H_d = -(mu0 V Ms0^2) D.h */
    double dm = 0.0;
    if (h) dm = -(OR_MU0 * V * s->Ms0 * s->Ms0 / kT) * (D[0] * h[p] + D[1] * h[N + p] + D[2] * h[2 * N + p]);
    out[5] = dm;
}

void or_energy(const or_sys* s, const or_class* cc, const double* m, const double* h, double E[6]) {
    int nx = s->nx, ny = s->ny, nz = s->nz;
    int64_t N = (int64_t)nx * ny * nz;
    double V = s->hx * s->hy * s->hz;
    for (int k = 0; k < 6; ++k) E[k] = 0.0;
    for (int64_t p = 0; p < N; ++p) {
        int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((int64_t)nx * ny));
        int cp = cls_of(s, p);
        double mi[3] = {m[p], m[N + p], m[2 * N + p]};
        /* bonds to +x, +y, +z */
        int64_t nbs[3] = {x < nx - 1 ? p + 1 : -1, y < ny - 1 ? p + nx : -1, z < nz - 1 ? p + (int64_t)nx * ny : -1};
        double hs[3] = {s->hx, s->hy, s->hz};
        for (int d = 0; d < 3; ++d) {
            int64_t q = nbs[d];
            if (q < 0) continue;
            double mj[3] = {m[q], m[N + q], m[2 * N + q]};
            double sc = (cls_of(s, q) != cp) ? s->bscale : 1.0;
            double d0 = mi[0] - mj[0], d1 = mi[1] - mj[1], d2 = mi[2] - mj[2];
            E[0] += sc * V * s->A0 * (d0 * d0 + d1 * d1 + d2 * d2) / (hs[d] * hs[d]);
            if (d == 0) E[1] += -V * s->D0 * (mi[2] * mj[0] - mi[0] * mj[2]) / s->hx;
            if (d == 1) E[1] += -V * s->D0 * (mi[2] * mj[1] - mi[1] * mj[2]) / s->hy;
        }
        double k1, k2;
        an_consts(s, &cc[cp], cp, &k1, &k2);
        E[2] += V * an_density(s, cp, k1, k2, mi);
        E[3] += -V * s->Ms0 * (mi[0] * s->B[0] + mi[1] * s->B[1] + mi[2] * s->B[2]);
        E[4] += OR_KB * T_of(s, cp) * fl_kT(&cc[cp], mi[0] * mi[0] + mi[1] * mi[1] + mi[2] * mi[2]);
        if (h) E[5] += -0.5 * OR_MU0 * V * s->Ms0 * s->Ms0 * (mi[0] * h[p] + mi[1] * h[N + p] + mi[2] * h[2 * N + p]);
    }
}

/* ------------------------------------------------------------------ */
/* The Metropolis sub-sweep                                                */
/* ------------------------------------------------------------------ */
static void philox_cell(const or_sys* s, int64_t p, uint64_t sweep, int tag, int colour, double u[4]) {
    uint32_t ctr[4] = {(uint32_t)p, (uint32_t)sweep, s->chain_id, (uint32_t)((tag << 1) | colour)};
    uint32_t key[2] = {(uint32_t)s->seed, (uint32_t)(s->seed >> 32)};
    uint32_t o[4];
    or_philox4x32_10(ctr, key, o);
    for (int k = 0; k < 4; ++k) u[k] = or_u01(o[k]);
}

/* Steps 1-2 of a move at cell p with uniforms u: rotation uniform on the cap
 * of 1 - cos(theta_c) = omc about the current direction, then the length
 * change.  Writes the proposal mB and ln(f) of the length factor f. */
static void propose(const or_sys* s, const or_class* c, const double* m, int64_t N, int64_t p, const double u[4],
                    double omc, double mB[3], double* lnf_out) {
    double mA[3] = {m[p], m[N + p], m[2 * N + p]};
    double len = sqrt(mA[0] * mA[0] + mA[1] * mA[1] + mA[2] * mA[2]);
    double n[3] = {mA[0] / len, mA[1] / len, mA[2] / len};
    /* 1) rotation: uniform on the cap of half-angle theta_c about n */
    double t = u[0] * omc;               /* 1 - cos(theta) */
    double ct = 1.0 - t, st = sqrt(t * (2.0 - t));
    double phi = 2.0 * M_PI * u[1];
    /* orthonormal frame of n: Duff et al., JCGT 6(1), 2017 */
    double sg = copysign(1.0, n[2]);
    double a = -1.0 / (sg + n[2]);
    double b = n[0] * n[1] * a;
    double e1[3] = {1.0 + sg * n[0] * n[0] * a, sg * b, -sg * n[0]};
    double e2[3] = {b, sg + n[1] * n[1] * a, -n[1]};
    double cp_ = cos(phi), sp_ = sin(phi);
    double nb[3];
    for (int k = 0; k < 3; ++k) nb[k] = ct * n[k] + st * (cp_ * e1[k] + sp_ * e2[k]);
    /* 2) length change */
    double lnf, f;
    if (s->lenmode == 0) { f = 1.0 - c->sigma + 2.0 * c->sigma * u[2]; lnf = log(f); }
    else { lnf = (2.0 * u[2] - 1.0) * log1p(c->sigma); f = exp(lnf); }
    for (int k = 0; k < 3; ++k) mB[k] = f * len * nb[k];
    *lnf_out = lnf;
}

int64_t or_subsweep(const or_sys* s, const or_class* cc, double* m, const double* h,
                    uint64_t sweep, int colour, double cone_deg,
                    int8_t* acc, double* margin, double* mB_out) {
    int nx = s->nx, ny = s->ny, nz = s->nz;
    int64_t N = (int64_t)nx * ny * nz;
    double omc = 2.0 * pow(sin(0.5 * cone_deg * M_PI / 180.0), 2);   /* 1 - cos(theta_c) */
    int64_t nacc = 0;
#pragma omp parallel for reduction(+ : nacc) schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((int64_t)nx * ny));
        if (((x + y + z) & 1) != colour) {
            if (acc) acc[p] = -1;
            if (margin) margin[p] = 0.0;
            continue;
        }
        const or_class* c = &cc[cls_of(s, p)];
        double u[4], mB[3], lnf;
        philox_cell(s, p, sweep, 0, colour, u);
        propose(s, c, m, N, p, u, omc, mB, &lnf);
        if (mB_out) { mB_out[p] = mB[0]; mB_out[N + p] = mB[1]; mB_out[2 * N + p] = mB[2]; }
        /* 3) free-energy change */
        double dF[6];
        or_delta_F(s, cc, m, h, p, mB, dF);
        double dFt = dF[0] + dF[1] + dF[2] + dF[3] + dF[4] + dF[5];
        /* 4) accept with min{1, (mB/mA)^k exp(-dF/kT)} (Eq. 5: k = 4) */
        double k = (s->lenmode == 0) ? 4.0 : 3.0;
        double mg = (k * lnf - dFt) - log(u[3]);
        int ok = mg > 0.0;
        if (margin) margin[p] = mg;
        if (acc) acc[p] = (int8_t)ok;
        if (ok) { m[p] = mB[0]; m[N + p] = mB[1]; m[2 * N + p] = mB[2]; nacc += 1; }
    }
    return nacc;
}

/* ------------------------------------------------------------------ */
/* Serial MMC with the exact demag interaction                             */
/* ------------------------------------------------------------------ */
struct or_serial {
    int nx, ny, nz;
    double* T;     /* 6 tensor components for every offset (dx, dy, dz) in [-(n-1), n-1]^3 */
};

static const double* ser_tensor(const or_serial* q, int dx, int dy, int dz) {
    int64_t ix = dx + q->nx - 1, iy = dy + q->ny - 1, iz = dz + q->nz - 1;
    return &q->T[6 * ((iz * (2 * q->ny - 1) + iy) * (2 * q->nx - 1) + ix)];
}

or_serial* or_serial_create(const or_sys* s) {
    or_serial* q = (or_serial*)calloc(1, sizeof(or_serial));
    q->nx = s->nx; q->ny = s->ny; q->nz = s->nz;
    int64_t n = (int64_t)(2 * s->nx - 1) * (2 * s->ny - 1) * (2 * s->nz - 1);
    q->T = (double*)malloc(sizeof(double) * 6 * n);
#pragma omp parallel for schedule(dynamic)
    for (int64_t o = 0; o < n; ++o) {
        int dx = (int)(o % (2 * s->nx - 1)) - (s->nx - 1);
        int dy = (int)((o / (2 * s->nx - 1)) % (2 * s->ny - 1)) - (s->ny - 1);
        int dz = (int)(o / ((int64_t)(2 * s->nx - 1) * (2 * s->ny - 1))) - (s->nz - 1);
        or_newell(dx * s->hx, dy * s->hy, dz * s->hz, s->hx, s->hy, s->hz, &q->T[6 * o]);
    }
    return q;
}

void or_serial_destroy(or_serial* q) {
    if (!q) return;
    free(q->T);
    free(q);
}

/* h_j += -N(j - p) dm for every cell j: the field change of a change dm at p. */
static void ser_field_update(const or_serial* q, int64_t N, int64_t p, const double dm[3], double* h) {
    int nx = q->nx, ny = q->ny;
    int px = (int)(p % nx), py = (int)((p / nx) % ny), pz = (int)(p / ((int64_t)nx * ny));
    for (int64_t j = 0; j < N; ++j) {
        int x = (int)(j % nx), y = (int)((j / nx) % ny), z = (int)(j / ((int64_t)nx * ny));
        const double* t = ser_tensor(q, x - px, y - py, z - pz);   /* xx yy zz xy xz yz */
        h[j] -= t[0] * dm[0] + t[3] * dm[1] + t[4] * dm[2];
        h[N + j] -= t[3] * dm[0] + t[1] * dm[1] + t[5] * dm[2];
        h[2 * N + j] -= t[4] * dm[0] + t[5] * dm[1] + t[2] * dm[2];
    }
}

void or_serial_field(const or_serial* q, const double* m, double* h) {
    int64_t N = (int64_t)q->nx * q->ny * q->nz;
    for (int64_t k = 0; k < 3 * N; ++k) h[k] = 0.0;
    for (int64_t p = 0; p < N; ++p) {
        double mp[3] = {m[p], m[N + p], m[2 * N + p]};
        ser_field_update(q, N, p, mp, h);
    }
}

int64_t or_serial_sweep(const or_serial* q, const or_sys* s, const or_class* cc, double* m, double* h,
                        uint64_t sweep, double cone_deg, int self_term, double* dE_accepted) {
    int nx = s->nx, ny = s->ny, nz = s->nz;
    int64_t N = (int64_t)nx * ny * nz;
    double omc = 2.0 * pow(sin(0.5 * cone_deg * M_PI / 180.0), 2);
    double V = s->hx * s->hy * s->hz;
    const double* N0 = s->demag ? ser_tensor(q, 0, 0, 0) : NULL;
    int64_t nacc = 0;
    for (int colour = 0; colour < 2; ++colour) {
        for (int64_t p = 0; p < N; ++p) {
            int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((int64_t)nx * ny));
            if (((x + y + z) & 1) != colour) continue;
            int cp = cls_of(s, p);
            double u[4], mB[3], lnf, dF[6];
            philox_cell(s, p, sweep, 0, colour, u);
            propose(s, &cc[cp], m, N, p, u, omc, mB, &lnf);
            or_delta_F(s, cc, m, s->demag ? h : NULL, p, mB, dF);
            double D[3] = {mB[0] - m[p], mB[1] - m[N + p], mB[2] - m[2 * N + p]};
            if (s->demag && self_term) {
                /* exact change of the total demag energy: the current-field term of
                 * Eq. 14 plus the cell's self term (mu0 V Ms0^2 / 2) D.N(0).D */
                double ND[3] = {N0[0] * D[0] + N0[3] * D[1] + N0[4] * D[2],
                                N0[3] * D[0] + N0[1] * D[1] + N0[5] * D[2],
                                N0[4] * D[0] + N0[5] * D[1] + N0[2] * D[2]};
                double kT = OR_KB * T_of(s, cp);
                dF[5] += 0.5 * OR_MU0 * V * s->Ms0 * s->Ms0 / kT * (D[0] * ND[0] + D[1] * ND[1] + D[2] * ND[2]);
            }
            double dFt = dF[0] + dF[1] + dF[2] + dF[3] + dF[4] + dF[5];
            double k = (s->lenmode == 0) ? 4.0 : 3.0;
            if ((k * lnf - dFt) - log(u[3]) > 0.0) {
                m[p] = mB[0]; m[N + p] = mB[1]; m[2 * N + p] = mB[2];
                if (s->demag) ser_field_update(q, N, p, D, h);
                if (dE_accepted) *dE_accepted += dFt * OR_KB * T_of(s, cp);
                nacc += 1;
            }
        }
    }
    return nacc;
}

void or_init_state(const or_sys* s, const or_class* cc, int kind, const double dir[3], double* m) {
    int64_t N = (int64_t)s->nx * s->ny * s->nz;
    double dl = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    for (int64_t p = 0; p < N; ++p) {
        double L = cc[cls_of(s, p)].m0, d[3];
        if (kind == 0) { d[0] = dir[0] / dl; d[1] = dir[1] / dl; d[2] = dir[2] / dl; }
        else {
            double u[4];
            philox_cell(s, p, 0, 1, 0, u);
            double ct = 2.0 * u[0] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct)), ph = 2.0 * M_PI * u[1];
            d[0] = st * cos(ph); d[1] = st * sin(ph); d[2] = ct;
        }
        m[p] = L * d[0]; m[N + p] = L * d[1]; m[2 * N + p] = L * d[2];
    }
}

void or_run(const or_sys* s, const or_class* cc, or_demag_plan* plan, double* m,
            uint64_t sweep0, int64_t n, int32_t* cone_deg, int32_t adapt_every,
            int64_t* window_accepts, double* series) {
    int64_t N = (int64_t)s->nx * s->ny * s->nz;
    double* h = NULL;
    if (s->demag) h = (double*)malloc(sizeof(double) * 3 * N);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t sw = sweep0 + (uint64_t)i;
        int64_t nacc = 0;
        for (int colour = 0; colour < 2; ++colour) {
            if (s->demag && (colour == 0 || s->refresh_per_sweep >= 2)) or_demag_plan_apply(plan, m, h);
            nacc += or_subsweep(s, cc, m, s->demag ? h : NULL, sw, colour, (double)*cone_deg, NULL, NULL, NULL);
        }
        *window_accepts += nacc;
        if (series) {
            double sx = 0, sy = 0, sz = 0, s2 = 0;
            for (int64_t p = 0; p < N; ++p) {
                double a = m[p], b = m[N + p], c = m[2 * N + p];
                sx += a; sy += b; sz += c; s2 += a * a + b * b + c * c;
            }
            series[5 * i + 0] = sx / N; series[5 * i + 1] = sy / N; series[5 * i + 2] = sz / N;
            series[5 * i + 3] = s2 / N; series[5 * i + 4] = (double)nacc;
        }
        /* cone adaptation every adapt_every sweeps: acceptance rate above
         * 0.55 -> +1 degree, below 0.45 -> -1 degree, kept in [1, 180] */
        if (adapt_every > 0 && (sw + 1) % (uint64_t)adapt_every == 0) {
            int64_t tot = (int64_t)adapt_every * N;
            if (100 * *window_accepts > 55 * tot && *cone_deg < 180) *cone_deg += 1;
            else if (100 * *window_accepts < 45 * tot && *cone_deg > 1) *cone_deg -= 1;
            *window_accepts = 0;
        }
    }
    free(h);
}
