// Host-side FP64 setup of libmmc: mean field (paper Eqs. 8-9), longitudinal
// and move coefficients (Eqs. 7, 13), and the cell-averaged demag tensor with
// its Fourier spectrum (Sec. III, Eq. 14).  Not on the sweep path.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "mmc_internal.h"

namespace mmc {

// ---------------------------------------------------------------------
// Mean field at zero field: m = B(k m), k = 3Tc/T (Langevin), Tc/T (J = 1/2).
// chi_par = (mu/kT) B'(k me) / (1 - k B'(k me)) (Eq. 8); above Tc me = 0.
// ---------------------------------------------------------------------
static double langevin(double x) {
    if (std::fabs(x) < 0.05) {
        const double x2 = x * x;
        return x * (1.0 / 3.0 - x2 / 45.0 + x2 * x2 * 2.0 / 945.0 - x2 * x2 * x2 / 4725.0 + x2 * x2 * x2 * x2 * 2.0 / 93555.0);
    }
    return 1.0 / std::tanh(x) - 1.0 / x;
}
static double langevin_prime(double x) {
    if (std::fabs(x) < 0.05) {
        const double x2 = x * x;
        return 1.0 / 3.0 - x2 / 15.0 + x2 * x2 * 2.0 / 189.0 - x2 * x2 * x2 / 675.0 + x2 * x2 * x2 * x2 * 2.0 / 10395.0;
    }
    const double s = std::sinh(x);
    return 1.0 / (x * x) - 1.0 / (s * s);
}

void meanfield(int model, double T, double Tc, double mu, double* me, double* inv_chi) {
    const bool lang = (model == MMC_MF_LANGEVIN);
    if (T >= Tc) {
        *me = 0.0;
        *inv_chi = (lang ? 3.0 : 1.0) * kB * (T - Tc) / mu;
        return;
    }
    const double k = lang ? 3.0 * Tc / T : Tc / T;
    auto B = [&](double x) { return lang ? langevin(x) : std::tanh(x); };
    auto dB = [&](double x) {
        if (lang) return langevin_prime(x);
        const double c = std::cosh(x);
        return 1.0 / (c * c);
    };
    // g(m) = B(k m) - m: positive on (0, me), negative on (me, 1]
    double lo = 0.0, hi = 1.0;
    while (true) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (B(k * mid) - mid > 0.0) lo = mid; else hi = mid;
    }
    const double m = 0.5 * (lo + hi);
    *me = m;
    const double d = dB(k * m);
    *inv_chi = (kB * T / mu) * (1.0 - d * k) / d;
}

// <m^2> of m^2 exp(-(lb m^2 + lbc m^4)) by Gauss-Legendre panels.
static double mean_m2_above(double lb, double lbc) {
    double w = 1e300;
    if (lb > 0) w = 1.0 / std::sqrt(lb);
    if (lbc > 0) w = std::min(w, std::pow(lbc, -0.25));
    const double Lmax = 12.0 * w;
    static const double gx[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831, 0.9061798459386640};
    static const double gw[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889, 0.4786286704993665, 0.2369268850561891};
    const int panels = 400;
    double s2 = 0.0, s4 = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double a = Lmax * p / panels, b = Lmax * (p + 1) / panels, c = 0.5 * (a + b), hw = 0.5 * (b - a);
        for (int j = 0; j < 5; ++j) {
            const double m = c + hw * gx[j], q = m * m;
            const double e = std::exp(-(lb * q + lbc * q * q)) * gw[j] * hw;
            s2 += q * e;
            s4 += q * q * e;
        }
    }
    return s4 / s2;
}

ClassCoef class_coef(const mmc_material& mat, double T, double T0, double V, double K1, double K2, const double* ea,
                     const double* cax6, bool kscale, double Tc, double sigma_fixed) {
    ClassCoef c{};
    double me = 0.0, ic = 0.0;
    meanfield(mat.mf, T, Tc, mat.mu_atomic, &me, &ic);
    const double kT = kB * T;
    double sigma;
    if (T < Tc) {
        c.below = 1.0f;
        c.me2 = me * me;
        c.la = (float)(V * mat.Ms0 * ic / (8.0 * me * me * kT));
        sigma = std::min(0.03, 2.0 * me * std::sqrt(kT / (V * mat.Ms0 * ic)));
        c.m0 = (float)me;
    } else {
        c.below = 0.0f;
        c.me2 = 0.0;
        const double lb = V * mat.Ms0 * ic / (2.0 * kT);
        // T >= Tc quartic coefficient V Ms0 c Tc /(2 chi kT (T - Tc)) in its
        // non-singular form; c = 3/10 (Langevin, as printed) or 1/6 (J = 1/2)
        const double lbc = (mat.mf == MMC_MF_LANGEVIN) ? 9.0 * V * mat.Ms0 * Tc / (20.0 * mat.mu_atomic * T)
                                                        : V * mat.Ms0 * Tc / (12.0 * mat.mu_atomic * T);
        c.lb = (float)lb;
        c.lbc = (float)lbc;
        sigma = 0.03;
        c.m0 = (float)std::sqrt(mean_m2_above(lb, lbc));
    }
    if (sigma_fixed > 0) sigma = sigma_fixed;
    c.sigma = (float)sigma;
    c.ln1ps = (float)std::log1p(sigma);
    if (cax6) {
        // crystal axes: e = a1/|a1|, f = a2 made orthogonal to e, g = e x f
        double e[3], f[3], g[3];
        const double n1 = std::sqrt(cax6[0] * cax6[0] + cax6[1] * cax6[1] + cax6[2] * cax6[2]);
        for (int k = 0; k < 3; ++k) e[k] = cax6[k] / n1;
        const double pr = cax6[3] * e[0] + cax6[4] * e[1] + cax6[5] * e[2];
        for (int k = 0; k < 3; ++k) f[k] = cax6[3 + k] - pr * e[k];
        const double n2 = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        for (int k = 0; k < 3; ++k) f[k] /= n2;
        g[0] = e[1] * f[2] - e[2] * f[1];
        g[1] = e[2] * f[0] - e[0] * f[2];
        g[2] = e[0] * f[1] - e[1] * f[0];
        c.ex = (float)e[0]; c.ey = (float)e[1]; c.ez = (float)e[2];
        c.fx = (float)f[0]; c.fy = (float)f[1]; c.fz = (float)f[2];
        c.gx = (float)g[0]; c.gy = (float)g[1]; c.gz = (float)g[2];
    } else {
        const double en = std::sqrt(ea[0] * ea[0] + ea[1] * ea[1] + ea[2] * ea[2]);
        c.ex = (float)(ea[0] / en); c.ey = (float)(ea[1] / en); c.ez = (float)(ea[2] / en);
    }
    // temperature law of the anisotropy constants (Sec. III, Fe film): order l
    // scales as me^{l(l+1)/2}; uniaxial orders 2 and 4, cubic orders 4 and 6
    double s1 = 1.0, s2 = 1.0;
    if (kscale) {
        const int l1 = cax6 ? 4 : 2, l2 = cax6 ? 6 : 4;
        s1 = std::pow(me, 0.5 * l1 * (l1 + 1));
        s2 = std::pow(me, 0.5 * l2 * (l2 + 1));
    }
    c.ka1 = (float)(V * K1 * s1 / kT);
    c.ka2 = (float)(V * K2 * s2 / kT);
    c.tsc = (float)(T0 / T);
    return c;
}

// ---------------------------------------------------------------------
// Cell-averaged demag tensor of two nx*ny*nz-free rectangular cells at
// offset R.  Near: Newell-Williams-Dunlop closed form (JGR 98, 9551, 1993),
// second differences of f (diagonal) and g (off-diagonal) in each axis.
// Far: the point-dipole kernel averaged over the two cells, expanded in the
// cell sizes: per axis the average is sum_n 2 (h d)^{2n} / (2n+2)!.
// ---------------------------------------------------------------------
static double f_nw(double x, double y, double z) {
    x = std::fabs(x); y = std::fabs(y); z = std::fabs(z);
    const double xx = x * x, yy = y * y, zz = z * z, R = std::sqrt(xx + yy + zz);
    if (R == 0.0) return 0.0;
    double v = (2.0 * xx - yy - zz) * R / 6.0;
    if (y > 0.0 && xx + zz > 0.0) v += 0.5 * y * (zz - xx) * std::asinh(y / std::sqrt(xx + zz));
    if (z > 0.0 && xx + yy > 0.0) v += 0.5 * z * (yy - xx) * std::asinh(z / std::sqrt(xx + yy));
    if (x > 0.0 && y > 0.0 && z > 0.0) v -= x * y * z * std::atan(y * z / (x * R));
    return v;
}

static double g_nw(double x, double y, double z) {
    const double sgn = ((x < 0) != (y < 0)) ? -1.0 : 1.0;
    x = std::fabs(x); y = std::fabs(y); z = std::fabs(z);
    const double xx = x * x, yy = y * y, zz = z * z, R = std::sqrt(xx + yy + zz);
    if (R == 0.0) return 0.0;
    double v = -x * y * R / 3.0;
    if (z > 0.0 && xx + yy > 0.0) v += x * y * z * std::asinh(z / std::sqrt(xx + yy));
    if (x > 0.0 && yy + zz > 0.0) v += y * (3.0 * zz - yy) / 6.0 * std::asinh(x / std::sqrt(yy + zz));
    if (y > 0.0 && xx + zz > 0.0) v += x * (3.0 * zz - xx) / 6.0 * std::asinh(y / std::sqrt(xx + zz));
    if (z > 0.0) v -= zz * z / 6.0 * std::atan(x * y / (z * R));
    if (y > 0.0) v -= z * yy / 2.0 * std::atan(x * z / (y * R));
    if (x > 0.0) v -= z * xx / 2.0 * std::atan(y * z / (x * R));
    return sgn * v;
}

template <class F>
static double second_diff3(F fn, double X, double Y, double Z, double a, double b, double c) {
    const double wt[3] = {-1.0, 2.0, -1.0};
    double acc = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                acc += wt[i] * wt[j] * wt[k] * fn(X + (i - 1) * a, Y + (j - 1) * b, Z + (k - 1) * c);
    return acc / (4.0 * kPi * a * b * c);
}

// d^a_x d^b_y d^c_z (1/r): sum over sets of same-axis index pairs; a pair
// gives a Kronecker delta, an unpaired index a coordinate factor.
static double pairings(int n, int m) {  // n! / (2^m m! (n-2m)!)
    double v = 1.0;
    for (int i = 0; i < 2 * m; ++i) v *= (n - i);
    for (int i = 1; i <= m; ++i) v /= (2.0 * i);
    return v;
}
static double deriv_inv_r(int a, int b, int c, double x, double y, double z) {
    const int n = a + b + c;
    const double r2 = x * x + y * y + z * z, r = std::sqrt(r2);
    double acc = 0.0;
    for (int i = 0; 2 * i <= a; ++i)
        for (int j = 0; 2 * j <= b; ++j)
            for (int k = 0; 2 * k <= c; ++k) {
                const int mm = i + j + k, q = n - mm;   // power of 1/r is 2q+1
                double df = 1.0;
                for (int t = 2 * q - 1; t > 1; t -= 2) df *= t;
                const double term = ((q & 1) ? -df : df) * pairings(a, i) * pairings(b, j) * pairings(c, k) *
                                    std::pow(x, a - 2 * i) * std::pow(y, b - 2 * j) * std::pow(z, c - 2 * k) /
                                    std::pow(r, 2 * q + 1);
                acc += term;
            }
    return acc;
}

static void newell_far(double X, double Y, double Z, double hx, double hy, double hz, int order, double out[6]) {
    static const int ij[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    const double h[3] = {hx, hy, hz};
    // coefficient of (h d)^{2n}: 2/(2n+2)!
    const double an[4] = {1.0, 1.0 / 12.0, 1.0 / 360.0, 1.0 / 20160.0};
    for (int q = 0; q < 6; ++q) {
        double acc = 0.0;
        for (int p0 = 0; p0 <= order; p0 += 2)
            for (int p1 = 0; p0 + p1 <= order; p1 += 2)
                for (int p2 = 0; p0 + p1 + p2 <= order; p2 += 2) {
                    const double coef = an[p0 / 2] * std::pow(h[0], p0) * an[p1 / 2] * std::pow(h[1], p1) *
                                        an[p2 / 2] * std::pow(h[2], p2);
                    int e[3] = {p0, p1, p2};
                    e[ij[q][0]]++;
                    e[ij[q][1]]++;
                    acc += coef * deriv_inv_r(e[0], e[1], e[2], X, Y, Z);
                }
        out[q] = -(hx * hy * hz) / (4.0 * kPi) * acc;
    }
}

void newell_tensor(double X, double Y, double Z, double hx, double hy, double hz, double out[6]) {
    const double hm = std::max(hx, std::max(hy, hz));
    const double rho = std::sqrt(X * X + Y * Y + Z * Z) / hm;
    if (rho < 12.0) {
        out[0] = second_diff3(f_nw, X, Y, Z, hx, hy, hz);
        out[1] = second_diff3(f_nw, Y, X, Z, hy, hx, hz);
        out[2] = second_diff3(f_nw, Z, Y, X, hz, hy, hx);
        out[3] = second_diff3(g_nw, X, Y, Z, hx, hy, hz);
        out[4] = second_diff3(g_nw, X, Z, Y, hx, hz, hy);
        out[5] = second_diff3(g_nw, Y, Z, X, hy, hz, hx);
        return;
    }
    const int order = rho >= 320.0 ? 2 : (rho >= 32.0 ? 4 : 6);
    newell_far(X, Y, Z, hx, hy, hz, order, out);
}

// ---------------------------------------------------------------------
// Spectrum.  For each layer offset dz >= 0 and component q the wrapped tensor
// plane (Px x Py) is Fourier transformed in FP64; xx,yy,zz,xy spectra are
// real and xz,yz imaginary (tensor parities), so one real number per bin is
// kept, for kx in [0,Px/2] and ky in [0,Py/2] (the other half follows from
// the parity in Y).  Multiplied by -1/(Px Py) (the field's sign and the
// unnormalised inverse transforms).
// ---------------------------------------------------------------------
using cd = std::complex<double>;

static void fft_inplace(cd* a, int n, const std::vector<cd>& w) {   // w: exp(-2 pi i j / n), j < n/2
    if (n <= 1) return;
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        const int step = n / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < len / 2; ++k) {
                const cd u = a[i + k], v = a[i + k + len / 2] * w[k * step];
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}

template <class Fn>
static void parallel_for(int n, Fn fn) {
    int nt = (int)std::thread::hardware_concurrency();
    nt = std::max(1, std::min(nt, 32));
    nt = std::min(nt, std::max(1, n));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (int i = t; i < n; i += nt) fn(i);
        });
    for (auto& x : th) x.join();
}

static void tensor_spectrum_compute(int nx, int ny, int nz, double hx, double hy, double hz, int Px, int Py,
                                    std::vector<float>& K) {
    const int L = Px / 2, hp = Py / 2;
    K.assign((size_t)(L + 1) * (hp + 1) * 6 * nz, 0.0f);
    std::vector<cd> wx(std::max(1, Px / 2)), wy(std::max(1, Py / 2));
    for (int j = 0; j < Px / 2; ++j) wx[j] = std::polar(1.0, -2.0 * kPi * j / Px);
    for (int j = 0; j < Py / 2; ++j) wy[j] = std::polar(1.0, -2.0 * kPi * j / Py);
    std::vector<double> oct((size_t)6 * nx * ny);
    std::vector<cd> plane((size_t)Px * Py);
    const double scale = -1.0 / ((double)Px * Py);
    for (int dz = 0; dz < nz; ++dz) {
        // octant X >= 0, Y >= 0 at this layer offset
        parallel_for(ny, [&](int j) {
            double t[6];
            for (int i = 0; i < nx; ++i) {
                newell_tensor(i * hx, j * hy, dz * hz, hx, hy, hz, t);
                for (int q = 0; q < 6; ++q) oct[((size_t)q * ny + j) * nx + i] = t[q];
            }
        });
        for (int q = 0; q < 6; ++q) {
            // parity of component q in X and Y (Z >= 0 here)
            const int px = (q == 3 || q == 4) ? -1 : 1;
            const int py = (q == 3 || q == 5) ? -1 : 1;
            std::fill(plane.begin(), plane.end(), cd(0.0, 0.0));
            for (int j = -(ny - 1); j <= ny - 1; ++j)
                for (int i = -(nx - 1); i <= nx - 1; ++i) {
                    double v = oct[((size_t)q * ny + std::abs(j)) * nx + std::abs(i)];
                    if (i < 0 && px < 0) v = -v;
                    if (j < 0 && py < 0) v = -v;
                    plane[(size_t)((j + Py) % Py) * Px + (i + Px) % Px] = v;
                }
            parallel_for(Py, [&](int j) { fft_inplace(&plane[(size_t)j * Px], Px, wx); });
            parallel_for(L + 1, [&](int i) {
                std::vector<cd> col(Py);
                for (int j = 0; j < Py; ++j) col[j] = plane[(size_t)j * Px + i];
                fft_inplace(col.data(), Py, wy);
                const bool imag = (q == 4 || q == 5);
                for (int j = 0; j <= hp; ++j) {
                    const double v = imag ? col[j].imag() : col[j].real();
                    K[(((size_t)i * (hp + 1) + j) * 6 + q) * nz + dz] = (float)(v * scale);
                }
            });
        }
    }
}

// Chains of equal grid and cell size share one spectrum: computed once per
// process and kept (a batch of chains typically repeats a few sizes).
void tensor_spectrum(int nx, int ny, int nz, double hx, double hy, double hz, int Px, int Py, std::vector<float>& K) {
    using Key = std::tuple<int, int, int, double, double, double, int, int>;
    static std::mutex mu;
    static std::map<Key, std::vector<float>> cache;
    const Key key{nx, ny, nz, hx, hy, hz, Px, Py};
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) { K = it->second; return; }
    }
    tensor_spectrum_compute(nx, ny, nz, hx, hy, hz, Px, Py, K);
    std::lock_guard<std::mutex> g(mu);
    if (cache.size() >= 16) cache.erase(cache.begin());
    cache[key] = K;
}

}  // namespace mmc
