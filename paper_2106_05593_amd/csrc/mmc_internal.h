// Internal declarations shared by the libmmc sources (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>
#include "../../include/mmc.h"

namespace mmc {

// Physical constants (SI): kB exact (2019 SI), mu0 = 4 pi 1e-7.
constexpr double kB = 1.380649e-23;
constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;
constexpr double kPi = 3.14159265358979323846;

// Per-class (grain) coefficients in units of kT, as the sweep kernel reads them.
struct alignas(16) ClassCoef {
    double me2;      // me^2 (double: (m^2 - me^2) is formed in FP64)
    float la;        // T < Tc: F_l/kT = la (m^2 - me^2)^2
    float lb, lbc;   // T >= Tc: F_l/kT = lb m^2 + lbc m^4
    float below;     // 1: T < Tc branch
    float sigma;     // length-move width
    float ln1ps;     // ln(1 + sigma)
    float m0;        // initial length
    float ex, ey, ez;  // uniaxial: easy axis; cubic: first crystal axis (unit)
    float ka1, ka2;  // V K1/kT, V K2/kT (uniaxial Eq. 11 or cubic Eq. 12 constants, temperature law applied)
    float tsc;       // T0/T of the class: factor on the terms the chain keeps in units of kT0
                     // (exchange, DMI, Zeeman, demag); 1 at a uniform temperature
    float fx, fy, fz;  // cubic: second crystal axis
    float gx, gy, gz;  // cubic: third crystal axis (e x f)
};
static_assert(sizeof(ClassCoef) == 96, "ClassCoef layout");

// Uniform per-chain constants of a colour pass (kT units).
struct SweepArgs {
    int nx, ny, nz, hw;          // hw = ceil(nx/2): cells per row and colour
    long long Nc;                // nz*ny*hw: slots per colour
    float wx, wy, wz;            // exchange V A0 / (h^2 kT)
    float cdx, cdy;              // DMI V D0 / (h kT)
    float bx, by, bz;            // Zeeman V Ms0 (mu0 H) / kT
    float cdm;                   // demag mu0 V Ms0^2 / kT
    float bscale;                // exchange scale across grain boundaries
    uint32_t k0, k1, chain;      // Philox key and chain id
};

// Device-resident run state: read by the kernels, advanced on the device,
// so a captured sequence of sweeps can be replayed.
struct DevState {
    unsigned long long sweep;        // sweeps completed
    unsigned long long window;       // accepts since the last cone adaptation
    unsigned long long accepts_last; // accepts in the last sweep
    int cone_deg;
    int adapt_every;
    float omc;                       // 1 - cos(cone)
    int pad;
    double last[4];                  // <mx>, <my>, <mz>, <|m|^2> after the last sweep
    double avg_sum[4];               // sums of those means over the sweeps since the last read-and-reset
    unsigned long long avg_n;        // sweeps in avg_sum
    unsigned long long pad2;
};

// Per-sweep statistics accumulators.  Blocks add fixed-point sums (scale
// 2^shift) of m_x, m_y, m_z, |m|^2 and the accepted-move count into one of
// kAccBins bins (one 64-byte line each, so concurrent atomics spread out).
constexpr int kAccBins = 256;
struct SweepAccum {
    long long bin[kAccBins][8];        // 4 sums, accepts, 3 spare
};

// Host-side physics setup (setup.cpp).
void meanfield(int model, double T, double Tc, double mu, double* me, double* inv_chi);
// T: the class's temperature; T0: the chain's reference temperature (kT0 units of SweepArgs).
// cax6 == NULL: uniaxial anisotropy about ea with constants K1, K2; else cubic, K1 and K2 the cubic
// constants and cax6 the first and second crystal axes (any length, not parallel).  kscale: each
// constant of order l times me^{l(l+1)/2}, me of the class at T.
ClassCoef class_coef(const mmc_material& mat, double T, double T0, double V, double K1, double K2, const double* ea,
                     const double* cax6, bool kscale, double Tc, double sigma_fixed);
// Demag tensor spectrum K[kx][ky'][q][dz] (kx in [0, Px/2], ky' in [0, Py/2],
// q = xx,yy,zz,xy,xz,yz, dz in [0,nz)), including the -1/(Px Py) factor.
void tensor_spectrum(int nx, int ny, int nz, double hx, double hy, double hz, int Px, int Py,
                     std::vector<float>& K);
void newell_tensor(double X, double Y, double Z, double hx, double hy, double hz, double out[6]);

// Kernel launchers (kernels.hip).
struct DemagPlan {
    int Px, Py, L, S;
    int logL, logPy;
    float2* X;        // [(L+1)][S][ny] complex work buffer
    float* K;         // tensor spectrum
    int rpt_f = 2, rpt_i = 2;   // x-pass rows per thread (1, 2 or 4), forward and inverse: the tuned tile shape
    int prec;         // y-pass DFT stages: 0 FP32 (vector units), 1 split BF16, 2 split FP16 (matrix cores)
    float kmax;       // largest magnitude in K (bounds for the FP16 scales)
    long long woff = 0;   // staged y pass: offset (complex elements) of its work buffer after X; 0: one-kernel y pass
};
// Everything a sweep-path kernel needs from one chain.  A single chain's is
// passed by value; for a batch the descriptors of chains of one shape (grid,
// material classes on/off, demag, move kind) sit in a device array and
// chain blockIdx.y (blockIdx.x for the end-of-sweep kernel) is served, so
// the chains advance in shared launches.
struct ChainDesc {
    SweepArgs a;
    const ClassCoef* ctab;
    const uint32_t* cid;   // per-cell class ids (colour-split) or NULL
    float* m;              // [2][3][Nc]
    float* h;              // [2][3][Nc]
    DevState* st;
    SweepAccum* acc;
    float2* X;             // demag work buffer or NULL
};
typedef const ChainDesc* DescList;

// The chains a launch serves: one chain passed by value (many == NULL), or
// n chains whose descriptors sit in a device array.
struct Chains {
    ChainDesc one;
    DescList many;
    int n;
};
template <bool B>
__device__ __forceinline__ const ChainDesc& chain_at(const ChainDesc& one, const ChainDesc* __restrict__ many,
                                                     unsigned i) {
    if constexpr (B) return many[i];
    else return one;
}

int ypass_E(int nz, int Py);                    // elements per thread of the y pass
int x_rpt_default(int L);                       // x-pass rows per thread without tuning
size_t x_pass_lds(int L, int rpt);              // LDS bytes of an x-pass block with rpt rows per thread
bool ypass_split_ok(int nz, int Py);            // split-precision y-pass stages available for this shape
bool ystage_needed(int nz, int Py);             // the shape needs the staged y pass (nz > 8 or the register budget)
int ystage_max_nz();                            // most layers the staged y pass mixes
long long ystage_work_elems(int L, int S, int Py);   // complex elements of its work buffer
hipError_t launch_init(const SweepArgs& a, const ClassCoef* ctab, const uint32_t* cid, float* m, int kind,
                       float dx, float dy, float dz, hipStream_t s);
hipError_t launch_to_split(const SweepArgs& a, const float* nat, float* split, hipStream_t s);
hipError_t launch_from_split(const SweepArgs& a, const float* split, float* nat, hipStream_t s);
// Sweep-path launches over the chains c, all of one shape (a: host copy of
// the shared geometry).
hipError_t launch_ystage(const Chains& c, const DemagPlan& p, int nz, const float2* tw, hipStream_t s);
hipError_t launch_demag_stage(int stage, const SweepArgs& a, const DemagPlan& p, const Chains& c, int colour_mask,
                              const float2* tw, hipStream_t s);
// Fills the x transforms' per-pass twiddle tables at tw + 8192 (tw holds
// 8192 + 4096 entries, the first 8192 the base table).
hipError_t launch_x_twiddles(const DemagPlan& p, float2* tw, hipStream_t s);
hipError_t launch_demag(const SweepArgs& a, const DemagPlan& p, const Chains& c, int colour_mask, const float2* tw,
                        hipStream_t s);
hipError_t launch_pass(const SweepArgs& a, bool classes, bool demag, bool exact, bool dmi, bool cubic, const Chains& c,
                       int colour, bool stats, int shift, uint8_t* dec, hipStream_t s);
hipError_t launch_end_sweep(const Chains& c, int shift, long long N, double* series, unsigned long long rec_base,
                            hipStream_t s);
// Fused colour pass (fused.hip): x-inverse of the field the pass reads, the
// four-cells-per-thread pass and (spec) the x-forward of the updated rows in
// one kernel; for uniform materials with nx % 8 == 0 and the field refreshed
// before each colour.  Without spec (the half form) the next x-forward runs
// as its own kernel.
bool fused_ok(const SweepArgs& a, int L, bool classes, bool spec);
hipError_t launch_fused(const SweepArgs& a, const DemagPlan& p, bool exact, bool dmi, const Chains& c, int colour,
                        int shift, const float2* tw, hipStream_t s, bool spec);
hipError_t launch_energy(const SweepArgs& a, bool classes, bool cubic, const ClassCoef* ctab, const uint32_t* cid,
                         const float* m, const float* h, double* part, hipStream_t s, int* nblk_out);
hipError_t launch_set_cone(DevState* st, int cone_deg, hipStream_t s);
// Persistent batched sweeps (persist.hip): one kernel advances every chain of
// a batch; chains of uniform material without DMI, demag off or FP32 with nz
// 1 or 2, x half-length 32..1024 and padded y 64..1024 (persist_shape_ok).
struct PersistChain {
    ChainDesc cd;
    const float* K;        // tensor spectrum (demag)
    const float2* tw;      // twiddle tables (demag)
    int L, Py;             // x half-length and padded y of the demag plan
    bool demag;
    int refresh_per_sweep;
    int shift;             // fixed-point scale of the statistics
};
struct PersistPlan {
    int nch = 0, W = 0, grid = 0;
    size_t lds = 0;
    bool exact = false;    // length move of every chain (one kernel per kind)
    void* mem = nullptr;   // device block holding the tables and counters
    void* pc = nullptr;
    int *off = nullptr, *pre = nullptr, *wc = nullptr;
    unsigned long long* ctr = nullptr;
    int* err = nullptr;
    std::vector<int> host_off, host_pre, host_wc;
};
bool persist_shape_ok(int nx, int ny, int nz, bool demag);
hipError_t persist_build(const PersistChain* in, int n, PersistPlan* out);   // out->exact set by the caller
// n sweeps of every chain: a counter reset and the persistent kernel on s;
// a wait longer than limit_s seconds sets the plan's error flag.
hipError_t persist_launch(const PersistPlan& p, int nsweeps, double limit_s, hipStream_t s);
void persist_free(PersistPlan* p);

// Energy partials: k_energy never runs more than kEnergyMaxBlocks blocks
// (it strides over the grid).
constexpr int kEnergyMaxBlocks = 2048;
// Allocation-free energy (kernels.hip): energy_scratch_init(device), called
// with that device current, looks up the device address of the static
// partial-sum array once per device; energy_scratch(device) returns it (NULL
// before the set-up).  launch_energy_sum writes the six terms times kT and
// their total (7 doubles) to out.
hipError_t energy_scratch_init(int device);
double* energy_scratch(int device);
hipError_t launch_energy_sum(const double* part, int nb, double kT, double* out, hipStream_t s);

}  // namespace mmc
