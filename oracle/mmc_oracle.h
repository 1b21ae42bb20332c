/*
 * mmc_oracle.h -- plain FP64 CPU oracle of the micromagnetic Monte Carlo (MMC)
 * method of Lepadatu, "Micromagnetic Monte Carlo method with variable
 * magnetization length based on the Landau-Lifshitz-Bloch equation"
 * (arXiv 2106.05593).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this library: it exists so that the tests, the smoke check and the
 * benchmark's CPU-baseline leg can check the GPU library against an
 * independent, slow, obviously correct implementation.  It shares no source,
 * header, table or constant generator with the GPU library.
 *
 * Everything here is double precision.  Arrays of magnetization are "natural
 * SoA": m[c*N + p] with c in {x,y,z}, p = x + nx*(y + ny*z), N = nx*ny*nz,
 * m = M/Ms0 (dimensionless, non-unit).  Demag fields h are in units of Ms0
 * (H_d = Ms0*h, A/m).  Energies are Joules unless a name ends in _kT.
 */
#ifndef MMC_ORACLE_H
#define MMC_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Physical constants (SI).  kB is exact in the 2019 SI; muB is CODATA 2018;
 * mu0 is taken as 4*pi*1e-7 exactly. */
#define OR_KB   1.380649e-23
#define OR_MUB  9.2740100783e-24
#define OR_MU0  (4.0e-7 * 3.14159265358979323846)

/* Counter-based generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* u = (x >> 8) * 2^-24, exact in binary32 and binary64, in [0, 1). */
double or_u01(uint32_t x);

/* Mean-field equilibrium length and relative longitudinal susceptibility
 * (paper Sec. II, Eqs. 8-9, taken at zero field).  model 0: Langevin (the
 * paper's classical form); model 1: Brillouin J=1/2 (m = tanh(m Tc/T)).
 * Returns me and inv_chi = 1/chi_par in tesla (chi_par in 1/T). */
void or_meanfield(int model, double T, double Tc, double mu, double* me, double* inv_chi);

/* Per-class coefficients (one class per grain; one class for a uniform
 * material).  All *_kT numbers are free energies divided by kB*T. */
typedef struct {
    double me, inv_chi;
    int    below;        /* 1: T < Tc branch of Eq. 7; 0: T >= Tc branch */
    double la;           /* below: F_l/kT = la*(m^2-me^2)^2 */
    double lb, lbc;      /* above: F_l/kT = lb*m^2 + lbc*m^4 */
    double sigma;        /* length-move width (Eq. 13 capped, or fixed) */
    double m0;           /* initial length: me below Tc, sqrt(<m^2>) above */
} or_class;

typedef struct {
    int32_t nx, ny, nz;
    double hx, hy, hz;          /* m */
    double Ms0, A0, D0;         /* A/m, J/m, J/m^2 */
    double T;                   /* K */
    double B[3];                /* mu0*H in tesla */
    int32_t mf;                 /* mean-field model, see or_meanfield */
    double mu;                  /* atomic moment, J/T */
    int32_t lenmode;            /* 0: paper (uniform factor, exponent 4); 1: exact (log-uniform factor, exponent 3) */
    int32_t demag;              /* 0 off, 1 on */
    int32_t refresh_per_sweep;  /* 1: one demag refresh per sweep, 2: before each colour */
    uint64_t seed;
    uint32_t chain_id;
    double sigma_fixed;         /* > 0 overrides Eq. 13 */
    int32_t nclass;             /* >= 1 */
    const uint32_t* cls;        /* N class ids, or NULL (all class 0) */
    const double* ea;           /* 3*nclass easy axes (unit) */
    const double* K1;           /* nclass, J/m^3 */
    const double* K2;           /* nclass, J/m^3 */
    const double* Tc;           /* nclass, K */
    double bscale;              /* exchange scale across class boundaries */
    const double* Tcl;          /* nclass temperatures (K) of a non-uniform temperature profile, or NULL:
                                 * every class at T.  A move at a cell of class c is judged at T_c: every
                                 * term of its dF is divided by kB*T_c (local detailed balance), and the
                                 * class's me, chi, sigma and Eq. 7 coefficients are taken at T_c. */
    int32_t anis;               /* 0: uniaxial anisotropy (Eq. 11) about ea with constants K1, K2;
                                 * 1: cubic anisotropy (Eq. 12) in place of it: K1, K2 are then the 4th and
                                 * 6th order cubic constants and cax holds the crystal axes */
    const double* cax;          /* anis 1: 9*nclass, three orthonormal cubic axes per class */
    int32_t kscale;             /* 1: each anisotropy constant of order l is multiplied by me^{l(l+1)/2}
                                 * (Sec. III, Fe film), me of the class at its temperature; 0: as given */
} or_sys;

/* Fill cls_out[nclass]. */
void or_class_coeffs(const or_sys* s, or_class* cls_out);

/* Cell-averaged demag tensor of two rectangular cells at offset (X,Y,Z) in
 * metres (Newell, Williams, Dunlop, JGR 98 (1993) 9551).  out = {xx,yy,zz,xy,xz,yz}.
 * Closed form near, multipole expansion of the cell average far. */
void or_newell(double X, double Y, double Z, double hx, double hy, double hz, double out[6]);
/* The two ingredients separately (for tests). */
void or_newell_exact(double X, double Y, double Z, double hx, double hy, double hz, double out[6]);
void or_newell_far(double X, double Y, double Z, double hx, double hy, double hz, int order, double out[6]);
/* d^a/dx^a d^b/dy^b d^c/dz^c of 1/r at (x,y,z). */
double or_dinvr(int a, int b, int c, double x, double y, double z);

/* Demag field h = -N * m (paper Sec. III, Eq. 14). */
void or_demag_direct(int nx, int ny, int nz, double hx, double hy, double hz, const double* m, double* h);
void or_demag_direct_at(int nx, int ny, int nz, double hx, double hy, double hz, const double* m,
                        const int64_t* cells, int ncells, double* h_out /* 3*ncells */);
typedef struct or_demag_plan or_demag_plan;
or_demag_plan* or_demag_plan_create(int nx, int ny, int nz, double hx, double hy, double hz);
void or_demag_plan_apply(or_demag_plan* pl, const double* m, double* h);
void or_demag_plan_destroy(or_demag_plan* pl);

/* Free-energy change in units of kT of replacing m_p by mB, split by term
 * {exchange, DMI, anisotropy, Zeeman, longitudinal, demag}.  h may be NULL. */
void or_delta_F(const or_sys* s, const or_class* cc, const double* m, const double* h,
                int64_t p, const double mB[3], double out_kT[6]);

/* Total free energy (J) split the same way; h (fresh field of m) may be NULL
 * (demag term then 0). */
void or_energy(const or_sys* s, const or_class* cc, const double* m, const double* h, double E[6]);

/* One colour sub-sweep (paper Sec. II, steps 1-4, red-black decomposition).
 * Updates m in place.  acc[p] (optional) = 1 accepted / 0 rejected / -1 not
 * of this colour.  margin[p] (optional) = (k ln f - dF/kT) - ln u3: the move
 * is accepted iff margin > 0.  mB_out (optional, 3N) gets the proposal.
 * Returns the number of accepted moves. */
int64_t or_subsweep(const or_sys* s, const or_class* cc, double* m, const double* h,
                    uint64_t sweep, int colour, double cone_deg,
                    int8_t* acc, double* margin, double* mB_out);

/* Serial MMC with the exact demag interaction (paper Sec. III, the comparison
 * of the parallel algorithm with a serial one; App. B): the cells are visited
 * one at a time (colour 0 cells in index order, then colour 1 cells), each
 * with the same compound move and Philox numbers as in the parallel sweep;
 * the demag field h = -N*m of every cell is kept current, updated after
 * every accepted move.  The demag part of dF is Eq. 14's -V mu0 dM.H_d with
 * that current field (self_term 0: the paper's serial version), or the exact
 * change of the total demag energy, which adds the cell's self term
 * (mu0 V Ms0^2 / 2) dm.N(0).dm (self_term 1).  With demag off a serial sweep
 * equals the two parallel colour passes.
 * or_serial_create tabulates the Newell tensor for every cell offset;
 * or_serial_field fills h from m by the direct sum over that table.
 * or_serial_sweep: one sweep, h in/out (current field of m on entry);
 * dE_accepted (optional) accumulates the accepted dF in Joules.  Returns the
 * number of accepted moves. */
typedef struct or_serial or_serial;
or_serial* or_serial_create(const or_sys* s);
void or_serial_destroy(or_serial* q);
void or_serial_field(const or_serial* q, const double* m, double* h);
int64_t or_serial_sweep(const or_serial* q, const or_sys* s, const or_class* cc, double* m, double* h,
                        uint64_t sweep, double cone_deg, int self_term, double* dE_accepted);

/* Initial state: kind 0 uniform along dir, kind 1 random directions
 * (Philox tag 1).  Length = class m0. */
void or_init_state(const or_sys* s, const or_class* cc, int kind, const double dir[3], double* m);

/* Full run of n sweeps from sweep index sweep0.  Cone angle is an integer
 * number of degrees, adapted every adapt_every sweeps (0: never) by the
 * +-1 degree rule targeting an acceptance rate of 0.5 +- 0.05.
 * series (optional) receives per sweep {<mx>,<my>,<mz>,<|m|^2>,accepts}.
 * plan may be NULL when demag is off. */
void or_run(const or_sys* s, const or_class* cc, or_demag_plan* plan, double* m,
            uint64_t sweep0, int64_t n, int32_t* cone_deg, int32_t adapt_every,
            int64_t* window_accepts, double* series);

#ifdef __cplusplus
}
#endif
#endif
