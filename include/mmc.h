/*
 * mmc.h -- C-ABI of libmmc, an MI355X (gfx950) implementation of the
 * micromagnetic Monte Carlo (MMC) method with variable magnetization length
 * (S. Lepadatu, arXiv 2106.05593).
 *
 * What the library computes (paper references are to that article):
 *   - Equilibrium states of a discretised ferromagnet sampled by a Markov
 *     chain whose stationary law is the Maxwell-Boltzmann-type density
 *     m^2 exp(-F(m)/kT) of Sec. II, Eq. 1.
 *   - One sweep ("MMC iteration", Sec. II, steps 1-4) gives every cell one
 *     compound trial move: a rotation uniform in a cone about the current
 *     direction, then a multiplicative length change, accepted with
 *     min{1, (mB/mA)^k exp(-dF/kT)} (Eq. 5, k = 4; see mmc_lenmove).
 *     Cells are updated in two colour passes of a red-black checkerboard
 *     (colour = (x+y+z) mod 2, colour 0 first), which makes every pass fully
 *     parallel.
 *   - dF sums exchange (Eq. 10, as the exact change of the bond energy
 *     sum_bonds V A0 |m_i - m_j|^2 / h^2), interfacial DMI (Eq. 15), uniaxial
 *     or cubic anisotropy (Eqs. 11-12), Zeeman, the longitudinal LLB term (exponent of
 *     Eq. 7, parameterised by me(T), Eq. 9 and chi_par(T), Eq. 8) and the
 *     demag term with a frozen field (Sec. III, Eq. 14): H_d = -N*M by
 *     zero-padded FFT convolution with the cell-averaged (Newell) tensor,
 *     refreshed before each colour pass (or once per sweep) and constant
 *     within a pass.
 *   - The cone half-angle is adapted every adapt_every sweeps by +-1 degree to
 *     keep the acceptance rate within 0.5 +- 0.05 (Sec. II).  The length
 *     move width sigma follows Eq. 13, capped at 0.03, and 0.03 at T >= Tc.
 *
 * Conventions
 *   - Units are SI.  Fields are given as mu0*H in tesla.  m = M/Ms0 is
 *     dimensionless and not unit length.  Demag fields h returned by the
 *     library are H_d/Ms0 (dimensionless).
 *   - Grids are nx*ny*nz cells, open boundaries.  "Natural SoA" arrays hold
 *     3*N floats: component c of cell (x,y,z) at c*N + x + nx*(y + ny*z).
 *   - Randomness is Philox4x32-10 (Salmon et al., SC'11) with key = seed and
 *     counter = (cell index, sweep mod 2^32, chain_id, 2*tag + colour);
 *     tag 0: trial moves, tag 1: random initial directions.  Each uniform is
 *     (x >> 8) * 2^-24.
 *   - The library owns every context and its device memory; the caller owns
 *     every pointer it passes in and keeps it valid for the call only.
 *   - on_device = 1 means the pointer is device memory on the context's GPU
 *     (e.g. a PyTorch tensor's data_ptr()); 0 means host memory.
 *   - Calls that enqueue work (mmc_sweep, mmc_batch_sweep) are asynchronous
 *     on the context's stream; getters synchronise that stream.
 *   - A context is not thread-safe; distinct contexts are.
 *   - Every call returns an mmc_status; no exception or abort crosses the ABI.
 *     On failure mmc_last_error() gives a thread-local message.  A device
 *     error (kernel fault, out of memory on the device) is returned as
 *     MMC_ERR_DEVICE and leaves the context unusable except for destroy.
 */
#ifndef MMC_H
#define MMC_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MMC_OK = 0,
    MMC_ERR_ARG = -1,          /* invalid argument (NULL, size, enum, negative count) */
    MMC_ERR_DOMAIN = -2,       /* physically invalid value (T <= 0, Ms0 <= 0, ...) */
    MMC_ERR_OOM = -3,          /* host or device allocation failed */
    MMC_ERR_DEVICE = -4,       /* HIP runtime or kernel error */
    MMC_ERR_STATE = -5,        /* call not valid in the current state */
    MMC_ERR_UNSUPPORTED = -6   /* valid request the library does not implement */
} mmc_status;

typedef struct { int32_t nx, ny, nz; } mmc_grid;          /* each >= 1; nx, ny <= 2048; N <= 2^28; nz <= 32 with demag */
typedef struct { double hx, hy, hz; } mmc_cellsize;       /* metres, > 0 */

/* Mean-field model behind me(T) and chi_par(T). */
typedef enum {
    MMC_MF_LANGEVIN = 0,        /* Eqs. 8-9 as printed (classical spins) */
    MMC_MF_BRILLOUIN_HALF = 1   /* J = 1/2: me = tanh(me Tc/T) */
} mmc_mf;

/* Length trial move and the acceptance exponent k of (mB/mA)^k. */
typedef enum {
    MMC_LEN_PAPER = 0,   /* factor uniform in [1-sigma, 1+sigma], k = 4 (Sec. II, Eq. 5) */
    MMC_LEN_EXACT = 1    /* ln(factor) uniform in [-ln(1+sigma), ln(1+sigma)], k = 3:
                            the exact Metropolis-Hastings ratio for the Eq. 1 target */
} mmc_lenmove;

/* Demag term (Sec. III, Eq. 14) and the precision of its FFT convolution.
 * The tensor spectrum is computed in FP64 and stored in FP32; the x-direction
 * transforms and the layer mixing run in FP32 in every mode.  Layers are
 * mixed directly (no transform along z), for 1 <= nz <= 32; with more than 8
 * layers, or when the 3 nz signals of a padded y column do not fit the
 * one-kernel y pass's registers, the y pass runs as three kernels through a
 * work buffer of (padded x / 2) * 3 nz * padded y complex FP32 values (same
 * arithmetic, more HBM traffic).  The split modes
 * run the radix-16 DFT stages of the y-direction transforms on the matrix
 * cores with each operand split into a high and a low 16-bit part and the
 * products hi*hi + hi*lo + lo*hi accumulated in FP32: BF16 parts keep 16
 * significant bits per operand, FP16 parts 22 (each stage's inputs scaled by a
 * power of two that keeps them in FP16 range).  The split modes need an even
 * nz and a padded y length (the power of two >= 2 ny - 1) of 512, 1024 or
 * 2048 (nz = 2, 4) or 256 or 1024 (nz = 6, 8); other shapes give
 * MMC_ERR_UNSUPPORTED. */
typedef enum {
    MMC_DEMAG_OFF = 0,
    MMC_DEMAG_FP32 = 1,         /* FFT convolution in FP32 */
    MMC_DEMAG_SPLIT_BF16 = 2,   /* y-direction DFT stages as split BF16 matrix products */
    MMC_DEMAG_SPLIT_FP16 = 3    /* y-direction DFT stages as split FP16 matrix products, scaled per stage */
} mmc_demag;

typedef struct {
    double Ms0;          /* zero-temperature saturation magnetization, A/m, > 0 */
    double A0;           /* exchange stiffness at T = 0 (A = A0 me^2), J/m, >= 0 */
    double D0;           /* interfacial DMI constant at T = 0 (D = D0 me^2), J/m^2 */
    double K1, K2;       /* uniaxial anisotropy constants, J/m^3 */
    double easy_axis[3]; /* need not be normalised, non-zero */
    double Tc;           /* Curie temperature, K, > 0 */
    double mu_atomic;    /* atomic moment, J/T, > 0 (Bohr magneton for J = 1/2, g = 2) */
    int32_t mf;          /* mmc_mf */
} mmc_material;

typedef struct {
    uint64_t seed;
    uint32_t chain_id;
    int32_t cone_deg;           /* initial cone half-angle, integer degrees in [1, 180] */
    int32_t adapt_every;        /* sweeps per cone adaptation; 0 disables (paper: 100) */
    double sigma_fixed;         /* > 0: fixed length-move width; <= 0: Eq. 13 capped at 0.03 */
    int32_t lenmove;            /* mmc_lenmove */
    int32_t demag;              /* mmc_demag */
    int32_t refresh_per_sweep;  /* 2: refresh H_d before each colour pass; 1: once per sweep */
    double T;                   /* temperature, K, > 0 */
    double B[3];                /* applied field mu0*H, tesla */
    int32_t init;               /* initial state: 0 uniform along init_dir, 1 random directions (tag 1);
                                   length me(T) below Tc, sqrt(<m^2>) of Eq. 7 at and above Tc */
    double init_dir[3];
} mmc_run;

typedef struct mmc_ctx mmc_ctx;
typedef struct mmc_batch mmc_batch;

/* Create a chain: validates arguments, solves the mean field (FP64, host),
 * builds the demag tensor spectrum (FP64, host), allocates device state and
 * writes the initial state.  hip_stream: a hipStream_t to enqueue on, or NULL
 * for a library-owned stream.  *out is set only on MMC_OK. */
mmc_status mmc_create(const mmc_grid* grid, const mmc_cellsize* cell, const mmc_material* mat,
                      const mmc_run* run, void* hip_stream, mmc_ctx** out);
void mmc_destroy(mmc_ctx* ctx);

/* Granular material (Sec. III, granular film): per-cell grain id (host, N values
 * < n_grains), per-grain easy axis, K1, K2 and Tc; exchange across grain
 * boundaries is scaled by boundary_exchange_scale.  Re-derives the per-grain
 * me, chi_par and sigma and re-initialises the state as mmc_run.init asks. */
mmc_status mmc_set_grains(mmc_ctx* ctx, const uint32_t* grain_of_cell, uint32_t n_grains,
                          const double* easy_axis3, const double* K1, const double* K2,
                          const double* Tc, double boundary_exchange_scale);

/* Applied field mu0*H (tesla) of the Zeeman term of dF (Sec. II); the state
 * is kept.  Errors: MMC_ERR_ARG for NULL, MMC_ERR_DOMAIN for non-finite. */
mmc_status mmc_set_field(mmc_ctx* ctx, const double mu0H_tesla[3]);
/* Chain temperature T > 0 (kelvin).  Re-solves on the host, in FP64, the mean
 * field at H = 0: me(T) (Eq. 9, or its J = 1/2 Brillouin form) and the
 * reduced longitudinal susceptibility chi_par(T) (Eq. 8), hence the Eq. 7
 * coefficients of the longitudinal term and the length-move width sigma
 * (Eq. 13, capped at 0.03); every kT-scaled constant of dF is rescaled.  The
 * state is kept; per-grain temperatures are cleared (every grain at T).
 * Synchronises the context's stream.  Errors: MMC_ERR_DOMAIN for T <= 0 or
 * non-finite. */
mmc_status mmc_set_temperature(mmc_ctx* ctx, double T_kelvin);

/* Non-uniform temperature profile (paper Sec. IV, laser-heated films): grain
 * k (as set by mmc_set_grains; bin the cells of a profile into grains of
 * equal temperature) is held at T_of_grain[k] kelvin (host array, n_grains =
 * the grain count, each > 0 and finite); NULL returns every grain to the
 * chain temperature.  A move at a cell of grain k is judged at T_k: every term
 * of its free-energy change is divided by kB*T_k, and the grain's me, chi_par,
 * sigma and Eq. 7 coefficients are taken at T_k.  The state is kept; a later
 * mmc_set_temperature or mmc_set_grains clears the profile.  Errors:
 * MMC_ERR_STATE without grains, MMC_ERR_ARG for a count mismatch,
 * MMC_ERR_DOMAIN for a non-positive or non-finite temperature. */
mmc_status mmc_set_grain_temperatures(mmc_ctx* ctx, const double* T_of_grain, uint32_t n_grains);

/* Magnetocrystalline anisotropy form (Sec. II, Eqs. 11-12) and temperature law
 * of its constants (Sec. III, Fe granular film). */
typedef enum {
    MMC_ANIS_UNIAXIAL = 0,   /* Eq. 11: K1 (1 - (m.e)^2) + K2 (1 - (m.e)^2)^2, m non-unit, per unit volume,
                                with the easy axes and constants of mmc_material or mmc_set_grains */
    MMC_ANIS_CUBIC = 1       /* Eq. 12 in place of Eq. 11: K1 (a^2 b^2 + a^2 g^2 + b^2 g^2) + K2 a^2 b^2 g^2,
                                a, b, g the direction cosines of m along the crystal axes */
} mmc_anis;
/* Selects the anisotropy of every cell.  kind MMC_ANIS_UNIAXIAL: axes6, K1, K2
 * must be NULL and n 0.  kind MMC_ANIS_CUBIC: n sets (host arrays), n = 1 for
 * every cell or n = the grain count of mmc_set_grains for one set per grain:
 * axes6[6k..6k+5] the first and second crystal axes of set k (any length, not
 * parallel; the second is made orthogonal to the first, the third is their
 * cross product), K1[k], K2[k] the 4th and 6th order cubic constants in
 * J/m^3.  me_scaling = 1 multiplies each constant of order l by
 * me^{l(l+1)/2}, me = me(T) of the grain at its own temperature (uniaxial K1,
 * K2 of orders 2 and 4 by me^3 and me^10; cubic K1, K2 of orders 4 and 6 by
 * me^10 and me^21; zero at and above Tc); 0 uses the constants as given.  The
 * cubic form runs the per-cell colour pass (one cell per thread).  The state
 * is kept; the setting survives mmc_set_field, mmc_set_temperature and
 * mmc_set_grain_temperatures; mmc_set_grains returns to the uniaxial form
 * without the temperature law.  Errors: MMC_ERR_ARG for an unknown kind or
 * flag, NULL or extra arrays, a set count that is neither 1 nor the grain
 * count, zero or parallel axes; MMC_ERR_DOMAIN for non-finite values. */
mmc_status mmc_set_anisotropy(mmc_ctx* ctx, int32_t kind, const double* axes6, const double* K1, const double* K2,
                              uint32_t n, int32_t me_scaling);

/* State in/out, natural SoA layout (3*N floats).  set: every |m_i| > 0 and
 * finite, else MMC_ERR_DOMAIN.  get synchronises the stream. */
mmc_status mmc_set_m(mmc_ctx* ctx, const float* m, int on_device);
mmc_status mmc_get_m(mmc_ctx* ctx, float* out, int on_device);

/* Enqueue n full sweeps (n >= 0), asynchronously on the context's stream.
 * One sweep is one MMC iteration (Sec. II, steps 1-4): for colour 0 then 1,
 * refresh the demag field (Sec. III, Eq. 14) when demag is on, then give every
 * cell of the colour one trial move (cone rotation, length change) accepted
 * by Eq. 5; then reduce the sweep's statistics (FP64), adapt the cone every
 * adapt_every sweeps (Sec. II) and advance the sweep counter, all on the
 * device.  For n >= 16 the launches of 16 sweeps are captured once as a HIP
 * graph on the context's stream (again after a setter changed kernel
 * arguments) and replayed, the rest launched directly: the same kernels in
 * the same order, so the same result bits; MMC_SWEEP_GRAPH=0 in the
 * environment keeps direct launches, and so does a call made while the
 * caller captures the context's stream (the sweeps go into that capture) or
 * on a stream that refuses capture.  Errors: MMC_ERR_ARG for n < 0,
 * MMC_ERR_STATE after a device error, MMC_ERR_DEVICE from a launch. */
mmc_status mmc_sweep(mmc_ctx* ctx, int32_t n);
/* As mmc_sweep, and copies per-sweep statistics to host `series` (n*5 doubles:
 * <mx>, <my>, <mz>, <|m|^2> (FP64 reductions) and the accepted-move count).
 * Blocking: synchronises the context's stream first (row i is the sweep that
 * starts from the device's sweep counter + i, whatever advanced it) and after
 * the copy.  Not for use while the caller captures the context's stream. */
mmc_status mmc_sweep_record(mmc_ctx* ctx, int32_t n, double* series);

/* Instrumented sweeps: as mmc_sweep, with HIP events recorded on the
 * context's stream before and after every kernel launch of sweeps
 * 0, every, 2*every, ... of the n (every >= 1; sampling keeps the event
 * overhead out of the other sweeps); synchronises and returns the summed
 * device time (ms) and the launch count per kernel kind over the sampled
 * sweeps:
 * 0 demag x-forward FFT, 1 demag y-pass (FFT, layer mixing, inverse FFT),
 * 2 demag x-inverse FFT, 3 colour pass, 4 end-of-sweep statistics,
 * 5 fused colour pass (chains of uniform material with nx % 8 == 0 and the
 * field refreshed before each colour, in the form mmc_get_tuning reports:
 * form 1, the x-inverse of the field, the colour pass and the x-forward of the
 * updated rows in one kernel, a sweep call then starting with one x-forward;
 * form 2, the x-inverse and the colour pass in one kernel, each colour
 * preceded by an x-forward). */
mmc_status mmc_sweep_timed(mmc_ctx* ctx, int32_t n, int32_t every, double ms_out[6], int32_t launches_out[6]);

/* Total free energy (J) of the current state and its split {exchange (Eq. 10
 * as the bond sum), DMI (Eq. 15), anisotropy (Eq. 11 or 12), Zeeman,
 * longitudinal (kT times the Eq. 7 exponent), demag (-mu0 V Ms0^2 / 2
 * sum m.h, Eq. 14 with a freshly computed field)}, each summed in FP64.
 * Synchronises the stream.  Either output may be NULL, not both. */
mmc_status mmc_energy(mmc_ctx* ctx, double* E_total_J, double E_terms_J[6]);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, hosts that forbid hipMalloc): mmc_energy without any
 * allocation, host copy or synchronisation.  Enqueues on the context's stream
 * the demag refresh (when demag is on), the energy kernel and a final FP64
 * sum, and writes 7 doubles to out_device (device memory on the context's GPU,
 * owned by the caller): the six terms of mmc_energy in its order, then the
 * total, in joules, equal to what mmc_energy returns for the same state.
 * The per-block partial sums go to a static device array of 2048 x 6 doubles
 * (96 KiB, one copy per GPU, held until the process ends; its address is
 * looked up once per GPU by mmc_create).  Every call on a GPU shares that
 * array: calls that overlap on one GPU (contexts on unordered streams) race,
 * so order them.  The energy kernel strides over the grid with at most 2048
 * blocks, so every grid size fits; a launch that needed more would be
 * rejected with MMC_ERR_UNSUPPORTED.  Errors: MMC_ERR_ARG for NULL,
 * MMC_ERR_STATE after a device error, MMC_ERR_DEVICE from a launch. */
mmc_status mmc_energy_noalloc(mmc_ctx* ctx, double* out_device);

/* Demag field h = H_d/Ms0 of the current state, natural SoA (3*N floats). */
mmc_status mmc_demag_field(mmc_ctx* ctx, float* h_out, int on_device);

/* One colour pass (Sec. II steps 1-4 for the cells of one colour) with the
 * given frozen field h (natural SoA, H_d/Ms0, device or NULL for none) at the
 * current sweep counter and cone angle; writes per-cell decisions (device,
 * N bytes: 1 accepted, 0 rejected, 255 other colour).  Counters and the
 * cone are left unchanged.  For checking the sweep against a reference. */
mmc_status mmc_subsweep(mmc_ctx* ctx, int32_t colour, const float* h_in_device, uint8_t* acc_out_device);

typedef struct {
    uint64_t sweeps;          /* sweeps done (the sweep counter) */
    uint64_t accepts_window;  /* accepted moves since the last cone adaptation */
    int32_t cone_deg;
    double sigma;             /* class 0 length-move width */
    double me;                /* class 0 equilibrium length */
    double m_mean[3];         /* <m> after the last sweep */
    double m2_mean;           /* <|m|^2> after the last sweep */
    uint64_t accepts_last;    /* accepted moves in the last sweep */
} mmc_stats;
/* Run statistics of the chain after the work queued so far (synchronises the
 * stream): the sweep counter, the accept window and cone angle of the
 * adaptation rule (Sec. II), sigma (Eq. 13) and me (Eq. 9) of class 0, and
 * the FP64 means <m>, <|m|^2> and accepted-move count of the last sweep. */
mmc_status mmc_get_stats(mmc_ctx* ctx, mmc_stats* out);

/* Running averages for averaging over chunks of sweeps (the hysteresis-loop
 * rule of Sec. III: chunk averages of the magnetization): every sweep adds
 * its <mx>, <my>, <mz>, <|m|^2> (FP64 means of the sweep's end state) to
 * device accumulators, in batches too.  This call synchronises the context's
 * stream (call mmc_batch_sync first for a chain in a batch), returns the
 * averages over the sweeps since the previous call (zeros when n_out = 0) and
 * their count, and resets the accumulators. */
mmc_status mmc_take_averages(mmc_ctx* ctx, double avg_out[4], uint64_t* n_out);

/* Tile shape of the demag x passes, tuned by the library at mmc_create: the
 * forward and inverse x transforms run with 1, 2 or 4 rows per thread (tiles
 * of 1-4 rows per group of threads that transforms one row); each candidate
 * is timed on the chain's own buffers, the fastest is kept (every candidate
 * gives the same bits) and the choice is cached for the process per (padded x
 * length, ny, nz).  MMC_TUNE=0 in the environment keeps the untuned default.
 * Returns the chosen rows per thread (forward, inverse) and, when
 * us_per_launch is not NULL, the measured microseconds per launch of the
 * candidates (forward 1, 2, 4, inverse 1, 2, 4; zeros when not tuned).
 * MMC_TUNE=1, 2 or 4 forces that many rows per thread in both directions.
 * Also decided at mmc_create: the form of the colour passes (see
 * mmc_sweep_timed, kind 5): 0 separate kernels; 1 fused with the x transforms
 * on either side of it (x-inverse of the field it reads and x-forward of the
 * rows it updated); 2 half fused (the x-inverse only; the x-forward stays a
 * kernel of its own).  For chains that allow it, one colour of each form is
 * timed from the state (restored afterwards, so the chain is unchanged; all
 * forms give the same bits), the fastest is kept and cached per shape;
 * MMC_FUSE=0, 1 or 2 forces a form.  *fused (may be NULL) is the form that
 * runs; fuse_us (may be NULL) the timed us per colour of forms 0, 1, 2 (zeros
 * when not timed).  Errors: MMC_ERR_STATE without demag. */
mmc_status mmc_get_tuning(mmc_ctx* ctx, int32_t rows_per_thread[2], double us_per_launch[6], int32_t* fused,
                          double fuse_us[3]);

/* Run state for checkpoint/resume: the sweep counter, cone angle and accept
 * window; with the state m (mmc_get_m / mmc_set_m) this restores a chain
 * bit-exactly (the generator is stateless).  get synchronises the stream;
 * set needs cone_deg in [1, 180] (else MMC_ERR_ARG). */
mmc_status mmc_get_state(mmc_ctx* ctx, uint64_t* sweep, int32_t* cone_deg, uint64_t* accepts_window);
mmc_status mmc_set_state(mmc_ctx* ctx, uint64_t sweep, int32_t cone_deg, uint64_t accepts_window);

/* Batches: independent chains (any sizes, temperatures, fields) advanced
 * together.  Chains of one shape (grid, cell size, grains on/off, demag and
 * its refresh cadence, move kind, DMI on/off) share every kernel launch, one
 * chain per grid row of blocks; the shape groups run on streams of their
 * own.  mmc_batch_sweep enqueues n sweeps of every chain as one HIP graph
 * launch on the first chain's stream (captured on the first call and again
 * whenever n or a chain's temperature, field or grains changed).  Work
 * enqueued on a chain's own stream before the call (mmc_sweep, say) runs
 * before the batch's sweeps, and work enqueued on it after the call (getters,
 * sweeps) runs after them; chains stay caller-owned, must outlive the batch
 * and must not be changed from another thread while a batch call runs.  All
 * chains must be on the same device.  Results equal
 * running each chain alone, bit for bit.  Errors: MMC_ERR_ARG (NULL, empty,
 * repeated chain, chains on different devices), MMC_ERR_STATE (a chain had a
 * device error), MMC_ERR_DEVICE / MMC_ERR_OOM from HIP. */
mmc_status mmc_batch_create(mmc_ctx* const* chains, int32_t n, mmc_batch** out);
mmc_status mmc_batch_sweep(mmc_batch* batch, int32_t n);
/* Synchronises the first chain's stream; MMC_ERR_DEVICE (and every chain of
 * the batch unusable) if a persistent launch raised its error flag. */
mmc_status mmc_batch_sync(mmc_batch* batch);
void mmc_batch_destroy(mmc_batch* batch);

/* How a batch's sweeps are scheduled (the results are the same bits in every
 * form: each is the single-chain sequence of kernels per chain).  In this
 * build the persistent form is switched off (its launches did not finish on
 * the GPU): requesting it gives MMC_ERR_UNSUPPORTED and MMC_SCHED_AUTO runs
 * the grouped form without trials.
 *   MMC_SCHED_GROUPS: chains of one shape share each launch of the
 *     single-chain sequence, shape groups on streams of their own, the whole
 *     captured as one HIP graph;
 *   MMC_SCHED_PERSISTENT: one persistent kernel per mmc_batch_sweep call
 *     (graph-captured with the reset of its counters) advances every chain:
 *     its blocks take work items (sweep, stage of the sweep, chain, tile) from
 *     a global counter and wait on per-chain completion counts, so small and
 *     large chains, temperatures and fields interleave in one launch.  It
 *     serves chains of uniform material without DMI, with demag off or FP32
 *     with nz 1 or 2, 17 <= nx <= 1024 and 17 <= ny <= 512, and one
 *     length-move kind across the batch (else MMC_ERR_UNSUPPORTED).  A wait
 *     that exceeds 5 s raises an error flag that mmc_batch_sync reports;
 *   MMC_SCHED_AUTO (default): on the first mmc_batch_sweep the library times
 *     three sweeps of each form that serves the chains, from the same state
 *     (restored afterwards, so the chains continue bit for bit), keeps the
 *     faster and caches the choice for batches of the same chain shapes.
 * set: the choice applies from the next mmc_batch_sweep.  get: the form in
 * use (MMC_SCHED_GROUPS before the first sweep under AUTO) and the trial
 * times in ms (groups, persistent; 0 when not timed); trial_ms may be NULL. */
typedef enum { MMC_SCHED_AUTO = 0, MMC_SCHED_GROUPS = 1, MMC_SCHED_PERSISTENT = 2 } mmc_sched;
mmc_status mmc_batch_set_schedule(mmc_batch* batch, int32_t sched);
mmc_status mmc_batch_get_schedule(mmc_batch* batch, int32_t* used, double trial_ms[2]);

/* Synchronise the context's stream. */
mmc_status mmc_sync(mmc_ctx* ctx);

const char* mmc_status_str(mmc_status s);
const char* mmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
