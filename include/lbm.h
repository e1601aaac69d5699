/*
 * lbm.h — C-ABI of liblbm.so: the D3Q19 MRT-Smagorinsky LES update with Guo
 * forcing on a periodic lattice, run by HIP kernels on one AMD Instinct MI355X
 * (gfx950).
 *
 * Method (Khan, Succi & Falcucci, "Validating the Boltzmann approach to the
 * large-eddy simulations of forced homogeneous incompressible turbulence",
 * arXiv:2512.23116):
 *   - lattice: D3Q19, App. B Fig. d3q19_table (velocities 0..18 here are the
 *     paper's 1..19; opposite pairs (0,1),(2,3),...,(16,17); rest = 18);
 *   - update: eq. mrt_les_guo (collide, then stream along c_a) with the
 *     moment matrix of eq. moment-matrix, the rates of eq. relaxation-matrix,
 *     the equilibrium and force moments of eq. meq_fm, the Guo velocity of
 *     eq. guo_velocity;
 *   - closure: per-cell tau_e = 1/2 + 3 (nu0 + C Delta^2 |S|)
 *     (eq. nu_eff_mrt, eq. eddy_visc, eq. les_viscosity) with |S| of
 *     eq. strain_norm from the strain of eq. yu_strain (s_1 = s_e, s_9 = 1/tau0,
 *     Delta = delta_x = delta_t = 1);
 *   - diagnostic: the turbulent Knudsen number K_t = sqrt(3) (tau_e - 1/2)
 *     (eq. Kt_definition with ell = delta_x, Sec. 2.4).
 *
 * Conventions for every call
 *   - Every entry point returns an lbm_status; no C++ exception crosses the
 *     ABI.  lbm_last_error() gives a message for the last failing call on a
 *     handle.
 *   - Host pointers are plain host memory owned by the caller, with the sizes
 *     stated per call; the library never keeps them after the call returns.
 *   - Cell index c = x + nx (y + ny z), x fastest, 0-based coordinates.
 *   - The observable state after n steps is the pre-collision, post-streaming
 *     population field f(x, n) of eq. mrt_dns_guo.  It does not depend on the
 *     streaming scheme or on the parity of n.
 *   - All work is issued on the handle's HIP stream.  lbm_step returns before
 *     the GPU finishes; kernel errors surface at the next synchronising call
 *     (every call that writes host memory synchronises the stream).
 *   - A handle is used from one host thread at a time.
 */
#ifndef LBM_H_
#define LBM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_ERR_INVALID_ARG = -1,  /* bad config or argument; nothing was changed */
    LBM_ERR_OUT_OF_MEMORY = -2,/* a device or host allocation failed          */
    LBM_ERR_DEVICE = -3,       /* a HIP call or a kernel failed               */
    LBM_ERR_UNSTABLE = -4,     /* the state holds NaN/Inf (reported by the
                                  diagnostic calls)                          */
    LBM_ERR_STATE = -5         /* call out of order (e.g. step before init)   */
} lbm_status;

/* Storage of the populations.  The device always stores the deviations
 * g = f - w rho0 (w: lattice weights); collisions run in FP64 for LBM_FP64
 * and in FP32 otherwise.  The FP16/BF16 forms store round-to-nearest-even
 * (sigma * g) with a per-run power-of-two scale sigma. */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16_DEV = 2, LBM_BF16_DEV = 3 } lbm_precision;

/* LBM_STREAM_AA: one array, updated in place with the AA access pattern
 *   (even steps read and write a cell's own slots, odd steps its neighbours').
 * LBM_STREAM_AB: two arrays, pull streaming from one into the other. */
typedef enum { LBM_STREAM_AA = 0, LBM_STREAM_AB = 1 } lbm_streaming;

/* Initial velocity field; the initial populations are the second-order
 * equilibrium of App. A eq. feq at rho = rho0 and that velocity.
 *   NOISE: u_a = A (2U - 1), U = (splitmix64(splitmix64(seed) ^ (3c + a)) >> 11) 2^-53
 *   TGV3D: u = A sin X cos Y cos Z, v = -A cos X sin Y cos Z, w = 0
 *          (X = 2 pi x/nx, ...; the Taylor-Green start of Sec. 2.2 and 3.1)
 *   TGV2D: u = A sin X cos Y, v = -A cos X sin Y, w = 0
 *   SHEAR: u = A sin Y
 *   REST : u = 0 */
typedef enum {
    LBM_INIT_NOISE = 0, LBM_INIT_TGV3D = 1, LBM_INIT_TGV2D = 2,
    LBM_INIT_SHEAR = 3, LBM_INIT_REST = 4
} lbm_init_kind;

/* One Fourier mode of the static body force (the general form of Sec. 2.2
 * eq. forcing_pattern):  F(x) += amp * sin(2 pi (k0 x/nx + k1 y/ny + k2 z/nz) + phase).
 * |k0| <= 2 is required (the force is evaluated per cell from x-harmonics 1
 * and 2 and a per-(y,z) coefficient table); k1 and k2 are free. */
typedef struct {
    int32_t k[3];
    int32_t reserved;   /* must be 0 */
    double amp[3];
    double phase;
} lbm_force_mode;

typedef struct {
    int32_t nx, ny, nz;      /* lattice size, each >= 1, nx*ny*nz < 2^31     */
    int32_t precision;       /* lbm_precision                                 */
    int32_t streaming;       /* lbm_streaming                                 */
    int32_t smag_form;       /* 0: nu_t = C |S| (the paper's linear constant, */
                             /*    eq. eddy_visc); 1: nu_t = C^2 |S|          */
    double tau0;             /* bare relaxation time 1/s_nu, > 1/2            */
    double smag_C;           /* Smagorinsky constant C >= 0; 0 gives DNS-MRT  */
    double rho0;             /* reference density (1 in the paper), > 0       */
    double s_e, s_eps, s_q, s_pi, s_m;  /* fixed rates of eq. relaxation-matrix:
                                           1.19, 1.4, 1.2, 1.4, 1.98         */
    double storage_scale;    /* sigma for FP16/BF16 storage; 0 selects the
                                default (2^15 for FP16, 1 for BF16)           */
    int32_t n_force_modes;   /* 0..64                                         */
    int32_t steps_per_graph; /* steps captured per HIP graph in lbm_step
                                (even, 2..1024); 0 disables graphs            */
    int32_t temporal_block;  /* 0 or 1: one time step per pass over memory.
                                2: pairs of steps run in one pass (A/B only,
                                FP32/FP16/BF16; steps_per_graph a multiple of
                                4 or 0): the intermediate level stays in LDS,
                                halving HBM traffic per step at ~19% more
                                arithmetic.  Results equal single steps up to
                                the rounding of the FP32 collision, and do not
                                depend on how a launch splits the work.        */
    int32_t tau_mode;        /* which relaxation rate enters the strain
                                estimate of App. B.1 eq. yu_strain:
                                0: s_1 = s_e and s_9 = 1/tau0 (explicit,
                                   default);
                                1: self-consistent s_9 = 1/tau_e with the
                                   s_1 (divergence) term dropped, solved in
                                   closed form: tau_e = (tau0 + sqrt(tau0^2
                                   + 4 c3 |S_1|)) / 2, S_1 = eq. yu_strain at
                                   s_1 = 0, s_9 = 1, c3 = 3 C or 3 C^2.      */
    const lbm_force_mode* force_modes; /* copied at create                   */
    void* hip_stream;        /* hipStream_t to run on; NULL = null stream     */
    void* device_buffer;     /* optional caller-owned device memory for the
                                population state (e.g. a torch tensor), at
                                least lbm_required_bytes() bytes, 256-B
                                aligned; kept alive by the caller until
                                lbm_destroy.  NULL: the library allocates.   */
    uint64_t device_buffer_bytes;
} lbm_config;

typedef struct lbm_handle lbm_handle;
typedef struct lbm_batch lbm_batch;

/* FP64 statistics of the state after the current step (Sec. 5.1 reports
 * domain statistics of tau_e - 1/2).  theta = tau_e - 1/2 and K_t = sqrt(3) theta
 * per cell; var is the population variance, skew = mu3/var^1.5,
 * flat = mu4/var^2 (NaN when var = 0). */
typedef struct {
    int64_t n_cells;
    int64_t steps;            /* steps done when the statistics were taken   */
    double theta_mean, theta_var, theta_skew, theta_flat, theta_min, theta_max;
    double kt_mean, kt_var, kt_skew, kt_flat, kt_min, kt_max;
    double mass;              /* sum of rho over cells                       */
    double momentum[3];       /* sum of rho u (with the half-force shift)     */
    double energy;            /* (1/2) <u.u>, unweighted domain mean          */
    double energy_rho;        /* (1/2) <rho u.u>                              */
    int64_t n_nonfinite;      /* cells whose populations or tau_e are NaN/Inf */
    double strain2;           /* <|S|^2> = 2 <S:S>, S the strain that sets tau_e
                                 (eq. yu_strain); nu0 <|S|^2> is the resolved
                                 dissipation 2 nu0 <S:S> of eq. energy_balance */
    double nut_strain2;       /* <nu_t |S|^2>, nu_t = (tau_e - tau0) / 3: the
                                 dissipation by the Smagorinsky viscosity     */
    double injection;         /* <F.u>: power injected by the forcing
                                 (eq. energy_balance)                          */
    double u_mean[3];         /* <u>                                           */
    double uu[6];             /* <u_i u_j>: xx, yy, zz, xy, xz, yz             */
} lbm_stats;

/* Fill *cfg with the paper's defaults: 32^3, FP32, AA, tau0 = 0.51, C = 0.1,
 * linear C, rho0 = 1, rates 1.19/1.4/1.2/1.4/1.98, no forcing, 64 steps per
 * graph, one step per pass, null stream, library-owned memory. */
void lbm_config_default(lbm_config* cfg);

/* Bytes of device memory the population state needs: 19 direction planes per
 * array (one array for AA, two for AB), each plane holding nx*ny*nz cells
 * rounded up to 64 plus 1728 cells of padding that staggers the plane starts
 * across HBM channels; 0 if cfg is invalid. */
size_t lbm_required_bytes(const lbm_config* cfg);

/* Validate cfg, allocate the state and the small per-lattice tables on the
 * current HIP device, evaluate the forcing tables on the device.  The state
 * is undefined until lbm_init_seeded or lbm_set_populations.
 * Errors: INVALID_ARG (cfg), OUT_OF_MEMORY, DEVICE.  *out is NULL on error. */
lbm_status lbm_create(const lbm_config* cfg, lbm_handle** out);

/* Set f(x, 0) = f_eq(rho0, u0(x)) (App. A eq. feq) for the velocity of
 * `kind` (lbm_init_kind) and amplitude A; resets the step count to 0. */
lbm_status lbm_init_seeded(lbm_handle* h, int32_t kind, double amplitude, uint64_t seed);

/* Set f(x, 0) = f_eq(rho(x), u(x)) (App. A eq. feq) from fields the caller
 * holds in device memory of the lattice's device: u[a * ncells + c] (a = x, y,
 * z; c = x + nx (y + ny z)), FP64 lattice units, and rho[c], or rho = NULL for
 * rho0 everywhere.  Starts a run from a given flow, e.g. one interpolated from
 * a coarser lattice.  Resets the step count to 0.  The kernel reads u and rho on
 * the lattice's stream after the call returns: the caller orders their writes
 * before it and keeps them alive until the stream has passed it (lbm_synchronize).
 * Errors: INVALID_ARG (u NULL, or u / rho not device memory of that device),
 * DEVICE. */
lbm_status lbm_init_velocity(lbm_handle* h, const double* u, const double* rho);

/* Advance n >= 0 steps of eq. mrt_les_guo, asynchronously on the stream.
 * Full graphs of steps_per_graph steps are replayed, the rest is launched. */
lbm_status lbm_step(lbm_handle* h, int64_t n);

/* Advance n >= 0 steps of free streaming: the left side of eq. mrt_dns_guo with
 * the collision replaced by the identity (f(x + c_i, t + 1) = f(x, t), no force),
 * i.e. every population moves one cell along its velocity, periodically.  It
 * performs exactly the loads and stores of lbm_step (same access pattern,
 * block order and state layout, no arithmetic), so its duration is the
 * ceiling of the step's data movement; the state stays exact in every storage
 * format.  Plain launches, asynchronous; counts as steps (lbm_steps_done). */
lbm_status lbm_stream_only(lbm_handle* h, int64_t n);

/* rho[c] and u[a * ncells + c] (a = x, y, z) of the current state, with the
 * half-force velocity of eq. guo_velocity.  Host arrays of ncells and
 * 3*ncells doubles; either may be NULL.  Synchronises. */
lbm_status lbm_moments(lbm_handle* h, double* rho, double* u);

/* Domain statistics of theta and K_t plus mass, momentum and energy, reduced
 * on the device in FP64 in a fixed order (bitwise reproducible).  tau_e is
 * computed by the same device code as the step.  Returns LBM_ERR_UNSTABLE
 * (with *out filled) when any cell is non-finite.  Synchronises. */
lbm_status lbm_kt_stats(lbm_handle* h, lbm_stats* out);

/* Per-cell K_t = sqrt(3) (tau_e - 1/2) of the current state, host float[ncells].
 * Synchronises. */
lbm_status lbm_kt_field(lbm_handle* h, float* kt);

/* The K_t map of one plane (Sec. 5.1 shows such slices): kt[x + nx y] = K_t of
 * cell (x, y, z), host float[nx*ny], the same values as lbm_kt_field for that
 * plane.  Only the plane is evaluated and copied.  0 <= z < nz, else
 * LBM_ERR_INVALID_ARG.  Synchronises. */
lbm_status lbm_kt_slice(lbm_handle* h, int32_t z, float* kt);

/* Canonical full populations f[a * ncells + c] of the current state (host,
 * 19 * ncells doubles).  Synchronises. */
lbm_status lbm_get_populations(lbm_handle* h, double* f);

/* Replace the state by the full populations f[a * ncells + c] (host, 19 *
 * ncells doubles) — converted to the storage precision — keeping the step
 * count.  Synchronises. */
lbm_status lbm_set_populations(lbm_handle* h, const double* f);

/* Canonical full populations of the listed cells: out[i * 19 + a] for cell
 * cells[i] (0 <= cells[i] < ncells).  Host arrays.  Synchronises. */
lbm_status lbm_sample_populations(lbm_handle* h, const int64_t* cells, int64_t n, double* out);

/* Fixed-bin histogram of theta = tau_e - 1/2 over the cells of the current
 * state (Sec. 5.1 shows its distribution; eq. les_viscosity), theta per cell as
 * in lbm_kt_field (FP64 from the kernel's tau_t):
 *   counts[0]          cells with theta < lo,
 *   counts[1 + b]      cells with floor((theta - lo) * (nbins / (hi - lo))) = b,
 *                      b = 0..nbins-1 (the product taken in FP64),
 *   counts[nbins + 1]  cells whose bin index would be >= nbins,
 *   counts[nbins + 2]  cells with a non-finite theta.
 * Host int64[nbins + 3]; exact integer counts (they sum to the cell count).
 * 1 <= nbins <= 4096, lo < hi finite.  Uses a device buffer the handle keeps
 * until lbm_destroy.  Synchronises. */
lbm_status lbm_theta_histogram(lbm_handle* h, double lo, double hi, int32_t nbins,
                               int64_t* counts);

/* The same histogram as lbm_theta_histogram, for callers that cannot allocate
 * device memory (code running while a HIP graph is being captured, tight
 * serving loops, harnesses that forbid hipMalloc): no hipMalloc, hipFree or
 * allocating library call.  The counts live in a static device array of the
 * library (4099 64-bit counters, 32.8 KB per GPU, held until the process
 * ends), looked up once per device; each call clears the counters it uses with
 * a kernel before counting.  Arguments, output and errors as in
 * lbm_theta_histogram; nbins > 4096 (beyond the static array) is
 * LBM_ERR_INVALID_ARG.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (several host threads or streams) race.  Synchronises. */
lbm_status lbm_theta_histogram_noalloc(lbm_handle* h, double lo, double hi, int32_t nbins,
                                       int64_t* counts);

/* Snapshot of the current state for a run that keeps stepping: its statistics
 * (as lbm_kt_stats), the K_t map of plane z (as lbm_kt_slice) and its spectrum
 * E[0..kmax] (as lbm_spectrum), without waiting for them.
 * lbm_snapshot_begin enqueues on the handle's stream, in order with the steps,
 * the kernels that read the state (reductions, K_t plane, velocity), the FFTs
 * and shell sums of the velocity, and the copies of the results to page-locked
 * host memory, and returns at once: the caller can enqueue the next lbm_step
 * before it waits, so the device never idles on the host.
 * lbm_snapshot_end waits for the snapshot and writes its results: stats (as
 * lbm_kt_stats, steps = the step count at lbm_snapshot_begin), E (host
 * double[kmax+1]) and kt_plane (host float[nx*ny]); any may be NULL.
 * 0 <= kmax <= 4096, 0 <= z < nz, else INVALID_ARG.  One snapshot per handle
 * at a time: begin while one is pending, or end with none pending, is
 * LBM_ERR_STATE, and so are the other analysis calls (spectra, structure
 * functions, turbulence scales) until lbm_snapshot_end.  UNSTABLE as in
 * lbm_kt_stats.  Buffers are kept until lbm_destroy. */
lbm_status lbm_snapshot_begin(lbm_handle* h, int32_t kmax, int32_t z);
lbm_status lbm_snapshot_end(lbm_handle* h, lbm_stats* stats, double* E, float* kt_plane);

/* Shell-binned kinetic-energy spectrum of the current state (Sec. 2.2,
 * eq. integral_length_scale with the squared modulus):
 *   E[k] = 1/2 sum_{k - 1/2 <= |q| < k + 1/2} |u_hat(q)|^2,  u_hat = FFT(u) / ncells,
 * for integer shells k = 0..kmax (0 <= kmax <= 4096), u the velocity with the
 * half-force shift of eq. guo_velocity.  FP64 FFT (hipFFT) on the device; the
 * shell sums run in a fixed order, so a state gives the same spectrum bit for
 * bit on every call (and through lbm_snapshot_begin/_end).  Host
 * double[kmax+1].  The first call creates the FFT plan and device buffers
 * (~32 bytes per cell, ~48 for lattices of up to 2^24 cells, whose three
 * velocity components are transformed in one batched call; plus kmax-sized
 * partial sums) that the handle keeps for later analysis calls until
 * lbm_destroy.
 * Synchronises. */
lbm_status lbm_spectrum(lbm_handle* h, int32_t kmax, double* E);

/* One-dimensional energy spectra and the spectral isotropy coefficient of the
 * current state (App. spectral isotropy: longitudinal and transverse spectra
 * E_11, E_22 and IC(k)):
 *   E[(3 c + a)(kmax + 1) + k] = sum of |u_hat_c(q)|^2 over the wavevectors q
 *   with |q_a| = k,  u_hat = FFT(u) / ncells,
 * for velocity component c and axis a (0, 1, 2 = x, y, z), integer k = 0..kmax
 * (0 <= kmax <= 2048; zero beyond n_a / 2), so that sum_k E[c][a][k] = <u_c^2>.
 * If ic is not NULL (cubic lattices only, else LBM_ERR_INVALID_ARG), ic[k] =
 * (E_L - k dE_L/dk) / (2 E_T) at k = 2..kmax-1 (NaN elsewhere and where
 * E_L(k +- 1) or E_T(k) is not positive): E_L, E_T are the means of the 3
 * longitudinal (c = a) and 6 transverse spectra, k dE_L/dk = E_L times the
 * central difference of ln E_L over ln k (exact for power laws).  The paper's printed
 * ratio does not equal 1 for isotropic fields; this is the isotropic relation
 * E_22 = (E_11 - k dE_11/dk) / 2, under which IC = 1.  FP64 FFT (hipFFT) on the
 * device, sums in a fixed order (bitwise the same on every call).  Host
 * double[9 (kmax+1)] and double[kmax+1].  Shares the analysis buffers and FFT
 * plan of lbm_spectrum.  Synchronises. */
lbm_status lbm_spectra_1d(lbm_handle* h, int32_t kmax, double* E, double* ic);

/* Longitudinal structure functions of the current state (Sec. 5.3): for each
 * separation rs[j] >= 1 (taken modulo the lattice size per axis),
 *   out[6 j + m] = mean over cells x and axes a of p_m(du),
 *   du = u_a(x + r e_a) - u_a(x) (periodic),  p = (du^2, du^3, |du|^3, du^4, |du|^5, du^6).
 * F4(r) = out[6j+3] / out[6j]^2.  FP64, reduced in a fixed order (bitwise
 * reproducible).  nr in 1..65535.  Uses the handle's analysis velocity buffer
 * (created on first use, 24 bytes per cell) and temporaries.  Synchronises. */
lbm_status lbm_structure_functions(lbm_handle* h, const int32_t* rs, int32_t nr, double* out);

/* Turbulence scales of the current state (Sec. 2.2, eq. integral_length_scale,
 * eq. kolmogorov_scale, eq. taylor_microscale, eq. rms_velocity,
 * eq. dissipation_rate, eq. energy_balance) on a cubic N^3 lattice.  Spectral
 * quantities use the shell spectrum of lbm_spectrum for shells 1..kmax
 * (kmax <= 0: every shell) with wavenumber kappa = 2 pi k / N (lattice units,
 * delta_x = 1; the paper's 2 pi box maps onto N cells) and the molecular
 * viscosity nu0 = (tau0 - 1/2)/3.  Real-space quantities come from the FP64
 * reductions of lbm_kt_stats.  INVALID_ARG for a non-cubic lattice.  Allocates
 * device temporaries.  Synchronises. */
typedef struct {
    int32_t kmax;             /* shells summed: 1..kmax                      */
    int32_t pad;
    double energy;            /* 1/2 <u.u> in real space (eq. energy_balance) */
    double energy_spec;       /* sum_{k=1..kmax} E(k) (the mean flow excluded) */
    double u_rms;             /* sqrt(2 energy_spec / 3)                      */
    double integral_scale;    /* L = (3 pi / 4) sum(E/kappa) / sum(E)         */
    double eps_spec;          /* 2 nu0 sum kappa^2 E(k)                       */
    double eps_strain;        /* 2 nu0 <S:S> = nu0 <|S|^2>, S of eq. yu_strain */
    double eps_sgs;           /* <nu_t |S|^2>: Smagorinsky dissipation         */
    double injection;         /* <F.u>                                       */
    double eta;               /* (nu0^3 / eps_spec)^(1/4)                     */
    double taylor;            /* sqrt(15 nu0 u_rms^2 / eps_spec)              */
    double re_lambda;         /* u_rms taylor / nu0                           */
    /* statistical isotropy (Sec. 3.3) from the Reynolds stresses
     * R_ij = <u_i u_j> - <u_i><u_j>: directional energy fractions R_ii / R_kk,
     * anisotropy b_ij = R_ij / R_kk - delta_ij / 3 (xx, yy, zz, xy, xz, yz), its
     * invariants II_b = -b_ij b_ji / 2, III_b = b_ij b_jk b_ki / 3 and the
     * Lumley-triangle coordinates xi = (III_b/2)^(1/3) (signed), eta = (-II_b/3)^(1/2) */
    double energy_frac[3];
    double b[6];
    double II_b, III_b, lumley_xi, lumley_eta;
} lbm_turbulence_stats;
lbm_status lbm_turbulence(lbm_handle* h, int32_t kmax, lbm_turbulence_stats* out);

/* Checkpoint / resume in the storage format: lbm_state_bytes() bytes of
 * opaque state (host memory) plus the step count.  Restoring into a handle
 * created with the same config reproduces the run bitwise.  Both synchronise.
 * INVALID_ARG if `bytes` differs from lbm_state_bytes(). */
size_t lbm_state_bytes(const lbm_handle* h);
lbm_status lbm_save_state(lbm_handle* h, void* host, size_t bytes, int64_t* steps);
lbm_status lbm_load_state(lbm_handle* h, const void* host, size_t bytes, int64_t steps);

/* Wait for all work issued on the handle's stream; DEVICE on kernel errors. */
lbm_status lbm_synchronize(lbm_handle* h);

/* Move the handle to another HIP stream (hipStream_t, or NULL for the null
 * stream): every later call on the handle, its graph replays included,
 * enqueues there.  Nothing is synchronised and nothing is launched: the caller
 * orders the new stream after the work still pending on the old one (for
 * instance with an event), as it would for any two streams.  Used by the
 * serving loop to set a lattice up and to read its final statistics on a side
 * stream while batched steps run on the main one.  Always LBM_OK for a
 * non-NULL handle. */
lbm_status lbm_set_stream(lbm_handle* h, void* hip_stream);

int64_t lbm_steps_done(const lbm_handle* h);
int64_t lbm_num_cells(const lbm_handle* h);

/* Release everything the handle owns (not a caller-provided device buffer).
 * NULL is allowed.  Synchronises the stream first. */
void lbm_destroy(lbm_handle* h);

const char* lbm_status_string(lbm_status s);
const char* lbm_last_error(const lbm_handle* h);

/* ---- Batched stepping of independent lattices (continuous batching) ------
 * A batch steps up to max_slots handles with one kernel launch per step: the
 * launch covers every slot's cells through a device-side slot table, so
 * independent runs of different sizes and parameters share the GPU.  The
 * handles must be FP32 with AA streaming, initialised, and created on the
 * batch's stream; each result is bitwise the same whether its handle is
 * stepped alone or with others.  Launches are captured once in a HIP graph of
 * steps_per_graph launches whose kernels read the slot table from device
 * memory, so changing the set of handles between calls does not recapture.
 * Calls that overlap on one batch must not be made from several threads.
 *
 * lbm_batch_create: max_slots in 1..1024; steps_per_graph even in 2..1024,
 *   or 0 for plain launches; hip_stream as in lbm_config.
 * lbm_batch_step: advance hs[i] by steps[i] (0 <= steps[i] <= steps_per_graph,
 *   or any >= 0 when steps_per_graph is 0) for i < n <= max_slots, handles
 *   distinct.  One graph replay when max steps[i] equals steps_per_graph, else
 *   max steps[i] plain launches.  Asynchronous; INVALID_ARG (nothing launched)
 *   on a bad argument.
 * lbm_batch_destroy: NULL allowed; synchronises the stream first. */
lbm_status lbm_batch_create(int32_t max_slots, int32_t steps_per_graph, void* hip_stream,
                            lbm_batch** out);
lbm_status lbm_batch_step(lbm_batch* b, lbm_handle* const* hs, const int32_t* steps, int32_t n);
const char* lbm_batch_last_error(const lbm_batch* b);
void lbm_batch_destroy(lbm_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H_ */
