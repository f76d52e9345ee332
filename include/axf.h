/*
 * axf.h -- C ABI of the MI355X axion-coupled Yee step (libaxf.so).
 *
 * The library advances, on one gfx950 GPU, the coupled system of
 * An et al., "Modeling of axion and electromagnetic fields coupling in a
 * particle-in-cell code" (arXiv 2406.16796), in natural units (c = 1):
 *
 *   Klein-Gordon axion      d_t^2 phi - lap phi + m^2 phi = g E0.B0     (Sec. II.A, eq. wave_axion)
 *   first-order EM (FPS)    d_t E1 = curl B1 - g[(d_t phi) B0 - E0 x grad phi],
 *                           d_t B1 = -curl E1                              (Sec. II.B, eq. curl-b1)
 *   zero-order EM (laser)   vacuum Maxwell for E0, B0; a static B_ext is
 *                           added to B0 wherever B0 enters a source term.
 *
 * on the staggered layout of Sec. II.C (phi at cell centres, E on faces, B on
 * edges) with the time discretisation of Sec. II.C (axion at half-integer
 * times, phi^n the mean of its neighbours), stored in the equivalent
 * leapfrog form E^{n-1/2}, B^n, phi^{n-1/2}, phi^{n+1/2}.  Axion boundaries:
 * periodic, reflect, outflow, PML (Sec. II.D).  EM boundaries: periodic, or
 * first-order Mur on the tangential E half a cell outside the boundary node
 * plane, with a laser entering through the x_min face.
 *
 * Conventions for every call:
 *   - every function returns 0 (AXF_OK) or a negative AXF_E* code and never
 *     throws or aborts; axf_last_error() gives a message for the calling thread;
 *   - device memory passed in is owned by the caller and must outlive the
 *     objects carved from it; the library never frees it;
 *   - `stream` is a hipStream_t (NULL = default stream); all GPU work of a run
 *     is enqueued on its stream and is asynchronous unless stated otherwise;
 *   - arrays crossing the ABI are dense, x fastest, with the storage extents
 *     of axf_extents() (n + 1 along Mur axes for nodal components, n otherwise).
 */
#ifndef AXF_H
#define AXF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
enum {
    AXF_OK = 0,
    AXF_EINVAL = -1,     /* bad argument or configuration */
    AXF_ENOMEM = -2,     /* caller buffer too small / budget exceeded */
    AXF_EHIP = -3,       /* a HIP runtime call failed */
    AXF_EUNSTABLE = -4,  /* time step beyond the Yee / Klein-Gordon limit */
    AXF_EBUSY = -5,      /* server full, or object still in use */
    AXF_ENOTFOUND = -6,  /* unknown request id or field */
    AXF_ESTATE = -7      /* call not allowed in the current state */
};

enum { AXF_F32 = 0, AXF_F64 = 1 };                       /* field storage precision */
enum { AXF_EM_PERIODIC = 0, AXF_EM_MUR = 1 };
enum { AXF_AX_PERIODIC = 0, AXF_AX_REFLECT = 1, AXF_AX_OUTFLOW = 2, AXF_AX_PML = 3 };
enum { AXF_ENV_CW = 0, AXF_ENV_GAUSS = 1 };
/* step kernels: PLAIN the unfused phases (one launch per phase of Sec. II.C);
   FUSED the fused step of the dimensionality (1D: multi-step LDS passes; 2D:
   the wavefront march, up to four steps per pass; 3D FP32: the one-pass z
   march; 3D FP64: the merged tile walks); AUTO takes FUSED wherever the run
   supports it.  Every path gives the same bits. */
enum { AXF_PATH_AUTO = 0, AXF_PATH_PLAIN = 1, AXF_PATH_FUSED = 2 };

/* field ids for axf_read_field / axf_write_field */
enum {
    AXF_E0X = 0, AXF_E0Y, AXF_E0Z, AXF_B0X, AXF_B0Y, AXF_B0Z,
    AXF_E1X, AXF_E1Y, AXF_E1Z, AXF_B1X, AXF_B1Y, AXF_B1Z,
    AXF_PHI_OLD,   /* phi at t_n - dt/2 */
    AXF_PHI_NEW,   /* phi at t_n + dt/2 */
    AXF_NFIELDS
};

/* ---------------------------------------------------------------- config
 * One run.  Axes 0..ndim-1 are active; n[d] = 1 for d >= ndim, and those
 * axes are periodic.  Active components per ndim (others are identically zero
 * for the allowed inputs and are not stored):
 *   ndim 1: E0y E0z B0y B0z, E1y E1z B1y B1z   (requires bext[0] == 0)
 *   ndim 2: E0x E0y B0z, all six E1/B1          (laser polarised along y)
 *   ndim 3: all twelve.
 */
typedef struct {
    int32_t ndim;            /* 1, 2 or 3 */
    int32_t n[3];            /* cells per axis */
    double  dx[3];           /* cell size per axis */
    double  dt;              /* time step; must satisfy dt^2 (sum 1/dx^2 + m^2/4) < 1 */
    int32_t precision;       /* AXF_F32 or AXF_F64 */
    int32_t em_bc[3];        /* AXF_EM_* per axis (both faces) */
    int32_t ax_bc[3];        /* AXF_AX_* per axis (both faces) */
    int32_t pml_n;           /* PML thickness in cells (Sec. III.A: 20) */
    double  pml_sigma_dt;    /* sigma_max * dt (Sec. III.A: 0.2) */
    double  m;               /* axion mass */
    double  g;               /* axion-photon coupling */
    double  bext[3];         /* static external B */
    int32_t slab_lo, slab_hi;/* B_ext present for cells slab_lo <= i < slab_hi along x */
    /* laser through x_min, along +x */
    int32_t laser_on;
    int32_t laser_pol;       /* 1: E along y, 2: E along z */
    int32_t laser_env;       /* AXF_ENV_CW (sin^2 ramp) or AXF_ENV_GAUSS */
    double  omega;           /* angular frequency */
    double  e_amp;           /* peak field */
    double  ramp_periods;    /* CW ramp length in periods */
    double  fwhm;            /* Gaussian intensity FWHM duration */
    double  t_center;        /* time the Gaussian peak crosses x = 0 */
    double  waist;           /* 1/e field radius at focus; 0 = plane wave */
    double  x_focus, y_c, z_c;
    double  cep;
    /* initial axion packet A exp(-(eta^2 + r_perp^2)/w^2) sin(k eta), eta = x - x0 - dir t,
       set at t = -dt/2 and +dt/2 (Sec. III.A) */
    int32_t packet_on;
    double  pk_amp, pk_k, pk_w, pk_x0, pk_y0, pk_z0;
    int32_t pk_dir;          /* +1 or -1 */
    /* execution */
    int32_t diag_every;      /* record energies every k steps (0: only on request) */
    int32_t path;            /* AXF_PATH_*: step kernels to use */
    /* moving window (Sec. III.B: the window follows the laser at c once it is
       in).  win_cells = 0: a fixed window.  Otherwise, before step n, once
       n dt >= win_t0, the window has moved win_cells * floor((n dt - win_t0) /
       (win_cells dx)) columns along +x: every field shifts left, new columns
       are vacuum, B_ext's slab stays where it is in the lab (it moves left in
       the window) and the laser is no longer injected; the x_min ghosts take
       the values that lay there before a move, the x_max ghosts are vacuum.
       Needs a Mur x axis, 1 <= win_cells <= 64, win_cells < n[0] and
       win_t0 >= dt; single runs only (not batches or served requests). */
    double  win_t0;
    int32_t win_cells;
    /* which order carries the injected laser: 0 (E0/B0) or 1 (E1/B1: the weak
       laser of Sec. III.D on a strong background).  1 needs the unfused path. */
    int32_t laser_order;
    /* Cold plasma electrons, the particle side of the first-order expansion
       (Sec. II.B): charge -1, mass 1, immobile neutralising ions; ppc[0] x
       ppc[1] particles per cell on a regular lattice in the cells
       plasma_lo <= i < plasma_hi along x and every cell along y, density
       plasma_n in critical densities (omega_p^2 = plasma_n), momentum
       u = p/(m c) = plasma_u at t = 0.  ppc[0] = 0: no particles.  Particles
       need ndim 2, a periodic y axis, the plasma at least two cells inside a
       Mur x axis, zero-order motion in the plane (plasma_u[2] = 0, B_ext
       along z), a fixed window and the unfused path (single runs only);
       otherwise axf_create fails with EINVAL.  A particle that comes within
       1.5 cells of a Mur face leaves the run (its density becomes 0). */
    int32_t ppc[2];
    double  plasma_n;
    int32_t plasma_lo, plasma_hi;
    double  plasma_u[3];
} axf_config;

/* one diagnostic record at integer time t = step * dt, all FP64, descaled
   (Sec. III.B/C: P_gamma->phi = H_phi / H_gamma(E0,B0), P_phi->gamma = H_gamma(E1,B1) / H_phi) */
typedef struct {
    int64_t step;
    double  t;
    double  h_phi;           /* axion energy: sum over cells of ((D_t phi)^2 + |D+ phi|^2 + m^2 phi^2)/2 dV */
    double  h_em0;           /* zero-order EM energy (laser only, B_ext excluded) */
    double  h_em1;           /* first-order EM energy */
    double  p_gen;           /* h_phi / h_em0 (0 if h_em0 == 0) */
    double  p_conv;          /* h_em1 / h_phi (0 if h_phi == 0) */
    int32_t finite;          /* 0 if any field was not finite */
    int32_t pad;
    double  x_laser;         /* laser centroid (Sec. III.D): sum x B1z^2 / sum B1z^2 over the
                                B1z points, x = i dx on the x nodes (0 if B1z == 0) */
} axf_diag_record;

typedef struct axf_run axf_run;
typedef struct axf_batch axf_batch;
typedef struct axf_server axf_server;

/* thread-local text of the last error of this thread (never NULL) */
const char *axf_last_error(void);
/* library version string */
const char *axf_version(void);

/* ------------------------------------------------------------ single run */

/* Device bytes one run of `cfg` needs: the state of the leapfrog form of
   Sec. II.C (E^{n-1/2} and B^n of both orders, the axion levels), the
   boundary planes (axion ghosts of Sec. II.D, Mur ghosts), the laser table
   and the diagnostic partials and records.  Pure host call, no GPU.
   Errors: EINVAL (bad config), EUNSTABLE (dt beyond the stability limit). */
int axf_footprint(const axf_config *cfg, size_t *bytes);

/* Storage extents nn[3] of the arrays crossing the ABI for `cfg` (the
   staggered layout of Sec. II.C: n + 1 along Mur axes, n otherwise).
   Pure host call.  Errors: EINVAL. */
int axf_extents(const axf_config *cfg, int32_t nn[3]);

/* Create a run: the problem statement of Sec. II.C (grid n, dx and time step
   dt), the axion mass m and coupling g of eq. wave_axion (Sec. II.A), the
   static field B0 = B_ext over the slab (Sec. III.B), the laser source
   (Sec. III.B), the initial axion at two time levels (Sec. III.A) and the
   boundary kinds (Sec. II.D).
   dev_buf: caller-owned device memory of `bytes` >= axf_footprint(cfg),
   256-byte aligned, holding the run until axf_destroy; never freed by the
   library.  stream: the hipStream_t every GPU operation of the run goes to
   (NULL: the default stream).  The analytic initial state (fields zero, the
   packet's two levels at t = -dt/2 and +dt/2, the laser table) is enqueued
   on the stream; the call returns before it runs.  *out receives the run.
   Errors: EINVAL (bad config or null argument), EUNSTABLE (dt), ENOMEM
   (buffer smaller than the footprint), EHIP (a HIP call failed). */
int axf_create(const axf_config *cfg, void *dev_buf, size_t bytes, void *stream, axf_run **out);

/* Overwrite field `field_id` (AXF_E0X .. AXF_PHI_NEW) of the initial state
   before the first step: the initial conditions of Sec. III.A, e.g. both
   axion levels of a packet, or any field of a synthetic test state.
   src: dense FP64 array of the true (unscaled) values with the extents of
   axf_extents, x fastest, src_bytes >= nn[0] nn[1] nn[2] * 8; in host memory
   (src_is_device = 0) or device memory (1), read before the call returns.
   Errors: EINVAL (bad id, size or pointer), ESTATE (the run has stepped), EHIP. */
int axf_write_field(axf_run *run, int32_t field_id, const void *src, size_t src_bytes, int32_t src_is_device);

/* Advance nsteps >= 0 full steps of Sec. II.C (eqs. update_E, update_B and
   update_axion, in the leapfrog form) with the axion boundaries of Sec. II.D
   and the Mur faces, recording the diagnostics every diag_every steps.
   Asynchronous on the run's stream.  Errors: EINVAL (nsteps < 0), EHIP. */
int axf_step(axf_run *run, int64_t nsteps);

/* Read field `field_id` at the current integer time t_n: phi, E1 and B1 (the
   perturbed fields of Sec. II.B, "perturbed laser field" of Sec. III.C) or
   E0 and B0, as dense FP64 true values (descaled), x fastest, the extents of
   axf_extents.  E fields are co-timed at t_n (mean of E^{n-1/2}, E^{n+1/2}),
   B at t_n, phi at t_n - dt/2 (AXF_PHI_OLD) and t_n + dt/2 (AXF_PHI_NEW).
   dst: host (dst_is_device = 0) or device memory of dst_bytes >= nn[0] nn[1]
   nn[2] * 8.  Synchronises the run's stream.  Errors: EINVAL, EHIP. */
int axf_read_field(axf_run *run, int32_t field_id, void *dst, size_t dst_bytes, int32_t dst_is_device);

/* Particle arrays of a run with a plasma (Sec. II.B), as dense FP64 true
   values (descaled) into host memory: id 0-2 position x^n, 3-5 momentum
   u^n = p/(mc), 6-8 the first-order position x1, 9-11 the first-order
   momentum u1, 12 the density each particle carries (0 once absorbed), at
   the current integer time t_n; `max` >= the particle count (*n on return).
   The currents are deposited with atomic additions, so a run is
   reproducible to their rounding order, not bit for bit.  Synchronises the
   run's stream.  Errors: EINVAL (no particles, bad id), ENOMEM (max too
   small), EHIP. */
int axf_read_particles(axf_run *run, int32_t id, double *dst, int64_t max, int64_t *n);

/* The diagnostic record of Sec. III.B/C at the current time t_n: H_phi,
   H_gamma0, H_gamma1 in FP64, P_gamma->phi = H_phi / H_gamma0,
   P_phi->gamma = H_gamma1 / H_phi, and x_laser (Sec. III.D).  *out is host
   memory.  Synchronises the run's stream.  Errors: EINVAL, EHIP. */
int axf_diag_now(axf_run *run, axf_diag_record *out);

/* For callers that cannot allocate device memory at the call (code under HIP
   graph capture, serving loops, harnesses that forbid hipMalloc): the record of
   axf_diag_now, computed by `rows` workgroups (1..1024, 0 = 1024, capped at one
   per 256 grid points) whose FP64 partials and record sit in a static device
   workspace of the library (1024 x 6 doubles + one record, 49.4 KB per device,
   held until the process ends).  Allocates nothing and uses nothing of the
   run's buffer beyond its state.  The sums are folded in another order than
   axf_diag_now's, so the two records agree to FP64 rounding, not bit for bit.
   Every call on one device shares that workspace and the call returns only
   once its record is copied out, so calls made at the same time from several
   host threads on one device race.  rows outside 0..1024 -> AXF_EINVAL. */
int axf_diag_now_static(axf_run *run, int32_t rows, axf_diag_record *out);

/* Copy up to `max` of the records taken every diag_every steps (the
   probabilities of Sec. III.B/C over time, oldest first) into host memory
   `out` and clear them; *n = the number copied.  The run keeps the last 4096.
   Synchronises the run's stream.  Errors: EINVAL, EHIP. */
int axf_read_diag(axf_run *run, axf_diag_record *out, int32_t max, int32_t *n);

/* Checkpoint and resume (a project facility; no passage of the paper): the
   raw state (fields, ghosts, the laser table, step counter) into or from a
   host buffer of axf_state_bytes bytes.  A state written back into a run of
   the same configuration continues bit for bit as the run it was read from.
   Both synchronise the stream and copy before they return; write also has
   the next step refill the laser table.  Errors: ENOMEM (buffer smaller than
   axf_state_bytes), EINVAL (a state of another configuration), EHIP. */
int axf_state_bytes(const axf_run *run, size_t *bytes);
int axf_read_state(axf_run *run, void *buf, size_t bytes);
int axf_write_state(axf_run *run, const void *buf, size_t bytes);

/* Wait for the run's stream.  Errors: EINVAL, EHIP. */
int axf_sync(axf_run *run);
/* Steps taken so far (host counter, no synchronisation). */
int axf_steps_done(const axf_run *run, int64_t *steps);
/* the step path this run takes: AXF_PATH_PLAIN or AXF_PATH_FUSED (AUTO resolved) */
int axf_path_in_use(const axf_run *run, int32_t *path);
/* release library-side handles (not the caller's device memory) */
int axf_destroy(axf_run *run);

/* Per-launch GPU time of the last `axf_step` call measured with HIP events on
   the run's stream: total ms over the steps and the number of step launches. */
int axf_last_step_timing(const axf_run *run, double *ms, int64_t *launches);

/* ------------------------------------------------------------ tuning
 * Launch shape of the fused 2D step, chosen by timing every candidate on a
 * scratch run: one step per pass (rows per wavefront march, prefetch
 * distance) or passes of two, three or four steps (temporal blocking: steps per
 * pass, rows per interior wavefront, rows per frame wavefront, prefetch
 * distance).  The best shape of each kind is kept in a process-wide table
 * keyed by dimensionality, precision, boundary kinds, PML width and the
 * power-of-two size class of the grid, with the faster kind; runs created
 * afterwards with a matching key use it (batches use the one-step shape, and
 * two-step passes with the multi-step rows).  The built-in shape is timed
 * first and again after the candidates (the faster of the two counts) and
 * stays unless a candidate beats it by more than 2%.  Configurations without a fused 2D
 * path report AXF_PATH_PLAIN and keep their launches.
 */
typedef struct {
    int32_t path;                /* AXF_PATH_FUSED or AXF_PATH_PLAIN */
    int32_t chunk;               /* rows per wavefront march (fused 2D; the
                                    interior of a pass of several steps) */
    int32_t prefetch;            /* rows prefetched ahead (fused 2D) */
    int32_t candidates;          /* shapes timed */
    int32_t steps_per_pass;      /* most steps per pass (2, 3 or 4), or 1 */
    int32_t frame_chunk;         /* rows per frame wavefront of a pass of several steps (0 if 1) */
    double  ms_per_step;         /* best */
    double  default_ms_per_step; /* the built-in default shape (faster of its two timings) */
} axf_tuning;

/* Time the candidates for `steps` steps each on a run carved from `scratch`
   (caller device memory of >= axf_footprint bytes; its contents are
   overwritten), record the best.  Synchronises `stream`. */
int axf_tune(const axf_config *cfg, void *scratch, size_t bytes, void *stream, int32_t steps, axf_tuning *out);
/* Forget every recorded choice (pure host call). */
int axf_tune_reset(void);

/* ------------------------------------------------------------ SI inputs
 * The paper's SI form of the equations (Sec. II.A: the axion field in units of
 * frequency, g_agg in units of time, as an SI particle-in-cell code takes them)
 * mapped to the normalised units of axf_config: times in 1/omega0, lengths in
 * 1/k0 (omega0 = k0 c = 2 pi c / lambda0 of a reference wavelength), fields in
 * m_e c omega0 / e (E) and m_e omega0 / e (B), masses as m_a c^2 / (hbar omega0).
 * The single coupling g of axf_config drives both the axion source and the
 * axion current; it is g = g_agg m_e c^(3/2) / (e sqrt(hbar mu0)) with the
 * axion field measured in omega0 s, s = m_e c^(3/2) / (e omega0 sqrt(hbar mu0)),
 * the scale at which the two SI couplings (g / (hbar mu0) and g / c) coincide.
 * Constants: CODATA 2018.
 */
typedef struct {
    double lambda0;          /* reference wavelength [m] (> 0) */
    double lambda_laser;     /* laser wavelength [m]; 0: lambda0 */
    double dx[3];            /* cell sizes [m] (> 0 on the run's axes) */
    double dt;               /* time step [s] (> 0) */
    double m_a;              /* axion mass m_a c^2 [eV] (>= 0) */
    double g_agg;            /* axion-photon coupling [hbar GeV^-1] */
    double bext[3];          /* static external field [T] */
    double e_amp;            /* laser peak field [V/m] */
    double fwhm;             /* laser intensity FWHM duration [s] */
    double t_center;         /* time the pulse peak crosses x = 0 [s] */
    double waist;            /* 1/e field radius at focus [m]; 0: plane wave */
    double x_focus, y_c, z_c;/* focus and transverse centre [m] */
} axf_si;

/* Fill dx (on the run's ndim axes), dt, m, g, bext, omega, e_amp, fwhm,
   t_center, waist, x_focus, y_c and z_c of *cfg from *si (every other field
   of *cfg is left as it is; set ndim first).  Pure host
   call; EINVAL for a non-positive wavelength, cell size or time step, or a
   negative mass. */
int axf_config_from_si(const axf_si *si, axf_config *cfg);

/* The axion-photon coupling of an axion model (Sec. III.B): f_a from
   m_a = 6.3 eV x 10^6 GeV / f_a, then g_agg = c_gamma 2 alpha / (pi f_a), in
   hbar GeV^-1 (c_gamma = -0.97 for KSVZ, 0.36 for DFSZ).  Pure host call;
   EINVAL for m_a <= 0 or a null output. */
int axf_axion_coupling(double m_a_eV, double c_gamma, double *g_agg);

/* ------------------------------------------------------------ batches
 * Many independent runs (parameter scans over m, g, B0, omega and grid size)
 * carved from one caller device buffer.  Runs are grouped by dimensionality,
 * precision and step path; one batched launch per kernel kind and group
 * advances every active run of the group by one step, or by a pass of two or
 * four steps (2D wavefront runs whose grid has an interior for it, where no
 * diagnostic record falls inside the pass), each run with its own step
 * counter.  Every run's result is bit-identical to the same run created with
 * axf_create and stepped alone.
 */

/* Device bytes of a batch: a launch table plus each run's footprint, each
   256-byte aligned.  Pure host call; EINVAL names the first bad configuration. */
int axf_batch_footprint(const axf_config *cfgs, int32_t count, size_t *bytes);
/* Create `count` runs in `dev_buf` (256-byte aligned, >= the batch footprint),
   all on `stream`.  Errors as axf_create, for the first run that fails. */
int axf_batch_create(const axf_config *cfgs, int32_t count, void *dev_buf, size_t bytes,
                     void *stream, axf_batch **out);
/* Advance run i by nsteps[i] >= 0 steps (array of `count`); runs with fewer
   steps drop out of the launches when done.  Asynchronous on the stream. */
int axf_batch_step(axf_batch *b, const int64_t *nsteps);
/* Borrowed view of run i for the single-run read, diagnostic and state
   calls; axf_step and axf_destroy on a view fail with AXF_ESTATE. */
int axf_batch_run(axf_batch *b, int32_t i, axf_run **view);
/* Synchronise the stream and release the batch (not the caller's memory). */
int axf_batch_destroy(axf_batch *b);

/* ------------------------------------------------------------ server
 * Continuous batching of conversion requests on one GPU.  A host thread
 * drives the GPU: each round it admits queued requests that fit (a free slot
 * and a first-fit range of the pool; a request passed over for more than a
 * few rounds blocks later ones from overtaking it), creates them in the pool,
 * and advances every resident run by a work slice of about
 * macro_steps x 2^20 cell-updates (at least one step, at most what remains)
 * through the batched launches (passes of at most two steps: four were slower
 * for its changing mix of runs).  Finished or cancelled runs are retired and
 * their memory returns to the pool.  A result's final record is bit-identical
 * to the same run stepped alone.
 */

/* Result of one served request.  Times are seconds on the server's clock. */
typedef struct {
    uint64_t id;
    int32_t  status;         /* 0 ok, AXF_E* on failure, 1 cancelled */
    int32_t  pad;
    int64_t  steps;          /* steps taken */
    int64_t  cells;          /* n[0] n[1] n[2] */
    double   t_submit, t_admit, t_done;
    axf_diag_record final;   /* record at the last step (status 0 only) */
} axf_result;

/* `pool` is caller device memory (256-byte aligned) of `pool_bytes`; the
   server keeps a small launch table at its start and carves resident runs
   from the rest.  At most `max_slots` runs are resident.  The server's thread
   enqueues all GPU work on `stream`. */
int axf_server_create(void *pool, size_t pool_bytes, int32_t max_slots, int32_t macro_steps,
                      void *stream, axf_server **out);
/* Queue a request of `nsteps` steps; *id identifies its result.  ENOMEM if
   the run can never fit the pool, EINVAL/EUNSTABLE for a bad configuration. */
int axf_server_submit(axf_server *s, const axf_config *cfg, int64_t nsteps, uint64_t *id);
/* Cancel a queued or resident request; its result has status 1.  ENOTFOUND
   if the request is neither queued nor resident. */
int axf_server_cancel(axf_server *s, uint64_t id);
/* Move up to `max` completed results (oldest first) to `out`; *n = count.
   Never blocks. */
int axf_server_poll(axf_server *s, axf_result *out, int32_t max, int32_t *n);
/* Queue depth, resident runs and pool bytes in use (any argument may be NULL). */
int axf_server_stats(axf_server *s, int32_t *queued, int32_t *resident, size_t *bytes_used);
/* Stop after the current round (resident runs end as cancelled, queued ones
   are dropped), join the thread, release the server. */
int axf_server_destroy(axf_server *s);

#ifdef __cplusplus
}
#endif
#endif
