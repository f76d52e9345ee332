/*
 * axion_oracle.h -- plain FP64 CPU reference of the axion-coupled Yee step.
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the GPU library.
 * Only the test suite, the package smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or helper
 * with the GPU path.
 *
 * Physics (natural units, c = 1), from An et al., "Modeling of axion and
 * electromagnetic fields coupling in a particle-in-cell code":
 *   - Klein-Gordon axion with source g E0.B0            (Sec. II.A, eq. wave_axion)
 *   - first-order fields E1/B1 driven by
 *     g[(dphi/dt) B0 - E0 x grad phi]                   (Sec. II.B, eq. curl-b1)
 *   - zero-order fields E0/B0: vacuum Maxwell (laser); a static external
 *     field B_ext is added to B0 wherever B0 enters a source term.
 *   - time stepping: the half-step sequence of Sec. II.C (eq. update_E,
 *     the B half-steps, eq. update_axion, then B and E again), with the
 *     axion at half-integer times and phi^n the average of its neighbours.
 *   - spatial layout: phi at cell centres, E on cell faces, B on cell edges
 *     (Sec. II.C, the averaging formulas for E0.B0 and E0 x grad phi).
 *   - axion boundaries: periodic, reflect, outflow, PML (Sec. II.D).
 *   - EM boundaries (not in the paper): periodic, or first-order Mur on the
 *     tangential E at ghost centres half a cell outside the boundary node
 *     plane, with a laser injected through the x_min face.
 *
 * Parity status per function is listed in the header comment of
 * axion_oracle.c.
 */
#ifndef AXION_ORACLE_H
#define AXION_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* boundary kinds */
enum { ORA_EM_PERIODIC = 0, ORA_EM_MUR = 1 };
enum { ORA_AX_PERIODIC = 0, ORA_AX_REFLECT = 1, ORA_AX_OUTFLOW = 2, ORA_AX_PML = 3 };
enum { ORA_ENV_CW = 0, ORA_ENV_GAUSS = 1 };

typedef struct {
    int    n[3];          /* cells per axis; an axis with n = 1 is degenerate (must be periodic) */
    double dx[3];         /* cell size per axis */
    double dt;            /* time step */
    int    em_bc[3];      /* ORA_EM_* per axis (both faces) */
    int    ax_bc[3];      /* ORA_AX_* per axis (both faces) */
    int    pml_n;         /* PML layer thickness in cells */
    double pml_sigma_dt;  /* sigma_max * dt */
    double m;             /* axion mass */
    double g;             /* coupling g_a-gamma-gamma */
    double bext[3];       /* static external B field vector */
    int    slab_lo, slab_hi; /* B_ext present in cells slab_lo <= i < slab_hi along x */
    /* laser injected through the x_min face, propagating along +x */
    int    laser_on;
    int    laser_pol;     /* 1: E along y, 2: E along z */
    int    laser_env;     /* ORA_ENV_* */
    double omega;         /* laser angular frequency */
    double e_amp;         /* peak electric field amplitude */
    double ramp_periods;  /* CW: sin^2 ramp length in laser periods */
    double fwhm;          /* Gaussian: intensity FWHM duration */
    double t_center;      /* Gaussian: time at which the peak crosses x = 0 */
    double waist;         /* 1/e field radius at focus (0: plane wave) */
    double x_focus;       /* focal plane position */
    double y_c, z_c;      /* beam axis */
    double cep;           /* carrier-envelope phase */
    /* axion packet phi = A exp(-(eta^2 + r_perp^2)/w^2) sin(k eta), eta = x - x0 - dir t */
    int    packet_on;
    double pk_amp, pk_k, pk_w, pk_x0, pk_y0, pk_z0;
    int    pk_dir;        /* +1 moves to +x, -1 moves to -x */
    /* which order carries the injected laser: 0 (E0/B0) or 1 (E1/B1, the weak
       laser of Sec. III.D riding on a strong background) */
    int    laser_order;
    /* cold plasma electrons (charge -1, mass 1; immobile neutralising ions),
       Sec. II.B: ppc[0] x ppc[1] particles per cell on a regular lattice in the
       cells plasma_lo <= i < plasma_hi along x and every cell along y; density
       plasma_n in critical densities (omega_p^2 = plasma_n), momentum u = p/(mc)
       plasma_u at t = 0.  ppc[0] = 0: no particles. */
    int    ppc[2];
    double plasma_n;
    int    plasma_lo, plasma_hi;
    double plasma_u[3];
} ora_config;

typedef struct ora_state ora_state;

/* field ids for ora_field */
enum {
    ORA_E0X = 0, ORA_E0Y, ORA_E0Z, ORA_B0X, ORA_B0Y, ORA_B0Z,
    ORA_E1X, ORA_E1Y, ORA_E1Z, ORA_B1X, ORA_B1Y, ORA_B1Z,
    ORA_PHI_OLD,  /* phi at t_n - dt/2 */
    ORA_PHI_NEW   /* phi at t_n + dt/2 */
};

/* returns 0 on success, -1 on an invalid configuration */
int    ora_create(const ora_config *cfg, ora_state **out);
void   ora_destroy(ora_state *s);
/* storage extents (nodal extents: n + 1 on Mur axes, n on periodic axes) */
void   ora_extents(const ora_state *s, int nn[3]);
/* pointer to the internal array of a field, laid out x fastest over nn[] */
double *ora_field(ora_state *s, int id);
/* axion ghost plane of axis d, side (0 lo, 1 hi), level (0: t_n - dt/2, 1: t_n + dt/2);
   laid out over the two other axes (first other axis fastest), sized by nn[] */
double *ora_axion_ghost(ora_state *s, int d, int side, int level);
/* after editing the initial arrays in place: recompute derived boundary history */
void   ora_refresh_initial(ora_state *s);
void   ora_step(ora_state *s, long nsteps);
int    ora_shift_window(ora_state *s, int cells);
long   ora_step_count(const ora_state *s);
/* particles: count, and their arrays (id 0-2 position x^n, 3-5 momentum u^n,
   6-8 first-order position, 9-11 first-order momentum, 12 weight (density
   carried; 0 once absorbed)); current at the E points of order o, component c
   (j at t_n, the value the next E half step uses), laid out as the fields */
long   ora_particles(const ora_state *s);
double *ora_particle_array(ora_state *s, int id);
double *ora_current(ora_state *s, int o, int c);
/* recompute j at t_n from the particle arrays as they are (after editing them) */
void   ora_redeposit(ora_state *s);
/* energies at the current integer time: out[0] = H_phi, out[1] = H_gamma(E0,B0), out[2] = H_gamma(E1,B1) */
void   ora_energies(const ora_state *s, double out[3]);
/* incident laser E component comp (1 = y, 2 = z) at (x, y, z, t); exposed for tests */
/* OpenMP threads the step loops use (1 without OpenMP) */
int    ora_threads(void);
void   ora_set_threads(int n);

double ora_incident(const ora_state *s, int comp, double x, double y, double z, double t);

#ifdef __cplusplus
}
#endif
#endif
