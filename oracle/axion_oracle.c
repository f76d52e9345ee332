/*
 * axion_oracle.c -- plain FP64 CPU reference of the axion-coupled Yee step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the package smoke
 * check and the CPU-baseline leg of the benchmark, never by the library.
 *
 * It follows An et al. (arXiv 2406.16796) literally, in natural units:
 *   - the half-step sequence of Sec. II.C: E1 and E0 half step with the
 *     axion current at t_n (eq. update_E), B half step, axion leapfrog to
 *     t_{n+3/2} (eq. update_axion), B half step, E0 and E1 half step with
 *     the axion current at t_{n+1};
 *   - phi^n as the average of the two neighbouring axion levels (Sec. II.C);
 *   - E0.B0 at cell centres from 2-point E and 4-point B averages, and the
 *     E0 x grad(phi) and (D_t phi) B0 terms formed at the two centres next to
 *     an E face and averaged onto it (Sec. II.C, the averaging formulas);
 *   - the axion boundaries of Sec. II.D: periodic, reflect (zero gradient),
 *     outflow (one-way wave equation plus Klein-Gordon at the ghost) and the
 *     PML damping layer obtained from d/dt -> d/dt + sigma, with the profile
 *     sigma = (1 - i/N)^3 sigma_max of Sec. III.A.
 *   - EM boundaries are not in the paper: periodic, or first-order Mur
 *     (G. Mur, IEEE Trans. EMC 23, 1981) on the tangential E at a ghost
 *     centre half a cell outside the boundary node plane, applied to the
 *     scattered part E - E_inc, with the laser as E_inc on the x_min face.
 *
 * Storage: every array has extents nn[d] (= n[d] + 1 on Mur axes, n[d] on
 * periodic axes), x fastest.  E_c is nodal along axis c and centred along
 * the others; B_c is centred along c and nodal along the others; phi is
 * centred everywhere.  Entries a component does not use stay zero.
 *
 * Pins (tests/test_oracle_*.py): Yee and Klein-Gordon discrete dispersion
 * relations (exact normal modes), the discrete EM and KG energy invariants,
 * div B, Gauss's law with the axion charge (kept exactly with E0 = 0, and
 * converging at second order with a laser wave on, which pins E0 x grad phi;
 * copies of this file with a planted sign or component slip fail it),
 * bit-exact linearity in g, exact-rational brute force of the half-step and
 * leapfrog forms, reflect boundary by the method of images, periodic
 * translation invariance, outflow/PML reflectivity against the 1% of
 * Sec. III.A, the conversion probability of Sec. III.B, the Mur faces
 * (plane-wave transmission of the injected laser; a normal pulse leaving
 * through x_max and y_max), and the first-order effect of the literal
 * reading of the time derivative (ORA_DTPHI_LITERAL).  Particles (Sec.
 * II.B): Boris gyration in closed form, the k = 0 Langmuir recurrence, and
 * the first-order particles and fields against a central difference of two
 * zero-order runs (copies with a planted slip fail it).  The Gaussian
 * envelope and focused profile of the injected laser have no formula in the
 * paper and no pin (parity unpinned).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include "axion_oracle.h"
#ifdef _OPENMP
#include <omp.h>
#endif

int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the following loops (timing only: every sum has a fixed order,
   so the results do not depend on the count) */
void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

struct ora_state {
    ora_config c;
    int    n[3], nn[3];
    long   ncell;
    double *E[2][3], *B[2][3];     /* order 0/1, component x/y/z, co-timed at t_n */
    double *phi[3];                /* rotating axion levels */
    int    la, lb;                 /* slots holding t_n - dt/2 and t_n + dt/2 */
    double *axg[3][2][3];          /* axion ghosts: axis, side, slot */
    double *mur_g[2][3][2][3];     /* Mur ghost E: order, axis, side, component */
    double *mur_a[2][3][2][3];     /* E at the interior centre next to that ghost, t_n - dt/2 */
    double *C[3];                  /* scratch: (D_t phi) B0 - E0 x grad phi at centres */
    double *Sax;                   /* scratch: g E0.B0 at centres */
    double *Eh[2][3];              /* E at t_n - dt/2 on the first ORA_WIN_KEEP x columns (window moves) */
    long   step;
    /* particles (Sec. II.B): zero-order position x^n and momentum u^n = p/(mc),
       first-order ones, density carried (0: absorbed); current at t_n on the E
       points of both orders */
    long   np;
    double *px[3], *pu[3], *px1[3], *pu1[3], *pw;
    double *J[2][3];
};

/* columns of E^{n-1/2} kept for a move of the window (the most one move shifts) */
#define ORA_WIN_KEEP 64

/* ---------------------------------------------------------------- helpers */

static void other_axes(int d, int *a, int *b)
{
    *a = (d == 0) ? 1 : 0;
    *b = (d == 2) ? 1 : 2;
}

static long IX(const ora_state *s, int i, int j, int k)
{
    return ((long)k * s->nn[1] + j) * s->nn[0] + i;
}

static int em_periodic(const ora_state *s, int d) { return s->c.em_bc[d] == ORA_EM_PERIODIC; }
static int ax_periodic(const ora_state *s, int d) { return s->c.ax_bc[d] == ORA_AX_PERIODIC; }

/* periodic index; stencil offsets never reach more than one period away */
static int wrapn(int i, int n)
{
    if (i < 0) i += n;
    if (i >= n) i -= n;
    return i;
}

/* number of points of a component along axis d: nodal or centred */
static int extent(const ora_state *s, int d, int nodal)
{
    return (nodal && !em_periodic(s, d)) ? s->n[d] + 1 : s->n[d];
}

static void die(const char *what)
{
    fprintf(stderr, "axion oracle: index out of range in %s\n", what);
    abort();
}

/* E_c of order o at index (i,j,k).  Indices outside the domain along an
   axis where E_c is centred and the EM boundary is Mur give the Mur ghost. */
static double E_at(const ora_state *s, int o, int c, int i, int j, int k)
{
    int id[3] = {i, j, k};
    for (int d = 0; d < 3; d++)
        if (em_periodic(s, d)) id[d] = wrapn(id[d], s->n[d]);
    for (int d = 0; d < 3; d++) {
        if (em_periodic(s, d) || d == c) continue;
        if (id[d] < 0 || id[d] >= s->n[d]) {
            if (id[d] < -1 || id[d] > s->n[d]) die("E ghost");
            int side = id[d] < 0 ? 0 : 1, a, b;
            other_axes(d, &a, &b);
            return s->mur_g[o][d][side][c][(long)id[b] * s->nn[a] + id[a]];
        }
    }
    if (id[c] < 0 || id[c] >= s->nn[c]) die("E nodal");
    return s->E[o][c][IX(s, id[0], id[1], id[2])];
}

static double B_at(const ora_state *s, int o, int c, int i, int j, int k)
{
    int id[3] = {i, j, k};
    for (int d = 0; d < 3; d++) {
        if (em_periodic(s, d)) id[d] = wrapn(id[d], s->n[d]);
        else if (id[d] < 0 || id[d] >= extent(s, d, d != c)) die("B");
    }
    return s->B[o][c][IX(s, id[0], id[1], id[2])];
}

/* phi at slot L, with the axion ghost values outside non-periodic faces */
static double phi_at(const ora_state *s, int L, int i, int j, int k)
{
    int id[3] = {i, j, k};
    for (int d = 0; d < 3; d++)
        if (ax_periodic(s, d)) id[d] = wrapn(id[d], s->n[d]);
    for (int d = 0; d < 3; d++) {
        if (ax_periodic(s, d)) continue;
        if (id[d] < 0 || id[d] >= s->n[d]) {
            if (id[d] < -1 || id[d] > s->n[d]) die("phi ghost");
            int side = id[d] < 0 ? 0 : 1, a, b;
            other_axes(d, &a, &b);
            return s->axg[d][side][L][(long)id[b] * s->nn[a] + id[a]];
        }
    }
    return s->phi[L][IX(s, id[0], id[1], id[2])];
}

static double bext_at(const ora_state *s, int comp, int i)
{
    return (i >= s->c.slab_lo && i < s->c.slab_hi) ? s->c.bext[comp] : 0.0;
}

/* ------------------------------------------------------ analytic inputs */

double ora_incident(const ora_state *s, int comp, double x, double y, double z, double t)
{
    const ora_config *c = &s->c;
    if (!c->laser_on || comp != c->laser_pol) return 0.0;
    double tau = t - x, env;
    if (c->laser_env == ORA_ENV_CW) {
        double tr = c->ramp_periods * 2.0 * M_PI / c->omega;
        if (tau <= 0.0) env = 0.0;
        else if (tau < tr) { double r = sin(0.5 * M_PI * tau / tr); env = r * r; }
        else env = 1.0;
    } else {
        double tau0 = c->fwhm / sqrt(2.0 * log(2.0));
        double u = (tau - c->t_center) / tau0;
        env = exp(-u * u);
    }
    double amp = 1.0, dphase = 0.0;
    int q = (s->n[1] > 1) + (s->n[2] > 1);
    if (q > 0 && c->waist > 0.0) {
        double r2 = 0.0;
        if (s->n[1] > 1) r2 += (y - c->y_c) * (y - c->y_c);
        if (s->n[2] > 1) r2 += (z - c->z_c) * (z - c->z_c);
        double zr = 0.5 * c->omega * c->waist * c->waist;
        double xi = x - c->x_focus;
        double w2 = c->waist * c->waist * (1.0 + (xi / zr) * (xi / zr));
        double inv_r = xi / (xi * xi + zr * zr);
        amp = pow(c->waist * c->waist / w2, 0.25 * q) * exp(-r2 / w2);
        dphase = -0.5 * c->omega * r2 * inv_r + 0.5 * q * atan(xi / zr);
    }
    return c->e_amp * amp * env * sin(c->omega * tau + dphase + c->cep);
}

static double packet(const ora_state *s, double x, double y, double z, double t)
{
    const ora_config *c = &s->c;
    if (!c->packet_on) return 0.0;
    double eta = x - c->pk_x0 - c->pk_dir * t, r2 = 0.0;
    if (s->n[1] > 1) r2 += (y - c->pk_y0) * (y - c->pk_y0);
    if (s->n[2] > 1) r2 += (z - c->pk_z0) * (z - c->pk_z0);
    return c->pk_amp * exp(-(eta * eta + r2) / (c->pk_w * c->pk_w)) * sin(c->pk_k * eta);
}

/* coordinate of index idx along axis d, nodal or centred */
static double coord(const ora_state *s, int d, int idx, int nodal)
{
    return nodal ? idx * s->c.dx[d] : (idx + 0.5) * s->c.dx[d];
}

/* ----------------------------------------------------------- stencils */

/* (curl B)_c at the E_c point (i,j,k): forward differences */
static double curl_B(const ora_state *s, int o, int c, int i, int j, int k)
{
    const double *h = s->c.dx;
    switch (c) {
    case 0:
        return (B_at(s, o, 2, i, j + 1, k) - B_at(s, o, 2, i, j, k)) / h[1]
             - (B_at(s, o, 1, i, j, k + 1) - B_at(s, o, 1, i, j, k)) / h[2];
    case 1:
        return (B_at(s, o, 0, i, j, k + 1) - B_at(s, o, 0, i, j, k)) / h[2]
             - (B_at(s, o, 2, i + 1, j, k) - B_at(s, o, 2, i, j, k)) / h[0];
    default:
        return (B_at(s, o, 1, i + 1, j, k) - B_at(s, o, 1, i, j, k)) / h[0]
             - (B_at(s, o, 0, i, j + 1, k) - B_at(s, o, 0, i, j, k)) / h[1];
    }
}

/* (curl E)_c at the B_c point (i,j,k): backward differences */
static double curl_E(const ora_state *s, int o, int c, int i, int j, int k)
{
    const double *h = s->c.dx;
    switch (c) {
    case 0:
        return (E_at(s, o, 2, i, j, k) - E_at(s, o, 2, i, j - 1, k)) / h[1]
             - (E_at(s, o, 1, i, j, k) - E_at(s, o, 1, i, j, k - 1)) / h[2];
    case 1:
        return (E_at(s, o, 0, i, j, k) - E_at(s, o, 0, i, j, k - 1)) / h[2]
             - (E_at(s, o, 2, i, j, k) - E_at(s, o, 2, i - 1, j, k)) / h[0];
    default:
        return (E_at(s, o, 1, i, j, k) - E_at(s, o, 1, i - 1, j, k)) / h[0]
             - (E_at(s, o, 0, i, j, k) - E_at(s, o, 0, i, j - 1, k)) / h[1];
    }
}

/* zero-order E averaged to the cell centre (i,j,k): 2 points along the component */
static void centre_E0(const ora_state *s, int i, int j, int k, double e[3])
{
    e[0] = 0.5 * (E_at(s, 0, 0, i + 1, j, k) + E_at(s, 0, 0, i, j, k));
    e[1] = 0.5 * (E_at(s, 0, 1, i, j + 1, k) + E_at(s, 0, 1, i, j, k));
    e[2] = 0.5 * (E_at(s, 0, 2, i, j, k + 1) + E_at(s, 0, 2, i, j, k));
}

/* zero-order B (laser plus external) at the cell centre: 4 points across the component */
static void centre_B0(const ora_state *s, int i, int j, int k, double b[3])
{
    b[0] = 0.25 * (B_at(s, 0, 0, i, j + 1, k + 1) + B_at(s, 0, 0, i, j + 1, k)
                 + B_at(s, 0, 0, i, j, k + 1) + B_at(s, 0, 0, i, j, k)) + bext_at(s, 0, i);
    b[1] = 0.25 * (B_at(s, 0, 1, i + 1, j, k + 1) + B_at(s, 0, 1, i + 1, j, k)
                 + B_at(s, 0, 1, i, j, k + 1) + B_at(s, 0, 1, i, j, k)) + bext_at(s, 1, i);
    b[2] = 0.25 * (B_at(s, 0, 2, i + 1, j + 1, k) + B_at(s, 0, 2, i + 1, j, k)
                 + B_at(s, 0, 2, i, j + 1, k) + B_at(s, 0, 2, i, j, k)) + bext_at(s, 2, i);
}

/* phi at the integer time between slots La and Lb (average of the two levels) */
static double phi_mid(const ora_state *s, int La, int Lb, int i, int j, int k)
{
    return 0.5 * (phi_at(s, Lb, i, j, k) + phi_at(s, La, i, j, k));
}

/* Reading of the time derivative in the second E1 half step (Sec. II.C,
   eq. update_E at t_{n+1}): the paper writes it at n + 1/2 beside fields at
   n + 1.  The default takes (D_t phi)^{n+1} = (phi^{n+3/2} - phi^{n+1/2}) / dt,
   which makes the two half steps one leapfrog step; ORA_DTPHI_LITERAL = 1 (a
   separate test build only) takes the literal centred derivative at n + 1/2,
   (phi^{n+3/2} - phi^{n-1/2}) / (2 dt). */
#ifndef ORA_DTPHI_LITERAL
#define ORA_DTPHI_LITERAL 0
#endif

/* C = (D_t phi) B0 - E0 x D phi at every centre, for the integer time between
   axion slots La (earlier) and Lb (later), with the E0, B0 arrays as they are;
   Lo: the slot before La (the literal reading's level), -1 for none */
static void compute_C(ora_state *s, int La, int Lb, int Lo)
{
    const double dt = s->c.dt, *h = s->c.dx;
    const int literal = ORA_DTPHI_LITERAL && Lo >= 0;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < s->n[2]; k++)
        for (int j = 0; j < s->n[1]; j++)
            for (int i = 0; i < s->n[0]; i++) {
                double e[3], b[3], gp[3];
                centre_E0(s, i, j, k, e);
                centre_B0(s, i, j, k, b);
                double dtphi = literal ? (phi_at(s, Lb, i, j, k) - phi_at(s, Lo, i, j, k)) / (2.0 * dt)
                                       : (phi_at(s, Lb, i, j, k) - phi_at(s, La, i, j, k)) / dt;
                gp[0] = (phi_mid(s, La, Lb, i + 1, j, k) - phi_mid(s, La, Lb, i - 1, j, k)) / (2.0 * h[0]);
                gp[1] = (phi_mid(s, La, Lb, i, j + 1, k) - phi_mid(s, La, Lb, i, j - 1, k)) / (2.0 * h[1]);
                gp[2] = (phi_mid(s, La, Lb, i, j, k + 1) - phi_mid(s, La, Lb, i, j, k - 1)) / (2.0 * h[2]);
                long id = IX(s, i, j, k);
                s->C[0][id] = dtphi * b[0] - (e[1] * gp[2] - e[2] * gp[1]);
                s->C[1][id] = dtphi * b[1] - (e[2] * gp[0] - e[0] * gp[2]);
                s->C[2][id] = dtphi * b[2] - (e[0] * gp[1] - e[1] * gp[0]);
            }
}

/* axion current term at the E_c face (i,j,k): mean of C_c at the two centres
   on either side; on a Mur face the one interior centre is used */
static double face_S(const ora_state *s, int c, int i, int j, int k)
{
    int lo[3] = {i, j, k}, hi[3] = {i, j, k};
    lo[c] -= 1;
    if (em_periodic(s, c)) {
        lo[c] = wrapn(lo[c], s->n[c]);
        hi[c] = wrapn(hi[c], s->n[c]);
    } else {
        if (lo[c] < 0) lo[c] = 0;
        if (hi[c] > s->n[c] - 1) hi[c] = s->n[c] - 1;
    }
    return 0.5 * (s->C[c][IX(s, lo[0], lo[1], lo[2])] + s->C[c][IX(s, hi[0], hi[1], hi[2])]);
}

/* E_o += h (curl B_o - j_o - g S) over every E point; g S only for order 1,
   j only with particles (the current at the time of the half step) */
static void update_E(ora_state *s, int o, double h, double g)
{
    for (int c = 0; c < 3; c++) {
        int e0 = extent(s, 0, c == 0), e1 = extent(s, 1, c == 1), e2 = extent(s, 2, c == 2);
        double *E = s->E[o][c];
        const double *J = s->J[o][c];
        #pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < e2; k++)
            for (int j = 0; j < e1; j++)
                for (int i = 0; i < e0; i++) {
                    double rhs = curl_B(s, o, c, i, j, k);
                    if (J) rhs = rhs - J[IX(s, i, j, k)];
                    if (o == 1) rhs = rhs - g * face_S(s, c, i, j, k);
                    E[IX(s, i, j, k)] += h * rhs;
                }
    }
}

/* B_o -= h curl E_o over every B point, both orders */
static void update_B(ora_state *s, double h)
{
    for (int o = 0; o < 2; o++)
        for (int c = 0; c < 3; c++) {
            int e0 = extent(s, 0, c != 0), e1 = extent(s, 1, c != 1), e2 = extent(s, 2, c != 2);
            double *B = s->B[o][c];
            #pragma omp parallel for collapse(2) schedule(static)
            for (int k = 0; k < e2; k++)
                for (int j = 0; j < e1; j++)
                    for (int i = 0; i < e0; i++)
                        B[IX(s, i, j, k)] -= h * curl_E(s, o, c, i, j, k);
        }
}

/* Mur ghosts at t_{n+1/2}, from the interior E just advanced to t_{n+1/2} */
static void mur_ghosts(ora_state *s)
{
    const double dt = s->c.dt;
    const double t_new = (s->step + 0.5) * dt, t_old = (s->step - 0.5) * dt;
    for (int d = 0; d < 3; d++) {
        if (em_periodic(s, d)) continue;
        double cm = (dt - s->c.dx[d]) / (dt + s->c.dx[d]);
        int a, b;
        other_axes(d, &a, &b);
        for (int side = 0; side < 2; side++) {
            int iadj = side ? s->n[d] - 1 : 0, igh = side ? s->n[d] : -1;
            int comps[2] = {a, b};
            for (int q = 0; q < 2; q++) {
                int c = comps[q];
                int ea = extent(s, a, c == a), eb = extent(s, b, c == b);
                for (int ib = 0; ib < eb; ib++)
                    for (int ia = 0; ia < ea; ia++) {
                        int id[3];
                        id[d] = iadj; id[a] = ia; id[b] = ib;
                        long f = (long)ib * s->nn[a] + ia;
                        double pa[3], pg[3];
                        for (int e = 0; e < 3; e++) {
                            pa[e] = coord(s, e, id[e], e == c);
                            pg[e] = pa[e];
                        }
                        pg[d] = coord(s, d, igh, 0);
                        for (int o = 0; o < 2; o++) {
                            int inj = (o == s->c.laser_order && d == 0 && side == 0);
                            double ia_new = inj ? ora_incident(s, c, pa[0], pa[1], pa[2], t_new) : 0.0;
                            double ia_old = inj ? ora_incident(s, c, pa[0], pa[1], pa[2], t_old) : 0.0;
                            double ig_new = inj ? ora_incident(s, c, pg[0], pg[1], pg[2], t_new) : 0.0;
                            double ig_old = inj ? ora_incident(s, c, pg[0], pg[1], pg[2], t_old) : 0.0;
                            double eadj = s->E[o][c][IX(s, id[0], id[1], id[2])];
                            double sc_adj_new = eadj - ia_new;
                            double sc_adj_old = s->mur_a[o][d][side][c][f] - ia_old;
                            double sc_gh_old = s->mur_g[o][d][side][c][f] - ig_old;
                            double sc_gh_new = sc_adj_old + cm * (sc_adj_new - sc_gh_old);
                            s->mur_g[o][d][side][c][f] = sc_gh_new + ig_new;
                            s->mur_a[o][d][side][c][f] = eadj;
                        }
                    }
            }
        }
    }
}

/* g E0.B0 at every centre with the E0, B0 arrays as they are */
static void compute_Sax(ora_state *s)
{
    const double g = s->c.g;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < s->n[2]; k++)
        for (int j = 0; j < s->n[1]; j++)
            for (int i = 0; i < s->n[0]; i++) {
                double e[3], b[3];
                centre_E0(s, i, j, k, e);
                centre_B0(s, i, j, k, b);
                s->Sax[IX(s, i, j, k)] = g * (e[0] * b[0] + e[1] * b[1] + e[2] * b[2]);
            }
}

static double pml_sigma(const ora_state *s, int i, int j, int k)
{
    int id[3] = {i, j, k};
    double smax = s->c.pml_sigma_dt / s->c.dt, sig = 0.0;
    for (int d = 0; d < 3; d++) {
        if (s->c.ax_bc[d] != ORA_AX_PML) continue;
        int dist = id[d] < s->n[d] - 1 - id[d] ? id[d] : s->n[d] - 1 - id[d];
        if (dist < s->c.pml_n) {
            double r = 1.0 - (double)dist / s->c.pml_n;
            double sd = smax * r * r * r;
            if (sd > sig) sig = sd;
        }
    }
    return sig;
}

/* axion leapfrog to slot Ln from slots La (t_{n-1/2}) and Lb (t_{n+1/2}) */
static void update_phi(ora_state *s, int La, int Lb, int Ln)
{
    const double dt = s->c.dt, m2 = s->c.m * s->c.m, *h = s->c.dx;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < s->n[2]; k++)
        for (int j = 0; j < s->n[1]; j++)
            for (int i = 0; i < s->n[0]; i++) {
                long id = IX(s, i, j, k);
                double pb = s->phi[Lb][id], pa = s->phi[La][id];
                double lap = (phi_at(s, Lb, i + 1, j, k) - 2.0 * pb + phi_at(s, Lb, i - 1, j, k)) / (h[0] * h[0])
                           + (phi_at(s, Lb, i, j + 1, k) - 2.0 * pb + phi_at(s, Lb, i, j - 1, k)) / (h[1] * h[1])
                           + (phi_at(s, Lb, i, j, k + 1) - 2.0 * pb + phi_at(s, Lb, i, j, k - 1)) / (h[2] * h[2]);
                double src = s->Sax[id], sig = pml_sigma(s, i, j, k), pn;
                if (sig == 0.0)
                    pn = 2.0 * pb - pa + dt * dt * (lap - m2 * pb + src);
                else
                    pn = (dt * dt * (src - m2 * pb + lap - sig * sig * pb) + sig * dt * pa + 2.0 * pb - pa)
                       / (1.0 + sig * dt);
                s->phi[Ln][id] = pn;
            }
}

/* ghost values of the new axion level Ln on every non-periodic face */
static void axion_ghosts(ora_state *s, int La, int Lb, int Ln)
{
    const double dt = s->c.dt, m2 = s->c.m * s->c.m;
    for (int d = 0; d < 3; d++) {
        if (ax_periodic(s, d)) continue;
        int a, b;
        other_axes(d, &a, &b);
        double r = dt / s->c.dx[d];
        for (int side = 0; side < 2; side++) {
            int iadj = side ? s->n[d] - 1 : 0;
            for (int ib = 0; ib < s->n[b]; ib++)
                for (int ia = 0; ia < s->n[a]; ia++) {
                    int id[3];
                    id[d] = iadj; id[a] = ia; id[b] = ib;
                    long f = (long)ib * s->nn[a] + ia, cell = IX(s, id[0], id[1], id[2]);
                    if (s->c.ax_bc[d] == ORA_AX_OUTFLOW) {
                        /* the paper's two equations at the ghost (one-way wave and
                           Klein-Gordon, both centred at the ghost at the previous level),
                           solved for the second ghost and the new first ghost */
                        double gB = s->axg[d][side][Lb][f], gA = s->axg[d][side][La][f];
                        double p1 = s->phi[Lb][cell], S1 = s->Sax[cell];
                        double X = (-2.0 * gB + 2.0 * gA - dt * dt * (S1 - m2 * gB)
                                    + r * p1 - r * r * (p1 - 2.0 * gB)) / (r + r * r);
                        s->axg[d][side][Ln][f] = gA + r * (p1 - X);
                    } else {
                        s->axg[d][side][Ln][f] = s->phi[Ln][cell];
                    }
                }
        }
    }
}

/* E^{n+1/2} of the first ORA_WIN_KEEP x columns, both orders */
static void keep_half_columns(ora_state *s)
{
    const int kc = s->nn[0] < ORA_WIN_KEEP ? s->nn[0] : ORA_WIN_KEEP;
    for (int o = 0; o < 2; o++)
        for (int c = 0; c < 3; c++)
            for (int k = 0; k < s->nn[2]; k++)
                for (int j = 0; j < s->nn[1]; j++)
                    for (int i = 0; i < kc; i++)
                        s->Eh[o][c][((long)k * s->nn[1] + j) * ORA_WIN_KEEP + i] = s->E[o][c][IX(s, i, j, k)];
}

/* ------------------------------------------------------------ particles */

/* Sec. II.B.  Zero order: cold electrons (q = -1, m = 1) pushed by E0 and
   B0 + B_ext (Boris); first order: the perturbations x1, u1 of the same push,
   driven by the fields a particle feels to first order,
     F_p = sum S(r - x0) F1 + sum (grad S(r - x0) . x1) F0,
   i.e. the push's derivative: dp1/dt = q (E_p + v0 x B_p + v1 x B_nop) with
   v1 = (gamma0^2 u1 - u0 (u0.u1)) / gamma0^3.  Currents, deposited at the E
   points with the same shape:
     j0 = q w S(r - x0) v0,   j1 = q w [(grad S(r - x0) . x1) v0 + S(r - x0) v1].
   The shape S is linear (one cell wide) along every active axis, on each
   component's own staggered points.  Time levels: x^n, u^n at integer times;
   a step drifts x half a step with v^n, kicks u with E^{n+1/2}, B^{n+1/2} at
   that midpoint, drifts again with v^{n+1}, and deposits j^{n+1} at x^{n+1}
   for the second E half step (and the first one of the next step). */

typedef struct {
    int i[2];            /* the two points */
    double w[2], dw[2];  /* weights and their d/dx */
    int m;               /* points used: 1 on a degenerate axis */
} ora_shape;

static void shape1(const ora_state *s, int d, int nodal, double x, ora_shape *sh)
{
    if (s->n[d] == 1) {
        sh->m = 1;
        sh->i[0] = sh->i[1] = 0;
        sh->w[0] = 1.0; sh->w[1] = 0.0;
        sh->dw[0] = sh->dw[1] = 0.0;
        return;
    }
    double u = x / s->c.dx[d] - (nodal ? 0.0 : 0.5);
    double f0 = floor(u), f = u - f0;
    int i0 = (int)f0, i1 = i0 + 1;
    if (em_periodic(s, d)) {
        i0 = wrapn(i0, s->n[d]);
        i1 = wrapn(i1, s->n[d]);
    } else if (i0 < 0 || i1 >= extent(s, d, nodal)) {
        die("particle shape");
    }
    sh->m = 2;
    sh->i[0] = i0; sh->i[1] = i1;
    sh->w[0] = 1.0 - f; sh->w[1] = f;
    sh->dw[0] = -1.0 / s->c.dx[d]; sh->dw[1] = 1.0 / s->c.dx[d];
}

static void shapes(const ora_state *s, int c, int isB, const double X[3], ora_shape sh[3])
{
    for (int d = 0; d < 3; d++) shape1(s, d, isB ? d != c : d == c, X[d], &sh[d]);
}

/* F(X) = sum S F and sum (grad S . dX) F for component c of F, on the E
   points or the B points (isB), the zero-order B with B_ext added (bext) */
static void gather(const ora_state *s, const double *F, int c, int isB, int bext, const double X[3],
                   const double dX[3], double *val, double *grad)
{
    ora_shape sh[3];
    shapes(s, c, isB, X, sh);
    double v = 0.0, g = 0.0;
    for (int a2 = 0; a2 < sh[2].m; a2++)
        for (int a1 = 0; a1 < sh[1].m; a1++)
            for (int a0 = 0; a0 < sh[0].m; a0++) {
                double f = F[IX(s, sh[0].i[a0], sh[1].i[a1], sh[2].i[a2])];
                if (bext) f += bext_at(s, c, sh[0].i[a0]);
                double w = sh[0].w[a0] * sh[1].w[a1] * sh[2].w[a2];
                double gw = sh[0].dw[a0] * sh[1].w[a1] * sh[2].w[a2] * dX[0]
                          + sh[0].w[a0] * sh[1].dw[a1] * sh[2].w[a2] * dX[1]
                          + sh[0].w[a0] * sh[1].w[a1] * sh[2].dw[a2] * dX[2];
                v += w * f;
                g += gw * f;
            }
    *val = v;
    *grad = g;
}

/* J_c += a S(r - X) + b (grad S(r - X) . dX) at the E_c points */
static void deposit(ora_state *s, double *J, int c, const double X[3], const double dX[3], double a, double b)
{
    ora_shape sh[3];
    shapes(s, c, 0, X, sh);
    for (int a2 = 0; a2 < sh[2].m; a2++)
        for (int a1 = 0; a1 < sh[1].m; a1++)
            for (int a0 = 0; a0 < sh[0].m; a0++) {
                double w = sh[0].w[a0] * sh[1].w[a1] * sh[2].w[a2];
                double gw = sh[0].dw[a0] * sh[1].w[a1] * sh[2].w[a2] * dX[0]
                          + sh[0].w[a0] * sh[1].dw[a1] * sh[2].w[a2] * dX[1]
                          + sh[0].w[a0] * sh[1].w[a1] * sh[2].dw[a2] * dX[2];
                J[IX(s, sh[0].i[a0], sh[1].i[a1], sh[2].i[a2])] += a * w + b * gw;
            }
}

/* on a Mur axis a particle counts while it stays 1.5 cells inside the
   faces (its shape then reaches interior points only); periodic axes wrap */
static int place(const ora_state *s, double X[3])
{
    for (int d = 0; d < 3; d++) {
        if (s->n[d] == 1) continue;
        double L = s->n[d] * s->c.dx[d];
        if (em_periodic(s, d)) {
            if (X[d] < 0.0) X[d] += L;
            if (X[d] >= L) X[d] -= L;
        } else if (X[d] < 1.5 * s->c.dx[d] || X[d] > L - 1.5 * s->c.dx[d]) {
            return 0;
        }
    }
    return 1;
}

static void cross(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Boris rotation (J. P. Boris 1970) of u by the fields E, B with
   hq = q dt / (2 m), and its derivative along (du, dE, dB) */
static void boris(const double u[3], const double du[3], const double E[3], const double dE[3], const double B[3],
                  const double dB[3], double hq, double un[3], double dun[3])
{
    double um[3], dum[3], t[3], dtv[3], up[3], dup[3], sv[3], ds[3], c1[3], c2[3];
    for (int q = 0; q < 3; q++) {
        um[q] = u[q] + hq * E[q];
        dum[q] = du[q] + hq * dE[q];
    }
    double g = sqrt(1.0 + dot(um, um)), dg = dot(um, dum) / g;
    for (int q = 0; q < 3; q++) {
        t[q] = hq * B[q] / g;
        dtv[q] = hq * dB[q] / g - hq * B[q] * dg / (g * g);
    }
    double tt = dot(t, t), dtt = 2.0 * dot(t, dtv), den = 1.0 + tt;
    for (int q = 0; q < 3; q++) {
        sv[q] = 2.0 * t[q] / den;
        ds[q] = 2.0 * dtv[q] / den - 2.0 * t[q] * dtt / (den * den);
    }
    cross(um, t, c1);
    for (int q = 0; q < 3; q++) up[q] = um[q] + c1[q];
    cross(dum, t, c1);
    cross(um, dtv, c2);
    for (int q = 0; q < 3; q++) dup[q] = dum[q] + c1[q] + c2[q];
    cross(up, sv, c1);
    double upl[3], dupl[3];
    for (int q = 0; q < 3; q++) upl[q] = um[q] + c1[q];
    cross(dup, sv, c1);
    cross(up, ds, c2);
    for (int q = 0; q < 3; q++) dupl[q] = dum[q] + c1[q] + c2[q];
    for (int q = 0; q < 3; q++) {
        un[q] = upl[q] + hq * E[q];
        dun[q] = dupl[q] + hq * dE[q];
    }
}

/* velocity v = u / gamma and its derivative (gamma^2 du - u (u.du)) / gamma^3 */
static void velocity(const double u[3], const double du[3], double v[3], double dv[3])
{
    double g = sqrt(1.0 + dot(u, u)), ud = dot(u, du);
    for (int q = 0; q < 3; q++) {
        v[q] = u[q] / g;
        dv[q] = (g * g * du[q] - u[q] * ud) / (g * g * g);
    }
}

static void zero_currents(ora_state *s)
{
    for (int o = 0; o < 2; o++)
        for (int c = 0; c < 3; c++)
            if (s->J[o][c]) memset(s->J[o][c], 0, sizeof(double) * s->ncell);
}

/* j0 and j1 of one particle at X, dX with velocity v, dv */
static void deposit_particle(ora_state *s, long p, const double X[3], const double dX[3], const double v[3],
                             const double dv[3])
{
    const double qw = -1.0 * s->pw[p];
    for (int c = 0; c < 3; c++) {
        deposit(s, s->J[0][c], c, X, dX, qw * v[c], 0.0);
        deposit(s, s->J[1][c], c, X, dX, qw * dv[c], qw * v[c]);
    }
}

void ora_redeposit(ora_state *s)
{
    if (!s->np) return;
    zero_currents(s);
    for (long p = 0; p < s->np; p++) {
        if (s->pw[p] == 0.0) continue;
        double X[3], dX[3], u[3], du[3], v[3], dv[3];
        for (int q = 0; q < 3; q++) {
            X[q] = s->px[q][p]; dX[q] = s->px1[q][p]; u[q] = s->pu[q][p]; du[q] = s->pu1[q][p];
        }
        velocity(u, du, v, dv);
        deposit_particle(s, p, X, dX, v, dv);
    }
}

/* one step of every particle with the fields as they are (E^{n+1/2},
   B^{n+1/2}), then j^{n+1}; particles in index order, so every sum has a
   fixed order */
static void push_particles(ora_state *s)
{
    if (!s->np) return;
    const double dt = s->c.dt, hq = -0.5 * dt;
    zero_currents(s);
    for (long p = 0; p < s->np; p++) {
        if (s->pw[p] == 0.0) continue;
        double X[3], dX[3], u[3], du[3], v[3], dv[3];
        for (int q = 0; q < 3; q++) {
            X[q] = s->px[q][p]; dX[q] = s->px1[q][p]; u[q] = s->pu[q][p]; du[q] = s->pu1[q][p];
        }
        velocity(u, du, v, dv);
        for (int q = 0; q < 3; q++) {
            X[q] += 0.5 * dt * v[q];
            dX[q] += 0.5 * dt * dv[q];
        }
        if (!place(s, X)) { s->pw[p] = 0.0; continue; }
        double E0[3], Ep[3], B0[3], Bp[3];
        for (int c = 0; c < 3; c++) {
            double f, gf, f1, g1;
            gather(s, s->E[0][c], c, 0, 0, X, dX, &f, &gf);
            gather(s, s->E[1][c], c, 0, 0, X, dX, &f1, &g1);
            E0[c] = f;
            Ep[c] = f1 + gf;
            gather(s, s->B[0][c], c, 1, 1, X, dX, &f, &gf);
            gather(s, s->B[1][c], c, 1, 0, X, dX, &f1, &g1);
            B0[c] = f;
            Bp[c] = f1 + gf;
        }
        double un[3], dun[3];
        boris(u, du, E0, Ep, B0, Bp, hq, un, dun);
        velocity(un, dun, v, dv);
        for (int q = 0; q < 3; q++) {
            X[q] += 0.5 * dt * v[q];
            dX[q] += 0.5 * dt * dv[q];
        }
        int in = place(s, X);
        for (int q = 0; q < 3; q++) {
            s->px[q][p] = X[q]; s->px1[q][p] = dX[q]; s->pu[q][p] = un[q]; s->pu1[q][p] = dun[q];
        }
        if (!in) { s->pw[p] = 0.0; continue; }
        deposit_particle(s, p, X, dX, v, dv);
    }
}

long ora_particles(const ora_state *s) { return s->np; }

double *ora_particle_array(ora_state *s, int id)
{
    if (!s->np || id < 0 || id > 12) return NULL;
    if (id < 3) return s->px[id];
    if (id < 6) return s->pu[id - 3];
    if (id < 9) return s->px1[id - 6];
    if (id < 12) return s->pu1[id - 9];
    return s->pw;
}

double *ora_current(ora_state *s, int o, int c)
{
    if (o < 0 || o > 1 || c < 0 || c > 2) return NULL;
    return s->J[o][c];
}

/* ------------------------------------------------------------ one step */

static void one_step(ora_state *s)
{
    const double h = 0.5 * s->c.dt, g = s->c.g;
    int La = s->la, Lb = s->lb, Ln = 3 - La - Lb;

    compute_C(s, La, Lb, -1);      /* axion current at t_n (uses E0^n, B0^n) */
    update_E(s, 0, h, 0.0);        /* E0^{n+1/2} */
    update_E(s, 1, h, g);          /* E1^{n+1/2}, eq. update_E */
    keep_half_columns(s);          /* for a move of the window at t_{n+1} */
    mur_ghosts(s);                 /* tangential E ghosts at t_{n+1/2} */
    update_B(s, h);                /* B^{n+1/2} */
    compute_Sax(s);                /* g E0.B0 at t_{n+1/2} */
    update_phi(s, La, Lb, Ln);     /* phi^{n+3/2}, eq. update_axion (PML form in the layer) */
    axion_ghosts(s, La, Lb, Ln);
    push_particles(s);             /* x, u to t_{n+1} with E, B at t_{n+1/2}; j^{n+1} (Sec. II.B) */
    update_B(s, h);                /* B^{n+1} */
    update_E(s, 0, h, 0.0);        /* E0^{n+1} */
    compute_C(s, Lb, Ln, La);      /* axion current at t_{n+1} (E0^{n+1}, B0^{n+1}) */
    update_E(s, 1, h, g);          /* E1^{n+1} */

    s->la = Lb;
    s->lb = Ln;
    s->step++;
}

void ora_step(ora_state *s, long nsteps)
{
    for (long it = 0; it < nsteps; it++) one_step(s);
}

long ora_step_count(const ora_state *s) { return s->step; }

/* ------------------------------------------------------------ moving window */

/* shift rows of length m (x fastest, `rows` of them) left by `cells`, vacuum after */
static void shift_rows(double *a, long rows, int m, int cells)
{
    if (!a) return;
    #pragma omp parallel for schedule(static)
    for (long r = 0; r < rows; r++) {
        double *row = a + r * m;
        for (int i = 0; i < m; i++) row[i] = i + cells < m ? row[i + cells] : 0.0;
    }
}

/* Sec. III.B: the simulation window moves along +x at c once the laser is
   in.  One move by `cells` columns at a step boundary: every field array and
   every plane of the y and z faces shifts left by `cells` columns, the new
   columns at x_max are vacuum, the B_ext slab and the laser (no longer
   injected) are taken in window coordinates.  The x_min ghosts become the
   values that lay there before the move: the Mur ghost and its adjacent
   history the E^{n-1/2} of columns cells - 1 and cells, the axion ghosts both
   levels of cell cells - 1; the x_max ghosts are vacuum.
   Needs a Mur x axis, 1 <= cells <= ORA_WIN_KEEP, cells < n_x, and at least
   one step taken (E^{n-1/2}).  Returns 0, or -1 for such a bad request. */
int ora_shift_window(ora_state *s, int cells)
{
    if (s->c.em_bc[0] != ORA_EM_MUR || cells < 1 || cells > ORA_WIN_KEEP || cells >= s->n[0] || s->step < 1)
        return -1;
    const int m = s->nn[0];
    const long rows = (long)s->nn[1] * s->nn[2];
    /* x faces first, from the columns before the move */
    for (int k = 0; k < s->nn[2]; k++)
        for (int j = 0; j < s->nn[1]; j++) {
            const long f = (long)k * s->nn[1] + j;
            for (int o = 0; o < 2; o++)
                for (int c = 1; c < 3; c++) {
                    const double *eh = s->Eh[o][c] + f * ORA_WIN_KEEP;
                    s->mur_g[o][0][0][c][f] = eh[cells - 1];
                    s->mur_a[o][0][0][c][f] = eh[cells];
                    s->mur_g[o][0][1][c][f] = 0.0;
                    s->mur_a[o][0][1][c][f] = 0.0;
                }
            if (!ax_periodic(s, 0) && j < s->n[1] && k < s->n[2])
                for (int L = 0; L < 3; L++) {
                    s->axg[0][0][L][f] = s->phi[L][IX(s, cells - 1, j, k)];
                    s->axg[0][1][L][f] = 0.0;
                }
        }
    for (int o = 0; o < 2; o++)
        for (int c = 0; c < 3; c++) {
            shift_rows(s->E[o][c], rows, m, cells);
            shift_rows(s->B[o][c], rows, m, cells);
        }
    for (int L = 0; L < 3; L++) shift_rows(s->phi[L], rows, m, cells);
    /* the planes of the y and z faces: rows along x */
    for (int d = 1; d < 3; d++) {
        const int b = d == 2 ? 1 : 2;
        for (int side = 0; side < 2; side++) {
            for (int L = 0; L < 3; L++) shift_rows(s->axg[d][side][L], s->nn[b], m, cells);
            for (int o = 0; o < 2; o++)
                for (int c = 0; c < 3; c++) {
                    shift_rows(s->mur_g[o][d][side][c], s->nn[b], m, cells);
                    shift_rows(s->mur_a[o][d][side][c], s->nn[b], m, cells);
                }
        }
    }
    s->c.slab_lo -= cells;
    s->c.slab_hi -= cells;
    s->c.laser_on = 0;
    return 0;
}

/* ------------------------------------------------------------ energies */

void ora_energies(const ora_state *s, double out[3])
{
    const double dt = s->c.dt, m2 = s->c.m * s->c.m;
    double dv = 1.0;
    for (int d = 0; d < 3; d++)
        if (s->n[d] > 1) dv *= s->c.dx[d];
    double hphi = 0.0;
    for (int k = 0; k < s->n[2]; k++)
        for (int j = 0; j < s->n[1]; j++)
            for (int i = 0; i < s->n[0]; i++) {
                double pm = phi_mid(s, s->la, s->lb, i, j, k);
                double dtp = (phi_at(s, s->lb, i, j, k) - phi_at(s, s->la, i, j, k)) / dt;
                double e = dtp * dtp + m2 * pm * pm;
                int id[3] = {i, j, k};
                for (int d = 0; d < 3; d++) {
                    if (s->n[d] == 1) continue;
                    if (!ax_periodic(s, d) && id[d] + 1 >= s->n[d]) continue;
                    int nb[3] = {i, j, k};
                    nb[d] += 1;
                    double gr = (phi_mid(s, s->la, s->lb, nb[0], nb[1], nb[2]) - pm) / s->c.dx[d];
                    e += gr * gr;
                }
                hphi += 0.5 * e;
            }
    out[0] = hphi * dv;
    for (int o = 0; o < 2; o++) {
        double sum = 0.0;
        for (int c = 0; c < 3; c++) {
            for (int isb = 0; isb < 2; isb++) {
                const double *A = isb ? s->B[o][c] : s->E[o][c];
                int e0 = extent(s, 0, isb ? c != 0 : c == 0);
                int e1 = extent(s, 1, isb ? c != 1 : c == 1);
                int e2 = extent(s, 2, isb ? c != 2 : c == 2);
                for (int k = 0; k < e2; k++)
                    for (int j = 0; j < e1; j++)
                        for (int i = 0; i < e0; i++) {
                            double v = A[IX(s, i, j, k)];
                            sum += 0.5 * v * v;
                        }
            }
        }
        out[1 + o] = sum * dv;
    }
}

/* --------------------------------------------------------- construction */

static double *zalloc(long n)
{
    double *p = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!p) { fprintf(stderr, "axion oracle: out of memory\n"); abort(); }
    return p;
}

/* E^{-1/2} next to each Mur ghost, by the backward half step from t = 0,
   and the ghost itself set to the incident field (no scattered field yet) */
static void init_mur_history(ora_state *s)
{
    const double dt = s->c.dt, h = 0.5 * dt, g = s->c.g, t_old = -0.5 * dt;
    compute_C(s, s->la, s->lb, -1);
    for (int d = 0; d < 3; d++) {
        if (em_periodic(s, d)) continue;
        int a, b;
        other_axes(d, &a, &b);
        for (int side = 0; side < 2; side++) {
            int iadj = side ? s->n[d] - 1 : 0, igh = side ? s->n[d] : -1;
            int comps[2] = {a, b};
            for (int q = 0; q < 2; q++) {
                int c = comps[q];
                int ea = extent(s, a, c == a), eb = extent(s, b, c == b);
                for (int ib = 0; ib < eb; ib++)
                    for (int ia = 0; ia < ea; ia++) {
                        int id[3];
                        id[d] = iadj; id[a] = ia; id[b] = ib;
                        long f = (long)ib * s->nn[a] + ia;
                        double pg[3];
                        for (int e = 0; e < 3; e++) pg[e] = coord(s, e, id[e], e == c);
                        pg[d] = coord(s, d, igh, 0);
                        for (int o = 0; o < 2; o++) {
                            double rhs = curl_B(s, o, c, id[0], id[1], id[2]);
                            if (s->J[o][c]) rhs = rhs - s->J[o][c][IX(s, id[0], id[1], id[2])];
                            if (o == 1) rhs = rhs - g * face_S(s, c, id[0], id[1], id[2]);
                            s->mur_a[o][d][side][c][f] = s->E[o][c][IX(s, id[0], id[1], id[2])] - h * rhs;
                            int inj = (o == s->c.laser_order && d == 0 && side == 0);
                            s->mur_g[o][d][side][c][f] = inj ? ora_incident(s, c, pg[0], pg[1], pg[2], t_old) : 0.0;
                        }
                    }
            }
        }
    }
}

static void copy_ghosts_from_interior(ora_state *s, int L, int outflow_too)
{
    for (int d = 0; d < 3; d++) {
        if (ax_periodic(s, d)) continue;
        if (s->c.ax_bc[d] == ORA_AX_OUTFLOW && !outflow_too) continue;
        int a, b;
        other_axes(d, &a, &b);
        for (int side = 0; side < 2; side++) {
            int iadj = side ? s->n[d] - 1 : 0;
            for (int ib = 0; ib < s->n[b]; ib++)
                for (int ia = 0; ia < s->n[a]; ia++) {
                    int id[3];
                    id[d] = iadj; id[a] = ia; id[b] = ib;
                    s->axg[d][side][L][(long)ib * s->nn[a] + ia] = s->phi[L][IX(s, id[0], id[1], id[2])];
                }
        }
    }
}

int ora_create(const ora_config *cfg, ora_state **out)
{
    *out = NULL;
    double inv2 = 0.0;
    for (int d = 0; d < 3; d++) {
        if (cfg->n[d] < 1 || !(cfg->dx[d] > 0.0)) return -1;
        if (cfg->n[d] == 1 && (cfg->em_bc[d] != ORA_EM_PERIODIC || cfg->ax_bc[d] != ORA_AX_PERIODIC)) return -1;
        if (cfg->em_bc[d] == ORA_EM_MUR && cfg->n[d] < 2) return -1;
        if (cfg->ax_bc[d] == ORA_AX_PML && (cfg->pml_n < 1 || 2 * cfg->pml_n > cfg->n[d])) return -1;
        if (cfg->n[d] > 1) inv2 += 1.0 / (cfg->dx[d] * cfg->dx[d]);
    }
    if (!(cfg->dt > 0.0) || cfg->dt * cfg->dt * inv2 >= 1.0) return -1;
    if (cfg->laser_on && (cfg->em_bc[0] != ORA_EM_MUR || (cfg->laser_pol != 1 && cfg->laser_pol != 2))) return -1;
    if (cfg->laser_order != 0 && cfg->laser_order != 1) return -1;
    if (cfg->ppc[0] > 0) {
        /* particles: 1D or 2D, periodic transverse axes, the plasma two cells
           inside a Mur x axis */
        if (cfg->n[2] > 1 || cfg->ppc[1] < 1 || cfg->plasma_lo < 0 || cfg->plasma_hi > cfg->n[0] ||
            cfg->plasma_lo >= cfg->plasma_hi || !(cfg->plasma_n > 0.0))
            return -1;
        if (cfg->n[1] > 1 && cfg->em_bc[1] != ORA_EM_PERIODIC) return -1;
        if (cfg->em_bc[0] == ORA_EM_MUR && (cfg->plasma_lo < 2 || cfg->plasma_hi > cfg->n[0] - 2)) return -1;
    }

    ora_state *s = (ora_state *)calloc(1, sizeof(ora_state));
    if (!s) return -1;
    s->c = *cfg;
    for (int d = 0; d < 3; d++) {
        s->n[d] = cfg->n[d];
        s->nn[d] = cfg->n[d] + (cfg->em_bc[d] == ORA_EM_MUR ? 1 : 0);
    }
    s->ncell = (long)s->nn[0] * s->nn[1] * s->nn[2];
    for (int o = 0; o < 2; o++)
        for (int c = 0; c < 3; c++) {
            s->E[o][c] = zalloc(s->ncell);
            s->B[o][c] = zalloc(s->ncell);
        }
    for (int L = 0; L < 3; L++) s->phi[L] = zalloc(s->ncell);
    for (int c = 0; c < 3; c++) s->C[c] = zalloc(s->ncell);
    s->Sax = zalloc(s->ncell);
    for (int o = 0; o < 2; o++)
        for (int c = 0; c < 3; c++) s->Eh[o][c] = zalloc((long)s->nn[1] * s->nn[2] * ORA_WIN_KEEP);
    for (int d = 0; d < 3; d++) {
        int a, b;
        other_axes(d, &a, &b);
        long fa = (long)s->nn[a] * s->nn[b];
        for (int side = 0; side < 2; side++) {
            if (!ax_periodic(s, d))
                for (int L = 0; L < 3; L++) s->axg[d][side][L] = zalloc(fa);
            if (!em_periodic(s, d))
                for (int o = 0; o < 2; o++)
                    for (int c = 0; c < 3; c++) {
                        if (c == d) continue;
                        s->mur_g[o][d][side][c] = zalloc(fa);
                        s->mur_a[o][d][side][c] = zalloc(fa);
                    }
        }
    }
    s->la = 0;
    s->lb = 1;
    s->step = 0;

    /* the plasma: a lattice of ppc[0] x ppc[1] particles per cell */
    if (cfg->ppc[0] > 0) {
        const int px = cfg->ppc[0], py = s->n[1] > 1 ? cfg->ppc[1] : 1;
        s->np = (long)(cfg->plasma_hi - cfg->plasma_lo) * s->n[1] * px * py;
        for (int q = 0; q < 3; q++) {
            s->px[q] = zalloc(s->np); s->pu[q] = zalloc(s->np);
            s->px1[q] = zalloc(s->np); s->pu1[q] = zalloc(s->np);
        }
        s->pw = zalloc(s->np);
        for (int o = 0; o < 2; o++)
            for (int c = 0; c < 3; c++) s->J[o][c] = zalloc(s->ncell);
        long p = 0;
        for (int j = 0; j < s->n[1]; j++)
            for (int i = cfg->plasma_lo; i < cfg->plasma_hi; i++)
                for (int b = 0; b < py; b++)
                    for (int a = 0; a < px; a++, p++) {
                        s->px[0][p] = (i + (a + 0.5) / px) * cfg->dx[0];
                        s->px[1][p] = s->n[1] > 1 ? (j + (b + 0.5) / py) * cfg->dx[1] : 0.0;
                        s->px[2][p] = 0.0;
                        for (int q = 0; q < 3; q++) s->pu[q][p] = cfg->plasma_u[q];
                        s->pw[p] = cfg->plasma_n / (px * py);
                    }
        ora_redeposit(s);          /* j^0 */
    }

    /* axion levels at t = -dt/2 and +dt/2 (the two-level start of Sec. III.A) */
    const double dt = cfg->dt;
    for (int k = 0; k < s->n[2]; k++)
        for (int j = 0; j < s->n[1]; j++)
            for (int i = 0; i < s->n[0]; i++) {
                double x = coord(s, 0, i, 0), y = coord(s, 1, j, 0), z = coord(s, 2, k, 0);
                s->phi[0][IX(s, i, j, k)] = packet(s, x, y, z, -0.5 * dt);
                s->phi[1][IX(s, i, j, k)] = packet(s, x, y, z, 0.5 * dt);
            }
    /* outflow ghosts start from the same analytic packet; the others copy */
    for (int d = 0; d < 3; d++) {
        if (s->c.ax_bc[d] != ORA_AX_OUTFLOW) continue;
        int a, b;
        other_axes(d, &a, &b);
        for (int side = 0; side < 2; side++) {
            int igh = side ? s->n[d] : -1;
            for (int ib = 0; ib < s->n[b]; ib++)
                for (int ia = 0; ia < s->n[a]; ia++) {
                    int id[3];
                    id[d] = igh; id[a] = ia; id[b] = ib;
                    double x = coord(s, 0, id[0], 0), y = coord(s, 1, id[1], 0), z = coord(s, 2, id[2], 0);
                    long f = (long)ib * s->nn[a] + ia;
                    s->axg[d][side][0][f] = packet(s, x, y, z, -0.5 * dt);
                    s->axg[d][side][1][f] = packet(s, x, y, z, 0.5 * dt);
                }
        }
    }
    copy_ghosts_from_interior(s, 0, 0);
    copy_ghosts_from_interior(s, 1, 0);
    init_mur_history(s);
    *out = s;
    return 0;
}

void ora_refresh_initial(ora_state *s)
{
    copy_ghosts_from_interior(s, s->la, 0);
    copy_ghosts_from_interior(s, s->lb, 0);
    init_mur_history(s);
}

void ora_destroy(ora_state *s)
{
    if (!s) return;
    for (int o = 0; o < 2; o++)
        for (int c = 0; c < 3; c++) { free(s->E[o][c]); free(s->B[o][c]); }
    for (int L = 0; L < 3; L++) free(s->phi[L]);
    for (int c = 0; c < 3; c++) free(s->C[c]);
    free(s->Sax);
    for (int o = 0; o < 2; o++)
        for (int c = 0; c < 3; c++) { free(s->Eh[o][c]); free(s->J[o][c]); }
    for (int q = 0; q < 3; q++) { free(s->px[q]); free(s->pu[q]); free(s->px1[q]); free(s->pu1[q]); }
    free(s->pw);
    for (int d = 0; d < 3; d++)
        for (int side = 0; side < 2; side++) {
            for (int L = 0; L < 3; L++) free(s->axg[d][side][L]);
            for (int o = 0; o < 2; o++)
                for (int c = 0; c < 3; c++) { free(s->mur_g[o][d][side][c]); free(s->mur_a[o][d][side][c]); }
        }
    free(s);
}

void ora_extents(const ora_state *s, int nn[3])
{
    for (int d = 0; d < 3; d++) nn[d] = s->nn[d];
}

double *ora_field(ora_state *s, int id)
{
    if (id >= ORA_E0X && id <= ORA_B1Z) {
        int o = id / 6, r = id % 6;
        return r < 3 ? s->E[o][r] : s->B[o][r - 3];
    }
    if (id == ORA_PHI_OLD) return s->phi[s->la];
    if (id == ORA_PHI_NEW) return s->phi[s->lb];
    return NULL;
}

double *ora_axion_ghost(ora_state *s, int d, int side, int level)
{
    if (d < 0 || d > 2 || side < 0 || side > 1 || ax_periodic(s, d)) return NULL;
    return s->axg[d][side][level ? s->lb : s->la];
}
