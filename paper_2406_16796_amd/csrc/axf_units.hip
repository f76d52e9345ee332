// axf_units.hip -- SI inputs to the normalised units of a run (host only).
//
// The derivation follows the SI form of the axion-Maxwell equations (Sec.
// II.A).  With t = t'/omega0, x = x'/k0, E = (m_e c omega0 / e) E',
// B = (m_e omega0 / e) B' and the axion field phi = s omega0 phi':
//   - the Klein-Gordon equation, divided by omega0^3 s / c^2, has the source
//     g m_e^2 c^3 / (hbar mu0 e^2 omega0 s) E'.B' and the mass term
//     (m_a c^2 / (hbar omega0))^2;
//   - Ampere's law, divided by m_e omega0^2 / (c e), has the axion current
//     g omega0 s [(d_t' phi') B' - E' x grad' phi'].
// The two couplings are equal for s = m_e c^(3/2) / (e omega0 sqrt(hbar mu0)),
// and then both are g m_e c^(3/2) / (e sqrt(hbar mu0)), independent of omega0.
#include <math.h>

#include "axf_internal.h"

namespace axf {
int fail(int code, const char *fmt, ...);
}

namespace {

// CODATA 2018 (exact where the SI defines them)
constexpr double kC = 299792458.0;                 // m / s
constexpr double kE = 1.602176634e-19;             // C
constexpr double kHbar = 1.054571817e-34;          // J s
constexpr double kMe = 9.1093837015e-31;           // kg
constexpr double kMu0 = 1.25663706212e-6;          // N / A^2
constexpr double kAlpha = 7.2973525693e-3;
constexpr double kPi = 3.14159265358979323846;

}  // namespace

extern "C" {

int axf_config_from_si(const axf_si *si, axf_config *cfg)
{
    using axf::fail;
    if (!si || !cfg) return fail(AXF_EINVAL, "null argument");
    if (!(si->lambda0 > 0.0)) return fail(AXF_EINVAL, "lambda0 must be positive");
    if (si->lambda_laser < 0.0) return fail(AXF_EINVAL, "lambda_laser must not be negative");
    const int nd = cfg->ndim;
    if (nd < 1 || nd > 3) return fail(AXF_EINVAL, "ndim must be 1, 2 or 3 (set it before the conversion)");
    for (int d = 0; d < nd; d++)
        if (!(si->dx[d] > 0.0)) return fail(AXF_EINVAL, "cell size on axis %d must be positive", d);
    if (!(si->dt > 0.0)) return fail(AXF_EINVAL, "dt must be positive");
    if (!(si->m_a >= 0.0)) return fail(AXF_EINVAL, "axion mass must not be negative");
    const double w0 = 2.0 * kPi * kC / si->lambda0, k0 = w0 / kC;
    for (int d = 0; d < nd; d++) cfg->dx[d] = k0 * si->dx[d];
    cfg->dt = w0 * si->dt;
    cfg->m = si->m_a * kE / (kHbar * w0);
    // hbar / GeV in seconds, then the normalised coupling
    const double g_s = si->g_agg * kHbar / (1e9 * kE);
    cfg->g = g_s * kMe * kC * sqrt(kC) / (kE * sqrt(kHbar * kMu0));
    const double b_unit = kMe * w0 / kE, e_unit = kMe * kC * w0 / kE;
    for (int d = 0; d < 3; d++) cfg->bext[d] = si->bext[d] / b_unit;
    cfg->omega = si->lambda_laser > 0.0 ? si->lambda0 / si->lambda_laser : 1.0;
    cfg->e_amp = si->e_amp / e_unit;
    cfg->fwhm = w0 * si->fwhm;
    cfg->t_center = w0 * si->t_center;
    cfg->waist = k0 * si->waist;
    cfg->x_focus = k0 * si->x_focus;
    cfg->y_c = k0 * si->y_c;
    cfg->z_c = k0 * si->z_c;
    return AXF_OK;
}

int axf_axion_coupling(double m_a_eV, double c_gamma, double *g_agg)
{
    using axf::fail;
    if (!g_agg) return fail(AXF_EINVAL, "null output");
    if (!(m_a_eV > 0.0)) return fail(AXF_EINVAL, "axion mass must be positive");
    const double f_a = 6.3e6 / m_a_eV;        // GeV
    *g_agg = c_gamma * 2.0 * kAlpha / (kPi * f_a);
    return AXF_OK;
}

}  // extern "C"
