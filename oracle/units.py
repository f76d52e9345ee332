"""SI inputs in the normalised units of a run, by way of natural units.

TEST INFRASTRUCTURE ONLY: the independent reference for the library's SI
front end.  The library derives every factor from the SI constants; this
module goes through energies in eV instead (hbar c, m_e c^2), so that a
wrong constant or a dropped factor on either side shows as a mismatch.

Normalised units: times in 1/omega0, lengths in 1/k0 with k0 = 2 pi / lambda0
and omega0 = c k0; fields in m_e c omega0 / e (E) and m_e omega0 / e (B);
masses as m_a c^2 / (hbar omega0).  The axion field is measured so that one
coupling drives both the axion source and the axion current of the SI
equations (Sec. II.A); in natural (Heaviside-Lorentz) units that coupling is
g_agg m_e c^2 / sqrt(4 pi alpha), g_agg in GeV^-1.
"""
import math

HBAR_C_EV_M = 1.973269804e-7      # hbar c [eV m] (CODATA 2018)
ME_C2_EV = 0.51099895000e6        # m_e c^2 [eV] (CODATA 2018)
C_M_S = 299792458.0               # c [m/s]
ALPHA = 7.2973525693e-3           # fine-structure constant (CODATA 2018)


def axion_coupling(m_a_eV, c_gamma):
    """g_agg [GeV^-1] of an axion model (Sec. III.B): the decay constant from
    m_a = 6.3 eV x 10^6 GeV / f_a, then g_agg = c_gamma 2 alpha / (pi f_a)."""
    f_a_GeV = 6.3 * 1e6 / m_a_eV
    return c_gamma * 2.0 * ALPHA / (math.pi * f_a_GeV)


def from_si(si, ndim):
    """The normalised run fields from SI inputs (dict with the keys of the
    library's SI struct; missing keys 0)."""
    lam = si["lambda0"]
    k0 = 2.0 * math.pi / lam                      # 1/m
    hbar_w0_eV = HBAR_C_EV_M * k0                 # photon energy of lambda0
    e_unit = ME_C2_EV * k0                        # V/m: (m_e c^2 / e) k0
    b_unit = e_unit / C_M_S                       # T
    out = {}
    out["dx"] = [k0 * si["dx"][d] for d in range(ndim)]
    out["dt"] = C_M_S * k0 * si["dt"]
    out["m"] = si.get("m_a", 0.0) / hbar_w0_eV
    out["g"] = si.get("g_agg", 0.0) * (ME_C2_EV * 1e-9) / math.sqrt(4.0 * math.pi * ALPHA)
    out["bext"] = [b / b_unit for b in si.get("bext", [0.0, 0.0, 0.0])]
    lam_l = si.get("lambda_laser", 0.0)
    out["omega"] = lam / lam_l if lam_l > 0 else 1.0
    out["e_amp"] = si.get("e_amp", 0.0) / e_unit
    for key in ("fwhm", "t_center"):
        out[key] = C_M_S * k0 * si.get(key, 0.0)
    for key in ("waist", "x_focus", "y_c", "z_c"):
        out[key] = k0 * si.get(key, 0.0)
    return out
