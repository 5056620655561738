"""Laboratory units -> the oscillator units of the energy functional (Sec. II).

The conversion itself is the library's host-only ``bec_params_from_physical``
(it needs no GPU); this module marshals arguments and returns the parameter
dict that ``solver.Context`` and ``solver.Batch`` take, together with the
oscillator length l in metres, by which the box edges are divided.

Readings of Sec. II used by the conversion:
  * contact couplings G_ij = 4 pi a_ij N_j / l by default, the coupling
    4 pi hbar^2 a / m for which the LHY prefactor of Eq. (1) reproduces the
    Lee-Huang-Yang energy; ``contact_2pi=True`` takes the 2 pi printed in Sec. II;
  * the dipolar input is the k-space amplitude Gdd_ij = (4 pi / 3) D_ij with
    D_ij = mu_0 mu_i mu_j N_j / (4 pi l^3 hbar omega_0) as printed in Sec. II;
  * one atomic mass for both components (the functional has one kinetic term).
"""
import ctypes as C

from . import binding as B


def physical_params(mass_amu: float, a_bohr, mu_bohr, N, f0_hz: float, trap_hz, r_cut_um: float,
                    c_lhy: float = 1.0, n_u: int = 16, contact_2pi: bool = False,
                    dip_cut: int = 0) -> tuple[dict, float]:
    """Parameters in oscillator units and the length unit l (m).

    mass_amu: atomic mass (u); a_bohr: 2x2 scattering lengths (Bohr radii);
    mu_bohr: the two magnetic moments along the field (Bohr magnetons, signed);
    N: atom numbers; f0_hz: omega_0 / 2 pi; trap_hz: omega_d / 2 pi (Hz);
    r_cut_um: dipolar cutoff radius (micrometres).  Raises BecError with the
    library's message on invalid input."""
    ph = B.Physical()
    ph.mass_amu = float(mass_amu)
    for i in range(2):
        ph.mu_bohr[i] = float(mu_bohr[i])
        ph.N[i] = float(N[i])
        for j in range(2):
            ph.a_bohr[i][j] = float(a_bohr[i][j])
    ph.f0_hz = float(f0_hz)
    for d in range(3):
        ph.trap_hz[d] = float(trap_hz[d])
    ph.c_lhy = float(c_lhy)
    ph.r_cut_um = float(r_cut_um)
    ph.n_u = int(n_u)
    ph.contact_2pi = 1 if contact_2pi else 0
    ph.dip_cut = int(dip_cut)
    P = B.Params()
    l = C.c_double(0.0)
    B.check(B.lib().bec_params_from_physical(C.byref(ph), C.byref(P), C.byref(l)), "bec_params_from_physical")
    return P.to_dict(), l.value


def box_in_units(lo_um, hi_um, length_m: float) -> tuple[list, list]:
    """Box edges given in micrometres -> units of the oscillator length."""
    return ([float(v) * 1e-6 / length_m for v in lo_um], [float(v) * 1e-6 / length_m for v in hi_um])
