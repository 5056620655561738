"""Laboratory-unit front end (bec_params_from_physical) pinned against physics.

The conversion into the oscillator units of Sec. II is checked end to end: the
dimensionless energies that the oracle computes from the converted parameters,
times hbar omega_0, must equal the same energies written in SI units from
textbook physics that is independent of the conversion formulas:
  * the Lee-Huang-Yang energy density e = (2 pi hbar^2 a n^2 / m)(128 / (15 sqrt(pi))) sqrt(n a^3)
    and its chemical potential (32 / (3 sqrt(pi))) g n sqrt(n a^3), g = 4 pi hbar^2 a / m,
    for a single component without dipoles: this fixes the contact prefactor
    4 pi (the 2 pi printed in Sec. II misses it by 2^(5/2) through the LHY term);
  * the mean-field contact energy (1/2) g_ij N_i N_j int n_i n_j of Gaussian clouds;
  * the dipolar energy of cylindrical Gaussian clouds with the k-space
    interaction (mu_0 mu_i mu_j / 3)(3 cos^2 alpha - 1), the Fourier transform
    of (mu_0 mu_i mu_j / 4 pi)(1 - 3 cos^2 theta) / r^3, for co- and counter-polarised pairs;
  * the dipolar lengths a_dd = mu_0 mu^2 m / (12 pi hbar^2) quoted in the
    literature for 164Dy (130.8 a_0) and 166Er (65.5 a_0).
No GPU is needed: the conversion is host code in the library.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2510_24543_amd import binding as B
from paper_2510_24543_amd import inputs, units

# CODATA 2018
HBAR = 1.054571817e-34
MU0 = 1.25663706212e-6
MUB = 9.2740100783e-24
A0 = 5.29177210903e-11
AMU = 1.66053906660e-27

M_DY164 = 163.9291819
M_ER166 = 165.9302995


def conv(**kw):
    base = dict(mass_amu=M_DY164, a_bohr=[[90.0, 40.0], [40.0, 70.0]], mu_bohr=[9.93, -6.98],
                N=[2.0e4, 3.0e4], f0_hz=120.0, trap_hz=[60.0, 80.0, 200.0], r_cut_um=6.0)
    base.update(kw)
    return units.physical_params(**base)


def unit_energy(mass_amu, f0_hz):
    return HBAR * 2 * math.pi * f0_hz


def grid_of(n, half):
    return {"n": list(n), "lo": [-h for h in half], "hi": list(half)}


def gaussian(grid, sig, c=(0.0, 0.0, 0.0)):
    x, y, z = inputs.coords(grid)
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    n = np.exp(-0.5 * ((X - c[0]) ** 2 / sig[0] ** 2 + (Y - c[1]) ** 2 / sig[1] ** 2
                       + (Z - c[2]) ** 2 / sig[2] ** 2)) / ((2 * np.pi) ** 1.5 * sig[0] * sig[1] * sig[2])
    return np.sqrt(n).astype(np.complex128)


# ---------------------------------------------------------------- LHY: textbook Lee-Huang-Yang
@pytest.mark.parametrize("a_bohr,n1", [(90.0, 0.02), (250.0, 0.3), (40.0, 1e-3)])
def test_lhy_reproduces_lee_huang_yang_in_si(orc, a_bohr, n1):
    N1, f0, m_amu = 2.5e4, 150.0, M_DY164
    P, l = conv(mass_amu=m_amu, a_bohr=[[a_bohr, 0.0], [0.0, 0.0]], mu_bohr=[0.0, 0.0], N=[N1, 1.0],
                f0_hz=f0, n_u=4)
    e, d1, _ = orc.lhy_point(P, n1, 0.0)
    m, a = m_amu * AMU, a_bohr * A0
    n_si = N1 * n1 / l ** 3
    e_textbook = 2 * math.pi * HBAR ** 2 * a * n_si ** 2 / m * 128 / (15 * math.sqrt(math.pi)) * math.sqrt(n_si * a ** 3)
    mu_textbook = 4 * math.pi * HBAR ** 2 * a * n_si / m * 32 / (3 * math.sqrt(math.pi)) * math.sqrt(n_si * a ** 3)
    eu = unit_energy(m_amu, f0)
    assert abs(e * eu / l ** 3 - e_textbook) < 1e-12 * e_textbook
    assert abs(d1 * eu / N1 - mu_textbook) < 1e-12 * mu_textbook
    # the prefactor printed in Sec. II gives the LHY energy 2^(-5/2) times the textbook one
    P2, _ = conv(mass_amu=m_amu, a_bohr=[[a_bohr, 0.0], [0.0, 0.0]], mu_bohr=[0.0, 0.0], N=[N1, 1.0],
                 f0_hz=f0, n_u=4, contact_2pi=True)
    e2 = orc.lhy_point(P2, n1, 0.0)[0]
    assert abs(e2 * eu / l ** 3 / e_textbook - 2 ** -2.5) < 1e-12


# ---------------------------------------------------------------- contact: mean-field energy
def test_contact_energy_in_si(orc):
    grid = grid_of((64, 64, 64), (12.0, 12.0, 12.0))
    s1, s2 = (1.0, 1.2, 0.9), (1.4, 0.8, 1.1)
    c1, c2 = (0.7, 0.0, 0.0), (-0.5, 0.3, 0.0)
    a = [[90.0, 40.0], [40.0, 70.0]]
    N = [2.0e4, 3.0e4]
    f0 = 120.0
    P, l = conv(a_bohr=a, mu_bohr=[0.0, 0.0], N=N, f0_hz=f0)
    psi = np.stack([gaussian(grid, s1, c1), gaussian(grid, s2, c2)])
    t, _, _, _ = orc.heval(grid, P, psi)
    m = M_DY164 * AMU

    def overlap_si(sa, ca, sb, cb):
        v = 1.0
        for d in range(3):
            var = (sa[d] ** 2 + sb[d] ** 2) * l * l
            v *= math.exp(-((ca[d] - cb[d]) * l) ** 2 / (2 * var)) / math.sqrt(2 * math.pi * var)
        return v

    shapes = ((s1, c1), (s2, c2))
    eu = unit_energy(M_DY164, f0)
    for i in range(2):
        for j in range(2):
            g = 4 * math.pi * HBAR ** 2 * a[i][j] * A0 / m
            # E_c[i][j] carries half of the pair energy g_ij N_i N_j int n_i n_j
            exact = 0.5 * g * N[i] * N[j] * overlap_si(*shapes[i], *shapes[j])
            assert abs(t["E_c"][i][j] * eu - exact) < 1e-11 * exact, (i, j)


# ---------------------------------------------------------------- dipolar: Gaussian clouds
def dipolar_gaussian_si(amp, sr, sz):
    """(1/2) amp int d^3k/(2 pi)^3 |n(k)|^2 (3 cos^2 alpha - 1) for a normalised
    cylindrical Gaussian density with standard deviations sr, sz (metres)."""
    f = lambda c: (3 * c * c - 1) * (sr ** 2 * (1 - c * c) + sz ** 2 * c * c) ** -1.5
    val, _ = integrate.quad(f, -1, 1, epsabs=0, epsrel=1e-13, limit=200)
    return amp / (32 * np.pi ** 1.5) * val


@pytest.mark.parametrize("mu", [(9.93, 9.93), (10.0, -10.0), (10.0, 7.07)])
def test_dipolar_energy_in_si(orc, mu):
    # both components share one elongated Gaussian; the cutoff radius (16 l) keeps
    # periodic images out and covers the cloud, so the cut interaction is the full one
    f0, N = 110.0, [3.0e4, 1.5e4]
    _, l = conv(f0_hz=f0)
    P, l = conv(a_bohr=[[0.0, 0.0], [0.0, 0.0]], mu_bohr=list(mu), N=N, f0_hz=f0, r_cut_um=16.0 * l * 1e6)
    assert abs(P["r_cut"] - 16.0) < 1e-12
    grid = grid_of((64, 64, 128), (16.0, 16.0, 16.0))
    sr, sz = 1.0, 1.6
    g = gaussian(grid, (sr, sr, sz))
    t, _, _, _ = orc.heval(grid, P, np.stack([g, g]))
    eu = unit_energy(M_DY164, f0)
    for i in range(2):
        for j in range(2):
            amp = MU0 * (mu[i] * MUB) * (mu[j] * MUB) / 3.0
            exact = N[i] * N[j] * dipolar_gaussian_si(amp, sr * l, sz * l)   # (1/2) N_i N_j U_ij pair term
            assert abs(t["E_dd"][i][j] * eu - exact) < 1e-10 * abs(exact), (i, j)
    if mu[0] * mu[1] < 0:
        assert t["E_dd"][0][1] > 0 > t["E_dd"][0][0]     # elongated along the field: attractive self term


# ---------------------------------------------------------------- dipolar lengths
@pytest.mark.parametrize("mass,mu,a_dd", [(M_DY164, 9.93, 130.8), (M_ER166, 6.98, 65.5)])
def test_dipolar_length_matches_literature(mass, mu, a_dd):
    for N, f0 in (([1e4, 1e4], 100.0), ([3e5, 3e5], 900.0)):
        P, _ = conv(mass_amu=mass, a_bohr=[[100.0, 0.0], [0.0, 100.0]], mu_bohr=[mu, mu], N=N, f0_hz=f0)
        # eps_dd = a_dd / a is independent of the unit frequency and of N
        assert abs(P["Gdd"][0][0] / P["G"][0][0] * 100.0 - a_dd) < 5e-3 * a_dd


# ---------------------------------------------------------------- scaling, signs, validation
def test_scaling_and_signs():
    P, l = conv()
    assert P["omega"] == pytest.approx([0.5, 80 / 120, 200 / 120], rel=1e-15)
    assert abs(P["r_cut"] - 6.0e-6 / l) < 1e-12 * P["r_cut"]
    m, w0 = M_DY164 * AMU, 2 * math.pi * 120.0
    assert abs(l - math.sqrt(HBAR / (m * w0))) < 1e-12 * l
    # N_i G_ij and N_i Gdd_ij symmetric; counter-polarised cross amplitude negative
    for k in ("G", "Gdd"):
        assert abs(P["N"][0] * P[k][0][1] - P["N"][1] * P[k][1][0]) < 1e-12 * abs(P["N"][0] * P[k][0][1])
    assert P["Gdd"][0][1] < 0 and P["Gdd"][0][0] > 0 and P["Gdd"][1][1] > 0
    # G_ij and Gdd_ij grow with N_j and with sqrt(omega_0)
    P4, _ = conv(f0_hz=480.0, N=[4.0e4, 3.0e4])
    assert abs(P4["G"][0][0] / P["G"][0][0] - 4.0) < 1e-12
    assert abs(P4["Gdd"][0][1] / P["Gdd"][0][1] - 2.0) < 1e-12
    assert abs(P4["Gdd"][1][0] / P["Gdd"][1][0] - 4.0) < 1e-12
    P2, _ = conv(contact_2pi=True)
    assert abs(P2["G"][1][1] / P["G"][1][1] - 0.5) < 1e-15 and P2["Gdd"] == P["Gdd"]
    lo, hi = units.box_in_units([-10.0, -10.0, -5.0], [10.0, 10.0, 5.0], l)
    assert abs(hi[0] - 10e-6 / l) < 1e-12 * hi[0] and lo[2] == -hi[2]


@pytest.mark.parametrize("bad", [dict(mass_amu=0.0), dict(f0_hz=-1.0), dict(N=[1e4, 0.0]),
                                 dict(a_bohr=[[90.0, 40.0], [41.0, 70.0]]), dict(trap_hz=[60.0, -1.0, 200.0]),
                                 dict(r_cut_um=0.0), dict(n_u=0), dict(n_u=65), dict(contact_2pi=2),
                                 dict(mu_bohr=[float("nan"), 1.0]), dict(c_lhy=float("inf"))])
def test_invalid_input_is_rejected(bad):
    if "contact_2pi" in bad:
        ph = B.Physical()
        ph.mass_amu, ph.f0_hz, ph.r_cut_um, ph.n_u, ph.contact_2pi = 160.0, 100.0, 5.0, 16, 2
        ph.N[0] = ph.N[1] = 1e4
        out = B.Params()
        assert B.lib().bec_params_from_physical(ph, out, None) == 1
        return
    with pytest.raises(B.BecError):
        conv(**bad)


def test_paper_setups_convert():
    """The laboratory parameter sets of Sec. VI convert into valid parameters."""
    # Sec. VI.A: 52Cr, counter-polarised 6 mu_B, trap 2 pi (100, 100, 800) Hz
    P, _ = units.physical_params(51.9405075, [[100.0, 100.0], [100.0, 100.0]], [6.0, -6.0], [5e5, 2.5e5],
                                 100.0, [100.0, 100.0, 800.0], r_cut_um=20.0)
    assert P["omega"] == [1.0, 1.0, 8.0] and P["Gdd"][0][1] < 0
    # Sec. VI.C: 162Dy, mu_1 = -mu_2 = 10 mu_B, a = (50, 70, 150) a_0, N = 3e4 each
    P, _ = units.physical_params(161.9268056, [[50.0, 150.0], [150.0, 70.0]], [10.0, -10.0], [3e4, 3e4],
                                 100.0, [50.0, 50.0, 250.0], r_cut_um=10.0)
    assert P["G"][0][1] / P["G"][0][0] == pytest.approx(3.0, rel=1e-14)
    assert P["Gdd"][0][0] / P["G"][0][0] > 2.5          # strongly dipolar: eps_dd ~ 2.6


def test_dip_cut_is_passed_through_and_checked():
    from paper_2510_24543_amd import binding as B
    args = (164.0, [[118.5, 57.65], [57.65, 58.95]], [10.0, 7.07], [1e6, 1e6], 900.0, [0.0, 0.0, 72.0])
    p, _ = units.physical_params(*args, r_cut_um=2.0, dip_cut=1)
    assert p["dip_cut"] == 1
    p, _ = units.physical_params(*args, r_cut_um=2.0)
    assert p["dip_cut"] == 0
    with pytest.raises(B.BecError, match="EINVAL"):
        units.physical_params(*args, r_cut_um=2.0, dip_cut=2)
