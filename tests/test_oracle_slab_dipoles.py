"""Pins of the oracle's slab-cut dipolar kernel (periodic x, y; the
interaction cut at |z - z'| < Z), the truncation for the periodic-xy setups of
Sec. VI.C.  Dipoles along z (Sec. VI.A).

Mixed representation.  The uncut kernel of unit amplitude, 3 kz^2/k^2 - 1 =
2 - 3 k_rho^2 / (k_rho^2 + kz^2), has the inverse Fourier transform in kz
  K(k_rho, u) = 2 delta(u) - (3/2) k_rho exp(-k_rho |u|)
(the Lorentzian 1/(a^2 + kz^2) transforms to exp(-a|u|)/(2a)).  Cutting the
interaction to |u| < Z multiplies the second term by theta(Z - |u|).  On a grid
periodic in z with 2 Z <= L_z the cut kernel fits in one period, so the discrete
convolution is exact for it.

Two layers.  n_j(x, y, z) = (1 + a_j cos(q x)) g(z - z_j) / (L_x L_y), g a
normalised Gaussian of width sigma (resolved by the grid, its periodic images
negligible).  Then
  X = integral n_1 (U * n_2) = [Kbar(0) + (a_1 a_2 / 2) Kbar(q)] / (L_x L_y),
  Kbar(k) = 2 G_s(dz) - (3/2) k integral_{-Z}^{Z} exp(-k |u|) G_s(u - dz) du,
with G_s the normalised Gaussian of width s = sqrt(2) sigma and dz = z_1 - z_2;
the u integral is a sum of erf terms (completing the square).  With a = 0 this
is the energy of a layer uniform in the plane: the contact-like value 2 n^2,
whatever Z (perpendicular dipoles in a uniform sheet).
"""
import math

import numpy as np
import pytest
from scipy.special import erf

from paper_2510_24543_amd import inputs


def gauss(u, s):
    return math.exp(-0.5 * (u / s) ** 2) / (math.sqrt(2 * math.pi) * s)


def half_line(k, c, s, Z):
    """integral_0^Z exp(-k u) G_s(u - c) du"""
    m = c - k * s * s
    pre = math.exp(-k * c + 0.5 * (k * s) ** 2)
    return pre * 0.5 * (erf((Z - m) / (s * math.sqrt(2))) - erf(-m / (s * math.sqrt(2))))


def kbar(k, dz, s, Z):
    if k == 0.0:
        return 2.0 * gauss(dz, s)
    I = half_line(k, dz, s, Z) + half_line(k, -dz, s, Z)      # integral over |u| < Z of exp(-k|u|) G_s(u - dz)
    return 2.0 * gauss(dz, s) - 1.5 * k * I


def layers(grid, a, zc, sigma, m):
    L = [grid["hi"][d] - grid["lo"][d] for d in range(3)]
    x, y, z = inputs.coords(grid)
    X, Y, Zg = np.meshgrid(x, y, z, indexing="ij")
    q = 2 * np.pi * m / L[0]
    out = []
    for j in range(2):
        g = np.exp(-0.5 * ((Zg - zc[j]) / sigma) ** 2) / (np.sqrt(2 * np.pi) * sigma)
        out.append(np.sqrt((1.0 + a[j] * np.cos(q * X)) * g / (L[0] * L[1])))
    return np.array(out, dtype=np.complex128), q, L


def unit_dipolar(Z):
    return {"N": [1.0, 1.0], "omega": [0.0, 0.0, 0.0], "G": [[0.0, 0.0], [0.0, 0.0]],
            "Gdd": [[1.0, 1.0], [1.0, 1.0]], "c_lhy": 0.0, "r_cut": Z, "n_u": 1, "dip_cut": 1}


GRID = {"n": [8, 16, 96], "lo": [-8.0, -8.0, -8.0], "hi": [8.0, 8.0, 8.0]}   # h_z = 1/6
SIGMA = 0.5


@pytest.mark.parametrize("Z,zc,a,m", [
    (8.0, (1.0, -1.5), (0.6, -0.4), 1),     # uncut within the box
    (1.5, (1.0, -1.5), (0.6, -0.4), 2),     # layers farther apart than the cut
    (2.5, (1.0, -1.5), (0.9, 0.7), 3),      # the cut inside the overlap region
    (4.0, (0.5, 0.5), (0.5, 0.5), 1),       # one layer: the self-energy
    (3.0, (1.0, -1.5), (0.0, 0.0), 1),      # uniform in the plane: 2 n^2, whatever Z
])
def test_layer_energy_closed_form(orc, Z, zc, a, m):
    psi, q, L = layers(GRID, a, zc, SIGMA, m)
    t = orc.heval(GRID, unit_dipolar(Z), psi)[0]
    s = math.sqrt(2.0) * SIGMA
    for (i, j) in ((0, 1), (0, 0), (1, 1)):
        dz = zc[i] - zc[j]
        X = (kbar(0.0, dz, s, Z) + 0.5 * a[i] * a[j] * kbar(q, dz, s, Z)) / (L[0] * L[1])
        got = 2.0 * t["E_dd"][i][j]            # E_dd[i][j] = 1/2 N_i Gdd_ij int n_i Phi_j
        assert abs(got - X) <= 1e-12 * max(abs(X), 1e-3), (i, j, got, X)


def test_cut_removes_the_interaction_beyond_Z(orc):
    """Layers 4 apart with Z = 1: only Gaussian tails reach |u| < Z."""
    psi, q, L = layers(GRID, (0.8, 0.8), (2.0, -2.0), 0.3, 1)
    t = orc.heval(GRID, unit_dipolar(1.0), psi)[0]
    full = orc.heval(GRID, unit_dipolar(8.0), psi)[0]
    assert abs(t["E_dd"][0][1]) < 1e-13 * t["E_dd"][0][0]        # round-off of the layers' own energies
    assert abs(full["E_dd"][0][1]) > 1e-2 * t["E_dd"][0][0]


def test_slab_cut_needs_the_kernel_inside_one_period(orc):
    psi, _, _ = layers(GRID, (0.0, 0.0), (0.0, 0.0), SIGMA, 1)
    with pytest.raises(RuntimeError, match="EINVAL"):
        orc.heval(GRID, unit_dipolar(8.5), psi)
