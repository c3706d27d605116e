"""Synthetic physics tables and their binary blob.

The paper loads its cross sections per interaction, material and energy from
data files before any transport starts (Sec. 2.2) and keeps them read-only on
the device (Sec. 2.3).  Those files (DPM's PENELOPE-derived data) are not
available, so this module writes a stand-in: closed-form textbook models for
the processes DPM simulates (Sec. 2.1), tabulated in FP64 on one shared
logarithmic energy grid.  The tables are *input data* to the transport, in the
same role as the paper's files; the transport itself (interpolation, majorant,
range inversion, sampling) is implemented separately by each consumer.

Quantities per material, per gram (the order is the blob's quantity index):

  0  mu_C/rho     Klein-Nishina Compton attenuation            cm^2/g
  1  mu_pe/rho    photoelectric, Z^4/E^3 model                 cm^2/g
  2  mu_pp/rho    pair production above 2 m c^2                cm^2/g
  3  R            restricted CSDA range                        g/cm^2
  4  1/(lambda1 rho)  elastic transport cross section          cm^2/g
  5  Sigma_M/rho  hard Moller cross section (W > W_cc)         cm^2/g
  6  Sigma_B/rho  hard bremsstrahlung cross section (W > W_cr) cm^2/g
  7  L_r/rho      restricted total stopping power              MeV cm^2/g
  8  mu_R/rho     Rayleigh (coherent) scattering, screened     cm^2/g
                  Thomson law (zero unless the tables enable it)
  9  1/(lambda2 rho)  second transport cross section (elastic)   cm^2/g
 10  R+           restricted CSDA range of positrons            g/cm^2
 11  Sigma_Bh/rho hard Bhabha cross section (W > W_cc)         cm^2/g
 12  L_r+/rho     restricted total stopping power of positrons  MeV cm^2/g
                  (10-12 are used when the tables enable Bhabha scattering;
                  otherwise positrons take the electron quantities)

Absorption energies are 200 keV (electrons) and 50 keV (photons) (Sec. 3);
the production thresholds W_cc and W_cr are taken equal to them.
"""
from __future__ import annotations

import math
import struct
from dataclasses import dataclass, field

import numpy as np
from scipy import integrate, optimize

# CODATA 2018
MC2 = 0.51099895                # electron rest energy, MeV
R_E = 2.8179403262e-13          # classical electron radius, cm
N_A = 6.02214076e23             # 1/mol
ALPHA = 1.0 / 137.035999084
HBARC = 1.973269804e-11         # MeV cm
A0 = 5.29177210903e-9           # Bohr radius, cm
MEV_PER_G_TO_GY = 1.602176634e-10

# Model constants of the synthetic processes.
C_PE = 1.213e-8                 # cm^2 MeV^3 / g, photoelectric
C_PP = 8.722e-4                 # cm^2 / g, pair
K_B = 5.07e-3                   # cm^2 / g, bremsstrahlung

N_E = 512
E_MIN = 1.0e-3                  # MeV
E_MAX = 20.0                    # MeV
N_Q = 13

(Q_MU_C, Q_MU_PE, Q_MU_PP, Q_RANGE, Q_LAMBDA1_INV, Q_SIGMA_M, Q_SIGMA_B, Q_L_R, Q_MU_R, Q_LAMBDA2_INV,
 Q_RANGE_POS, Q_SIGMA_BH, Q_L_R_POS) = range(13)
QUANTITY_NAMES = ("mu_C", "mu_pe", "mu_pp", "R", "lambda1_inv", "Sigma_M", "Sigma_B", "L_r", "mu_R",
                  "lambda2_inv", "R_pos", "Sigma_Bh", "L_r_pos")

BLOB_MAGIC = b"MCDTAB\x00\x01"
BLOB_VERSION = 4
FLAG_NO_HARD = 1                 # test variant: Sigma_M = Sigma_B = 0, unrestricted losses
FLAG_PE_ONLY = 2                 # test variant: photons interact only by photoabsorption
FLAG_ANGULAR = 4                 # emission angles of photoelectrons, bremsstrahlung photons
                                 # and pair leptons (same tables, different samplers)
FLAG_DENSITY = 8                 # collision stopping power with the density effect
                                 # (tables only: range and total stopping power change)
FLAG_RAYLEIGH = 16               # Rayleigh scattering tabulated (mu_R > 0)
FLAG_HINGE2 = 32                 # hinge angle matches the second Lewis moment too
FLAG_BHABHA = 64                 # positrons: Bhabha events and positron stopping power

E_ABS_E = 0.2                   # MeV
E_ABS_G = 0.05                  # MeV
KAPPA_STEP = 0.1
F_E = 0.2


@dataclass(frozen=True)
class Material:
    """Effective-atom description of a material (per-gram sums over elements)."""
    name: str
    rho: float          # nominal density, g/cm^3
    zoa: float          # Z/A
    i_ev: float         # mean excitation energy, eV
    b: float            # sum w Z^2/A
    ee: float           # sum w Z(Z+1)/A
    p: float            # sum w Z^4/A

    @property
    def zs(self) -> float:
        """Effective screening charge Z_s = B / (Z/A)."""
        return self.b / self.zoa


MATERIALS = (
    Material("air", 0.0012, 0.4991, 85.7, 3.673, 4.172, 222.4),
    # Lung: water composition at its own density.
    Material("lung", 0.26, 0.5551, 75.0, 3.664, 4.219, 227.5),
    Material("water", 1.00, 0.5551, 75.0, 3.664, 4.219, 227.5),
    Material("bone", 1.85, 0.5148, 106.4, 5.420, 5.935, 1210.0),
)
MAT_AIR, MAT_LUNG, MAT_WATER, MAT_BONE = range(4)


def water_bone_mixture(name: str, rho: float, w_bone: float) -> Material:
    """Effective atom of a mass fraction w_bone of bone in water: the per-gram
    sums (Z/A, B, Z(Z+1)/A, P) add by mass fraction, and ln I by Bragg's
    additivity rule, weighted by each part's electrons per gram."""
    a, b = MATERIALS[MAT_WATER], MATERIALS[MAT_BONE]
    wa = 1.0 - w_bone

    def lin(x, y):
        return wa * x + w_bone * y
    zoa = lin(a.zoa, b.zoa)
    ln_i = (wa * a.zoa * math.log(a.i_ev) + w_bone * b.zoa * math.log(b.i_ev)) / zoa
    return Material(name, rho, zoa, math.exp(ln_i), lin(a.b, b.b), lin(a.ee, b.ee), lin(a.p, b.p))


# Eight tissue classes of a CT-derived phantom: the four materials above plus
# adipose and muscle (water's atom at their densities), cartilage and
# spongiosa (10% and 40% of bone in water).  Eight materials is the most the
# device holds per table set; their tables (128 KiB in FP32) no longer leave
# room for two copies in a CU's LDS.
TISSUES8 = MATERIALS + (water_bone_mixture("adipose", 0.95, 0.0), water_bone_mixture("muscle", 1.05, 0.0),
                        water_bone_mixture("cartilage", 1.10, 0.1), water_bone_mixture("spongiosa", 1.18, 0.4))
MAT_ADIPOSE, MAT_MUSCLE, MAT_CARTILAGE, MAT_SPONGIOSA = range(4, 8)

# Elemental compositions (Z, A in g/mol, mass fraction) behind the effective
# atoms above, used where a quantity is summed element by element.  Air is
# dry air near sea level and water is H2O (their sums reproduce the effective
# atoms to 0.1%).  The bone of these synthetic tables is no tabulated tissue:
# its H, C, O and Ca fractions are the ones whose sum of w, w Z/A, w Z^2/A and
# w Z^4/A equal 1 and the bone atom's Z/A, B and P.
COMPOSITIONS = {
    "air": ((6, 12.0107, 0.000124), (7, 14.0067, 0.755268), (8, 15.9994, 0.231781),
            (18, 39.948, 0.012827)),
    "lung": ((1, 1.00794, 0.111894), (8, 15.9994, 0.888106)),
    "water": ((1, 1.00794, 0.111894), (8, 15.9994, 0.888106)),
    "bone": ((1, 1.00794, 0.030593), (6, 12.0107, 0.036078), (8, 15.9994, 0.674474),
             (20, 40.078, 0.258855)),
}


def energy_grid() -> np.ndarray:
    """E_i = E_min (E_max/E_min)^(i/511), i = 0..511 (MeV)."""
    i = np.arange(N_E, dtype=np.float64)
    return E_MIN * (E_MAX / E_MIN) ** (i / (N_E - 1))


# ----------------------------------------------------------------- photons

def sigma_kn(e: float) -> float:
    """Klein-Nishina total cross section per free electron (cm^2)."""
    k = e / MC2
    if k < 1e-4:
        # Series about k = 0: sigma_T (1 - 2k + 26k^2/5 - ...), avoids cancellation.
        return 8.0 * math.pi * R_E ** 2 / 3.0 * (1.0 - 2.0 * k + 5.2 * k * k - 13.3 * k ** 3)
    l = math.log1p(2.0 * k)
    t1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k)
    t2 = l / (2.0 * k)
    t3 = (1.0 + 3.0 * k) / (1.0 + 2.0 * k) ** 2
    return 2.0 * math.pi * R_E ** 2 * (t1 + t2 - t3)


def mu_compton(m: Material, e: float) -> float:
    return N_A * m.zoa * sigma_kn(e)


def mu_photo(m: Material, e: float) -> float:
    return C_PE * m.p / e ** 3


def rayleigh_b_coeff(m: Material) -> float:
    """b / E^2 of the Rayleigh form factor (MeV^-2): with the screening radius
    a = 0.885 a0 Z_s^(-1/3) and k = E / (hbar c), b = 2 (k a)^2, and
    q^2 a^2 = b (1 - cos)."""
    a = 0.885 * A0 * m.zs ** (-1.0 / 3.0)
    return 2.0 * a * a / (HBARC * HBARC)


def rayleigh_integral_quad(b: float) -> float:
    """I(b) = int_{-1}^{1} (1 + c^2) (1 + b (1 - c))^-4 dc by adaptive
    quadrature in s = 1 - c (break points where the form factor falls)."""
    pts = [p for p in (0.1 / b, 1.0 / b, 10.0 / b) if 0.0 < p < 2.0] if b > 0 else None
    f = lambda s: (1.0 + (1.0 - s) ** 2) * (1.0 + b * s) ** -4
    val, _ = integrate.quad(f, 0.0, 2.0, points=pts, epsabs=0.0, epsrel=1e-12, limit=400)
    return val


def rayleigh_integral_closed(b: float) -> float:
    """The same integral in closed form: with v = 1 + b s the integrand is a
    sum of powers of v, so I = [G(v)] from v = 1 to 1 + 2b over b, with
    G(v) = -(2/3 + 2/(3b) + 1/(3b^2)) v^-3 + (1/b + 1/b^2) v^-2 - v^-1 / b^2.
    Exact, but it cancels for small b."""
    def g(v):
        return (-(2.0 / 3.0 + 2.0 / (3.0 * b) + 1.0 / (3.0 * b * b)) / v ** 3
                + (1.0 / b + 1.0 / (b * b)) / v ** 2 - 1.0 / (b * b * v))
    return (g(1.0 + 2.0 * b) - g(1.0)) / b


def rayleigh_integral(b: float) -> float:
    """I(b): quadrature where the form factor is broad, closed form where it
    is sharp (b >= 1)."""
    return rayleigh_integral_closed(b) if b >= 1.0 else rayleigh_integral_quad(b)


def mu_rayleigh(m: Material, e: float) -> float:
    """Coherent scattering of the Z electrons of each atom: per atom
    dsigma/dOmega = (r_e^2 / 2)(1 + cos^2) Z^2 F(q)^2 with the screened form
    factor F = (1 + q^2 a^2)^-2; per gram N_A B pi r_e^2 I(b).  As E -> 0 it
    tends to Z^2 times the Thomson cross section."""
    return N_A * m.b * math.pi * R_E ** 2 * rayleigh_integral(rayleigh_b_coeff(m) * e * e)


def mu_pair(m: Material, e: float) -> float:
    thr = 2.0 * MC2
    if e <= thr:
        return 0.0
    g = (1.0 - thr / e) ** 3 * math.log1p(e / thr)
    return C_PP * m.b * g


# --------------------------------------------------------------- electrons

def _kin(t: float):
    tau = t / MC2
    pc = math.sqrt(t * (t + 2.0 * MC2))
    beta2 = (pc / (t + MC2)) ** 2
    return tau, pc, beta2


LN10 = math.log(10.0)
GAS_DENSITY = 0.01               # g/cm^3: below it a material takes the gas rules


def density_effect_params(m: Material):
    """Sternheimer-Peierls general parameters of the density-effect correction
    for a material at its nominal density (no conduction electrons):
      plasma energy  h w_p = 28.816 sqrt(rho Z/A) eV,
      C = 2 ln(I / h w_p) + 1,
      (X0, X1) from C by the rules for condensed materials (I below or above
      100 eV) or for gases, exponent k = 3, and a = (C - 2 ln10 X0) / (X1 - X0)^k
      so that the correction starts continuously at X0.
    Returns (C, X0, X1, a, k)."""
    hwp = 28.816 * math.sqrt(m.rho * m.zoa)
    c = 2.0 * math.log(m.i_ev / hwp) + 1.0
    if m.rho < GAS_DENSITY:
        rules = ((10.0, 1.6, 4.0), (10.5, 1.7, 4.0), (11.0, 1.8, 4.0), (11.5, 1.9, 4.0),
                 (12.25, 2.0, 4.0), (13.804, 2.0, 5.0))
        x0, x1 = 0.326 * c - 2.5, 5.0
        for c_top, x0_r, x1_r in rules:
            if c < c_top:
                x0, x1 = x0_r, x1_r
                break
    elif m.i_ev < 100.0:
        x1 = 2.0
        x0 = 0.2 if c < 3.681 else 0.326 * c - 1.0
    else:
        x1 = 3.0
        x0 = 0.2 if c < 5.215 else 0.326 * c - 1.5
    k = 3.0
    a = (c - 2.0 * LN10 * x0) / (x1 - x0) ** k
    return c, x0, x1, a, k


def density_delta(m: Material, t: float) -> float:
    """Density-effect correction delta at kinetic energy t, as a function of
    X = log10(p / (m c)):  0 below X0,  2 ln10 X - C + a (X1 - X)^k up to X1,
    2 ln10 X - C above."""
    c, x0, x1, a, k = density_effect_params(m)
    x = math.log10(math.sqrt(t * (t + 2.0 * MC2)) / MC2)
    if x < x0:
        return 0.0
    d = 2.0 * LN10 * x - c
    return d + a * (x1 - x) ** k if x < x1 else d


def l_col(m: Material, t: float, w_cut: float | None, density: bool = False) -> float:
    """Bethe collision stopping power with Moller F-, restricted to energy losses
    below w_cut (None: unrestricted); with `density`, less the density-effect
    correction delta of the material at its nominal density."""
    tau, _, beta2 = _kin(t)
    dmax = t / 2.0
    w = dmax if w_cut is None else min(w_cut, dmax)
    d = w / MC2
    i_mc2 = m.i_ev * 1e-6 / MC2
    f = (-1.0 - beta2 + math.log((tau - d) * d) + tau / (tau - d)
         + (d * d / 2.0 + (2.0 * tau + 1.0) * math.log1p(-d / tau)) / (tau + 1.0) ** 2)
    pref = 2.0 * math.pi * R_E ** 2 * MC2 * N_A * m.zoa / beta2
    delta = density_delta(m, t) if density else 0.0
    return pref * (math.log(2.0 * (tau + 2.0) / i_mc2 ** 2) + f - delta)


def l_col_positron(m: Material, t: float, w_cut: float | None, density: bool = False) -> float:
    """Bethe collision stopping power of positrons with the Bhabha term
    (Seltzer and Berger's restricted form), restricted to energy losses below
    w_cut (None: unrestricted; a positron can lose all of t).  With
    d = min(w_cut, t) / m c^2, y = 1 / (tau + 2):
      ln(2 (tau + 2) / (I/mc^2)^2) + ln(tau d)
        - (beta^2 / tau) [tau + 2d - y (3d^2/2 + y (d - d^3/3 + y (d^2/2 - tau d^3/3 + d^4/4)))]
    which at d = tau is ln(tau^2 (tau + 2) / (2 (I/mc^2)^2)) + F+(tau) with
    F+ = 2 ln 2 - (beta^2 / 12) (23 + 14 y + 10 y^2 + 4 y^3)."""
    tau, _, beta2 = _kin(t)
    w = t if w_cut is None else min(w_cut, t)
    d = w / MC2
    y = 1.0 / (tau + 2.0)
    i_mc2 = m.i_ev * 1e-6 / MC2
    poly = tau + 2.0 * d - y * (1.5 * d * d + y * (d - d ** 3 / 3.0
                                                   + y * (d * d / 2.0 - tau * d ** 3 / 3.0 + d ** 4 / 4.0)))
    pref = 2.0 * math.pi * R_E ** 2 * MC2 * N_A * m.zoa / beta2
    delta = density_delta(m, t) if density else 0.0
    return pref * (math.log(2.0 * (tau + 2.0) / i_mc2 ** 2) + math.log(tau * d) - beta2 / tau * poly - delta)


def bhabha_coeffs(t: float):
    """b1..b4 of the Bhabha cross section for a positron of kinetic energy t:
    dsigma/dW = (2 pi r_e^2 m c^2 / beta^2) W^-2 [1 - b1 e + b2 e^2 - b3 e^3 + b4 e^4],
    e = W / t (W the energy given to the electron, 0 < W < t)."""
    g = 1.0 + t / MC2
    a = ((g - 1.0) / g) ** 2
    return (a * (2.0 * (g + 1.0) ** 2 - 1.0) / (g * g - 1.0),
            a * (3.0 * (g + 1.0) ** 2 + 1.0) / (g + 1.0) ** 2,
            a * 2.0 * g * (g - 1.0) / (g + 1.0) ** 2,
            a * (g - 1.0) ** 2 / (g + 1.0) ** 2)


def sigma_bhabha_hard(m: Material, t: float, w_cc: float) -> float:
    """Bhabha cross section per gram for energy transfers above w_cc, in closed
    form: (1/t) int_{e_c}^1 e^-2 [1 - b1 e + ...] de, e_c = w_cc / t."""
    if t <= w_cc:
        return 0.0
    _, _, beta2 = _kin(t)
    b1, b2, b3, b4 = bhabha_coeffs(t)
    ec = w_cc / t
    br = (1.0 / ec - 1.0) + b1 * math.log(ec) + b2 * (1.0 - ec) - b3 * (1.0 - ec * ec) / 2.0 \
        + b4 * (1.0 - ec ** 3) / 3.0
    return N_A * m.zoa * 2.0 * math.pi * R_E ** 2 * MC2 / (beta2 * t) * br


def l_rad(m: Material, t: float, w_cut: float | None) -> float:
    """Radiative stopping power of the flat W dsigma/dW model, restricted to W < w_cut."""
    w = t if w_cut is None else min(w_cut, t)
    return K_B * m.b * (t + MC2) / t * w


def sigma_brems_hard(m: Material, t: float, w_cr: float) -> float:
    if t <= w_cr:
        return 0.0
    return K_B * m.b * (t + MC2) / t * math.log(t / w_cr)


def sigma_moller_hard(m: Material, t: float, w_cc: float) -> float:
    if t <= 2.0 * w_cc:
        return 0.0
    tau, _, beta2 = _kin(t)
    e0 = w_cc / t
    g = tau / (tau + 1.0)
    c = (2.0 * tau + 1.0) / (tau + 1.0) ** 2
    br = 1.0 / e0 - 1.0 / (1.0 - e0) + g * g * (0.5 - e0) - c * math.log((1.0 - e0) / e0)
    return N_A * m.zoa * 2.0 * math.pi * R_E ** 2 * MC2 / (beta2 * t) * br


def screening_charge(zs: float, t: float) -> float:
    """Moliere's screening parameter of an atom of charge zs for an electron of
    kinetic energy t: Thomas-Fermi radius 0.885 a0 zs^(-1/3), with his
    correction factor 1.13 + 3.76 (alpha zs / beta)^2."""
    _, pc, beta2 = _kin(t)
    beta = math.sqrt(beta2)
    return 0.25 * (HBARC / (0.885 * A0 * pc)) ** 2 * zs ** (2.0 / 3.0) * (
        1.13 + 3.76 * (ALPHA * zs / beta) ** 2)


def screening_moliere(m: Material, t: float) -> float:
    return screening_charge(m.zs, t)


def lambda1_inv(m: Material, t: float) -> float:
    """Transport cross section per gram of the screened-Rutherford (Wentzel) model."""
    _, pc, beta2 = _kin(t)
    a = screening_moliere(m, t)
    k = (R_E * MC2 / (math.sqrt(beta2) * pc)) ** 2
    return N_A * m.ee * 2.0 * math.pi * k * (math.log1p(1.0 / a) - 1.0 / (1.0 + a))


def lambda2_inv(m: Material, t: float) -> float:
    """Second transport cross section per gram of the same model,
    int (1 - P2(cos)) dsigma: with mu = (1 - cos)/2, 1 - P2 = 6 mu (1 - mu) and
    int_0^1 6 mu (1 - mu) / (mu + a)^2 dmu = 6 [(1 + 2a) ln(1 + 1/a) - 2]."""
    _, pc, beta2 = _kin(t)
    a = screening_moliere(m, t)
    k = (R_E * MC2 / (math.sqrt(beta2) * pc)) ** 2
    return N_A * m.ee * 2.0 * math.pi * k * 3.0 * ((1.0 + 2.0 * a) * math.log1p(1.0 / a) - 2.0)


def lambda1_inv_elements(comp, t: float) -> float:
    """1/(lambda1 rho) with each element screened by its own charge: the
    screened-Rutherford transport cross section summed over the elements
    (Z, A, w) of comp, each with the screening parameter of its Z."""
    _, pc, beta2 = _kin(t)
    k = (R_E * MC2 / (math.sqrt(beta2) * pc)) ** 2
    acc = 0.0
    for z, a_mol, w in comp:
        a = screening_charge(float(z), t)
        acc += w / a_mol * z * (z + 1) * (math.log1p(1.0 / a) - 1.0 / (1.0 + a))
    return N_A * 2.0 * math.pi * k * acc


def lambda2_inv_elements(comp, t: float) -> float:
    """1/(lambda2 rho) summed element by element, as lambda1_inv_elements."""
    _, pc, beta2 = _kin(t)
    k = (R_E * MC2 / (math.sqrt(beta2) * pc)) ** 2
    acc = 0.0
    for z, a_mol, w in comp:
        a = screening_charge(float(z), t)
        acc += w / a_mol * z * (z + 1) * ((1.0 + 2.0 * a) * math.log1p(1.0 / a) - 2.0)
    return N_A * 2.0 * math.pi * k * 3.0 * acc


def solve_a_hinge(kappa_step: float) -> float:
    """Screening A of the hinge's Wentzel angle whose mean mu equals the Lewis
    first moment of a step of kappa_step transport mean free paths:
    A[(1+A) ln((1+A)/A) - 1] = (1 - exp(-kappa_step)) / 2."""
    target = 0.5 * (1.0 - math.exp(-kappa_step))

    def mean_mu(a):
        return a * ((1.0 + a) * math.log((1.0 + a) / a) - 1.0)

    return optimize.brentq(lambda a: mean_mu(a) - target, 1e-12, 10.0, xtol=1e-16, rtol=1e-15)


# ------------------------------------------------------------------ tables

@dataclass
class Tables:
    """FP64 tables for every material plus the scalars the transport needs."""
    energies: np.ndarray
    data: np.ndarray                     # [n_mat, N_Q, N_E]
    materials: tuple = MATERIALS
    e_abs_e: float = E_ABS_E
    e_abs_g: float = E_ABS_G
    w_cc: float = E_ABS_E
    w_cr: float = E_ABS_G
    kappa_step: float = KAPPA_STEP
    f_e: float = F_E
    a_hinge: float = 0.0
    flags: int = 0

    def to_blob(self) -> bytes:
        return write_blob(self)


def _range_table(m: Material, e: np.ndarray, lr, kinks=(E_ABS_G, 2.0 * E_ABS_E)) -> np.ndarray:
    """R(E_i) = R_0 + int_{E_0}^{E_i} dT / L_r(T), R_0 = E_0 / L_r(E_0), by adaptive
    quadrature over each grid interval (kinks of L_r are passed as break points)."""
    r = np.empty_like(e)
    r[0] = e[0] / lr(e[0])
    for i in range(1, len(e)):
        a, b = e[i - 1], e[i]
        pts = [k for k in kinks if a < k < b]
        val, err = integrate.quad(lambda t: 1.0 / lr(t), a, b, points=pts or None,
                                  epsabs=0.0, epsrel=1e-13, limit=200)
        r[i] = r[i - 1] + val
    return r


def build_tables(materials=MATERIALS, variant: str = "standard", kappa_step: float = KAPPA_STEP) -> Tables:
    """Tabulate every quantity at the 512 grid nodes.

    variant:
      "standard"  restricted losses, hard Moller and bremsstrahlung events;
      "no_hard"   no hard events: unrestricted stopping power, Sigma_M = Sigma_B = 0
                  (the CSDA-track-length test case);
      "pe_only"   standard electrons, photons interact only by photoabsorption;
      "angular"   standard tables; photoelectrons leave at Sauter angles,
                  bremsstrahlung photons and pair leptons at forward-peaked
                  angles instead of along their parent;
      "density"   standard, with the density effect in the collision stopping
                  power (and so in the range);
      "rayleigh"  standard, with Rayleigh scattering tabulated;
      "hinge2"    standard tables; the hinge angle matches the second Lewis
                  moment exp(-s/lambda2) as well as the first;
      "bhabha"    standard tables; positrons take their own stopping power
                  and range and hard Bhabha events instead of Moller ones;
      "elements"  standard, with the elastic transport cross sections 1/lambda1
                  and 1/lambda2 summed element by element over COMPOSITIONS,
                  each element screened by its own charge (tables only; the
                  blob carries no flag for it);
      "refined"   every refinement above except "elements": angular, density,
                  rayleigh, hinge2, bhabha.
    The positron quantities are tabulated for every variant.
    """
    e = energy_grid()
    n_mat = len(materials)
    data = np.zeros((n_mat, N_Q, N_E))
    flags = 0
    if variant == "no_hard":
        flags |= FLAG_NO_HARD
    elif variant == "pe_only":
        flags |= FLAG_PE_ONLY
    elif variant == "angular":
        flags |= FLAG_ANGULAR
    elif variant == "density":
        flags |= FLAG_DENSITY
    elif variant == "rayleigh":
        flags |= FLAG_RAYLEIGH
    elif variant == "hinge2":
        flags |= FLAG_HINGE2
    elif variant == "bhabha":
        flags |= FLAG_BHABHA
    elif variant == "elements":
        pass
    elif variant == "refined":
        flags |= FLAG_ANGULAR | FLAG_DENSITY | FLAG_RAYLEIGH | FLAG_HINGE2 | FLAG_BHABHA
    elif variant != "standard":
        raise ValueError(f"unknown table variant {variant!r}")
    w_cc = None if flags & FLAG_NO_HARD else E_ABS_E
    w_cr = None if flags & FLAG_NO_HARD else E_ABS_G
    per_element = variant == "elements"
    for mi, m in enumerate(materials):
        dens = bool(flags & FLAG_DENSITY)
        if per_element and m.name not in COMPOSITIONS:
            raise ValueError(f"no elemental composition for material {m.name!r}")
        comp = COMPOSITIONS.get(m.name)

        def lr(t, m=m, dens=dens):
            return l_col(m, t, w_cc, dens) + l_rad(m, t, w_cr)

        def lr_pos(t, m=m, dens=dens):
            return l_col_positron(m, t, w_cc, dens) + l_rad(m, t, w_cr)
        for i, ei in enumerate(e):
            if not flags & FLAG_PE_ONLY:
                data[mi, Q_MU_C, i] = mu_compton(m, ei)
                data[mi, Q_MU_PP, i] = mu_pair(m, ei)
                if flags & FLAG_RAYLEIGH:
                    data[mi, Q_MU_R, i] = mu_rayleigh(m, ei)
            data[mi, Q_MU_PE, i] = mu_photo(m, ei)
            if per_element:
                data[mi, Q_LAMBDA1_INV, i] = lambda1_inv_elements(comp, ei)
                data[mi, Q_LAMBDA2_INV, i] = lambda2_inv_elements(comp, ei)
            else:
                data[mi, Q_LAMBDA1_INV, i] = lambda1_inv(m, ei)
                data[mi, Q_LAMBDA2_INV, i] = lambda2_inv(m, ei)
            if not flags & FLAG_NO_HARD:
                data[mi, Q_SIGMA_M, i] = sigma_moller_hard(m, ei, E_ABS_E)
                data[mi, Q_SIGMA_B, i] = sigma_brems_hard(m, ei, E_ABS_G)
            data[mi, Q_L_R, i] = lr(ei)
            data[mi, Q_L_R_POS, i] = lr_pos(ei)
            if not flags & FLAG_NO_HARD:
                data[mi, Q_SIGMA_BH, i] = sigma_bhabha_hard(m, ei, E_ABS_E)
        data[mi, Q_RANGE] = _range_table(m, e, lr)
        data[mi, Q_RANGE_POS] = _range_table(m, e, lr_pos, kinks=(E_ABS_G, E_ABS_E))
    return Tables(energies=e, data=data, materials=tuple(materials),
                  kappa_step=kappa_step, a_hinge=solve_a_hinge(kappa_step), flags=flags)


# -------------------------------------------------------------------- blob
#
# Little-endian layout:
#   char[8]  magic "MCDTAB\0\1"
#   u32      version, n_mat, n_e, n_q
#   f64      e_min, e_max, e_abs_e, e_abs_g, w_cc, w_cr, kappa_step, f_e, a_hinge
#   u32      flags, reserved
#   n_mat x { char[16] name; f64 rho, zoa, i_ev, b, ee, p; f64 q[n_q][n_e] }

_HDR = struct.Struct("<8s4I9d2I")
_MAT = struct.Struct("<16s6d")


def write_blob(t: Tables) -> bytes:
    n_mat = t.data.shape[0]
    out = bytearray(_HDR.pack(BLOB_MAGIC, BLOB_VERSION, n_mat, N_E, N_Q,
                              t.energies[0], t.energies[-1], t.e_abs_e, t.e_abs_g,
                              t.w_cc, t.w_cr, t.kappa_step, t.f_e, t.a_hinge, t.flags, 0))
    for mi in range(n_mat):
        m = t.materials[mi]
        out += _MAT.pack(m.name.encode()[:15], m.rho, m.zoa, m.i_ev, m.b, m.ee, m.p)
        out += np.ascontiguousarray(t.data[mi], dtype="<f8").tobytes()
    return bytes(out)


def read_blob(blob: bytes) -> Tables:
    (magic, ver, n_mat, n_e, n_q, emin, emax, eae, eag, wcc, wcr, ks, fe, ah, flags,
     _) = _HDR.unpack_from(blob, 0)
    if magic != BLOB_MAGIC or ver != BLOB_VERSION or n_e != N_E or n_q != N_Q:
        raise ValueError(f"not a version-{BLOB_VERSION} table blob")
    off = _HDR.size
    mats, data = [], np.empty((n_mat, n_q, n_e))
    for mi in range(n_mat):
        name, rho, zoa, iev, b, ee, p = _MAT.unpack_from(blob, off)
        off += _MAT.size
        mats.append(Material(name.rstrip(b"\0").decode(), rho, zoa, iev, b, ee, p))
        data[mi] = np.frombuffer(blob, dtype="<f8", count=n_q * n_e, offset=off).reshape(n_q, n_e)
        off += 8 * n_q * n_e
    return Tables(energies=energy_grid(), data=data, materials=tuple(mats), e_abs_e=eae,
                  e_abs_g=eag, w_cc=wcc, w_cr=wcr, kappa_step=ks, f_e=fe, a_hinge=ah,
                  flags=flags)


_CACHE: dict = {}


def standard_blob(variant: str = "standard", kappa_step: float = KAPPA_STEP) -> bytes:
    """The blob for the four standard materials (memoised; generation takes ~1 s)."""
    key = (variant, kappa_step)
    if key not in _CACHE:
        _CACHE[key] = build_tables(variant=variant, kappa_step=kappa_step).to_blob()
    return _CACHE[key]


def tissue_blob() -> bytes:
    """The standard blob for the eight tissue classes TISSUES8 (memoised)."""
    key = ("tissues8",)
    if key not in _CACHE:
        _CACHE[key] = build_tables(materials=TISSUES8).to_blob()
    return _CACHE[key]
