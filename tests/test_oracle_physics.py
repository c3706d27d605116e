"""Pins of the oracle's transport against closed forms, exact invariants and
textbook distributions (Woodcock tracking, samplers, CSDA range, energy
conservation, density scaling, symmetry and additivity)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from paper_0910_0329_amd.inputs import phantoms, sources
from paper_0910_0329_amd.inputs import tables as T
from paper_0910_0329_amd.inputs.sources import ELECTRON, PHOTON, POSITRON


def mu_total(m, e, rho):
    mat = T.MATERIALS[m]
    return rho * (T.mu_compton(mat, e) + T.mu_photo(mat, e) + T.mu_pair(mat, e))


# ------------------------------------------------------------ Woodcock

@pytest.mark.parametrize("e", [0.1, 1.0, 6.0, 20.0])
def test_narrow_beam_transmission_homogeneous_water(blob, e):
    """Uncollided fraction beyond depth x equals exp(-mu x)."""
    ph = phantoms.homogeneous(8, 8, 80, 0.5)            # 40 cm deep
    x, y = ph.centre_xy()
    n = 200_000
    z = oracle.first_interaction(blob, ph, sources.pencil(PHOTON, e, x + 0.1, y + 0.1), n, seed=11)
    mu = mu_total(T.MAT_WATER, e, 1.0)
    for depth in (1.0, 10.0, 30.0):
        p = math.exp(-mu * depth)
        phat = np.mean(z > depth)
        assert abs(phat - p) <= 4 * math.sqrt(p * (1 - p) / n) + 1e-12, (e, depth, phat, p)


def test_narrow_beam_transmission_slabs_with_virtual_events(blob):
    """Water-lung-water along z with one bone voxel off the beam: the bone raises
    the majorant so most stops in water and lung are virtual."""
    ph = phantoms.slab_phantom(8, 8, 0.5, 0.5, [(10, T.MAT_WATER, 1.0), (20, T.MAT_LUNG, 0.26),
                                                (30, T.MAT_WATER, 1.0)], 0.5)
    ph.mat[0, 0, 0] = T.MAT_BONE
    ph.rho[0, 0, 0] = 1.85
    x, y = ph.centre_xy()
    n = 200_000
    for e in (0.2, 2.0):
        z = oracle.first_interaction(blob, ph, sources.pencil(PHOTON, e, x + 0.1, y + 0.1), n, seed=12)
        mw, ml = mu_total(T.MAT_WATER, e, 1.0), mu_total(T.MAT_LUNG, e, 0.26)
        for depth, tau in ((4.0, 4.0 * mw), (12.0, 5.0 * mw + 7.0 * ml), (25.0, 5 * mw + 10 * ml + 10 * mw)):
            p = math.exp(-tau)
            phat = np.mean(z > depth)
            assert abs(phat - p) <= 4 * math.sqrt(p * (1 - p) / n), (e, depth, phat, p)
    r = oracle.simulate(blob, ph, sources.pencil(PHOTON, 2.0, x + 0.1, y + 0.1), 2000, seed=3)
    assert r["cnt"]["virtual"] > r["cnt"]["compton"]


@pytest.mark.parametrize("e,m", [(0.08, T.MAT_BONE), (1.5, T.MAT_WATER), (12.0, T.MAT_BONE)])
def test_interaction_branching_ratios(blob, e, m):
    """The kind of the first real interaction follows mu_C : mu_pe : mu_pp."""
    rho = 1.85 if m == T.MAT_BONE else 1.0
    ph = phantoms.homogeneous(8, 8, 400, 0.5, material=m, density=rho)
    x, y = ph.centre_xy()
    n = 100_000
    _, kind = oracle.first_interaction(blob, ph, sources.pencil(PHOTON, e, x + 0.1, y + 0.1), n,
                                       seed=13, kinds=True)
    mat = T.MATERIALS[m]
    mus = np.array([T.mu_compton(mat, e), T.mu_photo(mat, e), T.mu_pair(mat, e)])
    p = mus / mus.sum()
    inter = kind[kind != 6]
    for code, pk in zip((2, 3, 4), p):
        phat = np.mean(inter == code)
        assert abs(phat - pk) <= 4 * math.sqrt(pk * (1 - pk) / len(inter)) + 1e-9, (code, phat, pk)


@pytest.mark.parametrize("e,m", [(0.02, T.MAT_WATER), (0.03, T.MAT_BONE), (0.08, T.MAT_BONE)])
def test_rayleigh_branching_and_attenuation(e, m):
    """Rayleigh flag: coherent scattering is a fourth real interaction; the
    first one happens at depth distributed as exp(-(mu_C + mu_pe + mu_pp + mu_R) z)
    and its kind follows mu_C : mu_pe : mu_pp : mu_R."""
    blob = T.standard_blob("rayleigh")
    rho = 1.85 if m == T.MAT_BONE else 1.0
    ph = phantoms.homogeneous(8, 8, 400, 0.5, material=m, density=rho)
    x, y = ph.centre_xy()
    n = 100_000
    z, kind = oracle.first_interaction(blob, ph, sources.pencil(PHOTON, e, x + 0.1, y + 0.1), n,
                                       seed=17, kinds=True)
    mat = T.MATERIALS[m]
    mus = np.array([T.mu_compton(mat, e), T.mu_photo(mat, e), T.mu_pair(mat, e), T.mu_rayleigh(mat, e)])
    p = mus / mus.sum()
    assert p[3] > 0.005
    inter = kind[kind != 6]
    for code, pk in zip((2, 3, 4, 8), p):
        phat = np.mean(inter == code)
        assert abs(phat - pk) <= 4 * math.sqrt(pk * (1 - pk) / len(inter)) + 1e-9, (code, phat, pk)
    mu = rho * mus.sum()
    for depth in (0.5 / mu, 1.0 / mu, 2.0 / mu):
        q = math.exp(-mu * depth)
        qhat = np.mean(z > depth)
        assert abs(qhat - q) <= 4 * math.sqrt(q * (1 - q) / n), (depth, qhat, q)


def test_photoabsorption_only_layer_deposits(blob):
    """Photoabsorption-only tables, 0.1 MeV photons (photoelectrons below the
    electron cutoff are absorbed on the spot): the energy deposited in layer
    [z1, z2) is E (exp(-mu z1) - exp(-mu z2)) per photon."""
    b = T.standard_blob("pe_only")
    ph = phantoms.homogeneous(4, 4, 40, 0.5)
    x, y = ph.centre_xy()
    n = 100_000
    r = oracle.simulate(b, ph, sources.pencil(PHOTON, 0.1, x + 0.1, y + 0.1), n, seed=5)
    mu = T.mu_photo(T.MATERIALS[T.MAT_WATER], 0.1)
    layer = r["S"].reshape(40, 4, 4).sum(axis=(1, 2))
    for k in range(0, 40, 3):
        p = math.exp(-mu * 0.5 * k) - math.exp(-mu * 0.5 * (k + 1))
        assert abs(layer[k] / 0.1 / n - p) <= 4 * math.sqrt(p * (1 - p) / n), k
    assert r["cnt"]["compton"] == 0 and r["cnt"]["pair"] == 0


# ------------------------------------------------------------ samplers

def _chi2_pvalue(counts, probs):
    n = counts.sum()
    exp = probs * n
    ok = exp > 5
    chi2 = ((counts[ok] - exp[ok]) ** 2 / exp[ok]).sum()
    return stats.chi2.sf(chi2, ok.sum() - 1)


@pytest.mark.parametrize("e", [0.1, 1.0, 6.0, 20.0])
def test_compton_angles_follow_klein_nishina(blob, e):
    n = 300_000
    out = oracle.sample(blob, 0, e, n, seed=21)
    cost, tau = out[:, 0], out[:, 1]
    k = e / T.MC2
    # kinematics: E'/E = 1 / (1 + k (1 - cos)) per event
    np.testing.assert_allclose(tau, 1.0 / (1.0 + k * (1.0 - cost)), rtol=1e-12)

    def dcs(c):
        r = 1.0 / (1.0 + k * (1.0 - c))
        return r * r * (r + 1.0 / r - (1.0 - c * c))

    edges = np.linspace(-1, 1, 101)
    pb = np.array([integrate.quad(dcs, a, b)[0] for a, b in zip(edges[:-1], edges[1:])])
    pb /= pb.sum()
    counts = np.histogram(cost, edges)[0]
    assert _chi2_pvalue(counts, pb) > 1e-3
    # energy and 3-D momentum conservation of every event (MeV, MeV/c)
    d0 = np.array([0.3, -0.5, 0.8]) / math.sqrt(0.98)
    e1 = tau * e
    te = e - e1
    pe = np.sqrt(te * (te + 2 * T.MC2))
    p_after = e1[:, None] * out[:, 2:5] + pe[:, None] * out[:, 5:8]
    np.testing.assert_allclose(p_after, np.broadcast_to(e * d0, p_after.shape), atol=1e-9 * e)
    np.testing.assert_allclose(out[:, 2:5] @ d0, cost, atol=1e-12)


@pytest.mark.parametrize("t", [0.5, 3.0, 20.0])
def test_moller_sampler_follows_its_dcs(blob, t):
    n = 300_000
    out = oracle.sample(blob, 1, t, n, seed=22)
    eps, cos_d = out[:, 0], out[:, 1]
    e0 = T.E_ABS_E / t
    assert eps.min() >= e0 and eps.max() <= 0.5
    tau = t / T.MC2
    g = (tau / (tau + 1)) ** 2
    c = (2 * tau + 1) / (tau + 1) ** 2
    dcs = lambda x: 1 / x ** 2 + 1 / (1 - x) ** 2 + g - c / (x * (1 - x))
    edges = e0 / (1 - np.linspace(0, 1, 81) * (1 - 2 * e0))       # equal 1/eps^2 mass
    pb = np.array([integrate.quad(dcs, a, b)[0] for a, b in zip(edges[:-1], edges[1:])])
    pb /= pb.sum()
    assert _chi2_pvalue(np.histogram(eps, edges)[0], pb) > 1e-3
    # delta-ray angle from two-body kinematics: momentum along the primary
    w = eps * t
    p0 = math.sqrt(t * (t + 2 * T.MC2))
    pw = np.sqrt(w * (w + 2 * T.MC2))
    pr = np.sqrt((t - w) * (t - w + 2 * T.MC2))
    d0 = np.array([0.3, -0.5, 0.8]) / math.sqrt(0.98)
    p_after = pr[:, None] * out[:, 2:5] + pw[:, None] * out[:, 5:8]
    np.testing.assert_allclose(p_after, np.broadcast_to(p0 * d0, p_after.shape), atol=1e-9 * p0)
    np.testing.assert_allclose(out[:, 5:8] @ d0, cos_d, atol=1e-12)


@pytest.mark.parametrize("t", [0.3, 5.0, 20.0])
def test_bremsstrahlung_sampler_is_one_over_w(blob, t):
    n = 200_000
    w = oracle.sample(blob, 2, t, n, seed=23)[:, 0]
    assert w.min() >= T.E_ABS_G and w.max() <= t
    edges = np.exp(np.linspace(math.log(T.E_ABS_G), math.log(t), 51))
    assert _chi2_pvalue(np.histogram(w, edges)[0], np.full(50, 1 / 50)) > 1e-3


@pytest.mark.parametrize("t", [0.25, 1.0, 5.0])
def test_sauter_photoelectron_angles(t):
    """Angular flag: the photoelectron polar angle follows Sauter's K-shell
    distribution (1 - c^2)/(1 - beta c)^4 [1 + gamma(gamma-1)(gamma-2)(1 - beta c)/2],
    integrated here per bin by quadrature in c = cos(theta)."""
    blob = T.standard_blob("angular")
    c = oracle.sample(blob, 4, t, 300_000, seed=24)[:, 0]
    g = 1 + t / T.MC2
    beta = math.sqrt(1 - 1 / g ** 2)
    pdf = lambda x: (1 - x * x) / (1 - beta * x) ** 4 * (1 + 0.5 * g * (g - 1) * (g - 2) * (1 - beta * x))
    # bins of equal mass in 1/(1 - beta c)^3 resolve the forward peak
    edges = np.sort(np.concatenate([np.linspace(-1, 1, 41), 1 - np.geomspace(1e-4, 1, 40)]))
    edges = np.unique(np.clip(edges, -1, 1))
    pb = np.array([integrate.quad(pdf, a_, b_)[0] for a_, b_ in zip(edges[:-1], edges[1:])])
    pb /= pb.sum()
    assert c.min() >= -1 and c.max() <= 1
    assert _chi2_pvalue(np.histogram(c, edges)[0], pb) > 1e-3


@pytest.mark.parametrize("t", [0.3, 2.0, 15.0])
def test_forward_emission_angles(t):
    """Angular flag: bremsstrahlung photons and pair leptons leave at a polar
    angle with density proportional to (1 - beta cos)^-2 about the emitter."""
    blob = T.standard_blob("angular")
    c = oracle.sample(blob, 5, t, 300_000, seed=25)[:, 0]
    g = 1 + t / T.MC2
    beta = math.sqrt(1 - 1 / g ** 2)
    pdf = lambda x: 1 / (1 - beta * x) ** 2
    edges = np.unique(np.concatenate([np.linspace(-1, 1, 41), 1 - np.geomspace(1e-5, 1, 40)]))
    pb = np.array([integrate.quad(pdf, a_, b_)[0] for a_, b_ in zip(edges[:-1], edges[1:])])
    pb /= pb.sum()
    assert _chi2_pvalue(np.histogram(c, edges)[0], pb) > 1e-3
    # the mean of 1 - cos (which shrinks like 1/gamma) matches its quadrature
    assert np.mean(1 - c) == pytest.approx(quad_mean(pdf), rel=0.02)


def quad_mean(pdf):
    num = integrate.quad(lambda x: (1 - x) * pdf(x), -1, 1, limit=200, points=[0.999, 0.99999])[0]
    den = integrate.quad(pdf, -1, 1, limit=200, points=[0.999, 0.99999])[0]
    return num / den


@pytest.mark.parametrize("e,m", [(0.02, T.MAT_WATER), (0.1, T.MAT_BONE), (1.0, T.MAT_WATER)])
def test_rayleigh_angles_follow_screened_thomson(e, m):
    """Rayleigh polar angle: density (1 + c^2) (1 + b (1 - c))^-4 with
    b = 2 (k a)^2, k = E / (hbar c), a = 0.885 a0 Z_s^(-1/3) (the form factor
    of an exponentially screened atom), integrated per bin by quadrature."""
    blob = T.standard_blob("rayleigh")
    c = oracle.sample(blob, 6 + m, e, 300_000, seed=26)[:, 0]
    b = T.rayleigh_b_coeff(T.MATERIALS[m]) * e * e
    pdf = lambda x: (1 + x * x) / (1 + b * (1 - x)) ** 4
    edges = np.unique(np.concatenate([np.linspace(-1, 1, 41), 1 - np.geomspace(1e-6, 1, 40)]))
    pb = np.array([integrate.quad(pdf, a_, b_)[0] for a_, b_ in zip(edges[:-1], edges[1:])])
    pb /= pb.sum()
    assert c.min() >= -1 and c.max() <= 1
    assert _chi2_pvalue(np.histogram(c, edges)[0], pb) > 1e-3


def test_rayleigh_flag_conserves_energy_and_changes_only_photon_paths(blob):
    """Rayleigh flag: energy still balances; the source draws are unchanged; a
    pure Rayleigh-free run (standard tables) differs."""
    ph = phantoms.homogeneous(16, 16, 16, 1.0)
    src = sources.point_field(PHOTON, *ph.centre_xy(), 100.0, 3.0, 3.0, energy=0.2)
    a = oracle.simulate(blob, ph, src, 3000, seed=82)
    b = oracle.simulate(T.standard_blob("refined"), ph, src, 3000, seed=82)
    for r in (a, b):
        bal = r["bal"]
        closed = bal["E_csda"] + bal["E_local"] + bal["E_esc"] + bal["E_miss"]
        assert abs(closed - bal["E_src"]) <= 1e-9 * bal["E_src"]
    assert a["bal"]["E_src"] == b["bal"]["E_src"]
    assert a["cnt"]["rayleigh"] == 0 and b["cnt"]["rayleigh"] > 0
    assert not np.array_equal(a["S"], b["S"])


def test_angular_flag_keeps_energy_and_draw_structure(blob):
    """Same histories with and without the angular flag: energy is conserved,
    the source sampling is identical, and the angles change the dose."""
    ph = phantoms.homogeneous(16, 16, 16, 1.0)
    src = sources.point_field(PHOTON, *ph.centre_xy(), 100.0, 3.0, 3.0, energy=15.0)
    a = oracle.simulate(blob, ph, src, 3000, seed=81)
    b = oracle.simulate(T.standard_blob("angular"), ph, src, 3000, seed=81)
    for r in (a, b):
        bal = r["bal"]
        closed = bal["E_csda"] + bal["E_local"] + bal["E_esc"] + bal["E_miss"]
        assert abs(closed - bal["E_src"]) <= 1e-9 * bal["E_src"]
    assert a["bal"]["E_src"] == b["bal"]["E_src"]
    assert a["cnt"]["pair"] > 0 and a["cnt"]["photo"] >= 0
    assert not np.array_equal(a["S"], b["S"])


def test_hinge_reproduces_lewis_first_moment(tabs):
    n = 400_000
    out = oracle.sample(T.standard_blob(), 3, 1.0, n, seed=24)
    cost = out[:, 0]
    one_minus = 1 - cost
    target = 1 - math.exp(-tabs.kappa_step)
    assert abs(one_minus.mean() - target) <= 4 * one_minus.std() / math.sqrt(n)
    # the deflection is applied about the incoming direction, azimuth uniform
    d0 = np.array([0.3, -0.5, 0.8]) / math.sqrt(0.98)
    np.testing.assert_allclose(out[:, 2:5] @ d0, cost, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(out[:, 2:5], axis=1), 1.0, atol=1e-14)
    perp = out[:, 2:5] - (out[:, 2:5] @ d0)[:, None] * d0
    e1 = np.cross(d0, [0.0, 0.0, 1.0])
    e1 /= np.linalg.norm(e1)
    phi = np.arctan2(perp @ np.cross(d0, e1), perp @ e1)
    counts = np.histogram(phi, np.linspace(-math.pi, math.pi, 33))[0]
    assert _chi2_pvalue(counts, np.full(32, 1 / 32)) > 1e-3


# ------------------------------------------------------------ electrons

@pytest.mark.parametrize("m,e", [(T.MAT_WATER, 0.3), (T.MAT_WATER, 5.0), (T.MAT_BONE, 1.0),
                                 (T.MAT_BONE, 18.0)])
def test_second_moment_hinge_reproduces_both_lewis_moments(m, e):
    """hinge2 flag: after a step of kappa transport mean free paths the
    deflection has <P1(cos)> = exp(-kappa) and <P2(cos)> = exp(-kappa r),
    r = lambda1/lambda2 (Lewis); the hinge angle reproduces both.  The
    first-moment hinge reproduces the first and misses the second by many
    standard errors, so this pin tells the two apart."""
    blob = T.standard_blob("hinge2")
    n = 400_000
    out = oracle.sample(blob, 256 + m, e, n, seed=27)
    c, r = out[:, 0], out[0, 1]
    mat = T.MATERIALS[m]
    assert r == pytest.approx(T.lambda2_inv(mat, e) / T.lambda1_inv(mat, e), rel=1e-4)
    k = T.KAPPA_STEP
    assert c.min() >= -1 and c.max() <= 1
    p1, p2 = c, 1.5 * c * c - 0.5
    se = lambda x: x.std() / math.sqrt(n)
    assert abs(p1.mean() - math.exp(-k)) <= 5 * se(p1)
    assert abs(p2.mean() - math.exp(-k * r)) <= 5 * se(p2)
    c1 = oracle.sample(blob, 3, e, n, seed=27)[:, 0]
    q1, q2 = c1, 1.5 * c1 * c1 - 0.5
    assert abs(q1.mean() - math.exp(-k)) <= 5 * se(q1)
    assert abs(q2.mean() - math.exp(-k * r)) > 10 * se(q2)


@pytest.mark.parametrize("ratio", [1.2, 1.8, 2.4])
def test_second_moment_hinge_heavier_tail_branch(ratio):
    """lambda1/lambda2 set by hand so that the target <mu^2>/<mu> lies above
    the first-moment Wentzel law's (small ratios): the law then mixes
    undeflected hinges with a wider Wentzel angle.  Both Lewis moments still
    hold; some hinges do not deflect at all."""
    t = T.read_blob(T.standard_blob("hinge2"))
    t.data[:, T.Q_LAMBDA2_INV] = ratio * t.data[:, T.Q_LAMBDA1_INV]
    blob = T.write_blob(t)
    n = 400_000
    out = oracle.sample(blob, 256 + T.MAT_WATER, 2.0, n, seed=29)
    c, r = out[:, 0], out[0, 1]
    assert r == pytest.approx(ratio, rel=1e-12)
    k = T.KAPPA_STEP
    p1, p2 = c, 1.5 * c * c - 0.5
    se = lambda x: x.std() / math.sqrt(n)
    assert abs(p1.mean() - math.exp(-k)) <= 5 * se(p1)
    assert abs(p2.mean() - math.exp(-k * r)) <= 5 * se(p2)
    straight = np.mean(c == 1.0)
    m1 = 0.5 * (1 - math.exp(-k))
    m2 = m1 - (1 - math.exp(-k * r)) / 6
    a1 = t.a_hinge
    l1 = math.log1p(1 / a1)
    q1 = (a1 * ((1 + 2 * a1) - 2 * a1 * (1 + a1) * l1)) / (a1 * ((1 + a1) * l1 - 1))
    if m2 / m1 >= q1:
        assert straight > 0.01
    else:
        assert straight < 1e-4


def test_second_moment_hinge_flag_keeps_energy_and_draws(blob):
    """Same histories with and without the hinge2 flag: the source draws and
    the energy balance hold, the dose changes."""
    ph = phantoms.homogeneous(16, 16, 16, 1.0)
    src = sources.pencil(ELECTRON, 12.0, *ph.centre_xy())
    a = oracle.simulate(blob, ph, src, 1500, seed=83)
    b = oracle.simulate(T.standard_blob("hinge2"), ph, src, 1500, seed=83)
    for r in (a, b):
        bal = r["bal"]
        closed = bal["E_csda"] + bal["E_local"] + bal["E_esc"] + bal["E_miss"]
        assert abs(closed - bal["E_src"]) <= 1e-9 * bal["E_src"]
    assert a["bal"]["E_src"] == b["bal"]["E_src"]
    assert b["cnt"]["hinges"] > 0
    assert not np.array_equal(a["S"], b["S"])


def test_csda_track_length_equals_range_difference():
    """No hard events: each electron's path length is (R(T0) - R(E_abs)) / rho,
    whatever its deflections and voxel crossings."""
    b = T.standard_blob("no_hard")
    t = T.read_blob(b)
    ph = phantoms.homogeneous(40, 40, 40, 1.0)
    x, y = ph.centre_xy()
    for e0 in (20.0, 7.3, 1.1):
        r = oracle.simulate(b, ph, sources.pencil(ELECTRON, e0, x + 0.25, y + 0.25), 300, seed=31,
                            history=True)
        ln_e = np.log(t.energies)
        rr = t.data[T.MAT_WATER, T.Q_RANGE]
        expected = np.interp(math.log(e0), ln_e, rr) - np.interp(math.log(T.E_ABS_E), ln_e, rr)
        h = r["hist"]
        kept = h["escaped"] == 0                  # a few backscatter out of the top face
        assert kept.mean() > 0.9
        np.testing.assert_allclose(h["track_e"][kept], expected, rtol=1e-12)
        assert np.all(h["track_e"][~kept] < expected)
        # without escapes the whole kinetic energy is deposited
        np.testing.assert_allclose(h["edep"][kept], e0, rtol=1e-12)
        assert r["cnt"]["moller"] == 0 and r["cnt"]["brems"] == 0


def _blob_with_flags(variant, extra, e_abs_g=None):
    t = T.build_tables(variant=variant)
    t.flags |= extra
    if e_abs_g is not None:
        t.e_abs_g = e_abs_g
    return T.write_blob(t)


def test_positron_csda_track_length_uses_positron_range():
    """No hard events, Bhabha flag: a positron's path length is
    (R+(T0) - R+(E_abs)) / rho on the positron range; without the flag it is
    the electron range difference.  The photon cutoff is raised above m c^2 so
    the annihilation photons deposit on the spot and set no electrons moving."""
    for flags, q in ((T.FLAG_BHABHA, T.Q_RANGE_POS), (0, T.Q_RANGE)):
        b = _blob_with_flags("no_hard", flags, e_abs_g=0.6)
        t = T.read_blob(b)
        ph = phantoms.homogeneous(40, 40, 40, 1.0)
        x, y = ph.centre_xy()
        ln_e = np.log(t.energies)
        rr = t.data[T.MAT_WATER, q]
        for e0 in (15.0, 2.2):
            r = oracle.simulate(b, ph, sources.pencil(POSITRON, e0, x + 0.25, y + 0.25), 300, seed=34,
                                history=True)
            expected = np.interp(math.log(e0), ln_e, rr) - np.interp(math.log(T.E_ABS_E), ln_e, rr)
            h = r["hist"]
            full = np.isclose(h["track_e"], expected, rtol=1e-12)
            assert full.mean() > 0.9                  # the rest backscatter out of the top face
            assert np.all(h["track_e"][~full] < expected)
            assert r["cnt"]["bhabha"] == 0 and r["cnt"]["moller"] == 0


def test_bhabha_events_take_the_positron_cross_section():
    """Bhabha flag, energy-independent cross sections with Sigma_M = 0 and
    Sigma_B = 0: only positrons have hard events, at Sigma_Bh per g/cm^2 of
    their path.  A positron whose CSDA path would end inside the phantom is
    cut short by its first Bhabha event, so over 10 MeV primaries the number
    of events per history is Sigma_Bh times the mean positron path, which lies
    between the path to the first event and the CSDA range.  Without the flag
    positrons take Sigma_M = 0 and have none."""
    t = T.read_blob(T.standard_blob("bhabha"))
    s_bh = 0.2
    t.data[:, T.Q_SIGMA_BH] = s_bh
    t.data[:, T.Q_SIGMA_B] = 0.0
    t.data[:, T.Q_SIGMA_M] = 0.0
    b = T.write_blob(t)
    ph = phantoms.homogeneous(40, 40, 40, 1.0)
    x, y = ph.centre_xy()
    src = sources.pencil(POSITRON, 10.0, x + 0.25, y + 0.25)
    n = 2000
    r = oracle.simulate(b, ph, src, n, seed=35)
    c = r["cnt"]
    assert c["moller"] == 0 and c["brems"] == 0
    events = c["bhabha"] + c["void"]
    csda = np.interp(math.log(10.0), np.log(t.energies), t.data[T.MAT_WATER, T.Q_RANGE_POS])
    # at least one event per history unless the whole CSDA path has none
    p_none = math.exp(-s_bh * csda)
    assert events >= n * (1 - p_none) * 0.95
    assert events <= s_bh * csda * n * 1.05
    t.flags = 0
    r0 = oracle.simulate(T.write_blob(t), ph, src, n, seed=35)
    assert r0["cnt"]["bhabha"] == 0 and r0["cnt"]["moller"] == 0 and r0["cnt"]["void"] == 0


@pytest.mark.parametrize("t", [0.5, 3.0, 15.0])
def test_bhabha_sampler_follows_its_dcs(t):
    """Bhabha energy transfer e = W/T on [W_cc/T, 1] against quadrature of
    e^-2 [1 - b1 e + b2 e^2 - b3 e^3 + b4 e^4] per bin."""
    blob = T.standard_blob("bhabha")
    e = oracle.sample(blob, 512, t, 300_000, seed=28)[:, 0]
    b1, b2, b3, b4 = T.bhabha_coeffs(t)
    ec = T.E_ABS_E / t
    pdf = lambda x: (1 - b1 * x + b2 * x * x - b3 * x ** 3 + b4 * x ** 4) / (x * x)
    edges = np.geomspace(ec, 1.0, 41)
    pb = np.array([integrate.quad(pdf, a_, b_)[0] for a_, b_ in zip(edges[:-1], edges[1:])])
    pb /= pb.sum()
    assert e.min() >= ec and e.max() <= 1.0
    assert _chi2_pvalue(np.histogram(e, edges)[0], pb) > 1e-3


def test_hinge_and_hard_event_rates_along_a_track(blob):
    """With energy-independent transport and hard cross sections the step
    algorithm consumes them exactly, so over all electron paths L (g/cm^2):
    E[hinges] = (lambda1 rho)^-1 L / kappa_step and E[hard events] =
    (Sigma_M + Sigma_B) L, with Moller:brems selected as Sigma_M:Sigma_B."""
    t = T.read_blob(blob)
    lam_inv, s_m, s_b = 3.0, 0.35, 0.12            # cm^2/g
    t.data[:, T.Q_LAMBDA1_INV] = lam_inv
    t.data[:, T.Q_SIGMA_M] = s_m
    t.data[:, T.Q_SIGMA_B] = s_b
    b = T.write_blob(t)
    ph = phantoms.homogeneous(40, 40, 40, 1.0, density=1.0)
    x, y = ph.centre_xy()
    n = 3000
    r = oracle.simulate(b, ph, sources.pencil(ELECTRON, 10.0, x + 0.25, y + 0.25), n, seed=33)
    track = r["bal"]["track_e"]                     # cm at rho = 1
    c = r["cnt"]
    hinges_exp = lam_inv * track / t.kappa_step
    assert abs(c["hinges"] - hinges_exp) <= 4 * math.sqrt(hinges_exp / 4)
    hard = c["moller"] + c["brems"] + c["void"]
    hard_exp = (s_m + s_b) * track
    assert abs(hard - hard_exp) <= 4 * math.sqrt(hard_exp)
    pm = s_m / (s_m + s_b)
    assert abs((c["moller"] + c["void"]) / hard - pm) <= 4 * math.sqrt(pm * (1 - pm) / hard)


def test_spectrum_sampling_mean_energy(blob):
    ph = phantoms.homogeneous(10, 10, 4, 1.0)
    x, y = ph.centre_xy()
    edges, wts = sources.spectrum_6mv()
    src = sources.point_field(PHOTON, x, y, 100.0, 2.0, 2.0, spectrum=(edges, wts))
    n = 20000
    r = oracle.simulate(blob, ph, src, n, seed=35)
    c = 0.5 * (edges[1:] + edges[:-1])
    p = wts / wts.sum()
    mean = float(np.dot(p, c))
    var = float(np.dot(p, c * c + (edges[1] - edges[0]) ** 2 / 12)) - mean ** 2
    assert abs(r["bal"]["E_src"] / n - mean) <= 4 * math.sqrt(var / n)


CASES = [
    ("e20_wlw", lambda: (phantoms.water_lung_water_32(), "pencil", ELECTRON, 20.0)),
    ("g6mv_wbw", lambda: (phantoms.water_bone_water_61(), "field", PHOTON, None)),
    ("pos5_rf", lambda: (phantoms.random_field_phantom(24, 0.5, seed=9), "field", POSITRON, 5.0)),
    ("g15_rf", lambda: (phantoms.random_field_phantom(24, 0.5, seed=9), "field", PHOTON, 15.0)),
]


def _source(ph, kind, particle, e):
    x, y = ph.centre_xy()
    if kind == "pencil":
        return sources.pencil(particle, e, x, y)
    spec = sources.spectrum_6mv() if e is None else None
    return sources.point_field(particle, x, y, 100.0, 5.0, 5.0, energy=e, spectrum=spec)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_energy_conservation(blob, name, make):
    ph, kind, particle, e = make()
    r = oracle.simulate(blob, ph, _source(ph, kind, particle, e), 2000, seed=41)
    b = r["bal"]
    closed = b["E_csda"] + b["E_local"] + b["E_esc"] + b["E_miss"]
    assert abs(closed - b["E_src"]) <= 1e-9 * b["E_src"]
    assert r["S"].sum() == pytest.approx(b["E_csda"] + b["E_local"], rel=1e-12)
    assert np.all(r["Q"] >= 0) and np.all(r["S"] >= 0)
    # Q >= S^2 / N (Cauchy-Schwarz) and Q <= S * max history deposit
    assert np.all(r["Q"] * 2000 >= r["S"] ** 2 * (1 - 1e-12))


def test_density_scaling_is_exact(blob):
    """O'Connor: every coefficient is proportional to density, so water at
    rho = 0.5 with doubled voxels and doubled source geometry gives the same
    energy per voxel for the same keys (factor-2 scalings are exact in FP)."""
    a = phantoms.homogeneous(16, 16, 24, 0.5)
    b = phantoms.homogeneous(16, 16, 24, 1.0, density=0.5)
    for particle, e in ((ELECTRON, 12.0), (PHOTON, 4.0)):
        xa, ya = a.centre_xy()
        xb, yb = b.centre_xy()
        sa = sources.point_field(particle, xa, ya, 10.0, 1.5, 1.0, energy=e)
        sb = sources.point_field(particle, xb, yb, 20.0, 3.0, 2.0, energy=e)
        ra = oracle.simulate(blob, a, sa, 400, seed=51, history=True)
        rb = oracle.simulate(blob, b, sb, 400, seed=51, history=True)
        np.testing.assert_array_equal(ra["hist"]["hash"], rb["hist"]["hash"])
        np.testing.assert_allclose(ra["S"], rb["S"], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(rb["hist"]["track_e"], 2 * ra["hist"]["track_e"], rtol=1e-12)


def test_lateral_symmetry(blob):
    """Centred pencil beam on a laterally uniform phantom: D(x,y) = D(-x,y) = D(y,x) within 3 sigma."""
    ph = phantoms.slab_phantom(9, 9, 0.5, 0.5, [(4, T.MAT_WATER, 1.0), (6, T.MAT_BONE, 1.85),
                                                (6, T.MAT_WATER, 1.0)], 0.5)
    x, y = ph.centre_xy()
    n = 3000
    r = oracle.simulate(blob, ph, sources.pencil(ELECTRON, 8.0, x, y), n, seed=61)
    S = r["S"].reshape(16, 9, 9)
    Q = r["Q"].reshape(16, 9, 9)
    var = (Q / n - (S / n) ** 2) / (n - 1) * n * n
    for tr in (lambda a: a[:, :, ::-1], lambda a: a[:, ::-1, :], lambda a: a.transpose(0, 2, 1)):
        d = S - tr(S)
        s = np.sqrt(var + tr(var))
        sel = S > 0.05 * S.max()
        frac_ok = np.mean(np.abs(d[sel]) <= 3 * s[sel] + 1e-12)
        assert frac_ok > 0.97


def test_split_runs_add_up_and_runs_repeat(blob):
    ph = phantoms.water_lung_water_32()
    x, y = ph.centre_xy()
    src = sources.pencil(ELECTRON, 20.0, x, y)
    full = oracle.simulate(blob, ph, src, 600, seed=1, history=True)
    again = oracle.simulate(blob, ph, src, 600, seed=1, history=True)
    np.testing.assert_array_equal(full["S"], again["S"])
    np.testing.assert_array_equal(full["hist"], again["hist"])
    a = oracle.simulate(blob, ph, src, 250, seed=1, history=True)
    b = oracle.simulate(blob, ph, src, 350, seed=1, first=250, history=True)
    np.testing.assert_array_equal(np.concatenate([a["hist"], b["hist"]]), full["hist"])
    np.testing.assert_allclose(a["S"] + b["S"], full["S"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(a["Q"] + b["Q"], full["Q"], rtol=1e-12, atol=1e-15)
    # a different request key gives different histories
    other = oracle.simulate(blob, ph, src, 600, seed=1, key=7, history=True)
    assert np.mean(other["hist"]["hash"] == full["hist"]["hash"]) < 0.01


def test_source_sampling_field_and_miss(blob):
    ph = phantoms.homogeneous(10, 10, 4, 1.0)
    x, y = ph.centre_xy()
    # a field half outside the top face: about half the primaries miss
    src = sources.point_field(PHOTON, x, y, 100.0, 5.0, 2.0, energy=1.0, fx=x + 5.0)
    r = oracle.simulate(blob, ph, src, 4000, seed=71)
    frac = r["cnt"]["misses"] / 4000
    assert abs(frac - 0.5) < 4 * math.sqrt(0.25 / 4000)
    assert r["bal"]["E_miss"] == pytest.approx(r["cnt"]["misses"] * 1.0)


def test_finalize_hand_example():
    """Two voxels, N = 4 histories with deposits (MeV) per history:
    voxel 0: 1, 2, 0, 1 -> S = 4, Q = 6; voxel 1: 3, 3, 3, 3 -> S = 12, Q = 36."""
    ph = phantoms.Phantom(2, 1, 1, 1.0, 1.0, 1.0, mat=np.zeros((1, 1, 2), np.uint8),
                          rho=np.array([[[1.0, 2.0]]], np.float32))
    dose, sigma, dmax, sbar = oracle.finalize(ph, np.array([4.0, 12.0]), np.array([6.0, 36.0]), 4)
    gy = 1.602176634e-10
    assert dose[0] == pytest.approx(1.0 * gy) and dose[1] == pytest.approx(1.5 * gy)
    # sample variance of the mean: (Q/N - (S/N)^2) / (N - 1)
    assert sigma[0] == pytest.approx(math.sqrt((1.5 - 1.0) / 3) * gy)
    assert sigma[1] == 0.0
    assert dmax == pytest.approx(1.5 * gy)
    # both voxels exceed Dmax/2: mean of sigma/D = (0.408248/1 + 0) / 2
    assert sbar == pytest.approx(0.5 * math.sqrt(0.5 / 3))


def test_finalize_ignores_air_for_dmax_and_sigma_bar():
    """Voxel 2 is air (0.0012 g/cm^3): its dose (S/(N rho V)) is the largest
    but Dmax and sigma-bar cover tissue voxels (>= 0.05 g/cm^3) only; its dose
    and sigma are still reported.  Same rule for the group estimator."""
    rho = np.array([[[1.0, 0.26, 0.0012]]], np.float32)
    ph = phantoms.Phantom(3, 1, 1, 1.0, 1.0, 1.0, mat=np.zeros((1, 1, 3), np.uint8), rho=rho)
    S = np.array([4.0, 2.0, 1.0])
    Q = np.array([6.0, 2.0, 1.0])
    dose, sigma, dmax, sbar = oracle.finalize(ph, S, Q, 4)
    gy = 1.602176634e-10
    assert dose[2] == pytest.approx(0.25 / 0.0012 * gy, rel=1e-6) and sigma[2] > 0
    assert dmax == pytest.approx(0.5 / 0.26 * gy)          # the lung voxel
    # tissue voxels above Dmax/2 (0.96 gy-units): lung (1.92) and water (1.0)
    s_lung = math.sqrt((0.5 - 0.25) / 3) / 0.5
    s_water = math.sqrt((1.5 - 1.0) / 3) / 1.0
    assert sbar == pytest.approx(0.5 * (s_lung + s_water))
    # group estimator: 16 groups of one history each; all deposits in group 0
    Sb = np.zeros((16, 3))
    Sb[0] = S
    nb = np.ones(16)
    dose_g, _, dmax_g, _ = oracle.finalize_groups(ph, Sb, nb)
    assert dose_g[2] == pytest.approx(1.0 / 16 / 0.0012 * gy, rel=1e-6)
    assert dmax_g == pytest.approx(2.0 / 16 / 0.26 * gy)
