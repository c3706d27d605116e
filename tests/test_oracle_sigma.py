"""Pins of the oracle's uncertainty estimators (Sec. 3: sigma_D, the standard
deviation of the dose in a voxel, and its mean relative value over voxels above
half of Dmax).

The group ("batch") estimator sums histories into 16 groups (history mod 16)
and estimates the variance of the mean from the spread of the group means,
weighted by the group sizes, with B' - 1 degrees of freedom, then divides the
standard deviation by c4(B') so that it is not biased low.  These tests check
it against hand arithmetic with the closed forms c4(3) = Gamma(3/2) =
sqrt(pi)/2 and c4(2) = sqrt(2/pi), against a synthetic population whose
standard error is known exactly, and against the history-by-history estimator
on transported histories.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_0910_0329_amd.inputs import configs, phantoms

GY = 1.602176634e-10          # Gy per (MeV/g)


def _unit_phantom(nv, rho=1.0):
    return phantoms.Phantom(nv, 1, 1, 1.0, 1.0, 1.0, mat=np.zeros((1, 1, nv), np.uint8),
                            rho=np.full((1, 1, nv), rho, np.float32))


def test_group_sigma_hand_example_unequal_groups():
    """Three non-empty groups of 2, 3 and 5 histories (the other 13 empty).
    Deposits per history in the one voxel (MeV): group 0: 1, 3; group 1: 0,
    0, 3; group 2: 1, 1, 1, 1, 6.  Group totals 4, 3, 10 and means 2, 1, 2;
    N = 10, S = 17, m = 1.7.  Weighted spread: 2 (0.3)^2 + 3 (0.7)^2 +
    5 (0.3)^2 = 2.1, so s^2 = 2.1 / (3 - 1) = 1.05, sigma_mean^2 =
    1.05 / 10 = 0.105, and sigma = sqrt(0.105) / c4(3) with c4(3) =
    sqrt(pi) / 2."""
    ph = _unit_phantom(1)
    Sb = np.zeros((16, 1))
    nb = np.zeros(16)
    Sb[0, 0], nb[0] = 4.0, 2
    Sb[1, 0], nb[1] = 3.0, 3
    Sb[2, 0], nb[2] = 10.0, 5
    dose, sigma, dmax, sbar = oracle.finalize_groups(ph, Sb, nb)
    want = math.sqrt(0.105) / (math.sqrt(math.pi) / 2)
    assert dose[0] == pytest.approx(1.7 * GY, rel=1e-14)
    assert sigma[0] == pytest.approx(want * GY, rel=1e-12)
    assert dmax == pytest.approx(1.7 * GY, rel=1e-14)
    assert sbar == pytest.approx(want / 1.7, rel=1e-12)
    # the plausible slips all move sigma by far more than the tolerance
    assert abs(math.sqrt(2.1 / 3 / 10) / (math.sqrt(math.pi) / 2) - want) > 0.1 * want   # B' for B' - 1
    assert abs(math.sqrt(0.67 / 2 / 10) / (math.sqrt(math.pi) / 2) - want) > 0.1 * want  # no nb weight
    assert abs(math.sqrt(0.105) - want) > 0.1 * want                                     # no c4


def test_group_sigma_two_groups_and_groups_at_any_index():
    """Two non-empty groups (indices 5 and 11, sizes 1 and 3), two voxels of
    densities 1 and 2 g/cm^3.  Voxel 0: group totals 2 and 3 -> means 2 and 1,
    m = 5/4, spread 1 (0.75)^2 + 3 (0.25)^2 = 0.75, s^2 = 0.75 / 1,
    sigma_mean = sqrt(0.75 / 4); c4(2) = sqrt(2 / pi).  Voxel 1: totals 0 and
    6 -> means 0 and 2, m = 1.5, spread 1 (1.5)^2 + 3 (0.5)^2 = 3,
    sigma_mean = sqrt(3 / 4); its dose is S / (N rho V) = 6 / 4 / 2."""
    ph = phantoms.Phantom(2, 1, 1, 1.0, 1.0, 1.0, mat=np.zeros((1, 1, 2), np.uint8),
                          rho=np.array([[[1.0, 2.0]]], np.float32))
    Sb = np.zeros((16, 2))
    nb = np.zeros(16)
    Sb[5], nb[5] = (2.0, 0.0), 1
    Sb[11], nb[11] = (3.0, 6.0), 3
    dose, sigma, dmax, sbar = oracle.finalize_groups(ph, Sb, nb)
    c4 = math.sqrt(2 / math.pi)
    assert dose[0] == pytest.approx(1.25 * GY, rel=1e-14)
    assert dose[1] == pytest.approx(0.75 * GY, rel=1e-14)
    assert sigma[0] == pytest.approx(math.sqrt(0.75 / 4) / c4 * GY, rel=1e-12)
    assert sigma[1] == pytest.approx(math.sqrt(3 / 4) / c4 / 2 * GY, rel=1e-12)
    # Dmax = 1.25 GY-units; both voxels are above half of it
    assert dmax == pytest.approx(1.25 * GY, rel=1e-14)
    assert sbar == pytest.approx(0.5 * (sigma[0] / dose[0] + sigma[1] / dose[1]), rel=1e-12)


def test_group_sigma_single_group_is_zero():
    """One non-empty group leaves no spread to estimate from: sigma = 0."""
    ph = _unit_phantom(1)
    Sb = np.zeros((16, 1))
    nb = np.zeros(16)
    Sb[3, 0], nb[3] = 5.0, 4
    dose, sigma, _, _ = oracle.finalize_groups(ph, Sb, nb)
    assert dose[0] == pytest.approx(1.25 * GY) and sigma[0] == 0.0


def test_group_sigma_is_unbiased_for_a_known_population():
    """2e5 independent voxels whose per-history deposits have mean 5 and
    standard deviation 2: a group of nb histories then totals N(5 nb, 4 nb)
    (drawn exactly as such), and the standard error of the voxel mean is
    2 / sqrt(N), known exactly.  With uneven, partly empty groups (B' = 14)
    the estimator's mean over voxels must equal it to within 0.3%: the
    standard error of that mean is 0.05%, while c4(14) = 0.981, B' in place
    of B' - 1 (0.964) or dropping the nb weights are each off by 2% or more.
    The variance itself (sigma^2 c4^2) is unbiased as well."""
    rng = np.random.default_rng(20240611)
    nb = np.array([0, 3, 7, 1, 12, 5, 0, 9, 4, 2, 6, 8, 11, 1, 10, 2], dtype=np.float64)
    nv = 200_000
    mu, sd = 5.0, 2.0
    Sb = np.zeros((16, nv))
    for b in range(16):
        if nb[b] > 0:
            Sb[b] = rng.normal(mu * nb[b], sd * math.sqrt(nb[b]), nv)
    N = nb.sum()
    ph = phantoms.Phantom(1000, 200, 1, 1.0, 1.0, 1.0, mat=np.zeros((1, 200, 1000), np.uint8),
                          rho=np.ones((1, 200, 1000), np.float32))
    dose, sigma, _, _ = oracle.finalize_groups(ph, Sb, nb)
    se = sd / math.sqrt(N)
    ratio = sigma / GY / se
    assert np.mean(ratio) == pytest.approx(1.0, abs=0.003)
    k = int((nb > 0).sum())
    c4 = math.sqrt(2 / (k - 1)) * math.exp(math.lgamma(k / 2) - math.lgamma((k - 1) / 2))
    assert np.mean((ratio * c4) ** 2) == pytest.approx(1.0, abs=0.006)
    # the dose is the plain mean
    np.testing.assert_allclose(dose / GY, Sb.sum(axis=0) / N, rtol=1e-13)


def test_group_sigma_agrees_with_history_sigma_on_transport(blob):
    """16 x 2000 transported histories (20 MeV electrons, 10x10 cm field on
    the water-lung-water phantom): per voxel above Dmax/2 (about 7000), the
    group estimate over the history-by-history estimate is distributed like
    sqrt(chi2_15 / 15) / c4(16), 15 degrees of freedom, widened a little by
    the noise of the history-by-history estimate itself.  Its median must sit
    at the median of that law, few voxels may fall outside the law's
    0.1%-99.9% band, and the squared ratio times c4^2 (the variance
    estimates) must average to 1."""
    ph = configs.electron_20mev_wlw(1).phantom
    w = configs.electron_20mev_point_field(ph, 32_000)
    r = oracle.simulate(blob, w.phantom, w.source, w.n_histories, w.seed, w.request_key, groups=True)
    assert r["nb"].tolist() == [2000.0] * 16
    np.testing.assert_allclose(r["Sb"].sum(axis=0), r["S"], rtol=1e-12, atol=1e-12)
    d_h, s_h, dmax_h, _ = oracle.finalize(w.phantom, r["S"], r["Q"], w.n_histories)
    d_g, s_g, dmax_g, _ = oracle.finalize_groups(w.phantom, r["Sb"], r["nb"])
    np.testing.assert_allclose(d_g, d_h, rtol=1e-12, atol=0)
    sel = (d_h > 0.5 * dmax_h) & (s_h > 0)
    assert sel.sum() > 5000
    ratio = s_g[sel] / s_h[sel]
    c4 = math.sqrt(2 / 15) * math.exp(math.lgamma(8) - math.lgamma(7.5))
    law = lambda q: math.sqrt(stats.chi2.ppf(q, 15) / 15) / c4       # noqa: E731
    assert abs(np.median(ratio) - law(0.5)) < 0.015
    outside = np.mean((ratio < law(0.001)) | (ratio > law(0.999)))
    assert outside < 0.01
    assert np.mean((ratio * c4) ** 2) == pytest.approx(1.0, abs=0.04)
