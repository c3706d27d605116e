"""Source descriptors and seeded source-parameter generators.

The paper's sources are point sources with a rectangular field: a 20 MeV
monoenergetic electron beam or a 6 MV photon spectrum (Sec. 3).  A descriptor
holds data only; sampling a particle from it is part of the transport and is
implemented by each consumer.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PHOTON, ELECTRON, POSITRON = 0, 1, 2
MONO, HISTOGRAM = 0, 1
PENCIL, POINT_FIELD = 0, 1
MAX_BINS = 64


@dataclass
class Source:
    particle: int = PHOTON
    energy_kind: int = MONO
    e0: float = 1.0                           # MeV (mono)
    edges: np.ndarray = field(default_factory=lambda: np.zeros(0))     # n_bins + 1 (histogram)
    weights: np.ndarray = field(default_factory=lambda: np.zeros(0))   # n_bins
    beam_kind: int = PENCIL
    pos: tuple = (0.0, 0.0, 0.0)              # pencil: entry (x, y) on the top face; point: source point
    field_rect: tuple = (0.0, 0.0, 5.0, 5.0)  # centre x, centre y, half-widths hx, hy on the top face

    @property
    def n_bins(self) -> int:
        return len(self.weights)

    def mean_energy(self) -> float:
        if self.energy_kind == MONO:
            return self.e0
        c = 0.5 * (self.edges[1:] + self.edges[:-1])
        return float(np.dot(self.weights, c) / self.weights.sum())


def spectrum_6mv(n_bins: int = 64, e_lo: float = 0.1, e_hi: float = 6.0):
    """Synthetic 6 MV bremsstrahlung-like spectrum: equal bins on [0.1, 6] MeV with
    weights proportional to (6 - E_centre); mean energy 2.067 MeV."""
    edges = np.linspace(e_lo, e_hi, n_bins + 1)
    centres = 0.5 * (edges[1:] + edges[:-1])
    return edges, e_hi - centres


def pencil(particle, energy, x, y) -> Source:
    return Source(particle=particle, energy_kind=MONO, e0=energy, beam_kind=PENCIL, pos=(x, y, 0.0))


def point_field(particle, xc, yc, ssd, hx, hy, z0=0.0, energy=None, spectrum=None,
                fx=None, fy=None) -> Source:
    """Point source at (xc, yc, z0 - ssd) aiming at a rectangle of half-widths
    (hx, hy) centred at (fx, fy) on the phantom's top face z = z0."""
    s = Source(particle=particle, beam_kind=POINT_FIELD, pos=(xc, yc, z0 - ssd),
               field_rect=(xc if fx is None else fx, yc if fy is None else fy, hx, hy))
    if spectrum is not None:
        s.energy_kind = HISTOGRAM
        s.edges, s.weights = (np.asarray(a, dtype=np.float64) for a in spectrum)
    else:
        s.energy_kind = MONO
        s.e0 = float(energy)
    return s


def beamlets(phantom, seed: int = 4, n_x: int = 8, n_y: int = 16, side: float = 0.5,
             field: float = 10.0, ssd: float = 100.0, n_lo: float = 1e4, n_hi: float = 1e6):
    """128 beamlets of side x side cm on an n_x by n_y grid spanning the central
    field x field cm of the top face.  Even index: 6 MV photons; odd index:
    monoenergetic electrons with E ~ U(6, 20) MeV.  History counts are
    log-uniform on [n_lo, n_hi].  Returns (sources, n_histories)."""
    rng = np.random.default_rng(seed)
    xc, yc = phantom.centre_xy()
    spec = spectrum_6mv()
    srcs, ns = [], []
    for b in range(n_x * n_y):
        ix, iy = b % n_x, b // n_x
        fx = xc - field / 2 + (ix + 0.5) * field / n_x
        fy = yc - field / 2 + (iy + 0.5) * field / n_y
        e_el = rng.uniform(6.0, 20.0)
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        if b % 2 == 0:
            s = point_field(PHOTON, xc, yc, ssd, side / 2, side / 2, spectrum=spec, fx=fx, fy=fy)
        else:
            s = point_field(ELECTRON, xc, yc, ssd, side / 2, side / 2, energy=e_el, fx=fx, fy=fy)
        srcs.append(s)
        ns.append(n)
    return srcs, np.array(ns, dtype=np.uint64)


def poisson_arrivals(rate: float, duration: float, seed: int = 5) -> np.ndarray:
    """Arrival times (s) of a Poisson process of `rate` per second over `duration`."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return np.array(out)
        out.append(t)
