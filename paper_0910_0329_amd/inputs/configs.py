"""The synthetic workloads: phantoms and sources shaped like the paper's slab and
point-source experiments (Sec. 3), at the sizes this engine is measured on."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import phantoms, sources
from .sources import ELECTRON, PHOTON


@dataclass
class Workload:
    name: str
    phantom: phantoms.Phantom
    source: sources.Source
    n_histories: int
    seed: int
    request_key: int = 0


def electron_20mev_wlw(n: int = 10_000) -> Workload:
    """20 MeV electron pencil beam normally incident at the centre of the top face
    of a 32x32x30 water-lung-water phantom of 0.5 cm voxels; Philox seed 1."""
    ph = phantoms.water_lung_water_32()
    x, y = ph.centre_xy()
    return Workload("e20_wlw_32x32x30", ph, sources.pencil(ELECTRON, 20.0, x, y), n, 1)


def photon_6mv_wbw(n: int = 10_000_000) -> Workload:
    """6 MV synthetic spectrum from a point source at SSD 100 cm with a 10x10 cm
    field on a 61x61x60 water-bone-water phantom of 0.5 cm voxels; seed 2."""
    ph = phantoms.water_bone_water_61()
    x, y = ph.centre_xy()
    src = sources.point_field(PHOTON, x, y, 100.0, 5.0, 5.0, spectrum=sources.spectrum_6mv())
    return Workload("g6mv_wbw_61x61x60", ph, src, n, 2)


def photon_6mv_random_field(n: int = 100_000_000) -> Workload:
    """6 MV as above on a 256x256x160 random-field phantom of 0.2 cm voxels
    (field seed 3, transport seed 3)."""
    ph = phantoms.random_field_phantom(256, 0.2, seed=3, nz=160)
    x, y = ph.centre_xy()
    src = sources.point_field(PHOTON, x, y, 100.0, 5.0, 5.0, spectrum=sources.spectrum_6mv())
    return Workload("g6mv_rf_256x256x160", ph, src, n, 3)


def photon_6mv_ct8(n: int = 40_000_000) -> Workload:
    """6 MV as above on a 128^3 random-field phantom of 0.25 cm voxels (field
    seed 52) mapped to the eight tissue classes (tissue_blob tables); seed 7."""
    ph = phantoms.random_field_phantom(128, 0.25, seed=52)
    ph.mat = phantoms.tissue_from_density(ph.rho)
    x, y = ph.centre_xy()
    src = sources.point_field(PHOTON, x, y, 100.0, 5.0, 5.0, spectrum=sources.spectrum_6mv())
    return Workload("g6mv_ct8_128", ph, src, n, 7)


def electron_20mev_point_field(ph, n: int) -> Workload:
    """20 MeV electrons from a point source at SSD 100 cm with a 10x10 cm field."""
    x, y = ph.centre_xy()
    src = sources.point_field(ELECTRON, x, y, 100.0, 5.0, 5.0, energy=20.0)
    return Workload("e20_field", ph, src, n, 1)


# ------------------------------------------------------------ serving workload

SERVING_PHANTOMS = ((64, 0.5, 51), (128, 0.25, 52), (256, 0.2, 53))   # (n, voxel cm, field seed)


def serving_phantoms(sizes=SERVING_PHANTOMS):
    """The resident pool of the serving workload: random-field phantoms of
    64^3 x 0.5 cm, 128^3 x 0.25 cm and 256^3 x 0.2 cm (32, 32 and 51.2 cm)."""
    return [phantoms.random_field_phantom(n, d, seed=s) for n, d, s in sizes]


@dataclass
class ServeRequest:
    index: int              # arrival index, also the Philox request key
    t: float                # arrival time, s
    phantom: int            # index into the pool
    particle: int           # PHOTON (6 MV spectrum) or ELECTRON (mono)
    energy: float           # electron energy, MeV (photons: 0)
    side: float             # square field side at the surface, cm
    target: float           # target sigma-bar (0.01 or 0.02)


def serving_requests(rate: float = 20.0, duration: float = 60.0, seed: int = 5, n_phantoms: int = 3):
    """Poisson arrivals (rate per s over `duration` s); each request draws a
    phantom, a source (6 MV photons or electrons of U(6, 20) MeV), a square
    field side U(1, 10) cm and a target sigma-bar of 2% or 1%."""
    times = sources.poisson_arrivals(rate, duration, seed)
    rng = np.random.default_rng(seed + 1000)
    out = []
    for i, t in enumerate(times):
        ph = int(rng.integers(n_phantoms))
        particle = PHOTON if rng.random() < 0.5 else ELECTRON
        energy = float(rng.uniform(6.0, 20.0))
        side = float(rng.uniform(1.0, 10.0))
        target = 0.02 if rng.random() < 0.5 else 0.01
        out.append(ServeRequest(i, float(t), ph, particle, energy if particle == ELECTRON else 0.0, side,
                                target))
    return out


def serving_source(ph, particle: int, energy: float, side: float) -> sources.Source:
    """Point source at SSD 100 cm above the centre, square field of `side` cm."""
    x, y = ph.centre_xy()
    if particle == PHOTON:
        return sources.point_field(PHOTON, x, y, 100.0, side / 2, side / 2, spectrum=sources.spectrum_6mv())
    return sources.point_field(ELECTRON, x, y, 100.0, side / 2, side / 2, energy=energy)


# ------------------------------------------------ the paper's own geometry

PAPER_SSD = 90.0       # cm, source to phantom surface
PAPER_SAD = 100.0      # cm, where the 10x10 cm field is defined


def paper_workload(particle: int, middle: str, n: int) -> Workload:
    """The paper's benchmark geometry (Sec. 3, Table 1) on the synthetic
    physics: 61x61x150 voxels of 0.5x0.5x0.2 cm with 5 cm water, 5 cm lung or
    bone and 20 cm water; a point source at SSD 90 cm whose 10x10 cm field is
    defined at SAD 100 cm (9x9 cm on the surface); 20 MeV electrons or the
    6 MV spectrum.  Seeds: 6 (electrons), 7 (photons)."""
    ph = phantoms.paper_slab_phantom(middle)
    x, y = ph.centre_xy()
    half = 5.0 * PAPER_SSD / PAPER_SAD
    if particle == PHOTON:
        src = sources.point_field(PHOTON, x, y, PAPER_SSD, half, half, spectrum=sources.spectrum_6mv())
        name, seed = f"paper_g6mv_w{middle[0]}w_61x61x150", 7
    else:
        src = sources.point_field(ELECTRON, x, y, PAPER_SSD, half, half, energy=20.0)
        name, seed = f"paper_e20_w{middle[0]}w_61x61x150", 6
    return Workload(name, ph, src, n, seed)
