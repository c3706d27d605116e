"""The synthetic workloads: phantoms and sources shaped like the paper's slab and
point-source experiments (Sec. 3), at the sizes this engine is measured on."""
from __future__ import annotations

from dataclasses import dataclass

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


def electron_20mev_point_field(ph, n: int) -> Workload:
    """20 MeV electrons from a point source at SSD 100 cm with a 10x10 cm field."""
    x, y = ph.centre_xy()
    src = sources.point_field(ELECTRON, x, y, 100.0, 5.0, 5.0, energy=20.0)
    return Workload("e20_field", ph, src, n, 1)
