"""Host logic of the autotuner: search space, workload keys and the JSON cache."""
from paper_0910_0329_amd import autotune
from paper_0910_0329_amd.inputs import sources
from paper_0910_0329_amd.inputs.sources import ELECTRON, PHOTON


def items():
    g = sources.point_field(PHOTON, 0, 0, 100.0, 1, 1, spectrum=sources.spectrum_6mv())
    e = sources.pencil(ELECTRON, 10.0, 0, 0)
    return [(g, 50_000, 0), (e, 20_000, 1)]


def test_candidates_cover_the_space():
    c = list(autotune.candidates())
    # chunk sizes only with queues (regroup 1), table placement only with wave stacks (3)
    assert len(c) == (4 + 1 + 2) * 2
    assert len({tuple(sorted(d.items())) for d in c}) == len(c)
    assert {"regroup", "chunk_per_lane", "block_size", "table_placement"} == set(c[0])
    assert all(d["table_placement"] == 1 for d in c if d["regroup"] != 3)
    assert {d["table_placement"] for d in c if d["regroup"] == 3} == {1, 2}
    assert all(d["chunk_per_lane"] == 8 for d in c if d["regroup"] != 1)


def test_occupancy_candidates_below_the_resident_count():
    shape = {"grid_blocks": 512, "block_size": 512, "cu_count": 256, "resident_per_cu": 4}
    assert autotune.occupancy_candidates(shape) == [{"grid_blocks": 256}, {"grid_blocks": 512},
                                                   {"grid_blocks": 768}]
    assert autotune.occupancy_candidates({**shape, "resident_per_cu": 0}) == []
    assert autotune.occupancy_candidates({**shape, "resident_per_cu": 1}) == []


def test_workload_key_depends_on_shape_and_mix():
    k = autotune.workload_key("dev", 1000, items())
    assert k == autotune.workload_key("dev", 1000, items())
    assert k != autotune.workload_key("dev", 1001, items())
    assert k != autotune.workload_key("dev2", 1000, items())
    assert k != autotune.workload_key("dev", 1000, items()[:1])


def test_scaled_keeps_a_floor():
    s = autotune.scaled(items(), 8, 10_000)
    assert [n for _, n, _ in s] == [10_000, 10_000]
    s = autotune.scaled(items(), 2, 100)
    assert [n for _, n, _ in s] == [25_000, 10_000]


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(p) == {}
    autotune.store_cache("a", {"opts": {"regroup": 2}}, p)
    autotune.store_cache("b", {"opts": {"regroup": 1}}, p)
    d = autotune.load_cache(p)
    assert d["a"]["opts"] == {"regroup": 2} and d["b"]["opts"] == {"regroup": 1}
    with open(p, "w") as f:
        f.write("not json")
    assert autotune.load_cache(p) == {}
