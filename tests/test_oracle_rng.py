"""Pins of the oracle's random numbers: Philox4x32-10 against rocRAND's
independent implementation, the uniform conversion, and lineage substreams."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>
// Reads (k0, k1, c0, c1, c2, c3) records and writes rocRAND's Philox4x32-10
// block for key (k0, k1) and counter (c0, c1, c2, c3), calling the engine's own
// ten-round bijection.
struct Probe : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  uint32_t in[6];
  Probe p;
  while (fread(in, 4, 6, stdin) == 6) {
    uint4 r = p.block(uint4{in[2], in[3], in[4], in[5]}, uint2{in[0], in[1]});
    uint32_t o[4] = {r.x, r.y, r.z, r.w};
    fwrite(o, 4, 4, stdout);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_probe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h") or not os.path.exists(hipcc):
        pytest.skip("rocRAND headers or hipcc not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "probe.cpp")
    exe = os.path.join(d, "probe")
    open(src, "w").write(ROCRAND_PROBE)
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_probe):
    rng = np.random.default_rng(123)
    n = 20000
    recs = rng.integers(0, 2 ** 32, size=(n, 6), dtype=np.uint64).astype(np.uint32)
    recs[:100, 2:] = 0                       # small counters too
    recs[100:200, 5] = 0x80000000 | np.arange(100, dtype=np.uint32)
    out = subprocess.run([rocrand_probe], input=recs.tobytes(), capture_output=True, check=True).stdout
    ref = np.frombuffer(out, dtype=np.uint32).reshape(n, 4)
    for i in range(n):
        k0, k1, c0, c1, c2, c3 = (int(x) for x in recs[i])
        assert oracle.philox(k0, k1, (c0, c1, c2, c3)) == tuple(int(x) for x in ref[i]), i


def test_uniform_conversion_is_exact_and_open():
    for x in (0, 1, 255, 256, 0x7FFFFFFF, 0xFFFFFF00, 0xFFFFFFFF):
        u = oracle.uniform(x)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u          # exactly representable in FP32
        assert u == ((x >> 9) + 0.5) / 2 ** 23
        assert float(np.float32(1.0) - np.float32(u)) == 1.0 - u   # so is 1 - u
    assert oracle.uniform(0) == 2.0 ** -24
    assert oracle.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    # every value on the 2^-23 lattice shifted by half a step is exact in FP32
    ks = np.arange(0, 2 ** 23, 997, dtype=np.float64)
    us = (ks + 0.5) / 2 ** 23
    np.testing.assert_array_equal(us.astype(np.float32).astype(np.float64), us)


def test_uniform_moments_of_a_stream():
    xs = [oracle.philox(7, 9, (h, 0, 0, b)) for h in range(200) for b in range(50)]
    u = np.array([oracle.uniform(w) for blk in xs for w in blk])
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / len(u))
    assert abs((u * u).mean() - 1 / 3) < 4 * np.sqrt(4 / 45 / len(u))
    hist = np.bincount((u * 16).astype(int), minlength=16)
    exp = len(u) / 16
    assert ((hist - exp) ** 2 / exp).sum() < 50        # chi2 with 15 dof, p ~ 1e-5


def test_keys_and_lineages_give_distinct_streams():
    base = oracle.philox(1, 0, (5, 0, 0, 1))
    assert oracle.philox(1, 1, (5, 0, 0, 1)) != base        # request key
    assert oracle.philox(2, 0, (5, 0, 0, 1)) != base        # seed
    assert oracle.philox(1, 0, (6, 0, 0, 1)) != base        # history
    assert oracle.philox(1, 0, (5, 1, 0, 1)) != base        # lineage
    assert oracle.philox(1, 0, (5, 0, 0, 0x80000000)) != oracle.philox(1, 0, (5, 0, 0, 0))
