"""Pins of the oracle's random numbers: Philox4x32-10 against rocRAND's own
engine (a third-party implementation, built from its header on the host),
and the samplers against scipy's distributions."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  // stdin: lines "c0 c1 c2 c3 k0 k1" (hex); stdout: 4 hex words each
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long v = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
    rocrand_device::philox4x32_10_engine e(seed, subseq, 0);
    // advance the 64-bit block counter by v blocks of 4 numbers; one call
    // can skip fewer than 2^64 numbers, so take the blocks in four quarters
    for (int q = 0; q < 4; ++q) e.discard(4ull * (v >> 2));
    for (unsigned i = 0; i < (unsigned)(v & 3); ++i) e.discard(4ull);
    uint4 r = e.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_probe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "probe.cpp")
    exe = os.path.join(d, "probe")
    with open(src, "w") as f:
        f.write(ROCRAND_PROBE)
    subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_probe):
    rng = np.random.default_rng(0)
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6, [1, 2, 3, 4, 5, 6]]
    rows += rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64).tolist()
    # the counter layout the filters use: (slot, time, stream, attempt)
    rows += [[j, t, s, a, 7, 0] for j in (0, 1, 1023, 2**26 - 1) for t in (0, 1, 999)
             for s in (1, 2, 3, 4, 5, 16, 17) for a in (0, 1, 7)]
    inp = "\n".join(" ".join("%x" % v for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for r, line in zip(rows, out):
        want = [int(v, 16) for v in line.split()]
        assert orc.philox(r[:4], r[4:]) == want, r


def test_uniform_maps_open_interval(orc):
    for w in (0, 1, 255, 256, 2**31, 2**32 - 1):
        a, b = orc.u32(w), orc.u24(w)
        assert 0.0 < a < 1.0 and 0.0 < b < 1.0
        assert a == (w + 0.5) / 2**32
        assert b == ((w >> 8) + 0.5) / 2**24
        assert np.float32(b) == b  # exactly representable in single precision


def _philox_uniforms(orc, n, stream, fp32):
    out = []
    for j in range(n):
        w = orc.philox([j, 1, stream, 0], [11, 0])
        out.append([orc.u24(v) if fp32 else orc.u32(v) for v in w])
    return np.array(out)


@pytest.mark.parametrize("fp32", [False, True])
def test_box_muller_is_standard_normal(orc, fp32):
    u = _philox_uniforms(orc, 20000, 2, fp32)
    z = np.array([orc.box_muller(a, b) for a, b in u[:, :2]])
    for col in (0, 1):
        assert stats.kstest(z[:, col], "norm").pvalue > 1e-4
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.04


@pytest.mark.parametrize("a", [1.0, 2.0, 2.5, 10.0, 252.0])
@pytest.mark.parametrize("fp32", [False, True])
def test_marsaglia_tsang_gamma(orc, a, fp32):
    u = _philox_uniforms(orc, 20000, 3, fp32)
    g = []
    for j, row in enumerate(u):
        z0 = orc.box_muller(row[0], row[1])[0]
        g.append(orc.gamma_mt(a, z0, row[2], seed=11, j=j, t=1, g=0, fp32=fp32))
    g = np.array(g)
    assert stats.kstest(g, stats.gamma(a).cdf).pvalue > 1e-4
    # inverse gamma by reciprocal: IG(a, b) = b / Gamma(a)
    b = 3.0
    assert stats.kstest(b / g, stats.invgamma(a, scale=b).cdf).pvalue > 1e-4


def test_gamma_retries_use_their_own_stream(orc):
    # a first attempt that must be rejected (1 + c z <= 0) falls through to
    # the retry stream, which still yields a positive draw
    v = orc.gamma_mt(2.0, -100.0, 0.5, seed=3, j=5, t=7, g=1)
    assert v > 0
    assert v != orc.gamma_mt(2.0, -100.0, 0.5, seed=3, j=5, t=7, g=0)
