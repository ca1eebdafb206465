"""Oracle pins: the counter-based generator and the trial-move distribution.

Philox4x32-10 (Salmon et al., SC'11) is pinned against an independent
implementation, PyTorch's header-only ``at::philox_engine`` compiled on the
host; its counter is (offset lo, offset hi, subsequence lo, subsequence hi)
and its key (seed lo, seed hi).  The trial direction (Appendix A: a uniformly
random new spin direction) is pinned by its distribution.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

_REF_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>
int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    at::philox_engine e(seed, sub, off);
    uint32_t a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
}
"""


def _torch_include():
    try:
        import torch
    except Exception:
        return None
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    return inc if os.path.exists(os.path.join(inc, "ATen/core/PhiloxRNGEngine.h")) else None


def test_philox_matches_independent_implementation(orc):
    inc = _torch_include()
    if inc is None:
        pytest.skip("PyTorch C++ headers not present")
    rng = np.random.default_rng(12345)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 2, 3, 4, 5, 6)]
    for _ in range(200):
        cases.append(tuple(int(v) for v in rng.integers(0, 2**32, size=6)))
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "ref.cpp")
        exe = os.path.join(td, "ref")
        open(src, "w").write(_REF_SRC)
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-I" + inc, src, "-o", exe])
        lines = []
        for c0, c1, c2, c3, k0, k1 in cases:
            seed = k0 | (k1 << 32)
            sub = c2 | (c3 << 32)
            off = c0 | (c1 << 32)
            lines.append("%d %d %d" % (seed, sub, off))
        out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True,
                             text=True, check=True).stdout.split("\n")
    for (c0, c1, c2, c3, k0, k1), line in zip(cases, out):
        ref = [int(v) for v in line.split()]
        assert orc.philox4x32_10([c0, c1, c2, c3], [k0, k1]) == ref


def test_u01_open_interval(orc):
    assert orc.lib().orc_u01(0) == 2.0 ** -33
    assert orc.lib().orc_u01(0xFFFFFFFF) == 1.0 - 2.0 ** -33
    assert 0.0 < orc.lib().orc_u01(0x80000000) < 1.0


def test_draw_counter_layout(orc):
    """draw(seed, replica, sweep, site, purpose) uses counter (site, sweep, replica, purpose)."""
    seed = 0x0123456789ABCDEF
    x = orc.philox4x32_10([7, 11, 3, 1], [seed & 0xFFFFFFFF, seed >> 32])
    u = orc.draw(seed, 3, 11, 7, 1)
    assert np.array_equal(u, (np.array(x, dtype=np.float64) + 0.5) * 2.0 ** -32)


def test_uniform_chi_square(orc):
    n = 40000
    u = np.array([orc.draw(99, 0, 0, i, 1) for i in range(n // 4)]).ravel()
    hist, _ = np.histogram(u, bins=50, range=(0, 1))
    chi2, p = stats.chisquare(hist)
    assert p > 1e-4, (chi2, p)


def test_direction_uniform_on_sphere(orc):
    n = 20000
    S = np.array([orc.direction(*orc.draw(5, 2, 9, i, 1)[:2]) for i in range(n)])
    assert np.allclose(np.linalg.norm(S, axis=1), 1.0, atol=1e-14)
    # Archimedes: z is uniform on [-1, 1]; azimuth uniform on [0, 2 pi)
    assert stats.kstest(S[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-4
    phi = np.mod(np.arctan2(S[:, 1], S[:, 0]), 2 * np.pi)
    assert stats.kstest(phi, "uniform", args=(0, 2 * np.pi)).pvalue > 1e-4
    # isotropic second moment: E[S S^T] = I / 3
    assert np.abs(S.T @ S / n - np.eye(3) / 3).max() < 0.02


def test_direction_poles(orc):
    assert np.allclose(orc.direction(0.5, 0.0), [1.0, 0.0, 0.0], atol=1e-15)
    assert np.allclose(orc.direction(0.5, 0.25), [0.0, 1.0, 0.0], atol=1e-15)
    S = orc.direction(2.0 ** -33, 0.1)
    assert S[2] == 1.0 - 2.0 ** -32 and abs(np.linalg.norm(S) - 1) < 1e-15
