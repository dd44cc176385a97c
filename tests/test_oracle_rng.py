"""Pins of the oracle's random-number layer (CPU only).

The paper draws its bivariate-normal scattering pairs from C rand() uniforms through the
Marsaglia polar method and a covariance transform (Sec. II-B).  The oracle replaces
rand() by the counter-based Philox4x32-10 generator; these tests pin that generator to
an independent implementation (rocRAND's, compiled from its header) and pin the
transforms to their distributions.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "golden", "philox_rocrand_ref.cpp")],
                          cwd=str(tmp_path_factory.getbasetemp()))
    return exe


def test_philox_matches_rocrand(oracle, rocrand_ref):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 0, 0, 0, 0, 0), (0, 0, 0, 1, 0, 0),
             (0, 0, 0, 0, 0, 1)]
    cases += [tuple(int(v) for v in rng.integers(0, 2**32, 6, dtype=np.uint64)) for _ in range(200)]
    inp = "\n".join(" ".join(f"{v:x}" for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [[int(v, 16) for v in line.split()] for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        assert oracle.philox4x32_10(c[:4], c[4:]) == r, c


def test_draw64_layout(oracle):
    # counter (draw, stream, g_lo, g_hi), key (seed_lo, seed_hi); words (o0|o1<<32, o2|o3<<32)
    seed, stream, g, draw = 0x0123456789ABCDEF, 3, (5 << 32) | 17, 2
    o = oracle.philox4x32_10([draw, stream, g & 0xFFFFFFFF, g >> 32], [seed & 0xFFFFFFFF, seed >> 32])
    w0, w1 = oracle.draw64(seed, stream, g, draw)
    assert w0 == o[0] | (o[1] << 32)
    assert w1 == o[2] | (o[3] << 32)


def test_uniform53_edges(oracle):
    assert oracle.uniform53(0) == 0.0
    assert oracle.uniform53(2**64 - 1) == 1.0 - 2.0**-53
    assert oracle.uniform53(1 << 63) == 0.5
    assert oracle.uniform53((1 << 11) - 1) == 0.0  # low 11 bits are discarded


def test_offsets_uniform_ks(oracle):
    n = 50_000
    u = np.array([oracle.uniform53(oracle.draw64(12369, 0, g, 0)[0]) for g in range(n)])
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    v = np.array([oracle.uniform53(oracle.draw64(12369, 0, g, 0)[1]) for g in range(n)])
    assert stats.kstest(v, "uniform").pvalue > 1e-3
    # the two words of one draw are uncorrelated
    assert abs(np.corrcoef(u, v)[0, 1]) < 4.0 / math.sqrt(n)


def test_polar_normals(oracle):
    n = 100_000
    z = np.array([oracle.normal_pair(99, 2, g) for g in range(n)])
    z1, z2, att = z[:, 0], z[:, 1], z[:, 2]
    se = 1.0 / math.sqrt(n)
    assert abs(z1.mean()) < 4 * se and abs(z2.mean()) < 4 * se
    assert abs(z1.var() - 1.0) < 4 * math.sqrt(2.0 / n)
    assert abs(z2.var() - 1.0) < 4 * math.sqrt(2.0 / n)
    assert abs(np.corrcoef(z1, z2)[0, 1]) < 4 * se
    assert stats.kstest(z1, "norm").pvalue > 1e-3
    # acceptance probability of the polar method is pi/4: attempts are geometric
    p_acc = 1.0 / att.mean()
    assert abs(p_acc - math.pi / 4) < 4 * math.sqrt(p_acc * (1 - p_acc) / n) * 1.5
    assert att.min() >= 1


def test_bivariate_pair_correlation():
    """The covariance transform the oracle uses for the exit pair,
    (lat, ang) = (s_l z1, s_a (rho z1 + sqrt(1-rho^2) z2)), has the bivariate normal
    density of the paper with correlation rho (Sec. II-B): checked on normals from a
    library generator, independent of the oracle."""
    rng = np.random.default_rng(3)
    z1, z2 = rng.standard_normal((2, 200_000))
    for rho in (0.0, 0.5, math.sqrt(3) / 2):
        lat = 1.0 * z1
        ang = 0.01 * (rho * z1 + math.sqrt(1 - rho * rho) * z2)
        assert abs(np.corrcoef(lat, ang)[0, 1] - rho) < 0.01
        assert abs(ang.std() - 0.01) < 1e-4


def test_angle_table(oracle):
    for k, (c, s) in enumerate([(1, 0), (0, 1), (-1, 0), (0, -1), (1, 0)]):
        assert oracle.angle(0.0, 90.0, k) == (c, s)
    assert oracle.angle(-90.0, 0.0, 0) == (0.0, -1.0)
    for k in range(0, 360, 7):
        c, s = oracle.angle(0.5, 1.0, k)
        phi = math.radians(0.5 + k)
        assert abs(c - math.cos(phi)) < 1e-15 and abs(s - math.sin(phi)) < 1e-15


@pytest.mark.parametrize("P,K", [(10, 3), (92160, 90), (10_000_000, 90), (7, 7), (5, 9), (100_000_000, 180)])
def test_angle_major_split(oracle, P, K):
    """Angle k holds protons [floor(kP/K), floor((k+1)P/K)): brute force at the bounds."""
    starts = [(k * P) // K for k in range(K + 1)]
    for k in range(K):
        lo, hi = starts[k], starts[k + 1]
        for g in {lo, hi - 1, (lo + hi) // 2}:
            if lo <= g < hi:
                assert oracle.angle_of(g, P, K) == k
    assert sum(starts[k + 1] - starts[k] for k in range(K)) == P
