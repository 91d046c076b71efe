"""Pins of the oracle's pattern statistic (test infrastructure for the long
spinodal run, where pointwise parity ends at the FP32 chaotic horizon).

The radially averaged autocorrelation of a plane wave cos(k x) is, in the
continuum, the Bessel function J0(k r); the lattice ring average must put
its first zero at r = j_{0,1} / k within the binning error of the rings.
"""
import numpy as np
import pytest
from scipy.special import jn_zeros

import oracle as O


@pytest.mark.parametrize("lam,n,transpose", [(64, 256, False), (32, 256, True), (48, 192, False)])
def test_domain_size_of_a_plane_wave(lam, n, transpose):
    x = np.arange(n)
    phi = np.cos(2 * np.pi * x / lam)[None, :] * np.ones((n, 1))
    if transpose:
        phi = phi.T.copy()
    C = O.radial_correlation(phi)
    assert C[0] == pytest.approx(1.0, abs=1e-15)
    r0 = jn_zeros(0, 1)[0] * lam / (2 * np.pi)
    assert abs(O.domain_size(phi) - r0) < 0.01 * r0


def test_domain_size_scales_with_the_pattern():
    """A pattern stretched by 2 on a lattice twice as large has twice the size."""
    r = np.random.default_rng(5)
    base = r.standard_normal((64, 64))
    # smooth it (periodic box filter) so that domains span several nodes
    for _ in range(6):
        base = (base + np.roll(base, 1, 0) + np.roll(base, -1, 0) + np.roll(base, 1, 1)
                + np.roll(base, -1, 1)) / 5
    big = np.kron(base, np.ones((2, 2)))
    L1, L2 = O.domain_size(base), O.domain_size(big)
    assert abs(L2 / L1 - 2.0) < 0.05, (L1, L2)
