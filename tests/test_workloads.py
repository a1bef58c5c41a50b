"""Seeded input generators: determinism, normalisation, band limit, alias-free grids."""
import math

import numpy as np
import pytest

from workloads import configs, generate


def test_random_pw_deterministic_and_band_limited():
    shape, box = (24, 24, 24), (10.0, 10.0, 10.0)
    a = generate.random_pw(shape, box, 3, 5.0, seed=123)
    b = generate.random_pw(shape, box, 3, 5.0, seed=123)
    assert np.array_equal(a, b)
    dv = 1000.0 / 24 ** 3
    assert np.allclose(dv * np.sum(a.reshape(3, -1) ** 2, axis=1), 1.0, atol=1e-13)
    c = np.fft.fftn(a[0])
    m = np.fft.fftfreq(24, 1.0 / 24)
    g2 = (2 * math.pi / 10.0) ** 2 * (m[:, None, None] ** 2 + m[None, :, None] ** 2
                                      + m[None, None, :] ** 2)
    assert np.max(np.abs(c[0.5 * g2 > 5.0])) <= 1e-10 * np.max(np.abs(c))


def test_gaussians_localised():
    shape, box = (32, 32, 32), (12.0, 12.0, 12.0)
    psi, centres, widths = generate.gaussians(shape, box, 4, 20.0, seed=5)
    assert np.all((widths >= 1.2) & (widths <= 1.8))
    assert np.all((centres >= 0) & (centres < 12.0))
    # the maximum sits within one grid spacing (periodically) of the centre
    for o in range(4):
        iz, iy, ix = np.unravel_index(np.argmax(np.abs(psi[o])), shape)
        pos = np.array([ix, iy, iz]) * 12.0 / 32
        d = (pos - centres[o] + 6.0) % 12.0 - 6.0
        assert np.all(np.abs(d) <= 12.0 / 32 * 1.01)


@pytest.mark.parametrize("s", list(configs.ALL.values()), ids=lambda s: s.name)
def test_grids_alias_free(s):
    """Pair densities of orbitals band-limited to ecut fit the grid: 4 m_max + 1 <= n."""
    m_max = math.floor(math.sqrt(2 * s.ecut) * s.L / (2 * math.pi))
    assert 4 * m_max + 1 <= s.n
