"""The sampling facts behind the band-limited passes, checked on the generator's
orbitals with numpy FFTs (no library code).

Orbitals with plane waves only in (1/2)|G|^2 <= E_cut have integer frequencies
|m| <= floor(sqrt(2 E_cut) L / 2 pi) along each axis, so a pair density
psi_a psi_b has |k| <= k_max = 2 floor(sqrt(2 E_cut) L / 2 pi): the kz planes
beyond are empty (the skipped planes), and when 2 k_max + 1 <= n / 2 the even
grid points sample the pair density exactly: the length-n/2 DFT of the even
samples, doubled, equals the length-n DFT at every frequency |k| <= k_max
(frequency k lands on index k mod n/2).  The half-length forward z transform
of pass 1 and the half-height and half-width plane input of pass 2 rest on
this (along z, y and x; for a kz plane the even rows and columns together,
four times the quarter plane's 2D DFT); when the band does not fit, the
identity fails (aliasing), which the negative case shows.
"""
import math

import numpy as np
import pytest

from workloads import generate


def k_max(ecut, length):
    return 2 * math.floor(math.sqrt(2 * ecut) * length / (2 * math.pi) + 1e-9)


def _pair(n, box, ecut, seed):
    psi = generate.random_pw((n,) * 3, box, 3, ecut, seed)
    return psi[0] * psi[1]  # [z][y][x]


@pytest.mark.parametrize("n,L", [(64, 15.67), (96, 23.5), (120, 29.375)])
def test_pair_band_and_half_length_sampling(n, L):
    ecut = 5.0
    rho = _pair(n, (L,) * 3, ecut, seed=8100 + n)
    km = k_max(ecut, L)
    assert 2 * km + 1 <= n // 2
    freqs = np.fft.fftfreq(n, 1.0 / n).astype(int)
    # z (half-length forward z), y (half-height planes), x (half-width planes)
    for axis in (0, 1, 2):
        full = np.fft.fft(rho, axis=axis)
        scale = np.max(np.abs(full))
        out = np.abs(freqs) > km
        sl = [slice(None)] * 3
        sl[axis] = out
        # the pair band: nothing beyond k_max
        assert np.max(np.abs(full[tuple(sl)])) <= 1e-12 * scale
        even = [slice(None)] * 3
        even[axis] = slice(0, n, 2)
        half = 2.0 * np.fft.fft(rho[tuple(even)], axis=axis)
        for k in range(-km, km + 1):
            a = [slice(None)] * 3
            b = [slice(None)] * 3
            a[axis] = k % n
            b[axis] = k % (n // 2)
            assert np.max(np.abs(full[tuple(a)] - half[tuple(b)])) <= 1e-12 * scale


def test_half_length_sampling_fails_beyond_the_band():
    """20 Ha orbitals on 64^3 (L = 15.67): k_max = 30 > (n/2 - 1)/2, so the even
    points alias and the doubled half-length DFT differs from the full one."""
    n, L, ecut = 64, 15.67, 20.0
    rho = _pair(n, (L,) * 3, ecut, seed=8200)
    km = k_max(ecut, L)
    assert 2 * km + 1 > n // 2
    full = np.fft.fft(rho, axis=0)
    half = 2.0 * np.fft.fft(rho[0:n:2], axis=0)
    worst = max(np.max(np.abs(full[k % n] - half[k % (n // 2)])) for k in range(-15, 16))
    assert worst > 1e-3 * np.max(np.abs(full))


@pytest.mark.parametrize("n,L", [(72, 17.6), (108, 26.4)])
def test_quarter_plane_sampling(n, L):
    """The plane pass's quarter-plane input: a kz plane of a pair density
    (after the z transform) sampled at even y and even x; four times the
    (n/2 x n/2) DFT of those samples equals the plane's (n x n) DFT at every
    (ky, kx) in the band, half-length index k mapping to frequency k below n/4
    and to k - n/2 above it (the bin n/4 itself is beyond the band)."""
    ecut = 5.0
    rho = _pair(n, (L,) * 3, ecut, seed=8300 + n)
    km = k_max(ecut, L)
    assert 2 * km + 1 <= n // 2
    planes = np.fft.fft(rho, axis=0)
    h = n // 2
    for kz in (0, 1, km):
        plane = planes[kz]
        full = np.fft.fft2(plane)
        quarter = 4.0 * np.fft.fft2(plane[0::2, 0::2])
        scale = np.max(np.abs(full))
        assert np.max(np.abs(quarter[h // 2, :])) <= 1e-11 * scale
        assert np.max(np.abs(quarter[:, h // 2])) <= 1e-11 * scale
        for ky in range(h):
            for kx in range(h):
                if ky == h // 2 or kx == h // 2:
                    continue
                fy = ky if 2 * ky < h else ky - h
                fx = kx if 2 * kx < h else kx - h
                # in the band the two agree; beyond it (|f| > k_max) both vanish
                assert abs(full[fy % n, fx % n] - quarter[ky, kx]) <= 1e-11 * scale
