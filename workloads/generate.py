"""Seeded synthetic orbital generators shared by the oracle tests and the HIP tests.

This module holds only input synthesis: random band-limited real functions on
a periodic grid.  It contains none of the exchange arithmetic (no pair
densities, no Coulomb kernel, no orthonormalisation); both the oracle and the
HIP path receive its output and orthonormalise it themselves.

Two families stand in for the paper's condensed-phase systems (bulk water,
Fe3+ in water, 32-128 H2O boxes; Computational Details):

* ``random_pw``: delocalised real orbitals with Gaussian random plane-wave
  coefficients c(G) = exp(-|G|^2/8) (a + i b)/sqrt(2), a, b ~ N(0,1), on the
  sphere |G|^2/2 <= ecut, with c(-G) = conj(c(G)) and c(0) real.
* ``gaussians``: localised real orbitals exp(-|r-R|^2 / 2 s^2) with centres R
  uniform in the cell and widths s uniform in [s_lo, s_hi], built in
  reciprocal space as exp(-s^2 G^2 / 2) exp(-i G.R) on |G|^2/2 <= ecut, which
  makes them periodic, band-limited and real.

Every orbital is scaled to unit norm dV sum psi^2 = 1.  Arrays are float64
``[orb, z, y, x]``.  The random stream is numpy's PCG64 ``default_rng(seed)``.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

__all__ = ["random_pw", "gaussians", "white_noise", "ifft_real", "fd_direction"]


def _int_freqs(n):
    return np.fft.fftfreq(n, d=1.0 / n).astype(np.int64)


def _gvecs(shape, box):
    nz, ny, nx = shape
    lx, ly, lz = box
    mz = _int_freqs(nz)[:, None, None]
    my = _int_freqs(ny)[None, :, None]
    mx = _int_freqs(nx)[None, None, :]
    gx = 2.0 * math.pi * mx / lx
    gy = 2.0 * math.pi * my / ly
    gz = 2.0 * math.pi * mz / lz
    return (mz, my, mx), (gz, gy, gx)


def ifft_real(coef):
    """psi(r_n) = sum_G c(G) exp(i G r_n) for Hermitian c; returns the real part."""
    out = sfft.ifftn(coef, workers=os.cpu_count() or 1) * coef.size
    return np.ascontiguousarray(out.real)


def _normalise(psi, dv):
    nrm = np.sqrt(dv * np.sum(psi.reshape(psi.shape[0], -1) ** 2, axis=1))
    return psi / nrm.reshape((-1,) + (1,) * (psi.ndim - 1))


def random_pw(shape, box, n_orb, ecut, seed):
    """Delocalised random plane-wave orbitals (see the module docstring)."""
    rng = np.random.default_rng(seed)
    (mz, my, mx), (gz, gy, gx) = _gvecs(shape, box)
    g2 = gz ** 2 + gy ** 2 + gx ** 2
    inside = 0.5 * g2 <= ecut
    # canonical half space: mz > 0, or mz == 0 and my > 0, or mz == my == 0 and mx > 0
    half = (mz > 0) | ((mz == 0) & (my > 0)) | ((mz == 0) & (my == 0) & (mx > 0))
    sel = np.argwhere(inside & half)
    amp = np.exp(-g2 / 8.0)
    dv = box[0] * box[1] * box[2] / float(np.prod(shape))
    out = np.empty((n_orb,) + tuple(shape))
    nz, ny, nx = shape
    for o in range(n_orb):
        coef = np.zeros(shape, dtype=np.complex128)
        a = rng.standard_normal(len(sel))
        b = rng.standard_normal(len(sel))
        c = (a + 1j * b) / math.sqrt(2.0)
        iz, iy, ix = sel[:, 0], sel[:, 1], sel[:, 2]
        coef[iz, iy, ix] = c * amp[iz, iy, ix]
        coef[(-iz) % nz, (-iy) % ny, (-ix) % nx] = np.conj(coef[iz, iy, ix])
        coef[0, 0, 0] = rng.standard_normal() * amp[0, 0, 0]
        out[o] = ifft_real(coef)
    return _normalise(out, dv)


def gaussians(shape, box, n_orb, ecut, seed, s_lo=1.2, s_hi=1.8):
    """Localised Gaussian orbitals at random centres (see the module docstring).

    Returns (psi, centres, widths).
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_orb, 3)) * np.asarray(box, float)
    widths = rng.uniform(s_lo, s_hi, size=n_orb)
    (_, _, _), (gz, gy, gx) = _gvecs(shape, box)
    g2 = gz ** 2 + gy ** 2 + gx ** 2
    inside = 0.5 * g2 <= ecut
    dv = box[0] * box[1] * box[2] / float(np.prod(shape))
    out = np.empty((n_orb,) + tuple(shape))
    for o in range(n_orb):
        # exp(-s^2 G^2 / 2) exp(-i G.R) factorises over the three axes
        rx, ry, rz = centres[o]
        s2 = 0.5 * widths[o] ** 2
        fx = np.exp(-s2 * gx ** 2 - 1j * gx * rx)
        fy = np.exp(-s2 * gy ** 2 - 1j * gy * ry)
        fz = np.exp(-s2 * gz ** 2 - 1j * gz * rz)
        coef = (fz * fy) * fx
        coef[~inside] = 0.0
        out[o] = ifft_real(coef)
    return _normalise(out, dv), centres, widths


def white_noise(shape, box, n_orb, seed):
    """Full-spectrum real orbitals: independent N(0, 1) values at every grid
    point, scaled to unit norm.  Not band-limited: their pair densities fill
    every frequency of the grid, the Nyquist planes included, unlike the two
    families above."""
    rng = np.random.default_rng(seed)
    dv = box[0] * box[1] * box[2] / float(np.prod(shape))
    return _normalise(rng.standard_normal(size=(n_orb,) + tuple(shape)), dv)


def fd_direction(shape, dv, seed, k):
    """Direction k of a seeded set of perturbations D[orb, z, y, x] for finite
    differences: independent N(0, 1) values (numpy PCG64 stream seed + k),
    scaled to dV sum D^2 = 1.  ``shape`` includes the orbital axis."""
    rng = np.random.default_rng(seed + k)
    d = rng.standard_normal(size=tuple(shape))
    return d / math.sqrt(dv * float(np.sum(d * d)))
