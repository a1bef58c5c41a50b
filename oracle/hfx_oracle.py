"""CPU FP64 oracle for plane-wave Gamma-point Hartree-Fock exact exchange.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the HIP library (``paper_2309_00651_amd``) and never imports it.

What it computes (Methods, "MTACE Method for H-AIMD Simulation"):

* Eq. (vx):  V_X psi_i = - sum_j v_ij(r) psi_j                       (apply)
* Eq. (vij): v_ij(r)   = <psi_j | 1/r12 | psi_i>, the Coulomb potential of
             the pair density rho_ij = psi_i psi_j (a Poisson solve)
* Eq. (HFX): the exchange energy (prefactor reading below)
* ACE matrix M_kl = <psi_k | V_X | psi_l>  (same subsection, definition of M)
* ACE operator, Eq. (vx_ace): V_X^ACE = - sum_k |P_k><P_k| with P = W L^(-T),
  W_i = V_X psi_i and -M = L L^T (Cholesky)
* s-MTACE screening (same Methods subsection): only pairs with
  int |phi_i phi_j| dr >= rho_cut enter the exchange sums
* SCDM localisation of the orbitals the screening acts on (the same
  subsection cites the selected-columns-of-the-density-matrix method of
  Damle, Lin and Ying, 2015, without restating it; reading 6 below)

The FFT evaluates the periodic discrete convolution exactly up to rounding,
so the oracle is the plain definition written out, one pair at a time, in
float64, with numpy/scipy FFTs as the only library primitive.

Readings of points the paper leaves open (each repeated where it is used):

1. Energy prefactor.  The paper's Eq. (HFX) sums <psi_i|v_ij|psi_j> over all
   ordered pairs without a 1/2; we report the spin-orbital value
   E_x = 1/2 sum_i <psi_i | K psi_i> = -1/2 sum_ij e_ij, i.e. half of the
   paper's closed-shell sum.  No hybrid mixing fraction is applied.
2. Sign.  K == V_X (negative semidefinite), so E_x <= 0 and
   dE_x/dpsi_i(r_n) = 2 dV (K psi_i)(r_n).
3. Periodic kernel.  The paper writes only 1/r12.  Two periodic kernels:
   spherically truncated Coulomb v(G) = 4pi/G^2 (1 - cos G Rc),
   v(0) = 2 pi Rc^2, Rc = (3 Omega / 4 pi)^(1/3); and erfc-screened
   v(G) = 4pi/G^2 (1 - exp(-G^2 / 4 w^2)), v(0) = pi / w^2.  Evaluated in the
   cancellation-free forms 8 pi sin^2(G Rc / 2) / G^2 and
   -4 pi expm1(-G^2/4w^2) / G^2.
4. FFT convention.  rho~(G) = (1/N_r) sum_n rho(r_n) exp(-i G r_n);
   f(r_n) = sum_G f~(G) exp(+i G r_n).
5. Inner product.  <f|g> = dV sum_n f(r_n) g(r_n), dV = Omega / N_r.
6. SCDM (Gamma point, real orbitals).  Grid points c_1..c_N are selected by
   column-pivoted QR of the N_orb x N_r matrix Psi^T: step k takes the column
   (grid point) whose residual after projecting out the columns selected so
   far has the largest norm (ties: the smallest index).  The localised
   functions are the density-matrix columns at those points,
   xi_k(r) = sum_i psi_i(r) psi_i(c_k), orthonormalised by Loewdin.

Array layout: orbitals are float64 arrays ``psi[orb, z, y, x]`` (x fastest);
``box`` is (Lx, Ly, Lz) in bohr.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

__all__ = [
    "TRUNCATED", "ERFC", "volume", "grid_g2", "coulomb_kernel",
    "pair_potential", "pair_energy", "exchange", "apply_exchange_rows",
    "exchange_matrix", "overlap", "lowdin", "cholesky_orthonormalize",
    "ace_projectors", "ace_apply", "pair_overlap_abs", "screen_pairs",
    "scdm_pivots", "scdm",
]

TRUNCATED = 0
ERFC = 1


def volume(box):
    """Cell volume Omega of an orthorhombic box (Lx, Ly, Lz)."""
    return float(box[0]) * float(box[1]) * float(box[2])


def grid_g2(shape, box):
    """|G|^2 on the FFT grid, array [z, y, x].

    ``shape`` is (nz, ny, nx).  G = 2 pi (mx/Lx, my/Ly, mz/Lz) with the
    integer m in numpy's FFT order (0..n/2-1, -n/2..-1).
    """
    nz, ny, nx = shape
    lx, ly, lz = box
    mx = np.fft.fftfreq(nx, d=1.0 / nx)
    my = np.fft.fftfreq(ny, d=1.0 / ny)
    mz = np.fft.fftfreq(nz, d=1.0 / nz)
    gx = 2.0 * math.pi * mx / lx
    gy = 2.0 * math.pi * my / ly
    gz = 2.0 * math.pi * mz / lz
    return (gz[:, None, None] ** 2 + gy[None, :, None] ** 2
            + gx[None, None, :] ** 2)


def coulomb_kernel(shape, box, kind, param=0.0):
    """Periodic Coulomb kernel v(G) in float64 (reading 3 in the header).

    kind TRUNCATED: v = 8 pi sin^2(|G| Rc / 2) / G^2, v(0) = 2 pi Rc^2,
                    Rc = (3 Omega / 4 pi)^(1/3); ``param`` ignored.
    kind ERFC:      v = -4 pi expm1(-G^2 / 4 w^2) / G^2, v(0) = pi / w^2,
                    w = ``param`` (bohr^-1).
    """
    g2 = grid_g2(shape, box)
    v = np.empty_like(g2)
    nz0 = g2 > 0.0
    if kind == TRUNCATED:
        rc = (3.0 * volume(box) / (4.0 * math.pi)) ** (1.0 / 3.0)
        g = np.sqrt(g2[nz0])
        v[nz0] = 8.0 * math.pi * np.sin(0.5 * g * rc) ** 2 / g2[nz0]
        v[~nz0] = 2.0 * math.pi * rc * rc
    elif kind == ERFC:
        w = float(param)
        if not w > 0.0:
            raise ValueError("erfc kernel needs w > 0")
        v[nz0] = -4.0 * math.pi * np.expm1(-g2[nz0] / (4.0 * w * w)) / g2[nz0]
        v[~nz0] = math.pi / (w * w)
    else:
        raise ValueError(f"unknown kernel kind {kind!r}")
    return v


def pair_potential(rho, vg):
    """v(r) = sum_G v(G) rho~(G) exp(iGr) for a real density rho[z,y,x].

    Eq. (vij) solved in reciprocal space with the conventions of reading 4:
    forward transform divided by N_r, inverse transform unnormalised.
    """
    nr = rho.size
    rho_g = sfft.fftn(rho) / nr
    pot = sfft.ifftn(vg * rho_g) * nr
    imag = np.max(np.abs(pot.imag)) if pot.size else 0.0
    scale = np.max(np.abs(pot.real)) if pot.size else 0.0
    if imag > 1e-10 * max(scale, 1e-300):
        raise AssertionError("pair potential is not real: kernel not even?")
    return pot.real


def pair_energy(psi_i, psi_j, vg, dv):
    """e_ij = <rho_ij | v_ij> = dV sum_n rho_ij(r_n) v_ij(r_n)."""
    rho = psi_i * psi_j
    return dv * float(np.sum(rho * pair_potential(rho, vg)))


_FORKED = {}  # inputs of a forked pool, inherited by its workers (not pickled)


def _rows_worker(args):
    psi, vg, dv, rows, want_kpsi, keep = args
    n_orb = psi.shape[0]
    kpsi = np.zeros_like(psi) if want_kpsi else None
    e = np.zeros((n_orb, n_orb))
    for i in rows:
        for j in range(i, n_orb):
            if keep is not None and not keep[i, j]:
                continue                      # screened pair (s-MTACE)
            rho = psi[i] * psi[j]
            vij = pair_potential(rho, vg)
            e_ij = dv * float(np.sum(rho * vij))
            e[i, j] = e_ij
            e[j, i] = e_ij
            if want_kpsi:
                # Eq. (vx): V_X psi_i = -sum_j v_ij psi_j, and v_ij = v_ji.
                kpsi[i] -= vij * psi[j]
                if j != i:
                    kpsi[j] -= vij * psi[i]
    return kpsi, e


def _forked_rows(rows):
    f = _FORKED
    return _rows_worker((f["psi"], f["vg"], f["dv"], rows, f["want_kpsi"], f["keep"]))


def exchange(psi, box, vg, want_kpsi=True, workers=1, keep=None):
    """Exact exchange of real orbitals psi[orb, z, y, x] (float64).

    Returns a dict with
      ``ex``    E_x = -1/2 sum_{i,j} e_ij   (reading 1)
      ``e``     the symmetric matrix of pair energies e_ij (all >= 0)
      ``kpsi``  K psi_i = -sum_j v_ij psi_j (Eq. vx), or None
      ``dv``    the volume element Omega / N_r

    Pairs i <= j are evaluated once each; v_ij = v_ji because the pair density
    is symmetric in (i, j).  ``workers`` > 1 splits the rows i over forked
    processes; their private K psi blocks are summed in a fixed order.
    ``keep`` (symmetric boolean N_orb x N_orb, optional) restricts the sums
    to the pairs it marks, as the s-MTACE screening does (``screen_pairs``).
    """
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    n_orb = psi.shape[0]
    dv = volume(box) / psi[0].size
    if workers <= 1 or n_orb < 2:
        kpsi, e = _rows_worker((psi, vg, dv, range(n_orb), want_kpsi, keep))
    else:
        import multiprocessing as mp
        # Balance rows: row i has n_orb - i pairs; deal them round-robin.
        chunks = [list(range(w, n_orb, workers)) for w in range(workers)]
        # The workers inherit the inputs through fork (copy-on-write) instead
        # of receiving pickled copies, so a multi-GB Psi is held once.
        _FORKED.update(psi=psi, vg=vg, dv=dv, want_kpsi=want_kpsi, keep=keep)
        try:
            ctx = mp.get_context("fork")
            with ctx.Pool(workers) as pool:
                parts = pool.map(_forked_rows, chunks)
        finally:
            _FORKED.clear()
        kpsi = np.zeros_like(psi) if want_kpsi else None
        e = np.zeros((n_orb, n_orb))
        for kp, ep in parts:          # fixed summation order
            if want_kpsi:
                kpsi += kp
            e += ep
    ex = -0.5 * float(np.sum(e))
    return {"ex": ex, "e": e, "kpsi": kpsi, "dv": dv}


def apply_exchange_rows(psi, box, vg, rows, keep=None):
    """K psi_i = -sum_j v_ij psi_j for the selected orbitals only.

    Lets a full-size run be checked on a sample of orbitals: each row costs
    N_orb pair potentials.  ``keep`` (symmetric boolean, optional) restricts
    the sum to the kept pairs (i, j), as in ``exchange``.
    """
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    out = np.zeros((len(rows),) + psi.shape[1:])
    for r, i in enumerate(rows):
        for j in range(psi.shape[0]):
            if keep is not None and not keep[i, j]:
                continue                      # screened pair (s-MTACE)
            out[r] -= pair_potential(psi[i] * psi[j], vg) * psi[j]
    return out


def exchange_matrix(psi, kpsi, dv):
    """M_kl = <psi_k | K psi_l> = dV (Psi^T K Psi)_kl (the ACE matrix M)."""
    a = psi.reshape(psi.shape[0], -1)
    b = kpsi.reshape(kpsi.shape[0], -1)
    return dv * (a @ b.T)


def overlap(psi, dv):
    """S_kl = <psi_k | psi_l> = dV sum_n psi_k psi_l."""
    a = psi.reshape(psi.shape[0], -1)
    return dv * (a @ a.T)


def lowdin(psi, dv):
    """Loewdin (symmetric) orthonormalisation: Psi <- Psi S^(-1/2).

    S^(-1/2) from the eigendecomposition S = U diag(l) U^T.  The Kohn-Sham
    orbitals the exchange operator acts on are orthonormal (Methods, the
    occupied set in the definition of V_X).
    """
    s = overlap(psi, dv)
    lam, u = np.linalg.eigh(s)
    if lam[0] <= 0.0:
        raise ValueError("overlap matrix is not positive definite")
    s_mhalf = (u * lam ** -0.5) @ u.T
    out = s_mhalf @ psi.reshape(psi.shape[0], -1)
    return out.reshape(psi.shape), float(lam[0])


def cholesky_orthonormalize(psi, dv):
    """Psi <- Psi L^(-T) with S = L L^T (Cholesky orthonormalisation)."""
    s = overlap(psi, dv)
    low = np.linalg.cholesky(s)
    a = psi.reshape(psi.shape[0], -1)
    out = np.linalg.solve(low, a)
    return out.reshape(psi.shape)


def ace_projectors(kpsi, m):
    """P = W L^(-T) of Eq. (vx_ace): W_i = V_X psi_i (rows of ``kpsi``), L the
    lower Cholesky factor of -M.  Returned as rows, P[k] = |P_k>, i.e. the
    rows of L^(-1) W (column k of W L^(-T) is sum_i W_i (L^(-1))_ki).
    Raises if -M is not positive definite."""
    low = np.linalg.cholesky(-np.asarray(m, dtype=np.float64))
    w = kpsi.reshape(kpsi.shape[0], -1).astype(np.float64)
    return np.linalg.solve(low, w).reshape(kpsi.shape)


def ace_apply(p, phi, dv):
    """V_X^ACE phi_j = - sum_k P_k <P_k | phi_j> for every row of ``phi``
    (Eq. (vx_ace), inner product of reading 5)."""
    a = p.reshape(p.shape[0], -1)
    b = phi.reshape(phi.shape[0], -1)
    c = dv * (a @ b.T)          # <P_k | phi_j>
    return (-(c.T @ a)).reshape(phi.shape)


def pair_overlap_abs(psi, dv):
    """A_ij = int |phi_i(r) phi_j(r)| dr = dV sum_n |phi_i| |phi_j| (the
    quantity the s-MTACE screening compares with rho_cut)."""
    a = np.abs(psi.reshape(psi.shape[0], -1))
    return dv * (a @ a.T)


def screen_pairs(psi, dv, rho_cut):
    """Pairs kept by the s-MTACE criterion A_ij >= rho_cut (symmetric boolean
    matrix; the diagonal of normalised orbitals is 1 and always kept for
    rho_cut <= 1)."""
    return pair_overlap_abs(psi, dv) >= rho_cut


def scdm_pivots(psi):
    """Grid points selected by column-pivoted QR of Psi^T (reading 6).

    Plain greedy definition: keep the residual matrix R (initially Psi^T,
    N_orb x N_r), pick the column of largest norm, normalise it to q and
    remove its component from every column, R <- R - q (q^T R).  Returns the
    flat point indices c_1..c_N and, for each step, the relative gap between
    the largest and the second-largest residual norm (a tie test for callers
    that compare pivots computed in another summation order)."""
    r = np.array(psi.reshape(psi.shape[0], -1), dtype=np.float64)
    n = r.shape[0]
    piv, gaps = [], []
    taken = np.zeros(r.shape[1], dtype=bool)
    for _ in range(n):
        norms = np.einsum("ij,ij->j", r, r)
        norms[taken] = -1.0
        p = int(np.argmax(norms))            # first index among equal maxima
        top = norms[p]
        norms[p] = -1.0
        gaps.append((top - norms.max()) / top)
        q = r[:, p] / math.sqrt(top)
        r -= np.outer(q, q @ r)
        taken[p] = True
        piv.append(p)
    return np.array(piv), np.array(gaps)


def scdm(psi, dv):
    """SCDM-localised orthonormal orbitals (reading 6): xi_k = sum_i psi_i
    psi_i(c_k) at the pivots c_k of ``scdm_pivots``, then Loewdin in the
    dV inner product.  Returns (phi, pivots)."""
    a = psi.reshape(psi.shape[0], -1)
    piv, _ = scdm_pivots(psi)
    b = a[:, piv].T                          # b[k, i] = psi_i(c_k)
    xi = (b @ a).reshape(psi.shape)
    phi, _ = lowdin(xi, dv)
    return phi, piv
