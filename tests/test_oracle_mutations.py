"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins catch them.

Each mutation replaces one oracle function for the duration of a test; the
pin functions of ``test_oracle_pins`` must then fail.
"""
import math

import numpy as np
import pytest
import scipy.fft as sfft

import oracle
import oracle.hfx_oracle as ho
import test_oracle_pins as pins

_orig_kernel = ho.coulomb_kernel
_orig_potential = ho.pair_potential


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(ho, name, fn)
    monkeypatch.setattr(oracle, name, fn, raising=False)


def _small():
    from workloads import generate
    shape, box = (12, 12, 12), (6.0, 6.0, 6.0)
    psi = generate.random_pw(shape, box, 5, 4.0, seed=11)
    return psi, box, _orig_kernel(shape, box, oracle.TRUNCATED)


def mut_no_forward_normalisation(rho, vg):
    return sfft.ifftn(vg * sfft.fftn(rho)).real * rho.size


def mut_g0_dropped(shape, box, kind, param=0.0):
    v = _orig_kernel(shape, box, kind, param)
    v[0, 0, 0] = 0.0
    return v


def mut_rc_wrong(shape, box, kind, param=0.0):
    if kind != oracle.TRUNCATED:
        return _orig_kernel(shape, box, kind, param)
    g2 = oracle.grid_g2(shape, box)
    rc = 0.5 * (box[0] * box[1] * box[2]) ** (1 / 3)
    v = np.where(g2 > 0, 8 * math.pi * np.sin(0.5 * np.sqrt(g2) * rc) ** 2
                 / np.where(g2 > 0, g2, 1), 2 * math.pi * rc * rc)
    return v


def mut_axes_swapped(shape, box, kind, param=0.0):
    return _orig_kernel(shape, (box[2], box[1], box[0]), kind, param)


def mut_erfc_sign(shape, box, kind, param=0.0):
    if kind != oracle.ERFC:
        return _orig_kernel(shape, box, kind, param)
    g2 = oracle.grid_g2(shape, box)
    w = param
    return np.where(g2 > 0, 4 * math.pi * (1 + np.exp(-g2 / (4 * w * w)))
                    / np.where(g2 > 0, g2, 1), math.pi / (w * w))


def mut_rows_index_swapped(args):
    psi, vg, dv, rows, want_kpsi = args[:5]
    n = psi.shape[0]
    kpsi = np.zeros_like(psi)
    e = np.zeros((n, n))
    for i in rows:
        for j in range(i, n):
            rho = psi[i] * psi[j]
            vij = _orig_potential(rho, vg)
            e[i, j] = e[j, i] = dv * float(np.sum(rho * vij))
            kpsi[i] -= vij * psi[i]             # planted: psi_i instead of psi_j
            if j != i:
                kpsi[j] -= vij * psi[j]
    return kpsi, e


def mut_rows_offdiag_once(args):
    psi, vg, dv, rows, want_kpsi = args[:5]
    n = psi.shape[0]
    kpsi = np.zeros_like(psi)
    e = np.zeros((n, n))
    for i in rows:
        for j in range(i, n):
            rho = psi[i] * psi[j]
            vij = _orig_potential(rho, vg)
            e[i, j] = dv * float(np.sum(rho * vij))   # planted: e_ji never stored
            kpsi[i] -= vij * psi[j]
            if j != i:
                kpsi[j] -= vij * psi[i]
    return kpsi, e


def mut_rows_missing_symmetric_update(args):
    psi, vg, dv, rows, want_kpsi = args[:5]
    n = psi.shape[0]
    kpsi = np.zeros_like(psi)
    e = np.zeros((n, n))
    for i in rows:
        for j in range(i, n):
            rho = psi[i] * psi[j]
            vij = _orig_potential(rho, vg)
            e[i, j] = e[j, i] = dv * float(np.sum(rho * vij))
            kpsi[i] -= vij * psi[j]              # planted: K psi_j update dropped
    return kpsi, e


def _all_pins():
    psi_small = _small()
    return [
        lambda: pins.test_brute_force_direct_dft((6, 5, 4), (4.0, 3.5, 3.0), oracle.ERFC, 0.7),
        lambda: pins.test_brute_force_direct_dft((8, 6, 6), (5.0, 4.0, 4.2), oracle.TRUNCATED, 0.0),
        pins.test_gaussian_self_energy_truncated,
        pins.test_gaussian_self_energy_erfc_isolated,
        pins.test_gaussian_lattice_sum_erfc_long_range,
        pins.test_cosine_orbitals_closed_form,
        pins.test_constant_kernel_special_case,
        lambda: pins.test_energy_trace_identities(psi_small),
        lambda: pins.test_gradient_five_point_exact(psi_small),
    ]


def _count_failures():
    failed = 0
    for pin in _all_pins():
        try:
            pin()
        except AssertionError:
            failed += 1
    return failed


@pytest.mark.parametrize("name,fn", [
    ("pair_potential", mut_no_forward_normalisation),
    ("coulomb_kernel", mut_g0_dropped),
    ("coulomb_kernel", mut_rc_wrong),
    ("coulomb_kernel", mut_axes_swapped),
    ("coulomb_kernel", mut_erfc_sign),
    ("_rows_worker", mut_rows_index_swapped),
    ("_rows_worker", mut_rows_offdiag_once),
    ("_rows_worker", mut_rows_missing_symmetric_update),
])
def test_planted_mistake_is_caught(monkeypatch, name, fn):
    assert _count_failures() == 0          # the unmodified oracle passes every pin
    _patch(monkeypatch, name, fn)
    assert _count_failures() >= 1


# --------------------------------------------------------------------------
# SCDM: mistakes in the selection or in the density-matrix columns

_orig_pivots = ho.scdm_pivots


def mut_scdm_no_projection(psi):
    """Top column norms of Psi^T, without removing the selected directions."""
    a = psi.reshape(psi.shape[0], -1)
    norms = np.einsum("ij,ij->j", a, a)
    piv = np.argsort(-norms, kind="stable")[: a.shape[0]]
    return piv, np.ones(a.shape[0])


def mut_scdm_transposed_columns(psi, dv):
    a = psi.reshape(psi.shape[0], -1)
    piv, _ = _orig_pivots(psi)
    b = a[:, piv]                            # b[i, k] where b[k, i] is meant
    phi, _ = ho.lowdin((b @ a).reshape(psi.shape), dv)
    return phi, piv


def test_scdm_mutation_no_projection_is_caught(monkeypatch):
    _patch(monkeypatch, "scdm_pivots", mut_scdm_no_projection)
    with pytest.raises(AssertionError):
        pins.test_scdm_pivots_match_lapack_qrcp("pw", 24, 8, 3)


def test_scdm_mutation_transposed_columns_is_caught(monkeypatch):
    _patch(monkeypatch, "scdm", mut_scdm_transposed_columns)
    with pytest.raises(AssertionError):
        pins.test_scdm_orthonormal_same_span_and_rotation_invariant()


def mut_scdm_gram_schmidt(psi, dv):
    """The right pivots and columns, orthonormalised by Gram-Schmidt
    (Cholesky) instead of Loewdin."""
    a = psi.reshape(psi.shape[0], -1)
    piv, _ = _orig_pivots(psi)
    xi = (a[:, piv].T @ a).reshape(psi.shape)
    return ho.cholesky_orthonormalize(xi, dv), piv


def test_scdm_mutation_gram_schmidt_is_caught(monkeypatch):
    _patch(monkeypatch, "scdm", mut_scdm_gram_schmidt)
    # the other SCDM pins hold for any orthonormalisation of the same span
    pins.test_scdm_orthonormal_same_span_and_rotation_invariant()
    with pytest.raises(AssertionError):
        pins.test_scdm_final_step_is_loewdin()
