"""Parity on full-spectrum (white-noise) orbitals at every compiled kernel
configuration, against the float64 oracle, element by element.

The benchmark workloads are band-limited on alias-free grids, so their pair
densities vanish on the outermost frequencies of every axis.  White-noise
orbitals (independent N(0, 1) values, ``workloads.generate.white_noise``)
fill every frequency, the Nyquist planes of x, y and z included, so a wrong
kernel value, twiddle or codelet leg near Nyquist, or a wrong plane index
at the edge of the grid, changes K psi here (Eq. (vij): the potential of the
pair density at every G; Eq. (vx): K psi).

Bars: the energy bar of the other parity tests (float32 |dE_x|/|E_x| <=
1e-7, float64 1e-12); K psi element by element, float32 max|dK psi| <= 1e-5
absolute and <= 5e-7 of max|K psi| (white-noise K psi is small, so the
relative bar is the binding one: a few float32 roundings, 2^-24 each, per
stage of three transforms of length <= 128 and their inverses; measured
1.0-1.5e-7), float64 1e-10 of max|K psi|; the exchange matrix
from the plan's own K psi against the oracle's M to the Cauchy-Schwarz bar
sqrt(Omega) max|dK psi|.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import generate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import hfx  # noqa: E402

# (nx = ny, nz, box, n_orb, kernel, w): every compiled grid, cubic and slab
GRIDS = [(24, 24, (10.0, 10.0, 10.0), 5, hfx.TRUNCATED, 0.0),
         (64, 64, (12.0, 12.0, 12.0), 3, hfx.ERFC, 0.106),
         (72, 72, (17.6, 17.6, 17.6), 3, hfx.ERFC, 0.106),
         (80, 80, (19.6, 19.6, 19.6), 3, hfx.TRUNCATED, 0.0),
         (96, 96, (23.5, 23.5, 23.5), 3, hfx.ERFC, 0.106),
         (108, 108, (26.4, 26.4, 26.4), 2, hfx.TRUNCATED, 0.0),
         (120, 120, (29.4, 29.4, 29.4), 2, hfx.ERFC, 0.106),
         (128, 128, (29.6, 29.6, 29.6), 2, hfx.TRUNCATED, 0.0),
         (24, 48, (10.0, 10.0, 20.0), 5, hfx.TRUNCATED, 0.0),
         (64, 128, (15.7, 15.7, 31.3), 3, hfx.ERFC, 0.106)]
_REF = {}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _case(nxy, nz, box, n_orb, kernel, w):
    key = (nxy, nz)
    if key not in _REF:
        _REF.clear()
        shape = (nz, nxy, nxy)
        psi = generate.white_noise(shape, box, n_orb, seed=9000 + nxy + nz)
        vg = oracle.coulomb_kernel(shape, box, kernel, w)
        _REF[key] = (psi, oracle.exchange(psi, box, vg, workers=4))
    return _REF[key]


def _variant_names(nxy, nz, prec):
    if nxy == nz:
        return hfx.variants(nxy, prec)
    # slab grids: the compiled names carry the z length
    return [f"{'f32' if prec == hfx.FP32 else 'f64'}-n{nxy}x{nz}"]


@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("nxy,nz,box,n_orb,kernel,w", GRIDS,
                         ids=[f"n{g[0]}x{g[1]}" for g in GRIDS])
def test_white_noise_every_variant(nxy, nz, box, n_orb, kernel, w, prec):
    dev = _dev()
    psi, ref = _case(nxy, nz, box, n_orb, kernel, w)
    omega = box[0] * box[1] * box[2]
    dv = omega / psi[0].size
    kmax = float(np.max(np.abs(ref["kpsi"])))
    m_ref = oracle.exchange_matrix(psi, ref["kpsi"], dv)
    pt = torch.from_numpy(psi).to(dev)
    names = _variant_names(nxy, nz, prec)
    assert names, "no compiled variant"
    for v in names:
        print(f"case white noise {nxy}x{nxy}x{nz} n_orb={n_orb} prec={prec} variant={v}",
              flush=True)
        plan = hfx.Plan(hfx.SystemSpec((nxy, nxy, nz), box, n_orb, kernel, w), prec,
                        options=f"variant={v}", device=dev)
        kpsi, ex = plan.apply_exchange(pt)
        m = plan.exchange_matrix(pt, kpsi)
        torch.cuda.synchronize()
        k = kpsi.double().cpu().numpy()
        rel = abs(float(ex[0]) - ref["ex"]) / abs(ref["ex"])
        dk = float(np.max(np.abs(k - ref["kpsi"])))
        dm = float(np.max(np.abs(m.view(n_orb, n_orb).cpu().numpy() - m_ref)))
        print(f"  rel dE {rel:.2e}  max dK {dk:.2e} (max K {kmax:.2e}, rel {dk / kmax:.2e})"
              f"  max dM {dm:.2e}", flush=True)
        if prec == hfx.FP32:
            assert rel <= 1e-7
            assert dk <= 1e-5 and dk <= 5e-7 * kmax
        else:
            assert rel <= 1e-12
            assert dk <= 1e-10 * kmax
        assert dm <= math.sqrt(omega) * dk + 1e-13 * np.max(np.abs(m_ref))
        del plan
