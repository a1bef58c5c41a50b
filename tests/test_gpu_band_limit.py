"""Band-limited orbitals (plan option ecut=<Ha>) against the oracle.

Orbitals with plane-wave components only in (1/2)|G|^2 <= ecut have pair
densities with |kz| <= kz_max = 2 floor(sqrt(2 ecut) L_z / 2 pi); the passes
then skip the kz planes beyond (not stored, transformed or loaded).  The
oracle transforms the whole grid.  Covered: pruned planes on cubic grids
(the fused plane kernel, and at 108^3 in float64 the split rows + columns
path) and a slab grid, both precisions, E_x, K psi, M, the energy-only path and the
gradient; a screened plan; and a cutoff above the grid's reach, which must
give the unpruned result bit for bit.  Bars as in the parity tests.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import generate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import hfx  # noqa: E402

PRECS = [hfx.FP32, hfx.FP64]
IDS = ["fp32", "fp64"]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def bars(prec, ref_kpsi):
    if prec == hfx.FP32:
        return 1e-7, 1e-5
    return 1e-12, 1e-10 * np.max(np.abs(ref_kpsi))


def kz_max(ecut, lz):
    return 2 * math.floor(math.sqrt(2 * ecut) * lz / (2 * math.pi) + 1e-9)


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
@pytest.mark.parametrize("n,nz,box,n_orb", [
    (64, 64, (15.7, 15.7, 15.7), 13),
    (24, 48, (10.0, 10.0, 20.0), 11),
    (108, 108, (26.4, 26.4, 26.4), 3),   # float64: the split (rows + columns) plane path
])
def test_band_limited_planes_skipped(prec, n, nz, box, n_orb):
    ecut = 5.0
    shape = (nz, n, n)
    psi = generate.random_pw(shape, box, n_orb, ecut, seed=7000 + n)
    kzm = kz_max(ecut, box[2])
    assert 2 * kzm + 1 < nz  # planes are skipped
    print(f"case ecut={ecut} grid {n}x{n}x{nz} kz_max={kzm} prec={prec}", flush=True)
    vg = oracle.coulomb_kernel(shape, box, hfx.TRUNCATED, 0.0)
    ref = oracle.exchange(psi, box, vg, workers=4)
    dev = _dev()
    plan = hfx.Plan(hfx.SystemSpec((n, n, nz), box, n_orb), prec, options=f"ecut={ecut}",
                    device=dev)
    assert f"kz_max={kzm}" in plan.describe()
    # float32 plans whose pair band fits in half the z frequencies run the
    # forward z transform at half length on the even z points
    half = prec == hfx.FP32 and 2 * kzm + 1 <= nz // 2
    assert ("z_fwd=half" in plan.describe()) == half
    # at 64^3 the plane pass takes quarter planes: pass 1 on the even rows
    # and columns (the x and y bands fit in a quarter of the grid too)
    if prec == hfx.FP32 and n == 64:
        assert "y_rows=half" in plan.describe() and "x_cols=half" in plan.describe()
    pt = torch.from_numpy(psi).to(dev)
    kpsi, ex = plan.apply_exchange(pt)
    e_only = plan.exchange_energy(pt)
    m = plan.exchange_matrix(pt, kpsi)
    grad = plan.exchange_gradient(pt)
    torch.cuda.synchronize()
    e_bar, k_bar = bars(prec, ref["kpsi"])
    rel = abs(float(ex[0]) - ref["ex"]) / abs(ref["ex"])
    k = kpsi.double().cpu().numpy()
    dk = np.max(np.abs(k - ref["kpsi"]))
    print(f"  rel dE {rel:.2e} max dK {dk:.2e}", flush=True)
    assert rel <= e_bar and dk <= k_bar
    assert abs(float(e_only[0]) - float(ex[0])) <= 1e-13 * abs(float(ex[0]))
    dv = box[0] * box[1] * box[2] / psi[0].size
    m_ref = oracle.exchange_matrix(psi, ref["kpsi"], dv)
    omega = box[0] * box[1] * box[2]
    assert np.max(np.abs(m.view(n_orb, n_orb).cpu().numpy() - m_ref)) <= \
        np.sqrt(omega) * k_bar + 1e-12
    assert np.max(np.abs(grad.cpu().numpy() - 2 * dv * ref["kpsi"])) <= 2 * dv * k_bar


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_cutoff_beyond_the_grid_changes_nothing(prec):
    """ecut whose pair band reaches past the Nyquist plane skips no plane:
    results equal the plan without the option bit for bit."""
    n, L, n_orb = 24, 10.0, 9
    psi = generate.random_pw((n,) * 3, (L,) * 3, n_orb, 5.0, seed=7100)
    assert 2 * kz_max(40.0, L) + 1 >= n
    dev = _dev()
    pt = torch.from_numpy(psi).to(dev)
    out = []
    for opts in (None, "ecut=40"):
        plan = hfx.Plan(hfx.SystemSpec(n, (L,) * 3, n_orb), prec, options=opts, device=dev)
        assert "kz_max" not in plan.describe()
        k, e = plan.apply_exchange(pt)
        torch.cuda.synchronize()
        out.append((k.clone(), e.clone()))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


@pytest.mark.parametrize("n,L,n_orb,prec", [(64, 15.7, 24, hfx.FP32), (108, 26.4, 8, hfx.FP64)],
                         ids=["fp32-64", "fp64-108-split"])
def test_band_limited_screened_plan(n, L, n_orb, prec):
    """ecut together with s-MTACE screening (localised Gaussians at 5 Ha); at
    108^3 in float64 on the split plane path."""
    ecut = 5.0
    shape, box = (n,) * 3, (L,) * 3
    psi = generate.gaussians(shape, box, n_orb, ecut, seed=7200)[0]
    dv = L ** 3 / n ** 3
    a = oracle.pair_overlap_abs(psi, dv)
    vals = np.sort(a[np.triu_indices(n_orb, 1)])[::-1]
    mid = len(vals) // 2
    w = min(60, mid - 1)
    k = max(range(mid - w, mid + w), key=lambda i: (vals[i - 1] - vals[i]) / vals[i - 1])
    assert (vals[k - 1] - vals[k]) / vals[k - 1] > 1e-6
    rho_cut = 0.5 * (vals[k - 1] + vals[k])
    keep = oracle.screen_pairs(psi, dv, rho_cut)
    ref = oracle.exchange(psi, box, oracle.coulomb_kernel(shape, box, hfx.ERFC, 0.106),
                          keep=keep, workers=4)
    dev = _dev()
    plan = hfx.Plan(hfx.SystemSpec(n, box, n_orb, hfx.ERFC, 0.106), prec,
                    options=f"ecut={ecut}", device=dev)
    pt = torch.from_numpy(psi).to(dev)
    assert plan.screen(pt, rho_cut) == [int(np.triu(keep).sum())]
    kpsi, ex = plan.apply_exchange(pt)
    torch.cuda.synchronize()
    rel = abs(float(ex[0]) - ref["ex"]) / abs(ref["ex"])
    dk = np.max(np.abs(kpsi.double().cpu().numpy() - ref["kpsi"]))
    print(f"  screened rel dE {rel:.2e} max dK {dk:.2e}", flush=True)
    e_bar, k_bar = bars(prec, ref["kpsi"])
    assert rel <= e_bar and dk <= k_bar


_LARGE_REF = {}


@pytest.mark.parametrize("n,L,ecut", [(108, 26.4, 5.0), (108, 26.4, 20.0), (120, 29.4, 5.0),
                                      (120, 29.4, 20.0), (128, 29.6, 5.0), (128, 29.6, 20.0)])
def test_band_limited_every_large_variant(n, L, ecut):
    """Every float32 configuration of the grids whose plane fills the LDS
    (108, 120, 128), band-limited: at 5 Ha about half the kz planes are kept
    (pruned loads skipped, and band columns in the plane pass up to 120), at
    20 Ha nearly all (pruned legs read the zero block).  Covers the
    persistent plane kernels and the flat-load accumulation on pruned grids
    against the oracle's full transform, with several rows per tile pair so
    that the prefetching loop runs."""
    n_orb = 6
    shape, box = (n,) * 3, (L,) * 3
    key = (n, ecut)
    if key not in _LARGE_REF:
        _LARGE_REF.clear()
        psi = generate.random_pw(shape, box, n_orb, ecut, seed=7300 + n + int(ecut))
        vg = oracle.coulomb_kernel(shape, box, hfx.TRUNCATED, 0.0)
        _LARGE_REF[key] = (psi, oracle.exchange(psi, box, vg, workers=4))
    psi, ref = _LARGE_REF[key]
    dev = _dev()
    pt = torch.from_numpy(psi).to(dev)
    e_bar, k_bar = bars(hfx.FP32, ref["kpsi"])
    for v in hfx.variants(n, hfx.FP32):
        print(f"case ecut={ecut} grid {n}^3 variant={v}", flush=True)
        plan = hfx.Plan(hfx.SystemSpec(n, box, n_orb), hfx.FP32, options=f"ecut={ecut};variant={v}",
                        device=dev)
        assert "kz_max" in plan.describe()
        d = plan.describe()
        assert ("z_fwd=half" in d) == (ecut == 5.0)
        # cubic boxes: the x band fits a quarter of the grid exactly when the
        # y band does, so half-height input is half-width too
        assert ("x_cols=half" in d) == ("y_rows=half" in d)
        assert ecut == 5.0 or "y_rows=half" not in d
        kpsi, ex = plan.apply_exchange(pt)
        torch.cuda.synchronize()
        rel = abs(float(ex[0]) - ref["ex"]) / abs(ref["ex"])
        dk = np.max(np.abs(kpsi.double().cpu().numpy() - ref["kpsi"]))
        print(f"  rel dE {rel:.2e} max dK {dk:.2e}", flush=True)
        assert rel <= e_bar and dk <= k_bar
        del plan


@pytest.mark.parametrize("box,rows,cols", [
    ((16.0, 12.0, 14.0), True, False),   # x band 16 = n/4: band columns and half rows, full width
    ((12.0, 16.0, 14.0), False, False),  # y band 16 > 15: full planes
    ((12.0, 13.0, 14.0), True, True),    # both within 15: quarter planes
], ids=["half-rows", "full", "quarter"])
def test_band_limited_orthorhombic_decisions(box, rows, cols):
    """Orthorhombic boxes at 5 Ha on 64^3 (float32): the x and y bands differ,
    so the half-height and half-width decisions part (kx_max from L_x, ky_max
    from L_y; the half-length z transform from L_z); each combination
    against the oracle's full transform."""
    n, n_orb, ecut = 64, 9, 5.0
    shape = (n, n, n)
    psi = generate.random_pw(shape, box, n_orb, ecut, seed=7400)
    kx, ky = kz_max(ecut, box[0]), kz_max(ecut, box[1])
    print(f"case box={box} kx_max={kx} ky_max={ky}", flush=True)
    ref = oracle.exchange(psi, box, oracle.coulomb_kernel(shape, box, hfx.TRUNCATED, 0.0),
                          workers=4)
    dev = _dev()
    plan = hfx.Plan(hfx.SystemSpec(n, box, n_orb), hfx.FP32, options=f"ecut={ecut}", device=dev)
    d = plan.describe()
    assert ("y_rows=half" in d) == rows and ("x_cols=half" in d) == cols
    assert "z_fwd=half" in d
    kpsi, ex = plan.apply_exchange(torch.from_numpy(psi).to(dev))
    torch.cuda.synchronize()
    e_bar, k_bar = bars(hfx.FP32, ref["kpsi"])
    rel = abs(float(ex[0]) - ref["ex"]) / abs(ref["ex"])
    dk = np.max(np.abs(kpsi.double().cpu().numpy() - ref["kpsi"]))
    print(f"  rel dE {rel:.2e} max dK {dk:.2e}", flush=True)
    assert rel <= e_bar and dk <= k_bar
