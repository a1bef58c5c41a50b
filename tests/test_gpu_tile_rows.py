"""Tile pairs of R rows x 8 columns (plan option rows=R) against the oracle.

The schedule cuts each pair of R-orbital blocks into R/8 tile pairs; inside a
diagonal block only pairs i <= j are evaluated and a tile's rows stop at its
last column.  Covered here: ragged orbital counts (partial blocks, partial
last column tile, single orbital), both precisions, exact pair counts of the
schedule, two batch streams bit for bit, virtual groups adding up, the
clamp for variants that stage psi of I in LDS, and screening of a rows plan.
Bars as in the parity tests: float32 |dE|/|E| <= 1e-7, max|dK psi| <= 1e-5;
float64 1e-12 and 1e-10 max|K psi|.
"""
import numpy as np
import pytest

import oracle
from workloads import generate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import hfx  # noqa: E402

PRECS = [hfx.FP32, hfx.FP64]
IDS = ["fp32", "fp64"]
N, L = 24, 10.0
BOX = (L, L, L)


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def bars(prec, ref_kpsi):
    if prec == hfx.FP32:
        return 1e-7, 1e-5
    return 1e-12, 1e-10 * np.max(np.abs(ref_kpsi))


_REF = {}


def reference(n_orb, seed):
    key = (n_orb, seed)
    if key not in _REF:
        psi = generate.random_pw((N,) * 3, BOX, n_orb, 5.0, seed=seed)
        vg = oracle.coulomb_kernel((N,) * 3, BOX, hfx.TRUNCATED, 0.0)
        _REF[key] = (psi, oracle.exchange(psi, BOX, vg, workers=4))
    return _REF[key]


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
@pytest.mark.parametrize("rows", [16, 24, 32])
@pytest.mark.parametrize("n_orb", [1, 9, 13, 37, 70])
def test_rows_parity_ragged(n_orb, rows, prec):
    print(f"case rows={rows} n_orb={n_orb} prec={prec}", flush=True)
    psi, ref = reference(n_orb, 5100 + n_orb)
    dev = _dev()
    plan = hfx.Plan(hfx.SystemSpec(N, BOX, n_orb), prec, options=f"rows={rows}", device=dev)
    assert f"rows={rows}" in plan.describe()
    pt = torch.from_numpy(psi).to(dev)
    kpsi, ex = plan.apply_exchange(pt)
    e_only = plan.exchange_energy(pt)
    m = plan.exchange_matrix(pt, kpsi)
    torch.cuda.synchronize()
    e_bar, k_bar = bars(prec, ref["kpsi"])
    rel = abs(float(ex[0]) - ref["ex"]) / abs(ref["ex"])
    dk = np.max(np.abs(kpsi.double().cpu().numpy() - ref["kpsi"]))
    print(f"  rel dE {rel:.2e} max dK {dk:.2e}", flush=True)
    assert rel <= e_bar and dk <= k_bar
    assert abs(float(e_only[0]) - float(ex[0])) <= 1e-13 * abs(float(ex[0]))
    dv = L ** 3 / N ** 3
    m_ref = oracle.exchange_matrix(psi, ref["kpsi"], dv)
    assert np.max(np.abs(m.view(n_orb, n_orb).cpu().numpy() - m_ref)) <= \
        np.sqrt(L ** 3) * k_bar + 1e-12


@pytest.mark.parametrize("rows", [8, 16, 24, 32])
@pytest.mark.parametrize("n_orb", [1, 8, 9, 31, 33, 70, 256])
def test_rows_schedule_counts_every_pair_once(n_orb, rows):
    """The schedule evaluates n (n + 1) / 2 pairs, and its tile pairs and
    pair grids match the counts of the R x 8 tiling."""
    dev = _dev()
    plan = hfx.Plan(hfx.SystemSpec(N, BOX, n_orb), hfx.FP32, options=f"rows={rows}", device=dev)
    batches, tiles, grids, pairs = plan.schedule_info()
    assert pairs == n_orb * (n_orb + 1) // 2
    nb = -(-n_orb // rows)
    want_tiles = 0
    for bi in range(nb):
        for bj in range(bi, nb):
            for q in range(rows // 8):
                if bj * rows + q * 8 < n_orb:
                    want_tiles += 1
    assert tiles == want_tiles
    # grids: pairs (i, c) and (i, c + 1), c even, share one grid, which is
    # transformed when either pair has i <= j
    want_grids = sum(1 for i in range(n_orb) for c in range(0, n_orb, 2) if c + 1 >= i)
    assert grids == want_grids


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_rows_two_batch_streams_bitwise(prec):
    psi, _ = reference(37, 5300)
    dev = _dev()
    pt = torch.from_numpy(psi).to(dev)
    out = []
    for opts in ("rows=16;tiles=1", "rows=16;tiles=1;streams=2"):
        print(f"case {opts} prec={prec}", flush=True)
        plan = hfx.Plan(hfx.SystemSpec(N, BOX, 37), prec, options=opts, device=dev)
        k, e = plan.apply_exchange(pt)
        torch.cuda.synchronize()
        out.append((k.clone(), e.clone()))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_rows_shards_sum_to_full_plan(prec):
    psi, _ = reference(70, 5400)
    dev = _dev()
    spec = hfx.SystemSpec(N, BOX, 70)
    pt = torch.from_numpy(psi).to(dev)
    full = hfx.Plan(spec, prec, options="rows=32", device=dev)
    k_full, e_full = full.apply_exchange(pt)
    k_sum = torch.zeros(psi.shape, dtype=torch.float64, device=dev)
    e_sum = 0.0
    for g in range(2):
        plan = hfx.Plan(spec, prec, options=f"rows=32;shard={g}/2", device=dev)
        k, e = plan.apply_exchange(pt)
        k_sum += k.double()
        e_sum += float(e[0])
    torch.cuda.synchronize()
    ef = float(e_full[0])
    dk = float(torch.max(torch.abs(k_sum - k_full.double())))
    kmax = float(torch.max(torch.abs(k_full.double())))
    if prec == hfx.FP64:
        assert abs(e_sum - ef) <= 1e-12 * abs(ef) and dk <= 1e-12 * kmax
    else:
        assert abs(e_sum - ef) <= 1e-7 * abs(ef) and dk <= 1e-5


def test_rows_clamped_where_psi_i_is_staged():
    """Variants that stage psi of the I block in LDS take 8-row tiles."""
    dev = _dev()
    plan = hfx.Plan(hfx.SystemSpec(96, (23.5,) * 3, 40, hfx.ERFC, 0.106), hfx.FP32,
                    options="rows=32;variant=f32-n96-pi", device=dev)
    assert "rows=8" in plan.describe()
    plan = hfx.Plan(hfx.SystemSpec(96, (23.5,) * 3, 40, hfx.ERFC, 0.106), hfx.FP32,
                    options="rows=32;variant=f32-n96", device=dev)
    assert "rows=32" in plan.describe()


def test_rows_plan_screening_round_trip():
    """Screening a rows plan keeps its R x 8 tile pairs, now with masks of the
    kept pairs: K psi and E_x of the kept pairs match the oracle's screened
    exchange, and equal those of a screened 8-row plan to rounding; rho_cut =
    0 restores the unscreened schedule (equal to the plan's first result bit
    for bit)."""
    psi, _ = reference(37, 5500)
    dev = _dev()
    spec = hfx.SystemSpec(N, BOX, 37)
    pt = torch.from_numpy(psi).to(dev)
    p16 = hfx.Plan(spec, hfx.FP32, options="rows=16", device=dev)
    k0, e0 = p16.apply_exchange(pt)
    k0, e0 = k0.clone(), e0.clone()
    # a cut in a clear gap of the oracle's pair overlaps near the median, so
    # that both sides keep the same pairs
    dv = L ** 3 / N ** 3
    a = oracle.pair_overlap_abs(psi, dv)
    vals = np.sort(a[np.triu_indices(37, 1)])[::-1]
    mid = len(vals) // 2
    k = max(range(mid - 60, mid + 60), key=lambda i: (vals[i - 1] - vals[i]) / vals[i - 1])
    assert (vals[k - 1] - vals[k]) / vals[k - 1] > 1e-6
    rho_cut = 0.5 * (vals[k - 1] + vals[k])
    keep = oracle.screen_pairs(psi, dv, rho_cut)
    kept = p16.screen(pt, rho_cut)
    print(f"  rho_cut {rho_cut:.4f} kept {kept}", flush=True)
    assert kept == [int(np.triu(keep).sum())] and 0 < kept[0] < 37 * 38 // 2
    assert "rows=16" in p16.describe() and "screened=yes" in p16.describe()
    assert p16.schedule_info()[3] == kept[0]
    ks, es = p16.apply_exchange(pt)
    p8 = hfx.Plan(spec, hfx.FP32, options="rows=8", device=dev)
    assert p8.screen(pt, rho_cut) == kept
    k8, e8 = p8.apply_exchange(pt)
    torch.cuda.synchronize()
    assert abs(float(es[0]) - float(e8[0])) <= 1e-12 * abs(float(e8[0]))
    assert float(torch.max(torch.abs(ks - k8))) <= 1e-6
    ref = oracle.exchange(psi, BOX, oracle.coulomb_kernel((N,) * 3, BOX, hfx.TRUNCATED, 0.0),
                          keep=keep, workers=4)
    assert abs(float(es[0]) - ref["ex"]) <= 1e-7 * abs(ref["ex"])
    assert np.max(np.abs(ks.double().cpu().numpy() - ref["kpsi"])) <= 1e-5
    p16.screen(pt, 0.0)
    assert "rows=16" in p16.describe()
    kc, ec = p16.apply_exchange(pt)
    torch.cuda.synchronize()
    assert torch.equal(kc, k0) and torch.equal(ec, e0)


def test_rows_on_64_grid_against_oracle():
    """rows=32 on a 64^3 grid with 40 localised orbitals: two row blocks,
    three round-robin rounds, four column tiles per block pair."""
    n, Lb, n_orb = 64, 12.0, 40
    psi = generate.gaussians((n,) * 3, (Lb,) * 3, n_orb, 20.0, seed=5600)[0]
    vg = oracle.coulomb_kernel((n,) * 3, (Lb,) * 3, hfx.ERFC, 0.106)
    ref = oracle.exchange(psi, (Lb,) * 3, vg, workers=4)
    dev = _dev()
    pt = torch.from_numpy(psi).to(dev)
    for prec in PRECS:
        print(f"case n=64 rows=32 prec={prec}", flush=True)
        plan = hfx.Plan(hfx.SystemSpec(n, (Lb,) * 3, n_orb, hfx.ERFC, 0.106), prec,
                        options="rows=32", device=dev)
        kpsi, ex = plan.apply_exchange(pt)
        torch.cuda.synchronize()
        e_bar, k_bar = bars(prec, ref["kpsi"])
        rel = abs(float(ex[0]) - ref["ex"]) / abs(ref["ex"])
        dk = np.max(np.abs(kpsi.double().cpu().numpy() - ref["kpsi"]))
        print(f"  rel dE {rel:.2e} max dK {dk:.2e}", flush=True)
        assert rel <= e_bar and dk <= k_bar
