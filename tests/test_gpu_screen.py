"""s-MTACE pair screening on the GPU (through the C ABI) against the oracle.

The oracle evaluates the screened sums directly: the pairs kept by
int |phi_a phi_b| >= rho_cut (``oracle.screen_pairs``), each once, in plain
order.  The GPU plan reorders the orbitals (clusters of overlapping orbitals), drops
whole tile pairs and packs the rest into new batches, so a wrong permutation,
mask bit or packing shows up as a missing or doubled pair.  rho_cut is put in
the middle of a wide gap of the oracle's A values, so that both sides keep the
same pairs whatever the summation order of A.

Bars as in the unscreened parity tests: float32 |dE|/|E| <= 1e-7 and
max|dK psi| <= 1e-5; float64 1e-12 and 1e-10 max|K psi|.
"""
import numpy as np
import pytest

import oracle
from workloads import generate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import hfx  # noqa: E402

L = 23.5          # bohr: the water96 box at a coarser grid
ERFC, W = 1, 0.106
TOL = {hfx.FP32: (1e-7, 1e-5, None), hfx.FP64: (1e-12, None, 1e-10)}
_cache = {}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def gap_cut(a, keep_frac):
    """rho_cut in the widest relative gap of A's upper triangle near the
    fraction keep_frac of kept pairs (diagonal excluded from the choice)."""
    n = a.shape[0]
    vals = np.sort(a[np.triu_indices(n, 1)])[::-1]
    target = int(keep_frac * len(vals))
    lo, hi = max(1, target - len(vals) // 10), min(len(vals) - 1, target + len(vals) // 10)
    k = max(range(lo, hi), key=lambda i: (vals[i - 1] - vals[i]) / vals[i - 1])
    assert (vals[k - 1] - vals[k]) / vals[k - 1] > 1e-6
    return 0.5 * (vals[k - 1] + vals[k])


def case(n_orb, seed, keep_frac):
    key = (n_orb, seed, keep_frac)
    if key not in _cache:
        shape, box = (64, 64, 64), (L, L, L)
        psi = generate.gaussians(shape, box, n_orb, 20.0, seed)[0]
        dv = L ** 3 / psi[0].size
        a = oracle.pair_overlap_abs(psi, dv)
        rho = gap_cut(a, keep_frac)
        keep = oracle.screen_pairs(psi, dv, rho)
        vg = oracle.coulomb_kernel(shape, box, ERFC, W)
        print(f"  oracle: n_orb {n_orb} rho_cut {rho:.4e} kept "
              f"{int(np.triu(keep).sum())} of {n_orb * (n_orb + 1) // 2}", flush=True)
        ref = oracle.exchange(psi, box, vg, keep=keep, workers=8)
        _cache[key] = (psi, rho, keep, ref)
    return _cache[key]


def plan_for(n_orb, prec, options=None):
    return hfx.Plan(hfx.SystemSpec(64, (L, L, L), n_orb, ERFC, W), prec, options, _dev())


def check(ref, ex, kpsi, prec):
    e_bar, k_abs, k_rel = TOL[prec]
    rel = abs(ex - ref["ex"]) / abs(ref["ex"])
    dk = np.max(np.abs(kpsi - ref["kpsi"]))
    kmax = np.max(np.abs(ref["kpsi"]))
    print(f"  rel dE {rel:.2e}  max dK {dk:.2e} (max K {kmax:.2e})", flush=True)
    assert rel <= e_bar, rel
    assert dk <= (k_abs if k_abs is not None else k_rel * kmax), dk


@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64])
@pytest.mark.parametrize("n_orb,seed,keep_frac", [(64, 9101, 0.3), (61, 9102, 0.5)])
def test_screened_exchange_matches_oracle(prec, n_orb, seed, keep_frac):
    psi, rho, keep, ref = case(n_orb, seed, keep_frac)
    print(f"case: screen n_orb={n_orb} seed={seed} prec={prec}", flush=True)
    plan = plan_for(n_orb, prec)
    pt = torch.from_numpy(psi).to(_dev())
    full = plan.schedule_info()
    kept = plan.screen(pt, rho)
    info = plan.schedule_info()
    n_keep = int(np.triu(keep).sum())
    print(f"  schedule full {full} screened {info}", flush=True)
    assert kept == [n_keep]
    assert info[3] == n_keep
    assert info[2] < full[2]          # fewer pair grids are transformed
    kpsi, ex = plan.apply_exchange(pt)
    e_only = plan.exchange_energy(pt)
    grad = plan.exchange_gradient(pt)
    torch.cuda.synchronize()
    k = kpsi.double().cpu().numpy()
    check(ref, float(ex[0]), k, prec)
    assert abs(float(e_only[0]) - float(ex[0])) <= 1e-13 * abs(float(ex[0]))
    dv = L ** 3 / psi[0].size
    assert np.array_equal(grad.cpu().numpy(), 2 * dv * k) or \
        np.max(np.abs(grad.cpu().numpy() - 2 * dv * k)) <= 1e-15 * np.max(np.abs(2 * dv * k))


def test_screen_off_restores_unscreened_bitwise():
    psi, rho, _, _ = case(64, 9101, 0.3)
    dev = _dev()
    pt = torch.from_numpy(psi).to(dev)
    fresh = plan_for(64, hfx.FP32)
    k0, e0 = fresh.apply_exchange(pt)
    plan = plan_for(64, hfx.FP32)
    plan.screen(pt, rho)
    plan.apply_exchange(pt)
    assert plan.screen(pt, 0.0) == [64 * 65 // 2]
    assert plan.schedule_info() == fresh.schedule_info()
    k1, e1 = plan.apply_exchange(pt)
    torch.cuda.synchronize()
    assert torch.equal(k0, k1)
    assert torch.equal(e0, e1)


def test_screen_everything_gives_zero():
    psi, _, _, _ = case(64, 9101, 0.3)
    pt = torch.from_numpy(psi).to(_dev())
    plan = plan_for(64, hfx.FP32)
    # A_aa = 1 for normalised orbitals: a cut above 1 drops every pair
    assert plan.screen(pt, 2.0) == [0]
    assert plan.schedule_info() == (0, 0, 0, 0)
    kpsi, ex = plan.apply_exchange(pt)
    torch.cuda.synchronize()
    assert float(ex[0]) == 0.0
    assert float(kpsi.abs().max()) == 0.0


def test_tiny_cut_keeps_all_pairs_in_new_order():
    """A positive cut below every A_ab keeps all pairs but takes the screened
    schedule (reordered orbitals, repacked batches): the unscreened result."""
    psi, _, _, _ = case(64, 9101, 0.3)
    pt = torch.from_numpy(psi).to(_dev())
    shape, box = (64, 64, 64), (L, L, L)
    vg = oracle.coulomb_kernel(shape, box, ERFC, W)
    plan = plan_for(64, hfx.FP64)
    assert plan.screen(pt, 1e-300) == [64 * 65 // 2]
    kpsi, ex = plan.apply_exchange(pt)
    torch.cuda.synchronize()
    # sampled rows of the unscreened oracle (full K psi of 4 orbitals)
    rows = [0, 17, 40, 63]
    kr = oracle.apply_exchange_rows(psi, box, vg, rows)
    k = kpsi.cpu().numpy()
    for t, r in enumerate(rows):
        d = np.max(np.abs(k[r] - kr[t]))
        assert d <= 1e-10 * np.max(np.abs(kr[t])), (r, d)


def test_screened_two_streams_and_groups():
    """Two batch streams give the one-stream result bitwise; two virtual
    groups of the screened batches sum to the whole screened energy."""
    psi, rho, keep, ref = case(64, 9101, 0.3)
    dev = _dev()
    pt = torch.from_numpy(psi).to(dev)
    one = plan_for(64, hfx.FP32, "tiles=2")
    two = plan_for(64, hfx.FP32, "tiles=2;streams=2")
    g0 = plan_for(64, hfx.FP32, "shard=0/2")
    g1 = plan_for(64, hfx.FP32, "shard=1/2")
    for p in (one, two, g0, g1):
        p.screen(pt, rho)
    k1, e1 = one.apply_exchange(pt)
    k2, e2 = two.apply_exchange(pt)
    ka, ea = g0.apply_exchange(pt)
    kb, eb = g1.apply_exchange(pt)
    torch.cuda.synchronize()
    assert torch.equal(k1, k2) and torch.equal(e1, e2)
    check(ref, float(e1[0]), k1.double().cpu().numpy(), hfx.FP32)
    check(ref, float(ea[0]) + float(eb[0]), (ka.double() + kb.double()).cpu().numpy(),
          hfx.FP32)


def test_screen_rejects_bad_cut():
    psi, _, _, _ = case(64, 9101, 0.3)
    pt = torch.from_numpy(psi).to(_dev())
    plan = plan_for(64, hfx.FP32)
    with pytest.raises(RuntimeError):
        plan.screen(pt, float("nan"))


def test_screened_graph_replays_match_eager():
    """A graph captured after screening replays the screened schedule: every
    replay (with eager work and synchronisation between them) equals the
    eager screened call bitwise."""
    psi, rho, _, _ = case(64, 9101, 0.3)
    dev = _dev()
    pt = torch.from_numpy(psi).to(dev)
    plan = plan_for(64, hfx.FP32)
    plan.screen(pt, rho)
    k_ref, e_ref = plan.apply_exchange(pt)
    torch.cuda.synchronize()
    k = torch.empty_like(k_ref)
    e = torch.empty_like(e_ref)
    g = plan.graph(hfx.GRAPH_APPLY, pt, kpsi=k, ex=e)
    for rep in range(3):
        k.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(k, k_ref) and torch.equal(e, e_ref), rep
        plan.exchange_energy(pt)          # eager work between replays
        torch.cuda.synchronize()
    g.close()


def test_graph_captured_before_screening_keeps_its_schedule():
    """A graph captured before hfx_screen keeps replaying the unscreened
    schedule: the tables the screening replaces stay alive while the graph
    does.  Every replay equals the eager unscreened call made before the
    screening, bitwise, with screened eager calls in between; a second
    screening (tables replaced twice) and the graph's destruction follow."""
    psi, rho, _, _ = case(64, 9101, 0.3)
    dev = _dev()
    pt = torch.from_numpy(psi).to(dev)
    plan = plan_for(64, hfx.FP32)
    k_all, e_all = plan.apply_exchange(pt)
    torch.cuda.synchronize()
    k = torch.empty_like(k_all)
    e = torch.empty_like(e_all)
    g = plan.graph(hfx.GRAPH_APPLY, pt, kpsi=k, ex=e)
    plan.screen(pt, rho)
    k_scr, e_scr = plan.apply_exchange(pt)
    torch.cuda.synchronize()
    assert not torch.equal(e_scr, e_all)
    for rep in range(3):
        k.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(k, k_all) and torch.equal(e, e_all), rep
        k2, e2 = plan.apply_exchange(pt)        # eager screened work between replays
        torch.cuda.synchronize()
        assert torch.equal(k2, k_scr) and torch.equal(e2, e_scr), rep
        if rep == 1:
            plan.screen(pt, rho)                 # replace the tables once more
    g.close()
    k3, e3 = plan.apply_exchange(pt)
    plan.screen(pt, 0.0)                         # back to all pairs, no graph alive
    k4, e4 = plan.apply_exchange(pt)
    torch.cuda.synchronize()
    assert torch.equal(k3, k_scr) and torch.equal(e3, e_scr)
    assert torch.equal(k4, k_all) and torch.equal(e4, e_all)


def test_screened_open_shell_plan():
    """hfx_screen on a two-system plan screens each system on its own
    orbitals and reports one kept count per system."""
    psi, rho, keep, ref = case(64, 9101, 0.3)
    psi2, rho2, keep2, ref2 = case(61, 9102, 0.5)
    dev = _dev()
    # one cut for both systems: the first case's, checked to sit in a gap of
    # the second system's A as well
    dv = L ** 3 / psi2[0].size
    a2 = oracle.pair_overlap_abs(psi2, dv)
    vals = np.sort(a2[np.triu_indices(61)])
    lo, hi = vals[vals < rho].max(), vals[vals >= rho].min()
    assert (hi - lo) / hi > 1e-6 and abs(rho - lo) > 1e-9 * rho and abs(hi - rho) > 1e-9 * rho
    keep2 = oracle.screen_pairs(psi2, dv, rho)
    shape, box = (64, 64, 64), (L, L, L)
    vg = oracle.coulomb_kernel(shape, box, ERFC, W)
    ref2 = oracle.exchange(psi2, box, vg, keep=keep2, workers=8)
    plan = hfx.Plan([hfx.SystemSpec(64, box, 64, ERFC, W), hfx.SystemSpec(64, box, 61, ERFC, W)],
                    hfx.FP32, device=dev)
    pt = torch.from_numpy(np.concatenate([psi, psi2])).to(dev)
    kept = plan.screen(pt, rho)
    assert kept == [int(np.triu(keep).sum()), int(np.triu(keep2).sum())]
    kpsi, ex = plan.apply_exchange(pt)
    torch.cuda.synchronize()
    k = kpsi.double().cpu().numpy()
    check(ref, float(ex[0]), k[:64], hfx.FP32)
    check(ref2, float(ex[1]), k[64:], hfx.FP32)
