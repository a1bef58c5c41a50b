"""Size classes of a batched plan: systems with the same kernel configuration
(grid, precision), band and screening state share one launch per pass and
batch step (a table of the systems' pass arguments in the launch), up to
eight per class, with one staging, pair-mean and zero-fill launch for the
class; other systems run as their own class on a forked stream.  By default
only systems with small launches (below 512 workgroups) are grouped; group=1
groups every system it can, group=0 none.

Checked: the class layout that hfx_plan_describe reports; K psi, E_x, the
gradient and M of a plan whose classes hold several systems, bitwise equal
to the same plan without grouping (group=0) and to single-system plans;
graph replay of the grouped plan; an open-shell pair (two spin channels on
one grid, the use the classes are for) against the oracle; a screened class.
"""
import numpy as np
import pytest

import oracle
from workloads import generate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import hfx  # noqa: E402


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


# three 24^3 systems of different orbital counts and boxes (one class),
# a 64^3 system (its own class), a fifth on 24^3 again (same class as the first)
SYSTEMS = [(24, 10.0, 9, hfx.TRUNCATED, 0.0), (24, 11.0, 13, hfx.ERFC, 0.3),
           (64, 12.0, 6, hfx.ERFC, 0.106), (24, 10.0, 21, hfx.TRUNCATED, 0.0),
           (24, 9.0, 3, hfx.ERFC, 0.2)]


def _inputs():
    psis = [generate.random_pw((n,) * 3, (L,) * 3, no, 5.0, 300 + k)
            for k, (n, L, no, _, _) in enumerate(SYSTEMS)]
    specs = [hfx.SystemSpec(n, (L,) * 3, no, kind, w) for n, L, no, kind, w in SYSTEMS]
    return psis, specs


@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64], ids=["fp32", "fp64"])
def test_grouped_plan_equals_ungrouped_and_single_plans(prec):
    dev = _dev()
    psis, specs = _inputs()
    flat = torch.from_numpy(np.concatenate([p.reshape(-1) for p in psis])).to(dev)
    grouped = hfx.Plan(specs, prec, device=dev)
    plain = hfx.Plan(specs, prec, options="group=0", device=dev)
    forced = hfx.Plan(specs, prec, options="group=1", device=dev)
    assert "class=0/4" in forced.describe(0) and "class=1/1" in forced.describe(2)
    d = [grouped.describe(i) for i in range(len(specs))]
    print("\n".join(d), flush=True)
    assert all("class=0/4" in d[i] for i in (0, 1, 3, 4)) and "class=1/1" in d[2]
    assert all("/1" in plain.describe(i).split("class=")[1] for i in range(len(specs)))
    out = {}
    for name, plan in (("grouped", grouped), ("plain", plain), ("forced", forced)):
        k, e = plan.apply_exchange(flat)
        m = plan.exchange_matrix(flat, k)
        g = plan.exchange_gradient(flat)
        e2 = plan.exchange_energy(flat)
        m2 = torch.empty_like(m)
        e3 = torch.empty_like(e)
        plan.exchange_matrix(flat, m=m2, ex=e3)
        torch.cuda.synchronize()
        out[name] = (k.clone(), e.clone(), m.clone(), g.clone(), e2.clone(), m2, e3)
    for a, b, c in zip(out["grouped"], out["plain"], out["forced"]):
        assert torch.equal(a, b) and torch.equal(a, c)
    k, e, m, g, e2, m2, e3 = out["grouped"]
    assert torch.equal(e2, e) and torch.equal(e3, e) and torch.equal(m2, m)
    for i, (spec, psi) in enumerate(zip(specs, psis)):
        single = hfx.Plan(spec, prec, device=dev)
        k1, e1 = single.apply_exchange(torch.from_numpy(psi).to(dev))
        torch.cuda.synchronize()
        assert torch.equal(grouped.split(k)[i], k1.view_as(grouped.split(k)[i]))
        assert float(e1[0]) == float(e[i])
    # graph replay of the grouped plan, with eager work in between
    kk = torch.empty_like(k)
    ee = torch.empty_like(e)
    gr = grouped.graph(hfx.GRAPH_APPLY, flat, kpsi=kk, ex=ee)
    for rep in range(3):
        kk.fill_(float("nan"))
        gr.launch()
        torch.cuda.synchronize()
        assert torch.equal(kk, k) and torch.equal(ee, e), rep
        grouped.exchange_energy(flat)
        torch.cuda.synchronize()
    gr.close()


@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64], ids=["fp32", "fp64"])
def test_open_shell_pair_in_one_class_against_oracle(prec):
    """Spin-up and spin-down orbitals of one box: one class, one launch per
    pass; each channel's E_x and K psi against the oracle."""
    dev = _dev()
    n, L = 64, 15.0
    box = (L,) * 3
    up = generate.gaussians((n,) * 3, box, 11, 20.0, 310)[0]
    dn = generate.gaussians((n,) * 3, box, 7, 20.0, 311)[0]
    vg = oracle.coulomb_kernel((n,) * 3, box, hfx.ERFC, 0.106)
    refs = [oracle.exchange(p, box, vg, workers=4) for p in (up, dn)]
    specs = [hfx.SystemSpec(n, box, p.shape[0], hfx.ERFC, 0.106) for p in (up, dn)]
    plan = hfx.Plan(specs, prec, device=dev)
    assert "class=0/2" in plan.describe(0) and "class=0/2" in plan.describe(1)
    flat = torch.from_numpy(np.concatenate([up.reshape(-1), dn.reshape(-1)])).to(dev)
    k, e = plan.apply_exchange(flat)
    torch.cuda.synchronize()
    for i, ref in enumerate(refs):
        rel = abs(float(e[i]) - ref["ex"]) / abs(ref["ex"])
        dk = float(np.max(np.abs(plan.split(k)[i].double().cpu().numpy() - ref["kpsi"])))
        kmax = float(np.max(np.abs(ref["kpsi"])))
        print(f"  channel {i}: rel dE {rel:.2e} max dK {dk:.2e}", flush=True)
        if prec == hfx.FP32:
            assert rel <= 1e-7 and dk <= 1e-5
        else:
            assert rel <= 1e-12 and dk <= 1e-10 * kmax


def test_screened_class_equals_screened_single_plans():
    dev = _dev()
    n, L = 64, 15.0
    box = (L,) * 3
    psis = [generate.gaussians((n,) * 3, box, no, 20.0, 320 + no)[0] for no in (24, 17)]
    specs = [hfx.SystemSpec(n, box, p.shape[0], hfx.ERFC, 0.106) for p in psis]
    flat = torch.from_numpy(np.concatenate([p.reshape(-1) for p in psis])).to(dev)
    plan = hfx.Plan(specs, hfx.FP32, options="group=1", device=dev)
    kept = plan.screen(flat, 2.5e-2)
    assert "screened=yes" in plan.describe(0) and "class=0/2" in plan.describe(1)
    k, e = plan.apply_exchange(flat)
    torch.cuda.synchronize()
    for i, (spec, p) in enumerate(zip(specs, psis)):
        single = hfx.Plan(spec, hfx.FP32, device=dev)
        pt = torch.from_numpy(p).to(dev)
        assert single.screen(pt, 2.5e-2) == [kept[i]]
        k1, e1 = single.apply_exchange(pt)
        torch.cuda.synchronize()
        assert torch.equal(plan.split(k)[i], k1.view_as(plan.split(k)[i]))
        assert float(e1[0]) == float(e[i])
