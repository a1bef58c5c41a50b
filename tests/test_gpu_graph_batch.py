"""Multi-system plans and captured graphs (through the C ABI).

A plan over several systems forks them onto its own streams; every system's
results must equal (bitwise) those of a single-system plan.  Graph replays are
checked against the eager results after each of several replays, with eager
work and synchronisation in between.
"""
import numpy as np
import pytest

import oracle
from workloads import generate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import hfx  # noqa: E402

SYSTEMS = [(24, 10.0, 9, hfx.TRUNCATED, 0.0), (64, 15.7, 6, hfx.TRUNCATED, 0.0),
           (72, 17.6, 5, hfx.ERFC, 0.106)]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _inputs():
    return [generate.random_pw((n, n, n), (L, L, L), no, 5.0, seed=300 + n)
            for n, L, no, _, _ in SYSTEMS]


@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64], ids=["fp32", "fp64"])
def test_batched_plan_equals_single_plans(prec):
    dev = _dev()
    psis = _inputs()
    specs = [hfx.SystemSpec(n, (L, L, L), no, k, w) for n, L, no, k, w in SYSTEMS]
    flat = torch.from_numpy(np.concatenate([p.reshape(-1) for p in psis])).to(dev)
    plan = hfx.Plan(specs, prec, device=dev)
    kpsi, ex = plan.apply_exchange(flat)
    m = plan.exchange_matrix(flat, kpsi)
    torch.cuda.synchronize()
    moff = 0
    for i, (spec, p) in enumerate(zip(specs, psis)):
        single = hfx.Plan(spec, prec, device=dev)
        pt = torch.from_numpy(p).to(dev)
        k1, e1 = single.apply_exchange(pt)
        m1 = single.exchange_matrix(pt, k1)
        torch.cuda.synchronize()
        assert torch.equal(plan.split(kpsi)[i], k1)
        assert float(ex[i]) == float(e1[0])
        nn = spec.n_orb ** 2
        assert torch.equal(m[moff:moff + nn], m1)
        moff += nn
        # and against the oracle
        vg = oracle.coulomb_kernel((spec.n,) * 3, spec.box, spec.kernel, spec.param)
        ref = oracle.exchange(p, spec.box, vg)
        tol = 1e-7 if prec == hfx.FP32 else 1e-12
        assert abs(float(ex[i]) - ref["ex"]) <= tol * abs(ref["ex"])


# streams=2 with one tile per batch: eager calls alternate the batches over two
# streams, the captured graph keeps them on one; both must agree bit for bit
@pytest.mark.parametrize("options", [None, "tiles=1;streams=2"], ids=["default", "two_streams"])
def test_graph_replays_match_eager(options):
    dev = _dev()
    psis = _inputs()
    specs = [hfx.SystemSpec(n, (L, L, L), no, k, w) for n, L, no, k, w in SYSTEMS]
    flat = torch.from_numpy(np.concatenate([p.reshape(-1) for p in psis])).to(dev)
    print(f"case graph replay options={options}", flush=True)
    plan = hfx.Plan(specs, hfx.FP32, options=options, device=dev)
    # eager references
    k_ref, e_ref = plan.apply_exchange(flat)
    k_ref, e_ref = k_ref.clone(), e_ref.clone()
    e_only = plan.exchange_energy(flat).clone()
    kpsi = torch.zeros_like(k_ref)
    ex = torch.zeros_like(e_ref)
    g = plan.graph(hfx.GRAPH_APPLY, flat, kpsi=kpsi, ex=ex)
    ge = plan.graph(hfx.GRAPH_ENERGY, flat, ex=torch.zeros_like(e_ref))
    e_graph = ge._keep[2]
    for rep in range(4):
        kpsi.fill_(float("nan"))
        ex.fill_(0.0)
        e_graph.fill_(0.0)
        g.launch()
        ge.launch()
        torch.cuda.synchronize()
        assert torch.equal(kpsi, k_ref), rep
        assert torch.equal(ex, e_ref), rep
        assert torch.equal(e_graph, e_only), rep
        # eager work between replays
        k2, e2 = plan.apply_exchange(flat)
        torch.cuda.synchronize()
        assert torch.equal(k2, k_ref)
    g.close()
    ge.close()


def test_graph_step_matches_eager_step():
    dev = _dev()
    n, L, no = 64, 15.7, 6
    p = generate.random_pw((n, n, n), (L, L, L), no, 5.0, seed=9)
    plan = hfx.Plan(hfx.SystemSpec(n, (L, L, L), no), hfx.FP32, device=dev)
    a = torch.from_numpy(p).to(dev)
    plan.orthonormalize(a)
    ka, ea = plan.apply_exchange(a)
    ma = plan.exchange_matrix(a, ka)
    torch.cuda.synchronize()
    b = torch.from_numpy(p).to(dev)
    kb = torch.empty_like(ka)
    eb = torch.empty_like(ea)
    mb = torch.empty_like(ma)
    g = plan.graph(hfx.GRAPH_STEP, b, kpsi=kb, ex=eb, m=mb)
    for rep in range(3):
        b.copy_(torch.from_numpy(p).to(dev))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(b, a), rep
        assert torch.equal(kb, ka), rep
        assert torch.equal(eb, ea) and torch.equal(mb, ma), rep
    g.close()


@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64], ids=["fp32", "fp64"])
def test_batched_plan_with_different_row_tiles(prec):
    """Systems of 260 and 21 orbitals take 32- and 16-row tile pairs by
    default; in one plan each gives its single-system result bit for bit."""
    dev = _dev()
    L = 10.0
    psis = [generate.random_pw((24,) * 3, (L,) * 3, no, 5.0, seed=900 + no) for no in (260, 21)]
    specs = [hfx.SystemSpec(24, (L,) * 3, no) for no in (260, 21)]
    plan = hfx.Plan(specs, prec, device=dev)
    assert "rows=32" in plan.describe(0) and "rows=16" in plan.describe(1)
    flat = torch.from_numpy(np.concatenate([p.reshape(-1) for p in psis])).to(dev)
    kpsi, ex = plan.apply_exchange(flat)
    torch.cuda.synchronize()
    for i, (spec, p) in enumerate(zip(specs, psis)):
        single = hfx.Plan(spec, prec, device=dev)
        pt = torch.from_numpy(p).to(dev)
        k1, e1 = single.apply_exchange(pt)
        torch.cuda.synchronize()
        assert torch.equal(plan.split(kpsi)[i], k1)
        assert float(ex[i]) == float(e1[0])
    # the 21-orbital system against the oracle (the 260-orbital loop is long on the CPU)
    vg = oracle.coulomb_kernel((24,) * 3, (L,) * 3, hfx.TRUNCATED, 0.0)
    ref = oracle.exchange(psis[1], (L,) * 3, vg)
    tol = 1e-7 if prec == hfx.FP32 else 1e-12
    assert abs(float(ex[1]) - ref["ex"]) <= tol * abs(ref["ex"])
