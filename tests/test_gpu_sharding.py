"""Sharding emulation on one GPU: plans with shard=g/R run the tile rounds
r % R == g only; their K psi, E_x and M add up over g to the full plan's
(float64: 1e-12 relative; float32: the parity bars)."""
import numpy as np
import pytest

from workloads import generate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import hfx  # noqa: E402


@pytest.mark.parametrize("groups", [2, 3])
@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64], ids=["fp32", "fp64"])
def test_shards_sum_to_full_plan(prec, groups):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    n, L, n_orb = 24, 10.0, 37  # 5 orbital blocks: 5 tile rounds
    psi = generate.random_pw((n, n, n), (L, L, L), n_orb, 5.0, seed=61)
    spec = hfx.SystemSpec(n, (L,) * 3, n_orb)
    pt = torch.from_numpy(psi).to(dev)
    print(f"case shards R={groups} prec={prec}", flush=True)
    full = hfx.Plan(spec, prec, device=dev)
    k_full, e_full = full.apply_exchange(pt)
    m_full = full.exchange_matrix(pt, k_full)
    k_sum = torch.zeros(psi.shape, dtype=torch.float64, device=dev)
    m_sum = torch.zeros_like(m_full)
    e_sum = 0.0
    for g in range(groups):
        plan = hfx.Plan(spec, prec, options=f"shard={g}/{groups}", device=dev)
        k, e = plan.apply_exchange(pt)
        m = plan.exchange_matrix(pt, k)
        k_sum += k.double()
        m_sum += m
        e_sum += float(e[0])
    torch.cuda.synchronize()
    ef = float(e_full[0])
    dk = float(torch.max(torch.abs(k_sum - k_full.double())))
    kmax = float(torch.max(torch.abs(k_full.double())))
    dm = float(torch.max(torch.abs(m_sum - m_full)))
    print(f"  rel dE {abs(e_sum - ef) / abs(ef):.2e}  max dK {dk:.2e}  max dM {dm:.2e}", flush=True)
    if prec == hfx.FP64:
        assert abs(e_sum - ef) <= 1e-12 * abs(ef)
        assert dk <= 1e-12 * kmax
        assert dm <= 1e-12 * float(torch.max(torch.abs(m_full)))
    else:
        assert abs(e_sum - ef) <= 1e-7 * abs(ef)
        assert dk <= 1e-5
        assert dm <= 1e-6 * float(torch.max(torch.abs(m_full)))
