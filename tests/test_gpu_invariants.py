"""Invariants of the exchange functional on the GPU outputs (the oracle's pins
restated for the HIP path): E_x(s Psi) = s^4 E_x; rotation invariance
E_x(U^T Psi) = E_x(Psi) with K(U^T Psi) = U^T K Psi; M = M^T; -M positive
definite.  Bars: float64 1e-12 (K psi: 1e-10 max|K psi|); float32 the parity
bars (E: 1e-7 relative, K psi: 1e-5 absolute, M: 1e-6 relative)."""
import numpy as np
import pytest

from workloads import generate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import hfx  # noqa: E402


@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64], ids=["fp32", "fp64"])
def test_gpu_invariants(prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    n, L, n_orb = 64, 12.0, 12
    psi = generate.gaussians((n, n, n), (L, L, L), n_orb, 20.0, seed=71)[0]
    print(f"case invariants prec={prec}", flush=True)
    plan = hfx.Plan(hfx.SystemSpec(n, (L,) * 3, n_orb, hfx.ERFC, 0.106), prec, device=dev)
    pt = torch.from_numpy(psi).to(dev)
    k, e = plan.apply_exchange(pt)
    m = plan.exchange_matrix(pt, k).view(n_orb, n_orb)
    e0 = float(e[0])
    k0 = k.double().clone()
    # quartic scaling
    e_s = float(plan.exchange_energy((1.3 * pt).contiguous())[0])
    # rotation by a seeded orthogonal U
    q, _ = np.linalg.qr(np.random.default_rng(72).standard_normal((n_orb, n_orb)))
    qt = torch.from_numpy(q.T.copy()).to(dev)
    rot = (qt @ pt.view(n_orb, -1)).view(pt.shape).contiguous()
    k_r, e_r = plan.apply_exchange(rot)
    torch.cuda.synchronize()
    mm = m.cpu().numpy()
    k_rot_want = (qt @ k0.view(n_orb, -1)).view(pt.shape)
    dk_rot = float(torch.max(torch.abs(k_r.double() - k_rot_want)))
    kmax = float(torch.max(torch.abs(k0)))
    rel_s = abs(e_s - 1.3 ** 4 * e0) / abs(1.3 ** 4 * e0)
    rel_r = abs(float(e_r[0]) - e0) / abs(e0)
    asym = np.max(np.abs(mm - mm.T)) / np.max(np.abs(mm))
    lam = np.linalg.eigvalsh(-0.5 * (mm + mm.T))
    print(f"  scale {rel_s:.2e} rotE {rel_r:.2e} rotK {dk_rot:.2e} asym {asym:.2e} "
          f"min eig(-M) {lam[0]:.3e}", flush=True)
    assert e0 < 0 and lam[0] > 0
    if prec == hfx.FP64:
        assert rel_s <= 1e-12 and rel_r <= 1e-12
        assert dk_rot <= 1e-10 * kmax
        assert asym <= 1e-12
    else:
        assert rel_s <= 1e-7 and rel_r <= 1e-7
        assert dk_rot <= 1e-5
        assert asym <= 1e-6
