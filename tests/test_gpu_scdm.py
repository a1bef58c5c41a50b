"""SCDM localisation on the GPU (through the C ABI) against the oracle.

The pivots are integers decided by floating-point comparisons in another
summation order than the oracle's, so every case first checks on the oracle
that each step's largest residual norm leads the runner-up by a relative
margin (1e-9) far above that rounding; then the pivots must agree exactly
and the localised orthonormal orbitals to 1e-10 of their largest value
(float64 throughout, in either plan precision).
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


def _case(kind, n, L, n_orb, seed):
    shape, box = (n, n, n), (L, L, L)
    dv = L ** 3 / n ** 3
    if kind == "pw":
        psi = generate.random_pw(shape, box, n_orb, 5.0, seed)
    else:
        # localised Gaussians mixed by a random rotation: delocalised input
        g = generate.gaussians(shape, box, n_orb, 20.0, seed)[0]
        u, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n_orb, n_orb)))
        psi = (u.T @ g.reshape(n_orb, -1)).reshape(g.shape)
    psi, _ = oracle.lowdin(psi, dv)
    return psi, dv


@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("kind,n,L,n_orb,seed", [("pw", 24, 10.0, 8, 3), ("pw", 24, 10.0, 13, 4),
                                                  ("g", 64, 23.5, 40, 5)])
def test_scdm_matches_oracle(kind, n, L, n_orb, seed, prec):
    psi, dv = _case(kind, n, L, n_orb, seed)
    piv_ref, gaps = oracle.scdm_pivots(psi)
    assert gaps.min() > 1e-9, gaps.min()
    phi_ref, _ = oracle.scdm(psi, dv)
    print(f"case scdm {kind} n={n} n_orb={n_orb} prec={prec} min gap {gaps.min():.2e}",
          flush=True)
    dev = _dev()
    plan = hfx.Plan(hfx.SystemSpec(n, (L,) * 3, n_orb), prec, device=dev)
    pt = torch.from_numpy(psi).to(dev)
    phi, piv = plan.scdm(pt)
    torch.cuda.synchronize()
    assert np.array_equal(piv.cpu().numpy(), piv_ref)
    d = np.max(np.abs(phi.cpu().numpy() - phi_ref)) / np.max(np.abs(phi_ref))
    print(f"  rel max dphi {d:.2e}", flush=True)
    assert d <= 1e-10


def test_scdm_in_place_and_two_systems():
    """phi may overwrite psi; a two-system plan gives each system's result
    bit for bit, with the pivots of each system in its own slice."""
    dev = _dev()
    a, _ = _case("pw", 24, 10.0, 8, 3)
    b, _ = _case("g", 64, 23.5, 12, 6)
    singles = []
    for x, n, L in ((a, 24, 10.0), (b, 64, 23.5)):
        p = hfx.Plan(hfx.SystemSpec(n, (L,) * 3, x.shape[0]), hfx.FP64, device=dev)
        phi, piv = p.scdm(torch.from_numpy(x).to(dev))
        singles.append((phi.reshape(-1), piv))
    plan = hfx.Plan([hfx.SystemSpec(24, (10.0,) * 3, 8), hfx.SystemSpec(64, (23.5,) * 3, 12)],
                    hfx.FP64, device=dev)
    flat = torch.from_numpy(np.concatenate([a.reshape(-1), b.reshape(-1)])).to(dev)
    phi, piv = plan.scdm(flat, phi=flat)          # in place
    torch.cuda.synchronize()
    assert phi.data_ptr() == flat.data_ptr()
    assert torch.equal(phi[: a.size], singles[0][0]) and torch.equal(phi[a.size:], singles[1][0])
    assert torch.equal(piv[:8], singles[0][1]) and torch.equal(piv[8:], singles[1][1])


def test_scdm_then_screening_keeps_fewer_pairs():
    """The s-MTACE chain on a delocalised (rotated) set: after SCDM the pair
    overlaps int |phi_a phi_b| fall, so a cut keeps fewer pairs than on the
    rotated orbitals themselves."""
    psi, dv = _case("g", 64, 23.5, 40, 5)
    dev = _dev()
    plan = hfx.Plan(hfx.SystemSpec(64, (23.5,) * 3, 40, hfx.ERFC, 0.106), hfx.FP32, device=dev)
    pt = torch.from_numpy(psi).to(dev)
    before = plan.screen(pt, 2.5e-2)[0]
    phi, _ = plan.scdm(pt)
    after = plan.screen(phi, 2.5e-2)[0]
    print(f"  kept pairs: rotated {before}, SCDM {after} of {40 * 41 // 2}", flush=True)
    assert after < 0.5 * before
