"""Input check (plan option check=1): non-finite orbitals and orbitals that
break the plan's band limit (ecut=) are rejected with HFX_EINVAL before any
exchange launch; valid inputs give the unchecked plan's results bit for bit.

The band check is what makes skipping kz planes safe to rely on: a plan
told ecut skips the planes beyond the pair band 2 floor(sqrt(2 ecut) L_z /
2 pi), exact only for orbitals whose z spectrum stays within half of it.
"""
import numpy as np
import pytest

from workloads import generate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import hfx  # noqa: E402

N, L, NO = 64, 12.0, 10
SPEC = hfx.SystemSpec(N, (L,) * 3, NO, hfx.ERFC, 0.106)


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _gauss():
    return generate.gaussians((N,) * 3, (L,) * 3, NO, 20.0, 81)[0]


@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64], ids=["fp32", "fp64"])
def test_valid_inputs_pass_and_change_nothing(prec):
    dev = _dev()
    psi = torch.from_numpy(_gauss()).to(dev)
    plain = hfx.Plan(SPEC, prec, options="ecut=20", device=dev)
    checked = hfx.Plan(SPEC, prec, options="ecut=20;check=1", device=dev)
    assert "kz_max" in plain.describe()
    k1, e1 = plain.apply_exchange(psi)
    k2, e2 = checked.apply_exchange(psi)
    m2 = checked.exchange_matrix(psi)
    g2 = checked.exchange_gradient(psi)
    e3 = checked.exchange_energy(psi)
    torch.cuda.synchronize()
    assert torch.equal(k1, k2) and torch.equal(e1, e2) and torch.equal(e3, e1)
    assert torch.isfinite(m2).all() and torch.isfinite(g2).all()


def test_orbitals_beyond_the_band_rejected():
    dev = _dev()
    plan = hfx.Plan(SPEC, hfx.FP32, options="ecut=20;check=1", device=dev)
    noise = generate.white_noise((N,) * 3, (L,) * 3, NO, 82)
    with pytest.raises(hfx.HfxError) as e:
        plan.apply_exchange(torch.from_numpy(noise).to(dev))
    assert e.value.status == 1 and "ecut does not hold" in str(e.value)
    print(f"  {e.value}", flush=True)
    # a small out-of-band admixture: accepted below the tolerance, not above
    base = _gauss()
    for amp, ok in ((1e-9, True), (1e-4, False)):
        psi = torch.from_numpy(base + amp * noise).to(dev)
        if ok:
            plan.apply_exchange(psi)
            torch.cuda.synchronize()
        else:
            with pytest.raises(hfx.HfxError):
                plan.apply_exchange(psi)
    # without the band limit the same noise is valid input
    free = hfx.Plan(SPEC, hfx.FP32, options="check=1", device=dev)
    free.apply_exchange(torch.from_numpy(noise).to(dev))
    torch.cuda.synchronize()


def test_non_finite_orbitals_rejected():
    dev = _dev()
    plan = hfx.Plan(SPEC, hfx.FP64, options="check=1", device=dev)
    psi = _gauss()
    psi[3, 5, 6, 7] = np.nan
    with pytest.raises(hfx.HfxError) as e:
        plan.exchange_energy(torch.from_numpy(psi).to(dev))
    assert "orbital 3" in str(e.value) and "non-finite" in str(e.value)
    psi[3, 5, 6, 7] = np.inf
    with pytest.raises(hfx.HfxError):
        plan.exchange_gradient(torch.from_numpy(psi).to(dev))


@pytest.mark.parametrize("axis", ["x", "y"])
def test_orbitals_beyond_the_band_along_x_or_y_rejected(axis):
    """The band columns (x) and half-height planes (y) of the plane pass rely on
    the x and y bands as the skipped planes rely on the z band: an orbital
    whose z spectrum is fine but which holds a plane wave of |m| = 30 (beyond
    the 20 Ha band, |m| <= 12 on this machine) along x or y is rejected too."""
    dev = _dev()
    plan = hfx.Plan(SPEC, hfx.FP32, options="ecut=20;check=1", device=dev)
    psi = _gauss()
    wave = np.cos(2 * np.pi * 30 * np.arange(N) / N)
    if axis == "x":
        psi[2] += 1e-3 * wave[None, None, :]
    else:
        psi[2] += 1e-3 * wave[None, :, None]
    with pytest.raises(hfx.HfxError) as e:
        plan.apply_exchange(torch.from_numpy(psi).to(dev))
    assert e.value.status == 1 and f"|m_{axis}|" in str(e.value) and "orbital 2" in str(e.value)
    print(f"  {e.value}", flush=True)
