"""hfx_apply_exchange_noalloc (the entry point for callers that cannot
allocate) through the C ABI against hfx_apply_exchange on the same inputs:
two calls in a row, the second with a smaller input (another plan, fewer
orbitals and a smaller grid), each bitwise equal to the workspace entry
point's K psi and E_x (the same launch sequence), and both within the
parity bars of the oracle.  A plan whose K psi calls need more than the
static scratch is rejected with HFX_ENOMEM before any launch."""
import ctypes

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


def _noalloc(lib, plan, psi, kpsi, ex):
    vp = ctypes.c_void_p
    return lib.hfx_apply_exchange_noalloc(plan._h, vp(psi.data_ptr()), vp(kpsi.data_ptr()),
                                          vp(ex.data_ptr()),
                                          vp(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("prec", [hfx.FP32, hfx.FP64], ids=["fp32", "fp64"])
def test_noalloc_matches_workspace_entry_point(prec):
    dev = _dev()
    lib = hfx.load_library()
    lib.hfx_apply_exchange_noalloc.argtypes = [ctypes.c_void_p] * 5
    lib.hfx_apply_exchange_noalloc.restype = ctypes.c_int
    # one tile pair of 8 rows per batch keeps the 64^3 plan's workspace in
    # the scratch; the second call is the smaller input
    cases = [(64, 12.0, 21, hfx.ERFC, 0.106, "g", 61, "tiles=1;rows=8"),
             (24, 10.0, 7, hfx.TRUNCATED, 0.0, "pw", 62, None)]
    for n, L, n_orb, kernel, w, fam, seed, opts in cases:
        shape, box = (n, n, n), (L, L, L)
        if fam == "g":
            psi_h = generate.gaussians(shape, box, n_orb, 20.0, seed)[0]
        else:
            psi_h = generate.random_pw(shape, box, n_orb, 5.0, seed)
        print(f"case noalloc n={n} n_orb={n_orb} prec={prec}", flush=True)
        plan = hfx.Plan(hfx.SystemSpec(n, box, n_orb, kernel, w), prec, options=opts, device=dev)
        psi = torch.from_numpy(psi_h).to(dev)
        k_ref, e_ref = plan.apply_exchange(psi)
        kpsi = torch.full_like(k_ref, float("nan"))
        ex = torch.full_like(e_ref, float("nan"))
        assert _noalloc(lib, plan, psi, kpsi, ex) == 0, lib.hfx_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(kpsi, k_ref) and torch.equal(ex, e_ref)
        vg = oracle.coulomb_kernel(shape, box, kernel, w)
        ref = oracle.exchange(psi_h, box, vg, workers=4)
        rel = abs(float(ex[0]) - ref["ex"]) / abs(ref["ex"])
        dk = float(np.max(np.abs(kpsi.double().cpu().numpy() - ref["kpsi"])))
        kmax = float(np.max(np.abs(ref["kpsi"])))
        print(f"  rel dE {rel:.2e}  max dK {dk:.2e}", flush=True)
        if prec == hfx.FP32:
            assert rel <= 1e-7 and dk <= 1e-5
        else:
            assert rel <= 1e-12 and dk <= 1e-10 * kmax


def test_noalloc_rejects_plans_beyond_the_scratch():
    dev = _dev()
    lib = hfx.load_library()
    lib.hfx_apply_exchange_noalloc.argtypes = [ctypes.c_void_p] * 5
    lib.hfx_apply_exchange_noalloc.restype = ctypes.c_int
    # 96^3 with 64 orbitals and default batches: well over 256 MiB of workspace
    plan = hfx.Plan(hfx.SystemSpec(96, (23.5,) * 3, 64, hfx.ERFC, 0.106), hfx.FP32, device=dev)
    psi = torch.zeros(64 * 96 ** 3, dtype=torch.float64, device=dev)
    kpsi = torch.zeros(64 * 96 ** 3, dtype=torch.float32, device=dev)
    ex = torch.zeros(1, dtype=torch.float64, device=dev)
    assert _noalloc(lib, plan, psi, kpsi, ex) == 3
    assert "static scratch" in lib.hfx_last_error().decode()
    vp = ctypes.c_void_p
    assert lib.hfx_apply_exchange_noalloc(plan._h, vp(psi.data_ptr()), vp(0), vp(0), vp(0)) == 1
