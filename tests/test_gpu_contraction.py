"""The exchange-matrix contraction M = dV Psi^T (K Psi) on its own (the ACE
matrix M of the Methods' MTACE subsection), through the C ABI, separated
from the error of K psi.

Float32 plans compute it with psi (float64) split as hi = fl32(psi),
lo = fl32(psi - hi), both multiplied with the float32 K psi on float32 MFMA,
each float32 accumulator folded into float64 every 32 grid points, the
folds and chunk partials summed in float64 and scaled by dV once.

1. Exactness on short mantissas.  Inputs are built so that every product and
   every float32 partial sum of at most 32 terms is an integer multiple of a
   power of two below 2^24 in size: then the design computes the sum with no
   rounding at all, and M equals fl64(dV * S) bit for bit, S being the exact
   integer-arithmetic sum.  Two cases, each with a plausible wrong design that
   the same bar rejects (shown on the CPU, next to the GPU check):
   a) lo != 0: dropping the lo product (hi only) leaves sum lo*b out, a
      relative error near 1e-8;
   b) products near 2^19, so that 32-term sums stay below 2^24 but 64-term
      sums do not: folding every 64 points (or never) rounds.
2. Real orbitals: M from the plan's own float32 K psi against the float64
   product dV Psi^T float64(K psi), within the bound of the design
   (64 roundings of 2^-24 of sum |psi_k K psi_l| per fold, a deliberately
   loose worst case), and the K-psi-forming entry point
   hfx_exchange_matrix against apply + hfx_exchange_matrix_kpsi, bitwise.
"""
import numpy as np
import pytest

from workloads import generate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import hfx  # noqa: E402

N, L, N_ORB = 24, 10.0, 136       # 136 orbitals: two 128-row tiles, ragged
NR = N ** 3
DV = L ** 3 / NR


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _gpu_m(a, b):
    dev = _dev()
    plan = hfx.Plan(hfx.SystemSpec(N, (L, L, L), N_ORB), hfx.FP32, device=dev)
    m = plan.exchange_matrix(torch.from_numpy(a).to(dev),
                             kpsi=torch.from_numpy(b).to(dev))
    torch.cuda.synchronize()
    return m.view(N_ORB, N_ORB).cpu().numpy()


def _fold_emulation(hi, b, fold):
    """float32 accumulation of hi * b in 4-point MFMA steps, folded into
    float64 every `fold` points (CPU emulation of a design, for a few
    elements)."""
    prod = (hi.astype(np.float64) * b.astype(np.float64))        # exact (< 2^24)
    steps = prod.reshape(prod.shape[0], -1, 4).sum(axis=2)       # exact
    steps = steps.reshape(prod.shape[0], -1, fold // 4).astype(np.float32)
    part = np.cumsum(steps, axis=2, dtype=np.float32)[:, :, -1]  # sequential float32
    return part.astype(np.float64).sum(axis=1)


def test_split_contraction_exact_with_lo_part():
    rng = np.random.default_rng(31)
    hi = rng.integers(2048, 4096, size=(N_ORB, NR))      # exact in float32
    k = rng.integers(1, 64, size=(N_ORB, NR))           # lo = k 2^-20 < ulp(hi) / 2
    bint = rng.integers(1, 16, size=(N_ORB, NR))
    a = hi.astype(np.float64) + k.astype(np.float64) * 2.0 ** -20
    assert np.array_equal(a.astype(np.float32).astype(np.int64), hi)
    b = bint.astype(np.float32)
    s_hi = hi @ bint.T                                   # int64, < 2^30
    s_lo = k @ bint.T                                    # int64
    exact = s_hi.astype(np.float64) + s_lo.astype(np.float64) * 2.0 ** -20   # exact
    ref = DV * exact
    got = _gpu_m(a.reshape(N_ORB, N, N, N), b.reshape(N_ORB, N, N, N))
    bad = int(np.sum(got != ref))
    print(f"  split contraction: {bad} of {ref.size} entries differ from fl64(dV S)",
          flush=True)
    assert bad == 0
    hi_only = DV * s_hi.astype(np.float64)
    rel = np.max(np.abs(hi_only - ref) / np.abs(ref))
    print(f"  a hi-only product would be off by {rel:.2e} (relative)", flush=True)
    assert rel > 1e-9


def test_split_contraction_exact_with_long_sums():
    rng = np.random.default_rng(32)
    hi = rng.integers(2048, 4096, size=(N_ORB, NR))
    bint = rng.integers(64, 128, size=(N_ORB, NR))      # products in [2^17, 2^19)
    a = hi.astype(np.float64)
    b = bint.astype(np.float32)
    ref = DV * (hi @ bint.T).astype(np.float64)          # < 2^33: exact
    got = _gpu_m(a.reshape(N_ORB, N, N, N), b.reshape(N_ORB, N, N, N))
    bad = int(np.sum(got != ref))
    print(f"  long sums: {bad} of {ref.size} entries differ from fl64(dV S)", flush=True)
    assert bad == 0
    # the same products folded every 64 points round (16 elements emulated)
    rows = hi[:4].repeat(4, axis=0)
    cols = np.tile(bint[:4], (4, 1))
    s64 = _fold_emulation(rows, cols, 64)
    s32 = _fold_emulation(rows, cols, 32)
    ex = np.einsum("ij,ij->i", rows.astype(np.float64), cols.astype(np.float64))
    assert np.array_equal(s32, ex)
    print(f"  a 64-point fold would be off in {int(np.sum(s64 != ex))} of 16 emulated "
          f"entries", flush=True)
    assert np.any(s64 != ex)


def test_contraction_of_real_orbitals_and_kpsi_forming_call():
    dev = _dev()
    psi = generate.gaussians((64, 64, 64), (12.0,) * 3, 40, 20.0, seed=33)[0]
    dv = 12.0 ** 3 / 64 ** 3
    plan = hfx.Plan(hfx.SystemSpec(64, (12.0,) * 3, 40, hfx.ERFC, 0.106), hfx.FP32, device=dev)
    pt = torch.from_numpy(psi).to(dev)
    kpsi, ex = plan.apply_exchange(pt)
    m_kpsi = plan.exchange_matrix(pt, kpsi)
    m_new = torch.empty_like(m_kpsi)
    ex_new = torch.empty_like(ex)
    plan.exchange_matrix(pt, m=m_new, ex=ex_new)
    torch.cuda.synchronize()
    assert torch.equal(m_new, m_kpsi) and torch.equal(ex_new, ex)
    k64 = kpsi.double().cpu().numpy().reshape(40, -1)
    a = psi.reshape(40, -1)
    ref = dv * (a @ k64.T)
    scale = dv * (np.abs(a) @ np.abs(k64).T)
    err = np.abs(m_kpsi.view(40, 40).cpu().numpy() - ref)
    worst = float(np.max(err / scale))
    print(f"  max |dM| / (dV sum |psi||K psi|) = {worst:.2e}", flush=True)
    assert worst <= 64 * 2.0 ** -24
