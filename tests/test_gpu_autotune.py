"""Autotuner: every candidate it times meets the parity bar (covered per
variant in test_gpu_parity), the choice is cached, and a re-run with the cache
returns the same options without timing again."""
import json

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2309_00651_amd import autotune, hfx  # noqa: E402
from workloads import generate  # noqa: E402


def test_tune_and_cache(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n, L, no = 96, 23.5, 8
    spec = hfx.SystemSpec(n, (L, L, L), no, hfx.ERFC, 0.106)
    psi = torch.from_numpy(generate.gaussians((n,) * 3, (L,) * 3, no, 20.0, 7)[0]).cuda()
    cache = str(tmp_path / "tune.json")
    best = autotune.tune(spec, hfx.FP32, psi, cache_path=cache, reps=1)
    assert best in autotune.candidates(spec, hfx.FP32)
    rec = json.load(open(cache))
    assert len(rec) == 1
    (k, v), = rec.items()
    assert v["options"] == best and len(v["timings"]) == len(autotune.candidates(spec, hfx.FP32))
    assert autotune.cached_options(spec, hfx.FP32, cache) == best
    assert autotune.tune(spec, hfx.FP32, psi, cache_path=cache) == best
    plan = hfx.Plan(spec, hfx.FP32, options=best)
    kpsi, ex = plan.apply_exchange(psi)
    torch.cuda.synchronize()
    assert torch.isfinite(ex).all()
