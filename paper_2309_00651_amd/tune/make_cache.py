"""Tune the benchmark workloads' kernel configurations on this GPU into the
library's tune cache (``paper_2309_00651_amd/tune/mi355x.txt`` by default).

Runs ``hfx_autotune`` (through ``autotune.tune``) on the seeded synthetic
orbitals of each named workload, with the workload's orbital cutoff as a
base option, and prints each choice.  Entries of other builds or workloads
stay in the file; a re-run replaces the named workloads' entries only when
the cache lacks them (delete the file to time everything again).

Usage: python -m paper_2309_00651_amd.tune.make_cache [batched6 water96 large128]
                                                      [--cache PATH] [--reps 2]
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_CACHE = os.path.join(HERE, "mi355x.txt")


def main():
    import torch

    from paper_2309_00651_amd import autotune, hfx
    from workloads import configs

    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="*", default=["batched6", "water96"])
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--reps", type=int, default=2)
    a = ap.parse_args()
    dev = torch.device("cuda:0")
    for name in a.workloads:
        systems = configs.BATCHED6 if name == "batched6" else (configs.ALL[name],)
        for s in systems:
            spec = hfx.SystemSpec(s.n, s.box, s.n_orb, s.kernel, s.param)
            psi = torch.from_numpy(s.orbitals()).to(dev)
            best = autotune.tune(spec, hfx.FP32, psi, cache_path=a.cache, reps=a.reps,
                                 options=f"ecut={s.ecut:g}")
            print(f"{s.name}: {best}", flush=True)
            del psi
            torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
