"""Write full-size oracle reference values for a named workload.

Calls only the float64 CPU oracle (``oracle/``) and the seeded input
generators (``workloads/``).  Output ``tests/golden/<name>_oracle.json``:

  ex        E_x of the Loewdin-orthonormalised orbitals
  m_diag    <psi_i | K psi_i> = -sum_j e_ij for every orbital i
  samples   K psi values of a few orbitals at seeded grid points
            (orbital index, flat point index, value)

With --screen RHO it writes ``<name>_smtace_oracle.json`` instead: the same
quantities summed over the pairs kept by the s-MTACE criterion
int |psi_a psi_b| >= rho_cut (``oracle.screen_pairs``), with rho_cut moved to
the middle of the gap of A values that contains RHO (so that a different
summation order of A keeps the same pairs), and the number of kept pairs.

With --rows I,J,... it writes ``<name>_rows_oracle.json`` instead, for
workloads too large for the full pair loop: K psi of the listed orbitals only
(each row sums over all partners, ``oracle.apply_exchange_rows``), evaluated
on the raw generated orbitals (no orthonormalisation, as the batched
benchmark runs them), with <psi_i|K psi_i> of those rows and K psi at seeded
sample points.

With --scdm it writes ``<name>_scdm_oracle.json``: the SCDM pivots of the
Loewdin orbitals (``oracle.scdm_pivots``), the smallest relative lead of the
chosen residual norm over the runner-up across the steps, and the localised
orthonormal orbitals at seeded sample points.

With --full-raw it writes ``<name>_full_oracle.json``: the full pair loop on
the raw generated orbitals (exactly the input the batched and large-box
benchmarks feed), i.e. E_x and <psi_i|K psi_i> = -sum_j e_ij for every
orbital, plus K psi of orbitals spread over all orbital blocks (each summed
over all partners) at seeded sample points.

With --fd it writes ``<name>_fd_oracle.json``: E_x of the raw orbitals and of
psi + m h D_k for m = -2, -1, 1, 2, h = 1e-4 and the seeded directions D_k of
``workloads.generate.fd_direction`` (k = 0..15), all from the oracle's full
pair loop.

With --ace it writes ``<name>_ace_oracle.json``: the ACE projectors
P = W L^-T (``oracle.ace_projectors``) of the Loewdin orbitals, from the
oracle's full K psi and M, at seeded sample points of rows spread over the
Cholesky blocks, and the diagonal of L (from <P_k|psi_k> = -L_kk).

Usage: python tests/golden/make_golden.py water96 [--workers 8] [--screen 2.5e-2]
       python tests/golden/make_golden.py large128 --rows 0,1,255,511 [--workers 4]
The workload definitions live in workloads/configs.py; each record stores the
generator parameters it was made from.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import configs  # noqa: E402

SAMPLE_ORBITALS = (0, 1)
SAMPLE_POINTS = 256


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--screen", type=float, default=None)
    ap.add_argument("--rows", default=None)
    ap.add_argument("--scdm", action="store_true")
    ap.add_argument("--full-raw", action="store_true")
    ap.add_argument("--fd", action="store_true")
    ap.add_argument("--ace", action="store_true")
    a = ap.parse_args()
    s = configs.ALL[a.name]
    if a.full_raw:
        full_raw_mode(s, a.workers)
        return
    if a.fd:
        fd_mode(s, a.workers)
        return
    if a.ace:
        ace_mode(s, a.workers)
        return
    if a.scdm:
        scdm_mode(s)
        return
    if a.rows is not None:
        rows_mode(s, [int(r) for r in a.rows.split(",")], a.workers)
        return
    t0 = time.time()
    psi = s.orbitals()
    dv = oracle.volume(s.box) / psi[0].size
    psi_o, lam_min = oracle.lowdin(psi, dv)
    del psi
    vg = oracle.coulomb_kernel(s.shape, s.box, s.kernel, s.param)
    keep, extra, suffix = None, {}, ""
    if a.screen is not None:
        amat = oracle.pair_overlap_abs(psi_o, dv)
        vals = np.unique(amat[np.triu_indices(s.n_orb)])
        hi = vals[vals >= a.screen].min()
        lo = vals[vals < a.screen].max()
        rho = 0.5 * (lo + hi)
        keep = oracle.screen_pairs(psi_o, dv, rho)
        n_keep = int(np.triu(keep).sum())
        extra = {"rho_cut_requested": a.screen, "rho_cut": rho,
                 "gap_rel": (hi - lo) / hi, "pairs_kept": n_keep}
        suffix = "_smtace"
        print(f"screening at rho_cut {rho:.6e} (gap {(hi - lo) / hi:.2e}): {n_keep} pairs kept",
              flush=True)
    print(f"{s.name}: orthonormalised (min eig S {lam_min:.3e}), running "
          f"{s.n_pairs if keep is None else extra['pairs_kept']} pairs "
          f"on {a.workers} workers", flush=True)
    res = oracle.exchange(psi_o, s.box, vg, want_kpsi=False, workers=a.workers, keep=keep)
    m_diag = -res["e"].sum(axis=1)
    print(f"E_x = {res['ex']:.15f}  ({time.time() - t0:.0f} s)", flush=True)
    rng = np.random.default_rng(12345)
    pts = rng.choice(psi_o[0].size, size=SAMPLE_POINTS, replace=False)
    rows = oracle.apply_exchange_rows(psi_o, s.box, vg, list(SAMPLE_ORBITALS), keep=keep)
    samples = [[int(o), int(p), float(rows[k].reshape(-1)[p])]
               for k, o in enumerate(SAMPLE_ORBITALS) for p in pts]
    rec = {"name": s.name, "n": s.n, "L": s.L, "n_orb": s.n_orb, "kernel": s.kernel,
           "param": s.param, "family": s.family, "ecut": s.ecut, "seed": s.seed,
           "orthonormalisation": "Loewdin (oracle eigh)", "min_eig_overlap": lam_min,
           "ex": res["ex"], "m_diag": [float(x) for x in m_diag], "samples": samples,
           "seconds": time.time() - t0, "workers": a.workers, **extra}
    out = os.path.join(HERE, f"{s.name}{suffix}_oracle.json")
    with open(out, "w") as f:
        json.dump(rec, f)
    print(f"wrote {out} ({time.time() - t0:.0f} s)", flush=True)


_ROWS = {}  # inputs of the row jobs, inherited by the forked workers


def _row_job(i):
    return oracle.apply_exchange_rows(_ROWS["psi"], _ROWS["box"], _ROWS["vg"], [i])[0]


def rows_mode(s, rows, workers):
    import multiprocessing as mp
    t0 = time.time()
    psi = s.orbitals()
    dv = oracle.volume(s.box) / psi[0].size
    vg = oracle.coulomb_kernel(s.shape, s.box, s.kernel, s.param)
    print(f"{s.name}: {len(rows)} rows of {s.n_orb} partners each on {workers} workers",
          flush=True)
    _ROWS.update(psi=psi, box=s.box, vg=vg)
    with mp.get_context("fork").Pool(max(1, min(workers, len(rows)))) as pool:
        out = pool.map(_row_job, rows)
    rng = np.random.default_rng(12345)
    pts = rng.choice(psi[0].size, size=SAMPLE_POINTS, replace=False)
    samples = [[int(i), int(p), float(out[k].reshape(-1)[p])]
               for k, i in enumerate(rows) for p in pts]
    m_diag = [float(dv * np.sum(psi[i] * out[k])) for k, i in enumerate(rows)]
    rec = {"name": s.name, "n": s.n, "L": s.L, "n_orb": s.n_orb, "kernel": s.kernel,
           "param": s.param, "family": s.family, "ecut": s.ecut, "seed": s.seed,
           "orthonormalisation": "none (raw generated orbitals)", "rows": rows,
           "m_diag_rows": m_diag, "samples": samples, "seconds": time.time() - t0,
           "workers": workers}
    path = os.path.join(HERE, f"{s.name}_rows_oracle.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    print(f"wrote {path} ({time.time() - t0:.0f} s)", flush=True)


def spread_rows(n_orb):
    """Orbitals spread over the orbital blocks of any tiling: the first two,
    one in each quarter and the last."""
    return sorted({0, min(1, n_orb - 1), n_orb // 4 + 3 if n_orb > 8 else 0,
                   n_orb // 2 + 5 if n_orb > 16 else n_orb // 2,
                   3 * n_orb // 4 + 7 if n_orb > 32 else 3 * n_orb // 4, n_orb - 1})


def _record(s, **kw):
    return {"name": s.name, "n": s.n, "L": s.L, "n_orb": s.n_orb, "kernel": s.kernel,
            "param": s.param, "family": s.family, "ecut": s.ecut, "seed": s.seed, **kw}


def full_raw_mode(s, workers):
    import multiprocessing as mp
    t0 = time.time()
    psi = s.orbitals()
    dv = oracle.volume(s.box) / psi[0].size
    vg = oracle.coulomb_kernel(s.shape, s.box, s.kernel, s.param)
    print(f"{s.name}: full pair loop, {s.n_pairs} pairs on {workers} workers (raw orbitals)",
          flush=True)
    res = oracle.exchange(psi, s.box, vg, want_kpsi=False, workers=workers)
    m_diag = -res["e"].sum(axis=1)
    t1 = time.time()
    print(f"E_x = {res['ex']:.15f}  ({t1 - t0:.0f} s)", flush=True)
    rows = spread_rows(s.n_orb)
    _ROWS.update(psi=psi, box=s.box, vg=vg)
    with mp.get_context("fork").Pool(max(1, min(workers, len(rows)))) as pool:
        out = pool.map(_row_job, rows)
    _ROWS.clear()
    rng = np.random.default_rng(12345)
    pts = rng.choice(psi[0].size, size=SAMPLE_POINTS, replace=False)
    samples = [[int(i), int(p), float(out[k].reshape(-1)[p])]
               for k, i in enumerate(rows) for p in pts]
    m_rows = [float(dv * np.sum(psi[i] * out[k])) for k, i in enumerate(rows)]
    rec = _record(s, orthonormalisation="none (raw generated orbitals)", ex=res["ex"],
                  m_diag=[float(x) for x in m_diag], rows=rows, m_diag_rows=m_rows,
                  samples=samples, seconds=time.time() - t0, seconds_pair_loop=t1 - t0,
                  workers=workers, cpu_model=_cpu_model())
    path = os.path.join(HERE, f"{s.name}_full_oracle.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    print(f"wrote {path} ({time.time() - t0:.0f} s)", flush=True)


FD_H = 1e-4
FD_STEPS = (-2, -1, 1, 2)
FD_DIRECTIONS = 16


def fd_mode(s, workers):
    from workloads import generate
    t0 = time.time()
    psi = s.orbitals()
    dv = oracle.volume(s.box) / psi[0].size
    vg = oracle.coulomb_kernel(s.shape, s.box, s.kernel, s.param)
    e0 = oracle.exchange(psi, s.box, vg, want_kpsi=False, workers=workers)["ex"]
    print(f"{s.name}: E_x = {e0:.15f} ({time.time() - t0:.0f} s)", flush=True)
    energies = []
    for k in range(FD_DIRECTIONS):
        d = generate.fd_direction(psi.shape, dv, s.seed + 1000, k)
        row = []
        for m in FD_STEPS:
            row.append(oracle.exchange(psi + (m * FD_H) * d, s.box, vg, want_kpsi=False,
                                       workers=workers)["ex"])
        energies.append(row)
        print(f"direction {k}: {row} ({time.time() - t0:.0f} s)", flush=True)
    rec = _record(s, orthonormalisation="none (raw generated orbitals)", ex=e0, h=FD_H,
                  steps=list(FD_STEPS), direction_seed=s.seed + 1000, energies=energies,
                  seconds=time.time() - t0, workers=workers, cpu_model=_cpu_model())
    path = os.path.join(HERE, f"{s.name}_fd_oracle.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    print(f"wrote {path} ({time.time() - t0:.0f} s)", flush=True)


def ace_mode(s, workers):
    t0 = time.time()
    psi = s.orbitals()
    dv = oracle.volume(s.box) / psi[0].size
    psi_o, _ = oracle.lowdin(psi, dv)
    del psi
    vg = oracle.coulomb_kernel(s.shape, s.box, s.kernel, s.param)
    res = oracle.exchange(psi_o, s.box, vg, want_kpsi=True, workers=workers)
    m = oracle.exchange_matrix(psi_o, res["kpsi"], dv)
    print(f"{s.name}: K psi and M done ({time.time() - t0:.0f} s)", flush=True)
    p = oracle.ace_projectors(res["kpsi"], m)
    l_diag = -np.einsum("kn,kn->k", p.reshape(s.n_orb, -1), psi_o.reshape(s.n_orb, -1)) * dv
    rows = spread_rows(s.n_orb)
    rng = np.random.default_rng(12345)
    pts = rng.choice(psi_o[0].size, size=SAMPLE_POINTS, replace=False)
    samples = [[int(i), int(q), float(p[i].reshape(-1)[q])] for i in rows for q in pts]
    rec = _record(s, orthonormalisation="Loewdin (oracle eigh)", ex=res["ex"], rows=rows,
                  l_diag=[float(x) for x in l_diag], samples=samples,
                  seconds=time.time() - t0, workers=workers, cpu_model=_cpu_model())
    path = os.path.join(HERE, f"{s.name}_ace_oracle.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    print(f"wrote {path} ({time.time() - t0:.0f} s)", flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((ln.split(":", 1)[1].strip() for ln in f
                         if ln.startswith("model name")), None)
    except OSError:
        return None


def scdm_mode(s):
    t0 = time.time()
    psi = s.orbitals()
    dv = oracle.volume(s.box) / psi[0].size
    psi_o, _ = oracle.lowdin(psi, dv)
    del psi
    piv, gaps = oracle.scdm_pivots(psi_o)
    phi, _ = oracle.scdm(psi_o, dv)
    rng = np.random.default_rng(12345)
    pts = rng.choice(phi[0].size, size=SAMPLE_POINTS, replace=False)
    orbs = (0, 1, s.n_orb - 1)
    samples = [[int(o), int(p), float(phi[o].reshape(-1)[p])] for o in orbs for p in pts]
    rec = {"name": s.name, "n": s.n, "L": s.L, "n_orb": s.n_orb, "kernel": s.kernel,
           "param": s.param, "family": s.family, "ecut": s.ecut, "seed": s.seed,
           "orthonormalisation": "Loewdin (oracle eigh)", "pivots": [int(x) for x in piv],
           "min_gap": float(gaps.min()), "samples": samples, "seconds": time.time() - t0}
    path = os.path.join(HERE, f"{s.name}_scdm_oracle.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    print(f"wrote {path} (min gap {gaps.min():.2e}, {time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
