"""Sharding emulation on the oracle: the pair list split into R virtual groups
(the way pairs would be dealt over R devices); the partial K psi and pair
energies of the groups add up to the unsplit result."""
import numpy as np
import pytest

import oracle
from workloads import generate


@pytest.mark.parametrize("groups", [2, 3, 5])
def test_pair_groups_sum_to_full_result(groups):
    shape, box = (12, 12, 12), (6.0, 6.0, 6.0)
    psi = generate.random_pw(shape, box, 6, 4.0, seed=21)
    vg = oracle.coulomb_kernel(shape, box, oracle.TRUNCATED)
    full = oracle.exchange(psi, box, vg)
    dv = full["dv"]
    pairs = [(i, j) for i in range(len(psi)) for j in range(i, len(psi))]
    kpsi = np.zeros_like(psi)
    ex = 0.0
    for g in range(groups):
        part_k = np.zeros_like(psi)
        part_e = 0.0
        for i, j in pairs[g::groups]:
            v = oracle.pair_potential(psi[i] * psi[j], vg)
            e = dv * np.sum(psi[i] * psi[j] * v)
            part_k[i] -= v * psi[j]
            if i != j:
                part_k[j] -= v * psi[i]
            part_e += -0.5 * (1.0 if i == j else 2.0) * e
        kpsi += part_k
        ex += part_e
    assert np.max(np.abs(kpsi - full["kpsi"])) <= 1e-13 * np.max(np.abs(full["kpsi"]))
    assert abs(ex - full["ex"]) <= 1e-13 * abs(full["ex"])
