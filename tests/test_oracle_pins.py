"""Pins for the FP64 oracle against facts fixed by the mathematics.

The paper prints no exchange values, so the oracle is pinned by brute force,
closed forms, special cases and invariants.  Each test names the part of the
oracle it pins; ``test_oracle_mutations.py`` shows that plausible mistakes in
the oracle fail at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import generate


# --------------------------------------------------------------------------
# helpers written independently of the oracle (naive forms, explicit sums)

def naive_kernel(g2, box, kind, w=0.0):
    """v(G) from the textbook (non cancellation-safe) forms."""
    g2 = np.asarray(g2, float)
    out = np.empty_like(g2)
    om = box[0] * box[1] * box[2]
    nz = g2 > 0
    if kind == oracle.TRUNCATED:
        rc = (3 * om / (4 * math.pi)) ** (1 / 3)
        out[nz] = 4 * math.pi / g2[nz] * (1 - np.cos(np.sqrt(g2[nz]) * rc))
        out[~nz] = 2 * math.pi * rc * rc
    else:
        out[nz] = 4 * math.pi / g2[nz] * (1 - np.exp(-g2[nz] / (4 * w * w)))
        out[~nz] = math.pi / (w * w)
    return out


def explicit_grid(shape, box):
    """Real-space points and G vectors listed explicitly, index n = (z*ny + y)*nx + x."""
    nz, ny, nx = shape
    pts, gs = [], []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                pts.append((box[0] * x / nx, box[1] * y / ny, box[2] * z / nz))

    def m_of(k, n):
        return k if k < (n + 1) // 2 else k - n
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                gs.append((2 * math.pi * m_of(x, nx) / box[0],
                           2 * math.pi * m_of(y, ny) / box[1],
                           2 * math.pi * m_of(z, nz) / box[2]))
    return np.array(pts), np.array(gs)


def brute_force_exchange(psi, box, kind, w=0.0):
    """O(N_r^2) direct-DFT evaluation of K psi, e_ij and E_x."""
    shape = psi.shape[1:]
    nr = int(np.prod(shape))
    dv = box[0] * box[1] * box[2] / nr
    pts, gs = explicit_grid(shape, box)
    phase = np.exp(-1j * gs @ pts.T)              # [G, r]
    vg = naive_kernel(np.sum(gs * gs, axis=1), box, kind, w)
    flat = psi.reshape(psi.shape[0], nr)
    n = flat.shape[0]
    kpsi = np.zeros_like(flat)
    e = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            rho = flat[i] * flat[j]
            rho_g = phase @ rho / nr
            vij = (np.conj(phase).T @ (vg * rho_g)).real
            kpsi[i] -= vij * flat[j]
            e[i, j] = dv * np.sum(rho * vij)
    return kpsi.reshape(psi.shape), e, -0.5 * e.sum()


def centred_gaussian(shape, box, alpha):
    """psi = sqrt(rho), rho = (alpha/pi)^(3/2) exp(-alpha d^2), minimum-image d."""
    nz, ny, nx = shape
    c = [0.5 * b for b in box]
    x = np.arange(nx) * box[0] / nx - c[0]
    y = np.arange(ny) * box[1] / ny - c[1]
    z = np.arange(nz) * box[2] / nz - c[2]
    d2 = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
    return ((alpha / math.pi) ** 0.75 * np.exp(-0.5 * alpha * d2))[None]


# --------------------------------------------------------------------------
# brute force: pins the FFT, its normalisation and the pair loop

@pytest.mark.parametrize("shape,box,kind,w", [
    ((4, 4, 4), (3.0, 3.0, 3.0), oracle.TRUNCATED, 0.0),
    ((6, 5, 4), (4.0, 3.5, 3.0), oracle.ERFC, 0.7),
    ((8, 6, 6), (5.0, 4.0, 4.2), oracle.TRUNCATED, 0.0),
    ((5, 7, 6), (3.3, 4.1, 3.7), oracle.ERFC, 0.106),
])
def test_brute_force_direct_dft(shape, box, kind, w):
    rng = np.random.default_rng(7)
    psi = rng.standard_normal((3,) + shape)
    vg = oracle.coulomb_kernel(shape, box, kind, w)
    res = oracle.exchange(psi, box, vg)
    kb, eb, exb = brute_force_exchange(psi, box, kind, w)
    scale = np.max(np.abs(kb))
    assert np.max(np.abs(res["kpsi"] - kb)) <= 1e-12 * scale
    assert np.max(np.abs(res["e"] - eb)) <= 1e-12 * np.max(np.abs(eb))
    assert abs(res["ex"] - exb) <= 1e-12 * abs(exb)


def test_kernel_table_matches_naive_forms():
    shape, box = (10, 12, 9), (7.0, 8.0, 6.5)
    g2 = oracle.grid_g2(shape, box)
    for kind, w in ((oracle.TRUNCATED, 0.0), (oracle.ERFC, 0.106), (oracle.ERFC, 2.0)):
        v = oracle.coulomb_kernel(shape, box, kind, w)
        ref = naive_kernel(g2, box, kind, w)
        # the naive forms lose ~1e-12 relative to cancellation at small G
        assert np.allclose(v, ref, rtol=1e-9, atol=0)
        assert np.all(v > 0)


# --------------------------------------------------------------------------
# closed forms: pin the kernel, its G = 0 value and the normalisations

def test_gaussian_self_energy_truncated():
    """Normalised Gaussian density, truncated Coulomb (range Rc):
    e_11 = sqrt(2a/pi) (1 - exp(-a Rc^2 / 2)), E_x = -e_11 / 2."""
    L, n, a = 10.0, 64, 3.0
    box = (L, L, L)
    psi = centred_gaussian((n, n, n), box, a)
    vg = oracle.coulomb_kernel((n, n, n), box, oracle.TRUNCATED)
    ex = oracle.exchange(psi, box, vg)["ex"]
    rc = (3 * L ** 3 / (4 * math.pi)) ** (1 / 3)
    ref = -0.5 * math.sqrt(2 * a / math.pi) * (1 - math.exp(-a * rc * rc / 2))
    assert abs(ex - ref) <= 1e-10 * abs(ref)


def test_gaussian_self_energy_erfc_isolated():
    """Short-range erfc kernel (images negligible): with b = a/2,
    e_11 = sqrt(2a/pi) - 2 sqrt(b w^2 / (pi (b + w^2)))."""
    L, n, a, w = 10.0, 64, 3.0, 1.0
    box = (L, L, L)
    psi = centred_gaussian((n, n, n), box, a)
    vg = oracle.coulomb_kernel((n, n, n), box, oracle.ERFC, w)
    ex = oracle.exchange(psi, box, vg)["ex"]
    b = a / 2
    ref = -0.5 * (math.sqrt(2 * a / math.pi)
                  - 2 * math.sqrt(b * w * w / (math.pi * (b + w * w))))
    assert abs(ex - ref) <= 1e-10 * abs(ref)


def test_gaussian_lattice_sum_erfc_long_range():
    """w = 0.106 (images matter): Parseval with the analytic Fourier
    coefficients exp(-G^2 / 4a) / Omega of the periodic Gaussian density gives
    E_x = -1/(2 Omega) sum_G v(G) exp(-G^2 / 2a)."""
    L, n, a, w = 10.0, 48, 3.0, 0.106
    box = (L, L, L)
    psi = centred_gaussian((n, n, n), box, a)
    vg = oracle.coulomb_kernel((n, n, n), box, oracle.ERFC, w)
    ex = oracle.exchange(psi, box, vg)["ex"]
    _, gs = explicit_grid((n, n, n), box)
    g2 = np.sum(gs * gs, axis=1)
    ref = -0.5 / L ** 3 * np.sum(naive_kernel(g2, box, oracle.ERFC, w)
                                 * np.exp(-g2 / (2 * a)))
    assert abs(ex - ref) <= 1e-11 * abs(ref)


def test_cosine_orbitals_closed_form():
    """psi_k = sqrt(2/Omega) cos(G_k r): pair densities hold 2-4 plane waves,
    e_11 = (v(0) + v(2Ga)/2)/Omega, e_12 = (v(Ga+Gb) + v(Ga-Gb))/(2 Omega)."""
    L, n = 8.0, 16
    box = (L, L, L)
    om = L ** 3
    ma, mb = np.array([1, 0, 0]), np.array([0, 2, 1])     # (x, y, z)
    ga, gb = 2 * math.pi * ma / L, 2 * math.pi * mb / L
    x = np.arange(n) * L / n
    X = x[None, None, :]
    Y = x[None, :, None]
    Z = x[:, None, None]

    def cosine(g):
        return math.sqrt(2 / om) * np.cos(g[0] * X + g[1] * Y + g[2] * Z)
    psi = np.stack([cosine(ga), cosine(gb)])
    for kind, w in ((oracle.TRUNCATED, 0.0), (oracle.ERFC, 0.3)):
        vg = oracle.coulomb_kernel((n, n, n), box, kind, w)
        res = oracle.exchange(psi, box, vg)

        def v(g):
            return float(naive_kernel(np.array([g @ g]), box, kind, w)[0])
        e11 = (v(np.zeros(3)) + 0.5 * v(2 * ga)) / om
        e22 = (v(np.zeros(3)) + 0.5 * v(2 * gb)) / om
        e12 = 0.5 * (v(ga + gb) + v(ga - gb)) / om
        assert abs(res["e"][0, 0] - e11) <= 1e-12 * e11
        assert abs(res["e"][1, 1] - e22) <= 1e-12 * e22
        assert abs(res["e"][0, 1] - e12) <= 1e-12 * e12
        ref = -0.5 * (e11 + e22) - e12
        assert abs(res["ex"] - ref) <= 1e-12 * abs(ref)


def test_constant_kernel_special_case():
    """v(G) = c reduces the Poisson solve to v_ij = c rho_ij, so
    K psi_i = -c psi_i n(r) and E_x = -(c/2) dV sum n^2 with n = sum_j psi_j^2."""
    rng = np.random.default_rng(3)
    shape, box = (6, 8, 10), (4.0, 5.0, 6.0)
    psi = rng.standard_normal((4,) + shape)
    c = 1.7
    res = oracle.exchange(psi, box, np.full(shape, c))
    dens = np.sum(psi ** 2, axis=0)
    dv = box[0] * box[1] * box[2] / np.prod(shape)
    assert np.allclose(res["kpsi"], -c * psi * dens[None], rtol=0, atol=1e-12)
    ref = -0.5 * c * dv * np.sum(dens ** 2)
    assert abs(res["ex"] - ref) <= 1e-12 * abs(ref)


# --------------------------------------------------------------------------
# invariants of the exchange functional

@pytest.fixture(scope="module")
def small_system():
    shape, box = (12, 12, 12), (6.0, 6.0, 6.0)
    psi = generate.random_pw(shape, box, 5, 4.0, seed=11)
    vg = oracle.coulomb_kernel(shape, box, oracle.TRUNCATED)
    return psi, box, vg


def test_energy_trace_identities(small_system):
    psi, box, vg = small_system
    res = oracle.exchange(psi, box, vg)
    m = oracle.exchange_matrix(psi, res["kpsi"], res["dv"])
    ex = res["ex"]
    assert ex < 0
    assert abs(0.5 * np.trace(m) - ex) <= 1e-12 * abs(ex)
    half_sum = 0.5 * res["dv"] * np.sum(psi * res["kpsi"])
    assert abs(half_sum - ex) <= 1e-12 * abs(ex)
    assert np.max(np.abs(m - m.T)) <= 1e-12 * np.max(np.abs(m))
    assert np.all(np.linalg.eigvalsh(-0.5 * (m + m.T)) > 0)      # -M is PD
    assert np.all(res["e"] >= 0) and np.allclose(res["e"], res["e"].T, rtol=0, atol=0)


def test_single_orbital_energy(small_system):
    psi, box, vg = small_system
    res = oracle.exchange(psi[:1], box, vg)
    dv = res["dv"]
    assert abs(res["ex"] + 0.5 * oracle.pair_energy(psi[0], psi[0], vg, dv)) \
        <= 1e-14 * abs(res["ex"])


def test_rotation_invariance(small_system):
    psi, box, vg = small_system
    rng = np.random.default_rng(5)
    u, _ = np.linalg.qr(rng.standard_normal((psi.shape[0],) * 2))
    rot = np.einsum("ki,k...->i...", u, psi)          # Psi U (columns mixed)
    a = oracle.exchange(psi, box, vg)
    b = oracle.exchange(rot, box, vg)
    assert abs(a["ex"] - b["ex"]) <= 1e-12 * abs(a["ex"])
    # K is one operator: K (Psi U) = (K Psi) U
    krot = np.einsum("ki,k...->i...", u, a["kpsi"])
    assert np.max(np.abs(b["kpsi"] - krot)) <= 1e-11 * np.max(np.abs(krot))
    ma = oracle.exchange_matrix(psi, a["kpsi"], a["dv"])
    mb = oracle.exchange_matrix(rot, b["kpsi"], b["dv"])
    assert np.max(np.abs(mb - u.T @ ma @ u)) <= 1e-11 * np.max(np.abs(ma))


def test_quartic_scaling(small_system):
    psi, box, vg = small_system
    a = oracle.exchange(psi, box, vg)["ex"]
    b = oracle.exchange(1.3 * psi, box, vg)["ex"]
    assert abs(b - 1.3 ** 4 * a) <= 1e-12 * abs(b)


def test_gradient_five_point_exact(small_system):
    """E_x is a quartic in a displacement t D, so the five-point stencil is
    exact up to rounding: dE/dt = 2 dV <K psi, D>."""
    psi, box, vg = small_system
    rng = np.random.default_rng(9)
    res = oracle.exchange(psi, box, vg)
    dv = res["dv"]
    for _ in range(3):
        d = rng.standard_normal(psi.shape)
        d /= math.sqrt(dv * np.sum(d * d))
        h = 1e-2
        e = {s: oracle.exchange(psi + s * h * d, box, vg, want_kpsi=False)["ex"]
             for s in (-2, -1, 1, 2)}
        fd5 = (-e[2] + 8 * e[1] - 8 * e[-1] + e[-2]) / (12 * h)
        ana = 2 * dv * np.sum(res["kpsi"] * d)
        assert abs(fd5 - ana) <= 1e-9 * abs(ana)


def test_two_real_pairs_in_one_complex_transform(small_system):
    """The identity the packed GPU path relies on: for a real even kernel,
    Re / Im of IFFT(v FFT(a + i b)) are the potentials of a and b."""
    psi, box, vg = small_system
    a, b = psi[0] * psi[1], psi[2] * psi[3]
    nr = a.size
    c = np.fft.ifftn(vg * np.fft.fftn(a + 1j * b) / nr) * nr
    assert np.max(np.abs(c.real - oracle.pair_potential(a, vg))) <= 1e-13
    assert np.max(np.abs(c.imag - oracle.pair_potential(b, vg))) <= 1e-13


def test_parallel_rows_match_serial(small_system):
    psi, box, vg = small_system
    a = oracle.exchange(psi, box, vg, workers=1)
    b = oracle.exchange(psi, box, vg, workers=3)
    assert abs(a["ex"] - b["ex"]) <= 1e-14 * abs(a["ex"])
    assert np.max(np.abs(a["kpsi"] - b["kpsi"])) <= 1e-14
    rows = oracle.apply_exchange_rows(psi, box, vg, [0, 3])
    assert np.max(np.abs(rows - a["kpsi"][[0, 3]])) <= 1e-13


# --------------------------------------------------------------------------
# orthonormalisation

def gram_schmidt(psi, dv):
    out = []
    for v in psi:
        w = v.copy()
        for q in out:
            w = w - dv * np.sum(q * w) * q
        out.append(w / math.sqrt(dv * np.sum(w * w)))
    return np.array(out)


def test_lowdin_and_cholesky(small_system):
    psi, box, _ = small_system
    rng = np.random.default_rng(1)
    raw = psi + 0.2 * rng.standard_normal(psi.shape)     # clearly non-orthogonal
    dv = box[0] * box[1] * box[2] / psi[0].size
    low, lam_min = oracle.lowdin(raw, dv)
    assert lam_min > 0
    assert np.allclose(oracle.overlap(low, dv), np.eye(len(raw)), atol=1e-12)
    # Loewdin's characterisation: the map Psi -> Psi S^-1/2 has a symmetric
    # positive-definite coefficient matrix <psi'_k | psi_l>.
    c = dv * low.reshape(len(raw), -1) @ raw.reshape(len(raw), -1).T
    assert np.max(np.abs(c - c.T)) <= 1e-12
    assert np.all(np.linalg.eigvalsh(c) > 0)
    # Cholesky orthonormalisation is classical Gram-Schmidt in orbital order.
    cho = oracle.cholesky_orthonormalize(raw, dv)
    assert np.max(np.abs(cho - gram_schmidt(raw, dv))) <= 1e-10


# --------------------------------------------------------------------------
# ACE operator (Eq. (vx_ace)): V_X^ACE = -sum_k |P_k><P_k|, P = W L^(-T)

def _ace_setup(small_system):
    psi, box, vg = small_system
    res = oracle.exchange(psi, box, vg)
    m = oracle.exchange_matrix(psi, res["kpsi"], res["dv"])
    return psi, res, m, oracle.ace_projectors(res["kpsi"], m)


def test_ace_reproduces_exchange_on_the_orbitals(small_system):
    """<P_k|psi_j> = (L^-1 M)_kj = -L^T, so V^ACE psi_j = (L P)_j = W_j exactly
    (the orbitals need not be orthonormal: small_system's are raw)."""
    psi, res, m, p = _ace_setup(small_system)
    out = oracle.ace_apply(p, psi, res["dv"])
    assert np.max(np.abs(out - res["kpsi"])) <= 1e-12 * np.max(np.abs(res["kpsi"]))
    # <P_k | psi_j> = -L^T (upper triangular) for the Cholesky factor of -M
    low = np.linalg.cholesky(-m)
    c = res["dv"] * (p.reshape(len(p), -1) @ psi.reshape(len(psi), -1).T)
    assert np.max(np.abs(c + low.T)) <= 1e-12 * np.max(np.abs(low))


def test_ace_equals_w_minv_w(small_system):
    """Another route to the same operator: V^ACE phi = W M^-1 <W|phi> (linear
    solve with M instead of the Cholesky factor), for random phi."""
    psi, res, m, p = _ace_setup(small_system)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal((3,) + psi.shape[1:])
    w = res["kpsi"].reshape(len(psi), -1)
    c = res["dv"] * (w @ phi.reshape(3, -1).T)            # <W_i | phi_j>
    want = (np.linalg.solve(m, c).T @ w).reshape(phi.shape)
    got = oracle.ace_apply(p, phi, res["dv"])
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))


def test_ace_is_negative_semidefinite_and_vanishes_off_span(small_system):
    psi, res, m, p = _ace_setup(small_system)
    dv = res["dv"]
    rng = np.random.default_rng(6)
    phi = rng.standard_normal((4,) + psi.shape[1:])
    out = oracle.ace_apply(p, phi, dv)
    quad = dv * np.sum(phi.reshape(4, -1) * out.reshape(4, -1), axis=1)
    assert np.all(quad <= 0)
    # remove the span of W from phi: the operator then gives zero
    w = res["kpsi"].reshape(len(psi), -1)
    q, _ = np.linalg.qr(w.T)
    f = phi.reshape(4, -1)
    f = f - (f @ q) @ q.T
    z = oracle.ace_apply(p, f.reshape(phi.shape), dv)
    assert np.max(np.abs(z)) <= 1e-12 * np.max(np.abs(out))


def test_ace_pins_catch_planted_mistakes(small_system):
    """The reproduction identity fails for plausible slips in building P:
    solving with L^T instead of L, multiplying by L instead of solving, and
    a dropped sign in the application."""
    psi, res, m, p = _ace_setup(small_system)
    w = res["kpsi"].reshape(len(psi), -1)
    low = np.linalg.cholesky(-m)
    ref = res["kpsi"]
    scale = np.max(np.abs(ref))
    for bad in (np.linalg.solve(low.T, w), low @ w):
        out = oracle.ace_apply(bad.reshape(psi.shape), psi, res["dv"])
        assert np.max(np.abs(out - ref)) > 1e-6 * scale
    out = -oracle.ace_apply(p, psi, res["dv"])
    assert np.max(np.abs(out - ref)) > 1e-6 * scale


# --------------------------------------------------------------------------
# s-MTACE pair screening: int |phi_i phi_j| >= rho_cut

def test_pair_overlap_abs_two_gaussians_closed_form():
    """psi_k = (2 pi s^2)^(-3/4) exp(-|r - R_k|^2 / 4 s^2): int psi_1 psi_2 =
    exp(-d^2 / 8 s^2) (both positive, so the absolute value changes nothing);
    box large enough for the periodic images to vanish."""
    n, L, s = 64, 24.0, 1.0
    x = np.arange(n) * (L / n)
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    r1, r2 = np.array([10.0, 11.0, 12.0]), np.array([13.0, 11.5, 10.0])

    def g(c):
        d2 = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2
        return (2 * math.pi * s * s) ** -0.75 * np.exp(-d2 / (4 * s * s))
    psi = np.stack([g(r1), -g(r2)])          # a sign flip: |.| makes it positive
    a = oracle.pair_overlap_abs(psi, (L / n) ** 3)
    d2 = float(np.sum((r1 - r2) ** 2))
    assert abs(a[0, 1] - math.exp(-d2 / (8 * s * s))) <= 1e-10
    assert abs(a[0, 0] - 1.0) <= 1e-10 and abs(a[1, 1] - 1.0) <= 1e-10


def test_screening_limits(small_system):
    psi, box, vg = small_system
    dv = box[0] * box[1] * box[2] / psi[0].size
    a = oracle.pair_overlap_abs(psi, dv)
    full = oracle.exchange(psi, box, vg)
    # below every overlap: nothing is screened
    keep = oracle.screen_pairs(psi, dv, 0.5 * float(np.min(a)))
    assert keep.all()
    low = oracle.exchange(psi, box, vg, keep=keep)
    assert low["ex"] == full["ex"] and np.array_equal(low["kpsi"], full["kpsi"])
    # above every off-diagonal overlap: only the self terms remain
    off = a[~np.eye(len(psi), dtype=bool)]
    diag = np.diag(a)
    cut = 0.5 * (float(off.max()) + float(diag.min()))
    assert off.max() < cut < diag.min()
    keep = oracle.screen_pairs(psi, dv, cut)
    assert np.array_equal(keep, np.eye(len(psi), dtype=bool))
    res = oracle.exchange(psi, box, vg, keep=keep)
    want_e = -0.5 * sum(oracle.pair_energy(p, p, vg, dv) for p in psi)
    want_k = np.stack([-oracle.pair_potential(p * p, vg) * p for p in psi])
    assert abs(res["ex"] - want_e) <= 1e-13 * abs(want_e)
    assert np.max(np.abs(res["kpsi"] - want_k)) <= 1e-13 * np.max(np.abs(want_k))


def test_screening_keeps_symmetric_pairs_and_diagonal(small_system):
    psi, box, vg = small_system
    dv = box[0] * box[1] * box[2] / psi[0].size
    a = oracle.pair_overlap_abs(psi, dv)
    keep = oracle.screen_pairs(psi, dv, float(np.median(a)))
    assert np.array_equal(keep, keep.T)
    assert np.diag(keep).all()


def test_screened_rows_match_screened_exchange(small_system):
    """Rows of K psi summed directly over the kept partners j agree with the
    pair loop's i <= j sums with symmetric updates; a partial keep makes the
    two differ from the unscreened rows."""
    psi, box, vg = small_system
    dv = box[0] * box[1] * box[2] / psi[0].size
    a = oracle.pair_overlap_abs(psi, dv)
    keep = oracle.screen_pairs(psi, dv, float(np.median(a)))
    assert not keep.all()
    res = oracle.exchange(psi, box, vg, keep=keep)
    rows = oracle.apply_exchange_rows(psi, box, vg, list(range(len(psi))), keep=keep)
    assert np.max(np.abs(rows - res["kpsi"])) <= 1e-13 * np.max(np.abs(rows))
    full = oracle.apply_exchange_rows(psi, box, vg, list(range(len(psi))))
    assert np.max(np.abs(full - rows)) > 1e-6 * np.max(np.abs(full))


# --------------------------------------------------------------------------
# SCDM localisation (reading 6 of the oracle)

def _scdm_case(kind, n, n_orb, seed):
    shape, box = (n, n, n), (10.0, 10.0, 10.0)
    if kind == "pw":
        psi = generate.random_pw(shape, box, n_orb, 5.0, seed)
    else:
        psi = generate.gaussians(shape, box, n_orb, 20.0 if n >= 32 else 5.0, seed)[0]
    dv = 1000.0 / n ** 3
    return oracle.lowdin(psi, dv)[0], dv


@pytest.mark.parametrize("kind,n,n_orb,seed", [("pw", 24, 8, 3), ("pw", 24, 13, 4),
                                                ("g", 32, 10, 5)])
def test_scdm_pivots_match_lapack_qrcp(kind, n, n_orb, seed):
    """The greedy selection equals LAPACK's column-pivoted QR (geqp3) of
    Psi^T wherever no near-tie makes the choice rounding-dependent."""
    import scipy.linalg as sl
    psi, _ = _scdm_case(kind, n, n_orb, seed)
    piv, gaps = oracle.scdm_pivots(psi)
    assert gaps.min() > 1e-8
    _, _, p = sl.qr(psi.reshape(n_orb, -1), pivoting=True, mode="economic")
    assert np.array_equal(piv, p[:n_orb])


def test_scdm_orthonormal_same_span_and_rotation_invariant():
    psi, dv = _scdm_case("g", 32, 10, 5)
    phi, piv = oracle.scdm(psi, dv)
    a, f = psi.reshape(10, -1), phi.reshape(10, -1)
    assert np.max(np.abs(dv * f @ f.T - np.eye(10))) <= 1e-12
    o = dv * f @ a.T                    # overlaps <phi_k|psi_i>: orthogonal when the spans agree
    assert np.max(np.abs(o @ o.T - np.eye(10))) <= 1e-12
    # the density matrix, hence the selected columns, ignores any rotation of psi
    rng = np.random.default_rng(8)
    u, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    psi_u = (u.T @ a).reshape(psi.shape)
    phi_u, piv_u = oracle.scdm(psi_u, dv)
    assert np.array_equal(piv, piv_u)
    assert np.max(np.abs(phi_u - phi)) <= 1e-11 * np.max(np.abs(phi))


def test_scdm_final_step_is_loewdin():
    """Loewdin's characterisation, independent of how the orthonormalisation
    is computed: among all orthonormal Phi = T Xi spanning the density-matrix
    columns Xi, the symmetric (Loewdin) one has T = S^(-1/2) symmetric
    positive definite, i.e. the overlaps C = <phi_k|xi_l> = (T S)_kl =
    S^(1/2) are symmetric positive definite with C C = S = <xi_k|xi_l>.
    Gram-Schmidt or Cholesky would give a triangular C instead."""
    psi, dv = _scdm_case("g", 32, 10, 5)
    phi, piv = oracle.scdm(psi, dv)
    a = psi.reshape(10, -1)
    xi = a[:, piv].T @ a                 # xi_k(r) = sum_i psi_i(c_k) psi_i(r)
    f = phi.reshape(10, -1)
    c = dv * f @ xi.T
    s = dv * xi @ xi.T
    assert np.max(np.abs(c - c.T)) <= 1e-12 * np.max(np.abs(c))
    assert np.linalg.eigvalsh(0.5 * (c + c.T)).min() > 0.0
    assert np.max(np.abs(c @ c - s)) <= 1e-11 * np.max(np.abs(s))


def test_scdm_relocalises_mixed_gaussians():
    """Localised Gaussians mixed by a random rotation are delocalised; the
    SCDM functions of the mixture are localised again (inverse participation
    ratio sum |phi|^4 / (sum |phi|^2)^2 back near that of the Gaussians)."""
    psi, dv = _scdm_case("g", 32, 10, 5)
    a = psi.reshape(10, -1)
    rng = np.random.default_rng(9)
    u, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    mixed = (u.T @ a).reshape(psi.shape)
    phi, _ = oracle.scdm(mixed, dv)

    def ipr(x):
        x = x.reshape(x.shape[0], -1)
        return np.mean(np.sum(x ** 4, axis=1) / np.sum(x ** 2, axis=1) ** 2)
    assert ipr(mixed) < 0.5 * ipr(psi)
    assert ipr(phi) > 0.7 * ipr(psi)
