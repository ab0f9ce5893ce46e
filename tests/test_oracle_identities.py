"""Pins of the oracle's constants and closed-form pieces against what the
paper and the mathematics fix (no GPU).

Each test checks an oracle piece against something other than the oracle:
printed values of the paper, textbook definitions of the D2Q9 moment basis,
moment identities stated in the paper, or closed forms of the discrete
operators.
"""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_blocks(path):
    blocks, cur = {}, None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            blocks[cur] = []
            continue
        blocks[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


def test_matrices_match_printed_eq_a1(oracle):
    M, Mi36, *_ = oracle.tables()
    g = _read_blocks(os.path.join(GOLD, "eq_a1_matrices.txt"))
    np.testing.assert_array_equal(M, g["M"])
    np.testing.assert_array_equal(Mi36, g["36*Minv"])


def test_lattice_matches_eq5(oracle):
    _, _, ex, ey, w, opp = oracle.tables()
    rows = np.loadtxt(os.path.join(GOLD, "eq5_lattice.txt"))
    np.testing.assert_array_equal(ex, rows[:, 1])
    np.testing.assert_array_equal(ey, rows[:, 2])
    np.testing.assert_allclose(36 * w, rows[:, 3], rtol=0, atol=1e-14)
    # the closed forms of Eq. (5) evaluated directly
    for i in range(1, 5):
        a = (i - 1) * np.pi / 2
        assert (ex[i], ey[i]) == (round(np.cos(a)), round(np.sin(a)))
    for i in range(5, 9):
        a = (2 * i - 9) * np.pi / 4
        assert (ex[i], ey[i]) == (round(np.sqrt(2) * np.cos(a)), round(np.sqrt(2) * np.sin(a)))
    for i in range(9):
        assert ex[opp[i]] == -ex[i] and ey[opp[i]] == -ey[i]


def test_weights_are_isotropic(oracle):
    """sum w = 1, second moment cs^2 delta, fourth moment cs^4 (dd+dd+dd)."""
    _, _, ex, ey, w, _ = oracle.tables()
    e = np.stack([ex, ey], 1).astype(float)
    cs2 = 1 / 3
    assert abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, e, e), cs2 * np.eye(2), atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia->a", w, e), 0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, e, e, e), 0, atol=1e-15)
    d = np.eye(2)
    iso4 = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e), iso4, atol=1e-15)


def test_M_rows_are_the_polynomial_moment_basis(oracle):
    """Rows of M are the standard D2Q9 moment polynomials of e_i (density,
    energy, energy squared, momentum, energy flux, stress)."""
    M, _, ex, ey, *_ = oracle.tables()
    ex = ex.astype(float)
    ey = ey.astype(float)
    e2 = ex ** 2 + ey ** 2
    basis = np.stack([np.ones(9), -4 + 3 * e2, 4 - 10.5 * e2 + 4.5 * e2 ** 2, ex,
                      (-5 + 3 * e2) * ex, ey, (-5 + 3 * e2) * ey, ex ** 2 - ey ** 2, ex * ey])
    np.testing.assert_array_equal(M, basis)
    # orthogonal rows with the usual norms
    np.testing.assert_array_equal(M @ M.T, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]))


def test_M_times_Minv_is_identity(oracle):
    M, Mi36, *_ = oracle.tables()
    # exact in integers: M @ (36 M^-1) = 36 I
    np.testing.assert_array_equal(M @ Mi36, 36 * np.eye(9))


def _random_states(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        phi = rng.uniform(0.05, 1.0)
        rho = rng.uniform(0.8, 1.2)
        ux, uy = rng.uniform(-0.1, 0.1, 2)
        kappa = rng.uniform(0.0, 1.0)
        yield phi, rho, ux, uy, kappa


def test_equilibrium_moments_of_eq15(oracle):
    """The adjusted equilibrium (Eq. 14) has the 0th-3rd moments of Eq. (15)."""
    _, _, ex, ey, *_ = oracle.tables()
    e = np.stack([ex, ey], 1).astype(float)
    cs2 = 1 / 3
    for phi, rho, ux, uy, kappa in _random_states(50, 1):
        f = oracle.feq(phi, rho, ux, uy, kappa)
        u = np.array([ux, uy])
        assert abs(f.sum() - phi * rho) < 1e-14
        np.testing.assert_allclose(e.T @ f, phi * rho * u, atol=1e-15)
        P2 = np.einsum("i,ia,ib->ab", f, e, e)
        np.testing.assert_allclose(P2, phi * rho * np.outer(u, u) + kappa * rho * cs2 * np.eye(2),
                                   atol=1e-14)
        P3 = np.einsum("i,ia,ib,ic->abc", f, e, e, e)
        d = np.eye(2)
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    sym = u[c] * d[a, b] + u[b] * d[a, c] + u[a] * d[b, c]
                    coef = phi if (a == b == c) else kappa
                    assert abs(P3[a, b, c] - coef * rho * cs2 * sym) < 1e-14


def test_eq18_is_M_times_eq14(oracle):
    M, *_ = oracle.tables()
    for phi, rho, ux, uy, kappa in _random_states(50, 2):
        np.testing.assert_allclose(M @ oracle.feq(phi, rho, ux, uy, kappa),
                                   oracle.meq(phi, rho, ux, uy, kappa), rtol=0, atol=2e-14)


def test_eq19_is_M_times_guo_force_eq6(oracle):
    """S of Eq. (19) equals M applied to Guo's discrete force of Eq. (6)."""
    M, _, ex, ey, w, _ = oracle.tables()
    e = np.stack([ex, ey], 1).astype(float)
    cs2 = 1 / 3
    rng = np.random.default_rng(3)
    for _ in range(50):
        u = rng.uniform(-0.1, 0.1, 2)
        F = rng.uniform(-1e-3, 1e-3, 2)
        Fi = np.array([w[i] * (((e[i] - u) / cs2 + (e[i] @ u) / cs2 ** 2 * e[i]) @ F)
                       for i in range(9)])
        np.testing.assert_allclose(M @ Fi, oracle.force_moments(u[0], u[1], F[0], F[1]),
                                   rtol=0, atol=1e-17)


def _periodic(oracle, nx, ny, **kw):
    return oracle.Oracle(nx, ny, np.ones((ny, nx)), **kw)


@pytest.mark.parametrize("k,q", [(1, 0), (0, 2), (3, 5), (7, 2)])
def test_gradient_symbol_on_fourier_modes(oracle, k, q):
    """Eq. (10) acting on sin(kx x + a) sin(ky y + b) has the closed-form
    symbol d_x -> 2i sin(kx) (2 + cos ky)/6 (and x<->y)."""
    nx, ny = 24, 20
    kx, ky = 2 * np.pi * k / nx, 2 * np.pi * q / ny
    o = _periodic(oracle, nx, ny)
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    psi = np.sin(kx * x + 0.3) * np.sin(ky * y + 0.7)
    gx, gy = o.gradient(psi)
    ex_x = np.cos(kx * x + 0.3) * np.sin(ky * y + 0.7) * np.sin(kx) * (2 + np.cos(ky)) / 3
    ex_y = np.sin(kx * x + 0.3) * np.cos(ky * y + 0.7) * np.sin(ky) * (2 + np.cos(kx)) / 3
    np.testing.assert_allclose(gx, ex_x, atol=1e-14)
    np.testing.assert_allclose(gy, ex_y, atol=1e-14)


def test_gradient_exact_for_quadratics_away_from_walls(oracle):
    nx, ny = 12, 10
    o = oracle.Oracle(nx, ny, np.ones((ny, nx)), bc_x="wall", bc_y="wall")
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    psi = 0.3 + 0.2 * x - 0.7 * y + 0.05 * x * x - 0.02 * x * y + 0.09 * y * y
    gx, gy = o.gradient(psi)
    s = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(gx[s], (0.2 + 0.1 * x - 0.02 * y)[s], atol=1e-13)
    np.testing.assert_allclose(gy[s], (-0.7 - 0.02 * x + 0.18 * y)[s], atol=1e-13)


def test_gradient_wall_images(oracle):
    """At a half-way wall Eq. (10) with the mirror image equals the centred
    difference of the field's even (scalars) or odd (velocity-like)
    continuation across the wall."""
    nx, ny = 8, 9
    H = float(ny)
    o = oracle.Oracle(nx, ny, np.ones((ny, nx)), bc_y="wall")
    d = (np.arange(ny)[:, None] + 0.5) * np.ones((1, nx))  # distance from the lower wall
    dd = np.arange(-1, ny + 1)[:, None] + 0.5  # one ghost row beyond each wall
    even = lambda z: np.cos(2 * np.pi * z / H)  # even about both walls
    odd = lambda z: np.sin(np.pi * z / H)  # odd about both walls, zero on them
    for fun, is_odd in ((even, False), (odd, True)):
        gx, gy = o.gradient(fun(d), odd=is_odd)
        v = fun(dd)
        cd = (v[2:] - v[:-2]) / 2 * np.ones((1, nx))
        np.testing.assert_allclose(gy, cd, atol=1e-14)
        np.testing.assert_allclose(gx, 0, atol=1e-14)
