"""Pins of the CPU oracle to mathematics (not to itself).

Each test ties one oracle function to something fixed outside it: exact
results on polynomials with the Taylor defect constants, Fourier symbols of
the five-point formulas, an observed convergence order against continuum
derivatives, the closed form of RK4 on a pure mode, discrete energy, the
adjoint identity, finite-difference gradients and dense-matrix brute force
(numpy / torch CPU autograd).  A dropped term, wrong sign, wrong index or a
transposed operand in the oracle fails at least one of them.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workload as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def poly_box(n, g, h, f, x0=(0.0, 0.0, 0.0)):
    """Whole ghosted array (ghosts included) sampled from f(x, y, z) at x0 + i h, i in [-g, n+g)."""
    nx, ny, nz = n
    X = x0[0] + h * np.arange(-g, nx + g)[None, None, :]
    Y = x0[1] + h * np.arange(-g, ny + g)[None, :, None]
    Z = x0[2] + h * np.arange(-g, nz + g)[:, None, None]
    return np.ascontiguousarray(np.broadcast_to(f(X, Y, Z), (nz + 2 * g, ny + 2 * g, nx + 2 * g)).astype(np.float64)), X, Y, Z


# --------------------------------------------------------------------------- ghost fill

@pytest.mark.parametrize("n,g", [((5, 6, 7), 2), ((3, 4, 5), 3), ((8, 2, 3), 2), ((4, 4, 4), 4)])
def test_fill_matches_numpy_wrap(n, g):
    nx, ny, nz = n
    inner = W.uniform_pm1(7, 0, (nz, ny, nx))
    a = O.embed(inner, g, np.nan)
    O.fill_ghosts_periodic(a, g)
    np.testing.assert_array_equal(a, np.pad(inner, g, mode="wrap"))


# --------------------------------------------------------------------------- P1 polynomials

H = 2.0 ** -5


@pytest.mark.parametrize("p", range(0, 5))
def test_d1_exact_up_to_degree4(p):
    n, g = (9, 7, 6), 2
    for axis in range(3):
        f, X, Y, Z = poly_box(n, g, H, lambda x, y, z: [x, y, z][axis] ** p, x0=(0.3125, -0.5, 0.125))
        c = [X, Y, Z][axis]
        want = np.broadcast_to(p * c ** (p - 1) if p > 0 else 0.0 * c, f.shape)
        got = O.d1(f, g, axis, H)
        assert np.max(np.abs(O.interior(got - want, g))) <= 8 * np.finfo(float).eps * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("p", range(0, 6))
def test_d2_exact_up_to_degree5(p):
    n, g = (9, 7, 6), 2
    for axis in range(3):
        f, X, Y, Z = poly_box(n, g, H, lambda x, y, z: [x, y, z][axis] ** p, x0=(0.3125, -0.5, 0.125))
        c = [X, Y, Z][axis]
        want = np.broadcast_to(p * (p - 1) * c ** (p - 2) if p > 1 else 0.0 * c, f.shape)
        got = O.d2(f, g, axis, H)
        assert np.max(np.abs(O.interior(got - want, g))) <= 16 * np.finfo(float).eps * max(1.0, np.max(np.abs(want)))


def test_taylor_defects_pin_coefficients():
    """D1 x^5 = 5x^4 - 4h^4 and D2 x^6 = 30x^4 - 8h^4 exactly: the next Taylor term
    fixes the weights completely (any other 5-point weights give another defect)."""
    n, g = (10, 5, 5), 2
    T = GOLD["taylor_defects"]
    for axis in range(3):
        f, X, Y, Z = poly_box(n, g, H, lambda x, y, z: [x, y, z][axis] ** 5)
        c = [X, Y, Z][axis]
        want = T["D1_x5"]["value_coeff_x4"] * c ** 4 + T["D1_x5"]["defect_coeff_h4"] * H ** 4
        got = O.d1(f, g, axis, H)
        assert np.max(np.abs(O.interior(got - want, g))) <= 1e-14 * np.max(np.abs(want))
        f, X, Y, Z = poly_box(n, g, H, lambda x, y, z: [x, y, z][axis] ** 6)
        c = [X, Y, Z][axis]
        want = T["D2_x6"]["value_coeff_x4"] * c ** 4 + T["D2_x6"]["defect_coeff_h4"] * H ** 4
        got = O.d2(f, g, axis, H)
        assert np.max(np.abs(O.interior(got - want, g))) <= 1e-14 * np.max(np.abs(want))


def test_mixed_exact_on_products():
    """D_ab (x_a^p x_b^q) = p q x_a^(p-1) x_b^(q-1) for p, q <= 4; other axes untouched."""
    n, g = (7, 8, 6), 2
    pairs = [(0, 1), (0, 2), (1, 2)]
    for a, b in pairs:
        for p, q in [(1, 1), (2, 3), (4, 1), (3, 4)]:
            def fn(x, y, z):
                c = [x, y, z]
                return c[a] ** p * c[b] ** q + 0.5 * c[3 - a - b] ** 3
            f, X, Y, Z = poly_box(n, g, H, fn, x0=(0.25, 0.5, -0.375))
            c = [X, Y, Z]
            want = np.broadcast_to(p * q * c[a] ** (p - 1) * c[b] ** (q - 1), f.shape)
            ha, hb = H, H
            got = O.dmix(f, g, a, b, ha, hb)
            assert np.max(np.abs(O.interior(got - want, g))) <= 64 * np.finfo(float).eps * max(1.0, np.max(np.abs(want)))


def test_laplacian_and_wave_rhs_on_quadratic_with_c2():
    n, g = (6, 7, 8), 2
    dx = (H, 2 * H, 4 * H)
    # per-axis spacing: sample with the matching spacing along each axis
    nx, ny, nz = n
    X = dx[0] * np.arange(-g, nx + g)[None, None, :]
    Y = dx[1] * np.arange(-g, ny + g)[None, :, None]
    Z = dx[2] * np.arange(-g, nz + g)[:, None, None]
    u = np.ascontiguousarray(np.broadcast_to(3 * X ** 2 - 2 * Y ** 3 + Z ** 4 + X * Y * Z, (nz + 2 * g, ny + 2 * g, nx + 2 * g)))
    want = 6.0 - 12.0 * Y + 12.0 * Z ** 2
    got = O.laplacian(u, g, dx)
    assert rel(O.interior(got, g), O.interior(np.broadcast_to(want, u.shape), g)) < 1e-13
    c2 = O.embed(1.0 + 0.5 * W.uniform01(3, 1, (nz, ny, nx)), g, np.nan)
    got2 = O.wave_rhs(u, g, dx, c2)
    assert rel(O.interior(got2, g), O.interior(c2 * np.broadcast_to(want, u.shape), g)) < 1e-13
    # c2 = None means c = 1
    np.testing.assert_array_equal(O.wave_rhs(u, g, dx, None), got)


# --------------------------------------------------------------------------- P2 Fourier symbols

def symbols(kappa, n):
    """s_a, lambda_a of the five-point formulas for mode numbers kappa (x,y,z) on n (x,y,z), h = 1/n."""
    s, lam = [], []
    for a in range(3):
        h = 1.0 / n[a]
        th = 2 * np.pi * kappa[a] * h
        s.append((8 * np.sin(th) - np.sin(2 * th)) / (6 * h))
        lam.append((-2 * np.cos(2 * th) + 32 * np.cos(th) - 30) / (12 * h * h))
    return s, lam


def mode(n, kappa, phi):
    nx, ny, nz = n
    X = np.arange(nx)[None, None, :] / nx
    Y = np.arange(ny)[None, :, None] / ny
    Z = np.arange(nz)[:, None, None] / nz
    psi = 2 * np.pi * (kappa[0] * X + kappa[1] * Y + kappa[2] * Z) + phi
    return np.sin(psi), np.cos(psi)


@pytest.mark.parametrize("kappa", [(1, 0, 0), (0, 2, 0), (0, 0, 3), (1, -2, 3), (3, 1, -1)])
def test_fourier_symbols(kappa):
    n, g = (16, 12, 20), 2
    S, C = mode(n, kappa, 0.37)
    s, lam = symbols(kappa, n)
    f = O.fill_ghosts_periodic(O.embed(S, g), g)
    dx = [1.0 / v for v in n]
    for a in range(3):
        assert np.max(np.abs(O.interior(O.d1(f, g, a, dx[a]), g) - s[a] * C)) < 1e-10 * max(1, abs(s[a]))
        assert np.max(np.abs(O.interior(O.d2(f, g, a, dx[a]), g) - lam[a] * S)) < 1e-9 * max(1, abs(lam[a]))
    for a, b in [(0, 1), (0, 2), (1, 2)]:
        got = O.interior(O.dmix(f, g, a, b, dx[a], dx[b]), g)
        assert np.max(np.abs(got + s[a] * s[b] * S)) < 1e-9 * max(1, abs(s[a] * s[b]))
    assert np.max(np.abs(O.interior(O.laplacian(f, g, dx), g) - sum(lam) * S)) < 1e-9 * max(1, abs(sum(lam)))


def test_mixed_kernel_fourier_closed_form():
    """The whole multi-field output for a sum of sine modes, in closed form."""
    n, g = (12, 16, 10), 2
    modes = W.sine_modes(99, 1, nmodes=5, kmax=3)
    a, kap, phi = modes
    A = W.random_symmetric3(99, 2)
    A[0, 1] += 0.25  # also exercise a non-symmetric A: the formula uses A as given
    dx = [1.0 / v for v in n]
    fin = W.sine_sum(n, modes)
    want = np.zeros_like(fin)
    d1 = [np.zeros_like(fin) for _ in range(3)]
    for m in range(len(a)):
        S, C = mode(n, kap[m], phi[m])
        s, lam = symbols(kap[m], n)
        want += a[m] * sum(lam) * S
        for p, q in [(0, 1), (0, 2), (1, 2)]:
            want += -a[m] * s[p] * s[q] * S
        for p in range(3):
            d1[p] += a[m] * s[p] * C
    for p in range(3):
        for q in range(3):
            want += A[p, q] * d1[p] * d1[q]
    f = O.fill_ghosts_periodic(O.embed(fin, g), g)
    got = O.interior(O.deriv_mixed(f, g, dx, A), g)
    assert rel(got, want) < 1e-11


# --------------------------------------------------------------------------- P3 convergence

def test_convergence_order_four():
    errs = []
    ns = [16, 32, 64]
    for n in ns:
        S = W.sine_mode_111(n)
        f = O.fill_ghosts_periodic(O.embed(S, 2), 2)
        L = O.interior(O.laplacian(f, 2, 1.0 / n), 2)
        errs.append(np.max(np.abs(L - GOLD["continuum_laplacian_mode111"]["value"] * S)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders) > 3.95 and max(orders) < 4.1, orders


def test_mixed_kernel_converges_to_continuum():
    """Against the continuum operator on analytic sine modes (exact derivatives)."""
    modes = W.sine_modes(5, 3, nmodes=3, kmax=2)
    a, kap, phi = modes
    A = W.random_symmetric3(5, 4)
    errs = []
    for n in (24, 48):
        nn = (n, n, n)
        fin = W.sine_sum(nn, modes)
        want = np.zeros_like(fin)
        d1 = [np.zeros_like(fin) for _ in range(3)]
        for m in range(len(a)):
            S, C = mode(nn, kap[m], phi[m])
            k = 2 * np.pi * np.asarray(kap[m], dtype=float)
            want += -a[m] * (k @ k) * S
            want += -a[m] * (k[0] * k[1] + k[0] * k[2] + k[1] * k[2]) * S
            for p in range(3):
                d1[p] += a[m] * k[p] * C
        for p in range(3):
            for q in range(3):
                want += A[p, q] * d1[p] * d1[q]
        f = O.fill_ghosts_periodic(O.embed(fin, 2), 2)
        got = O.interior(O.deriv_mixed(f, 2, 1.0 / n, A), 2)
        errs.append(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    order = math.log2(errs[0] / errs[1])
    assert 3.8 < order < 4.3, (errs, order)


# --------------------------------------------------------------------------- P4 pure-mode RK4

def rk4_matrix(lam, dt):
    A = np.array([[0.0, 1.0], [lam, 0.0]])
    Z = dt * A
    P = np.eye(2)
    T = np.eye(2)
    for k in range(1, 5):
        T = T @ Z / k
        P = P + T
    return P


def test_rk4_pure_mode_closed_form():
    n = 32
    d = W.wave32()
    S = W.sine_mode_111(n)
    s, lam = symbols((1, 1, 1), (n, n, n))
    lam_tot = sum(lam)
    assert abs(lam_tot - (-118.4333)) < 1e-4  # discrete symbol of the 4th-order Laplacian
    g = 2
    u, r = O.rk4(O.embed(S, g), O.embed(np.zeros_like(S), g), g, d["dx"], d["dt"], 10)
    P = np.linalg.matrix_power(rk4_matrix(lam_tot, d["dt"]), 10)
    assert np.max(np.abs(O.interior(u, g) - P[0, 0] * S)) < 1e-12
    assert np.max(np.abs(O.interior(r, g) - P[1, 0] * S)) < 1e-12 * abs(lam_tot) ** 0.5


def test_rk4_order_against_matrix_exponential():
    """One step of RK4 on a pure mode differs from exp(dt A) by O(dt^5)."""
    from scipy.linalg import expm
    n = 16
    s, lam = symbols((1, 2, 1), (n, n, n))
    A = np.array([[0.0, 1.0], [sum(lam), 0.0]])
    errs = [np.max(np.abs(rk4_matrix(sum(lam), dt) - expm(dt * A))) for dt in (0.02, 0.01)]
    assert 4.7 < math.log2(errs[0] / errs[1]) < 5.3
    # the oracle step reproduces the matrix on the grid
    S, _ = mode((n, n, n), (1, 2, 1), 0.0)
    u, r = O.rk4(O.embed(S, 2), O.embed(0 * S, 2), 2, 1.0 / n, 0.01, 1)
    M = rk4_matrix(sum(lam), 0.01)
    assert np.max(np.abs(O.interior(u, 2) - M[0, 0] * S)) < 1e-13
    assert np.max(np.abs(O.interior(r, 2) - M[1, 0] * S)) < 1e-11


# --------------------------------------------------------------------------- P5 energy

def energy(u, rho, g, dx):
    uf = O.fill_ghosts_periodic(u.copy(), g)
    Lu = O.interior(O.laplacian(uf, g, dx), g)
    return 0.5 * np.sum(O.interior(rho, g) ** 2) - 0.5 * np.sum(O.interior(u, g) * Lu)


def test_laplacian_symmetric():
    n, g = (10, 9, 8), 2
    a = O.fill_ghosts_periodic(O.embed(W.uniform_pm1(1, 1, n[::-1]), g), g)
    b = O.fill_ghosts_periodic(O.embed(W.uniform_pm1(1, 2, n[::-1]), g), g)
    dx = (0.1, 0.2, 0.3)
    lhs = np.sum(O.interior(a, g) * O.interior(O.laplacian(b, g, dx), g))
    rhs = np.sum(O.interior(b, g) * O.interior(O.laplacian(a, g, dx), g))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs) * 100


def test_energy_ratio_pure_mode():
    n, g = 16, 2
    S, C = mode((n, n, n), (2, 1, 3), 0.3)
    s, lam = symbols((2, 1, 3), (n, n, n))
    w = math.sqrt(-sum(lam))
    dt = 0.25 / n
    u0, r0 = O.embed(S, g), O.embed(0.7 * w * C, g)
    E0 = energy(u0, r0, g, 1.0 / n)
    u1, r1 = O.rk4(u0, r0, g, 1.0 / n, dt, 1)
    E1 = energy(u1, r1, g, 1.0 / n)
    y = w * dt
    R = GOLD["rk4_energy_ratio"]
    want = 1 + R["coeff_y6"] * y ** 6 + R["coeff_y8"] * y ** 8
    assert abs(E1 / E0 - want) < 1e-12


def test_energy_random_data_bounds():
    n, g = 12, 2
    d = W.wave_cube(n, 4, "none")
    u, r = O.embed(d["u"], g), O.embed(d["rho"], g)
    E0 = energy(u, r, g, d["dx"])
    u, r = O.rk4(u, r, g, d["dx"], d["dt"], 1)
    E1 = energy(u, r, g, d["dx"])
    assert 0.98785 - 1e-12 <= E1 / E0 <= 1.0 + 1e-12


# --------------------------------------------------------------------------- P6 adjoint identity

def test_adjoint_identity_rhs_and_step():
    n, g = (7, 6, 5), 2
    nn = n[::-1]
    c2 = O.embed(1.0 + 0.5 * W.uniform_pm1(2, 9, nn), g)
    v = [O.embed(W.uniform_pm1(2, k, nn), g) for k in (1, 2)]
    w = [O.embed(W.uniform_pm1(2, k, nn), g) for k in (3, 4)]
    dx = (0.2, 0.15, 0.1)
    ip = lambda a, b: np.sum(O.interior(a, g) * O.interior(b, g))
    # RHS: A v = (rho, c^2 L_p u)
    uf = O.fill_ghosts_periodic(v[0].copy(), g)
    Av = (v[1], O.wave_rhs(uf, g, dx, c2))
    ATw = O.wave_adjoint_rhs(w[0], w[1], g, dx, c2)
    lhs = ip(Av[0], w[0]) + ip(Av[1], w[1])
    rhs = ip(v[0], ATw[0]) + ip(v[1], ATw[1])
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + 1)
    # one RK4 step M (linear in y): <M v, w> = <v, M^T w>
    dt = 0.01
    Mv = O.rk4(v[0], v[1], g, dx, dt, 1, c2)
    MTw = O.rk4_adjoint_step(v[0], v[1], w[0], w[1], g, dx, dt, c2)
    lhs = ip(Mv[0], w[0]) + ip(Mv[1], w[1])
    rhs = ip(v[0], MTw[0]) + ip(v[1], MTw[1])
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


# --------------------------------------------------------------------------- P7 FD gradients

def test_fd_gradient_checks():
    n, g = (6, 5, 7), 2
    nn = n[::-1]
    dx = (1 / 6, 1 / 5, 1 / 7)
    dt, nsteps = 0.02, 4
    c2 = O.embed(1.0 + 0.5 * W.uniform_pm1(3, 1, nn), g)
    u0 = O.embed(W.uniform_pm1(3, 2, nn), g)
    r0 = O.embed(W.uniform_pm1(3, 3, nn), g)
    ut = O.embed(W.uniform_pm1(3, 4, nn), g)
    J, gu, gr, gc = O.wave_loss_grad(u0, r0, c2, ut, g, dx, dt, nsteps)

    def loss(u, r, c):
        uN, _ = O.rk4(u, r, g, dx, dt, nsteps, c)
        return 0.5 * np.sum(O.interior(uN - ut, g) ** 2)

    assert abs(J - loss(u0, r0, c2)) < 1e-14 * J
    for k, (grad, which) in enumerate([(gu, 0), (gr, 1), (gc, 2)]):
        e = O.embed(W.uniform_pm1(3, 10 + k, nn), g)
        eps = 1e-3 if which < 2 else 1e-5
        args_p = [u0, r0, c2]
        args_m = [u0, r0, c2]
        args_p = [a + eps * e if i == which else a for i, a in enumerate(args_p)]
        args_m = [a - eps * e if i == which else a for i, a in enumerate(args_m)]
        fd = (loss(*args_p) - loss(*args_m)) / (2 * eps)
        an = np.sum(O.interior(grad, g) * O.interior(e, g))
        tol = 1e-9 if which < 2 else 1e-6
        assert abs(fd - an) < tol * max(abs(an), 1e-3), (which, fd, an)
    # ghosts of the gradients stay zero
    for grad in (gu, gr, gc):
        mask = np.ones(grad.shape, bool)
        mask[g:-g, g:-g, g:-g] = False
        assert not np.any(grad[mask])


# --------------------------------------------------------------------------- P8 brute force

def circulant(n, weights, scale):
    M = np.zeros((n, n))
    for i in range(n):
        for p, w in zip(range(-2, 3), weights):
            M[i, (i + p) % n] += w * scale
    return M


def dense_ops(n, dx):
    """Dense D1_a, D2_a on the flattened (z, y, x) interior of a periodic box."""
    nx, ny, nz = n
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    D1 = [circulant(m, [1, -8, 0, 8, -1], 1 / (12 * h)) for m, h in zip(n, dx)]
    D2 = [circulant(m, [-1, 16, -30, 16, -1], 1 / (12 * h * h)) for m, h in zip(n, dx)]
    ax = lambda Ma, a: [np.kron(Iz, np.kron(Iy, Ma)), np.kron(Iz, np.kron(Ma, Ix)), np.kron(Ma, np.kron(Iy, Ix))][a]
    return [ax(D1[a], a) for a in range(3)], [ax(D2[a], a) for a in range(3)]


@pytest.mark.parametrize("n", [(5, 6, 7), (8, 5, 6), (5, 5, 5)])
def test_brute_force_dense(n):
    g = 2
    nn = n[::-1]
    dx = (0.3, 0.25, 0.2)
    D1, D2 = dense_ops(n, dx)
    L = D2[0] + D2[1] + D2[2]
    N = int(np.prod(n))
    # Laplacian and mixed kernel
    f_in = W.uniform_pm1(8, 1, nn)
    f = O.fill_ghosts_periodic(O.embed(f_in, g), g)
    assert rel(O.interior(O.laplacian(f, g, dx), g).ravel(), L @ f_in.ravel()) < 1e-13
    A = W.random_symmetric3(8, 2)
    d1 = [D @ f_in.ravel() for D in D1]
    want = L @ f_in.ravel() + sum(D1[a] @ (D1[b] @ f_in.ravel()) for a, b in [(0, 1), (0, 2), (1, 2)])
    want += sum(A[a, b] * d1[a] * d1[b] for a in range(3) for b in range(3))
    assert rel(O.interior(O.deriv_mixed(f, g, dx, A), g).ravel(), want) < 1e-13
    # one RK4 step as the matrix polynomial p(dt A)
    c2 = 1.0 + 0.5 * W.uniform_pm1(8, 3, nn)
    Amat = np.block([[np.zeros((N, N)), np.eye(N)], [np.diag(c2.ravel()) @ L, np.zeros((N, N))]])
    dt = 0.02
    M = np.eye(2 * N)
    T = np.eye(2 * N)
    for k in range(1, 5):
        T = T @ (dt * Amat) / k
        M = M + T
    u0, r0 = W.uniform_pm1(8, 4, nn), W.uniform_pm1(8, 5, nn)
    y = M @ np.concatenate([u0.ravel(), r0.ravel()])
    uo, ro = O.rk4(O.embed(u0, g), O.embed(r0, g), g, dx, dt, 1, O.embed(c2, g))
    assert rel(np.concatenate([O.interior(uo, g).ravel(), O.interior(ro, g).ravel()]), y) < 1e-13
    # adjoint step = M^T, on both components
    lu, lr = W.uniform_pm1(8, 6, nn), W.uniform_pm1(8, 7, nn)
    yb = M.T @ np.concatenate([lu.ravel(), lr.ravel()])
    bu, br, _ = O.rk4_adjoint_step(O.embed(u0, g), O.embed(r0, g), O.embed(lu, g), O.embed(lr, g), g, dx, dt, O.embed(c2, g))
    assert rel(np.concatenate([O.interior(bu, g).ravel(), O.interior(br, g).ravel()]), yb) < 1e-13


def test_brute_force_gradient_torch_autograd():
    """dJ/du0, dJ/drho0, dJ/dc2 against torch CPU float64 autograd of the dense formulation."""
    torch = pytest.importorskip("torch")
    n, g = (5, 4, 6), 2
    nn = n[::-1]
    dx = (0.2, 0.25, 1 / 6)
    _, D2 = dense_ops(n, dx)
    L = torch.tensor(D2[0] + D2[1] + D2[2])
    dt, nsteps = 0.03, 3
    c2n = 1.0 + 0.5 * W.uniform_pm1(4, 1, nn)
    u0n, r0n, utn = (W.uniform_pm1(4, k, nn) for k in (2, 3, 4))
    c2 = torch.tensor(c2n.ravel(), requires_grad=True)
    u = torch.tensor(u0n.ravel(), requires_grad=True)
    r = torch.tensor(r0n.ravel(), requires_grad=True)

    def F(uu, rr):
        return rr, c2 * (L @ uu)

    uu, rr = u, r
    for _ in range(nsteps):
        k1 = F(uu, rr)
        k2 = F(uu + dt / 2 * k1[0], rr + dt / 2 * k1[1])
        k3 = F(uu + dt / 2 * k2[0], rr + dt / 2 * k2[1])
        k4 = F(uu + dt * k3[0], rr + dt * k3[1])
        uu = uu + dt / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        rr = rr + dt / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
    J = 0.5 * torch.sum((uu - torch.tensor(utn.ravel())) ** 2)
    J.backward()
    Jo, gu, gr, gc = O.wave_loss_grad(O.embed(u0n, g), O.embed(r0n, g), O.embed(c2n, g), O.embed(utn, g), g, dx, dt, nsteps)
    assert abs(Jo - J.item()) < 1e-13 * J.item()
    assert rel(O.interior(gu, g).ravel(), u.grad.numpy()) < 1e-12
    assert rel(O.interior(gr, g).ravel(), r.grad.numpy()) < 1e-12
    assert rel(O.interior(gc, g).ravel(), c2.grad.numpy()) < 1e-12


def test_mixed_is_composition_of_first_derivatives():
    """The tensor-product reading: D_ab f = D1_a(D1_b f) with a periodic fill in between."""
    n, g = (9, 8, 7), 2
    f = O.fill_ghosts_periodic(O.embed(W.uniform_pm1(6, 1, n[::-1]), g), g)
    dx = (0.1, 0.2, 0.3)
    for a, b in [(0, 1), (0, 2), (1, 2)]:
        inner = O.fill_ghosts_periodic(O.d1(f, g, b, dx[b]), g)
        comp = O.interior(O.d1(inner, g, a, dx[a]), g)
        assert rel(O.interior(O.dmix(f, g, a, b, dx[a], dx[b]), g), comp) < 1e-13
