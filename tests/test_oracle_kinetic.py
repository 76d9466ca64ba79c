"""Pins of the oracle's gas-kinetic point functions (CPU only).

Every expected value here comes from something other than the oracle's own
moment recursions: brute-force Gauss-Hermite / adaptive quadrature of the
Maxwellian, the Euler flux in closed form, the Chapman-Enskog Navier-Stokes
flux written out from its textbook definition, and complex-step Jacobians of
the Euler flux.
"""
import itertools

import numpy as np
import pytest
from scipy import integrate

import oracle

GAMMA = 1.4


def prim(W):
    d = len(W) - 2
    rho = W[0]
    u = W[1:1 + d] / rho
    p = (GAMMA - 1) * (W[-1] - 0.5 * rho * u @ u)
    return rho, u, p


def K_of(d):
    return (5 - 3 * GAMMA) / (GAMMA - 1) if d == 3 else (4 - 2 * GAMMA) / (GAMMA - 1)


def random_state(rng, d):
    rho = rng.uniform(0.6, 1.6)
    u = rng.uniform(-0.6, 0.6, d)
    p = rng.uniform(0.4, 1.2)
    W = np.zeros(d + 2)
    W[0], W[1:1 + d], W[-1] = rho, rho * u, p / (GAMMA - 1) + 0.5 * rho * u @ u
    return W


def gh_nodes(U, lam, n):
    x, w = np.polynomial.hermite.hermgauss(n)
    return U + x / np.sqrt(lam), w / np.sqrt(np.pi)


def brute_grid(W, n=10):
    """Tensor Gauss-Hermite nodes of the normalised Maxwellian of W:
    returns arrays (u, v, w, xi2, weight) over the grid, with the K internal
    degrees of freedom sampled individually."""
    d = len(W) - 2
    rho, u, p = prim(W)
    lam = rho / (2 * p)
    K = int(round(K_of(d)))
    axes = []
    for a in range(d):
        axes.append(gh_nodes(u[a], lam, n))
    for _ in range(K):
        axes.append(gh_nodes(0.0, lam, n))
    nodes = np.meshgrid(*[a[0] for a in axes], indexing="ij")
    wts = np.meshgrid(*[a[1] for a in axes], indexing="ij")
    wt = np.ones_like(nodes[0])
    for ww in wts:
        wt = wt * ww
    U = nodes[0].ravel()
    V = nodes[1].ravel()
    Wz = nodes[2].ravel() if d == 3 else np.zeros_like(U)
    xi2 = sum(nodes[d + k] ** 2 for k in range(K)).ravel()
    return U, V, Wz, xi2, wt.ravel()


def psi(d, U, V, Wz, xi2):
    out = [np.ones_like(U), U, V]
    if d == 3:
        out.append(Wz)
    out.append(0.5 * (U * U + V * V + Wz * Wz + xi2))
    return out


@pytest.mark.parametrize("d", [2, 3])
def test_full_moments_match_gauss_hermite(d):
    rng = np.random.default_rng(11 + d)
    for _ in range(3):
        W = random_state(rng, d)
        U, V, Wz, xi2, wt = brute_grid(W, n=8)
        for a, b, c, e in itertools.product(range(7), range(4), range(4 if d == 3 else 1), range(3)):
            ref = np.sum(wt * U ** a * V ** b * Wz ** c * xi2 ** e)
            got = oracle.moment(W, a, b, c, e)
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (a, b, c, e, got, ref)


@pytest.mark.parametrize("d", [2, 3])
def test_half_moments_match_quadrature(d):
    rng = np.random.default_rng(5)
    for _ in range(3):
        W = random_state(rng, d)
        rho, u, p = prim(W)
        lam = rho / (2 * p)
        g = lambda x: np.sqrt(lam / np.pi) * np.exp(-lam * (x - u[0]) ** 2)
        for a in range(7):
            for half, lo, hi in ((1, 0.0, np.inf), (-1, -np.inf, 0.0)):
                ref = integrate.quad(lambda x: x ** a * g(x), lo, hi, epsabs=1e-15, epsrel=1e-13)[0]
                got = oracle.moment(W, a, 0, 0, 0, half=half)
                assert abs(got - ref) <= 1e-11 * max(1.0, abs(ref)), (a, half, got, ref)


@pytest.mark.parametrize("d", [2, 3])
def test_micro_slope_reproduces_gradient(d):
    """<a psi> = dW/rho, with the expectation taken by brute-force quadrature."""
    rng = np.random.default_rng(7)
    for _ in range(4):
        W = random_state(rng, d)
        dWdx = rng.normal(size=d + 2) * 0.3
        a = oracle.micro_slope(W, dWdx)
        U, V, Wz, xi2, wt = brute_grid(W, n=6)
        ps = psi(d, U, V, Wz, xi2)
        aval = sum(a[k] * ps[k] for k in range(d + 2))
        got = np.array([np.sum(wt * ps[p] * aval) for p in range(d + 2)])
        np.testing.assert_allclose(got, dWdx / W[0], rtol=0, atol=1e-12)


def euler_flux(W, n):
    d = len(W) - 2
    rho = W[0]
    u = W[1:1 + d] / rho
    p = (GAMMA - 1) * (W[-1] - 0.5 * rho * u @ u)
    un = u @ n
    F = np.zeros(d + 2, dtype=W.dtype)
    F[0] = rho * un
    F[1:1 + d] = W[1:1 + d] * un + p * n
    F[-1] = (W[-1] + p) * un
    return F


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("mu", [0.0, 0.05, 0.3])
def test_zero_gradient_flux_is_euler(d, mu):
    """With a uniform equilibrium state the flux is the Euler flux for any
    collision time, and nothing changes in time."""
    rng = np.random.default_rng(3)
    for _ in range(4):
        W = random_state(rng, d)
        F0, Ft, Wt = oracle.gks_flux(W, np.zeros((d, d + 2)), mu=mu)
        n = np.zeros(d)
        n[0] = 1
        np.testing.assert_allclose(F0, euler_flux(W, n), rtol=0, atol=2e-15 * np.abs(W).max() * 4)
        assert np.all(Ft == 0) and np.all(Wt == 0)


def ns_flux_x(W, dW, mu, Pr):
    """Navier-Stokes flux along x from the Chapman-Enskog closure of BGK:
    stress mu (grad U + grad U^T - (2/N) div U I), N = 2/(gamma-1) total
    degrees of freedom, heat flux -mu cp grad T / Pr, cp = gamma/(gamma-1)."""
    d = len(W) - 2
    rho, u, p = prim(W)
    T = p / rho
    drho = dW[:, 0]
    du = (dW[:, 1:1 + d] - np.outer(drho, u)) / rho           # du[j, k] = d_j u_k
    dp = (GAMMA - 1) * (dW[:, -1] - dW[:, 1:1 + d] @ u + 0.5 * (u @ u) * drho)
    dT = (dp - T * drho) / rho
    N = 2.0 / (GAMMA - 1.0)
    div = np.trace(du)
    sig = mu * (du + du.T - (2.0 / N) * div * np.eye(d))
    q = -mu * GAMMA / (GAMMA - 1) * dT / Pr
    n = np.zeros(d)
    n[0] = 1
    F = euler_flux(W, n)
    F[1:1 + d] -= sig[0]
    F[-1] -= sig[0] @ u - q[0]
    return F


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("Pr", [1.0, 0.72])
def test_flux_equals_navier_stokes_closed_form(d, Pr):
    rng = np.random.default_rng(21)
    for _ in range(5):
        W = random_state(rng, d)
        dW = rng.normal(size=(d, d + 2)) * 0.4
        mu = rng.uniform(0.01, 0.2)
        F0, _, _ = oracle.gks_flux(W, dW, mu=mu, Pr=Pr)
        np.testing.assert_allclose(F0, ns_flux_x(W, dW, mu, Pr), rtol=0, atol=1e-13)


def jac_vec(f, W, v):
    h = 1e-30
    return np.imag(f(W.astype(complex) + 1j * h * v)) / h


@pytest.mark.parametrize("d", [2, 3])
def test_time_derivatives_equal_euler_chain_rule(d):
    """W_t = -sum_j dF_j/dW dW/dx_j and F_t = dF_x/dW W_t (exact for the
    Maxwellian's time derivative fixed by compatibility)."""
    rng = np.random.default_rng(31)
    eye = np.eye(d)
    for _ in range(5):
        W = random_state(rng, d)
        dW = rng.normal(size=(d, d + 2)) * 0.4
        _, Ft, Wt = oracle.gks_flux(W, dW, mu=0.1)
        Wt_ref = -sum(jac_vec(lambda X: euler_flux(X, eye[j]), W, dW[j]) for j in range(d))
        Ft_ref = jac_vec(lambda X: euler_flux(X, eye[0]), W, Wt_ref)
        np.testing.assert_allclose(Wt, Wt_ref, rtol=0, atol=1e-13)
        np.testing.assert_allclose(Ft, Ft_ref, rtol=0, atol=1e-13)


def test_two_d_flux_is_three_d_flux_of_extended_state():
    """3-D (K=2) flux of a state with w = 0 and no z-variation equals the 2-D
    (K=3) flux: both carry 2/(gamma-1) degrees of freedom."""
    rng = np.random.default_rng(41)
    for _ in range(5):
        W2 = random_state(rng, 2)
        dW2 = rng.normal(size=(2, 4)) * 0.3
        W3 = np.array([W2[0], W2[1], W2[2], 0.0, W2[3]])
        dW3 = np.zeros((3, 5))
        dW3[:2, [0, 1, 2, 4]] = dW2
        for mu, Pr in ((0.0, 1.0), (0.1, 1.0), (0.1, 0.72)):
            a = oracle.gks_flux(W2, dW2, mu=mu, Pr=Pr)
            b = oracle.gks_flux(W3, dW3, mu=mu, Pr=Pr)
            for x, y in zip(a, b):
                np.testing.assert_allclose(x, y[[0, 1, 2, 4]], rtol=0, atol=1e-14)
                assert abs(y[3]) < 1e-15


def half_flux_ref(W, d, sign):
    """(state moments, flux moments) over the half space sign*u > 0 by 1-D quadrature."""
    rho, u, p = prim(W)
    lam = rho / (2 * p)
    K = K_of(d)
    g = lambda x: np.sqrt(lam / np.pi) * np.exp(-lam * (x - u[0]) ** 2)
    lo, hi = (0.0, np.inf) if sign > 0 else (-np.inf, 0.0)
    m = [integrate.quad(lambda x: x ** k * g(x), lo, hi, epsabs=1e-16, epsrel=1e-13)[0] for k in range(4)]
    tang2 = sum(u[a] ** 2 + 1 / (2 * lam) for a in range(1, d)) + K / (2 * lam)
    Wh = np.zeros(d + 2)
    Fh = np.zeros(d + 2)
    Wh[0], Fh[0] = rho * m[0], rho * m[1]
    Wh[1], Fh[1] = rho * m[1], rho * m[2]
    for a in range(1, d):
        Wh[1 + a], Fh[1 + a] = rho * m[0] * u[a], rho * m[1] * u[a]
    Wh[-1] = 0.5 * rho * (m[2] + m[0] * tang2)
    Fh[-1] = 0.5 * rho * (m[3] + m[1] * tang2)
    return Wh, Fh


@pytest.mark.parametrize("d", [2, 3])
def test_halfspace_state_and_kfvs_match_quadrature(d):
    rng = np.random.default_rng(51)
    for _ in range(4):
        WL, WR = random_state(rng, d), random_state(rng, d)
        wl, fl = half_flux_ref(WL, d, +1)
        wr, fr = half_flux_ref(WR, d, -1)
        np.testing.assert_allclose(oracle.halfspace_state(WL, WR), wl + wr, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(oracle.kfvs(WL, WR), fl + fr, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_kfvs_limits(d):
    """KFVS(U, U) is the Euler flux; far supersonic it is the upwind Euler flux;
    equal left and right states give back that state at the interface."""
    rng = np.random.default_rng(61)
    n = np.zeros(d)
    n[0] = 1
    for _ in range(4):
        W = random_state(rng, d)
        np.testing.assert_allclose(oracle.kfvs(W, W), euler_flux(W, n), rtol=0, atol=1e-14)
        np.testing.assert_allclose(oracle.halfspace_state(W, W), W, rtol=0, atol=1e-14)
        rho, u, p = prim(W)
        c = np.sqrt(GAMMA * p / rho)
        Ws = W.copy()
        Ws[1] = rho * 12 * c
        Ws[-1] = p / (GAMMA - 1) + 0.5 * rho * (Ws[1:1 + d] / rho) @ (Ws[1:1 + d] / rho)
        # right state supersonic in +n as well: no particle moves towards -n
        Wr = random_state(rng, d)
        rr, ur, pr = prim(Wr)
        Wr[1] = rr * 12 * np.sqrt(GAMMA * pr / rr)
        Wr[-1] = pr / (GAMMA - 1) + 0.5 * rr * (Wr[1:1 + d] / rr) @ (Wr[1:1 + d] / rr)
        np.testing.assert_allclose(oracle.kfvs(Ws, Wr), euler_flux(Ws, n), rtol=1e-14, atol=1e-13)
