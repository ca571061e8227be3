"""Reference values of Y0 = u(0, x0) for the benchmark problems (Sec. 4).
TEST INFRASTRUCTURE.

* Black–Scholes–Barenblatt: the closed form u(t,x) = exp((r + s^2)(T - t)) |x|^2
  printed in Sec. 4.
* Hamilton–Jacobi–Bellman: the Cole–Hopf formula of Sec. 4,
  u(t,x) = -ln E[exp(-g(x + sqrt(2) W_{T-t}))] (the subscript is T - t), with
  x = 0 so that |sqrt(2) W_T|^2 = 2 T chi^2_d; evaluated as a 1-D quadrature
  over the chi-square density, and by plain Monte Carlo.
* Allen–Cahn: no closed form.  x0 = 0 and g is radial, so u(t,x) = v(T-t,|x|)
  with v_tau = v_rr + (d-1)/r v_r + v - v^3 (the PDE of Sec. 4 with sigma =
  sqrt(2) and driver y^3 - y, in time-to-go tau).  Solved by Strang splitting:
  exact logistic-cubic reaction half steps around a Crank–Nicolson radial
  diffusion step, Neumann condition at r = R.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, linalg, stats


def bsb_y0(d: int = 100, T: float = 1.0, r: float = 0.05, sigma: float = 0.4, x0=None) -> float:
    if x0 is None:
        x0 = np.array([1.0 if i % 2 == 0 else 0.5 for i in range(d)])
    return float(math.exp((r + sigma * sigma) * T) * float(np.dot(x0, x0)))


def bsb_u(t, x, T=1.0, r=0.05, sigma=0.4):
    return math.exp((r + sigma * sigma) * (T - t)) * float(np.dot(x, x))


def hjb_y0_quad(d: int = 100, T: float = 1.0, lam: float = 1.0) -> float:
    """-(1/lam) ln E[(2 / (1 + 2 T q))^lam], q ~ chi^2_d, by adaptive
    quadrature (u(0, 0) of the Cole–Hopf formula; lam = 1 in Sec. 4)."""
    lo, hi = stats.chi2.ppf(1e-15, d), stats.chi2.ppf(1.0 - 1e-15, d)
    f = lambda q: (2.0 / (1.0 + 2.0 * T * q)) ** lam * stats.chi2.pdf(q, d)
    val, _err = integrate.quad(f, lo, hi, limit=500, epsabs=0.0, epsrel=1e-13)
    return float(-math.log(val) / lam)


def hjb_mean_g(d: int = 100, T: float = 1.0) -> float:
    """E[g(X_T)] = E[ln((1 + 2 T q) / 2)], q ~ chi^2_d: the value Y0 would take
    without the driver (lam = 0)."""
    lo, hi = stats.chi2.ppf(1e-15, d), stats.chi2.ppf(1.0 - 1e-15, d)
    f = lambda q: math.log(0.5 * (1.0 + 2.0 * T * q)) * stats.chi2.pdf(q, d)
    val, _err = integrate.quad(f, lo, hi, limit=500, epsabs=0.0, epsrel=1e-13)
    return float(val)


def hjb_y0_mc(d: int = 100, T: float = 1.0, n: int = 10 ** 6, seed: int = 7):
    """Plain Monte Carlo of the Cole–Hopf expectation; returns (value, stderr)."""
    rng = np.random.default_rng(seed)
    acc, acc2, done = 0.0, 0.0, 0
    while done < n:
        k = min(100_000, n - done)
        W = rng.standard_normal((k, d)) * math.sqrt(T)
        X = math.sqrt(2.0) * W
        e = 2.0 / (1.0 + np.einsum("ij,ij->i", X, X))
        acc += e.sum()
        acc2 += (e * e).sum()
        done += k
    mean = acc / n
    var = acc2 / n - mean * mean
    se = math.sqrt(var / n)
    return float(-math.log(mean)), float(se / mean)


def hjb_grad_u(tau, X, lam: float = 1.0, n_par: int = 160, n_perp: int = 48):
    """grad u of the Hamilton–Jacobi–Bellman problem at time-to-go tau > 0 and
    points X [K][d], from the Cole–Hopf formula of Sec. 4:
    u = -(1/lam) ln w, w(tau, x) = E[exp(-lam g(x + sqrt(2) W_tau))] with
    g(y) = ln((1 + |y|^2) / 2), so exp(-g) = 2 / (1 + |y|^2) (the formula is
    written for lam = 1; other lam use exp(-lam g) = (2 / (1 + |y|^2))^lam).
    grad w = E[-lam exp(-lam g(y)) 2 y / (1 + |y|^2)] and grad u = -grad w / (lam w).
    Both expectations depend on x through rho = |x| only: with s = sqrt(2 tau)
    and x along e_1, |y|^2 = (rho + s xi)^2 + s^2 q, xi ~ N(0, 1) and
    q ~ chi^2_{d-1} independent, and grad w points along x.  Gauss–Hermite in
    xi times generalized Gauss–Laguerre in q / 2 (exact for the chi-square
    weight); returns (u [K], grad u [K][d])."""
    from numpy.polynomial.hermite_e import hermegauss
    from scipy.special import roots_genlaguerre
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    K, d = X.shape
    s = math.sqrt(2.0 * tau)
    xi, wx = hermegauss(n_par)
    wx = wx / math.sqrt(2.0 * math.pi)
    if d > 1:
        r, wr = roots_genlaguerre(n_perp, 0.5 * (d - 1) - 1.0)
        wr = wr / math.gamma(0.5 * (d - 1))
        q = 2.0 * r
    else:
        q, wr = np.zeros(1), np.ones(1)
    rho = np.sqrt((X * X).sum(1))
    u = np.empty(K)
    gr = np.empty(K)
    for a in range(0, K, 256):
        b = min(K, a + 256)
        yp = rho[a:b, None, None] + s * xi[None, :, None]          # component along x
        y2 = yp * yp + s * s * q[None, None, :]
        e = (2.0 / (1.0 + y2)) ** lam                               # exp(-lam g(y))
        wgt = wx[None, :, None] * wr[None, None, :]
        w = (e * wgt).sum((1, 2))
        dw = (-lam * e * 2.0 * yp / (1.0 + y2) * wgt).sum((1, 2))
        u[a:b] = -np.log(w) / lam
        gr[a:b] = -dw / (lam * w)
    with np.errstate(invalid="ignore", divide="ignore"):
        unit = np.where(rho[:, None] > 0, X / rho[:, None], 0.0)
    return u, gr[:, None] * unit


def radial_heat_quad(d: int, tau: float, g) -> float:
    """E[g(|sqrt(2) W_tau|)] for a radial g: the linear (no reaction) version
    of the Allen–Cahn solve, used to pin the radial finite differences."""
    lo, hi = stats.chi2.ppf(1e-15, d), stats.chi2.ppf(1.0 - 1e-15, d)
    f = lambda q: g(math.sqrt(2.0 * tau * q)) * stats.chi2.pdf(q, d)
    val, _ = integrate.quad(f, lo, hi, limit=500, epsabs=0.0, epsrel=1e-12)
    return float(val)


def radial_solve(d: int, tau_end: float, g, reaction: bool = True, R: float = 40.0,
                 K: int = 4000, steps: int = 600) -> float:
    """v(tau_end, 0) of v_tau = v_rr + (d-1)/r v_r [+ v - v^3], v(0, r) = g(r)."""
    h = R / K
    r = np.arange(K + 1) * h
    v = np.array([g(x) for x in r])
    dt = tau_end / steps
    # Laplacian matrix A (tridiagonal) with the symmetric condition at r = 0
    # (Laplacian -> d v_rr) and zero flux at r = R.
    lower = np.zeros(K + 1)
    diag = np.zeros(K + 1)
    upper = np.zeros(K + 1)
    diag[0] = -2.0 * d / h ** 2
    upper[0] = 2.0 * d / h ** 2
    i = np.arange(1, K)
    diag[i] = -2.0 / h ** 2
    upper[i] = 1.0 / h ** 2 + (d - 1) / (2.0 * h * r[i])
    lower[i] = 1.0 / h ** 2 - (d - 1) / (2.0 * h * r[i])
    diag[K] = -2.0 / h ** 2
    lower[K] = 2.0 / h ** 2

    def apply(x):
        y = diag * x
        y[:-1] += upper[:-1] * x[1:]
        y[1:] += lower[1:] * x[:-1]
        return y

    # banded form of (I - dt/2 A)
    ab = np.zeros((3, K + 1))
    ab[0, 1:] = -0.5 * dt * upper[:-1]
    ab[1, :] = 1.0 - 0.5 * dt * diag
    ab[2, :-1] = -0.5 * dt * lower[1:]

    def react(x, t):
        # exact flow of v' = v - v^3
        e2 = math.exp(2.0 * t)
        return x * math.exp(t) / np.sqrt(1.0 + x * x * (e2 - 1.0))

    for _ in range(steps):
        if reaction:
            v = react(v, 0.5 * dt)
        v = linalg.solve_banded((1, 1), ab, v + 0.5 * dt * apply(v))
        if reaction:
            v = react(v, 0.5 * dt)
    return float(v[0])


def ac_y0(d: int = 20, T: float = 0.3, **kw) -> float:
    return radial_solve(d, T, lambda x: 1.0 / (2.0 + 0.4 * x * x), reaction=True, **kw)


def ac_mean_g(d: int, T: float = 0.3) -> float:
    """E[g(X_T)] for Allen–Cahn (the reaction-free value; Y0 must exceed it
    because v - v^3 > 0 on (0, 1))."""
    return radial_heat_quad(d, T, lambda x: 1.0 / (2.0 + 0.4 * x * x))



