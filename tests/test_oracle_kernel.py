"""Pins of the oracle's Kelvin tensor (Sec. 4.1) against the elasticity it solves.

The kernel is pinned by physics, not by retyping its formula:
  * symmetry S_ab = S_ba, evenness S(-r) = S(r), homogeneity S(l r) = S(r)/l;
  * the Navier system (Sec. 1) mu Lap u + (lambda + mu) grad div u = 0 holds for
    u = S e_b away from the origin (finite differences);
  * point-force equilibrium: with Hooke's law and the Lame constants of Sec. 1,
    the traction of u = S e_b integrated over any sphere around the origin equals
    -e_b. This fixes the 1/(8 pi) constant (a constant of 1/8, read from the
    garbled prefactor of eq. Vh, would give -pi e_b).
"""
import json
import os

import numpy as np
import pytest

import oracle as O

MATERIALS = [(1.0, 0.3), (2.5, 0.2), (0.7, 0.45)]


def lame(E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return lam, mu


def test_symmetry_evenness_homogeneity():
    rng = np.random.default_rng(5)
    for E, nu in MATERIALS:
        for _ in range(20):
            r = rng.standard_normal(3)
            S = O.kelvin(r, E, nu)
            assert np.allclose(S, S.T, rtol=0, atol=1e-15 * np.abs(S).max())
            assert np.allclose(O.kelvin(-r, E, nu), S, rtol=1e-15, atol=0)
            lam = 3.7
            assert np.allclose(O.kelvin(lam * r, E, nu), S / lam, rtol=1e-14, atol=0)
            # 1/E scaling
            assert np.allclose(O.kelvin(r, 2 * E, nu), S / 2, rtol=1e-14, atol=0)


def test_golden_values():
    """Hand-evaluated values (tests/golden/kelvin_points.json) of the Sec. 4.1 tensor."""
    path = os.path.join(os.path.dirname(__file__), "golden", "kelvin_points.json")
    with open(path) as f:
        g = json.load(f)
    for case in g["cases"]:
        S = O.kelvin(case["r"], case["E"], case["nu"])
        assert np.allclose(S, np.array(case["S"]), rtol=1e-12, atol=1e-15), case


def _u(x, b, E, nu):
    return O.kelvin(x, E, nu)[:, b]


def _grad(x, b, E, nu, h):
    """G[i, j] = d u_j / d x_i by 4th-order central differences."""
    G = np.zeros((3, 3))
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        G[i] = (-_u(x + 2 * e, b, E, nu) + 8 * _u(x + e, b, E, nu) - 8 * _u(x - e, b, E, nu)
                + _u(x - 2 * e, b, E, nu)) / (12 * h)
    return G


@pytest.mark.parametrize("E,nu", MATERIALS)
def test_navier_equation(E, nu):
    lam, mu = lame(E, nu)
    rng = np.random.default_rng(7)
    h = 1e-3
    for _ in range(6):
        x = rng.standard_normal(3)
        x *= 1.3 / np.linalg.norm(x)
        for b in range(3):
            lap = np.zeros(3)
            hess = np.zeros((3, 3, 3))  # hess[i, k, j] = d_i d_k u_j
            for i in range(3):
                for k in range(3):
                    ei = np.zeros(3); ei[i] = h
                    ek = np.zeros(3); ek[k] = h
                    hess[i, k] = (_u(x + ei + ek, b, E, nu) - _u(x + ei - ek, b, E, nu)
                                  - _u(x - ei + ek, b, E, nu) + _u(x - ei - ek, b, E, nu)) / (4 * h * h)
            for i in range(3):
                lap += hess[i, i]
            grad_div = np.array([sum(hess[i, k, k] for k in range(3)) for i in range(3)])
            t1 = mu * lap
            t2 = (lam + mu) * grad_div
            res = t1 + t2
            scale = np.abs(t1).max() + np.abs(t2).max()
            assert np.abs(res).max() <= 2e-5 * scale, (res, scale)


def _sphere_rule(n_theta=24, n_phi=48):
    ct, wt = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    pts, wts = [], []
    for c, w in zip(ct, wt):
        s = np.sqrt(1 - c * c)
        for p in phi:
            pts.append((s * np.cos(p), s * np.sin(p), c))
            wts.append(w * 2 * np.pi / n_phi)
    return np.array(pts), np.array(wts)


@pytest.mark.parametrize("E,nu", MATERIALS)
@pytest.mark.parametrize("R", [0.5, 2.0])
def test_point_force_equilibrium(E, nu, R):
    lam, mu = lame(E, nu)
    pts, wts = _sphere_rule()
    h = 1e-4 * R
    for b in range(3):
        F = np.zeros(3)
        for n, w in zip(pts, wts):
            x = R * n
            G = _grad(x, b, E, nu, h)  # G[i, j] = d_i u_j
            eps = 0.5 * (G + G.T)
            sigma = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps  # Hooke's law (Sec. 1)
            F += w * R * R * sigma @ n
        expect = -np.eye(3)[b]
        assert np.abs(F - expect).max() < 1e-7, (b, F)
