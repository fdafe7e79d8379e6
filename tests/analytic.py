"""Closed-form solutions used to pin the oracle (test infrastructure).

Each function states where its formula comes from: the paper's closed forms
(Sections 4.1 and 4.2) or textbook solutions of the incompressible
Navier-Stokes equations.  Arrays are numpy-ordered ([y, x] / [z, y, x]).
"""
import math

import numpy as np


def rel_l2(exact, numeric):
    """Relative L2 error of Section 4: |phi_a - phi_n|_2 / |phi_a|_2."""
    exact = np.asarray(exact, np.float64)
    numeric = np.asarray(numeric, np.float64)
    return float(np.linalg.norm((exact - numeric).ravel()) / np.linalg.norm(exact.ravel()))


def taylor_green_2d(N, u0, nu, t):
    """Decaying 2D Taylor-Green vortex (textbook exact NSE solution) on an N x N
    periodic box, nodes at (i + 1/2, j + 1/2), k = 2 pi / N:
      u = -u0 cos kx sin ky e^{-2 nu k^2 t},  v = u0 sin kx cos ky e^{-2 nu k^2 t},
      P = -(u0^2/4)(cos 2kx + cos 2ky) e^{-4 nu k^2 t},
      omega = dv/dx - du/dy = 2 u0 k cos kx cos ky e^{-2 nu k^2 t}."""
    k = 2 * math.pi / N
    x = np.arange(N) + 0.5
    X, Y = np.meshgrid(x, x, indexing="xy")
    e = math.exp(-2 * nu * k * k * t)
    u = -u0 * np.cos(k * X) * np.sin(k * Y) * e
    v = u0 * np.sin(k * X) * np.cos(k * Y) * e
    P = -(u0 * u0 / 4) * (np.cos(2 * k * X) + np.cos(2 * k * Y)) * e * e
    g = np.empty((2, 2, N, N))
    g[0, 0] = u0 * k * np.sin(k * X) * np.sin(k * Y) * e
    g[0, 1] = -u0 * k * np.cos(k * X) * np.cos(k * Y) * e
    g[1, 0] = u0 * k * np.cos(k * X) * np.cos(k * Y) * e
    g[1, 1] = -u0 * k * np.sin(k * X) * np.sin(k * Y) * e
    vort = 2 * u0 * k * np.cos(k * X) * np.cos(k * Y) * e
    return {"u": np.stack([u, v]), "P": P, "grad": g, "vort": vort}


def taylor_green_3d_linear(N, u0, nu, t):
    """Velocity of the 3D Taylor-Green field in its linear (Stokes) regime,
    u = u0 sin x cos y cos z e^{-3 nu k^2 t}, v = -u0 cos x sin y cos z e^{...},
    w = 0, with x = k (i + 1/2), k = 2 pi / N.  Exact for the Stokes
    equations; the nonlinear correction is O(u0^2)."""
    k = 2 * math.pi / N
    c = (np.arange(N) + 0.5) * k
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    e = math.exp(-3 * nu * k * k * t)
    u = u0 * np.sin(X) * np.cos(Y) * np.cos(Z) * e
    v = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z) * e
    return np.stack([u, v, np.zeros_like(u)])


def poiseuille(F, nu, H, y):
    """Section 4.1 closed forms with the wall at y = 0 and y = H:
    u1 = F/(2 nu) y (H - y); du1/dy = F/(2 nu)(H - 2y); S_xy = du1/dy / 2;
    omega = -du1/dy."""
    u1 = F / (2 * nu) * y * (H - y)
    g = F / (2 * nu) * (H - 2 * y)
    return {"u1": u1, "du1dy": g, "Sxy": 0.5 * g, "vort": -g}


def four_roll_mill(N, U0, shift=0.5):
    """Section 4.2 closed forms on [0, 2 pi]^2 (physical units):
    u1 = U0 sin x cos y, u2 = -U0 cos x sin y, S_xx = U0 cos x cos y = -S_yy,
    omega = 2 U0 sin x sin y."""
    dx = 2 * math.pi / N
    x = (np.arange(N) + shift) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    return {
        "u1": U0 * np.sin(X) * np.cos(Y),
        "u2": -U0 * np.cos(X) * np.sin(Y),
        "Sxx": U0 * np.cos(X) * np.cos(Y),
        "Syy": -U0 * np.cos(X) * np.cos(Y),
        "vort": 2 * U0 * np.sin(X) * np.sin(Y),
    }


def couette(U, H, y):
    """Plane Couette flow between a resting wall at y = 0 and a wall moving
    with U at y = H: u1 = U y / H (textbook)."""
    return U * y / H
