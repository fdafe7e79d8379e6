"""Vortex centres of a lid-driven cavity (test infrastructure).

The stream function is integrated from the bottom wall (psi = 0 there):
psi(x, y_j) = sum_{j' < j} u(x, y_j') dy + u(x, y_j) dy / 2 for cell-centred
nodes y_j = (j + 1/2) dy.  A vortex centre is a local extremum of psi,
refined by a quadratic fit through the 3 x 3 neighbourhood; the vorticity
there is interpolated bilinearly.  Positions are returned in units of the
cavity side (x, y in [0, 1])."""
import numpy as np


def stream_function(u, dy=1.0):
    """u: [y, x] horizontal velocity; returns psi[y, x]."""
    cum = np.cumsum(u, axis=0) * dy
    return cum - 0.5 * u * dy


def _refine(psi, j, i):
    """Quadratic fit of psi around (j, i); returns sub-node offsets."""
    ny, nx = psi.shape
    if not (0 < j < ny - 1 and 0 < i < nx - 1):
        return 0.0, 0.0
    fxx = psi[j, i + 1] - 2 * psi[j, i] + psi[j, i - 1]
    fyy = psi[j + 1, i] - 2 * psi[j, i] + psi[j - 1, i]
    fx = 0.5 * (psi[j, i + 1] - psi[j, i - 1])
    fy = 0.5 * (psi[j + 1, i] - psi[j - 1, i])
    fxy = 0.25 * (psi[j + 1, i + 1] - psi[j + 1, i - 1] - psi[j - 1, i + 1] + psi[j - 1, i - 1])
    H = np.array([[fxx, fxy], [fxy, fyy]])
    g = np.array([fx, fy])
    try:
        d = -np.linalg.solve(H, g)
    except np.linalg.LinAlgError:
        return 0.0, 0.0
    d = np.clip(d, -1.0, 1.0)
    return float(d[1]), float(d[0])     # (dy, dx)


def _bilinear(f, y, x):
    ny, nx = f.shape
    x = min(max(x, 0.0), nx - 1.0)
    y = min(max(y, 0.0), ny - 1.0)
    i0, j0 = int(np.floor(x)), int(np.floor(y))
    i1, j1 = min(i0 + 1, nx - 1), min(j0 + 1, ny - 1)
    tx, ty = x - i0, y - j0
    return float((1 - ty) * ((1 - tx) * f[j0, i0] + tx * f[j0, i1]) + ty * ((1 - tx) * f[j1, i0] + tx * f[j1, i1]))


def find_vortex(psi, vort, region, kind):
    """Extremum of psi inside region = (x0, x1, y0, y1) (fractions of the
    side); kind 'min' or 'max'.  Returns (omega, x, y)."""
    ny, nx = psi.shape
    x0, x1, y0, y1 = region
    i0, i1 = int(x0 * nx), max(int(x1 * nx), int(x0 * nx) + 1)
    j0, j1 = int(y0 * ny), max(int(y1 * ny), int(y0 * ny) + 1)
    sub = psi[j0:j1, i0:i1]
    k = np.argmin(sub) if kind == "min" else np.argmax(sub)
    j, i = np.unravel_index(k, sub.shape)
    j, i = j + j0, i + i0
    dy, dx = _refine(psi, j, i)
    yc, xc = j + dy, i + dx
    w = _bilinear(vort, yc, xc)
    return w, (xc + 0.5) / nx, (yc + 0.5) / ny
