"""ctypes front end of the plain-C FP64 oracle (``mdf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the CPU
baseline leg of the benchmark.  It never imports the GPU package and the GPU
package never imports it.

Arrays use numpy order: a 2D field is ``a[y, x]``, a 3D field ``a[z, y, x]``;
vector fields carry the component first (``u[b, y, x]``), the gradient is
``grad[a, b] = d u_a / d x_b`` (eq. 3-16).  Populations are the oracle's own
array-of-structures ``f[node, set, dir]`` (pre-collision, time t).
"""
import ctypes
import os

import numpy as np

from . import build as _build

D2Q5 = 0
D3Q7 = 1
D2Q4 = 4
D3Q6 = 5
D2Q9 = 8
D3Q15 = 9
# a lattice per set: the velocity sets on D2Q9 / D3Q15, the set a = 0 on D2Q5 / D3Q7
D2Q9_Q5 = 12
D3Q15_Q7 = 13
_DQ = {D2Q5: (2, 5), D3Q7: (3, 7), D2Q4: (2, 4), D3Q6: (3, 6), D2Q9: (2, 9), D3Q15: (3, 15),
       D2Q9_Q5: (2, 9), D3Q15_Q7: (3, 15)}
PERIODIC = 0
WALL = 1
PLAIN = 0        # forcing of eq. 3-21
SCHEME2 = 1      # forcing of Scheme II, eq. 2-3c / 2-7a
BINARY16 = 2     # 16-bit deviation storage formats (orc_store16)
BFLOAT16 = 3
FORMATS = {"f16dev": BINARY16, "bf16dev": BFLOAT16}

_LIB = None


class OrcCase(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("s0", ctypes.c_double),
        ("s1", ctypes.c_double),
        ("s2", ctypes.c_double),
        ("bc", ctypes.c_int32 * 6),
        ("wall_u", (ctypes.c_double * 3) * 6),
        ("force", ctypes.c_double * 3),
        ("R", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("forcing", ctypes.c_int32),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        cp = ctypes.POINTER(OrcCase)
        L.orc_lattice_info.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), dp, dp, dp]
        L.orc_collision_matrix.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, dp]
        L.orc_init.argtypes = [cp, u8p, dp, dp, dp, dp, dp]
        L.orc_collide.argtypes = [cp, u8p, dp, dp, dp]
        L.orc_stream.argtypes = [cp, u8p, dp, dp]
        L.orc_fields.argtypes = [cp, u8p, dp, dp, dp]
        L.orc_num_fields.argtypes = [ctypes.c_int]
        L.orc_step.argtypes = [cp, u8p, dp, dp, dp]
        L.orc_run.argtypes = [cp, u8p, dp, dp, dp, ctypes.c_long]
        L.orc_invariants.argtypes = [cp, u8p, dp, dp, dp]
        L.orc_set0_lattice.argtypes = [ctypes.c_int]
        fp = ctypes.POINTER(ctypes.c_float)
        L.orc_round16.argtypes = [ctypes.c_int, fp, dp, ctypes.c_long]
        L.orc_store16.argtypes = [cp, u8p, ctypes.c_int, ctypes.c_double, dp]
        L.orc_run16.argtypes = [cp, u8p, dp, ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_long]
        for name in ("orc_lattice_info", "orc_collision_matrix", "orc_init", "orc_collide",
                     "orc_stream", "orc_fields", "orc_num_fields", "orc_step", "orc_run",
                     "orc_invariants", "orc_round16", "orc_store16", "orc_run16", "orc_set0_lattice"):
            getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _ok(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def lattice_info(lattice):
    d, q = ctypes.c_int(), ctypes.c_int()
    c = (ctypes.c_int * 45)()
    w = np.zeros(15)
    cs2 = np.zeros(1)
    M = np.zeros(225)
    _ok(lib().orc_lattice_info(lattice, ctypes.byref(d), ctypes.byref(q), c, _dp(w), _dp(cs2),
                               _dp(M)), "lattice_info")
    qn = q.value
    return {
        "d": d.value,
        "q": qn,
        "c": np.array(list(c)[: 3 * qn], dtype=np.int64).reshape(qn, 3)[:, : d.value],
        "w": w[:qn].copy(),
        "cs2": float(cs2[0]),
        "M": M[: qn * qn].reshape(qn, qn).copy(),
    }


def set0_lattice(lattice):
    """Lattice id of the set a = 0 (differs from `lattice` only for the ids
    with a lattice per set)."""
    r = lib().orc_set0_lattice(int(lattice))
    if r < 0:
        raise ValueError(f"unknown lattice {lattice}")
    return r


def collision_matrix(lattice, s0, s1, s2=0.0):
    q = lattice_info(lattice)["q"]
    out = np.zeros(q * q)
    _ok(lib().orc_collision_matrix(lattice, s0, s1, s2, _dp(out)), "collision_matrix")
    return out.reshape(q, q)


class Case:
    """One simulation case for the oracle (lattice units)."""

    def __init__(self, lattice, shape, s1, s0=1.0, s2=0.0, bc=None, wall_u=None, force=None,
                 R=0.0, rho0=1.0, forcing=0):
        self.lattice = lattice
        self.d, self.q = _DQ[lattice]
        shape = tuple(int(s) for s in shape)
        if self.d == 2:
            nx, ny = shape
            nz = 1
        else:
            nx, ny, nz = shape
        self.nx, self.ny, self.nz = nx, ny, nz
        self.N = nx * ny * nz
        self.s0, self.s1, self.s2 = float(s0), float(s1), float(s2)
        self.bc = list(bc) if bc is not None else [PERIODIC] * 6
        self.wall_u = np.zeros((6, 3)) if wall_u is None else np.asarray(wall_u, float).reshape(6, 3)
        self.force = np.zeros(3)
        if force is not None:
            self.force[: len(force)] = force
        self.R = float(R)
        self.rho0 = float(rho0)
        self.forcing = int(forcing)      # PLAIN: eq. 3-21; SCHEME2: eq. 2-3c / 2-7a

    @property
    def fshape(self):
        return (self.nz, self.ny, self.nx) if self.d == 3 else (self.ny, self.nx)

    def c_struct(self):
        s = OrcCase()
        s.lattice = self.lattice
        s.nx, s.ny, s.nz = self.nx, self.ny, self.nz
        s.s0, s.s1, s.s2 = self.s0, self.s1, self.s2
        for k in range(6):
            s.bc[k] = int(self.bc[k])
            for b in range(3):
                s.wall_u[k][b] = float(self.wall_u[k, b])
        for b in range(3):
            s.force[b] = float(self.force[b])
        s.R = self.R
        s.rho0 = self.rho0
        s.forcing = self.forcing
        return s


class Oracle:
    """FP64 reference solver for one case.  ``f`` is the pre-collision state."""

    def __init__(self, case, solid=None, force_field=None):
        self.case = case
        self._cs = case.c_struct()
        self.solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
        self.force_field = (None if force_field is None
                            else np.ascontiguousarray(force_field, dtype=np.float64).reshape(-1))
        if self.force_field is not None:
            assert self.force_field.size == case.d * case.N
        ns = case.d + 1
        self.f = np.zeros(case.N * ns * case.q)
        self._tmp = np.zeros_like(self.f)
        self.t = 0

    def init(self, P, u, grad=None):
        c = self.case
        P = np.ascontiguousarray(np.broadcast_to(np.asarray(P, float), c.fshape)).reshape(-1).copy()
        u = np.ascontiguousarray(np.asarray(u, float).reshape(c.d, -1))
        assert u.shape[1] == c.N
        g = None
        if grad is not None:
            g = np.ascontiguousarray(np.asarray(grad, float).reshape(c.d * c.d, -1))
        _ok(lib().orc_init(ctypes.byref(self._cs), _u8(self.solid), _dp(self.force_field), _dp(P), _dp(u), _dp(g),
                           _dp(self.f)), "init")
        self.t = 0
        return self

    def set_populations(self, f):
        """f given as [set][dir][node] (set-major), converted to the oracle's
        layout.  With a lattice per set, the set a = 0 uses the first q0
        directions (the rest must be zero)."""
        c = self.case
        f = np.asarray(f, float).reshape(c.d + 1, c.q, c.N)
        self.f[:] = np.ascontiguousarray(f.transpose(2, 0, 1)).reshape(-1)
        self.t = 0
        return self

    def populations(self):
        """Pre-collision f(., t) as [set][dir] + field shape."""
        c = self.case
        f = self.f.reshape(c.N, c.d + 1, c.q).transpose(1, 2, 0)
        return np.ascontiguousarray(f).reshape((c.d + 1, c.q) + c.fshape)

    def run(self, nsteps):
        _ok(lib().orc_run(ctypes.byref(self._cs), _u8(self.solid), _dp(self.force_field),
                          _dp(self.f), _dp(self._tmp), int(nsteps)), "run")
        self.t += int(nsteps)
        return self

    def run16(self, nsteps, fmt, u_ref):
        """nsteps steps with the post-collision populations stored through
        the 16-bit deviation format `fmt` (BINARY16 or BFLOAT16) with scale
        u_ref (orc_run16)."""
        _ok(lib().orc_run16(ctypes.byref(self._cs), _u8(self.solid), _dp(self.force_field), int(fmt),
                            float(u_ref), _dp(self.f), _dp(self._tmp), int(nsteps)), "run16")
        self.t += int(nsteps)
        return self

    def post16(self, fmt, u_ref):
        """Post-collision f*(., t) stored through the 16-bit deviation format
        `fmt` with scale u_ref (orc_collide, then orc_store16), as [set][dir] +
        field shape (state unchanged)."""
        c = self.case
        out = np.zeros_like(self.f)
        _ok(lib().orc_collide(ctypes.byref(self._cs), _u8(self.solid), _dp(self.force_field),
                              _dp(self.f), _dp(out)), "collide")
        _ok(lib().orc_store16(ctypes.byref(self._cs), _u8(self.solid), int(fmt), float(u_ref), _dp(out)),
            "store16")
        f = out.reshape(c.N, c.d + 1, c.q).transpose(1, 2, 0)
        return np.ascontiguousarray(f).reshape((c.d + 1, c.q) + c.fshape)

    def collide(self):
        """Post-collision f*(., t) as [set][dir] + field shape (state unchanged)."""
        c = self.case
        out = np.zeros_like(self.f)
        _ok(lib().orc_collide(ctypes.byref(self._cs), _u8(self.solid), _dp(self.force_field),
                              _dp(self.f), _dp(out)), "collide")
        f = out.reshape(c.N, c.d + 1, c.q).transpose(1, 2, 0)
        return np.ascontiguousarray(f).reshape((c.d + 1, c.q) + c.fshape)

    def fields(self):
        c = self.case
        nch = lib().orc_num_fields(c.lattice)
        out = np.zeros(nch * c.N)
        _ok(lib().orc_fields(ctypes.byref(self._cs), _u8(self.solid), _dp(self.force_field), _dp(self.f), _dp(out)),
            "fields")
        out = out.reshape((nch,) + c.fshape)
        d = c.d
        nsym = d * (d + 1) // 2
        k = 0
        res = {"ubar0": out[0]}
        res["u"] = out[1: d + 1]
        k = d + 1
        res["P"] = out[k]
        k += 1
        res["grad"] = out[k: k + d * d].reshape((d, d) + c.fshape)
        k += d * d
        res["div"] = out[k]
        k += 1
        res["S"] = out[k: k + nsym]
        k += nsym
        res["sigma"] = out[k: k + nsym]
        k += nsym
        res["vort"] = out[k] if d == 2 else out[k: k + 3]
        return res

    def invariants(self):
        c = self.case
        out = np.zeros(c.d + 2)
        _ok(lib().orc_invariants(ctypes.byref(self._cs), _u8(self.solid), _dp(self.force_field), _dp(self.f), _dp(out)),
            "invariants")
        return out


def round16(fmt, x):
    """The 16-bit value (BINARY16 or BFLOAT16) nearest to each binary32 value
    of x, ties to even, as float64 (orc_round16)."""
    a = np.ascontiguousarray(np.asarray(x, np.float32).reshape(-1))
    out = np.zeros(a.size)
    _ok(lib().orc_round16(int(fmt), a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _dp(out), a.size),
        "round16")
    return out.reshape(np.shape(x))


def residual(u_now, u_prev, K):
    """Steady-state residual over K steps, |u^n - u^{n-K}|_2 / (K |u^n|_2), with
    the sums taken in FP64 over every component and node."""
    a = np.asarray(u_now, np.float64)
    b = np.asarray(u_prev, np.float64)
    num = np.sqrt(np.sum((a - b) ** 2))
    den = np.sqrt(np.sum(a ** 2))
    return float(num / (K * den)) if den > 0 else float("inf")
