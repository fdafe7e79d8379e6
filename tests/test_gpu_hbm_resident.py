"""Parity on contexts whose population buffers exceed the 256 MB Infinity
Cache, where the step kernels store populations with a non-temporal hint and
address nodes by 32-bit byte offsets: the 2D cavity in FP32 and FP64
(two-step and one-step launches) and the 3D Taylor-Green vortex at its full
256^3 size in FP32.  After some steps from
the GPU's own run, one and then two or three more steps are checked node by
node against the FP64 oracle on sampled patches (corners, walls, periodic
faces, interior); the oracle starts from the GPU's state on each patch
widened by the dependence radius."""
import sys

import numpy as np
import pytest
import torch

from paper_2108_08591_amd import cases as C
from paper_2108_08591_amd import mdf
from helpers import oracle_for, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f64": 1e-12, "f32": 1e-5}
CACHE_BYTES = 256 << 20


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _pop_bytes(solver, spec):
    nbytes = solver.dtype.itemsize
    return 2 * solver.nsets * solver.q * int(np.prod(spec.shape)) * nbytes


def _cavity_patch_oracle(spec, f_t, x0, y0, P, h):
    """Oracle on the P x P patch at (x0, y0) widened by h on every side that
    is not a wall; a widened side that is not a wall is made periodic (its
    halo values are wrong but reach only h - 1 nodes inward in h steps)."""
    NX, NY = spec.shape
    ex0, ex1 = max(x0 - h, 0), min(x0 + P + h, NX)
    ey0, ey1 = max(y0 - h, 0), min(y0 + P + h, NY)
    bc = [C.WALL if ex0 == 0 else C.PERIODIC, C.WALL if ex1 == NX else C.PERIODIC,
          C.WALL if ey0 == 0 else C.PERIODIC, C.WALL if ey1 == NY else C.PERIODIC, 0, 0]
    for ax in range(2):                      # periodic faces come in pairs
        if bc[2 * ax] != bc[2 * ax + 1]:
            bc[2 * ax] = bc[2 * ax + 1] = C.WALL
    sub = C.CaseSpec(C.D2Q5, (ex1 - ex0, ey1 - ey0), spec.s1, bc=tuple(bc), wall_u=spec.wall_velocity().copy())
    o = oracle_for(sub).set_populations(_np(f_t[:, :, ey0:ey1, ex0:ex1]))
    return o, (slice(y0 - ey0, y0 - ey0 + P), slice(x0 - ex0, x0 - ex0 + P))


@pytest.mark.parametrize("storage,N,form", [("f32", 1600, 2), ("f32", 1600, 0), ("f64", 1200, 2),
                                            ("f64", 1200, 0)])
def test_cavity_beyond_the_cache(storage, N, form):
    spec = C.cavity_case(N=N, Re=1000.0)
    _say(f"[hbm-resident] cavity {N}^2 {storage} form {form}")
    s = mdf.Solver([spec], storage=storage, device=DEV)
    assert _pop_bytes(s, spec) > CACHE_BYTES
    s.set_launch(128, 2, 8, form)
    s.step(200)
    P = 16
    patches = [(0, 0), (N - P, 0), (0, N - P), (N - P, N - P), (N // 2, N - P), (0, N // 3), (N - P, N // 2),
               (N // 4, 0), (N // 2, N // 2), (137, 251)]
    for nsteps in (1, 3):
        f_t = s.populations()
        s.step(nsteps)
        f_t1 = s.populations()
        fl = s.fields(mdf.FIELD_ALL)
        big = {k: float(v.abs().max()) for k, v in fl.items() if k in ("u", "vort", "S", "P")}
        for (x0, y0) in patches:
            o, (iy, ix) = _cavity_patch_oracle(spec, f_t, x0, y0, P, nsteps)
            o.run(nsteps)
            got = _np(f_t1[:, :, y0:y0 + P, x0:x0 + P])
            assert rel_err(o.populations()[:, :, iy, ix], got) < TOL[storage], (nsteps, x0, y0)
            fo = o.fields()
            for key in big:
                ref = fo[key][..., iy, ix]
                g = _np(fl[key][..., y0:y0 + P, x0:x0 + P])
                assert np.abs(ref - g).max() <= TOL[storage] * big[key], (nsteps, key, x0, y0)
        del f_t, f_t1, fl


@pytest.mark.parametrize("storage,form", [("f32", 0), ("f32", 2), ("f64", 2)])
def test_tgv3d_full_size_beyond_the_cache(storage, form):
    """3D Taylor-Green at 256^3 (3.8 GB of populations in FP32, 7.5 GB in
    FP64), one node per thread (form 0) and two steps per launch with tiles
    walking z-planes (form 2): patches of 8^3 nodes, some wrapping across the
    periodic faces, after one step and after three more (one two-step launch
    and one one-step launch)."""
    N = 256
    spec = C.tgv3d_case(N=N, u0=0.05, Re=100.0)
    _say(f"[hbm-resident] tgv3d 256^3 {storage} form {form}")
    Pf, u = C.taylor_green_3d_initial(N, 0.05)
    dt = np.float64 if storage == "f64" else np.float32
    init = torch.tensor(np.concatenate([Pf[None], u]).astype(dt))
    del Pf, u
    s = mdf.Solver([spec], storage=storage, init=("fields", [init]), device=DEV)
    del init
    assert _pop_bytes(s, spec) > CACHE_BYTES
    s.set_launch(64, 4, 8, form)
    s.step(20)
    P = 8
    corners = [(0, 0, 0), (N - 4, 3, 250), (128, 128, 128), (17, 200, N - 8), (N - 8, N - 8, N - 8), (60, 0, 99),
               (31, 7, 31), (32, 8, 32)]
    for nsteps in (1, 3):
        f_t = s.populations()
        s.step(nsteps)
        f_t1 = s.populations()
        h = nsteps
        for (x0, y0, z0) in corners:
            ext = [torch.arange(a - h, a + P + h, device=DEV) % N for a in (z0, y0, x0)]
            inn = [torch.arange(a, a + P, device=DEV) % N for a in (z0, y0, x0)]
            sub_in = f_t.index_select(2, ext[0]).index_select(3, ext[1]).index_select(4, ext[2])
            sub = C.CaseSpec(C.D3Q7, (P + 2 * h,) * 3, spec.s1)
            o = oracle_for(sub).set_populations(_np(sub_in))
            o.run(nsteps)
            ref = o.populations()[:, :, h:h + P, h:h + P, h:h + P]
            got = _np(f_t1.index_select(2, inn[0]).index_select(3, inn[1]).index_select(4, inn[2]))
            assert rel_err(ref, got) < TOL[storage], (nsteps, x0, y0, z0)
        del f_t, f_t1

