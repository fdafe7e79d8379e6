"""Forces on the HIP path: per-node force fields (eq. 2-6 with a
space-dependent F) through mdf_set_force_field, and the Scheme II forcing of
eq. 2-3c / 2-7a.  Parity with the FP64 oracle at fixed step counts, the
four-roll mill of Section 4.2 (Table 1) solved on the GPU, and the exact
Poiseuille profile of Scheme II.

A force field set on a context enters every later collision; the state
already held by the context (the collision done by mdf_init) keeps the force
it was collided with.  The oracle reproduces that by taking the first step
without the field and the rest with it.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2108_08591_amd import cases as C
from paper_2108_08591_amd import mdf
import analytic as A
from helpers import compare_fields, gpu_fields_np, oracle_for, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f64": 1e-12, "f32": 1e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cast(a, storage):
    a = np.asarray(a, np.float64)
    return a if storage == "f64" else a.astype(np.float32).astype(np.float64)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _oracle_run(spec, solid, FF, nsteps):
    """nsteps steps from rest: the first collision without the field (as
    mdf_init does it), the remaining ones with it."""
    o0 = oracle_for(spec, solid=solid).init(0.0, np.zeros((spec.d,) + spec.fshape))
    o0.run(1)
    o = oracle_for(spec, solid=solid, force_field=FF).set_populations(o0.populations())
    o.run(nsteps - 1)
    return o


def _force(spec, seed, amp=2e-4):
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(spec.d,) + spec.fshape)


def _walled_2d():
    wall = np.zeros((6, 3))
    wall[3] = (0.05, 0.0, 0.0)
    spec = C.CaseSpec(C.D2Q5, (70, 45), 0.83, bc=(C.PERIODIC, C.PERIODIC, C.WALL, C.WALL, 0, 0),
                      wall_u=wall, force=(3e-5, -1e-5))
    mask = np.zeros((45, 70), np.uint8)
    mask[18:26, 30:41] = 1
    return spec, mask


@pytest.mark.parametrize("form", [0, 2])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_force_field_parity_2d(storage, form):
    """Ragged 70 x 45 channel with a moving wall, an obstacle, a uniform force
    and a random per-node force on top; one and two steps per launch."""
    spec, mask = _walled_2d()
    FF = _cast(_force(spec, 11), storage)
    _say(f"[force] 2d 70x45 {storage} form {form}")
    s = mdf.Solver([spec], storage=storage, solid=[mask], device=DEV)
    s.set_launch(64, 4, 8, form)
    s.set_force_field(FF)
    s.step(57)
    o = _oracle_run(spec, mask, FF, 57)
    assert rel_err(o.populations(), _np(s.populations())) < TOL[storage]
    compare_fields(o.fields(), gpu_fields_np(s, mdf.FIELD_ALL), TOL[storage])


def test_force_field_parity_3d_and_removal():
    """D3Q7 box (periodic x, walls elsewhere, ragged) in FP64; then the field
    is removed and the next steps match the oracle without it."""
    spec = C.CaseSpec(C.D3Q7, (21, 14, 11), 1.1, bc=(C.PERIODIC, C.PERIODIC, C.WALL, C.WALL, C.WALL, C.WALL),
                      force=(1e-5, 0.0, 2e-5))
    FF = _force(spec, 5)
    _say("[force] 3d 21x14x11 f64")
    s = mdf.Solver([spec], storage="f64", device=DEV)
    s.set_force_field(FF)
    s.step(33)
    o = _oracle_run(spec, None, FF, 33)
    assert rel_err(o.populations(), _np(s.populations())) < 1e-12
    compare_fields(o.fields(), gpu_fields_np(s, mdf.FIELD_ALL), 1e-12)
    # the state at t = 33 was already collided with the field: the oracle
    # takes that collision with it, the next eight without
    s.set_force_field(None)
    s.step(9)
    o.run(1)
    o2 = oracle_for(spec).set_populations(o.populations())
    o2.run(8)
    assert rel_err(o2.populations(), _np(s.populations())) < 1e-12


def test_force_field_per_case_in_a_batch():
    """Three cases in one context (batched launch): a field on cases 0 and 2
    only; each case matches its own oracle."""
    specs = [C.CaseSpec(C.D2Q5, (40, 33), 1.2, force=(2e-5, 0.0)),
             C.CaseSpec(C.D2Q5, (65, 20), 0.9, bc=(C.PERIODIC, C.PERIODIC, C.WALL, C.WALL, 0, 0)),
             C.CaseSpec(C.D2Q5, (31, 47), 1.5)]
    fields = [_force(specs[0], 1), None, _force(specs[2], 2)]
    _say("[force] batch of 3, f64")
    s = mdf.Solver(specs, storage="f64", device=DEV)
    for k, FF in enumerate(fields):
        if FF is not None:
            s.set_force_field(FF, case=k)
    s.step(25)
    for k, (spec, FF) in enumerate(zip(specs, fields)):
        o = _oracle_run(spec, None, FF, 25)
        assert rel_err(o.populations(), _np(s.populations(k))) < 1e-12, k


def test_force_field_rejects_wrong_size():
    spec, mask = _walled_2d()
    s = mdf.Solver([spec], storage="f32", solid=[mask], device=DEV)
    with pytest.raises(ValueError):
        s.set_force_field(np.zeros((2, 10, 10)))


def _table_1():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    return g["four_roll_mill_table_1"]


@pytest.mark.parametrize("k", [0, 1, 2])
def test_four_roll_mill_table_1_on_gpu(k):
    """Section 4.2, Table 1 on the GPU path: the 64 x 64 four-roll mill at
    s1 = 0.7, 1.2, 1.7 solved to steady state in FP64; the five printed
    relative errors (u1, u2, S_xx, S_yy, vorticity) matched to 1e-4 relative."""
    g = _table_1()
    s1 = g["s1"][k]
    spec, FF, dt, dx = C.four_roll_mill(64, s1)
    _say(f"[force] four-roll mill 64^2 s1={s1} f64")
    s = mdf.Solver([spec], storage="f64", device=DEV)
    s.set_force_field(FF)
    st, steps, res = s.run_steady(1e-12, 100, 400000)
    assert st[0] == 0 and res[0] < 1e-12, (st, steps, res)
    fl = gpu_fields_np(s, mdf.FIELD_ALL)
    ex = A.four_roll_mill(64, 1e-4)
    ul = dt / dx
    got = {
        "E_u1": A.rel_l2(ex["u1"] * ul, fl["u"][0]),
        "E_u2": A.rel_l2(ex["u2"] * ul, fl["u"][1]),
        "E_Sxx": A.rel_l2(ex["Sxx"] * dt, fl["S"][0]),
        "E_Syy": A.rel_l2(ex["Syy"] * dt, fl["S"][2]),
        "E_vort": A.rel_l2(ex["vort"] * dt, fl["vort"]),
    }
    for key, val in got.items():
        assert abs(val / g[key][k] - 1) < 1e-4, (key, val, g[key][k])


# ---------------------------------------------------------------- Scheme II

@pytest.mark.parametrize("form", [0, 2])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_scheme2_parity_2d(storage, form):
    """Scheme II on the walled 2D case with an obstacle, a uniform force, a
    mass source and a per-node force field."""
    spec, mask = _walled_2d()
    spec.forcing = C.SCHEME2
    spec.R = 1e-4
    FF = _cast(_force(spec, 12), storage)
    _say(f"[scheme2] 2d 70x45 {storage} form {form}")
    s = mdf.Solver([spec], storage=storage, solid=[mask], device=DEV)
    s.set_launch(64, 4, 8, form)
    s.set_force_field(FF)
    s.step(57)
    o = _oracle_run(spec, mask, FF, 57)
    assert rel_err(o.populations(), _np(s.populations())) < TOL[storage]
    compare_fields(o.fields(), gpu_fields_np(s, mdf.FIELD_ALL), TOL[storage])
    inv = s.invariants()
    ref = o.invariants()
    assert np.allclose(inv, ref, rtol=TOL[storage], atol=TOL[storage] * np.abs(ref).max())


def test_scheme2_parity_3d():
    spec = C.CaseSpec(C.D3Q7, (21, 14, 11), 1.1, bc=(C.PERIODIC, C.PERIODIC, C.WALL, C.WALL, C.WALL, C.WALL),
                      force=(1e-5, 0.0, 2e-5), R=5e-5, forcing=C.SCHEME2)
    FF = _force(spec, 6)
    _say("[scheme2] 3d 21x14x11 f64")
    s = mdf.Solver([spec], storage="f64", device=DEV)
    s.set_force_field(FF)
    s.step(33)
    o = _oracle_run(spec, None, FF, 33)
    assert rel_err(o.populations(), _np(s.populations())) < 1e-12
    compare_fields(o.fields(), gpu_fields_np(s, mdf.FIELD_ALL), 1e-12)


def test_scheme2_and_plain_cases_in_one_batch():
    """One batched context holding both forcing schemes; each case matches
    its own oracle."""
    specs = [C.CaseSpec(C.D2Q5, (40, 33), 1.2, force=(2e-5, 1e-5), forcing=C.SCHEME2),
             C.CaseSpec(C.D2Q5, (65, 20), 0.9, bc=(C.PERIODIC, C.PERIODIC, C.WALL, C.WALL, 0, 0),
                        force=(3e-5, 0.0)),
             C.CaseSpec(C.D2Q5, (31, 47), 1.5, force=(0.0, -2e-5), R=1e-4, forcing=C.SCHEME2)]
    _say("[scheme2] batch of 3, f64")
    s = mdf.Solver(specs, storage="f64", device=DEV)
    s.step(25)
    for k, spec in enumerate(specs):
        o = _oracle_run(spec, None, None, 25)
        assert rel_err(o.populations(), _np(s.populations(k))) < 1e-12, k


def test_scheme2_velocity_sets_equal_full_form():
    """Scheme II with only the d velocity sets (Remark IV) agrees bit for bit
    with all d + 1 sets (the source R of the set a = 0 reaches nothing), and
    with the oracle's sets a = 1..d within the FP32 bar."""
    spec, mask = _walled_2d()
    spec.forcing = C.SCHEME2
    spec.R = 1e-4
    _say("[scheme2] velocity sets vs full, f32")
    full = mdf.Solver([spec], storage="f32", solid=[mask], device=DEV)
    vel = mdf.Solver([spec], storage="f32", solid=[mask], device=DEV, sets="velocity")
    FF = _force(spec, 13)
    for x in (full, vel):
        x.set_force_field(FF)
        x.step(41)
    assert torch.equal(full.populations()[1:], vel.populations())
    assert torch.equal(full.gradients(mdf.FIELD_ALL)[1:], vel.gradients(mdf.FIELD_ALL)[1:])
    # and against the oracle's velocity sets a = 1..d with the same field
    o = _oracle_run(spec, mask, _cast(FF, "f32"), 41)
    fluid = mask == 0
    assert rel_err(o.populations()[1:][..., fluid], _np(vel.populations())[..., fluid]) < TOL["f32"]
    compare_fields(o.fields(), gpu_fields_np(vel, mdf.FIELD_ALL), TOL["f32"],
                   keys=("u", "P", "grad", "div", "S", "sigma", "vort"))


def test_scheme2_poiseuille_exact_on_gpu():
    """Section 4.1 geometry under Scheme II on the GPU in FP64: the steady
    profile is the parabola to the rounding floor (eq. 3-21 leaves Fbar/2)."""
    spec = C.poiseuille_paper_case()
    spec.forcing = C.SCHEME2
    _say("[scheme2] poiseuille 32x32 f64")
    s = mdf.Solver([spec], storage="f64", device=DEV)
    st, steps, res = s.run_steady(1e-15, 1000, 200000)
    assert st[0] == 0, (st, steps, res)
    got = gpu_fields_np(s, mdf.FIELD_ALL)
    F, H = spec.force[0], 32
    nu = (1 / spec.s1 - 0.5) / 3
    y = (np.arange(H) + 0.5)[:, None] * np.ones((1, 32))
    ex = A.poiseuille(F, nu, H, y)
    assert A.rel_l2(ex["u1"], got["u"][0]) < 1e-10
    assert A.rel_l2(ex["du1dy"], got["grad"][0, 1]) < 1e-12


@pytest.mark.parametrize("k", [0, 1, 2])
def test_scheme2_four_roll_mill_on_gpu(k):
    """Table 1 under Scheme II on the GPU in FP64: E(u1) equals the printed
    E(u1) minus nu_lat (k dx)^2, the part a Fbar/2 offset contributes under
    eq. 3-21, to the table's 5 digits."""
    g = _table_1()
    s1 = g["s1"][k]
    spec, FF, dt, dx = C.four_roll_mill(64, s1)
    spec.forcing = C.SCHEME2
    _say(f"[scheme2] four-roll mill 64^2 s1={s1} f64")
    s = mdf.Solver([spec], storage="f64", device=DEV)
    s.set_force_field(FF)
    st, steps, res = s.run_steady(1e-12, 100, 400000)
    assert st[0] == 0 and res[0] < 1e-12, (st, steps, res)
    fl = gpu_fields_np(s, mdf.FIELD_ALL)
    ex = A.four_roll_mill(64, 1e-4)
    e1 = A.rel_l2(ex["u1"] * dt / dx, fl["u"][0])
    nu_lat = (1 / s1 - 0.5) / 3
    assert abs(e1 / (g["E_u1"][k] - nu_lat * (2 * np.pi / 64) ** 2) - 1) < 1e-4, e1
