"""Checkpoint and resume through mdf_save / mdf_load: a run interrupted,
saved, and continued in a new context gives the populations, fields and
residuals of the uninterrupted run bit for bit, in single-case contexts (two
steps per launch) and batched ones, through device or host memory."""
import os
import sys
import tempfile

import numpy as np
import pytest
import torch

from paper_2108_08591_amd import cases as C
from paper_2108_08591_amd import mdf

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cavity():
    spec = C.cavity_case(N=96, Re=200.0, U=0.1)
    spec.shape = (98, 71)
    return spec


@pytest.mark.parametrize("storage", ["f32", "f64", "f16dev"])
def test_resume_equals_uninterrupted_run(storage):
    spec = _cavity()
    _say(f"[checkpoint] single case {storage}")
    a = mdf.Solver([spec], storage=storage, device=DEV, u_ref=0.1)
    a.step(37)
    a.check()                                   # residual snapshot at t = 37
    blob = a.save()
    fields_at_save = a.gradients(mdf.FIELD_ALL).clone()
    a.step(25)
    res_a = a.check()[0]
    b = mdf.Solver([spec], storage=storage, device=DEV, u_ref=0.1)
    b.step(3)                                   # a different state, overwritten by the load
    b.load(blob)
    assert torch.equal(b.gradients(mdf.FIELD_ALL), fields_at_save)
    b.step(25)
    assert torch.equal(b.populations(), a.populations())
    assert torch.equal(b.gradients(mdf.FIELD_ALL), a.gradients(mdf.FIELD_ALL))
    assert b.check()[0][0] == res_a[0]
    assert lib_time(b) == lib_time(a) == 62


def lib_time(s):
    return mdf.lib().mdf_time(s._ctx, 0)


def test_resume_batched_through_a_file():
    """Three uneven cases (one with an obstacle) in a batched context; the
    state goes through pinned host memory and a file, and the resumed steady
    solve stops at the same step with the same residual."""
    specs = [C.cavity_case(N=64, Re=100.0), C.poiseuille_case(nx=80, ny=24),
             C.CaseSpec(C.D2Q5, (45, 37), 1.3, force=(1e-5, 0.0))]
    mask = np.zeros((37, 45), np.uint8)
    mask[10:15, 20:26] = 1
    masks = [None, None, mask]
    _say("[checkpoint] batch of 3 through a file")
    a = mdf.Solver(specs, storage="f64", solid=masks, device=DEV)
    a.step(150)
    blob = a.save(device="cpu")
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "state.pt")
        torch.save(blob, path)
        back = torch.load(path, weights_only=True)
    st_a, steps_a, res_a = a.run_steady(1e-9, 100, 200000)
    b = mdf.Solver(specs, storage="f64", solid=masks, device=DEV)
    b.load(back)
    st_b, steps_b, res_b = b.run_steady(1e-9, 100, 200000)
    assert np.array_equal(st_a, st_b) and np.array_equal(steps_a, steps_b)
    assert np.array_equal(res_a, res_b)
    for k in range(3):
        assert torch.equal(a.populations(k), b.populations(k)), k


def test_load_rejects_a_different_context():
    spec = _cavity()
    a = mdf.Solver([spec], storage="f32", device=DEV)
    a.step(5)
    blob = a.save()
    other = C.cavity_case(N=96, Re=200.0)          # 96 x 96, not 98 x 71
    b = mdf.Solver([other], storage="f32", device=DEV)
    with pytest.raises(mdf.MdfError):
        b.load(blob)
    c = mdf.Solver([spec], storage="f64", device=DEV)
    with pytest.raises(mdf.MdfError):
        c.load(blob)
    d = mdf.Solver([spec], storage="f32", device=DEV)
    with pytest.raises(mdf.MdfError):
        d.load(blob[:-16])
    bad = blob.clone()
    bad[0] = 0
    with pytest.raises(mdf.MdfError):
        d.load(bad)
    d.load(blob)                                     # the context is still usable
    d.step(2)
    a.step(2)
    assert torch.equal(d.populations(), a.populations())
