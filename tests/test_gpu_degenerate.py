"""Degenerate grids against the FP64 oracle: one-node-wide rows and columns
(periodic, where a node pulls from itself, or between walls), a single
node, a 2 x 2 walled box with a moving lid and thin 3D boxes, in every launch
form (one node per thread, vector, two steps per launch); the 16-bit
storages give the same codes in every form; calls of zero steps leave the
state untouched."""
import sys

import numpy as np
import pytest
import torch

from paper_2108_08591_amd import cases as C
from paper_2108_08591_amd import mdf
from helpers import compare_fields, gpu_fields_np, oracle_for, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
P_, W_ = C.PERIODIC, C.WALL


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _lid(face, ux, uy=0.0):
    w = np.zeros((6, 3))
    w[face] = (ux, uy, 0.0)
    return w


def _cases():
    return [
        ("column 1x9, walls in y", C.CaseSpec(C.D2Q5, (1, 9), 1.2, bc=(P_, P_, W_, W_, P_, P_),
                                              wall_u=_lid(3, 0.05), force=(1e-5, 0.0, 0.0))),
        ("row 9x1, periodic", C.CaseSpec(C.D2Q5, (9, 1), 1.1, force=(0.0, 2e-5, 0.0))),
        ("row 13x1 between walls", C.CaseSpec(C.D2Q5, (13, 1), 0.9, bc=(P_, P_, W_, W_, P_, P_),
                                               wall_u=_lid(3, 0.04))),
        ("single node", C.CaseSpec(C.D2Q5, (1, 1), 1.3)),
        ("2x2 walled box, lid", C.CaseSpec(C.D2Q5, (2, 2), 1.4, bc=(W_, W_, W_, W_, P_, P_),
                                           wall_u=_lid(3, 0.08))),
        ("3D column 1x1x7, walls in z", C.CaseSpec(C.D3Q7, (1, 1, 7), 1.2, bc=(P_, P_, P_, P_, W_, W_),
                                                   wall_u=_lid(5, 0.03, 0.02))),
        ("3D slab 3x1x2", C.CaseSpec(C.D3Q7, (3, 1, 2), 1.1, force=(1e-5, 0.0, -1e-5))),
    ]


def _init(spec, storage):
    P, u = C.smooth_random_fields(spec, seed=3, amp=0.02)
    arr = np.concatenate([np.asarray(P)[None], np.asarray(u)], axis=0)
    if storage != "f64":
        arr = arr.astype(np.float32)
    return P, u, ("fields", [torch.tensor(arr)])


@pytest.mark.parametrize("form", [0, 1, 2])
def test_degenerate_grids_match_oracle(form):
    for name, spec in _cases():
        _say(f"[gpu] degenerate {name} form {form}")
        P, u, init = _init(spec, "f64")
        s = mdf.Solver([spec], storage="f64", init=init, device=DEV)
        s.set_launch(64, 4, 8, form)
        o = oracle_for(spec).init(P, u)
        for nsteps in (1, 4):
            s.step(nsteps)
            o.run(nsteps)
            ref = o.populations()
            got = s.populations().detach().cpu().numpy()
            assert rel_err(ref, got) < 1e-12, (name, nsteps)
            compare_fields(o.fields(), gpu_fields_np(s, mdf.FIELD_ALL), 1e-12)


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_degenerate_grids_16bit_forms_agree(storage):
    for name, spec in _cases():
        states = []
        for form in (0, 1, 2):
            _say(f"[gpu] degenerate {name} {storage} form {form}")
            _, _, init = _init(spec, storage)
            s = mdf.Solver([spec], storage=storage, init=init, device=DEV, u_ref=0.05)
            s.set_launch(64, 4, 8, form)
            s.step(5)
            states.append((s.populations(), s.gradients(mdf.FIELD_ALL)))
        for pops, flds in states[1:]:
            assert torch.equal(pops, states[0][0]), name
            assert torch.equal(flds, states[0][1]), name


def test_zero_steps_leave_the_state_untouched():
    spec = C.cavity_case(N=40, Re=100.0)
    s = mdf.Solver([spec], storage="f32", device=DEV)
    s.step(3)
    before = s.populations()
    out = [torch.full((mdf.n_channels(2, mdf.FIELD_VORT),) + spec.fshape, 7.0, device=DEV)]
    s.step(0)
    s.step_emit(0, mdf.FIELD_VORT, out)
    assert s.time() == 3
    assert torch.equal(s.populations(), before)
    assert bool((out[0] == 7.0).all())
