"""Failure paths of the HIP path, forced from the host: non-finite initial
fields, one poisoned case in a batch, NaN-filled ping-pong buffers, and
whether batched chunks ran as captured HIP graphs.

None of these makes a kernel fault or hang: a NaN is an ordinary value to
the kernels, and the residual check (FP64 sums with a non-finite count)
turns it into MDF_EUNSTABLE on the host.
"""
import sys

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


def _fields(spec, seed, dtype, nan_at=None):
    P, u = C.smooth_random_fields(spec, seed=seed, amp=0.02)
    arr = np.concatenate([np.asarray(P)[None], np.asarray(u)], axis=0).astype(np.float64)
    if nan_at is not None:
        arr[(1,) + tuple(nan_at)] = np.nan
    return torch.tensor(arr, dtype=dtype)


def _dtype(storage):
    return torch.float64 if storage == "f64" else torch.float32


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
def test_nan_initial_field_is_reported_unstable(storage):
    """A NaN in the initial velocity: mdf_check returns MDF_EUNSTABLE with
    status 1, and so does mdf_run_steady (case status 1)."""
    spec = C.cavity_case(N=48, Re=100.0)
    _say(f"[failure] NaN init field {storage}")
    s = mdf.Solver([spec], storage=storage, init=("fields", [_fields(spec, 3, _dtype(storage), (20, 17))]),
                   device=DEV, u_ref=0.05)
    st = mdf.lib().mdf_check(s._ctx, None, None, mdf._stream_ptr(None))
    assert st == mdf.EUNSTABLE
    res, status = s.check()
    assert status[0] == 1
    status, steps, res = s.run_steady(1e-8, 10, 200)
    assert status[0] == 1
    assert steps[0] <= 10


def test_bad_rate_is_rejected_before_launch():
    """s1 outside (0, 2) is refused on the host (MDF_EINVAL), nothing runs."""
    spec = C.cavity_case(N=32, Re=100.0)
    spec.s1 = 2.0
    with pytest.raises(mdf.MdfError) as e:
        mdf.Solver([spec], storage="f32", device=DEV)
    assert e.value.status == mdf.EINVAL


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_poisoned_case_leaves_the_batch_unchanged(storage):
    """One case of a batched context starts with a NaN: it is reported
    non-finite (status 1) while every other case advances bitwise as its
    own single-case run, through plain steps and a steady solve."""
    specs = [C.cavity_case(N=64, Re=100.0),
             C.CaseSpec(C.D2Q5, (70, 45), 1.1, bc=(C.PERIODIC, C.PERIODIC, C.WALL, C.WALL, 0, 0),
                        force=(2e-5, 0.0)),
             C.cavity_case(N=96, Re=300.0)]
    inits = [_fields(sp, 10 + k, _dtype(storage)) for k, sp in enumerate(specs)]
    bad = 1
    inits[bad] = _fields(specs[bad], 10 + bad, _dtype(storage), (7, 30))
    _say(f"[failure] poisoned case in a batch of 3 {storage}")
    stream = torch.cuda.Stream()
    batch = mdf.Solver(specs, storage=storage, init=("fields", inits), device=DEV, stream=stream)
    singles = [mdf.Solver([sp], storage=storage, init=("fields", [inits[k]]), device=DEV)
               for k, sp in enumerate(specs)]
    batch.step(37)
    for s in singles:
        s.step(37)
    torch.cuda.synchronize()
    for k in range(3):
        if k == bad:
            assert not torch.isfinite(batch.populations(k)).all()
            continue
        assert torch.equal(batch.populations(k), singles[k].populations())
    status, steps, res = batch.run_steady(1e-300, 20, 60)
    for s in singles:
        s.run_steady(1e-300, 20, 60)
    torch.cuda.synchronize()
    assert status[bad] == 1
    for k in range(3):
        if k != bad:
            assert status[k] == 2 and steps[k] == 60
            assert torch.equal(batch.populations(k), singles[k].populations())


@pytest.mark.parametrize("form", [0, 2])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "bf16dev"])
def test_nan_poisoned_write_buffer_is_never_read(storage, form):
    """Before every call the buffer the next step overwrites is filled with
    NaN bytes: the populations, fields and residual stay finite and equal
    bit for bit to an unpoisoned twin (no kernel reads memory it has not
    written first), for calls of every length, in 2D and 3D, one and two
    steps per launch."""
    cav = C.cavity_case(N=70, Re=100.0)
    cav.shape = (70, 37)
    box = C.CaseSpec(C.D3Q7, (26, 14, 11), 1.2, bc=(C.PERIODIC, C.PERIODIC, C.WALL, C.WALL, C.WALL, C.WALL),
                     wall_u=((0, 0, 0), (0, 0, 0), (0, 0, 0), (0.04, 0, 0), (0, 0, 0), (0, 0, 0)))
    for spec in (cav, box):
        _say(f"[failure] NaN-poisoned write buffer {storage} form {form} d={spec.d}")
        runs = []
        for poison in (False, True):
            s = mdf.Solver([spec], storage=storage, device=DEV, u_ref=0.05)
            s.set_launch(64, 4, 8, form)
            rec = []
            for n in (1, 2, 3, 5, 8):
                if poison:
                    s.population_buffer(1).fill_(255)     # NaN in every storage format
                s.step(n)
                rec.append((s.populations(), s.gradients(mdf.FIELD_ALL)))
            # (mdf_run_steady starts with a read of buffer 1 unless the
            # residual snapshot is current, so it is not poisoned here)
            st, steps, res = s.run_steady(1e-300, 7, 21)
            rec.append((s.populations(), float(res[0])))
            runs.append(rec)
        for a, b in zip(runs[0], runs[1]):
            assert torch.isfinite(b[0]).all()
            assert torch.equal(a[0], b[0])
            if isinstance(a[1], torch.Tensor):
                assert torch.equal(a[1], b[1])
            else:
                assert np.isfinite(b[1]) and a[1] == b[1]


def test_batched_chunks_run_as_captured_graphs():
    """A batched context on a side stream captures each K-step chunk once as
    a HIP graph and replays it; on the null stream it launches plainly.
    Both give the same populations."""
    specs = [C.cavity_case(N=64, Re=100.0), C.cavity_case(N=96, Re=200.0)]
    _say("[failure] graph capture of batched chunks")
    stream = torch.cuda.Stream()
    g = mdf.Solver(specs, storage="f32", device=DEV, stream=stream)
    for _ in range(3):
        g.step(10)
    stream.synchronize()
    st = g.graph_stats()
    assert st["failed"] == 0, st
    assert st["captured"] == 1 and st["replayed"] == 3, st
    p = mdf.Solver(specs, storage="f32", device=DEV)
    for _ in range(3):
        p.step(10)
    torch.cuda.synchronize()
    sp = p.graph_stats()
    assert sp["captured"] == 0 and sp["plain"] == 3, sp
    for k in range(2):
        assert torch.equal(g.populations(k), p.populations(k))
    # a steady solve on the side stream replays its chunk graphs too
    g.run_steady(1e-300, 10, 40)
    stream.synchronize()
    st2 = g.graph_stats()
    assert st2["captured"] >= 2 and st2["replayed"] >= 3 + 4 and st2["failed"] == 0, st2
