"""Batched contexts (several uneven cases per persistent launch) against the
single-case path (bitwise) and the FP64 oracle (seeded subset)."""
import sys

import numpy as np
import pytest
import torch

from paper_2108_08591_amd import cases as C
from paper_2108_08591_amd import mdf
from helpers import compare_fields, gpu_fields_np, oracle_for

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed_cases():
    specs = []
    specs.append(C.cavity_case(N=96, Re=200.0, U=0.08))
    ch = C.poiseuille_case(70, 45, umax=0.05, s1=1.3)
    specs.append(ch)
    cav = C.cavity_case(N=64, Re=50.0, U=0.1)
    cav.shape = (77, 51)
    specs.append(cav)
    specs.append(C.CaseSpec(C.D2Q5, (130, 33), 1.1, force=(1e-5, 2e-6)))
    specs.append(C.cavity_case(N=40, Re=400.0, U=0.06))
    return specs


def _masks(specs):
    masks = []
    for k, s in enumerate(specs):
        if k == 2:
            m = np.zeros(s.fshape, np.uint8)
            m[20:30, 30:45] = 1
            masks.append(m)
        else:
            masks.append(None)
    return masks


@pytest.mark.parametrize("with_mask,form", [(False, 0), (True, 0), (False, 2), (True, 2)])
def test_batch_bitwise_equals_single_cases(with_mask, form):
    """Batched launches (one step, or two steps per launch) against
    one-step single-case contexts: populations and fields bit for bit."""
    specs = _mixed_cases()
    masks = _masks(specs) if with_mask else None
    stream = torch.cuda.Stream()
    _say(f"[batch] bitwise vs single, mask={with_mask}, form={form}")
    b = mdf.Solver(specs, storage="f32", solid=masks, device=DEV, stream=stream)
    b.set_launch(64, 4, 8, form)
    fields = mdf.FIELD_VORT | mdf.FIELD_STRAIN
    out_b = b.new_field_buffers(fields)
    b.step(7)                      # odd count: buffer parity flips per case
    b.step_emit(10, fields, out_b)  # graph-captured chunk
    b.step(5)
    stream.synchronize()
    for k, s in enumerate(specs):
        single = mdf.Solver([s], storage="f32", solid=None if masks is None else [masks[k]], device=DEV,
                            stream=stream)
        out_s = single.new_field_buffers(fields)
        single.step(7)
        single.step_emit(10, fields, out_s)
        single.step(5)
        stream.synchronize()
        assert torch.equal(b.populations(k), single.populations()), k
        assert torch.equal(out_b[k], out_s[0]), k
        assert b.time(k) == 22


@pytest.mark.parametrize("storage,form", [("f32", 0), ("f32", 2), ("f16dev", 0), ("f16dev", 2)])
def test_batch_beyond_the_cache_bitwise_equals_single_cases(storage, form):
    """A batch whose population buffers together exceed the 256 MB Infinity
    Cache (336 MB in FP32, 341 MB in FP16): its launches store with the
    non-temporal hint and address nodes by 32-bit offsets (the 16-bit pull
    then reads every set of a direction with one offset), while each case
    alone fits the cache and runs the plain form.  Populations and fields
    agree bit for bit, walls, a moving lid, a channel force and an obstacle
    included."""
    f = 1.0 if storage == "f32" else 1.45
    n = lambda v: int(round(v * f / 4)) * 4
    cav = C.cavity_case(N=n(1100), Re=1000.0)
    ch = C.poiseuille_case(n(900), n(700), umax=0.05, s1=1.3)
    box = C.cavity_case(N=n(1000), Re=400.0, U=0.08)
    box.shape = (n(1000), n(900))
    specs = [cav, ch, box]
    mask = np.zeros(box.fshape, np.uint8)
    mask[300:360, 400:470] = 1
    masks = [None, None, mask]
    stream = torch.cuda.Stream()
    _say(f"[batch] beyond the cache, bitwise vs single, {storage} form={form}")
    b = mdf.Solver(specs, storage=storage, solid=masks, device=DEV, stream=stream, u_ref=0.1)
    sb = 4 if storage == "f32" else 2
    pitch = 128 // sb
    sizes = [2 * 15 * sb * ((s.shape[0] + pitch - 1) // pitch * pitch) * s.shape[1] for s in specs]
    assert sum(sizes) > 256 << 20 and max(sizes) < 256 << 20
    b.set_launch(128, 2, 8, form)
    fields = mdf.FIELD_VORT | mdf.FIELD_STRAIN
    out_b = b.new_field_buffers(fields)
    b.step(5)
    b.step_emit(6, fields, out_b)
    stream.synchronize()
    for k, s in enumerate(specs):
        single = mdf.Solver([s], storage=storage, solid=[masks[k]] if masks[k] is not None else None, device=DEV,
                            stream=stream, u_ref=0.1)
        out_s = single.new_field_buffers(fields)
        single.step(5)
        single.step_emit(6, fields, out_s)
        stream.synchronize()
        assert torch.equal(b.populations(k), single.populations()), k
        assert torch.equal(out_b[k], out_s[0]), k
        del single


@pytest.mark.parametrize("form", [0, 2])
def test_batch_run_steady_matches_single_cases(form):
    """Per-case convergence inside one batch: same stopping step, same FP64
    residual and same state as solving each case alone."""
    specs = [C.cavity_case(N=32, Re=20.0, U=0.08), C.poiseuille_case(40, 24, umax=0.03, s1=1.0),
             C.cavity_case(N=48, Re=60.0, U=0.1)]
    stream = torch.cuda.Stream()
    _say(f"[batch] run_steady vs single, form={form}")
    b = mdf.Solver(specs, storage="f64", device=DEV, stream=stream)
    b.set_launch(64, 4, 8, form)
    st_b, steps_b, res_b = b.run_steady(1e-7, 100, 60000)
    assert (st_b == 0).all(), (st_b, steps_b, res_b)
    assert len(set(steps_b.tolist())) > 1          # cases stopped at different times
    for k, s in enumerate(specs):
        single = mdf.Solver([s], storage="f64", device=DEV, stream=stream)
        st, steps, res = single.run_steady(1e-7, 100, 60000)
        assert st[0] == 0 and steps[0] == steps_b[k], (k, steps, steps_b)
        assert res[0] == res_b[k]
        assert torch.equal(b.populations(k), single.populations())


def test_batch_seeded_subset_vs_oracle():
    """Three cases of the seeded uneven workload (sizes scaled down to 40..96)
    after 300 steps in one batch match the FP64 oracle (FP32 bar)."""
    bc = C.batch_cases(n=3, seed=210808591, nmin=40, nmax=96, step=8)
    specs = [c.spec for c in bc]
    _say("[batch] seeded subset vs oracle: " + ", ".join(f"{c.kind}{c.N}/Re{c.Re:.0f}" for c in bc))
    b = mdf.Solver(specs, storage="f32", device=DEV, stream=torch.cuda.Stream())
    b.step(300)
    for k, s in enumerate(specs):
        o = oracle_for(s).init(0.0, np.zeros((2,) + s.fshape)).run(300)
        compare_fields(o.fields(), gpu_fields_np(b, mdf.FIELD_ALL, k), 1e-5)


def test_autotune_keeps_results():
    specs = _mixed_cases()[:3]
    stream = torch.cuda.Stream()
    _say("[batch] autotune")
    a = mdf.Solver(specs, storage="f32", device=DEV, stream=stream)
    chosen, ms = a.autotune(trial_steps=5)
    assert chosen[0] % 32 == 0 and ms > 0
    n = a.time(0)
    ref = mdf.Solver(specs, storage="f32", device=DEV, stream=stream)
    ref.step(n)
    for k in range(len(specs)):
        assert torch.equal(a.populations(k), ref.populations(k))


def test_set_active_freezes_disabled_cases():
    specs = _mixed_cases()[:3]
    stream = torch.cuda.Stream()
    _say("[batch] set_active")
    b = mdf.Solver(specs, storage="f32", device=DEV, stream=stream)
    b.step(6)
    frozen = b.populations(1).clone()
    b.set_active([1, 0, 1])
    b.step(9)
    assert b.time(1) == 6 and b.time(0) == 15 and b.time(2) == 15
    assert torch.equal(b.populations(1), frozen)
    st, steps, res = b.run_steady(1e-30, 50, 100)
    assert st[1] == 3 and steps[1] == 0 and b.time(1) == 6
    ref = mdf.Solver([specs[0]], storage="f32", device=DEV, stream=stream)
    ref.step(115)
    assert torch.equal(b.populations(0), ref.populations())
