"""Storage precision of the 3D Taylor-Green vortex (D3Q7, four sets, u0 =
0.05, Re = 100 and 1600) against the FP64 CPU oracle: FP64, FP32, FP16- and
BF16-deviation storage (FP32 collision in the last three), relative L2 error
of u, P (against |u|, as P is formed from populations of size |u|) and the
vorticity after each step count.

The grids the oracle can afford (32^3, 64^3) take the lattice parameters of
the configuration's 256^3 runs: the same u0, s1 and s2, hence the same cell
Reynolds number and stability (Re = 100: s1 = 1.7197 with the s2 of
Section 4.1; Re = 1600: s1 = 1.9798 with s2 = 1.5, the even-moment rate of
Section 4.1 diverging there).  On N^3 their nominal Reynolds number is
Re N / 256.  (At the nominal Re on 64^3, s1 = 1.92 and 1.995, both runs
diverge, in the oracle as on the GPU.)

test_precision_small runs by default (32^3, 600 steps).  The full study on
64^3 (5000 steps, errors at 1000 / 2500 / 5000) runs when
MDF_PRECISION_STUDY is set, and writes its table to the file
MDF_PRECISION_OUT names (if any)."""
import json
import os
import sys

import numpy as np
import pytest
import torch

from paper_2108_08591_amd import cases as C
from paper_2108_08591_amd import mdf
from helpers import oracle_for, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
STORAGES = ("f64", "f32", "f16dev", "bf16dev")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _spec(N, Re):
    """N^3 box with the relaxation rates of the 256^3 run at Re."""
    ref = C.tgv3d_case(N=256, u0=0.05, Re=Re)
    spec = C.CaseSpec(C.D3Q7, (N, N, N), ref.s1)
    if Re > 1000.0:
        spec.s2 = 1.5
    return spec


def _fields(d):
    return {k: np.asarray(d[k], np.float64) for k in ("u", "P", "vort")}


def study(N, steps):
    out = []
    P, u = C.taylor_green_3d_initial(N, 0.05)
    for Re in (100.0, 1600.0):
        spec = _spec(N, Re)
        _say(f"[precision] oracle {N}^3, rates of Re {Re:g} at 256^3, s1 {spec.s1:.5f}")
        o = oracle_for(spec).init(P, u)
        ref, done = {}, 0
        for t in steps:
            o.run(t - done)
            done = t
            ref[t] = _fields(o.fields())
        for st in STORAGES:
            dt = np.float64 if st == "f64" else np.float32
            init = torch.tensor(np.concatenate([P[None], u], axis=0).astype(dt))
            s = mdf.Solver([spec], storage=st, init=("fields", [init]), device=DEV, u_ref=0.05)
            rec = {"N": N, "Re_256": Re, "Re_nominal": Re * N / 256, "s1": spec.s1,
                   "s2": spec.s2 if spec.s2 > 0 else 8 * (2 - spec.s1) / (8 - spec.s1), "storage": st,
                   "errors": {}}
            done = 0
            for t in steps:
                s.step(t - done)
                done = t
                f = s.fields(mdf.FIELD_MOMENTS | mdf.FIELD_VORT)
                got = {k: v.detach().cpu().numpy().astype(np.float64) for k, v in f.items()}
                uscale = np.linalg.norm(ref[t]["u"].ravel())
                finite = all(np.isfinite(got[k]).all() for k in ("u", "P", "vort"))
                rec["errors"][str(t)] = {"finite": bool(finite),
                                         "u": rel_err(ref[t]["u"], got["u"]),
                                         "P": rel_err(ref[t]["P"], got["P"], uscale),
                                         "vort": rel_err(ref[t]["vort"], got["vort"]),
                                         "u_rms_oracle": float(np.sqrt(np.mean(ref[t]["u"] ** 2)))}
            _say(json.dumps(rec))
            out.append(rec)
            del s
            torch.cuda.empty_cache()
    return out


def _check(res, last):
    for rec in res:
        e = rec["errors"][str(last)]
        assert e["finite"], rec
        if rec["storage"] == "f64":
            assert max(e["u"], e["P"], e["vort"]) < 1e-10, rec
        elif rec["storage"] == "f32":
            assert max(e["u"], e["P"], e["vort"]) < 1e-4, rec


def test_precision_small():
    res = study(32, (200, 600))
    _check(res, 600)


@pytest.mark.skipif(not os.environ.get("MDF_PRECISION_STUDY"), reason="full precision study: set MDF_PRECISION_STUDY")
def test_precision_c3_64():
    res = study(64, (1000, 2500, 5000))
    path = os.environ.get("MDF_PRECISION_OUT")
    if path:
        with open(path, "w") as fh:
            json.dump(res, fh, indent=1)
    _check(res, 5000)
