"""Shared helpers of the GPU tests: build the oracle and the GPU solver from
one CaseSpec (inputs only; no arithmetic of the method lives here)."""
import numpy as np

from oracle import oracle as O


def oracle_for(spec, solid=None, force_field=None):
    case = O.Case(spec.lattice, spec.shape, spec.s1, s0=spec.s0, s2=spec.s2, bc=spec.bc,
                  wall_u=spec.wall_velocity(), force=spec.force, R=spec.R, rho0=spec.rho0,
                  forcing=spec.forcing)
    return O.Oracle(case, solid=solid, force_field=force_field)


def rel_err(ref, got, scale=None):
    ref = np.asarray(ref, np.float64)
    got = np.asarray(got, np.float64)
    den = np.linalg.norm(ref.ravel())
    if scale is not None:
        den = max(den, scale)
    num = np.linalg.norm((ref - got).ravel())
    if den == 0.0:
        return num
    return num / den


def gpu_fields_np(solver, fields, case=0):
    """GPU fields as numpy, keyed like the oracle's fields()."""
    from paper_2108_08591_amd import mdf
    f = solver.fields(fields, case)
    out = {}
    for k, v in f.items():
        out[k] = v.detach().cpu().numpy().astype(np.float64)
    if "ubar" in out:
        out["ubar0"] = out["ubar"][0]
    return out


FIELD_KEYS = ("ubar0", "u", "P", "grad", "div", "S", "sigma", "vort")


def compare_fields(ref, got, rtol, keys=FIELD_KEYS):
    """Per-field relative L2 error; fields that vanish identically (div) are
    measured against the size of the velocity gradient."""
    gscale = np.linalg.norm(np.asarray(ref["grad"]).ravel())
    # P = (sum_a J_aa - |u|^2)/d (eq. 3-15) is formed from populations of
    # size ~|u| (lattice units), so storage rounding resolves it to eps |u|,
    # not eps |u|^2: its error is measured against max(|P|, |u|)
    pscale = np.linalg.norm(np.asarray(ref["u"]).ravel())
    errs = {}
    for k in keys:
        scale = gscale if k in ("div", "S", "sigma", "vort", "grad") else None
        if k == "P":
            scale = pscale
        errs[k] = rel_err(ref[k], got[k], scale)
    bad = {k: e for k, e in errs.items() if not e <= rtol}
    assert not bad, f"fields beyond {rtol:g}: {bad} (all: {errs})"
    return errs
