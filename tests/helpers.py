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

# Unit roundoff of the compute dtype of a parity bar: FP64 bars are below
# 1e-9, FP32 bars above.
def unit_roundoff(rtol):
    return 2.0 ** -53 if rtol < 1e-9 else 2.0 ** -24


# P = (sum_a J_aa - |u|^2) / d (eq. 3-15) is formed from populations of
# size ~|u| (lattice units), so rounding the stored populations perturbs it
# by ~eps |u| although P itself is ~|u|^2.  Its error is taken against its
# own norm, with the bar max(rtol, P_ROUNDING_FLOOR * eps * |u| / |P|): the
# parity bar where P is not much smaller than u, and a fixed number of
# rounding units of the populations where it is.
P_ROUNDING_FLOOR = 64.0


def compare_fields(ref, got, rtol, keys=FIELD_KEYS):
    """Per-field relative L2 error; fields that vanish identically (div) are
    measured against the size of the velocity gradient, and P against its
    own norm with the rounding floor above."""
    gscale = np.linalg.norm(np.asarray(ref["grad"]).ravel())
    unorm = np.linalg.norm(np.asarray(ref["u"]).ravel())
    errs, bars = {}, {}
    for k in keys:
        scale = gscale if k in ("div", "S", "sigma", "vort", "grad") else None
        errs[k] = rel_err(ref[k], got[k], scale)
        bars[k] = rtol
        if k == "P":
            pnorm = np.linalg.norm(np.asarray(ref["P"]).ravel())
            floor = P_ROUNDING_FLOOR * unit_roundoff(rtol) * unorm / pnorm if pnorm > 0 else 0.0
            bars[k] = max(rtol, floor)
    bad = {k: (e, bars[k]) for k, e in errs.items() if not e <= bars[k]}
    assert not bad, f"fields beyond their bars (error, bar): {bad} (all: {errs})"
    return errs
