"""Learned warm start of steady cavity solves: data generation with the
batched solver, training of the encoder-decoder of nn.py on the GPU, and the
warm-versus-cold comparison.

The solver decides the answer in both cases: a warm start only replaces the
rest state by f^eq + f^ne built from the predicted (P, u, grad u) (inverse
of eq. 3-16); the cold start from rest is the fallback whenever the warm
solve goes non-finite or does not converge.
"""
from __future__ import annotations

import json
import math
import time
from typing import Callable, Dict, List, Optional

import numpy as np
import torch

from . import cases as C
from . import mdf
from . import nn

FIELDS = mdf.FIELD_MOMENTS | mdf.FIELD_GRAD


def warmstart_cases(n: int, N: int = 128, seed: int = 20210819) -> List[dict]:
    """Seeded lid-driven cavities with 0..3 circular/rectangular obstacles:
    Re log-uniform in [10, 1000], lid speed uniform in [0.05, 0.1]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        Re = float(10.0 ** rng.uniform(1.0, 3.0))
        U = float(rng.uniform(0.05, 0.1))
        mask = C.obstacle_mask(N, rng)
        spec = C.cavity_case(N=N, Re=Re, U=U)
        out.append({"spec": spec, "mask": mask, "Re": Re, "U": U, "N": N})
    return out


def solve(cases: List[dict], storage="f32", tol=1e-8, K=100, max_steps=400000, init=None, stream=None,
          window=20000, log: Optional[Callable[[str], None]] = None):
    """Run every case to residual `tol` in one batched context.  init: None
    (rest) or a list of channel-major field arrays [P, u, v, (grad 4)] per
    case.  Returns (solver, status, steps, residual, wall seconds)."""
    specs = [c["spec"] for c in cases]
    masks = [c["mask"] for c in cases]
    t0 = time.perf_counter()
    if init is None:
        solver = mdf.Solver(specs, storage=storage, solid=masks, stream=stream)
    else:
        kind = "fields_grad" if init[0].shape[0] == 7 else "fields"
        solver = mdf.Solver(specs, storage=storage, solid=masks, init=(kind, [torch.tensor(a) for a in init]),
                            stream=stream)
    n = len(cases)
    st = np.full(n, 2)
    steps = np.zeros(n, np.int64)
    res = np.full(n, np.inf)
    active = np.ones(n, bool)
    done = 0
    while active.any() and done < max_steps:
        solver.set_active(active)
        w = min(window, max_steps - done)
        s, k, r = solver.run_steady(tol, K, w)
        done += w
        for i in np.nonzero(active)[0]:
            steps[i] += k[i]
            res[i] = r[i]
            if s[i] in (0, 1):
                st[i] = s[i]
                active[i] = False
        if log:
            log(json.dumps({"solve_steps": done, "converged": int((st == 0).sum()), "nonfinite": int((st == 1).sum()),
                            "running": int(active.sum()), "wall_s": round(time.perf_counter() - t0, 1)}))
    torch.cuda.synchronize()
    return solver, st, steps, res, time.perf_counter() - t0


def solve_warm(cases: List[dict], init, storage="f64", tol=1e-8, K=100, max_steps=400000, stream=None,
               window=20000, log: Optional[Callable[[str], None]] = None):
    """Warm solves with the cold start as fallback: every case first runs
    from its predicted initial state (init, as in solve()); each case that
    goes non-finite or does not converge within max_steps is solved again
    from rest, and its steps and wall time are added.  Returns (where,
    status, steps, residual, wall seconds, fallback case indices), with
    where[k] = (solver, index) holding case k's final state."""
    warm, st, steps, res, wall = solve(cases, storage, tol=tol, K=K, max_steps=max_steps, init=init,
                                       stream=stream, window=window, log=log)
    where = [(warm, k) for k in range(len(cases))]
    bad = [k for k in range(len(cases)) if st[k] != 0]
    if bad:
        cold, cst, csteps, cres, cwall = solve([cases[k] for k in bad], storage, tol=tol, K=K,
                                               max_steps=max_steps, stream=stream, window=window, log=log)
        for j, k in enumerate(bad):
            where[k] = (cold, j)
            st[k] = cst[j]
            steps[k] += csteps[j]
            res[k] = cres[j]
        wall += cwall
    return where, st, steps, res, wall, bad


def coarse_cases(cases: List[dict], factor: int = 2, s1_max: float = 1.85) -> List[dict]:
    """The same cavities on a grid `factor` times coarser: same lid speed
    (the same flow in lattice velocity units) and Re, a node solid when any of
    the fine nodes it covers is solid, one fluid ring at the walls.  Where the
    coarse grid cannot resolve the flow stably (s1 above s1_max, the cell
    Reynolds number too high), the coarse case takes the lowest viscosity
    with s1 = s1_max instead: a lower-Re flow that still serves as a first
    guess (its Re is recorded as "Re")."""
    nu_min = (1.0 / s1_max - 0.5) / 3.0
    out = []
    for c in cases:
        N = c["N"]
        n = N // factor
        m = c["mask"].reshape(n, factor, n, factor).max(axis=(1, 3)).astype(np.uint8)
        m[:1, :] = 0
        m[-1:, :] = 0
        m[:, :1] = 0
        m[:, -1:] = 0
        nu = max(c["U"] * n / c["Re"], nu_min)
        re_c = c["U"] * n / nu
        out.append({"spec": C.cavity_case(N=n, Re=re_c, U=c["U"]), "mask": m, "Re": re_c, "U": c["U"], "N": n})
    return out


def upsampled_init(cases: List[dict], coarse: List[dict], solver, status, factor: int = 2):
    """Steady fields of the coarse solves, interpolated (bilinear, cell
    centred) to the fine grids as channel-major [P, u, v, grad(4)] init data;
    gradients rescaled to the fine node spacing, solid nodes zeroed, the
    divergence of the gradient removed.  None for a coarse solve that did not
    converge."""
    from scipy.ndimage import zoom
    out = []
    for k, c in enumerate(cases):
        if status[k] != 0:
            out.append(None)
            continue
        a = solution_init(solver, k)
        up = np.stack([zoom(a[ch], factor, order=1, grid_mode=True, mode="nearest") for ch in range(7)])
        up[3:] /= factor
        div = up[3] + up[6]
        up[3] -= 0.5 * div
        up[6] -= 0.5 * div
        up[:, c["mask"].astype(bool)] = 0.0
        out.append(up.astype(np.float32))
    return out


def dataset(cases: List[dict], solver, log: Optional[Callable[[str], None]] = None,
            coarse: Optional[List[Optional[np.ndarray]]] = None,
            coarse2: Optional[List[Optional[np.ndarray]]] = None) -> Dict[str, torch.Tensor]:
    """Inputs (bf16 [n, N, N, IN_CH]), raw targets (f32 [n, N*N, OUT_CH])
    and fluid weights (f32 [n, N*N]) from solved cases.  With `coarse`
    (upsampled coarse solutions, or None per case) the inputs carry them and
    the targets are the corrections to them; `coarse2` (a second, coarser
    level) is an input only."""
    X, T, Wt = [], [], []
    for k, c in enumerate(cases):
        if log and k % 2048 == 0:
            log(json.dumps({"dataset_cases": k, "of": len(cases)}))
        N = c["N"]
        base = None
        if coarse is not None and coarse[k] is not None:
            base = nn.scaled_fields(coarse[k], N, c["U"], c["Re"], c["mask"])
        base2 = None
        if coarse2 is not None and coarse2[k] is not None:
            base2 = nn.scaled_fields(coarse2[k], N, c["U"], c["Re"], c["mask"])
        X.append(torch.tensor(nn.input_features(N, c["mask"], c["Re"], c["U"], base, base2)))
        f = solver.fields(FIELDS, k)
        t = nn.raw_targets(f, N, c["U"], c["Re"]).cpu()
        if base is not None:
            t = t - torch.tensor(base)
        T.append(t.reshape(N * N, nn.OUT_CH))
        Wt.append(torch.tensor((c["mask"] == 0).astype(np.float32).reshape(-1)))
    torch.cuda.synchronize()
    return {"X": torch.stack(X), "T": torch.stack(T), "W": torch.stack(Wt)}


def fit_normalisation(T, W):
    """Per-channel mean/std of the raw targets over fluid nodes."""
    w = W.reshape(-1, 1)
    t = T.reshape(-1, T.shape[-1])
    mean = (t * w).sum(0) / w.sum()
    std = torch.sqrt(((t - mean) ** 2 * w).sum(0) / w.sum()).clamp_min(1e-6)
    return {"mean": mean.numpy().astype(np.float32), "std": std.numpy().astype(np.float32)}


def train(model: nn.UNet, data: Dict[str, torch.Tensor], epochs=30, batch=16, lr=2e-3, seed=0, clip=None,
          val: Optional[Dict[str, torch.Tensor]] = None, log: Optional[Callable[[str], None]] = None):
    """Adam on the weighted MSE of the normalised targets; inputs and
    targets are moved to the device once.  clip (in standard deviations)
    bounds the normalised targets, so that the few nodes at the singular lid
    corners do not dominate the loss.  Returns the per-epoch losses (and
    the held-out losses when `val` is given)."""
    dev = model.device
    model.norm = fit_normalisation(data["T"], data["W"])
    mean = torch.tensor(model.norm["mean"], device=dev)
    std = torch.tensor(model.norm["std"], device=dev)

    def prep(d):
        X = nn.to_bf16(d["X"].to(dev))
        T = (d["T"].to(dev) - mean) / std
        if clip is not None:
            T = T.clamp(-clip, clip)
        return X, T.contiguous(), d["W"].to(dev).contiguous()

    X, T, W = prep(data)
    Xv, Tv, Wv = prep(val) if val is not None else (None, None, None)
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    history, val_hist = [], []
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    it = 0
    for ep in range(epochs):
        perm = rng.permutation(n)
        acc = 0.0
        for b in range(steps_per_epoch):
            idx = torch.tensor(perm[b * batch:(b + 1) * batch], device=dev)
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).reshape(-1, nn.OUT_CH).contiguous()
            wb = W.index_select(0, idx).reshape(-1).contiguous()
            model.forward(xb)
            loss, g = model.loss_and_grad(tb, wb)
            model.backward(g)
            # cosine learning-rate schedule
            cur = lr * 0.5 * (1 + math.cos(math.pi * it / total))
            model.adam_step(cur)
            it += 1
            acc += float(loss.item())
        history.append(acc / steps_per_epoch)
        rec = {"epoch": ep + 1, "loss": round(history[-1], 6)}
        if Xv is not None and ((ep + 1) % 10 == 0 or ep + 1 == epochs):
            vl = 0.0
            for b in range(0, Xv.shape[0], batch):
                model.forward(Xv[b:b + batch].contiguous())
                l, _ = model.loss_and_grad(Tv[b:b + batch].reshape(-1, nn.OUT_CH).contiguous(),
                                           Wv[b:b + batch].reshape(-1).contiguous())
                vl += float(l.item()) * min(batch, Xv.shape[0] - b)
            rec["val_loss"] = round(vl / Xv.shape[0], 6)
            val_hist.append((ep + 1, rec["val_loss"]))
        if log:
            log(json.dumps(rec))
    return (history, val_hist) if Xv is not None else history


def predict(model: nn.UNet, cases: List[dict], with_grad=True, batch=16,
            coarse: Optional[List[Optional[np.ndarray]]] = None,
            coarse2: Optional[List[Optional[np.ndarray]]] = None) -> List[np.ndarray]:
    """Initial fields per case from the network ([P, u, v] or
    [P, u, v, grad(4)], channel-major float64); with `coarse`, the network
    corrects the upsampled coarse solutions it is given (`coarse2`: a second,
    coarser level as further input)."""
    out = []
    dev = model.device
    for s in range(0, len(cases), batch):
        part = cases[s:s + batch]
        N = part[0]["N"]
        bases, bases2 = [], []
        for k, c in enumerate(part):
            cf = coarse[s + k] if coarse is not None else None
            bases.append(None if cf is None else nn.scaled_fields(cf, N, c["U"], c["Re"], c["mask"]))
            cf2 = coarse2[s + k] if coarse2 is not None else None
            bases2.append(None if cf2 is None else nn.scaled_fields(cf2, N, c["U"], c["Re"], c["mask"]))
        X = torch.stack([torch.tensor(nn.input_features(N, c["mask"], c["Re"], c["U"], bases[k], bases2[k]))
                         for k, c in enumerate(part)])
        y = model.forward(nn.to_bf16(X.to(dev)))
        y = y.reshape(len(part), N, N, nn.OUT_CH).cpu().numpy()
        for k, c in enumerate(part):
            fl = nn.fields_from_prediction(y[k], N, c["U"], c["Re"], c["mask"], model.norm, bases[k])
            out.append(fl if with_grad else fl[:3].copy())
    return out


def solution_init(solver, k) -> np.ndarray:
    """The steady fields of case k as channel-major [P, u, v, grad(4)]
    init data (float64): the warm start an exact predictor would give."""
    f = solver.fields(FIELDS, k)
    P = f["P"].double().cpu().numpy()
    u = f["u"].double().cpu().numpy()
    g = f["grad"].double().cpu().numpy()
    return np.stack([P, u[0], u[1], g[0, 0], g[0, 1], g[1, 0], g[1, 1]])


CHANNELS = ("P", "u", "v", "du/dx", "du/dy", "dv/dx", "dv/dy")


def prediction_error(init: np.ndarray, exact: np.ndarray, mask) -> Dict[str, float]:
    """Relative L2 error per channel of a predicted init over fluid nodes
    (P with its mean removed from both, since only its gradient acts)."""
    fl = mask == 0
    out = {}
    for c, name in enumerate(CHANNELS):
        a, b = init[c][fl], exact[c][fl]
        if c == 0:
            a, b = a - a.mean(), b - b.mean()
        out[name] = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    return out


def field_error(solver_a, solver_b, k, kb=None) -> float:
    """Relative L2 distance of the velocity fields of case k in solver_a and
    case kb (default k) in solver_b."""
    ua = solver_a.fields(mdf.FIELD_MOMENTS, k)["u"].double()
    ub = solver_b.fields(mdf.FIELD_MOMENTS, k if kb is None else kb)["u"].double()
    torch.cuda.synchronize()
    return float(torch.linalg.vector_norm(ua - ub) / torch.linalg.vector_norm(ua))
