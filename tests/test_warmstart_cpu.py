"""Host logic of the warm-start pipeline (no GPU): coarse cases, the
scaling between lattice fields and network targets, and the interpolation of
a coarse solution to the fine grid."""
import numpy as np
import torch

from paper_2108_08591_amd import nn
from paper_2108_08591_amd import warmstart as WS


def test_coarse_cases_keep_flow_parameters_and_pool_the_mask():
    cases = WS.warmstart_cases(24, N=64, seed=3)
    coarse = WS.coarse_cases(cases, s1_max=1.85)
    capped = 0
    for c, k in zip(cases, coarse):
        assert k["N"] == 32 and k["spec"].shape == (32, 32)
        assert k["U"] == c["U"]
        nu_f = 1.0 / 3.0 * (1.0 / c["spec"].s1 - 0.5)
        nu_c = 1.0 / 3.0 * (1.0 / k["spec"].s1 - 0.5)
        if abs(k["Re"] - c["Re"]) < 1e-9 * c["Re"]:
            # same lid speed and Reynolds number: the viscosity scales with N
            assert abs(nu_f / nu_c - 2.0) < 1e-9
            assert k["spec"].s1 <= 1.85 + 1e-12
        else:
            # too fine a viscosity for the coarse grid: capped at s1 = 1.85
            capped += 1
            assert k["Re"] < c["Re"] and abs(k["spec"].s1 - 1.85) < 1e-9
        pooled = c["mask"].reshape(32, 2, 32, 2).max(axis=(1, 3))
        inner = (slice(1, -1), slice(1, -1))
        assert np.array_equal(k["mask"][inner], pooled[inner])
        assert k["mask"][0].sum() == 0 and k["mask"][:, -1].sum() == 0
    assert 0 < capped < len(cases)


def test_scaled_fields_round_trip():
    rng = np.random.default_rng(0)
    N, U, Re = 32, 0.07, 250.0
    mask = np.zeros((N, N), np.uint8)
    mask[10:14, 12:20] = 1
    fl = rng.normal(size=(7, N, N)) * np.array([1e-4, 0.05, 0.05, 1e-3, 1e-3, 1e-3, 1e-3])[:, None, None]
    fl[6] = -fl[3]                                  # trace-free gradient
    fl[:, mask.astype(bool)] = 0.0
    fl[0][mask == 0] -= fl[0][mask == 0].mean()     # pressure gauge: zero fluid mean
    base = nn.scaled_fields(fl, N, U, Re, mask)
    norm = {"mean": np.zeros(nn.OUT_CH, np.float32), "std": np.ones(nn.OUT_CH, np.float32)}
    back = nn.fields_from_prediction(np.zeros((N, N, nn.OUT_CH)), N, U, Re, mask, norm, base)
    assert np.allclose(back, fl, rtol=1e-5, atol=1e-9)
    # the target scales agree with raw_targets on the same fields
    f = {"P": torch.tensor(fl[0]), "u": torch.tensor(fl[1:3]),
         "grad": torch.tensor(fl[3:7].reshape(2, 2, N, N))}
    t = nn.raw_targets(f, N, U, Re).numpy()
    fluid = mask == 0
    for ch in range(1, nn.OUT_CH):
        assert np.allclose(t[..., ch][fluid], base[..., ch][fluid], rtol=1e-5, atol=1e-6)


class _ConstSolver:
    """Stands in for a solver whose steady fields are given arrays."""

    def __init__(self, fields):
        self.f = fields

    def fields(self, which, k):
        a = self.f[k]
        return {"P": torch.tensor(a[0]), "u": torch.tensor(a[1:3]), "grad": torch.tensor(a[3:7].reshape(2, 2, *a.shape[1:]))}


def test_upsampled_init_interpolates_and_rescales_gradients():
    cases = WS.warmstart_cases(2, N=32, seed=9)
    for c in cases:
        c["mask"][:] = 0
    coarse = WS.coarse_cases(cases)
    n = 16
    y, x = np.mgrid[0:n, 0:n] + 0.5
    a = np.zeros((7, n, n))
    a[1] = 0.01 * x                     # u linear in x: du/dx = 0.01 per coarse node
    a[3] = 0.01
    a[6] = -0.01
    a[2] = -0.01 * y
    up = WS.upsampled_init(cases, coarse, _ConstSolver([a, a]), [0, 1])
    X = (np.arange(32) + 0.5) / 2.0     # fine centres in coarse units
    # interior of the bilinear interpolation of a linear field is exact
    assert np.allclose(up[0][1][:, 2:-2], 0.01 * X[None, 2:-2], atol=1e-7)
    assert np.allclose(up[0][3], 0.005) and np.allclose(up[0][6], -0.005)
    # a coarse solve that did not converge (status != 0) gives no init
    assert up[1] is None
    other = WS.upsampled_init(cases, coarse, _ConstSolver([a, a]), [1, 0])
    assert other[0] is None and other[1] is not None


def test_input_features_carry_one_or_two_coarse_levels():
    """The coarse solutions sit in their own channel blocks, each followed by
    a flag; absent levels leave zeros; everything fits the padded width."""
    N = 32
    mask = np.zeros((N, N), np.uint8)
    mask[10:14, 8:12] = 1
    a = np.full((N, N, nn.OUT_CH), 0.25, np.float32)
    b = np.full((N, N, nn.OUT_CH), -0.5, np.float32)
    k1, k2 = nn.FEATURES, nn.FEATURES + nn.COARSE_FEATURES
    assert k2 + nn.COARSE_FEATURES <= nn.IN_CH
    none = nn.input_features(N, mask, 100.0, 0.08)
    one = nn.input_features(N, mask, 100.0, 0.08, coarse=a)
    two = nn.input_features(N, mask, 100.0, 0.08, coarse=a, coarse2=b)
    assert np.array_equal(none[..., :k1], two[..., :k1])
    assert not none[..., k1:].any()
    assert np.all(one[..., k1:k1 + nn.OUT_CH] == 0.25) and np.all(one[..., k1 + nn.OUT_CH] == 1.0)
    assert not one[..., k2:].any()
    assert np.array_equal(two[..., :k2], one[..., :k2])
    assert np.all(two[..., k2:k2 + nn.OUT_CH] == -0.5) and np.all(two[..., k2 + nn.OUT_CH] == 1.0)
    assert not two[..., k2 + nn.COARSE_FEATURES:].any()
