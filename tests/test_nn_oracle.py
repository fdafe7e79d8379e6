"""Pins of the FP64 layer oracle (oracle/conv_oracle.py): central finite
differences for every backward, a delta-kernel shift identity, adjoint
identities of pooling / up-sampling and the closed form of the first Adam
step.  CPU only."""
import numpy as np

from oracle import conv_oracle as R


def _fd(f, x, h=1e-6):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = x[i]
        x[i] = old + h
        fp = f()
        x[i] = old - h
        fm = f()
        x[i] = old
        g[i] = (fp - fm) / (2 * h)
    return g


def test_conv_backward_by_finite_differences():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 4, 5, 3))
    w = rng.normal(size=(2, 9, 3))
    b = rng.normal(size=2)
    g = rng.normal(size=(2, 4, 5, 2))
    L = lambda: float((g * R.conv3x3(x, w, b)).sum())
    assert np.allclose(R.conv3x3_dgrad(g, w), _fd(L, x), atol=1e-6)
    dw, db = R.conv3x3_wgrad(x, g)
    assert np.allclose(dw, _fd(L, w), atol=1e-6)
    assert np.allclose(db, _fd(L, b), atol=1e-6)


def test_conv_delta_kernel_is_a_shift():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 6, 7, 2))
    for t, (dy, dx) in enumerate(R.TAPS):
        w = np.zeros((2, 9, 2))
        w[:, t, :] = np.eye(2)
        y = R.conv3x3(x, w)
        ref = np.zeros_like(x)
        for yy in range(6):
            for xx in range(7):
                if 0 <= yy + dy < 6 and 0 <= xx + dx < 7:
                    ref[0, yy, xx] = x[0, yy + dy, xx + dx]
        assert np.array_equal(y, ref)


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 6, 8, 3))
    y = rng.normal(size=(2, 3, 4, 3))
    assert np.isclose((R.avgpool2(x) * y).sum(), (x * R.avgpool2_bwd(y)).sum())
    z = rng.normal(size=(2, 12, 16, 3))
    assert np.isclose((R.upsample2(x) * z).sum(), (x * R.upsample2_bwd(z)).sum())
    assert np.allclose(R.avgpool2(R.upsample2(x)), x)


def test_head_and_loss_by_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(7, 4))
    w = rng.normal(size=(3, 4))
    b = rng.normal(size=3)
    t = rng.normal(size=(7, 3))
    wt = rng.uniform(0, 1, size=7)
    L = lambda: R.mse(R.head(x, w, b), t, wt)[0]
    _, dy = R.mse(R.head(x, w, b), t, wt)
    dx, dw, db = R.head_bwd(x, dy, w)
    assert np.allclose(dx, _fd(L, x), atol=1e-7)
    assert np.allclose(dw, _fd(L, w), atol=1e-7)
    assert np.allclose(db, _fd(L, b), atol=1e-7)


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = R.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8))
