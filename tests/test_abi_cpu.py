"""Host-side checks of the C ABI (no GPU needed, no compute calls).

The library loads, exports every function include/mdf.h declares, and the
host validation rejects bad arguments before anything is launched.
"""
import ctypes
import os
import re

import pytest

from paper_2108_08591_amd import cases as C
from paper_2108_08591_amd import mdf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "mdf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = mdf.lib()
    declared = _declared_functions()
    assert "mdf_init" in declared and "mdf_step" in declared
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(mdf.EXPORTED) == declared


def _declared_nn_functions():
    text = open(os.path.join(ROOT, "include", "mdfnn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdfnn_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_network_symbol():
    from paper_2108_08591_amd import nn
    L = nn._lib()
    declared = _declared_nn_functions()
    assert "mdfnn_conv3x3_fwd" in declared and "mdfnn_mse_noalloc" in declared
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(nn.NN_EXPORTED) == declared


def test_noalloc_loss_refuses_sizes_beyond_its_scratch():
    """mdfnn_mse_noalloc checks P against its static scratch before touching
    the device: MDFNN_ETOOBIG (-2) above the maximum, MDFNN_EINVAL (-1) for
    null pointers; nothing is launched (the pointers are never read)."""
    from paper_2108_08591_amd import nn
    L = nn._lib()
    fake = ctypes.c_void_p(256)
    assert L.mdfnn_mse_noalloc(fake, fake, fake, nn.MSE_NOALLOC_MAX_P + 1, 7, fake, fake, None) == -2
    assert L.mdfnn_mse_noalloc(None, fake, fake, 16, 7, fake, fake, None) == -1
    assert L.mdfnn_mse_noalloc(fake, fake, fake, 0, 7, fake, fake, None) == -1


def _ws(spec, storage=mdf.F32, solid=0):
    c = (mdf.MdfCase * 1)(mdf._case_struct(spec))
    return mdf.lib().mdf_workspace_size(spec.lattice, storage, c, 1, solid)


def test_workspace_size_scales_with_storage_and_grid():
    spec = C.cavity_case(N=128, Re=100)
    w64, w32, w16 = _ws(spec, mdf.F64), _ws(spec, mdf.F32), _ws(spec, mdf.F16DEV)
    assert w64 > w32 > w16 > 0
    # two population buffers dominate: 2 * 15 * 128^2 * bytes
    assert w32 >= 2 * 15 * 128 * 128 * 4
    assert _ws(spec, mdf.F32, solid=1) > w32
    big = C.cavity_case(N=256, Re=100)
    assert _ws(big) > 3.5 * w32


def test_planes_beyond_4gib_are_refused():
    """The step kernels address nodes by 32-bit byte offsets within a plane:
    a case whose padded population plane would exceed 4 GiB (a 1 x 40 M FP32
    column pads every row to 32 values: 5.1 GB per plane, with only 6e8
    populations) is refused; one just below the bound is accepted."""
    narrow = C.CaseSpec(C.D2Q5, (1, 40_000_000), 1.2)
    assert _ws(narrow) == 0
    assert "4 GiB" in mdf.lib().mdf_last_error(None).decode()
    ok = C.CaseSpec(C.D2Q5, (1, 33_554_432), 1.2)          # 32 * 2^25 * 4 B = 4 GiB exactly
    assert _ws(ok) > 0


def test_velocity_set_lattices_store_d_of_d_plus_one_sets():
    """MDF_D2Q5_V / MDF_D3Q7_V keep only the d velocity sets (Remark IV):
    the population part of the workspace shrinks by d/(d+1)."""
    for spec, d in ((C.cavity_case(N=256, Re=100), 2), (C.tgv3d_case(N=64, u0=0.05, Re=100.0), 3)):
        c = (mdf.MdfCase * 1)(mdf._case_struct(spec))
        full = mdf.lib().mdf_workspace_size(spec.lattice, mdf.F32, c, 1, 0)
        vel = mdf.lib().mdf_workspace_size(spec.lattice + 2, mdf.F32, c, 1, 0)
        q = 5 if d == 2 else 7
        one_set = 2 * q * spec.nodes * 4          # both ping-pong buffers, FP32
        assert full - vel == pytest.approx(one_set, rel=0.02)
        assert full > (d + 1) * one_set
    assert mdf.lib().mdf_workspace_size(14, mdf.F32, c, 1, 0) == 0
    assert mdf.lib().mdf_workspace_size(-1, mdf.F32, c, 1, 0) == 0


def test_rest_free_lattices_store_q_minus_one_planes():
    """MDF_D2Q4 / MDF_D3Q6 (eq. d2q4, d3q6) keep 4 and 6 planes per set
    against 5 and 7 for D2Q5 / D3Q7; a 3D case on a 2D lattice is rejected."""
    for spec, lat, q_full, q in ((C.cavity_case(N=256, Re=100), mdf.D2Q4, 5, 4),
                                 (C.tgv3d_case(N=64, u0=0.05, Re=100.0), mdf.D3Q6, 7, 6)):
        c = (mdf.MdfCase * 1)(mdf._case_struct(spec))
        full = mdf.lib().mdf_workspace_size(spec.lattice, mdf.F32, c, 1, 0)
        rest_free = mdf.lib().mdf_workspace_size(lat, mdf.F32, c, 1, 0)
        plane = 2 * (spec.d + 1) * spec.nodes * 4        # one plane per set, both buffers
        assert full - rest_free == pytest.approx((q_full - q) * plane, rel=0.02)
    c3 = (mdf.MdfCase * 1)(mdf._case_struct(C.tgv3d_case(N=16, u0=0.05, Re=100.0)))
    assert mdf.lib().mdf_workspace_size(mdf.D2Q4, mdf.F32, c3, 1, 0) == 0


def test_diagonal_lattices_store_q_planes():
    """MDF_D2Q9 / MDF_D3Q15 (eq. d2q9, d3q15) keep 9 and 15 planes per set."""
    for spec, lat, q_full, q in ((C.cavity_case(N=256, Re=100), mdf.D2Q9, 5, 9),
                                 (C.tgv3d_case(N=64, u0=0.05, Re=100.0), mdf.D3Q15, 7, 15)):
        c = (mdf.MdfCase * 1)(mdf._case_struct(spec))
        base = mdf.lib().mdf_workspace_size(spec.lattice, mdf.F32, c, 1, 0)
        diag = mdf.lib().mdf_workspace_size(lat, mdf.F32, c, 1, 0)
        plane = 2 * (spec.d + 1) * spec.nodes * 4
        assert diag - base == pytest.approx((q - q_full) * plane, rel=0.02)


def test_lattice_per_set_stores_fewer_set0_planes():
    """MDF_D2Q9_Q5 / MDF_D3Q15_Q7 (a lattice per set, remark after eq. d3q15)
    keep the set a = 0 on D2Q5 / D3Q7: 5 + 2 x 9 and 7 + 3 x 15 planes per
    buffer, against (d + 1) q for D2Q9 / D3Q15."""
    for spec, pure, mixed, saved in ((C.cavity_case(N=256, Re=100), mdf.D2Q9, mdf.D2Q9_Q5, 9 - 5),
                                     (C.tgv3d_case(N=64, u0=0.05, Re=100.0), mdf.D3Q15, mdf.D3Q15_Q7, 15 - 7)):
        c = (mdf.MdfCase * 1)(mdf._case_struct(spec))
        full = mdf.lib().mdf_workspace_size(pure, mdf.F32, c, 1, 0)
        per_set = mdf.lib().mdf_workspace_size(mixed, mdf.F32, c, 1, 0)
        plane = 2 * spec.nodes * 4                    # one plane, both buffers, FP32
        assert full - per_set == pytest.approx(saved * plane, rel=0.02)
    c3 = (mdf.MdfCase * 1)(mdf._case_struct(C.tgv3d_case(N=16, u0=0.05, Re=100.0)))
    assert mdf.lib().mdf_workspace_size(mdf.D2Q9_Q5, mdf.F32, c3, 1, 0) == 0


@pytest.mark.parametrize("mutate,msg", [
    (lambda s: setattr(s, "s1", 2.0), "s1"),
    (lambda s: setattr(s, "s1", 0.0), "s1"),
    (lambda s: setattr(s, "bc", (0, 1, 0, 0, 0, 0)), "periodic"),
    (lambda s: setattr(s, "shape", (0, 8)), "grid"),
    (lambda s: setattr(s, "rho0", -1.0), "rho0"),
])
def test_invalid_cases_are_rejected(mutate, msg):
    spec = C.cavity_case(N=16, Re=10)
    mutate(spec)
    assert _ws(spec) == 0
    err = mdf.lib().mdf_last_error(None).decode()
    assert msg in err


def test_init_rejects_before_touching_the_device():
    L = mdf.lib()
    spec = C.cavity_case(N=16, Re=10)
    cases = (mdf.MdfCase * 1)(mdf._case_struct(spec))
    ctx = ctypes.c_void_p()
    # NULL workspace
    st = L.mdf_init(ctypes.byref(ctx), mdf.D2Q5, mdf.F32, cases, 1, None, 0, None, 0, None, None)
    assert st == mdf.EINVAL and not ctx.value
    # misaligned workspace
    st = L.mdf_init(ctypes.byref(ctx), mdf.D2Q5, mdf.F32, cases, 1, ctypes.c_void_p(16), 1 << 30,
                    None, 0, None, None)
    assert st == mdf.EINVAL and "aligned" in L.mdf_last_error(None).decode()
    # workspace too small
    st = L.mdf_init(ctypes.byref(ctx), mdf.D2Q5, mdf.F32, cases, 1, ctypes.c_void_p(256), 1024,
                    None, 0, None, None)
    assert st == mdf.ENOMEM
    # bad lattice / storage / init kind
    assert L.mdf_init(ctypes.byref(ctx), 14, mdf.F32, cases, 1, ctypes.c_void_p(256), 1 << 30,
                      None, 0, None, None) == mdf.EINVAL
    assert L.mdf_init(ctypes.byref(ctx), mdf.D2Q5, 9, cases, 1, ctypes.c_void_p(256), 1 << 30,
                      None, 0, None, None) == mdf.EINVAL
    assert L.mdf_init(ctypes.byref(ctx), mdf.D2Q5, mdf.F32, cases, 1, ctypes.c_void_p(256), 1 << 30,
                      None, 1, None, None) == mdf.EINVAL
    # D2Q5 case with nz != 1
    bad = (mdf.MdfCase * 1)(mdf._case_struct(spec))
    bad[0].nz = 2
    assert L.mdf_init(ctypes.byref(ctx), mdf.D2Q5, mdf.F32, bad, 1, ctypes.c_void_p(256), 1 << 30,
                      None, 0, None, None) == mdf.EINVAL


def test_null_context_calls_fail_cleanly():
    L = mdf.lib()
    assert L.mdf_state_size(None) == 0
    assert L.mdf_save(None, None, 0, None) == mdf.EINVAL
    assert L.mdf_load(None, None, 0, None) == mdf.EINVAL
    assert L.mdf_step(None, 1, None) == mdf.EINVAL
    assert L.mdf_set_launch(None, 64, 4, 8, 1) == mdf.EINVAL
    assert L.mdf_time(None, 0) == -1
    stats = (ctypes.c_int64 * 4)()
    assert L.mdf_graph_stats(None, stats, None) == mdf.EINVAL
    ptr, nbytes = ctypes.c_void_p(), ctypes.c_size_t()
    assert L.mdf_population_buffer(None, 0, 0, ctypes.byref(ptr), ctypes.byref(nbytes)) == mdf.EINVAL
    assert L.mdf_destroy(None) == mdf.OK


def test_field_layout_channel_counts():
    assert mdf.n_channels(2, mdf.FIELD_ALL) == 4 + 4 + 1 + 3 + 3 + 1
    assert mdf.n_channels(3, mdf.FIELD_ALL) == 5 + 9 + 1 + 6 + 6 + 3
    assert mdf.n_channels(2, mdf.FIELD_VORT | mdf.FIELD_STRAIN) == 4
