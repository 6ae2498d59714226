"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, validates arguments before touching the device, and its host
helpers agree with the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1511_00242_amd import inputs as I
from paper_1511_00242_amd import lbfv as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbfv.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert "lbfv_create" in names and "dugks_step" in names and "bkg_step" in names
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_strerror_covers_every_status():
    for s in range(0, -7, -1):
        assert L.lib().lbfv_strerror(s) not in (b"", b"unknown status")


def _mesh(nx=8, ny=6):
    return I.uniform_faces(nx), I.uniform_faces(ny)


@pytest.mark.parametrize("bad", [
    dict(nx=1), dict(ny=1), dict(tau=0.0), dict(tau=-1.0), dict(dt=0.0), dict(rt=0.0),
    dict(q=19), dict(nonmono=True), dict(compute=0, storage=2), dict(compute=0, storage=1),
    dict(compute=7),
])
def test_create_rejects_bad_arguments(bad):
    nx, ny = bad.get("nx", 8), bad.get("ny", 6)
    xf, yf = I.uniform_faces(nx), I.uniform_faces(ny)
    if bad.get("nonmono"):
        xf = xf.copy(); xf[3] = xf[2]
    m = L._Mesh(nx, ny, L._p(xf), L._p(yf))
    v = L._Velset(bad.get("q", 9), bad.get("rt", 1 / 3))
    o = L._Opts(bad.get("compute", 0), bad.get("storage", 0), 1.0, 100, None)
    h = C.c_void_p()
    st = L.lib().lbfv_create(C.byref(m), C.byref(v), bad.get("tau", 0.1), bad.get("dt", 0.01),
                             C.byref(o), C.byref(h))
    assert st == L.LBFV_EINVAL
    assert not h.value
    assert L.lib().lbfv_last_error(None)


def test_null_pointers_are_rejected():
    lib = L.lib()
    assert lib.lbfv_create(None, None, 0.1, 0.1, None, None) == L.LBFV_EINVAL
    assert lib.lbfv_destroy(None) == L.LBFV_EINVAL
    assert lib.dugks_step(None, 1) == L.LBFV_EINVAL
    assert lib.bkg_step(None, 1) == L.LBFV_EINVAL
    assert lib.lbfv_batch_create(0, None, None, None, None) == L.LBFV_EINVAL
    assert lib.lbfv_batch_nonfinite(None, None) == L.LBFV_EINVAL
    assert lib.lbfv_batch_autotune(None, 0, 10, None) == L.LBFV_EINVAL
    assert lib.lbfv_batch_get_shape(None, None, None) == L.LBFV_EINVAL
    assert lib.lbfv_batch_set_time_block(None, 2) == L.LBFV_EINVAL
    assert lib.lbfv_batch_get_time_block(None, None) == L.LBFV_EINVAL
    assert lib.lbfv_batch_set_grid_form(None, 1) == L.LBFV_EINVAL
    assert lib.lbfv_batch_get_grid_form(None, None) == L.LBFV_EINVAL
    assert lib.lbfv_batch_last_error(None) is not None


def test_state_errors_before_any_device_work():
    xf, yf = _mesh()
    ctx = L.Context(xf, yf, 0.1, 0.01)
    # sides unset -> ESTATE
    assert L.lib().dugks_step(ctx.h, 1) == L.LBFV_ESTATE
    ctx.set_sides(["periodic"] * 4)
    # no state -> ESTATE
    assert L.lib().bkg_step(ctx.h, 1) == L.LBFV_ESTATE
    with pytest.raises(L.LbfvError) as e:
        ctx.dugks_step(1)
    assert e.value.status == L.LBFV_ESTATE
    # bad setter arguments
    assert L.lib().lbfv_set_wall(ctx.h, 7, 0.0, 0.0) == L.LBFV_EINVAL
    assert L.lib().lbfv_set_outflow_extrap(ctx.h, 0, 2) == L.LBFV_EINVAL
    assert L.lib().lbfv_set_inflow_eq(ctx.h, 0, -1.0, 0.0, 0.0) == L.LBFV_EINVAL
    assert L.lib().lbfv_set_periodic(ctx.h, 5) == L.LBFV_EINVAL
    assert L.lib().lbfv_set_tile(ctx.h, 8, 3) == L.LBFV_EINVAL
    assert L.lib().lbfv_set_time_block(ctx.h, 5) == L.LBFV_EINVAL
    assert L.lib().lbfv_set_time_block(ctx.h, 0) == L.LBFV_EINVAL
    assert L.lib().lbfv_set_time_block(ctx.h, 4) == L.LBFV_EINVAL   # 8 x 6 mesh: 4 steps need 8 per side
    L._check(L.lib().lbfv_set_time_block(ctx.h, 3), ctx.h)      # periodic, no state yet
    L._check(L.lib().lbfv_set_time_block(ctx.h, 2), ctx.h)
    L._check(L.lib().lbfv_set_time_block(ctx.h, 1), ctx.h)
    assert L.lib().lbfv_set_wave_pairs(ctx.h, 2) == L.LBFV_EINVAL
    assert ctx.get_wave_pairs() is False
    ctx.set_wave_pairs(True)
    assert ctx.get_wave_pairs() is True
    ctx.set_wave_pairs(False)
    assert L.lib().lbfv_get_wave_pairs(ctx.h, None) == L.LBFV_EINVAL
    # the allocation-free totals need a state (and the mesh metrics on the device)
    assert L.lib().lbfv_totals_device(ctx.h, None) == L.LBFV_EINVAL
    assert L.lib().lbfv_totals_device(None, None) == L.LBFV_EINVAL
    assert L.lib().dugks_step(ctx.h, -1) == L.LBFV_EINVAL
    assert L.lib().lbfv_step(ctx.h, 4, 1) == L.LBFV_EINVAL
    assert L.lib().lbfv_step(ctx.h, -1, 1) == L.LBFV_EINVAL
    assert L.lib().lbfv_step(ctx.h, L.LBFV_UPWIND, 1) == L.LBFV_ESTATE    # no state yet
    # symmetry sides and wall segments
    assert L.lib().lbfv_set_symmetry(ctx.h, 4) == L.LBFV_EINVAL
    assert L.lib().lbfv_set_wall_from(ctx.h, L.LBFV_WEST, 2, 0.0, 0.0) == L.LBFV_EINVAL   # x-side
    assert L.lib().lbfv_set_wall_from(ctx.h, L.LBFV_SOUTH, 2, 0.0, 0.0) == L.LBFV_EINVAL  # periodic side
    L._check(L.lib().lbfv_set_symmetry(ctx.h, L.LBFV_SOUTH), ctx.h)
    assert L.lib().lbfv_set_wall_from(ctx.h, L.LBFV_SOUTH, 8, 0.0, 0.0) == L.LBFV_EINVAL  # past nx - 1
    assert L.lib().lbfv_set_wall_from(ctx.h, L.LBFV_SOUTH, -1, 0.0, 0.0) == L.LBFV_EINVAL
    L._check(L.lib().lbfv_set_wall_from(ctx.h, L.LBFV_SOUTH, 3, 0.01, 0.0), ctx.h)
    assert L.lib().dugks_step(ctx.h, 1) == L.LBFV_ESTATE      # north left unset by the switch
    assert L.lib().lbfv_set_time_block(ctx.h, 2) == L.LBFV_EINVAL  # a side is unset
    ctx.set_sides(["periodic"] * 4)
    # replacing one side of a periodic axis leaves the other side unset
    L._check(L.lib().lbfv_set_wall(ctx.h, L.LBFV_WEST, 0.0, 0.0), ctx.h)
    assert L.lib().dugks_step(ctx.h, 1) == L.LBFV_ESTATE
    L._check(L.lib().lbfv_set_wall(ctx.h, L.LBFV_EAST, 0.0, 0.0), ctx.h)
    assert L.lib().lbfv_set_time_block(ctx.h, 3) == L.LBFV_EINVAL   # walls: at most two steps per launch
    L._check(L.lib().lbfv_set_time_block(ctx.h, 2), ctx.h)
    # the reference velocity belongs to deviation storage
    assert L.lib().lbfv_set_reference_velocity(ctx.h, 0.1, 0.0) == L.LBFV_EINVAL
    ctx.close()


def test_reference_velocity_setter():
    xf, yf = _mesh()
    ctx = L.Context(xf, yf, 0.1, 0.01, compute=L.LBFV_FP32, storage=L.LBFV_STORE_DEV_FP32)
    assert L.lib().lbfv_set_reference_velocity(ctx.h, float("nan"), 0.0) == L.LBFV_EINVAL
    assert ctx.get_reference_velocity() == (0.0, 0.0)
    ctx.set_reference_velocity(0.1, 0.0)          # no state yet: nothing to re-encode
    assert ctx.get_reference_velocity() == (0.1, 0.0)
    ctx.set_sides(["periodic", "periodic", "symmetry", "symmetry"])
    assert L.lib().dugks_step(ctx.h, 1) == L.LBFV_ESTATE        # no state
    assert "initial state" in L.lib().lbfv_last_error(ctx.h).decode()
    ctx.set_reference_velocity(0.1, 0.02)         # normal to the symmetry sides
    assert L.lib().dugks_step(ctx.h, 1) == L.LBFV_ESTATE
    assert "symmetry" in L.lib().lbfv_last_error(ctx.h).decode()
    ctx.close()


def test_required_bytes_layout():
    xf, yf = I.uniform_faces(100), I.uniform_faces(7)
    for compute, storage, esize in ((0, 0, 8), (1, 0, 4), (1, 1, 4), (1, 2, 2), (1, 3, 2)):
        ctx = L.Context(xf, yf, 0.1, 0.01, compute=compute, storage=storage)
        assert ctx.required_bytes() == 9 * 7 * 128 * esize   # two 62-column strips, 64 slots each
        ctx.close()


def test_dt_from_cfl_matches_oracle():
    from oracle import oracle as O
    for xf, yf in ((I.uniform_faces(32, 0, 6.28), I.uniform_faces(32, 0, 6.28)),
                   (I.tanh_faces(40, 2.0), I.geometric_faces(30, 0.01, 2.0))):
        for cfl in (0.5, 1.1):
            assert L.dt_from_cfl(xf, yf, 1 / 3, cfl) == pytest.approx(O.dt_from_cfl(xf, yf, 1 / 3, cfl),
                                                                       rel=1e-15)
    with pytest.raises(L.LbfvError):
        L.dt_from_cfl(xf, yf, -1.0, 0.5)
