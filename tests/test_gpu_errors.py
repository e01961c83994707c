"""Error paths of the C-ABI: argument errors returned synchronously and
device-side failures reported by last_status.  Every kernel launched here
exits normally: the bad cells only make the bounded Newton solve fail or
leave the fit range, which sets the context's error word."""
import ctypes

import numpy as np
import pytest

from synth import fields, mechanism

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1309_7327_amd import narrowsdc as N  # noqa: E402
import gpu_util as G  # noqa: E402

L = N._lib
SHAPE = (6, 7, 8)
DX = 1e-4


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.fixture(scope="module")
def good():
    m = mechanism.load("mech9")
    ctx = N.Context(0)
    ctx.set_mechanism(m)
    prim = fields.sines(SHAPE, DX, 9, 3)
    bx, U = G.device_state(ctx, prim, DX)
    yield m, ctx, bx, U
    ctx.close()


def test_rhs_eval_before_set_mechanism_is_enomech():
    ctx = N.Context(0)
    bx = N.box(8, 7, 6, DX)
    U = torch.zeros(N.ghosted_shape(14, 6, 7, 8), dtype=torch.float64, device="cuda")
    F = torch.zeros((14, 6, 7, 8), dtype=torch.float64, device="cuda")
    assert L.rhs_eval(ctx.h, ctypes.byref(bx), _ptr(U), _ptr(F), N.RHS_ALL, _stream()) == N.SDC_ENOMECH
    sch = N.scheme(4, 2, 0, 1)
    n = ctypes.c_size_t()
    assert L.sdc_workspace_size(ctx.h, 1, ctypes.byref(bx), ctypes.byref(sch), ctypes.byref(n)) == N.SDC_ENOMECH
    assert L.sdc_step(ctx.h, ctypes.byref(bx), _ptr(U), 1e-9, 1, ctypes.byref(sch), _ptr(U), 8,
                      _stream()) == N.SDC_ENOMECH
    assert b"mechanism" in L.last_error_message(ctx.h)
    ctx.close()


def test_bad_arguments_are_einval(good):
    m, ctx, bx, U = good
    F = torch.zeros((14,) + SHAPE, dtype=torch.float64, device="cuda")
    s = _stream()
    for bad in (N.BoxDesc(8, 7, 6, 3, DX, DX, DX),      # ghost layers must be 4
                N.BoxDesc(0, 7, 6, 4, DX, DX, DX),      # empty box
                N.BoxDesc(8, -1, 6, 4, DX, DX, DX),
                N.BoxDesc(8, 7, 6, 4, 0.0, DX, DX),     # non-positive spacing
                N.BoxDesc(8, 7, 6, 4, DX, DX, float("nan"))):
        assert L.rhs_eval(ctx.h, ctypes.byref(bad), _ptr(U), _ptr(F), N.RHS_ALL, s) == N.SDC_EINVAL
    assert L.rhs_eval(ctx.h, ctypes.byref(bx), None, _ptr(F), N.RHS_ALL, s) == N.SDC_EINVAL
    assert L.rhs_eval(ctx.h, ctypes.byref(bx), _ptr(U), None, N.RHS_ALL, s) == N.SDC_EINVAL
    assert L.rhs_eval(ctx.h, None, _ptr(U), _ptr(F), N.RHS_ALL, s) == N.SDC_EINVAL
    assert L.rhs_eval(ctx.h, ctypes.byref(bx), _ptr(U), _ptr(F), 0, s) == N.SDC_EINVAL
    assert L.rhs_eval(ctx.h, ctypes.byref(bx), _ptr(U), _ptr(F), 8, s) == N.SDC_EINVAL
    assert L.rhs_eval(None, ctypes.byref(bx), _ptr(U), _ptr(F), N.RHS_ALL, s) == N.SDC_EINVAL
    sch = N.scheme(4, 2, 0, 1)
    ws, nb = N.workspace(ctx, [bx], sch)
    assert L.sdc_step(ctx.h, ctypes.byref(bx), _ptr(U), -1e-9, 1, ctypes.byref(sch), _ptr(ws), nb,
                      s) == N.SDC_EINVAL
    assert L.sdc_step(ctx.h, ctypes.byref(bx), _ptr(U), 1e-9, 0, ctypes.byref(sch), _ptr(ws), nb,
                      s) == N.SDC_EINVAL
    assert L.sdc_step(ctx.h, ctypes.byref(bx), _ptr(U), 1e-9, 1, ctypes.byref(sch), None, nb,
                      s) == N.SDC_EINVAL
    assert L.sdc_step(ctx.h, ctypes.byref(bx), _ptr(U), 1e-9, 1, ctypes.byref(sch), _ptr(ws), nb - 8,
                      s) == N.SDC_ENOMEM
    bad_sch = N.scheme(1, 2, 0, 1)
    assert L.sdc_step(ctx.h, ctypes.byref(bx), _ptr(U), 1e-9, 1, ctypes.byref(bad_sch), _ptr(ws), nb,
                      s) == N.SDC_EINVAL
    # tile shapes: each all zero (automatic) or all positive, at most 256
    # threads, the interior one whole waves
    for bad in ((64, 0, 1, 0, 0, 0, 0), (0, 0, 0, 16, 0, 16, 0), (64, 4, -1, 0, 0, 0, 0),
                (64, 8, 1, 0, 0, 0, 0), (32, 3, 1, 0, 0, 0, 0), (0, 0, 0, 0, 0, 0, -1)):
        assert L.sdc_set_tiles(ctx.h, *bad) == N.SDC_EINVAL
    # nothing was launched by the rejected calls: the state is intact
    ctx.check_status()


def _with_bad_cell(U, kind):
    V = U.clone()
    i, j, k = 4 + 3, 4 + 2, 4 + 1           # an interior cell (ghosted indices)
    rho = V[0, i, j, k].item()
    ke = 0.5 * (V[1, i, j, k] ** 2 + V[2, i, j, k] ** 2 + V[3, i, j, k] ** 2).item() / rho
    if kind == "energy_below_kinetic":
        # rho E below the kinetic energy by 1e8 J/kg: E includes the
        # formation enthalpies, so e < 0 alone can be a valid state; this e
        # lies far below e(T_lo) of any mixture
        V[1, i, j, k] = rho * 400.0
        V[4, i, j, k] = 0.5 * rho * 400.0 ** 2 - rho * 1e8
    elif kind == "negative_density":
        V[0, i, j, k] = -rho
    elif kind == "nan":
        V[4, i, j, k] = float("nan")
    elif kind == "too_hot":
        V[4, i, j, k] = rho * 1e8 + ke * rho    # far above the fit range's energy
    return V


@pytest.mark.parametrize("kind", ["energy_below_kinetic", "negative_density", "nan", "too_hot"])
def test_bad_cells_set_etemp(good, kind):
    m, ctx, bx, U = good
    F = torch.zeros((14,) + SHAPE, dtype=torch.float64, device="cuda")
    assert ctx.last_status() == N.SDC_OK
    V = _with_bad_cell(U, kind)
    ctx.rhs_eval(bx, V, F, N.RHS_ALL)           # the call itself is accepted
    assert ctx.last_status() == N.SDC_ETEMP
    assert b"device error flags" in L.last_error_message(ctx.h)
    assert ctx.last_status() == N.SDC_OK        # the error word was cleared
    # the same through a time step
    sch = N.scheme(4, 2, 0, 1)
    ws, nb = N.workspace(ctx, [bx], sch)
    V = _with_bad_cell(U, kind)
    ctx.sdc_step(bx, V, 1e-9, 1, sch, ws, nb)
    assert ctx.last_status() == N.SDC_ETEMP
    # and a good state afterwards reports nothing
    ctx.rhs_eval(bx, U.clone(), F, N.RHS_ALL)
    assert ctx.last_status() == N.SDC_OK
    assert torch.isfinite(F).all()
