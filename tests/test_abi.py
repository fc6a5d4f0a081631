"""C ABI checks that need no GPU: the library loads, exports every entry point
the header declares, validates parameters and computes its plan on the host."""
import ctypes
import math
import os
import re

import pytest

from paper_2105_10517_amd import binding, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gp_spin1.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(gp_spin1_\w+)\s*\(", src, re.M)))


def test_header_matches_binding_exports():
    assert declared() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for name in declared():
        assert hasattr(lib, name), name


def test_strerror_covers_every_status():
    lib = binding.load()
    seen = set()
    for st in range(0, -7, -1):
        msg = lib.gp_spin1_strerror(st).decode()
        assert msg and msg != "unknown status"
        seen.add(msg)
    assert len(seen) == 7


BASE = inputs.params(64, 48, 0.1, dt=1e-3, c0=10.0, c2=-1.0, gamma=0.5, omega=0.3)


@pytest.mark.parametrize("change,status", [
    ({"nx": 2}, binding.GP_EINVAL), ({"ny": 1}, binding.GP_EINVAL),
    ({"dx": 0.0}, binding.GP_EINVAL), ({"dy": -0.1}, binding.GP_EINVAL),
    ({"dt": 0.0}, binding.GP_EINVAL), ({"dt": math.inf}, binding.GP_EINVAL),
    ({"c0": math.nan}, binding.GP_EINVAL), ({"eta": 0}, binding.GP_EINVAL),
    ({"omega": math.inf}, binding.GP_EINVAL), ({"x0": math.inf}, binding.GP_EINVAL),
    ({"nx": 9000}, binding.GP_EUNSUPPORTED),
])
def test_validation(change, status):
    p = dict(BASE, **change)
    with pytest.raises(binding.GPError) as ei:
        binding.plan_query(p, True)
    assert ei.value.status == status


def test_plan_of_the_workloads():
    c1 = binding.plan_query(inputs.config_c1(), True)
    assert c1["stable"] == 1 and c1["y_solver"] == binding.GP_YSOLVER_WINDOW and c1["y_halo"] == 0
    c2 = binding.plan_query(inputs.config_c2(), False)
    assert c2["stable"] == 1 and c2["y_solver"] == binding.GP_YSOLVER_WINDOW
    # the window halo makes decay^h fall below 2^-60
    assert c2["decay_y"] ** c2["y_halo"] < 2.0 ** -60
    assert c2["y_rows_out"] == c2["y_segments"] * c2["y_rows_per_thread"] - 2 * c2["y_halo"]
    for prec in ("fp64", "fp32"):
        # large grids: chain x windows (two points per lane in FP64, where they
        # write 3/4 of what they load; four in FP32) and stacked y windows by default
        c3 = binding.plan_query(inputs.config_c3(4096), True, prec)
        assert c3["stable"] == 1 and c3["y_solver"] == binding.GP_YSOLVER_STACK and c3["y_segments"] == 16
        kx = 2 if prec == "fp64" else 4
        assert c3["x_solver"] == binding.GP_XSOLVER_CHAIN and c3["x_points_per_thread"] == kx
        assert c3["x_points_out"] == 64 * kx - 2 * c3["x_halo"] and c3["decay_x"] ** c3["x_halo"] < 2.0 ** -32
        assert 4 * c3["x_points_out"] >= 3 * 64 * kx
        # and the scanned windows / whole rows when asked for
        w = binding.plan_query(inputs.config_c3(4096), True, prec, y_solver="window", x_solver="scan")
        assert w["y_solver"] == binding.GP_YSOLVER_WINDOW and w["x_solver"] == binding.GP_XSOLVER_SCAN
        assert w["x_points_per_thread"] * w["x_threads_per_row"] >= 4096
    th = binding.plan_query(inputs.config_c2(), False, y_solver="thomas")
    assert th["y_solver"] == binding.GP_YSOLVER_THOMAS


def test_decay_matches_closed_form():
    # imaginary time without rotation or SO: (I + a h) has b = 1 + beta, a = e = -beta/2
    # (beta = dt/(2 dx^2)); the converged Thomas multiplier is the small root of
    # beta/2 r^2 - (1 + beta) r + beta/2 = 0
    dx, dt = 0.1, 1e-3
    p = inputs.params(64, 64, dx, dt=dt)
    pl = binding.plan_query(p, True)
    beta = dt / (2 * dx * dx)
    r = ((1 + beta) - math.sqrt((1 + beta) ** 2 - beta * beta)) / beta
    assert abs(pl["decay_x"] - r) < 1e-14 and abs(pl["decay_y"] - r) < 1e-14


def test_stability_checks():
    # imaginary-time Cayley bound (dt/4)(|Omega| L + |gamma|)^2 < 1
    p = inputs.params(64, 64, 0.3, dt=0.05, omega=0.9, gamma=1.0)
    assert binding.plan_query(p, True)["stable"] == 0 and binding.plan_query(p, False)["stable"] == 1
    # real time with a huge dt and strong rotation loses diagonal dominance
    q = inputs.params(64, 64, 0.1, dt=5.0, omega=5.0)
    assert binding.plan_query(q, False)["stable"] == 0
    assert binding.plan_query(inputs.config_c2(), False)["stable"] == 1


def test_batch_create_validates_before_touching_the_device():
    import ctypes
    lib = binding.load()
    out = ctypes.c_void_p()
    # no parameter array, or no output pointer
    assert lib.gp_spin1_batch_create(None, 2, None, ctypes.byref(out)) == binding.GP_EINVAL
    arr = (binding.Params * 2)(binding.make_params(BASE, "fp64"), binding.make_params(BASE, "fp32"))
    # slots of different precision
    assert lib.gp_spin1_batch_create(arr, 2, None, ctypes.byref(out)) == binding.GP_EINVAL
    # empty batch
    assert lib.gp_spin1_batch_create(arr, 0, None, ctypes.byref(out)) == binding.GP_EINVAL
    # null handles
    assert lib.gp_spin1_batch_step(None, None, None, None, None) == binding.GP_EINVAL
    assert lib.gp_spin1_batch_destroy(None) == binding.GP_EINVAL
    assert lib.gp_spin1_batch_last_error(None).decode() == "null batch"


@pytest.mark.parametrize("change", [
    {"fix_m": 1, "magnetization": 0.2},                       # gamma != 0 in BASE
    {"fix_m": 1, "magnetization": 1.0, "gamma": 0.0},         # |m| must be < 1
    {"split": 2}, {"gx": -1.0}, {"gy": math.inf},
])
def test_validation_of_the_next_row_options(change):
    p = dict(BASE, **change)
    with pytest.raises(binding.GPError) as ei:
        binding.plan_query(p, True)
    assert ei.value.status == binding.GP_EINVAL


def test_block_orders_of_the_windowed_sweeps():
    # default: x windows grouped by XCD, y windows grouped only on grids of about one wave of blocks
    small = binding.plan_query(inputs.config_c2(), False, x_solver="window")
    assert small["x_solver"] == binding.GP_XSOLVER_WINDOW and small["x_block_order"] == 1
    assert small["y_block_order"] == 1
    big = binding.plan_query(inputs.config_c3(4096), True, y_solver="window", x_solver="scan")
    assert big["y_solver"] == binding.GP_YSOLVER_WINDOW and big["y_block_order"] == 0
    assert big["x_block_order"] == 0  # whole-row x sweep: no windows to order
    chain = binding.plan_query(inputs.config_c3(4096), True)  # chain x and stacked y windows
    assert chain["x_block_order"] == 1 and chain["y_block_order"] == 0
    for order, wx, wy in (("hardware", 0, 0), ("xcd", 1, 1), ("bands", 1, 2), ("rows", 3, 3)):
        for p, imag in ((inputs.config_c2(), False), (inputs.config_c3(4096), True)):
            pl = binding.plan_query(p, imag, x_solver="window", block_order=order)
            assert pl["x_block_order"] == wx and pl["y_block_order"] == wy
    # row bands on the whole-row x sweep
    pl = binding.plan_query(inputs.config_c2(), False, block_order="rows")
    assert pl["x_solver"] == binding.GP_XSOLVER_SCAN and pl["x_block_order"] == 3 and pl["y_block_order"] == 3
    bad = binding.make_params(BASE)
    bad.block_order = 5
    pl = binding.Plan()
    assert binding.load().gp_spin1_plan_query(ctypes.byref(bad), 1, ctypes.byref(pl)) == binding.GP_EINVAL


def test_tile_options():
    p = dict(BASE, nx=700, ny=600, dx=0.1, dy=0.1)
    for t in range(1, 9):
        pl = binding.plan_query(p, True, x_solver="window", x_tile=t, y_tile=t)
        assert pl["x_tile"] == t and pl["y_tile"] == t
    lib, pl = binding.load(), binding.Plan()
    for field, value in (("x_tile", 9), ("x_tile", -1), ("y_tile", 9)):
        q = binding.make_params(p, x_solver="window")
        setattr(q, field, value)
        assert lib.gp_spin1_plan_query(ctypes.byref(q), 1, ctypes.byref(pl)) == binding.GP_EINVAL, (field, value)
    # a tile for the x windows without the x windows
    q = binding.make_params(p, x_tile=2)
    assert lib.gp_spin1_plan_query(ctypes.byref(q), 1, ctypes.byref(pl)) == binding.GP_EINVAL


def test_plane_stride_validation():
    n = BASE["nx"] * BASE["ny"]
    for stride in (0, n, n + 4160):
        binding.plan_query(dict(BASE, plane_stride=stride), True)
    for stride in (n - 1, -5):
        with pytest.raises(binding.GPError) as ei:
            binding.plan_query(dict(BASE, plane_stride=stride), True)
        assert ei.value.status == binding.GP_EINVAL


def test_unit_helper_reproduces_the_printed_couplings():
    # Eq. (S.4) with the paper's 87Rb / 23Na inputs (l0 / sqrt(kappa) = 4 micrometres)
    import json
    from paper_2105_10517_amd import units
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "couplings_rb87_na23.json")))
    for c in g["cases"]:
        for kappa in (1.0, 20.0):
            l0 = g["l0_over_sqrt_kappa_m"] * math.sqrt(kappa)
            c0, c2 = units.couplings(c["N"], c["a0_bohr"], c["a2_bohr"], l0, kappa)
            assert round(c0, c["c0_digits"]) == c["c0_printed"]
            assert round(c2, c["c2_digits"]) == c["c2_printed"]
    # oscillator length of 87Rb in a 2 pi x 20 Hz trap: about 2.4 micrometres
    assert abs(units.oscillator_length(86.909 * 1.66053906660e-27, 2 * math.pi * 20.0) - 2.41e-6) < 0.02e-6


def test_check_psi_refuses_host_and_misshaped_tensors():
    torch = pytest.importorskip("torch")
    p = {"nx": 8, "ny": 6}
    with pytest.raises(ValueError):
        binding.check_psi(torch.zeros((3, 6, 8), dtype=torch.complex128), torch.complex128, p)
    with pytest.raises(ValueError):
        binding.check_psi(torch.zeros((3, 8, 6), dtype=torch.complex128), torch.complex128, p)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_row_band_tiles_split_evenly_over_the_xcds(precision):
    # under row bands the y row tile shrinks so that the number of row tiles is
    # a multiple of the 8 XCDs; the window span stays, the halo grows
    for n in (512, 700, 2048):
        p = inputs.params(n, n, 0.05, dt=1e-4, c0=200.0, c2=5.0, gamma=1.0, eta=-1, rabi=0.2, omega=0.9)
        for imag in (False, True):
            base = binding.plan_query(p, imag, precision=precision, block_order="hardware")
            rows = binding.plan_query(p, imag, precision=precision, block_order="rows")
            if base["y_solver"] != binding.GP_YSOLVER_WINDOW or base["y_rows_out"] >= n:
                continue
            nrt = -(-n // rows["y_rows_out"])
            assert nrt % 8 == 0 or nrt < 8, (n, imag, rows["y_rows_out"])
            assert rows["y_rows_out"] <= base["y_rows_out"] and rows["y_halo"] >= base["y_halo"]
            span = 16 * rows["y_rows_per_thread"]
            assert rows["y_halo"] + rows["y_rows_out"] <= span
            assert span - rows["y_halo"] - rows["y_rows_out"] >= base["y_halo"]


def test_size_limits():
    # the longest row the whole-row x sweep holds on chip is 8192 points; a grid
    # of more than 4e9 values (3 nx ny) is refused
    ok = inputs.params(8192, 16, 0.01, dt=1e-5)
    assert binding.plan_query(ok, True)["stable"] == 1
    for nx, ny in ((8193, 16), (8192, 170000)):
        with pytest.raises(binding.GPError) as ei:
            binding.plan_query(inputs.params(nx, ny, 0.01, dt=1e-5), True)
        assert ei.value.status == binding.GP_EUNSUPPORTED
