"""Parity of the gfx950 HIP path (called through the C ABI) with the FP64 CPU
oracle, element by element on the same seeded inputs.

Tolerances: FP64 substeps 1e-13 relative L2 (rounding only); FP64 full runs
1e-10 relative L2 on psi after up to 1000 steps; FP32 bulk: density 1e-5
relative to the peak density, chemical potential 1e-6 relative.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2105_10517_amd import binding, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def gpu_run(p, psi0, nsteps, imag, precision="fp64", y_solver="auto", autotune=False):
    s = binding.Solver(p, precision, y_solver, autotune=autotune)
    t = dev(psi0, s.dtype)
    (s.step_imag if imag else s.step_real)(t, nsteps)
    s.sync()
    out = host(t)
    obs = s.observables(t)
    s.close()
    return out, obs


def all_couplings(nx, ny, dx, dy=None, dt=0.01, eta=1, **kw):
    base = dict(c0=35.0, c2=-3.0, gamma=0.6, eta=eta, rabi=0.25, omega=0.45)
    base.update(kw)
    return inputs.params(nx, ny, dx, dy=dy, dt=dt, **base)


# ---------------------------------------------------------------------------
# Substeps on random input
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("imag", [True, False])
def test_local_substep(imag):
    p = all_couplings(53, 37, 0.21, dt=0.02)
    psi = inputs.random_state(53, 37, seed=21, scale=0.6)
    s = binding.Solver(p)
    t = dev(psi)
    s.substep(t, binding.SUB_LOCAL, imag)
    got = host(t)
    want = oracle.pointwise(p, psi, imag)
    assert rel(got, want) < 1e-13


@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("nx", [3, 53, 128, 130, 700, 1024, 1500, 4096, 5000, 8192])
def test_x_sweep(imag, nx):
    ny = 5
    p = all_couplings(nx, ny, 24.0 / nx + 0.001, dy=0.2, dt=0.004, eta=-1 if nx % 2 else 1)
    psi = inputs.random_state(nx, ny, seed=nx)
    s = binding.Solver(p)
    t = dev(psi)
    s.substep(t, binding.SUB_X, imag)
    got = host(t)
    want = oracle.sweep_x(p, psi, imag)
    assert rel(got, want) < 1e-13, s.plan(imag)


@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("nx", [3, 53, 128, 131, 700, 1024, 4096])
def test_x_sweep_windows(imag, nx):
    # truncated windows along the rows: one window (no halo) up to 16 KX points, overlapping windows beyond
    p = all_couplings(nx, 5, 0.05, dy=0.2, dt=0.001, eta=-1 if nx % 2 else 1)
    psi = inputs.random_state(nx, 5, seed=nx + 7)
    s = binding.Solver(p, x_solver="window")
    assert s.plan(imag)["x_solver"] == binding.GP_XSOLVER_WINDOW
    t = dev(psi)
    s.substep(t, binding.SUB_X, imag)
    got = host(t)
    want = oracle.sweep_x(p, psi, imag)
    assert rel(got, want) < 1e-13, s.plan(imag)


@pytest.mark.parametrize("tile", range(1, 9))
def test_every_window_tile(tile):
    # each tile shape of both windowed sweeps (5..8 solve the three lines one at a time), several windows
    # per line and a ragged last window, both propagation modes
    for imag in (True, False):
        p = all_couplings(700, 5, 0.1, dy=0.2, dt=0.001)
        psi = inputs.random_state(700, 5, seed=40 + tile)
        s = binding.Solver(p, x_solver="window", x_tile=tile)
        pl = s.plan(imag)
        assert pl["x_tile"] == tile and pl["x_points_out"] < 700
        t = dev(psi)
        s.substep(t, binding.SUB_X, imag)
        assert rel(host(t), oracle.sweep_x(p, psi, imag)) < 1e-13, (tile, imag, pl)
        s.close()
        q = all_couplings(9, 600, 0.2, dy=0.1, dt=0.001)
        psi = inputs.random_state(9, 600, seed=50 + tile)
        s = binding.Solver(q, y_tile=tile)
        pl = s.plan(imag)
        assert pl["y_tile"] == tile and pl["y_rows_out"] < 600
        t = dev(psi)
        s.substep(t, binding.SUB_Y, imag)
        assert rel(host(t), oracle.sweep_y(q, psi, imag)) < 1e-13, (tile, imag, pl)
        s.close()


@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_x_windows_full_steps(imag, precision):
    # whole steps (local substep and pending scale fused into the windowed x sweep)
    p = all_couplings(700, 61, 0.06, dy=0.1, dt=0.0015)
    psi0 = inputs.gaussian(700, 61, 0.06, 0.1, x0=p["x0"], y0=p["y0"], seed=15, center=(4.0, 0.3))
    s = binding.Solver(p, precision, x_solver="window")
    assert s.plan(imag)["x_points_out"] < 700  # several windows per row
    t = dev(psi0, s.dtype)
    (s.step_imag if imag else s.step_real)(t, 60)
    s.sync()
    got = host(t)
    s.close()
    want = oracle.step(p, psi0, 60, imag)
    if precision == "fp64":
        assert rel(got, want) < 1e-11
    else:
        rho_g, rho_w = np.abs(got) ** 2, np.abs(want) ** 2
        assert float(np.abs(rho_g - rho_w).max() / rho_w.max()) < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_block_orders_give_identical_results(precision):
    # orders 0-2 only change which workgroup computes which window: the states,
    # and the imaginary-time norm partials (stored per window and summed in
    # window order), agree to the bit; row bands also shorten the y row tile so
    # that the tiles split evenly over the XCDs (other window ends: agreement to
    # rounding); 700 x 500 spans several windows in both directions and a
    # ragged last window
    p = all_couplings(700, 500, 0.06, dy=0.05, dt=0.0015)
    psi0 = inputs.gaussian(700, 500, 0.06, 0.05, x0=p["x0"], y0=p["y0"], seed=16, center=(3.0, -2.0))
    for imag, xs in ((True, "window"), (False, "window"), (True, "scan"), (False, "scan")):
        out = []
        for order, wy in (("hardware", 0), ("xcd", 1), ("bands", 2), ("rows", 3)):
            s = binding.Solver(p, precision, x_solver=xs, block_order=order)
            pl = s.plan(imag)
            assert pl["y_rows_out"] < 500 and pl["y_block_order"] == wy
            if xs == "window":
                assert pl["x_points_out"] < 700 and pl["x_block_order"] == {"hardware": 0, "rows": 3}.get(order, 1)
            else:
                assert pl["x_block_order"] == (3 if order == "rows" else 0)
            t = dev(psi0, s.dtype)
            (s.step_imag if imag else s.step_real)(t, 7)
            s.sync()
            out.append(host(t))
            s.close()
        assert all(np.array_equal(out[0], o) for o in out[1:3]), (imag, xs)
        err = np.linalg.norm(out[3] - out[0]) / np.linalg.norm(out[0])
        assert err < (1e-13 if precision == "fp64" else 2e-6), (imag, xs, err)


@pytest.mark.parametrize("imag", [True, False])
def test_row_bands_with_row_zero_in_a_later_tile(imag):
    # row bands shorten the y row tile (130 rows over 8 XCDs: tiles of 17 rows
    # with a halo of 55), so row 0 of the columns lies in the halo of tiles
    # after the first; those tiles apply the line-start correction with the
    # increment of line point 0 (not of their first written row)
    p = all_couplings(256, 130, 0.02, dt=4e-4)
    psi0 = inputs.gaussian(256, 130, 0.02, 0.02, x0=p["x0"], y0=p["y0"], seed=17, phase_noise=0.3)
    pl = binding.plan_query(p, imag, "fp64", block_order="rows")
    assert pl["y_block_order"] == 3 and pl["y_rows_out"] <= pl["y_halo"]
    out = {}
    for order in ("hardware", "rows"):
        s = binding.Solver(p, "fp64", block_order=order)
        t = dev(psi0)
        (s.step_imag if imag else s.step_real)(t, 5)
        s.sync()
        out[order] = host(t)
        s.close()
    want = oracle.step(p, psi0, 5, imag)
    assert rel(out["rows"], out["hardware"]) < 1e-13
    assert rel(out["rows"], want) < 1e-13


@pytest.mark.parametrize("imag", [True, False])
def test_slowly_decaying_rows(imag):
    # the pivots' transient spans hundreds of points: the whole-row sweep takes a
    # shape whose line-start correction fits (or the long-row path), and refuses
    # a requested shape where it would not
    p = all_couplings(2000, 5, 0.005, dt=0.01)
    psi = inputs.random_state(2000, 5, seed=77)
    s = binding.Solver(p)
    t = dev(psi)
    s.substep(t, binding.SUB_X, imag)
    assert rel(host(t), oracle.sweep_x(p, psi, imag)) < 1e-12, s.plan(imag)
    s.close()
    with pytest.raises(binding.GPError) as ei:
        binding.Solver(p, x_points=2)
    assert ei.value.status == binding.GP_EUNSUPPORTED


def test_x_windows_refused_when_the_decay_is_slow():
    p = all_couplings(2000, 5, 0.005, dt=0.01)
    with pytest.raises(binding.GPError) as ei:
        binding.Solver(p, x_solver="window")
    assert ei.value.status == binding.GP_EUNSUPPORTED


@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("solver", ["window", "thomas"])
@pytest.mark.parametrize("ny", [3, 100, 128, 129, 600, 1000])
def test_y_sweep(imag, solver, ny):
    nx = 19 if ny % 2 else 40
    p = all_couplings(nx, ny, 0.2, dy=24.0 / ny + 0.001, dt=5e-4, eta=1 if ny % 3 else -1)
    psi = inputs.random_state(nx, ny, seed=ny + 7)
    s = binding.Solver(p, y_solver=solver)
    plan = s.plan(imag)
    t = dev(psi)
    s.substep(t, binding.SUB_Y, imag)
    got = host(t)
    want = oracle.sweep_y(p, psi, imag)
    assert rel(got, want) < 1e-13, plan
    if solver == "window":
        assert plan["y_solver"] == binding.GP_YSOLVER_WINDOW
        if ny > plan["y_segments"] * plan["y_rows_per_thread"]:
            assert plan["y_halo"] > 0  # the truncated-window path is exercised
    else:
        assert plan["y_solver"] == binding.GP_YSOLVER_THOMAS


def test_normalize_substep():
    p = all_couplings(33, 29, 0.3)
    psi = inputs.random_state(33, 29, seed=5)
    s = binding.Solver(p)
    t = dev(psi)
    s.substep(t, binding.SUB_NORMALIZE, True)
    assert rel(host(t), oracle.normalize(p, psi)) < 1e-14


# ---------------------------------------------------------------------------
# Whole steps
# ---------------------------------------------------------------------------
def test_c1_imaginary_time_200_steps():
    # 128 x 128, dx = 0.1, dt = 5e-4, c0 = 50, c2 = -1, Rashba gamma = 0.5, Omega = 0.5
    p = inputs.config_c1()
    psi0 = inputs.gaussian(128, 128, 0.1, 0.1, seed=1, phase_noise=0.1)
    got, obs = gpu_run(p, psi0, 200, True)
    want = oracle.step(p, psi0, 200, True)
    assert rel(got, want) < 1e-10
    o = oracle.observables(p, want)
    for k in ("energy", "mu_total", "e_kin", "e_trap", "e_int", "e_rot", "e_so", "lz", "magnetization"):
        assert abs(obs[k] - o[k]) <= 1e-10 * max(1.0, abs(o[k])), k
    assert abs(obs["norm_total"] - 1.0) < 1e-13


@pytest.mark.parametrize("imag", [True, False])
def test_1000_steps(imag):
    # spec bar: relative L2 <= 1e-10 on psi after 1000 FP64 steps
    if imag:
        p = inputs.config_c1()
        psi0 = inputs.gaussian(128, 128, 0.1, 0.1, seed=1, phase_noise=0.1)
    else:
        # the real-time workload's couplings on a 128^2 grid of the same box
        p = inputs.params(128, 128, 0.2, dt=4e-4, c0=200.0, c2=5.0, gamma=1.0, eta=-1, rabi=0.2, omega=0.9)
        psi0 = inputs.add_noise(inputs.gaussian(128, 128, 0.2, 0.2, seed=2), 0.2, 0.2, 1e-3, seed=3)
    got, obs = gpu_run(p, psi0, 1000, imag)
    want = oracle.step(p, psi0, 1000, imag)
    assert rel(got, want) < 1e-10
    if not imag:
        assert abs(obs["norm_total"] - 1.0) < 1e-12  # unitary real-time step


@pytest.mark.parametrize("imag", [True, False])
def test_ragged_rectangular_grid(imag):
    p = all_couplings(97, 61, 0.17, dy=0.23, dt=0.005, eta=-1)
    p["x0"], p["y0"] = -7.3, -6.1
    psi0 = inputs.gaussian(97, 61, 0.17, 0.23, x0=p["x0"], y0=p["y0"], seed=4, center=(0.3, -0.2))
    got, _ = gpu_run(p, psi0, 100, imag)
    want = oracle.step(p, psi0, 100, imag)
    assert rel(got, want) < 1e-11


@pytest.mark.parametrize("shape", [(3, 3), (3, 200), (200, 3), (5, 131)])
def test_degenerate_small_grids(shape):
    nx, ny = shape
    p = all_couplings(nx, ny, 0.4, dt=0.003)
    psi0 = inputs.random_state(nx, ny, seed=nx * ny, scale=0.3)
    for imag in (True, False):
        got, _ = gpu_run(p, psi0, 20, imag)
        want = oracle.step(p, psi0, 20, imag)
        assert rel(got, want) < 1e-11


def test_window_and_thomas_agree_on_tall_grid():
    p = all_couplings(48, 1100, 0.25, dy=0.02, dt=2e-4)
    psi0 = inputs.gaussian(48, 1100, 0.25, 0.02, seed=8)
    a, _ = gpu_run(p, psi0, 30, True, y_solver="window")
    b, _ = gpu_run(p, psi0, 30, True, y_solver="thomas")
    assert rel(a, b) < 1e-13
    want = oracle.step(p, psi0, 30, True)
    assert rel(a, want) < 1e-12


def test_observables_match_oracle():
    p = all_couplings(64, 56, 0.3, eta=-1)
    psi = inputs.gaussian(64, 56, 0.3, 0.3, seed=9, phase_noise=0.5, windings=(1, 0, -1))
    s = binding.Solver(p)
    t = dev(psi)
    dens = torch.empty((3, 56, 64), dtype=torch.float64, device=DEV)
    obs = s.observables(t, dens)
    o = oracle.observables(p, psi)
    for k in ("norm_total", "magnetization", "energy", "e_kin", "e_trap", "e_int", "e_rot", "e_so",
              "e_rabi", "lz", "mu_total"):
        assert abs(obs[k] - o[k]) <= 1e-12 * max(1.0, abs(o[k])), k
    for m in range(3):
        assert abs(obs["mu"][m] - o["mu"][m]) <= 1e-12 * max(1.0, abs(o["mu"][m]))
        assert abs(obs["norm"][m] - o["norm"][m]) <= 1e-13
    assert np.abs(dens.cpu().numpy() - np.abs(psi) ** 2).max() < 1e-15


def test_empty_component_chemical_potential():
    # a component of zero norm reports mu = 0 (as the oracle), and the call succeeds
    p = all_couplings(40, 36, 0.3, gamma=0.0, rabi=0.0)
    psi = inputs.gaussian(40, 36, 0.3, 0.3, seed=9)
    psi[0] = 0.0
    psi[2] = 0.0
    s = binding.Solver(p)
    obs = s.observables(dev(psi))
    o = oracle.observables(p, psi)
    assert obs["mu"][0] == 0.0 and obs["mu"][2] == 0.0 and o["mu"][0] == 0.0
    assert abs(obs["mu"][1] - o["mu"][1]) <= 1e-12 * abs(o["mu"][1])
    s.close()


# ---------------------------------------------------------------------------
# FP32 bulk with FP64 reductions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("imag", [True, False])
def test_fp32_bulk(imag):
    if imag:
        p = inputs.config_c1()
        psi0 = inputs.gaussian(128, 128, 0.1, 0.1, seed=1, phase_noise=0.1)
        n = 200
    else:
        p = inputs.params(128, 128, 0.2, dt=4e-4, c0=200.0, c2=5.0, gamma=1.0, eta=-1, rabi=0.2, omega=0.9)
        psi0 = inputs.add_noise(inputs.gaussian(128, 128, 0.2, 0.2, seed=2), 0.2, 0.2, 1e-3, seed=3)
        n = 1000
    got, obs = gpu_run(p, psi0, n, imag, precision="fp32")
    want = oracle.step(p, psi0, n, imag)
    o = oracle.observables(p, want)
    rho_g, rho_w = np.abs(got) ** 2, np.abs(want) ** 2
    dens_err = float(np.abs(rho_g - rho_w).max() / rho_w.max())
    mu_err = abs(obs["mu_total"] - o["mu_total"]) / abs(o["mu_total"])
    print(f"fp32 {'imag' if imag else 'real'}: density err {dens_err:.2e}, mu err {mu_err:.2e}")
    assert dens_err < 1e-5
    assert mu_err < 1e-6


# ---------------------------------------------------------------------------
# Full workload sizes, in the launch configuration the benchmark times
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c2_full_size_steps(precision):
    # the 512^2 real-time workload in the benchmark's launch configuration (tuned shapes)
    p = inputs.config_c2()
    psi0 = inputs.add_noise(inputs.gaussian(512, 512, 0.05, 0.05, seed=2), 0.05, 0.05, 1e-3, seed=3)
    got, obs = gpu_run(p, psi0, 3, False, precision=precision, autotune=True)
    want = oracle.step(p, psi0, 3, False)
    if precision == "fp64":
        assert rel(got, want) < 1e-13
    else:
        rho_g, rho_w = np.abs(got) ** 2, np.abs(want) ** 2
        assert float(np.abs(rho_g - rho_w).max() / rho_w.max()) < 1e-6
    # many steps: the unitary real-time step keeps the norm
    s = binding.Solver(p, precision, autotune=True)
    t = dev(psi0, s.dtype)
    s.step_real(t, 2000)
    assert abs(s.observables(t)["norm_total"] - 1.0) < (1e-11 if precision == "fp64" else 1e-6)


_C2_1000 = {}


def c2_oracle_1000():
    """The oracle's 1000 real-time steps of the 512^2 workload (shared by the precisions)."""
    if not _C2_1000:
        p = inputs.config_c2()
        psi0 = inputs.add_noise(inputs.gaussian(512, 512, 0.05, 0.05, seed=2), 0.05, 0.05, 1e-3, seed=3)
        want = oracle.step(p, psi0, 1000, False)
        _C2_1000.update(p=p, psi0=psi0, want=want, obs=oracle.observables(p, want))
    return _C2_1000


def fp32_errors(got, obs, want, o):
    """FP32 result against the FP64 oracle: the density error relative to the
    peak density, and the relative errors of mu_total and of each mu_m."""
    rho_g, rho_w = np.abs(got) ** 2, np.abs(want) ** 2
    dens = float(np.abs(rho_g - rho_w).max() / rho_w.max())
    mu = abs(obs["mu_total"] - o["mu_total"]) / abs(o["mu_total"])
    mum = max(abs(obs["mu"][m] - o["mu"][m]) / abs(o["mu"][m]) for m in range(3))
    return dens, mu, mum


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c2_full_size_1000_steps(precision):
    # 1000 steps of the full 512^2 real-time workload in the benchmark's launch
    # configuration (tuned shapes): FP64 to the 1e-10 relative L2 bar; FP32 bulk
    # to density 1e-5 (relative to the peak density) and chemical potentials 1e-6
    c = c2_oracle_1000()
    got, obs = gpu_run(c["p"], c["psi0"], 1000, False, precision=precision, autotune=True)
    if precision == "fp64":
        assert rel(got, c["want"]) < 1e-10
        assert abs(obs["norm_total"] - 1.0) < 1e-12
    else:
        dens, mu, mum = fp32_errors(got, obs, c["want"], c["obs"])
        print(f"c2 fp32 1000 steps: density err {dens:.2e}, mu err {mu:.2e}, mu_m err {mum:.2e}, "
              f"psi rel L2 {rel(got, c['want']):.2e}")
        assert dens < 1e-5
        assert mu < 1e-6 and mum < 1e-6


@pytest.mark.parametrize("n", [2048, 4096])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c3_full_size_steps(precision, n):
    # the large imaginary-time grid; 4096^2 in the benchmark's launch configuration (tuned shapes)
    p = inputs.config_c3(n)
    psi0 = inputs.gaussian(n, n, 0.02, 0.02, seed=4, full_phase=True)
    got, obs = gpu_run(p, psi0, 2, True, precision=precision, autotune=(n == 4096))
    want = oracle.step(p, psi0, 2, True)
    if precision == "fp64":
        assert rel(got, want) < 1e-13
        assert abs(obs["norm_total"] - 1.0) < 1e-13
    else:
        dens, mu, mum = fp32_errors(got, obs, want, oracle.observables(p, want))
        print(f"c3 {n} fp32 2 steps: density err {dens:.2e}, mu err {mu:.2e}, mu_m err {mum:.2e}, "
              f"psi rel L2 {rel(got, want):.2e}")
        assert dens < 1e-5
        assert mu < 1e-6 and mum < 1e-6
        assert abs(obs["norm_total"] - 1.0) < 1e-6


# ---------------------------------------------------------------------------
# Error paths (forced from the host; every kernel still exits normally)
# ---------------------------------------------------------------------------
def test_unstable_parameters_are_refused():
    # the imaginary-time Cayley bound fails, the real-time lines stay diagonally dominant
    p = inputs.params(64, 64, 0.3, dt=0.05, omega=0.9, gamma=1.0)
    assert binding.plan_query(p, True)["stable"] == 0 and binding.plan_query(p, False)["stable"] == 1
    s = binding.Solver(p)
    t = dev(inputs.gaussian(64, 64, 0.3, 0.3, seed=1))
    with pytest.raises(binding.GPError) as ei:
        s.step_imag(t, 1)
    assert ei.value.status == binding.GP_EUNSTABLE
    s.step_real(t, 1)  # real time stays available on this handle
    s.sync()
    s.close()
    # neither propagation stable (real-time lines not diagonally dominant): refused at create
    q = inputs.params(64, 64, 0.1, dt=5.0, omega=5.0)
    assert binding.plan_query(q, False)["stable"] == 0 and binding.plan_query(q, True)["stable"] == 0
    with pytest.raises(binding.GPError) as ei:
        binding.Solver(q)
    assert ei.value.status == binding.GP_EUNSTABLE


@pytest.mark.parametrize("imag", [True, False])
def test_longest_row_full_steps(imag):
    # 8192-point rows (the longest the library handles) through whole steps: by
    # default the chain windows (the whole-row solve would hold 16 points per
    # thread), and the whole-row solve when asked for
    p = all_couplings(8192, 12, 0.0015, dy=0.3, dt=2e-5)
    psi0 = inputs.random_state(8192, 12, seed=91, scale=0.4)
    want = oracle.step(p, psi0, 3, imag)
    for xs, solver in (("auto", binding.GP_XSOLVER_CHAIN), ("scan", binding.GP_XSOLVER_SCAN)):
        s = binding.Solver(p, x_solver=xs)
        assert s.plan(imag)["x_solver"] == solver
        t = dev(psi0)
        (s.step_imag if imag else s.step_real)(t, 3)
        s.sync()
        assert rel(host(t), want) < 1e-12, xs
        s.close()


def test_zero_steps_and_invalid_counts():
    # zero steps leave psi untouched (imaginary time included: no pending scale
    # is applied); negative counts and unknown substeps are refused
    p = all_couplings(40, 30, 0.3, dt=0.01)
    psi0 = inputs.gaussian(40, 30, 0.3, 0.3, seed=5)
    s = binding.Solver(p)
    for step in (s.step_imag, s.step_real):
        t = dev(psi0)
        step(t, 0)
        s.sync()
        assert np.array_equal(host(t), psi0)
        with pytest.raises(binding.GPError) as ei:
            step(t, -1)
        assert ei.value.status == binding.GP_EINVAL
    t = dev(psi0)
    with pytest.raises(binding.GPError) as ei:
        s.substep(t, 4, True)
    assert ei.value.status == binding.GP_EINVAL
    s.step_imag(t, 1)
    one = host(t)
    s.step_imag(t, 0)
    assert np.array_equal(host(t), one)
    s.close()


def test_host_buffers_are_refused_before_any_launch():
    # the binding hands the library device pointers only
    p = inputs.params(32, 24, 0.3, dt=0.01)
    s = binding.Solver(p)
    host = torch.zeros((3, 24, 32), dtype=torch.complex128)
    with pytest.raises(ValueError):
        s.step_imag(host, 1)
    t = dev(inputs.gaussian(32, 24, 0.3, 0.3, seed=1))
    with pytest.raises(ValueError):
        s.observables(t, torch.zeros((3, 24, 32), dtype=torch.float64))
    s.observables(t, torch.zeros((3, 24, 32), dtype=torch.float64, device=DEV))
    s.close()


def test_nonfinite_is_reported():
    p = all_couplings(40, 40, 0.3)
    psi = inputs.gaussian(40, 40, 0.3, 0.3, seed=1)
    psi[1, 20, 20] = complex(math.nan, 0.0)
    s = binding.Solver(p)
    t = dev(psi)
    s.step_imag(t, 2)
    with pytest.raises(binding.GPError) as ei:
        s.sync()
    assert ei.value.status == binding.GP_ENONFINITE
    with pytest.raises(binding.GPError) as ei:
        s.observables(t)
    assert ei.value.status == binding.GP_ENONFINITE
    s.sync()  # the flag was cleared


def test_imaginary_time_with_many_y_blocks():
    # enough y windows that the next x sweep does not sum the norm partials itself
    # (a separate one-block reduction between the steps)
    p = all_couplings(256, 4000, 0.1, dy=0.05, dt=0.002, omega=0.3)
    q = binding.plan_query(p, True)
    assert q["y_solver"] == binding.GP_YSOLVER_WINDOW
    # y blocks (32 column strips x windows of y_rows_out rows) far more than the x threads can sum
    nyb = (256 // q["y_tile_cols"]) * -(-4000 // q["y_rows_out"])
    assert 3 * nyb > 8 * q["x_threads_per_row"] * q["x_rows_per_block"]
    psi0 = inputs.gaussian(256, 4000, 0.1, 0.05, x0=p["x0"], y0=p["y0"], seed=12, center=(0.5, 20.0))
    got, obs = gpu_run(p, psi0, 12, True)
    want = oracle.step(p, psi0, 12, True)
    assert rel(got, want) < 1e-11
    assert abs(obs["norm_total"] - 1.0) < 1e-13
