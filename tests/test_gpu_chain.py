"""Chain windows (GP_XSOLVER_CHAIN, GP_YSOLVER_CHAIN): the windowed sweeps
with each lane's carry formed from the ceil((h - 1) / K) lanes before and after it.
Every point a window writes lies at least h from both window ends, so the
result equals the exact line solve to the rounding level: the FP64 parity
bars are those of the scanned windows (1e-13 for a substep, 1e-11 after tens
of steps), FP32 the density and chemical-potential bounds.

Cases: every chain tile of both sweeps and both propagation modes, lines of
several windows with a ragged last window, lines shorter than one window,
slow decay (wide halos), the line-start correction, Strang and fixed
magnetisation, padded planes, block orders, and the full 4096^2 grid.
"""
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


def all_couplings(nx, ny, dx, dy=None, dt=0.01, eta=1, **kw):
    base = dict(c0=35.0, c2=-3.0, gamma=0.6, eta=eta, rabi=0.25, omega=0.45)
    base.update(kw)
    return inputs.params(nx, ny, dx, dy=dy, dt=dt, **base)


@pytest.mark.parametrize("tile", range(1, 9))
def test_every_chain_tile_x(tile):
    for imag in (True, False):
        for nx in (3, 200, 1500, 4100):
            dx = min(12.0 / nx + 0.01, 0.3)
            p = all_couplings(nx, 5, dx, dy=0.2, dt=0.4 * dx * dx, eta=-1 if nx % 2 else 1)
            psi = inputs.random_state(nx, 5, seed=60 + tile + nx)
            s = binding.Solver(p, x_solver="chain", x_tile=tile)
            pl = s.plan(imag)
            assert pl["x_solver"] == binding.GP_XSOLVER_CHAIN and pl["x_tile"] == tile
            t = dev(psi)
            s.substep(t, binding.SUB_X, imag)
            assert rel(host(t), oracle.sweep_x(p, psi, imag)) < 1e-13, (tile, imag, nx, pl)
            s.close()


@pytest.mark.parametrize("tile", range(1, 9))
def test_every_chain_tile_y(tile):
    for imag in (True, False):
        for ny in (3, 90, 700, 1501):
            dy = min(12.0 / ny + 0.01, 0.3)
            p = all_couplings(9, ny, 0.2, dy=dy, dt=0.4 * dy * dy, eta=1 if ny % 3 else -1)
            psi = inputs.random_state(9, ny, seed=80 + tile + ny)
            s = binding.Solver(p, y_solver="chain", y_tile=tile)
            pl = s.plan(imag)
            assert pl["y_solver"] == binding.GP_YSOLVER_CHAIN and pl["y_tile"] == tile
            t = dev(psi)
            s.substep(t, binding.SUB_Y, imag)
            assert rel(host(t), oracle.sweep_y(p, psi, imag)) < 1e-13, (tile, imag, ny, pl)
            s.close()


@pytest.mark.parametrize("tile", range(1, 7))
def test_every_stacked_tile_y(tile):
    # stacked windows: 16 columns per block (ragged column strips included), 16 or 32 segments over the waves
    for imag in (True, False):
        for nx, ny in ((9, 3), (37, 90), (21, 700), (50, 1501)):
            dy = min(12.0 / ny + 0.01, 0.3)
            p = all_couplings(nx, ny, 0.2, dy=dy, dt=0.4 * dy * dy, eta=1 if ny % 3 else -1)
            psi = inputs.random_state(nx, ny, seed=90 + tile + ny)
            s = binding.Solver(p, y_solver="stack", y_tile=tile)
            pl = s.plan(imag)
            assert pl["y_solver"] == binding.GP_YSOLVER_STACK and pl["y_tile"] == tile
            t = dev(psi)
            s.substep(t, binding.SUB_Y, imag)
            assert rel(host(t), oracle.sweep_y(p, psi, imag)) < 1e-13, (tile, imag, ny, pl)
            s.close()


@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_stacked_full_steps(imag, precision):
    p = all_couplings(700, 530, 0.06, dy=0.05, dt=0.0015)
    psi0 = inputs.gaussian(700, 530, 0.06, 0.05, x0=p["x0"], y0=p["y0"], seed=25, center=(-3.0, 0.7))
    s = binding.Solver(p, precision, x_solver="chain", y_solver="stack")
    t = dev(psi0, s.dtype)
    (s.step_imag if imag else s.step_real)(t, 30)
    s.sync()
    got = host(t)
    obs = s.observables(t)
    s.close()
    want = oracle.step(p, psi0, 30, imag)
    if precision == "fp64":
        assert rel(got, want) < 1e-11
    else:
        o = oracle.observables(p, want)
        rho_g, rho_w = np.abs(got) ** 2, np.abs(want) ** 2
        assert float(np.abs(rho_g - rho_w).max() / rho_w.max()) < 1e-5
        assert abs(obs["mu_total"] - o["mu_total"]) / abs(o["mu_total"]) < 1e-6


@pytest.mark.parametrize("imag", [True, False])
def test_chain_wide_halo(imag):
    # slow decay (dt above dx dy): halos of tens of points, several carry lanes
    p = all_couplings(900, 700, 0.02, dy=0.025, dt=0.001, omega=0.1, gamma=0.2)
    psi = inputs.random_state(900, 700, seed=5)
    for prec in ("fp64",):
        s = binding.Solver(p, prec, x_solver="chain", y_solver="chain")
        pl = s.plan(imag)
        assert pl["x_halo"] > 16 and pl["y_halo"] > 16, pl
        t = dev(psi)
        s.substep(t, binding.SUB_X, imag)
        assert rel(host(t), oracle.sweep_x(p, psi, imag)) < 1e-13, pl
        t = dev(psi)
        s.substep(t, binding.SUB_Y, imag)
        assert rel(host(t), oracle.sweep_y(p, psi, imag)) < 1e-13, pl
        s.close()


@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_chain_full_steps(imag, precision):
    # whole steps (local substep and pending scale fused into the x chain windows, norm partials in y)
    p = all_couplings(700, 530, 0.06, dy=0.05, dt=0.0015)
    psi0 = inputs.gaussian(700, 530, 0.06, 0.05, x0=p["x0"], y0=p["y0"], seed=15, center=(4.0, 0.3))
    s = binding.Solver(p, precision, x_solver="chain", y_solver="chain")
    pl = s.plan(imag)
    assert pl["x_points_out"] < 700 and pl["y_rows_out"] < 530
    t = dev(psi0, s.dtype)
    (s.step_imag if imag else s.step_real)(t, 40)
    s.sync()
    got = host(t)
    obs = s.observables(t)
    s.close()
    want = oracle.step(p, psi0, 40, imag)
    if precision == "fp64":
        assert rel(got, want) < 1e-11
    else:
        o = oracle.observables(p, want)
        rho_g, rho_w = np.abs(got) ** 2, np.abs(want) ** 2
        assert float(np.abs(rho_g - rho_w).max() / rho_w.max()) < 1e-5
        assert abs(obs["mu_total"] - o["mu_total"]) / abs(o["mu_total"]) < 1e-6


@pytest.mark.parametrize("imag", [True, False])
def test_chain_with_scanned_other_sweep(imag):
    # mixed plans: chain x with the scanned y windows, scanned x windows with chain y
    p = all_couplings(600, 450, 0.06, dy=0.06, dt=0.0015)
    psi0 = inputs.gaussian(600, 450, 0.06, 0.06, x0=p["x0"], y0=p["y0"], seed=16)
    want = oracle.step(p, psi0, 12, imag)
    for xs, ys in (("chain", "window"), ("window", "chain"), ("scan", "chain")):
        s = binding.Solver(p, "fp64", x_solver=xs, y_solver=ys)
        t = dev(psi0)
        (s.step_imag if imag else s.step_real)(t, 12)
        s.sync()
        assert rel(host(t), want) < 1e-12, (xs, ys)
        s.close()


def test_chain_strang_and_fixed_magnetisation():
    p = all_couplings(500, 420, 0.06, dy=0.06, dt=0.0015, split=1)
    psi0 = inputs.gaussian(500, 420, 0.06, 0.06, x0=p["x0"], y0=p["y0"], seed=17)
    for imag in (True, False):
        s = binding.Solver(p, "fp64", x_solver="chain", y_solver="chain")
        t = dev(psi0)
        (s.step_imag if imag else s.step_real)(t, 10)
        s.sync()
        assert rel(host(t), oracle.step(p, psi0, 10, imag)) < 1e-12, imag
        s.close()
    q = inputs.params(500, 420, 0.06, dy=0.06, dt=0.0015, c0=40.0, c2=-2.0, omega=0.3, fix_m=1, magnetization=0.2)
    psi0 = inputs.gaussian(500, 420, 0.06, 0.06, x0=q["x0"], y0=q["y0"], seed=18)
    s = binding.Solver(q, "fp64", x_solver="chain", y_solver="chain")
    t = dev(psi0)
    s.step_imag(t, 10)
    s.sync()
    assert rel(host(t), oracle.step(q, psi0, 10, True)) < 1e-12
    s.close()


def test_chain_padded_planes_and_block_orders():
    p = all_couplings(640, 480, 0.05, dy=0.05, dt=0.001)
    psi0 = inputs.gaussian(640, 480, 0.05, 0.05, x0=p["x0"], y0=p["y0"], seed=19)
    out = []
    for order in ("hardware", "xcd", "bands"):
        s = binding.Solver(p, "fp64", x_solver="chain", y_solver="chain", block_order=order)
        t = dev(psi0)
        s.step_imag(t, 6)
        s.sync()
        out.append(host(t))
        s.close()
    assert all(np.array_equal(out[0], o) for o in out[1:])
    t, q = binding.padded_psi(psi0, p, torch.complex128)
    s = binding.Solver(q, "fp64", x_solver="chain", y_solver="chain", block_order="hardware")
    s.step_imag(t, 6)
    s.sync()
    assert np.array_equal(host(t), out[0])
    s.close()
    assert rel(out[0], oracle.step(p, psi0, 6, True)) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_chain_full_size_4096(precision):
    # the 4096^2 imaginary-time workload through chain windows in both sweeps
    p = inputs.config_c3(4096)
    psi0 = inputs.gaussian(4096, 4096, 0.02, 0.02, seed=4, full_phase=True)
    s = binding.Solver(p, precision, x_solver="chain", y_solver="chain")
    t = dev(psi0, s.dtype)
    s.step_imag(t, 2)
    s.sync()
    got = host(t)
    obs = s.observables(t)
    s.close()
    want = oracle.step(p, psi0, 2, True)
    if precision == "fp64":
        assert rel(got, want) < 1e-13
    else:
        o = oracle.observables(p, want)
        rho_g, rho_w = np.abs(got) ** 2, np.abs(want) ** 2
        assert float(np.abs(rho_g - rho_w).max() / rho_w.max()) < 1e-5
        assert abs(obs["mu_total"] - o["mu_total"]) / abs(o["mu_total"]) < 1e-6


def test_seeded_random_plans_match_oracle():
    # seeded random grids (ragged sizes, rectangular cells), couplings, time
    # steps and chain / stacked tiles, in both propagation modes, against the
    # oracle; cases whose decay fits no chosen tile are drawn again
    rng = np.random.default_rng(2024)
    done = 0
    while done < 16:
        nx, ny = int(rng.integers(3, 260)), int(rng.integers(3, 260))
        dx, dy = float(rng.uniform(0.04, 0.3)), float(rng.uniform(0.04, 0.3))
        dt = float(rng.uniform(0.05, 1.0)) * min(dx, dy) ** 2
        p = inputs.params(nx, ny, dx, dy=dy, dt=dt, c0=float(rng.uniform(0, 200)), c2=float(rng.uniform(-10, 10)),
                          gamma=float(rng.uniform(0, 1)), eta=int(rng.choice([-1, 1])),
                          rabi=float(rng.uniform(0, 0.5)), omega=float(rng.uniform(0, 0.9)))
        imag = bool(rng.integers(0, 2))
        kw = dict(x_solver="chain", x_tile=int(rng.integers(1, 9)), y_solver=str(rng.choice(["chain", "stack"])))
        kw["y_tile"] = int(rng.integers(1, 9 if kw["y_solver"] == "chain" else 7))
        pl = binding.plan_query(p, imag, **kw)
        if (not pl["stable"] or pl["x_solver"] != binding.GP_XSOLVER_CHAIN
                or pl["y_solver"] not in (binding.GP_YSOLVER_CHAIN, binding.GP_YSOLVER_STACK)):
            continue
        # the amplitude keeps the nonlinear phase of one step near 0.3 rad
        # (the workloads turn through far less): in real time each local
        # substep multiplies a difference in rounding by about that phase
        # times the mean density, in both implementations alike
        g = dt * (p["c0"] + abs(p["c2"]))
        psi0 = inputs.random_state(nx, ny, seed=500 + done, scale=min(1.0, (0.05 / max(g, 1e-30)) ** 0.5))
        s = binding.Solver(p, "fp64", **kw)
        t = dev(psi0)
        (s.step_imag if imag else s.step_real)(t, 3)
        got = host(t)
        s.close()
        want = oracle.step(p, psi0, 3, imag)
        assert rel(got, want) < 1e-12, (nx, ny, dx, dy, dt, imag, kw, pl)
        done += 1
