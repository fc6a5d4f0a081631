"""Batched launches over many condensates (C ABI gp_spin1_batch_*).

A condensate advanced inside a batch must give the wave function of the same
condensate advanced alone on a handle with the batch's launch shape: the same
blocking, scans and reduction order, so the two agree to rounding (the
batched and single kernels are separate instantiations of one source, and
the compiler may contract a product and a sum into an FMA in one and not the
other, a last-bit difference).  Tolerance: relative L2 1e-12 (FP64) and 2e-6
(FP32) after up to 30 steps.  Against the oracle: the FP64 parity bar.

Both batched shapes are covered: chain x windows with stacked chain y windows
(the default when the group fits them) and whole-row scans with scanned y
windows (asked for per slot, or when a slot does not fit the chain tiles).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2105_10517_amd import binding, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(DEV)


def mixed_slots():
    """Different grids (ragged, rectangular), couplings, SO types and time steps."""
    ps = [
        inputs.params(64, 64, 0.25, dt=0.1 * 0.25 ** 2, c0=40.0, c2=-2.0, gamma=0.5, eta=1, rabi=0.1, omega=0.4),
        inputs.params(96, 160, 0.15, dy=0.12, dt=0.004, c0=120.0, c2=4.0, gamma=0.9, eta=-1, rabi=0.3, omega=0.7),
        inputs.params(200, 130, 0.1, dt=0.002, c0=300.0, c2=-8.0, gamma=0.3, eta=1, rabi=0.0, omega=0.9),
        inputs.params(37, 45, 0.3, dt=0.01, c0=10.0, c2=1.0, gamma=0.0, eta=1, rabi=0.5, omega=0.0),
        inputs.params(256, 256, 0.1, dt=0.001, c0=500.0, c2=15.0, gamma=1.0, eta=-1, rabi=0.2, omega=0.95),
    ]
    return ps


def initial(p, seed):
    return inputs.gaussian(p["nx"], p["ny"], p["dx"], p["dy"], x0=p["x0"], y0=p["y0"], seed=seed)


def same(got, want, precision):
    tol = 1e-12 if precision == "fp64" else 2e-6
    err = float(torch.linalg.vector_norm((got - want).flatten()) / torch.linalg.vector_norm(want.flatten()))
    return err <= tol, err


def alone(p, psi0, n, mode, precision, info, dtype):
    """The same condensate on a single handle with the batch's launch shape."""
    md = 0 if mode == "imag" else 1
    if info["x_solver"][md] == binding.GP_XSOLVER_CHAIN:
        assert info["y_solver"][md] == binding.GP_YSOLVER_STACK
        s = binding.Solver(p, precision, x_solver="chain", x_tile=info["x_tile"][md], y_solver="stack",
                           y_tile=info["y_tile"][md])
    else:
        s = binding.Solver(p, precision, x_points=info["x_points"][md], y_tile=info["y_tile"][md])
    t = dev(psi0, dtype)
    (s.step_imag if mode == "imag" else s.step_real)(t, n)
    s.sync()
    out = t.cpu()
    s.close()
    return out


SHAPES = {"chain": dict(), "scan": dict(x_solver="scan", y_solver="window")}
SHAPE_SOLVER = {"chain": binding.GP_XSOLVER_CHAIN, "scan": binding.GP_XSOLVER_SCAN}


@pytest.mark.parametrize("shape", ["chain", "scan"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_single_handles(precision, shape):
    ps = mixed_slots()
    modes = ["imag", "real", "imag", "real", "imag"]
    nsteps = [30, 12, 7, 30, 19]  # several phases
    b = binding.Batch(ps, precision, **SHAPES[shape])
    psi0 = [initial(p, 10 + k) for k, p in enumerate(ps)]
    ts = [dev(a, b.dtype) for a in psi0]
    b.step(ts, nsteps, modes)
    b.sync()
    info = b.info()
    assert info["grouped"] == len(ps) and info["individual"] == 0
    assert info["phases"] == len(set(nsteps))
    assert info["x_solver"] == [SHAPE_SOLVER[shape]] * 2, info
    for k, p in enumerate(ps):
        want = alone(p, psi0[k], nsteps[k], modes[k], precision, info, b.dtype)
        got = ts[k].cpu()
        ok, err = same(got, want, precision)
        assert ok, f"slot {k}: relative L2 {err:.3e}"
    b.close()


@pytest.mark.parametrize("shape", ["chain", "scan"])
def test_batch_matches_oracle(shape):
    ps = mixed_slots()[:4]
    modes = ["imag", "real", "real", "imag"]
    nsteps = [25, 25, 10, 40]
    b = binding.Batch(ps, "fp64", **SHAPES[shape])
    psi0 = [initial(p, 20 + k) for k, p in enumerate(ps)]
    ts = [dev(a, torch.complex128) for a in psi0]
    b.step(ts, nsteps, modes)
    b.sync()
    for k, p in enumerate(ps):
        want = oracle.step(p, psi0[k], nsteps[k], modes[k] == "imag")
        got = ts[k].cpu().numpy()
        err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        assert err < 1e-11, (k, err)
    b.close()


def test_empty_and_inactive_slots_are_untouched():
    ps = mixed_slots()[:3]
    b = binding.Batch([ps[0], None, ps[2]], "fp64")
    psi0 = [initial(p, 30 + k) for k, p in enumerate(ps)]
    t0, t2 = dev(psi0[0], torch.complex128), dev(psi0[2], torch.complex128)
    before2 = t2.clone()
    b.step([t0, None, t2], [5, 0, 5], ["imag", "imag", "real"], active=[True, False, False])
    b.sync()
    assert torch.equal(t2, before2)
    assert not torch.equal(t0.cpu(), torch.from_numpy(psi0[0]))
    with pytest.raises(binding.GPError):
        b.step([t0, t0, t2], [1, 1, 1], ["imag", "imag", "imag"])  # slot 1 is empty
    b.close()


def test_set_slot_admits_a_new_condensate():
    ps = mixed_slots()
    b = binding.Batch([ps[0], ps[1]], "fp64")
    b.set_slot(1, ps[4])
    psi = [initial(ps[0], 40), initial(ps[4], 41)]
    ts = [dev(a, torch.complex128) for a in psi]
    b.step(ts, [8, 8], ["imag", "real"])
    b.sync()
    info = b.info()
    want = alone(ps[4], psi[1], 8, "real", "fp64", info, torch.complex128)
    assert same(ts[1].cpu(), want, "fp64")[0]
    b.set_slot(0, None)
    with pytest.raises(binding.GPError):
        b.step(ts, [1, 1], ["imag", "real"])
    b.close()


def test_slot_outside_the_batch_tile_runs_alone():
    # a tall grid with slow decay in y (large dt / dy^2) needs a bigger window
    # than any tile (scanned or stacked); it runs on its own plan
    small = inputs.params(48, 48, 0.3, dt=0.009, c0=20.0, c2=-1.0, gamma=0.4, eta=1, rabi=0.1, omega=0.3)
    tall = inputs.params(40, 700, 0.2, dy=0.05, dt=0.05, c0=20.0, c2=-1.0, gamma=0.4, eta=1, rabi=0.1, omega=0.3)
    assert binding.plan_query(tall, True)["stable"] == 1
    if binding.plan_query(tall, True)["y_solver"] == binding.GP_YSOLVER_WINDOW:
        pytest.skip("the tall grid windows with every tile here")
    b = binding.Batch([small, tall], "fp64")
    psi = [initial(small, 50), initial(tall, 51)]
    ts = [dev(a, torch.complex128) for a in psi]
    b.step(ts, [6, 6], ["imag", "imag"])
    b.sync()
    info = b.info()
    assert info["individual"] == 1 and info["grouped"] == 1
    # (the tall grid fits no stacked tile either: the group takes the scanned shapes)
    assert info["x_solver"][0] == binding.GP_XSOLVER_SCAN
    s = binding.Solver(tall, "fp64")
    t = dev(psi[1], torch.complex128)
    s.step_imag(t, 6)
    s.sync()
    assert torch.equal(ts[1].cpu(), t.cpu())  # the same kernels and plan: bit for bit
    s.close()
    b.close()


def test_batch_nonfinite_names_the_slot():
    ps = mixed_slots()[:2]
    b = binding.Batch(ps, "fp64")
    bad = initial(ps[1], 60)
    bad[0, 10, 10] = complex(math.nan, 0.0)
    ts = [dev(initial(ps[0], 61), torch.complex128), dev(bad, torch.complex128)]
    b.step(ts, [3, 3], ["imag", "imag"])
    with pytest.raises(binding.GPError) as ei:
        b.sync()
    assert ei.value.status == binding.GP_ENONFINITE and "slot 1" in str(ei.value)
    b.close()


def test_batch_scan_workload_sample():
    """The 32 k x 32 k parameter-scan grids (k = 4..16), FP32 bulk, against
    single handles with the batch shape (a sample of the scan, few steps)."""
    ps = inputs.batch_scan(24, seed=5)
    b = binding.Batch(ps, "fp32")
    psi0 = [initial(p, 1000 + k) for k, p in enumerate(ps)]
    ts = [dev(a, torch.complex64) for a in psi0]
    b.step(ts, [20] * len(ps), ["imag"] * len(ps))
    b.sync()
    info = b.info()
    assert info["grouped"] + info["individual"] == len(ps)
    for k in (0, 7, 23):
        want = alone(ps[k], psi0[k], 20, "imag", "fp32", info, torch.complex64)
        assert same(ts[k].cpu(), want, "fp32")[0]
    b.close()


def test_batch_scan_fp32_matches_oracle():
    """The full 256-condensate parameter scan, FP32 bulk in one batch, 100
    imaginary-time steps; the smallest, a middle and the largest grid of the
    scan against the FP64 oracle: density 1e-5 (relative to the peak density)
    and chemical potentials 1e-6 (relative)."""
    ps = inputs.batch_scan(256, seed=5)
    b = binding.Batch(ps, "fp32")
    ts = [dev(initial(p, 1000 + k), torch.complex64) for k, p in enumerate(ps)]
    b.step(ts, [100] * len(ps), ["imag"] * len(ps))
    b.sync()
    sizes = [p["nx"] for p in ps]
    picks = (int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), int(np.argmax(sizes)))
    for k in picks:
        p = ps[k]
        want = oracle.step(p, initial(p, 1000 + k), 100, True)
        o = oracle.observables(p, want)
        obs = b.observables(k, ts[k])
        got = ts[k].cpu().numpy().astype(np.complex128)
        rho_g, rho_w = np.abs(got) ** 2, np.abs(want) ** 2
        dens = float(np.abs(rho_g - rho_w).max() / rho_w.max())
        mu = abs(obs["mu_total"] - o["mu_total"]) / abs(o["mu_total"])
        mum = max(abs(obs["mu"][m] - o["mu"][m]) / abs(o["mu"][m]) for m in range(3))
        print(f"scan slot {k} ({p['nx']}^2): density err {dens:.2e}, mu err {mu:.2e}, mu_m err {mum:.2e}")
        assert dens < 1e-5 and mu < 1e-6 and mum < 1e-6, k
    b.close()


def test_condensate_beyond_the_block_map_runs_alone():
    # a grouped condensate's blocks are named by map entries with 20 bits of
    # block index; beside a 48-point-wide slot the x sweep takes one row per
    # block, so 3 x 1.2M points need more blocks than that and run on their own
    # plan, while the same shape 2000 rows tall is grouped
    small = inputs.params(48, 48, 0.3, dt=0.009, c0=20.0, c2=-1.0, gamma=0.4, eta=1, rabi=0.1, omega=0.3)
    nx, ny = 3, 1_200_000
    kw = dict(dt=5e-4, c0=10.0, c2=1.0, gamma=0.2, eta=-1, rabi=0.1)
    huge = inputs.params(nx, ny, 0.1, **kw)
    short = inputs.params(nx, 2000, 0.1, **kw)
    assert ny > (1 << 20)
    if binding.plan_query(huge, True, y_solver="window")["y_solver"] != binding.GP_YSOLVER_WINDOW:
        pytest.skip("the tall grid does not window here")
    b = binding.Batch([small, short], "fp32", **SHAPES["scan"])
    b.step([dev(initial(small, 71), torch.complex64), dev(initial(short, 72), torch.complex64)], [2, 2], ["imag", "imag"])
    b.sync()
    assert b.info()["grouped"] == 2
    b.close()
    # a Gaussian strip about the centre; zero elsewhere
    psi = np.zeros((3, ny, nx), np.complex64)
    j = np.arange(ny // 2 - 400, ny // 2 + 400)
    y = (j - ny // 2) * 0.1
    x = (np.arange(nx) - nx // 2) * 0.1
    g = np.exp(-0.5 * (y[:, None] ** 2 + x[None, :] ** 2))
    rng = np.random.default_rng(70)
    for m, w in enumerate((0.25, 0.5, 0.25)):
        psi[m, j, :] = np.sqrt(w) * g * np.exp(1j * rng.uniform(-np.pi, np.pi, g.shape))
    psi /= np.sqrt((np.abs(psi.astype(np.complex128)) ** 2).sum() * 0.01)
    b = binding.Batch([small, huge], "fp32", **SHAPES["scan"])
    ts = [dev(initial(small, 71), torch.complex64), torch.from_numpy(psi).cuda()]
    b.step(ts, [3, 3], ["imag", "imag"])
    b.sync()
    info = b.info()
    assert info["individual"] == 1 and info["grouped"] == 1
    s = binding.Solver(huge, "fp32", x_solver="scan", y_solver="window")
    t = torch.from_numpy(psi).cuda()
    s.step_imag(t, 3)
    s.sync()
    assert torch.equal(ts[1], t)  # the same kernels and plan: bit for bit
    assert abs(s.observables(t)["norm_total"] - 1.0) < 1e-6
    s.close()
    b.close()


def test_more_condensates_than_one_launch_names():
    # a launch's map names at most 4096 condensates; the rest of the batch run
    # on their own plans
    n = 4100
    p = inputs.params(8, 8, 0.5, dt=0.02, c0=5.0, c2=0.5, gamma=0.3, eta=1, rabi=0.1)
    b = binding.Batch([p] * n, "fp32")
    psi = [initial(p, 80 + k % 7) for k in range(n)]
    ts = [dev(a, torch.complex64) for a in psi]
    b.step(ts, [2] * n, ["imag"] * n)
    b.sync()
    info = b.info()
    assert info["grouped"] == 4096 and info["individual"] == n - 4096
    for k in (0, 4095):
        ok, err = same(ts[k].cpu(), alone(p, psi[k], 2, "imag", "fp32", info, torch.complex64), "fp32")
        assert ok, f"slot {k}: relative L2 {err:.3e}"
    s = binding.Solver(p, "fp32")
    for k in (4096, n - 1):
        t = dev(psi[k], torch.complex64)
        s.step_imag(t, 2)
        s.sync()
        assert torch.equal(ts[k], t), k  # its own plan: bit for bit
    s.close()
    b.close()
