"""gp_spin1_step_static: steps without device allocation (a static scratch
array per GPU) against the handle path with the same parameters, which runs
the same kernels with the same launch plan: FP64 to the 1e-13 bar of a few
steps (bit-identical in practice), FP32 to 2e-6 relative L2.  Two calls in a
row, the second on a smaller grid (the array keeps the first call's
contents), both propagation modes; a grid larger than the array and a request
for autotuning are refused."""
import numpy as np
import pytest

import oracle
from paper_2105_10517_amd import binding, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def couplings(nx, ny, dx, dy, dt):
    return inputs.params(nx, ny, dx, dy=dy, dt=dt, c0=60.0, c2=-4.0, gamma=0.7, eta=-1, rabi=0.2, omega=0.5)


def handle_run(p, psi0, n, mode, prec):
    s = binding.Solver(p, prec)
    t = torch.from_numpy(psi0).to(s.dtype).to(DEV)
    (s.step_imag if mode == "imag" else s.step_real)(t, n)
    s.sync()
    out = t.cpu().numpy().astype(np.complex128)
    s.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_static_steps_match_the_handle_path(prec):
    dtype = torch.complex128 if prec == "fp64" else torch.complex64
    tol = 1e-13 if prec == "fp64" else 2e-6
    cases = [(couplings(300, 260, 0.06, 0.07, 0.002), 25), (couplings(180, 150, 0.08, 0.08, 0.003), 17)]
    for mode in ("imag", "real"):
        for k, (p, n) in enumerate(cases):  # the second call on a smaller grid
            psi0 = inputs.gaussian(p["nx"], p["ny"], p["dx"], p["dy"], x0=p["x0"], y0=p["y0"], seed=70 + k)
            t = torch.from_numpy(psi0).to(dtype).to(DEV)
            binding.step_static(p, t, n, mode, prec)
            got = t.cpu().numpy().astype(np.complex128)
            want = handle_run(p, psi0, n, mode, prec)
            err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
            print(f"{prec} {mode} {p['nx']}x{p['ny']}: rel L2 vs handle {err:.2e}, identical {np.array_equal(got, want)}")
            assert err <= tol, (prec, mode, k, err)
            if prec == "fp64" and k == 0:
                ref = oracle.step(p, psi0, n, mode == "imag")
                assert float(np.linalg.norm(got - ref) / np.linalg.norm(ref)) < 1e-12


def test_static_refusals():
    p = couplings(1200, 1200, 0.02, 0.02, 4e-5)  # 69 MB of FP64 work wave function
    t = torch.zeros((3, 1200, 1200), dtype=torch.complex128, device=DEV)
    with pytest.raises(binding.GPError) as ei:
        binding.step_static(p, t, 1, "imag", "fp64")
    assert ei.value.status == binding.GP_ENOMEM and "static scratch" in str(ei.value)
    q = dict(couplings(64, 64, 0.2, 0.2, 0.005))
    t = torch.from_numpy(inputs.gaussian(64, 64, 0.2, 0.2, seed=1)).to(DEV)
    lib = binding.load()
    pp = binding.make_params(q, "fp64", autotune=True)
    import ctypes
    rc = lib.gp_spin1_step_static(ctypes.byref(pp), ctypes.c_void_p(t.data_ptr()), 1, 0,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == binding.GP_EINVAL
    # after the refusals, a good call still runs
    binding.step_static(q, t, 3, "real", "fp64")
