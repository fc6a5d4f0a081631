"""Steps replayed from captured HIP graphs (gp_spin1_step_graph).

A graph holds the launch sequence of the stepping calls, so every replay must
equal the same steps run eagerly, bit for bit.  Each graph is replayed several
times with eager work and synchronisations of the program between the
replays, and every replay is checked (imaginary time with the folded and the
separate norm kernels, real time, both precisions, the chain windows, Strang
splitting), and against the oracle once.
"""
import numpy as np
import pytest

import oracle
from paper_2105_10517_amd import binding, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def all_couplings(nx, ny, dx, dy=None, dt=0.01, **kw):
    base = dict(c0=35.0, c2=-3.0, gamma=0.6, eta=1, rabi=0.25, omega=0.45)
    base.update(kw)
    return inputs.params(nx, ny, dx, dy=dy, dt=dt, **base)


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(DEV)


CASES = [
    # (nx, ny, dx, dt, solver options, split)
    (128, 128, 0.1, 5e-4, {}, 0),                                 # small grid: norm folded into the x sweep
    (300, 260, 0.06, 0.0015, {"x_solver": "chain", "y_solver": "stack"}, 0),
    (200, 150, 0.08, 0.002, {}, 1),                               # Strang splitting
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_equal_eager_steps(case, imag, precision):
    nx, ny, dx, dt, kw, split = CASES[case]
    p = all_couplings(nx, ny, dx, dt=dt, split=split)
    psi0 = inputs.gaussian(nx, ny, dx, dx, x0=p["x0"], y0=p["y0"], seed=30 + case)
    s = binding.Solver(p, precision, **kw)
    step = s.step_imag if imag else s.step_real
    n = 7
    g = dev(psi0, s.dtype)   # advanced by graph replays
    e = dev(psi0, s.dtype)   # advanced eagerly, the same steps
    other = dev(psi0, s.dtype)
    for rep in range(4):
        s.step_graph(g, n, imag)
        # the program's own eager work between replays (another wave function, a sync)
        step(other, 3)
        s.sync()
        step(e, n)
        s.sync()
        assert torch.equal(g, e), (case, imag, precision, rep)
    # a second graph (other step count) beside the first, then the first again
    s.step_graph(g, 2, imag)
    step(e, 2)
    s.step_graph(g, n, imag)
    step(e, n)
    s.sync()
    assert torch.equal(g, e)
    if precision == "fp64" and case == 0:
        want = oracle.step(p, psi0, 4 * n + 2 + n, imag)
        got = g.cpu().numpy()
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-11
    s.close()


def test_graph_refuses_bad_arguments():
    p = all_couplings(64, 64, 0.2, dt=0.01)
    s = binding.Solver(p)
    t = dev(inputs.gaussian(64, 64, 0.2, 0.2, seed=1), torch.complex128)
    with pytest.raises(binding.GPError) as ei:
        s.step_graph(t, -1, True)
    assert ei.value.status == binding.GP_EINVAL
    s.step_graph(t, 0, True)  # zero steps: nothing captured, nothing run
    s.sync()
    s.close()
