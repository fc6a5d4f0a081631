"""Wave functions with padded component planes (gp_spin1_params.plane_stride):
every entry point must give the same bits as on a contiguous array (the
kernels only address the planes differently) and must never touch the gaps
between the planes."""
import numpy as np
import pytest

from paper_2105_10517_amd import binding, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SENTINEL = 7.0 + 7.0j


def couplings(nx, ny, dx, dy, dt, **kw):
    base = dict(c0=35.0, c2=-3.0, gamma=0.6, eta=1, rabi=0.25, omega=0.45)
    base.update(kw)
    return inputs.params(nx, ny, dx, dy=dy, dt=dt, **base)


def padded(psi, p, dtype):
    t, q = binding.padded_psi(psi, p, dtype, DEV)
    buf = t.as_strided((t.untyped_storage().nbytes() // t.element_size(),), (1,), 0)
    gaps = []
    n = p["nx"] * p["ny"]
    for m in range(2):
        g = buf[m * q["plane_stride"] + n:(m + 1) * q["plane_stride"]]
        g.fill_(SENTINEL)
        gaps.append(g)
    return t, q, gaps


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(300, 200), (256, 256)])
def test_padded_planes_match_contiguous(precision, shape):
    nx, ny = shape
    dtype = torch.complex128 if precision == "fp64" else torch.complex64
    p = couplings(nx, ny, 0.06, 0.05, 0.0015)
    psi0 = inputs.gaussian(nx, ny, 0.06, 0.05, x0=p["x0"], y0=p["y0"], seed=17, center=(2.0, -1.0))
    a = torch.from_numpy(psi0).to(dtype).to(DEV)
    b, q, gaps = padded(psi0, p, dtype)
    assert tuple(b.stride()) == (q["plane_stride"], nx, 1)
    sa, sb = binding.Solver(p, precision), binding.Solver(q, precision)
    for s, t in ((sa, a), (sb, b)):
        s.step_imag(t, 9)
        s.step_real(t, 7)
        for which in range(4):
            s.substep(t, which, which % 2 == 0)
        s.sync()
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    da = torch.empty(3, ny, nx, dtype=sa.real_dtype, device=DEV)
    db = torch.empty_like(da)
    oa, ob = sa.observables(a, da), sb.observables(b, db)
    assert oa == ob and torch.equal(da, db)
    for g in gaps:
        assert bool((g == SENTINEL).all())
    # a contiguous tensor is refused by the padded handle, and the other way round
    with pytest.raises(ValueError):
        sb.step_real(a, 1)
    with pytest.raises(ValueError):
        sa.step_real(b, 1)
    sa.close()
    sb.close()


def test_padded_planes_in_a_batch():
    dtype = torch.complex64
    ps = [couplings(96, 80, 0.12, 0.12, 0.0015, omega=0.3 + 0.1 * k) for k in range(3)]
    psis = [inputs.gaussian(96, 80, 0.12, 0.12, x0=p["x0"], y0=p["y0"], seed=30 + k) for k, p in enumerate(ps)]
    plain = [torch.from_numpy(x).to(dtype).to(DEV) for x in psis]
    pads = [padded(x, p, dtype) for x, p in zip(psis, ps)]
    ba = binding.Batch(ps, "fp32")
    bb = binding.Batch([q for _, q, _ in pads], "fp32")
    modes = ["imag", "real", "imag"]
    ba.step(plain, [5, 6, 7], modes)
    bb.step([t for t, _, _ in pads], [5, 6, 7], modes)
    ba.sync()
    bb.sync()
    for t, (u, _, gaps) in zip(plain, pads):
        assert np.array_equal(t.cpu().numpy(), u.cpu().numpy())
        for g in gaps:
            assert bool((g == SENTINEL).all())
    ba.close()
    bb.close()
