"""The line-solve scheme of the GPU sweeps, checked on the host against dense
solves (no GPU, no library): every point of a tridiagonal Crank-Nicolson line
is eliminated with the converged Thomas pivots, the carries are cut at the
line ends, the blocks of K points held by the threads are joined by
scans of their affine transfer maps, and the line start is corrected by the
rank-one (Sherman-Morrison) term, since the converged pivots factor the matrix
whose first diagonal entry is the limit pivot w instead of b:
A = A_inf + (b - w) e0 e0^T,  A^{-1} r = z - (b - w) z_0 g / (1 + (b - w) g_0),
z = A_inf^{-1} r, g = A_inf^{-1} e0.  Lines are padded on both sides as in the
windowed kernels (points outside [0, n) are held but not part of the line)."""
import numpy as np
import pytest


def limit_pivot(a, b, e):
    w1 = (b + np.sqrt(b * b - 4 * a * e)) / 2
    w2 = (b - np.sqrt(b * b - 4 * a * e)) / 2
    return w1 if abs(w1) >= abs(w2) else w2  # the attracting fixed point of w -> b - a e / w


def partitioned_solve(a, b, e, r, n, K, start, nthreads):
    w = limit_pivot(a, b, e)
    m, nam, ncp = 1 / w, -a / w, -e / w
    idx = [[start + t * K + k for k in range(K)] for t in range(nthreads)]
    rr, maps = [], []
    for t in range(nthreads):
        E, P, blk = 0j, 1 + 0j, []
        for i in idx[t]:
            na = 0 if i <= 0 else nam  # no carry into the line start
            E = na * E + m * (r[i] if 0 <= i < n else 0)
            P *= na
            blk.append(E)
        rr.append(blk)
        maps.append((P, E))
    carry = 0j
    for t in range(nthreads):  # forward exclusive scan, then the carry times the running product
        Q = 1 + 0j
        for k, i in enumerate(idx[t]):
            Q *= 0 if i <= 0 else nam
            rr[t][k] += carry * Q
        carry = maps[t][0] * carry + maps[t][1]
    bmaps = []
    for t in range(nthreads):
        G, R = 0j, 1 + 0j
        for k in range(K - 1, -1, -1):
            nc = 0 if idx[t][k] >= n - 1 else ncp  # no carry past the line end
            G = nc * G + rr[t][k]
            R *= nc
            rr[t][k] = G
        bmaps.append((R, G))
    z = np.zeros(n, dtype=complex)
    carry = 0j
    for t in range(nthreads - 1, -1, -1):
        S = 1 + 0j
        for k in range(K - 1, -1, -1):
            i = idx[t][k]
            S *= 0 if i >= n - 1 else ncp
            if 0 <= i < n:
                z[i] = carry * S + rr[t][k]
        carry = bmaps[t][0] * carry + bmaps[t][1]
    # the rank-one line-start correction
    A_inf = np.diag(np.full(n, b, dtype=complex)) + np.diag(np.full(n - 1, a), -1) + np.diag(np.full(n - 1, e), 1)
    A_inf[0, 0] = w
    g = np.linalg.solve(A_inf, np.eye(n)[0])
    return z - (b - w) * z[0] / (1 + (b - w) * g[0]) * g


@pytest.mark.parametrize("seed", range(6))
def test_scheme_matches_dense_solves(seed):
    rng = np.random.default_rng(seed)
    for _ in range(40):
        n = int(rng.integers(3, 150))
        K = int(rng.choice([1, 2, 4, 8]))
        # alpha = i dt/2 (real time) or dt/2 (imaginary time) over dx^2, first-derivative part c
        alpha = complex(0, rng.uniform(0.01, 3)) if rng.random() < 0.5 else complex(rng.uniform(0.01, 3), 0)
        c = complex(0, rng.uniform(-0.6, 0.6))
        a, e, b = -alpha * (1 - c), -alpha * (1 + c), 1 + 2 * alpha
        r = rng.normal(size=n) + 1j * rng.normal(size=n)
        A = np.diag(np.full(n, b)) + np.diag(np.full(n - 1, a), -1) + np.diag(np.full(n - 1, e), 1)
        start = -int(rng.integers(0, 3 * K)) if rng.random() < 0.5 else 0
        nthreads = (n - start + K - 1) // K + int(rng.integers(0, 3))
        got = partitioned_solve(a, b, e, r, n, K, start, nthreads)
        want = np.linalg.solve(A, r)
        assert np.abs(got - want).max() < 1e-11 * np.abs(want).max(), (n, K, start)


def test_without_the_correction_the_start_is_wrong():
    # the converged pivots alone solve A_inf, not A: the correction is what makes the scheme exact
    a, e, b = -0.8j, -0.8j, 1 + 1.6j
    n = 40
    r = np.arange(1, n + 1) + 0j
    A = np.diag(np.full(n, b)) + np.diag(np.full(n - 1, a), -1) + np.diag(np.full(n - 1, e), 1)
    w = limit_pivot(a, b, e)
    A_inf = A.copy()
    A_inf[0, 0] = w
    z = np.linalg.solve(A_inf, r)
    want = np.linalg.solve(A, r)
    assert np.abs(z - want)[0] > 1e-3 * np.abs(want).max()
    assert np.allclose(partitioned_solve(a, b, e, r, n, 4, 0, 10), want, rtol=0, atol=1e-12 * np.abs(want).max())
