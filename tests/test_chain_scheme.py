"""The chain-window scheme on the host (numpy), against dense solves.

A window of W = 64 K points solves its own system with the converged pivot
from its first point and zero carries at both ends, in lanes of K points:
each lane runs its forward (backward) pass from a zero carry, and the carry
entering lane l is formed from the nc lanes before (after) it only,
c_in(l) = sum_{j=1..nc} P^{j-1} f(l - j), P = (-a m)^K.  The window writes the
points at least h from both of its ends, h the halo at which decay^h falls
below the tolerance.  With nc = ceil((h - 1) / K) every dropped carry crosses
at least h points, so every written point agrees with the exact solution to
that tolerance; one lane fewer must break it for some window (the count is
not an overestimate that a smaller one would also pass).  The tolerance here
is 1e-7 instead of the kernels' 2^-60 so that double precision resolves the
truncation.
"""
import math

import numpy as np
import pytest


def converged_pivot(a, b, e):
    # w = b - a e / w, the root with |w| > |a e / w| (the stable one)
    disc = np.sqrt(b * b - 4 * a * e)
    w1, w2 = (b + disc) / 2, (b - disc) / 2
    return w1 if abs(w1) > abs(w2) else w2


def chain_window(r, a, e, w, K, nc, past_end):
    """Solve A_inf x = r over one window (W = 64 K points) the chain way;
    past_end marks the points beyond the line end, whose forward values are
    zeroed so that no carry comes back across it."""
    m = 1.0 / w
    nam, ncp = -a * m, -e * m
    lanes = len(r) // K
    v = (m * r).reshape(lanes, K)
    # forward: value each lane passes on from a zero carry
    f = np.zeros(lanes, complex)
    for l in range(lanes):
        x = 0.0
        for k in range(K):
            x = x * nam + v[l, k]
        f[l] = x
    P = nam ** K
    z = np.zeros_like(v)
    for l in range(lanes):
        c = 0.0
        for j in range(nc, 0, -1):  # sum_{j=1..nc} P^{j-1} f(l - j)
            c = c * P + (f[l - j] if l - j >= 0 else 0.0)
        x = c
        for k in range(K):
            x = x * nam + v[l, k]
            if past_end[l * K + k]:
                x = 0.0
            z[l, k] = x
    # backward, the same way round
    b = np.zeros(lanes, complex)
    for l in range(lanes):
        x = 0.0
        for k in range(K - 1, -1, -1):
            x = x * ncp + z[l, k]
        b[l] = x
    R = ncp ** K
    out = np.zeros_like(v)
    for l in range(lanes):
        c = 0.0
        for j in range(nc, 0, -1):
            c = c * R + (b[l + j] if l + j < lanes else 0.0)
        x = c
        for k in range(K - 1, -1, -1):
            x = x * ncp + z[l, k]
            out[l, k] = x
    return out.reshape(-1)


def dense_line(n, a, b, e, w):
    """A_inf of the whole line: first diagonal entry w, then b."""
    A = np.diag(np.full(n, b, complex)) + np.diag(np.full(n - 1, a, complex), -1) + np.diag(np.full(n - 1, e, complex), 1)
    A[0, 0] = w
    return A


def worst_window_error(K, nc, h, a, b, e, rng, nwin=4):
    W = 64 * K
    L = W - 2 * h
    n = L * nwin
    w = converged_pivot(a, b, e)
    r = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    exact = np.linalg.solve(dense_line(n, a, b, e, w), r)
    worst = 0.0
    for win in range(nwin):
        s0 = win * L - h  # window covers [s0, s0 + W), writes [s0 + h, s0 + h + L)
        idx = np.arange(s0, s0 + W)
        rr = np.where((idx >= 0) & (idx < n), r[np.clip(idx, 0, n - 1)], 0.0)
        got = chain_window(rr, a, e, w, K, nc, idx >= n)
        wr = np.arange(h, h + L)
        wr = wr[(idx[wr] >= 0) & (idx[wr] < n)]
        # the first window starts at the line start: its pivot w is the line's own
        worst = max(worst, float(np.max(np.abs(got[wr] - exact[idx[wr]])) / np.max(np.abs(exact))))
    return worst


# (beta = 20 with K = 2: the halo, 68 points, does not fit a 128-point window)
@pytest.mark.parametrize("K,beta", [(2, 0.3), (2, 3.0), (4, 0.3), (4, 3.0), (4, 20.0), (8, 0.3), (8, 3.0), (8, 20.0)])
def test_chain_carries_reach_the_tolerance(K, beta):
    # CN line of the imaginary-time kinetic term with a first-derivative part:
    # b = 1 + beta, a, e = -beta / 2 -+ i c
    rng = np.random.default_rng(int(10 * beta) + K)
    a, e = -beta / 2 - 0.1j * beta, -beta / 2 + 0.1j * beta  # diagonally dominant: 2 |a| < |b|
    b = 1 + beta
    w = converged_pivot(a, b, e)
    decay = max(abs(a / w), abs(e / w))
    tol = 1e-7
    h = math.ceil(math.log(tol) / math.log(decay)) + 1
    assert 64 * K - 2 * h >= 4
    nc = max(1, math.ceil((h - 1) / K))
    assert nc * K + 1 >= h
    err = worst_window_error(K, nc, h, a, b, e, rng)
    assert err < tol, (K, beta, h, nc, err)
    if nc > 1:
        # one carry lane fewer leaves carries that crossed fewer than h points
        bad = worst_window_error(K, nc - 1, h, a, b, e, np.random.default_rng(int(10 * beta) + K))
        assert bad > err, (K, beta, h, nc, err, bad)
