"""The single-reduction order of COCG used by the FP64 kernels (CPU).

The FP64 solver on the GPU reorganises COCG (section 3.1.5.1) so that one
global reduction per iteration suffices: the product is applied to
z = D^-1 r, and with w = A z, s = A p,

    gamma = r^T z,  delta = z^T w,  mu = z^T s_old
    beta  = -mu / pi_old,   pi = delta + 2 beta mu + beta^2 pi_old,   alpha = gamma / pi
    p = z + beta p,  s = w + beta s,  x += alpha p,  z -= alpha D^-1 s.

These tests restate those formulas in numpy and pin them to the oracle's
COCG: in exact arithmetic the iterates are the same, so over a few steps on
assembled systems (where rounding has not yet separated them) x_k and the
residual norms must agree to rounding.  A wrong sign or a dropped term in
beta or pi breaks the agreement at the second step.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fem, solve


def single_reduction_steps(A, b, k):
    """k steps of the reorganised recurrence from x = 0; returns x_k and the
    residual norms ||r_j|| / ||b||, j = 0..k, with r = D z carried as z."""
    d = A.diagonal()
    dinv = 1.0 / d
    x = np.zeros_like(b)
    z = dinv * b
    p = np.zeros_like(b)
    s = np.zeros_like(b)
    pi_old = 0.0
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(d * z) / nb]
    for _ in range(k):
        w = A @ z
        r = d * z
        gamma, delta, mu = r @ z, z @ w, z @ s
        if pi_old == 0.0:
            beta, pi = 0.0, delta
        else:
            beta = -mu / pi_old
            pi = delta + 2.0 * beta * mu + beta * beta * pi_old
        alpha = gamma / pi
        p = z + beta * p
        s = w + beta * s
        x = x + alpha * p
        z = z - alpha * (dinv * s)
        pi_old = pi
        hist.append(np.linalg.norm(d * z) / nb)
    return x, np.array(hist)


def _system(name):
    rng = np.random.default_rng(5)
    if name == "free_cube_4":
        prob, waves = W.free_cube(4)
    elif name == "pec_lossy":
        prob = W.random_small(rng, n=(4, 3, 5), n_pec=3, lossy=True)
        waves = [W.random_wave(rng)]
    else:
        prob, waves = W.mirrored_pec_cube(6, cut_x=True, cut_y=True)
    A = fem.assemble(prob).tocsr()
    b = np.asarray(fem.rhs(prob, waves[:1])).reshape(A.shape[0], -1)[:, 0].astype(np.complex128)
    return A, b


@pytest.mark.parametrize("name", ["free_cube_4", "pec_lossy", "planes_6"])
def test_same_iterates_as_oracle_cocg(name):
    A, b = _system(name)
    k = 6
    ref = solve.cocg(A, b, rtol=1e-30, maxiter=k)
    assert ref.iters == k and not ref.breakdown
    x, hist = single_reduction_steps(A, b, k)
    assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    np.testing.assert_allclose(hist, ref.history, rtol=1e-9)


def test_dropping_the_cross_term_is_detected():
    """Taking pi = delta (mu's terms dropped) must not reproduce COCG, so the
    comparison above does test the conjugation terms."""
    A, b = _system("free_cube_4")
    ref = solve.cocg(A, b, rtol=1e-30, maxiter=4)
    d = A.diagonal()
    z = b / d
    p = np.zeros_like(b)
    x = np.zeros_like(b)
    for _ in range(4):
        w = A @ z
        alpha = ((d * z) @ z) / (z @ w)
        p = z
        x = x + alpha * p
        z = z - alpha * (w / d)
    assert np.linalg.norm(x - ref.x) > 1e-6 * np.linalg.norm(ref.x)
