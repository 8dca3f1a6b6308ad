"""Pins of the oracle's direct sum (the plain definition the FMM approximates).

phi_i = sum_{j: x_j != x_i} q_j/|x_i - x_j|,  E_i = -grad_i phi_i
(kernel without 1/(4 pi), coincident pairs skipped).
"""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle


def _bodies(n, seed, dup=0):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3))
    q = rng.uniform(-1, 1, n)
    if dup:
        x[-dup:] = x[:dup]  # coincident bodies: their mutual term is skipped
    return x, q


def test_direct_matches_vectorised_library_evaluation():
    # scipy's pairwise distance matrix; a different summation route entirely
    x, q = _bodies(300, 1, dup=5)
    phi, E = oracle.direct(x, q)
    r = cdist(x, x)
    with np.errstate(divide="ignore"):
        inv = np.where(r > 0, 1.0 / r, 0.0)
    phi_ref = inv @ q
    inv3 = inv ** 3
    E_ref = np.einsum("ij,j,ijd->id", inv3, q, x[:, None, :] - x[None, :, :])
    assert np.allclose(phi, phi_ref, rtol=1e-13, atol=1e-12)
    assert np.allclose(E, E_ref, rtol=1e-12, atol=1e-11)


def test_two_body_closed_form():
    x = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    q = np.array([2.0, -5.0])
    phi, E = oracle.direct(x, q)
    assert phi[0] == pytest.approx(-1.0, rel=1e-15)        # -5/5
    assert phi[1] == pytest.approx(0.4, rel=1e-15)          # 2/5
    # E_0 = q_1 (x_0 - x_1)/r^3 = -5 * (-3,-4,0)/125
    assert np.allclose(E[0], [0.12, 0.16, 0.0], rtol=1e-15)


def test_newtons_third_law_and_translation_invariance():
    x, q = _bodies(400, 2)
    phi, E = oracle.direct(x, q)
    F = q[:, None] * E
    assert np.abs(F.sum(0)).max() < 1e-10 * np.abs(F).sum()
    phi2, E2 = oracle.direct(x + np.array([0.25, -0.5, 0.125]), q)
    assert np.allclose(phi2, phi, rtol=1e-12)
    assert np.allclose(E2, E, rtol=1e-10, atol=1e-12)


def test_field_is_minus_gradient():
    x, q = _bodies(64, 3)
    h = 1e-5
    _, E = oracle.direct(x, q, targets=np.array([7]))
    g = np.zeros(3)
    for d in range(3):
        xp = x.copy(); xp[7, d] += h
        xm = x.copy(); xm[7, d] -= h
        pp, _ = oracle.direct(xp, q, targets=np.array([7]))
        pm, _ = oracle.direct(xm, q, targets=np.array([7]))
        g[d] = (pp[0] - pm[0]) / (2 * h)
    assert np.allclose(E[0], -g, rtol=1e-6, atol=1e-6)


def test_energy_symmetry_and_targets_subset():
    x, q = _bodies(500, 4)
    w = np.random.default_rng(9).uniform(-1, 1, 500)
    pq, _ = oracle.direct(x, q)
    pw, _ = oracle.direct(x, w)
    assert abs(w @ pq - q @ pw) < 1e-12 * (np.abs(w) @ np.abs(pq))
    t = np.array([0, 17, 499, 250])
    ps, Es = oracle.direct(x, q, targets=t)
    _, E = oracle.direct(x, q)
    assert np.array_equal(ps, pq[t]) and np.array_equal(Es, E[t])
