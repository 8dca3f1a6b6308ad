"""Pins of the oracle's O(p^3) M2L (rotate the offset onto +z, translate along
z, rotate back; the O(P^3) end of the operator cost range of Section III.A):
Wigner's d-matrices against their closed forms at degree 1, orthogonality and
the rotation law of the oracle's own harmonics, and the rotation M2L against
the dense M2L of the addition theorem (pinned elsewhere against the direct
sum)."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def test_wigner_degree_one_closed_form():
    # the textbook table of d^1(b), rows and columns m = -1, 0, 1
    for b in (0.0, 0.4, 1.3, math.pi / 2, 2.9, math.pi):
        c, s = math.cos(b), math.sin(b)
        want = np.array([[(1 + c) / 2, s / math.sqrt(2), (1 - c) / 2],
                         [-s / math.sqrt(2), c, s / math.sqrt(2)],
                         [(1 - c) / 2, -s / math.sqrt(2), (1 + c) / 2]])
        assert np.allclose(oracle.wigner_d(1, b), want, atol=1e-15), b


@pytest.mark.parametrize("n", [0, 2, 5, 9, 12, 15])
def test_wigner_orthogonal_identity_and_composition(n):
    tol = 1e-13 if n <= 9 else 1e-11
    for b in (0.3, 1.1, math.pi / 2, 2.7):
        d = oracle.wigner_d(n, b)
        assert np.abs(d @ d.T - np.eye(2 * n + 1)).max() < tol
        # rotations about one axis compose: d(a) d(b) = d(a + b)
        assert np.abs(oracle.wigner_d(n, 0.2) @ d - oracle.wigner_d(n, b + 0.2)).max() < tol
    assert np.abs(oracle.wigner_d(n, 0.0) - np.eye(2 * n + 1)).max() < 1e-14


def _ry(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


@pytest.mark.parametrize("n", [1, 3, 7, 11])
def test_wigner_rotates_the_oracles_harmonics(n):
    # C_n^m(Ry(b)^-1 u) = sum_k d^n_{k m}(b) C_n^k(u), with C_n^m = s_m R_n^m
    # for a unit vector (s_m = sqrt((n+m)!(n-m)!)), the law the rotation M2L
    # relies on
    rng = np.random.default_rng(40 + n)
    b = 0.83
    d = oracle.wigner_d(n, b)
    sm = np.array([math.sqrt(math.factorial(n + m) * math.factorial(n - m)) for m in range(-n, n + 1)])
    for _ in range(4):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        R = np.zeros(2 * (n + 1) ** 2)
        oracle.lib().oracle_harmonics(oracle._d(u), n + 1, oracle._d(R), None)
        Cu = (R.view(np.complex128)[n * n:(n + 1) ** 2]) * sm
        v = _ry(b).T @ u
        R2 = np.zeros(2 * (n + 1) ** 2)
        oracle.lib().oracle_harmonics(oracle._d(v), n + 1, oracle._d(R2), None)
        Cv = (R2.view(np.complex128)[n * n:(n + 1) ** 2]) * sm
        assert np.abs(Cv - d.T @ Cu).max() < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 6, 10, 12, 16])
def test_rotation_m2l_equals_dense_m2l(p):
    rng = np.random.default_rng(100 + p)
    offsets = [rng.normal(size=3) * 3.0 for _ in range(4)]
    # on the axis (both directions), in the plane z = 0, along -y
    offsets += [np.array([0.0, 0.0, 2.5]), np.array([0.0, 0.0, -2.5]), np.array([2.0, 1.0, 0.0]),
                np.array([0.0, -3.0, 0.0])]
    tol = 1e-12 if p <= 12 else 1e-11
    for D in offsets:
        M = rng.normal(size=p * p) + 1j * rng.normal(size=p * p)
        cB = rng.normal(size=3)
        a = oracle.op_m2l(M, cB, cB + D, p)
        b = oracle.op_m2l_rot(M, cB, cB + D, p)
        assert np.abs(a - b).max() <= tol * np.abs(a).max(), (p, D)


def test_rotation_m2l_planted_mistake_is_seen():
    # dropping the back-rotation's phase (a plausible slip) must fail the pin:
    # emulate it by rotating the offset about z, which leaves the axial
    # translation alone but not the local coefficients
    p = 6
    rng = np.random.default_rng(7)
    M = rng.normal(size=p * p) + 1j * rng.normal(size=p * p)
    D = np.array([1.5, 2.0, 1.0])
    a = oracle.op_m2l(M, np.zeros(3), D, p)
    Dz = np.array([-2.0, 1.5, 1.0])  # D turned by 90 degrees about z
    b = oracle.op_m2l_rot(M, np.zeros(3), Dz, p)
    assert np.abs(a - b).max() > 1e-3 * np.abs(a).max()
