"""Pins of the oracle's solid harmonics and of its five expansion operators.

Each check compares against something the oracle does not compute itself:
scipy's Legendre functions, the Legendre addition theorem, the closed form of
the axisymmetric double series, bidegree Taylor coefficients of 1/|D+t-a|
extracted by contour integration (2-D FFT), and exactness identities of the
translations (degree < p is preserved exactly by M2M and L2L).
"""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, lpmv

import oracle


def _cos(u, v):
    return float(np.dot(u, v) / (np.linalg.norm(u) * np.linalg.norm(v)))


@pytest.mark.parametrize("xv", [-0.93, -0.2, 0.0, 0.41, 0.999])
def test_legendre_matches_scipy(xv):
    nmax = 14
    P = oracle.legendre(xv, nmax)
    for n in range(nmax):
        for m in range(n + 1):
            ref = lpmv(m, n, xv)  # includes the Condon-Shortley phase
            # absolute slack on the function's natural scale sqrt((n+m)!/(n-m)!)
            scale = math.sqrt(math.factorial(n + m) / math.factorial(n - m))
            assert P[n * (n + 1) // 2 + m] == pytest.approx(ref, rel=1e-11, abs=1e-14 * scale)


def test_regular_harmonics_on_axis_and_homogeneity():
    z = 0.7
    R, _ = oracle.harmonics([0.0, 0.0, z], 10)
    for n in range(10):
        for m in range(-n, n + 1):
            exp = z ** n / math.factorial(n) if m == 0 else 0.0
            assert abs(R[n * n + n + m] - exp) < 1e-15
    v = np.array([0.3, -0.45, 0.2])
    R1, I1 = oracle.harmonics(v, 9)
    R2, I2 = oracle.harmonics(2.5 * v, 9)
    for n in range(9):
        sl = slice(n * n, (n + 1) * (n + 1))
        assert np.allclose(R2[sl], 2.5 ** n * R1[sl], rtol=1e-13, atol=1e-300)
        assert np.allclose(I2[sl], 2.5 ** (-n - 1) * I1[sl], rtol=1e-13, atol=1e-300)


def test_inverse_distance_expansion():
    # 1/|x - y| = sum_{n,m} conj(R_n^m(y)) I_n^m(x) for |y| < |x|
    x = np.array([0.9, -1.1, 0.7])
    y = np.array([-0.2, 0.15, 0.3])
    nmax = 32
    R, _ = oracle.harmonics(y, nmax)
    _, I = oracle.harmonics(x, nmax)
    s = np.sum(np.conj(R) * I)
    assert abs(s.imag) < 1e-14
    assert s.real == pytest.approx(1.0 / np.linalg.norm(x - y), rel=1e-13)


def test_regular_addition_theorem():
    # R_n^m(a + b) = sum_{k<=n, l} R_k^l(a) R_{n-k}^{m-l}(b): the identity
    # behind M2M and L2L
    a = np.array([0.31, -0.22, 0.17])
    b = np.array([-0.12, 0.4, 0.26])
    nmax = 8
    Ra, _ = oracle.harmonics(a, nmax)
    Rb, _ = oracle.harmonics(b, nmax)
    Rab, _ = oracle.harmonics(a + b, nmax)

    def g(H, n, m):
        return H[n * n + n + m] if (0 <= n and abs(m) <= n) else 0.0

    for n in range(nmax):
        for m in range(-n, n + 1):
            s = sum(g(Ra, k, l) * g(Rb, n - k, m - l) for k in range(n + 1) for l in range(-k, k + 1))
            assert abs(s - g(Rab, n, m)) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 12])
def test_p2m_matches_legendre_addition_theorem(p):
    # one charge at c + s, multipole series at c + x:
    # q sum_{n<p} |s|^n / |x|^{n+1} P_n(cos gamma)
    c = np.array([0.1, 0.2, -0.3])
    s = np.array([0.05, -0.11, 0.07])
    q = -1.7
    M = oracle.op_p2m((c + s)[None], np.array([q]), c, p)
    for xv in ([0.9, 0.3, -0.4], [-0.2, -0.6, 0.5]):
        xv = np.array(xv)
        got = oracle.op_m2p(M, c, p, c + xv)
        g = _cos(s, xv)
        ref = q * sum(np.linalg.norm(s) ** n / np.linalg.norm(xv) ** (n + 1) * eval_legendre(n, g) for n in range(p))
        assert got == pytest.approx(ref, rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("p", [1, 4, 7, 10])
def test_local_expansion_of_a_far_charge(p):
    # unit charge at c_B (multipole = monopole), M2L to c_A, evaluate at
    # c_A + t: sum_{j<p} |t|^j / |D|^{j+1} P_j(cos gamma), gamma between t
    # and -D
    cB = np.array([0.0, 0.0, 0.0])
    cA = np.array([1.3, -0.7, 0.9])
    D = cA - cB
    M = oracle.op_p2m(cB[None], np.array([1.0]), cB, p)
    L = oracle.op_m2l(M, cB, cA, p)
    for t in ([0.1, 0.05, -0.2], [-0.15, 0.12, 0.03]):
        t = np.array(t)
        phi, _ = oracle.op_l2p(L, cA, p, (cA + t)[None])
        g = _cos(t, -D)
        ref = sum(np.linalg.norm(t) ** j / np.linalg.norm(D) ** (j + 1) * eval_legendre(j, g) for j in range(p))
        assert phi[0] == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("p", [2, 4, 8, 10])
def test_m2l_axisymmetric_closed_form(p):
    # everything on the z axis: result sum_{n,j<p} C(n+j,n) a^n (-t)^j / D^{n+j+1}
    D, a, t = 2.0, 0.3, -0.25
    cB = np.zeros(3)
    cA = np.array([0.0, 0.0, D])
    M = oracle.op_p2m(np.array([[0.0, 0.0, a]]), np.array([1.0]), cB, p)
    L = oracle.op_m2l(M, cB, cA, p)
    phi, _ = oracle.op_l2p(L, cA, p, np.array([[0.0, 0.0, D + t]]))
    ref = sum(math.comb(n + j, n) * a ** n * (-t) ** j / D ** (n + j + 1) for n in range(p) for j in range(p))
    assert phi[0] == pytest.approx(ref, rel=1e-14)


def _bidegree_taylor(t, D, a, p, K=48):
    """K_p(t, D, a): sum over j<p, n<p of the (alpha^j beta^n) Taylor
    coefficients of 1/|D + alpha t - beta a|, from a 2-D trapezoidal contour
    integral on |alpha| = |beta| = 1 (requires |t| + |a| <~ 0.3 |D|)."""
    w = np.exp(2j * np.pi * np.arange(K) / K)
    al = w[:, None]
    be = w[None, :]
    v = [D[d] + al * t[d] - be * a[d] for d in range(3)]
    f = 1.0 / np.sqrt(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    c = np.fft.fft2(f) / (K * K)  # c[j, n] multiplies alpha^j beta^n
    return c[:p, :p].sum().real


@pytest.mark.parametrize("p", [1, 3, 6, 9])
def test_p2m_m2l_l2p_equals_bidegree_taylor(p):
    rng = np.random.default_rng(p)
    for _ in range(3):
        D = rng.normal(size=3)
        D *= 1.5 / np.linalg.norm(D)
        a = rng.normal(size=3); a *= 0.2 / np.linalg.norm(a)
        t = rng.normal(size=3); t *= 0.22 / np.linalg.norm(t)
        cB = rng.normal(size=3)
        cA = cB + D
        M = oracle.op_p2m((cB + a)[None], np.array([1.0]), cB, p)
        L = oracle.op_m2l(M, cB, cA, p)
        phi, _ = oracle.op_l2p(L, cA, p, (cA + t)[None])
        assert phi[0] == pytest.approx(_bidegree_taylor(t, D, a, p), rel=1e-12)


def test_l2p_field_is_minus_gradient_of_its_potential():
    p = 7
    cB = np.zeros(3)
    cA = np.array([0.9, 1.1, -0.8])
    rng = np.random.default_rng(5)
    xs = cB + 0.1 * rng.normal(size=(6, 3))
    M = oracle.op_p2m(xs, rng.uniform(-1, 1, 6), cB, p)
    L = oracle.op_m2l(M, cB, cA, p)
    x0 = cA + np.array([0.07, -0.05, 0.11])
    _, E = oracle.op_l2p(L, cA, p, x0[None])
    h = 1e-5
    g = np.zeros(3)
    for d in range(3):
        e = np.zeros(3); e[d] = h
        pp, _ = oracle.op_l2p(L, cA, p, (x0 + e)[None])
        pm, _ = oracle.op_l2p(L, cA, p, (x0 - e)[None])
        g[d] = (pp[0] - pm[0]) / (2 * h)
    assert np.allclose(E[0], -g, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("p", [2, 5, 8, 12])
def test_m2m_is_exact(p):
    rng = np.random.default_rng(10 + p)
    cpar = np.array([0.5, 0.5, 0.5])
    cch = cpar + 0.125 * np.array([1, -1, 1])
    xs = cch + 0.125 * (rng.random((20, 3)) - 0.5)
    q = rng.uniform(-1, 1, 20)
    Mch = oracle.op_p2m(xs, q, cch, p)
    Mpar_direct = oracle.op_p2m(xs, q, cpar, p)
    Mpar = oracle.op_m2m(Mch, cch, cpar, p)
    scale = np.abs(Mpar_direct).max()
    assert np.abs(Mpar - Mpar_direct).max() < 1e-14 * scale


@pytest.mark.parametrize("p", [2, 5, 8, 12])
def test_l2l_is_exact(p):
    rng = np.random.default_rng(20 + p)
    cB = np.array([3.0, -1.0, 2.0])
    xs = cB + 0.2 * (rng.random((10, 3)) - 0.5)
    M = oracle.op_p2m(xs, rng.uniform(-1, 1, 10), cB, p)
    cpar = np.array([0.0, 0.0, 0.0])
    L = oracle.op_m2l(M, cB, cpar, p)
    cch = cpar + 0.25 * np.array([-1, 1, 1])
    Lch = oracle.op_l2l(L, cpar, cch, p)
    pts = cch + 0.25 * (rng.random((5, 3)) - 0.5)
    f1, E1 = oracle.op_l2p(L, cpar, p, pts)
    f2, E2 = oracle.op_l2p(Lch, cch, p, pts)
    assert np.allclose(f2, f1, rtol=1e-13, atol=1e-16)
    assert np.allclose(E2, E1, rtol=1e-12, atol=1e-15)


def test_m2m_then_m2l_equals_m2l_from_the_parent_center():
    p = 6
    rng = np.random.default_rng(3)
    cpar = np.zeros(3)
    cch = np.array([0.1, 0.1, -0.1])
    xs = cch + 0.1 * (rng.random((12, 3)) - 0.5)
    q = rng.uniform(-1, 1, 12)
    cA = np.array([1.6, 0.4, -1.2])
    L1 = oracle.op_m2l(oracle.op_m2m(oracle.op_p2m(xs, q, cch, p), cch, cpar, p), cpar, cA, p)
    L2 = oracle.op_m2l(oracle.op_p2m(xs, q, cpar, p), cpar, cA, p)
    assert np.abs(L1 - L2).max() < 1e-13 * np.abs(L2).max()
