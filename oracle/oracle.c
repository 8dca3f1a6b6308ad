/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the per-rank fast multipole
 * evaluation whose hot path the HIP library implements.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg load it; the
 * product path never links, loads or calls anything in this directory, and
 * this file shares no code, header, table or helper with the HIP library.
 *
 * What it computes (paper: Section II.A, the six FMM operators P2M, M2M,
 * M2L, L2L, L2P, P2P; Section II.C, upward pass, dual tree traversal and
 * downward pass; Section III and Table I, parameters P, theta, N_crit):
 *
 *   direct sum     phi_i = sum_{j: x_j != x_i} q_j / |x_i - x_j|,
 *                  E_i   = sum_{j: x_j != x_i} q_j (x_i - x_j) / |x_i - x_j|^3
 *                  (the plain definition that the FMM approximates)
 *   local octree   root cube from the local bounding box, 64-bit Morton keys
 *                  (3 bits per level, 21 levels; Section II.B), stable sort,
 *                  a cell is split while it holds more than N_crit bodies
 *   dual traversal recursive cell-pair walk (Section II.C, after Dehnen 2002)
 *                  emitting M2L pairs (acceptance criterion met) and P2P
 *                  pairs (both leaves), with a symmetric split rule
 *   expansions     complex solid harmonics of degree n < p built from their
 *                  textbook definition (associated Legendre functions and
 *                  e^{i m phi}); translations from the addition theorem of
 *                  the regular solid harmonics
 *   M2L by rotation the O(P^3) form of the same operator (Section III.A):
 *                  rotate D onto +z with Wigner's explicit d-matrices,
 *                  translate along z, rotate back
 *   mutual P2P     the near field with every unordered body pair of the
 *                  P2P lists evaluated once and both bodies updated (mutual
 *                  interactions, listed among the features in Section II.C)
 *
 * Every target output is accumulated by one thread in a fixed order, so the
 * result is bit-identical for any OpenMP thread count.
 *
 * Pins (tests/test_oracle_*.py): direct sum against an independent
 * vectorised evaluation and physical invariants; Legendre functions against
 * scipy; multipole and local series against the Legendre addition theorem;
 * M2L against the axisymmetric closed form and against bidegree Taylor
 * coefficients extracted by contour integrals; M2M/L2L exactness; the tree
 * against an independent recursive octree and published cell counts; list
 * invariants and lattice counts; the a priori error bound of the whole FMM;
 * energy symmetry; scaling and axis-permutation invariance; frozen-tree
 * finite differences; Wigner matrices against closed forms, orthogonality
 * and the rotation of the harmonics; rotation M2L against the dense M2L;
 * the mutual near field against a numpy sum over the exported P2P list, the
 * direct sum and Newton's third law.
 * No function here is "parity unpinned".
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_MAXP 16
#define ORC_LEVELS 21
#define ORC_HMAX (2 * ORC_MAXP) /* harmonics needed up to degree 2p-2 */

/* ------------------------------------------------------------------------ */
/* Direct sum: the plain definition of potential and field.                 */
/* ------------------------------------------------------------------------ */

/* targets == NULL: every body is a target (outputs in input order, n rows);
 * otherwise nt target indices, outputs in target order.                    */
int oracle_direct(int64_t n, const double *x, const double *q, int64_t nt,
                  const int64_t *targets, double *phi, double *field)
{
    if (n < 0 || nt < 0 || (n > 0 && (!x || !q))) return 1;
    int64_t ntg = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ntg; ++t) {
        int64_t i = targets ? targets[t] : t;
        double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
        double p = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double dx = xi - x[3 * j], dy = yi - x[3 * j + 1], dz = zi - x[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            double qr = q[j] / r;
            double qr3 = qr / r2;
            p += qr;
            ex += qr3 * dx;
            ey += qr3 * dy;
            ez += qr3 * dz;
        }
        if (phi) phi[t] = p;
        if (field) {
            field[3 * t] = ex;
            field[3 * t + 1] = ey;
            field[3 * t + 2] = ez;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Associated Legendre functions and solid harmonics (textbook definitions). */
/* ------------------------------------------------------------------------ */

static double fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

#define PIDX(n, m) ((n) * ((n) + 1) / 2 + (m))
#define HIDX(n, m) ((n) * (n) + (n) + (m))

/* P_n^m(x) for 0 <= m <= n < nmax, with the Condon-Shortley phase (-1)^m,
 * from the standard recurrences in n at fixed m.                          */
void oracle_legendre(double x, int nmax, double *P)
{
    double s = sqrt(fmax(0.0, (1.0 - x) * (1.0 + x)));
    double pmm = 1.0;
    for (int m = 0; m < nmax; ++m) {
        if (m > 0) pmm *= -(2.0 * m - 1.0) * s;
        P[PIDX(m, m)] = pmm;
        if (m + 1 < nmax) P[PIDX(m + 1, m)] = x * (2.0 * m + 1.0) * pmm;
        for (int n = m + 2; n < nmax; ++n)
            P[PIDX(n, m)] = ((2.0 * n - 1.0) * x * P[PIDX(n - 1, m)] - (n + m - 1.0) * P[PIDX(n - 2, m)]) / (double)(n - m);
    }
}

/* Solid harmonics of v for degrees n < nmax and all orders -n..n:
 *   R_n^m(v) = r^n P_n^m(cos t) e^{i m f} / (n+m)!        (m >= 0)
 *   I_n^m(v) = (n-m)! P_n^m(cos t) e^{i m f} / r^{n+1}     (m >= 0)
 *   X_n^{-m} = (-1)^m conj(X_n^m)
 * With these, 1/|x - y| = sum_{n,m} conj(R_n^m(y)) I_n^m(x) for |y| < |x|,
 * and R_n^m(a + b) = sum_{k,l} R_k^l(a) R_{n-k}^{m-l}(b).
 * Either output may be NULL; the irregular ones need v != 0.               */
static void harmonics(const double v[3], int nmax, cplx *Rh, cplx *Ih)
{
    double P[(ORC_HMAX + 1) * (ORC_HMAX + 2) / 2];
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double ct = r > 0.0 ? v[2] / r : 1.0;
    double ph = atan2(v[1], v[0]);
    oracle_legendre(ct, nmax, P);
    for (int n = 0; n < nmax; ++n) {
        double rn = pow(r, (double)n);
        double rin = (Ih && r > 0.0) ? 1.0 / pow(r, (double)(n + 1)) : 0.0;
        for (int m = 0; m <= n; ++m) {
            cplx e = cos(m * ph) + sin(m * ph) * I;
            double sg = (m & 1) ? -1.0 : 1.0;
            if (Rh) {
                cplx val = rn * P[PIDX(n, m)] * e / fact(n + m);
                Rh[HIDX(n, m)] = val;
                Rh[HIDX(n, -m)] = sg * conj(val);
            }
            if (Ih) {
                cplx val = fact(n - m) * P[PIDX(n, m)] * e * rin;
                Ih[HIDX(n, m)] = val;
                Ih[HIDX(n, -m)] = sg * conj(val);
            }
        }
    }
}

/* Exported for the pins: complex values as (re, im) pairs, index n*n+n+m. */
void oracle_harmonics(const double *v, int nmax, double *R, double *Iout)
{
    cplx Rh[(ORC_HMAX + 1) * (ORC_HMAX + 1)], Ih[(ORC_HMAX + 1) * (ORC_HMAX + 1)];
    if (nmax > ORC_HMAX + 1) return;
    harmonics(v, nmax, R ? Rh : NULL, Iout ? Ih : NULL);
    for (int k = 0; k < nmax * nmax; ++k) {
        if (R) { R[2 * k] = creal(Rh[k]); R[2 * k + 1] = cimag(Rh[k]); }
        if (Iout) { Iout[2 * k] = creal(Ih[k]); Iout[2 * k + 1] = cimag(Ih[k]); }
    }
}

static cplx hget(const cplx *H, int n, int m)
{
    if (n < 0 || m > n || m < -n) return 0.0;
    return H[HIDX(n, m)];
}

/* ------------------------------------------------------------------------ */
/* The five expansion operators on complex coefficient vectors of length p^2 */
/* (index n*n+n+m, 0 <= n < p, -n <= m <= n).                                */
/* ------------------------------------------------------------------------ */

/* P2M (Section II.A): M_n^m = sum_j q_j conj(R_n^m(x_j - c)).              */
static void p2m_add(const double *xj, double qj, const double c[3], int p, cplx *M)
{
    cplx Rh[ORC_MAXP * ORC_MAXP];
    double v[3] = {xj[0] - c[0], xj[1] - c[1], xj[2] - c[2]};
    harmonics(v, p, Rh, NULL);
    for (int k = 0; k < p * p; ++k) M[k] += qj * conj(Rh[k]);
}

/* M2M (Section II.A): re-expansion of a child multipole about the parent
 * center; x_j - c_par = (x_j - c_ch) + (c_ch - c_par) with the regular
 * addition theorem gives M_n^m += sum_{k,l} M'_k^l conj(R_{n-k}^{m-l}(d)).  */
static void m2m_add(const cplx *Mc, const double cch[3], const double cpar[3], int p, cplx *Mp)
{
    cplx Rh[ORC_MAXP * ORC_MAXP];
    double d[3] = {cch[0] - cpar[0], cch[1] - cpar[1], cch[2] - cpar[2]};
    harmonics(d, p, Rh, NULL);
    for (int n = 0; n < p; ++n)
        for (int m = -n; m <= n; ++m) {
            cplx s = 0.0;
            for (int k = 0; k <= n; ++k)
                for (int l = -k; l <= k; ++l) s += Mc[HIDX(k, l)] * conj(hget(Rh, n - k, m - l));
            Mp[HIDX(n, m)] += s;
        }
}

/* M2L (Section II.A): with D = c_A - c_B and t = x - c_A,
 * I_n^m(D + t) = sum_{j,s} (-1)^j conj(R_j^s(t)) I_{n+j}^{m+s}(D), so the
 * local coefficients (of conj(R_j^s(t))) are
 *   L_j^s += (-1)^j sum_{n<p,m} M_n^m I_{n+j}^{m+s}(D),   j < p.           */
static void m2l_add(const cplx *M, const double cB[3], const double cA[3], int p, cplx *L)
{
    cplx Ih[(2 * ORC_MAXP) * (2 * ORC_MAXP)];
    double D[3] = {cA[0] - cB[0], cA[1] - cB[1], cA[2] - cB[2]};
    harmonics(D, 2 * p - 1, NULL, Ih);
    for (int j = 0; j < p; ++j) {
        double sj = (j & 1) ? -1.0 : 1.0;
        for (int s = -j; s <= j; ++s) {
            cplx acc = 0.0;
            for (int n = 0; n < p; ++n)
                for (int m = -n; m <= n; ++m) acc += M[HIDX(n, m)] * hget(Ih, n + j, m + s);
            L[HIDX(j, s)] += sj * acc;
        }
    }
}

/* M2L by rotation, O(p^3) per pair.  The operators' cost ranges from O(P^3)
 * to O(P^6) with the basis (Section III.A); with spherical harmonics the
 * O(P^3) form rotates the frame so that D = c_A - c_B lies on +z, translates
 * along z and rotates back (White & Head-Gordon 1996).
 *
 * Both R_n^m and I_n^m are multiples of C_n^m = sqrt((n-m)!/(n+m)!) P_n^m
 * e^{i m f}:  R_n^m = r^n C_n^m / s_m,  I_n^m = s_m C_n^m / r^{n+1},  with
 * s_m = sqrt((n+m)! (n-m)!).  Let Q = Ry(-t) Rz(-f) (t, f: polar and azimuth
 * angles of D), so Q D = (0, 0, d).  The angular functions rotate as
 * C_n^m(Q u) = sum_k U_{m k} C_n^k(u) with U_{m k} = d^n_{k m}(t) e^{-i k f},
 * d^n the Wigner small-d matrix (for an active rotation R, Y(R^-1 u) =
 * sum_k D_{k m}(R) Y_k(u)).  Writing the source's series in the rotated
 * frame, sum_m M_m I^m(u) = sum_m Mt_m I^m(Q u), gives
 *     Mt_m = sum_k conj(U_{m k}) (s_k / s_m) M_k;
 * along z only I_k^0((0, 0, d)) = k! / d^{k+1} survives, so
 *     Lt_j^s = (-1)^j sum_{n >= |s|} Mt_n^{-s} (n + j)! / d^{n+j+1};
 * and sum_s Lt_s conj(R^s(Q t)) = sum_s L_s conj(R^s(t)) gives
 *     L_k += sum_s Lt_s conj(U_{s k}) (s_k / s_s).
 * The result equals m2l_add's up to rounding. */

/* Wigner small-d matrix element d^n_{mp m}(b), Wigner's explicit sum. */
static double wigner_d(int n, int mp, int m, double b)
{
    double c = cos(0.5 * b), sn = sin(0.5 * b), acc = 0.0;
    double pre = sqrt(fact(n + m) * fact(n - m) * fact(n + mp) * fact(n - mp));
    for (int k = 0; k <= 2 * n; ++k) {
        int a1 = n + m - k, a3 = n - k - mp, a4 = k - m + mp;
        if (a1 < 0 || a3 < 0 || a4 < 0) continue;
        double term = pre / (fact(a1) * fact(k) * fact(a3) * fact(a4)) * pow(c, 2 * n - 2 * k + m - mp) *
                      pow(sn, 2 * k - m + mp);
        acc += (a4 & 1) ? -term : term;
    }
    return acc;
}

static double sfac(int n, int m) { return sqrt(fact(n + m) * fact(n - m)); }

static void m2l_rot_add(const cplx *M, const double cB[3], const double cA[3], int p, cplx *L)
{
    double D[3] = {cA[0] - cB[0], cA[1] - cB[1], cA[2] - cB[2]};
    double d = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    double ct = fmax(-1.0, fmin(1.0, D[2] / d));
    double t = acos(ct), f = (D[0] == 0.0 && D[1] == 0.0) ? 0.0 : atan2(D[1], D[0]);
    cplx Mt[ORC_MAXP * ORC_MAXP], Lt[ORC_MAXP * ORC_MAXP];
    for (int n = 0; n < p; ++n)
        for (int m = -n; m <= n; ++m) {
            cplx acc = 0.0;
            for (int k = -n; k <= n; ++k)  /* conj(U_{m k}) = d^n_{k m}(t) e^{+i k f} */
                acc += wigner_d(n, k, m, t) * cexp(I * (double)k * f) * (sfac(n, k) / sfac(n, m)) * M[HIDX(n, k)];
            Mt[HIDX(n, m)] = acc;
        }
    for (int j = 0; j < p; ++j)
        for (int s = -j; s <= j; ++s) {
            cplx acc = 0.0;
            int as = s < 0 ? -s : s;
            for (int n = as; n < p; ++n) acc += Mt[HIDX(n, -s)] * (fact(n + j) / pow(d, (double)(n + j + 1)));
            Lt[HIDX(j, s)] = (j & 1) ? -acc : acc;
        }
    for (int j = 0; j < p; ++j)
        for (int k = -j; k <= j; ++k) {
            cplx acc = 0.0;
            for (int s = -j; s <= j; ++s)  /* conj(U_{s k}) = d^j_{k s}(t) e^{+i k f} */
                acc += Lt[HIDX(j, s)] * wigner_d(j, k, s, t) * (sfac(j, k) / sfac(j, s));
            L[HIDX(j, k)] += acc * cexp(I * (double)k * f);
        }
}

/* L2L (Section II.A): with t = t' + d (d = c_child - c_parent),
 * conj(R_j^s(t)) = sum_{k,l} conj(R_k^l(t')) conj(R_{j-k}^{s-l}(d)), so
 *   L'_k^l += sum_{j>=k,s} L_j^s conj(R_{j-k}^{s-l}(d)).                    */
static void l2l_add(const cplx *Lp, const double cpar[3], const double cch[3], int p, cplx *Lc)
{
    cplx Rh[ORC_MAXP * ORC_MAXP];
    double d[3] = {cch[0] - cpar[0], cch[1] - cpar[1], cch[2] - cpar[2]};
    harmonics(d, p, Rh, NULL);
    for (int k = 0; k < p; ++k)
        for (int l = -k; l <= k; ++l) {
            cplx s = 0.0;
            for (int j = k; j < p; ++j)
                for (int ss = -j; ss <= j; ++ss) s += Lp[HIDX(j, ss)] * conj(hget(Rh, j - k, ss - l));
            Lc[HIDX(k, l)] += s;
        }
}

/* L2P (Section II.A): phi(x) = sum_{j,s} L_j^s conj(R_j^s(x - c)) (real),
 * E = -grad phi, using dR_n^m/dz = R_{n-1}^m,
 * dR_n^m/dx = (R_{n-1}^{m+1} - R_{n-1}^{m-1})/2,
 * dR_n^m/dy = -i (R_{n-1}^{m-1} + R_{n-1}^{m+1})/2.                        */
static void l2p_eval(const cplx *L, const double c[3], int p, const double *x, double *phi, double *E)
{
    cplx Rh[ORC_MAXP * ORC_MAXP];
    double v[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    harmonics(v, p, Rh, NULL);
    cplx f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int j = 0; j < p; ++j)
        for (int s = -j; s <= j; ++s) {
            cplx Ljs = L[HIDX(j, s)];
            f += Ljs * conj(hget(Rh, j, s));
            if (j > 0) {
                cplx dz = hget(Rh, j - 1, s);
                cplx dx = 0.5 * (hget(Rh, j - 1, s + 1) - hget(Rh, j - 1, s - 1));
                cplx dy = -0.5 * I * (hget(Rh, j - 1, s - 1) + hget(Rh, j - 1, s + 1));
                gx += Ljs * conj(dx);
                gy += Ljs * conj(dy);
                gz += Ljs * conj(dz);
            }
        }
    *phi = creal(f);
    E[0] = -creal(gx);
    E[1] = -creal(gy);
    E[2] = -creal(gz);
}

/* Multipole series evaluated at x (for the pins): sum M_n^m I_n^m(x - c).  */
static double m2p_eval(const cplx *M, const double c[3], int p, const double *x)
{
    cplx Ih[ORC_MAXP * ORC_MAXP];
    double v[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    harmonics(v, p, NULL, Ih);
    cplx f = 0.0;
    for (int k = 0; k < p * p; ++k) f += M[k] * Ih[k];
    return creal(f);
}

/* ---- exported single-operator entry points for the pins (interleaved
 *      (re, im) doubles, p^2 complex coefficients) ---------------------- */
static void to_c(const double *a, int k, cplx *z)
{
    for (int i = 0; i < k; ++i) z[i] = a[2 * i] + a[2 * i + 1] * I;
}
static void from_c(const cplx *z, int k, double *a)
{
    for (int i = 0; i < k; ++i) { a[2 * i] = creal(z[i]); a[2 * i + 1] = cimag(z[i]); }
}

void oracle_op_p2m(int64_t n, const double *x, const double *q, const double *c, int p, double *Mout)
{
    cplx M[ORC_MAXP * ORC_MAXP] = {0};
    for (int64_t j = 0; j < n; ++j) p2m_add(x + 3 * j, q[j], c, p, M);
    from_c(M, p * p, Mout);
}
double oracle_op_m2p(const double *Min, const double *c, int p, const double *x)
{
    cplx M[ORC_MAXP * ORC_MAXP];
    to_c(Min, p * p, M);
    return m2p_eval(M, c, p, x);
}
void oracle_op_m2m(const double *Min, const double *cch, const double *cpar, int p, double *Mout)
{
    cplx Mc[ORC_MAXP * ORC_MAXP], Mp[ORC_MAXP * ORC_MAXP] = {0};
    to_c(Min, p * p, Mc);
    m2m_add(Mc, cch, cpar, p, Mp);
    from_c(Mp, p * p, Mout);
}
void oracle_op_m2l(const double *Min, const double *cB, const double *cA, int p, double *Lout)
{
    cplx M[ORC_MAXP * ORC_MAXP], L[ORC_MAXP * ORC_MAXP] = {0};
    to_c(Min, p * p, M);
    m2l_add(M, cB, cA, p, L);
    from_c(L, p * p, Lout);
}
void oracle_op_m2l_rot(const double *Min, const double *cB, const double *cA, int p, double *Lout)
{
    cplx M[ORC_MAXP * ORC_MAXP], L[ORC_MAXP * ORC_MAXP] = {0};
    to_c(Min, p * p, M);
    m2l_rot_add(M, cB, cA, p, L);
    from_c(L, p * p, Lout);
}

/* d^n_{mp m}(b) for all mp, m (row-major, (2n+1)^2 values). */
void oracle_wigner_d(int n, double b, double *out)
{
    for (int mp = -n; mp <= n; ++mp)
        for (int m = -n; m <= n; ++m) out[(mp + n) * (2 * n + 1) + (m + n)] = wigner_d(n, mp, m, b);
}

void oracle_op_l2l(const double *Lin, const double *cpar, const double *cch, int p, double *Lout)
{
    cplx Lp[ORC_MAXP * ORC_MAXP], Lc[ORC_MAXP * ORC_MAXP] = {0};
    to_c(Lin, p * p, Lp);
    l2l_add(Lp, cpar, cch, p, Lc);
    from_c(Lc, p * p, Lout);
}
void oracle_op_l2p(const double *Lin, const double *c, int p, int64_t n, const double *x, double *phi, double *E)
{
    cplx L[ORC_MAXP * ORC_MAXP];
    to_c(Lin, p * p, L);
    for (int64_t i = 0; i < n; ++i) l2p_eval(L, c, p, x + 3 * i, phi + i, E + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* Local octree (Section II.B: Morton keys, 3 bits per level, 21 levels in a */
/* 64-bit key; Section II.C: tree from the local bounding box).              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    int32_t ncrit;
    double theta, t4;
    double lo[3], S, scale;
    uint64_t *key;    /* sorted keys            [n]  */
    int32_t *perm;    /* sorted -> input index  [n]  */
    int64_t ncell, nleaf;
    int32_t depth;
    int32_t *lvl, *beg, *end, *par, *cbeg, *nch;
    uint64_t *ckey;
    int32_t *ix;      /* lattice coordinates at the cell's own level [3*ncell] */
    double *ctr;      /* lattice centers [3*ncell] */
    /* lists (CSR by target cell; source ascending).  With a target subset only
     * the target cells that matter are stored; the counts are always full.  */
    int64_t n_m2l, n_p2p, n_m2l_stored, n_p2p_stored;
    uint64_t h_m2l, h_p2p; /* list digests (mix64 sums) */
    int64_t *m2l_off, *p2p_off;
    int32_t *m2l_src, *p2p_src;
    uint8_t *need;    /* target cell is an ancestor of (or is) a sampled leaf */
    int tight;        /* acceptance also by the cells' own radii (rad)        */
    int64_t *rad;     /* [ncell] radius in units of S 2^-22, or NULL          */
} otree;

typedef struct { uint64_t k; int64_t i; } kv;

static int cmp_kv(const void *a, const void *b)
{
    const kv *x = (const kv *)a, *y = (const kv *)b;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;
    return (x->i > y->i) - (x->i < y->i);
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Key of one body (step T2): i_d = min(2^21 - 1, floor((x_d - lo_d) * scale)),
 * bit b of i_x at key bit 3b+2, of i_y at 3b+1, of i_z at 3b.            */
static uint64_t body_key(const double *x, const double lo[3], double scale)
{
    uint64_t c[3];
    for (int d = 0; d < 3; ++d) {
        double s = (x[d] - lo[d]) * scale;
        double f = floor(s);
        uint64_t v = f < 0.0 ? 0 : (uint64_t)f;
        if (v > (1u << ORC_LEVELS) - 1) v = (1u << ORC_LEVELS) - 1;
        c[d] = v;
    }
    uint64_t k = 0;
    for (int b = 0; b < ORC_LEVELS; ++b) {
        k |= ((c[0] >> b) & 1ull) << (3 * b + 2);
        k |= ((c[1] >> b) & 1ull) << (3 * b + 1);
        k |= ((c[2] >> b) & 1ull) << (3 * b);
    }
    return k;
}

/* Multipole acceptance (step T6): R_A + R_B < theta |c_A - c_B| with R the
 * radius of the cube's bounding sphere, decided exactly on the lattice of
 * half-units of the finer cell (see the tree documentation).               */
static int mac(const otree *t, int a, int b)
{
    int la = t->lvl[a], lb = t->lvl[b];
    int f = la > lb ? la : lb;
    int64_t sa = (int64_t)1 << (f - la + 1), sb = (int64_t)1 << (f - lb + 1);
    int64_t d2 = 0;
    for (int d = 0; d < 3; ++d) {
        int64_t ca = (2 * (int64_t)t->ix[3 * a + d] + 1) << (f - la);
        int64_t cb = (2 * (int64_t)t->ix[3 * b + d] + 1) << (f - lb);
        d2 += (ca - cb) * (ca - cb);
    }
    double lhs = (double)(3 * (sa + sb) * (sa + sb));
    if (lhs < t->t4 * (double)d2) return 1;
    if (!t->tight) return 0;
    /* the cells' own radii (integers in units u = S 2^-22, centers at
     * (2 i + 1) 2^(21 - l) u): 4 (r_A + r_B)^2 < (4 theta^2) D^2            */
    int64_t D2 = 0;
    for (int d = 0; d < 3; ++d) {
        int64_t ca = (2 * (int64_t)t->ix[3 * a + d] + 1) << (ORC_LEVELS - la);
        int64_t cb = (2 * (int64_t)t->ix[3 * b + d] + 1) << (ORC_LEVELS - lb);
        D2 += (ca - cb) * (ca - cb);
    }
    const int64_t rs = t->rad[a] + t->rad[b];
    return (double)(4 * rs * rs) < t->t4 * (double)D2;
}

static int is_leaf(const otree *t, int c) { return t->nch[c] == 0; }

/* ---- growable pair buffer ---- */
typedef struct { uint64_t *v; int64_t n, cap; } pbuf;
static void pb_push(pbuf *b, uint64_t x)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->v = (uint64_t *)realloc(b->v, (size_t)b->cap * sizeof(uint64_t));
    }
    b->v[b->n++] = x;
}

/* Order-independent list digest: the sum, mod 2^64, of mix64(target << 32 |
 * source) over the pairs, with mix64 the output finaliser of SplitMix64
 * (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014).  Two lists have equal digests when they hold the same pairs
 * (up to a 2^-64 accident), whatever order they were produced in.          */
static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

typedef struct {
    otree *t;
    pbuf m2l, p2p;
    int prune;
    int64_t n_m2l, n_p2p;
    uint64_t h_m2l, h_p2p;
} tctx;

/* One step of the dual tree traversal (step T7, Section II.C): 0 = the pair
 * is an M2L pair, 1 = a P2P pair, 2 = split A and/or B (symmetric rule: the
 * coarser cell, both on equal levels, never a leaf).                       */
static int classify(const otree *t, int a, int b, int *split_a, int *split_b)
{
    if (mac(t, a, b)) return 0;
    int la = is_leaf(t, a), lb = is_leaf(t, b);
    if (la && lb) return 1;
    if (la) { *split_a = 0; *split_b = 1; }
    else if (lb) { *split_a = 1; *split_b = 0; }
    else if (t->lvl[a] < t->lvl[b]) { *split_a = 1; *split_b = 0; }
    else if (t->lvl[b] < t->lvl[a]) { *split_a = 0; *split_b = 1; }
    else { *split_a = 1; *split_b = 1; }
    return 2;
}

/* Records a terminal pair (packed target << 32 | source); returns 1 when the
 * pair was split instead, with the split flags set. */
static int visit(tctx *c, int a, int b, int *split_a, int *split_b)
{
    otree *t = c->t;
    int kind = classify(t, a, b, split_a, split_b);
    if (kind == 2) return 1;
    const uint64_t pr = ((uint64_t)a << 32) | (uint32_t)b;
    if (kind == 0) {
        c->n_m2l++;
        c->h_m2l += mix64(pr);
        if (t->need[a]) pb_push(&c->m2l, pr);
    } else {
        c->n_p2p++;
        c->h_p2p += mix64(pr);
        if (t->need[a]) pb_push(&c->p2p, pr);
    }
    return 0;
}

static void interact(tctx *c, int a, int b)
{
    otree *t = c->t;
    /* pruned walk: a pair whose target is not kept has no kept descendant
     * (the kept set is closed under ancestors) */
    if (c->prune && !t->need[a]) return;
    int split_a = 0, split_b = 0;
    if (!visit(c, a, b, &split_a, &split_b)) return;
    if (split_a && split_b) {
        for (int i = 0; i < t->nch[a]; ++i)
            for (int j = 0; j < t->nch[b]; ++j) interact(c, t->cbeg[a] + i, t->cbeg[b] + j);
    } else if (split_a) {
        for (int i = 0; i < t->nch[a]; ++i) interact(c, t->cbeg[a] + i, b);
    } else {
        for (int j = 0; j < t->nch[b]; ++j) interact(c, a, t->cbeg[b] + j);
    }
}

static void pb_append(pbuf *dst, const pbuf *src)
{
    for (int64_t k = 0; k < src->n; ++k) pb_push(dst, src->v[k]);
}

/* The whole walk from (root, root).  The first generations are expanded
 * breadth-first until the frontier holds enough pairs; the frontier's pairs
 * are then walked depth-first by independent threads.  Each pair is visited
 * exactly once either way, so the lists (sorted afterwards), counts and
 * digests do not depend on the thread count.                                */
static void traverse_all(tctx *cx)
{
    otree *t = cx->t;
    pbuf front = {0}, next = {0};
    pb_push(&front, 0);
    for (int gen = 0; gen < 6 && front.n > 0 && front.n < 4096; ++gen) {
        next.n = 0;
        for (int64_t k = 0; k < front.n; ++k) {
            int a = (int)(front.v[k] >> 32), b = (int)(front.v[k] & 0xffffffffu);
            if (cx->prune && !t->need[a]) continue;
            int split_a = 0, split_b = 0;
            if (!visit(cx, a, b, &split_a, &split_b)) continue;
            int na = split_a ? t->nch[a] : 1, nb = split_b ? t->nch[b] : 1;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    uint64_t ca = split_a ? (uint64_t)(t->cbeg[a] + i) : (uint64_t)a;
                    uint64_t cb = split_b ? (uint64_t)(t->cbeg[b] + j) : (uint64_t)b;
                    pb_push(&next, (ca << 32) | cb);
                }
        }
        pbuf tmp = front; front = next; next = tmp;
    }
#pragma omp parallel
    {
        tctx lc = {t, {0}, {0}, cx->prune, 0, 0, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < front.n; ++k)
            interact(&lc, (int)(front.v[k] >> 32), (int)(front.v[k] & 0xffffffffu));
#pragma omp critical
        {
            cx->n_m2l += lc.n_m2l;
            cx->n_p2p += lc.n_p2p;
            cx->h_m2l += lc.h_m2l;
            cx->h_p2p += lc.h_p2p;
            pb_append(&cx->m2l, &lc.m2l);
            pb_append(&cx->p2p, &lc.p2p);
        }
        free(lc.m2l.v);
        free(lc.p2p.v);
    }
    free(front.v);
    free(next.v);
}

static void csr_from_pairs(pbuf *b, int64_t ncell, int64_t **off, int32_t **src)
{
    qsort(b->v, (size_t)b->n, sizeof(uint64_t), cmp_u64);
    *off = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    *src = (int32_t *)malloc((size_t)(b->n ? b->n : 1) * sizeof(int32_t));
    for (int64_t k = 0; k < b->n; ++k) {
        (*off)[(b->v[k] >> 32) + 1]++;
        (*src)[k] = (int32_t)(b->v[k] & 0xffffffffu);
    }
    for (int64_t c = 0; c < ncell; ++c) (*off)[c + 1] += (*off)[c];
    free(b->v);
    b->v = NULL;
}

/* Build the tree and the lists.  targets (nt indices into the input order)
 * restrict which target cells keep their lists: leaves holding a target and
 * their ancestors.  targets == NULL keeps everything; nt < 0 keeps nothing
 * (count only).  prune != 0 (with targets) walks only pairs whose target is
 * kept; the counts then cover the kept lists only.  Returns NULL on invalid
 * input.                                                                    */
void *oracle_tree_new3(int64_t n, const double *x, int32_t ncrit, double theta,
                       int64_t nt, const int64_t *targets, int prune, int tight);

/* Smallest r >= 0 with r^2 >= v (exact integer square root, rounded up). */
static int64_t isqrt_ceil(int64_t v)
{
    int64_t r = (int64_t)sqrt((double)v);
    while (r * r < v) ++r;
    while (r > 0 && (r - 1) * (r - 1) >= v) --r;
    return r;
}

/* Radius of every cell about its lattice center, tight to its bodies: the
 * largest distance from the center to a corner of a member body's lattice
 * cell (the body lies inside that cell), in units u = S 2^-22, rounded up
 * to an integer.  Never above the cube's own bounding radius by more than
 * one unit.                                                                */
static void tight_radii(otree *t)
{
    t->rad = (int64_t *)calloc((size_t)t->ncell, sizeof(int64_t));
    for (int64_t c = 0; c < t->ncell; ++c) {
        const int l = t->lvl[c];
        int64_t C[3], best = 0;
        for (int d = 0; d < 3; ++d) C[d] = (2 * (int64_t)t->ix[3 * c + d] + 1) << (ORC_LEVELS - l);
        for (int32_t j = t->beg[c]; j < t->end[c]; ++j) {
            const uint64_t k = t->key[j];
            int64_t r2 = 0;
            for (int d = 0; d < 3; ++d) {
                int64_t v = 0;
                for (int b = 0; b < ORC_LEVELS; ++b) v |= (int64_t)((k >> (3 * b + 2 - d)) & 1ull) << b;
                const int64_t lo = 2 * v - C[d], hi = 2 * v + 2 - C[d];
                const int64_t m = llabs(lo) > llabs(hi) ? llabs(lo) : llabs(hi);
                r2 += m * m;
            }
            if (r2 > best) best = r2;
        }
        t->rad[c] = isqrt_ceil(best);
    }
}

void *oracle_tree_new2(int64_t n, const double *x, int32_t ncrit, double theta,
                       int64_t nt, const int64_t *targets, int prune)
{
    return oracle_tree_new3(n, x, ncrit, theta, nt, targets, prune, 0);
}

/* As oracle_tree_new2; tight != 0 also accepts a pair when the cells' own
 * radii about their lattice centers (tight_radii) meet the criterion.      */
void *oracle_tree_new3(int64_t n, const double *x, int32_t ncrit, double theta,
                       int64_t nt, const int64_t *targets, int prune, int tight)
{
    if (n <= 0 || !x || ncrit < 1 || !(theta > 0.0 && theta < 1.0)) return NULL;
    otree *t = (otree *)calloc(1, sizeof(otree));
    t->tight = tight ? 1 : 0;
    t->n = n;
    t->ncrit = ncrit;
    t->theta = theta;
    t->t4 = 4.0 * theta * theta;

    /* T1: root cube anchored at the per-axis minima, side = largest extent. */
    double hi[3];
    for (int d = 0; d < 3; ++d) { t->lo[d] = x[d]; hi[d] = x[d]; }
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            if (x[3 * i + d] < t->lo[d]) t->lo[d] = x[3 * i + d];
            if (x[3 * i + d] > hi[d]) hi[d] = x[3 * i + d];
        }
    t->S = 0.0;
    for (int d = 0; d < 3; ++d)
        if (hi[d] - t->lo[d] > t->S) t->S = hi[d] - t->lo[d];
    if (t->S == 0.0) t->S = 1.0;
    t->scale = ldexp(1.0, ORC_LEVELS) / t->S;

    /* T2 + T3: keys, stable sort with ties broken by input index. */
    kv *a = (kv *)malloc((size_t)n * sizeof(kv));
    for (int64_t i = 0; i < n; ++i) { a[i].k = body_key(x + 3 * i, t->lo, t->scale); a[i].i = i; }
    qsort(a, (size_t)n, sizeof(kv), cmp_kv);
    t->key = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    t->perm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) { t->key[i] = a[i].k; t->perm[i] = (int32_t)a[i].i; }
    free(a);

    /* T4: cells in breadth-first order, which is (level, key) order. */
    int64_t cap = 1024;
    t->lvl = (int32_t *)malloc(cap * sizeof(int32_t));
    t->beg = (int32_t *)malloc(cap * sizeof(int32_t));
    t->end = (int32_t *)malloc(cap * sizeof(int32_t));
    t->par = (int32_t *)malloc(cap * sizeof(int32_t));
    t->cbeg = (int32_t *)malloc(cap * sizeof(int32_t));
    t->nch = (int32_t *)malloc(cap * sizeof(int32_t));
    t->ckey = (uint64_t *)malloc(cap * sizeof(uint64_t));
    int64_t nc = 1;
    t->lvl[0] = 0; t->beg[0] = 0; t->end[0] = (int32_t)n; t->par[0] = -1; t->ckey[0] = 0;
    for (int64_t c = 0; c < nc; ++c) {
        int l = t->lvl[c];
        t->cbeg[c] = -1;
        t->nch[c] = 0;
        if (!(t->end[c] - t->beg[c] > ncrit && l < ORC_LEVELS)) continue;
        int shift = 3 * (ORC_LEVELS - l - 1);
        int64_t i = t->beg[c];
        while (i < t->end[c]) {
            uint64_t ck = t->key[i] >> shift;
            int64_t j = i;
            while (j < t->end[c] && (t->key[j] >> shift) == ck) ++j;
            if (nc == cap) {
                cap *= 2;
                t->lvl = (int32_t *)realloc(t->lvl, cap * sizeof(int32_t));
                t->beg = (int32_t *)realloc(t->beg, cap * sizeof(int32_t));
                t->end = (int32_t *)realloc(t->end, cap * sizeof(int32_t));
                t->par = (int32_t *)realloc(t->par, cap * sizeof(int32_t));
                t->cbeg = (int32_t *)realloc(t->cbeg, cap * sizeof(int32_t));
                t->nch = (int32_t *)realloc(t->nch, cap * sizeof(int32_t));
                t->ckey = (uint64_t *)realloc(t->ckey, cap * sizeof(uint64_t));
            }
            if (t->nch[c] == 0) t->cbeg[c] = (int32_t)nc;
            t->nch[c]++;
            t->lvl[nc] = l + 1; t->beg[nc] = (int32_t)i; t->end[nc] = (int32_t)j;
            t->par[nc] = (int32_t)c; t->ckey[nc] = ck;
            ++nc;
            i = j;
        }
    }
    t->ncell = nc;
    t->nleaf = 0;
    t->depth = 0;
    for (int64_t c = 0; c < nc; ++c) {
        if (t->nch[c] == 0) t->nleaf++;
        if (t->lvl[c] > t->depth) t->depth = t->lvl[c];
    }

    /* T5: lattice coordinates and centers c_d = lo_d + (i_d + 1/2) h_l. */
    t->ix = (int32_t *)malloc((size_t)nc * 3 * sizeof(int32_t));
    t->ctr = (double *)malloc((size_t)nc * 3 * sizeof(double));
    for (int64_t c = 0; c < nc; ++c) {
        uint64_t k = t->ckey[c];
        int l = t->lvl[c];
        int32_t v[3] = {0, 0, 0};
        for (int b = 0; b < l; ++b) {
            v[0] |= (int32_t)(((k >> (3 * b + 2)) & 1ull) << b);
            v[1] |= (int32_t)(((k >> (3 * b + 1)) & 1ull) << b);
            v[2] |= (int32_t)(((k >> (3 * b)) & 1ull) << b);
        }
        double h = ldexp(t->S, -l);
        for (int d = 0; d < 3; ++d) {
            t->ix[3 * c + d] = v[d];
            double off = ((double)v[d] + 0.5) * h;
            t->ctr[3 * c + d] = t->lo[d] + off;
        }
    }

    if (t->tight) tight_radii(t);

    /* Which target cells keep lists. */
    t->need = (uint8_t *)calloc((size_t)nc, 1);
    if (!targets && nt >= 0) {
        memset(t->need, 1, (size_t)nc);
    } else if (targets && nt > 0) {
        int32_t *leaf_of = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        for (int64_t c = 0; c < nc; ++c)
            if (t->nch[c] == 0)
                for (int32_t i = t->beg[c]; i < t->end[c]; ++i) leaf_of[t->perm[i]] = (int32_t)c;
        for (int64_t s = 0; s < nt; ++s)
            for (int32_t c = leaf_of[targets[s]]; c >= 0; c = t->par[c]) t->need[c] = 1;
        free(leaf_of);
    }

    /* T7: lists. */
    tctx cx = {t, {0}, {0}, (prune && targets) ? 1 : 0, 0, 0, 0, 0};
    traverse_all(&cx);
    t->n_m2l = cx.n_m2l;
    t->n_p2p = cx.n_p2p;
    t->h_m2l = cx.h_m2l;
    t->h_p2p = cx.h_p2p;
    t->n_m2l_stored = cx.m2l.n;
    t->n_p2p_stored = cx.p2p.n;
    csr_from_pairs(&cx.m2l, nc, &t->m2l_off, &t->m2l_src);
    csr_from_pairs(&cx.p2p, nc, &t->p2p_off, &t->p2p_src);
    return t;
}

void *oracle_tree_new(int64_t n, const double *x, int32_t ncrit, double theta,
                      int64_t nt, const int64_t *targets)
{
    return oracle_tree_new2(n, x, ncrit, theta, nt, targets, 0);
}

void oracle_tree_free(void *h)
{
    otree *t = (otree *)h;
    if (!t) return;
    free(t->key); free(t->perm);
    free(t->lvl); free(t->beg); free(t->end); free(t->par); free(t->cbeg); free(t->nch); free(t->ckey);
    free(t->ix); free(t->ctr); free(t->need); free(t->rad);
    free(t->m2l_off); free(t->m2l_src); free(t->p2p_off); free(t->p2p_src);
    free(t);
}

/* radii of the tight criterion (units S 2^-22); zeros without it          */
void oracle_tree_radii(const void *h, int64_t *out)
{
    const otree *t = (const otree *)h;
    for (int64_t c = 0; c < t->ncell; ++c) out[c] = t->rad ? t->rad[c] : 0;
}

/* out: [digest of the M2L list, digest of the P2P list] over every pair the
 * walk visited (the full lists unless the walk was pruned).               */
void oracle_tree_digest(const void *h, uint64_t *out)
{
    const otree *t = (const otree *)h;
    out[0] = t->h_m2l;
    out[1] = t->h_p2p;
}

/* info: [ncell, nleaf, depth, n_m2l, n_p2p, n_m2l_stored, n_p2p_stored]
 * box:  [lo_x, lo_y, lo_z, S, scale]                                      */
void oracle_tree_info(const void *h, int64_t *info, double *box)
{
    const otree *t = (const otree *)h;
    if (info) {
        info[0] = t->ncell; info[1] = t->nleaf; info[2] = t->depth;
        info[3] = t->n_m2l; info[4] = t->n_p2p;
        info[5] = t->n_m2l_stored; info[6] = t->n_p2p_stored;
    }
    if (box) {
        for (int d = 0; d < 3; ++d) box[d] = t->lo[d];
        box[3] = t->S;
        box[4] = t->scale;
    }
}

/* Any pointer may be NULL.  Lists are exported as (target, source) pairs in
 * canonical (target, source) order.                                        */
void oracle_tree_export(const void *h, uint64_t *keys, int32_t *perm, int32_t *lvl, uint64_t *ckey,
                        int32_t *beg, int32_t *end, int32_t *par, int32_t *cbeg, int32_t *nch,
                        double *centers, int32_t *m2l, int32_t *p2p)
{
    const otree *t = (const otree *)h;
    if (keys) memcpy(keys, t->key, (size_t)t->n * sizeof(uint64_t));
    if (perm) memcpy(perm, t->perm, (size_t)t->n * sizeof(int32_t));
    if (lvl) memcpy(lvl, t->lvl, (size_t)t->ncell * sizeof(int32_t));
    if (ckey) memcpy(ckey, t->ckey, (size_t)t->ncell * sizeof(uint64_t));
    if (beg) memcpy(beg, t->beg, (size_t)t->ncell * sizeof(int32_t));
    if (end) memcpy(end, t->end, (size_t)t->ncell * sizeof(int32_t));
    if (par) memcpy(par, t->par, (size_t)t->ncell * sizeof(int32_t));
    if (cbeg) memcpy(cbeg, t->cbeg, (size_t)t->ncell * sizeof(int32_t));
    if (nch) memcpy(nch, t->nch, (size_t)t->ncell * sizeof(int32_t));
    if (centers) memcpy(centers, t->ctr, (size_t)t->ncell * 3 * sizeof(double));
    if (m2l)
        for (int64_t c = 0; c < t->ncell; ++c)
            for (int64_t k = t->m2l_off[c]; k < t->m2l_off[c + 1]; ++k) {
                m2l[2 * k] = (int32_t)c;
                m2l[2 * k + 1] = t->m2l_src[k];
            }
    if (p2p)
        for (int64_t c = 0; c < t->ncell; ++c)
            for (int64_t k = t->p2p_off[c]; k < t->p2p_off[c + 1]; ++k) {
                p2p[2 * k] = (int32_t)c;
                p2p[2 * k + 1] = t->p2p_src[k];
            }
}

/* ------------------------------------------------------------------------ */
/* FMM evaluation on a built tree (steps T8-T10).                            */
/* ------------------------------------------------------------------------ */

/* xpos == NULL: the coordinates the tree was built from.  Otherwise the
 * bodies sit at xpos (input order) while the tree, centers and lists stay
 * frozen (used for finite differences of the frozen-tree FMM).
 * targets == NULL: all bodies, outputs in input order; else nt targets, which
 * must be a subset of the targets the tree was built for.                  */
int oracle_fmm_at(const void *h, const double *xpos, const double *q, int p,
                  int64_t nt, const int64_t *targets, double *phi, double *field)
{
    const otree *t = (const otree *)h;
    if (!t || !q || p < 1 || p > ORC_MAXP) return 1;
    const int64_t n = t->n, nc = t->ncell;
    const int P2 = p * p;
    (void)n;
    /* Sorted body coordinates. */
    double *xs = (double *)malloc((size_t)t->n * 3 * sizeof(double));
    double *qs = (double *)malloc((size_t)t->n * sizeof(double));
    if (!xpos) return (free(xs), free(qs), 2);
    for (int64_t i = 0; i < t->n; ++i) {
        int32_t o = t->perm[i];
        for (int d = 0; d < 3; ++d) xs[3 * i + d] = xpos[3 * (int64_t)o + d];
        qs[i] = q[o];
    }
    cplx *M = (cplx *)calloc((size_t)nc * P2, sizeof(cplx));
    cplx *L = (cplx *)calloc((size_t)nc * P2, sizeof(cplx));

    /* Upward pass (Section II.C): P2M at leaves, then M2M from the finest
     * level up; each parent gathers its children in order.                 */
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t c = 0; c < nc; ++c)
        if (t->nch[c] == 0)
            for (int32_t i = t->beg[c]; i < t->end[c]; ++i) p2m_add(xs + 3 * (int64_t)i, qs[i], t->ctr + 3 * c, p, M + c * P2);
    for (int l = t->depth - 1; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t c = 0; c < nc; ++c) {
            if (t->lvl[c] != l || t->nch[c] == 0) continue;
            for (int k = 0; k < t->nch[c]; ++k) {
                int64_t ch = t->cbeg[c] + k;
                m2m_add(M + ch * P2, t->ctr + 3 * ch, t->ctr + 3 * c, p, M + c * P2);
            }
        }
    }

    /* M2L over each (kept) target cell's list, sources ascending. */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < nc; ++c)
        for (int64_t k = t->m2l_off[c]; k < t->m2l_off[c + 1]; ++k) {
            int64_t s = t->m2l_src[k];
            m2l_add(M + s * P2, t->ctr + 3 * s, t->ctr + 3 * c, p, L + c * P2);
        }

    /* Downward pass: L2L from the root down. */
    for (int l = 1; l <= t->depth; ++l) {
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t c = 0; c < nc; ++c) {
            if (t->lvl[c] != l || !t->need[c]) continue;
            int64_t pa = t->par[c];
            l2l_add(L + pa * P2, t->ctr + 3 * pa, t->ctr + 3 * c, p, L + c * P2);
        }
    }

    /* Targets: sorted position -> leaf. */
    int32_t *leaf_of_sorted = (int32_t *)malloc((size_t)t->n * sizeof(int32_t));
    int32_t *inv = (int32_t *)malloc((size_t)t->n * sizeof(int32_t));
    for (int64_t c = 0; c < nc; ++c)
        if (t->nch[c] == 0)
            for (int32_t i = t->beg[c]; i < t->end[c]; ++i) leaf_of_sorted[i] = (int32_t)c;
    for (int64_t i = 0; i < t->n; ++i) inv[t->perm[i]] = (int32_t)i;

    int64_t ntg = targets ? nt : t->n;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t s = 0; s < ntg; ++s) {
        int64_t orig = targets ? targets[s] : s;
        int64_t i = inv[orig];
        int64_t c = leaf_of_sorted[i];
        if (!t->need[c]) { bad |= 1; continue; }
        const double *xi = xs + 3 * i;
        /* P2P (Section II.A): source leaves ascending, bodies in sorted order. */
        double pp = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (int64_t k = t->p2p_off[c]; k < t->p2p_off[c + 1]; ++k) {
            int64_t b = t->p2p_src[k];
            for (int32_t j = t->beg[b]; j < t->end[b]; ++j) {
                double dx = xi[0] - xs[3 * (int64_t)j], dy = xi[1] - xs[3 * (int64_t)j + 1], dz = xi[2] - xs[3 * (int64_t)j + 2];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) continue;
                double r = sqrt(r2);
                double qr = qs[j] / r;
                double qr3 = qr / r2;
                pp += qr;
                ex += qr3 * dx;
                ey += qr3 * dy;
                ez += qr3 * dz;
            }
        }
        /* L2P. */
        double lp, E[3];
        l2p_eval(L + c * P2, t->ctr + 3 * c, p, xi, &lp, E);
        if (phi) phi[s] = lp + pp;
        if (field) {
            field[3 * s] = E[0] + ex;
            field[3 * s + 1] = E[1] + ey;
            field[3 * s + 2] = E[2] + ez;
        }
    }
    free(leaf_of_sorted);
    free(inv);
    free(xs);
    free(qs);
    free(M);
    free(L);
    return bad ? 3 : 0;
}

/* ------------------------------------------------------------------------ */
/* Mutual interactions (Section II.C lists them among the features of the    */
/* code the paper builds on): every unordered pair of bodies in the near     */
/* field is evaluated once and both bodies are updated.                      */
/* ------------------------------------------------------------------------ */

/* Near field (P2P only, no expansions) of every body, input order.  The
 * leaves are taken in ascending order; for leaf A each source B >= A of its
 * P2P list (sources ascending) is visited once: B == A gives the pairs
 * i < j of A's bodies, B > A every pair (i in A, j in B).  One distance, one
 * reciprocal and one cube serve both updates: body i gains q_j / r and
 * q_j (x_i - x_j) / r^3, body j gains q_i / r and q_i (x_j - x_i) / r^3.
 * Coincident bodies are skipped, as in the one-sided sums.  Serial: the
 * updates of B's bodies would race across leaves.  Needs a tree built for
 * every target, at the coordinates x (input order) it was built from.     */
int oracle_near_mutual(const void *h, const double *x, const double *q, double *phi, double *field)
{
    const otree *t = (const otree *)h;
    if (!t || !x || !q || !phi || !field) return 1;
    const int64_t n = t->n;
    for (int64_t c = 0; c < t->ncell; ++c)
        if (t->nch[c] == 0 && !t->need[c]) return 3;
    double *xs = (double *)malloc((size_t)n * 3 * sizeof(double) + 1);
    double *acc = (double *)calloc((size_t)n * 4 + 1, sizeof(double)); /* phi, Ex, Ey, Ez per sorted body */
    if (!xs || !acc) return (free(xs), free(acc), 2);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) xs[3 * i + d] = x[3 * (int64_t)t->perm[i] + d];
    for (int64_t a = 0; a < t->ncell; ++a) {
        if (t->nch[a] != 0) continue;
        for (int64_t k = t->p2p_off[a]; k < t->p2p_off[a + 1]; ++k) {
            const int64_t b = t->p2p_src[k];
            if (b < a) continue;
            for (int32_t i = t->beg[a]; i < t->end[a]; ++i) {
                const int32_t j0 = b == a ? i + 1 : t->beg[b];
                for (int32_t j = j0; j < t->end[b]; ++j) {
                    const double dx = xs[3 * (int64_t)i] - xs[3 * (int64_t)j];
                    const double dy = xs[3 * (int64_t)i + 1] - xs[3 * (int64_t)j + 1];
                    const double dz = xs[3 * (int64_t)i + 2] - xs[3 * (int64_t)j + 2];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 == 0.0) continue;
                    const double r = sqrt(r2);
                    const double qi = q[t->perm[i]], qj = q[t->perm[j]];
                    const double ri = 1.0 / r, ri3 = ri / r2;
                    acc[4 * (int64_t)i] += qj * ri;
                    acc[4 * (int64_t)i + 1] += qj * ri3 * dx;
                    acc[4 * (int64_t)i + 2] += qj * ri3 * dy;
                    acc[4 * (int64_t)i + 3] += qj * ri3 * dz;
                    acc[4 * (int64_t)j] += qi * ri;
                    acc[4 * (int64_t)j + 1] -= qi * ri3 * dx;
                    acc[4 * (int64_t)j + 2] -= qi * ri3 * dy;
                    acc[4 * (int64_t)j + 3] -= qi * ri3 * dz;
                }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        const int64_t o = t->perm[i];
        phi[o] = acc[4 * i];
        for (int d = 0; d < 3; ++d) field[3 * o + d] = acc[4 * i + 1 + d];
    }
    free(xs);
    free(acc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Virtual ranks (Section II.B: orthogonal recursive bisection weighted by   */
/* the work of Eq. (1); Section II.C: local trees from local bounding boxes, */
/* the local essential tree sent by each rank and grafted by the receiver).  */
/* ------------------------------------------------------------------------ */

typedef struct { double c; int64_t i; } okey;

static int cmp_okey(const void *a, const void *b)
{
    const okey *x = (const okey *)a, *y = (const okey *)b;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    return (x->i > y->i) - (x->i < y->i);
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* ORB of the bodies mem[0..cnt) (ascending input indices) over the m ranks
 * r0 .. r0+m-1.  The box is split across its longest side (the first of the
 * longest when several tie): bodies in ascending (coordinate, index) order,
 * the lower part taking the first k bodies with k the smallest count whose
 * weight reaches the share floor(m/2)/m of the box's weight (unit weights
 * when the box weighs nothing), and at least one body on each side when
 * there are two or more.  Each part keeps ascending input order.           */
static void orb_split(const double *x, const int64_t *w, int64_t *mem, int64_t cnt, int m, int r0, int32_t *rank)
{
    if (cnt == 0) return;
    if (m <= 1) {
        for (int64_t k = 0; k < cnt; ++k) rank[mem[k]] = r0;
        return;
    }
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = x[3 * mem[0] + d];
    for (int64_t k = 1; k < cnt; ++k)
        for (int d = 0; d < 3; ++d) {
            double v = x[3 * mem[k] + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    int axis = 0;
    for (int d = 1; d < 3; ++d)
        if (hi[d] - lo[d] > hi[axis] - lo[axis]) axis = d;
    okey *ks = (okey *)malloc((size_t)cnt * sizeof(okey));
    for (int64_t k = 0; k < cnt; ++k) { ks[k].c = x[3 * mem[k] + axis]; ks[k].i = mem[k]; }
    qsort(ks, (size_t)cnt, sizeof(okey), cmp_okey);
    __int128 W = 0;
    for (int64_t k = 0; k < cnt; ++k) W += w ? w[ks[k].i] : 1;
    const int unit = (!w || W == 0);
    if (unit) W = cnt;
    const int mL = m / 2;
    /* smallest k with P(k) m >= W mL, P(k) the weight of the first k bodies */
    int64_t k = 0;
    __int128 P = 0;
    const __int128 goal = W * mL;
    while (k < cnt && P * m < goal) {
        P += unit ? 1 : w[ks[k].i];
        ++k;
    }
    if (cnt >= 2) {
        if (k < 1) k = 1;
        if (k > cnt - 1) k = cnt - 1;
    }
    for (int64_t j = 0; j < cnt; ++j) mem[j] = ks[j].i;
    free(ks);
    qsort(mem, (size_t)k, sizeof(int64_t), cmp_i64);
    qsort(mem + k, (size_t)(cnt - k), sizeof(int64_t), cmp_i64);
    orb_split(x, w, mem, k, mL, r0, rank);
    orb_split(x, w, mem + k, cnt - k, m - mL, r0 + mL, rank);
}

typedef struct {
    int64_t n;
    int R;
    int32_t ncrit;
    double theta, t4;
    double *x;                /* [3n] coordinates (input order)                     */
    int32_t *rank;            /* [n] rank of every body                            */
    int64_t *rstart, *rcount; /* [R] members of rank r: mem[rstart[r] .. + rcount[r]) */
    int64_t *mem;             /* [n] input indices grouped by rank, ascending inside */
    otree **T;                /* [R] local trees (NULL for an empty rank)           */
    uint8_t **kind;           /* [R*R] (receiver r, sender s): kind of s's cells      */
    pbuf *rm2l, *rp2p, *rm2p; /* [R*R] remote pairs (A of r) << 32 | (B of s), sorted */
    int64_t *cnt;             /* [R*R*4] LET cells, multipole-only leaves, body leaves, bodies */
} olet;

/* Side of a cell's cube: h_l = S 2^-l. */
static double cell_h(const otree *t, int c) { return ldexp(t->S, -t->lvl[c]); }

/* The sender's test against the receiver's root cube (lo, lo + S): the
 * acceptance criterion with the whole cube on the target side, R_B < theta d
 * with d the distance from the cell's center to the cube (0 inside), in the
 * form 3 h_B^2 < 4 theta^2 d^2 (R = sqrt(3)/2 h).                        */
static int let_far(const otree *s, int b, const otree *r, double t4)
{
    double d[3];
    for (int k = 0; k < 3; ++k) {
        const double c = s->ctr[3 * b + k], lo = r->lo[k], hi = r->lo[k] + r->S;
        d[k] = c < lo ? lo - c : (c > hi ? c - hi : 0.0);
    }
    const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double h = cell_h(s, b);
    return 3.0 * h * h < t4 * d2;
}

/* Acceptance criterion between cells of two different trees (no common
 * lattice): R_A + R_B < theta |c_A - c_B| as 3 (h_A + h_B)^2 < 4 theta^2 D^2. */
static int mac_cross(const otree *ta, int a, const otree *tb, int b, double t4)
{
    const double dx = ta->ctr[3 * a] - tb->ctr[3 * b], dy = ta->ctr[3 * a + 1] - tb->ctr[3 * b + 1],
                 dz = ta->ctr[3 * a + 2] - tb->ctr[3 * b + 2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double sh = cell_h(ta, a) + cell_h(tb, b);
    return 3.0 * sh * sh < t4 * d2;
}

/* LET of sender s for receiver r, top-down over s's cells (a parent precedes
 * its children in (level, key) order): kind 0 = not sent, 1 = sent with its
 * multipole and its children, 2 = sent with its multipole only (accepted
 * against the receiver's cube), 3 = a leaf sent with its multipole and its
 * bodies.  cnt: cells sent, kind-2 cells, kind-3 leaves, bodies sent.      */
static void let_select(const otree *s, const otree *r, double t4, uint8_t *kind, int64_t *cnt)
{
    cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0;
    for (int64_t c = 0; c < s->ncell; ++c) {
        const int32_t pa = s->par[c];
        if (pa >= 0 && kind[pa] != 1) { kind[c] = 0; continue; }
        if (let_far(s, (int)c, r, t4)) kind[c] = 2;
        else if (s->nch[c] == 0) kind[c] = 3;
        else kind[c] = 1;
        cnt[0]++;
        if (kind[c] == 2) cnt[1]++;
        if (kind[c] == 3) { cnt[2]++; cnt[3] += s->end[c] - s->beg[c]; }
    }
}

typedef struct {
    const otree *ta, *tb;
    const uint8_t *kind;
    double t4;
    pbuf *m2l, *p2p, *m2p;
} lctx;

/* The receiver's dual traversal of its tree (A) against the grafted remote
 * tree (B): accepted pairs are M2L; a leaf against a sent leaf is P2P (bodies
 * sent) or M2P (multipole only, evaluated at the leaf's bodies, which all lie
 * in the receiver's cube where the sender found the series convergent);
 * otherwise a sent leaf splits A, a leaf A splits B, and else the larger cube
 * is split (both when equal).                                             */
static void let_interact(lctx *c, int a, int b)
{
    const uint64_t pr = ((uint64_t)a << 32) | (uint32_t)b;
    if (mac_cross(c->ta, a, c->tb, b, c->t4)) { pb_push(c->m2l, pr); return; }
    const int aleaf = c->ta->nch[a] == 0, bk = c->kind[b], bleaf = (bk == 2 || bk == 3);
    if (aleaf && bleaf) {
        pb_push(bk == 3 ? c->p2p : c->m2p, pr);
        return;
    }
    int sa, sb;
    if (bleaf) { sa = 1; sb = 0; }
    else if (aleaf) { sa = 0; sb = 1; }
    else {
        const double ha = cell_h(c->ta, a), hb = cell_h(c->tb, b);
        sa = ha >= hb;
        sb = hb >= ha;
    }
    const int na = sa ? c->ta->nch[a] : 1, nb = sb ? c->tb->nch[b] : 1;
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j)
            let_interact(c, sa ? c->ta->cbeg[a] + i : a, sb ? c->tb->cbeg[b] + j : b);
}

static void pb_sort(pbuf *b) { qsort(b->v, (size_t)b->n, sizeof(uint64_t), cmp_u64); }

/* Partition, local trees, LETs and remote lists.  w (nullable) holds integer
 * weights >= 0; count_only != 0 keeps no local list (counts only).  Returns
 * NULL on invalid input.                                                   */
void *oracle_let_new(int64_t n, const double *x, const int64_t *w, int32_t R, int32_t ncrit, double theta,
                     int count_only)
{
    if (n <= 0 || !x || R < 1 || ncrit < 1 || !(theta > 0.0 && theta < 1.0)) return NULL;
    if (w)
        for (int64_t i = 0; i < n; ++i)
            if (w[i] < 0 || w[i] >= ((int64_t)1 << 40)) return NULL;
    olet *L = (olet *)calloc(1, sizeof(olet));
    L->n = n;
    L->R = R;
    L->ncrit = ncrit;
    L->theta = theta;
    L->t4 = 4.0 * theta * theta;
    L->x = (double *)malloc((size_t)n * 3 * sizeof(double));
    memcpy(L->x, x, (size_t)n * 3 * sizeof(double));
    L->rank = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    L->mem = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) L->mem[i] = i;
    orb_split(x, w, L->mem, n, R, 0, L->rank);
    /* members grouped by rank, ascending input index inside a rank */
    L->rstart = (int64_t *)calloc((size_t)R, sizeof(int64_t));
    L->rcount = (int64_t *)calloc((size_t)R, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) L->rcount[L->rank[i]]++;
    for (int r = 1; r < R; ++r) L->rstart[r] = L->rstart[r - 1] + L->rcount[r - 1];
    {
        int64_t *fill = (int64_t *)calloc((size_t)R, sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i) {
            const int r = L->rank[i];
            L->mem[L->rstart[r] + fill[r]++] = i;
        }
        free(fill);
    }
    L->T = (otree **)calloc((size_t)R, sizeof(otree *));
    double *xr = (double *)malloc((size_t)n * 3 * sizeof(double));
    for (int64_t k = 0; k < n; ++k)
        for (int d = 0; d < 3; ++d) xr[3 * k + d] = x[3 * L->mem[k] + d];
    for (int r = 0; r < R; ++r)
        if (L->rcount[r] > 0)
            L->T[r] = (otree *)oracle_tree_new2(L->rcount[r], xr + 3 * L->rstart[r], ncrit, theta,
                                                count_only ? -1 : 0, NULL, 0);
    free(xr);
    const int64_t RR = (int64_t)R * R;
    L->kind = (uint8_t **)calloc((size_t)RR, sizeof(uint8_t *));
    L->rm2l = (pbuf *)calloc((size_t)RR, sizeof(pbuf));
    L->rp2p = (pbuf *)calloc((size_t)RR, sizeof(pbuf));
    L->rm2p = (pbuf *)calloc((size_t)RR, sizeof(pbuf));
    L->cnt = (int64_t *)calloc((size_t)RR * 4, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t rs = 0; rs < RR; ++rs) {
        const int r = (int)(rs / R), s = (int)(rs % R);
        if (r == s || !L->T[r] || !L->T[s]) continue;
        L->kind[rs] = (uint8_t *)malloc((size_t)L->T[s]->ncell);
        let_select(L->T[s], L->T[r], L->t4, L->kind[rs], L->cnt + 4 * rs);
        lctx c = {L->T[r], L->T[s], L->kind[rs], L->t4, &L->rm2l[rs], &L->rp2p[rs], &L->rm2p[rs]};
        let_interact(&c, 0, 0);
        pb_sort(&L->rm2l[rs]);
        pb_sort(&L->rp2p[rs]);
        pb_sort(&L->rm2p[rs]);
    }
    return L;
}

void oracle_let_free(void *h)
{
    olet *L = (olet *)h;
    if (!L) return;
    const int64_t RR = (int64_t)L->R * L->R;
    for (int r = 0; r < L->R; ++r) oracle_tree_free(L->T[r]);
    for (int64_t k = 0; k < RR; ++k) {
        free(L->kind[k]);
        free(L->rm2l[k].v);
        free(L->rp2p[k].v);
        free(L->rm2p[k].v);
    }
    free(L->T); free(L->kind); free(L->rm2l); free(L->rp2p); free(L->rm2p); free(L->cnt);
    free(L->x); free(L->rank); free(L->rstart); free(L->rcount); free(L->mem);
    free(L);
}

/* rank of every body; members (input indices grouped by rank); rstart, rcount */
void oracle_let_partition(const void *h, int32_t *rank, int64_t *mem, int64_t *rstart, int64_t *rcount)
{
    const olet *L = (const olet *)h;
    if (rank) memcpy(rank, L->rank, (size_t)L->n * sizeof(int32_t));
    if (mem) memcpy(mem, L->mem, (size_t)L->n * sizeof(int64_t));
    if (rstart) memcpy(rstart, L->rstart, (size_t)L->R * sizeof(int64_t));
    if (rcount) memcpy(rcount, L->rcount, (size_t)L->R * sizeof(int64_t));
}

/* the local tree of rank r (owned by the LET; NULL for an empty rank) */
void *oracle_let_rank_tree(const void *h, int32_t r)
{
    const olet *L = (const olet *)h;
    return (r >= 0 && r < L->R) ? L->T[r] : NULL;
}

/* per (receiver r, sender s), r-major, 11 values: [LET cells, multipole-only
 * leaves, body leaves, bodies, remote M2L, remote P2P, M2P, digest M2L, digest
 * P2P, digest M2P, digest of the LET] -- digests are mix64 sums like the
 * local lists' (of (A << 32 | B) for the lists, of (cell << 8 | kind) over the
 * cells sent for the LET).  For r == s: [0, 0, 0, 0, local M2L, local P2P, 0,
 * local M2L digest, local P2P digest, 0, 0].                              */
void oracle_let_counts(const void *h, int64_t *out)
{
    const olet *L = (const olet *)h;
    const int64_t RR = (int64_t)L->R * L->R;
    for (int64_t rs = 0; rs < RR; ++rs) {
        int64_t *o = out + 11 * rs;
        const int r = (int)(rs / L->R), s = (int)(rs % L->R);
        for (int k = 0; k < 11; ++k) o[k] = 0;
        if (r == s) {
            if (L->T[r]) {
                o[4] = L->T[r]->n_m2l;
                o[5] = L->T[r]->n_p2p;
                o[7] = (int64_t)L->T[r]->h_m2l;
                o[8] = (int64_t)L->T[r]->h_p2p;
            }
            continue;
        }
        for (int k = 0; k < 4; ++k) o[k] = L->cnt[4 * rs + k];
        o[4] = L->rm2l[rs].n;
        o[5] = L->rp2p[rs].n;
        o[6] = L->rm2p[rs].n;
        const pbuf *b[3] = {&L->rm2l[rs], &L->rp2p[rs], &L->rm2p[rs]};
        for (int k = 0; k < 3; ++k) {
            uint64_t d = 0;
            for (int64_t j = 0; j < b[k]->n; ++j) d += mix64(b[k]->v[j]);
            o[7 + k] = (int64_t)d;
        }
        uint64_t dk = 0;
        if (L->kind[rs])
            for (int64_t c = 0; c < L->T[s]->ncell; ++c)
                if (L->kind[rs][c]) dk += mix64(((uint64_t)c << 8) | L->kind[rs][c]);
        o[10] = (int64_t)dk;
    }
}

/* kind of sender s's cells in the LET for receiver r (s's cell order)     */
void oracle_let_kind(const void *h, int32_t r, int32_t s, uint8_t *kind)
{
    const olet *L = (const olet *)h;
    const int64_t rs = (int64_t)r * L->R + s;
    if (L->kind[rs]) memcpy(kind, L->kind[rs], (size_t)L->T[s]->ncell);
}

/* the remote lists of (r, s) as (A, B) pairs in ascending order           */
void oracle_let_lists(const void *h, int32_t r, int32_t s, int32_t *m2l, int32_t *p2p, int32_t *m2p)
{
    const olet *L = (const olet *)h;
    const int64_t rs = (int64_t)r * L->R + s;
    int32_t *dst[3] = {m2l, p2p, m2p};
    const pbuf *b[3] = {&L->rm2l[rs], &L->rp2p[rs], &L->rm2p[rs]};
    for (int k = 0; k < 3; ++k)
        if (dst[k])
            for (int64_t j = 0; j < b[k]->n; ++j) {
                dst[k][2 * j] = (int32_t)(b[k]->v[j] >> 32);
                dst[k][2 * j + 1] = (int32_t)(b[k]->v[j] & 0xffffffffu);
            }
}

/* Work of every body (input order), the l_i and r_i of Eq. (1): bodies of the
 * leaves in its leaf's P2P list plus cells in the M2L lists of its leaf and
 * the leaf's ancestors, for the local lists (l) and the remote ones (r, M2P
 * cells of its leaf included).  Needs the local lists (not count_only).    */
void oracle_let_work(const void *h, int64_t *lw, int64_t *rw)
{
    const olet *L = (const olet *)h;
    const int R = L->R;
    for (int r = 0; r < R; ++r) {
        const otree *t = L->T[r];
        if (!t) continue;
        int64_t *own = (int64_t *)calloc((size_t)t->ncell, sizeof(int64_t));
        int64_t *rem = (int64_t *)calloc((size_t)t->ncell, sizeof(int64_t));
        for (int64_t c = 0; c < t->ncell; ++c) {
            own[c] = t->m2l_off[c + 1] - t->m2l_off[c];
            if (t->nch[c] == 0)
                for (int64_t k = t->p2p_off[c]; k < t->p2p_off[c + 1]; ++k)
                    own[c] += t->end[t->p2p_src[k]] - t->beg[t->p2p_src[k]];
        }
        for (int s = 0; s < R; ++s) {
            const int64_t rs = (int64_t)r * R + s;
            if (s == r || !L->T[s]) continue;
            const otree *ts = L->T[s];
            for (int64_t j = 0; j < L->rm2l[rs].n; ++j) rem[L->rm2l[rs].v[j] >> 32] += 1;
            for (int64_t j = 0; j < L->rm2p[rs].n; ++j) rem[L->rm2p[rs].v[j] >> 32] += 1;
            for (int64_t j = 0; j < L->rp2p[rs].n; ++j) {
                const int b = (int)(L->rp2p[rs].v[j] & 0xffffffffu);
                rem[L->rp2p[rs].v[j] >> 32] += ts->end[b] - ts->beg[b];
            }
        }
        /* down the tree: a cell's count includes its ancestors' */
        for (int64_t c = 1; c < t->ncell; ++c) {
            own[c] += own[t->par[c]];
            rem[c] += rem[t->par[c]];
        }
        for (int64_t c = 0; c < t->ncell; ++c)
            if (t->nch[c] == 0)
                for (int32_t i = t->beg[c]; i < t->end[c]; ++i) {
                    const int64_t orig = L->mem[L->rstart[r] + t->perm[i]];
                    if (lw) lw[orig] = own[c];
                    if (rw) rw[orig] = rem[c];
                }
        free(own);
        free(rem);
    }
}

/* Multipole series of a cell evaluated at x, with its field: the local
 * expansion about x itself of the truncated multipole series (the M2L of
 * the pinned operator, degrees j <= 1 kept) gives the value and gradient of
 * that series exactly at its center.                                      */
static void m2p_add(const cplx *M, const double cB[3], int p, const double *x, double *phi, double E[3])
{
    cplx Lx[ORC_MAXP * ORC_MAXP] = {0};
    cplx Ih[(2 * ORC_MAXP) * (2 * ORC_MAXP)];
    double D[3] = {x[0] - cB[0], x[1] - cB[1], x[2] - cB[2]};
    harmonics(D, p + 1, NULL, Ih);
    const int jmax = p > 1 ? 2 : 1;
    for (int j = 0; j < jmax; ++j) {
        double sj = (j & 1) ? -1.0 : 1.0;
        for (int s = -j; s <= j; ++s) {
            cplx acc = 0.0;
            for (int nn = 0; nn < p; ++nn)
                for (int m = -nn; m <= nn; ++m) acc += M[HIDX(nn, m)] * hget(Ih, nn + j, m + s);
            Lx[HIDX(j, s)] += sj * acc;
        }
    }
    double ph, Ev[3];
    l2p_eval(Lx, x, jmax, x, &ph, Ev);
    *phi += ph;
    E[0] += Ev[0];
    E[1] += Ev[1];
    E[2] += Ev[2];
}

/* The FMM over the virtual ranks at every body (input order): each rank's
 * upward pass; local expansions from the local M2L list and then from each
 * sender's remote M2L pairs (senders ascending, pairs in order); the
 * downward pass; at every body L2P, the local P2P list, the remote P2P
 * pairs and the M2P pairs (senders ascending).  Needs the local lists.     */
int oracle_let_fmm(const void *h, const double *q, int p, double *phi, double *field)
{
    const olet *L = (const olet *)h;
    if (!L || !q || p < 1 || p > ORC_MAXP) return 1;
    const int R = L->R, P2 = p * p;
    if (R < 1) return 1;
    for (int r = 0; r < R; ++r)
        if (L->T[r] && L->T[r]->n_m2l_stored != L->T[r]->n_m2l) return 2;  /* built count_only */
    cplx **M = (cplx **)calloc((size_t)R, sizeof(cplx *));
    cplx **Lc = (cplx **)calloc((size_t)R, sizeof(cplx *));
    double **xs = (double **)calloc((size_t)R, sizeof(double *));
    double **qs = (double **)calloc((size_t)R, sizeof(double *));
    for (int r = 0; r < R; ++r) {
        const otree *t = L->T[r];
        if (!t) continue;
        const int64_t nc = t->ncell;
        xs[r] = (double *)malloc((size_t)t->n * 3 * sizeof(double));
        qs[r] = (double *)malloc((size_t)t->n * sizeof(double));
        for (int64_t i = 0; i < t->n; ++i) {
            const int64_t o = L->mem[L->rstart[r] + t->perm[i]];
            for (int d = 0; d < 3; ++d) xs[r][3 * i + d] = L->x[3 * o + d];
            qs[r][i] = q[o];
        }
        /* upward pass of rank r */
        cplx *Mr = M[r] = (cplx *)calloc((size_t)nc * P2, sizeof(cplx));
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t c = 0; c < nc; ++c)
            if (t->nch[c] == 0)
                for (int32_t i = t->beg[c]; i < t->end[c]; ++i)
                    p2m_add(xs[r] + 3 * (int64_t)i, qs[r][i], t->ctr + 3 * c, p, Mr + c * P2);
        for (int l = t->depth - 1; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 8)
            for (int64_t c = 0; c < nc; ++c) {
                if (t->lvl[c] != l || t->nch[c] == 0) continue;
                for (int k = 0; k < t->nch[c]; ++k) {
                    int64_t ch = t->cbeg[c] + k;
                    m2m_add(Mr + ch * P2, t->ctr + 3 * ch, t->ctr + 3 * c, p, Mr + c * P2);
                }
            }
        }
    }
    for (int r = 0; r < R; ++r) {
        const otree *t = L->T[r];
        if (!t) continue;
        const int64_t nc = t->ncell;
        cplx *Lr = Lc[r] = (cplx *)calloc((size_t)nc * P2, sizeof(cplx));
        /* remote pairs of each sender as CSR over the receiver's cells */
        int64_t **off = (int64_t **)calloc((size_t)R * 3, sizeof(int64_t *));
        for (int s = 0; s < R; ++s) {
            const int64_t rs = (int64_t)r * R + s;
            const pbuf *b[3] = {&L->rm2l[rs], &L->rp2p[rs], &L->rm2p[rs]};
            for (int k = 0; k < 3; ++k) {
                int64_t *o = off[3 * s + k] = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
                for (int64_t j = 0; j < b[k]->n; ++j) o[(b[k]->v[j] >> 32) + 1]++;
                for (int64_t c = 0; c < nc; ++c) o[c + 1] += o[c];
            }
        }
        /* M2L: the local list, then the senders in order */
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t c = 0; c < nc; ++c) {
            for (int64_t k = t->m2l_off[c]; k < t->m2l_off[c + 1]; ++k) {
                int64_t s = t->m2l_src[k];
                m2l_add(M[r] + s * P2, t->ctr + 3 * s, t->ctr + 3 * c, p, Lr + c * P2);
            }
            for (int s = 0; s < R; ++s) {
                const int64_t rs = (int64_t)r * R + s;
                const int64_t *o = off[3 * s];
                for (int64_t k = o[c]; k < o[c + 1]; ++k) {
                    const int64_t b = (int64_t)(L->rm2l[rs].v[k] & 0xffffffffu);
                    m2l_add(M[s] + b * P2, L->T[s]->ctr + 3 * b, t->ctr + 3 * c, p, Lr + c * P2);
                }
            }
        }
        /* downward pass */
        for (int l = 1; l <= t->depth; ++l) {
#pragma omp parallel for schedule(dynamic, 8)
            for (int64_t c = 0; c < nc; ++c) {
                if (t->lvl[c] != l) continue;
                int64_t pa = t->par[c];
                l2l_add(Lr + pa * P2, t->ctr + 3 * pa, t->ctr + 3 * c, p, Lr + c * P2);
            }
        }
        /* bodies */
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t c = 0; c < nc; ++c) {
            if (t->nch[c] != 0) continue;
            for (int32_t i = t->beg[c]; i < t->end[c]; ++i) {
                const double *xi = xs[r] + 3 * (int64_t)i;
                double pp = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
                /* local P2P, then the senders' bodies */
                for (int s = -1; s < R; ++s) {
                    const otree *ts = s < 0 ? t : L->T[s];
                    const double *xsrc = s < 0 ? xs[r] : xs[s];
                    const double *qsrc = s < 0 ? qs[r] : qs[s];
                    int64_t k0, k1;
                    const uint64_t *pv = NULL;
                    if (s < 0) { k0 = t->p2p_off[c]; k1 = t->p2p_off[c + 1]; }
                    else {
                        const int64_t *o = off[3 * s + 1];
                        k0 = o[c];
                        k1 = o[c + 1];
                        pv = L->rp2p[(int64_t)r * R + s].v;
                    }
                    for (int64_t k = k0; k < k1; ++k) {
                        const int64_t b = pv ? (int64_t)(pv[k] & 0xffffffffu) : t->p2p_src[k];
                        for (int32_t j = ts->beg[b]; j < ts->end[b]; ++j) {
                            double dx = xi[0] - xsrc[3 * (int64_t)j], dy = xi[1] - xsrc[3 * (int64_t)j + 1],
                                   dz = xi[2] - xsrc[3 * (int64_t)j + 2];
                            double r2 = dx * dx + dy * dy + dz * dz;
                            if (r2 == 0.0) continue;
                            double rr = sqrt(r2);
                            double qr = qsrc[j] / rr;
                            double qr3 = qr / r2;
                            pp += qr;
                            ex += qr3 * dx;
                            ey += qr3 * dy;
                            ez += qr3 * dz;
                        }
                    }
                }
                /* M2P of the multipole-only cells of the senders */
                double mp = 0.0, Em[3] = {0.0, 0.0, 0.0};
                for (int s = 0; s < R; ++s) {
                    const int64_t rs = (int64_t)r * R + s;
                    const int64_t *o = off[3 * s + 2];
                    for (int64_t k = o[c]; k < o[c + 1]; ++k) {
                        const int64_t b = (int64_t)(L->rm2p[rs].v[k] & 0xffffffffu);
                        m2p_add(M[s] + b * P2, L->T[s]->ctr + 3 * b, p, xi, &mp, Em);
                    }
                }
                double lp, E[3];
                l2p_eval(Lr + c * P2, t->ctr + 3 * c, p, xi, &lp, E);
                const int64_t orig = L->mem[L->rstart[r] + t->perm[i]];
                if (phi) phi[orig] = lp + pp + mp;
                if (field) {
                    field[3 * orig] = E[0] + ex + Em[0];
                    field[3 * orig + 1] = E[1] + ey + Em[1];
                    field[3 * orig + 2] = E[2] + ez + Em[2];
                }
            }
        }
        for (int k = 0; k < 3 * R; ++k) free(off[k]);
        free(off);
    }
    for (int r = 0; r < R; ++r) {
        free(M[r]); free(Lc[r]); free(xs[r]); free(qs[r]);
    }
    free(M); free(Lc); free(xs); free(qs);
    return 0;
}

/* Convenience: one-shot FMM at the coordinates the tree was built from.   */
int oracle_fmm(const void *h, const double *x, const double *q, int p, int64_t nt,
               const int64_t *targets, double *phi, double *field)
{
    return oracle_fmm_at(h, x, q, p, nt, targets, phi, field);
}

/* For the a priori error bound: per M2L pair the ratio pieces are computed
 * by the tests from the exported lists and centers; nothing else needed.   */

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the later parallel regions (timing of the serial oracle). */
void oracle_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}
