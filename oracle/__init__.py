"""ctypes wrapper for the FP64 CPU oracle (test infrastructure only).

Only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  Nothing here is used by the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_u64p = C.POINTER(C.c_uint64)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.oracle_direct.argtypes = [C.c_int64, _dp, _dp, C.c_int64, _i64p, _dp, _dp]
        L.oracle_direct.restype = C.c_int
        L.oracle_legendre.argtypes = [C.c_double, C.c_int, _dp]
        L.oracle_harmonics.argtypes = [_dp, C.c_int, _dp, _dp]
        L.oracle_op_p2m.argtypes = [C.c_int64, _dp, _dp, _dp, C.c_int, _dp]
        L.oracle_op_m2p.argtypes = [_dp, _dp, C.c_int, _dp]
        L.oracle_op_m2p.restype = C.c_double
        L.oracle_op_m2m.argtypes = [_dp, _dp, _dp, C.c_int, _dp]
        L.oracle_op_m2l.argtypes = [_dp, _dp, _dp, C.c_int, _dp]
        L.oracle_op_m2l_rot.argtypes = [_dp, _dp, _dp, C.c_int, _dp]
        L.oracle_wigner_d.argtypes = [C.c_int, C.c_double, _dp]
        L.oracle_op_l2l.argtypes = [_dp, _dp, _dp, C.c_int, _dp]
        L.oracle_op_l2p.argtypes = [_dp, _dp, C.c_int, C.c_int64, _dp, _dp, _dp]
        L.oracle_tree_new.argtypes = [C.c_int64, _dp, C.c_int32, C.c_double, C.c_int64, _i64p]
        L.oracle_tree_new.restype = C.c_void_p
        L.oracle_tree_new2.argtypes = [C.c_int64, _dp, C.c_int32, C.c_double, C.c_int64, _i64p, C.c_int]
        L.oracle_tree_new2.restype = C.c_void_p
        L.oracle_tree_new3.argtypes = [C.c_int64, _dp, C.c_int32, C.c_double, C.c_int64, _i64p, C.c_int, C.c_int]
        L.oracle_tree_new3.restype = C.c_void_p
        L.oracle_tree_radii.argtypes = [C.c_void_p, _i64p]
        L.oracle_tree_free.argtypes = [C.c_void_p]
        L.oracle_tree_info.argtypes = [C.c_void_p, _i64p, _dp]
        L.oracle_tree_digest.argtypes = [C.c_void_p, _u64p]
        L.oracle_tree_export.argtypes = [C.c_void_p, _u64p, _i32p, _i32p, _u64p, _i32p, _i32p,
                                         _i32p, _i32p, _i32p, _dp, _i32p, _i32p]
        L.oracle_fmm_at.argtypes = [C.c_void_p, _dp, _dp, C.c_int, C.c_int64, _i64p, _dp, _dp]
        L.oracle_fmm_at.restype = C.c_int
        L.oracle_near_mutual.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.oracle_near_mutual.restype = C.c_int
        L.oracle_let_new.argtypes = [C.c_int64, _dp, _i64p, C.c_int32, C.c_int32, C.c_double, C.c_int]
        L.oracle_let_new.restype = C.c_void_p
        L.oracle_let_free.argtypes = [C.c_void_p]
        L.oracle_let_partition.argtypes = [C.c_void_p, _i32p, _i64p, _i64p, _i64p]
        L.oracle_let_rank_tree.argtypes = [C.c_void_p, C.c_int32]
        L.oracle_let_rank_tree.restype = C.c_void_p
        L.oracle_let_counts.argtypes = [C.c_void_p, _i64p]
        L.oracle_let_kind.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_uint8)]
        L.oracle_let_lists.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _i32p, _i32p, _i32p]
        L.oracle_let_work.argtypes = [C.c_void_p, _i64p, _i64p]
        L.oracle_let_fmm.argtypes = [C.c_void_p, _dp, C.c_int, _dp, _dp]
        L.oracle_let_fmm.restype = C.c_int
        L.oracle_num_threads.restype = C.c_int
        L.oracle_set_num_threads.argtypes = [C.c_int]
        L.oracle_set_num_threads.restype = None
        _LIB = L
    return _LIB


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(k: int) -> None:
    """Threads of the oracle's later parallel regions (results do not depend
    on it: every target is summed by one thread in a fixed order)."""
    lib().oracle_set_num_threads(int(k))


def direct(x, q, targets=None):
    """O(N^2) FP64 direct sum: (phi, E) at all bodies or at ``targets``."""
    x = _f64(x).reshape(-1, 3)
    q = _f64(q)
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = targets.size, targets.ctypes.data_as(_i64p)
    phi = np.empty(nt)
    E = np.empty((nt, 3))
    rc = lib().oracle_direct(n, _d(x), _d(q), nt, tp, _d(phi), _d(E))
    if rc:
        raise ValueError("oracle_direct failed")
    return phi, E


def legendre(xv: float, nmax: int):
    P = np.zeros(nmax * (nmax + 1) // 2)
    lib().oracle_legendre(float(xv), nmax, _d(P))
    return P


def harmonics(v, nmax: int):
    """(R, I) complex arrays of length nmax^2, index n*n+n+m."""
    v = _f64(v)
    R = np.zeros(2 * nmax * nmax)
    I = np.zeros(2 * nmax * nmax)
    lib().oracle_harmonics(_d(v), nmax, _d(R), _d(I))
    return R.view(np.complex128), I.view(np.complex128)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128).view(np.float64)


def op_p2m(x, q, c, p):
    x = _f64(x).reshape(-1, 3)
    q = _f64(q)
    M = np.zeros(2 * p * p)
    lib().oracle_op_p2m(x.shape[0], _d(x), _d(q), _d(_f64(c)), p, _d(M))
    return M.view(np.complex128)


def op_m2p(M, c, p, x):
    return lib().oracle_op_m2p(_d(_c(M)), _d(_f64(c)), p, _d(_f64(x)))


def op_m2m(M, cch, cpar, p):
    out = np.zeros(2 * p * p)
    lib().oracle_op_m2m(_d(_c(M)), _d(_f64(cch)), _d(_f64(cpar)), p, _d(out))
    return out.view(np.complex128)


def op_m2l(M, cB, cA, p):
    out = np.zeros(2 * p * p)
    lib().oracle_op_m2l(_d(_c(M)), _d(_f64(cB)), _d(_f64(cA)), p, _d(out))
    return out.view(np.complex128)


def op_m2l_rot(M, cB, cA, p):
    """M2L by rotating D onto +z, translating along z and rotating back:
    O(p^3) per pair, the same operator as op_m2l up to rounding."""
    out = np.zeros(2 * p * p)
    lib().oracle_op_m2l_rot(_d(_c(M)), _d(_f64(cB)), _d(_f64(cA)), p, _d(out))
    return out.view(np.complex128)


def wigner_d(n, b):
    """Wigner small-d matrix d^n_{m' m}(b), rows m' and columns m from -n to n."""
    out = np.zeros((2 * n + 1) * (2 * n + 1))
    lib().oracle_wigner_d(int(n), float(b), _d(out))
    return out.reshape(2 * n + 1, 2 * n + 1)


def op_l2l(L, cpar, cch, p):
    out = np.zeros(2 * p * p)
    lib().oracle_op_l2l(_d(_c(L)), _d(_f64(cpar)), _d(_f64(cch)), p, _d(out))
    return out.view(np.complex128)


def op_l2p(L, c, p, x):
    x = _f64(x).reshape(-1, 3)
    phi = np.zeros(x.shape[0])
    E = np.zeros((x.shape[0], 3))
    lib().oracle_op_l2p(_d(_c(L)), _d(_f64(c)), p, x.shape[0], _d(x), _d(phi), _d(E))
    return phi, E


class Tree:
    """Oracle octree + dual-traversal lists for one body set.

    targets=None keeps every list; an index array keeps only what those
    targets need; count_only=True keeps no list (counts are always full).
    prune=True (with targets) walks only the pairs the targets need, so the
    counts then cover only the kept lists (for very large trees).
    """

    def __init__(self, x, ncrit, theta, targets=None, count_only=False, prune=False, tight=False, _handle=None,
                 _owner=None):
        if _handle is not None:
            # a tree owned by another object (a rank of a LET): no build, no free
            self._adopt(_handle, x, ncrit, theta, _owner)
            return
        self.x = _f64(x).reshape(-1, 3)
        self.n = self.x.shape[0]
        self.ncrit, self.theta = int(ncrit), float(theta)
        if count_only:
            nt, tp = -1, None
            self.targets = None
        elif targets is None:
            nt, tp = 0, None
            self.targets = None
        else:
            self.targets = np.ascontiguousarray(targets, dtype=np.int64)
            nt, tp = self.targets.size, self.targets.ctypes.data_as(_i64p)
        self.tight = bool(tight)
        h = lib().oracle_tree_new3(self.n, _d(self.x), self.ncrit, self.theta, nt, tp, 1 if prune else 0,
                                   1 if tight else 0)
        if not h:
            raise ValueError("oracle_tree_new: invalid input")
        self._h = h
        self._owned = True
        self._read_info()

    def _adopt(self, h, x, ncrit, theta, owner):
        self.x = _f64(x).reshape(-1, 3)
        self.n = self.x.shape[0]
        self.ncrit, self.theta = int(ncrit), float(theta)
        self.targets = None
        self._h = h
        self._owned = False
        self._owner = owner  # keeps the owner (and the tree) alive
        self._read_info()

    def _read_info(self):
        h = self._h
        info = np.zeros(7, dtype=np.int64)
        box = np.zeros(5)
        lib().oracle_tree_info(h, info.ctypes.data_as(_i64p), _d(box))
        (self.ncell, self.nleaf, self.depth, self.n_m2l, self.n_p2p,
         self.n_m2l_stored, self.n_p2p_stored) = (int(v) for v in info)
        dg = np.zeros(2, dtype=np.uint64)
        lib().oracle_tree_digest(h, dg.ctypes.data_as(_u64p))
        self.digest_m2l, self.digest_p2p = int(dg[0]), int(dg[1])
        self.lo = box[:3].copy()
        self.S = float(box[3])
        self.scale = float(box[4])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and getattr(self, "_owned", True):
            lib().oracle_tree_free(h)
        self._h = None

    def radii(self):
        """Radius of every cell tight to its bodies, in units S 2^-22 (zeros
        unless the tree uses the tight criterion)."""
        out = np.zeros(self.ncell, np.int64)
        lib().oracle_tree_radii(self._h, out.ctypes.data_as(_i64p))
        return out

    def export(self):
        n, nc = self.n, self.ncell
        out = dict(
            keys=np.zeros(n, np.uint64), perm=np.zeros(n, np.int32),
            level=np.zeros(nc, np.int32), ckey=np.zeros(nc, np.uint64),
            begin=np.zeros(nc, np.int32), end=np.zeros(nc, np.int32),
            parent=np.zeros(nc, np.int32), child_begin=np.zeros(nc, np.int32),
            nchild=np.zeros(nc, np.int32), centers=np.zeros((nc, 3)),
            m2l=np.zeros((self.n_m2l_stored, 2), np.int32),
            p2p=np.zeros((self.n_p2p_stored, 2), np.int32),
        )
        i32 = lambda a: a.ctypes.data_as(_i32p)
        lib().oracle_tree_export(
            self._h, out["keys"].ctypes.data_as(_u64p), i32(out["perm"]), i32(out["level"]),
            out["ckey"].ctypes.data_as(_u64p), i32(out["begin"]), i32(out["end"]),
            i32(out["parent"]), i32(out["child_begin"]), i32(out["nchild"]),
            _d(out["centers"]), i32(out["m2l"]), i32(out["p2p"]))
        return out

    def fmm(self, q, p, targets=None, x=None):
        """FP64 FMM potential and field at all bodies or at ``targets``.

        x (optional) moves the bodies while the tree stays frozen."""
        q = _f64(q)
        xp = self.x if x is None else _f64(x).reshape(-1, 3)
        if targets is None:
            nt, tp = self.n, None
        else:
            targets = np.ascontiguousarray(targets, dtype=np.int64)
            nt, tp = targets.size, targets.ctypes.data_as(_i64p)
        phi = np.zeros(nt)
        E = np.zeros((nt, 3))
        rc = lib().oracle_fmm_at(self._h, _d(xp), _d(q), int(p), nt, tp, _d(phi), _d(E))
        if rc:
            raise ValueError(f"oracle_fmm failed ({rc})")
        return phi, E

    def near_mutual(self, q):
        """Near field (the P2P part alone) of every body, each unordered body
        pair of the P2P lists evaluated once with both bodies updated
        (mutual interactions, Section II.C).  Input order."""
        q = _f64(q)
        phi = np.zeros(self.n)
        E = np.zeros((self.n, 3))
        rc = lib().oracle_near_mutual(self._h, _d(self.x), _d(q), _d(phi), _d(E))
        if rc:
            raise ValueError(f"oracle_near_mutual failed ({rc})")
        return phi, E


class Let:
    """The evaluation split over R virtual ranks (ORB partition with integer
    weights, local trees, LET selection, the remote traversal), FP64.

    count_only=True keeps no local list (counts and digests only)."""

    NSTAT = 11

    def __init__(self, x, R, ncrit, theta, weights=None, count_only=False):
        self.x = _f64(x).reshape(-1, 3)
        self.n = self.x.shape[0]
        self.R, self.ncrit, self.theta = int(R), int(ncrit), float(theta)
        wp = None
        if weights is not None:
            self._w = np.ascontiguousarray(weights, dtype=np.int64)
            wp = self._w.ctypes.data_as(_i64p)
        h = lib().oracle_let_new(self.n, _d(self.x), wp, self.R, self.ncrit, self.theta, 1 if count_only else 0)
        if not h:
            raise ValueError("oracle_let_new: invalid input")
        self._h = h
        self.rank = np.zeros(self.n, np.int32)
        self.members = np.zeros(self.n, np.int64)
        self.rstart = np.zeros(self.R, np.int64)
        self.rcount = np.zeros(self.R, np.int64)
        lib().oracle_let_partition(h, self.rank.ctypes.data_as(_i32p), self.members.ctypes.data_as(_i64p),
                                   self.rstart.ctypes.data_as(_i64p), self.rcount.ctypes.data_as(_i64p))
        st = np.zeros(self.R * self.R * self.NSTAT, np.int64)
        lib().oracle_let_counts(h, st.ctypes.data_as(_i64p))
        self.pair_stats = st.reshape(self.R, self.R, self.NSTAT)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_let_free(h)
            self._h = None

    def tree(self, r):
        """The local tree of rank r (an oracle Tree view), or None."""
        h = lib().oracle_let_rank_tree(self._h, int(r))
        if not h:
            return None
        m = self.members[self.rstart[r]:self.rstart[r] + self.rcount[r]]
        return Tree(self.x[m], self.ncrit, self.theta, _handle=h, _owner=self)

    def kind(self, r, s):
        """LET kind of sender s's cells for receiver r (0 not sent, 1 opened,
        2 multipole only, 3 leaf with bodies)."""
        t = self.tree(s)
        out = np.zeros(t.ncell, np.uint8)
        lib().oracle_let_kind(self._h, int(r), int(s), out.ctypes.data_as(C.POINTER(C.c_uint8)))
        return out

    def lists(self, r, s):
        """Remote (M2L, P2P, M2P) pairs (A of r, B of s), ascending."""
        n = self.pair_stats[r, s, 4:7]
        out = [np.zeros((int(k), 2), np.int32) for k in n]
        ptr = lambda a: a.ctypes.data_as(_i32p) if a.size else None
        lib().oracle_let_lists(self._h, int(r), int(s), *(ptr(a) for a in out))
        return tuple(out)

    def work(self):
        """(l, r) work counts of every body (input order)."""
        lw = np.zeros(self.n, np.int64)
        rw = np.zeros(self.n, np.int64)
        lib().oracle_let_work(self._h, lw.ctypes.data_as(_i64p), rw.ctypes.data_as(_i64p))
        return lw, rw

    def fmm(self, q, p):
        """FP64 potential and field at every body (input order)."""
        q = _f64(q)
        phi = np.zeros(self.n)
        E = np.zeros((self.n, 3))
        rc = lib().oracle_let_fmm(self._h, _d(q), int(p), _d(phi), _d(E))
        if rc:
            raise ValueError(f"oracle_let_fmm failed ({rc})")
        return phi, E
