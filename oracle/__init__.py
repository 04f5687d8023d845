"""FP64 CPU oracle for the Barnes-Hut dipolar field -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the CPU-baseline leg of the benchmark may import this
package.  The GPU library never loads it; the two share no code.  Arithmetic lives in ``oracle.c`` (plain
C, FP64, built with gcc and ``-ffp-contract=off``); this module only builds that file and marshals numpy
arrays into it.  ``md.py`` holds the integrator reference.

Vector fields are float64 arrays of shape (3, n).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]
# The timing build of the CPU baseline: the same source and the same arithmetic (no contraction, no
# fast-math), optimised for the host it runs on; built on that host, never shipped.
_NATIVE_LIB = os.path.join(_HERE, "liboracle_native.so")
NATIVE_CFLAGS = ["-O3", "-march=native", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                 "-shared"]


def _native() -> bool:
    return os.environ.get("FFBH_ORACLE_NATIVE") == "1"


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc); with FFBH_ORACLE_NATIVE=1 the timing build
    liboracle_native.so instead."""
    out, flags = (_NATIVE_LIB, NATIVE_CFLAGS) if _native() else (_LIB, _CFLAGS)
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.run(["gcc", *flags, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        path = _NATIVE_LIB if _native() else _LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(path)
        P = C.c_void_p
        i64 = C.c_int64
        L.or_allpairs_field.argtypes = [i64, P, P, P]
        L.or_allpairs_field_subset.argtypes = [i64, P, P, i64, P, P]
        L.or_energy.argtypes = [i64, P, P, P]
        L.or_energy.restype = C.c_double
        L.or_allpairs_grad_r.argtypes = [i64, P, P, P]
        L.or_allpairs_grad_r_subset.argtypes = [i64, P, P, i64, P, P]
        L.or_tree_build.argtypes = [i64, P, P, C.c_int]
        L.or_tree_build.restype = P
        L.or_tree_free.argtypes = [P]
        L.or_tree_num_nodes.argtypes = [P]
        L.or_tree_num_nodes.restype = i64
        L.or_tree_export.argtypes = [P] + [P] * 13
        L.or_bh_field.argtypes = [P, C.c_double, P, P, P]
        L.or_bh_field_order.argtypes = [P, C.c_double, C.c_int, P, P, P]
        L.or_tree_export_D.argtypes = [P, P]
        L.or_bh_field_subset.argtypes = [P, C.c_double, i64, P, P, P, P]
        L.or_bh_lists.argtypes = [P, C.c_double, P, P, P, P]
        L.or_bh_vjp.argtypes = [P, C.c_double, P, P, P]
        L.or_energy_frozen.argtypes = [i64, P, P, P, i64, P, P, P, P, P, P, P, P]
        L.or_energy_frozen.restype = C.c_double
        L.or_fd_grad_frozen.argtypes = [i64, P, P, P, i64, P, P, P, P, P, P, P, C.c_double, P, P]
        L.or_bh_vjp_order.argtypes = [P, C.c_double, C.c_int, P, P, P]
        L.or_energy_frozen_order.argtypes = [i64, P, P, P, i64, P, P, P, P, P, P, P, C.c_int, P]
        L.or_energy_frozen_order.restype = C.c_double
        L.or_fd_grad_frozen_order.argtypes = [i64, P, P, P, i64, P, P, P, P, P, P, P, C.c_double, C.c_int, P, P]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().or_num_threads()


def allpairs_field(pos, mom):
    pos, mom = _f64(pos), _f64(mom)
    H = np.empty_like(pos)
    assert lib().or_allpairs_field(pos.shape[1], _p(pos), _p(mom), _p(H)) == 0
    return H


def allpairs_field_subset(pos, mom, targets):
    pos, mom = _f64(pos), _f64(mom)
    t = np.ascontiguousarray(targets, dtype=np.int64)
    H = np.empty((3, t.size))
    assert lib().or_allpairs_field_subset(pos.shape[1], _p(pos), _p(mom), t.size, _p(t), _p(H)) == 0
    return H


def energy(mom, H, hext=None) -> float:
    mom, H = _f64(mom), _f64(H)
    he = None if hext is None else _f64(hext)
    return lib().or_energy(mom.shape[1], _p(mom), _p(H), _p(he))


def allpairs_grad_r(pos, mom):
    pos, mom = _f64(pos), _f64(mom)
    g = np.empty_like(pos)
    assert lib().or_allpairs_grad_r(pos.shape[1], _p(pos), _p(mom), _p(g)) == 0
    return g


def allpairs_grad_r_subset(pos, mom, targets):
    pos, mom = _f64(pos), _f64(mom)
    t = np.ascontiguousarray(targets, dtype=np.int64)
    g = np.empty((3, t.size))
    assert lib().or_allpairs_grad_r_subset(pos.shape[1], _p(pos), _p(mom), t.size, _p(t), _p(g)) == 0
    return g


class Tree:
    """The uncollapsed octree of the oracle, with pseudo-particles (Eq. magCenter)."""

    def __init__(self, pos, mom, leaf_size: int = 16):
        self.pos, self.mom = _f64(pos), _f64(mom)
        self.n = self.pos.shape[1]
        self.leaf_size = leaf_size
        h = lib().or_tree_build(self.n, _p(self.pos), _p(self.mom), leaf_size)
        if not h:
            raise ValueError("oracle tree build rejected its arguments")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_tree_free(self._h)
            self._h = None

    @property
    def num_nodes(self) -> int:
        return lib().or_tree_num_nodes(self._h)

    def export(self) -> dict:
        n, nn = self.n, self.num_nodes
        d = dict(bbox=np.empty(5), code=np.empty(n, np.uint64), perm=np.empty(n, np.int64),
                 level=np.empty(nn, np.int32), first=np.empty(nn, np.int64),
                 count=np.empty(nn, np.int64), nchild=np.empty(nn, np.int32),
                 child=np.empty((nn, 8), np.int64), parent=np.empty(nn, np.int64),
                 S=np.empty((nn, 3)), M=np.empty((nn, 3)), c=np.empty((nn, 3)), s2=np.empty(nn))
        keys = ["bbox", "code", "perm", "level", "first", "count", "nchild", "child", "parent", "S",
                "M", "c", "s2"]
        lib().or_tree_export(self._h, *[_p(d[k]) for k in keys])
        return d

    def field(self, theta: float, order: int = 1):
        """(H (3, n), n_far (n,), n_near (n,)) for every particle.  order 1: the paper's pseudo-particles
        (Eq. magCenter); order 2: plus the first-moment term of every accepted cell (beyond the paper)."""
        H = np.empty((3, self.n))
        nf = np.empty(self.n, np.int64)
        nr = np.empty(self.n, np.int64)
        if order == 1:
            assert lib().or_bh_field(self._h, theta, _p(H), _p(nf), _p(nr)) == 0
        else:
            assert lib().or_bh_field_order(self._h, theta, order, _p(H), _p(nf), _p(nr)) == 0
        return H, nf, nr

    def first_moments(self):
        """(nn, 3, 3): D[c, k, b] = sum over the members j of cell c of (r_j - c_c)_k m_j,b."""
        D = np.empty((self.num_nodes, 3, 3))
        lib().or_tree_export_D(self._h, _p(D))
        return D

    def field_subset(self, theta: float, targets):
        t = np.ascontiguousarray(targets, dtype=np.int64)
        H = np.empty((3, t.size))
        nf = np.empty(t.size, np.int64)
        nr = np.empty(t.size, np.int64)
        assert lib().or_bh_field_subset(self._h, theta, t.size, _p(t), _p(H), _p(nf), _p(nr)) == 0
        return H, nf, nr

    def lists(self, theta: float) -> dict:
        n = self.n
        fp = np.zeros(n + 1, np.int64)
        npt = np.zeros(n + 1, np.int64)
        assert lib().or_bh_lists(self._h, theta, _p(fp), None, _p(npt), None) == 0
        fn = np.empty(max(int(fp[-1]), 1), np.int64)
        ni = np.empty(max(int(npt[-1]), 1), np.int64)
        assert lib().or_bh_lists(self._h, theta, _p(fp), _p(fn), _p(npt), _p(ni)) == 0
        return dict(far_ptr=fp, far_node=fn, near_ptr=npt, near_idx=ni)

    def vjp(self, theta: float, hbar, order: int = 1):
        """(dL/dr, dL/dm) for L = sum_i hbar_i . H_i with the structure frozen (cells of the given order)."""
        hb = _f64(hbar)
        dr = np.empty((3, self.n))
        dm = np.empty((3, self.n))
        if order == 1:
            assert lib().or_bh_vjp(self._h, theta, _p(hb), _p(dr), _p(dm)) == 0
        else:
            assert lib().or_bh_vjp_order(self._h, theta, order, _p(hb), _p(dr), _p(dm)) == 0
        return dr, dm

    def energy_grad(self, theta: float, hext=None, order: int = 1):
        """(H, E, dE/dr, dE/dm) for E = -1/2 sum m.H - sum m.H_ext, structure frozen; H is linear in the
        moments for either order, so dE/dm = -1/2 H - H_ext + the adjoint of -1/2 m."""
        H, _, _ = self.field(theta, order)
        E = energy(self.mom, H, hext)
        dr, dm = self.vjp(theta, -0.5 * self.mom, order)
        he = np.zeros(3) if hext is None else _f64(hext)
        dm = dm - 0.5 * H - he[:, None]
        return H, E, dr, dm


def frozen_structure(tree: Tree, theta: float) -> dict:
    d = tree.export()
    d.update(tree.lists(theta))
    return d


def energy_frozen(pos, mom, hext, st: dict, order: int = 1) -> float:
    pos, mom = _f64(pos), _f64(mom)
    he = None if hext is None else _f64(hext)
    nn = st["first"].size
    scr = np.empty(15 * nn)
    return lib().or_energy_frozen_order(pos.shape[1], _p(pos), _p(mom), _p(he), nn, _p(st["first"]),
                                        _p(st["count"]), _p(st["perm"]), _p(st["far_ptr"]),
                                        _p(st["far_node"]), _p(st["near_ptr"]), _p(st["near_idx"]),
                                        order, _p(scr))


def fd_grad_frozen(pos, mom, hext, st: dict, h: float = 1e-6, order: int = 1):
    """Central differences (step h) of the frozen-structure energy in every coordinate."""
    pos, mom = _f64(pos), _f64(mom)
    he = None if hext is None else _f64(hext)
    dr = np.empty_like(pos)
    dm = np.empty_like(mom)
    nn = st["first"].size
    assert lib().or_fd_grad_frozen_order(pos.shape[1], _p(pos), _p(mom), _p(he), nn, _p(st["first"]),
                                         _p(st["count"]), _p(st["perm"]), _p(st["far_ptr"]),
                                         _p(st["far_node"]), _p(st["near_ptr"]), _p(st["near_idx"]),
                                         h, order, _p(dr), _p(dm)) == 0
    return dr, dm
