"""ctypes access to the C oracle in oracle.c (test infrastructure only).

Every function here is marshalling: the arithmetic lives in oracle.c.
The library is compiled by build() (plain gcc, no GPU code) and loaded from
this directory.
"""
import ctypes
import os
import subprocess

import numpy as np

MONO, QUAD, SPLIT_QUAD, SPLIT_MONO, QUAD_SOFT = 0, 1, 2, 3, 4
# how the split kernel's cutoff decision is taken (see orc_split_keep)
MASK_ABS, MASK_F64_OFS = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)


def build():
    """Compile oracle.c into liboracle.so (always recompiles)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)


def lib():
    """Load liboracle.so, compiling it first only if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.orc_build.restype = ctypes.c_int
        L.orc_build.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_double,
                                ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_void_p)]
        L.orc_free.argtypes = [ctypes.c_void_p]
        L.orc_sizes.argtypes = [ctypes.c_void_p, _I64]
        L.orc_export_lists.argtypes = [ctypes.c_void_p, _I64, _I64, _I32,
                                       _I64, _I64, _I64, _I32]
        L.orc_export_nodes.argtypes = [ctypes.c_void_p, _D, _D, _D, _D, _D,
                                       _D, _I64]
        L.orc_eval.argtypes = [ctypes.c_int, ctypes.c_int64, _I64, _I64, _D,
                               _D, _I64, _D, _D, _I64, _D, _D, _D, _D,
                               ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, _D, _D, _D]
        L.orc_count_keep.argtypes = [ctypes.c_int, ctypes.c_int64, _I64, _I64, _D, _I64, _D,
                                     _I64, _D, ctypes.c_double, ctypes.c_double, _D, _I64]
        L.orc_mask_flips.restype = ctypes.c_int64
        L.orc_mask_flips.argtypes = [ctypes.c_int64, _I64, _I64, _D, _I64, _D, _I64,
                                     _D, ctypes.c_double, ctypes.c_double, _D]
        L.orc_split_keep.restype = ctypes.c_int
        L.orc_split_keep.argtypes = [ctypes.c_int, _D, _D, _D, ctypes.c_double,
                                     ctypes.c_double]
        L.orc_direct.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_int64,
                                 _I64, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, _D, _D]
        L.orc_moments.argtypes = [ctypes.c_int64, _I64, _D, _D, _D, _D, _D, _D]
        L.orc_pp_plummer.argtypes = [_D, ctypes.c_double, ctypes.c_double, _D, _D]
        L.orc_pc_quad.argtypes = [_D, ctypes.c_double, _D, ctypes.c_double,
                                  _D, _D]
        L.orc_pc_mono.argtypes = [_D, ctypes.c_double, ctypes.c_double, _D, _D]
        L.orc_pc_quad_soft.argtypes = [_D, ctypes.c_double, _D, ctypes.c_double,
                                       ctypes.c_double, _D, _D]
        L.orc_pc_split.argtypes = [_D, ctypes.c_double, _D, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, _D, _D]
        L.orc_pp_split.argtypes = [_D, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, _D, _D]
        L.orc_split_derivs.argtypes = [ctypes.c_double, ctypes.c_double, _D,
                                       _D, _D, _D]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(_I64) if a is not None else None


def _cd(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads():
    return lib().orc_num_threads()


def set_threads(n):
    """Threads for the oracle's later parallel loops (results unchanged)."""
    lib().orc_set_threads(int(n))


class Tree:
    """Tree, groups and interaction lists built by the oracle (exported as
    numpy arrays; the C object is freed on construction)."""

    def __init__(self, x, m, theta, ncrit, nleaf=8, maxdepth=21, box=0.0,
                 rcut=0.0, walk_stride=1):
        x = _cd(x).reshape(-1, 3)
        m = _cd(m)
        n = x.shape[0]
        h = ctypes.c_void_p()
        rc = lib().orc_build(n, _dp(x), _dp(m), float(theta), int(ncrit),
                             int(nleaf), int(maxdepth), float(box), float(rcut),
                             int(walk_stride), ctypes.byref(h))
        if rc != 0:
            raise RuntimeError("orc_build failed with code %d" % rc)
        try:
            sz = np.zeros(4, np.int64)
            lib().orc_sizes(h, _ip(sz))
            ng, njp, njc, nn = (int(v) for v in sz)
            self.n, self.ngroups, self.nnodes = n, ng, nn
            self.perm = np.zeros(n, np.int64)
            self.i_off = np.zeros(ng + 1, np.int64)
            self.gnode = np.zeros(ng, np.int32)
            self.jp_off = np.zeros(ng + 1, np.int64)
            self.jp_idx = np.zeros(njp, np.int64)
            self.jc_off = np.zeros(ng + 1, np.int64)
            self.jc_node = np.zeros(njc, np.int32)
            lib().orc_export_lists(h, _ip(self.perm), _ip(self.i_off),
                                   self.gnode.ctypes.data_as(_I32),
                                   _ip(self.jp_off), _ip(self.jp_idx),
                                   _ip(self.jc_off),
                                   self.jc_node.ctypes.data_as(_I32))
            self.center = np.zeros((nn, 3))
            self.side = np.zeros(nn)
            self.mass = np.zeros(nn)
            self.com = np.zeros((nn, 3))
            self.q = np.zeros((nn, 6))
            self.trace = np.zeros(nn)
            ints = np.zeros((nn, 8), np.int64)
            lib().orc_export_nodes(h, _dp(self.center), _dp(self.side),
                                   _dp(self.mass), _dp(self.com), _dp(self.q),
                                   _dp(self.trace), _ip(ints))
            self.first, self.count = ints[:, 0].copy(), ints[:, 1].copy()
            self.parent, self.depth = ints[:, 2].copy(), ints[:, 3].copy()
            self.leaf = ints[:, 4].astype(bool)
        finally:
            lib().orc_free(h)
        self.theta, self.ncrit, self.box, self.rcut = theta, ncrit, box, rcut
        self.walk_stride = walk_stride

    def sample_mat(self, x, m, groups):
        """Materialised lists of the given groups only (their i-particles in
        original indexing), e.g. the groups a strided walk visited."""
        x = _cd(x).reshape(-1, 3)
        m = _cd(m)
        groups = np.asarray(groups, np.int64)
        i_idx, i_off, jp_off, jc_off, jp, jc = [], [0], [0], [0], [], []
        for g in groups:
            i_idx.append(self.perm[self.i_off[g]:self.i_off[g + 1]])
            i_off.append(i_off[-1] + self.i_off[g + 1] - self.i_off[g])
            jp.append(self.jp_idx[self.jp_off[g]:self.jp_off[g + 1]])
            jc.append(self.jc_node[self.jc_off[g]:self.jc_off[g + 1]].astype(np.int64))
            jp_off.append(jp_off[-1] + len(jp[-1]))
            jc_off.append(jc_off[-1] + len(jc[-1]))
        jp = np.concatenate(jp)
        jc = np.concatenate(jc)
        return dict(i_idx=np.concatenate(i_idx), i_off=np.array(i_off),
                    gcenter=self.center[self.gnode[groups]],
                    gside=self.side[self.gnode[groups]],
                    jp_off=np.array(jp_off), jp_x=x[jp], jp_m=m[jp],
                    jc_off=np.array(jc_off), jc_x=self.com[jc],
                    jc_m=self.mass[jc], jc_q=self.q[jc], jc_t=self.trace[jc])

    @property
    def n_jp(self):
        return int(self.jp_off[-1])

    @property
    def n_jc(self):
        return int(self.jc_off[-1])

    def interaction_counts(self):
        """(n_pp, n_pc): sum over groups of n_i * list length."""
        ni = np.diff(self.i_off)
        return (int(np.sum(ni * np.diff(self.jp_off))),
                int(np.sum(ni * np.diff(self.jc_off))))


def build_tree(x, m, theta, ncrit, **kw):
    return Tree(x, m, theta, ncrit, **kw)


def materialise(tree, x, m):
    """The lists with their j-data copied out (the layout the GPU library
    takes): returns a dict of FP64 arrays."""
    x = _cd(x).reshape(-1, 3)
    m = _cd(m)
    jc = tree.jc_node.astype(np.int64)
    gcenter = tree.center[tree.gnode]
    return dict(
        i_idx=tree.perm, i_off=tree.i_off, gcenter=gcenter,
        gside=tree.side[tree.gnode],
        jp_off=tree.jp_off, jp_x=x[tree.jp_idx], jp_m=m[tree.jp_idx],
        jc_off=tree.jc_off, jc_x=tree.com[jc], jc_m=tree.mass[jc],
        jc_q=tree.q[jc], jc_t=tree.trace[jc],
    )


def eval_lists(kind, mat, x, eps2, box=0.0, rs=0.0, rcut=0.0,
               mask=MASK_ABS):
    """Oracle evaluation of materialised lists (see orc_eval).  Returns
    (a[n,3], phi[n]) in original particle order; particles not in any group
    are left at zero.  mask: how the split kernel's cutoff is decided."""
    x = _cd(x).reshape(-1, 3)
    eps2 = _cd(np.broadcast_to(eps2, (x.shape[0],)))
    n = x.shape[0]
    a = np.zeros((n, 3))
    phi = np.zeros(n)
    i_idx = np.ascontiguousarray(mat["i_idx"], np.int64)
    i_off = np.ascontiguousarray(mat["i_off"], np.int64)
    jp_off = np.ascontiguousarray(mat["jp_off"], np.int64)
    jc_off = np.ascontiguousarray(mat["jc_off"], np.int64)
    jp_x, jp_m = _cd(mat["jp_x"]), _cd(mat["jp_m"])
    jc_x, jc_m, jc_q = _cd(mat["jc_x"]), _cd(mat["jc_m"]), _cd(mat["jc_q"])
    jc_t = _cd(mat["jc_t"]) if mat.get("jc_t") is not None else None
    ng = i_off.shape[0] - 1
    gc = _cd(mat["gcenter"]) if mask != MASK_ABS else None
    lib().orc_eval(int(kind), ng, _ip(i_idx), _ip(i_off), _dp(x), _dp(eps2),
                   _ip(jp_off), _dp(jp_x), _dp(jp_m), _ip(jc_off), _dp(jc_x),
                   _dp(jc_m), _dp(jc_q), _dp(jc_t), float(box), float(rs),
                   float(rcut), int(mask), _dp(gc), _dp(a), _dp(phi))
    return a, phi


def mask_flips(mat, x, box, rcut):
    """Number of terms of the materialised lists on which the cutoff
    decision from absolute FP64 separations (the definition, MASK_ABS) and
    the one from FP64 offsets to the group centres (MASK_F64_OFS) differ."""
    x = _cd(x).reshape(-1, 3)
    i_idx = np.ascontiguousarray(mat["i_idx"], np.int64)
    i_off = np.ascontiguousarray(mat["i_off"], np.int64)
    jp_off = np.ascontiguousarray(mat["jp_off"], np.int64)
    jc_off = np.ascontiguousarray(mat["jc_off"], np.int64)
    ng = i_off.shape[0] - 1
    return int(lib().orc_mask_flips(ng, _ip(i_idx), _ip(i_off), _dp(x), _ip(jp_off),
                                    _dp(_cd(mat["jp_x"])), _ip(jc_off),
                                    _dp(_cd(mat["jc_x"])), float(box), float(rcut),
                                    _dp(_cd(mat["gcenter"]))))


def count_keep(mat, x, box, rcut, mask=MASK_ABS):
    """(particle terms, cell terms) of the materialised lists that the
    cutoff keeps under the given decision."""
    x = _cd(x).reshape(-1, 3)
    i_off = np.ascontiguousarray(mat["i_off"], np.int64)
    out = np.zeros(2, np.int64)
    lib().orc_count_keep(int(mask), i_off.shape[0] - 1,
                         _ip(np.ascontiguousarray(mat["i_idx"], np.int64)), _ip(i_off), _dp(x),
                         _ip(np.ascontiguousarray(mat["jp_off"], np.int64)),
                         _dp(_cd(mat["jp_x"])),
                         _ip(np.ascontiguousarray(mat["jc_off"], np.int64)),
                         _dp(_cd(mat["jc_x"])), float(box), float(rcut),
                         _dp(_cd(mat["gcenter"])), _ip(out))
    return int(out[0]), int(out[1])


def direct(x, m, eps2=0.0, targets=None, split=False, box=0.0, rs=0.0,
           rcut=0.0):
    """Direct summation (Sec. 4, eq. 8 reference) for the given targets."""
    x = _cd(x).reshape(-1, 3)
    m = _cd(m)
    n = x.shape[0]
    eps2 = _cd(np.broadcast_to(eps2, (n,)))
    if targets is None:
        nt, tp, tgt = n, None, None
    else:
        tgt = np.ascontiguousarray(targets, np.int64)
        nt, tp = tgt.shape[0], _ip(tgt)
    a = np.zeros((nt, 3))
    phi = np.zeros(nt)
    lib().orc_direct(n, _dp(x), _dp(m), _dp(eps2), nt, tp, int(bool(split)),
                     float(box), float(rs), float(rcut), _dp(a), _dp(phi))
    return a, phi


def moments(x, m):
    """(M, com[3], q[6], T) of a particle set, computed directly (eq. 2)."""
    x = _cd(x).reshape(-1, 3)
    m = _cd(m)
    M = ctypes.c_double()
    T = ctypes.c_double()
    com = np.zeros(3)
    q = np.zeros(6)
    lib().orc_moments(x.shape[0], None, _dp(x), _dp(m), ctypes.byref(M),
                      _dp(com), _dp(q), ctypes.byref(T))
    return M.value, com, q, T.value


def _single(fn, d, *args):
    d = _cd(d)
    a = np.zeros(3)
    phi = ctypes.c_double(0.0)
    fn(_dp(d), *args, _dp(a), ctypes.byref(phi))
    return a, phi.value


def pp_plummer(d, m, eps2):
    return _single(lib().orc_pp_plummer, d, float(m), float(eps2))


def pc_quad(d, M, q, eps2):
    q = _cd(q)
    return _single(lib().orc_pc_quad, d, float(M), _dp(q), float(eps2))


def pc_quad_soft(d, M, q, T, eps2):
    """Plummer cell, complete second-order expansion (with the trace T)."""
    q = _cd(q)
    return _single(lib().orc_pc_quad_soft, d, float(M), _dp(q), float(T),
                   float(eps2))


def pc_mono(d, M, eps2):
    return _single(lib().orc_pc_mono, d, float(M), float(eps2))


def pc_split(d, M, q, T, rs, rcut, use_quad=True):
    q = _cd(q)
    return _single(lib().orc_pc_split, d, float(M), _dp(q), float(T),
                   float(rs), float(rcut), int(bool(use_quad)))


def pp_split(d, m, rs, rcut):
    return _single(lib().orc_pp_split, d, float(m), float(rs), float(rcut))


def split_keep(mode, xj, xi, c, box, rcut):
    return bool(lib().orc_split_keep(int(mode), _dp(_cd(xj)), _dp(_cd(xi)),
                                     _dp(_cd(c)), float(box), float(rcut)))


def split_derivs(r, rs):
    out = [ctypes.c_double() for _ in range(4)]
    lib().orc_split_derivs(float(r), float(rs), *[ctypes.byref(o) for o in out])
    return tuple(o.value for o in out)


def relative_errors(a_test, a_ref):
    """Per-particle |a_test - a_ref| / |a_ref| (Sec. 4, eq. 8)."""
    a_test = np.asarray(a_test, np.float64).reshape(-1, 3)
    a_ref = np.asarray(a_ref, np.float64).reshape(-1, 3)
    return (np.linalg.norm(a_test - a_ref, axis=1) /
            np.linalg.norm(a_ref, axis=1))


def leapfrog(x, v, m, eps, dt, nsteps, theta, ncrit, kind=QUAD, nleaf=8, box=0.0,
             rs=0.0, rcut=0.0, pm_mesh=0):
    """Kick-drift-kick leapfrog (second order, time reversible; the
    integrator of the paper's cold-collapse runs), forces from the oracle's
    own tree and lists, rebuilt after every drift:
        v += dt/2 a(x);  x += dt v;  v += dt/2 a(x).
    Periodic TreePM (box > 0, split kinds): the split tree force (cutoff
    decided in FP64 from group-relative offsets) plus, when pm_mesh > 0,
    the particle-mesh long-range force of oracle.pm, with positions mapped
    to [0, box) after each drift by x - box floor(x / box) (and one more box
    off if that rounds to box).  Returns (x, v, a, phi) after nsteps, FP64."""
    from . import pm as _pm
    x = np.array(x, np.float64).reshape(-1, 3)
    v = np.array(v, np.float64).reshape(-1, 3)
    m = np.asarray(m, np.float64)
    split = kind in (SPLIT_QUAD, SPLIT_MONO)

    def force(xx):
        T = Tree(xx, m, theta, ncrit, nleaf, box=box, rcut=rcut)
        if split:
            a, phi = eval_lists(kind, materialise(T, xx, m), xx, 0.0, box=box, rs=rs,
                                rcut=rcut, mask=MASK_F64_OFS)
            if pm_mesh:
                al, pl = _pm.pm(xx, m, box, pm_mesh, rs)
                a, phi = a + al, phi + pl
            return a, phi
        return eval_lists(kind, materialise(T, xx, m), xx, eps * eps)

    def wrap(xx):
        if box <= 0.0:
            return xx
        y = xx - box * np.floor(xx / box)
        return np.where(y >= box, y - box, y)

    a, phi = force(x)
    for _ in range(nsteps):
        v = v + (0.5 * dt) * a
        x = wrap(x + dt * v)
        a, phi = force(x)
        v = v + (0.5 * dt) * a
    return x, v, a, phi
