"""ctypes wrapper of the FP64 dense-array oracle in ``lbm_oracle.c``.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Arrays use the dense
layout f[i, z, y, x] (x fastest) and mask[z, y, x] with True = solid.

Physics (arXiv 1703.08015): BGK collision Eq. (2); quasi-compressible
equilibrium Eq. (3) and velocity Eq. (5) (``model=QUASI``, the default) or
incompressible equilibrium Eq. (4) and velocity Eq. (6)
(``model=INCOMPRESSIBLE``); LBGK update Eq. (7), or the MRT collision of
Eq. (8) when ``mrt`` rates are given (published orthogonal moment bases, see
the C source); propagation only between
non-solid nodes (Sec. 3.2) as half-way bounce-back, gather form of
propagation (Sec. 3, Fig. 5).  Body force: Guo forcing (the paper has none).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

_lib = None

QUASI, INCOMPRESSIBLE = 0, 1
_MODELS = {"quasi": QUASI, "quasi-compressible": QUASI, "incompressible": INCOMPRESSIBLE}


def _model(m):
    if isinstance(m, str):
        return _MODELS[m]
    if m not in (QUASI, INCOMPRESSIBLE):
        raise ValueError("unknown model %r" % (m,))
    return int(m)


def build(force=False):
    """Compile the oracle with gcc (FP64, no contraction, OpenMP for timing)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c99",
           "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u32, dbl = ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
        lib.ora_lattice.argtypes = [ctypes.c_int, P, P, P]
        I = ctypes.c_int
        lib.ora_feq.argtypes = [I, I, dbl, P, P]
        lib.ora_guo.argtypes = [I, I, dbl, P, P, P]
        lib.ora_collide.argtypes = [I, I, P, dbl, P, P, P]
        lib.ora_mrt_matrix.argtypes = [I, P, P]
        lib.ora_init.argtypes = [I, I, P, P, dbl, P, P, P]
        lib.ora_step.argtypes = [I, I, P, u32, P, dbl, P, P, P, P, P, i64, I]
        lib.ora_moments.argtypes = [I, I, P, P, P, P, P, P]
        for fn in (lib.ora_lattice, lib.ora_feq, lib.ora_guo, lib.ora_collide, lib.ora_init,
                   lib.ora_step, lib.ora_moments, lib.ora_mrt_matrix):
            fn.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc):
    if rc != 0:
        raise ValueError("oracle call failed (%d)" % rc)


def lattice(q):
    """Velocities c[q,3] (int), weights w[q], opposite index opp[q]."""
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q, np.float64)
    opp = np.zeros(q, np.int32)
    _check(_load().ora_lattice(q, _p(c), _p(w), _p(opp)))
    return c, w, opp


def feq(q, rho, u, model=QUASI):
    out = np.zeros(q)
    u = np.ascontiguousarray(u, np.float64)
    _check(_load().ora_feq(q, _model(model), float(rho), _p(u), _p(out)))
    return out


def guo(q, rho, u, g, model=QUASI):
    """Guo source term without the (1 - omega/2) factor."""
    out = np.zeros(q)
    u = np.ascontiguousarray(u, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    _check(_load().ora_guo(q, _model(model), float(rho), _p(u), _p(g), _p(out)))
    return out


MRT_CLASSES = ("conserved", "e", "eps", "q", "nu", "pi", "m")


def _mrt(mrt):
    """None (BGK) or the rates (s_e, s_eps, s_q, s_pi, s_m) as a C array."""
    if mrt is None:
        return None
    r = np.ascontiguousarray(mrt, np.float64)
    if r.shape != (5,):
        raise ValueError("mrt rates are (s_e, s_eps, s_q, s_pi, s_m)")
    return r


def mrt_matrix(q):
    """Moment basis M[q, q] (rows = moments) and each row's relaxation class
    (index into MRT_CLASSES)."""
    M = np.zeros((q, q))
    cls = np.zeros(q, np.int32)
    _check(_load().ora_mrt_matrix(q, _p(M), _p(cls)))
    return M, cls


def collide(q, f, tau, g, model=QUASI, mrt=None):
    f = np.ascontiguousarray(f, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    out = np.zeros(q)
    r = _mrt(mrt)
    _check(_load().ora_collide(q, _model(model), _p(f), float(tau), _p(g), None if r is None else _p(r), _p(out)))
    return out


def _shape3(mask):
    nz, ny, nx = mask.shape
    return np.array([nx, ny, nz], np.int32)


def _periodic_bits(periodic):
    if isinstance(periodic, (int, np.integer)):
        return int(periodic)
    return int(bool(periodic[0])) | (int(bool(periodic[1])) << 1) | (int(bool(periodic[2])) << 2)


def init(q, mask, rho0=1.0, rho=None, u=None, model=QUASI):
    """Post-collision state at t = 0: f*_i = f_eq_i(rho, u) on fluid nodes."""
    mask = np.ascontiguousarray(mask, np.uint8)
    f = np.zeros((q,) + mask.shape, np.float64)
    rho = None if rho is None else np.ascontiguousarray(rho, np.float64)
    u = None if u is None else np.ascontiguousarray(u, np.float64)
    rp = None if rho is None else _p(rho)
    up = None if u is None else _p(u)
    _check(_load().ora_init(q, _model(model), _p(_shape3(mask)), _p(mask), float(rho0), rp, up, _p(f)))
    return f


def step(q, mask, f, tau, g, nsteps, periodic=7, nthreads=1, model=QUASI, mrt=None, lid=None):
    """lid: None or (axis, side, (u_x, u_y, u_z), rho_w): the face of a non-periodic axis beyond the last
    (side 1) or before the first (side 0) node moves with velocity u_w (moving-wall bounce-back)."""
    """Advance the post-collision state ``f`` by ``nsteps`` steps (in place copy)."""
    mask = np.ascontiguousarray(mask, np.uint8)
    f = np.array(f, np.float64, order="C", copy=True)
    tmp = np.empty_like(f)
    g = np.ascontiguousarray(g, np.float64)
    r = _mrt(mrt)
    lw = None
    if lid is not None:
        axis, side, uw, rho_w = lid
        lw = np.array([axis, side, uw[0], uw[1], uw[2], rho_w], np.float64)
    _check(_load().ora_step(q, _model(model), _p(_shape3(mask)), _periodic_bits(periodic), _p(mask),
                            float(tau), _p(g), None if r is None else _p(r), None if lw is None else _p(lw), _p(f),
                            _p(tmp), int(nsteps), int(nthreads)))
    return f


def moments(q, mask, f, g, model=QUASI):
    """rho[z,y,x], u[3,z,y,x] of the stored post-collision state; solid = 0."""
    mask = np.ascontiguousarray(mask, np.uint8)
    f = np.ascontiguousarray(f, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    rho = np.zeros(mask.shape)
    u = np.zeros((3,) + mask.shape)
    _check(_load().ora_moments(q, _model(model), _p(_shape3(mask)), _p(mask), _p(g), _p(f), _p(rho), _p(u)))
    return rho, u
