"""FP64 CPU oracle of the D3Q27 (and, Appendix A, D3Q19) cascaded LBM of
arXiv:1801.04586 (Fei, Luo & Li).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_1801_04586_amd``: the arithmetic lives in
``clbm_oracle.c`` (plain dense 27x27 matrices built from the paper's
definitions, Steps 1-4 of Sec. II B), and this module only marshals numpy
arrays into it.

Array conventions (all float64 unless stated):
  * populations ``f``: shape (27, nz, ny, nx), population order of Eq. (1)
    (D3Q19: (19, nz, ny, nx), order of Eq. (A1)); these are the
    *pre-collision* populations f(x, t) of the paper;
  * velocity ``u``: shape (3, nz, ny, nx); density ``rho``: (nz, ny, nx);
  * force field: (3, nz, ny, nx) force density, added to the uniform force;
  * solid mask: uint8 (nz, ny, nx), 1 = solid.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "clbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

Q = 27
RATE_NAMES = ("s0", "s1", "s2", "s2b", "s3", "s3b", "s4", "s4b", "s5", "s6")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        L.orc_matrix_K.argtypes = [dp, dp]
        L.orc_matrix_M.argtypes = [dp]
        L.orc_matrix_N.argtypes = [dp, dp]
        L.orc_matrix_Ninv.argtypes = [dp, dp]
        L.orc_matrix_Minv.argtypes = [dp]
        L.orc_matrix_S.argtypes = [dp, dp]
        L.orc_invert.argtypes = [ctypes.c_int, dp, dp]
        L.orc_teq.argtypes = [ctypes.c_double, dp]
        L.orc_cvec.argtypes = [dp, dp]
        L.orc_velocities.argtypes = [ip]
        L.orc_exponents.argtypes = [ip]
        L.orc_collide.argtypes = [dp, dp, dp, dp]
        L.orc_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.orc_step.argtypes = [ip, dp, dp, dp, u8, dp, dp]
        L.orc_macro.argtypes = [ip, dp, dp, u8, dp, dp, dp]
        L.orc_init.argtypes = [ip, dp, dp, dp]
        L.orc_adjoint_step.argtypes = [ip, dp, dp, dp, u8, dp, dp, dp, dp, dp]
        L.orc_loss_seed.argtypes = [ip, dp, dp, u8, dp, dp, dp, dp, dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = None
        for name in ("orc19_matrix_M", "orc19_matrix_Minv"):
            getattr(L, name).argtypes = [dp]
        L.orc19_matrix_K.argtypes = [dp, dp]
        L.orc19_matrix_N.argtypes = [dp, dp]
        L.orc19_matrix_S.argtypes = [dp, dp]
        L.orc19_teq.argtypes = [ctypes.c_double, dp]
        L.orc19_cvec.argtypes = [dp, dp]
        L.orc19_velocities.argtypes = [ip]
        L.orc19_exponents.argtypes = [ip]
        L.orc19_collide.argtypes = [dp, dp, dp, dp]
        L.orc19_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.orc19_step.argtypes = [ip, dp, dp, dp, u8, dp, dp]
        L.orc19_step_ex.argtypes = [ip, dp, dp, dp, u8, dp, dp, dp]
        L.orc19_macro.argtypes = [ip, dp, dp, u8, dp, dp, dp]
        L.orc19_init.argtypes = [ip, dp, dp, dp]
        L.orc_mrt_feq.argtypes = [ctypes.c_double, dp, dp]
        L.orc_mrt_guo.argtypes = [dp, dp, dp]
        L.orc_mrt_collide.argtypes = [dp, dp, dp, dp]
        L.orc_mrt_init.argtypes = [ip, dp, dp, dp]
        L.orc_step_ex.argtypes = [ip, dp, dp, dp, u8, dp, ctypes.c_int, dp, dp]
        _lib = L
    return _lib


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's later loops (n >= 1)."""
    lib().orc_set_num_threads(int(n))


# --------------------------------------------------------------------------- helpers
def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _rates(s):
    s = np.ascontiguousarray(np.asarray(s, dtype=np.float64).reshape(10))
    return s


def _vec3(v):
    if v is None:
        return None
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3))


class Geometry:
    """Lattice of dims (nx, ny, nz) with per-axis walls, optionally a window of it.

    ``walls[a]`` is 0 for a periodic axis, 1 for half-way bounce-back walls at
    both ends.  A window covers ``[origin, origin + wdims)`` in global
    coordinates (wrapped on periodic axes); by default the whole lattice.
    """

    def __init__(self, dims, walls=(0, 0, 0), origin=(0, 0, 0), wdims=None):
        self.dims = tuple(int(d) for d in dims)
        self.walls = tuple(int(w) for w in walls)
        self.origin = tuple(int(o) for o in origin)
        self.wdims = tuple(int(d) for d in (wdims if wdims is not None else dims))
        self._arr = np.array(self.dims + self.walls + self.origin + self.wdims, dtype=np.int32)

    @property
    def shape(self):
        nx, ny, nz = self.wdims
        return (nz, ny, nx)

    @property
    def n(self):
        return int(np.prod(self.wdims))

    def ptr(self):
        return self._arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


# --------------------------------------------------------------------------- matrices
def velocities() -> np.ndarray:
    """Eq. (1) velocities, shape (27, 3) int."""
    e = np.zeros(81, dtype=np.int32)
    lib().orc_velocities(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return e.reshape(27, 3).astype(np.int64)


def exponents() -> np.ndarray:
    """Eq. (12) exponents (m, n, p) of the 27 moments, shape (27, 3) int."""
    p = np.zeros(81, dtype=np.int32)
    lib().orc_exponents(p.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return p.reshape(27, 3).astype(np.int64)


def matrix_M() -> np.ndarray:
    out = np.zeros((27, 27))
    lib().orc_matrix_M(_d(out))
    return out


def matrix_Minv() -> np.ndarray:
    out = np.zeros((27, 27))
    rc = lib().orc_matrix_Minv(_d(out))
    assert rc == 0
    return out


def matrix_K(u) -> np.ndarray:
    out = np.zeros((27, 27))
    lib().orc_matrix_K(_d(_vec3(u)), _d(out))
    return out


def matrix_N(u) -> np.ndarray:
    out = np.zeros((27, 27))
    lib().orc_matrix_N(_d(_vec3(u)), _d(out))
    return out


def matrix_Ninv(u) -> np.ndarray:
    out = np.zeros((27, 27))
    lib().orc_matrix_Ninv(_d(_vec3(u)), _d(out))
    return out


def matrix_S(s) -> np.ndarray:
    out = np.zeros((27, 27))
    lib().orc_matrix_S(_d(_rates(s)), _d(out))
    return out


def invert(A) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    out = np.zeros_like(A)
    rc = lib().orc_invert(n, _d(A), _d(out))
    if rc:
        raise np.linalg.LinAlgError("singular")
    return out


def teq(rho) -> np.ndarray:
    out = np.zeros(27)
    lib().orc_teq(float(rho), _d(out))
    return out


def cvec(F) -> np.ndarray:
    out = np.zeros(27)
    lib().orc_cvec(_d(_vec3(F)), _d(out))
    return out


def collide(f, F, s) -> np.ndarray:
    """Steps 1-3 at a single node: pre-collision f (27) -> post-collision f* (27)."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(27)
    out = np.zeros(27)
    rc = lib().orc_collide(_d(f), _d(_vec3(F)), _d(_rates(s)), _d(out))
    assert rc == 0
    return out


def equilibrium(rho, u) -> np.ndarray:
    out = np.zeros(27)
    rc = lib().orc_equilibrium(float(rho), _d(_vec3(u)), _d(out))
    assert rc == 0
    return out


# --------------------------------------------------------------------------- D3Q19 (Appendix A)
def q19_velocities() -> np.ndarray:
    """Eq. (A1) velocities, shape (19, 3) int."""
    e = np.zeros(57, dtype=np.int32)
    lib().orc19_velocities(e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return e.reshape(19, 3).astype(np.int64)


def q19_exponents() -> np.ndarray:
    """Eq. (A2) exponents of the 19 moments, shape (19, 3) int."""
    p = np.zeros(57, dtype=np.int32)
    lib().orc19_exponents(p.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return p.reshape(19, 3).astype(np.int64)


def q19_matrix_M() -> np.ndarray:
    out = np.zeros((19, 19))
    lib().orc19_matrix_M(_d(out))
    return out


def q19_matrix_Minv() -> np.ndarray:
    out = np.zeros((19, 19))
    assert lib().orc19_matrix_Minv(_d(out)) == 0
    return out


def q19_matrix_K(u) -> np.ndarray:
    out = np.zeros((19, 19))
    lib().orc19_matrix_K(_d(_vec3(u)), _d(out))
    return out


def q19_matrix_N(u) -> np.ndarray:
    out = np.zeros((19, 19))
    lib().orc19_matrix_N(_d(_vec3(u)), _d(out))
    return out


def q19_matrix_S(s) -> np.ndarray:
    out = np.zeros((19, 19))
    lib().orc19_matrix_S(_d(_rates(s)), _d(out))
    return out


def q19_teq(rho) -> np.ndarray:
    out = np.zeros(19)
    lib().orc19_teq(float(rho), _d(out))
    return out


def q19_cvec(F) -> np.ndarray:
    out = np.zeros(19)
    lib().orc19_cvec(_d(_vec3(F)), _d(out))
    return out


def q19_collide(f, F, s) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(19)
    out = np.zeros(19)
    assert lib().orc19_collide(_d(f), _d(_vec3(F)), _d(_rates(s)), _d(out)) == 0
    return out


def q19_equilibrium(rho, u) -> np.ndarray:
    out = np.zeros(19)
    assert lib().orc19_equilibrium(float(rho), _d(_vec3(u)), _d(out)) == 0
    return out


# --------------------------------------------------------------------------- MRT (Appendix B)
def mrt_feq(rho, u) -> np.ndarray:
    """Discrete equilibrium f_D^eq of Sec. II B (27 values)."""
    out = np.zeros(27)
    lib().orc_mrt_feq(float(rho), _d(_vec3(u)), _d(out))
    return out


def mrt_guo(u, F) -> np.ndarray:
    """Guo forcing term R_G of Appendix B (27 values)."""
    out = np.zeros(27)
    lib().orc_mrt_guo(_d(_vec3(u)), _d(_vec3(F)), _d(out))
    return out


def mrt_collide(f, F, s) -> np.ndarray:
    """Raw-moment MRT collision of Appendix B at one node: f (27) -> f* (27)."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(27)
    out = np.zeros(27)
    assert lib().orc_mrt_collide(_d(f), _d(_vec3(F)), _d(_rates(s)), _d(out)) == 0
    return out


# --------------------------------------------------------------------------- lattice
LATTICES = ("d3q27", "d3q19")
MODELS = ("cascaded", "mrt")


def _wall_u(wall_velocity):
    """wall_velocity: {(axis, side): (ux, uy, uz)} or a (6, 3) array, face 2*axis + side."""
    if wall_velocity is None:
        return None
    if isinstance(wall_velocity, dict):
        w = np.zeros((6, 3))
        for (a, sd), v in wall_velocity.items():
            w[2 * a + sd] = v
        return w
    return np.ascontiguousarray(np.asarray(wall_velocity, dtype=np.float64).reshape(6, 3))


def _q(lattice: str) -> int:
    if lattice not in LATTICES:
        raise ValueError(f"lattice must be one of {LATTICES}")
    return 27 if lattice == "d3q27" else 19


def init(geom: Geometry, rho0=None, u0=None, lattice: str = "d3q27", model: str = "cascaded") -> np.ndarray:
    """f = f_eq(rho0, u0) at every node; rho0 (nz,ny,nx) or None (=1), u0 (3,nz,ny,nx) or None.
    The cascaded scheme starts from its generalized equilibrium, the MRT from f_D^eq."""
    assert model in MODELS and (model == "cascaded" or lattice == "d3q27")
    f = np.zeros((_q(lattice),) + geom.shape)
    if model == "mrt":
        fn = lib().orc_mrt_init
    else:
        fn = lib().orc_init if lattice == "d3q27" else lib().orc19_init
    rc = fn(geom.ptr(), _d(_f64(rho0)), _d(_f64(u0)), _d(f))
    assert rc == 0
    return f


def step(geom: Geometry, f, s, force=(0.0, 0.0, 0.0), force_field=None, solid=None,
         lattice: str = "d3q27", model: str = "cascaded", wall_velocity=None) -> np.ndarray:
    """One time step (Steps 1-4); returns the pre-collision populations at t+1.

    model "mrt": the raw-moment MRT of Appendix B (D3Q27); wall_velocity: moving
    walls, {(axis, side): (ux, uy, uz)}."""
    f = _f64(f)
    assert f.shape[0] == _q(lattice) and model in MODELS
    out = np.empty_like(f)
    solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    args = (_d(_rates(s)), _d(_vec3(force)), _d(_f64(force_field)), _u8(solid))
    if lattice == "d3q19":
        assert model == "cascaded"
        rc = lib().orc19_step_ex(geom.ptr(), *args, _d(_wall_u(wall_velocity)), _d(f), _d(out))
    elif model == "cascaded" and wall_velocity is None:
        rc = lib().orc_step(geom.ptr(), *args, _d(f), _d(out))
    else:
        assert lattice == "d3q27"
        rc = lib().orc_step_ex(geom.ptr(), *args, _d(_wall_u(wall_velocity)), MODELS.index(model), _d(f), _d(out))
    assert rc == 0, rc
    return out


def run(geom: Geometry, f, s, nsteps, force=(0.0, 0.0, 0.0), force_field=None, solid=None,
        lattice: str = "d3q27", model: str = "cascaded", wall_velocity=None) -> np.ndarray:
    for _ in range(int(nsteps)):
        f = step(geom, f, s, force, force_field, solid, lattice, model, wall_velocity)
    return f


def macro(geom: Geometry, f, force=(0.0, 0.0, 0.0), force_field=None, solid=None, lattice: str = "d3q27"):
    """Eq. (9): returns (rho (nz,ny,nx), u (3,nz,ny,nx))."""
    f = _f64(f)
    assert f.shape[0] == _q(lattice)
    rho = np.zeros(geom.shape)
    u = np.zeros((3,) + geom.shape)
    solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    fn = lib().orc_macro if lattice == "d3q27" else lib().orc19_macro
    rc = fn(geom.ptr(), _d(_vec3(force)), _d(_f64(force_field)), _u8(solid), _d(f), _d(rho), _d(u))
    assert rc == 0
    return rho, u


def adjoint_step(geom: Geometry, f_t, lam_next, s, force=(0.0, 0.0, 0.0), force_field=None, solid=None,
                 gF=None, gs=None):
    """lambda(t) = (dPhi/df)^T P^T lambda(t+1); accumulates dJ/dF into gF (3,...) and dJ/ds into gs (10)."""
    f_t = _f64(f_t)
    lam_next = _f64(lam_next)
    lam = np.empty_like(lam_next)
    if gF is None:
        gF = np.zeros((3,) + geom.shape)
    if gs is None:
        gs = np.zeros(10)
    solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    rc = lib().orc_adjoint_step(geom.ptr(), _d(_rates(s)), _d(_vec3(force)), _d(_f64(force_field)), _u8(solid),
                                _d(f_t), _d(lam_next), _d(lam), _d(gF), _d(gs))
    assert rc == 0
    return lam, gF, gs


def loss_seed(geom: Geometry, f, u_target, force=(0.0, 0.0, 0.0), force_field=None, solid=None, gF=None):
    """J = 1/2 sum_fluid |u - u_target|^2; returns (J, dJ/df, gF with the direct dJ/dF added)."""
    f = _f64(f)
    lam = np.empty_like(f)
    if gF is None:
        gF = np.zeros((3,) + geom.shape)
    J = ctypes.c_double(0.0)
    solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
    rc = lib().orc_loss_seed(geom.ptr(), _d(_vec3(force)), _d(_f64(force_field)), _u8(solid), _d(f),
                             _d(_f64(u_target)), _d(lam), _d(gF), ctypes.byref(J))
    assert rc == 0
    return J.value, lam, gF


def loss_and_grads(geom: Geometry, f0, s, nsteps, u_target, force=(0.0, 0.0, 0.0), force_field=None,
                   solid=None):
    """Run nsteps from f0, J = 1/2 sum |u(T) - u_t|^2, and the exact discrete adjoint.

    Returns (J, dJ/dF field (3,...), dJ/ds (10), dJ/df0 (27,...)).  Stores every state.
    """
    states = [_f64(f0)]
    for _ in range(int(nsteps)):
        states.append(step(geom, states[-1], s, force, force_field, solid))
    J, lam, gF = loss_seed(geom, states[-1], u_target, force, force_field, solid)
    gs = np.zeros(10)
    for t in range(int(nsteps) - 1, -1, -1):
        lam, gF, gs = adjoint_step(geom, states[t], lam, s, force, force_field, solid, gF, gs)
    return J, gF, gs, lam
