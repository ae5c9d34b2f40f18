"""ctypes binding of libclbm.so (include/clbm.h): argument marshalling only.

Every step of the method runs in the HIP kernels of the library; this module
passes torch tensors' device pointers and the current HIP stream through the C
ABI and turns status codes into exceptions.  There is no fallback: if the
library is missing or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclbm.so")

CLBM_F64, CLBM_F32, CLBM_F16, CLBM_BF16 = 0, 1, 2, 3
STORAGE = {"f64": CLBM_F64, "f32": CLBM_F32, "f16": CLBM_F16, "bf16": CLBM_BF16}
STORAGE_TORCH = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
# arithmetic / adjoint / force-field type per storage
REAL_TORCH = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float32, "bf16": torch.float32}
RATE_NAMES = ("s0", "s1", "s2", "s2b", "s3", "s3b", "s4", "s4b", "s5", "s6")
ABI_VERSION = 7  # CLBM_ABI_VERSION of include/clbm.h
CLBM_D3Q27, CLBM_D3Q19 = 0, 1
LATTICE = {"d3q27": CLBM_D3Q27, "d3q19": CLBM_D3Q19}
LATTICE_Q = {"d3q27": 27, "d3q19": 19}
CLBM_CASCADED, CLBM_MRT = 0, 1
COLLISION = {"cascaded": CLBM_CASCADED, "mrt": CLBM_MRT}
_STORAGE_DTYPE = {STORAGE[k]: v for k, v in STORAGE_TORCH.items()}


class ClbmError(RuntimeError):
    def __init__(self, func: str, code: int, msg: str):
        super().__init__(f"{func} failed ({code}): {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("wall", ctypes.c_int32 * 3),
        ("storage", ctypes.c_int32),
        ("lattice", ctypes.c_int32),
        ("s", ctypes.c_double * 10),
        ("force_uniform", ctypes.c_double * 3),
        ("force_scale", ctypes.c_double),
        ("force", ctypes.c_void_p),
        ("solid", ctypes.c_void_p),
        ("collision", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("wall_velocity", ctypes.c_double * 18),
        ("plane_stride", ctypes.c_int64),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libclbm.so and declare its C signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(path)
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    sig = {
        "clbm_abi_version": ([], ctypes.c_int),
        "clbm_default_plane_stride": ([i32, i32, i32, i32], ctypes.c_int64),
        "clbm_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "clbm_last_error": ([vp], ctypes.c_char_p),
        "clbm_create": ([ctypes.POINTER(vp), ctypes.POINTER(Desc), vp], ctypes.c_int),
        "clbm_destroy": ([vp], ctypes.c_int),
        "clbm_set_stream": ([vp, vp], ctypes.c_int),
        "clbm_set_rates": ([vp, dp], ctypes.c_int),
        "clbm_set_force": ([vp, dp, vp, ctypes.c_double], ctypes.c_int),
        "clbm_init": ([vp, vp, vp, vp], ctypes.c_int),
        "clbm_step": ([vp, vp, vp], ctypes.c_int),
        "clbm_run": ([vp, vp, vp, i32, ctypes.POINTER(vp)], ctypes.c_int),
        "clbm_trajectory": ([vp, vp, ctypes.POINTER(vp), i32], ctypes.c_int),
        "clbm_set_options": ([vp, ctypes.c_uint32], ctypes.c_int),
        "clbm_fused_pairs": ([vp], ctypes.c_int),
        "clbm_copy": ([vp, vp, vp], ctypes.c_int),
        "clbm_moments": ([vp, vp, vp, vp, dp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "clbm_get_populations": ([vp, vp, vp], ctypes.c_int),
        "clbm_set_populations": ([vp, vp, vp], ctypes.c_int),
        "clbm_sample_populations": ([vp, vp, vp, i32, vp], ctypes.c_int),
        "clbm_adjoint_step": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "clbm_loss_seed": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "clbm_adjoint_step_noalloc": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "clbm_adjoint_noalloc_max_nodes": ([], ctypes.c_int64),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    if L.clbm_abi_version() != ABI_VERSION:
        raise ImportError("libclbm.so ABI version mismatch")
    _lib = L
    return L


def strerror(code: int) -> str:
    return load_library().clbm_strerror(code).decode()


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """Owns a clbm_ctx.  Method names follow the C ABI (clbm_<name>)."""

    def __init__(self, desc: Desc, device: torch.device):
        self.lib = load_library()
        self.device = device
        self._h = ctypes.c_void_p()
        rc = self.lib.clbm_create(ctypes.byref(self._h), ctypes.byref(desc), _stream(device))
        if rc:
            raise ClbmError("clbm_create", rc, self.lib.clbm_last_error(None).decode())
        self.desc = desc
        n = desc.nx * desc.ny * desc.nz
        q = 19 if desc.lattice == CLBM_D3Q19 else 27
        es = {CLBM_F64: 8, CLBM_F32: 4}.get(desc.storage, 2)
        self.state_bytes = q * (desc.plane_stride or n) * es  # size of one state buffer

    def _state(self, t: Optional[torch.Tensor]):
        """Pointer of a state buffer, after checking that it holds Q x P elements of the storage type."""
        if t is None:
            raise ValueError("state buffer is None")
        want = _STORAGE_DTYPE[self.desc.storage]
        if t.dtype != want:
            raise ValueError(f"state buffer has dtype {t.dtype}, {want} needed (the storage type)")
        if t.numel() * t.element_size() < self.state_bytes:
            raise ValueError(f"state buffer of {t.numel() * t.element_size()} bytes, {self.state_bytes} needed "
                             "(Q x plane_stride elements)")
        return _ptr(t)

    def _call(self, name, *args):
        fn = getattr(self.lib, name)
        self.lib.clbm_set_stream(self._h, _stream(self.device))
        rc = fn(self._h, *args)
        if rc:
            raise ClbmError(name, rc, self.lib.clbm_last_error(self._h).decode())
        return rc

    def close(self):
        if self._h:
            self.lib.clbm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- ABI mirrors
    def set_rates(self, s):
        arr = (ctypes.c_double * 10)(*[float(v) for v in s])
        self._call("clbm_set_rates", arr)

    def set_force(self, uniform, field: Optional[torch.Tensor], scale: float):
        u = (ctypes.c_double * 3)(*[float(v) for v in uniform])
        self._call("clbm_set_force", u, _ptr(field), ctypes.c_double(float(scale)))

    def init(self, state, rho0=None, u0=None):
        self._call("clbm_init", self._state(state), _ptr(rho0), _ptr(u0))

    def step(self, src, dst):
        self._call("clbm_step", self._state(src), self._state(dst))

    def run(self, a, b, nsteps: int) -> bool:
        """Runs nsteps; returns True when the final state is in b."""
        res = ctypes.c_void_p()
        self._call("clbm_run", self._state(a), self._state(b), ctypes.c_int32(int(nsteps)), ctypes.byref(res))
        return res.value == b.data_ptr()

    def trajectory(self, src, states):
        """clbm_trajectory: states[k] gets the state after k + 1 steps from src."""
        arr = (ctypes.c_void_p * max(len(states), 1))(*[self._state(t) for t in states])
        self._call("clbm_trajectory", self._state(src), arr, ctypes.c_int32(len(states)))

    def set_options(self, options: int):
        self._call("clbm_set_options", ctypes.c_uint32(int(options)))

    def fused_pairs(self) -> bool:
        r = self.lib.clbm_fused_pairs(self._h)
        if r < 0:
            raise ClbmError("clbm_fused_pairs", r, self.lib.clbm_last_error(self._h).decode())
        return r == 1

    def copy(self, src, dst):
        self._call("clbm_copy", self._state(src), self._state(dst))

    def moments(self, state, rho=None, u=None, want_totals=True):
        totals = (ctypes.c_double * 4)() if want_totals else None
        nbad = ctypes.c_int64(0) if want_totals else None
        fn = self.lib.clbm_moments
        self.lib.clbm_set_stream(self._h, _stream(self.device))
        rc = fn(self._h, self._state(state), _ptr(rho), _ptr(u), totals, ctypes.byref(nbad) if want_totals else None)
        if rc and rc != 5:
            raise ClbmError("clbm_moments", rc, self.lib.clbm_last_error(self._h).decode())
        if not want_totals:
            return None, None
        return np.array(list(totals)), int(nbad.value)

    def get_populations(self, state, out):
        self._call("clbm_get_populations", self._state(state), _ptr(out))

    def set_populations(self, f, state):
        self._call("clbm_set_populations", _ptr(f), self._state(state))

    def sample_populations(self, state, nodes, out):
        self._call("clbm_sample_populations", self._state(state), _ptr(nodes), ctypes.c_int32(int(nodes.numel())),
                   _ptr(out))

    def _buf(self, t: Optional[torch.Tensor], name: str, dtype: torch.dtype, numel: int, optional: bool = False):
        """Pointer of an adjoint-side buffer after checking its dtype and element count (the library
        reads and writes exactly that many elements of that type)."""
        if t is None:
            if optional:
                return None
            raise ValueError(f"{name} is None")
        if t.dtype != dtype:
            raise ValueError(f"{name} has dtype {t.dtype}, {dtype} needed")
        if t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, {numel} needed")
        return _ptr(t)

    @property
    def adjoint_dtype(self) -> torch.dtype:
        """Type of lambda, dJ/dF and the loss target: FP64 for FP64 storage, FP32 otherwise."""
        return torch.float64 if self.desc.storage == CLBM_F64 else torch.float32

    def adjoint_step(self, state_t, lam_next, lam_out, dJdF=None, dJds=None):
        n, r = self.desc.nx * self.desc.ny * self.desc.nz, self.adjoint_dtype
        self._call("clbm_adjoint_step", self._state(state_t), self._buf(lam_next, "lam_next", r, 27 * n),
                   self._buf(lam_out, "lam_out", r, 27 * n), self._buf(dJdF, "dJdF", r, 3 * n, True),
                   self._buf(dJds, "dJds", torch.float64, 10, True))

    def adjoint_step_noalloc(self, state_t, lam_next, lam_out, dJdF=None, dJds=None):
        """clbm_adjoint_step_noalloc: clbm_adjoint_step without any allocation (lattices <= 2^25 nodes)."""
        n, r = self.desc.nx * self.desc.ny * self.desc.nz, self.adjoint_dtype
        self._call("clbm_adjoint_step_noalloc", self._state(state_t), self._buf(lam_next, "lam_next", r, 27 * n),
                   self._buf(lam_out, "lam_out", r, 27 * n), self._buf(dJdF, "dJdF", r, 3 * n, True),
                   self._buf(dJds, "dJds", torch.float64, 10, True))

    def loss_seed(self, state, u_target, lam_out, dJdF=None, J=None):
        n, r = self.desc.nx * self.desc.ny * self.desc.nz, self.adjoint_dtype
        self._call("clbm_loss_seed", self._state(state), self._buf(u_target, "u_target", r, 3 * n),
                   self._buf(lam_out, "lam_out", r, 27 * n), self._buf(dJdF, "dJdF", r, 3 * n, True),
                   self._buf(J, "J", torch.float64, 1, True))


def wall_velocity_array(wall_velocity) -> np.ndarray:
    """Face velocities as a (6, 3) array, face 2 * axis + side (side 1 beyond n - 1); accepts
    None, a {(axis, side): (ux, uy, uz)} dict or anything shaped (6, 3)."""
    w = np.zeros((6, 3))
    if wall_velocity is None:
        return w
    if isinstance(wall_velocity, dict):
        for (a, sd), v in wall_velocity.items():
            w[2 * int(a) + int(sd)] = v
        return w
    return np.asarray(wall_velocity, dtype=np.float64).reshape(6, 3).copy()


def default_plane_stride(dims, storage) -> int:
    """clbm_default_plane_stride: N rounded up to 256 B plus 4 KiB, in elements."""
    nx, ny, nz = (int(v) for v in dims)
    P = load_library().clbm_default_plane_stride(nx, ny, nz, STORAGE[storage])
    if P < 0:
        raise ValueError("invalid lattice dims or storage")
    return int(P)


def make_desc(dims, walls=(0, 0, 0), storage="f32", rates=None, force=(0.0, 0.0, 0.0), force_field=None,
              force_scale=1.0, solid=None, lattice="d3q27", collision="cascaded", wall_velocity=None,
              plane_stride=0) -> Desc:
    d = Desc()
    d.plane_stride = int(plane_stride)
    d.collision = COLLISION[collision]
    d.reserved = 0
    for k, v in enumerate(wall_velocity_array(wall_velocity).reshape(18)):
        d.wall_velocity[k] = float(v)
    d.nx, d.ny, d.nz = (int(v) for v in dims)
    for a in range(3):
        d.wall[a] = int(walls[a])
    d.storage = STORAGE[storage]
    d.lattice = LATTICE[lattice]
    rates = [1.0] * 10 if rates is None else [float(v) for v in rates]
    for k in range(10):
        d.s[k] = rates[k]
    for a in range(3):
        d.force_uniform[a] = float(force[a])
    d.force_scale = float(force_scale)
    d.force = None if force_field is None else force_field.data_ptr()
    d.solid = None if solid is None else solid.data_ptr()
    return d


def _dev_tensor(a, dtype, device, shape=None) -> Optional[torch.Tensor]:
    if a is None:
        return None
    t = torch.as_tensor(np.asarray(a) if not isinstance(a, torch.Tensor) else a)
    t = t.to(device=device, dtype=dtype).contiguous()
    if shape is not None:
        t = t.reshape(shape)
    return t


class Lattice:
    """A cascaded-LBM lattice on one GPU: two state buffers and a context.

    dims = (nx, ny, nz); walls per axis (0 periodic, 1 half-way bounce-back);
    storage in {"f64", "f32", "f16", "bf16"}; rates = the 10 rates of Eq. (13);
    force = uniform force density; force_field = (3, nz, ny, nx) field added to
    it (times force_scale); solid = (nz, ny, nx) mask, nonzero = solid;
    lattice = "d3q27" (Eq. (1)) or "d3q19" (Appendix A); collision = "cascaded"
    (Sec. II) or "mrt" (the raw-moment MRT of Appendix B, D3Q27); wall_velocity =
    moving wall faces, {(axis, side): (ux, uy, uz)} (side 1 beyond n - 1);
    plane_stride = plane stride P of the state buffers (None: the library's
    default, N plus a little padding; 0: P = N).

    State buffers are contiguous (Q, P) tensors whose padding is zero; view()
    gives the (Q, nz, ny, nx) part that holds the lattice.
    """

    def __init__(self, dims: Sequence[int], walls=(0, 0, 0), storage="f32", rates=None, force=(0.0, 0.0, 0.0),
                 force_field=None, force_scale=1.0, solid=None, device=None, lattice="d3q27", collision="cascaded",
                 wall_velocity=None, plane_stride=None):
        if not torch.cuda.is_available():
            raise RuntimeError("clbm needs a GPU (HIP); none is visible")
        self.device = torch.device(device if device is not None else "cuda")
        self.dims = tuple(int(v) for v in dims)
        nx, ny, nz = self.dims
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self.walls = tuple(int(w) for w in walls)
        self.storage = storage
        self.lattice = lattice
        self.collision = collision
        self.wall_velocity = wall_velocity_array(wall_velocity)
        self.q = LATTICE_Q[lattice]
        self.real = REAL_TORCH[storage]
        self.force_field = _dev_tensor(force_field, self.real, self.device, (3,) + self.shape)
        self.solid = _dev_tensor(solid, torch.uint8, self.device, self.shape)
        self.rates = np.array([1.0] * 10 if rates is None else rates, dtype=np.float64)
        self.force = tuple(float(v) for v in force)
        self.force_scale = float(force_scale)
        if plane_stride is None:
            plane_stride = default_plane_stride(self.dims, storage)
        self.P = int(plane_stride) if plane_stride else self.n
        desc = make_desc(self.dims, self.walls, storage, self.rates, self.force, self.force_field, force_scale,
                         self.solid, lattice, collision, self.wall_velocity, plane_stride)
        self.ctx = Context(desc, self.device)
        self.bufs = [self.new_state() for _ in range(2)]
        self.cur = 0
        self.t = 0

    # ---- state
    def new_state(self) -> torch.Tensor:
        """A zeroed state buffer (Q, P) of this lattice."""
        return torch.zeros((self.q, self.P), dtype=STORAGE_TORCH[self.storage], device=self.device)

    def view(self, t: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The (Q, nz, ny, nx) lattice part of a state buffer (default: the current state)."""
        t = self.state if t is None else t
        return t[:, : self.n].view((self.q,) + self.shape)

    @property
    def state(self) -> torch.Tensor:
        return self.bufs[self.cur]

    @property
    def other(self) -> torch.Tensor:
        return self.bufs[1 - self.cur]

    def init(self, rho0=None, u0=None):
        r = _dev_tensor(rho0, torch.float64, self.device, self.shape)
        u = _dev_tensor(u0, torch.float64, self.device, (3,) + self.shape)
        self.ctx.init(self.state, r, u)
        self.t = 0
        return self

    def step(self, n: int = 1):
        n = int(n)
        if n <= 0:
            return self
        if self.ctx.run(self.state, self.other, n):
            self.cur = 1 - self.cur
        self.t += n
        return self

    def set_fused_steps(self, enabled: Optional[bool]):
        """Fused two-step launches of clbm_run: None = chosen by lattice size (default),
        True = whenever the lattice allows them, False = never."""
        self.ctx.set_options(0 if enabled is None else (2 if enabled else 1))

    @property
    def uses_fused_pairs(self) -> bool:
        """Whether step(n) runs pairs of steps as one fused launch (asks clbm_fused_pairs)."""
        return self.ctx.fused_pairs()

    def set_rates(self, rates):
        self.rates = np.asarray(rates, dtype=np.float64)
        self.ctx.set_rates(self.rates)

    def set_force(self, force=(0.0, 0.0, 0.0), force_field=None, force_scale=1.0):
        self.force = tuple(float(v) for v in force)
        self.force_field = _dev_tensor(force_field, self.real, self.device, (3,) + self.shape)
        self.force_scale = float(force_scale)
        self.ctx.set_force(self.force, self.force_field, self.force_scale)

    def set_force_scale(self, scale: float):
        """Rescale the per-node force field (time-dependent forcing, F(t) at the collision of step t)."""
        self.force_scale = float(scale)
        self.ctx.set_force(self.force, self.force_field, self.force_scale)

    # ---- observables
    def moments(self, fields: bool = True):
        """Returns (rho (nz,ny,nx) f64, u (3,nz,ny,nx) f64, totals [mass, px, py, pz], n_bad)."""
        rho = torch.empty(self.shape, dtype=torch.float64, device=self.device) if fields else None
        u = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device) if fields else None
        totals, nbad = self.ctx.moments(self.state, rho, u, want_totals=True)
        return rho, u, totals, nbad

    def populations(self) -> torch.Tensor:
        """Pre-collision populations f(x, t) as f64 (Q, nz, ny, nx), Eq. (1) / (A1) order."""
        out = torch.empty((self.q,) + self.shape, dtype=torch.float64, device=self.device)
        self.ctx.get_populations(self.state, out)
        return out

    def set_populations(self, f):
        ft = _dev_tensor(f, torch.float64, self.device, (self.q,) + self.shape)
        self.ctx.set_populations(ft, self.state)

    def sample(self, xyz) -> np.ndarray:
        """Pre-collision populations (Q, k) f64 at the nodes xyz = [(x, y, z), ...]."""
        nx, ny, _ = self.dims
        ids = torch.tensor([x + nx * (y + ny * z) for x, y, z in xyz], dtype=torch.int32, device=self.device)
        out = torch.empty((self.q, len(xyz)), dtype=torch.float64, device=self.device)
        self.ctx.sample_populations(self.state, ids, out)
        return out.cpu().numpy()

    def close(self):
        self.ctx.close()
