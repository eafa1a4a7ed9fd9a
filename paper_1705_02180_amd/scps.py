"""Python binding of libscps (include/scps.h): argument marshalling only.

Every computation happens in the HIP library.  Device arrays are torch
tensors on the current GPU; the library queues its work on torch's current
stream.  Importing this module loads ``libscps.so`` and raises if it has not
been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
# SCPS_LIB: another build of the same sources (e.g. one with host-side sanitizers)
LIB_PATH = os.environ.get("SCPS_LIB") or os.path.join(_HERE, "libscps.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1705_02180_amd.build`")

CV_STRIDE = 8
CV_Z, CV_ZM, CV_EB, CV_S, CV_W, CV_SM, CV_WM, CV_T = range(8)   # CV_T: bias functional T[X]
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "SHAPE", -3: "OOM", -4: "HIP", -5: "STATE",
          -6: "NONFINITE", -7: "NO_SUCCESS"}


class ScpsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"scps {STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("integrator", C.c_int32), ("bias_mode", C.c_int32), ("exec_mode", C.c_int32),
        ("nb_excl", C.c_int32), ("min_seq_sep", C.c_int32), ("replica_base", C.c_int32),
        ("w_form", C.c_int32), ("reserved", C.c_int32),
        ("dt", C.c_double), ("gamma", C.c_double), ("kT", C.c_double),
        ("k_bond", C.c_double), ("r_bond", C.c_double),
        ("lj_eps", C.c_double), ("lj_sigma", C.c_double),
        ("dh_prefactor", C.c_double), ("dh_kappa", C.c_double),
        ("r0_contact", C.c_double), ("r_cut_contact", C.c_double), ("r_cut_nb", C.c_double),
        ("k_R", C.c_double), ("lam", C.c_double), ("k_s", C.c_double), ("k_w", C.c_double),
        ("seed", C.c_uint64),
    ]


class Topology(C.Structure):
    _fields_ = [
        ("n_systems", C.c_int32),
        ("n_particles", C.POINTER(C.c_int32)), ("n_contact", C.POINTER(C.c_int32)),
        ("contact_idx", C.POINTER(C.c_int32)),
        ("mass", C.POINTER(C.c_float)), ("charge", C.POINTER(C.c_float)),
    ]


_lib = C.CDLL(LIB_PATH)
_vp, _i32, _i64, _u64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
_lib.scps_init_system.restype = C.c_int
_lib.scps_init_system.argtypes = [C.POINTER(Params), C.POINTER(Topology), _i32, _vp, _vp, C.POINTER(_vp)]
_lib.scps_set_reference_map.restype = C.c_int
_lib.scps_set_reference_map.argtypes = [_vp, _i32, _i32, _vp, _vp, _d]
_lib.scps_step_replicas.restype = C.c_int
_lib.scps_step_replicas.argtypes = [_vp, _vp, _vp, _vp, _i64, _u64, _i32, _vp]
_lib.scps_eval_z_and_grad.restype = C.c_int
_lib.scps_eval_z_and_grad.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.scps_ratchet_energy.restype = C.c_int
_lib.scps_ratchet_energy.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.scps_update_reference_from_paths.restype = C.c_int
_lib.scps_update_reference_from_paths.argtypes = [_vp, _i32, _vp, _i32, _i32, _vp, _vp]
_lib.scps_set_stream.restype = C.c_int
_lib.scps_set_stream.argtypes = [_vp, _vp]
_lib.scps_sync.restype = C.c_int
_lib.scps_sync.argtypes = [_vp, _vp, _vp]
_lib.scps_autotune.restype = C.c_int
_lib.scps_autotune.argtypes = [_vp, _vp, _vp, _vp, _i64, _vp]
_lib.scps_set_launch.restype = C.c_int
_lib.scps_set_launch.argtypes = [_vp, _i32, _i32]
_lib.scps_get_launch.restype = C.c_int
_lib.scps_get_launch.argtypes = [_vp, _vp]
_lib.scps_set_graph_steps.restype = C.c_int
_lib.scps_set_graph_steps.argtypes = [_vp, _i32]
_lib.scps_least_biased_path.restype = C.c_int
_lib.scps_least_biased_path.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.scps_eval_tube.restype = C.c_int
_lib.scps_eval_tube.argtypes = [_vp, _i32, _vp, _vp, _vp]
_lib.scps_eval_sigma.restype = C.c_int
_lib.scps_eval_sigma.argtypes = [_vp, _i32, _vp, _vp, _vp]
_lib.scps_path_distance.restype = C.c_int
_lib.scps_path_distance.argtypes = [_vp, _i64, _vp, _i64, _d, _d, _d, _i32, _i32, _vp, C.POINTER(C.c_double)]
_lib.scps_time_passes.restype = C.c_int
_lib.scps_time_passes.argtypes = [_vp, _i32]
_lib.scps_pass_times.restype = C.c_int
_lib.scps_pass_times.argtypes = [_vp, _vp, _vp]
_lib.scps_path_distance_noalloc.restype = C.c_int
_lib.scps_path_distance_noalloc.argtypes = _lib.scps_path_distance.argtypes
_lib.scps_funnel_steps.restype = C.c_int
_lib.scps_funnel_steps.argtypes = [C.c_void_p, _i32, _i32, _vp, _vp, _i64, _u64, _i32, _vp, _i32, _vp, _vp]
_lib.scps_funnel_mean_path.restype = C.c_int
_lib.scps_funnel_mean_path.argtypes = [_i32, _i32, _vp, _vp, _vp, _vp]
_lib.scps_scale_by_replica.restype = C.c_int
_lib.scps_scale_by_replica.argtypes = [_vp, _vp, _vp, _vp]
_lib.scps_eval_zbias.restype = C.c_int
_lib.scps_eval_zbias.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
_lib.scps_zbias_backward.restype = C.c_int
_lib.scps_zbias_backward.argtypes = [_vp, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp]
_lib.scps_destroy.restype = None
_lib.scps_destroy.argtypes = [_vp]
_lib.scps_last_error.restype = C.c_char_p
_lib.scps_last_error.argtypes = []

EXPORTS = ["scps_init_system", "scps_set_reference_map", "scps_step_replicas", "scps_eval_z_and_grad",
           "scps_ratchet_energy", "scps_update_reference_from_paths", "scps_set_stream", "scps_sync",
           "scps_autotune", "scps_set_launch", "scps_get_launch", "scps_set_graph_steps", "scps_least_biased_path", "scps_eval_tube", "scps_eval_sigma", "scps_path_distance",
           "scps_path_distance_noalloc", "scps_time_passes", "scps_pass_times",
           "scps_funnel_steps", "scps_funnel_mean_path", "scps_scale_by_replica", "scps_eval_zbias",
           "scps_zbias_backward", "scps_destroy",
           "scps_last_error"]


def _check(status: int):
    if status != 0:
        raise ScpsError(status, _lib.scps_last_error().decode())


def _stream() -> C.c_void_p:
    if not torch.cuda.is_available():      # host-side argument checks only
        return C.c_void_p(None)
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: Optional[torch.Tensor], dtype, numel: Optional[int] = None, name: str = "tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _dev_vec(t: Optional[torch.Tensor], dtype, n: int, name: str):
    """(pointer, element stride) of a 1-D device tensor of n elements that may
    be strided or broadcast (stride 0, as the gradient of a sum arrives)."""
    if t is None:
        return None, 0
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 1 or t.shape[0] != n:
        raise ValueError(f"{name} must have shape [{n}], got {list(t.shape)}")
    stride = t.stride(0) if n > 1 else 0
    if stride < 0:
        raise ValueError(f"{name} must have a non-negative stride")
    return C.c_void_p(t.data_ptr()), stride


def make_params(d: dict, exec_mode: int = 0, replica_base: int = 0) -> Params:
    return Params(
        integrator=int(d["integrator"]), bias_mode=int(d["bias_mode"]), exec_mode=int(exec_mode),
        nb_excl=int(d["nb_excl"]), min_seq_sep=int(d["min_seq_sep"]), replica_base=int(replica_base),
        w_form=int(d.get("w_form", 0)), reserved=0,
        dt=d["dt"], gamma=d["gamma"], kT=d["kT"], k_bond=d["k_bond"], r_bond=d["r_bond"],
        lj_eps=d["lj_eps"], lj_sigma=d["lj_sigma"], dh_prefactor=d["dh_prefactor"],
        dh_kappa=d["dh_kappa"], r0_contact=d["r0_contact"], r_cut_contact=d["r_cut_contact"],
        r_cut_nb=d.get("r_cut_nb", 0.0), k_R=d["k_R"], lam=d["lam"], k_s=d["k_s"], k_w=d["k_w"], seed=int(d["seed"]))


class Context:
    """Owns one scps_ctx.  Methods mirror the C entry points."""

    def __init__(self, params: dict, n_particles: Sequence[int], contact_idx: Sequence[np.ndarray],
                 mass: Sequence[np.ndarray], charge: Sequence[np.ndarray], replica_system: Sequence[int],
                 exec_mode: int = 0, replica_base: int = 0):
        self.params = dict(params)
        self.n = np.ascontiguousarray(n_particles, dtype=np.int32)
        self.nc = np.ascontiguousarray([len(c) for c in contact_idx], dtype=np.int32)
        self._cidx = np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.int32) for c in contact_idx])
                                          if len(contact_idx) else np.zeros(0, np.int32))
        self._mass = np.ascontiguousarray(np.concatenate([np.asarray(m, dtype=np.float32) for m in mass]))
        self._charge = np.ascontiguousarray(np.concatenate([np.asarray(q, dtype=np.float32) for q in charge]))
        self.replica_system = np.ascontiguousarray(replica_system, dtype=np.int32)
        self.R = len(self.replica_system)
        self._p = make_params(self.params, exec_mode, replica_base)
        topo = Topology(
            n_systems=len(self.n),
            n_particles=self.n.ctypes.data_as(C.POINTER(C.c_int32)),
            n_contact=self.nc.ctypes.data_as(C.POINTER(C.c_int32)),
            contact_idx=self._cidx.ctypes.data_as(C.POINTER(C.c_int32)),
            mass=self._mass.ctypes.data_as(C.POINTER(C.c_float)),
            charge=self._charge.ctypes.data_as(C.POINTER(C.c_float)))
        h = C.c_void_p()
        _check(_lib.scps_init_system(C.byref(self._p), C.byref(topo), self.R,
                                     self.replica_system.ctypes.data_as(C.c_void_p), _stream(), C.byref(h)))
        self._h = h
        sizes = self.n[self.replica_system].astype(np.int64)
        self.offsets = np.zeros(self.R + 1, dtype=np.int64)
        self.offsets[1:] = np.cumsum(sizes)
        self.sumN = int(self.offsets[-1])

    @classmethod
    def from_workload(cls, w, exec_mode: int = 0, params: Optional[dict] = None, replica_system=None,
                      replica_base: int = 0):
        rs = w.replica_system if replica_system is None else replica_system
        return cls(params or w.params, [s.n for s in w.systems], [s.contact_idx for s in w.systems],
                   [s.mass for s in w.systems], [s.charge for s in w.systems], rs, exec_mode, replica_base)

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.scps_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ctx(self):
        if not self._h:
            raise ScpsError(-5, "context is closed")
        _check(_lib.scps_set_stream(self._h, _stream()))
        return self._h

    def n_pairs(self, system: int) -> int:
        nc = int(self.nc[system])
        return nc * (nc - 1) // 2

    # -- entry points -----------------------------------------------------------
    def set_reference_map(self, system: int, maps: Optional[np.ndarray] = None,
                          native_xyz: Optional[np.ndarray] = None, z0_norm: float = 0.0):
        if maps is not None:
            maps = np.ascontiguousarray(maps, dtype=np.float64)
            n_maps = 1 if maps.ndim == 1 else maps.shape[0]
            if maps.size != n_maps * self.n_pairs(system):
                raise ValueError("maps must hold n_maps x P packed entries")
        else:
            n_maps = 1
        if native_xyz is not None:
            native_xyz = np.ascontiguousarray(native_xyz, dtype=np.float64)
            if native_xyz.size != 3 * int(self.n[system]):
                raise ValueError("native_xyz must be [3][N]")
        _check(_lib.scps_set_reference_map(
            self._ctx(), int(system), int(n_maps),
            None if maps is None else maps.ctypes.data_as(C.c_void_p),
            None if native_xyz is None else native_xyz.ctypes.data_as(C.c_void_p), float(z0_norm)))

    def step_replicas(self, x: torch.Tensor, v: Optional[torch.Tensor], cvstate: torch.Tensor,
                      n_steps: int, step0: int = 0, record_every: int = 0,
                      frames: Optional[torch.Tensor] = None):
        n3 = 3 * self.sumN
        px = _dev(x, torch.float32, n3, "x")
        pv = _dev(v, torch.float32, n3, "v")
        pc = _dev(cvstate, torch.float64, self.R * CV_STRIDE, "cvstate")
        pf = None
        if record_every > 0:
            pf = _dev(frames, torch.float32, (n_steps // record_every + 1) * n3, "frames")
        _check(_lib.scps_step_replicas(self._ctx(), px, pv, pc, int(n_steps), int(step0),
                                       int(record_every), pf))

    def eval_z_and_grad(self, x: torch.Tensor, z: torch.Tensor, grad: Optional[torch.Tensor] = None,
                        grad_coef: Optional[torch.Tensor] = None):
        n3 = 3 * self.sumN
        _check(_lib.scps_eval_z_and_grad(self._ctx(), _dev(x, torch.float32, n3, "x"),
                                         _dev(z, torch.float64, self.R, "z"),
                                         _dev(grad, torch.float32, n3, "grad"),
                                         _dev(grad_coef, torch.float64, self.R, "grad_coef")))

    def ratchet_energy(self, z: torch.Tensor, z_m: torch.Tensor, E_b: Optional[torch.Tensor] = None,
                       gz: Optional[torch.Tensor] = None, gE: Optional[torch.Tensor] = None,
                       coef: Optional[torch.Tensor] = None):
        R = self.R
        _check(_lib.scps_ratchet_energy(self._ctx(), _dev(z, torch.float64, R, "z"),
                                        _dev(z_m, torch.float64, R, "z_m"), _dev(E_b, torch.float64, R, "E_b"),
                                        _dev(gz, torch.float64, R, "gz"), _dev(gE, torch.float64, R, "gE"),
                                        _dev(coef, torch.float64, R, "coef")))

    def update_reference_from_paths(self, system: int, frames: torch.Tensor, n_paths: int, n_frames: int,
                                    success: Sequence[int], want_maps: bool = False):
        n = int(self.n[system])
        pf = _dev(frames, torch.float32, n_frames * n_paths * 3 * n, "frames")
        succ = np.ascontiguousarray(np.asarray(success, dtype=np.uint8))
        if succ.size != n_paths:
            raise ValueError("success must have n_paths entries")
        out = np.zeros((n_frames, self.n_pairs(system))) if want_maps else None
        _check(_lib.scps_update_reference_from_paths(
            self._ctx(), int(system), pf, int(n_paths), int(n_frames), succ.ctypes.data_as(C.c_void_p),
            None if out is None else out.ctypes.data_as(C.c_void_p)))
        return out

    def scale_by_replica(self, inp: torch.Tensor, coef: torch.Tensor, out: torch.Tensor):
        n3 = 3 * self.sumN
        _check(_lib.scps_scale_by_replica(self._ctx(), _dev(inp, torch.float32, n3, "in"),
                                          _dev(coef, torch.float64, self.R, "coef"),
                                          _dev(out, torch.float32, n3, "out")))

    def eval_zbias(self, x: torch.Tensor, z_m: torch.Tensor, z: torch.Tensor, E_b: torch.Tensor,
                   grad_z: Optional[torch.Tensor] = None):
        n3, R = 3 * self.sumN, self.R
        _check(_lib.scps_eval_zbias(self._ctx(), _dev(x, torch.float32, n3, "x"), _dev(z_m, torch.float64, R, "z_m"),
                                    _dev(z, torch.float64, R, "z"), _dev(E_b, torch.float64, R, "E_b"),
                                    _dev(grad_z, torch.float32, n3, "grad_z")))

    def zbias_backward(self, z: torch.Tensor, z_m: torch.Tensor, g_z: Optional[torch.Tensor],
                       g_E: Optional[torch.Tensor], grad_z: torch.Tensor, grad_x: torch.Tensor):
        n3, R = 3 * self.sumN, self.R
        pz, sz = _dev_vec(g_z, torch.float64, R, "g_z")
        pe, se = _dev_vec(g_E, torch.float64, R, "g_E")
        _check(_lib.scps_zbias_backward(self._ctx(), _dev(z, torch.float64, R, "z"),
                                        _dev(z_m, torch.float64, R, "z_m"), pz, int(sz), pe, int(se),
                                        _dev(grad_z, torch.float32, n3, "grad_z"),
                                        _dev(grad_x, torch.float32, n3, "grad_x")))

    def autotune(self, x: torch.Tensor, v: Optional[torch.Tensor], cvstate: torch.Tensor, n_steps: int):
        """Time the launch configurations on copies of the state and keep the
        fastest; returns (path, param): path 0 persistent, 1 per-step, 2
        packed, and the persistent kernel's threads per replica or the packed
        kernel's replicas per workgroup (an SCPS context: 1 when its
        nonbonded pass overlaps the distance pass, else 0)."""
        px = _dev(x, torch.float32, 3 * self.sumN, "x")
        pv = _dev(v, torch.float32, 3 * self.sumN, "v")
        pc = _dev(cvstate, torch.float64, self.R * CV_STRIDE, "cvstate")
        out = np.zeros(2, dtype=np.int32)
        _check(_lib.scps_autotune(self._ctx(), px, pv, pc, int(n_steps), out.ctypes.data_as(C.c_void_p)))
        return int(out[0]), int(out[1])

    def set_launch(self, path: int, param: int = 0):
        """Fix the launch configuration: path 0 persistent (param = threads
        per workgroup), 1 per-step, 2 packed (param = wavefronts per
        workgroup)."""
        _check(_lib.scps_set_launch(self._ctx(), int(path), int(param)))

    def set_graph_steps(self, steps: int):
        """Steps per captured HIP graph on the per-step path (0: none)."""
        _check(_lib.scps_set_graph_steps(self._ctx(), int(steps)))

    def get_launch(self):
        """The launch the next step_replicas takes, as (path, parameter) in
        autotune's encoding."""
        out = np.zeros(2, dtype=np.int32)
        _check(_lib.scps_get_launch(self._ctx(), out.ctypes.data_as(C.c_void_p)))
        return int(out[0]), int(out[1])

    def eval_tube(self, stack_system: int, x: torch.Tensor, s: Optional[torch.Tensor] = None,
                  w: Optional[torch.Tensor] = None):
        """s_lambda, w_lambda of every replica against system stack_system's frame stack."""
        _check(_lib.scps_eval_tube(self._ctx(), int(stack_system), _dev(x, torch.float32, 3 * self.sumN, "x"),
                                   _dev(s, torch.float64, self.R, "s"), _dev(w, torch.float64, self.R, "w")))

    def eval_sigma(self, stack_systems: Sequence[int], x: torch.Tensor, sigma: torch.Tensor):
        """sigma(X) = mean over the stacks of 1 - s_lambda^k(X)."""
        st = np.ascontiguousarray(np.asarray(stack_systems, dtype=np.int32))
        _check(_lib.scps_eval_sigma(self._ctx(), int(st.size), st.ctypes.data_as(C.c_void_p),
                                    _dev(x, torch.float32, 3 * self.sumN, "x"),
                                    _dev(sigma, torch.float64, self.R, "sigma")))

    def least_biased_path(self, cvstate: torch.Tensor, success: Optional[Sequence[int]] = None):
        """(replica id, T) of the candidate with the smallest bias functional
        T (cvstate[:, CV_T]); success selects the candidates (None = all)."""
        pc = _dev(cvstate, torch.float64, self.R * CV_STRIDE, "cvstate")
        ps = None
        if success is not None:
            succ = np.ascontiguousarray(np.asarray(success, dtype=np.uint8))
            if succ.size != self.R:
                raise ValueError("success must have one entry per replica")
            ps = succ.ctypes.data_as(C.c_void_p)
        idx = C.c_int32(-1)
        t = C.c_double(0.0)
        _check(_lib.scps_least_biased_path(self._ctx(), pc, ps, C.byref(idx), C.byref(t)))
        return int(idx.value), float(t.value)

    def time_passes(self, enable=True):
        """Start (or stop: False / 0) recording HIP events around the SCPS
        step's distance and bias passes; True or 1 times every step, an int
        k >= 1 every k-th."""
        _check(_lib.scps_time_passes(self._ctx(), int(enable)))

    def pass_times(self):
        """({"distance": ms, "bias": ms} summed, steps timed) since time_passes."""
        ms = (C.c_double * 2)()
        n = (C.c_int64 * 2)()
        _check(_lib.scps_pass_times(self._ctx(), ms, n))
        return {"distance": float(ms[0]), "bias": float(ms[1])}, int(n[0])

    def sync(self):
        bad = np.zeros(self.R, dtype=np.int32)
        nb = C.c_int32(0)
        st = _lib.scps_sync(self._h, bad.ctypes.data_as(C.c_void_p), C.byref(nb))
        if st == -6:
            raise ScpsError(st, f"{_lib.scps_last_error().decode()}: replicas {bad[:nb.value].tolist()}")
        _check(st)


# module-level names matching the C entry points
def init_system(params: dict, n_particles, contact_idx, mass, charge, replica_system, exec_mode: int = 0):
    return Context(params, n_particles, contact_idx, mass, charge, replica_system, exec_mode)


def set_reference_map(ctx: Context, system: int, maps=None, native_xyz=None, z0_norm: float = 0.0):
    return ctx.set_reference_map(system, maps, native_xyz, z0_norm)


def autotune(ctx: Context, x, v, cvstate, n_steps):
    return ctx.autotune(x, v, cvstate, n_steps)


def step_replicas(ctx: Context, x, v, cvstate, n_steps, step0=0, record_every=0, frames=None):
    return ctx.step_replicas(x, v, cvstate, n_steps, step0, record_every, frames)


def eval_z_and_grad(ctx: Context, x, z, grad=None, grad_coef=None):
    return ctx.eval_z_and_grad(x, z, grad, grad_coef)


def update_reference_from_paths(ctx: Context, system, frames, n_paths, n_frames, success, want_maps=False):
    return ctx.update_reference_from_paths(system, frames, n_paths, n_frames, success, want_maps)


def eval_zbias(ctx: Context, x, z_m, z, E_b, grad_z=None):
    return ctx.eval_zbias(x, z_m, z, E_b, grad_z)


def zbias_backward(ctx: Context, z, z_m, g_z, g_E, grad_z, grad_x):
    return ctx.zbias_backward(z, z_m, g_z, g_E, grad_z, grad_x)


class ZBias(torch.autograd.Function):
    """z(X) and the rMD bias energy E_b = 1/2 k_R (z - z_m)^2 theta(z - z_m) as a
    differentiable function of the coordinates.  When x needs a gradient,
    forward runs the z + dz/dx pair pass once and keeps dz/dx (O(N) per
    replica; no map of the current contacts is stored); backward scales it by
    g_z + g_E k_R (z - z_m) theta per replica.  Otherwise forward evaluates z
    alone.  Forward and backward are one library call each (scps_eval_zbias,
    scps_zbias_backward): three launches in all beside the pair pass."""

    @staticmethod
    def forward(ctx_, x: torch.Tensor, z_m: torch.Tensor, lib_ctx: Context):
        z = torch.empty(lib_ctx.R, dtype=torch.float64, device=x.device)
        Eb = torch.empty_like(z)
        dz = torch.empty_like(x) if ctx_.needs_input_grad[0] else None
        lib_ctx.eval_zbias(x, z_m, z, Eb, dz)
        ctx_.save_for_backward(z, z_m, dz)
        ctx_.lib_ctx = lib_ctx
        return z, Eb

    @staticmethod
    def backward(ctx_, gz: torch.Tensor, gE: torch.Tensor):
        # gz, gE arrive broadcast (stride 0) from a sum: the library reads them strided
        z, z_m, dz = ctx_.saved_tensors
        gz = None if gz is None else gz.to(torch.float64)
        gE = None if gE is None else gE.to(torch.float64)
        grad = torch.empty_like(dz)
        ctx_.lib_ctx.zbias_backward(z, z_m, gz, gE, dz, grad)
        return grad, None, None


def zbias(x: torch.Tensor, z_m: torch.Tensor, lib_ctx: Context):
    return ZBias.apply(x, z_m, lib_ctx)


def path_distance(xy_a: torch.Tensor, xy_b: torch.Tensor, x0: float, y0: float, cell: float, nx: int,
                  ny: int) -> float:
    """Frobenius distance between the unit-norm binary occupancy matrices of
    two sets of 2-D projections (device float32 [n][2]) on an nx x ny grid."""
    for t, name in ((xy_a, "xy_a"), (xy_b, "xy_b")):
        if t.dim() != 2 or t.shape[1] != 2:
            raise ValueError(f"{name} must have shape [n, 2]")
    D = C.c_double(0.0)
    _check(_lib.scps_path_distance(_dev(xy_a, torch.float32, None, "xy_a"), int(xy_a.shape[0]),
                                   _dev(xy_b, torch.float32, None, "xy_b"), int(xy_b.shape[0]), float(x0), float(y0),
                                   float(cell), int(nx), int(ny), _stream(), C.byref(D)))
    return float(D.value)


def path_distance_noalloc(xy_a: torch.Tensor, xy_b: torch.Tensor, x0: float, y0: float, cell: float, nx: int,
                          ny: int) -> float:
    """path_distance without device allocation (grids of at most 2^20 cells,
    scratch in a fixed device array per GPU; overlapping calls on one GPU race)."""
    for t, name in ((xy_a, "xy_a"), (xy_b, "xy_b")):
        if t.dim() != 2 or t.shape[1] != 2:
            raise ValueError(f"{name} must have shape [n, 2]")
    D = C.c_double(0.0)
    _check(_lib.scps_path_distance_noalloc(_dev(xy_a, torch.float32, None, "xy_a"), int(xy_a.shape[0]),
                                           _dev(xy_b, torch.float32, None, "xy_b"), int(xy_b.shape[0]), float(x0),
                                           float(y0), float(cell), int(nx), int(ny), _stream(), C.byref(D)))
    return float(D.value)


class FunnelParams(C.Structure):
    _fields_ = [
        ("A1", C.c_double), ("A2", C.c_double), ("A3", C.c_double),
        ("s1", C.c_double), ("s2", C.c_double), ("s3", C.c_double),
        ("w", C.c_double), ("xm", C.c_double), ("ym", C.c_double),
        ("kT", C.c_double), ("mobility_dt", C.c_double),
        ("bias_mode", C.c_int32), ("w_form", C.c_int32),
        ("k_R", C.c_double), ("lam", C.c_double), ("k_s", C.c_double), ("k_w", C.c_double),
        ("seed", C.c_uint64),
    ]


def funnel_steps(params: dict, xy: torch.Tensor, cvstate: torch.Tensor, n_steps: int, step0: int = 0,
                 record_every: int = 0, frames: Optional[torch.Tensor] = None,
                 mean_path: Optional[torch.Tensor] = None, first_id: int = 0):
    """Toy model: advance the trajectories xy [n][2] (float64) in place."""
    n = int(xy.shape[0])
    fp = FunnelParams(A1=params["A1"], A2=params["A2"], A3=params["A3"], s1=params["s1"], s2=params["s2"],
                      s3=params["s3"], w=params["w"], xm=params["xm"], ym=params["ym"], kT=params["kT"],
                      mobility_dt=params["mob_dt"], bias_mode=int(params["bias_mode"]),
                      w_form=int(params.get("w_form", 0)), k_R=params["k_R"], lam=params["lam"], k_s=params["k_s"], k_w=params["k_w"],
                      seed=int(params["seed"]))
    K = 0 if mean_path is None else int(mean_path.shape[0])
    pf = None
    if record_every > 0:
        pf = _dev(frames, torch.float64, (n_steps // record_every + 1) * n * 2, "frames")
    _check(_lib.scps_funnel_steps(C.byref(fp), n, int(first_id), _dev(xy, torch.float64, 2 * n, "xy"),
                                  _dev(cvstate, torch.float64, n * CV_STRIDE, "cvstate"), int(n_steps), int(step0),
                                  int(record_every), pf, K,
                                  None if mean_path is None else _dev(mean_path, torch.float64, 2 * K, "mean_path"),
                                  _stream()))


def funnel_mean_path(frames: torch.Tensor, success: Sequence[int]) -> torch.Tensor:
    """Mean over the successful trajectories of every frame of frames [F][n][2]."""
    n_frames, n = int(frames.shape[0]), int(frames.shape[1])
    succ = np.ascontiguousarray(np.asarray(success, dtype=np.uint8))
    if succ.size != n:
        raise ValueError("success must have one entry per trajectory")
    out = torch.empty((n_frames, 2), dtype=torch.float64, device=frames.device)
    _check(_lib.scps_funnel_mean_path(n, n_frames, _dev(frames, torch.float64, n_frames * n * 2, "frames"),
                                      succ.ctypes.data_as(C.c_void_p), _dev(out, torch.float64, 2 * n_frames, "out"),
                                      _stream()))
    return out
