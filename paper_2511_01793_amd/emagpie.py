"""Python binding of libemagpie (ctypes; argument marshalling only).

Every step of the reconstruction runs in the HIP kernels of libemagpie.so.
PyTorch supplies device memory (tensors) and the current HIP stream.  If the
built library is missing this module raises at import of `lib()`; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libemagpie.so")

PATHS = {"plain": 0, "fused": 1, "graph": 2, "persistent": 3, "auto": 4, "chain": 5}
PATH_NAMES = {v: k for k, v in PATHS.items()}
TUNE = -1  # fft_plan / finalize_shape: choose by timing at init
F32, F64 = 0, 1

STATUS = {
    0: "OK", -1: "E_ARG", -2: "E_SHAPE", -3: "E_POSITION", -4: "E_DATA",
    -5: "E_DEGENERATE", -6: "E_WORKSPACE", -7: "E_HIP", -8: "E_UNSUPPORTED",
}

EXPORTS = [
    "emagpie_workspace_size", "emagpie_init", "emagpie_destroy", "emagpie_dp_avg",
    "emagpie_normalize_probe", "emagpie_step_minibatch", "emagpie_epoch", "emagpie_mg_cycle",
    "emagpie_misfit", "emagpie_grad", "emagpie_permutation", "emagpie_last_error",
    "emagpie_version", "emagpie_profile_enable", "emagpie_profile_read",
    "emagpie_group_workspace_size", "emagpie_group_create", "emagpie_group_epoch",
    "emagpie_group_destroy", "emagpie_plan_get", "emagpie_plan_describe", "emagpie_check_step",
    "emagpie_phase_memory_reset", "emagpie_workspace_size_many", "emagpie_init_many",
    "emagpie_epoch_many", "emagpie_many_member", "emagpie_debug_barrier", "emagpie_measure_peaks",
    "emagpie_misfit_noalloc",
]


class EmagpieError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Config(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32), ("m", ctypes.c_int32),
        ("n_pos", ctypes.c_int32),
        ("minibatch", ctypes.c_int32), ("levels", ctypes.c_int32),
        ("alpha", ctypes.c_float), ("alpha_z", ctypes.c_float),
        ("update_probe", ctypes.c_int32), ("joint_step", ctypes.c_int32), ("path", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("fft_plan", ctypes.c_int32), ("finalize_shape", ctypes.c_int32),
        ("tune_cache", ctypes.c_char_p), ("zero_phase_memory", ctypes.c_int32),
    ]


class Plan(ctypes.Structure):
    _fields_ = [
        ("fft_plan", ctypes.c_int32), ("r1", ctypes.c_int32), ("r2", ctypes.c_int32),
        ("threads", ctypes.c_int32), ("finalize_shape", ctypes.c_int32),
        ("fin_threads", ctypes.c_int32), ("fin_tile", ctypes.c_int32), ("fin_order", ctypes.c_int32),
        ("path", ctypes.c_int32), ("tuned", ctypes.c_int32), ("n_fft_plans", ctypes.c_int32),
        ("fft_us", ctypes.c_float * 4), ("n_fin_shapes", ctypes.c_int32), ("fin_us", ctypes.c_float * 12),
        ("path_ms", ctypes.c_float * 8),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if not k.endswith(("_us", "_ms"))}
        d["fft_us"] = list(self.fft_us)[:self.n_fft_plans]
        d["fin_us"] = list(self.fin_us)[:self.n_fin_shapes]
        d["path_ms"] = {PATH_NAMES[i]: t for i, t in enumerate(self.path_ms) if t >= 0}
        d["path"] = PATH_NAMES.get(self.path, self.path)
        d["tuned"] = {0: "fixed", 1: "timed", 2: "cache"}.get(self.tuned, self.tuned)
        return d


_lib = None


def lib() -> ctypes.CDLL:
    """Load libemagpie.so (built by `__graft_entry__.build()`); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sz = ctypes.c_size_t
    cfgp = ctypes.POINTER(Config)
    sig = {
        "emagpie_workspace_size": [cfgp, ctypes.POINTER(sz)],
        "emagpie_init": [ctypes.POINTER(vp), cfgp, vp, vp, vp, sz, vp],
        "emagpie_destroy": [vp],
        "emagpie_dp_avg": [vp, ctypes.POINTER(ctypes.c_double)],
        "emagpie_normalize_probe": [vp, vp, vp],
        "emagpie_step_minibatch": [vp, vp, vp, vp, i32, vp, vp],
        "emagpie_epoch": [vp, vp, vp, i64, vp, vp, vp],
        "emagpie_mg_cycle": [vp, vp, vp, vp, i32, vp, vp],
        "emagpie_misfit": [vp, vp, vp, vp, vp],
        "emagpie_grad": [vp, vp, vp, vp, vp, vp, i32, vp],
        "emagpie_permutation": [u64, i64, i32, vp],
        "emagpie_profile_enable": [vp, i32],
        "emagpie_profile_read": [vp, vp, vp],
        "emagpie_group_workspace_size": [i32, vp, ctypes.POINTER(sz)],
        "emagpie_group_create": [ctypes.POINTER(vp), i32, vp, vp, sz, vp],
        "emagpie_group_epoch": [vp, vp, vp, i64, vp, vp],
        "emagpie_group_destroy": [vp],
        "emagpie_plan_get": [vp, ctypes.POINTER(Plan)],
        "emagpie_check_step": [vp, vp, vp, vp, i32, vp, vp],
        "emagpie_phase_memory_reset": [vp, vp],
        "emagpie_plan_describe": [i32, i32, i32, ctypes.POINTER(Plan), ctypes.POINTER(i32)],
        "emagpie_workspace_size_many": [i32, vp, ctypes.POINTER(sz)],
        "emagpie_init_many": [ctypes.POINTER(vp), i32, vp, vp, vp, vp, sz, vp],
        "emagpie_epoch_many": [vp, vp, vp, i64, vp, vp],
        "emagpie_many_member": [vp, i32, ctypes.POINTER(vp)],
        "emagpie_debug_barrier": [vp, ctypes.c_uint32, ctypes.c_uint32],
        "emagpie_measure_peaks": [vp, sz, i32, vp, vp],
        "emagpie_misfit_noalloc": [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.emagpie_last_error.restype = ctypes.c_char_p
    L.emagpie_last_error.argtypes = [vp]
    L.emagpie_version.restype = ctypes.c_char_p
    L.emagpie_version.argtypes = []
    _lib = L
    return L


def _check(st: int, ctx=None):
    """Raise on a failed call; the message is ctx's last failure (or the thread's)."""
    if st != 0:
        raise EmagpieError(st, last_error(ctx))


def last_error(ctx=None) -> str:
    """Message of the last failure of a call on ctx (a ctypes handle), or on this thread."""
    h = None if ctx is None else (ctx.value if isinstance(ctx, ctypes.c_void_p) else ctx)
    return lib().emagpie_last_error(h).decode()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def workspace_size(cfg: Config) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().emagpie_workspace_size(ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def permutation(seed: int, epoch: int, n: int) -> np.ndarray:
    """The library's scan order for (seed, epoch) (host computation)."""
    out = np.empty(n, dtype=np.int32)
    _check(lib().emagpie_permutation(seed, epoch, n, out.ctypes.data))
    return out


def plan_describe(m: int, fft_plan: int = 0, finalize_shape: int = 0) -> dict:
    """Shape of FFT plan `fft_plan` and finalize shape `finalize_shape` for probe side m (host)."""
    p, cnt = Plan(), ctypes.c_int32(0)
    _check(lib().emagpie_plan_describe(m, fft_plan, finalize_shape, ctypes.byref(p), ctypes.byref(cnt)))
    d = {k: getattr(p, k) for k in ("fft_plan", "r1", "r2", "threads", "finalize_shape",
                                    "fin_threads", "fin_tile", "fin_order")}
    d["fft_plans"] = cnt.value
    return d


def _expect(t: torch.Tensor, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or tuple(t.shape) != tuple(shape) \
            or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape {tuple(shape)}")


class Reconstruction:
    """One reconstruction problem bound to a libemagpie context.

    positions: (N, 2) int (row, col) top-left corners; intensities: (N, m, m) float32 CUDA
    tensor (unshifted); n: the object side, or its (rows, cols).  The object (rows x cols)
    and probe (m x m) are complex64 CUDA tensors owned by the caller and updated in place.
    """

    def __init__(self, positions, intensities: torch.Tensor, n, *, minibatch: int,
                 levels: int = 1, alpha: float = 0.05, alpha_z: float = 1.0,
                 update_probe: bool = True, joint_step: bool = True, path: str = "graph",
                 seed: int = 0, fft_plan: int = 0, finalize_shape: int = 0,
                 tune_cache: str | None = None, zero_phase_memory: bool = False):
        pos = np.ascontiguousarray(np.asarray(positions, dtype=np.int32).reshape(-1, 2))
        if intensities.dim() != 3 or intensities.dtype != torch.float32 or not intensities.is_cuda:
            raise ValueError("intensities must be a (N, m, m) float32 CUDA tensor")
        intensities = intensities.contiguous()
        N, m, m2 = intensities.shape
        if m != m2 or N != pos.shape[0]:
            raise ValueError("intensities must be (N, m, m) with N = len(positions)")
        rows, cols = (int(n), int(n)) if np.ndim(n) == 0 else (int(n[0]), int(n[1]))
        self.shape = (rows, cols)
        self.n = rows if rows == cols else self.shape
        self.m, self.n_pos = int(m), int(N)
        self.cfg = Config(n_rows=rows, n_cols=cols, m=self.m, n_pos=self.n_pos, minibatch=int(minibatch),
                          levels=int(levels), alpha=float(alpha), alpha_z=float(alpha_z),
                          update_probe=int(bool(update_probe)), joint_step=int(bool(joint_step)),
                          path=PATHS[path],
                          seed=int(seed) & ((1 << 64) - 1), fft_plan=int(fft_plan),
                          finalize_shape=int(finalize_shape),
                          tune_cache=None if tune_cache is None else os.fsencode(tune_cache),
                          zero_phase_memory=int(bool(zero_phase_memory)))
        nbytes = workspace_size(self.cfg)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=intensities.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        self.positions = pos
        self._ctx = ctypes.c_void_p(None)
        _check(lib().emagpie_init(ctypes.byref(self._ctx), ctypes.byref(self.cfg), pos.ctypes.data,
                                  intensities.data_ptr(), self._ws_ptr, nbytes, _stream()))

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            torch.cuda.current_stream().synchronize()
            lib().emagpie_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- timing -----------------------------------------------------------
    def profile(self, enable: bool = True):
        _check(lib().emagpie_profile_enable(self._ctx, int(bool(enable))), self._ctx)

    def profile_read(self):
        """{'patch': (ms, launches), 'finalize': (...), 'persistent': (...)} since the last read."""
        ms = np.zeros(3, dtype=np.float64)
        cnt = np.zeros(3, dtype=np.int64)
        _check(lib().emagpie_profile_read(self._ctx, ms.ctypes.data, cnt.ctypes.data), self._ctx)
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(["patch", "finalize", "persistent"])}

    # -- operations -------------------------------------------------------
    @property
    def dp_avg(self) -> float:
        out = ctypes.c_double(0)
        _check(lib().emagpie_dp_avg(self._ctx, ctypes.byref(out)), self._ctx)
        return out.value

    @property
    def plan(self) -> dict:
        """The kernel plan this context runs with (after any autotuning at init)."""
        p = Plan()
        _check(lib().emagpie_plan_get(self._ctx, ctypes.byref(p)), self._ctx)
        return p.as_dict()

    def _state(self, obj, probe, dtype=torch.complex64):
        _expect(obj, dtype, self.shape, "object")
        _expect(probe, dtype, (self.m, self.m), "probe")

    def normalize_probe(self, probe: torch.Tensor):
        _expect(probe, torch.complex64, (self.m, self.m), "probe")
        _check(lib().emagpie_normalize_probe(self._ctx, probe.data_ptr(), _stream()), self._ctx)

    def _indices(self, idx) -> torch.Tensor:
        t = torch.as_tensor(idx, dtype=torch.int32)
        host = t.cpu().numpy() if t.is_cuda else t.numpy()
        if host.ndim != 1 or host.size < 1 or host.size > self.cfg.minibatch:
            raise ValueError("index list must be 1-D with 1..minibatch entries")
        if host.min() < 0 or host.max() >= self.n_pos or len(set(host.tolist())) != host.size:
            raise ValueError("indices must be distinct and in [0, N)")
        return t.to(device="cuda").contiguous()

    def step(self, obj, probe, idx, sampled: torch.Tensor | None = None):
        self._state(obj, probe)
        d_idx = self._indices(idx)
        _check(lib().emagpie_step_minibatch(self._ctx, obj.data_ptr(), probe.data_ptr(),
                                            d_idx.data_ptr(), d_idx.numel(), _ptr(sampled), _stream()), self._ctx)
        return d_idx

    def epoch(self, obj, probe, epoch: int, perm: torch.Tensor | None = None,
              sampled: torch.Tensor | None = None):
        self._state(obj, probe)
        if perm is not None:
            _expect(perm, torch.int32, (self.n_pos,), "perm")
        _check(lib().emagpie_epoch(self._ctx, obj.data_ptr(), probe.data_ptr(), int(epoch),
                                   _ptr(perm), _ptr(sampled), _stream()), self._ctx)

    def reset_phase_memory(self):
        """Zero-bin phase memory back to the first-sweep state (theta = 0 everywhere)."""
        _check(lib().emagpie_phase_memory_reset(self._ctx, _stream()), self._ctx)

    def debug_barrier(self, spin_limit: int = 0, target_skew: int = 0):
        """Fault injection for the persistent path's error reporting (tests only): grid
        barriers of later persistent epochs poll at most spin_limit times (0: default) and
        wait for target_skew extra arrivals, so with target_skew > 0 every wait gives up and
        the next call raises E_HIP."""
        _check(lib().emagpie_debug_barrier(self._ctx, int(spin_limit), int(target_skew)), self._ctx)

    @property
    def last_error(self) -> str:
        return last_error(self._ctx)

    def check_step(self, obj, probe, idx) -> torch.Tensor:
        """One minibatch update (as step()) that also returns, in float64 on the device,
        [Phi_B before, surrogate of Eq. 3 after (R frozen before), Phi_B after]."""
        self._state(obj, probe)
        t = self._indices(idx)
        out = torch.empty(3, dtype=torch.float64, device="cuda")
        _check(lib().emagpie_check_step(self._ctx, obj.data_ptr(), probe.data_ptr(), t.data_ptr(),
                                        t.numel(), out.data_ptr(), _stream()), self._ctx)
        return out

    def mg_cycle(self, obj, probe, idx) -> torch.Tensor:
        self._state(obj, probe)
        d_idx = self._indices(idx)
        out = torch.empty((d_idx.numel(), self.m, self.m), dtype=torch.complex64, device="cuda")
        _check(lib().emagpie_mg_cycle(self._ctx, obj.data_ptr(), probe.data_ptr(), d_idx.data_ptr(),
                                      d_idx.numel(), out.data_ptr(), _stream()), self._ctx)
        return out

    def misfit(self, obj, probe, out: torch.Tensor | None = None) -> torch.Tensor:
        self._state(obj, probe)
        if out is None:
            out = torch.empty((), dtype=torch.float64, device="cuda")
        _check(lib().emagpie_misfit(self._ctx, obj.data_ptr(), probe.data_ptr(), out.data_ptr(),
                                    _stream()), self._ctx)
        return out

    def grad(self, obj, probe):
        """(grad_obj, grad_probe, Phi) with gradient = d/dx + i d/dy (float32 or float64)."""
        f64 = obj.dtype == torch.complex128
        self._state(obj, probe, torch.complex128 if f64 else torch.complex64)
        gobj = torch.empty_like(obj)
        gprobe = torch.empty_like(probe)
        phi = torch.empty((), dtype=torch.float64, device="cuda")
        _check(lib().emagpie_grad(self._ctx, obj.data_ptr(), probe.data_ptr(), gobj.data_ptr(),
                                  gprobe.data_ptr(), phi.data_ptr(), F64 if f64 else F32, _stream()), self._ctx)
        return gobj, gprobe, phi


class AmplitudeMisfit(torch.autograd.Function):
    """Phi(Q, z) of Eq. 1 with its hand-written adjoint (libemagpie grad kernels).

    forward(obj, probe, rec) -> real scalar; backward returns grad_output times the CR
    gradient d/dx + i d/dy, which is torch's convention for real losses of complex inputs.
    Double backward is not supported.
    """

    @staticmethod
    def forward(ctx, obj, probe, rec: Reconstruction):
        gobj, gprobe, phi = rec.grad(obj.detach().contiguous(), probe.detach().contiguous())
        ctx.save_for_backward(gobj, gprobe)
        real = torch.float64 if obj.dtype == torch.complex128 else torch.float32
        return phi.to(real)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g):
        gobj, gprobe = ctx.saved_tensors
        return g.to(gobj.real.dtype) * gobj, g.to(gprobe.real.dtype) * gprobe, None


class Group:
    """Several independent reconstructions advanced together (one sweep each per call).

    Every member keeps its own configuration, data and state; a group epoch gives
    bitwise the same result as calling `Reconstruction.epoch` on each member.
    """

    def __init__(self, recs):
        self.recs = list(recs)
        n = len(self.recs)
        self._ctxs = (ctypes.c_void_p * n)(*[r._ctx.value for r in self.recs])
        nbytes = ctypes.c_size_t(0)
        _check(lib().emagpie_group_workspace_size(n, self._ctxs, ctypes.byref(nbytes)))
        self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        ptr = (self._ws.data_ptr() + 255) & ~255
        self._g = ctypes.c_void_p(None)
        _check(lib().emagpie_group_create(ctypes.byref(self._g), n, self._ctxs, ptr, nbytes.value,
                                          _stream()))

    def epoch(self, objs, probes, epoch: int, sampled: torch.Tensor | None = None):
        n = len(self.recs)
        if len(objs) != n or len(probes) != n:
            raise ValueError("one object and one probe per member")
        for r, o, q in zip(self.recs, objs, probes):
            r._state(o, q)
        if sampled is not None:
            _expect(sampled, torch.float64, (n,), "sampled")
        op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in objs])
        pp = (ctypes.c_void_p * n)(*[q.data_ptr() for q in probes])
        _check(lib().emagpie_group_epoch(self._g, op, pp, int(epoch), _ptr(sampled), _stream()))

    def close(self):
        if getattr(self, "_g", None) is not None and self._g.value:
            torch.cuda.current_stream().synchronize()
            lib().emagpie_group_destroy(self._g)
            self._g = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Many:
    """Several independent reconstructions behind one library context
    (emagpie_init_many / emagpie_epoch_many); member i is a Reconstruction-like view for the
    per-instance calls.  Bitwise the same as a Group of separately made Reconstructions.

    problems: a list of dicts with the Reconstruction arguments (positions, intensities, n,
    minibatch, levels, alpha, alpha_z, update_probe, joint_step, path, seed, fft_plan,
    finalize_shape, zero_phase_memory).
    """

    def __init__(self, problems):
        n = len(problems)
        cfgs = (Config * n)()
        self._pos, self._inten, self.members = [], [], []
        for i, pr in enumerate(problems):
            pos = np.ascontiguousarray(np.asarray(pr["positions"], dtype=np.int32).reshape(-1, 2))
            d = pr["intensities"].contiguous()
            N, m, _ = d.shape
            nn = pr["n"]
            rows, cols = (int(nn), int(nn)) if np.ndim(nn) == 0 else (int(nn[0]), int(nn[1]))
            cfgs[i] = Config(n_rows=rows, n_cols=cols, m=int(m), n_pos=int(N),
                             minibatch=int(pr["minibatch"]), levels=int(pr.get("levels", 1)),
                             alpha=float(pr.get("alpha", 0.05)), alpha_z=float(pr.get("alpha_z", 1.0)),
                             update_probe=int(bool(pr.get("update_probe", True))),
                             joint_step=int(bool(pr.get("joint_step", True))),
                             path=PATHS[pr.get("path", "graph")],
                             seed=int(pr.get("seed", 0)) & ((1 << 64) - 1),
                             fft_plan=int(pr.get("fft_plan", 0)),
                             finalize_shape=int(pr.get("finalize_shape", 0)), tune_cache=None,
                             zero_phase_memory=int(bool(pr.get("zero_phase_memory", False))))
            self._pos.append(pos)
            self._inten.append(d)
        self._cfgs = cfgs
        nbytes = ctypes.c_size_t(0)
        _check(lib().emagpie_workspace_size_many(n, cfgs, ctypes.byref(nbytes)))
        self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        ptr = (self._ws.data_ptr() + 255) & ~255
        pos_arr = (ctypes.c_void_p * n)(*[p.ctypes.data for p in self._pos])
        int_arr = (ctypes.c_void_p * n)(*[d.data_ptr() for d in self._inten])
        self._ctx = ctypes.c_void_p(None)
        _check(lib().emagpie_init_many(ctypes.byref(self._ctx), n, cfgs, pos_arr, int_arr, ptr,
                                       nbytes.value, _stream()))
        self._inten = None  # copied into the workspace at init
        for i in range(n):
            h = ctypes.c_void_p(None)
            _check(lib().emagpie_many_member(self._ctx, i, ctypes.byref(h)), self._ctx)
            self.members.append(_Member(h, cfgs[i], self._pos[i]))

    def epoch(self, objs, probes, epoch: int, sampled: torch.Tensor | None = None):
        n = len(self.members)
        if len(objs) != n or len(probes) != n:
            raise ValueError("one object and one probe per member")
        for r, o, q in zip(self.members, objs, probes):
            r._state(o, q)
        if sampled is not None:
            _expect(sampled, torch.float64, (n,), "sampled")
        op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in objs])
        pp = (ctypes.c_void_p * n)(*[q.data_ptr() for q in probes])
        _check(lib().emagpie_epoch_many(self._ctx, op, pp, int(epoch), _ptr(sampled), _stream()),
               self._ctx)

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            torch.cuda.current_stream().synchronize()
            for r in self.members:
                r._ctx = ctypes.c_void_p(None)  # owned by the many-context
            lib().emagpie_destroy(self._ctx)
            self._ctx = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Member(Reconstruction):
    """A member context of a Many (borrowed handle: closing it does nothing)."""

    def __init__(self, handle, cfg, positions):  # noqa: D401 - no Reconstruction.__init__
        self._ctx = handle
        self.cfg = cfg
        self.shape = (int(cfg.n_rows), int(cfg.n_cols))
        self.n = self.shape[0] if self.shape[0] == self.shape[1] else self.shape
        self.m, self.n_pos = int(cfg.m), int(cfg.n_pos)
        self.positions = positions

    def close(self):
        pass


def measure_peaks(nbytes: int = 1 << 30, reps: int = 5) -> dict:
    """Measured copy bandwidth (GB/s) and FP32 FMA rate (TFLOP/s) of the current device."""
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ptr = (buf.data_ptr() + 255) & ~255
    out = np.zeros(2, dtype=np.float64)
    _check(lib().emagpie_measure_peaks(ptr, nbytes, int(reps), out.ctypes.data, _stream()))
    return {"copy_GBs": float(out[0]), "fp32_fma_TFLOPs": float(out[1]), "copy_bytes": nbytes,
            "reps": reps}


def misfit_noalloc(positions: torch.Tensor, intensities: torch.Tensor, obj: torch.Tensor,
                   probe: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Phi of Eq. 1 through emagpie_misfit_noalloc (no context, no workspace): positions
    (N, 2) int32 and intensities (N, m, m) float32 (natural order), object and probe
    complex64, all CUDA tensors."""
    N = positions.shape[0]
    m = probe.shape[0]
    _expect(positions, torch.int32, (N, 2), "positions")
    _expect(intensities, torch.float32, (N, m, m), "intensities")
    _expect(probe, torch.complex64, (m, m), "probe")
    _expect(obj, torch.complex64, tuple(obj.shape), "object")
    if out is None:
        out = torch.empty((), dtype=torch.float64, device="cuda")
    _check(lib().emagpie_misfit_noalloc(obj.shape[0], obj.shape[1], m, N, positions.data_ptr(),
                                        intensities.data_ptr(), obj.data_ptr(), probe.data_ptr(),
                                        out.data_ptr(), _stream()))
    return out
