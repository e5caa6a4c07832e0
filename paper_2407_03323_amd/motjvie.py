"""Python binding of libmotjvie.so (C interface in include/motjvie.h).

Argument marshalling only: every step of the march runs in the HIP library.  Device
buffers are torch CUDA tensors (float64, contiguous); PyTorch provides device memory
and the stream, nothing else.  The library must have been built (paper_2407_03323_amd/
build.py); importing this module on a machine without it raises immediately.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmotjvie.so")

MJ_OK, MJ_EINVAL, MJ_ENOMEM, MJ_EHIP, MJ_ENOCONV, MJ_EUNSTABLE, MJ_ESTATE = 0, -1, -2, -3, -4, -5, -6
_NAMES = {MJ_EINVAL: "MJ_EINVAL", MJ_ENOMEM: "MJ_ENOMEM", MJ_EHIP: "MJ_EHIP", MJ_ENOCONV: "MJ_ENOCONV",
          MJ_EUNSTABLE: "MJ_EUNSTABLE", MJ_ESTATE: "MJ_ESTATE"}


class MotJvieError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


# device allocator callbacks of mj_config (alloc(bytes, ctx) -> ptr, free_(ptr, ctx))
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class mj_config(ctypes.Structure):
    _fields_ = [
        ("U", ctypes.c_int32), ("V", ctypes.c_int32), ("W", ctypes.c_int32),
        ("h", ctypes.c_double), ("c_dt", ctypes.c_double),
        ("eps_r", ctypes.POINTER(ctypes.c_double)),
        ("fir", ctypes.POINTER(ctypes.c_double)), ("n_fir", ctypes.c_int32),
        ("n_rhs", ctypes.c_int32),
        ("cg_rtol", ctypes.c_double), ("cg_maxit", ctypes.c_int32),
        ("time_block", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("quad_order", ctypes.c_int32),
        ("fft_pencils", ctypes.c_int32),
        ("hy", ctypes.c_double), ("hz", ctypes.c_double),
        ("alloc", ALLOC_FN), ("free_", FREE_FN), ("alloc_ctx", ctypes.c_void_p),
        ("outer_block", ctypes.c_int32), ("z0_solver", ctypes.c_int32), ("z0_graphs", ctypes.c_int32),
        ("outer_overlap", ctypes.c_int32),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmotjvie.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libmotjvie.so not built (run paper_2407_03323_amd/build.py): %s" % path)
    L = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
    L.mj_create.argtypes = [ctypes.POINTER(mj_config), ctypes.POINTER(vp)]
    L.mj_destroy.argtypes = [vp]
    L.mj_destroy.restype = None
    L.mj_last_error.argtypes = [vp]
    L.mj_last_error.restype = ctypes.c_char_p
    L.mj_info.argtypes = [vp, dp, ctypes.c_int32]
    L.mj_set_plane_waves.argtypes = [vp, dp, dp, dp, dp, dp, dp]
    L.mj_run.argtypes = [vp, ctypes.c_int32, vp]
    L.mj_reset.argtypes = [vp]
    L.mj_history_sum.argtypes = [vp, vp, ctypes.c_int32, vp]
    L.mj_kernel_values.argtypes = [vp, ctypes.c_int32, ip, ip, dp]
    L.mj_kernel_values_noalloc.argtypes = [vp, ctypes.c_int32, ip, ip, dp]
    L.mj_stats.argtypes = [vp, dp, ctypes.c_int32]
    L.mj_fft_roundtrip.argtypes = [vp, vp, vp, vp]
    L.mj_set_probes.argtypes = [vp, ctypes.c_int32, dp]
    L.mj_march.argtypes = [vp, ctypes.c_int32, vp, vp]
    L.mj_step.argtypes = [vp, vp, vp]
    L.mj_march_every.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp]
    L.mj_probe_kernel_values.argtypes = [vp, ctypes.c_int32, ip, ip, ip, dp]
    L.mj_set_eps.argtypes = [vp, dp]
    L.mj_adjoint_gradient.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, dp, vp, vp]
    L.mj_get_state.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
    L.mj_set_state.argtypes = [vp, vp, ctypes.c_size_t]
    for f in ("mj_create", "mj_info", "mj_set_plane_waves", "mj_run", "mj_reset", "mj_history_sum",
              "mj_kernel_values", "mj_stats", "mj_fft_roundtrip", "mj_set_probes", "mj_march",
              "mj_probe_kernel_values", "mj_set_eps", "mj_adjoint_gradient", "mj_get_state", "mj_set_state",
              "mj_step", "mj_march_every", "mj_kernel_values_noalloc"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _tptr(t, what):
    """Device pointer of a float64 contiguous CUDA tensor (or None)."""
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("%s must be a contiguous float64 CUDA tensor" % what)
    return ctypes.c_void_p(t.data_ptr())


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def torch_allocator(stream=None):
    """alloc / free_ callbacks that take the library's device memory from PyTorch's caching
    allocator on `stream` (a raw stream handle; default torch's current stream).  The returned
    pair must stay referenced for as long as the solver lives."""
    import torch
    dev = torch.cuda.current_device()
    handle = int(stream.value if isinstance(stream, ctypes.c_void_p) else
                 (stream if stream is not None else torch.cuda.current_stream().cuda_stream))

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, handle)
        except Exception:
            return None   # NULL: the library reports MJ_ENOMEM

    def _free(ptr, ctx):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass

    return ALLOC_FN(_alloc), FREE_FN(_free)


class Solver:
    """One MOT-JVIE march on the device (see include/motjvie.h for the exact semantics)."""

    def __init__(self, U, V, W, eps, fir=None, h=1.0, c_dt=None, n_rhs=1, cg_rtol=0.0, cg_maxit=0,
                 time_block=0, quad_order=0, stream=None, fft_pencils=0, hy=0.0, hz=0.0, allocator=None,
                 outer_block=0, z0_solver=0, z0_graphs=0, outer_overlap=0):
        """allocator: None (the library's hipMalloc) or "torch" (PyTorch's caching allocator,
        through mj_config.alloc / free_)."""
        self._lib = load_library()
        self._h = ctypes.c_void_p()
        eps = np.ascontiguousarray(np.asarray(eps, dtype=np.float64).reshape(W, V, U))
        fir = np.ascontiguousarray(np.zeros(0) if fir is None else np.asarray(fir, dtype=np.float64))
        self.U, self.V, self.W, self.n_rhs = int(U), int(V), int(W), int(n_rhs)
        self.M = self.U * self.V * self.W
        cfg = mj_config()
        cfg.U, cfg.V, cfg.W = self.U, self.V, self.W
        cfg.h = float(h)
        cfg.c_dt = float(h if c_dt is None else c_dt)
        cfg.eps_r = _dptr(eps)
        cfg.fir = _dptr(fir) if len(fir) else None
        cfg.n_fir = len(fir)
        cfg.n_rhs = self.n_rhs
        cfg.cg_rtol = float(cg_rtol)
        cfg.cg_maxit = int(cg_maxit)
        cfg.time_block = int(time_block)
        cfg.stream = stream if stream is not None else _current_stream()
        cfg.quad_order = int(quad_order)
        cfg.fft_pencils = int(fft_pencils)
        cfg.hy, cfg.hz = float(hy), float(hz)
        cfg.outer_block = int(outer_block)
        cfg.z0_solver = int(z0_solver)
        cfg.z0_graphs = int(z0_graphs)
        cfg.outer_overlap = int(outer_overlap)
        self._alloc_fns = None
        if allocator == "torch":
            self._alloc_fns = torch_allocator(cfg.stream)
            cfg.alloc, cfg.free_ = self._alloc_fns
        elif allocator is not None:
            raise ValueError("allocator must be None or 'torch'")
        self._keep = (eps, fir)
        rc = self._lib.mj_create(ctypes.byref(cfg), ctypes.byref(self._h))
        if rc != MJ_OK:
            raise MotJvieError(rc, self._lib.mj_last_error(None).decode())

    # ------------------------------------------------------------------ helpers
    def _check(self, rc):
        if rc != MJ_OK:
            raise MotJvieError(rc, self._lib.mj_last_error(self._h).decode())

    def close(self):
        if self._h:
            self._lib.mj_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        out = np.zeros(24)
        self._check(self._lib.mj_info(self._h, _dptr(out), 24))
        keys = ["ell", "Nx", "Ny", "Nz", "time_block", "real_depth", "n_rhs", "n", "device_bytes",
                "gen_ms", "spectra_ms", "n_fir", "n_probes", "probe_window", "probe_pairs", "probe_gen_ms",
                "fft_pencils_x", "fft_pencils_y", "fft_pencils_z", "outer_block", "z0_solver", "lam_lo", "lam_hi",
                "outer_overlap"]
        ms = ("gen_ms", "spectra_ms", "probe_gen_ms", "lam_lo", "lam_hi")
        return {k: (int(v) if k not in ms else float(v)) for k, v in zip(keys, out)}

    @property
    def ell(self) -> int:
        return self.info()["ell"]

    # ------------------------------------------------------------------ march
    def set_plane_waves(self, waves):
        """waves: sequence (one per right-hand side) of objects with khat, pol, width, t0, amp, r_ref."""
        assert len(waves) == self.n_rhs
        k = np.ascontiguousarray([w.khat for w in waves], dtype=np.float64)
        p = np.ascontiguousarray([w.pol for w in waves], dtype=np.float64)
        wd = np.ascontiguousarray([w.width for w in waves], dtype=np.float64)
        t0 = np.ascontiguousarray([w.t0 for w in waves], dtype=np.float64)
        a = np.ascontiguousarray([w.amp for w in waves], dtype=np.float64)
        rr = np.ascontiguousarray([w.r_ref for w in waves], dtype=np.float64)
        self._check(self._lib.mj_set_plane_waves(self._h, _dptr(k), _dptr(p), _dptr(wd), _dptr(t0), _dptr(a),
                                                 _dptr(rr)))

    def set_probes(self, pos):
        """Probe points [n][3] (units of h, origin at the grid corner); before the first step."""
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
        self.n_probes = len(pos)
        self._check(self._lib.mj_set_probes(self._h, len(pos), _dptr(pos) if len(pos) else None))

    def run(self, n_steps: int, J_out=None, probes_out=None, j_every: int = 1):
        """March n_steps; J_out (optional) is a CUDA tensor [n_steps // j_every][n_rhs][3][W][V][U]
        receiving J of every j_every-th step, probes_out (optional) a CUDA tensor
        [n_steps][n_rhs][n_probes][3]."""
        if J_out is not None:
            assert J_out.numel() == (n_steps // j_every) * self.n_rhs * 3 * self.M
        if probes_out is not None:
            assert probes_out.numel() == n_steps * self.n_rhs * getattr(self, "n_probes", 0) * 3
        if j_every != 1:
            self._check(self._lib.mj_march_every(self._h, int(n_steps), int(j_every), _tptr(J_out, "J_out"),
                                                 _tptr(probes_out, "probes_out")))
        elif probes_out is None:
            self._check(self._lib.mj_run(self._h, int(n_steps), _tptr(J_out, "J_out")))
        else:
            self._check(self._lib.mj_march(self._h, int(n_steps), _tptr(J_out, "J_out"),
                                           _tptr(probes_out, "probes_out")))

    def step(self, J_out=None, probe_out=None):
        """One step; J_out [n_rhs][3][W][V][U] and probe_out [n_rhs][n_probes][3] are optional
        CUDA tensors."""
        if J_out is not None:
            assert J_out.numel() == self.n_rhs * 3 * self.M
        if probe_out is not None:
            assert probe_out.numel() == self.n_rhs * getattr(self, "n_probes", 0) * 3
        self._check(self._lib.mj_step(self._h, _tptr(J_out, "J_out"), _tptr(probe_out, "probe_out")))

    def probe_kernel_values(self, probe, voxels, lags) -> np.ndarray:
        probe = np.ascontiguousarray(np.asarray(probe, dtype=np.int32))
        vox = np.ascontiguousarray(np.asarray(voxels, dtype=np.int32).reshape(-1, 3))
        lags = np.ascontiguousarray(np.asarray(lags, dtype=np.int32))
        out = np.zeros((len(lags), 6))
        ip = ctypes.POINTER(ctypes.c_int32)
        self._check(self._lib.mj_probe_kernel_values(self._h, len(lags), probe.ctypes.data_as(ip),
                                                     vox.ctypes.data_as(ip), lags.ctypes.data_as(ip), _dptr(out)))
        return out

    def reset(self):
        self._check(self._lib.mj_reset(self._h))

    def get_state(self) -> np.ndarray:
        """The march state (step count and every history the next steps read) as host bytes."""
        nb = ctypes.c_size_t(0)
        self._check(self._lib.mj_get_state(self._h, None, ctypes.byref(nb)))
        buf = np.empty(nb.value, dtype=np.uint8)
        self._check(self._lib.mj_get_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nb)))
        return buf

    def set_state(self, buf):
        """Resume from get_state() of a solver with the same configuration (and probes)."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self._lib.mj_set_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes))

    def history_sum(self, J_hist, P):
        """P_{n-1} for the explicit history J_hist[k-1] = J_{n-k} (CUDA tensors)."""
        depth = J_hist.shape[0]
        assert J_hist.numel() == depth * 3 * self.M and P.numel() == 3 * self.M
        self._check(self._lib.mj_history_sum(self._h, _tptr(J_hist, "J_hist"), int(depth), _tptr(P, "P")))

    def kernel_values(self, lags, offsets) -> np.ndarray:
        lags = np.ascontiguousarray(np.asarray(lags, dtype=np.int32))
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
        out = np.zeros((len(lags), 6))
        ip = ctypes.POINTER(ctypes.c_int32)
        self._check(self._lib.mj_kernel_values(self._h, len(lags), lags.ctypes.data_as(ip),
                                               offs.ctypes.data_as(ip), _dptr(out)))
        return out

    def kernel_values_noalloc(self, lags, offsets) -> np.ndarray:
        """kernel_values through the library's fixed staging array (no device allocation)."""
        lags = np.ascontiguousarray(np.asarray(lags, dtype=np.int32))
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
        out = np.zeros((len(lags), 6))
        ip = ctypes.POINTER(ctypes.c_int32)
        self._check(self._lib.mj_kernel_values_noalloc(self._h, len(lags), lags.ctypes.data_as(ip),
                                                       offs.ctypes.data_as(ip), _dptr(out)))
        return out

    def set_eps(self, eps):
        """New eps_r [W][V][U] for the same grid (kernels kept); at n = 0."""
        e = np.ascontiguousarray(np.asarray(eps, dtype=np.float64).reshape(self.W, self.V, self.U))
        self._keep = (e,) + tuple(self._keep[1:])
        self._check(self._lib.mj_set_eps(self._h, _dptr(e)))

    def adjoint_gradient(self, n_steps: int, grad_out, ckpt_every: int = 0, probes_out=None) -> float:
        """Phi = sum |E^s|^2 over n_steps and the probes; grad_out (CUDA tensor [W][V][U])
        receives dPhi/deps_r.  Returns Phi."""
        assert grad_out.numel() == self.M
        phi = ctypes.c_double()
        self._check(self._lib.mj_adjoint_gradient(self._h, int(n_steps), int(ckpt_every), ctypes.byref(phi),
                                                  _tptr(grad_out, "grad_out"), _tptr(probes_out, "probes_out")))
        return phi.value

    def stats(self) -> dict:
        out = np.zeros(21)
        self._check(self._lib.mj_stats(self._h, _dptr(out), 21))
        keys = ["fft_fwd_ms", "mac_ms", "fft_inv_ms", "epilogue_ms", "z0_ms", "step_ms", "cg_iters",
                "cg_res_max", "steps", "cg_iters_max", "far_launch_ms", "far_launches", "near_launch_ms",
                "probe_ms", "adjoint_forward_ms", "adjoint_backward_ms", "adjoint_segments",
                "adjoint_checkpoint_bytes", "mid_launch_ms", "side_launch_ms", "side_launches"]
        return dict(zip(keys, out.tolist()))

    def fft_roundtrip(self, x, X=None, y=None):
        self._check(self._lib.mj_fft_roundtrip(self._h, _tptr(x, "x"), _tptr(X, "X"), _tptr(y, "y")))


def solver_for(problem, **kw) -> Solver:
    """Solver for a workloads.Problem, with its plane waves set."""
    s = Solver(problem.U, problem.V, problem.W, problem.eps, fir=problem.fir, h=problem.h, c_dt=problem.c_dt,
               hy=getattr(problem, "hy", 0.0), hz=getattr(problem, "hz", 0.0),
               n_rhs=kw.pop("n_rhs", len(problem.waves) or 1), **kw)
    if problem.waves:
        s.set_plane_waves(problem.waves)
    return s


class ProbeObjective:
    """Phi(eps_r) = sum_n sum_p |E^s_p(n)|^2 as a torch.autograd.Function: forward runs the
    march and the transposed march (mj_adjoint_gradient) on one Solver whose probes and
    plane waves are set; backward returns grad_output * dPhi/deps_r.  The kernels stay, only
    eps changes between calls (mj_set_eps)."""

    def __init__(self, solver: Solver, n_steps: int, ckpt_every: int = 0):
        self.solver = solver
        self.n_steps = int(n_steps)
        self.ckpt_every = int(ckpt_every)
        self._fn = None

    def function(self):
        import torch
        outer = self

        class _Phi(torch.autograd.Function):
            @staticmethod
            def forward(ctx, eps):
                s = outer.solver
                s.reset()
                s.set_eps(eps.detach().double().cpu().numpy())
                grad = torch.zeros((s.W, s.V, s.U), dtype=torch.float64, device="cuda")
                phi = s.adjoint_gradient(outer.n_steps, grad, outer.ckpt_every)
                ctx.save_for_backward(grad.to(eps.device, eps.dtype))
                return torch.tensor(phi, dtype=eps.dtype, device=eps.device)

            @staticmethod
            def backward(ctx, g):
                (grad,) = ctx.saved_tensors
                return g * grad

        return _Phi

    def __call__(self, eps):
        if self._fn is None:
            self._fn = self.function()
        return self._fn.apply(eps)

