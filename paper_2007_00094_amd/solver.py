"""Python face of the library: a Solver over one Q1 mesh, a BatchSolver
over many independent meshes.

State tensors are torch.float64 on the current HIP device, [n_nodes, dim+2]
contiguous, in the caller's node order; calls are ordered on the torch
stream that was current when the Solver was created.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import capi


def _require_torch_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the IDP library needs a HIP device (none visible)")
    return torch


class Solver:
    def __init__(self, mesh=None, *, dim=None, coords=None, cells=None,
                 dirichlet=None, gamma=1.4, cfl=0.5, passes=2, newton_max=2,
                 newton_tol=1e-10, asynchronous=False, stream=None, staging=True,
                 sell_sigma=0, renumber=False, relax=False, split_p=False):
        torch = _require_torch_gpu()
        if mesh is not None:
            dim, coords, cells = mesh.dim, mesh.coords, mesh.cells
            if dirichlet is None:
                dirichlet = mesh.boundary
        self.dim = int(dim)
        self.nc = self.dim + 2
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        self.n = int(coords.shape[0])
        L = capi.lib()
        p = capi.idp_params()
        capi.check("idp_default_params", L.idp_default_params(C.byref(p), self.dim))
        p.gamma, p.cfl = float(gamma), float(cfl)
        p.limiter_passes, p.newton_max_iter = int(passes), int(newton_max)
        p.newton_tol = float(newton_tol)
        p.flags = (capi.IDP_FLAG_ASYNC if asynchronous else 0) | \
            (0 if staging else capi.IDP_FLAG_NO_STAGING) | \
            (capi.IDP_FLAG_RENUMBER if renumber else 0) | \
            (capi.IDP_FLAG_SPLIT_P if split_p else 0)
        p.sell_sigma = int(sell_sigma)
        p.relax_bounds = 1 if relax else 0
        self.params = p
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        hd = None
        if dirichlet is not None:
            hd = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        h = C.c_void_p()
        rc = L.idp_create(C.byref(h), C.byref(p), self.n,
                          coords.ctypes.data_as(capi._dp), int(cells.shape[0]),
                          cells.ctypes.data_as(capi._i64p),
                          hd.ctypes.data_as(capi._u8p) if hd is not None else None,
                          C.c_void_p(self._stream.cuda_stream))
        capi.check("idp_create", rc)
        self._h = h
        nn, nz, nb = C.c_int64(), C.c_int64(), C.c_size_t()
        capi.check("idp_info", L.idp_info(h, C.byref(nn), C.byref(nz), C.byref(nb)))
        self.nnz = int(nz.value)
        self.device_bytes = int(nb.value)

    # ---------------------------------------------------------------- life
    def close(self):
        h = getattr(self, "_h", None)
        if h:
            capi.lib().idp_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _u(self, U):
        torch = _require_torch_gpu()
        if not (isinstance(U, torch.Tensor) and U.is_cuda and U.dtype == torch.float64
                and U.is_contiguous() and tuple(U.shape) == (self.n, self.nc)):
            raise ValueError(f"state must be a contiguous float64 device tensor "
                             f"of shape ({self.n}, {self.nc})")
        return C.c_void_p(U.data_ptr())

    # ------------------------------------------------------------- calls
    def max_dt(self, U) -> float:
        out = C.c_double()
        capi.check("idp_max_dt", capi.lib().idp_max_dt(self._h, self._u(U), C.byref(out)))
        return out.value

    def step(self, U, dt: float = 0.0):
        """One SSP-RK3 step in place; returns (dt_used, status)."""
        used = C.c_double(0.0)
        rc = capi.lib().idp_step(self._h, self._u(U), float(dt), C.byref(used))
        capi.check("idp_step", rc)
        return used.value, rc

    def euler_stage(self, U, tau: float, out=None):
        """E(U) with step tau into out (allocated if None); returns (out, status)."""
        torch = _require_torch_gpu()
        if out is None:
            out = torch.empty_like(U)
        rc = capi.lib().idp_euler_stage(self._h, self._u(U), float(tau), self._u(out))
        capi.check("idp_euler_stage", rc)
        return out, rc

    def status(self) -> int:
        return capi.check("idp_get_status", capi.lib().idp_get_status(self._h))

    # ----------------------------------------------------------- adjoint
    def euler_stage_vjp(self, U, tau: float, Ebar):
        """(dE/dU)^T Ebar for the forward-Euler update with step tau."""
        torch = _require_torch_gpu()
        out = torch.empty_like(U)
        capi.check("idp_euler_stage_vjp", capi.lib().idp_euler_stage_vjp(
            self._h, self._u(U), float(tau), self._u(Ebar), self._u(out)))
        return out

    def step_vjp(self, U, dt: float, Ubar_next):
        """(dS/dU)^T Ubar_next for one SSP-RK3 step from U with step dt."""
        torch = _require_torch_gpu()
        out = torch.empty_like(U)
        capi.check("idp_step_vjp", capi.lib().idp_step_vjp(
            self._h, self._u(U), float(dt), self._u(Ubar_next), self._u(out)))
        return out

    checkpoint_generation = 0

    def forward_checkpoints(self, U, dts, every: int):
        """len(dts) steps in place with the given steps, checkpoints kept
        (replacing those of the previous run; checkpoint_generation counts
        the runs)."""
        d = np.ascontiguousarray(dts, dtype=np.float64)
        self.checkpoint_generation += 1
        return capi.check("idp_forward_checkpoints", capi.lib().idp_forward_checkpoints(
            self._h, self._u(U), len(d), d.ctypes.data_as(capi._dp), int(every)))

    def trace_decisions(self, U, dts, out=None):
        """len(dts) steps in place with the given steps, every stage's
        decisions into a device byte tensor (allocated if out is None);
        returns (trace [3 len(dts), stage_bytes] uint8, stage_bytes)."""
        torch = _require_torch_gpu()
        d = np.ascontiguousarray(dts, dtype=np.float64)
        sb = C.c_int64(0)
        capi.check("idp_trace_decisions", capi.lib().idp_trace_decisions(
            self._h, None, 0, None, None, 0, C.byref(sb)))
        nb = int(sb.value)
        if out is None:
            out = torch.empty((3 * len(d), nb), dtype=torch.uint8, device=U.device)
        capi.check("idp_trace_decisions", capi.lib().idp_trace_decisions(
            self._h, self._u(U), len(d), d.ctypes.data_as(capi._dp),
            C.c_void_p(out.data_ptr()), out.numel(), C.byref(sb)))
        return out, nb

    def adjoint_checkpoints(self, dts, every: int, Ubar_final):
        """Cotangent of the initial state of the last forward_checkpoints run."""
        torch = _require_torch_gpu()
        d = np.ascontiguousarray(dts, dtype=np.float64)
        out = torch.empty_like(Ubar_final)
        capi.check("idp_adjoint_checkpoints", capi.lib().idp_adjoint_checkpoints(
            self._h, len(d), d.ctypes.data_as(capi._dp), int(every), self._u(Ubar_final),
            self._u(out)))
        return out

    # ----------------------------------------------------------- exports
    def matrices(self):
        n, z, d = self.n, self.nnz, self.dim
        rp = np.empty(n + 1, np.int64)
        col = np.empty(z, np.int32)
        mi = np.empty(n)
        mij = np.empty(z)
        cij = np.empty((z, d))
        capi.check("idp_export_matrices", capi.lib().idp_export_matrices(
            self._h, rp.ctypes.data_as(capi._i64p), col.ctypes.data_as(capi._i32p),
            mi.ctypes.data_as(capi._dp), mij.ctypes.data_as(capi._dp),
            cij.ctypes.data_as(capi._dp)))
        return {"row_ptr": rp, "col": col, "m_i": mi, "m_ij": mij, "c_ij": cij}

    _DBG_SHAPE = {
        capi.IDP_DBG_D: "z", capi.IDP_DBG_L1: "z", capi.IDP_DBG_L2: "z",
        capi.IDP_DBG_ALPHA: "n", capi.IDP_DBG_TAUI: "n", capi.IDP_DBG_R: "nc",
        capi.IDP_DBG_UL: "nc", capi.IDP_DBG_UPASS: "nc", capi.IDP_DBG_BOUNDS: "n3",
        capi.IDP_DBG_P: "zc", capi.IDP_DBG_L1RAW: "z", capi.IDP_DBG_L2RAW: "z",
    }

    def debug(self, what: int) -> np.ndarray:
        kind = self._DBG_SHAPE[what]
        shape = {"z": (self.nnz,), "n": (self.n,), "nc": (self.n, self.nc),
                 "n3": (self.n, 3), "zc": (self.nnz, self.nc)}[kind]
        out = np.empty(shape)
        capi.check("idp_debug_export", capi.lib().idp_debug_export(
            self._h, int(what), out.ctypes.data_as(capi._dp)))
        return out

    # ------------------------------------------------------------ timing
    def set_timing(self, on: bool):
        capi.check("idp_set_timing", capi.lib().idp_set_timing(self._h, int(bool(on))))

    def kernel_times(self):
        names = (C.c_char_p * 32)()
        ms = np.zeros(32)
        cnt = np.zeros(32, np.int64)
        k = capi.check("idp_kernel_times", capi.lib().idp_kernel_times(
            self._h, 32, names, ms.ctypes.data_as(capi._dp), cnt.ctypes.data_as(capi._i64p)))
        return {names[i].decode(): (float(ms[i]), int(cnt[i])) for i in range(k)}

    def device_math(self, kind: int, x, y=None):
        torch = _require_torch_gpu()
        out = torch.empty_like(x)
        yp = C.c_void_p(y.data_ptr()) if y is not None else None
        capi.check("idp_device_math", capi.lib().idp_device_math(
            self._h, int(kind), int(x.numel()), C.c_void_p(x.data_ptr()), yp,
            C.c_void_p(out.data_ptr())))
        return out


class BatchSolver:
    """Many independent Q1 meshes advanced together, each with its own tau.

    The state is one contiguous float64 device tensor [N, dim+2]; instance k
    owns rows offsets[k]:offsets[k+1] (its own node order).  Results are
    bit-identical to a Solver per instance.
    """

    def __init__(self, meshes, *, dirichlet=None, gamma=1.4, cfl=0.5, passes=2,
                 newton_max=2, newton_tol=1e-10, stream=None, staging=True, sell_sigma=0):
        torch = _require_torch_gpu()
        meshes = list(meshes)
        if not meshes:
            raise ValueError("empty batch")
        self.dim = int(meshes[0].dim)
        if any(int(m.dim) != self.dim for m in meshes):
            raise ValueError("every instance must have the same dimension")
        self.nc = self.dim + 2
        self.count = len(meshes)
        L = capi.lib()
        p = capi.idp_params()
        capi.check("idp_default_params", L.idp_default_params(C.byref(p), self.dim))
        p.gamma, p.cfl = float(gamma), float(cfl)
        p.limiter_passes, p.newton_max_iter = int(passes), int(newton_max)
        p.newton_tol = float(newton_tol)
        p.flags = 0 if staging else capi.IDP_FLAG_NO_STAGING
        p.sell_sigma = int(sell_sigma)
        self.params = p
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        K = self.count
        self._keep = []
        co = (capi._dp * K)()
        ce = (capi._i64p * K)()
        hd = (capi._u8p * K)()
        nn = (C.c_int64 * K)()
        ncell = (C.c_int64 * K)()
        for k, m in enumerate(meshes):
            x = np.ascontiguousarray(m.coords, dtype=np.float64)
            c = np.ascontiguousarray(m.cells, dtype=np.int64)
            d = m.boundary if dirichlet is None else dirichlet[k]
            d = np.ascontiguousarray(d, dtype=np.uint8) if d is not None else None
            self._keep += [x, c, d]
            co[k] = x.ctypes.data_as(capi._dp)
            ce[k] = c.ctypes.data_as(capi._i64p)
            hd[k] = d.ctypes.data_as(capi._u8p) if d is not None else None
            nn[k] = x.shape[0]
            ncell[k] = c.shape[0]
        h = C.c_void_p()
        rc = L.idp_create_batch(C.byref(h), C.byref(p), K, nn, co, ncell, ce, hd,
                                C.c_void_p(self._stream.cuda_stream))
        self._keep = None
        capi.check("idp_create_batch", rc)
        self._h = h
        off = np.empty(K + 1, np.int64)
        capi.check("idp_batch_info", L.idp_batch_info(h, None, off.ctypes.data_as(capi._i64p)))
        self.offsets = off
        self.n = int(off[-1])
        nz, nb = C.c_int64(), C.c_size_t()
        capi.check("idp_info", L.idp_info(h, None, C.byref(nz), C.byref(nb)))
        self.nnz = int(nz.value)
        self.device_bytes = int(nb.value)

    close = Solver.close
    __del__ = Solver.__del__
    _u = Solver._u
    set_timing = Solver.set_timing
    kernel_times = Solver.kernel_times

    @staticmethod
    def schedule(kind, tile=0):
        """kind: "launches" or "persistent"."""
        k = {"launches": capi.IDP_SCHED_LAUNCHES, "persistent": capi.IDP_SCHED_PERSISTENT}[kind]
        return capi.idp_schedule(k, int(tile))

    def steps(self, U, n_steps: int, dt=None, schedule=None):
        """n_steps SSP-RK3 steps of every instance in place.  dt: None (each
        instance's CFL tau at every step) or one tau per instance.  Returns
        (tau [n_steps, count], status)."""
        K = self.count
        used = np.zeros((max(int(n_steps), 0), K))
        dta = None
        if dt is not None:
            dta = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, np.float64), (K,)))
        rc = capi.lib().idp_batch_steps(
            self._h, self._u(U), int(n_steps),
            dta.ctypes.data_as(capi._dp) if dta is not None else None,
            used.ctypes.data_as(capi._dp),
            C.byref(schedule) if schedule is not None else None)
        capi.check("idp_batch_steps", rc)
        return used, rc

    def max_dt(self, U) -> np.ndarray:
        out = np.empty(self.count)
        capi.check("idp_batch_max_dt", capi.lib().idp_batch_max_dt(
            self._h, self._u(U), out.ctypes.data_as(capi._dp)))
        return out

    def tune(self, U, n_steps: int = 2):
        """Time every candidate schedule on a scratch copy of U; the fastest
        becomes the default.  Returns (best schedule, {name: ms})."""
        best = capi.idp_schedule()
        ms = np.zeros(16)
        nc = C.c_int()
        capi.check("idp_batch_tune", capi.lib().idp_batch_tune(
            self._h, self._u(U), int(n_steps), C.byref(best), ms.ctypes.data_as(capi._dp),
            C.byref(nc)))
        names = (["launches"] + [f"persistent_tile{t}" for t in (4, 16, 32, 64, 128, 256)] +
                 [f"persistent_{n}_items_per_instance" for n in (8, 32, 128)])
        return best, {names[i]: float(ms[i]) for i in range(nc.value)}


def tune_layout(mesh, U0, steps: int = 2, sigmas=(0, 64), staging=(True, False), **kw):
    """Layout autotuner for one mesh: times `steps` SSP-RK3 steps from U0
    (host array) under every combination of the SELL sorting window
    (`sell_sigma`) and the LDS staging of the row sweeps, each in a fresh
    context, and returns (the fastest combination as Solver keyword
    arguments, {(sigma, staging): ms per step}).  Every combination must
    give the same state bit for bit; a mismatch raises."""
    import time
    torch = _require_torch_gpu()
    times, ref, best = {}, None, None
    for sg in sigmas:
        for st in staging:
            s = Solver(mesh, asynchronous=True, sell_sigma=sg, staging=st, **kw)
            U = torch.tensor(U0, device="cuda")
            s.step(U)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                s.step(U)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            status = s.status()
            s.close()
            if status not in (0, 1):
                raise RuntimeError(f"step failed under sigma={sg}, staging={st}: {status}")
            out = U.cpu().numpy()
            if ref is None:
                ref = out
            elif not np.array_equal(out, ref):
                raise RuntimeError(f"sigma={sg}, staging={st} changed the result")
            times[(sg, st)] = ms
            if best is None or ms < times[best]:
                best = (sg, st)
    return {"sell_sigma": best[0], "staging": best[1]}, times
