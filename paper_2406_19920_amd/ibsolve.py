"""ctypes binding of libibsolve.so (declared in include/ibsolve.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  The functions keep the C names; ``Solver`` is a small convenience
that owns torch device buffers (constants, workspace) for one plan.  Torch is
used for device memory and streams only.

Importing this module loads the library; if it has not been built, the
import fails loudly (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibsolve.so")

IBS_OK = 0
IBS_ERR_INVALID_ARG = 1
IBS_ERR_UNSUPPORTED = 2
IBS_ERR_WORKSPACE_TOO_SMALL = 3
IBS_ERR_HIP = 4
IBS_ERR_NOT_CONVERGED = 5
IBS_ERR_INCOMPATIBLE_RHS = 6
IBS_ERR_NOT_UPLOADED = 7

IBS_FP64, IBS_REFINED_FP16X2, IBS_REFINED_BF16X3, IBS_REFINED_AUTO = 0, 1, 2, 3
IBS_PERIODIC, IBS_DIRICHLET, IBS_NEUMANN = 0, 1, 2
IBS_OP_POISSON, IBS_OP_HELMHOLTZ_U, IBS_OP_HELMHOLTZ_V, IBS_OP_HELMHOLTZ_W = 0, 1, 2, 3

# every exported entry point of include/ibsolve.h
EXPORTS = ("solver_plan", "solver_plan_bytes", "solver_plan_upload", "solver_plan_destroy",
           "solve_poisson", "solve_poisson_noalloc", "solve_helmholtz_batch", "residual",
           "ibs_divergence", "ibs_wall_data", "ibs_stage_bytes", "ibs_rk_stage",
           "ibs_correct", "ibs_plan_export", "ibs_profile", "ibs_profile_read",
           "ibs_batch_build", "ibs_batch_build_sched", "ibs_batch_autotune", "ibs_batch_build_multigrid",
           "ibs_batch_launch", "ibs_batch_destroy",
           "ibs_autotune_bytes", "ibs_autotune", "ibs_plan_set_tiles",
           "ibs_last_error", "ibs_version")

IBS_NUM_TUNE = 2

PROFILE_KERNELS = ("xgemm_f64", "zgemm_f64", "tridiag_f64", "divergence", "correct", "residual",
                   "xgemm_split", "zgemm_split", "tridiag_f32", "update", "explicit", "ibm")


class ibs_grid_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("beta", ctypes.c_double), ("y_faces", ctypes.POINTER(ctypes.c_double)),
                ("bc_x", ctypes.c_int32), ("bc_z", ctypes.c_int32),
                ("bc_y_vel", ctypes.c_int32), ("bc_y_p", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("strict_compat", ctypes.c_int32),
                ("x_faces", ctypes.POINTER(ctypes.c_double)),
                ("z_faces", ctypes.POINTER(ctypes.c_double))]


class ibs_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("rel_correction", ctypes.c_double),
                ("removed_mean", ctypes.c_double)]


INFO_BYTES = ctypes.sizeof(ibs_solve_info)


class ibs_batch_job(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("op", ctypes.c_int32), ("ncomp", ctypes.c_int32),
                ("comp", ctypes.c_int32 * 3), ("c", ctypes.c_double * 3),
                ("rhs", ctypes.c_void_p * 3), ("x", ctypes.c_void_p * 3),
                ("work", ctypes.c_void_p), ("work_bytes", ctypes.c_size_t),
                ("info", ctypes.c_void_p)]


class ibs_rk_coef(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("zeta", ctypes.c_double), ("dt", ctypes.c_double), ("re", ctypes.c_double)]


class ibs_stage_fields(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("v", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("p", ctypes.c_void_p), ("nu", ctypes.c_void_p), ("nv", ctypes.c_void_p),
                ("nw", ctypes.c_void_p), ("markers", ctypes.c_void_p), ("ud", ctypes.c_void_p),
                ("dvol", ctypes.c_void_p), ("force", ctypes.c_void_p), ("nmarkers", ctypes.c_int32)]


class IbsError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2406_19920_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
    L.solver_plan.argtypes = [ctypes.POINTER(ibs_grid_desc), ctypes.POINTER(vp)]
    L.solver_plan_bytes.argtypes = [vp, i32, i32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.solver_plan_upload.argtypes = [vp, vp, sz, vp]
    L.solver_plan_destroy.argtypes = [vp]
    L.solve_poisson.argtypes = [vp, vp, vp, vp, sz, vp, vp]
    L.solve_poisson_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.solve_helmholtz_batch.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl),
                                        ctypes.POINTER(vp), ctypes.POINTER(vp), vp, sz, vp, vp]
    L.residual.argtypes = [vp, i32, dbl, vp, vp, vp, vp, vp, sz, vp]
    L.ibs_divergence.argtypes = [vp, vp, vp, vp, vp, dbl, vp]
    L.ibs_wall_data.argtypes = [vp, i32, dbl, vp, vp, vp, vp]
    L.ibs_stage_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.ibs_rk_stage.argtypes = [vp, ctypes.POINTER(ibs_rk_coef), ctypes.POINTER(ibs_stage_fields), vp, sz,
                               vp, vp]
    L.ibs_correct.argtypes = [vp, vp, vp, vp, vp, dbl, vp, vp, dbl, vp]
    L.ibs_plan_export.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(sz)]
    L.ibs_profile.argtypes = [vp, i32]
    L.ibs_autotune_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.ibs_autotune.argtypes = [vp, vp, sz, ctypes.POINTER(i32), vp]
    L.ibs_plan_set_tiles.argtypes = [vp, ctypes.POINTER(i32), i32]
    L.ibs_batch_build.argtypes = [ctypes.POINTER(ibs_batch_job), i32, i32, ctypes.POINTER(vp)]
    L.ibs_batch_build_sched.argtypes = [ctypes.POINTER(ibs_batch_job), i32, i32, i32, ctypes.POINTER(vp)]
    L.ibs_batch_build_multigrid.argtypes = [ctypes.POINTER(ibs_batch_job), i32, ctypes.POINTER(vp)]
    L.ibs_batch_autotune.argtypes = [ctypes.POINTER(ibs_batch_job), i32, i32, ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float), vp]
    L.ibs_batch_launch.argtypes = [vp, vp]
    L.ibs_batch_destroy.argtypes = [vp]
    L.ibs_profile_read.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    for name in EXPORTS:
        if name in ("ibs_last_error", "ibs_version"):
            getattr(L, name).restype = ctypes.c_char_p
        else:
            getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def ibs_last_error() -> str:
    return lib.ibs_last_error().decode()


def ibs_version() -> str:
    return lib.ibs_version().decode()


def _check(st: int, where: str):
    if st != IBS_OK:
        raise IbsError(st, where, ibs_last_error())


def make_desc(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0, beta=0.0, y_faces=None,
              precision=IBS_FP64, tol=1e-10, max_iter=0, strict_compat=0,
              bc_x=IBS_PERIODIC, bc_z=IBS_PERIODIC, bc_y_vel=IBS_DIRICHLET,
              bc_y_p=IBS_NEUMANN, x_faces=None, z_faces=None):
    d = ibs_grid_desc()
    d.nx, d.ny, d.nz = nx, ny, nz
    d.lx, d.ly, d.lz = lx, ly, lz
    d.beta = beta
    d._keep = []
    for name, faces in (("y_faces", y_faces), ("x_faces", x_faces), ("z_faces", z_faces)):
        if faces is not None:
            arr = (ctypes.c_double * len(faces))(*[float(t) for t in faces])
            d._keep.append(arr)
            setattr(d, name, ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)))
    d.bc_x, d.bc_z, d.bc_y_vel, d.bc_y_p = bc_x, bc_z, bc_y_vel, bc_y_p
    d.precision, d.tol, d.max_iter, d.strict_compat = precision, tol, max_iter, strict_compat
    return d


def solver_plan(desc: ibs_grid_desc) -> int:
    h = ctypes.c_void_p()
    _check(lib.solver_plan(ctypes.byref(desc), ctypes.byref(h)), "solver_plan")
    return h.value


def solver_plan_bytes(plan: int, op: int, ncomp: int = 1):
    cb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.solver_plan_bytes(plan, op, ncomp, ctypes.byref(cb), ctypes.byref(wb)),
           "solver_plan_bytes")
    return cb.value, wb.value


def solver_plan_upload(plan: int, dev_const: int, nbytes: int, stream: int):
    _check(lib.solver_plan_upload(plan, dev_const, nbytes, stream), "solver_plan_upload")


def solver_plan_destroy(plan: int):
    _check(lib.solver_plan_destroy(plan), "solver_plan_destroy")


def solve_poisson(plan, b, phi, work, work_bytes, info, stream):
    _check(lib.solve_poisson(plan, b, phi, work, work_bytes, info, stream), "solve_poisson")


IBS_NOALLOC_SCRATCH_BYTES = 64 << 20


def solve_poisson_noalloc(plan, b, phi, info, stream):
    _check(lib.solve_poisson_noalloc(plan, b, phi, info, stream), "solve_poisson_noalloc")


def solve_helmholtz_batch(plan, comps, cs, rs, xs, work, work_bytes, info, stream):
    n = len(comps)
    ca = (ctypes.c_int32 * n)(*comps)
    da = (ctypes.c_double * n)(*cs)
    ra = (ctypes.c_void_p * n)(*rs)
    xa = (ctypes.c_void_p * n)(*xs)
    _check(lib.solve_helmholtz_batch(plan, n, ca, da, ra, xa, work, work_bytes, info, stream),
           "solve_helmholtz_batch")


def residual(plan, op, c, x, b, r, norms2, work, work_bytes, stream):
    _check(lib.residual(plan, op, c, x, b, r, norms2, work, work_bytes, stream), "residual")


def ibs_divergence(plan, u, v, w, b, scale, stream):
    _check(lib.ibs_divergence(plan, u, v, w, b, scale, stream), "ibs_divergence")


def ibs_stage_bytes(plan) -> int:
    n = ctypes.c_size_t()
    _check(lib.ibs_stage_bytes(plan, ctypes.byref(n)), "ibs_stage_bytes")
    return n.value


def ibs_rk_stage(plan, coef, fields, work, work_bytes, info, stream):
    _check(lib.ibs_rk_stage(plan, ctypes.byref(coef), ctypes.byref(fields), work, work_bytes, info,
                            stream), "ibs_rk_stage")


def ibs_wall_data(plan, op, c, lo, hi, rhs, stream):
    _check(lib.ibs_wall_data(plan, op, c, lo, hi, rhs, stream), "ibs_wall_data")


def ibs_correct(plan, phi, u, v, w, g, p, lap_phi, cp, stream):
    _check(lib.ibs_correct(plan, phi, u, v, w, g, p, lap_phi, cp, stream), "ibs_correct")


def ibs_plan_export(plan, table: int):
    import numpy as np
    n = ctypes.c_size_t()
    _check(lib.ibs_plan_export(plan, table, None, ctypes.byref(n)), "ibs_plan_export")
    out = np.zeros(n.value)
    _check(lib.ibs_plan_export(plan, table, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(n)), "ibs_plan_export")
    return out


def ibs_profile(plan, enable: bool):
    _check(lib.ibs_profile(plan, 1 if enable else 0), "ibs_profile")


def ibs_profile_read(plan, kernel: int):
    ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib.ibs_profile_read(plan, kernel, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl),
                                ctypes.byref(by)), "ibs_profile_read")
    return dict(ms=ms.value, launches=n.value, flops=fl.value, bytes=by.value)


def ibs_autotune_bytes(plan) -> int:
    n = ctypes.c_size_t()
    _check(lib.ibs_autotune_bytes(plan, ctypes.byref(n)), "ibs_autotune_bytes")
    return n.value


def ibs_autotune(plan, scratch_ptr: int, scratch_bytes: int, stream: int = 0):
    """Time the tile candidates on device; returns the chosen indices."""
    ch = (ctypes.c_int32 * IBS_NUM_TUNE)()
    _check(lib.ibs_autotune(plan, scratch_ptr, scratch_bytes, ch, stream), "ibs_autotune")
    return list(ch)


def ibs_plan_set_tiles(plan, choices):
    arr = (ctypes.c_int32 * len(choices))(*choices)
    _check(lib.ibs_plan_set_tiles(plan, arr, len(choices)), "ibs_plan_set_tiles")


IBS_SCHED_BALANCED, IBS_SCHED_IN_ORDER = 0, 1


def ibs_batch_build(jobs, nlanes: int, policy: int = IBS_SCHED_BALANCED) -> int:
    arr = (ibs_batch_job * len(jobs))(*jobs)
    h = ctypes.c_void_p()
    _check(lib.ibs_batch_build_sched(arr, len(jobs), nlanes, policy, ctypes.byref(h)), "ibs_batch_build_sched")
    return h.value


def ibs_batch_build_multigrid(jobs) -> int:
    """Multi-grid batch: one persistent launch per solve stage over all jobs."""
    arr = (ibs_batch_job * len(jobs))(*jobs)
    h = ctypes.c_void_p()
    _check(lib.ibs_batch_build_multigrid(arr, len(jobs), ctypes.byref(h)), "ibs_batch_build_multigrid")
    return h.value


def ibs_batch_autotune(jobs, reps: int, stream: int):
    """Returns (nlanes, policy, ms per replay) of the fastest schedule."""
    arr = (ibs_batch_job * len(jobs))(*jobs)
    nl, pol, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    _check(lib.ibs_batch_autotune(arr, len(jobs), reps, ctypes.byref(nl), ctypes.byref(pol), ctypes.byref(ms),
                                  stream), "ibs_batch_autotune")
    return nl.value, pol.value, ms.value


def ibs_batch_launch(batch: int, stream: int):
    _check(lib.ibs_batch_launch(batch, stream), "ibs_batch_launch")


def ibs_batch_destroy(batch: int):
    _check(lib.ibs_batch_destroy(batch), "ibs_batch_destroy")


# ---------------------------------------------------------------------------
# torch-owned buffers around one plan
def info_record(row) -> ibs_solve_info:
    """Decode one report record from a device or host float64 row."""
    raw = row.cpu().numpy().tobytes()[:INFO_BYTES]
    return ibs_solve_info.from_buffer_copy(raw)


# ---------------------------------------------------------------------------
class Solver:
    """One plan plus the device buffers it needs (torch allocations)."""

    def __init__(self, nx, ny, nz, device="cuda", plan=None, alloc_work=True, **kw):
        """plan: an already built handle for the same description (ownership
        passes to the Solver); built here when None.  alloc_work=False leaves
        the workspace to the caller (set .work and .work_bytes before use)."""
        import torch
        self.torch = torch
        self.desc = make_desc(nx, ny, nz, **kw)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.plan = plan if plan is not None else solver_plan(self.desc)
        dv = torch.device(device)
        if dv.type == "cuda" and dv.index is None:
            dv = torch.device("cuda", torch.cuda.current_device())
        self.device = dv
        cb, self.work_p = solver_plan_bytes(self.plan, IBS_OP_POISSON)
        _, self.work_h = solver_plan_bytes(self.plan, IBS_OP_HELMHOLTZ_U, 3)
        self.const = torch.empty(cb, dtype=torch.uint8, device=self.device)
        self.work = (torch.empty(max(self.work_p, self.work_h), dtype=torch.uint8, device=self.device)
                     if alloc_work else None)
        self.info = torch.zeros((8, INFO_BYTES // 8), dtype=torch.float64, device=self.device)
        solver_plan_upload(self.plan, self.const.data_ptr(), cb, self.stream())
        self.work_bytes = self.work.numel() if self.work is not None else 0

    def autotune(self):
        """Pick the fastest tile shapes for this grid (bitwise-identical
        results whatever the choice); returns the chosen indices."""
        n = ibs_autotune_bytes(self.plan)
        scratch = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        ch = ibs_autotune(self.plan, scratch.data_ptr(), n, self.stream())
        del scratch
        return ch

    def stream(self) -> int:
        return self.torch.cuda.current_stream(self.device).cuda_stream

    @property
    def periodic_y(self) -> bool:
        """Triply periodic plan: no walls, v has ny faces."""
        return self.desc.bc_y_vel == IBS_PERIODIC

    def shape(self, op=IBS_OP_POISSON):
        walls = op == IBS_OP_HELMHOLTZ_V and not self.periodic_y
        return (self.nz, self.ny + 1 if walls else self.ny, self.nx)

    def empty(self, op=IBS_OP_POISSON):
        return self.torch.empty(self.shape(op), dtype=self.torch.float64, device=self.device)

    def _chk(self, t, op):
        assert t.dtype == self.torch.float64 and t.is_contiguous() and t.device == self.device
        assert tuple(t.shape) == self.shape(op), (tuple(t.shape), self.shape(op))

    def _info_ptr(self, info, slot, n):
        """Device address of n report records: rows of `info` (a float64
        tensor [>= n][INFO_BYTES/8] of the caller's) or the Solver's own."""
        if info is None:
            return self.info[slot].data_ptr()
        assert info.dtype == self.torch.float64 and info.is_contiguous() and info.device == self.device
        assert info.shape[0] >= n and info.shape[1] * 8 >= INFO_BYTES
        return info.data_ptr()

    def poisson(self, b, phi=None, info=None):
        self._chk(b, IBS_OP_POISSON)
        phi = self.empty() if phi is None else phi
        self._chk(phi, IBS_OP_POISSON)
        solve_poisson(self.plan, b.data_ptr(), phi.data_ptr(), self.work.data_ptr(),
                      self.work_bytes, self._info_ptr(info, 0, 1), self.stream())
        return phi

    def helmholtz(self, comps, cs, rs, xs=None, info_slot=0, info=None):
        ops = [c + 1 for c in comps]
        if xs is None:
            xs = [self.empty(op) for op in ops]
        for r, x, op in zip(rs, xs, ops):
            self._chk(r, op)
            self._chk(x, op)
        solve_helmholtz_batch(self.plan, list(comps), list(cs), [r.data_ptr() for r in rs],
                              [x.data_ptr() for x in xs], self.work.data_ptr(), self.work_bytes,
                              self._info_ptr(info, info_slot, len(comps)), self.stream())
        return xs

    def residual(self, op, c, x, b, r=None, norms=False):
        r = self.empty(op) if r is None else r
        n2 = self.torch.zeros(2, dtype=self.torch.float64, device=self.device) if norms else None
        residual(self.plan, op, c, x.data_ptr(), b.data_ptr(), r.data_ptr(),
                 n2.data_ptr() if n2 is not None else None, self.work.data_ptr(),
                 self.work_bytes, self.stream())
        return (r, n2) if norms else r

    def divergence(self, u, v, w, scale=1.0, b=None):
        b = self.empty() if b is None else b
        ibs_divergence(self.plan, u.data_ptr(), v.data_ptr(), w.data_ptr(), b.data_ptr(), scale,
                       self.stream())
        return b

    def rk_stage(self, u, v, w, p, nu, nv, nw, coef, markers=None, ud=None, dvol=None, force=None,
                 work=None, info_slot=4):
        """One Runge-Kutta sub-step in place on u, v, w, p (eqs. a-h); nu, nv,
        nw: N of the stage before on input (read when zeta != 0), N of the
        input velocity on output.  coef: dict alpha, beta, gamma, zeta, dt,
        re.  Marker arrays: device tensors [nm][3], [nm][3], [nm] (and
        force [nm][3] or None).  Reports in info slots info_slot..+3."""
        torch = self.torch
        for t, op in ((u, 1), (v, 2), (w, 3), (p, 0), (nu, 1), (nv, 2), (nw, 3)):
            self._chk(t, op)
        c = ibs_rk_coef(coef["alpha"], coef["beta"], coef["gamma"], coef["zeta"], coef["dt"], coef["re"])
        f = ibs_stage_fields()
        f.u, f.v, f.w, f.p = u.data_ptr(), v.data_ptr(), w.data_ptr(), p.data_ptr()
        f.nu, f.nv, f.nw = nu.data_ptr(), nv.data_ptr(), nw.data_ptr()
        nm = 0 if markers is None else int(markers.shape[0])
        if nm:
            for t in (markers, ud, dvol):
                assert t.dtype == torch.float64 and t.is_contiguous() and t.device == self.device
            f.markers, f.ud, f.dvol = markers.data_ptr(), ud.data_ptr(), dvol.data_ptr()
            f.force = force.data_ptr() if force is not None else None
        f.nmarkers = nm
        nb = ibs_stage_bytes(self.plan)
        if work is None:
            if getattr(self, "_stage_work", None) is None or self._stage_work.numel() < nb:
                self._stage_work = torch.empty(nb, dtype=torch.uint8, device=self.device)
            work = self._stage_work
        ibs_rk_stage(self.plan, c, f, work.data_ptr(), work.numel(), self.info[info_slot].data_ptr(),
                     self.stream())

    def wall_data(self, op, rhs, lo=None, hi=None, c=0.0):
        """Add the wall data's contribution to rhs in place (lo, hi:
        [nz][nx] device tensors or None)."""
        self._chk(rhs, op)
        for d in (lo, hi):
            if d is not None:
                assert d.dtype == self.torch.float64 and d.is_contiguous()
                assert tuple(d.shape) == (self.nz, self.nx)
        ibs_wall_data(self.plan, op, c, lo.data_ptr() if lo is not None else None,
                      hi.data_ptr() if hi is not None else None, rhs.data_ptr(), self.stream())
        return rhs

    def correct(self, phi, u, v, w, g, p=None, lap_phi=None, cp=0.0):
        ibs_correct(self.plan, phi.data_ptr(), u.data_ptr(), v.data_ptr(), w.data_ptr(), g,
                    p.data_ptr() if p is not None else None,
                    lap_phi.data_ptr() if lap_phi is not None else None, cp, self.stream())

    def poisson_job(self, b, phi, info_slot=0, work=None):
        """An ibs_batch_job record for a Poisson solve (buffers must outlive the
        batch); work: a workspace tensor of its own instead of the solver's."""
        self._chk(b, IBS_OP_POISSON)
        self._chk(phi, IBS_OP_POISSON)
        j = ibs_batch_job()
        j.plan, j.op, j.ncomp = self.plan, IBS_OP_POISSON, 1
        j.rhs[0], j.x[0] = b.data_ptr(), phi.data_ptr()
        if work is None:
            j.work, j.work_bytes = self.work.data_ptr(), self.work_bytes
        else:
            j.work, j.work_bytes = work.data_ptr(), work.numel() * work.element_size()
        j.info = self.info[info_slot].data_ptr()
        return j

    def helmholtz_job(self, comps, cs, rs, xs, info_slot=0):
        """An ibs_batch_job record for a Helmholtz batch (info slots info_slot..)."""
        j = ibs_batch_job()
        j.plan, j.op, j.ncomp = self.plan, IBS_OP_HELMHOLTZ_U, len(comps)
        for q, (cp, cv, r, x) in enumerate(zip(comps, cs, rs, xs)):
            self._chk(r, cp + 1)
            self._chk(x, cp + 1)
            j.comp[q], j.c[q], j.rhs[q], j.x[q] = cp, cv, r.data_ptr(), x.data_ptr()
        j.work, j.work_bytes = self.work.data_ptr(), self.work_bytes
        j.info = self.info[info_slot].data_ptr()
        return j

    def read_info(self, q=0):
        return info_record(self.info[q])

    def new_info(self, n=4):
        """A zeroed device buffer for n report records (see _info_ptr)."""
        return self.torch.zeros((n, INFO_BYTES // 8), dtype=self.torch.float64, device=self.device)

    def close(self):
        if self.plan:
            solver_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
