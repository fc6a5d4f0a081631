"""ctypes binding of the C ABI declared in include/gp_spin1.h.

Argument marshalling only: every step of the SSCN path runs in the HIP
kernels of libgp_spin1.so.  PyTorch supplies the device memory (a complex128
or complex64 tensor of shape (3, ny, nx)) and the stream; the library borrows
the tensor's storage for the duration of each call.

The library is loaded on first use and a missing build raises
``LibraryNotBuilt``: there is no fallback of any kind.
"""
import ctypes
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libgp_spin1.so")

GP_OK, GP_EINVAL, GP_EUNSTABLE, GP_ENOMEM, GP_EHIP, GP_ENONFINITE, GP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
GP_FP64, GP_FP32 = 0, 1
GP_YSOLVER_AUTO, GP_YSOLVER_WINDOW, GP_YSOLVER_THOMAS, GP_YSOLVER_CHAIN, GP_YSOLVER_STACK = 0, 1, 2, 3, 4
GP_XSOLVER_AUTO, GP_XSOLVER_SCAN, GP_XSOLVER_WINDOW, GP_XSOLVER_CHAIN = 0, 1, 2, 3
GP_ORDER_AUTO, GP_ORDER_HARDWARE, GP_ORDER_XCD, GP_ORDER_BANDS, GP_ORDER_ROWS = 0, 1, 2, 3, 4
SUB_LOCAL, SUB_X, SUB_Y, SUB_NORMALIZE = 0, 1, 2, 3

# Every entry point the header declares (checked by the CPU test suite).
EXPORTS = ("gp_spin1_create", "gp_spin1_destroy", "gp_spin1_step_imag", "gp_spin1_step_real", "gp_spin1_step_graph",
           "gp_spin1_substep", "gp_spin1_observables", "gp_spin1_sync", "gp_spin1_get_plan",
           "gp_spin1_plan_query", "gp_spin1_timing_enable", "gp_spin1_timing_read",
           "gp_spin1_strerror", "gp_spin1_last_error",
           "gp_spin1_batch_create", "gp_spin1_batch_set_slot", "gp_spin1_batch_step", "gp_spin1_batch_sync",
           "gp_spin1_batch_observables", "gp_spin1_batch_info_read", "gp_spin1_batch_destroy",
           "gp_spin1_batch_last_error", "gp_spin1_serve", "gp_spin1_step_static", "gp_spin1_static_last_error")


class LibraryNotBuilt(RuntimeError):
    pass


class GPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("dt", ctypes.c_double),
                ("c0", ctypes.c_double), ("c2", ctypes.c_double), ("gamma", ctypes.c_double),
                ("eta", ctypes.c_int32), ("rabi", ctypes.c_double), ("omega", ctypes.c_double),
                ("precision", ctypes.c_int32), ("y_solver", ctypes.c_int32),
                ("x_points", ctypes.c_int32), ("y_tile", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("trap_gx", ctypes.c_double), ("trap_gy", ctypes.c_double), ("split", ctypes.c_int32),
                ("fix_magnetization", ctypes.c_int32), ("magnetization", ctypes.c_double),
                ("x_solver", ctypes.c_int32), ("block_order", ctypes.c_int32),
                ("x_tile", ctypes.c_int32), ("plane_stride", ctypes.c_int64)]


class Obs(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double * 3), ("norm_total", ctypes.c_double),
                ("magnetization", ctypes.c_double), ("energy", ctypes.c_double),
                ("e_kin", ctypes.c_double), ("e_trap", ctypes.c_double), ("e_int", ctypes.c_double),
                ("e_rot", ctypes.c_double), ("e_so", ctypes.c_double), ("e_rabi", ctypes.c_double),
                ("lz", ctypes.c_double), ("mu", ctypes.c_double * 3), ("mu_total", ctypes.c_double)]


class Timing(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 4), ("ms", ctypes.c_double * 4)]


TIMING_KINDS = ("x_sweep", "y_sweep", "norm_finalize", "renormalise")


class Plan(ctypes.Structure):
    _fields_ = [("x_points_per_thread", ctypes.c_int32), ("x_threads_per_row", ctypes.c_int32),
                ("x_rows_per_block", ctypes.c_int32), ("y_solver", ctypes.c_int32),
                ("y_halo", ctypes.c_int32), ("y_rows_out", ctypes.c_int32),
                ("y_tile", ctypes.c_int32), ("y_tile_cols", ctypes.c_int32), ("y_segments", ctypes.c_int32),
                ("y_rows_per_thread", ctypes.c_int32), ("pivots_x", ctypes.c_int32),
                ("pivots_y", ctypes.c_int32), ("decay_x", ctypes.c_double), ("decay_y", ctypes.c_double),
                ("stable", ctypes.c_int32), ("x_solver", ctypes.c_int32), ("x_halo", ctypes.c_int32),
                ("x_points_out", ctypes.c_int32), ("x_tile", ctypes.c_int32),
                ("x_block_order", ctypes.c_int32), ("y_block_order", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("x_points", ctypes.c_int32 * 2), ("x_block", ctypes.c_int32 * 2), ("y_tile", ctypes.c_int32 * 2),
                ("grouped", ctypes.c_int32), ("individual", ctypes.c_int32), ("phases", ctypes.c_int32),
                ("launches", ctypes.c_int64), ("x_solver", ctypes.c_int32 * 2), ("y_solver", ctypes.c_int32 * 2),
                ("x_tile", ctypes.c_int32 * 2)]


class Request(ctypes.Structure):
    _fields_ = [("arrival", ctypes.c_double), ("p", Params), ("nsteps", ctypes.c_int64), ("mode", ctypes.c_int32),
                ("psi_dev", ctypes.c_void_p)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_double),
                ("chunk_steps", ctypes.c_int64), ("time_scale", ctypes.c_double)]


class RequestResult(ctypes.Structure):
    _fields_ = [("start", ctypes.c_double), ("finish", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("pt_steps", ctypes.c_double), ("served_rate", ctypes.c_double),
                ("offered_rate", ctypes.c_double), ("p50_latency", ctypes.c_double),
                ("p99_latency", ctypes.c_double), ("mean_latency", ctypes.c_double),
                ("max_latency", ctypes.c_double), ("completed", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("mean_active", ctypes.c_double), ("gpu_busy", ctypes.c_double),
                ("admit_ms", ctypes.c_double)]


_lib = None


def load():
    """Load libgp_spin1.so (built in-tree by ``paper_2105_10517_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise LibraryNotBuilt(f"{LIBPATH} is missing: run `python -m paper_2105_10517_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded
    # (the wave functions are torch allocations; loading the library first
    # can leave two runtimes in the process, and the library's calls fail)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIBPATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "gp_spin1_create": [ctypes.POINTER(Params), vp, ctypes.POINTER(vp)],
        "gp_spin1_destroy": [vp],
        "gp_spin1_step_imag": [vp, vp, i64],
        "gp_spin1_step_real": [vp, vp, i64],
        "gp_spin1_step_graph": [vp, vp, i64, i32],
        "gp_spin1_substep": [vp, vp, i32, i32],
        "gp_spin1_observables": [vp, vp, ctypes.POINTER(Obs), vp],
        "gp_spin1_sync": [vp],
        "gp_spin1_get_plan": [vp, i32, ctypes.POINTER(Plan)],
        "gp_spin1_plan_query": [ctypes.POINTER(Params), i32, ctypes.POINTER(Plan)],
        "gp_spin1_timing_enable": [vp, i32],
        "gp_spin1_timing_read": [vp, ctypes.POINTER(Timing)],
    }
    sig.update({
        "gp_spin1_batch_create": [ctypes.POINTER(Params), i32, vp, ctypes.POINTER(vp)],
        "gp_spin1_batch_set_slot": [vp, i32, ctypes.POINTER(Params)],
        "gp_spin1_batch_step": [vp, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                ctypes.POINTER(ctypes.c_uint8)],
        "gp_spin1_batch_sync": [vp],
        "gp_spin1_batch_observables": [vp, i32, vp, ctypes.POINTER(Obs), vp],
        "gp_spin1_batch_info_read": [vp, ctypes.POINTER(BatchInfo)],
        "gp_spin1_batch_destroy": [vp],
    })
    sig["gp_spin1_serve"] = [ctypes.POINTER(Request), i32, ctypes.POINTER(ServeConfig), vp,
                             ctypes.POINTER(RequestResult), ctypes.POINTER(ServeStats)]
    sig["gp_spin1_step_static"] = [ctypes.POINTER(Params), vp, i64, i32, vp]
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.gp_spin1_strerror.argtypes = [ctypes.c_int]
    lib.gp_spin1_strerror.restype = ctypes.c_char_p
    lib.gp_spin1_last_error.argtypes = [vp]
    lib.gp_spin1_last_error.restype = ctypes.c_char_p
    lib.gp_spin1_batch_last_error.argtypes = [vp]
    lib.gp_spin1_batch_last_error.restype = ctypes.c_char_p
    lib.gp_spin1_static_last_error.argtypes = []
    lib.gp_spin1_static_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def make_params(p: dict, precision: str = "fp64", y_solver: str = "auto", x_points: int = 0, y_tile: int = 0,
                autotune: bool = False, x_solver: str = "auto", block_order: str = "auto", x_tile: int = 0) -> Params:
    """Params from a plain mapping (keys nx, ny, dx, dy, x0, y0, dt, c0, c2,
    gamma, eta, rabi, omega; missing x0/y0 select the default -n d / 2;
    optional gx, gy (trap), split (0 Lie, 1 Strang), fix_m and magnetization)."""
    prec = {"fp64": GP_FP64, "fp32": GP_FP32}[precision]
    ys = {"auto": GP_YSOLVER_AUTO, "window": GP_YSOLVER_WINDOW, "thomas": GP_YSOLVER_THOMAS,
          "chain": GP_YSOLVER_CHAIN, "stack": GP_YSOLVER_STACK}[y_solver]
    return Params(int(p["nx"]), int(p["ny"]), float(p["dx"]), float(p.get("dy", p["dx"])),
                  float(p.get("x0", math.nan)), float(p.get("y0", math.nan)), float(p["dt"]),
                  float(p.get("c0", 0.0)), float(p.get("c2", 0.0)), float(p.get("gamma", 0.0)),
                  int(p.get("eta", 1)), float(p.get("rabi", 0.0)), float(p.get("omega", 0.0)), prec, ys,
                  int(x_points), int(y_tile), int(bool(autotune)), float(p.get("gx", 1.0)), float(p.get("gy", 1.0)),
                  int(p.get("split", 0)), int(bool(p.get("fix_m", 0))), float(p.get("magnetization", 0.0)),
                  {"auto": GP_XSOLVER_AUTO, "scan": GP_XSOLVER_SCAN, "window": GP_XSOLVER_WINDOW,
                   "chain": GP_XSOLVER_CHAIN}[x_solver],
                  {"auto": GP_ORDER_AUTO, "hardware": GP_ORDER_HARDWARE, "xcd": GP_ORDER_XCD,
                   "bands": GP_ORDER_BANDS, "rows": GP_ORDER_ROWS}[block_order],
                  int(x_tile), int(p.get("plane_stride", 0)))


def plane_stride(p: dict) -> int:
    """Elements between the component planes of the wave functions of p."""
    return int(p.get("plane_stride", 0)) or int(p["nx"]) * int(p["ny"])


def check_psi(t, dtype, p: dict, what: str = "psi", device=None):
    """Device pointer of a (3, ny, nx) CUDA tensor whose rows are contiguous
    and whose planes are plane_stride(p) elements apart (contiguous when p
    has no plane_stride), on GPU `device` when given (the handle's)."""
    nx, ny = int(p["nx"]), int(p["ny"])
    if t.dtype != dtype or tuple(t.shape) != (3, ny, nx) or not t.is_cuda or \
            tuple(t.stride()) != (plane_stride(p), nx, 1):
        raise ValueError(f"{what} must be a CUDA {dtype} tensor of shape (3, {ny}, {nx}) with strides "
                         f"({plane_stride(p)}, {nx}, 1)")
    if device is not None and t.device.index != device:
        raise ValueError(f"{what} is on cuda:{t.device.index}, the handle on cuda:{device}")
    return t.data_ptr()


PLANE_PAD = 4160  # elements of padding between planes that padded_psi adds


def padded_psi(psi, p: dict, dtype, device="cuda"):
    """Copy of psi (array-like (3, ny, nx)) on the device with planes
    nx ny + PLANE_PAD elements apart, and p updated with that plane_stride.
    Planes a power of two apart make a sweep's three read (and three write)
    streams fall on the same HBM channels; the pad spreads them."""
    import torch
    nx, ny = int(p["nx"]), int(p["ny"])
    stride = nx * ny + PLANE_PAD
    buf = torch.zeros(2 * stride + nx * ny, dtype=dtype, device=device)
    t = torch.as_strided(buf, (3, ny, nx), (stride, nx, 1))
    t.copy_(torch.as_tensor(psi).to(dtype))
    return t, dict(p, plane_stride=stride)


def _obs_dict(o: Obs) -> dict:
    return {"norm": list(o.norm), "norm_total": o.norm_total, "magnetization": o.magnetization,
            "energy": o.energy, "e_kin": o.e_kin, "e_trap": o.e_trap, "e_int": o.e_int, "e_rot": o.e_rot,
            "e_so": o.e_so, "e_rabi": o.e_rabi, "lz": o.lz, "mu": list(o.mu), "mu_total": o.mu_total}


def plan_query(p: dict, imag: bool, precision: str = "fp64", y_solver: str = "auto", x_points: int = 0,
               y_tile: int = 0, x_solver: str = "auto", block_order: str = "auto", x_tile: int = 0) -> dict:
    """Host-only plan (no GPU needed): pivot table lengths, decay factors,
    y solver and stability flag for these parameters."""
    lib = load()
    pl = Plan()
    pp = make_params(p, precision, y_solver, x_points, y_tile, x_solver=x_solver, block_order=block_order,
                     x_tile=x_tile)
    rc = lib.gp_spin1_plan_query(ctypes.byref(pp), int(bool(imag)), ctypes.byref(pl))
    if rc != GP_OK:
        raise GPError(rc, "gp_spin1_plan_query: " + lib.gp_spin1_strerror(rc).decode())
    return {k: getattr(pl, k) for k, _ in Plan._fields_}


class Solver:
    """One condensate on one stream: a handle of the C ABI."""

    def __init__(self, p: dict, precision: str = "fp64", y_solver: str = "auto", stream=None, x_points: int = 0,
                 y_tile: int = 0, autotune: bool = False, x_solver: str = "auto", block_order: str = "auto",
                 x_tile: int = 0):
        import torch
        self._lib = load()
        self.precision = precision
        self.params = dict(p)
        self.nx, self.ny = int(p["nx"]), int(p["ny"])
        self.dtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.real_dtype = torch.float64 if precision == "fp64" else torch.float32
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = torch.cuda.current_device()  # the handle's GPU (current at creation)
        self._h = ctypes.c_void_p()
        pp = make_params(p, precision, y_solver, x_points, y_tile, autotune, x_solver, block_order, x_tile)
        rc = self._lib.gp_spin1_create(ctypes.byref(pp), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(self._h))
        if rc != GP_OK:
            raise GPError(rc, "gp_spin1_create: " + self._lib.gp_spin1_strerror(rc).decode())

    def _check(self, rc, what):
        if rc != GP_OK:
            msg = self._lib.gp_spin1_last_error(self._h).decode()
            raise GPError(rc, f"{what}: {self._lib.gp_spin1_strerror(rc).decode()}: {msg}")

    def _psi(self, psi):
        return ctypes.c_void_p(check_psi(psi, self.dtype, self.params, device=self.device))

    def step_imag(self, psi, nsteps: int):
        self._check(self._lib.gp_spin1_step_imag(self._h, self._psi(psi), int(nsteps)), "step_imag")

    def step_real(self, psi, nsteps: int):
        self._check(self._lib.gp_spin1_step_real(self._h, self._psi(psi), int(nsteps)), "step_real")

    def step_graph(self, psi, nsteps: int, imag: bool):
        """nsteps steps replayed from a captured HIP graph (captured on the
        first call with these arguments)."""
        self._check(self._lib.gp_spin1_step_graph(self._h, self._psi(psi), int(nsteps), 0 if imag else 1),
                    "step_graph")

    def substep(self, psi, which: int, imag: bool):
        self._check(self._lib.gp_spin1_substep(self._h, self._psi(psi), int(which), int(bool(imag))), "substep")

    def observables(self, psi, dens=None) -> dict:
        o = Obs()
        dp = None
        if dens is not None:
            if dens.dtype != self.real_dtype or tuple(dens.shape) != (3, self.ny, self.nx) or not dens.is_contiguous() \
                    or not dens.is_cuda or dens.device.index != self.device:
                raise ValueError("dens must be a contiguous real CUDA tensor of shape (3, ny, nx) in the solver "
                                 "precision, on the handle's device")
            dp = ctypes.c_void_p(dens.data_ptr())
        self._check(self._lib.gp_spin1_observables(self._h, self._psi(psi), ctypes.byref(o), dp), "observables")
        return _obs_dict(o)

    def sync(self):
        self._check(self._lib.gp_spin1_sync(self._h), "sync")

    def plan(self, imag: bool) -> dict:
        pl = Plan()
        self._check(self._lib.gp_spin1_get_plan(self._h, int(bool(imag)), ctypes.byref(pl)), "get_plan")
        return {k: getattr(pl, k) for k, _ in Plan._fields_}

    def timing(self, enable: bool):
        self._check(self._lib.gp_spin1_timing_enable(self._h, int(bool(enable))), "timing_enable")

    def timing_read(self) -> dict:
        t = Timing()
        self._check(self._lib.gp_spin1_timing_read(self._h, ctypes.byref(t)), "timing_read")
        return {k: {"launches": int(t.launches[i]), "ms": float(t.ms[i])} for i, k in enumerate(TIMING_KINDS)}

    def close(self):
        if self._h:
            self._lib.gp_spin1_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


MODES = {"imag": 0, "real": 1, 0: 0, 1: 1}


def step_static(p: dict, psi, nsteps: int, mode, precision: str = "fp64", stream=None):
    """gp_spin1_step_static: nsteps steps of psi with no device allocation
    (the library's static scratch array; blocks until done)."""
    import torch
    lib = load()
    dtype = torch.complex128 if precision == "fp64" else torch.complex64
    ptr = check_psi(psi, dtype, p, device=torch.cuda.current_device())
    if stream is None:
        stream = torch.cuda.current_stream()
    pp = make_params(p, precision)
    rc = lib.gp_spin1_step_static(ctypes.byref(pp), ctypes.c_void_p(ptr), int(nsteps), MODES[mode],
                                  ctypes.c_void_p(stream.cuda_stream))
    if rc != GP_OK:
        raise GPError(rc, "gp_spin1_step_static: " + lib.gp_spin1_strerror(rc).decode() + ": "
                      + lib.gp_spin1_static_last_error().decode())


class Batch:
    """Independent condensates advanced together (one launch per sweep over
    all of them).  ``params`` holds one parameter mapping per slot, or None
    for an empty slot; every slot has the batch precision and the solver
    requests x_solver / y_solver ("auto": chain shapes when the group fits
    them; "scan" / "window": the whole-row scans and scanned windows)."""

    def __init__(self, params, precision: str = "fp64", stream=None, x_solver: str = "auto", y_solver: str = "auto"):
        import torch
        self._lib = load()
        self.precision = precision
        self.x_solver, self.y_solver = x_solver, y_solver
        self.n = len(params)
        self.dtype = torch.complex128 if precision == "fp64" else torch.complex64
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = torch.cuda.current_device()
        self.params = [dict(p) if p is not None else None for p in params]
        arr = (Params * self.n)(*[self._mk(p) for p in params])
        self._h = ctypes.c_void_p()
        rc = self._lib.gp_spin1_batch_create(arr, self.n, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(self._h))
        if rc != GP_OK:
            raise GPError(rc, "gp_spin1_batch_create: " + self._lib.gp_spin1_strerror(rc).decode())

    def _mk(self, p):
        if p is None:
            q = Params()
            q.precision = {"fp64": GP_FP64, "fp32": GP_FP32}[self.precision]
            return q
        return make_params(p, self.precision, self.y_solver, x_solver=self.x_solver)

    def _check(self, rc, what):
        if rc != GP_OK:
            msg = self._lib.gp_spin1_batch_last_error(self._h).decode()
            raise GPError(rc, f"{what}: {self._lib.gp_spin1_strerror(rc).decode()}: {msg}")

    def set_slot(self, slot: int, p):
        q = self._mk(p)
        self._check(self._lib.gp_spin1_batch_set_slot(self._h, int(slot), ctypes.byref(q)), "batch_set_slot")
        self.params[slot] = dict(p) if p is not None else None

    def _psi(self, slot, psi):
        p = self.params[slot]
        if p is None:
            return psi.data_ptr()  # the library reports the empty slot
        return check_psi(psi, self.dtype, p, f"slot {slot}: psi", device=self.device)

    def step(self, psis, nsteps, modes, active=None):
        """psis[s]: tensor or None (slot skipped); nsteps[s] >= 0; modes[s] in
        {'imag', 'real', 0, 1}; active: optional sequence of booleans."""
        n = self.n
        ptrs = (ctypes.c_void_p * n)()
        ns = (ctypes.c_int64 * n)()
        md = (ctypes.c_int32 * n)()
        ac = (ctypes.c_uint8 * n)()
        for s in range(n):
            on = psis[s] is not None and (active is None or bool(active[s])) and int(nsteps[s]) > 0
            ac[s] = 1 if on else 0
            ns[s] = int(nsteps[s]) if on else 0
            md[s] = MODES[modes[s]] if on else 0
            ptrs[s] = self._psi(s, psis[s]) if on else None
        self._check(self._lib.gp_spin1_batch_step(self._h, ptrs, ns, md, ac), "batch_step")

    def sync(self):
        self._check(self._lib.gp_spin1_batch_sync(self._h), "batch_sync")

    def observables(self, slot: int, psi) -> dict:
        o = Obs()
        self._check(self._lib.gp_spin1_batch_observables(self._h, int(slot), ctypes.c_void_p(self._psi(slot, psi)),
                                                         ctypes.byref(o), None), "batch_observables")
        return _obs_dict(o)

    def info(self) -> dict:
        b = BatchInfo()
        self._check(self._lib.gp_spin1_batch_info_read(self._h, ctypes.byref(b)), "batch_info_read")
        out = {}
        for k, _ in BatchInfo._fields_:
            v = getattr(b, k)
            out[k] = list(v) if k in ("x_points", "x_block", "y_tile", "x_solver", "y_solver", "x_tile") else v
        return out

    def close(self):
        if self._h:
            self._lib.gp_spin1_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def serve(requests, precision: str = "fp32", max_slots: int = 64, hbm_budget_bytes: float = 200e9,
          chunk_steps: int = 250, time_scale: float = 1.0, stream=None):
    """Replay a request trace through the library's serving loop.  Each
    request is a mapping with keys arrival (s), params (mapping), nsteps,
    mode ('imag' / 'real') and psi (device tensor, advanced in place).
    Returns (per-request [(start, finish)], stats dict)."""
    import torch
    lib = load()
    n = len(requests)
    arr = (Request * n)()
    dtype = torch.complex128 if precision == "fp64" else torch.complex64
    device = torch.cuda.current_device()
    for k, r in enumerate(requests):
        p = r["params"]
        t = r["psi"]
        ptr = check_psi(t, dtype, p, f"request {k}: psi", device=device)
        arr[k] = Request(float(r["arrival"]), make_params(p, precision), int(r["nsteps"]), MODES[r["mode"]],
                         ctypes.c_void_p(ptr))
    cfg = ServeConfig(int(max_slots), float(hbm_budget_bytes), int(chunk_steps), float(time_scale))
    out = (RequestResult * n)()
    st = ServeStats()
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = lib.gp_spin1_serve(arr, n, ctypes.byref(cfg), ctypes.c_void_p(stream.cuda_stream), out, ctypes.byref(st))
    if rc != GP_OK:
        raise GPError(rc, "gp_spin1_serve: " + lib.gp_spin1_strerror(rc).decode())
    return [(o.start, o.finish) for o in out], {k: getattr(st, k) for k, _ in ServeStats._fields_}
