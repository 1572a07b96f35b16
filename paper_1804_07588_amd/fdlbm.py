"""Python binding of the HIP library libfdlbm.so (C ABI in include/fdlbm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides the device workspace (one uint8 tensor) and the
stream.  If the library is not built, importing works but creating a `Sim`
raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FDLBM_LIB names another build of the same library (the host-sanitized
# build of build.py, for instance); by default the in-tree libfdlbm.so
LIB_PATH = os.environ.get("FDLBM_LIB") or os.path.join(HERE, "libfdlbm.so")

# constants mirrored from include/fdlbm.h
OK, E_INVALID, E_GEOMETRY, E_ALIGN, E_HIP, E_UNSTABLE, E_STATE = 0, -1, -2, -3, -4, -5, -6
D2Q9, D3Q19 = 2, 3
F64, F32, F16, BF16 = 0, 1, 2, 3  # F16/BF16: 16-bit population storage, FP32 arithmetic
CORR_DIFFUSION, CORR_VISCOUS, CORR_ENERGY, CORR_PRANDTL, CORR_ALL = 1, 2, 4, 8, 15
WALL_REACTIVE, WALL_ISOTHERMAL = 0, 1
FIELD_RHO, FIELD_U, FIELD_T, FIELD_TS, FIELD_POP, FIELD_KIND, FIELD_WALL_R, FIELD_WALL_DE, FIELD_X = range(9)
K_WALL, K_MOMENTS, K_COLLIDE, K_SOLID = range(4)
RATE_PER_NODE, RATE_PER_AREA = 0, 1
SOURCE_LATTICE, SOURCE_FLUX = 0, 1
WALL_ON_NODE, WALL_HALFWAY = 0, 1
KERNEL_NAMES = ["k_wall", "k_moments", "k_collide", "k_solid"]
MAX_SPECIES = 8

EXPORTS = ["fdlbm_create", "fdlbm_destroy", "fdlbm_last_error", "fdlbm_set_geometry",
           "fdlbm_set_species", "fdlbm_set_solid", "fdlbm_set_reaction", "fdlbm_set_flow",
           "fdlbm_workspace_bytes", "fdlbm_bind_workspace", "fdlbm_init_fields", "fdlbm_step",
           "fdlbm_sync", "fdlbm_observe", "fdlbm_get_field", "fdlbm_state_bytes",
           "fdlbm_save_state", "fdlbm_load_state", "fdlbm_set_profiling", "fdlbm_kernel_times",
           "fdlbm_counts", "fdlbm_residual", "fdlbm_set_overlap", "fdlbm_set_prandtl", "fdlbm_set_solid_scheme",
           "fdlbm_set_lj_transport", "fdlbm_batch_create", "fdlbm_batch_destroy",
           "fdlbm_batch_last_error", "fdlbm_batch_workspace_bytes", "fdlbm_batch_bind_workspace",
           "fdlbm_batch_set_active", "fdlbm_batch_step", "fdlbm_batch_set_grid",
           "fdlbm_batch_get_grid", "fdlbm_batch_autotune", "fdlbm_batch_set_overlap",
           "fdlbm_set_sync_check", "fdlbm_last_step", "fdlbm_observe_noalloc", "fdlbm_set_rate_scaling",
           "fdlbm_set_wall_source", "fdlbm_get_field_device", "fdlbm_batch_check",
           "fdlbm_set_wall_position", "fdlbm_add_reaction",
           "fdlbm_set_solid_coupling"]
BATCH_KINDS = ["wall_fast", "wall_slow", "gas_fast", "gas_slow", "collide", "solid"]


class FdlbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fdlbm error {code}: {msg}")
        self.code = code


class Desc(ct.Structure):
    _fields_ = [("lattice", ct.c_int), ("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
                ("periodic", ct.c_int * 3), ("precision", ct.c_int), ("n_species", ct.c_int),
                ("hip_stream", ct.c_void_p)]


class Obs(ct.Structure):
    _fields_ = [("mass", ct.c_double * MAX_SPECIES), ("e_gas", ct.c_double),
                ("e_solid", ct.c_double), ("moles_reacted", ct.c_double),
                ("heat_released", ct.c_double), ("heat_boundary", ct.c_double),
                ("work_body", ct.c_double), ("T_min", ct.c_double), ("T_max", ct.c_double),
                ("u_max", ct.c_double), ("rho_min", ct.c_double), ("Ts_min", ct.c_double),
                ("Ts_max", ct.c_double), ("step", ct.c_int64), ("bad", ct.c_int32),
                ("n_gas", ct.c_int32), ("n_wall", ct.c_int32), ("n_solid", ct.c_int32)]

    def as_dict(self, ns: int) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "mass"}
        d["mass"] = np.array(self.mass[:ns])
        return d


_lib = None


def lib() -> ct.CDLL:
    """Load libfdlbm.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FdlbmError(E_STATE, f"{LIB_PATH} is not built (run paper_1804_07588_amd/build.py)")
        L = ct.CDLL(LIB_PATH)
        vp, dp, i64 = ct.c_void_p, ct.POINTER(ct.c_double), ct.c_int64
        L.fdlbm_create.argtypes = [ct.POINTER(Desc), ct.POINTER(vp)]
        L.fdlbm_destroy.argtypes = [vp]
        L.fdlbm_destroy.restype = None
        L.fdlbm_last_error.argtypes = [vp]
        L.fdlbm_last_error.restype = ct.c_char_p
        L.fdlbm_set_geometry.argtypes = [vp, ct.POINTER(ct.c_uint8), ct.c_int]
        L.fdlbm_set_species.argtypes = [vp, dp, dp, ct.c_double, dp, ct.c_double, ct.c_double,
                                        ct.c_double, ct.c_double, ct.c_double, ct.c_uint]
        L.fdlbm_set_solid.argtypes = [vp, ct.c_double, ct.c_double, dp]
        L.fdlbm_set_reaction.argtypes = [vp, dp, dp, ct.c_double, ct.c_double, ct.c_double,
                                         ct.c_double, ct.c_int, ct.c_double, ct.c_double, ct.c_int]
        L.fdlbm_set_flow.argtypes = [vp, dp, dp, ct.c_double, ct.c_double]
        L.fdlbm_workspace_bytes.argtypes = [vp, ct.POINTER(ct.c_size_t)]
        L.fdlbm_bind_workspace.argtypes = [vp, vp, ct.c_size_t]
        L.fdlbm_init_fields.argtypes = [vp, dp, dp, dp, dp]
        L.fdlbm_step.argtypes = [vp, i64]
        L.fdlbm_sync.argtypes = [vp]
        L.fdlbm_observe.argtypes = [vp, ct.POINTER(Obs)]
        L.fdlbm_observe_noalloc.argtypes = [vp, ct.POINTER(Obs)]
        L.fdlbm_get_field.argtypes = [vp, ct.c_int, ct.c_int, dp]
        L.fdlbm_state_bytes.argtypes = [vp, ct.POINTER(ct.c_size_t)]
        L.fdlbm_save_state.argtypes = [vp, vp, ct.c_size_t]
        L.fdlbm_load_state.argtypes = [vp, vp, ct.c_size_t]
        L.fdlbm_set_profiling.argtypes = [vp, ct.c_int]
        L.fdlbm_kernel_times.argtypes = [vp, dp, ct.POINTER(i64)]
        L.fdlbm_counts.argtypes = [vp, ct.POINTER(i64), ct.POINTER(i64), ct.POINTER(i64)]
        L.fdlbm_residual.argtypes = [vp, dp]
        L.fdlbm_set_overlap.argtypes = [vp, ct.c_int]
        L.fdlbm_set_prandtl.argtypes = [vp, dp]
        L.fdlbm_set_solid_scheme.argtypes = [vp, ct.c_int]
        L.fdlbm_set_lj_transport.argtypes = [vp, dp, ct.c_double, ct.c_double, ct.c_double, ct.c_int, dp, dp]
        L.fdlbm_set_sync_check.argtypes = [vp, i64]
        L.fdlbm_set_rate_scaling.argtypes = [vp, ct.c_int]
        L.fdlbm_set_wall_source.argtypes = [vp, ct.c_int]
        L.fdlbm_set_wall_position.argtypes = [vp, ct.c_int]
        L.fdlbm_add_reaction.argtypes = [vp, dp, dp, ct.c_double, ct.c_double, ct.c_double, ct.c_double]
        L.fdlbm_get_field_device.argtypes = [vp, ct.c_int, ct.c_int, vp]
        L.fdlbm_batch_check.argtypes = [vp, ct.POINTER(ct.c_int), ct.POINTER(i64)]
        L.fdlbm_set_solid_coupling.argtypes = [vp, ct.c_int]
        L.fdlbm_last_step.argtypes = [vp, ct.POINTER(i64)]
        ip = ct.POINTER(ct.c_int)
        L.fdlbm_batch_create.argtypes = [ct.POINTER(vp), ct.c_int, ct.POINTER(vp)]
        L.fdlbm_batch_destroy.argtypes = [vp]
        L.fdlbm_batch_destroy.restype = None
        L.fdlbm_batch_last_error.argtypes = [vp]
        L.fdlbm_batch_last_error.restype = ct.c_char_p
        L.fdlbm_batch_workspace_bytes.argtypes = [vp, ct.POINTER(ct.c_size_t)]
        L.fdlbm_batch_bind_workspace.argtypes = [vp, vp, ct.c_size_t]
        L.fdlbm_batch_set_active.argtypes = [vp, ct.POINTER(ct.c_uint8)]
        L.fdlbm_batch_step.argtypes = [vp, i64]
        L.fdlbm_batch_set_grid.argtypes = [vp, ip, ct.c_int]
        L.fdlbm_batch_get_grid.argtypes = [vp, ip, ip]
        L.fdlbm_batch_autotune.argtypes = [vp, ct.c_int, ip]
        L.fdlbm_batch_set_overlap.argtypes = [vp, ct.c_int]
        _lib = L
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def configure(h, cfg: dict) -> None:
    """Hand a context everything of the configuration dict up to the
    workspace: geometry, species, transport options, solid, reaction and
    flow.  Host-side work only (no HIP call); raises FdlbmError with the
    library's message on a rejected value."""
    L = lib()

    def check(rc: int):
        if rc != OK:
            raise FdlbmError(rc, L.fdlbm_last_error(h).decode())

    mask = np.ascontiguousarray(np.asarray(cfg["mask"], dtype=np.uint8).reshape(-1))
    check(L.fdlbm_set_geometry(h, mask.ctypes.data_as(ct.POINTER(ct.c_uint8)),
                               int(cfg.get("inout", 0))))
    sp = cfg["species"]
    M, mu0, Djk = _arr(sp["M"]), _arr(sp["mu0"]), _arr(sp["Djk0"]).reshape(-1)
    check(L.fdlbm_set_species(h, _d(M), _d(mu0), sp["mu_T_exp"], _d(Djk), sp["D_T_exp"],
                              sp["D_p_exp"], sp["T_ref"], sp["p_ref"], sp["Pr"], int(sp["flags"])))
    if sp.get("Pr_j") is not None:
        prj = _arr(sp["Pr_j"])
        check(L.fdlbm_set_prandtl(h, _d(prj)))
    lj = sp.get("lj")
    if lj is not None:
        eps, omu, omd = _arr(lj["eps_over_k"]), _arr(lj["omega_mu"]), _arr(lj["omega_d"])
        check(L.fdlbm_set_lj_transport(h, _d(eps), lj["T_unit"], lj["tstar_min"], lj["tstar_max"],
                                       len(omu), _d(omu), _d(omd)))
    so = cfg["solid"]
    tbc = _arr(so["T_bc"])
    if so.get("scheme", 0):
        check(L.fdlbm_set_solid_scheme(h, int(so["scheme"])))
    check(L.fdlbm_set_solid(h, so["alpha_s"], so["C_s"], _d(tbc)))
    if so.get("coupling", 0):
        check(L.fdlbm_set_solid_coupling(h, int(so["coupling"])))
    rx = cfg["reaction"]
    nu, order = _arr(rx["nu"]), _arr(rx["order"])
    check(L.fdlbm_set_reaction(h, _d(nu), _d(order), rx["k0"], rx["ea"], rx["T_ref"],
                               rx["dH"], int(rx["wall_mode"]), rx["T_iso"], rx["tol"], int(rx["max_iter"])))
    if rx.get("rate_area"):
        check(L.fdlbm_set_rate_scaling(h, RATE_PER_AREA))
    if rx.get("source_flux"):
        check(L.fdlbm_set_wall_source(h, SOURCE_FLUX))
    if rx.get("halfway"):
        check(L.fdlbm_set_wall_position(h, WALL_HALFWAY))
    for more in rx.get("more", ()):
        # further reactions at every wall node (same keys as the first)
        mnu, mord = _arr(more["nu"]), _arr(more["order"])
        check(L.fdlbm_add_reaction(h, _d(mnu), _d(mord), more["k0"], more["ea"], more["T_ref"], more["dH"]))
    fl = cfg["flow"]
    F, Xin = _arr(fl["F"]), _arr(fl["X_in"])
    check(L.fdlbm_set_flow(h, _d(F), _d(Xin), fl["p_in"], fl["T_in"]))



class RunLog:
    """JSON-lines run log: one object per line, flushed at once, so the log
    of a run that stops is complete up to its last record.  The first line
    ({"event": "open", ...}) carries the caller's metadata; each record
    ({"event": "step", ...}) the step, seconds since the log opened, every
    observable of Sim.observe() and whatever the caller adds (a residual
    dict, a label).  Usable from any object with an observe() method."""

    def __init__(self, path: str, meta: dict | None = None):
        import json
        import time
        self._json, self._time = json, time
        self._t0 = time.perf_counter()
        self._fh = open(path, "a", buffering=1)
        self._write({"event": "open", "unix_time": time.time(), **(meta or {})})

    @staticmethod
    def _plain(v):
        if isinstance(v, np.ndarray):
            return v.tolist()
        if isinstance(v, (np.floating, np.integer)):
            return v.item()
        if isinstance(v, dict):
            return {k: RunLog._plain(x) for k, x in v.items()}
        return v

    def _write(self, obj: dict):
        self._fh.write(self._json.dumps(self._plain(obj), allow_nan=True) + "\n")

    def record(self, sim, **extra):
        o = sim.observe()
        self._write({"event": "step", "step": int(o["step"]), "t": self._time.perf_counter() - self._t0,
                     **o, **extra})

    def close(self):
        if self._fh:
            self._write({"event": "close", "t": self._time.perf_counter() - self._t0})
            self._fh.close()
            self._fh = None


class Sim:
    """One simulation on the current HIP device, built from a workload dict
    (see workloads.py).  precision: F64, F32, or F16 / BF16 (16-bit
    population storage, FP32 arithmetic).  stream: a torch.cuda.Stream or
    None for torch's current stream."""

    def __init__(self, cfg: dict, precision: int = F32, init: dict | None = None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise FdlbmError(E_STATE, "no HIP device available")
        L = lib()
        self.cfg = cfg
        self.ns = len(cfg["species"]["M"])
        self.nx, self.ny, self.nz = cfg["nx"], cfg["ny"], cfg["nz"]
        self.n = self.nx * self.ny * self.nz
        self.Q = 9 if cfg["lattice"] == 2 else 19
        self.precision = precision
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        d = Desc(cfg["lattice"], self.nx, self.ny, self.nz,
                 (ct.c_int * 3)(*[int(p) for p in cfg["periodic"]]), precision, self.ns,
                 ct.c_void_p(self.stream.cuda_stream))
        h = ct.c_void_p()
        rc = L.fdlbm_create(ct.byref(d), ct.byref(h))
        if rc != OK:
            raise FdlbmError(rc, "fdlbm_create rejected the description")
        self.h = h
        configure(h, cfg)
        nbytes = ct.c_size_t()
        self._check(L.fdlbm_workspace_bytes(h, ct.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        ptr = self.workspace.data_ptr()
        aligned = (ptr + 255) & ~255
        self._check(L.fdlbm_bind_workspace(h, ct.c_void_p(aligned), nbytes.value))
        if init is not None:
            self.init_fields(init)

    def _check(self, rc: int):
        if rc != OK:
            raise FdlbmError(rc, lib().fdlbm_last_error(self.h).decode())

    def counts(self) -> tuple[int, int, int]:
        a, b, c = ct.c_int64(), ct.c_int64(), ct.c_int64()
        self._check(lib().fdlbm_counts(self.h, ct.byref(a), ct.byref(b), ct.byref(c)))
        return a.value, b.value, c.value

    def init_fields(self, init: dict):
        rho, u = _arr(init["rho"]).reshape(-1), _arr(init["u"]).reshape(-1)
        T, Ts = _arr(init["T"]), _arr(init["Ts"])
        self._check(lib().fdlbm_init_fields(self.h, _d(rho), _d(u), _d(T), _d(Ts)))

    def step(self, n: int = 1):
        self._check(lib().fdlbm_step(self.h, int(n)))

    def sync(self):
        self._check(lib().fdlbm_sync(self.h))

    def set_sync_check(self, every: int):
        """Check the stability record every `every` steps inside step() (0: off);
        step() then raises FdlbmError with code E_UNSTABLE."""
        self._check(lib().fdlbm_set_sync_check(self.h, int(every)))

    def last_step(self) -> int:
        """First step with a non-finite or negative density or temperature, or -1."""
        v = ct.c_int64()
        self._check(lib().fdlbm_last_step(self.h, ct.byref(v)))
        return v.value

    def observe(self) -> dict:
        o = Obs()
        self._check(lib().fdlbm_observe(self.h, ct.byref(o)))
        return o.as_dict(self.ns)

    def observe_noalloc(self) -> dict:
        """fdlbm_observe_noalloc: the observables without any allocation."""
        o = Obs()
        self._check(lib().fdlbm_observe_noalloc(self.h, ct.byref(o)))
        return o.as_dict(self.ns)

    def field(self, fid: int, comp: int = 0) -> np.ndarray:
        size = self.Q * self.n if fid == FIELD_POP else self.n
        out = np.zeros(size)
        self._check(lib().fdlbm_get_field(self.h, fid, comp, _d(out)))
        return out

    def field_device(self, fid: int, comp: int = 0, out=None):
        """The field as a float64 torch tensor on the device (n values, node
        order), filled on the context's stream without a host round trip;
        `out` (a contiguous float64 device tensor of n values) is reused if
        given."""
        import torch
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() == self.n):
            raise FdlbmError(E_INVALID, "out must be a contiguous float64 device tensor of n values")
        self._check(lib().fdlbm_get_field_device(self.h, fid, comp, ct.c_void_p(out.data_ptr())))
        return out

    def save_state(self) -> bytes:
        nb = ct.c_size_t()
        self._check(lib().fdlbm_state_bytes(self.h, ct.byref(nb)))
        buf = ct.create_string_buffer(nb.value)
        self._check(lib().fdlbm_save_state(self.h, buf, nb.value))
        return buf.raw

    def load_state(self, data: bytes):
        buf = ct.create_string_buffer(data, len(data))
        self._check(lib().fdlbm_load_state(self.h, buf, len(data)))

    def residual(self) -> dict:
        """Steady-state residual since the previous call (inf on the first):
        per field group X, T, u, Ts and their maximum."""
        r = np.zeros(5)
        self._check(lib().fdlbm_residual(self.h, _d(r)))
        return dict(X=r[0], T=r[1], u=r[2], Ts=r[3], max=r[4])

    def set_overlap(self, on: bool):
        self._check(lib().fdlbm_set_overlap(self.h, 1 if on else 0))

    def set_profiling(self, on: bool):
        self._check(lib().fdlbm_set_profiling(self.h, 1 if on else 0))

    def kernel_times(self) -> tuple[dict, int]:
        avg = np.zeros(len(KERNEL_NAMES))
        cnt = ct.c_int64()
        self._check(lib().fdlbm_kernel_times(self.h, _d(avg), ct.byref(cnt)))
        return {name: float(avg[k]) for k, name in enumerate(KERNEL_NAMES)}, cnt.value

    def close(self):
        if getattr(self, "h", None):
            lib().fdlbm_destroy(self.h)
            self.h = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many Sims (same lattice, species count, precision and stream) advanced
    by shared persistent launches replayed from captured HIP graphs.  The
    Sims stay usable on their own (observe, residual, field) between batch
    steps; do not call Sim.step on an active member."""

    def __init__(self, sims: list):
        import torch
        L = lib()
        self.sims = list(sims)
        arr = (ct.c_void_p * len(self.sims))(*[s.h for s in self.sims])
        h = ct.c_void_p()
        rc = L.fdlbm_batch_create(arr, len(self.sims), ct.byref(h))
        if rc != OK:
            raise FdlbmError(rc, L.fdlbm_last_error(self.sims[0].h).decode())
        self.h = h
        nbytes = ct.c_size_t()
        self._check(L.fdlbm_batch_workspace_bytes(h, ct.byref(nbytes)))
        with torch.cuda.stream(self.sims[0].stream):
            self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self._check(L.fdlbm_batch_bind_workspace(h, ct.c_void_p(aligned), nbytes.value))
        self.active = np.ones(len(self.sims), dtype=np.uint8)

    def _check(self, rc: int):
        if rc != OK:
            raise FdlbmError(rc, lib().fdlbm_batch_last_error(self.h).decode())

    def step(self, n: int = 1):
        self._check(lib().fdlbm_batch_step(self.h, int(n)))

    def check(self):
        """Synchronise and read every sample's stability record: None if all
        are sound, else raise FdlbmError (code E_UNSTABLE) whose `sample` and
        `step` name the lowest unstable sample and its first unstable step."""
        s, st = ct.c_int(), ct.c_int64()
        rc = lib().fdlbm_batch_check(self.h, ct.byref(s), ct.byref(st))
        if rc != OK:
            err = FdlbmError(rc, lib().fdlbm_batch_last_error(self.h).decode())
            err.sample, err.step = s.value, st.value
            raise err
        return None

    def set_active(self, active):
        a = np.ascontiguousarray(np.asarray(active, dtype=np.uint8).reshape(-1))
        if a.size != len(self.sims):
            raise ValueError("one flag per sample")
        self._check(lib().fdlbm_batch_set_active(self.h, a.ctypes.data_as(ct.POINTER(ct.c_uint8))))
        self.active = a.copy()

    def set_grid(self, grid=None, graph_steps: int = 0):
        g = None
        if grid is not None:
            g = (ct.c_int * len(BATCH_KINDS))(*[int(v) for v in grid])
        self._check(lib().fdlbm_batch_set_grid(self.h, g, int(graph_steps)))

    def set_overlap(self, on: bool):
        self._check(lib().fdlbm_batch_set_overlap(self.h, 1 if on else 0))

    def grid(self) -> tuple[list, int]:
        g = (ct.c_int * len(BATCH_KINDS))()
        k = ct.c_int()
        self._check(lib().fdlbm_batch_get_grid(self.h, g, ct.byref(k)))
        return list(g), k.value

    def autotune(self, steps: int = 5) -> dict:
        g = (ct.c_int * len(BATCH_KINDS))()
        self._check(lib().fdlbm_batch_autotune(self.h, int(steps), g))
        return dict(zip(BATCH_KINDS, list(g)))

    def close(self):
        if getattr(self, "h", None):
            lib().fdlbm_batch_destroy(self.h)
            self.h = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
