"""ctypes wrapper around the FP64 CPU oracle (oracle/fdlbm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports this module.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SAN_PATH = os.path.join(HERE, "liboracle_san.so")
SOURCES = [os.path.join(HERE, "fdlbm_oracle.c")]

MAXS = 8
OF_RHO, OF_U, OF_T, OF_TS, OF_POP, OF_KIND, OF_WALL_R, OF_WALL_DE = range(8)


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so; with sanitize,
    an AddressSanitizer + UndefinedBehaviorSanitizer build liboracle_san.so
    (load it by naming it in FDLBM_ORACLE_LIB, in a process that preloads
    gcc's libasan)."""
    out = SAN_PATH if sanitize else LIB_PATH
    if force or not os.path.exists(out):
        opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
        cmd = ["gcc", *opt, "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", out + ".tmp",
               *SOURCES, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return out


class Obs(ct.Structure):
    _fields_ = [("mass", ct.c_double * MAXS), ("e_gas", ct.c_double), ("e_solid", ct.c_double),
                ("moles_reacted", ct.c_double), ("heat_released", ct.c_double),
                ("heat_boundary", ct.c_double), ("work_body", ct.c_double),
                ("T_min", ct.c_double), ("T_max", ct.c_double),
                ("u_max", ct.c_double), ("rho_min", ct.c_double), ("Ts_min", ct.c_double),
                ("Ts_max", ct.c_double), ("step", ct.c_int64), ("bad", ct.c_int32),
                ("n_gas", ct.c_int32), ("n_wall", ct.c_int32), ("n_solid", ct.c_int32)]

    def as_dict(self, ns: int) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "mass"}
        d["mass"] = np.array(self.mass[:ns])
        return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("FDLBM_ORACLE_LIB") or LIB_PATH
        if not os.path.exists(path):
            build(sanitize=path == SAN_PATH)
        L = ct.CDLL(path)
        dp = ct.POINTER(ct.c_double)
        L.oracle_create.restype = ct.c_void_p
        L.oracle_create.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                    ct.POINTER(ct.c_int), ct.c_int]
        L.oracle_destroy.argtypes = [ct.c_void_p]
        L.oracle_error.restype = ct.c_char_p
        L.oracle_error.argtypes = [ct.c_void_p]
        L.oracle_set_geometry.argtypes = [ct.c_void_p, ct.POINTER(ct.c_uint8), ct.c_int]
        L.oracle_set_species.argtypes = [ct.c_void_p, dp, dp, ct.c_double, dp, ct.c_double,
                                         ct.c_double, ct.c_double, ct.c_double, ct.c_double,
                                         ct.c_uint]
        L.oracle_set_solid.argtypes = [ct.c_void_p, ct.c_double, ct.c_double, dp]
        L.oracle_set_prandtl.argtypes = [ct.c_void_p, dp]
        L.oracle_set_solid_scheme.argtypes = [ct.c_void_p, ct.c_int]
        L.oracle_set_lj.argtypes = [ct.c_void_p, dp, ct.c_double, ct.c_double, ct.c_double, ct.c_int,
                                    dp, dp]
        L.oracle_set_reaction.argtypes = [ct.c_void_p, dp, dp, ct.c_double, ct.c_double,
                                          ct.c_double, ct.c_double, ct.c_int, ct.c_double,
                                          ct.c_double, ct.c_int]
        L.oracle_set_flow.argtypes = [ct.c_void_p, dp, dp, ct.c_double, ct.c_double]
        L.oracle_set_wall_velocity.argtypes = [ct.c_void_p, dp]
        L.oracle_set_pops.argtypes = [ct.c_void_p, ct.c_int, dp]
        L.oracle_state_bytes.restype = ct.c_size_t
        L.oracle_state_bytes.argtypes = [ct.c_void_p]
        L.oracle_save_state.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t]
        L.oracle_load_state.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_size_t]
        L.oracle_set_literal_eq6.argtypes = [ct.c_void_p, ct.c_int]
        L.oracle_set_rate_area.argtypes = [ct.c_void_p, ct.c_int]
        L.oracle_set_source_flux.argtypes = [ct.c_void_p, ct.c_int]
        L.oracle_set_wall_position.argtypes = [ct.c_void_p, ct.c_int]
        L.oracle_add_reaction.argtypes = [ct.c_void_p, dp, dp, ct.c_double, ct.c_double, ct.c_double,
                                          ct.c_double]
        L.oracle_set_coupling.argtypes = [ct.c_void_p, ct.c_int]
        L.oracle_set_threads.argtypes = [ct.c_int]
        L.oracle_init_fields.argtypes = [ct.c_void_p, dp, dp, dp, dp]
        L.oracle_step.argtypes = [ct.c_void_p, ct.c_int64]
        L.oracle_observe.argtypes = [ct.c_void_p, ct.POINTER(Obs)]
        L.oracle_get_field.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, dp]
        L.oracle_equilibrium.argtypes = [ct.c_int, ct.c_double, ct.c_double, dp, ct.c_double, dp]
        L.oracle_shape.argtypes = [ct.c_int, ct.c_int, dp]
        L.oracle_interp_weights.argtypes = [ct.c_int, ct.c_double, dp, ct.POINTER(ct.c_int),
                                            ct.POINTER(ct.c_int)]
        L.oracle_velocities.argtypes = [ct.c_int, ct.POINTER(ct.c_int)]
        L.oracle_deviations.argtypes = [ct.c_int, ct.c_double, ct.c_double, dp, ct.c_double, dp,
                                        dp, dp]
        L.oracle_transport.argtypes = [ct.c_void_p, dp, ct.c_double, dp, dp]
        _lib = L
    return _lib


def _d(a) -> ct.POINTER(ct.c_double):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def set_threads(n: int) -> int:
    """Threads of the oracle's node loops (results do not depend on it)."""
    return int(lib().oracle_set_threads(int(n)))


def velocities(lattice: int) -> np.ndarray:
    c = (ct.c_int * 57)()
    q = lib().oracle_velocities(lattice, c)
    return np.array(c[:3 * q]).reshape(q, 3)


def equilibrium(lattice: int, rho: float, M: float, u, T: float) -> np.ndarray:
    q = 9 if lattice == 2 else 19
    out = np.zeros(q)
    u3 = _arr(list(u) + [0.0] * (3 - len(u)))
    lib().oracle_equilibrium(lattice, rho, M, _d(u3), T, _d(out))
    return out


def deviations(lattice: int, rho: float, M: float, u, T: float):
    q3, r9 = np.zeros(3), np.zeros(9)
    qxyz = ct.c_double()
    u3 = _arr(list(u) + [0.0] * (3 - len(u)))
    lib().oracle_deviations(lattice, rho, M, _d(u3), T, _d(q3), ct.byref(qxyz), _d(r9))
    return q3, qxyz.value, r9.reshape(3, 3)


def shape(lattice: int, which: int) -> np.ndarray:
    q = 9 if lattice == 2 else 19
    out = np.zeros(q)
    lib().oracle_shape(lattice, which, _d(out))
    return out


def interp_weights(cls: int, s: float):
    w = np.zeros(3)
    t = (ct.c_int * 3)()
    m = ct.c_int()
    lib().oracle_interp_weights(cls, s, _d(w), t, ct.byref(m))
    return w[:m.value], list(t[:m.value])


class OracleSim:
    """One oracle simulation built from a workload dict (see workloads.py)."""

    def __init__(self, cfg: dict, init: dict | None = None):
        L = lib()
        self.cfg = cfg
        self.ns = len(cfg["species"]["M"])
        self.nx, self.ny, self.nz = cfg["nx"], cfg["ny"], cfg["nz"]
        self.n = self.nx * self.ny * self.nz
        self.Q = 9 if cfg["lattice"] == 2 else 19
        per = (ct.c_int * 3)(*[int(p) for p in cfg["periodic"]])
        h = L.oracle_create(cfg["lattice"], self.nx, self.ny, self.nz, per, self.ns)
        if not h:
            raise ValueError("oracle_create failed")
        self.h = h
        mask = np.ascontiguousarray(np.asarray(cfg["mask"], dtype=np.uint8).reshape(-1))
        self._check(L.oracle_set_geometry(h, mask.ctypes.data_as(ct.POINTER(ct.c_uint8)),
                                          int(cfg.get("inout", 0))))
        sp = cfg["species"]
        M, mu0, Djk = _arr(sp["M"]), _arr(sp["mu0"]), _arr(sp["Djk0"]).reshape(-1)
        self._check(L.oracle_set_species(h, _d(M), _d(mu0), sp["mu_T_exp"], _d(Djk), sp["D_T_exp"],
                                         sp["D_p_exp"], sp["T_ref"], sp["p_ref"], sp["Pr"],
                                         int(sp["flags"])))
        if sp.get("Pr_j") is not None:
            prj = _arr(sp["Pr_j"])
            self._check(L.oracle_set_prandtl(h, _d(prj)))
        lj = sp.get("lj")
        if lj is not None:
            eps, omu, omd = _arr(lj["eps_over_k"]), _arr(lj["omega_mu"]), _arr(lj["omega_d"])
            self._check(L.oracle_set_lj(h, _d(eps), lj["T_unit"], lj["tstar_min"], lj["tstar_max"],
                                        len(omu), _d(omu), _d(omd)))
        so = cfg["solid"]
        tbc = _arr(so["T_bc"])
        if so.get("scheme", 0):
            self._check(L.oracle_set_solid_scheme(h, int(so["scheme"])))
        self._check(L.oracle_set_solid(h, so["alpha_s"], so["C_s"], _d(tbc)))
        if so.get("coupling", 0):
            self._check(L.oracle_set_coupling(h, int(so["coupling"])))
        rx = cfg["reaction"]
        nu, order = _arr(rx["nu"]), _arr(rx["order"])
        self._check(L.oracle_set_reaction(h, _d(nu), _d(order), rx["k0"], rx["ea"], rx["T_ref"],
                                          rx["dH"], int(rx["wall_mode"]), rx["T_iso"], rx["tol"],
                                          int(rx["max_iter"])))
        fl = cfg["flow"]
        F, Xin = _arr(fl["F"]), _arr(fl["X_in"])
        self._check(L.oracle_set_flow(h, _d(F), _d(Xin), fl["p_in"], fl["T_in"]))
        if rx.get("rate_area"):
            self._check(L.oracle_set_rate_area(h, 1))
        if rx.get("source_flux"):
            self._check(L.oracle_set_source_flux(h, 1))
        if rx.get("halfway"):
            self._check(L.oracle_set_wall_position(h, 1))
        for more in rx.get("more", ()):
            # further reactions at every wall node (same keys as the first)
            mnu, mord = _arr(more["nu"]), _arr(more["order"])
            self._check(L.oracle_add_reaction(h, _d(mnu), _d(mord), more["k0"], more["ea"], more["T_ref"],
                                              more["dH"]))
        if cfg.get("literal_eq6"):
            self._check(L.oracle_set_literal_eq6(h, 1))
        if cfg.get("wall_u") is not None:
            # per-node wall velocity [3][n] (Eq.(39)'s U_w), read at wall nodes
            wu = _arr(cfg["wall_u"]).reshape(-1)
            assert wu.size == 3 * self.n
            self._wall_u = wu
            self._check(L.oracle_set_wall_velocity(h, _d(wu)))
        if init is not None:
            self.init_fields(init)

    def _check(self, rc: int):
        if rc != 0:
            raise ValueError(lib().oracle_error(self.h).decode())

    def init_fields(self, init: dict):
        rho, u = _arr(init["rho"]).reshape(-1), _arr(init["u"]).reshape(-1)
        T, Ts = _arr(init["T"]), _arr(init["Ts"])
        self._check(lib().oracle_init_fields(self.h, _d(rho), _d(u), _d(T), _d(Ts)))

    def step(self, n: int = 1):
        self._check(lib().oracle_step(self.h, int(n)))

    def observe(self) -> dict:
        o = Obs()
        self._check(lib().oracle_observe(self.h, ct.byref(o)))
        return o.as_dict(self.ns)

    def field(self, fid: int, comp: int = 0) -> np.ndarray:
        size = self.Q * self.n if fid == OF_POP else self.n
        out = np.zeros(size)
        self._check(lib().oracle_get_field(self.h, fid, comp, _d(out)))
        return out

    def set_pops(self, comp: int, g) -> None:
        """Overwrite species comp's populations ([Q*n], the OF_POP layout)."""
        a = _arr(g).reshape(-1)
        assert a.size == self.Q * self.n
        self._check(lib().oracle_set_pops(self.h, int(comp), _d(a)))

    def save_state(self) -> bytes:
        """Checkpoint: populations, solid temperature, the last step's node
        fields and the cumulative counters."""
        nb = lib().oracle_state_bytes(self.h)
        buf = ct.create_string_buffer(nb)
        self._check(lib().oracle_save_state(self.h, buf, nb))
        return buf.raw

    def load_state(self, state: bytes) -> None:
        buf = ct.create_string_buffer(state, len(state))
        self._check(lib().oracle_load_state(self.h, buf, len(state)))

    def transport(self, rho, T):
        t1, t2 = np.zeros(self.ns), np.zeros(self.ns)
        r = _arr(rho)
        self._check(lib().oracle_transport(self.h, _d(r), T, _d(t1), _d(t2)))
        return t1, t2

    def close(self):
        if getattr(self, "h", None):
            lib().oracle_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


R_GAS = 8.314462618


def lattice_units(dx_m: float, T0_K: float, M0_kg_per_mol: float) -> dict:
    """Eq.(28)-(32): velocity scale U' = sqrt(3 R T0 / M0) (the lightest
    species moves one lattice constant per step), length scale L' = dx,
    time scale t' = L'/U', temperature scale T0/(1/3), mu' = D' = kappa' = L'U',
    pressure scale U'^2, density scale 1."""
    U = (3.0 * R_GAS * T0_K / M0_kg_per_mol) ** 0.5
    return dict(U=U, L=dx_m, t=dx_m / U, T=T0_K / (1.0 / 3.0), mu=dx_m * U, D=dx_m * U,
                kappa=dx_m * U, P=U * U, rho=1.0)
