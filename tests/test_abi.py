"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/fdlbm.h and include/fdlbm_unet.h, validates its inputs and classifies geometry
like the oracle does.  No call here touches a HIP device."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_1804_07588_amd import fdlbm, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name="fdlbm.h"):
    src = open(os.path.join(ROOT, "include", name)).read()
    return sorted(set(re.findall(r"\b(fdlbm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(fdlbm.LIB_PATH):
        pytest.skip("libfdlbm.so not built")
    return fdlbm.lib()


def test_exports_match_header(L):
    names = header_functions()
    assert len(names) >= 20
    for nme in names:
        assert hasattr(L, nme), nme
    assert sorted(fdlbm.EXPORTS) == names
    from paper_1804_07588_amd import surrogate
    unet = header_functions("fdlbm_unet.h")
    for nme in unet:
        assert hasattr(L, nme), nme
    assert sorted(surrogate.UNET_EXPORTS) == unet


def make_ctx(L, cfg, precision=fdlbm.F64):
    d = fdlbm.Desc(cfg["lattice"], cfg["nx"], cfg["ny"], cfg["nz"],
                   (ct.c_int * 3)(*cfg["periodic"]), precision, len(cfg["species"]["M"]), None)
    h = ct.c_void_p()
    assert L.fdlbm_create(ct.byref(d), ct.byref(h)) == fdlbm.OK
    return h


def set_geom(L, h, cfg):
    m = np.ascontiguousarray(np.asarray(cfg["mask"], np.uint8).reshape(-1))
    return L.fdlbm_set_geometry(h, m.ctypes.data_as(ct.POINTER(ct.c_uint8)), int(cfg["inout"]))


@pytest.mark.parametrize("cfg_name", ["c1", "bed", "noisy2d"])
def test_geometry_counts_match_oracle(L, oracle_lib, cfg_name):
    if cfg_name == "c1":
        cfg = W.channel_c1()
    elif cfg_name == "bed":
        mask, _ = W.sphere_pack_mask(24, radius=3.0, porosity=0.6, seed=5, buffer=4)
        cfg = W.packed_bed(mask=mask)
    else:
        rng = np.random.default_rng(11)
        mask = (rng.random((1, 24, 32)) < 0.3).astype(np.uint8)
        mask[:, :2, :] = 1
        mask[:, -2:, :] = 1
        cfg = W.with_changes(W.channel_c1(), mask=mask, nx=32, ny=24)
    h = make_ctx(L, cfg)
    assert set_geom(L, h, cfg) == fdlbm.OK
    ng, nw, nsol = ct.c_int64(), ct.c_int64(), ct.c_int64()
    assert L.fdlbm_counts(h, ct.byref(ng), ct.byref(nw), ct.byref(nsol)) == fdlbm.OK
    o = oracle_lib.OracleSim(cfg).observe()
    assert (ng.value, nw.value, nsol.value) == (o["n_gas"], o["n_wall"], o["n_solid"])
    L.fdlbm_destroy(h)


def test_invalid_inputs_are_rejected(L):
    cfg = W.channel_c1()
    bad = fdlbm.Desc(7, 4, 4, 1, (ct.c_int * 3)(1, 1, 1), 0, 1, None)
    h = ct.c_void_p()
    assert L.fdlbm_create(ct.byref(bad), ct.byref(h)) == fdlbm.E_INVALID
    h = make_ctx(L, cfg)
    # step / init before the workspace exists
    assert L.fdlbm_step(h, 1) == fdlbm.E_STATE
    dp = ct.POINTER(ct.c_double)
    # unstable solid diffusivity (forward Euler bound 1/(2D))
    assert L.fdlbm_set_solid(h, 0.3, 1.0, None) == fdlbm.E_INVALID
    assert b"alpha_s" in L.fdlbm_last_error(h)
    # masses must be >= 1 (relative to the lightest species)
    M = np.array([0.5, 1.0])
    mu = np.array([0.1, 0.1])
    Dj = np.array([0, 0.05, 0.05, 0.0])
    assert L.fdlbm_set_species(h, M.ctypes.data_as(dp), mu.ctypes.data_as(dp), 0.5,
                               Dj.ctypes.data_as(dp), 1.5, 1.0, 1 / 3, 1 / 3, 1.0, 15) == fdlbm.E_INVALID
    # non-integer reaction order
    nu = np.array([-1.0, 1.0])
    order = np.array([1.5, 0.0])
    assert L.fdlbm_set_reaction(h, nu.ctypes.data_as(dp), order.ctypes.data_as(dp), 1e-3, 0, 1 / 3,
                                -0.1, 0, 1 / 3, 1e-12, 20) == fdlbm.E_INVALID
    # binding before the geometry, then a misaligned workspace
    assert L.fdlbm_bind_workspace(h, ct.c_void_p(256), 1 << 30) == fdlbm.E_STATE
    assert set_geom(L, h, cfg) == fdlbm.OK
    assert L.fdlbm_bind_workspace(h, ct.c_void_p(4096 + 8), 1 << 40) == fdlbm.E_ALIGN
    L.fdlbm_destroy(h)


def test_geometry_errors(L):
    cfg = W.channel_c1()
    h = make_ctx(L, cfg)
    solid = dict(cfg, mask=np.ones((1, 40, 64), np.uint8))
    assert set_geom(L, h, solid) == fdlbm.E_GEOMETRY
    # gas against the closed y edge
    open_edge = dict(cfg, mask=np.zeros((1, 40, 64), np.uint8))
    assert set_geom(L, h, open_edge) == fdlbm.E_GEOMETRY
    L.fdlbm_destroy(h)
