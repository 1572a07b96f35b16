"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only *generates inputs*: geometry masks, species/transport tables
and initial states.  It contains none of the method's arithmetic (no
equilibria, no interpolation, no boundary rule), so that the GPU library and
the CPU oracle can both be fed from it without sharing any of the scheme.

Geometries follow the paper's setups: a straight channel between solid walls
(Sec. 5, the quasi-1D and 2D channel benchmarks) and a random porous bed
(Sec. 6 uses three cubes; here overlapping spheres generalise it to 3-D).
Units are lattice units throughout: the lightest species has mass 1 and
lattice speed 1, the reference temperature is 1/3 (Sec. 4.1, units paragraph).
"""
from __future__ import annotations

import copy
import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood 2014): the published 64-bit mixer."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


# ---------------------------------------------------------------------------
# geometry masks: uint8, 0 = gas, 1 = solid, x fastest (index x + nx*(y + ny*z))
# ---------------------------------------------------------------------------

def channel_mask(nx: int, ny: int, wall: int, nz: int = 1) -> np.ndarray:
    """Channel along x bounded by `wall` solid rows at both y ends."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[:, :wall, :] = 1
    m[:, ny - wall:, :] = 1
    return m


def slab_mask(nx: int, ny: int, solid_lo: int, solid_hi: int, nz: int = 1) -> np.ndarray:
    """Solid for y in [solid_lo, solid_hi), gas elsewhere (periodic slab stack)."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[:, solid_lo:solid_hi, :] = 1
    return m


def sphere_pack_mask(n: int = 128, radius: float = 6.0, porosity: float = 0.6,
                     seed: int = 12345, buffer: int = 8, ny: int | None = None,
                     nz: int | None = None, fill_closed: bool = True) -> tuple[np.ndarray, int]:
    """Random overlapping spheres in a box of n (x) by ny by nz nodes.

    Sphere centres are i.i.d. uniform over the bed x in [buffer, n-buffer),
    y in [0, ny), z in [0, nz), drawn three SplitMix64 doubles per sphere in
    (x, y, z) order.  A node is solid when its squared distance to a centre is
    <= radius**2, with y and z periodic and x clipped to the bed.  Spheres are
    added until the gas fraction of the bed region drops to `porosity` or below.
    The `buffer` planes at both x ends stay gas (inlet / outlet buffers).
    With `fill_closed`, gas cavities with no lattice path to the inlet plane
    are then filled (fill_closed_pores).
    Returns (mask[nz, ny, nx], number of spheres placed).
    """
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    nx = n
    rng = SplitMix64(seed)
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    x0, x1 = buffer, nx - buffer
    bed_nodes = (x1 - x0) * ny * nz
    solid = 0
    r = radius
    ri = int(np.ceil(r))
    off = np.arange(-ri, ri + 1)
    dz, dy, dx = np.meshgrid(off, off, off, indexing="ij")
    placed = 0
    while True:
        cx = x0 + rng.uniform() * (x1 - x0)
        cy = rng.uniform() * ny
        cz = rng.uniform() * nz
        ix = np.floor(cx).astype(int) + dx
        iy = np.floor(cy).astype(int) + dy
        iz = np.floor(cz).astype(int) + dz
        d2 = (ix - cx) ** 2 + (iy - cy) ** 2 + (iz - cz) ** 2
        sel = (d2 <= r * r) & (ix >= x0) & (ix < x1)
        xs = ix[sel]
        ys = np.mod(iy[sel], ny)
        zs = np.mod(iz[sel], nz)
        newly = m[zs, ys, xs] == 0
        solid += int(np.count_nonzero(newly))
        m[zs, ys, xs] = 1
        placed += 1
        if (bed_nodes - solid) / bed_nodes <= porosity:
            break
    if fill_closed:
        m = fill_closed_pores(m, periodic=(0, 1, 1))
    return m, placed


def _link_offsets(dims: int) -> list[tuple[int, int, int]]:
    """(dz, dy, dx) of the D2Q9 / D3Q19 links: face and edge neighbours."""
    out = []
    rng = (-1, 0, 1)
    for dz in (rng if dims == 3 else (0,)):
        for dy in rng:
            for dx in rng:
                k = abs(dx) + abs(dy) + abs(dz)
                if 0 < k <= 2:
                    out.append((dz, dy, dx))
    return out


def fill_closed_pores(mask: np.ndarray, periodic=(0, 1, 1)) -> np.ndarray:
    """Turn gas that no lattice path joins to the x = 0 plane into solid.

    Connectivity is that of the lattice links (face and edge neighbours, the
    D3Q19 / D2Q9 velocity set), across the periodic y / z faces where
    `periodic` (x, y, z flags) says so.  Closed cavities, often single nodes
    walled in by overlapping spheres, exchange nothing with the flow; they are
    standard pore-space preprocessing debris, so they are removed.
    """
    from scipy import ndimage

    nz, ny, nx = mask.shape
    dims = 2 if nz == 1 else 3
    gas = mask == 0
    st = ndimage.generate_binary_structure(3, 2)
    if dims == 2:
        st[0] = False
        st[2] = False
    lab, nl = ndimage.label(gas, structure=st)
    parent = np.arange(nl + 1)

    def find(a: int) -> int:
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    # links that wrap across a periodic face join labels the plain labelling split
    for dz, dy, dx in _link_offsets(dims):
        nb = np.roll(lab, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
        ok = (lab > 0) & (nb > 0) & (lab != nb)
        for ax, d, per, size in ((2, dx, periodic[0], nx), (1, dy, periodic[1], ny),
                                 (0, dz, periodic[2], nz)):
            if d != 0 and not per:
                idx = [slice(None)] * 3
                idx[ax] = size - 1 if d > 0 else 0
                ok[tuple(idx)] = False
        for a, b in set(zip(lab[ok].tolist(), nb[ok].tolist())):
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(a) for a in range(nl + 1)])
    keep = np.zeros(nl + 1, dtype=bool)
    keep[np.unique(roots[lab[:, :, 0][lab[:, :, 0] > 0]])] = True
    keep[0] = False
    open_gas = keep[roots[lab]]
    out = mask.copy()
    out[gas & ~open_gas] = 1
    return out


# ---------------------------------------------------------------------------
# parameter sets (plain numbers; see the module docstring for units)
# ---------------------------------------------------------------------------

# Correction-term switches (bit flags, same values in the C-ABI header).
CORR_DIFFUSION = 1   # diffusion-velocity correction (momentum)
CORR_VISCOUS = 2     # third-moment deviation correction
CORR_ENERGY = 4      # energy-flux deviation correction
CORR_PRANDTL = 8     # variable-Prandtl-number correction
CORR_ALL = 15

WALL_REACTIVE = 0
WALL_ISOTHERMAL = 1


def channel_c1(nx: int = 64, ny: int = 40, wall: int = 4, pr: float = 1.0) -> dict:
    """2-D D2Q9 channel, species A and B (both mass 1), A -> B first order.

    Gas rows wall..ny-wall-1, solid rows at both ends, x periodic, outer
    solid faces held at T0 = 1/3.  tau1 = 0.3 (mu0 = tau1*C*T0 with C = 1),
    tau2 = 0.15 (D_AB = tau2*T0/M), solid volumetric heat capacity 100x the
    gas value (c_p per mole is 2 in 2-D), solid/gas conductivity ratio 10.
    """
    T0 = 1.0 / 3.0
    tau1, tau2 = 0.3, 0.15
    mu0 = tau1 * 1.0 * T0
    dab = tau2 * T0 / 1.0
    kappa_f = (2 + 2) * tau1 * 1.0 * T0 / (2 * 1.0 * pr)
    cs = 100.0 * 2.0
    return dict(
        lattice=2, nx=nx, ny=ny, nz=1, periodic=(1, 0, 1),
        mask=channel_mask(nx, ny, wall),
        inout=0,
        species=dict(names=["A", "B"], M=[1.0, 1.0], mu0=[mu0, mu0], mu_T_exp=0.5,
                     Djk0=[[0.0, dab], [dab, 0.0]], D_T_exp=1.5, D_p_exp=1.0,
                     T_ref=T0, p_ref=T0, Pr=pr, flags=CORR_ALL),
        solid=dict(alpha_s=10.0 * kappa_f / cs, C_s=cs,
                   T_bc=[float("nan"), float("nan"), T0, T0, float("nan"), float("nan")]),
        reaction=dict(nu=[-1.0, 1.0], order=[1.0, 0.0], k0=1e-3, ea=0.0, T_ref=T0,
                      dH=-0.1, wall_mode=WALL_REACTIVE, T_iso=T0, tol=1e-13, max_iter=64),
        flow=dict(F=[1e-6, 0.0, 0.0], X_in=[1.0 - 1e-6, 1e-6], p_in=T0, T_in=T0),
        init=dict(X=[1.0 - 1e-6, 1e-6], C=1.0, T=T0, Ts=T0, u=[0.0, 0.0, 0.0]),
    )


def channel_two_reactions(kind: str = "parallel", k: tuple = (1e-2, 5e-3), dH: tuple = (-0.1, -0.04),
                          M: tuple = (1.0, 1.0, 1.0)) -> dict:
    """The D2Q9 channel with three species A, B, C and two first-order surface
    reactions at every wall node: A -> B and A -> C ("parallel") or A -> B and
    B -> C ("consecutive"); rate constants k, reaction enthalpies dH; inlet
    and initial mole fractions 0.6, 0.25, 0.15."""
    cfg = channel_c1()
    T0 = 1.0 / 3.0
    mu0 = cfg["species"]["mu0"][0]
    dab = cfg["species"]["Djk0"][0][1]
    X = [0.6, 0.25, 0.15]
    cfg["species"].update(names=["A", "B", "C"], M=list(M), mu0=[mu0 * float(np.sqrt(m)) for m in M],
                          Djk0=[[0.0 if a == b else dab for b in range(3)] for a in range(3)])
    second = ([-1.0, 0.0, 1.0], [1.0, 0.0, 0.0]) if kind == "parallel" else ([0.0, -1.0, 1.0], [0.0, 1.0, 0.0])
    cfg["reaction"].update(nu=[-1.0, 1.0, 0.0], order=[1.0, 0.0, 0.0], k0=k[0], ea=0.0, T_ref=T0, dH=dH[0],
                           more=[dict(nu=second[0], order=second[1], k0=k[1], ea=0.0, T_ref=T0, dH=dH[1])])
    cfg["flow"]["X_in"] = list(X)
    cfg["init"]["X"] = list(X)
    return cfg


# Water-gas shift species (masses relative to H2, Sec. 4.4 / Sec. 6).
WGS_NAMES = ["CO", "H2O", "CO2", "H2", "N2"]
WGS_M = [14.0, 9.0, 22.0, 1.0, 14.0]


def packed_bed(n: int = 128, radius: float = 6.0, porosity: float = 0.6,
               seed: int = 12345, buffer: int = 8, mask: np.ndarray | None = None,
               k0: float = 1e-3, force: float = 1e-5, mu_scale: float = 0.0218,
               d_scale: float = 0.0471, trace: float = 1e-4) -> dict:
    """3-D D3Q19 packed bed with water-gas-shift chemistry on the sphere surfaces.

    Species CO, H2O, CO2, H2, N2 (masses 14, 9, 22, 1, 14 relative to H2);
    inlet mole fractions 0.1, 0.3, `trace`, `trace` (products start as traces:
    a zero density has no species velocity), rest N2; T0 = 1/3 (403 K),
    C = 1.  Rate r = k0 exp[ea (1 - T_ref/T_w)] C_CO C_H2O with ea = 84 kJ/mol /
    (R 403 K) = 25.07, reaction enthalpy -4.1 kJ/mol = -0.408 lattice units
    (one lattice energy per mole = 3 R 403 K).  Synthetic transport:
    mu_j = mu_scale * sqrt(M_j) (T/T0)^0.5 and
    D_jk = d_scale * sqrt((1/M_j + 1/M_k)/2) (T/T0)^1.5 (p0/p), Pr = 0.71.
    Flow is driven by a body force along x; the x ends are inlet / outlet.
    The wall rate is taken per unit wetted area (rate_area): a sphere pack
    has the concave corners and one-link wall nodes the paper's walls avoid.
    """
    T0 = 1.0 / 3.0
    if mask is None:
        mask, _ = sphere_pack_mask(n, radius, porosity, seed, buffer)
    M = WGS_M
    ns = len(M)
    djk = [[0.0 if j == k else d_scale * float(np.sqrt(0.5 * (1.0 / M[j] + 1.0 / M[k])))
            for k in range(ns)] for j in range(ns)]
    X_in = [0.1, 0.3, trace, trace]
    X_in.append(1.0 - sum(X_in))
    cs = 100.0 * 2.5
    nz, ny, nx = mask.shape
    return dict(
        lattice=3, nx=nx, ny=ny, nz=nz, periodic=(0, 1, 1),
        mask=mask, inout=1,
        species=dict(names=list(WGS_NAMES), M=list(M),
                     mu0=[mu_scale * float(np.sqrt(m)) for m in M], mu_T_exp=0.5,
                     Djk0=djk, D_T_exp=1.5, D_p_exp=1.0, T_ref=T0, p_ref=T0, Pr=0.71,
                     flags=CORR_ALL),
        solid=dict(alpha_s=0.03, C_s=cs, T_bc=[float("nan")] * 6),
        reaction=dict(nu=[-1.0, -1.0, 1.0, 1.0, 0.0], order=[1.0, 1.0, 0.0, 0.0, 0.0],
                      k0=k0, ea=84000.0 / (8.314462618 * 403.0), T_ref=T0, dH=-0.408,
                      wall_mode=WALL_REACTIVE, T_iso=T0, tol=1e-7, max_iter=32,
                      rate_area=True),
        flow=dict(F=[force, 0.0, 0.0], X_in=X_in, p_in=T0, T_in=T0),
        init=dict(X=list(X_in), C=1.0, T=T0, Ts=T0, u=[0.0, 0.0, 0.0]),
    )


def batch_beds(count: int = 64, n_min: int = 48, n_max: int = 96, por_min: float = 0.4,
               por_max: float = 0.7, seed: int = 2024, radius: float = 6.0, buffer: int = 8,
               **bed_kw) -> list[dict]:
    """`count` packed beds of uneven size for batched runs: per sample three
    SplitMix64 draws give the cube edge (uniform integer in [n_min, n_max]),
    the bed porosity (uniform in [por_min, por_max)) and the seed of its
    sphere pack.  Each is a packed_bed() workload (same chemistry and
    transport); `bed_kw` passes further packed_bed arguments.  The body force
    is scaled with the Kozeny-Carman permeability, eps^3 / (1 - eps)^2, from
    the reference bed (porosity 0.6, force 1e-5), so that every sample flows
    at about the reference speed (peak near 0.03): a fixed force would drive
    the open beds several times faster, beyond the speeds the scheme holds
    for the heavy species (lattice sound speed 0.12 for CO2).  The force is
    capped at 3e-5: the tight beds' throats run faster than their mean."""
    rng = SplitMix64(seed)
    out = []
    kc = lambda e: e ** 3 / (1.0 - e) ** 2
    for _ in range(count):
        n = n_min + int(rng.uniform() * (n_max - n_min + 1))
        por = por_min + rng.uniform() * (por_max - por_min)
        s = int(rng.next_u64() & 0x7FFFFFFF)
        mask, _ = sphere_pack_mask(n, radius=radius, porosity=por, seed=s, buffer=buffer)
        kw = dict(bed_kw)
        kw.setdefault("force", min(1e-5 * kc(0.6) / kc(por), 3e-5))
        cfg = packed_bed(mask=mask, **kw)
        cfg["sample"] = dict(n=n, porosity=por, seed=s)
        out.append(cfg)
    return out


def with_changes(cfg: dict, **sections) -> dict:
    """Deep copy of `cfg` with the given sub-dict entries replaced."""
    out = copy.deepcopy(cfg)
    for sec, upd in sections.items():
        if isinstance(upd, dict) and isinstance(out.get(sec), dict):
            out[sec].update(upd)
        else:
            out[sec] = upd
    return out


def uniform_init(cfg: dict) -> dict:
    """Per-node initial arrays (rho_j, u, T, Ts) from cfg['init'], float64."""
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    M = np.asarray(cfg["species"]["M"], dtype=np.float64)
    X = np.asarray(cfg["init"]["X"], dtype=np.float64)
    C = cfg["init"]["C"]
    rho = np.repeat((M * X * C)[:, None], n, axis=1)
    u = np.repeat(np.asarray(cfg["init"]["u"], dtype=np.float64)[:, None], n, axis=1)
    T = np.full(n, cfg["init"]["T"], dtype=np.float64)
    Ts = np.full(n, cfg["init"]["Ts"], dtype=np.float64)
    return dict(rho=rho, u=u, T=T, Ts=Ts)


def perturbed_init(cfg: dict, seed: int, amp_rho: float = 0.02, amp_u: float = 0.01,
                   amp_T: float = 0.01) -> dict:
    """Uniform state plus seeded smooth random perturbations (for parity runs).

    Perturbations are sums of a few low Fourier modes with SplitMix64 phases,
    so fields are smooth on the lattice scale like a developing flow.
    """
    base = uniform_init(cfg)
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    rng = SplitMix64(seed)
    # broadcast views instead of full coordinate grids (same values)
    z, y, x = (np.arange(nz)[:, None, None], np.arange(ny)[None, :, None], np.arange(nx)[None, None, :])

    def field(amp):
        f = np.zeros((nz, ny, nx))
        for _ in range(3):
            kx, ky, kz = (1 + int(rng.uniform() * 2)), (1 + int(rng.uniform() * 2)), \
                (1 + int(rng.uniform() * 2))
            ph = 2 * np.pi * rng.uniform()
            a = amp * (0.5 + rng.uniform())
            f += a * np.sin(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / max(nz, 1)) + ph)
        return f.reshape(-1) / 3.0

    rho = base["rho"] * (1.0 + np.stack([field(amp_rho) for _ in range(base["rho"].shape[0])]))
    u = np.stack([field(amp_u) for _ in range(3)])
    if cfg["lattice"] == 2:
        u[2] = 0.0
    T = base["T"] * (1.0 + field(amp_T))
    Ts = base["Ts"] * (1.0 + field(amp_T))
    return dict(rho=rho, u=u, T=T, Ts=Ts)


# ---------------------------------------------------------------------------
# learned warm start: the U-Net's layer table and seeded initial parameters
# (architecture data and random numbers only; the network arithmetic lives in
# the HIP library and, independently, in the oracle)
# ---------------------------------------------------------------------------
# (c_in, c_out, level, relu) per convolution, level = log2 of the pooling
UNET_LAYERS = [(32, 32, 0, 1), (32, 32, 0, 1), (32, 64, 1, 1), (64, 64, 1, 1),
               (64, 160, 2, 1), (160, 160, 2, 1), (224, 64, 1, 1), (64, 64, 1, 1),
               (96, 32, 0, 1), (32, 32, 0, 1), (32, 32, 0, 0)]


def unet_layout(layers=None) -> tuple[list, int]:
    """[(w_off, b_off)] per layer and the parameter count: each layer's
    weights W[c_out][27][c_in] followed by its biases [c_out]."""
    layers = UNET_LAYERS if layers is None else layers
    offs, p = [], 0
    for ci, co, _, _ in layers:
        offs.append((p, p + co * 27 * ci))
        p += co * 27 * ci + co
    return offs, p


def unet_init_params(seed: int = 1, layers=None, bias_scale: float = 0.0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (27 c_in))) and zero (or small normal)
    biases, float32, from numpy's PCG64 generator."""
    layers = UNET_LAYERS if layers is None else layers
    offs, n = unet_layout(layers)
    rng = np.random.default_rng(seed)
    p = np.zeros(n, dtype=np.float64)
    for (ci, co, _, _), (wo, bo) in zip(layers, offs):
        p[wo:bo] = rng.standard_normal(co * 27 * ci) * np.sqrt(2.0 / (27 * ci))
        if bias_scale:
            p[bo:bo + co] = rng.standard_normal(co) * bias_scale
    return p.astype(np.float32)
