"""Seeded synthetic inputs for the two-phase oil-water simulator.

This module produces *inputs only*: grid geometry, rock property fields, well
locations and controls, fluid constants and step schedules.  It holds none of
the simulator's arithmetic (no property law, no residual, no well index, no
initial state); the CPU oracle and the device library each derive those from
these inputs on their own.

The workloads stand in for the SPE10 model and the CMG IMEX decks the paper
runs on (Examples 1-3 and 6-7), which are not available here.  Cell size,
fluid constants and the reference depth/pressure follow Example 2 of the
paper (constants of the mxspe1 deck: oil 46.244 and water 62.238 lbm/ft^3,
4800 psi at 8400 ft, top-layer centre at 8335 ft, well radius 0.25 ft).

Cell numbering is natural: c = i + nx*(j + ny*k), k counted from the top
layer downward.  Every per-cell array is float64 of length n = nx*ny*nz in
that order.
"""
from __future__ import annotations

import numpy as np

# Well kinds and controls (Eq 11-14 of the paper: BHP, water, oil, liquid rate).
INJ, PROD = 0, 1
BHP, WRATE, ORATE, LRATE = 0, 1, 2, 3


def default_constants():
    """Field-unit constants shared by every workload (paper, Example 2)."""
    return dict(
        beta_c=0.001127,      # Darcy conversion, bbl*cP/(day*mD*ft*psi)
        alpha_c=5.614583,     # ft^3 per bbl
        rho_o=46.244,         # oil reference density, lbm/ft^3
        rho_w=62.238,         # water reference density, lbm/ft^3
        p_ref=4800.0,         # reference pressure of fluids and rock, psi
        z_ref=8400.0,         # depth of the reference pressure, ft
        c_o=1e-5, c_w=1e-5, c_r=1e-5,   # compressibilities, 1/psi
        mu_o=5.0, mu_w=1.0,   # viscosities, cP
        grav=1.0,             # 1 = gravity on, 0 = off
    )


def _grid(nx, ny, nz, dx=20.0, dy=20.0, dz=2.0, top=8335.0):
    return dict(nx=int(nx), ny=int(ny), nz=int(nz), n=int(nx * ny * nz),
                dx=float(dx), dy=float(dy), dz=float(dz), top=float(top))


def _vertical_well(g, i, j, kind, ctrl, target, k0=0, k1=None, rw=0.25, skin=0.0):
    k1 = g["nz"] if k1 is None else k1
    cells = np.array([i + g["nx"] * (j + g["ny"] * k) for k in range(k0, k1)],
                     dtype=np.int32)
    return dict(cells=cells, kind=int(kind), ctrl=int(ctrl), target=float(target),
                rw=float(rw), skin=float(skin))


def gaussian_field(shape, corr_len, rng, pad=30):
    """Standardised Gaussian random field, covariance exp(-(r/corr_len)^2).

    Spectral (FFT) method on a periodic grid padded by >= `pad` cells per axis,
    then cropped to `shape` and standardised to mean 0 and variance 1.
    `shape` is (nz, ny, nx).
    """
    full = []
    for s in shape:
        m = s + pad
        # next size with only small prime factors, for a quick FFT
        while max(_factors(m)) > 7:
            m += 1
        full.append(m)
    axes = [np.minimum(np.arange(m), m - np.arange(m)).astype(np.float64) for m in full]
    r2 = (axes[0][:, None, None] ** 2 + axes[1][None, :, None] ** 2
          + axes[2][None, None, :] ** 2)
    cov = np.exp(-r2 / corr_len ** 2)
    spec = np.abs(np.fft.rfftn(cov))
    noise = rng.standard_normal(full)
    field = np.fft.irfftn(np.sqrt(spec) * np.fft.rfftn(noise), s=full, axes=(0, 1, 2))
    field = field[: shape[0], : shape[1], : shape[2]]
    field = (field - field.mean()) / field.std()
    return field


def _factors(m):
    out, d = [], 2
    while d * d <= m:
        while m % d == 0:
            out.append(d)
            m //= d
        d += 1
    if m > 1:
        out.append(m)
    return out or [1]


def make_small(seed=0):
    """20x20x5 quarter five-spot with iid lognormal permeability (2,000 cells).

    ln k ~ N(4.6, 1.0^2) per cell (mD), kx = ky = kz; porosity U(0.15, 0.25);
    water-rate injector at (0,0), liquid-rate producer at (19,19), both
    200 STB/day through all layers; 10 steps of 10 days.
    """
    g = _grid(20, 20, 5)
    rng = np.random.default_rng(seed)
    lnk = rng.normal(4.6, 1.0, g["n"])
    phi = rng.uniform(0.15, 0.25, g["n"])
    k = np.exp(lnk)
    wells = [_vertical_well(g, 0, 0, INJ, WRATE, 200.0),
             _vertical_well(g, 19, 19, PROD, LRATE, 200.0)]
    return dict(name="quarter-five-spot 20x20x5", grid=g, kx=k.copy(), ky=k.copy(),
                kz=k.copy(), phi=phi, wells=wells, const=default_constants(),
                steps=10, dt=10.0, seed=seed)


def make_gaussian(nx=200, ny=200, nz=50, seed=1, corr_len=10.0, sigma=2.0,
                  well_pattern=5, inj_rate=4000.0, prod_bhp=4000.0):
    """Correlated lognormal model (default 200x200x50 = 2,000,000 cells).

    ln kh = 4.6 + sigma*G, G a standardised Gaussian field with correlation
    length `corr_len` cells; kz = 0.1 kh; porosity U(0.1, 0.3).  Vertical
    wells on a `well_pattern` x `well_pattern` lattice (spacing nx/pattern,
    offset half a spacing); (a+b) even -> water-rate injector, odd -> BHP
    producer; perforated in every layer.  30 steps of 10 days.
    """
    g = _grid(nx, ny, nz)
    rng = np.random.default_rng(seed)
    G = gaussian_field((nz, ny, nx), corr_len, rng)
    kh = np.exp(4.6 + sigma * G).reshape(-1)
    phi = rng.uniform(0.1, 0.3, g["n"])
    wells = []
    for a in range(well_pattern):
        for b in range(well_pattern):
            i = int((a + 0.5) * nx / well_pattern)
            j = int((b + 0.5) * ny / well_pattern)
            if (a + b) % 2 == 0:
                wells.append(_vertical_well(g, i, j, INJ, WRATE, inj_rate))
            else:
                wells.append(_vertical_well(g, i, j, PROD, BHP, prod_bhp))
    return dict(name=f"gaussian {nx}x{ny}x{nz}", grid=g, kx=kh.copy(), ky=kh.copy(),
                kz=0.1 * kh, phi=phi, wells=wells, const=default_constants(),
                steps=30, dt=10.0, seed=seed)


def make_channels(nx=640, ny=640, nz=160, seed=4, n_channels=60, well_pattern=20):
    """Channelised model (default 640x640x160 = 65,536,000 cells).

    Shale background ln k = 0 with ~`n_channels` sinuous sand channels of
    ln k = ln 1000: centreline y = y0 + A sin(2 pi x / lam + ph), A in [20, 60],
    lam in [150, 400], width 8-16 and thickness 4-8 cells, random x/y
    orientation and layer band; plus N(0, 1.5^2) noise on ln k; kz = 0.1 kh;
    porosity clip(0.08 + 0.025 ln k, 0.03, 0.35).  Wells on a 20x20 lattice
    (i, j = 16 + 32a), checkerboard injectors (4,000 STB/day) and BHP
    producers (4,000 psi).
    """
    g = _grid(nx, ny, nz)
    rng = np.random.default_rng(seed)
    lnk = np.zeros((nz, ny, nx), dtype=np.float64)
    xs = np.arange(nx, dtype=np.float64)
    ys = np.arange(ny, dtype=np.float64)
    for _ in range(n_channels):
        amp = rng.uniform(20, 60)
        lam = rng.uniform(150, 400)
        ph = rng.uniform(0, 2 * np.pi)
        width = rng.uniform(8, 16)
        thick = int(rng.integers(4, 9))
        along_x = rng.random() < 0.5
        k0 = int(rng.integers(0, max(1, nz - thick)))
        if along_x:
            y0 = rng.uniform(0, ny)
            centre = y0 + amp * np.sin(2 * np.pi * xs / lam + ph)       # per x
            mask2 = np.abs(ys[:, None] - centre[None, :]) <= width / 2  # (ny, nx)
        else:
            x0 = rng.uniform(0, nx)
            centre = x0 + amp * np.sin(2 * np.pi * ys / lam + ph)       # per y
            mask2 = np.abs(xs[None, :] - centre[:, None]) <= width / 2
        lnk[k0:k0 + thick][:, mask2] = np.log(1000.0)
    lnk += rng.normal(0.0, 1.5, lnk.shape)
    kh = np.exp(lnk).reshape(-1)
    phi = np.clip(0.08 + 0.025 * lnk.reshape(-1), 0.03, 0.35)
    wells = []
    for a in range(well_pattern):
        for b in range(well_pattern):
            i, j = 16 + 32 * a, 16 + 32 * b
            if i >= nx or j >= ny:
                continue
            if (a + b) % 2 == 0:
                wells.append(_vertical_well(g, i, j, INJ, WRATE, 4000.0))
            else:
                wells.append(_vertical_well(g, i, j, PROD, BHP, 4000.0))
    return dict(name=f"channels {nx}x{ny}x{nz}", grid=g, kx=kh.copy(), ky=kh.copy(),
                kz=0.1 * kh, phi=phi, wells=wells, const=default_constants(),
                steps=10, dt=10.0, seed=seed)


def make_column(nz=20, seed=0, k=100.0, phi=0.2):
    """One vertical column of `nz` cells, no wells, homogeneous rock.

    Starting from a non-equilibrium water saturation profile (water on top
    of oil) it exercises gravity segregation; the Jacobian is block
    tridiagonal, so block ILU(0) is an exact factorisation.
    """
    g = _grid(1, 1, nz)
    rng = np.random.default_rng(seed)
    sw0 = np.clip(0.6 - 0.5 * np.arange(nz) / nz + 0.05 * rng.random(nz), 0.0, 1.0)
    return dict(name=f"column 1x1x{nz}", grid=g, kx=np.full(nz, k), ky=np.full(nz, k),
                kz=np.full(nz, k), phi=np.full(nz, phi), wells=[],
                const=default_constants(), steps=1, dt=1.0, seed=seed, sw0=sw0)


def make_1d(nx=100, length=1000.0, k=100.0, phi=0.2, rate=10.0, bhp=4000.0,
            mu_ratio=5.0):
    """1D horizontal core for the Darcy and Buckley-Leverett checks.

    nx cells along x, one cell in y and z, homogeneous rock, incompressible
    fluids (all compressibilities 0), gravity off.  Water-rate injector in
    the first cell, BHP producer in the last cell.  Viscosity ratio
    mu_o/mu_w = `mu_ratio` with mu_w = 1 cP.
    """
    dx = length / nx
    g = _grid(nx, 1, 1, dx=dx, dy=20.0, dz=20.0)
    c = default_constants()
    c.update(c_o=0.0, c_w=0.0, c_r=0.0, grav=0.0, mu_w=1.0, mu_o=float(mu_ratio))
    n = g["n"]
    wells = [_vertical_well(g, 0, 0, INJ, WRATE, rate),
             _vertical_well(g, nx - 1, 0, PROD, BHP, bhp)]
    return dict(name=f"1d core {nx}", grid=g, kx=np.full(n, k), ky=np.full(n, k),
                kz=np.full(n, k), phi=np.full(n, phi), wells=wells, const=c,
                steps=1, dt=1.0, seed=0)


def make_tiny(nx=4, ny=4, nz=2, seed=3):
    """Tiny heterogeneous model with one injector and one producer (dense checks)."""
    g = _grid(nx, ny, nz)
    rng = np.random.default_rng(seed)
    k = np.exp(rng.normal(4.6, 1.0, g["n"]))
    phi = rng.uniform(0.15, 0.25, g["n"])
    wells = [_vertical_well(g, 0, 0, INJ, WRATE, 50.0),
             _vertical_well(g, nx - 1, ny - 1, PROD, BHP, 4700.0)]
    return dict(name=f"tiny {nx}x{ny}x{nz}", grid=g, kx=k.copy(), ky=k.copy(),
                kz=0.5 * k, phi=phi, wells=wells, const=default_constants(),
                steps=3, dt=5.0, seed=seed)


# The five workload sizes used throughout: quarter five-spot (2,000 cells),
# the 2M-cell correlated model (plain, mixed-precision and learned forms
# share it), and the 65.5M-cell channelised model.
def make_config(index, seed=None):
    if index == 0:
        return make_small(0 if seed is None else seed)
    if index in (1, 2, 3):
        return make_gaussian(seed=1 if seed is None else seed)
    if index == 4:
        return make_channels(seed=4 if seed is None else seed)
    raise ValueError(f"no workload {index}")


def random_state(w, rng, p_spread=50.0, tie_free=False):
    """A random reservoir state (p, sw per cell; p_b per well), interleaved.

    Used by consistency checks that need states away from equilibrium.
    Returns float64 array of length 2*(n + nw): [p0, s0, p1, s1, ..., pb0, 0, ...].
    """
    n = w["grid"]["n"]
    nw = len(w["wells"])
    x = np.zeros(2 * (n + nw))
    x[0:2 * n:2] = w["const"]["p_ref"] + p_spread * rng.standard_normal(n)
    x[1:2 * n:2] = rng.uniform(0.05, 0.95, n)
    x[2 * n::2] = w["const"]["p_ref"] + p_spread * rng.standard_normal(nw)
    return x


def developed_state(w, x0, rng, p_mound=300.0, length=15.0, radius=10.0):
    """A state shaped like one some days into the run, from a base state x0
    (the hydrostatic start, length 2*(n + nw)): a pressure mound of
    `p_mound` psi around every injector and a sink of the same depth around
    every producer (exp(-r/length), r in cells), and a water plume around
    every injector whose radius varies per layer (s_w = 0.8 (1 - r/R_k)
    inside R_k = radius * U(0.3, 1.5)).  Geometry and seeded noise only.
    """
    g = w["grid"]
    nx, ny, nz, n = g["nx"], g["ny"], g["nz"], g["n"]
    x = np.array(x0, dtype=np.float64, copy=True)
    c = np.arange(n)
    ci, cj, ck = c % nx, (c // nx) % ny, c // (nx * ny)
    dp = np.zeros(n)
    sw = np.zeros(n)
    for wl in w["wells"]:
        i0, j0 = wl["cells"][0] % nx, (wl["cells"][0] // nx) % ny
        r = np.hypot(ci - i0, cj - j0)
        sign = 1.0 if wl["kind"] == INJ else -1.0
        dp += sign * p_mound * np.exp(-r / length)
        if wl["kind"] == INJ:
            R = radius * rng.uniform(0.3, 1.5, nz)[ck]
            sw = np.maximum(sw, 0.8 * np.clip(1.0 - r / R, 0.0, 1.0))
    x[0:2 * n:2] += dp
    x[1:2 * n:2] = sw
    for k, wl in enumerate(w["wells"]):
        x[2 * (n + k)] += dp[wl["cells"][0]]
    return x


def flat_wells(w):
    """Wells as flat arrays: ptr[nw+1], cells, kind, ctrl, target, rw, skin."""
    wells = w["wells"]
    ptr = np.zeros(len(wells) + 1, dtype=np.int32)
    for i, wl in enumerate(wells):
        ptr[i + 1] = ptr[i] + len(wl["cells"])
    cells = (np.concatenate([wl["cells"] for wl in wells]).astype(np.int32)
             if wells else np.zeros(0, np.int32))
    return dict(ptr=ptr, cells=cells,
                kind=np.array([wl["kind"] for wl in wells], dtype=np.int32),
                ctrl=np.array([wl["ctrl"] for wl in wells], dtype=np.int32),
                target=np.array([wl["target"] for wl in wells], dtype=np.float64),
                rw=np.array([wl["rw"] for wl in wells], dtype=np.float64),
                skin=np.array([wl["skin"] for wl in wells], dtype=np.float64))
