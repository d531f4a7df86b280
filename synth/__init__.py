"""Seeded synthetic workloads shared by the HIP path's tests and the oracle.

This module holds problem descriptions (grid, incident wave, absorber, TF/SF
box, equivalence surface, time window) and seeded potential generators.  It
contains none of the scattering method's arithmetic: no reduced-unit scaling,
no stability bound, no tables, no FFTs.  Each consumer derives what it needs
from these raw inputs on its own.

Grid convention used by every workload: index (i, j, k) along (x, y, z) maps to
the physical point ((i - Nx/2) hx, (j - Ny/2) hy, (k - Nz/2) hz); 3D arrays are
stored C-ordered as [k][j][i] (x fastest).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "square_barrier", "gaussian_bumps", "smoothed_prior",
    "plain_barrier", "plain_barrier_refined", "square_barrier_160", "bumps_288", "uneven_batch", "voxel_potential_160", "tiny", "fresnel_plane", "fd_voxels",
    "paper_u0",
]


@dataclass
class Problem:
    """Raw description of one scattering run (physical units unless noted).

    tfsf[a] = (y0, y1, y2, y3): grid indices of the taper ramps along axis a
    (zeta = 0 at and outside y0 / y3, 1 on [y1, y2]).
    abc_U0 is in units of the central angular frequency E0/hbar; abc_alpha is
    per grid cell; abc_cells[a] is the absorber width in cells.
    surf_lo / surf_hi are the grid indices of the box equivalence surface.
    dt == 0 selects 0.9 of the critical step for |V| <= v_max.
    """
    n: tuple
    h: tuple
    k0: float
    hbar: float = 1.0
    mass: float = 1.0
    theta: float = 0.0
    phi: float = 0.0
    abc_cells: tuple = (8, 8, 8)
    abc_U0: float = 10.0
    abc_alpha: float = 0.5
    abc_UR: float = 0.0            # real part of a complex absorbing potential (units of E0)
    abc_alphaR: float = 0.0        # its decay per cell; 0: abc_alpha
    scheme: int = 0                # 0: spectral step; 1: the eighth-order FDTD variant
    tfsf: tuple = ((12, 18, 30, 36),) * 3
    v_max: float = 0.0
    dt: float = 0.0
    force_dt: bool = False
    ramp_periods: float = 4.0
    n_steps: int = 0
    dft_begin: int = 0
    dft_end: int = 0
    surf_lo: tuple = (10, 10, 10)
    surf_hi: tuple = (38, 38, 38)
    eta_on_source: bool = False
    sub_core: tuple = ()
    sub_halo: int = 0
    sub_taper: int = 0
    surface_kind: int = 0          # 0: box faces; 1: sphere (an addition, not in the paper)
    sphere_radius: float = 0.0     # physical, centred at the origin
    sphere_nodes: tuple = (64, 128)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    @property
    def cells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


def paper_u0(alpha: float, dxbar: float, width: int) -> float:
    """Absorber height giving the same one-way integral of gamma over the layer
    as the paper's square-potential run (U0 = 5, alpha = 0.1 per cell, 40 cells,
    cell pi/10 in reduced length): 5*pi*tanh(4) reduced units."""
    target = 5.0 * math.pi * math.tanh(4.0)
    return target * alpha / (dxbar * math.tanh(alpha * width))


# ----------------------------------------------------------------------------
# potentials (energy units, layout [k][j][i])
# ----------------------------------------------------------------------------

def square_barrier(n, h, radius, height, sub=8):
    """Central square barrier of the given radius, voxelised by volume fraction.

    Each cell (centred on its grid point) is split into sub^3 sub-cells; a
    sub-cell counts as inside when its centre lies within the sphere.  The test
    is done in exact integer arithmetic: with s = 0..sub-1 the sub-cell centre
    offset is (2s - sub + 1)/(2 sub) cells.
    """
    nx, ny, nz = (int(v) for v in n)
    assert abs(h[0] - h[1]) < 1e-15 and abs(h[0] - h[2]) < 1e-15, "cubic cells"
    r_cells = radius / h[0]
    scale = 2 * sub
    # exact when radius/h * 2*sub is an integer (true for every workload here)
    rr = r_cells * scale
    rr2 = int(round(rr * rr)) if abs(rr - round(rr)) < 1e-9 else rr * rr
    s = np.arange(sub)
    off = 2 * s - sub + 1  # in units of 1/(2 sub) cells

    def axis_sq(N):
        idx = np.arange(N) - N // 2
        return (idx[:, None] * scale + off[None, :]) ** 2  # [N, sub]

    ax, ay, az = axis_sq(nx), axis_sq(ny), axis_sq(nz)
    V = np.zeros((nz, ny, nx), dtype=np.float64)
    # only cells near the centre can be touched
    reach = int(math.ceil(r_cells)) + 1
    ks = range(max(0, nz // 2 - reach), min(nz, nz // 2 + reach + 1))
    js = range(max(0, ny // 2 - reach), min(ny, ny // 2 + reach + 1))
    is_ = np.arange(max(0, nx // 2 - reach), min(nx, nx // 2 + reach + 1))
    sub3 = float(sub ** 3)
    for k in ks:
        for j in js:
            t = az[k][:, None] + ay[j][None, :]  # [sub, sub]
            d = t[None, :, :, None] + ax[is_][:, None, None, :]  # [ni, sub, sub, sub]
            frac = (d <= rr2).sum(axis=(1, 2, 3)) / sub3
            V[k, j, is_] = height * frac
    return V


def gaussian_bumps(n, h, count, ball_radius, sigma_range, height_std, seed,
                   core_lo, core_hi, sigma_floor=0.0):
    """Sum of axis-aligned anisotropic Gaussian bumps, truncated to the TF core.

    Centres: uniform in a ball (radius * u^(1/3) along an isotropic direction);
    standard deviations per axis ~ U[sigma_range]; heights ~ N(0, height_std).
    Values outside the index box [core_lo, core_hi] (inclusive) are set to 0.
    Returns (V, params) with V in energy units, layout [k][j][i].
    """
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(count, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = ball_radius * rng.random(count) ** (1.0 / 3.0)
    centres = d * rad[:, None]
    sig = rng.uniform(sigma_range[0], sigma_range[1], size=(count, 3))
    sig = np.maximum(sig, sigma_floor)
    heights = rng.normal(0.0, height_std, size=count)
    nx, ny, nz = (int(v) for v in n)
    x = (np.arange(nx) - nx // 2) * h[0]
    y = (np.arange(ny) - ny // 2) * h[1]
    z = (np.arange(nz) - nz // 2) * h[2]
    V = np.zeros((nz, ny, nx))
    for b in range(count):
        gx = np.exp(-0.5 * ((x - centres[b, 0]) / sig[b, 0]) ** 2)
        gy = np.exp(-0.5 * ((y - centres[b, 1]) / sig[b, 1]) ** 2)
        gz = np.exp(-0.5 * ((z - centres[b, 2]) / sig[b, 2]) ** 2)
        V += heights[b] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    mask = np.zeros_like(V, dtype=bool)
    mask[core_lo[2]:core_hi[2] + 1, core_lo[1]:core_hi[1] + 1, core_lo[0]:core_hi[0] + 1] = True
    V[~mask] = 0.0
    return V, dict(centres=centres, sigmas=sig, heights=heights)


def smoothed_prior(n, core_lo, core_hi, std, sigma_cells, seed):
    """i.i.d. N(0,1) on the TF-core voxels, separable Gaussian smoothing
    (sigma in cells, truncated at 4 sigma), rescaled to standard deviation std
    over the core.  Zero outside the core."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in n)
    lo, hi = core_lo, core_hi
    shape = (hi[2] - lo[2] + 1, hi[1] - lo[1] + 1, hi[0] - lo[0] + 1)
    w = rng.normal(size=shape)
    r = int(math.ceil(4 * sigma_cells))
    t = np.arange(-r, r + 1)
    ker = np.exp(-0.5 * (t / sigma_cells) ** 2)
    ker /= ker.sum()
    for ax in range(3):
        w = np.apply_along_axis(lambda v: np.convolve(v, ker, mode="same"), ax, w)
    w *= std / w.std()
    V = np.zeros((nz, ny, nx))
    V[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = w
    return V


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def plain_barrier():
    """Square barrier r = 0.6, V0 = 0.5 E0, k0 = pi/(4h) along +z; 32^3 cells
    inside an 8-cell absorber (FFT grid 48^3).  6649 steps at 0.9 of the
    critical step cover T = 4.0; the phasor window is the last 4 periods."""
    h = 0.1
    k0 = math.pi / (4 * h)
    E0 = k0 * k0 / 2
    n = (48, 48, 48)
    P = 8
    alpha = 4.0 / P
    prob = Problem(n=n, h=(h, h, h), k0=k0, abc_cells=(P,) * 3, abc_alpha=alpha,
                   abc_U0=paper_u0(alpha, k0 * h, P), tfsf=((12, 18, 30, 36),) * 3,
                   v_max=0.5 * E0, n_steps=6649, dft_begin=6649 - 1354, dft_end=6649,
                   surf_lo=(10, 10, 10), surf_hi=(38, 38, 38))
    V = square_barrier(n, prob.h, 0.6, 0.5 * E0)
    return prob, V


# Absorber parameters for an 8-cell layer at 8 points per wavelength (k0 h =
# pi/4), found by minimising the far-field difference between the plain-
# method workload and the same problem with a 32-cell layer on a 96^3 grid
# (wide_layer_reference).  The mask alone, and the mask with a real part
# (a complex absorbing potential).
TUNED_MASK_8 = dict(abc_U0=9.835, abc_alpha=0.3386)
TUNED_COMPLEX_8 = dict(abc_U0=23.71, abc_alpha=0.3959, abc_UR=-0.6635, abc_alphaR=0.2705)


def wide_layer_reference(prob, V, n_fft=96, width=32):
    """The same problem (spacing, taper, box planes and potential about the
    grid centre, steps, window) on a cubic grid of n_fft points with a
    `width`-cell layer of the paper's profile (alpha = 4 / width, U0 from the
    paper's one-way absorption): its far field stands for the thin-layer
    problem's without absorber reflections."""
    n0 = prob.n[0]
    assert prob.n == (n0, n0, n0) and (n_fft - n0) % 2 == 0 and n_fft > n0
    sh = (n_fft - n0) // 2
    alpha = 4.0 / width
    p = prob.replace(n=(n_fft,) * 3, abc_cells=(width,) * 3, abc_alpha=alpha,
                     abc_U0=paper_u0(alpha, prob.k0 * prob.h[0], width), abc_UR=0.0, abc_alphaR=0.0,
                     tfsf=tuple(tuple(y + sh for y in t) for t in prob.tfsf),
                     surf_lo=tuple(x + sh for x in prob.surf_lo), surf_hi=tuple(x + sh for x in prob.surf_hi))
    W = np.zeros((n_fft,) * 3)
    W[sh:sh + n0, sh:sh + n0, sh:sh + n0] = V
    return p, W


def x3_square_potential(s, n_fft=288, n_steps=36000, ramp_periods=2.0):
    """The paper's own run of Section 4 at its scale on one grid: central
    square potential V = s E0 for r_bar <= 4 pi (Eq. sphericalV), 20 points
    per wavelength (dxb = pi/10), dtau = pi/1000, incident along +y; per axis
    a 40-cell absorber (U0 = 5, alpha = 0.1 per cell), 41 scattered-field
    cells, a 12-cell taper, box planes on the middle planes of the
    scattered-field region.  The paper's 288 x 290 x 288 (two overlapping
    y subdomains) becomes one n_fft^3 grid; the window is the last 4
    periods.  36000 steps settle s = 1, 0.5, -0.5; the deep well s = -1
    holds a slowly decaying quasi-bound state and needs about 60000."""
    h = 0.1
    k0 = math.pi / (10 * h)
    E0 = k0 * k0 / 2
    N = n_fft
    P = 40
    y0, y1 = P + 41, P + 41 + 12
    tf = (y0, y1, N - 1 - y1, N - 1 - y0)
    mid = P + 20
    dtau = math.pi / 1000
    window = int(round(4 * 2 * math.pi / dtau))
    prob = Problem(n=(N,) * 3, h=(h, h, h), k0=k0, theta=math.pi / 2, phi=math.pi / 2,
                   abc_cells=(P,) * 3, abc_U0=5.0, abc_alpha=0.1, tfsf=(tf,) * 3,
                   v_max=abs(s) * E0, dt=dtau / E0, ramp_periods=ramp_periods, n_steps=n_steps,
                   dft_begin=n_steps - window, dft_end=n_steps,
                   surf_lo=(mid,) * 3, surf_hi=(N - 1 - mid,) * 3)
    V = square_barrier(prob.n, prob.h, 4 * math.pi / k0, s * E0)
    return prob, V


def plain_barrier_refined():
    """The plain-method barrier (r = 0.6, V0 = E0/2, k0 = pi/(4h0), h0 = 0.1)
    at half the spacing, h = 0.05, with an absorber twice as wide (32 cells,
    1.6 length units) and the same time T = 4.0: FFT grid 128^3, TF/SF walls
    of 12 cells, box surface 4 cells outside the TF box."""
    h = 0.05
    k0 = math.pi / 0.4
    E0 = k0 * k0 / 2
    n = (128, 128, 128)
    P = 32
    alpha = 4.0 / P
    dtau = 0.9 / (math.pi ** 2 * 3 / (k0 * h) ** 2 + 0.5)
    steps = int(math.ceil(4.0 * E0 / dtau))
    window = int(round(4 * 2 * math.pi / dtau))
    prob = Problem(n=n, h=(h, h, h), k0=k0, abc_cells=(P,) * 3, abc_alpha=alpha,
                   abc_U0=paper_u0(alpha, k0 * h, P), tfsf=((40, 52, 76, 88),) * 3,
                   v_max=0.5 * E0, n_steps=steps, dft_begin=steps - window, dft_end=steps,
                   surf_lo=(36, 36, 36), surf_hi=(92, 92, 92))
    V = square_barrier(n, prob.h, 0.6, 0.5 * E0)
    return prob, V


def square_barrier_160(n_fft=160, transition=12):
    """Square barrier r = 2.4, V0 = 0.5 E0; 128^3 cells inside a 16-cell absorber
    (FFT grid 160^3); box surface at i = 40, 120.  The taper is one on the
    core +-2.4 (N/2 -+ 24 cells) and ramps over `transition` cells outside it:
    12 cells keep the TF/SF leakage at 1e-4 of the scattered amplitude (4 cells
    leak 2.2 %, 8 cells 0.09 %, measured on the V = 0 run); pulsed runs on the
    sphere of radius 5.6, whose shell must lie where the taper is zero, take
    4 (the taper box's corners at 4.85)."""
    h = 0.1
    k0 = math.pi / (4 * h)
    E0 = k0 * k0 / 2
    n = (n_fft,) * 3
    P = 16
    alpha = 4.0 / P
    c = n_fft // 2
    tf = (c - 24 - transition, c - 24, c + 24, c + 24 + transition)
    prob = Problem(n=n, h=(h, h, h), k0=k0, abc_cells=(P,) * 3, abc_alpha=alpha,
                   abc_U0=paper_u0(alpha, k0 * h, P), tfsf=(tf,) * 3,
                   v_max=0.5 * E0, n_steps=14440, dft_begin=14440 - 1354, dft_end=14440,
                   surf_lo=(c - 40,) * 3, surf_hi=(c + 40,) * 3)
    V = square_barrier(n, prob.h, 2.4, 0.5 * E0)
    return prob, V


def bumps_288(n_fft=288, seed=3):
    """32 anisotropic Gaussian bumps (centres in a radius-8 ball, sigma in
    U[0.3, 1.2], heights N(0, 0.3 E0)) on a 256^3 interior (FFT grid 288^3)."""
    h = 0.1
    k0 = math.pi / (4 * h)
    E0 = k0 * k0 / 2
    n = (n_fft,) * 3
    P = 16
    alpha = 4.0 / P
    tf = (24, 28, n_fft - 28, n_fft - 24)
    core_lo, core_hi = (tf[1],) * 3, (tf[2],) * 3
    V, _ = gaussian_bumps(n, (h,) * 3, 32, 8.0, (0.3, 1.2), 0.3 * E0, seed, core_lo, core_hi)
    prob = Problem(n=n, h=(h, h, h), k0=k0, abc_cells=(P,) * 3, abc_alpha=alpha,
                   abc_U0=paper_u0(alpha, k0 * h, P), tfsf=(tf,) * 3,
                   v_max=float(np.abs(V).max()), n_steps=1000, dft_begin=0, dft_end=0,
                   surf_lo=(20,) * 3, surf_hi=(n_fft - 20,) * 3,
                   sub_core=(48, 48, 48), sub_halo=8, sub_taper=3)
    return prob, V


BATCH_LENGTHS = (96, 100, 108, 120, 128, 144, 150, 160, 162, 180, 192)


def uneven_batch(count=64, seed=4, lengths=BATCH_LENGTHS):
    """Uneven batched instances: per-axis FFT lengths drawn from `lengths`,
    isotropic incident directions, k0 ~ U[pi/(8h), pi/(3h)], Gaussian bumps
    scaled to each instance's TF core."""
    rng = np.random.default_rng(seed)
    h = 0.1
    P = 16
    out = []
    for b in range(count):
        n = tuple(int(v) for v in rng.choice(lengths, size=3))
        k0 = float(rng.uniform(math.pi / (8 * h), math.pi / (3 * h)))
        u, w = rng.random(), rng.random()
        theta = math.acos(1 - 2 * u)
        phi = 2 * math.pi * w
        tf = tuple((P + 4, P + 8, N - P - 8, N - P - 4) for N in n)
        core_lo = tuple(t[1] for t in tf)
        core_hi = tuple(t[2] for t in tf)
        half = min((t[2] - t[1]) * h / 2 for t in tf)
        s = half / 11.6
        E0 = k0 * k0 / 2
        V, _ = gaussian_bumps(n, (h,) * 3, 32, 8.0 * s, (0.3 * s, 1.2 * s), 0.3 * E0,
                              seed * 1000 + b, core_lo, core_hi, sigma_floor=1.5 * h)
        alpha = 4.0 / P
        prob = Problem(n=n, h=(h, h, h), k0=k0, theta=theta, phi=phi,
                       abc_cells=(P,) * 3, abc_alpha=alpha,
                       abc_U0=paper_u0(alpha, k0 * h, P), tfsf=tf,
                       v_max=float(np.abs(V).max()), n_steps=1000,
                       surf_lo=tuple(P + 2 for _ in n), surf_hi=tuple(N - P - 2 for N in n))
        out.append((prob, V))
    return out


def voxel_potential_160(seed_prior=5, seed_hidden=55, n_fft=160):
    """Voxel potential on the TF core of a 128^3 interior (FFT grid 160^3):
    smoothed N(0, 0.1 E0) prior and a hidden potential from the same recipe."""
    h = 0.1
    k0 = math.pi / (4 * h)
    E0 = k0 * k0 / 2
    n = (n_fft,) * 3
    P = 16
    alpha = 4.0 / P
    tf = (20, 24, n_fft - 24, n_fft - 20)
    core_lo, core_hi = (tf[1],) * 3, (tf[2],) * 3
    V0 = smoothed_prior(n, core_lo, core_hi, 0.1 * E0, 2.0, seed_prior)
    Vh = smoothed_prior(n, core_lo, core_hi, 0.1 * E0, 2.0, seed_hidden)
    vmax = max(float(np.abs(V0).max()), float(np.abs(Vh).max())) * 1.5
    prob = Problem(n=n, h=(h, h, h), k0=k0, abc_cells=(P,) * 3, abc_alpha=alpha,
                   abc_U0=paper_u0(alpha, k0 * h, P), tfsf=(tf,) * 3,
                   v_max=vmax, n_steps=6000, dft_begin=0, dft_end=6000,
                   surf_lo=(18,) * 3, surf_hi=(n_fft - 18,) * 3)
    return prob, V0, Vh


def voxel_potential_48(seed_prior=5, seed_hidden=55):
    """The voxel-potential recipe of voxel_potential_160 on a 48^3 FFT grid
    (32^3 inside an 8-cell absorber): taper 10/14/34/38, voxel potential on
    the 21^3 core (smoothed N(0, 0.1 E0) prior, sigma 2 cells; hidden
    potential from another seed), box planes at 9 and 39, 6000 steps with the
    window over all of them.  Small enough for the FP64 oracle's adjoint at
    the full step count."""
    h = 0.1
    k0 = math.pi / (4 * h)
    E0 = k0 * k0 / 2
    n = (48, 48, 48)
    P = 8
    alpha = 4.0 / P
    tf = (10, 14, 34, 38)
    core_lo, core_hi = (tf[1],) * 3, (tf[2],) * 3
    V0 = smoothed_prior(n, core_lo, core_hi, 0.1 * E0, 2.0, seed_prior)
    Vh = smoothed_prior(n, core_lo, core_hi, 0.1 * E0, 2.0, seed_hidden)
    vmax = max(float(np.abs(V0).max()), float(np.abs(Vh).max())) * 1.5
    prob = Problem(n=n, h=(h, h, h), k0=k0, abc_cells=(P,) * 3, abc_alpha=alpha,
                   abc_U0=paper_u0(alpha, k0 * h, P), tfsf=(tf,) * 3,
                   v_max=vmax, n_steps=6000, dft_begin=0, dft_end=6000,
                   surf_lo=(9,) * 3, surf_hi=(39,) * 3)
    return prob, V0, Vh


def fresnel_plane(n_side, spacing, z):
    """n_side x n_side detector points (physical xyz) at height z, centred on
    the z axis, lateral spacing `spacing`; row-major in (y, x)."""
    g = (np.arange(n_side) - (n_side - 1) / 2.0) * spacing
    X, Y = np.meshgrid(g, g, indexing="xy")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, float(z))], axis=1)


def fd_voxels(prob, count, seed):
    """`count` distinct seed-chosen voxels (k, j, i) of the TF core."""
    rng = np.random.default_rng(seed)
    lo = [prob.tfsf[a][1] for a in range(3)]
    hi = [prob.tfsf[a][2] for a in range(3)]
    seen, out = set(), []
    while len(out) < count:
        v = (int(rng.integers(lo[2], hi[2] + 1)), int(rng.integers(lo[1], hi[1] + 1)),
             int(rng.integers(lo[0], hi[0] + 1)))
        if v not in seen:
            seen.add(v)
            out.append(v)
    return out


def tiny(n=(24, 24, 24), P=4, transition=3, theta=0.0, phi=0.0, k_ppw=8,
         steps=40, v0=0.5, radius_cells=3, dft=(0, 40)):
    """Small anisotropic-capable workload for parity tests.  The TF box sits
    two cells inside the absorber, the surface one cell outside the TF box."""
    h = 0.1
    k0 = 2 * math.pi / (k_ppw * h)
    E0 = k0 * k0 / 2
    tf = tuple((P + 2, P + 2 + transition, N - P - 2 - transition, N - P - 2) for N in n)
    surf_lo = tuple(P + 1 for _ in n)
    surf_hi = tuple(N - P - 1 for N in n)
    alpha = 4.0 / P
    prob = Problem(n=tuple(n), h=(h, h, h), k0=k0, theta=theta, phi=phi,
                   abc_cells=(P,) * 3, abc_alpha=alpha, abc_U0=paper_u0(alpha, k0 * h, P),
                   tfsf=tf, v_max=max(abs(v0), 1e-12) * E0, n_steps=steps,
                   dft_begin=dft[0], dft_end=dft[1], surf_lo=surf_lo, surf_hi=surf_hi)
    if radius_cells > 0 and v0 != 0.0:
        V = square_barrier(n, prob.h, radius_cells * h, v0 * E0) if len(set(n)) == 1 else \
            _ellipsoid(n, h, radius_cells, v0 * E0)
    else:
        V = np.zeros((n[2], n[1], n[0]))
    return prob, V


def _ellipsoid(n, h, r_cells, height):
    nx, ny, nz = n
    x = np.arange(nx) - nx // 2
    y = np.arange(ny) - ny // 2
    z = np.arange(nz) - nz // 2
    d = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
    return np.where(d <= r_cells * r_cells, height, 0.0)


def random_state(n, seed, scale=1.0):
    """Seeded complex field of shape [Nz][Ny][Nx] (for single-step parity)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    a = rng.normal(size=(nz, ny, nx)) + 1j * rng.normal(size=(nz, ny, nx))
    return scale * a


def gaussian_pulse_1d(n1d, delta, k_c, sigma, d0):
    """A Gaussian packet on the periodic 1D grid d_j = j delta (reduced
    units): exp(-(d - d0)^2 / (2 sigma^2)) exp(i k_c (d - d0)), with d - d0
    taken at the nearest periodic image."""
    L = n1d * delta
    x = np.arange(n1d) * delta - d0
    x = (x + L / 2) % L - L / 2
    return np.exp(-x * x / (2 * sigma * sigma)) * np.exp(1j * k_c * x)
