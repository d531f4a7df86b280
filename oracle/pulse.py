"""FP64 oracle of pulsed (broadband) incidence.  Test infrastructure only:
imported by tests, never by the product.

Section 2.2.3, calculation of the incident wave: a plane-wave packet of any
shape reaches the transition layer; since cells on one wavefront share its
value, the packet is a 1D problem along k_hat, solved in free space next to
the 3D model and deployed to the layer each step.  The 1D axis starts at the
corner of the taper box the front reaches first (Eq. Oinc); a cell sits at
d = k_hat . (x - x_O) on it (Eq. inc_d); the packet and its gradient there
come from the spectral interpolation of the 1D grid (Eqs. pstd_psiinc,
pstd_dpsiinc).  Section 3.3: with a pulse the surface DFT runs over the
whole run at several frequencies, each normalised by the incident phasor
(Eqs. psiphasor-scaleddpsiphasor).

Readings (the paper leaves these open):
  * the 1D equation is stepped with the 3D model's leapfrog (Eq.
    PSTDupdating in 1D, no potential, no mask), eta on the kinetic term, on
    a periodic grid d_j = j Delta, j = 0 .. N-1, so every mode has the 3D
    scheme's dispersion sin(theta) = dtau eta k^2;
  * the start psi^0 is given; psi^{-1} moves each mode one step back along
    its physical root, so the packet travels one way;
  * the 3D step n -> n+1 uses the 1D field of step n (the 1D field is
    updated first, then deployed, then the 3D model is stepped);
  * the phasor at wavenumber k uses the scheme's frequency W(k): sin(W
    dtau) = dtau eta k^2 (W(1) = 1), weight exp(i W tau_n);
  * the incident phasor of the normalisation is taken at the grid origin,
    the reference point of the far-field amplitude, not at x_O: the two
    differ by the phase exp(-i k k_hat . x_O) only.
"""
from __future__ import annotations

import math

import numpy as np

from . import fft as _fft
from . import pstd as _pstd


def kbar1d(N, delta):
    """Wavenumbers of the 1D grid in FFT order: 2 pi l / (N Delta), l in
    [-N/2, N/2) (the Nyquist index at -N/2, as in Eq. pstd_psiinc)."""
    l = np.arange(N)
    l = np.where(l >= N // 2, l - N, l)
    return 2.0 * math.pi * l / (N * delta)


def scheme_frequency(k, dtau, eta):
    """W with sin(W dtau) = dtau eta k^2: the frequency at which wavenumber
    k oscillates under the leapfrog of Eq. PSTDupdating (free space)."""
    return np.arcsin(dtau * eta * np.asarray(k, dtype=np.float64) ** 2) / dtau


class Pulse1D:
    """The 1D free-space leapfrog of the incident packet."""

    def __init__(self, psi0, delta, dtau, eta):
        self.psi0 = np.asarray(psi0, dtype=np.complex128)
        self.N = self.psi0.size
        self.delta = float(delta)
        self.dtau = dtau
        self.eta = eta
        self.k = kbar1d(self.N, self.delta)
        if np.max(dtau * eta * self.k ** 2) >= 1.0:
            raise ValueError("the 1D grid holds modes beyond the leapfrog's bound")
        th = scheme_frequency(self.k, dtau, eta) * dtau
        self.prev = _fft.ifft(np.exp(1j * th) * _fft.fft(self.psi0))
        self.cur = self.psi0.copy()

    def step(self):
        lap = _fft.ifft(self.k ** 2 * _fft.fft(self.cur))
        nxt = self.prev - 2j * self.eta * self.dtau * lap
        self.prev, self.cur = self.cur, nxt

    def at(self, d):
        """Eqs. pstd_psiinc and pstd_dpsiinc: the packet and its derivative
        along the axis at the points d (any shape)."""
        d = np.asarray(d, dtype=np.float64)
        F = _fft.fft(self.cur)
        E = np.exp(1j * np.multiply.outer(d.reshape(-1), self.k))
        psi = (E @ F) / self.N
        dpsi = (E @ (1j * self.k * F)) / self.N
        return psi.reshape(d.shape), dpsi.reshape(d.shape)


def origin_corner(prob, kh):
    """Eq. Oinc: the outer corner of the taper box (y0 or y3 per axis) that
    the incident front reaches first."""
    lo = [prob.tfsf[a][0] for a in range(3)]
    hi = [prob.tfsf[a][3] for a in range(3)]
    return _pstd.o_inc(kh, lo, hi)


def axis_coordinate(model, O):
    """Eq. inc_d on the whole grid, [k][j][i]."""
    n = model.prob.n
    d = np.zeros((n[2], n[1], n[0]))
    for a in range(3):
        d = d + _pstd._bcast((np.arange(n[a]) - O[a]) * model.dxb[a] * model.kh[a], a)
    return d


class PulseModel:
    def __init__(self, prob, V, psi0, delta):
        self.m = _pstd.build(prob, V)
        self.O = origin_corner(prob, self.m.kh)
        self.d = axis_coordinate(self.m, self.O)
        self.layer = (self.m.lap_zeta != 0) | (self.m.grad_zeta[0] != 0) | (self.m.grad_zeta[1] != 0) | \
            (self.m.grad_zeta[2] != 0)
        self.pulse = Pulse1D(psi0, delta, self.m.dtau, self.m.eta)
        # the grid origin on the 1D axis (reference point of the normalisation)
        self.d_origin = sum((prob.n[a] // 2 - self.O[a]) * self.m.dxb[a] * self.m.kh[a] for a in range(3))

    def source(self):
        """lap(zeta) psi_inc + 2 grad(zeta) . grad(psi_inc) with the 1D
        field of the current step; grad psi_inc = k_hat dpsi/dd."""
        m = self.m
        S = np.zeros(m.v.shape, np.complex128)
        psi, dpsi = self.pulse.at(self.d[self.layer])
        g = sum(m.grad_zeta[a][self.layer] * m.kh[a] for a in range(3))
        S[self.layer] = m.lap_zeta[self.layer] * psi + 2.0 * g * dpsi
        return S

    def step(self, psi_prev, psi_cur, n):
        """3D step n -> n+1 of Eq. PSTDupdating with the pulse's source."""
        m = self.m
        S = self.source()
        if m.prob.eta_on_source:
            S = m.eta * S
        out = _pstd.step(m, psi_prev, psi_cur, n, with_source=False) - m.Gamma * (2j * m.dtau * S)
        return out


class MultiShellDFT:
    """Eq. psiphasor on the shell cells at several wavenumbers, and Eq.
    incpsiphasor at the grid origin for each.  The shell must lie where the
    taper is zero (scattered field only), so nothing is removed."""

    def __init__(self, pm, sphere, kbars):
        self.pm = pm
        self.mask = sphere.shell_mask()
        if np.any(pm.m.zeta[self.mask] != 0):
            raise ValueError("the shell reaches the taper")
        self.k = np.asarray(kbars, dtype=np.float64)
        self.W = scheme_frequency(self.k, pm.m.dtau, pm.m.eta)
        self.phi = np.zeros((self.k.size, int(self.mask.sum())), np.complex128)
        self.inc = np.zeros(self.k.size, np.complex128)

    def accumulate(self, psi, n):
        w = np.exp(1j * self.W * n * self.pm.m.dtau)
        self.phi += np.multiply.outer(w, psi[self.mask])
        p0, _ = self.pm.pulse.at(np.array([self.pm.d_origin]))
        self.inc += w * p0[0]

    def normalized(self, f):
        out = np.zeros(self.pm.m.v.shape, np.complex128)
        out[self.mask] = self.phi[f] / self.inc[f]
        return out


class MultiSurfaceDFT:
    """Eqs. psiphasor and dpsiphasor on the six box planes (values and the
    spectral normal derivative) at several wavenumbers, and Eq.
    incpsiphasor at the grid origin for each.  The planes must lie where
    the taper is zero (at or outside the taper box), so nothing is
    removed."""

    def __init__(self, pm, kbars):
        p = pm.m.prob
        for a in range(3):
            if not (p.surf_lo[a] <= p.tfsf[a][0] and p.surf_hi[a] >= p.tfsf[a][3]):
                raise ValueError("a box plane reaches the taper")
        self.pm = pm
        self.k = np.asarray(kbars, dtype=np.float64)
        self.W = scheme_frequency(self.k, pm.m.dtau, pm.m.eta)
        shapes = [_pstd.plane(pm.m.v, _pstd.FACES[f][0], 0).shape for f in range(6)]
        self.phi = [[np.zeros(sh, np.complex128) for sh in shapes] for _ in self.k]
        self.dphi = [[np.zeros(sh, np.complex128) for sh in shapes] for _ in self.k]
        self.inc = np.zeros(self.k.size, np.complex128)

    def accumulate(self, psi, n):
        m = self.pm.m
        w = np.exp(1j * self.W * n * m.dtau)
        ders = [_pstd.derivative(m, psi, a) for a in range(3)]
        for f in range(6):
            a, _ = _pstd.FACES[f]
            idx = _pstd.face_index(m.prob, f)
            v = _pstd.plane(psi, a, idx)
            d = _pstd.plane(ders[a], a, idx)
            for q in range(self.k.size):
                self.phi[q][f] += w[q] * v
                self.dphi[q][f] += w[q] * d
        p0, _ = self.pm.pulse.at(np.array([self.pm.d_origin]))
        self.inc += w * p0[0]

    def normalized(self, q):
        return [x / self.inc[q] for x in self.phi[q]], [x / self.inc[q] for x in self.dphi[q]]


def run(prob, V, psi0, delta, n_steps=None, sphere=None, kbars=(), box=False):
    """March from rest with the pulse; with a sphere (or box=True, the box
    planes), the phasors at the wavenumbers kbars over [dft_begin,
    dft_end)."""
    pm = PulseModel(prob, V, psi0, delta)
    n_steps = prob.n_steps if n_steps is None else n_steps
    prev = np.zeros(pm.m.v.shape, np.complex128)
    cur = np.zeros(pm.m.v.shape, np.complex128)
    if box:
        sd = MultiSurfaceDFT(pm, kbars)
    else:
        sd = MultiShellDFT(pm, sphere, kbars) if sphere is not None else None
    for n in range(n_steps):
        if sd is not None and prob.dft_begin <= n < prob.dft_end:
            sd.accumulate(cur, n)
        prev, cur = cur, pm.step(prev, cur, n)
        pm.pulse.step()
    return pm, prev, cur, sd
