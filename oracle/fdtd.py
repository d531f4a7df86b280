"""FP64 oracle of the FDTD variant of the internal model (Section 2.2.1, FDTD
version of TF/SF).  Test infrastructure only: imported by tests, never by
the product.

Reduced units as in `pstd.py` (x_bar = k0 x, tau = E0 t / hbar): the
Laplacian is the eighth-order central stencil of Eq. y_stencil with the
coefficients of Eq. stencil_alpha along every axis (periodic grid, like the
spectral passes), time is the central difference of Eq. FDTDupdatePsi,

    psi^{n+1} = psi^{n-1} - 2i dtau v psi^n + 2i dtau lap_8 psi^n,

(the potential term multiplies psi^n, which the printed equation drops), the
total-field region is the box y1 <= i <= y2 of every axis with a sharp
interface, and the incident plane wave enters through the consistency terms
of Eqs. FDTDpsi_extraJminus1-FDTDpsiJplus4 on the four cells either side of
each wall, accumulated wall by wall on the lines whose transverse indices lie
in the total-field box, at the scheme's discrete frequency for k_hat.  The
mask of Eq. expmask multiplies the update as in the spectral scheme.  No eta
correction: the FDTD scheme has none.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import pstd as _pstd

# Eq. stencil_alpha
ALPHA = (-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0)


def stencil_symbol(theta):
    """alpha_0 + 2 sum_l alpha_l cos(l theta): the stencil applied to
    exp(i theta j), per unit spacing squared."""
    theta = np.asarray(theta, dtype=np.float64)
    return ALPHA[0] + 2.0 * sum(ALPHA[l] * np.cos(l * theta) for l in range(1, 5))


def critical_dtau(dxb, vmax_over_E0):
    """Largest stable reduced step of the central-difference leapfrog: dtau
    times the largest |eigenvalue| of -lap_8 + v at most 1; -lap_8 peaks at
    the Nyquist corner, |symbol(pi)| / dxb_a^2 per axis."""
    lam = float(abs(stencil_symbol(math.pi))) * float(np.sum(1.0 / np.asarray(dxb) ** 2))
    return 1.0 / (lam + vmax_over_E0)


def dtau_of(prob):
    E0 = _pstd.central_energy(prob)
    if prob.dt > 0:
        return E0 * prob.dt / prob.hbar
    return 0.9 * critical_dtau(_pstd.dxbar(prob), prob.v_max / E0)


def laplacian8(psi, dxb):
    """sum_a lap_8 along axis a (Eq. y_stencil), periodic."""
    out = np.zeros_like(psi, dtype=np.complex128)
    for a in range(3):
        ax = _pstd.NPAX[a]
        s = ALPHA[0] * psi
        for l in range(1, 5):
            s = s + ALPHA[l] * (np.roll(psi, l, axis=ax) + np.roll(psi, -l, axis=ax))
        out += s / dxb[a] ** 2
    return out


@dataclass
class Model:
    prob: object
    dtau: float
    dxb: np.ndarray
    v: np.ndarray          # V / E0 (plus the absorber's real part), [k][j][i]
    Gamma: np.ndarray      # mask, Eq. Gamma
    box: tuple             # per axis (lo, hi): total field for lo <= i <= hi
    phase: np.ndarray      # exp(i k_hat . r_bar)
    kh: np.ndarray
    tau_r: float
    omega: float           # discrete frequency of the incident wave (discrete_frequency)


def discrete_frequency(kh, dxb, dtau):
    """The frequency at which the plane wave exp(i k_hat . r_bar) solves the
    discrete scheme exactly with v = 0: sin(W dtau) = dtau k_h^2, k_h^2 =
    -sum_a symbol(kh_a dxb_a) / dxb_a^2 (1 + O(dtau^2) + O(dxb^8)).  The
    walls drive the incident wave at W, so that the consistency terms cancel
    the stencil's dispersion (the paper states no frequency; the spectral
    scheme reaches the same end with eta)."""
    k2 = -sum(float(stencil_symbol(kh[a] * dxb[a])) / dxb[a] ** 2 for a in range(3))
    return math.asin(dtau * k2) / dtau


def build(prob, V):
    E0 = _pstd.central_energy(prob)
    dxb = _pstd.dxbar(prob)
    dtau = dtau_of(prob)
    n = prob.n
    v = np.asarray(V, dtype=np.float64) / E0 + _pstd.absorber_real_3d(prob)
    G = np.ones((n[2], n[1], n[0]))
    for a in range(3):
        G = G * _pstd._bcast(_pstd.mask_1d(n[a], prob.abc_cells[a], prob.abc_U0, prob.abc_alpha, dtau), a)
    box = tuple((prob.tfsf[a][1], prob.tfsf[a][2]) for a in range(3))
    kh = _pstd.khat(prob.theta, prob.phi)
    X = [_pstd._bcast(_pstd.coords(n[a], dxb[a]), a) for a in range(3)]
    phase = np.exp(1j * (kh[0] * X[0] + kh[1] * X[1] + kh[2] * X[2])) * np.ones_like(G, dtype=np.complex128)
    return Model(prob, dtau, dxb, v, G, box, phase, kh, 2 * math.pi * prob.ramp_periods,
                 discrete_frequency(kh, dxb, dtau))


def total_field_mask(model):
    """1 on the total-field box, 0 elsewhere (Eq. psiTFvsNTF)."""
    n = model.prob.n
    T = np.ones((n[2], n[1], n[0]))
    for a in range(3):
        lo, hi = model.box[a]
        t = np.zeros(n[a])
        t[lo:hi + 1] = 1.0
        T = T * _pstd._bcast(t, a)
    return T


def incident(model, n):
    """R(tau_n) exp(i(k_hat . r_bar - W tau_n)), W the discrete frequency."""
    tau = n * model.dtau
    return _pstd.ramp(tau, model.tau_r) * np.exp(-1j * model.omega * tau) * model.phase


def wall_terms(model, psi_inc):
    """The consistency terms of the six walls, accumulated wall by wall
    (the bracket that multiplies 2i dtau / dxb_a^2 in Eqs. FDTDpsi_extra...):
    on a line along axis a whose other indices lie in the box, the four
    total-field cells next to a wall gain alpha_l times the incident wave at
    the scattered-field cells their stencil reaches, and the four scattered-
    field cells lose alpha_l times it at the total-field cells they reach."""
    n = model.prob.n
    W = np.zeros((n[2], n[1], n[0]), dtype=np.complex128)
    for a in range(3):
        ax = _pstd.NPAX[a]
        # lines whose transverse indices lie in the box
        sel = [slice(None)] * 3
        for b in range(3):
            if b != a:
                lo, hi = model.box[b]
                sel[_pstd.NPAX[b]] = slice(lo, hi + 1)
        lo, hi = model.box[a]
        inc = psi_inc[tuple(sel)]
        acc = np.zeros_like(inc)

        def at(i):
            s = [slice(None)] * 3
            s[ax] = i % n[a]
            return tuple(s)

        for m in range(4):
            # high wall: total-field cell hi - m reaches hi + 1 ... (scattered)
            acc[at(hi - m)] += sum(ALPHA[l] * inc[at(hi - m + l)] for l in range(m + 1, 5))
            # low wall: total-field cell lo + m reaches lo - 1 ...
            acc[at(lo + m)] += sum(ALPHA[l] * inc[at(lo + m - l)] for l in range(m + 1, 5))
        for m in range(1, 5):
            # scattered-field cells hi + m and lo - m reach into the box
            acc[at(hi + m)] -= sum(ALPHA[l] * inc[at(hi + m - l)] for l in range(m, 5))
            acc[at(lo - m)] -= sum(ALPHA[l] * inc[at(lo - m + l)] for l in range(m, 5))
        W[tuple(sel)] += acc / model.dxb[a] ** 2
    return W


def step(model, psi_prev, psi_cur, n, with_source=True, psi_inc=None):
    """One step of Eq. FDTDupdatePsi plus the wall terms, under the mask.
    psi_inc overrides the incident wave at step n (default: incident())."""
    dt = model.dtau
    rhs = psi_prev + 2j * dt * laplacian8(psi_cur, model.dxb) - 2j * dt * model.v * psi_cur
    if with_source:
        inc = incident(model, n) if psi_inc is None else psi_inc
        rhs = rhs + 2j * dt * wall_terms(model, inc)
    return model.Gamma * rhs


def run(prob, V, n_steps=None):
    model = build(prob, V)
    n_steps = prob.n_steps if n_steps is None else n_steps
    prev = np.zeros(model.v.shape, np.complex128)
    cur = np.zeros(model.v.shape, np.complex128)
    for n in range(n_steps):
        prev, cur = cur, step(model, prev, cur, n)
    return model, prev, cur


class ShellDFT:
    """Eq. psiphasor on the shell cells of a spherical surface, for the FDTD
    variant: step n weighs exp(i W tau_n), W the incident wave's discrete
    frequency, and the normalised phasor has the incident part removed.  The
    stored field is psi_s + T psi_inc (T the total-field box, Eq.
    psiTFvsNTF); the DFT of T R(tau_n) exp(i(k_hat . r_bar - W tau_n)) with
    these weights is T exp(i k_hat . r_bar) sum_n R(tau_n), so after the
    normalisation by sum_n R(tau_n) the incident part is T exp(i k_hat .
    r_bar) exactly."""

    def __init__(self, model, sphere):
        self.m = model
        self.mask = sphere.shell_mask()
        self.phi = np.zeros(model.v.shape, np.complex128)
        self.inc = 0.0

    def accumulate(self, psi, n):
        tau = n * self.m.dtau
        self.phi[self.mask] += np.exp(1j * self.m.omega * tau) * psi[self.mask]
        self.inc += _pstd.ramp(tau, self.m.tau_r)

    def normalized(self):
        out = self.phi / self.inc - total_field_mask(self.m) * self.m.phase
        return np.where(self.mask, out, 0.0)


def run_sphere(prob, V, sphere, n_steps=None):
    """The FDTD march from rest with the shell DFT over [dft_begin, dft_end)."""
    model = build(prob, V)
    n_steps = prob.n_steps if n_steps is None else n_steps
    prev = np.zeros(model.v.shape, np.complex128)
    cur = np.zeros(model.v.shape, np.complex128)
    sd = ShellDFT(model, sphere)
    for n in range(n_steps):
        if prob.dft_begin <= n < prob.dft_end:
            sd.accumulate(cur, n)
        prev, cur = cur, step(model, prev, cur, n)
    return model, cur, sd
