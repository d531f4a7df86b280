"""FP64 oracle of the Fresnel-plane intensity misfit and its gradient with
respect to the voxel potential (the exact discrete adjoint of the PSTD run,
Eq. PSTDupdating, of the surface DFT, Eqs. psiphasor / dpsiphasor /
scaledphsiphasor, and of the box projection, Eqs. bottomPsi_lm ... Psi).

Misfit (total-field detector intensity, incident wave exp(i k.r)):
    J(V) = 1/2 sum_o (|psi_inc(r_o) + Psi_o(V)|^2 - I_o)^2.

Discrete forward model (reduced units), n = 0 .. N-1, psi^{-1} = psi^0 = 0:
    psi^{n+1} = Gamma (psi^{n-1} - i A psi^n - i sigma_n s),
    A = 2 dtau (eta K + v),  v = V / E0,  K = sum_a F_a^-1 kbar_a^2 F_a.
A is real and symmetric, Gamma real and diagonal.  With the Lagrange
multipliers mu of the step equations, stationarity gives, m = N .. 1,
    mu^m = Gamma mu^{m+2} + i A Gamma mu^{m+1} + e_m,   mu^{N+1} = mu^{N+2} = 0,
where e_m is the adjoint of the surface DFT applied to h = G^H g / Phi_inc
(G the projection, g_o = dJ/d conj(Psi_o) = (|T_o|^2 - I_o) T_o), and
    dJ/dV_c = (4 dtau / E0) Gamma_c sum_{n=0}^{N-1} Im(conj(mu_c^{n+1}) psi_c^n).

Every linear map has its adjoint written out below; dot-product tests and
finite differences pin them (tests/test_oracle_adjoint.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import fft as _fft
from . import ntdf as _ntdf
from . import pstd as _pstd


# ----------------------------------------------------------------------------
# forward pieces as explicit linear maps
# ----------------------------------------------------------------------------

def forward_states(model, n_steps):
    """psi^0 .. psi^N of the forward run from rest (all kept: small grids)."""
    shape = model.v.shape
    prev = np.zeros(shape, np.complex128)
    cur = np.zeros(shape, np.complex128)
    states = [cur]
    for n in range(n_steps):
        prev, cur = cur, _pstd.step(model, prev, cur, n)
        states.append(cur)
    return states


def surface_phasors(model, states):
    """Normalised phasors (Eqs. psiphasor, dpsiphasor, scaledphsiphasor) over
    the window [dft_begin, dft_end) of the given states."""
    p = model.prob
    sd = _pstd.SurfaceDFT(model)
    for n in range(p.dft_begin, min(p.dft_end, len(states) - 1)):
        sd.accumulate(states[n], n)
    phi, dphi = sd.normalized()
    return phi, dphi, sd.inc.real


def surface_adjoint(model, n, hphi, hdphi, inc):
    """e_n = conj(w_n) B^H h / Phi_inc: the adjoint of psi^n -> w_n B psi^n / Phi_inc,
    B = (plane values, plane values of the spectral normal derivative)."""
    p = model.prob
    out = np.zeros(model.v.shape, np.complex128)
    w = np.exp(1j * n * model.dtau)
    for f in range(6):
        a, _ = _pstd.FACES[f]
        idx = _pstd.face_index(p, f)
        ax = _pstd.NPAX[a]
        # plane extraction^H: put h on the plane
        inj = np.zeros_like(out)
        sl = [slice(None)] * 3
        sl[ax] = idx
        inj[tuple(sl)] = hdphi[f]
        # derivative^H = F^-1 conj(i kbar) F applied to the injected plane
        d = _fft.ifft(np.conj(1j * _pstd._bcast(model.kb[a], a)) * _fft.fft(inj, axis=ax), axis=ax)
        out += d
        out[tuple(sl)] += hphi[f]
    return np.conj(w) * out / inc


# ----------------------------------------------------------------------------
# projection and its adjoint (Taylor form of the cell formula)
# ----------------------------------------------------------------------------

class Projection:
    """Psi(points) = G (phi, dphi) with the 8th-order sinc expansion; the
    map is linear in the phasors: plane DFT -> expansion tables -> cell sums."""

    def __init__(self, box, points, order=8, k=1.0):
        self.box = box
        self.points = np.atleast_2d(np.asarray(points, dtype=np.float64))
        self.order = order
        self.k = k
        self.faces = []
        for f in range(6):
            a, b, c, idx, sign = box.face(f)
            U = self._table(b, order)   # [p, L, Nb]
            Vt = self._table(c, order)  # [q, M, Nc]
            Nb, Nc = box.n[b], box.n[c]
            db, dc = box.dxb[b], box.dxb[c]
            xa = box.coord(a, idx)
            yb = box.cell_centres(b)[None, :]
            yc = box.cell_centres(c)[:, None]
            pref = sign * db * dc / (4 * math.pi * Nb * Nc)
            # per point: weights W[o, p, q, m, l] folded with the Green factor
            Wp, Wd = [], []
            for r in self.points:
                Ra = r[a] - xa
                Rb = r[b] - yb
                Rc = r[c] - yc
                Rn = np.sqrt(Ra * Ra + Rb * Rb + Rc * Rc)
                ab = k * db * (Rb / Rn) / 2
                ac = k * dc * (Rc / Rn) / 2
                E = pref * np.exp(1j * k * Rn) / Rn
                coef = (1j * k - 1.0 / Rn) * (Ra / Rn)
                powb = np.stack([ab ** p for p in range(order + 1)])  # [p, M, L]
                powc = np.stack([ac ** q for q in range(order + 1)])
                base = powb[:, None] * powc[None, :]                 # [p, q, M, L]
                Wd.append(base * E)
                Wp.append(base * E * coef)
            self.faces.append((U, Vt, np.array(Wp), np.array(Wd)))

    def _table(self, ax, order):
        box = self.box
        N = box.n[ax]
        L = N * box.dxb[ax]
        bp = _ntdf.signed_index(N)
        s = _ntdf.sinc_taylor_coeffs(math.pi * bp / N, order)
        xcs = box.cell_centres(ax)
        base = np.where(bp % 2 == 0, 1.0, -1.0)[None, :] * np.exp(2j * math.pi * xcs[:, None] * bp[None, :] / L)
        return base[None, :, :] * s[:, None, :]

    def apply(self, phi, dphi):
        out = np.zeros(len(self.points), np.complex128)
        for f in range(6):
            U, Vt, Wp, Wd = self.faces[f]
            Fp = _fft.fft2(phi[f])
            Fd = _fft.fft2(dphi[f])
            Qp = np.einsum("qmc,cb,plb->pqml", Vt, Fp, U, optimize=True)
            Qd = np.einsum("qmc,cb,plb->pqml", Vt, Fd, U, optimize=True)
            out += np.einsum("opqml,pqml->o", Wp, Qp, optimize=True)
            out += np.einsum("opqml,pqml->o", Wd, Qd, optimize=True)
        return out

    def adjoint(self, g):
        """(G^H g) split into per-face psi and dpsi planes."""
        hphi, hdphi = [], []
        for f in range(6):
            U, Vt, Wp, Wd = self.faces[f]
            Qp_bar = np.einsum("opqml,o->pqml", np.conj(Wp), g, optimize=True)
            Qd_bar = np.einsum("opqml,o->pqml", np.conj(Wd), g, optimize=True)
            # Q = V F U^T  ->  F_bar = sum_pq V^H Q_bar conj(U)
            Fp_bar = np.einsum("qmc,pqml,plb->cb", np.conj(Vt), Qp_bar, np.conj(U), optimize=True)
            Fd_bar = np.einsum("qmc,pqml,plb->cb", np.conj(Vt), Qd_bar, np.conj(U), optimize=True)
            # F = fft2(x) -> x_bar = fft2^H(F_bar) = N_b N_c ifft2(F_bar)
            nb = Fp_bar.shape[0] * Fp_bar.shape[1]
            hphi.append(nb * _fft.ifft(_fft.ifft(Fp_bar, axis=0), axis=1))
            hdphi.append(nb * _fft.ifft(_fft.ifft(Fd_bar, axis=0), axis=1))
        return hphi, hdphi


# ----------------------------------------------------------------------------
# misfit, gradient
# ----------------------------------------------------------------------------

def misfit(prob, V, points_phys, target_I, n_steps=None, order=8):
    """J, and the intermediate quantities the gradient needs."""
    model = _pstd.build(prob, V)
    n_steps = prob.n_steps if n_steps is None else n_steps
    states = forward_states(model, n_steps)
    phi, dphi, inc = surface_phasors(model, states)
    box = _ntdf.Box(prob.n, model.dxb, prob.surf_lo, prob.surf_hi)
    pts = np.atleast_2d(points_phys) * prob.k0
    G = Projection(box, pts, order=order)
    Psi = G.apply(phi, dphi)
    # incident wave at the detector, exp(i k_hat . r_bar)
    T = np.exp(1j * pts @ model.kh) + Psi
    r = np.abs(T) ** 2 - np.asarray(target_I)
    J = 0.5 * float(np.sum(r * r))
    return J, dict(model=model, states=states, inc=inc, G=G, T=T, r=r, Psi=Psi)


def intensity(prob, V, points_phys, n_steps=None, order=8):
    _, aux = misfit(prob, V, points_phys, np.zeros(len(np.atleast_2d(points_phys))), n_steps, order)
    return np.abs(aux["T"]) ** 2


def gradient(prob, V, points_phys, target_I, n_steps=None, order=8):
    """dJ/dV (energy units) by the discrete adjoint."""
    J, aux = misfit(prob, V, points_phys, target_I, n_steps, order)
    model, states, inc, G = aux["model"], aux["states"], aux["inc"], aux["G"]
    g = aux["r"] * aux["T"]                     # dJ / d conj(Psi)
    hphi, hdphi = G.adjoint(g)
    N = len(states) - 1
    p = model.prob
    dt = model.dtau
    shape = model.v.shape
    mu_next2 = np.zeros(shape, np.complex128)   # mu^{m+2}
    mu_next1 = np.zeros(shape, np.complex128)   # mu^{m+1}
    grad = np.zeros(shape)
    Gam = model.Gamma
    for m in range(N, 0, -1):
        x = Gam * mu_next1
        Ax = 2 * dt * (model.eta * _pstd.kinetic(model, x) + model.v * x)
        mu = Gam * mu_next2 + 1j * Ax
        if p.dft_begin <= m < min(p.dft_end, N):   # psi^N is not in the window sum
            mu = mu + surface_adjoint(model, m, hphi, hdphi, inc)
        # mu^m pairs with psi^{m-1}
        grad += Gam * np.imag(np.conj(mu) * states[m - 1])
        mu_next2, mu_next1 = mu_next1, mu
    E0 = _pstd.central_energy(p)
    return J, (4 * dt / E0) * grad


def tangent(prob, V, dV, points_phys, target_I, n_steps=None, order=8):
    """dJ in the direction dV by the tangent-linear model (forward mode)."""
    J, aux = misfit(prob, V, points_phys, target_I, n_steps, order)
    model, states, inc, G = aux["model"], aux["states"], aux["inc"], aux["G"]
    E0 = _pstd.central_energy(prob)
    dv = np.asarray(dV) / E0
    dt = model.dtau
    N = len(states) - 1
    shape = model.v.shape
    dprev = np.zeros(shape, np.complex128)
    dcur = np.zeros(shape, np.complex128)
    dstates = [dcur]
    for n in range(N):
        rhs = dprev - 2j * dt * (model.eta * _pstd.kinetic(model, dcur) + model.v * dcur) \
            - 2j * dt * dv * states[n]
        dprev, dcur = dcur, model.Gamma * rhs
        dstates.append(dcur)
    sd = _pstd.SurfaceDFT(model)
    for n in range(prob.dft_begin, min(prob.dft_end, N)):
        sd.accumulate(dstates[n], n)
    dphi = [x / inc for x in sd.phi]
    ddphi = [x / inc for x in sd.dphi]
    dPsi = G.apply(dphi, ddphi)
    g = aux["r"] * aux["T"]
    return J, 2.0 * float(np.real(np.vdot(g, dPsi)))
