"""FP64 oracle of the overlapping-subdomain PSTD with local Fourier basis
(Section 2.6, Eq. weight).

The global grid is cut into blocks whose cores tile it.  Each block holds a
local array of core + 2 * halo points per axis; the halo is copied from the
neighbouring cores and multiplied by smoothing weights, counted from the
distal end: one zero point (against FFT wrap-around), n_t points weighted
w[l] = xi(l / (n_t + 1)), l = 1..n_t, and the remaining halo points unchanged
(at least 4 of them: halo >= n_t + 5).  Eq. PSTDupdating then runs with the
local FFT lengths, and only core points are updated.  Points of a local array
outside the global grid are zero.

Readings: weights are separable over the three axes; edge and corner halos
are read from the global array like the face halos.
"""
from __future__ import annotations

import math

import numpy as np

from . import fft as _fft
from .pstd import NPAX, _bcast, kbar, ramp, step as global_step, xi


def halo_weights(halo, n_t):
    """Weights of one halo, distal to proximal (Eq. weight)."""
    if halo < n_t + 5:
        raise ValueError("the halo must be at least n_t + 5 points")
    w = np.ones(halo)
    w[0] = 0.0
    for l in range(1, n_t + 1):
        w[l] = xi(l / (n_t + 1))
    return w


def local_weights(core, halo, n_t):
    w = halo_weights(halo, n_t)
    return np.concatenate([w, np.ones(core), w[::-1]])


class Blocks:
    def __init__(self, n, core, halo, n_t):
        self.n = tuple(n)
        self.core = tuple(core)
        self.halo = halo
        self.n_t = n_t
        for a in range(3):
            if self.n[a] % self.core[a]:
                raise ValueError("cores must tile the global grid")
        self.count = tuple(self.n[a] // self.core[a] for a in range(3))
        self.nloc = tuple(self.core[a] + 2 * halo for a in range(3))
        self.w = [local_weights(self.core[a], halo, n_t) for a in range(3)]

    def window(self, a, b):
        """Global indices of block b's local points along axis a."""
        return np.arange(b * self.core[a] - self.halo, (b + 1) * self.core[a] + self.halo)

    def local(self, psi, bx, by, bz):
        """Weighted local array of block (bx, by, bz), [k][j][i]."""
        idx = [self.window(0, bx), self.window(1, by), self.window(2, bz)]
        out = np.zeros((self.nloc[2], self.nloc[1], self.nloc[0]), np.complex128)
        ok = [(g >= 0) & (g < self.n[a]) for a, g in enumerate(idx)]
        sub = psi[np.ix_(idx[2][ok[2]], idx[1][ok[1]], idx[0][ok[0]])]
        out[np.ix_(np.where(ok[2])[0], np.where(ok[1])[0], np.where(ok[0])[0])] = sub
        W = _bcast(self.w[0], 0) * _bcast(self.w[1], 1) * _bcast(self.w[2], 2)
        return out * W


def kinetic(model, blocks, psi):
    """sum_a F_a^-1[kbar_a^2 F_a] evaluated block by block on the weighted
    local arrays; each global point takes the value of the block whose core
    holds it."""
    out = np.zeros_like(psi, dtype=np.complex128)
    kb2 = [kbar(blocks.nloc[a], model.dxb[a]) ** 2 for a in range(3)]
    h = blocks.halo
    for bz in range(blocks.count[2]):
        for by in range(blocks.count[1]):
            for bx in range(blocks.count[0]):
                loc = blocks.local(psi, bx, by, bz)
                L = np.zeros_like(loc)
                for a in range(3):
                    ax = NPAX[a]
                    L += _fft.ifft(_bcast(kb2[a], a) * _fft.fft(loc, axis=ax), axis=ax)
                c = blocks.core
                out[bz * c[2]:(bz + 1) * c[2], by * c[1]:(by + 1) * c[1], bx * c[0]:(bx + 1) * c[0]] = \
                    L[h:h + c[2], h:h + c[1], h:h + c[0]]
    return out


def derivative(model, blocks, psi, a, idx):
    """Spectral normal derivative on the plane idx of axis a, from the local
    arrays of the blocks whose cores contain that plane."""
    b = idx // blocks.core[a]
    shape = list(psi.shape)
    shape[NPAX[a]] = 1
    out = np.zeros(shape, np.complex128).squeeze(axis=NPAX[a])
    kb = kbar(blocks.nloc[a], model.dxb[a])
    h = blocks.halo
    c = blocks.core
    local_pos = idx - b * c[a] + h
    for bz in range(blocks.count[2]):
        for by in range(blocks.count[1]):
            for bx in range(blocks.count[0]):
                if (bx, by, bz)[a] != b:
                    continue
                loc = blocks.local(psi, bx, by, bz)
                ax = NPAX[a]
                d = _fft.ifft(1j * _bcast(kb, a) * _fft.fft(loc, axis=ax), axis=ax)
                d = np.take(d, local_pos, axis=ax)
                # core part of the two transverse axes
                sl = []
                for t in range(3):
                    if t == a:
                        continue
                    sl.append(slice(h, h + c[t]))
                tgt = []
                for t in range(3):
                    if t == a:
                        continue
                    bb = (bx, by, bz)[t]
                    tgt.append(slice(bb * c[t], (bb + 1) * c[t]))
                # plane arrays are [slow][fast] = reversed transverse axis order
                out[tgt[1], tgt[0]] = d[sl[1], sl[0]]
    return out


def step(model, blocks, psi_prev, psi_cur, n):
    """Eq. PSTDupdating with the kinetic term of the local blocks."""
    dt = model.dtau
    tau = n * dt
    amp = ramp(tau, model.tau_r) * np.exp(-1j * tau)
    pinc = amp * model.phase
    S = model.lap_zeta * pinc + 2.0 * sum(model.grad_zeta[a] * 1j * model.kh[a] * pinc for a in range(3))
    if model.prob.eta_on_source:
        S = model.eta * S
    rhs = psi_prev - 2j * model.eta * dt * kinetic(model, blocks, psi_cur) - 2j * dt * model.v * psi_cur \
        - 2j * dt * S
    return model.Gamma * rhs


def step_at(model, blocks, psi_prev, psi_cur, n, points):
    """psi^{n+1} of the subdomain scheme at selected points.  A point lies in
    the core of exactly one block; there the weights of the two transverse
    axes are 1, so each axis term needs only the weighted local pencil
    along that axis."""
    from .pstd import step_at as global_step_at  # source, potential and mask terms
    out = []
    dt = model.dtau
    h = blocks.halo
    for (i, j, k) in points:
        pos = (i, j, k)
        kin = 0.0 + 0.0j
        for a in range(3):
            b = pos[a] // blocks.core[a]
            idx = blocks.window(a, b)
            ok = (idx >= 0) & (idx < blocks.n[a])
            pen = np.zeros(blocks.nloc[a], np.complex128)
            full = (psi_cur[k, j, :], psi_cur[k, :, i], psi_cur[:, j, i])[a]
            pen[ok] = full[idx[ok]]
            pen = pen * blocks.w[a]
            kb2 = kbar(blocks.nloc[a], model.dxb[a]) ** 2
            kin += _fft.ifft(kb2 * _fft.fft(pen))[pos[a] - b * blocks.core[a] + h]
        ref_global = global_step_at(model, psi_prev, psi_cur, n, [pos])[0]
        # replace the global kinetic term of the same formula by the local one
        glob_kin = 0.0 + 0.0j
        for a in range(3):
            full = (psi_cur[k, j, :], psi_cur[k, :, i], psi_cur[:, j, i])[a]
            glob_kin += _fft.ifft(model.kb2[a] * _fft.fft(full))[pos[a]]
        out.append(ref_global - model.Gamma[k, j, i] * 2j * model.eta * dt * (kin - glob_kin))
    return np.array(out)
