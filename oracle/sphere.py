"""FP64 oracle of the spherical equivalence surface.

The paper integrates over the six faces of a box (Sections 3.1-3.2); a
sphere (the paper allows any closed surface) serves the 160^3 square-barrier
workload.  Test infrastructure only: imported by tests, never by the product.

Definition (reduced units, k = 1, x_bar = k0 x):
  * nodes s_q on the sphere of radius R: Gauss-Legendre in cos(theta)
    (n_theta nodes) times uniform phi (n_phi nodes), weights
    w_q = R^2 w_GL 2 pi / n_phi;
  * the running DFT (Eq. psiphasor, weight exp(i tau_n)) is taken on the
    shell of grid cells the interpolation stencils touch;
  * the incident part zeta psi_inc of the stored field is removed from the
    shell phasors (so stencils may reach into the taper walls);
  * node values psi_q and normal derivatives d_n psi_q come from separable
    Lagrange interpolation of `order` points per axis around each node
    (index space, derivative of the interpolant), normalised by the incident
    phasor at the origin like the box phasors (Eq. scaledphsiphasor);
  * Kirchhoff surface integral with G = exp(ikR)/(4 pi R), outward normal
    (k = 1 for the central wave, another reduced wavenumber for a phasor of
    a pulsed run):
      Psi(r) = -(1/4pi) sum_q w_q exp(ikR_q)/R_q
               [d_n psi_q + (-ik + 1/R_q) (n_q . (s_q - r) / R_q) psi_q],
      R_q = |r - s_q|;
    far field f(r_hat) = lim r e^{-ikr} Psi:
      f = -(1/4pi) sum_q w_q [d_n psi_q + ik (n_q . r_hat) psi_q] exp(-ik r_hat . s_q),
    in physical length units f / k0.
"""
from __future__ import annotations

import math

import numpy as np

from . import pstd as _pstd


def gauss_legendre(n):
    """Nodes and weights of n-point Gauss-Legendre quadrature on [-1, 1]
    (Newton iteration on P_n from the Chebyshev guess)."""
    x = np.cos(math.pi * (np.arange(1, n + 1) - 0.25) / (n + 0.5))
    for _ in range(100):
        p0 = np.ones_like(x)
        p1 = x.copy()
        for k in range(2, n + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        dp = n * (x * p1 - p0) / (x * x - 1)
        dx = p1 / dp
        x -= dx
        if np.abs(dx).max() < 1e-16:
            break
    p0 = np.ones_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    dp = n * (x * p1 - p0) / (x * x - 1)
    w = 2.0 / ((1 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order], w[order]


def lagrange(u, order):
    """Stencil start i0 and the `order` Lagrange weights (and derivative
    weights, per unit index) at fractional index u."""
    i0 = int(math.floor(u)) - (order // 2 - 1)
    xs = i0 + np.arange(order)
    L = np.ones(order)
    dL = np.zeros(order)
    for m in range(order):
        others = [xs[j] for j in range(order) if j != m]
        den = np.prod([xs[m] - xj for xj in others])
        L[m] = np.prod([u - xj for xj in others]) / den
        s = 0.0
        for a in range(order - 1):
            s += np.prod([u - others[b] for b in range(order - 1) if b != a])
        dL[m] = s / den
    return i0, L, dL


class Sphere:
    def __init__(self, prob, radius, n_theta=64, n_phi=128, order=8):
        self.prob = prob
        self.order = order
        self.k0 = prob.k0
        self.R = radius * prob.k0                     # reduced radius
        self.dxb = _pstd.dxbar(prob)
        ct, wt = gauss_legendre(n_theta)
        ph = 2 * math.pi * np.arange(n_phi) / n_phi
        st = np.sqrt(1 - ct * ct)
        C, P = np.meshgrid(ct, ph, indexing="ij")       # [theta][phi]
        S = np.sqrt(1 - C * C)
        self.normal = np.stack([S * np.cos(P), S * np.sin(P), C], -1).reshape(-1, 3)
        self.nodes = self.R * self.normal
        self.weights = (self.R ** 2 * wt[:, None] * (2 * math.pi / n_phi) * np.ones_like(P)).reshape(-1)
        del st
        # stencils in index space: u_a = x_a / h_a + N_a / 2
        self.stencils = []
        cells = set()
        n = prob.n
        for s in self.nodes:
            st3 = []
            for a in range(3):
                u = s[a] / self.dxb[a] + n[a] // 2
                i0, L, dL = lagrange(u, order)
                if i0 < 0 or i0 + order > n[a]:
                    raise ValueError("an interpolation stencil leaves the grid")
                st3.append((i0, L, dL))
            self.stencils.append(st3)
            (ix, _, _), (iy, _, _), (iz, _, _) = st3
            for k in range(iz, iz + order):
                for j in range(iy, iy + order):
                    for i in range(ix, ix + order):
                        cells.add((k, j, i))
        self.shell = sorted(cells)                    # (k, j, i), x fastest order

    def shell_mask(self):
        n = self.prob.n
        m = np.zeros((n[2], n[1], n[0]), dtype=bool)
        for (k, j, i) in self.shell:
            m[k, j, i] = True
        return m

    def node_values(self, field):
        """psi and d_n psi at the nodes from a [k][j][i] array of phasors (only
        shell cells are read)."""
        o = self.order
        val = np.zeros(len(self.nodes), np.complex128)
        dn = np.zeros(len(self.nodes), np.complex128)
        for q, ((ix, Lx, dLx), (iy, Ly, dLy), (iz, Lz, dLz)) in enumerate(self.stencils):
            blk = field[iz:iz + o, iy:iy + o, ix:ix + o]
            v = np.einsum("kji,k,j,i->", blk, Lz, Ly, Lx)
            gx = np.einsum("kji,k,j,i->", blk, Lz, Ly, dLx) / self.dxb[0]
            gy = np.einsum("kji,k,j,i->", blk, Lz, dLy, Lx) / self.dxb[1]
            gz = np.einsum("kji,k,j,i->", blk, dLz, Ly, Lx) / self.dxb[2]
            nq = self.normal[q]
            val[q] = v
            dn[q] = nq[0] * gx + nq[1] * gy + nq[2] * gz
        return val, dn

    def project(self, psi_q, dpsi_q, points_reduced, k=1.0):
        """Psi at reduced points outside the sphere (Kirchhoff integral with
        G = exp(ikR)/(4 pi R); k = 1 is the central wave)."""
        out = np.zeros(len(points_reduced), np.complex128)
        for o, r in enumerate(np.atleast_2d(points_reduced)):
            d = self.nodes - r[None, :]                  # s - r
            Rq = np.sqrt(np.sum(d * d, axis=1))
            ndr = np.sum(self.normal * d, axis=1) / Rq
            term = dpsi_q + (-1j * k + 1.0 / Rq) * ndr * psi_q
            out[o] = -np.sum(self.weights * np.exp(1j * k * Rq) / Rq * term) / (4 * math.pi)
        return out

    def far_field(self, psi_q, dpsi_q, dirs, k=1.0):
        """f(r_hat) in physical length units, for the wavenumber k (reduced)."""
        dirs = np.atleast_2d(dirs)
        out = np.zeros(len(dirs), np.complex128)
        for o, rh in enumerate(dirs):
            nr = self.normal @ rh
            ph = np.exp(-1j * k * (self.nodes @ rh))
            out[o] = -np.sum(self.weights * (dpsi_q + 1j * k * nr * psi_q) * ph) / (4 * math.pi)
        return out / self.k0


class ShellDFT:
    """Eq. psiphasor on the shell cells: Phi_c += exp(i tau_n) psi_c^n, and the
    incident phasor at the origin for the normalisation."""

    def __init__(self, model, sphere):
        self.m = model
        self.mask = sphere.shell_mask()
        self.phi = np.zeros(model.v.shape, np.complex128)
        self.inc = 0.0

    def accumulate(self, psi, n):
        tau = n * self.m.dtau
        self.phi[self.mask] += np.exp(1j * tau) * psi[self.mask]
        self.inc += _pstd.ramp(tau, self.m.tau_r)

    def normalized(self):
        """Scattered-field phasors on the shell: the total-field phasor minus
        the incident part.  The stored field is psi_s + zeta psi_inc (Eq.
        PSTD_TF-SF) and the DFT of zeta R(tau_n) exp(i(k.x - tau_n)) with
        weights exp(i tau_n) is zeta exp(i k.x) sum_n R(tau_n), so after the
        normalisation the incident part is zeta exp(i k.x) exactly."""
        out = self.phi / self.inc - self.m.zeta * self.m.phase
        return np.where(self.mask, out, 0.0)


def run(prob, V, sphere, n_steps=None):
    """The oracle march with the shell DFT over [dft_begin, dft_end)."""
    model = _pstd.build(prob, V)
    n_steps = prob.n_steps if n_steps is None else n_steps
    shape = model.v.shape
    prev = np.zeros(shape, np.complex128)
    cur = np.zeros(shape, np.complex128)
    sd = ShellDFT(model, sphere)
    for n in range(n_steps):
        if prob.dft_begin <= n < prob.dft_end:
            sd.accumulate(cur, n)
        prev, cur = cur, _pstd.step(model, prev, cur, n)
    return model, cur, sd
