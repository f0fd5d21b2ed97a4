"""Independent forms of the discrete equations, used to pin the oracle.

The oracle assembles the per-cell matrix of the paper's eq. (Aj) and the
right-hand side of eq. (rhs_sg).  This module does not: it writes the four
corner-balance equations (scb-mb-a..d) as residuals, with the cell-midpoint
closure (average of the two corners) and the upstream edge closure spelled out
as edge values, exactly as the balances read.  A wrong entry, sign or index in
the oracle's matrix or right-hand side therefore makes the oracle's answers
disagree with the solutions and spectra computed here.

Quadrature comes from numpy's leggauss, not from the oracle.

Everything is vectorised over a leading batch axis so the global matrix of
the discrete system can be built column by column (the residual is affine in
the unknowns).
"""
from __future__ import annotations

import numpy as np


def quadrature(N):
    mu, w = np.polynomial.legendre.leggauss(N)
    return mu, w


def residual(prob, psi, psi_prev, q=None, q_ang=None, inc_l=None, inc_r=None,
             periodic=False, nb_factor=None, scatter=True):
    """Residuals of eqs. (scb-mb-a..d) for every (cell, group, angle).

    psi      [..., J, G, N, 4]  (k,L), (k,R), (k+1/2,L), (k+1/2,R)
    psi_prev [..., J, G, N, 2]  corners at t_{k-1/2}
    q        [J, G, 4] isotropic source, or q_ang [J, G, N, 4] angular source
    nb_factor  optional pair (fl, fr) multiplying every value taken from the
               left / right neighbour (Fourier modes; implies periodic)
    scatter  False drops the scattering source (for the SI splitting)
    Returns R [..., J, G, N, 4] with R = 0 for the discrete solution.
    """
    J, N, G = prob["J"], prob["N"], prob["G"]
    mu, w = quadrature(N)
    dx = prob["dx"][:, None, None]                      # [J,1,1]
    sig = prob["sigma_t"][:, :, None]                   # [J,G,1]
    v = prob["speed"][None, :, None]                    # [1,G,1]
    dt = prob["dt"]
    m = mu[None, None, :]                               # [1,1,N]
    kL, kR, hL, hR = (psi[..., u] for u in range(4))
    pL, pR = psi_prev[..., 0], psi_prev[..., 1]

    # scalar flux and scattering source, per corner/time level
    phi = np.einsum("n,...jgnu->...jgu", w, psi)         # [...,J,G,4]
    if scatter:
        scat = np.einsum("jgh,...jhu->...jgu", prob["sigma_s"], phi)
    else:
        scat = np.zeros_like(phi)
    # source density in the balances: (1/2)(Ss phi + Q) isotropic, or q_ang
    src = 0.5 * scat[..., None, :]                      # [...,J,G,1,4]
    if q_ang is not None:
        src = src + q_ang
    elif q is not None:
        src = src + 0.5 * q[:, :, None, :]

    # edge values from the upstream closure
    pos = (mu > 0)[None, None, :]
    fl, fr = (1.0, 1.0) if nb_factor is None else nb_factor
    per = periodic or nb_factor is not None

    def from_left(x):      # value of the right corner of cell j-1
        y = np.roll(x, 1, axis=-3) * fl
        if not per:
            y = y.copy()
            y[..., 0, :, :] = 0.0
        return y

    def from_right(x):     # value of the left corner of cell j+1
        y = np.roll(x, -1, axis=-3) * fr
        if not per:
            y = y.copy()
            y[..., -1, :, :] = 0.0
        return y

    def inc_edge(inc, lev, side):
        out = np.zeros(kL.shape[-3:])
        if inc is not None and not per:
            h = N // 2
            if side == "l":
                out[0, :, h:] = inc[lev]
            else:
                out[-1, :, :h] = inc[lev]
        return out

    # left edge x_{j-1/2} and right edge x_{j+1/2} at time levels k and k+1/2
    eL_k = np.where(pos, from_left(kR) + inc_edge(inc_l, 0, "l"), kL)
    eR_k = np.where(pos, kR, from_right(kL) + inc_edge(inc_r, 0, "r"))
    eL_h = np.where(pos, from_left(hR) + inc_edge(inc_l, 1, "l"), hL)
    eR_h = np.where(pos, hR, from_right(hL) + inc_edge(inc_r, 1, "r"))

    half = dx / 2.0
    Ra = (half / v * (hL - pL) / dt + m * ((kL + kR) / 2 - eL_k) + half * sig * kL
          - half * src[..., 0])
    Rb = (half / v * (hR - pR) / dt + m * (eR_k - (kL + kR) / 2) + half * sig * kR
          - half * src[..., 1])
    Rc = (half / v * (hL - kL) / (dt / 2) + m * ((hL + hR) / 2 - eL_h) + half * sig * hL
          - half * src[..., 2])
    Rd = (half / v * (hR - kR) / (dt / 2) + m * (eR_h - (hL + hR) / 2) + half * sig * hR
          - half * src[..., 3])
    return np.stack([Ra, Rb, Rc, Rd], axis=-1)


def direct_solve(prob, psi_prev, q=None, q_ang=None, inc_l=None, inc_r=None,
                 periodic=False):
    """Solve the whole discrete system of one time step with numpy (tiny sizes)."""
    J, N, G = prob["J"], prob["N"], prob["G"]
    nu = J * G * N * 4
    zero_prev = np.zeros_like(psi_prev)
    eye = np.eye(nu).reshape(nu, J, G, N, 4)
    M = residual(prob, eye, zero_prev, periodic=periodic).reshape(nu, nu).T
    f = -residual(prob, np.zeros((J, G, N, 4)), psi_prev, q=q, q_ang=q_ang,
                  inc_l=inc_l, inc_r=inc_r, periodic=periodic).reshape(nu)
    return np.linalg.solve(M, f).reshape(J, G, N, 4)


def _mode_matrices(prob1, theta):
    """Per-mode operators of the homogeneous single-cell problem.

    Returns (A_own, A_nb, S) with the residual of a Fourier mode a e^{i theta j}
    being (A_own + A_nb) a; A_own excludes the values taken from neighbours and
    S is the scattering part of A_own (sign as in the residual).
    """
    J, N, G = 1, prob1["N"], prob1["G"]
    nu = G * N * 4
    eye = np.eye(nu, dtype=complex).reshape(nu, 1, G, N, 4)
    zp = np.zeros((1, G, N, 2))
    f = (np.exp(-1j * theta), np.exp(1j * theta))
    full = residual(prob1, eye, zp, nb_factor=f).reshape(nu, nu).T
    own = residual(prob1, eye, zp, nb_factor=(0.0, 0.0)).reshape(nu, nu).T
    own_ns = residual(prob1, eye, zp, nb_factor=(0.0, 0.0), scatter=False).reshape(nu, nu).T
    del J
    return own, full - own, own - own_ns


def oci_symbol(prob1, theta):
    """Fourier symbol of the OCI iteration, T = -(A_own)^-1 A_nb."""
    own, nb, _ = _mode_matrices(prob1, theta)
    return -np.linalg.solve(own, nb)


def si_symbol(prob1, theta):
    """Fourier symbol of SI, T = -(A_own - S + A_nb)^-1 S (scattering lagged)."""
    own, nb, S = _mode_matrices(prob1, theta)
    return -np.linalg.solve(own - S + nb, S)


def one_cell(prob, j=0):
    """The single-cell problem with the material of cell j (for symbols)."""
    return dict(J=1, N=prob["N"], G=prob["G"], dx=prob["dx"][j:j + 1],
                sigma_t=prob["sigma_t"][j:j + 1], sigma_s=prob["sigma_s"][j:j + 1],
                speed=prob["speed"], dt=prob["dt"])
