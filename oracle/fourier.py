"""Closed-form convergence factors of the Robin-Schwarz iteration.

Test infrastructure (oracle).

Continuous, two half-spaces (Sec. 3: Omega = R^2, f = 0, Fourier transform in
the tangential variable): a tangential mode of frequency k is multiplied per
double iteration by

    rho(k) = (k - L1)(k - L2) / ((k + L1)(k + L2)),   L_s = Lambda^(s)(k),

with Lambda^(s) the symbol of the transmission operator; the non-local choice
L_s = |k| gives rho = 0 (convergence in two iterations, Sec. 3). For the
local family of Sec. 3 the symbol is read as p_s + q_s k^2 (a second-order
tangential operator whose symbol is positive; with the opposite sign the
coefficients of Table 1 give rates above one). For a finite subdomain of depth
a with a homogeneous Dirichlet far end, |k| is replaced by the exact
Dirichlet-to-Neumann symbol k coth(k a).

Discrete, one tangential mode: for a box split in two along x, a mode
v = v_y (x) v_z of the tangential generalised eigenproblems K v = mu M v stays
a single mode through the iteration, and the Robin datum is multiplied per
half iteration by (p - S)/(p + S), S the Schur complement at the interface
node of the 1D operator Kx + mu Mx on one side.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .direct import assemble_1d


def rho_halfspace(k, p1, q1=0.0, p2=None, q2=None):
    """rho(k) for the transmission symbols p_s + q_s k^2 (two half-spaces)."""
    p2 = p1 if p2 is None else p2
    q2 = q1 if q2 is None else q2
    k = np.asarray(k, float)
    L1 = p1 + q1 * k * k
    L2 = p2 + q2 * k * k
    return np.abs((k - L1) * (k - L2) / ((k + L1) * (k + L2)))


def rho_max(p1, q1, p2, q2, kmin, kmax, n=200001):
    """max of rho_halfspace over a frequency range (dense sampling)."""
    k = np.linspace(kmin, kmax, n)
    return float(np.max(rho_halfspace(k, p1, q1, p2, q2)))


def rho_finite_depth(k, p, depth):
    """Symmetric Robin p, both subdomains of the given depth with a Dirichlet
    far end: per double iteration ((s - p)/(s + p))^2, s = k coth(k depth)."""
    s = k / np.tanh(k * depth)
    return ((s - p) / (s + p)) ** 2


def tangential_modes(n_elem, h, lo, hi):
    """Generalised eigenpairs (mu, V) of the 1D Dirichlet-reduced factors."""
    K, M = assemble_1d(n_elem, h, lo, hi)
    mu, V = sla.eigh(K, M)
    return mu, V


def schur_interface(n_elem, h, mu, dirichlet_far=True, far_at_start=True):
    """Schur complement at the interface node of K + mu M on a 1D interval of
    n_elem Q2 elements, the other end Dirichlet (removed)."""
    if far_at_start:
        K, M = assemble_1d(n_elem, h, 1 if dirichlet_far else 0, 2 * n_elem)
        B = K + mu * M
        return 1.0 / np.linalg.inv(B)[-1, -1]
    K, M = assemble_1d(n_elem, h, 0, 2 * n_elem - (1 if dirichlet_far else 0))
    B = K + mu * M
    return 1.0 / np.linalg.inv(B)[0, 0]


def rho_discrete_two(n_elem_x, hx, mu, p):
    """Per double iteration factor ((S - p)/(S + p))^2 of a tangential mode with
    eigenvalue mu for a symmetric split into two halves of n_elem_x elements."""
    S = schur_interface(n_elem_x, hx, mu)
    return ((S - p) / (S + p)) ** 2


def grid_minimax(kind, kmin, kmax, n_grid=241, n_k=1001, lo=1e-3, hi=1e2):
    """Brute-force minimax of rho_max over a log-spaced grid of the two free
    coefficients (kind 1: p1, p2 of the zeroth-order unsymmetric condition;
    kind 2: p, q of the second-order symmetric condition). Returns
    (best rho_max, coefficients (p1, q1, p2, q2))."""
    k = np.linspace(kmin, kmax, n_k)
    g = np.exp(np.linspace(np.log(lo), np.log(hi), n_grid))
    best, arg = np.inf, None
    for a in g:
        if kind == 1:
            L1 = np.full_like(k, a)[None, :]
            L2 = g[:, None] + 0.0 * k[None, :]
            pq = lambda b: (a, 0.0, b, 0.0)
        elif kind == 2:
            L1 = a + g[:, None] * k[None, :] ** 2
            L2 = L1
            pq = lambda b: (a, b, a, b)
        else:
            raise ValueError(kind)
        r = np.abs((k - L1) * (k - L2) / ((k + L1) * (k + L2))).max(axis=1)
        j = int(np.argmin(r))
        if r[j] < best:
            best, arg = float(r[j]), pq(g[j])
    return best, arg


def oo0_symmetric_optimum(kmin, kmax):
    """Closed-form minimax of ((k - p)/(k + p))^2 on [kmin, kmax]: the two end
    frequencies equioscillate at p = sqrt(kmin kmax)."""
    p = np.sqrt(kmin * kmax)
    return p, ((np.sqrt(kmax) - np.sqrt(kmin)) / (np.sqrt(kmax) + np.sqrt(kmin))) ** 2
