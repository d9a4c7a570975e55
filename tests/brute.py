"""Brute-force references used to pin the oracle (dense, tiny dimensions only).

These are independent formulations of what the oracle computes:
  * the Liouvillian as an explicit n^2 x n^2 superoperator built from Kronecker
    products (row-major vectorisation: vec(A X B) = (A kron B^T) vec(X)),
    instead of the oracle's sparse commutator / anticommutator products;
  * the RK4 step as the Taylor polynomial P(z) = sum_{k<=4} z^k / k! of h*S;
  * the exact solution as scipy.linalg.expm(t S);
  * closed forms of the Jaynes-Cummings single-excitation sector and of a
    damped cavity.
"""
from __future__ import annotations

from math import factorial

import numpy as np
import scipy.linalg as sl


def dense(m):
    return m.toarray() if hasattr(m, "toarray") else np.asarray(m, np.complex128)


def superop(H, C, Hc=(), u=()):
    """S with vec(L y) = S vec(y) for L y = -i[H, y] + sum_k D[C_k] y."""
    H = dense(H).astype(np.complex128)
    for Hj, uj in zip(Hc, u):
        H = H + uj * dense(Hj)
    n = H.shape[0]
    Id = np.eye(n)
    S = -1j * (np.kron(H, Id) - np.kron(Id, H.T))
    for c in C:
        c = dense(c)
        cdc = c.conj().T @ c
        S = S + np.kron(c, c.conj()) - 0.5 * np.kron(cdc, Id) - 0.5 * np.kron(Id, cdc.T)
    return S


def comm_superop(V):
    """vec(-i[V, y]) = comm_superop(V) vec(y)."""
    V = dense(V)
    n = V.shape[0]
    Id = np.eye(n)
    return -1j * (np.kron(V, Id) - np.kron(Id, V.T))


def taylor(Z, order):
    out = np.eye(Z.shape[0], dtype=np.complex128)
    term = np.eye(Z.shape[0], dtype=np.complex128)
    for k in range(1, order + 1):
        term = term @ Z / k
        out = out + term
    return out


def rk4_map(S, h):
    """The RK4 step on a linear constant ODE equals P(hS), P = 4th-order Taylor."""
    return taylor(h * S, 4)


def dopri5_map(S, h):
    """Stability function of the Dormand-Prince fifth-order solution,
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/120 + z^6/600
    (Hairer & Wanner, Solving ODEs II, Sec. IV.2)."""
    Z = h * S
    return taylor(Z, 5) + np.linalg.matrix_power(Z, 6) / 600.0


def vec(rho):
    return np.asarray(rho, np.complex128).reshape(-1)


def unvec(v, n):
    return np.asarray(v).reshape(n, n)


def trace_distance(a, b):
    """T = 1/2 sum of singular values of (a - b)."""
    return 0.5 * np.sum(np.linalg.svd(np.asarray(a) - np.asarray(b), compute_uv=False))


def expm_states(S, rho0, times, t0=0.0):
    n = rho0.shape[0]
    return np.array([unvec(sl.expm((t - t0) * S) @ vec(rho0), n) for t in times])


def jc_single_excitation(t, wc, wa, g, kappa, gamma):
    """Closed form in the sector {|1,g>, |0,e>} of the damped JC model at zero
    temperature: the no-jump amplitude psi(t) = exp(-i Heff t) (1, 0), with
    Heff = [[wc - i kappa/2, g], [g, wa - i gamma/2]]; every jump lands in
    |0,g>, which carries no photon and sigma_z = -1.
    Returns (<a^+a>, <sigma_z>)."""
    Heff = np.array([[wc - 0.5j * kappa, g], [g, wa - 0.5j * gamma]])
    psi = sl.expm(-1j * Heff * t) @ np.array([1.0, 0.0])
    p1, p2 = abs(psi[0]) ** 2, abs(psi[1]) ** 2
    p0 = 1.0 - p1 - p2
    return p1, p2 - p1 - p0


def fact(k):
    return float(factorial(k))


def dopri5_error_map(S, h):
    """Embedded error estimate of one Dormand-Prince step on a linear constant
    ODE: y5 - y4 = E(hS) y with E = R - Rhat, where R is the fifth-order
    stability function above and Rhat that of the embedded fourth-order
    solution (with the first-same-as-last seventh stage),
    Rhat(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + 1097 z^5/120000
              + 161 z^6/120000 + z^7/24000,
    both obtained from the published Dormand & Prince (1980) tableau as
    1 + sum_k z^k b^T A^(k-1) 1.  Written as the difference polynomial
    E(z) = (-97 z^5 + 39 z^6 - 5 z^7) / 120000 to avoid cancellation."""
    Z = h * S
    Z5 = np.linalg.matrix_power(Z, 5)
    return (-97.0 * Z5 + 39.0 * Z5 @ Z - 5.0 * Z5 @ Z @ Z) / 120000.0


def rms_scaled(v, sc):
    """RMS over the complex moduli of v / sc (the adaptive error norm)."""
    return float(np.sqrt(np.mean((np.abs(v) / sc) ** 2)))


def heff(H, C):
    """Dense effective Hamiltonian H - (i/2) sum_n C_n^+ C_n (the non-Hermitian
    generator of the no-jump evolution)."""
    Hd = dense(H).astype(np.complex128)
    for c in C:
        c = dense(c)
        Hd = Hd - 0.5j * (c.conj().T @ c)
    return Hd


def nojump_state(H, C, psi0, t):
    """exp(-i H_eff t) psi0 (unnormalised)."""
    return sl.expm(-1j * heff(H, C) * t) @ np.asarray(psi0, np.complex128)
