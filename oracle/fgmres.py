"""Flexible GMRES (oracle, test infrastructure only).

Right-preconditioned flexible GMRES in the recurrence of Algorithm 1
(x0 = 0, r0 = b - A x0, v1 = r0/beta; z_j = M(v_j); w = A z_j; modified
Gram-Schmidt against v_1..v_j -- the paper's inner loop subtracts h_ij v_j,
read as v_i; h_{j+1,j} = ||w||; least-squares update y_j and x_j = x0 + Z_j y_j).

The least-squares problem is solved with complex Givens rotations:
for the pair (a, b) = (H[j,j], H[j+1,j]),
    rho = sqrt(|a|^2 + |b|^2),  c = |a|/rho,  s = (a/|a|) conj(b)/rho
    (c = 0, s = 1 when a = 0),
so [c s; -conj(s) c] [a; b] = [(a/|a|) rho; 0], and the residual estimate is
updated as gamma_{j+1} = -conj(s) gamma_j, gamma_j <- c gamma_j.

``fgmres``       restarted outer solver; the stopping test compares |gamma|/||b||
                 with tol and confirms with an explicit residual at cycle end.
``fgmres_fixed`` no-restart inner solver (Algorithm 1 inference branch) that stops
                 when |gamma_{j+1}|/||b|| <= r_th or after N steps.
"""
from __future__ import annotations

import numpy as np


def givens(a, b):
    if a == 0:
        return 0.0, 1.0 + 0j
    rho = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    c = abs(a) / rho
    s = (a / abs(a)) * np.conj(b) / rho
    return c, s


def _arnoldi_cycle(Aop, M, r0, beta, bnorm, tol, max_steps, hist, breakdown_rtol):
    n = r0.shape[0]
    V = np.zeros((max_steps + 1, n), dtype=np.complex128)
    Z = np.zeros((max_steps, n), dtype=np.complex128)
    H = np.zeros((max_steps + 1, max_steps), dtype=np.complex128)
    cs = np.zeros(max_steps)
    sn = np.zeros(max_steps, dtype=np.complex128)
    gam = np.zeros(max_steps + 1, dtype=np.complex128)
    gam[0] = beta
    V[0] = r0 / beta
    k = 0
    converged = False
    for j in range(max_steps):
        out = M(V[j])
        if isinstance(out, tuple):
            z, w = out
            w = np.array(w, dtype=np.complex128)
        else:
            z = out
            w = Aop(z)
        Z[j] = z
        wnorm_pre = np.linalg.norm(w)
        for i in range(j + 1):                     # modified Gram-Schmidt
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        for i in range(j):                         # previous rotations
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        c, s = givens(H[j, j], H[j + 1, j])
        cs[j], sn[j] = c, s
        H[j, j] = c * H[j, j] + s * H[j + 1, j]
        H[j + 1, j] = 0.0
        gam[j + 1] = -np.conj(s) * gam[j]
        gam[j] = c * gam[j]
        k = j + 1
        res = abs(gam[j + 1]) / bnorm
        hist.append(res)
        breakdown = np.linalg.norm(w) <= breakdown_rtol * wnorm_pre
        if res <= tol or breakdown:
            converged = res <= tol
            break
        V[j + 1] = w / np.linalg.norm(w)
    y = np.zeros(k, dtype=np.complex128)
    for i in range(k - 1, -1, -1):                 # back substitution H y = gamma
        y[i] = (gam[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    return Z[:k].T @ y, k, converged


def fgmres(Aop, b, M=None, tol=1e-6, restart=30, max_iters=1000, x0=None,
           breakdown_rtol=1e-14):
    """Restarted flexible GMRES; M(v) returns z or (z, A z).

    Returns (x, iters, hist, explicit_rel_residual).  ``iters`` counts
    preconditioner applications; ``hist`` holds |gamma_{j+1}|/||b|| per step.
    """
    if M is None:
        M = lambda v: v.copy()
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    hist = []
    iters = 0
    if bnorm == 0:
        return np.zeros_like(b), 0, hist, 0.0
    while True:
        r = b - Aop(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol or iters >= max_iters:
            return x, iters, hist, beta / bnorm
        steps = min(restart, max_iters - iters)
        dx, k, _ = _arnoldi_cycle(Aop, M, r, beta, bnorm, tol, steps, hist, breakdown_rtol)
        x = x + dx
        iters += k


def fgmres_fixed(Aop, b, M, r_th, N, breakdown_rtol=1e-14):
    """Inner NN-FGMRES: x0 = 0, no restart, stop at |gamma|/||b|| <= r_th or N steps.

    Returns (x, steps, hist).
    """
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0 or N <= 0:
        return np.zeros_like(b), 0, []
    hist = []
    x, k, _ = _arnoldi_cycle(Aop, M, b, bnorm, bnorm, r_th, N, hist, breakdown_rtol)
    return x, k, hist
