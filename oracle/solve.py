"""Master equation, dense direct solve, block-diagonal preconditioner and
reference GMRES and BiCGSTAB solvers (paper, Section 2.2 eqs.
"masterequation" and "M"; Section 3.2 and 3.2.1).

    M^{ii'}_{nn'} = delta_{nn'} delta_{ii'} - T^i_{nn} W^{ii'}_{nn'}     (T diagonal)
    M b = T a_in
"""
import math

import numpy as np
import scipy.linalg as sla

from .translation import coupling_matrix
from .mie import T_vector


def wavenumber(n0, wavelength):
    return 2.0 * math.pi * n0 / wavelength


def master_matrix(pos, radii, n_sphere, n0, wavelength, L, hankel=None):
    k = wavenumber(n0, wavelength)
    W = coupling_matrix(pos, k, L, hankel)
    t = T_vector(L, k, radii, n_sphere, n0).reshape(-1)
    M = np.eye(W.shape[0], dtype=np.complex128) - t[:, None] * W
    return M, W, t


def solve_dense(M, rhs):
    """b = M^{-1} rhs by LU with partial pivoting (LAPACK getrf/getrs)."""
    lu, piv = sla.lu_factor(M)
    return sla.lu_solve((lu, piv), rhs)


def partition(pos, edge):
    """Cuboid partition of Section 3.2.1, step 1.

    Cells are cubes of the given edge anchored at the minimum corner of the
    centres' bounding box; a sphere belongs to cell floor((r - r_min)/edge).
    Spheres are re-ordered by (cell linear index with x fastest, then y, then
    z; original index), empty cells are skipped.  Returns (perm, offsets):
    perm[new] = old, block j holds perm[offsets[j]:offsets[j+1]].
    """
    pos = np.asarray(pos, dtype=np.float64)
    lo = pos.min(axis=0)
    c = np.floor((pos - lo) / edge).astype(np.int64)
    nc = c.max(axis=0) + 1
    lin = c[:, 0] + nc[0] * (c[:, 1] + nc[1] * c[:, 2])
    perm = np.lexsort((np.arange(pos.shape[0]), lin))
    sl = lin[perm]
    starts = np.nonzero(np.r_[True, sl[1:] != sl[:-1]])[0]
    offsets = np.r_[starts, pos.shape[0]]
    return perm, offsets


class BlockDiagonalPreconditioner:
    """Blocks M_j of M restricted to each cuboid (steps 2-4 of Section
    3.2.1), LU-factorised; apply = solve L_j U_j x = P_j y per block."""

    def __init__(self, M, nmax, perm, offsets):
        self.nmax = nmax
        self.blocks = []
        for j in range(len(offsets) - 1):
            sph = perm[offsets[j]:offsets[j + 1]]
            ix = (sph[:, None] * nmax + np.arange(nmax)[None, :]).reshape(-1)
            self.blocks.append((ix, sla.lu_factor(M[np.ix_(ix, ix)])))

    def __call__(self, y):
        x = np.zeros_like(y)
        for ix, lu in self.blocks:
            x[ix] = sla.lu_solve(lu, y[ix])
        return x


def gmres(matvec, rhs, tol=1e-10, restart=100, maxiter=10000, precond=None, x0=None):
    """Restarted GMRES, right-preconditioned (M P^{-1} u = rhs, x = P^{-1} u),
    modified Gram-Schmidt Arnoldi, Givens rotations.  Converges on the true
    relative residual ||rhs - M x|| / ||rhs||.  Returns (x, iterations,
    history of true residuals at restarts)."""
    P = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(rhs) if x0 is None else np.array(x0, dtype=np.complex128)
    nb = np.linalg.norm(rhs)
    if nb == 0:
        return np.zeros_like(rhs), 0, [0.0]
    its = 0
    hist = []
    while True:
        r = rhs - matvec(x)
        res = np.linalg.norm(r) / nb
        hist.append(res)
        if res <= tol or its >= maxiter:
            return x, its, hist
        beta = np.linalg.norm(r)
        V = [r / beta]
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        kk = 0
        for kk in range(restart):
            w = matvec(P(V[kk]))
            for i in range(kk + 1):
                H[i, kk] = np.vdot(V[i], w)
                w = w - H[i, kk] * V[i]
            H[kk + 1, kk] = np.linalg.norm(w)
            # complex Givens rotation [[conj(c), conj(s)], [-s, c]] with
            # c = a/r, s = b/r, r = sqrt(|a|^2 + |b|^2), annihilating H[k+1, k]
            for i in range(kk):
                t = np.conj(cs[i]) * H[i, kk] + np.conj(sn[i]) * H[i + 1, kk]
                H[i + 1, kk] = -sn[i] * H[i, kk] + cs[i] * H[i + 1, kk]
                H[i, kk] = t
            a, b = H[kk, kk], H[kk + 1, kk]
            den = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
            cs[kk] = a / den if den != 0 else 1.0
            sn[kk] = b / den if den != 0 else 0.0
            H[kk, kk] = den
            H[kk + 1, kk] = 0.0
            g[kk + 1] = -sn[kk] * g[kk]
            g[kk] = np.conj(cs[kk]) * g[kk]
            its += 1
            if H[kk + 1, kk] == 0 and den == 0:
                break
            V.append(w / (np.linalg.norm(w) if np.linalg.norm(w) > 0 else 1.0))
            if abs(g[kk + 1]) / nb <= tol or its >= maxiter:
                break
        m = kk + 1
        y = np.linalg.solve(np.triu(H[:m, :m]), g[:m])
        u = sum(y[i] * V[i] for i in range(m))
        x = x + P(u)


def bicgstab(matvec, rhs, tol=1e-10, maxiter=10000, precond=None, x0=None, trace=None):
    """Right-preconditioned BiCGSTAB, the alternative iterative solver of
    Section 3.2 (the method as given in the iterative-templates reference the
    paper cites, Barrett et al. 1994).  Notation: rho, alpha, omega, beta;
    p_hat = P^{-1} p, s_hat = P^{-1} s; the shadow residual r_tilde is the
    residual at the start of a run.

    One iteration costs two products with the master matrix.  A run ends when
    the updated residual ||s|| or ||r|| drops to tol * ||rhs|| or on a
    breakdown (rho = 0, r_tilde^H v = 0, omega = 0); the true residual
    rhs - M x is then evaluated and, if it is still above the tolerance, a new
    run starts from the current x (a stalled run that makes no iteration ends
    the solve).  Returns (x, iterations, history of true residuals at run
    starts and at the end).  `trace`, if a list, receives per iteration a
    dict with the vectors s, t, r (updated), x after the iteration and the
    shadow residual r_tilde."""
    P = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(rhs) if x0 is None else np.array(x0, dtype=np.complex128)
    nb = np.linalg.norm(rhs)
    if nb == 0:
        return np.zeros_like(rhs), 0, [0.0]
    its = 0
    hist = []
    while True:
        r = rhs - matvec(x)
        res = np.linalg.norm(r) / nb
        hist.append(res)
        if res <= tol or its >= maxiter:
            return x, its, hist
        r_tilde = r.copy()
        rho_old = alpha = omega = 1.0
        p = np.zeros_like(r)
        v = np.zeros_like(r)
        run_its = 0
        while its < maxiter:
            rho = np.vdot(r_tilde, r)
            if rho == 0:
                break
            if run_its == 0:
                p = r.copy()
            else:
                beta = (rho / rho_old) * (alpha / omega)
                p = r + beta * (p - omega * v)
            p_hat = P(p)
            v = matvec(p_hat)
            rv = np.vdot(r_tilde, v)
            if rv == 0:
                break
            alpha = rho / rv
            s = r - alpha * v
            its += 1
            run_its += 1
            if np.linalg.norm(s) / nb <= tol:
                x = x + alpha * p_hat
                if trace is not None:
                    trace.append({"s": s, "t": None, "r": s, "x": x.copy(), "r_tilde": r_tilde})
                break
            s_hat = P(s)
            t = matvec(s_hat)
            tt = np.vdot(t, t).real
            omega = np.vdot(t, s) / tt if tt > 0 else 0.0
            x = x + alpha * p_hat + omega * s_hat
            r = s - omega * t
            rho_old = rho
            if trace is not None:
                trace.append({"s": s, "t": t, "r": r, "x": x.copy(), "r_tilde": r_tilde})
            if np.linalg.norm(r) / nb <= tol or omega == 0:
                break
        if run_its == 0:
            hist.append(np.linalg.norm(rhs - matvec(x)) / nb)
            return x, its, hist


def subsystem_initial_guess(pos, radii, n_sphere, n0, wavelength, L, a_in, idx, hankel=None):
    """Custom initial condition of Section 4.2: the solution of the master
    equation of a sub-ensemble (the spheres idx, under the same incident
    field) placed at those spheres, zero at all others.  a_in: [N][nmax]
    incident coefficients of the whole ensemble (a sphere's coefficients
    depend only on its own position, so the sub-ensemble's are the rows idx);
    hankel: None or a Hankel table built for the sub-ensemble.  Returns the
    initial guess [N][nmax]."""
    idx = np.asarray(idx, dtype=np.int64)
    pos = np.asarray(pos, dtype=float)
    M, W, t = master_matrix(pos[idx], np.asarray(radii)[idx], np.asarray(n_sphere)[idx], n0, wavelength, L, hankel)
    rhs = t * np.asarray(a_in)[idx].reshape(-1)
    b = solve_dense(M, rhs).reshape(len(idx), -1)
    x0 = np.zeros_like(np.asarray(a_in, dtype=np.complex128))
    x0[idx] = b
    return x0
