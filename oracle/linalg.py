"""Oracle for the linear-algebra end of the path: assembly, SVD, truncated SVD / Tikhonov
reconstruction and residual (FP64, numpy / scipy LAPACK).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Definitions followed (paper, Sections 3, 3.1, 4.3 and Algorithm "Main" of Section 5.1):
  H        = counts / N                                    (eq. WoE_matrix_MC, Voronoi counting form)
  nu_i     = 1 / sqrt(M_D)                                 (Section 5.2, equal weights, sum nu^2 = 1)
  B        = diag(nu) H[:, Gamma_1] diag(sigma_1)^{-1/2}   (the matrix inside A^{nu,dagger,r})
  b        = u^D - H[:, Gamma_0] u^0                        (remark on non-zero Gamma_0 data)
  B        = U Sigma V^T (thin), eigenvalues of Lambda^nu = B B^T are s^2   (eq. SVD)
  u_1      = diag(sigma_1)^{-1/2} V diag(phi(s)) U^T diag(nu) b
             TSVD: phi_i = 1/s_i for i <= r, else 0        (eq. u1r / A^{nu,dagger,r})
             Tikhonov: phi_i = s_i / (s_i^2 + alpha^2)
  u_hat^D  = H[:, Gamma_1] u_1 + H[:, Gamma_0] u^0          (residual check, Section 5.2 item (iv))
Truncation by the discrepancy principle: smallest r with |B w_r - nu b| <= tau * delta; Tikhonov
alpha solves |B w_alpha - nu b| = tau * delta.
Products (Section 5.2, items (i)-(iv)):
  rho_i(l) = H_il / sigma_l                                  (eq. rho omega1 MC, cell indicators as weights)
  Lambda^nu = diag(nu) H_1 diag(sigma_1)^{-1} H_1^T diag(nu)  (eq. Lambda_tilde_nu), eigenpairs by eigh
  u_j      = lambda_j^{-1/2} sum_i nu_i [u_j]_i rho_i         (eq. eigenfunctions_MC) on the Gamma_1 cells
  sweep    : u_1^(r), u_hat^{D,r} and |nu b - B w_r| for r = 1..r_max (items (iii), (iv))
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.optimize as sopt

TSVD_RANK, TSVD_DISCREPANCY, TIKHONOV = 0, 1, 2


def assemble(counts, n_walks, gamma1_mask, sigma, uD=None, u0=None, nu=None):
    counts = np.asarray(counts)
    H = counts.astype(np.float64) / float(n_walks)
    g1 = np.asarray(gamma1_mask).astype(bool)
    M_D = H.shape[0]
    nu = np.full(M_D, 1.0 / np.sqrt(M_D)) if nu is None else np.asarray(nu, float)
    B = nu[:, None] * H[:, g1] / np.sqrt(np.asarray(sigma, float)[g1])[None, :]
    out = dict(H=H, B=B, nu=nu, g1=g1)
    if uD is not None:
        b = np.asarray(uD, float).copy()
        if u0 is not None and (~g1).any():
            b = b - H[:, ~g1] @ np.asarray(u0, float)
        out["b"] = b
        out["q"] = nu * b
    return out


def svd(B):
    """Thin SVD by LAPACK dgesvd; singular values descending."""
    U, s, Vt = sla.svd(B, full_matrices=False, lapack_driver="gesvd")
    return U, s, Vt


def residual_norms_tsvd(U, s, q):
    """|q - B w_r| for r = 0..k, computed directly from the truncated projections."""
    c = U.T @ q
    k = len(s)
    out = np.empty(k + 1)
    for r in range(k + 1):
        out[r] = np.linalg.norm(q - U[:, :r] @ c[:r])
    return out


def tikhonov_residual(U, s, q, alpha):
    c = U.T @ q
    phi_s = s * s / (s * s + alpha * alpha)
    return np.linalg.norm(q - U @ (phi_s * c))


def reconstruct(U, s, Vt, sigma1, q, kind=TSVD_RANK, rank=1, alpha=0.0, delta=0.0, tau=1.1,
                rank_tol=None):
    """u_1 on Gamma_1 and the regularisation actually used (rank, alpha)."""
    s = np.asarray(s, float)
    k = len(s)
    if rank_tol is None:
        rank_tol = max(U.shape[0], Vt.shape[1]) * np.finfo(float).eps * (s[0] if k else 0.0)
    k_pos = int(np.sum(s > rank_tol))
    c = U.T @ q
    phi = np.zeros(k)
    r_used, a_used = 0, 0.0
    if kind == TSVD_RANK:
        r_used = max(0, min(int(rank), k_pos))
        phi[:r_used] = 1.0 / s[:r_used]
    elif kind == TSVD_DISCREPANCY:
        res = residual_norms_tsvd(U, s, q)
        r_used = k_pos
        for r in range(1, k_pos + 1):
            if res[r] <= tau * delta:
                r_used = r
                break
        phi[:r_used] = 1.0 / s[:r_used]
    elif kind == TIKHONOV:
        if alpha > 0:
            a_used = float(alpha)
        else:
            target = tau * delta
            lo, hi = np.log(s[0] * 1e-16), np.log(s[0] * 1e4)
            f = lambda la: tikhonov_residual(U, s, q, np.exp(la)) - target
            if f(lo) >= 0:
                a_used = float(np.exp(lo))
            elif f(hi) <= 0:
                a_used = float(np.exp(hi))
            else:
                a_used = float(np.exp(sopt.brentq(f, lo, hi, xtol=1e-14, rtol=1e-15, maxiter=500)))
        phi = s / (s * s + a_used * a_used)
    else:
        raise ValueError(kind)
    w = Vt.T @ (phi * c)
    u1 = w / np.sqrt(np.asarray(sigma1, float))
    return u1, r_used, a_used


def predicted_data(H, g1, u1, u0=None):
    g1 = np.asarray(g1).astype(bool)
    out = H[:, g1] @ u1
    if u0 is not None and (~g1).any():
        out = out + H[:, ~g1] @ u0
    return out


def density(counts, n_walks, sigma):
    """rho[i, l] = (counts[i, l] / N) / sigma_l on every boundary cell (eq. rho omega1 MC with the
    cell indicators as the weight functions)."""
    H = np.asarray(counts).astype(np.float64) / float(n_walks)
    return H / np.asarray(sigma, float)[None, :]


def mean_density(counts, n_walks, sigma):
    """The density averaged over the points x^D_i."""
    return density(counts, n_walks, sigma).mean(axis=0)


def eigenfunctions(H, g1, sigma, nu=None, n_fun=None):
    """Eigenvalues of Lambda^nu (descending, eq. Lambda_tilde_nu) and the eigenfunction estimators of
    eq. eigenfunctions_MC on the Gamma_1 cells (n1 x n_fun), formed as written there: the eigenvectors
    of Lambda^nu from LAPACK dsyevd, then lambda^{-1/2} sum_i nu_i [u_j]_i rho_i."""
    g1 = np.asarray(g1).astype(bool)
    H1 = np.asarray(H, float)[:, g1]
    M_D = H1.shape[0]
    nu = np.full(M_D, 1.0 / np.sqrt(M_D)) if nu is None else np.asarray(nu, float)
    sig1 = np.asarray(sigma, float)[g1]
    Lam = (nu[:, None] * H1 / sig1[None, :]) @ (H1.T * nu[None, :])
    lam, E = sla.eigh(Lam, driver="evd")
    order = np.argsort(lam)[::-1]
    lam, E = lam[order], E[:, order]
    if n_fun is None:  # the eigenbasis of the orthogonal complement of the kernel
        n_fun = int(np.sum(lam > max(H1.shape) * np.finfo(float).eps * lam[0]))
    rho = H1 / sig1[None, :]                               # rho_i on the Gamma_1 cells
    ef = rho.T @ (nu[:, None] * E[:, :n_fun]) / np.sqrt(lam[:n_fun])[None, :]
    return lam[:n_fun], ef


def tsvd_sweep(U, s, Vt, sigma1, q, B, r_max, H=None, g1=None, u0=None, rank_tol=None):
    """Items (iii) and (iv) of Section 5.2 for every truncation r = 1..r_max: columns r - 1 of
    u1_all (the r-TSVD solution of reconstruct) and of pred_all (H_1 u1 + H_0 u0), and the residual
    norms |q - B w_r| for r = 0..r_max, w_r = diag(sigma_1)^{1/2} u1^(r) evaluated with B itself."""
    n1 = Vt.shape[1]
    u1_all = np.zeros((n1, r_max))
    pred_all = None if H is None else np.zeros((H.shape[0], r_max))
    resid = np.empty(r_max + 1)
    resid[0] = np.linalg.norm(q)
    sq = np.sqrt(np.asarray(sigma1, float))
    for r in range(1, r_max + 1):
        u1, _, _ = reconstruct(U, s, Vt, sigma1, q, kind=TSVD_RANK, rank=r, rank_tol=rank_tol)
        u1_all[:, r - 1] = u1
        resid[r] = np.linalg.norm(q - B @ (sq * u1))
        if H is not None:
            pred_all[:, r - 1] = predicted_data(H, g1, u1, u0)
    return u1_all, pred_all, resid

