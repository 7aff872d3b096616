"""CPU FP64 oracle for the H-IDBF-LU hot path (test infrastructure only).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module.  It shares no code with the GPU
library; the only thing both sides consume is the seeded input generator
module.

Everything here is the plain dense definition of what the GPU path
approximates, in complex128 with NumPy/SciPy:

* the TM_z EFIE impedance matrix of the paper (Sec. 3.1, the entry formula
  with the closed-form self term), rescaled as in Sec. 3.1 / Sec. 4;
* y = A x, and x = A^{-1} b by LU with partial pivoting;
* the approximate-LU preconditioner built from the triangular parts of A
  (Sec. 3.1, the definitions of L~ and U~, and the split system solved with
  them), in two readings: the paper's point-wise triangular parts, and the
  block form whose leaf blocks are the exact n0 x n0 diagonal blocks;
* a restarted, right-preconditioned GMRES and TFQMR (the paper's Krylov
  method) used for iteration counts;
* a far-field objective and its gradient through the adjoint system.

The Hankel function is SciPy's ``hankel2`` (AMOS); the GPU library carries
its own independent implementation.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.special as sps

EULER_GAMMA_EXP = math.exp(0.57721566490153286060651209)  # gamma ~ 1.781 (Sec. 3.1)
E = math.e                                                 # e ~ 2.718 (Sec. 3.1)
ETA0 = 376.730313668


# ---------------------------------------------------------------------------
# geometry: pulse basis on line segments (Sec. 3.1: rho_i and w_i are the
# centre and length of the i-th segment)
# ---------------------------------------------------------------------------

def segments(xy: np.ndarray, node_off: np.ndarray):
    """Centres rho (N, 2) and lengths w (N,) of the chords between
    consecutive nodes of every curve, curves concatenated in order."""
    rho, w = [], []
    for c in range(len(node_off) - 1):
        p = np.asarray(xy[node_off[c]:node_off[c + 1]], dtype=np.float64)
        d = p[1:] - p[:-1]
        rho.append(0.5 * (p[1:] + p[:-1]))
        w.append(np.hypot(d[:, 0], d[:, 1]))
    return np.concatenate(rho, axis=0), np.concatenate(w)


# ---------------------------------------------------------------------------
# entries of the impedance matrix (Sec. 3.1, entry formula for A_ij)
# ---------------------------------------------------------------------------

def hankel2_0(x):
    """Zeroth-order Hankel function of the second kind, H0^(2)(x) = J0 - i Y0."""
    return sps.hankel2(0, x)


def self_term(w, kappa, eta0=ETA0):
    """Diagonal entry (Sec. 3.1): (kappa eta0 w / 4) [1 - i (2/pi) ln(gamma kappa w / (4 e))]."""
    w = np.asarray(w, dtype=np.float64)
    return (kappa * eta0 * w / 4.0) * (1.0 - 1j * (2.0 / math.pi)
                                       * np.log(EULER_GAMMA_EXP * kappa * w / (4.0 * E)))


def entries(rows, cols, rho, w, kappa, eta0=ETA0, z=None):
    """A[rows][:, cols] with A = Z + diag(z): off-diagonal entries
    (kappa eta0 w_j / 4) H0^(2)(kappa |rho_i - rho_j|) (the source-segment
    length w_j), diagonal entries from the closed form."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    dx = rho[rows, 0][:, None] - rho[cols, 0][None, :]
    dy = rho[rows, 1][:, None] - rho[cols, 1][None, :]
    r = np.hypot(dx, dy)
    same = rows[:, None] == cols[None, :]
    rr = np.where(same, 1.0, r)
    out = (kappa * eta0 * w[cols][None, :] / 4.0) * hankel2_0(kappa * rr)
    if same.any():
        ii, jj = np.nonzero(same)
        d = self_term(w[rows[ii]], kappa, eta0)
        if z is not None:
            d = d + z[rows[ii]]
        out[ii, jj] = d
    return out


def dense_A(rho, w, kappa, eta0=ETA0, z=None):
    n = rho.shape[0]
    idx = np.arange(n)
    return entries(idx, idx, rho, w, kappa, eta0, z)


def exact_rows_matvec(rows, x, rho, w, kappa, eta0=ETA0, z=None, chunk=64):
    """(A x)[rows] evaluated matrix-free, row block by row block; x is (N,) or
    (N, R).  Used where a dense A does not fit in memory."""
    rows = np.asarray(rows)
    n = rho.shape[0]
    cols = np.arange(n)
    x2 = x.reshape(n, -1)
    out = np.empty((len(rows), x2.shape[1]), dtype=np.complex128)
    for s in range(0, len(rows), chunk):
        r = rows[s:s + chunk]
        out[s:s + chunk] = entries(r, cols, rho, w, kappa, eta0, z) @ x2
    return out.reshape((len(rows),) + x.shape[1:])


# ---------------------------------------------------------------------------
# rescaling (Sec. 3.1: the system is rescaled so that the largest diagonal
# entry has unit magnitude, Sec. 4; the analysis of Sec. 3.3.1 assumes
# A(i,i) ~ 1).  Reading: a = 1 / A[i*, i*], i* = argmax |A_ii| (lowest index on
# ties), a complex scalar.
# ---------------------------------------------------------------------------

def scale_factor(diag_entries):
    d = np.asarray(diag_entries)
    i = int(np.argmax(np.abs(d)))
    return 1.0 / d[i]


# ---------------------------------------------------------------------------
# dense results
# ---------------------------------------------------------------------------

def matvec(A, x):
    return A @ x


def lu_solve(A, b):
    lu = sla.lu_factor(A)
    return sla.lu_solve(lu, b)


def relres(A, x, b):
    """||b - A x||_2 / ||b||_2 per right-hand side (columns, or a vector)."""
    r = b - A @ x
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)


# ---------------------------------------------------------------------------
# the approximate-LU preconditioner (Sec. 3.1, the definitions of L~ and U~
# and the split system built from them; Sec. 3.2.2 solves with them by block
# forward / back substitution over a dyadic partition with leaves <= n0)
# ---------------------------------------------------------------------------

def leaf_partition(n: int, n0: int):
    """Dyadic bisection of [0, n) until pieces have at most n0 indices; the
    first half of a piece of size m has ceil(m/2) indices."""
    out = []

    def rec(lo, hi):
        if hi - lo <= n0:
            out.append((lo, hi))
            return
        mid = lo + (hi - lo + 1) // 2
        rec(lo, mid)
        rec(mid, hi)

    rec(0, n)
    return out


def block_parts(A, n0):
    """D = blockdiag(A[leaf, leaf]); A_low / A_up = strictly block-lower /
    block-upper parts of A for the leaf partition."""
    n = A.shape[0]
    D = np.zeros_like(A)
    mask_low = np.zeros((n, n), dtype=bool)
    leaves = leaf_partition(n, n0)
    for (lo, hi) in leaves:
        D[lo:hi, lo:hi] = A[lo:hi, lo:hi]
        mask_low[hi:, lo:hi] = True
    A_low = np.where(mask_low, A, 0)
    A_up = np.where(mask_low.T, A, 0)
    return D, A_low, A_up


def precond_block_matrix(A, n0):
    """P_blk = (D + A_low) D^{-1} (D + A_up): the paper's L~ U~ with its unit
    scalar diagonal replaced by the exact leaf blocks (so L~ = I + A_low D^-1,
    U~ = D + A_up)."""
    D, A_low, A_up = block_parts(A, n0)
    return (D + A_low) @ np.linalg.solve(D, D + A_up)


def precond_block_apply(A, r, n0, adjoint=False):
    """P_blk^{-1} r by the two block substitutions: t = (D + A_low)^{-1} r,
    s = D t, x = (D + A_up)^{-1} s.  With adjoint=True, P_blk^{-H} r."""
    D, A_low, A_up = block_parts(A, n0)
    if not adjoint:
        t = np.linalg.solve(D + A_low, r)
        s = D @ t
        return np.linalg.solve(D + A_up, s)
    # P^H = (D + A_up)^H D^{-H} (D + A_low)^H
    t = np.linalg.solve((D + A_up).conj().T, r)
    s = D.conj().T @ t
    return np.linalg.solve((D + A_low).conj().T, s)


def precond_paper_matrices(A):
    """The paper's point-wise factors for the rescaled matrix a*A
    (Sec. 3.1, definitions of L~ and U~): L~ = I + tril(aA, -1), U~ = triu(aA).
    In unscaled terms P_pt = L~ U~ / a = (I + a A_sl)(diag A + A_su)."""
    a = scale_factor(np.diag(A))
    n = A.shape[0]
    Lt = np.eye(n, dtype=A.dtype) + np.tril(a * A, -1)
    Ut = np.triu(A)
    return Lt, Ut, a


def precond_paper_apply(A, r, adjoint=False):
    """P_pt^{-1} r = (diag A + A_su)^{-1} (I + a A_sl)^{-1} r (adjoint: the
    conjugate-transposed composition)."""
    Lt, Ut, _ = precond_paper_matrices(A)
    if not adjoint:
        y = sla.solve_triangular(Lt, r, lower=True, unit_diagonal=True)
        return sla.solve_triangular(Ut, y, lower=False)
    y = sla.solve_triangular(Ut.conj().T, r, lower=True)
    return sla.solve_triangular(Lt.conj().T, y, lower=False, unit_diagonal=True)


# ---------------------------------------------------------------------------
# restarted right-preconditioned GMRES (iteration-count reference only)
# ---------------------------------------------------------------------------

def gmres(apply_A, apply_Minv, b, tol=1e-6, restart=50, maxiter=1000):
    """Solve A x = b with x0 = 0 and right preconditioning A M^{-1} y = b,
    x = M^{-1} y; classical Gram-Schmidt applied twice, Givens rotations.
    Returns (x, iterations, relres_history)."""
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    hist = []
    it = 0
    r = b.copy()
    while it < maxiter:
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            break
        V = np.zeros((n, restart + 1), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(restart):
            w = apply_A(apply_Minv(V[:, j]))
            for _ in range(2):
                h = V[:, :j + 1].conj().T @ w
                w = w - V[:, :j + 1] @ h
                H[:j + 1, j] += h
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = np.conj(cs[i]) * hi + np.conj(sn[i]) * hi1
                H[i + 1, j] = -sn[i] * hi + cs[i] * hi1
            a_, b_ = H[j, j], H[j + 1, j]
            den = math.hypot(abs(a_), abs(b_))
            # G = [conj(c) conj(s); -s c] with c = a/den, s = b/den maps (a, b) to (den, 0)
            cs[j], sn[j] = (a_ / den, b_ / den) if den else (1.0, 0.0)
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if hist[-1] <= tol or it >= maxiter:
                break
        y = sla.solve_triangular(H[:j_done, :j_done], g[:j_done], lower=False)
        x = x + apply_Minv(V[:, :j_done] @ y)
        r = b - apply_A(x)
    return x, it, hist


def tfqmr(apply_A, apply_Minv, b, tol=1e-6, maxiter=1000):
    """Transpose-free QMR (Freund, SIAM J. Sci. Comput. 14, 1993), the Krylov
    method of the paper's experiments (Sec. 4), on the right-preconditioned
    system A M^{-1} u = b with x0 = 0, x = M^{-1} u, shadow vector r~ = b.
    Each iteration is two half steps with one product by A M^{-1} each; the
    iteration stops when the quasi-residual bound tau sqrt(half steps + 1)
    falls to tol ||b|| (and the true residual confirms it).
    Returns (x, iterations, bound_history)."""
    bnorm = np.linalg.norm(b)
    op = lambda v: apply_A(apply_Minv(v))
    u = np.zeros_like(b)           # solution of the preconditioned system
    w = b.copy()
    y1 = b.copy()
    rt = b.copy()
    Ay1 = op(y1)
    v = Ay1.copy()
    d = np.zeros_like(b)
    tau = bnorm
    theta = 0.0
    eta = 0.0
    rho = np.vdot(rt, w)
    hist = []
    half = 0

    def half_step(y, Ay):
        nonlocal w, d, theta, tau, eta, u, half
        w = w - alpha * Ay
        d = y + (theta ** 2 * eta / alpha) * d
        theta = np.linalg.norm(w) / tau
        c = 1.0 / math.sqrt(1.0 + theta ** 2)
        tau = tau * theta * c
        eta = c ** 2 * alpha
        u = u + eta * d
        half += 1
        hist.append(tau * math.sqrt(half + 1) / bnorm)
        if hist[-1] <= tol:
            x = apply_Minv(u)
            return np.linalg.norm(b - apply_A(x)) <= tol * bnorm
        return False

    for it in range(maxiter):
        sigma = np.vdot(rt, v)
        if sigma == 0 or rho == 0:
            break
        alpha = rho / sigma
        y2 = y1 - alpha * v
        if half_step(y1, Ay1):
            return apply_Minv(u), it + 1, hist
        Ay2 = op(y2)
        if half_step(y2, Ay2):
            return apply_Minv(u), it + 1, hist
        rho_new = np.vdot(rt, w)
        beta = rho_new / rho
        rho = rho_new
        y1 = w + beta * y2
        Ay1 = op(y1)
        v = Ay1 + beta * (Ay2 + beta * v)
    return apply_Minv(u), maxiter, hist


# ---------------------------------------------------------------------------
# differentiable workload: far-field objective and its gradient.  The paper
# defines no far field; reading: F(phi) = sum_j w_j x_j exp(+i kappa (rho_j .
# u(phi))) (constant prefactor dropped), J = sum_m |F(phi_m)|^2.
# ---------------------------------------------------------------------------

def farfield_matrix(rho, w, kappa, angles):
    ph = kappa * (np.outer(np.cos(angles), rho[:, 0]) + np.outer(np.sin(angles), rho[:, 1]))
    return w[None, :] * np.exp(1j * ph)            # C[m, j]


def objective(x, C):
    F = C @ x
    return float(np.sum(np.abs(F) ** 2))


def objective_grad_x(x, C):
    """dJ/dRe x + i dJ/dIm x = 2 C^H C x (PyTorch's convention for a real
    function of complex inputs)."""
    return 2.0 * (C.conj().T @ (C @ x))


def adjoint_gradients(A, b, C):
    """x = A^{-1} b, J(x); returns (J, grad_b, grad_z) with grad_b = A^{-H} g,
    grad_z = -grad_b * conj(x) (the derivative of A = Z + diag(z) w.r.t. z)."""
    x = lu_solve(A, b)
    g = objective_grad_x(x, C)
    lam = lu_solve(A.conj().T, g)
    return objective(x, C), lam, -lam * np.conj(x)
