"""Dense FP64 building blocks of the oracle (test infrastructure only).

* Householder reflectors in the LAPACK convention: H = I - tau v v^T with
  v[0] = 1, H x = beta e_1, beta = -sign(alpha) ||x|| with sign(0) = +1, and
  tau = 0 when x[1:] is zero; an alpha at rounding level (|alpha| <=
  64 u ||x||) counts as 0.  This is the block Householder QR used to
  eliminate clusters (Section 2.3) and to scale interfaces (Section 2.4).
* Column-pivoted Householder QR truncated by the paper's rank rule
  |R_ii| >= eps |R_11| (Section 4, the low-rank approximations of
  Section 2.5).  Pivot = largest remaining column 2-norm, first index on
  ties; norms are downdated after each step and recomputed from the matrix
  when cancellation makes the downdate unreliable, following Drmac and
  Bujanovic, "On the failure of rank-revealing QR factorization software"
  (LAPACK Working Note 176).

Every routine is unblocked: one reflector at a time, in column order.
"""
from __future__ import annotations

import math

import numpy as np

EPS = np.finfo(np.float64).eps


# |alpha| at or below this multiple of u ||x|| is rounding error: its sign
# carries no information and counts as +1
SIGN_FLOOR = 64.0


def house(x: np.ndarray, unit: float = EPS / 2):
    """Return (v, tau, beta) with (I - tau v v^T) x = beta e_1, v[0] = 1.

    LAPACK's convention beta = -sign(alpha) ||x|| with sign(0) = +1, where
    an alpha of at most SIGN_FLOOR * unit * ||x|| counts as 0: such an
    alpha is a structural zero carrying rounding error, and two correct
    evaluations may give it either sign."""
    alpha = float(x[0])
    xnorm = float(np.sqrt(np.dot(x[1:], x[1:]))) if x.shape[0] > 1 else 0.0
    v = np.zeros_like(x)
    v[0] = 1.0
    if xnorm == 0.0:
        return v, 0.0, alpha
    nrm = math.hypot(alpha, xnorm)
    sgn = alpha if abs(alpha) > SIGN_FLOOR * unit * nrm else 1.0
    beta = -math.copysign(nrm, sgn)
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def householder_qr(F: np.ndarray, ncols: int | None = None):
    """In-place Householder QR of the leading ``ncols`` columns of F.

    The reflectors are applied to all remaining columns of F.  On return the
    leading ``min(m, ncols)`` rows hold R (zeros written below its diagonal
    in the factored columns) and the trailing rows hold the transformed
    remainder.  Returns the list of (v, tau) pairs.
    """
    m, n = F.shape
    if ncols is None:
        ncols = n
    refl = []
    for k in range(min(m, ncols)):
        v, tau, beta = house(F[k:, k])
        if tau != 0.0 and k + 1 < n:
            w = v @ F[k:, k + 1:]
            F[k:, k + 1:] -= tau * np.outer(v, w)
        F[k, k] = beta
        F[k + 1:, k] = 0.0
        refl.append((v, tau))
    return refl


NOISE = 1000.0


def pivoted_qr(C: np.ndarray, eps: float, noise: float = NOISE):
    """Column-pivoted Householder QR of C (m x n), stopped by the rank rule.

    Returns (rank, rows, perm, V, tau) where ``rows`` (rank x n) are the first
    ``rank`` rows of Q^T C in the ORIGINAL column order, ``perm[i]`` is the
    original index of the i-th pivot, ``V`` (m x rank) holds the reflectors
    (unit diagonal, zeros above) and ``tau`` their scalars, so that
    Q = H_0 H_1 ... H_{rank-1}.

    Rank rule: rank = number of leading steps i with |R_ii| >= eps |R_00|
    and |R_ii| > noise * u * ||C||_F (u the unit roundoff).  The second
    condition stops at the numerical rank: past it the reflectors would be
    built from rounding error.  rank = 0 for an all-zero or empty matrix.
    """
    A = np.array(C, dtype=np.float64, copy=True)
    m, n = A.shape
    perm = np.arange(n)
    vn1 = np.sqrt(np.einsum("ij,ij->j", A, A)) if m > 0 else np.zeros(n)
    vn2 = vn1.copy()
    floor = noise * (EPS / 2) * float(np.sqrt(np.sum(vn1 * vn1)))
    tol3z = math.sqrt(EPS)
    V = np.zeros((m, min(m, n)))
    taus = []
    rank = 0
    r00 = 0.0
    for i in range(min(m, n)):
        pvt = i + int(np.argmax(vn1[i:]))
        if pvt != i:
            A[:, [i, pvt]] = A[:, [pvt, i]]
            perm[[i, pvt]] = perm[[pvt, i]]
            vn1[[i, pvt]] = vn1[[pvt, i]]
            vn2[[i, pvt]] = vn2[[pvt, i]]
        v, tau, beta = house(A[i:, i])
        if abs(beta) <= floor:
            break
        if i == 0:
            r00 = abs(beta)
        elif abs(beta) < eps * r00:
            break
        if tau != 0.0 and i + 1 < n:
            w = v @ A[i:, i + 1:]
            A[i:, i + 1:] -= tau * np.outer(v, w)
        A[i, i] = beta
        A[i + 1:, i] = 0.0
        V[i:, i] = v
        taus.append(tau)
        rank = i + 1
        # norm downdate of the remaining columns (LAPACK Working Note 176)
        for j in range(i + 1, n):
            if vn1[j] != 0.0:
                temp = 1.0 - (abs(A[i, j]) / vn1[j]) ** 2
                temp = max(temp, 0.0)
                temp2 = temp * (vn1[j] / vn2[j]) ** 2
                if temp2 <= tol3z:
                    vn1[j] = float(np.sqrt(np.dot(A[i + 1:, j], A[i + 1:, j]))) if i + 1 < m else 0.0
                    vn2[j] = vn1[j]
                else:
                    vn1[j] *= math.sqrt(temp)
    rows = np.zeros((rank, n))
    rows[:, perm] = np.triu(A[:rank, :])
    return rank, rows, perm[:rank].copy(), V[:, :rank].copy(), np.array(taus)


def apply_q(V: np.ndarray, tau: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Q x with Q = H_0 ... H_{r-1} (apply H_{r-1} first)."""
    y = np.array(x, dtype=np.float64, copy=True)
    for i in range(V.shape[1] - 1, -1, -1):
        y -= tau[i] * np.multiply.outer(V[:, i], V[:, i] @ y)
    return y


def apply_qt(V: np.ndarray, tau: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Q^T x with Q = H_0 ... H_{r-1} (apply H_0 first)."""
    y = np.array(x, dtype=np.float64, copy=True)
    for i in range(V.shape[1]):
        y -= tau[i] * np.multiply.outer(V[:, i], V[:, i] @ y)
    return y
