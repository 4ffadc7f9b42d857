"""Binary64 oracle of the iterative use of the product -- TEST INFRASTRUCTURE ONLY.

The paper's motivation (Sect. 2.1) is an iterative solver that stays in the permuted basis
from its first to its last step.  The solver here is the symmetric Lanczos recurrence
(Lanczos 1950; the three-term form of Paige 1972), run for m steps from a start vector v:

    v_0 = v / ||v||,  beta_0 = 0,  v_{-1} = 0
    for j = 0 .. m-1:
        w        = A v_j - beta_j v_{j-1}
        alpha_j  = w . v_j
        w        = w - alpha_j v_j
        beta_{j+1} = ||w||
        v_{j+1}  = w / beta_{j+1}

It returns alpha_0..alpha_{m-1} and beta_0..beta_m.  The coefficients do not depend on the
basis: running on P A P^T from P v gives the same numbers as A from v.  Products come from
the oracle's plain CSR product; dot products and norms are numpy's.

``axpby`` is the plain definition of y = a (A x) + b z.
"""
from __future__ import annotations

import numpy as np

import oracle


def axpby(A, x: np.ndarray, a: float, b: float, z: np.ndarray | None) -> np.ndarray:
    y = a * oracle.csr_spmv(A, x)
    if z is not None:
        y = y + b * np.asarray(z, np.float64)
    return y


def lanczos(A, v: np.ndarray, m: int) -> tuple[np.ndarray, np.ndarray]:
    v = np.asarray(v, np.float64)
    vj = v / np.linalg.norm(v)
    vprev = np.zeros_like(vj)
    alpha = np.zeros(m)
    beta = np.zeros(m + 1)
    for j in range(m):
        w = oracle.csr_spmv(A, vj) - beta[j] * vprev
        alpha[j] = w @ vj
        w = w - alpha[j] * vj
        beta[j + 1] = np.linalg.norm(w)
        vprev, vj = vj, w / beta[j + 1]
    return alpha, beta


def ritz_values(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Eigenvalues of the m x m tridiagonal matrix tridiag(beta_1.., alpha, beta_1..)."""
    m = len(alpha)
    T = np.diag(alpha) + np.diag(beta[1:m], 1) + np.diag(beta[1:m], -1)
    return np.linalg.eigvalsh(T)
