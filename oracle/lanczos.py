"""Lowest eigenpair of a Hermitian operator given only as a matvec (Sec. 4.2).

The paper's minimiser takes the current tensor as the initial guess and a
contractor that applies H_eff; it hands both to an external iterative sparse
eigensolver.  Here that solver is plain Lanczos in FP64:

  v_0 = theta / |theta|
  for j = 0 .. kmax-1:
      w = H v_j ;  alpha_j = Re <v_j, w>
      w -= alpha_j v_j + beta_{j-1} v_{j-1}
      two passes of full re-orthogonalisation  w -= V (V^H w)
      beta_j = |w| ; stop at j = kmax-1 or when beta_j <= tol * max(1, |alpha_0|)
      v_{j+1} = w / beta_j
  lowest eigenpair (t, y) of the tridiagonal T(alpha, beta)
  psi = V y / |V y| ;  E = Re <psi, H psi> ;  r = |H psi - E psi|

The final E is the Rayleigh quotient with the (FP64) matvec; r is the
residual norm.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal


def lanczos_ground(matvec, x0, kmax=20, tol=1e-12, refine=None):
    """Returns dict(psi, E, E_ritz, residual, steps, alpha, beta).

    matvec: callable on flat complex128 vectors (the operator used inside the
    iteration); refine: the FP64 matvec used for the final Rayleigh quotient
    (defaults to matvec).
    """
    refine = matvec if refine is None else refine
    nrm = np.linalg.norm(x0)
    V = [x0 / nrm]
    alpha, beta = [], []
    for j in range(kmax):
        w = matvec(V[j])
        a = float(np.real(np.vdot(V[j], w)))
        w = w - a * V[j]
        if j > 0:
            w = w - beta[j - 1] * V[j - 1]
        Vm = np.array(V)
        for _ in range(2):
            c = Vm.conj() @ w
            w = w - Vm.T @ c
        b = float(np.linalg.norm(w))
        alpha.append(a)
        if j == kmax - 1 or b <= tol * max(1.0, abs(alpha[0])):
            break
        beta.append(b)
        V.append(w / b)
    k = len(alpha)
    if k == 1:
        evals, evecs = np.array([alpha[0]]), np.ones((1, 1))
    else:
        evals, evecs = eigh_tridiagonal(np.array(alpha), np.array(beta[:k - 1]))
    y = evecs[:, 0]
    psi = np.zeros_like(V[0])
    for i in range(k):
        psi = psi + y[i] * V[i]
    psi = psi / np.linalg.norm(psi)
    hpsi = refine(psi)
    E = float(np.real(np.vdot(psi, hpsi)))
    r = float(np.linalg.norm(hpsi - E * psi))
    return {"psi": psi, "E": E, "E_ritz": float(evals[0]), "residual": r,
            "steps": k, "alpha": alpha, "beta": beta[:k - 1]}
