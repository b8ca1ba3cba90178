"""Iterative solution of second-kind boundary integral equations with GIGAQBX applies.

The paper uses the fast layer potential inside an integral-equation solver: it checks Green's
formula on a discretized surface and solves Laplace boundary value problems (Section 6 and
its introduction).  This module supplies the solver around the evaluation:

* `gmres`: restarted GMRES (Arnoldi with two passes of classical Gram-Schmidt, Givens
  rotations on the small Hessenberg matrix), for any linear map on device vectors.
* `gmres_ir`: iterative refinement in two precisions.  The correction equation is solved
  by GMRES with a cheaper, less accurate apply (the split-precision translations), and the
  residual is recomputed with the accurate one (FP64), so the final residual reaches the
  accurate operator's level while most applies use the cheap one.

Both work on torch vectors (any device); every operator apply is a call into the HIP
library through `Plan.apply`.  The vector arithmetic here (a few dot products and updates
per iteration on N-vectors) is outside the evaluation path and costs a small fraction of
one apply.
"""

from __future__ import annotations

import math

import numpy as np


def plan_operator(plan, stream=None):
    """A vector -> vector map x -> plan.apply(x) for a plan with one density whose targets
    correspond one-to-one to its density values (a square operator)."""
    import torch

    if plan.n_densities != 1 or plan.n_tgt != plan.n_density_cols:
        raise ValueError("plan_operator needs one density and as many targets as density "
                         "values")

    def apply(x):
        out = torch.empty((1, plan.n_tgt), dtype=torch.float64, device=x.device)
        plan.apply(x.reshape(1, -1).contiguous(), out, stream=stream)
        return out.reshape(-1)

    return apply


def gmres(apply, b, *, tol=1e-8, maxiter=200, restart=60, x0=None):
    """Solve A x = b by restarted GMRES.

    Stops when the Arnoldi residual estimate |b - A x| <= tol |b| or after `maxiter` applies
    of A (the restart's residual recomputation counts as one).  Returns (x, applies,
    history), where history holds the relative residual estimate after each iteration.
    """
    import torch

    bnorm = float(torch.linalg.vector_norm(b))
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    history = []
    if bnorm == 0.0:
        return x, 0, [0.0]
    applies = 0
    if x0 is None:
        r = b.clone()
    else:
        r = b - apply(x)
        applies += 1
    beta = float(torch.linalg.vector_norm(r))
    history.append(beta / bnorm)
    while beta > tol * bnorm and applies < maxiter:
        m = min(restart, maxiter - applies)
        V = torch.empty((m + 1, b.numel()), dtype=b.dtype, device=b.device)
        V[0] = r / beta
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k_used = 0
        for k in range(m):
            w = apply(V[k])
            applies += 1
            Vk = V[: k + 1]
            h = Vk @ w
            w = w - Vk.T @ h
            h2 = Vk @ w  # second Gram-Schmidt pass restores orthogonality in floating point
            w = w - Vk.T @ h2
            hcol = (h + h2).cpu().numpy()
            hnext = float(torch.linalg.vector_norm(w))
            H[: k + 1, k] = hcol
            H[k + 1, k] = hnext
            for i in range(k):
                a, c = H[i, k], H[i + 1, k]
                H[i, k] = cs[i] * a + sn[i] * c
                H[i + 1, k] = -sn[i] * a + cs[i] * c
            d = math.hypot(H[k, k], H[k + 1, k])
            cs[k], sn[k] = (1.0, 0.0) if d == 0.0 else (H[k, k] / d, H[k + 1, k] / d)
            H[k, k] = d
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            k_used = k + 1
            history.append(abs(g[k + 1]) / bnorm)
            if abs(g[k + 1]) <= tol * bnorm or hnext == 0.0:
                break
            V[k + 1] = w / hnext
        y = _upper_solve(H[:k_used, :k_used], g[:k_used])
        x = x + V[:k_used].T @ torch.as_tensor(y, dtype=b.dtype, device=b.device)
        if abs(g[k_used]) <= tol * bnorm or applies >= maxiter:
            break
        r = b - apply(x)
        applies += 1
        beta = float(torch.linalg.vector_norm(r))
        history.append(beta / bnorm)
    return x, applies, history


def _upper_solve(R, g):
    y = np.zeros_like(g)
    for i in range(len(g) - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:] @ y[i + 1:]) / R[i, i]
    return y


def gmres_ir(apply_lo, apply_hi, b, *, tol=1e-10, inner_tol=1e-6, max_applies=200,
             restart=60):
    """Solve A x = b to |b - A_hi x| <= tol |b| by iterative refinement.

    Each refinement step solves A_lo d = r (r the current accurate residual) by GMRES to the
    relative tolerance `inner_tol`, updates x += d and recomputes r = b - A_hi x.  The
    budget `max_applies` counts applies of both operators.  Returns (x, info) where info
    has the outer relative residuals, the inner iteration counts and the apply counts.
    """
    import torch

    bnorm = float(torch.linalg.vector_norm(b))
    x = torch.zeros_like(b)
    r = b.clone()
    rel = 1.0 if bnorm > 0 else 0.0
    info = {"outer_residuals": [rel], "inner_iterations": [], "applies_lo": 0, "applies_hi": 0,
            "converged": rel <= tol}
    while rel > tol:
        used = info["applies_lo"] + info["applies_hi"]
        if used + 2 > max_applies:
            break
        d, k, _ = gmres(apply_lo, r, tol=inner_tol, maxiter=max_applies - used - 1,
                        restart=restart)
        info["applies_lo"] += k
        info["inner_iterations"].append(k)
        x = x + d
        r = b - apply_hi(x)
        info["applies_hi"] += 1
        rel = float(torch.linalg.vector_norm(r)) / bnorm
        info["outer_residuals"].append(rel)
    info["converged"] = rel <= tol
    return x, info
