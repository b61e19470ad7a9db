"""Minimal-residual initial guess for Newton's method (section 2.2.1,
eq. MinRes2).

Parity: pinned (tests/test_oracle_mr.py): with eps = 0 the objective is a
linear least-squares problem in beta and the result equals numpy's lstsq
solution; a combination that reproduces an exact solution is found with
a zero objective; the finite-difference gradient matches the closed-form
gradient of the cubic residual; every accepted step lowers the objective.

The initial guess for time step n is a combination sum_j alpha_j x_{n-j} of
s previous solutions x = (z, uhat), with alpha minimising the squared norm
of the nonlinear residual (both blocks, eq. MinRes2), found by
Levenberg-Marquardt with finite-difference gradients.

The paper's residual is that of the IEDG Navier-Stokes discretisation,
which a synthetic workload does not have.  This module uses the residual of
the uncondensed Newton system plus a cubic term (a reading; eps = 0 gives
the linear residual):

  R_NS,e = F_e - A_e z_e - B_e uhat_e - eps z_e^3,
  R_FL   = G - sum_e P_e^T (C_e z_e + D_e uhat_e) - eps uhat^3   (componentwise cubes).

Levenberg-Marquardt (Marquardt's damped Gauss-Newton step with the diagonal
of J^T J as scaling; the paper fixes none of these details, so they are
readings too):

* start at beta = e_1 (the most recent solution alone), lambda = lambda0;
* J[:, i] = (R(x(beta + h_i e_i)) - R(x(beta))) / h_i, h_i = fd * max(1, |beta_i|);
* step: (J^T J + lambda diag(J^T J)) d = -J^T r;
* accept when the objective decreases (lambda /= 10, floor 1e-12), else
  lambda *= 10 and retry with the same J (at most 10 tries);
* stop after max_iters accepted steps, when no try is accepted, when
  max|d| <= tol (1 + max|beta|), when an accepted step lowers the
  objective by no more than ftol of its value, or when it is zero.
"""
import numpy as np


def combine(Zs, Us, beta):
    """x(beta) = sum_j beta_j (Z_j, U_j); Zs [s][E][n], Us [s][N_t]."""
    beta = np.asarray(beta, dtype=np.float64)
    z = np.tensordot(beta, np.asarray(Zs), axes=1)
    u = np.tensordot(beta, np.asarray(Us), axes=1)
    return z, u


def nonlinear_residual(tmesh, blocks, G, eps, z, uhat):
    """(R_NS [E][n], R_FL [N_t]) at (z, uhat), as defined above."""
    rG = np.array(G, dtype=np.float64, copy=True) - eps * uhat ** 3
    rF = np.empty((tmesh.n_elem, blocks[0]["A"].shape[0]))
    for e, blk in enumerate(blocks):
        dofs = tmesh.element_dofs(e)
        ue = uhat[dofs]
        rF[e] = blk["F"] - blk["A"] @ z[e] - blk["B"] @ ue - eps * z[e] ** 3
        np.subtract.at(rG, dofs, blk["C"] @ z[e] + blk["D"] @ ue)
    return rF, rG


def residual_vector(tmesh, blocks, G, eps, Zs, Us, beta):
    """R(x(beta)) as one vector (element rows first, then the trace)."""
    z, u = combine(Zs, Us, beta)
    rF, rG = nonlinear_residual(tmesh, blocks, G, eps, z, u)
    return np.concatenate([rF.ravel(), rG])


def fd_jacobian(res, beta, r0, fd):
    """Columns (R(beta + h_i e_i) - R(beta)) / h_i, h_i = fd max(1, |beta_i|)."""
    s = len(beta)
    J = np.empty((r0.size, s))
    for i in range(s):
        h = fd * max(1.0, abs(beta[i]))
        bi = np.array(beta, dtype=np.float64)
        bi[i] += h
        J[:, i] = (res(bi) - r0) / h
    return J


def mr_guess(tmesh, blocks, G, eps, Zs, Us, max_iters=20, lambda0=1e-3, fd=1e-7, tol=1e-10, ftol=1e-10):
    """Levenberg-Marquardt for eq. MinRes2.  Returns (alpha, info) with info
    keys obj0 (objective at e_1), obj, iters (accepted steps), evals
    (residual evaluations) and history (objective after each accepted step)."""
    s = len(Zs)
    evals = [0]

    def res(b):
        evals[0] += 1
        return residual_vector(tmesh, blocks, G, eps, Zs, Us, b)

    beta = np.zeros(s)
    beta[0] = 1.0
    r = res(beta)
    obj = float(r @ r)
    obj0 = obj
    lam = lambda0
    iters = 0
    history = []
    while iters < max_iters and obj > 0.0:
        J = fd_jacobian(res, beta, r, fd)
        H = J.T @ J
        g = J.T @ r
        accepted = False
        for _ in range(10):
            d = np.linalg.solve(H + lam * np.diag(np.diag(H)), -g)
            bt = beta + d
            rt = res(bt)
            ot = float(rt @ rt)
            if ot < obj:
                decrease = obj - ot
                beta, r, obj = bt, rt, ot
                lam = max(lam / 10.0, 1e-12)
                accepted = True
                break
            lam *= 10.0
        if not accepted:
            break
        iters += 1
        history.append(obj)
        if np.max(np.abs(d)) <= tol * (1.0 + np.max(np.abs(beta))) or decrease <= ftol * (obj + decrease):
            break
    return beta, {"obj0": obj0, "obj": obj, "iters": iters, "evals": evals[0], "history": history}
