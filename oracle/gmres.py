"""Left-preconditioned restarted GMRES(m) with iterated classical
Gram-Schmidt (section 2.2.2, eq. LS1; Saad and Schultz 1986).

Parity: pinned.  Tests check the Arnoldi relation
M^{-1} K V_m = V_{m+1} Hbar_m, orthonormality of V, a non-increasing residual
estimate, finite termination in at most N steps without restart, and the
solution against a dense direct solve.

Readings (the paper names the method only):
* ICGS is taken as classical Gram-Schmidt applied twice per step (the second
  pass always taken), with the two coefficient vectors summed into H.
* x0 = 0.  Each cycle starts from the true residual r = R - K x; the solve is
  accepted when ||r|| / ||R|| <= rtol (unpreconditioned, checked at cycle
  starts).  The inner Arnoldi loop stops when the Givens residual estimate
  |g_{j+1}| drops to inner_factor * rtol * ||M^{-1} R||, at j = m, or on a
  happy breakdown (||w|| after orthogonalisation <= 1e-14 of its norm
  before).  The Hessenberg system is solved by back substitution.
"""
import numpy as np


def _rotation(a, b):
    if b == 0.0:
        return 1.0, 0.0, a
    r = np.hypot(a, b)
    return a / r, b / r, r


def gmres(Kmv, Minv, R, restart, rtol, max_cycles=200, inner_factor=0.1,
          record=False):
    R = np.asarray(R, dtype=np.float64)
    N = R.shape[0]
    nR = np.linalg.norm(R)
    x = np.zeros(N)
    info = {"iters": 0, "cycles": 0, "converged": False, "true_hist": [],
            "est_hist": []}
    if nR == 0.0:
        info["converged"] = True
        info["rel_resid"] = 0.0
        return x, info
    beta0 = np.linalg.norm(Minv(R))
    inner_tol = inner_factor * rtol * beta0
    m = restart
    for cycle in range(max_cycles):
        r = R - Kmv(x)
        rho = np.linalg.norm(r) / nR
        info["true_hist"].append(rho)
        if rho <= rtol:
            info["converged"] = True
            break
        info["cycles"] += 1
        z = Minv(r)
        beta = np.linalg.norm(z)
        V = np.zeros((m + 1, N))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = z / beta
        k = 0
        for j in range(m):
            w = Minv(Kmv(V[j]))
            w_norm0 = np.linalg.norm(w)
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            if record:
                info.setdefault("H_raw", []).append(H[:j + 2, j].copy())
            for i in range(j):
                a, bb = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * bb
                H[i + 1, j] = -sn[i] * a + cs[i] * bb
            cs[j], sn[j], H[j, j] = _rotation(H[j, j], H[j + 1, j])
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info["iters"] += 1
            info["est_hist"].append(abs(g[j + 1]))
            k = j + 1
            breakdown = hn <= 1e-14 * w_norm0
            if not breakdown:
                V[j + 1] = w / hn
            if abs(g[j + 1]) <= inner_tol or breakdown:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + V[:k].T @ y
        if record:
            info.setdefault("V", []).append(V[:k + 1].copy())
    else:
        r = R - Kmv(x)
        info["true_hist"].append(np.linalg.norm(r) / nR)
    info["rel_resid"] = info["true_hist"][-1]
    return x, info
