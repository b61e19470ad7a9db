"""Pins of the oracle's minimal-residual initial guess (oracle/mr.py,
section 2.2.1, eq. MinRes2) against what the mathematics fixes: the linear
case is a least-squares problem with a closed-form solution, an exact
solution among the previous ones is recovered, the finite-difference
gradient agrees with the closed-form gradient of the cubic residual, and
the nonlinear minimiser agrees with MINPACK's Levenberg-Marquardt."""
import numpy as np
import pytest
import scipy.optimize as so

import oracle
from oracle.mr import mr_guess, residual_vector, fd_jacobian, combine

from helpers import host_case, dense_uncondensed


def _case(dims=(2, 1, 1), p=1, s=3, seed=5):
    m, spec, blocks, G = host_case(dims, p)
    tm = oracle.TraceMesh(m.elem_faces(), m.n_face, spec.b)
    M, rhs = dense_uncondensed(tm, blocks, G)
    x = np.linalg.solve(M, rhs)
    E, n = tm.n_elem, spec.n
    rng = np.random.default_rng(seed)
    xs = [(1.0 + 0.1 * (j + 1)) * x + 0.05 * rng.standard_normal(x.size) for j in range(s)]
    Zs = [v[:E * n].reshape(E, n) for v in xs]
    Us = [v[E * n:] for v in xs]
    return tm, blocks, G, M, rhs, x, Zs, Us


def test_linear_case_is_least_squares():
    tm, blocks, G, M, rhs, x, Zs, Us = _case()
    Y = np.stack([M @ np.concatenate([z.ravel(), u]) for z, u in zip(Zs, Us)], axis=1)
    beta_ls, *_ = np.linalg.lstsq(Y, rhs, rcond=None)
    obj_ls = float(np.sum((rhs - Y @ beta_ls) ** 2))
    alpha, info = mr_guess(tm, blocks, G, 0.0, Zs, Us)
    assert np.max(np.abs(alpha - beta_ls)) <= 1e-7 * np.max(np.abs(beta_ls))
    assert abs(info["obj"] - obj_ls) <= 1e-9 * obj_ls
    assert info["obj"] < 0.2 * info["obj0"]


def test_exact_solution_among_previous_is_recovered():
    tm, blocks, G, M, rhs, x, Zs, Us = _case()
    E, n = len(Zs[0]), Zs[0].shape[1]
    Zs[1] = x[:E * n].reshape(E, n)
    Us[1] = x[E * n:]
    alpha, info = mr_guess(tm, blocks, G, 0.0, Zs, Us)
    assert np.max(np.abs(alpha - np.array([0.0, 1.0, 0.0]))) <= 1e-8
    assert info["obj"] <= 1e-20 * info["obj0"]


def test_fd_gradient_matches_closed_form():
    tm, blocks, G, M, rhs, x, Zs, Us = _case()
    eps = 0.05
    beta = np.array([0.7, 0.2, 0.15])
    res = lambda b: residual_vector(tm, blocks, G, eps, Zs, Us, b)
    r0 = res(beta)
    J = fd_jacobian(res, beta, r0, 1e-7)
    z, u = combine(Zs, Us, beta)
    xb = np.concatenate([z.ravel(), u])
    # R(x) = rhs - M x - eps x^3 componentwise, so dR/dbeta_i = -(M + 3 eps diag(x^2)) x_i
    for i in range(3):
        xi = np.concatenate([Zs[i].ravel(), Us[i]])
        exact = -(M @ xi) - 3.0 * eps * xb ** 2 * xi
        assert np.linalg.norm(J[:, i] - exact) <= 1e-6 * np.linalg.norm(exact)
    # and the residual itself is that formula
    assert np.linalg.norm(r0 - (rhs - M @ xb - eps * xb ** 3)) <= 1e-13 * np.linalg.norm(rhs)


@pytest.mark.parametrize("eps", [0.05, 0.5])
def test_nonlinear_minimiser_matches_minpack(eps):
    tm, blocks, G, M, rhs, x, Zs, Us = _case(s=4, seed=9)
    alpha, info = mr_guess(tm, blocks, G, eps, Zs, Us)
    # MINPACK's LM on R(x(beta)) = rhs - M x - eps x^3, from the same start
    X = np.stack([np.concatenate([z.ravel(), u]) for z, u in zip(Zs, Us)], axis=1)
    f = lambda b: rhs - M @ (X @ b) - eps * (X @ b) ** 3
    ref = so.least_squares(f, np.eye(4)[0], method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15)
    obj_ref = float(ref.fun @ ref.fun)
    assert abs(info["obj"] - obj_ref) <= 1e-8 * obj_ref
    assert np.max(np.abs(alpha - ref.x)) <= 1e-5 * np.max(np.abs(ref.x))
    h = info["history"]
    assert all(b < a for a, b in zip([info["obj0"]] + h[:-1], h))
    assert info["obj"] < 0.5 * info["obj0"]
