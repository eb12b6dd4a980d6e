"""Checks that tie the FP64 oracle to what the paper and the mathematics fix.

Each check takes the function under test as an argument, so the same check
runs on the real oracle (tests/test_oracle.py) and on deliberately broken
copies of it (tests/test_oracle_mutants.py), which shows that a plausible
mistake fails at least one check.
"""
from __future__ import annotations

import numpy as np

import synth


def small_problem(n=10, m=20, N=64, p=0.1, sigma=0.0, frac=0.2, seed=7):
    return synth.make_problem(n, m, N, p, sigma, frac, seed)


def monotone_violation(forward, lipschitz, pb, T=200):
    """Largest increase F(z^(t+1)) - F(z^(t)) along ISTA (alpha = 1/L).

    Section 3: one ISTA step minimises the majorizer Q_{x,L} of Eq. (7), so
    F never increases. Returns a number that must be <= 0 (up to rounding)."""
    L = lipschitz(pb.D)
    _, F = forward(pb.D, pb.X, pb.lam, np.full(T, 1.0 / L))
    inc = np.diff(F, axis=0)
    return float(np.max(inc / np.maximum(1.0, np.abs(F[:-1]))))


def rate_violation(forward, lipschitz, objective, zstar, pb, T=100):
    """max_t,i of (F(z^t) - F*) - L ||z*||^2 / (2t): the classical ISTA rate
    quoted in Section 3 after Prop. 3.2 (from z^(0) = 0). Must be <= 0."""
    L = lipschitz(pb.D)
    _, F = forward(pb.D, pb.X, pb.lam, np.full(T, 1.0 / L))
    Fs = objective(pb.D, pb.X, zstar, pb.lam)
    bound = L * np.sum(zstar ** 2, axis=1)[None, :] / (2.0 * np.arange(1, T + 1)[:, None])
    return float(np.max((F[1:] - Fs[None, :]) - bound))


def kkt_after_long_run(forward, kkt_residual, lipschitz, pb, T=4000):
    """A fixed point of the ISTA map satisfies Lemma 2.1; after many layers the
    KKT residual of the iterate must be tiny."""
    L = lipschitz(pb.D)
    Z, _ = forward(pb.D, pb.X, pb.lam, np.full(T, 1.0 / L))
    return float(np.max(kkt_residual(pb.D, pb.X, Z, pb.lam)))


def orthogonal_one_step_error(forward, kkt_residual, seed=3, n=12, N=16, lam=0.3):
    """Orthogonal D (D^T D = I, so L = 1): one step with alpha = 1 gives
    ST(D^T x, lam), which is already the Lasso solution (Section 3, after
    Prop. 3.2: ISTA converges in one iteration for orthogonal D). Returns the
    KKT residual of z^(1) plus its distance to ST(D^T x, lam) computed here."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    X = rng.standard_normal((N, n))
    Z1, _ = forward(Q, X, lam, np.array([1.0]))
    C = X @ Q
    direct = np.sign(C) * np.maximum(np.abs(C) - lam, 0.0)
    return float(np.max(kkt_residual(Q, X, Z1, lam)) + np.max(np.abs(Z1 - direct)))


def lemma42_case(seed=11, n=24, m=48, j=5, lam=0.4, shrink=0.5):
    """Build x = D_j + eps with eps orthogonal to D_j and ||eps|| < lam(1-c),
    c = max_{l != j} |D_l^T D_j|. Lemma 4.2: z* = (1 - lam) e_j, and then
    F* = 1/2 (lam^2 + ||eps||^2) + lam (1 - lam) (the residual is lam D_j + eps)."""
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((n, m))
    D /= np.linalg.norm(D, axis=0, keepdims=True)
    dj = D[:, j]
    c = np.max(np.abs(np.delete(D.T @ dj, j)))
    assert c < 1.0
    e = rng.standard_normal(n)
    e -= (e @ dj) * dj
    e *= shrink * lam * (1.0 - c) / np.linalg.norm(e)
    x = dj + e
    zstar = np.zeros(m)
    zstar[j] = 1.0 - lam
    Fstar = 0.5 * (lam ** 2 + e @ e) + lam * (1.0 - lam)
    return D, x[None, :], lam, zstar[None, :], Fstar


def fd_gradient(forward, D, X, lam, alpha, dZ, dF, h=1e-6):
    """Central finite differences of J = sum dF_i F_i(z^T) + <dZ, z^T> in alpha."""
    def J(a):
        Z, F = forward(D, X, lam, a)
        val = 0.0
        if dF is not None:
            val += float(np.sum(dF * F[-1]))
        if dZ is not None:
            val += float(np.sum(dZ * Z))
        return val
    g = np.zeros_like(alpha)
    for t in range(len(alpha)):
        ap, am = alpha.copy(), alpha.copy()
        ap[t] += h
        am[t] -= h
        g[t] = (J(ap) - J(am)) / (2.0 * h)
    return g


def one_layer_gradient(D, X, lam, a, dF):
    """Closed form for T = 1: z^(1) = ST(a c, lam a) = a ST(c, lam) (a > 0) with
    c = D^T x, so F(z^(1)) = 1/2 ||x - a D s||^2 + lam a ||s||_1, s = ST(c, lam),
    and dF/da = -(x - a D s)^T D s + lam ||s||_1."""
    C = X @ D
    S = np.sign(C) * np.maximum(np.abs(C) - lam, 0.0)
    DS = S @ D.T
    R = X - a * DS
    per = -np.sum(R * DS, axis=1) + lam * np.sum(np.abs(S), axis=1)
    return float(np.sum(dF * per))
