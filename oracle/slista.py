"""FP64 oracle for the unfolded ISTA / Step-LISTA hot path.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Every function works in float64 with plain numpy / scipy primitives, follows
the paper's formulas in the paper's order, and does no blocking or fusion.
Layout is sample-major: X is [N, n], Z is [N, m] (row i = sample i), D is
[n, m]. The paper's column vectors are the rows here, so D z_i is row i of
Z @ D.T and D^T r_i is row i of R @ D.

Paper: Ablin, Moreau, Massias, Gramfort, "Learning step sizes for unfolded
sparse coding" (NeurIPS 2019, arXiv 1905.11071).

Pins (tests that tie each function to something other than itself) are
listed per function; none of them is left "parity unpinned".
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np
import scipy.linalg

__all__ = [
    "soft_threshold",
    "lipschitz",
    "lambda_max",
    "objective",
    "forward",
    "forward_backward",
    "adjoint",
    "kkt_residual",
    "lasso_solution",
    "brute_force_lasso",
    "train_steps",
    "support_lipschitz",
    "fista_momentum",
    "fista",
    "oista",
    "lista_layer",
    "lista_forward",
    "lista_forward_backward",
]


def _f64(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)


def soft_threshold(u, theta):
    """ST(u, theta) = sign(u) * max(|u| - theta, 0), with sign(0) = 0.

    Section 1, the definition following Eq. (2); the sign convention is the
    one of the Notation paragraph of Section 2.
    Pinned by a hand-computed table (tests/golden/soft_threshold.json).
    """
    u = _f64(u)
    return np.sign(u) * np.maximum(np.abs(u) - theta, 0.0)


def lipschitz(D) -> float:
    """L = greatest eigenvalue of D^T D (Section 1, after Eq. (2)).

    LAPACK symmetric eigensolver on the m x m Gram matrix. Pinned against
    the squared top singular value of D, the bounds 1 <= L <= m for
    unit-norm columns, and L = 1 for an orthogonal D.
    """
    D = _f64(D)
    return float(scipy.linalg.eigvalsh(D.T @ D)[-1])


def lambda_max(D, X) -> np.ndarray:
    """Per-sample lambda_max = ||D^T x||_inf (Section 2): below it the Lasso
    solution is non-zero, at or above it the solution is exactly 0."""
    return np.max(np.abs(_f64(X) @ _f64(D)), axis=1)


def objective(D, X, Z, lam) -> np.ndarray:
    """Per-sample Lasso cost F_x(z) = 1/2 ||x - D z||^2 + lam ||z||_1, Eq. (1).

    Pinned by F(0) = 1/2 ||x||^2 and by the closed-form cost of the
    Lemma 4.2 solution.
    """
    D, X, Z = _f64(D), _f64(X), _f64(Z)
    R = X - Z @ D.T
    return 0.5 * np.sum(R * R, axis=1) + lam * np.sum(np.abs(Z), axis=1)


def forward(D, X, lam, alpha, return_iterates: bool = False, dtype=np.float64):
    """T layers of Step-LISTA / proximal gradient with a step sequence.

    z^(0) = 0 and z^(t+1) = ST(z^(t) - alpha_t D^T (D z^(t) - x), lam alpha_t)
    (Section 3, Eq. (5); Section 4, Eq. (14)). With alpha_t = 1/L for every
    t this is ISTA, Eq. (2).

    The gradient is taken in the paper's factored form D^T (D z - x): a
    residual in R^n, then its correlation with the atoms.

    Returns Z^(T) [N, m] and the objective trace F [T+1, N] with
    F[t] = F_x(z^(t)). With return_iterates, also returns the list
    [z^(0), ..., z^(T)].

    Pins: monotone decrease of F for alpha_t <= 1/L (Section 3, Eq. (6)-(7)
    majorization), the sublinear ISTA rate of Section 3 (after Prop. 3.2),
    exact zeros when lam >= lambda_max (Section 2), one-step convergence for
    an orthogonal dictionary (Section 3, after Prop. 3.2), KKT at
    convergence (Lemma 2.1) and the Lemma 4.2 closed-form solution.

    dtype: the type every array of the recursion is held in. float64 is the
    oracle; float32 runs the same recursion with 32-bit rounding (the
    objective trace is still evaluated in float64), which the tests use as a
    measured rounding floor for 32-bit results, never as a reference.
    """
    D, X = np.asarray(D, dtype), np.asarray(X, dtype)
    alpha = np.asarray(alpha, dtype).reshape(-1)
    N, m = X.shape[0], D.shape[1]
    Z = np.zeros((N, m), dtype)
    iterates = [Z]
    trace = [objective(D, X, Z, lam)]
    for a in alpha:
        R = Z @ D.T - X                      # D z - x, per sample
        U = Z - a * (R @ D)                  # z - alpha D^T (D z - x)
        Z = soft_threshold(U, a * dtype(lam)).astype(dtype)
        iterates.append(Z)
        trace.append(objective(D, X, Z, lam))
    F = np.stack(trace)
    if return_iterates:
        return Z, F, iterates
    return Z, F


def forward_backward(D, X, lam, alpha, dZ=None, dF=None, return_adjoints: bool = False, dtype=np.float64):
    """Forward pass plus the reverse-mode derivative with respect to the steps.

    The scalar differentiated is J = sum_i dF_i F_{x_i}(z_i^(T)) + <dZ, Z^(T)>.
    With dF_i = 1/N and dZ = 0, J is the empirical unsupervised loss of
    Section 4, Eq. (15), which the paper differentiates by automatic
    differentiation (Appendix D, "Training the networks"). Here the
    derivative is written out by hand:

      seed       g = dZ + dF_i (D^T (D z^(T) - x) + lam sign z^(T))
                 (a sub-gradient of F, sign(0) = 0)
      for t = T-1 ... 0, with u = z^(t) - alpha_t D^T (D z^(t) - x):
        mask     M = [ |u| > lam alpha_t ]   (derivative of ST; 0 at the kink)
        v        = g * M
        dJ/dalpha_t = - sum v * (D^T (D z^(t) - x) + lam sign u)
        g        = v - alpha_t D^T D v       (back through the linear step)

    Returns (Z^(T), F [T+1, N], dalpha [T]); with return_adjoints also the
    iterates [z^(0) .. z^(T)] and the masked adjoints [v^(0) .. v^(T-1)]
    (v^(t) = g * M at layer t). Pinned against central finite differences of
    `forward` and against the closed form for T = 1. dtype as in `forward`
    (dalpha is summed in float64 either way).
    """
    Z, F, iterates = forward(D, X, lam, alpha, return_iterates=True, dtype=dtype)
    dalpha, adjoints = adjoint(D, X, lam, alpha, iterates, dZ=dZ, dF=dF, dtype=dtype)
    if return_adjoints:
        return Z, F, dalpha, iterates, adjoints
    return Z, F, dalpha


def adjoint(D, X, lam, alpha, iterates, dZ=None, dF=None, dtype=np.float64):
    """The reverse pass of `forward_backward` along given iterates
    z^(0) .. z^(T) (each [N, m]): the same recursion, with z^(t) taken from
    `iterates` instead of recomputed. Along the oracle's own iterates it is
    forward_backward's derivative; along iterates computed elsewhere (in
    another precision) it is the exact derivative of J at that trajectory's
    layers, which separates the error of a reverse pass from the error of
    the forward pass that fed it. Returns (dalpha [T], the masked adjoints
    [v^(0) .. v^(T-1)]). dtype as in `forward`."""
    D, X = np.asarray(D, dtype), np.asarray(X, dtype)
    alpha = np.asarray(alpha, dtype).reshape(-1)
    lam = dtype(lam)
    iterates = [np.asarray(z, dtype) for z in iterates]
    N, m = X.shape[0], D.shape[1]
    Z = iterates[len(alpha)]
    if dZ is None and dF is None:
        raise ValueError("forward_backward needs dZ and/or dF")
    g = np.zeros((N, m), dtype) if dZ is None else np.array(dZ, dtype)
    if dF is not None:
        dF = np.asarray(dF, dtype).reshape(-1)
        grad_T = (Z @ D.T - X) @ D
        g = g + dF[:, None] * (grad_T + lam * np.sign(Z))
    dalpha = np.zeros(len(alpha))
    adjoints = [None] * len(alpha)
    for t in range(len(alpha) - 1, -1, -1):
        a = alpha[t]
        Zt = iterates[t]
        grad = (Zt @ D.T - X) @ D            # D^T (D z^(t) - x)
        U = Zt - a * grad
        M = np.abs(U) > lam * a
        v = np.where(M, g, dtype(0))
        dalpha[t] = -np.sum(v * (grad + lam * np.sign(U)), dtype=np.float64)
        adjoints[t] = v
        g = v - a * ((v @ D.T) @ D)
    return dalpha, adjoints


def kkt_residual(D, X, Z, lam) -> np.ndarray:
    """Per-sample distance to the Lasso optimality conditions, Lemma 2.1, Eq. (3).

    With r_j = D_j^T (x - D z): for z_j != 0 the condition is
    r_j = lam sign z_j, for z_j = 0 it is |r_j| <= lam. Returns
    max_j of the violation (0 exactly at a solution).
    """
    D, X, Z = _f64(D), _f64(X), _f64(Z)
    Rc = (X - Z @ D.T) @ D
    viol = np.where(Z != 0.0, np.abs(Rc - lam * np.sign(Z)),
                    np.maximum(np.abs(Rc) - lam, 0.0))
    return np.max(viol, axis=1)


def _polish(D, x, z, lam, tol):
    """Exact solution on the support of z: solve the restricted optimality
    system D_S^T D_S z_S = D_S^T x - lam s_S (Eq. (3) on the support) and
    accept it only if it keeps the signs and satisfies Eq. (3) off the support.
    Returns the polished vector or None."""
    S = np.flatnonzero(z)
    out = np.zeros_like(z)
    if S.size:
        s = np.sign(z[S])
        DS = D[:, S]
        try:
            zS = np.linalg.solve(DS.T @ DS, DS.T @ x - lam * s)
        except np.linalg.LinAlgError:
            return None
        if np.any(np.sign(zS) != s):
            return None
        out[S] = zS
    r = D.T @ (x - D @ out)
    off = np.ones(z.shape[0], bool)
    off[S] = False
    if off.any() and np.max(np.abs(r[off])) > lam + tol:
        return None
    return out


def lasso_solution(D, X, lam, tol: float = 1e-10, max_iter: int = 200_000,
                   chunk: int = 500) -> np.ndarray:
    """The Lasso minimiser z*(x) of Eq. (1) for every sample, to machine precision.

    FISTA (Beck and Teboulle 2009; the accelerated method the paper compares
    against in Section 3) runs until every sample's support and signs are
    stable, then each sample is polished on its support (see `_polish`) and
    certified by the KKT conditions of Lemma 2.1 to `tol`. Unique under
    Assumption 2.2 (continuous D). Pinned against `brute_force_lasso` for
    m <= 8, against the Lemma 4.2 closed form, and by the KKT certificate.
    """
    D, X = _f64(D), _f64(X)
    N, m = X.shape[0], D.shape[1]
    L = lipschitz(D)
    C = X @ D
    G = D.T @ D
    Z = np.zeros((N, m))
    Y = Z.copy()
    tk = 1.0
    done = np.zeros(N, bool)
    out = np.zeros((N, m))
    it = 0
    while it < max_iter:
        for _ in range(chunk):
            Zn = soft_threshold(Y - (Y @ G - C) / L, lam / L)
            tn = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * tk * tk))
            Y = Zn + ((tk - 1.0) / tn) * (Zn - Z)
            Z, tk = Zn, tn
        it += chunk
        for i in np.flatnonzero(~done):
            p = _polish(D, X[i], Z[i], lam, tol)
            if p is not None and kkt_residual(D, X[i:i + 1], p[None], lam)[0] <= tol:
                out[i] = p
                done[i] = True
        if done.all():
            return out
    raise RuntimeError(f"lasso_solution: {int((~done).sum())} samples not certified")


def brute_force_lasso(D, x, lam) -> np.ndarray:
    """Exact Lasso solution by enumerating all 3^m sign patterns (m <= 8).

    For each pattern s in {-1, 0, +1}^m with support S (|S| <= n), the
    smooth cost restricted to the open orthant face {sign z = s} has its
    stationary point at D_S^T D_S z_S = D_S^T x - lam s_S; keep it if its
    signs match s and return the candidate of least F_x (Eq. (1)). The
    global minimiser lies in the relative interior of the face of its own
    sign pattern, so it is among the candidates.
    """
    D, x = _f64(D), _f64(x).reshape(-1)
    n, m = D.shape
    if m > 8:
        raise ValueError("brute_force_lasso is for m <= 8")
    best, best_f = np.zeros(m), 0.5 * float(x @ x)
    for code in range(3 ** m):
        s = np.empty(m)
        c = code
        for j in range(m):
            s[j] = (c % 3) - 1
            c //= 3
        S = np.flatnonzero(s)
        if S.size == 0 or S.size > n:
            continue
        DS = D[:, S]
        A = DS.T @ DS
        if np.linalg.matrix_rank(A) < S.size:
            continue
        zS = np.linalg.solve(A, DS.T @ x - lam * s[S])
        if np.any(np.sign(zS) != s[S]):
            continue
        z = np.zeros(m)
        z[S] = zS
        f = 0.5 * float(np.sum((x - D @ z) ** 2)) + lam * float(np.sum(np.abs(z)))
        if f < best_f:
            best, best_f = z, f
    return best


def train_steps(D, X, lam, alpha0, iters: int, lr: float, max_halvings: int = 30):
    """Full-batch sub-gradient descent on the step sizes with a backtracking
    learning rate (Appendix D, "Training the networks"), on the mean loss of
    Eq. (15). The paper does not spell the backtracking rule out; the reading
    taken: from the current steps alpha with loss J and gradient g, try
    alpha' = max(alpha - eta g, 0); if J(alpha') < J accept it and double eta,
    otherwise halve eta and try again, at most max_halvings times per
    iteration (no decrease found: stop).

    Returns (alpha [T], losses [accepted + 1], eta). Pinned by: the loss
    sequence decreases strictly; the first accepted step equals
    max(alpha0 - eta g, 0) with g from forward_backward; the learned steps of
    the paper's 10 x 20, lambda = 0.2 setting exceed 1/L in the late layers
    and stay below the largest 1/L_S of the supports reached (Section 4.1).
    """
    D, X = _f64(D), _f64(X)
    alpha = _f64(alpha0).reshape(-1).copy()
    N = X.shape[0]
    dF = np.full(N, 1.0 / N)
    _, F, g = forward_backward(D, X, lam, alpha, dF=dF)
    J = float(np.mean(F[-1]))
    losses = [J]
    eta = float(lr)
    for _ in range(iters):
        accepted = False
        for _ in range(max_halvings + 1):
            cand = np.maximum(alpha - eta * g, 0.0)
            Jc = float(np.mean(forward(D, X, lam, cand)[1][-1]))
            if Jc < J:
                alpha, J = cand, Jc
                _, _, g = forward_backward(D, X, lam, alpha, dF=dF)
                eta *= 2.0
                accepted = True
                break
            eta *= 0.5
        if not accepted:
            break
        losses.append(J)
    return alpha, np.array(losses), eta


def support_lipschitz(D, z) -> float:
    """L_S = greatest eigenvalue of D_S^T D_S for the support S of z (Section
    3, Oracle-ISTA); 0 for an empty support."""
    D = _f64(D)
    S = np.flatnonzero(_f64(z) != 0.0)
    if S.size == 0:
        return 0.0
    return float(scipy.linalg.eigvalsh(D[:, S].T @ D[:, S])[-1])


def fista_momentum(T: int) -> np.ndarray:
    """Momentum weights of FISTA (Beck & Teboulle 2009), the accelerated
    baseline of the paper's Figures 2 and D.2: tau_0 = 1,
    tau_{t+1} = (1 + sqrt(1 + 4 tau_t^2)) / 2, beta_t = (tau_t - 1) / tau_{t+1}
    (so beta_0 = 0)."""
    beta = np.zeros(T)
    tau = 1.0
    for t in range(T):
        tau_next = (1.0 + np.sqrt(1.0 + 4.0 * tau * tau)) / 2.0
        beta[t] = (tau - 1.0) / tau_next
        tau = tau_next
    return beta


def fista(D, X, lam, alpha, return_iterates: bool = False):
    """T layers of FISTA from z^(0) = y^(0) = 0, in the factored form:
        z^(t+1) = ST(y^(t) - alpha_t D^T (D y^(t) - x), lam alpha_t)
        y^(t+1) = z^(t+1) + beta_t (z^(t+1) - z^(t))
    with beta_t from fista_momentum. Returns (Z [N, m], F [T+1, N] of the z^(t),
    and the iterates z^(t) if asked). Pinned by: its first two layers equal
    ISTA's (beta_0 = 0), and with alpha = 1/L it meets the O(1/t^2) bound
    F(z^(t)) - F* <= 2 L ||z*||^2 / (t+1)^2."""
    D, X = _f64(D), _f64(X)
    alpha = _f64(alpha).reshape(-1)
    T = alpha.shape[0]
    beta = fista_momentum(T)
    N, m = X.shape[0], D.shape[1]
    z = np.zeros((N, m))
    y = np.zeros((N, m))
    F = np.empty((T + 1, N))
    F[0] = objective(D, X, z, lam)
    its = [z.copy()]
    for t in range(T):
        a = alpha[t]
        grad = (y @ D.T - X) @ D            # D^T (D y^(t) - x)
        z_next = soft_threshold(y - a * grad, lam * a)
        y = z_next + beta[t] * (z_next - z)
        z = z_next
        F[t + 1] = objective(D, X, z, lam)
        if return_iterates:
            its.append(z.copy())
    return (z, F, its) if return_iterates else (z, F)


def oista(D, X, lam, T: int, return_steps: bool = False):
    """Oracle-ISTA (Section 3, Algorithm 1), per sample, from z^(0) = 0:
        S = supp(z^(t)), L_S = greatest eigenvalue of D_S^T D_S (L_empty = L),
        y = psi_{1/L_S}(z^(t), x) = ST(z - (1/L_S) D^T (D z - x), lam / L_S);
        z^(t+1) = y if supp(y) is inside S (condition (*)),
                  else psi_{1/L}(z^(t), x).
    Returns (Z [N, m], F [T+1, N]) and, if asked, the step used by every
    sample at every layer [T, N]. Pinned by: its first layer equals ISTA's
    (S is empty at z^(0) = 0); F decreases at every layer (majorization by
    the tighter surrogate, Eq. (7)); on a long run it reaches z*."""
    D, X = _f64(D), _f64(X)
    N, m = X.shape[0], D.shape[1]
    L = lipschitz(D)
    Z = np.zeros((N, m))
    F = np.empty((T + 1, N))
    F[0] = objective(D, X, Z, lam)
    steps = np.empty((T, N))
    for t in range(T):
        for i in range(N):
            z, x = Z[i], X[i]
            S = z != 0.0
            LS = support_lipschitz(D, z) if S.any() else L
            grad = D.T @ (D @ z - x)
            y = soft_threshold(z - grad / LS, lam / LS)
            if np.all(S | (y == 0.0)):
                Z[i], steps[t, i] = y, 1.0 / LS
            else:
                Z[i], steps[t, i] = soft_threshold(z - grad / L, lam / L), 1.0 / L
        F[t + 1] = objective(D, X, Z, lam)
    return (Z, F, steps) if return_steps else (Z, F)


def lista_layer(D, X, lam, Z, W, a, b) -> np.ndarray:
    """One coupled LISTA layer, Section 4, Eq. (11):
        phi_theta(z, x) = ST(z - a W^T (D z - x), b lam),  theta = (W, a, b),
    W in R^{n x m} (the coupling W_z = I - W_x^T D that precedes Eq. (11))."""
    D, X, Z, W = _f64(D), _f64(X), _f64(Z), _f64(W)
    R = Z @ D.T - X                          # D z - x
    return soft_threshold(Z - a * (R @ W), lam * b)


def lista_forward(D, X, lam, W, alpha, beta, return_iterates: bool = False):
    """The LISTA network of Section 4, Eq. (12): z^(0) = 0 and
    z^(t+1) = phi_{theta_t}(z^(t), x) with per-layer theta_t = (W_t, alpha_t, beta_t),
    W [T, n, m]. With W_t = D and alpha_t = beta_t this is the Step-LISTA /
    ISTA recursion (the remark after Eq. (12)).

    Returns Z^(T) [N, m] and F [T+1, N] (F[t] = F_x(z^(t)), Eq. (1)), plus the
    iterates if asked. Pins: ISTA equivalence for W_t = D, alpha_t = beta_t;
    the closed form of one layer from z^(0) = 0, z^(1) = ST(alpha_0 W_0^T x,
    beta_0 lam); a Lasso solution is a fixed point of every layer with
    alpha W = beta D (the "if" direction of Lemma 4.3)."""
    D, X, W = _f64(D), _f64(X), _f64(W)
    alpha = _f64(alpha).reshape(-1)
    beta = _f64(beta).reshape(-1)
    if W.ndim != 3 or W.shape[0] != alpha.shape[0] or beta.shape != alpha.shape:
        raise ValueError("W must be [T, n, m] with alpha, beta of length T")
    N, m = X.shape[0], D.shape[1]
    Z = np.zeros((N, m))
    iterates = [Z]
    trace = [objective(D, X, Z, lam)]
    for t in range(alpha.shape[0]):
        Z = lista_layer(D, X, lam, Z, W[t], alpha[t], beta[t])
        iterates.append(Z)
        trace.append(objective(D, X, Z, lam))
    F = np.stack(trace)
    return (Z, F, iterates) if return_iterates else (Z, F)


def lista_forward_backward(D, X, lam, W, alpha, beta, dZ=None, dF=None):
    """LISTA forward pass plus the reverse-mode derivative of
    J = sum_i dF_i F_{x_i}(z_i^(T)) + <dZ, Z^(T)> with respect to every layer's
    (W_t, alpha_t, beta_t); with dF_i = 1/N, J is the unsupervised loss of
    Eq. (15) that the paper trains LISTA on (Section 5 / Appendix D).

    Written out by hand (the paper uses automatic differentiation): with
    r = D z^(t) - x, u = z^(t) - alpha_t W_t^T r, M = [|u| > beta_t lam],
      seed         g = dZ + dF_i (D^T (D z^(T) - x) + lam sign z^(T))
      v            = g * M
      dJ/dalpha_t  = - sum v * (W_t^T r)
      dJ/dbeta_t   = - lam sum v * sign(u)
      dJ/dW_t      = - alpha_t sum_i r_i v_i^T          ([n, m])
      g            = v - alpha_t D^T (W_t v)             (back through the layer)

    Returns (Z [N, m], F [T+1, N], dW [T, n, m], dalpha [T], dbeta [T]).
    Pins: central finite differences of lista_forward; for W_t = D and
    alpha_t = beta_t, dalpha + dbeta equals the Step-LISTA derivative of
    forward_backward; the rescaling (W, alpha) -> (c W, alpha / c) leaves the
    network unchanged, so sum W_t * dW_t = alpha_t dalpha_t for every t."""
    D, X, W = _f64(D), _f64(X), _f64(W)
    alpha = _f64(alpha).reshape(-1)
    beta = _f64(beta).reshape(-1)
    Z, F, iterates = lista_forward(D, X, lam, W, alpha, beta, return_iterates=True)
    if dZ is None and dF is None:
        raise ValueError("lista_forward_backward needs dZ and/or dF")
    N, m = X.shape[0], D.shape[1]
    g = np.zeros((N, m)) if dZ is None else _f64(dZ).copy()
    if dF is not None:
        dF = _f64(dF).reshape(-1)
        g = g + dF[:, None] * ((Z @ D.T - X) @ D + lam * np.sign(Z))
    T = alpha.shape[0]
    dW = np.zeros_like(W)
    dalpha = np.zeros(T)
    dbeta = np.zeros(T)
    for t in range(T - 1, -1, -1):
        a, b, Wt, Zt = alpha[t], beta[t], W[t], iterates[t]
        R = Zt @ D.T - X                     # D z^(t) - x
        WR = R @ Wt                          # W_t^T (D z^(t) - x)
        U = Zt - a * WR
        v = np.where(np.abs(U) > lam * b, g, 0.0)
        dalpha[t] = -np.sum(v * WR)
        dbeta[t] = -lam * np.sum(v * np.sign(U))
        dW[t] = -a * (R.T @ v)
        g = v - a * ((v @ Wt.T) @ D)
    return Z, F, dW, dalpha, dbeta
