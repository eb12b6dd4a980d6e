"""Pins for the FP64 oracle: every oracle function is checked against values,
closed forms, invariants or brute force fixed by the paper and the
mathematics, not against itself. CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_soft_threshold_table():
    with open(os.path.join(GOLDEN, "soft_threshold.json")) as f:
        table = json.load(f)
    for case in table["cases"]:
        got = oracle.soft_threshold(np.array([case["u"]]), case["theta"])[0]
        assert got == pytest.approx(case["st"], abs=1e-15), case
        # sign(0) = 0: no negative zero leaks through as a non-zero
        if case["st"] == 0.0:
            assert got == 0.0


def test_lipschitz_matches_svd_and_bounds():
    pb = pins.small_problem(n=30, m=90, N=4)
    L = oracle.lipschitz(pb.D)
    s0 = np.linalg.svd(pb.D, compute_uv=False)[0]
    assert L == pytest.approx(s0 * s0, rel=1e-12)
    # unit-norm columns: diag(G) = 1 and trace(G) = m, so 1 <= L <= m
    assert 1.0 <= L <= pb.m


def test_lipschitz_orthogonal_is_one():
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((16, 16)))
    assert oracle.lipschitz(Q) == pytest.approx(1.0, abs=1e-13)


def test_objective_at_zero_and_lemma42():
    pb = pins.small_problem()
    F0 = oracle.objective(pb.D, pb.X, np.zeros((pb.N, pb.m)), pb.lam)
    np.testing.assert_allclose(F0, 0.5 * np.sum(pb.X ** 2, axis=1), rtol=1e-14)
    D, X, lam, zstar, Fstar = pins.lemma42_case()
    assert oracle.objective(D, X, zstar, lam)[0] == pytest.approx(Fstar, rel=1e-13)


def test_lambda_max_threshold():
    pb = pins.small_problem()
    lm = oracle.lambda_max(pb.D, pb.X)
    assert np.all(lm >= 0) and np.max(lm) > 0   # all-zero codes give x = 0, lambda_max = 0
    # lambda >= lambda_max(x) for every sample => every layer is exactly 0
    L = oracle.lipschitz(pb.D)
    Z, F = oracle.forward(pb.D, pb.X, float(np.max(lm)), np.full(25, 1.0 / L))
    assert np.all(Z == 0.0)
    np.testing.assert_array_equal(F[-1], F[0])


def test_forward_monotone_ista():
    pb = pins.small_problem()
    assert pins.monotone_violation(oracle.forward, oracle.lipschitz, pb) <= 1e-14


def test_forward_monotone_any_step_below_one_over_L():
    pb = pins.small_problem(seed=9)
    L = oracle.lipschitz(pb.D)
    alpha = np.random.default_rng(1).uniform(0.1, 1.0, 60) / L
    _, F = oracle.forward(pb.D, pb.X, pb.lam, alpha)
    assert np.max(np.diff(F, axis=0)) <= 1e-13


def test_forward_rate_bound():
    pb = pins.small_problem(N=32)
    zs = oracle.lasso_solution(pb.D, pb.X, pb.lam)
    v = pins.rate_violation(oracle.forward, oracle.lipschitz, oracle.objective, zs, pb)
    assert v <= 1e-12


def test_forward_kkt_at_convergence():
    pb = pins.small_problem(N=16)
    assert pins.kkt_after_long_run(oracle.forward, oracle.kkt_residual, oracle.lipschitz, pb) <= 1e-9


def test_forward_orthogonal_one_step():
    assert pins.orthogonal_one_step_error(oracle.forward, oracle.kkt_residual) <= 1e-13


def test_forward_reaches_lemma42_solution():
    D, X, lam, zstar, Fstar = pins.lemma42_case()
    L = oracle.lipschitz(D)
    Z, F = oracle.forward(D, X, lam, np.full(3000, 1.0 / L))
    np.testing.assert_allclose(Z, zstar, atol=1e-9)
    assert F[-1, 0] == pytest.approx(Fstar, rel=1e-12)


def test_forward_trace_matches_objective():
    pb = pins.small_problem(N=8)
    L = oracle.lipschitz(pb.D)
    alpha = np.full(5, 1.0 / L)
    Z, F, its = oracle.forward(pb.D, pb.X, pb.lam, alpha, return_iterates=True)
    assert F.shape == (6, 8)
    for t, Zt in enumerate(its):
        np.testing.assert_allclose(F[t], oracle.objective(pb.D, pb.X, Zt, pb.lam), rtol=0)
    np.testing.assert_array_equal(its[-1], Z)


def test_zero_layers():
    pb = pins.small_problem(N=4)
    Z, F = oracle.forward(pb.D, pb.X, pb.lam, np.zeros(0))
    assert np.all(Z == 0) and F.shape == (1, 4)
    np.testing.assert_allclose(F[0], 0.5 * np.sum(pb.X ** 2, axis=1))


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_lasso_solution_vs_brute_force(seed):
    pb = synth.make_problem(5, 8, 6, 0.3, 0.05, 0.3, seed=100 + seed)
    zs = oracle.lasso_solution(pb.D, pb.X, pb.lam)
    for i in range(pb.N):
        zb = oracle.brute_force_lasso(pb.D, pb.X[i], pb.lam)
        np.testing.assert_allclose(zs[i], zb, atol=1e-10)
        assert np.array_equal(np.sign(zs[i]), np.sign(zb))
    assert np.max(oracle.kkt_residual(pb.D, pb.X, zs, pb.lam)) <= 1e-10


def test_lasso_solution_lemma42():
    D, X, lam, zstar, _ = pins.lemma42_case(seed=5)
    np.testing.assert_allclose(oracle.lasso_solution(D, X, lam), zstar, atol=1e-12)


def test_brute_force_zero_above_lambda_max():
    pb = synth.make_problem(4, 6, 3, 0.3, 0.0, 0.5, seed=3)
    for i in range(3):
        lm = float(oracle.lambda_max(pb.D, pb.X[i:i + 1])[0])
        assert np.all(oracle.brute_force_lasso(pb.D, pb.X[i], lm * 1.0001) == 0.0)
        assert np.any(oracle.brute_force_lasso(pb.D, pb.X[i], lm * 0.5) != 0.0)


def test_kkt_residual_definition_points():
    D, X, lam, zstar, _ = pins.lemma42_case(seed=2)
    assert oracle.kkt_residual(D, X, zstar, lam)[0] <= 1e-13
    bad = zstar.copy()
    bad[0, 5] *= 0.9
    assert oracle.kkt_residual(D, X, bad, lam)[0] > 1e-3


@pytest.mark.parametrize("use_dz", [False, True])
def test_adjoint_vs_finite_differences(use_dz):
    pb = synth.make_problem(8, 16, 24, 0.2, 0.01, 0.1, seed=21)
    L = oracle.lipschitz(pb.D)
    alpha = synth.perturbed_steps(L, 6, seed=4)
    dF = np.full(pb.N, 1.0 / pb.N)
    dZ = np.random.default_rng(5).standard_normal((pb.N, pb.m)) if use_dz else None
    _, _, g = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dZ=dZ, dF=dF)
    fd = pins.fd_gradient(oracle.forward, pb.D, pb.X, pb.lam, alpha, dZ, dF)
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_adjoint_one_layer_closed_form():
    pb = synth.make_problem(8, 16, 24, 0.2, 0.01, 0.1, seed=22)
    a = 0.7 / oracle.lipschitz(pb.D)
    dF = np.random.default_rng(3).uniform(0.5, 1.5, pb.N)
    _, _, g = oracle.forward_backward(pb.D, pb.X, pb.lam, np.array([a]), dF=dF)
    assert g[0] == pytest.approx(pins.one_layer_gradient(pb.D, pb.X, pb.lam, a, dF), rel=1e-12)


def test_adjoint_is_linear_in_seeds():
    pb = synth.make_problem(6, 12, 10, 0.2, 0.0, 0.1, seed=23)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 5, seed=1)
    rng = np.random.default_rng(8)
    dZ, dF = rng.standard_normal((10, 12)), rng.standard_normal(10)
    _, _, g1 = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dZ=dZ)
    _, _, g2 = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dF=dF)
    _, _, g3 = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dZ=dZ, dF=dF)
    np.testing.assert_allclose(g3, g1 + g2, rtol=1e-12, atol=1e-14)


# --- step-size training (Appendix D) and per-support Lipschitz constants ------

def test_support_lipschitz_special_cases():
    pb = synth.make_problem(10, 20, 4, 0.1, 0.0, 0.1, seed=31)
    z = np.zeros(20)
    assert oracle.support_lipschitz(pb.D, z) == 0.0
    z[3] = 1.0                                    # one atom: L_S = ||D_j||^2 (1 up to the FP32 rounding of D)
    assert abs(oracle.support_lipschitz(pb.D, z) - float(pb.D[:, 3] @ pb.D[:, 3])) < 1e-14
    assert abs(oracle.support_lipschitz(pb.D, np.ones(20)) - oracle.lipschitz(pb.D)) < 1e-10
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((6, 6)))
    assert abs(oracle.support_lipschitz(Q, np.ones(6)) - 1.0) < 1e-12   # orthogonal D


def test_train_steps_update_rule_and_monotone_loss():
    """Each accepted iterate is max(alpha - eta g, 0) with g the oracle's
    gradient at the previous iterate, and the loss decreases strictly."""
    pb = synth.make_binf_problem(10, 20, 300, 0.2, seed=1101)
    L = oracle.lipschitz(pb.D)
    a0 = np.full(12, 1.0 / L)
    a1, l1, eta1 = oracle.train_steps(pb.D, pb.X, pb.lam, a0, 1, lr=1.0 / L)
    assert len(l1) == 2 and l1[1] < l1[0]
    _, _, g0 = oracle.forward_backward(pb.D, pb.X, pb.lam, a0, dF=np.full(pb.N, 1.0 / pb.N))
    assert np.allclose(a1, np.maximum(a0 - (eta1 / 2.0) * g0, 0.0), rtol=0, atol=1e-15)
    _, l20, _ = oracle.train_steps(pb.D, pb.X, pb.lam, a0, 20, lr=1.0 / L)
    assert np.all(np.diff(l20) < 0)


def test_learned_steps_exceed_one_over_L_within_support_range():
    """Section 4.1 / Fig. 4 setting (10 x 20 dictionary, lambda = 0.2, 1000
    samples on B_inf, 20 layers): the learned steps of the late layers are
    larger than 1/L and no larger than the largest 1/L_S of the supports the
    layer's outputs reach."""
    pb = synth.make_binf_problem(10, 20, 1000, 0.2, seed=1101)
    L = oracle.lipschitz(pb.D)
    T = 20
    alpha, losses, _ = oracle.train_steps(pb.D, pb.X, pb.lam, np.full(T, 1.0 / L), 200, lr=1.0 / L)
    assert losses[-1] < losses[0]
    _, _, its = oracle.forward(pb.D, pb.X, pb.lam, alpha, return_iterates=True)
    for t in range(T // 2, T):
        assert alpha[t] > 1.0 / L
        inv_ls = [1.0 / oracle.support_lipschitz(pb.D, z) for z in its[t + 1] if np.any(z)]
        assert alpha[t] <= max(inv_ls)


# --- FISTA (the accelerated baseline of Figs. 2 and D.2) ------------------------

def test_fista_momentum_closed_values():
    beta = oracle.fista_momentum(4)
    tau1 = (1 + 5 ** 0.5) / 2
    tau2 = (1 + (1 + 4 * tau1 ** 2) ** 0.5) / 2
    assert beta[0] == 0.0
    assert abs(beta[1] - (tau1 - 1) / tau2) < 1e-15
    assert np.all(np.diff(beta) > 0) and np.all(beta < 1)


def test_fista_first_two_layers_are_ista():
    pb = synth.make_problem(16, 40, 50, 0.1, 0.01, 0.1, seed=41)
    a = np.full(2, 1.0 / oracle.lipschitz(pb.D))
    Zf, Ff = oracle.fista(pb.D, pb.X, pb.lam, a)
    Zi, Fi = oracle.forward(pb.D, pb.X, pb.lam, a)[:2]
    assert np.array_equal(Zf, Zi)
    assert np.allclose(Ff, Fi, rtol=0, atol=0)


def test_fista_meets_its_rate_bound():
    """Beck & Teboulle (2009), Thm 4.4, from z^(0) = 0 with step 1/L."""
    pb = synth.make_problem(20, 50, 40, 0.1, 0.0, 0.1, seed=43)
    L = oracle.lipschitz(pb.D)
    T = 60
    _, F = oracle.fista(pb.D, pb.X, pb.lam, np.full(T, 1.0 / L))
    zs = oracle.lasso_solution(pb.D, pb.X, pb.lam)
    Fs = oracle.objective(pb.D, pb.X, zs, pb.lam)
    bound = 2.0 * L * np.sum(zs * zs, axis=1)
    for t in range(1, T + 1):
        assert np.all(F[t] - Fs <= bound / (t + 1) ** 2 + 1e-12)


# --- Oracle-ISTA (Section 3, Algorithm 1) -------------------------------------

def test_oista_first_layer_is_ista_and_descends():
    pb = synth.make_binf_problem(10, 50, 30, 0.5, seed=1201)
    L = oracle.lipschitz(pb.D)
    Z1, _ = oracle.oista(pb.D, pb.X, pb.lam, 1)           # S is empty at z^(0) = 0: L_S = L
    Zi, _ = oracle.forward(pb.D, pb.X, pb.lam, np.array([1.0 / L]))[:2]
    np.testing.assert_allclose(Z1, Zi, rtol=1e-13, atol=1e-15)   # same step; only the BLAS order differs
    _, F = oracle.oista(pb.D, pb.X, pb.lam, 80)
    assert np.all(np.diff(F, axis=0) <= 1e-14 * np.abs(F[:-1]))   # every layer lowers F


def test_oista_converges_faster_than_ista_and_reaches_kkt():
    """Fig. 2 setting (10 x 50 dictionary, lambda = 0.5, samples on B_inf)."""
    pb = synth.make_binf_problem(10, 50, 30, 0.5, seed=1201)
    L = oracle.lipschitz(pb.D)
    T = 100
    Zo, Fo, steps = oracle.oista(pb.D, pb.X, pb.lam, T, return_steps=True)
    _, Fi = oracle.forward(pb.D, pb.X, pb.lam, np.full(T, 1.0 / L))[:2]
    zs = oracle.lasso_solution(pb.D, pb.X, pb.lam)
    Fs = oracle.objective(pb.D, pb.X, zs, pb.lam)
    assert np.mean(Fo[T] - Fs) < 1e-2 * np.mean(Fi[T] - Fs)
    assert np.all(steps >= 1.0 / L * (1 - 1e-12)) and np.any(steps > 1.5 / L)
    _, Flong = oracle.oista(pb.D, pb.X, pb.lam, 400)
    assert np.max(Flong[-1] - Fs) < 1e-9


# --- coupled LISTA (Section 4, Eq. (11)-(12); Lemma 4.3, Theorem 4.4) -------

def _lista_params(pb, T, seed, spread=0.3):
    """Per-layer parameters near the ISTA point: W_t = D + spread E_t,
    alpha_t, beta_t around 1/L."""
    rng = np.random.default_rng(seed)
    L = oracle.lipschitz(pb.D)
    W = pb.D[None] + spread * rng.standard_normal((T, pb.n, pb.m)) / np.sqrt(pb.n)
    alpha = (1.0 / L) * rng.uniform(0.6, 1.4, T)
    beta = (1.0 / L) * rng.uniform(0.6, 1.4, T)
    return W, alpha, beta


def test_lista_coupled_to_dictionary_is_ista():
    """W_t = D, alpha_t = beta_t gives the Step-LISTA recursion (the remark
    after Eq. (12)); with alpha_t = 1/L, ISTA."""
    pb = synth.make_problem(8, 16, 30, 0.2, 0.01, 0.1, seed=31)
    L = oracle.lipschitz(pb.D)
    for alpha in (np.full(7, 1.0 / L), synth.perturbed_steps(L, 7, seed=2)):
        W = np.repeat(pb.D[None], 7, axis=0)
        Zl, Fl = oracle.lista_forward(pb.D, pb.X, pb.lam, W, alpha, alpha)
        Zs, Fs = oracle.forward(pb.D, pb.X, pb.lam, alpha)
        np.testing.assert_allclose(Zl, Zs, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(Fl, Fs, rtol=1e-13)


def test_lista_one_layer_closed_form():
    """From z^(0) = 0 the residual is -x, so z^(1) = ST(alpha W^T x, beta lam)
    = sign(W^T x) max(alpha |W^T x| - beta lam, 0), checked coordinate by
    coordinate with plain Python arithmetic."""
    pb = synth.make_problem(5, 9, 4, 0.3, 0.01, 0.1, seed=32)
    W, a, b = _lista_params(pb, 1, seed=3)
    Z, _ = oracle.lista_forward(pb.D, pb.X, pb.lam, W, a, b)
    for i in range(pb.N):
        for j in range(pb.m):
            wx = sum(W[0, k, j] * pb.X[i, k] for k in range(pb.n))
            mag = a[0] * abs(wx) - b[0] * pb.lam
            want = (1.0 if wx > 0 else -1.0) * mag if mag > 0 else 0.0
            assert Z[i, j] == pytest.approx(want, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("use_dz", [False, True])
def test_lista_adjoint_vs_finite_differences(use_dz):
    pb = synth.make_problem(6, 12, 20, 0.25, 0.01, 0.1, seed=33)
    T = 5
    W, alpha, beta = _lista_params(pb, T, seed=4)
    dF = np.full(pb.N, 1.0 / pb.N)
    rng = np.random.default_rng(6)
    dZ = rng.standard_normal((pb.N, pb.m)) if use_dz else None
    _, _, dW, da, db = oracle.lista_forward_backward(pb.D, pb.X, pb.lam, W, alpha, beta, dZ=dZ, dF=dF)

    def J(W_, a_, b_):
        Z, F = oracle.lista_forward(pb.D, pb.X, pb.lam, W_, a_, b_)
        return float(np.sum(dF * F[-1])) + (float(np.sum(dZ * Z)) if use_dz else 0.0)

    h = 1e-6
    for t in range(T):
        e = np.zeros(T)
        e[t] = h
        fa = (J(W, alpha + e, beta) - J(W, alpha - e, beta)) / (2 * h)
        fb = (J(W, alpha, beta + e) - J(W, alpha, beta - e)) / (2 * h)
        assert da[t] == pytest.approx(fa, rel=1e-5, abs=1e-7 * max(1.0, abs(fa)))
        assert db[t] == pytest.approx(fb, rel=1e-5, abs=1e-7 * max(1.0, abs(fb)))
    scale = np.max(np.abs(dW))
    for _ in range(25):
        t, k, j = rng.integers(T), rng.integers(pb.n), rng.integers(pb.m)
        Wp, Wm = W.copy(), W.copy()
        Wp[t, k, j] += h
        Wm[t, k, j] -= h
        fd = (J(Wp, alpha, beta) - J(Wm, alpha, beta)) / (2 * h)
        assert abs(dW[t, k, j] - fd) <= 1e-6 * scale


def test_lista_adjoint_reduces_to_step_lista():
    """With W_t = D and alpha_t = beta_t = a_t, a_t drives both the step and the
    threshold, so the Step-LISTA derivative (itself pinned by finite
    differences) is dalpha_t + dbeta_t of the LISTA network."""
    pb = synth.make_problem(8, 16, 24, 0.2, 0.01, 0.1, seed=34)
    L = oracle.lipschitz(pb.D)
    a = synth.perturbed_steps(L, 6, seed=5)
    dF = np.full(pb.N, 1.0 / pb.N)
    W = np.repeat(pb.D[None], 6, axis=0)
    _, _, _, da, db = oracle.lista_forward_backward(pb.D, pb.X, pb.lam, W, a, a, dF=dF)
    _, _, g = oracle.forward_backward(pb.D, pb.X, pb.lam, a, dF=dF)
    np.testing.assert_allclose(da + db, g, rtol=1e-10, atol=1e-14)


def test_lista_adjoint_rescaling_invariant():
    """(W_t, alpha_t) -> (c W_t, alpha_t / c) leaves every layer unchanged, so
    the derivative along that direction vanishes: <W_t, dW_t> = alpha_t dalpha_t."""
    pb = synth.make_problem(8, 20, 30, 0.2, 0.01, 0.1, seed=35)
    W, alpha, beta = _lista_params(pb, 6, seed=7, spread=0.5)
    _, _, dW, da, _ = oracle.lista_forward_backward(pb.D, pb.X, pb.lam, W, alpha, beta,
                                                    dF=np.full(pb.N, 1.0 / pb.N))
    lhs = np.einsum("tkj,tkj->t", W, dW)
    np.testing.assert_allclose(lhs, alpha * da, rtol=1e-10, atol=1e-14)


def test_lista_fixed_point_iff_aligned_lemma43():
    """Lemma 4.3 on the Lemma 4.2 construction: z* = (1 - lam) e_j is a fixed
    point of a layer with alpha W = beta D, and is moved by a layer whose
    column j is not aligned with D_j."""
    D, X, lam, Z, _ = pins.lemma42_case()
    rng = np.random.default_rng(8)
    for a, b in ((0.3, 0.3), (0.5, 0.2), (0.1, 0.4)):
        W = (b / a) * D
        np.testing.assert_allclose(oracle.lista_layer(D, X, lam, Z, W, a, b), Z, atol=1e-12)
    j = int(np.flatnonzero(Z[0])[0])
    W = D.copy()
    W[:, j] += 0.5 * rng.standard_normal(D.shape[0])
    assert np.max(np.abs(oracle.lista_layer(D, X, lam, Z, W, 0.3, 0.3) - Z)) > 1e-3


def test_adjoint_along_its_own_iterates_is_forward_backward():
    """The reverse pass along given iterates reproduces forward_backward's
    derivative along the oracle's own trajectory (whose finite-difference and
    closed-form pins above then pin it), and its adjoints are the masked
    vectors the recursion multiplies by the layers' Jacobians."""
    pb = pins.small_problem(N=40)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 7, seed=3)
    dF = np.full(pb.N, 1.0 / pb.N)
    _, _, da, its, adj = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dF=dF, return_adjoints=True)
    da2, adj2 = oracle.adjoint(pb.D, pb.X, pb.lam, alpha, its, dF=dF)
    assert np.array_equal(da, da2)
    assert all(np.array_equal(a, b) for a, b in zip(adj, adj2))
    # the last adjoint is the seed restricted to the last layer's mask
    Z = its[-1]
    seed = dF[:, None] * ((Z @ pb.D.T - pb.X) @ pb.D + pb.lam * np.sign(Z))
    a = alpha[-1]
    U = its[-2] - a * ((its[-2] @ pb.D.T - pb.X) @ pb.D)
    np.testing.assert_array_equal(adj[-1], np.where(np.abs(U) > pb.lam * a, seed, 0.0))


def test_float32_evaluation_runs_in_float32_and_stays_near_float64():
    """dtype=float32 evaluates the same recursion with 32-bit arrays (the
    tests' measured rounding floor for 32-bit results): the iterates are
    float32, and z^T and dalpha stay within a few thousand unit roundoffs of
    the float64 oracle on a small problem."""
    pb = pins.small_problem(N=40)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 12, seed=5)
    dF = np.full(pb.N, 1.0 / pb.N)
    Z64, _, da64, its64, _ = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dF=dF, return_adjoints=True)
    Z32, _, da32, its32, adj32 = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dF=dF, return_adjoints=True,
                                                         dtype=np.float32)
    assert all(z.dtype == np.float32 for z in its32) and all(v.dtype == np.float32 for v in adj32)
    assert np.max(np.abs(Z32 - Z64)) <= 1e-4 * np.max(np.abs(Z64))
    assert np.max(np.abs(da32 - da64)) <= 1e-4 * np.max(np.abs(da64))
    assert np.max(np.abs(da32 - da64)) > 0.0   # it did round
