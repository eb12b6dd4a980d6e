"""Planted mistakes, on the CPU: a broken copy of an oracle function must fail
at least one of the pins in tests/pins.py. This is what makes the pins
evidence: a dropped term, a wrong sign, a wrong threshold or a transposed
operand does not pass silently."""
import numpy as np

import oracle
from tests import pins


def _st(u, th):
    return np.sign(u) * np.maximum(np.abs(u) - th, 0.0)


def _forward_factory(step_sign=-1.0, thresh_scale_alpha=True, transpose=False):
    def fwd(D, X, lam, alpha):
        D, X = np.asarray(D, float), np.asarray(X, float)
        Z = np.zeros((X.shape[0], D.shape[1]))
        tr = [oracle.objective(D, X, Z, lam)]
        for a in np.asarray(alpha, float):
            if transpose:
                g = (Z @ D - X) @ D.T      # D and D^T swapped (only square D runs)
            else:
                g = (Z @ D.T - X) @ D
            Z = _st(Z + step_sign * a * g, lam * a if thresh_scale_alpha else lam)
            tr.append(oracle.objective(D, X, Z, lam))
        return Z, np.stack(tr)
    return fwd


def test_mutant_wrong_step_sign_is_caught():
    pb = pins.small_problem()
    bad = _forward_factory(step_sign=+1.0)
    assert pins.monotone_violation(bad, oracle.lipschitz, pb) > 1e-6


def test_mutant_threshold_without_alpha_is_caught():
    pb = pins.small_problem(N=16)
    bad = _forward_factory(thresh_scale_alpha=False)
    assert pins.kkt_after_long_run(bad, oracle.kkt_residual, oracle.lipschitz, pb, T=500) > 1e-3


def test_mutant_transposed_operand_is_caught():
    bad = _forward_factory(transpose=True)
    assert pins.orthogonal_one_step_error(bad, oracle.kkt_residual) > 1e-3


def test_mutant_objective_without_half_is_caught():
    D, X, lam, zstar, Fstar = pins.lemma42_case()

    def bad_objective(D, X, Z, lam):
        R = X - Z @ D.T
        return np.sum(R * R, axis=1) + lam * np.sum(np.abs(Z), axis=1)
    assert abs(bad_objective(D, X, zstar, lam)[0] - Fstar) > 1e-3


def test_mutant_adjoint_without_l1_term_is_caught():
    import synth
    pb = synth.make_problem(8, 16, 24, 0.2, 0.01, 0.1, seed=21)
    L = oracle.lipschitz(pb.D)
    alpha = synth.perturbed_steps(L, 6, seed=4)
    dF = np.full(pb.N, 1.0 / pb.N)

    def bad_adjoint(D, X, lam, alpha):
        Z, F, its = oracle.forward(D, X, lam, alpha, return_iterates=True)
        g = dF[:, None] * ((Z @ D.T - X) @ D)          # lam * sign(z) dropped
        da = np.zeros_like(alpha)
        for t in range(len(alpha) - 1, -1, -1):
            grad = (its[t] @ D.T - X) @ D
            U = its[t] - alpha[t] * grad
            v = np.where(np.abs(U) > lam * alpha[t], g, 0.0)
            da[t] = -np.sum(v * (grad + lam * np.sign(U)))
            g = v - alpha[t] * ((v @ D.T) @ D)
        return da
    fd = pins.fd_gradient(oracle.forward, pb.D, pb.X, pb.lam, alpha, None, dF)
    assert np.max(np.abs(bad_adjoint(pb.D, pb.X, pb.lam, alpha) - fd)) > 1e-3 * np.max(np.abs(fd))


def test_mutant_adjoint_without_mask_is_caught():
    pb = pins.small_problem(N=8)
    a = 0.7 / oracle.lipschitz(pb.D)
    dF = np.ones(pb.N)

    def bad_one_layer(D, X, lam, a):
        # forgets the ST mask: differentiates through the thresholded-away entries
        C = X @ D
        Z = _st(a * C, lam * a)
        g = dF[:, None] * ((Z @ D.T - X) @ D + lam * np.sign(Z))
        return -np.sum(g * (-C + lam * np.sign(a * C)))
    want = pins.one_layer_gradient(pb.D, pb.X, pb.lam, a, dF)
    assert abs(bad_one_layer(pb.D, pb.X, pb.lam, a) - want) > 1e-6 * abs(want)


# --- coupled LISTA: planted mistakes in the adjoint and the layer -----------

def _lista_fb_factory(dw_alpha=True, swap_back=False, dbeta_sign=1.0):
    """A copy of the LISTA forward/backward with one planted mistake."""
    def fb(D, X, lam, W, alpha, beta, dF):
        D, X, W = (np.asarray(a, float) for a in (D, X, W))
        Z, F, its = oracle.lista_forward(D, X, lam, W, alpha, beta, return_iterates=True)
        g = dF[:, None] * ((Z @ D.T - X) @ D + lam * np.sign(Z))
        dW, da, db = np.zeros_like(W), np.zeros(len(alpha)), np.zeros(len(alpha))
        for t in range(len(alpha) - 1, -1, -1):
            a, b, Wt, Zt = alpha[t], beta[t], W[t], its[t]
            R = Zt @ D.T - X
            WR = R @ Wt
            U = Zt - a * WR
            v = np.where(np.abs(U) > lam * b, g, 0.0)
            da[t] = -np.sum(v * WR)
            db[t] = -dbeta_sign * lam * np.sum(v * np.sign(U))
            dW[t] = -(a if dw_alpha else 1.0) * (R.T @ v)
            g = v - a * (((v @ D.T) @ Wt) if swap_back else ((v @ Wt.T) @ D))
        return dW, da, db
    return fb


def _lista_case():
    import synth
    pb = synth.make_problem(6, 12, 20, 0.25, 0.01, 0.1, seed=33)
    rng = np.random.default_rng(4)
    L = oracle.lipschitz(pb.D)
    T = 4
    W = pb.D[None] + 0.3 * rng.standard_normal((T, pb.n, pb.m)) / np.sqrt(pb.n)
    a = (1.0 / L) * rng.uniform(0.6, 1.4, T)
    b = (1.0 / L) * rng.uniform(0.6, 1.4, T)
    return pb, W, a, b, np.full(pb.N, 1.0 / pb.N)


def _lista_pin_failures(fb):
    """How many LISTA adjoint pins a candidate breaks: finite differences of
    the (correct) forward in alpha, beta and a few W entries; the rescaling
    invariant <W_t, dW_t> = alpha_t dalpha_t; the Step-LISTA reduction."""
    pb, W, a, b, dF = _lista_case()
    dW, da, db = fb(pb.D, pb.X, pb.lam, W, a, b, dF)

    def J(W_, a_, b_):
        return float(np.sum(dF * oracle.lista_forward(pb.D, pb.X, pb.lam, W_, a_, b_)[1][-1]))
    h, fails = 1e-6, 0
    e = np.zeros(len(a))
    e[1] = h
    if abs((J(W, a + e, b) - J(W, a - e, b)) / (2 * h) - da[1]) > 1e-6 * max(1.0, abs(da[1])):
        fails += 1
    if abs((J(W, a, b + e) - J(W, a, b - e)) / (2 * h) - db[1]) > 1e-6 * max(1.0, abs(db[1])):
        fails += 1
    Wp, Wm = W.copy(), W.copy()
    Wp[0, 2, 3] += h
    Wm[0, 2, 3] -= h
    if abs((J(Wp, a, b) - J(Wm, a, b)) / (2 * h) - dW[0, 2, 3]) > 1e-6 * np.max(np.abs(dW)):
        fails += 1
    if np.max(np.abs(np.einsum("tkj,tkj->t", W, dW) - a * da)) > 1e-10:
        fails += 1
    Wd = np.repeat(pb.D[None], len(a), axis=0)
    _, da2, db2 = fb(pb.D, pb.X, pb.lam, Wd, a, a, dF)
    g = oracle.forward_backward(pb.D, pb.X, pb.lam, a, dF=dF)[2]
    if np.max(np.abs(da2 + db2 - g)) > 1e-10 * np.max(np.abs(g)):
        fails += 1
    return fails


def test_lista_correct_adjoint_passes_every_pin():
    assert _lista_pin_failures(_lista_fb_factory()) == 0


def test_mutant_lista_weight_gradient_without_alpha_is_caught():
    assert _lista_pin_failures(_lista_fb_factory(dw_alpha=False)) > 0


def test_mutant_lista_backward_through_swapped_operators_is_caught():
    assert _lista_pin_failures(_lista_fb_factory(swap_back=True)) > 0


def test_mutant_lista_threshold_gradient_sign_is_caught():
    assert _lista_pin_failures(_lista_fb_factory(dbeta_sign=-1.0)) > 0


def test_mutant_lista_threshold_with_step_size_is_caught():
    """A layer thresholding at lam alpha_t instead of lam beta_t fails the
    one-layer closed form z^(1) = ST(alpha W^T x, beta lam)."""
    pb, W, a, b, _ = _lista_case()
    good = oracle.soft_threshold(a[0] * (pb.X @ W[0]), b[0] * pb.lam)
    bad = oracle.soft_threshold(a[0] * (pb.X @ W[0]), a[0] * pb.lam)
    assert np.max(np.abs(bad - good)) > 1e-6
