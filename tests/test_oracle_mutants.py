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
