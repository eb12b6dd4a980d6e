"""Seeded synthetic Lasso problems for the unfolded-ISTA / Step-LISTA path.

This module only draws random inputs. It holds none of the iteration's
arithmetic, and it is the one piece of code that both the CPU oracle's tests
and the GPU path's tests, smoke check and benchmark use, so that both sides
see bit-identical inputs.

Recipe (the paper's synthetic setting, Section 5 and Appendix D):
  * dictionary D in R^{n x m}: i.i.d. N(0, 1) entries, then every column is
    divided by its l2 norm (unit-norm atoms);
  * codes z0 in R^m: Bernoulli(p) mask times N(0, 1) values;
  * samples x = D z0 + sigma * eps with eps ~ N(0, I_n);
  * lambda = frac * max_i ||D^T x_i||_inf  (lambda_max of Section 2, taken
    over the batch, so a single scalar lambda per problem).
  * an alternative sample recipe on the equiregularization set B_inf of
    Section 2: x = x_hat / ||D^T x_hat||_inf with x_hat ~ N(0, I_n).

Everything is drawn in float64 with numpy's PCG64 and rounded once to
float32; the returned float64 arrays are those float32 values widened, so
the FP64 oracle and the FP32 device path start from the same numbers.

Layout is sample-major: X is [N, n], codes are [N, m] (row i = sample i).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List

import numpy as np

__all__ = [
    "Problem",
    "make_dictionary",
    "make_problem",
    "make_binf_problem",
    "perturbed_steps",
    "CONFIGS",
    "UNEVEN",
    "uneven_problem_specs",
]


@dataclasses.dataclass
class Problem:
    """One Lasso problem instance (float32-representable values held in float64)."""

    D: np.ndarray  # [n, m]
    X: np.ndarray  # [N, n]
    Z0: np.ndarray  # [N, m] generating codes (not the Lasso solution)
    lam: float
    seed: int

    @property
    def n(self) -> int:
        return self.D.shape[0]

    @property
    def m(self) -> int:
        return self.D.shape[1]

    @property
    def N(self) -> int:
        return self.X.shape[0]

    def D32(self) -> np.ndarray:
        return np.ascontiguousarray(self.D, dtype=np.float32)

    def X32(self) -> np.ndarray:
        return np.ascontiguousarray(self.X, dtype=np.float32)


def _f32(a: np.ndarray) -> np.ndarray:
    """Round to float32 and widen back, so both sides see identical values."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def make_dictionary(rng: np.random.Generator, n: int, m: int) -> np.ndarray:
    """Gaussian dictionary with unit-norm columns (Section 5, synthetic case)."""
    D = rng.standard_normal((n, m))
    D /= np.linalg.norm(D, axis=0, keepdims=True)
    return _f32(D)


def make_problem(n: int, m: int, N: int, p: float, sigma: float, lam_frac: float,
                 seed: int) -> Problem:
    """Dictionary, Bernoulli(p)-Gaussian codes, noisy samples, lambda = frac*lambda_max."""
    rng = np.random.default_rng(seed)
    D = make_dictionary(rng, n, m)
    mask = rng.random((N, m)) < p
    Z0 = np.where(mask, rng.standard_normal((N, m)), 0.0)
    X = Z0 @ D.T
    if sigma > 0.0:
        X = X + sigma * rng.standard_normal((N, n))
    X = _f32(X)
    lam_max = float(np.max(np.abs(X @ D)))
    return Problem(D=D, X=X, Z0=Z0, lam=float(np.float32(lam_frac * lam_max)), seed=seed)


def make_binf_problem(n: int, m: int, N: int, lam: float, seed: int) -> Problem:
    """Samples on B_inf = {x : ||D^T x||_inf = 1} (Section 2, Appendix D)."""
    rng = np.random.default_rng(seed)
    D = make_dictionary(rng, n, m)
    Xh = rng.standard_normal((N, n))
    X = _f32(Xh / np.max(np.abs(Xh @ D), axis=1, keepdims=True))
    return Problem(D=D, X=X, Z0=np.zeros((N, m)), lam=float(np.float32(lam)), seed=seed)


def perturbed_steps(L: float, T: int, seed: int, spread: float = 0.3) -> np.ndarray:
    """Step sizes alpha_t = (1/L)(1 + spread*U[0,1)), rounded to float32.

    Used wherever the layers must not all be identical (gradient checks)."""
    rng = np.random.default_rng(seed)
    a = (1.0 / L) * (1.0 + spread * rng.random(T))
    return _f32(a)


def lista_params(D: np.ndarray, L: float, T: int, seed: int, spread: float):
    """Per-layer LISTA parameters near the ISTA point, rounded to float32:
    W_t = D + spread E_t / sqrt(n) with E_t standard normal [n, m], and
    alpha_t, beta_t drawn uniformly from (0.6 / L, 1.4 / L). Returns
    (W [T, n, m], alpha [T], beta [T])."""
    rng = np.random.default_rng(seed)
    n, m = D.shape
    W = np.asarray(D, np.float64)[None] + spread * rng.standard_normal((T, n, m)) / np.sqrt(n)
    a = (1.0 / L) * rng.uniform(0.6, 1.4, T)
    b = (1.0 / L) * rng.uniform(0.6, 1.4, T)
    return _f32(W), _f32(a), _f32(b)


# The five workloads. Seeds: config k uses 1000 + k; problem p of the uneven
# batch uses 5000 + p.
CONFIGS: Dict[str, dict] = {
    # Plain ISTA on a 10x20 dictionary, per-iteration objective trace.
    "ista_10x20": dict(n=10, m=20, N=1000, T=100, p=0.1, sigma=0.0, lam_frac=0.1, seed=1001),
    # Batched forward, 64x256, T=40, fixed step 1/L.
    "fwd_64x256": dict(n=64, m=256, N=10_000, T=40, p=0.05, sigma=0.01, lam_frac=0.1, seed=1002),
    # Learned steps with the adjoint, 64x256, N=4096, T=20.
    "grad_64x256": dict(n=64, m=256, N=4096, T=20, p=0.05, sigma=0.01, lam_frac=0.1, seed=1003),
    # Precision study, 256x1024, N=65536, T=50, forward+backward.
    "prec_256x1024": dict(n=256, m=1024, N=65_536, T=50, p=0.02, sigma=0.0, lam_frac=0.05, seed=1004),
    # Coupled LISTA (per-layer W_t, alpha_t, beta_t) on the 64x256 Gaussian
    # setting, forward+backward with the weight gradient.
    "lista_64x256": dict(n=64, m=256, N=10_000, T=40, p=0.05, sigma=0.01, lam_frac=0.1, seed=1006, spread=0.2),
}

# The uneven batch (sizes from uneven_problem_specs): common depth and checkpoint spacing.
UNEVEN: dict = dict(P=64, T=100, ckpt_every=10, seed=1005)


def uneven_problem_specs(P: int = 64, seed: int = 1005, n_lo: int = 32, n_hi: int = 512,
                         N_lo: int = 128, N_hi: int = 8192) -> List[dict]:
    """Sizes of the uneven multi-problem batch: n ~ U{n_lo..n_hi}, m = 4n,
    N ~ U{N_lo..N_hi} (inclusive), p = 0.05, sigma = 0, lambda = 0.1 lambda_max."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=P)
    Ns = rng.integers(N_lo, N_hi + 1, size=P)
    return [dict(n=int(n), m=4 * int(n), N=int(N), p=0.05, sigma=0.0, lam_frac=0.1,
                 seed=5000 + i) for i, (n, N) in enumerate(zip(ns, Ns))]
