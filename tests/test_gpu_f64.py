"""The FP64 forward (slista_forward_f64) against the FP64 oracle.

The double-precision ISTA workload (n = 10, m = 20, N = 1000, T = 100,
alpha = 1/L, lambda = 0.1 lambda_max, the objective at every layer) and a
ragged shape with perturbed steps. Both sides compute in FP64 from the same
FP32-representable inputs (D, X, lambda, and the same alpha array), so they
differ only in the order of their sums: z^T within 1e-13 of the largest
code, every F trace entry and the loss within 1e-13 relative, and the mean
objective gap within 1e-11 relative (gaps are about 1e-4 of F* at 10x20,
which magnifies a relative gap error; measured 1.5e-16, 6e-16 and 6e-14)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import mean_gap_rel_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sl():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1905_11071_amd as sl
    return sl


def _run(sl, pb, alpha, f_trace=True):
    d = sl.Dictionary(torch.tensor(pb.D32(), device=DEV))
    X = torch.tensor(pb.X, device=DEV, dtype=torch.float64)
    a = torch.tensor(alpha, device=DEV, dtype=torch.float64)
    Z, F, loss = sl.forward_f64(d, X, pb.lam, a, f_trace=f_trace)
    torch.cuda.synchronize()
    out = Z.cpu().numpy(), F.cpu().numpy(), float(loss.item())
    d.close()
    return out


@pytest.mark.parametrize("case", ["ista_10x20", "ragged_37x150"])
def test_f64_forward_matches_oracle(sl, case):
    if case == "ista_10x20":
        c = synth.CONFIGS[case]
        pb = synth.make_problem(c["n"], c["m"], c["N"], c["p"], c["sigma"], c["lam_frac"], c["seed"])
        alpha = np.full(c["T"], 1.0 / oracle.lipschitz(pb.D))
    else:
        pb = synth.make_problem(37, 150, 77, 0.1, 0.01, 0.1, seed=77)
        alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 9, seed=78)
    assert np.array_equal(pb.D, pb.D32().astype(np.float64))
    Zg, Fg, loss = _run(sl, pb, alpha)
    Zo, Fo = oracle.forward(pb.D, pb.X, pb.lam, alpha)
    zerr = np.max(np.abs(Zg - Zo)) / np.max(np.abs(Zo))
    ferr = np.max(np.abs(Fg - Fo) / np.maximum(Fo, 1e-300))
    lerr = abs(loss - np.mean(Fo[-1])) / np.mean(Fo[-1])
    Zs = oracle.lasso_solution(pb.D, pb.X, pb.lam)
    gerr, g_gpu, g_orc = mean_gap_rel_error(pb.D, pb.X, pb.lam, Zg, Zo, Zs)
    _say(f"[{case} fp64] z {zerr:.2e}, F trace {ferr:.2e}, loss {lerr:.2e}, mean-gap rel err {gerr:.2e} "
         f"(gap {g_orc:.3e}, gap/F* {g_orc / np.mean(oracle.objective(pb.D, pb.X, Zs, pb.lam)):.2e})")
    assert Fg.shape == (len(alpha) + 1, pb.N)
    assert zerr <= 1e-13
    assert ferr <= 1e-13
    assert lerr <= 1e-13
    assert gerr <= 1e-11
    # exact zeros stay exact: the support matches the oracle's wherever the
    # oracle's code is not within rounding of the threshold
    assert np.array_equal(Zg[np.abs(Zo) > 1e-9] != 0, Zo[np.abs(Zo) > 1e-9] != 0)


def test_f64_forward_edge_cases(sl):
    pb = synth.make_problem(12, 40, 33, 0.1, 0.0, 0.2, seed=5)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 4, seed=6)
    # T = 0: z = 0 and F = 1/2 ||x||^2
    Zg, Fg, loss = _run(sl, pb, alpha[:0])
    assert not Zg.any()
    np.testing.assert_allclose(Fg[0], 0.5 * np.sum(pb.X ** 2, axis=1), rtol=1e-14)
    # F of z^T only (no trace) equals the trace's last row
    Zt, Ft, _ = _run(sl, pb, alpha, f_trace=True)
    Zn, Fn, _ = _run(sl, pb, alpha, f_trace=False)
    assert np.array_equal(Zt, Zn) and np.array_equal(Ft[-1], Fn)
    # lambda >= lambda_max: every code is exactly zero (Section 2)
    d = sl.Dictionary(torch.tensor(pb.D32(), device=DEV))
    X = torch.tensor(pb.X, device=DEV, dtype=torch.float64)
    a = torch.tensor(alpha, device=DEV, dtype=torch.float64)
    lam_big = float(np.max(oracle.lambda_max(pb.D, pb.X))) * 1.0001
    Z, _, _ = sl.forward_f64(d, X, lam_big, a)
    assert not Z.cpu().numpy().any()
    # N = 0
    Z0, F0, l0 = sl.forward_f64(d, X[:0], pb.lam, a)
    torch.cuda.synchronize()
    assert Z0.shape == (0, pb.m) and l0.item() == 0.0
    # wrong dtype is rejected before any launch
    with pytest.raises(ValueError):
        sl.forward_f64(d, X.float(), pb.lam, a)
    d.close()
