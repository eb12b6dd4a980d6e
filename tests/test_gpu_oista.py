"""Oracle-ISTA (slista_oista) against the FP64 oracle's Algorithm 1: the
step each sample takes at each layer (1/L_S or 1/L), the objective gap of
z^T, and the speed-up over ISTA the paper reports (Fig. 2 setting)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import GAP_TOL

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


def _gpu(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device=DEV)


def _case(name):
    if name == "fig2_10x50":
        return synth.make_binf_problem(10, 50, 200, 0.5, seed=1201), 40
    return synth.make_problem(64, 256, 600, 0.05, 0.01, 0.1, seed=1202), 25


# The 10 x 50 setting of Fig. 2 converges to a gap of 3e-5 of F* within its
# layers, which BF16 operands cannot resolve (their rounding moves the mean gap
# by about 2e-2 there); it is checked in FP32, and the BF16 path on the 64 x 256
# setting, whose gap the 2e-2 bar resolves.
@pytest.mark.parametrize("name,prec", [("fig2_10x50", "fp32"), ("gauss_64x256", "fp32"), ("gauss_64x256", "bf16")])
def test_oista_vs_oracle(sl, name, prec):
    pb, T = _case(name)
    L = oracle.lipschitz(pb.D)
    d = sl.Dictionary(_gpu(pb.D))
    Lg, _ = d.lipschitz(max_iter=200_000, rtol=1e-14)
    Z, F, loss, steps = sl.oista(d, _gpu(pb.X), pb.lam, Lg, T, prec=prec)
    torch.cuda.synchronize()
    Zg = Z.cpu().numpy().astype(np.float64)
    sg = steps.cpu().numpy().astype(np.float64)
    Zo, Fo, so = oracle.oista(pb.D, pb.X, pb.lam, T, return_steps=True)
    # the branch each sample took at each layer: the same step up to the FP32 accuracy of G
    same = np.isclose(sg, so, rtol=1e-4)
    frac = float(np.mean(same))
    # where both took 1/L_S, the device's L_S (Lanczos on the FP32 Gram matrix) against LAPACK's
    ls = same & (so > 1.0001 / L)
    ls_err = float(np.max(np.abs(sg[ls] - so[ls]) / so[ls])) if ls.any() else 0.0
    zs = oracle.lasso_solution(pb.D, pb.X, pb.lam)
    Fs = oracle.objective(pb.D, pb.X, zs, pb.lam)
    g_gpu = float(np.mean(oracle.objective(pb.D, pb.X, Zg, pb.lam) - Fs))
    g_orc = float(np.mean(Fo[-1] - Fs))
    rel = abs(g_gpu - g_orc) / g_orc
    tol = GAP_TOL[prec]
    _say(f"[{name} {prec}] steps agreeing {frac:.4f}, larger than 1/L {np.mean(so > 1.0001 / L):.3f}, "
         f"1/L_S rel err {ls_err:.2e}; mean-gap rel err {rel:.2e} (tolerance {tol:.2e}), "
         f"gap/F* {g_orc / np.mean(Fs):.2e}")
    # FP32 follows the oracle's trajectory, so it takes the same branch; BF16
    # contractions move the trajectory (and with it the supports), so there
    # the agreement is only a sanity bound and the gap carries the claim
    assert frac >= (0.999 if prec == "fp32" else 0.9)
    if prec == "fp32":  # the FP32 Gram matrix moves L_S by a few units of FP32 rounding
        assert ls_err <= 1e-5
    assert rel <= tol
    np.testing.assert_allclose(F.cpu().numpy(), oracle.objective(pb.D, pb.X, Zg, pb.lam),
                               rtol=1e-4 if prec == "fp32" else 2e-2)
    d.close()


def test_oista_beats_ista(sl):
    """Fig. 2: at the same number of layers Oracle-ISTA is much closer to F*."""
    pb, T = _case("fig2_10x50")
    d = sl.Dictionary(_gpu(pb.D))
    Lg, _ = d.lipschitz(max_iter=200_000, rtol=1e-14)
    X = _gpu(pb.X)
    _, _, lo, _ = sl.oista(d, X, pb.lam, Lg, T)
    _, _, li, _ = sl.forward(d, X, pb.lam, _gpu(np.full(T, np.float32(1.0 / Lg))))
    zs = oracle.lasso_solution(pb.D, pb.X, pb.lam)
    fs = float(np.mean(oracle.objective(pb.D, pb.X, zs, pb.lam)))
    _say(f"T={T}: OISTA gap {lo.item() - fs:.3e}, ISTA gap {li.item() - fs:.3e}")
    assert lo.item() - fs < 0.1 * (li.item() - fs)
    d.close()
