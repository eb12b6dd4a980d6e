"""Learning the step sizes on the GPU (slista_train through the C ABI): the
backtracking sub-gradient loop of Appendix D against the FP64 oracle's loop
(oracle.train_steps), on the paper's 10 x 20, lambda = 0.2 setting (1000
samples on B_inf, 20 layers) and on the 64 x 256 learned-step workload."""
import sys

import numpy as np
import pytest

import oracle
import synth

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


def _setting(name):
    if name == "fig4_10x20":
        pb = synth.make_binf_problem(10, 20, 1000, 0.2, seed=1101)
        T = 20
    else:
        c = synth.CONFIGS["grad_64x256"]
        pb = synth.make_problem(c["n"], c["m"], c["N"], c["p"], c["sigma"], c["lam_frac"], c["seed"])
        T = c["T"]
    L = oracle.lipschitz(pb.D)
    a0 = np.full(T, np.float32(1.0 / L), dtype=np.float64)
    return pb, a0, L


@pytest.mark.parametrize("name,iters", [("fig4_10x20", 12), ("grad_64x256", 4)])
def test_training_matches_oracle_fp32(sl, name, iters):
    """Same accept/reject sequence, loss trace within 1e-5 and learned steps
    within 1e-4 of the FP64 loop (each step moves alpha by eta * dalpha, and
    dalpha agrees to 1e-5)."""
    pb, a0, L = _setting(name)
    lr = 1.0 / L
    ao, lo, eta_o = oracle.train_steps(pb.D, pb.X, pb.lam, a0, iters, lr=lr)
    d = sl.Dictionary(_gpu(pb.D))
    alpha = _gpu(a0)
    losses, eta = sl.train(d, _gpu(pb.X), pb.lam, alpha, iters, lr, prec="fp32")
    a = alpha.cpu().numpy().astype(np.float64)
    _say(f"[{name}] accepted gpu {len(losses) - 1} oracle {len(lo) - 1}; loss {losses[0]:.6g} -> {losses[-1]:.6g} "
         f"(oracle {lo[-1]:.6g}); max |dalpha_t| / alpha_t {np.max(np.abs(a - ao) / ao):.2e}; eta {eta:.4g} / {eta_o:.4g}")
    assert len(losses) == len(lo)
    assert eta == pytest.approx(eta_o, rel=0, abs=0)
    np.testing.assert_allclose(losses, lo, rtol=1e-5)
    np.testing.assert_allclose(a, ao, rtol=1e-4)
    d.close()


def test_training_bf16_descends_and_learns_larger_steps(sl):
    """BF16 contractions: the accepted losses decrease, the trained network
    beats ISTA (alpha = 1/L), and the late layers learn steps above 1/L, as
    the FP64 loop does (Section 4.1)."""
    pb, a0, L = _setting("fig4_10x20")
    d = sl.Dictionary(_gpu(pb.D))
    alpha = _gpu(a0)
    losses, _ = sl.train(d, _gpu(pb.X), pb.lam, alpha, 60, 1.0 / L, prec="bf16")
    a = alpha.cpu().numpy().astype(np.float64)
    _say(f"[bf16] {len(losses) - 1} accepted, loss {losses[0]:.6g} -> {losses[-1]:.6g}; alpha*L {np.round(a * L, 2)}")
    assert len(losses) > 10
    assert np.all(np.diff(losses) < 0)
    ista = float(np.mean(oracle.forward(pb.D, pb.X, pb.lam, a0)[1][-1]))
    trained = float(np.mean(oracle.forward(pb.D, pb.X, pb.lam, a)[1][-1]))
    assert trained < ista
    assert np.all(a[len(a) // 2:] > 1.0 / L)
    d.close()


def test_training_rejects_bad_arguments(sl):
    pb, a0, L = _setting("fig4_10x20")
    d = sl.Dictionary(_gpu(pb.D))
    with pytest.raises(sl.SlistaError):
        sl.train(d, _gpu(pb.X), pb.lam, _gpu(a0), 3, -1.0)
    with pytest.raises(sl.SlistaError):
        sl.train(d, _gpu(pb.X), pb.lam, _gpu(a0), 3, 1.0, max_halvings=-1)
    d.close()
