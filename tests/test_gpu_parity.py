"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on the
same seeded inputs. Runs on an MI355X only."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import DALPHA_TOL, GAP_TOL, mean_gap_rel_error, z_tolerance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sl():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1905_11071_amd as sl
    return sl


DEV = "cuda:0"


def _gpu(a, dtype=np.float32):
    return torch.tensor(np.ascontiguousarray(a, dtype=dtype), device=DEV)


def _run_forward(sl, pb, alpha, prec, f_trace=False, ckpt_every=0):
    d = sl.Dictionary(_gpu(pb.D))
    Z, F, loss, _ = sl.forward(d, _gpu(pb.X), pb.lam, _gpu(alpha), prec=prec, f_trace=f_trace,
                               ckpt_every=ckpt_every)
    torch.cuda.synchronize()
    out = Z.cpu().numpy().astype(np.float64), F.cpu().numpy().astype(np.float64), float(loss.item())
    d.close()
    return out


def test_single_hip_runtime(sl):
    sl.Dictionary(_gpu(np.eye(4, 8)))
    maps = open("/proc/self/maps").read()
    paths = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(paths) == 1, paths


def test_gram_and_lipschitz(sl):
    pb = synth.make_problem(64, 256, 4, 0.05, 0.0, 0.1, seed=1003)
    d = sl.Dictionary(_gpu(pb.D))
    G = d.gram().cpu().numpy().astype(np.float64)
    Go = pb.D.T @ pb.D
    # FP64 accumulation, one rounding to FP32: |error| <= u |G|
    assert np.max(np.abs(G - Go)) <= 2.0 ** -24 * np.max(np.abs(Go)) * 1.0001
    L, it = d.lipschitz(max_iter=200_000, rtol=1e-14)
    _say(f"L gpu={L!r} iters={it} oracle={oracle.lipschitz(pb.D)!r}")
    import scipy.linalg
    L_same = scipy.linalg.eigvalsh(G)[-1]   # same FP32 G widened to FP64
    assert abs(L - L_same) <= 1e-8 * L_same
    assert abs(L - oracle.lipschitz(pb.D)) <= 1e-6 * L
    d.close()


@pytest.mark.parametrize("prec", ["fp32"])
def test_forward_ista_10x20_trace(sl, prec):
    """Plain ISTA on the 10x20 dictionary, N=1000, T=100, alpha = 1/L, with the
    per-iteration objective trace. This workload is specified in FP64; the
    device computes it in FP32 and is held to the FP32 tolerances (BF16
    operands are specified for the 256x1024 precision workload, not here)."""
    cfg = synth.CONFIGS["ista_10x20"]
    pb = synth.make_problem(cfg["n"], cfg["m"], cfg["N"], cfg["p"], cfg["sigma"], cfg["lam_frac"], cfg["seed"])
    T = cfg["T"]
    alpha = np.full(T, np.float32(1.0 / oracle.lipschitz(pb.D)), dtype=np.float64)
    Zg, Fg, loss = _run_forward(sl, pb, alpha, prec, f_trace=True)
    Zo, Fo, its = oracle.forward(pb.D, pb.X, pb.lam, alpha, return_iterates=True)
    zs = oracle.lasso_solution(pb.D, pb.X, pb.lam)
    rel, gg, go = mean_gap_rel_error(pb.D, pb.X, pb.lam, Zg, Zo, zs)
    _say(f"[{prec}] 10x20 gap gpu={gg:.3e} oracle={go:.3e} rel={rel:.2e} max|dZ|={np.max(np.abs(Zg - Zo)):.2e}")
    assert rel <= GAP_TOL[prec]
    assert Fg.shape == (T + 1, pb.N)
    # trace row 0 is 1/2||x||^2 exactly up to the FP32 output rounding
    np.testing.assert_allclose(Fg[0], Fo[0], rtol=1e-6)
    if prec == "fp32":
        tol = z_tolerance(pb.D, pb.X, alpha, its)
        assert np.max(np.abs(Zg - Zo)) <= tol
        # in-kernel objective (FP32, Gram form): monitoring accuracy
        np.testing.assert_allclose(Fg, Fo, rtol=1e-4, atol=1e-5 * np.max(Fo))
        assert abs(loss - np.mean(Fo[-1])) <= 1e-5 * np.mean(Fo[-1])


def test_forward_ragged_shapes_fp32(sl):
    """m not a multiple of 64, n not a multiple of 4, N not a multiple of 128."""
    pb = synth.make_problem(50, 200, 1037, 0.1, 0.01, 0.1, seed=77)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 15, seed=3)
    Zg, Fg, _ = _run_forward(sl, pb, alpha, "fp32")
    Zo, Fo, its = oracle.forward(pb.D, pb.X, pb.lam, alpha, return_iterates=True)
    err = float(np.max(np.abs(Zg - Zo)))
    tol = z_tolerance(pb.D, pb.X, alpha, its)
    _say(f"ragged max|dZ|={err:.2e} tol={tol:.2e}")
    assert err <= tol
    np.testing.assert_allclose(Fg, Fo[-1], rtol=1e-4)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_forward_64x256_full_batch(sl, prec):
    """Batched forward at its full size (N=10000, T=40, alpha = 1/L); the
    oracle checks every 10th sample (samples are independent)."""
    cfg = synth.CONFIGS["fwd_64x256"]
    pb = synth.make_problem(cfg["n"], cfg["m"], cfg["N"], cfg["p"], cfg["sigma"], cfg["lam_frac"], cfg["seed"])
    T = cfg["T"]
    alpha = np.full(T, np.float32(1.0 / oracle.lipschitz(pb.D)), dtype=np.float64)
    Zg, Fg, _ = _run_forward(sl, pb, alpha, prec)
    idx = np.arange(0, pb.N, 10)
    Xs = pb.X[idx]
    Zo, Fo, its = oracle.forward(pb.D, Xs, pb.lam, alpha, return_iterates=True)
    zs = oracle.lasso_solution(pb.D, Xs, pb.lam)
    rel, gg, go = mean_gap_rel_error(pb.D, Xs, pb.lam, Zg[idx], Zo, zs)
    _say(f"[{prec}] 64x256 gap gpu={gg:.3e} oracle={go:.3e} rel={rel:.2e} max|dZ|={np.max(np.abs(Zg[idx] - Zo)):.2e}")
    assert rel <= GAP_TOL[prec]
    if prec == "fp32":
        assert np.max(np.abs(Zg[idx] - Zo)) <= z_tolerance(pb.D, Xs, alpha, its)


def _grad_problem():
    cfg = synth.CONFIGS["grad_64x256"]
    pb = synth.make_problem(cfg["n"], cfg["m"], cfg["N"], cfg["p"], cfg["sigma"], cfg["lam_frac"], cfg["seed"])
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), cfg["T"], seed=11)
    return pb, alpha


@pytest.fixture(scope="module")
def grad_reference():
    pb, alpha = _grad_problem()
    Zo, Fo, dao = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dF=np.full(pb.N, 1.0 / pb.N))
    return pb, alpha, Zo, Fo, dao


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_dalpha_64x256(sl, grad_reference, prec):
    """d(mean F)/d alpha_t through T=20 learned-step layers, N=4096."""
    pb, alpha, Zo, Fo, dao = grad_reference
    d = sl.Dictionary(_gpu(pb.D))
    Z, F, loss, da, _ = sl.forward_backward(d, _gpu(pb.X), pb.lam, _gpu(alpha), prec=prec, ckpt_every=1)
    torch.cuda.synchronize()
    da = da.cpu().numpy().astype(np.float64)
    err = float(np.max(np.abs(da - dao)) / np.max(np.abs(dao)))
    lerr = abs(loss.item() - np.mean(Fo[-1])) / np.mean(Fo[-1])
    _say(f"[{prec}] dalpha rel err={err:.2e} loss rel err={lerr:.2e}")
    assert err <= DALPHA_TOL[prec]
    if prec == "fp32":
        assert lerr <= 1e-5
    d.close()


def test_dalpha_with_upstream_dz_and_weights(sl):
    pb = synth.make_problem(40, 160, 777, 0.08, 0.01, 0.1, seed=91)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 9, seed=2)
    rng = np.random.default_rng(0)
    dZ = rng.standard_normal((pb.N, pb.m)).astype(np.float32).astype(np.float64)
    dF = rng.uniform(0.0, 2.0, pb.N).astype(np.float32).astype(np.float64)
    _, _, dao = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dZ=dZ, dF=dF)
    d = sl.Dictionary(_gpu(pb.D))
    X, a = _gpu(pb.X), _gpu(alpha)
    _, _, _, ws = sl.forward(d, X, pb.lam, a, ckpt_every=1)
    da = sl.backward(d, X, pb.lam, a, ws, dZ=_gpu(dZ), dF=_gpu(dF), ckpt_every=1).cpu().numpy()
    err = float(np.max(np.abs(da - dao)) / np.max(np.abs(dao)))
    _say(f"dZ+dF dalpha rel err={err:.2e}")
    assert err <= DALPHA_TOL["fp32"]
    d.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_checkpointing_is_bitwise_neutral(sl, prec):
    pb = synth.make_problem(32, 128, 900, 0.08, 0.01, 0.1, seed=5)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 13, seed=6)
    d = sl.Dictionary(_gpu(pb.D))
    X, a = _gpu(pb.X), _gpu(alpha)
    outs = []
    for k in (1, 2, 5, 13, 40):
        Z, F, loss, da, _ = sl.forward_backward(d, X, pb.lam, a, prec=prec, ckpt_every=k)
        outs.append((Z.cpu().numpy(), F.cpu().numpy(), da.cpu().numpy()))
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x, y)
    d.close()


def test_run_to_run_determinism(sl):
    pb = synth.make_problem(64, 256, 3000, 0.05, 0.01, 0.1, seed=8)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 10, seed=7)
    d = sl.Dictionary(_gpu(pb.D))
    X, a = _gpu(pb.X), _gpu(alpha)
    r1 = [t.cpu().numpy() for t in sl.forward_backward(d, X, pb.lam, a, prec="bf16")[:4]]
    r2 = [t.cpu().numpy() for t in sl.forward_backward(d, X, pb.lam, a, prec="bf16")[:4]]
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)
    d.close()


def test_autograd_function_matches_fused_call(sl):
    pb = synth.make_problem(32, 128, 500, 0.08, 0.01, 0.1, seed=12)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 7, seed=1)
    d = sl.Dictionary(_gpu(pb.D))
    X = _gpu(pb.X)
    a = _gpu(alpha).requires_grad_(True)
    Z, F = sl.slista(a, d, X, pb.lam, "fp32", 1)
    F.mean().backward()
    _, _, _, da, _ = sl.forward_backward(d, X, pb.lam, a.detach(), prec="fp32")
    np.testing.assert_allclose(a.grad.cpu().numpy(), da.cpu().numpy(), rtol=1e-6, atol=1e-9)
    d.close()


def test_finite_difference_on_gpu_forward(sl, grad_reference):
    """Central differences (h = 1e-4) of the GPU FP32 forward's loss against
    the adjoint, on the learned-step workload (64 x 256, N = 4096, T = 20,
    perturbed steps). The loss of each perturbed forward is evaluated in FP64
    on the device (slista_kkt's objective) from the FP32 codes, so the
    difference quotient is not limited by an FP32 loss value."""
    pb, alpha, _, _, dao = grad_reference
    d = sl.Dictionary(_gpu(pb.D))
    X = _gpu(pb.X)
    _, _, _, da, _ = sl.forward_backward(d, X, pb.lam, _gpu(alpha))
    da = da.cpu().numpy()
    h = 1e-4
    fd = np.zeros_like(alpha)
    for t in range(len(alpha)):
        vals = []
        for s in (+1, -1):
            a2 = alpha.copy()
            a2[t] += s * h
            Z, _, _, _ = sl.forward(d, X, pb.lam, _gpu(a2), want_f=False, want_loss=False)
            _, F = sl.kkt(d, X, pb.lam, Z)
            vals.append(float(F.mean().item()))
        fd[t] = (vals[0] - vals[1]) / (2 * h)
    err = float(np.max(np.abs(fd - da)) / np.max(np.abs(da)))
    err_o = float(np.max(np.abs(fd - dao)) / np.max(np.abs(dao)))
    _say(f"gpu FD vs adjoint rel err={err:.2e}, vs oracle gradient {err_o:.2e}")
    assert err <= 5e-3 and err_o <= 5e-3
    d.close()


def test_edge_cases(sl):
    pb = synth.make_problem(16, 48, 70, 0.1, 0.0, 0.1, seed=14)
    d = sl.Dictionary(_gpu(pb.D))
    X = _gpu(pb.X)
    L = oracle.lipschitz(pb.D)
    # T = 0: z = 0, F = 1/2 ||x||^2
    Z, F, loss, _ = sl.forward(d, X, pb.lam, _gpu(np.zeros(0)))
    assert np.all(Z.cpu().numpy() == 0)
    np.testing.assert_allclose(F.cpu().numpy(), 0.5 * np.sum(pb.X ** 2, axis=1), rtol=1e-6)
    # T = 1 forward + backward vs oracle
    a1 = np.array([np.float32(0.8 / L)], dtype=np.float64)
    Z, F, loss, da, _ = sl.forward_backward(d, X, pb.lam, _gpu(a1))
    Zo, Fo, dao = oracle.forward_backward(pb.D, pb.X, pb.lam, a1, dF=np.full(pb.N, 1.0 / pb.N))
    np.testing.assert_allclose(Z.cpu().numpy(), Zo, atol=1e-6)
    np.testing.assert_allclose(da.cpu().numpy(), dao, rtol=1e-5)
    # lambda >= lambda_max: every layer exactly zero
    lam_big = float(np.max(oracle.lambda_max(pb.D, pb.X))) * 1.0001
    Z, F, loss, da, _ = sl.forward_backward(d, X, lam_big, _gpu(np.full(5, 1.0 / L)))
    assert np.all(Z.cpu().numpy() == 0)
    # N = 0
    Z, F, loss, da, _ = sl.forward_backward(d, _gpu(np.zeros((0, 16))), pb.lam, _gpu(np.full(3, 1.0 / L)))
    assert Z.shape == (0, 48) and np.all(da.cpu().numpy() == 0)
    d.close()


def test_error_paths_reach_no_kernel(sl):
    pb = synth.make_problem(16, 48, 70, 0.1, 0.0, 0.1, seed=15)
    d = sl.Dictionary(_gpu(pb.D))
    X = _gpu(pb.X)
    a = _gpu(np.full(4, 0.1))
    with pytest.raises(sl.SlistaError, match="EINVAL"):
        sl.forward(d, X, -1.0, a)
    with pytest.raises(sl.SlistaError, match="EINVAL"):
        sl.forward(d, X, float("nan"), a)
    small = torch.empty(256, dtype=torch.uint8, device=DEV)
    with pytest.raises(sl.SlistaError, match="workspace"):
        sl.forward(d, X, 0.1, a, ws=small)
    with pytest.raises(sl.SlistaError, match="EINVAL"):
        sl.backward(d, X, 0.1, a, d.workspace(70, 4, "fp32", 1), ckpt_every=1)
    d.close()


@pytest.fixture(scope="module")
def full_prec_problem():
    cfg = synth.CONFIGS["prec_256x1024"]
    pb = synth.make_problem(cfg["n"], cfg["m"], cfg["N"], cfg["p"], cfg["sigma"], cfg["lam_frac"], cfg["seed"])
    rows = np.arange(0, pb.N, 256)      # 256 sampled rows, the same on both sides
    return pb, cfg["T"], rows


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_full_size_256x1024(sl, full_prec_problem, prec):
    """The benchmark's workload and launch configuration (N=65536, m=1024,
    T=50, fused forward+backward, every iterate kept): sampled rows of z^(T)
    against the oracle run on those rows alone (samples are independent), and
    d alpha of the loss restricted to those rows (dF = 1/256 on them, 0
    elsewhere) against the oracle's."""
    pb, T, rows = full_prec_problem
    _say(f"[{prec}] full size N={pb.N} m={pb.m} T={T}")
    d = sl.Dictionary(_gpu(pb.D))
    L, _ = d.lipschitz(max_iter=200_000, rtol=1e-13)
    alpha = np.full(T, np.float32(1.0 / L), dtype=np.float64)
    X, a = _gpu(pb.X), _gpu(alpha)
    Z, F, loss, _, ws = sl.forward_backward(d, X, pb.lam, a, prec=prec, ckpt_every=1)
    dF = np.zeros(pb.N)
    dF[rows] = 1.0 / len(rows)
    da = sl.backward(d, X, pb.lam, a, ws, dF=_gpu(dF), prec=prec, ckpt_every=1)
    torch.cuda.synchronize()
    Zg = Z.cpu().numpy().astype(np.float64)[rows]
    da = da.cpu().numpy().astype(np.float64)
    del ws
    d.close()
    Xs = pb.X[rows]
    Zo, Fo, dao = oracle.forward_backward(pb.D, Xs, pb.lam, alpha, dF=np.full(len(rows), 1.0 / len(rows)))
    zs = oracle.lasso_solution(pb.D, Xs, pb.lam)
    rel, gg, go = mean_gap_rel_error(pb.D, Xs, pb.lam, Zg, Zo, zs)
    derr = float(np.max(np.abs(da - dao)) / np.max(np.abs(dao)))
    # per sample: the objective of the device codes against the oracle's codes
    Fs = oracle.objective(pb.D, Xs, zs, pb.lam)
    Fg, Foz = oracle.objective(pb.D, Xs, Zg, pb.lam), oracle.objective(pb.D, Xs, Zo, pb.lam)
    per_F = np.abs(Fg - Foz) / Foz
    per_gap = np.abs(Fg - Foz) / np.maximum(Foz - Fs, 1e-300)
    _say(f"[{prec}] 256x1024 gap gpu={gg:.4e} oracle={go:.4e} rel={rel:.2e} dalpha rel={derr:.2e} "
         f"max|dZ|={np.max(np.abs(Zg - Zo)):.2e}; per sample |dF|/F max {per_F.max():.2e}, "
         f"|dF|/gap median {np.median(per_gap):.2e} max {per_gap.max():.2e}")
    assert rel <= GAP_TOL[prec]
    assert derr <= DALPHA_TOL[prec]
    if prec == "fp32":
        # every code of every sampled row within the FP32 forward-error bound
        _, _, its = oracle.forward(pb.D, Xs, pb.lam, alpha, return_iterates=True)
        tol = z_tolerance(pb.D, Xs, alpha, its)
        _say(f"[fp32] 256x1024 max|dZ| / bound = {np.max(np.abs(Zg - Zo)) / tol:.2e}")
        assert np.max(np.abs(Zg - Zo)) <= tol
        assert per_F.max() <= 1e-5
    else:
        # each sample's objective: within the BF16 bar relative to its own gap
        # for the typical sample, and within 1e-3 of F for every sample (no
        # elementwise bound exists for BF16 operands: the worst-case forward
        # error bound exceeds the codes themselves)
        assert np.median(per_gap) <= GAP_TOL["bf16"]
        assert per_F.max() <= 1e-3


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
# N covers every remainder mod 4 (the persistent kernels keep the tape and c
# in four-row groups; the last group of a ragged N is part padding)
# m = 600 (m_pad 640): the four-pass kernels with the last pass partly past m_pad
@pytest.mark.parametrize("shape", [(50, 200, 1037, 9), (64, 256, 3000, 12), (80, 448, 515, 6), (96, 1024, 702, 7),
                                   (40, 600, 333, 5), (40, 1100, 300, 5)])
def test_kernel_families_agree(sl, prec, shape):
    """The persistent kernels (a workgroup carries a sample tile through all
    layers; four tile variants) and the per-layer kernels use the same K
    order and epilogue arithmetic: z^(T) is bitwise identical; dalpha differs
    only by the grouping of its FP64 partial sums."""
    n, m, N, T = shape
    pb = synth.make_problem(n, m, N, 0.08, 0.01, 0.1, seed=300 + m)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=4)
    d = sl.Dictionary(_gpu(pb.D))
    X, a = _gpu(pb.X), _gpu(alpha)
    res = {}
    try:
        for fam, variants in (("layer", (0,)), ("persistent", (1, 2, 3, 4))):
            sl.set_kernel_family(fam)
            for v in variants:
                sl.set_tile_variant(v)
                for k in (1, 3):
                    Z, F, loss, da, _ = sl.forward_backward(d, X, pb.lam, a, prec=prec, ckpt_every=k)
                    res[(fam, v, k)] = (Z.cpu().numpy(), F.cpu().numpy(), da.cpu().numpy())
    finally:
        sl.set_kernel_family("auto")
        sl.set_tile_variant(0)
    ref = res[("layer", 0, 1)]
    for key, (Z, F, da) in res.items():
        assert np.array_equal(Z, ref[0]), key
        np.testing.assert_allclose(da, ref[2], rtol=1e-6, atol=1e-12 * np.max(np.abs(ref[2])))
        np.testing.assert_allclose(F, ref[1], rtol=1e-5)
    d.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_wide_dictionary_on_the_per_layer_kernels(sl, prec):
    """m_pad > 2048 (n = 40, m = 2600): past the persistent kernels' column
    passes the layers run on the per-layer kernels. Codes (FP32: within the
    forward-error bound), the mean gap and d alpha against the oracle."""
    pb = synth.make_problem(40, 2600, 150, 0.02, 0.01, 0.1, seed=2600)
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), 5, seed=2601)
    d = sl.Dictionary(_gpu(pb.D))
    Z, F, loss, da, _ = sl.forward_backward(d, _gpu(pb.X), pb.lam, _gpu(alpha), prec=prec, ckpt_every=2)
    torch.cuda.synchronize()
    Zg, da = Z.cpu().numpy().astype(np.float64), da.cpu().numpy().astype(np.float64)
    d.close()
    Zo, Fo, dao, its, _ = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dF=np.full(pb.N, 1.0 / pb.N),
                                                 return_adjoints=True)
    zs = oracle.lasso_solution(pb.D, pb.X, pb.lam)
    rel, gg, go = mean_gap_rel_error(pb.D, pb.X, pb.lam, Zg, Zo, zs)
    err = float(np.max(np.abs(da - dao)) / np.max(np.abs(dao)))
    zerr = float(np.max(np.abs(Zg - Zo)))
    _say(f"[{prec}] 40x2600: mean-gap rel err {rel:.2e}, dalpha rel err {err:.2e}, max|dZ| {zerr:.2e}")
    assert rel <= GAP_TOL[prec]
    assert err <= DALPHA_TOL[prec]
    if prec == "fp32":
        assert zerr <= z_tolerance(pb.D, pb.X, alpha, its)


def test_objective_entry_point(sl):
    """slista_objective evaluates Eq. (1) for given codes; compared with the
    oracle's FP64 objective on sparse and dense codes (FP32 residual: the
    relative error is a few units of 2^-24 times the cancellation factor)."""
    pb = synth.make_problem(64, 256, 777, 0.05, 0.01, 0.1, seed=19)
    d = sl.Dictionary(_gpu(pb.D))
    rng = np.random.default_rng(3)
    for Z in (pb.Z0, rng.standard_normal((pb.N, pb.m)) * (rng.random((pb.N, pb.m)) < 0.3)):
        Z = Z.astype(np.float32).astype(np.float64)
        Fg = sl.objective(d, _gpu(pb.X), pb.lam, _gpu(Z)).cpu().numpy()
        Fo = oracle.objective(pb.D, pb.X, Z, pb.lam)
        np.testing.assert_allclose(Fg, Fo, rtol=2e-5, atol=1e-6)
    d.close()


def test_autotune_keeps_results(sl, tmp_path):
    """The autotuner times every tile variant on the problem and makes the
    fastest the default for its class; the variants compute the same bits,
    so results before and after tuning agree exactly. The tuning table
    survives a save / load round trip."""
    pb = synth.make_problem(64, 256, 3000, 0.05, 0.01, 0.1, seed=23)
    T = 6
    alpha = _gpu(synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=4))
    d = sl.Dictionary(_gpu(pb.D))
    X = _gpu(pb.X)
    for prec in ("bf16", "fp32"):
        Z0, F0, l0, da0, _ = sl.forward_backward(d, X, pb.lam, alpha, prec=prec)
        best, ms = sl.autotune(d, X, pb.lam, alpha, prec=prec)
        _say(f"{prec}: best variant {best}, ms by variant {ms}")
        assert best in (1, 2, 3, 4)
        timed = [x for x in ms if x > 0]
        assert len(timed) >= 2 and ms[best - 1] == min(timed)
        Z1, F1, l1, da1, _ = sl.forward_backward(d, X, pb.lam, alpha, prec=prec)
        assert np.array_equal(Z0.cpu().numpy(), Z1.cpu().numpy())
        assert np.array_equal(da0.cpu().numpy(), da1.cpu().numpy())
        assert l0.item() == l1.item()
    path = str(tmp_path / "tune.txt")
    sl.tune_save(path)
    recs = [list(map(int, ln.split())) for ln in open(path).read().splitlines() if ln.strip()]
    assert any(r[0] == 1 and r[1] == 1 and r[2] == 11 for r in recs), recs  # bf16, one pass, log2(3000)
    sl.tune_load(path)
    d.close()


def test_checkpoint_spacing_for_a_memory_budget(sl):
    """slista_ckpt_for_budget picks the smallest spacing whose workspace fits;
    the autograd node's "auto" mode uses it and gives the same gradient as
    keeping every layer (checkpointing is bitwise neutral on the codes)."""
    pb = synth.make_problem(32, 128, 700, 0.08, 0.01, 0.1, seed=14)
    T = 24
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=3)
    d = sl.Dictionary(_gpu(pb.D))
    full = d.workspace_bytes(pb.N, T, "fp32", 1)
    assert d.ckpt_for_budget(pb.N, T, "fp32", budget=full) == 1
    sizes = {k: d.workspace_bytes(pb.N, T, "fp32", k) for k in range(1, T + 1)}
    budget = (full + min(sizes.values())) // 2
    k = d.ckpt_for_budget(pb.N, T, "fp32", budget=budget)
    assert sizes[k] <= budget and all(sizes[j] > budget for j in range(1, k))
    with pytest.raises(sl.SlistaError):
        d.ckpt_for_budget(pb.N, T, "fp32", budget=min(sizes.values()) - 1)
    X = _gpu(pb.X)
    a = _gpu(alpha).requires_grad_(True)
    Z, F = sl.slista(a, d, X, pb.lam, "fp32", "auto")
    F.mean().backward()
    _, _, _, da, _ = sl.forward_backward(d, X, pb.lam, a.detach(), prec="fp32", ckpt_every=1)
    np.testing.assert_allclose(a.grad.cpu().numpy(), da.cpu().numpy(), rtol=1e-6, atol=1e-9)
    d.close()
