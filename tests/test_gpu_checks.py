"""Device-side checks through the C ABI, against the FP64 oracle and against
what the paper fixes in closed form:

* slista_kkt (FP64 optimality conditions of Lemma 2.1 and the cost of
  Eq. (1) on the device) against the oracle's kkt_residual / objective;
* after a long ISTA run on the device the iterate satisfies Lemma 2.1 to the
  bound the arithmetic allows (a fixed point of the computed layer satisfies
  the optimality conditions up to that layer's rounding error / alpha);
* Lemma 4.2: x = D_j + eps with eps orthogonal to D_j and ||eps|| <
  lam (1 - c) has the solution (1 - lam) e_j, which a long device run reaches;
* slista_lambda_max (Section 2) against the oracle, and lambda at the device
  value giving exact zeros;
* the backward entry point without a prior forward, the non-finite check
  flag, the FP32-tail precision schedule and the one-call batch."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import DALPHA_TOL, GAP_TOL, U16, U32, mean_gap_rel_error

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


def _layer_error_bound(D, X, Z, alpha, prec):
    """Elementwise bound on one computed layer's rounding error at codes Z,
    per sample (max over coordinates): the contraction (Higham's gamma_m for
    FP32 accumulation, plus the rounding of z and of G to BF16 operands in
    BF16 mode, plus G's own rounding to FP32), the correlation c = D^T x
    (gamma_n) and a few elementwise operations."""
    D = np.asarray(D, np.float64)
    X = np.asarray(X, np.float64)
    n, m = D.shape
    absG = np.abs(D.T @ D)
    gz = np.abs(Z) @ absG
    cabs = np.abs(X) @ np.abs(D)
    c = np.abs(X @ D)
    k_prod = (m + 1) * U32 + (2 * U16 if prec == "bf16" else 0.0)
    e = alpha * (k_prod * gz + n * U32 * cabs) + 4 * U32 * (np.abs(Z) + alpha * c)
    return np.max(e, axis=1)


def test_kkt_entry_point_matches_oracle(sl):
    pb = synth.make_problem(48, 200, 300, 0.08, 0.01, 0.1, seed=31)
    rng = np.random.default_rng(2)
    Z = pb.Z0 * rng.uniform(0.5, 1.5, pb.Z0.shape)
    Z = Z.astype(np.float32).astype(np.float64)
    d = sl.Dictionary(_gpu(pb.D))
    kkt, F = sl.kkt(d, _gpu(pb.X), pb.lam, _gpu(Z))
    kkt, F = kkt.cpu().numpy(), F.cpu().numpy()
    ko = oracle.kkt_residual(pb.D, pb.X, Z, np.float64(np.float32(pb.lam)))
    Fo = oracle.objective(pb.D, pb.X, Z, np.float64(np.float32(pb.lam)))
    # both FP64 from the same FP32 values: only the order of the sums differs
    scale = np.max(np.abs(pb.X)) * np.max(np.sum(np.abs(pb.D), axis=1)) + np.max(np.abs(Z)) * 64
    assert np.max(np.abs(kkt - ko)) <= 1e-12 * scale
    np.testing.assert_allclose(F, Fo, rtol=1e-12)
    d.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_long_device_ista_satisfies_lemma_2_1(sl, prec):
    """T = 3000 ISTA layers (alpha = 1/L) on the 64 x 256 Gaussian setting: the
    device's z^T is a fixed point of the computed layer, so the optimality
    conditions hold up to that layer's rounding error divided by alpha."""
    pb = synth.make_problem(64, 256, 512, 0.05, 0.01, 0.1, seed=1002)
    d = sl.Dictionary(_gpu(pb.D))
    L, _ = d.lipschitz(max_iter=200_000, rtol=1e-13)
    a = float(np.float32(1.0 / L))
    T = 3000
    X = _gpu(pb.X)
    Z, _, _, _ = sl.forward(d, X, pb.lam, _gpu(np.full(T, a)), prec=prec, want_f=False, want_loss=False)
    kkt, _ = sl.kkt(d, X, pb.lam, Z)
    Zg = Z.cpu().numpy().astype(np.float64)
    kkt = kkt.cpu().numpy()
    bound = _layer_error_bound(pb.D, pb.X, Zg, a, prec) / a
    _say(f"[{prec}] kkt after {T} layers: max {kkt.max():.3e}, bound {bound.max():.3e}, "
         f"worst ratio {np.max(kkt / bound):.3e}")
    assert np.all(kkt <= bound)
    d.close()


def _lemma42_batch(n=64, m=256, N=96, lam=0.4, shrink=0.5, seed=17):
    """One dictionary, N samples x_i = D_j + eps_i (j = j_i) with eps_i
    orthogonal to D_j and ||eps_i|| = shrink lam (1 - c_j) (Lemma 4.2)."""
    rng = np.random.default_rng(seed)
    D = synth.make_dictionary(rng, n, m)
    G = D.T @ D
    X = np.zeros((N, n))
    js = rng.integers(0, m, N)
    for i, j in enumerate(js):
        dj = D[:, j] / np.linalg.norm(D[:, j])
        c = np.max(np.abs(np.delete(G[:, j], j))) / np.linalg.norm(D[:, j])
        assert c < 1.0
        e = rng.standard_normal(n)
        e -= (e @ dj) * dj
        e *= shrink * lam * (1.0 - c) / np.linalg.norm(e)
        X[i] = D[:, j] + e
    return D, X.astype(np.float32).astype(np.float64), lam, js


def test_long_device_ista_reaches_lemma_4_2_solution(sl):
    D, X, lam, js = _lemma42_batch()
    N, m = X.shape[0], D.shape[1]
    d = sl.Dictionary(_gpu(D))
    L, _ = d.lipschitz(max_iter=200_000, rtol=1e-13)
    T = 2000
    Z, _, _, _ = sl.forward(d, _gpu(X), lam, _gpu(np.full(T, 1.0 / L)), prec="fp32", want_f=False,
                            want_loss=False)
    Zg = Z.cpu().numpy().astype(np.float64)
    # closed form (1 - lam) e_j; for the FP32 inputs the one-atom solution is
    # (D_j^T x - lam) / ||D_j||^2, within ~1e-7 of it
    zj_exact = np.array([(D[:, j] @ X[i] - np.float32(lam)) / (D[:, j] @ D[:, j]) for i, j in enumerate(js)])
    assert np.max(np.abs(zj_exact - (1.0 - lam))) <= 1e-6
    off = Zg.copy()
    off[np.arange(N), js] = 0.0
    assert np.all(off == 0.0), "coordinates off the Lemma 4.2 support must be exactly zero"
    err = np.max(np.abs(Zg[np.arange(N), js] - zj_exact))
    _say(f"Lemma 4.2 on the device: max |z_j - z_j*| = {err:.2e}")
    assert err <= 1e-5
    d.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_lambda_max_on_device(sl, prec):
    pb = synth.make_problem(64, 256, 1000, 0.05, 0.01, 0.1, seed=1002)
    d = sl.Dictionary(_gpu(pb.D))
    X = _gpu(pb.X)
    lm, rows = sl.lambda_max(d, X)
    rows = rows.cpu().numpy().astype(np.float64)
    lo = oracle.lambda_max(pb.D, pb.X)
    # FP32 dot products of length n: |error| <= n u (|D|^T |x|)
    tol = pb.n * U32 * np.max(np.abs(pb.X) @ np.abs(pb.D), axis=1)
    assert np.all(np.abs(rows - lo) <= tol)
    assert lm == float(np.float32(rows.max()))
    # lambda at the device value: every layer exactly zero (Section 2)
    L, _ = d.lipschitz(max_iter=200_000, rtol=1e-12)
    Z, F, loss, da, _ = sl.forward_backward(d, X, lm, _gpu(np.full(5, 1.0 / L)), prec=prec)
    assert np.all(Z.cpu().numpy() == 0.0)
    # just below it some code is non-zero
    Z2, _, _, _, _ = sl.forward_backward(d, X, float(np.float32(lm * 0.999)), _gpu(np.full(5, 1.0 / L)), prec=prec)
    assert np.any(Z2.cpu().numpy() != 0.0)
    d.close()


@pytest.mark.parametrize("name", ["fp32", "bf16", "bf16+tail3"])
def test_backward_without_a_prior_forward(sl, name):
    """slista_backward on a fresh workspace runs the forward itself; on a
    workspace holding another forward's tape (other precision) it does the
    same instead of reading that tape; after a fused call (whose backward has
    recomputed earlier segments into the slots of the last one) it recomputes
    what it needs; all equal the fused call's gradient, also when called
    twice in a row on one tape."""
    prec = {"fp32": "fp32", "bf16": "bf16", "bf16+tail3": sl.bf16_fp32_tail(3)}[name]
    pb = synth.make_problem(40, 160, 777, 0.08, 0.01, 0.1, seed=91)
    T = 9
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=2)
    d = sl.Dictionary(_gpu(pb.D))
    X, a = _gpu(pb.X), _gpu(alpha)
    for k in (1, 3):
        _, _, _, da_ref, ws_fused = sl.forward_backward(d, X, pb.lam, a, prec=prec, ckpt_every=k)
        ws = d.workspace(pb.N, T, prec, k)
        dF = torch.full((pb.N,), 1.0 / pb.N, device=DEV)
        da_fresh = sl.backward(d, X, pb.lam, a, ws, dF=dF, prec=prec, ckpt_every=k)
        da_again = sl.backward(d, X, pb.lam, a, ws, dF=dF, prec=prec, ckpt_every=k)
        other = "fp32" if name != "fp32" else "bf16"
        sl.forward(d, X, pb.lam, a, prec=other, ckpt_every=k, ws=ws)
        da_other = sl.backward(d, X, pb.lam, a, ws, dF=dF, prec=prec, ckpt_every=k)
        # the tape of a matching forward is used as it is
        sl.forward(d, X, pb.lam, a, prec=prec, ckpt_every=k, ws=ws)
        da_tape = sl.backward(d, X, pb.lam, a, ws, dF=dF, prec=prec, ckpt_every=k)
        da_after_fused = sl.backward(d, X, pb.lam, a, ws_fused, dF=dF, prec=prec, ckpt_every=k)
        ref = da_ref.cpu().numpy()
        for got in (da_fresh, da_again, da_other, da_tape, da_after_fused):
            np.testing.assert_allclose(got.cpu().numpy(), ref, rtol=1e-6, atol=1e-12 * np.max(np.abs(ref)))
    d.close()


def test_backward_under_another_kernel_family(sl):
    """A forward under one kernel family leaves its tape in that family's
    layout; a backward under the other family must not read it (the tape
    record includes the family) and recomputes: its gradient equals the fused
    call's of either family."""
    pb = synth.make_problem(40, 160, 333, 0.08, 0.01, 0.1, seed=93)
    T, k = 7, 2
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=4)
    d = sl.Dictionary(_gpu(pb.D))
    X, a = _gpu(pb.X), _gpu(alpha)
    dF = torch.full((pb.N,), 1.0 / pb.N, device=DEV)
    try:
        sl.set_kernel_family("persistent")
        _, _, _, da_ref, _ = sl.forward_backward(d, X, pb.lam, a, prec="fp32", ckpt_every=k)
        ws = d.workspace(pb.N, T, "fp32", k)
        for fwd_fam, bwd_fam in (("persistent", "layer"), ("layer", "persistent")):
            sl.set_kernel_family(fwd_fam)
            sl.forward(d, X, pb.lam, a, prec="fp32", ckpt_every=k, ws=ws)
            sl.set_kernel_family(bwd_fam)
            da = sl.backward(d, X, pb.lam, a, ws, dF=dF, prec="fp32", ckpt_every=k)
            ref = da_ref.cpu().numpy()
            np.testing.assert_allclose(da.cpu().numpy(), ref, rtol=1e-6, atol=1e-12 * np.max(np.abs(ref)))
    finally:
        sl.set_kernel_family("auto")
    d.close()


def test_check_finite_flag(sl):
    pb = synth.make_problem(16, 48, 70, 0.1, 0.0, 0.1, seed=14)
    d = sl.Dictionary(_gpu(pb.D))
    X = pb.X.copy()
    X[3, 2] = np.nan
    a = _gpu(np.full(4, 0.1))
    sl.set_check_finite(True)
    try:
        sl.forward(d, _gpu(pb.X), pb.lam, a)  # finite: passes
        with pytest.raises(sl.SlistaError, match="ENONFINITE"):
            sl.forward(d, _gpu(X), pb.lam, a)
        with pytest.raises(sl.SlistaError, match="ENONFINITE"):
            sl.forward_backward(d, _gpu(X), pb.lam, a)
        Dbad = pb.D.copy()
        Dbad[0, 0] = np.inf
        with pytest.raises(sl.SlistaError, match="ENONFINITE"):
            sl.Dictionary(_gpu(Dbad))
    finally:
        sl.set_check_finite(False)
    # off: no error; the NaN sample's objective is NaN (its codes are not:
    # the soft-threshold maps a NaN argument to 0)
    Z, F, _, _ = sl.forward(d, _gpu(X), pb.lam, a)
    assert np.isnan(F.cpu().numpy()[3]) and np.all(np.isfinite(F.cpu().numpy()[np.arange(pb.N) != 3]))
    d.close()


@pytest.mark.parametrize("family", ["persistent", "layer"])
def test_fp32_tail_schedule(sl, family):
    """BF16 layers followed by an FP32 tail: tail = T is the FP32 network and
    tail = 0 the BF16 one, bit for bit; a mid-network switch gives the same
    bits in both kernel families and with or without checkpoints, its codes
    sit within the FP32 forward bound of the oracle over the tail's start, and
    its step gradient meets the BF16 tolerance."""
    pb = synth.make_problem(50, 200, 1037, 0.08, 0.01, 0.1, seed=77)
    T = 12
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=5)
    d = sl.Dictionary(_gpu(pb.D))
    X, a = _gpu(pb.X), _gpu(alpha)
    sl.set_kernel_family(family)
    try:
        def run(prec, k=1):
            Z, F, loss, da, _ = sl.forward_backward(d, X, pb.lam, a, prec=prec, ckpt_every=k)
            return Z.cpu().numpy(), F.cpu().numpy(), da.cpu().numpy()
        full32, full16 = run("fp32"), run("bf16")
        for x, y in zip(run(sl.bf16_fp32_tail(T)), full32):
            assert np.array_equal(x, y)
        for x, y in zip(run(sl.bf16_fp32_tail(0)), full16):
            assert np.array_equal(x, y)
        mixed = run(sl.bf16_fp32_tail(6))
        for k in (2, 3, 6):
            other = run(sl.bf16_fp32_tail(6), k)
            assert np.array_equal(other[0], mixed[0])
            np.testing.assert_allclose(other[2], mixed[2], rtol=1e-6, atol=1e-12 * np.max(np.abs(mixed[2])))
        with pytest.raises(sl.SlistaError, match="checkpoint"):
            run(sl.bf16_fp32_tail(5), 2)
    finally:
        sl.set_kernel_family("auto")
    _, _, dao = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dF=np.full(pb.N, 1.0 / pb.N))
    err = float(np.max(np.abs(mixed[2] - dao)) / np.max(np.abs(dao)))
    _say(f"[{family}] tail 6 of 12: dalpha rel err {err:.2e}")
    assert err <= DALPHA_TOL["bf16"]
    d.close()


def test_fp32_tail_across_families_bitwise(sl):
    pb = synth.make_problem(64, 256, 900, 0.05, 0.01, 0.1, seed=9)
    T = 10
    alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=8)
    d = sl.Dictionary(_gpu(pb.D))
    X, a = _gpu(pb.X), _gpu(alpha)
    out = {}
    try:
        for fam in ("layer", "persistent"):
            sl.set_kernel_family(fam)
            Z, F, loss, _ = sl.forward(d, X, pb.lam, a, prec=sl.bf16_fp32_tail(4), ckpt_every=0)
            out[fam] = Z.cpu().numpy()
    finally:
        sl.set_kernel_family("auto")
    assert np.array_equal(out["layer"], out["persistent"])
    d.close()


def test_batched_one_call(sl):
    """slista_batched_fwd_bwd (planned once, then replayed) equals the explicit
    batch object, with and without the graph, with and without an FP32 tail."""
    specs = [(32, 128, 300), (50, 200, 1037), (100, 400, 129), (300, 1200, 257), (16, 64, 1000)]
    T = 8
    inputs = []
    for i, (n, m, N) in enumerate(specs):
        pb = synth.make_problem(n, m, N, 0.05, 0.0, 0.1, seed=900 + i)
        dd = sl.Dictionary(_gpu(pb.D))
        inputs.append((dd, _gpu(pb.X), pb.lam, _gpu(synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=i))))
    for prec in ("bf16", sl.bf16_fp32_tail(4)):
        ref = sl.Batch(inputs, prec=prec, ckpt_every=2)
        ref.run()
        one = sl.BatchedCall(inputs, prec=prec, ckpt_every=2)
        for use_graph in (False, True, True):
            for z in one.Z:
                z.zero_()
            one(use_graph=use_graph)
            torch.cuda.synchronize()
            for i in range(len(inputs)):
                assert np.array_equal(one.Z[i].cpu().numpy(), ref.Z[i].cpu().numpy())
                assert np.array_equal(one.dalpha[i].cpu().numpy(), ref.dalpha[i].cpu().numpy())
                assert one.loss[i].item() == ref.loss[i].item()
        ref.close()
    sl.batched_release()
    for dd, _, _, _ in inputs:
        dd.close()
