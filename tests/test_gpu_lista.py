"""Coupled LISTA (slista_lista_* through the C ABI) against the FP64 oracle
(oracle.lista_forward_backward): z^(T), F(z^(T)), the mean loss of Eq. (15)
and its gradient in every layer's (W_t, alpha_t, beta_t), on the paper's
Fig. 5 setting (10 x 20, lambda = 0.05, 1000 samples on B_inf, 40 layers),
the 64 x 256 Gaussian workload and a shape with ragged n, m and N."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"

# FP32: every layer rounds z, the residual and W^T r once (unit roundoff
# 6e-8); over 40 layers and through the adjoint's sums the relative error
# measured on MI355X stays at or below 7e-7, so the FP32 bar of 1e-5 holds
# for the iterates and the gradients as for the objective. BF16: the loss,
# z^T and the step gradients d alpha, d beta are held to the BF16 bar of 2e-2
# (relative to their largest entry; measured <= 4.2e-3). dW is held to its
# direction (cosine >= 0.995, measured >= 0.9989): an entry of dW sums
# R_i v_j over the samples whose support holds atom j, and BF16 operands move
# those supports, so single entries differ by up to 0.14 of the largest one
# while the matrix keeps its direction and scale.
Z_TOL_FP32 = 1e-5
GRAD_TOL_FP32 = 1e-5
LOSS_TOL = {"fp32": 1e-5, "bf16": 2e-2}
BF16_TOL = 2e-2
DW_COS_BF16 = 0.995


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


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _params(pb, T, seed, spread):
    """FP32 parameters near the ISTA point, so both sides see the same values."""
    return synth.lista_params(pb.D, oracle.lipschitz(pb.D), T, seed, spread)


def _case(name):
    if name == "fig5_10x20":
        pb = synth.make_binf_problem(10, 20, 1000, 0.05, seed=1301)
        return pb, 40, 0.1
    if name == "gauss_64x256":
        return synth.make_problem(64, 256, 2000, 0.05, 0.01, 0.1, seed=1302), 20, 0.2
    return synth.make_problem(37, 150, 333, 0.1, 0.01, 0.1, seed=1303), 7, 0.3


_REF = {}


def _reference(name):
    if name not in _REF:
        pb, T, spread = _case(name)
        W, a, b = _params(pb, T, 7, spread)
        out = oracle.lista_forward_backward(pb.D, pb.X, pb.lam, W, a, b, dF=np.full(pb.N, 1.0 / pb.N))
        _REF[name] = (pb, W, a, b) + tuple(out)
    return _REF[name]


def _rel(x, ref):
    return float(np.max(np.abs(np.asarray(x, np.float64) - ref)) / np.max(np.abs(ref)))


def _cos(x, ref):
    x = np.asarray(x, np.float64).ravel()
    ref = ref.ravel()
    return float(x @ ref / (np.linalg.norm(x) * np.linalg.norm(ref)))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["fig5_10x20", "gauss_64x256", "ragged_37x150"])
def test_lista_forward_backward_vs_oracle(sl, name, prec):
    pb, W, a, b, Zo, Fo, dWo, dao, dbo = _reference(name)
    d = sl.Dictionary(_gpu(pb.D))
    Z, F, loss, dW, da, db, _ = sl.lista_forward_backward(d, _gpu(pb.X), pb.lam, _gpu(W), _gpu(a), _gpu(b),
                                                          prec=prec)
    torch.cuda.synchronize()
    Zg = Z.cpu().numpy().astype(np.float64)
    lo = float(np.mean(Fo[-1]))
    lerr = abs(loss.item() - lo) / lo
    zerr = _rel(Zg, Zo)
    errs = {k: _rel(v.cpu().numpy(), r) for k, v, r in (("dW", dW, dWo), ("dalpha", da, dao), ("dbeta", db, dbo))}
    coss = {k: _cos(v.cpu().numpy(), r) for k, v, r in (("dW", dW, dWo), ("dalpha", da, dao), ("dbeta", db, dbo))}
    _say(f"[{name} {prec}] z rel {zerr:.2e}, loss rel {lerr:.2e}, grads rel "
         + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
         + "; cos " + ", ".join(f"{k} {v:.6f}" for k, v in coss.items()))
    # the kernel's own F agrees with F evaluated in FP64 on the Z it returned
    np.testing.assert_allclose(F.cpu().numpy(), oracle.objective(pb.D, pb.X, Zg, pb.lam),
                               rtol=1e-4 if prec == "fp32" else 2e-2, atol=1e-6)
    assert lerr <= LOSS_TOL[prec]
    if prec == "fp32":
        assert zerr <= Z_TOL_FP32
        for k, v in errs.items():
            assert v <= GRAD_TOL_FP32, k
    else:
        assert zerr <= BF16_TOL
        assert errs["dalpha"] <= BF16_TOL and errs["dbeta"] <= BF16_TOL
        assert coss["dW"] >= DW_COS_BF16
    d.close()


def test_lista_coupled_to_dictionary_matches_step_lista(sl):
    """W_t = D, alpha_t = beta_t: the LISTA network is Step-LISTA (the remark
    after Eq. (12)), so z^(T) matches slista_forward and dalpha + dbeta matches
    the Step-LISTA gradient."""
    pb = synth.make_problem(64, 256, 1500, 0.05, 0.01, 0.1, seed=1304)
    T = 15
    a = _f32(synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=3))
    d = sl.Dictionary(_gpu(pb.D))
    X, ag = _gpu(pb.X), _gpu(a)
    W = _gpu(np.repeat(pb.D[None], T, axis=0))
    Zl, _, ll, _, da, db, _ = sl.lista_forward_backward(d, X, pb.lam, W, ag, ag, want_dW=False)
    Zs, _, ls, das, _ = sl.forward_backward(d, X, pb.lam, ag, ckpt_every=1)
    torch.cuda.synchronize()
    zerr = _rel(Zl.cpu().numpy(), Zs.cpu().numpy().astype(np.float64))
    gerr = _rel((da + db).cpu().numpy(), das.cpu().numpy().astype(np.float64))
    _say(f"LISTA(W=D, a=b) vs Step-LISTA: z rel {zerr:.2e}, loss {ll.item():.7g} / {ls.item():.7g}, grad rel {gerr:.2e}")
    assert zerr <= Z_TOL_FP32
    assert ll.item() == pytest.approx(ls.item(), rel=1e-5)
    assert gerr <= GRAD_TOL_FP32
    d.close()


def test_lista_autograd_with_upstream_dz(sl):
    """ListaFunction: J = mean F + <G, Z> through torch autograd equals the
    oracle's gradient with dZ = G, dF = 1/N; skipping dW leaves dalpha and
    dbeta bitwise unchanged."""
    pb = synth.make_problem(24, 96, 500, 0.1, 0.01, 0.1, seed=1305)
    T = 6
    W, a, b = _params(pb, T, 11, 0.3)
    G = _f32(np.random.default_rng(4).standard_normal((pb.N, pb.m)) * 1e-3)
    _, _, dWo, dao, dbo = oracle.lista_forward_backward(pb.D, pb.X, pb.lam, W, a, b, dZ=G,
                                                        dF=np.full(pb.N, 1.0 / pb.N))
    d = sl.Dictionary(_gpu(pb.D))
    Wt, at, bt = (_gpu(v).requires_grad_(True) for v in (W, a, b))
    Z, F = sl.lista(Wt, at, bt, d, _gpu(pb.X), pb.lam)
    J = F.mean() + (Z * _gpu(G)).sum()
    J.backward()
    for k, v, r in (("dW", Wt.grad, dWo), ("dalpha", at.grad, dao), ("dbeta", bt.grad, dbo)):
        err = _rel(v.cpu().numpy(), r)
        _say(f"autograd {k} rel {err:.2e}")
        assert err <= GRAD_TOL_FP32, k
    # alpha, beta only: the weight-gradient launches are skipped
    Z2, F2, _, ws = sl.lista_forward(d, _gpu(pb.X), pb.lam, Wt.detach(), at.detach(), bt.detach(), tape=True)
    dW, da, db = sl.lista_backward(d, pb.N, pb.lam, at.detach(), bt.detach(), ws, dZ=_gpu(G),
                                   dF=torch.full((pb.N,), 1.0 / pb.N, device=DEV), want_dW=False)
    assert dW is None
    dW1, da1, db1 = sl.lista_backward(d, pb.N, pb.lam, at.detach(), bt.detach(), ws, dZ=_gpu(G),
                                      dF=torch.full((pb.N,), 1.0 / pb.N, device=DEV))
    assert torch.equal(da, da1) and torch.equal(db, db1)
    d.close()


def test_lista_edge_cases(sl):
    pb = synth.make_problem(10, 20, 50, 0.2, 0.01, 0.1, seed=1306)
    d = sl.Dictionary(_gpu(pb.D))
    X = _gpu(pb.X)
    # T = 0: z = 0 and F = 1/2 |x|^2
    empty = torch.empty(0, device=DEV)
    Z, F, loss, _ = sl.lista_forward(d, X, pb.lam, torch.empty(0, 10, 20, device=DEV), empty, empty)
    torch.cuda.synchronize()
    assert float(Z.abs().max()) == 0.0
    np.testing.assert_allclose(F.cpu().numpy(), 0.5 * np.sum(pb.X ** 2, axis=1), rtol=1e-6)
    # N = 0: zero loss and gradients
    W, a, b = _params(pb, 3, 1, 0.1)
    Z, F, loss, dW, da, db, _ = sl.lista_forward_backward(d, torch.empty(0, 10, device=DEV), pb.lam, _gpu(W),
                                                          _gpu(a), _gpu(b))
    torch.cuda.synchronize()
    assert loss.item() == 0.0 and float(dW.abs().max()) == 0.0
    assert float(da.abs().max()) == 0.0 and float(db.abs().max()) == 0.0
    # invalid arguments are refused before any launch
    with pytest.raises(sl.SlistaError):
        sl.lista_forward(d, X, -1.0, _gpu(W), _gpu(a), _gpu(b))
    with pytest.raises(ValueError):
        sl.lista_forward(d, X, pb.lam, _gpu(W[:, :, :5]), _gpu(a), _gpu(b))
    with pytest.raises(sl.SlistaError):
        sl.lista_backward(d, pb.N, pb.lam, _gpu(a), _gpu(b), sl.lista_workspace(d, pb.N, 3, tape=True))
    d.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_lista_persistent_matches_per_layer(sl, prec):
    """The persistent kernels (one workgroup carries 32 samples through every
    layer) and the per-layer kernels compute the same network: same operand
    rounding, different accumulation order."""
    pb, W, a, b, *_ = _reference("gauss_64x256")
    d = sl.Dictionary(_gpu(pb.D))
    args = (d, _gpu(pb.X), pb.lam, _gpu(W), _gpu(a), _gpu(b))
    try:
        sl.set_kernel_family("layer")
        ref = sl.lista_forward_backward(*args, prec=prec)
        sl.set_kernel_family("persistent")
        got = sl.lista_forward_backward(*args, prec=prec)
    finally:
        sl.set_kernel_family("auto")
    torch.cuda.synchronize()
    tol = 1e-5 if prec == "fp32" else 5e-2
    for k, i in (("Z", 0), ("F", 1), ("dW", 3), ("dalpha", 4), ("dbeta", 5)):
        r = ref[i].cpu().numpy().astype(np.float64)
        err = _rel(got[i].cpu().numpy(), r)
        _say(f"[{prec}] persistent vs per-layer {k}: rel {err:.2e}")
        assert err <= tol, k
    d.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shape", [(100, 600, 300, 5), (64, 1500, 200, 3)])
def test_lista_wide_dictionaries(sl, shape, prec):
    """100 x 600 (n_pad 128, m_pad 640): the persistent kernels with several
    column-block groups per wave and a partial last group; 64 x 1500 (m_pad
    1536): the tile exceeds LDS and the per-layer kernels take over. Both
    against the oracle."""
    n, m, N, T = shape
    pb = synth.make_problem(n, m, N, 0.05, 0.01, 0.1, seed=1307 + m)
    W, a, b = _params(pb, T, 5, 0.2)
    Zo, Fo, dWo, dao, dbo = oracle.lista_forward_backward(pb.D, pb.X, pb.lam, W, a, b, dF=np.full(N, 1.0 / N))
    d = sl.Dictionary(_gpu(pb.D))
    Z, F, loss, dW, da, db, _ = sl.lista_forward_backward(d, _gpu(pb.X), pb.lam, _gpu(W), _gpu(a), _gpu(b),
                                                          prec=prec)
    torch.cuda.synchronize()
    lo = float(np.mean(Fo[-1]))
    lerr = abs(loss.item() - lo) / lo
    errs = {k: _rel(v.cpu().numpy(), r) for k, v, r in (("Z", Z, Zo), ("dW", dW, dWo), ("dalpha", da, dao),
                                                        ("dbeta", db, dbo))}
    coss = {k: _cos(v.cpu().numpy(), r) for k, v, r in (("dW", dW, dWo), ("dalpha", da, dao), ("dbeta", db, dbo))}
    _say(f"[{n}x{m} {prec}] loss rel {lerr:.2e}; " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items())
         + "; cos " + ", ".join(f"{k} {v:.6f}" for k, v in coss.items()))
    assert lerr <= LOSS_TOL[prec]
    if prec == "fp32":
        for k, v in errs.items():
            assert v <= GRAD_TOL_FP32, k
    else:
        assert errs["Z"] <= BF16_TOL
        assert errs["dalpha"] <= BF16_TOL and errs["dbeta"] <= BF16_TOL
        assert coss["dW"] >= DW_COS_BF16
    d.close()


@pytest.mark.parametrize("N,T", [(5, 1), (33, 2), (1, 3)])
def test_lista_small_batches_and_depths(sl, N, T):
    """One partial 32-sample tile (N = 5, 1), a full tile plus one sample
    (N = 33), and a single layer (T = 1: the seed goes straight to the
    weight gradient), FP32 against the oracle."""
    pb = synth.make_problem(20, 80, N, 0.1, 0.01, 0.1, seed=1310 + N)
    W, a, b = _params(pb, T, 9, 0.2)
    Zo, Fo, dWo, dao, dbo = oracle.lista_forward_backward(pb.D, pb.X, pb.lam, W, a, b, dF=np.full(N, 1.0 / N))
    d = sl.Dictionary(_gpu(pb.D))
    Z, F, loss, dW, da, db, _ = sl.lista_forward_backward(d, _gpu(pb.X), pb.lam, _gpu(W), _gpu(a), _gpu(b))
    torch.cuda.synchronize()
    errs = {k: _rel(v.cpu().numpy(), r) for k, v, r in (("Z", Z, Zo), ("dW", dW, dWo), ("dalpha", da, dao),
                                                        ("dbeta", db, dbo)) if np.max(np.abs(r)) > 0}
    lo = float(np.mean(Fo[-1]))
    _say(f"[N={N} T={T}] loss rel {abs(loss.item() - lo) / lo:.2e}; " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert abs(loss.item() - lo) / lo <= LOSS_TOL["fp32"]
    for k, v in errs.items():
        assert v <= GRAD_TOL_FP32, k
    d.close()
