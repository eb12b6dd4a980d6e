"""Uneven multi-problem batches through the C ABI: each problem of a batch
gives the same results as its own single-problem call, graph replays equal
eager runs, and the step gradients match the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import DALPHA_TOL

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


def _problems(specs, T, seed0):
    out = []
    for i, (n, m, N) in enumerate(specs):
        pb = synth.make_problem(n, m, N, 0.05, 0.0, 0.1, seed=seed0 + i)
        alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=i)
        out.append((pb, alpha))
    return out


# sizes across all four column-pass buckets, ragged N and m
SPECS = [(32, 128, 300), (50, 200, 1037), (80, 320, 513), (100, 400, 129), (160, 640, 700),
         (300, 1200, 257), (16, 64, 1000)]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("ckpt", [1, 3])
def test_batch_equals_single_calls(sl, prec, ckpt):
    T = 7
    probs = _problems(SPECS, T, 700)
    dicts = [sl.Dictionary(_gpu(pb.D)) for pb, _ in probs]
    inputs = [(d, _gpu(pb.X), pb.lam, _gpu(a)) for d, (pb, a) in zip(dicts, probs)]
    b = sl.Batch(inputs, prec=prec, ckpt_every=ckpt)
    b.run()
    torch.cuda.synchronize()
    for i, (d, X, lam, a) in enumerate(inputs):
        Z, F, loss, da, _ = sl.forward_backward(d, X, lam, a, prec=prec, ckpt_every=ckpt)
        assert np.array_equal(b.Z[i].cpu().numpy(), Z.cpu().numpy()), i
        assert np.array_equal(b.F[i].cpu().numpy(), F.cpu().numpy()), i
        assert np.array_equal(b.dalpha[i].cpu().numpy(), da.cpu().numpy()), i
        assert b.loss[i].item() == loss.item()
    b.close()


def test_batch_graph_replays_equal_eager(sl):
    T = 6
    probs = _problems(SPECS[:5], T, 800)
    dicts = [sl.Dictionary(_gpu(pb.D)) for pb, _ in probs]
    inputs = [(d, _gpu(pb.X), pb.lam, _gpu(a)) for d, (pb, a) in zip(dicts, probs)]
    b = sl.Batch(inputs, prec="bf16", ckpt_every=2)
    b.run()
    torch.cuda.synchronize()
    ref = [(z.cpu().numpy(), da.cpu().numpy()) for z, da in zip(b.Z, b.dalpha)]
    b.capture()
    for rep in range(3):
        for z in b.Z:
            z.zero_()
        for da in b.dalpha:
            da.fill_(-1.0)
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for i, (zr, dr) in enumerate(ref):
            assert np.array_equal(b.Z[i].cpu().numpy(), zr), (rep, i)
            assert np.array_equal(b.dalpha[i].cpu().numpy(), dr), (rep, i)
        # eager work between replays
        sl.forward(dicts[0], inputs[0][1], inputs[0][2], inputs[0][3])
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_gradients_vs_oracle(sl, prec):
    T = 8
    probs = _problems(SPECS[:4] + SPECS[5:6], T, 900)
    dicts = [sl.Dictionary(_gpu(pb.D)) for pb, _ in probs]
    inputs = [(d, _gpu(pb.X), pb.lam, _gpu(a)) for d, (pb, a) in zip(dicts, probs)]
    b = sl.Batch(inputs, prec=prec, ckpt_every=3)
    b.run()
    torch.cuda.synchronize()
    for i, (pb, alpha) in enumerate(probs):
        Zo, Fo, dao = oracle.forward_backward(pb.D, pb.X, pb.lam, alpha, dF=np.full(pb.N, 1.0 / pb.N))
        err = float(np.max(np.abs(b.dalpha[i].cpu().numpy() - dao)) / np.max(np.abs(dao)))
        lerr = abs(b.loss[i].item() - Fo[-1].mean()) / Fo[-1].mean()
        _say(f"[{prec}] problem {i} n={pb.n} m={pb.m} N={pb.N}: dalpha rel err {err:.2e}, loss rel err {lerr:.2e}")
        assert err <= DALPHA_TOL[prec] and lerr <= (1e-5 if prec == "fp32" else 2e-2)
    b.close()


def test_batch_autotune_keeps_results(sl):
    """Tuning a batch changes only its tile shapes: the outputs stay the same
    bits, before and after graph capture."""
    T = 5
    probs = _problems(SPECS, T, 1000)
    dicts = [sl.Dictionary(_gpu(pb.D)) for pb, _ in probs]
    inputs = [(d, _gpu(pb.X), pb.lam, _gpu(a)) for d, (pb, a) in zip(dicts, probs)]
    b = sl.Batch(inputs, prec="bf16", ckpt_every=2)
    b.run()
    torch.cuda.synchronize()
    ref = [(z.cpu().numpy(), da.cpu().numpy()) for z, da in zip(b.Z, b.dalpha)]
    chosen = b.autotune()
    _say(f"tuned variants by column passes: {chosen}")
    assert set(chosen) == {1, 2, 4, 8} and all(v in (1, 2, 3, 4) for v in chosen.values())
    b.run()
    torch.cuda.synchronize()
    for i, (zr, dr) in enumerate(ref):
        assert np.array_equal(b.Z[i].cpu().numpy(), zr), i
        assert np.array_equal(b.dalpha[i].cpu().numpy(), dr), i
    b.capture()
    for z in b.Z:
        z.zero_()
    b.replay()
    torch.cuda.synchronize()
    for i, (zr, dr) in enumerate(ref):
        assert np.array_equal(b.Z[i].cpu().numpy(), zr), i
        assert np.array_equal(b.dalpha[i].cpu().numpy(), dr), i
    b.close()
