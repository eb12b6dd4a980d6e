"""slista_forward_scratch (the forward pass on the library's static per-device
scratch, for callers that cannot allocate) against slista_forward on a
caller workspace, through the C ABI: two calls in a row, the second smaller,
must give the same bits as the existing entry point (same kernels, same
order of every sum). Sizes past the scratch are rejected on the host."""
import ctypes
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


def _scratch_call(sl, d, X, lam, alpha, prec, f_trace):
    from paper_1905_11071_amd._lib import lib
    N, T = int(X.shape[0]), int(alpha.shape[0])
    Z = torch.full((N, d.m), float("nan"), device=DEV)
    F = torch.full((T + 1, N) if f_trace else (N,), float("nan"), device=DEV)
    loss = torch.full((1,), float("nan"), device=DEV)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib().slista_forward_scratch(d.handle, X.data_ptr(), N, float(lam), alpha.data_ptr(), T,
                                      sl.PRECISIONS[prec], Z.data_ptr(), F.data_ptr(), int(f_trace),
                                      loss.data_ptr(), s)
    assert st == 0, lib().slista_last_error()
    torch.cuda.synchronize()
    return Z.cpu().numpy(), F.cpu().numpy(), loss.cpu().numpy()


# the second case is smaller in every dimension than the first, so stale
# contents of the shared scratch would show up in its results
CASES = [((64, 256, 3000, 12), "bf16", False), ((32, 128, 517, 7), "fp32", True)]


def test_scratch_forward_equals_workspace_forward(sl):
    for (n, m, N, T), prec, trace in CASES:
        _say(f"scratch forward: n={n} m={m} N={N} T={T} {prec} trace={trace}")
        pb = synth.make_problem(n, m, N, 0.05, 0.01, 0.1, seed=400 + m)
        alpha = synth.perturbed_steps(oracle.lipschitz(pb.D), T, seed=9)
        d = sl.Dictionary(_gpu(pb.D))
        X, a = _gpu(pb.X), _gpu(alpha)
        Zs, Fs, ls = _scratch_call(sl, d, X, pb.lam, a, prec, trace)
        Zw, Fw, lw, _ = sl.forward(d, X, pb.lam, a, prec=prec, f_trace=trace, ckpt_every=0)
        torch.cuda.synchronize()
        assert np.array_equal(Zs, Zw.cpu().numpy())
        assert np.array_equal(Fs, Fw.cpu().numpy())
        assert np.array_equal(ls, lw.cpu().numpy())
        if prec == "fp32":
            # and the codes sit within the FP32 forward-error bound of the oracle
            from tests.gpu_common import z_tolerance
            Zo, _, its = oracle.forward(pb.D, pb.X, pb.lam, alpha, return_iterates=True)
            assert np.max(np.abs(Zs - Zo)) <= z_tolerance(pb.D, pb.X, alpha, its)
        d.close()


def test_scratch_forward_rejects_sizes_past_the_scratch(sl):
    from paper_1905_11071_amd._lib import lib
    pb = synth.make_problem(16, 1024, 8, 0.05, 0.0, 0.1, seed=3)
    d = sl.Dictionary(_gpu(pb.D))
    N = 5000  # m_pad = 1024: past the 64 MiB scratch (about 4000 samples)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = ctypes.c_void_p(16)  # never dereferenced: the size check comes first
    st = lib().slista_forward_scratch(d.handle, p, N, 0.1, p, 3, 0, p, None, 0, None, s)
    assert st == -1
    assert b"scratch" in lib().slista_last_error()
    d.close()
