"""The uneven batch at its full size, in the configuration bench.py times: 64
problems (n in [32, 512], m = 4n, N in [128, 8192]), T = 100 layers with
per-problem step sizes, a checkpoint every 10 layers, autotuned tiles, one
captured HIP graph. Samples are independent, so every problem is checked on
sampled rows against the FP64 oracle run on those rows alone, and batch
results equal single-problem calls bit for bit.

Precisions: FP32, and BF16 with an FP32 tail (the last 40 of the 100 layers
contract in FP32). At T = 100 the problems are converged to a gap of about
4e-6 of F*, below the rounding floor of BF16 operands: BF16 throughout
misses the 2e-2 objective-gap bar (kept below as an expected failure),
while FP32 layers at the end contract the BF16 floor away (a CPU emulation
of the schedule measured 9e-3 with 30 of them and 4.5e-3 with 40 on a subset
of the problems; 40 also keep the step gradients of the late layers within
2e-2).

The mean gap's reference F* is the best objective an FP64 FISTA run of 1000
iterations reaches on the same rows: F* <= that value, so the gap used in the
denominator is a lower bound and the relative errors are, if anything,
overstated."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import DALPHA_TOL, GAP_TOL, z_tolerance

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
ROWS = 16          # sampled rows per problem for the codes and the gap
GRAD_ROWS = 64     # sampled rows of the largest problem per bucket for dalpha
TAIL = 40          # FP32 layers at the end of the BF16 schedule
FISTA_ITERS = 1000


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sl():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1905_11071_amd as sl
    return sl


def _bucket(m):
    mp = -(-m // 64) * 64
    return 1 if mp <= 256 else 2 if mp <= 512 else 4 if mp <= 1024 else 8


@pytest.fixture(scope="module")
def uneven(sl):
    """Device inputs of the 64 problems and the oracle on each problem's
    sampled rows (z^T, iterates, a FISTA reference for F*); for the largest
    problem of each column-pass bucket also the step gradient of the mean
    objective over GRAD_ROWS sampled rows."""
    T = synth.UNEVEN["T"]
    specs = synth.uneven_problem_specs(P=synth.UNEVEN["P"], seed=synth.UNEVEN["seed"])
    rng = np.random.default_rng(7)
    largest = {}
    for i, sp in enumerate(specs):
        b = _bucket(sp["m"])
        if b not in largest or sp["m"] * sp["N"] > specs[largest[b]]["m"] * specs[largest[b]]["N"]:
            largest[b] = i
    probs, inputs = [], []
    for i, sp in enumerate(specs):
        pb = synth.make_problem(sp["n"], sp["m"], sp["N"], sp["p"], sp["sigma"], sp["lam_frac"], sp["seed"])
        d = sl.Dictionary(torch.tensor(pb.D32(), device=DEV))
        L, _ = d.lipschitz(max_iter=20_000, rtol=1e-7)
        alpha = synth.perturbed_steps(L, T, seed=sp["seed"])
        rows = np.sort(rng.choice(pb.N, size=min(ROWS, pb.N), replace=False))
        Xs = pb.X[rows]
        Zo, Fo, its = oracle.forward(pb.D, Xs, pb.lam, alpha, return_iterates=True)
        Lo = oracle.lipschitz(pb.D)
        _, Ff = oracle.fista(pb.D, Xs, pb.lam, np.full(FISTA_ITERS, 1.0 / Lo))
        ref = {"rows": rows, "Zo": Zo, "Fo": Fo[-1], "ztol": z_tolerance(pb.D, Xs, alpha, its),
               "Fstar_ub": np.minimum(Ff.min(axis=0), Fo[-1])}
        if largest.get(_bucket(pb.m)) == i:
            grows = np.sort(rng.choice(pb.N, size=min(GRAD_ROWS, pb.N), replace=False))
            dFg = np.full(len(grows), 1.0 / len(grows))
            _, _, dao, its_g, adj_g = oracle.forward_backward(pb.D, pb.X[grows], pb.lam, alpha, dF=dFg,
                                                              return_adjoints=True)
            _, _, da32 = oracle.forward_backward(pb.D, pb.X[grows], pb.lam, alpha, dF=dFg, dtype=np.float32)
            scale = np.max(np.abs(dao))
            u = 2.0 ** -24
            ref["grad_rows"], ref["dalpha_rows"] = grows, dao
            ref["floor32"] = np.max(np.abs(da32 - dao)) / scale
            ref["cancel"] = np.array([u / alpha[t] * np.sum(np.abs(adj_g[t]) * (np.abs(its_g[t]) + 2 * np.abs(its_g[t + 1])))
                                      for t in range(T)]) / scale
        probs.append((pb, ref))
        inputs.append((d, torch.tensor(pb.X32(), device=DEV), pb.lam,
                       torch.tensor(alpha, device=DEV, dtype=torch.float32)))
    _say(f"uneven batch: {len(probs)} problems and their oracle references ready; "
         f"largest per bucket {sorted(largest.items())}")
    yield probs, inputs
    for d, _, _, _ in inputs:
        d.close()


def _prec(sl, name):
    return {"fp32": "fp32", "bf16": "bf16", "bf16+tail": sl.bf16_fp32_tail(TAIL)}[name]


def _run_batch(sl, inputs, prec):
    b = sl.Batch(inputs, prec=prec, ckpt_every=synth.UNEVEN["ckpt_every"])
    b.run()
    torch.cuda.synchronize()
    tuned = b.autotune()
    b.capture()
    for z in b.Z:
        z.zero_()
    b.replay()
    torch.cuda.synchronize()
    return b, tuned


def _gap_error(probs, b):
    gap_gpu = gap_orc = f_sum = 0.0
    for i, (pb, ref) in enumerate(probs):
        Xs = pb.X[ref["rows"]]
        Zg = b.Z[i].cpu().numpy().astype(np.float64)[ref["rows"]]
        Fg = oracle.objective(pb.D, Xs, Zg, pb.lam)
        gap_gpu += float(np.sum(Fg - ref["Fstar_ub"]))
        gap_orc += float(np.sum(ref["Fo"] - ref["Fstar_ub"]))
        f_sum += float(np.sum(ref["Fstar_ub"]))
    return abs(gap_gpu - gap_orc) / gap_orc, gap_orc / f_sum


@pytest.mark.parametrize("name", ["fp32", "bf16+tail"])
def test_uneven_batch_full_size(sl, uneven, name):
    probs, inputs = uneven
    prec = _prec(sl, name)
    b, tuned = _run_batch(sl, inputs, prec)
    _say(f"[{name}] tuned variants {tuned}")
    worst_z = 0.0
    for i, (pb, ref) in enumerate(probs):
        rows = ref["rows"]
        Zg = b.Z[i].cpu().numpy().astype(np.float64)[rows]
        Fg = b.F[i].cpu().numpy().astype(np.float64)[rows]
        # in-kernel objective (FP32 Gram form) against the FP64 residual form
        np.testing.assert_allclose(Fg, ref["Fo"], rtol=1e-4)
        if name == "fp32":
            err = float(np.max(np.abs(Zg - ref["Zo"])))
            worst_z = max(worst_z, err / ref["ztol"])
            assert err <= ref["ztol"], (i, err, ref["ztol"])
    rel, gap_f = _gap_error(probs, b)
    tol = GAP_TOL["fp32" if name == "fp32" else "bf16"]
    _say(f"[{name}] {ROWS} sampled rows of 64 problems: mean-gap rel err {rel:.2e} (tolerance {tol:.0e}; "
         f"gap / F* = {gap_f:.2e}), worst |dZ|/bound {worst_z:.2e}")
    assert rel <= tol
    # every problem's outputs equal its own single-problem call bit for bit;
    # checked on problems spanning the four column-pass buckets
    by_bucket = {}
    for i, (pb, _) in enumerate(probs):
        by_bucket.setdefault(_bucket(pb.m), []).append(i)
    picks = sorted({ids[0] for ids in by_bucket.values()} | {ids[-1] for ids in by_bucket.values()})
    for i in picks:
        d, X, lam, a = inputs[i]
        Z, F, loss, da, _ = sl.forward_backward(d, X, lam, a, prec=prec, ckpt_every=synth.UNEVEN["ckpt_every"])
        torch.cuda.synchronize()
        assert np.array_equal(b.Z[i].cpu().numpy(), Z.cpu().numpy()), i
        assert np.array_equal(b.dalpha[i].cpu().numpy(), da.cpu().numpy()), i
        assert b.loss[i].item() == loss.item(), i
    _say(f"[{name}] batch equals single calls on problems {picks}")
    b.close()


@pytest.mark.xfail(strict=True, raises=AssertionError, reason="BF16 operands in all 100 layers leave the converged problems at a "
                                       "rounding floor about 36x the 2e-2 objective-gap bar; the FP32 tail "
                                       "schedule above meets it")
def test_uneven_batch_bf16_throughout_misses_the_gap(sl, uneven):
    probs, inputs = uneven
    b, _ = _run_batch(sl, inputs, "bf16")
    rel, _ = _gap_error(probs, b)
    _say(f"[bf16 throughout] mean-gap rel err {rel:.2e}")
    b.close()
    assert rel <= GAP_TOL["bf16"]



@pytest.mark.parametrize("name", ["fp32", "bf16+tail"])
def test_uneven_dalpha_on_the_largest_problems(sl, uneven, name):
    """d alpha of the mean objective over GRAD_ROWS sampled rows (dF = 1 /
    rows there, 0 elsewhere) on the largest problem of every column-pass
    bucket, in the batch's configuration (checkpoints every 10 layers), on
    all T layers, against the FP64 oracle on those rows. The batch's own
    gradients equal these single calls' (bit for bit, tested above).

    Tolerance per layer t, relative to max |dalpha|: BF16 (with the FP32
    tail) 2e-2. FP32 max(1e-5, 4 f + c_t), because at T = 100 on converged
    problems with m up to 1856 the 32-bit rounding floor itself exceeds 1e-5:
      f   the oracle's recursion evaluated in float32 on the same rows, its
          largest distance from the float64 oracle over the layers: a
          measured floor of 32-bit arithmetic for these problems (forward
          and reverse pass; 2.8e-6 to 3.3e-5 on the four problems), with a
          factor 4 for the device's different summation order;
      c_t the rounding of the difference form the kernels use,
          dalpha_t = -(1/alpha_t) sum v^t (z^t - z^{t+1}) with 32-bit
          iterates: the stored iterates are rounded once each, so the form
          differs from the gradient form by at most
          (u / alpha_t) sum |v^t| (|z^t| + 2 |z^{t+1}|), u = 2^-24, which
          grows as z^t - z^{t+1} shrinks on the converged layers.
    Both terms come from the oracle alone."""
    probs, inputs = uneven
    prec = _prec(sl, name)
    k = synth.UNEVEN["ckpt_every"]
    T = synth.UNEVEN["T"]
    for i, (pb, ref) in enumerate(probs):
        if "grad_rows" not in ref:
            continue
        d, X, lam, a = inputs[i]
        _, _, _, _, ws = sl.forward_backward(d, X, lam, a, prec=prec, ckpt_every=k)
        grows = ref["grad_rows"]
        dF = np.zeros(pb.N, np.float32)
        dF[grows] = 1.0 / len(grows)
        da = sl.backward(d, X, lam, a, ws, dF=torch.tensor(dF, device=DEV), prec=prec, ckpt_every=k)
        da = da.cpu().numpy().astype(np.float64)
        del ws
        dao = ref["dalpha_rows"]
        err = np.abs(da - dao) / np.max(np.abs(dao))
        if name == "fp32":
            tol = np.maximum(DALPHA_TOL["fp32"], 4.0 * ref["floor32"] + ref["cancel"])
        else:
            tol = np.full(T, DALPHA_TOL["bf16"])
        worst = int(np.argmax(err / tol))
        _say(f"[{name}] problem {i} n={pb.n} m={pb.m} N={pb.N}: max rel err {err.max():.2e} (layer "
             f"{int(err.argmax())}); float32 oracle floor {ref['floor32']:.2e}; worst err / tolerance "
             f"{err[worst] / tol[worst]:.2f} at layer {worst} (tolerance {tol[worst]:.2e}); layers at or "
             f"below 1e-5: {int(np.sum(err <= 1e-5))} of {T}")
        assert np.all(err <= tol), (i, np.flatnonzero(err > tol))
