"""The C ABI library loads and exports every symbol include/slista.h declares,
and its host-side argument checks reject bad calls before any device work.
CPU only: none of these calls reaches the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slista.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SLISTA_API\s+[\w\s\*]+?\b(slista_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1905_11071_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libslista.so is not built (run __graft_entry__.build())")
    return _lib.lib()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for want in ["slista_dict_create", "slista_dict_lipschitz", "slista_forward", "slista_backward",
                 "slista_forward_backward", "slista_workspace_size"]:
        assert want in syms


def test_every_declared_symbol_is_exported(lib):
    from paper_1905_11071_amd import _lib
    syms = declared_symbols()
    assert syms, "no declarations parsed"
    for s in syms:
        assert hasattr(lib, s), f"{s} declared but not exported"
        assert s in _lib.SIGNATURES, f"{s} has no ctypes signature in the binding"
    assert set(_lib.SIGNATURES) == set(syms)


def test_abi_version_and_status_strings(lib):
    assert lib.slista_abi_version() == 1
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.slista_status_string(code)
    assert lib.slista_status_string(12345) == b"unknown status"


def test_null_dict_rejected(lib):
    vp = ctypes.c_void_p
    st = lib.slista_forward(None, vp(16), 4, 0.1, vp(16), 3, 0, vp(16), None, 0, None, 0, vp(256), 1 << 20, None)
    assert st == -1
    assert b"dict" in lib.slista_last_error()
    st = lib.slista_backward(None, vp(16), 4, 0.1, vp(16), 3, 0, None, None, vp(16), 1, vp(256), 1 << 20, None)
    assert st == -1


def test_dict_create_rejects_bad_sizes(lib):
    h = ctypes.c_void_p()
    assert lib.slista_dict_create(None, 4, 8, None, ctypes.byref(h)) == -1
    assert lib.slista_dict_create(ctypes.c_void_p(256), 0, 8, None, ctypes.byref(h)) == -1
    assert lib.slista_dict_create(ctypes.c_void_p(256), 4, 0, None, ctypes.byref(h)) == -1
    assert lib.slista_dict_create(ctypes.c_void_p(256), 4, 9000, None, ctypes.byref(h)) == -1
    assert h.value is None
    assert lib.slista_dict_destroy(None) == 0


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_1905_11071_amd as sl
    with pytest.raises(ValueError):
        sl.Dictionary(torch.zeros(4, 8))


def test_options_are_checked_on_the_host(lib):
    assert lib.slista_set_option(1, 3) == -1          # kernel family outside [0, 2]
    assert lib.slista_set_option(2, 5) == -1          # tile variant outside [0, 4]
    assert lib.slista_set_option(99, 0) == -1         # unknown option
    assert lib.slista_set_option(2, 4) == 0
    assert lib.slista_set_option(2, 0) == 0
    assert lib.slista_set_option(1, 0) == 0


def test_tuning_table_round_trip(lib, tmp_path):
    """slista_tune_load keeps only well-formed records (precision, column
    passes, log2 N, variant); slista_tune_save writes them back. Host only."""
    src = tmp_path / "in.txt"
    src.write_text("1 4 16 4\n0 8 12 1\n1 3 10 2\n0 2 9 7\n1 1 30 2\n")
    assert lib.slista_tune_load(str(src).encode()) == 0
    out = tmp_path / "out.txt"
    assert lib.slista_tune_save(str(out).encode()) == 0
    recs = {tuple(map(int, ln.split())) for ln in out.read_text().splitlines() if ln.strip()}
    assert {(1, 4, 16, 4), (0, 8, 12, 1), (1, 1, 30, 2)} <= recs
    assert (1, 3, 10, 2) not in recs and (0, 2, 9, 7) not in recs   # bad passes / variant dropped
    assert lib.slista_tune_load(str(tmp_path / "missing.txt").encode()) == -1
    assert lib.slista_tune_save(None) == -1


def test_batch_and_autotune_reject_null_arguments(lib):
    best = ctypes.c_int()
    assert lib.slista_autotune(None, None, 1, ctypes.c_float(0.1), None, 1, 0, 1, None, None, None, 0, None,
                               ctypes.byref(best), None) == -1
    assert lib.slista_batch_autotune(None, None, None) == -1
    out = ctypes.c_void_p()
    assert lib.slista_batch_create(None, 1, 5, 0, 1, ctypes.byref(out)) == -1
    assert lib.slista_batch_run(None, None) == -1
    assert lib.slista_batch_replay(None, None) == -1
    assert lib.slista_batch_destroy(None) == 0


def test_bf16_rounding_helper_matches_torch():
    """The tests' BF16 rounding (used for the gap resolution floor) is
    round-to-nearest-even, as torch's float32 -> bfloat16 conversion."""
    import numpy as np
    import torch
    from tests.gpu_common import round_to_bf16
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-20, 20, 10000),
                        [0.0, -0.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).double().numpy()
    assert np.array_equal(round_to_bf16(x), ref)


def test_lista_entry_points_reject_bad_arguments(lib):
    """The coupled-LISTA entry points validate on the host, before any launch."""
    vp = ctypes.c_void_p
    size = ctypes.c_size_t()
    assert lib.slista_lista_workspace_size(None, 4, 3, 0, 1, ctypes.byref(size)) == -1
    assert b"dict" in lib.slista_last_error()
    st = lib.slista_lista_forward(None, vp(16), 4, ctypes.c_float(0.1), vp(16), vp(16), vp(16), 3, 0, vp(16), None,
                                  None, 1, vp(256), ctypes.c_size_t(1 << 20), None)
    assert st == -1
    st = lib.slista_lista_backward(None, 4, ctypes.c_float(0.1), vp(16), vp(16), 3, 0, None, None, None, vp(16),
                                   vp(16), vp(256), ctypes.c_size_t(1 << 20), None)
    assert st == -1
    st = lib.slista_lista_forward_backward(None, vp(16), 4, ctypes.c_float(0.1), vp(16), vp(16), vp(16), 3, 0,
                                           vp(16), None, None, None, vp(16), vp(16), vp(256),
                                           ctypes.c_size_t(1 << 20), None)
    assert st == -1


def test_check_and_batched_entry_points_reject_bad_arguments(lib):
    """The device checks, lambda_max, the one-call batch and the options
    validate on the host, before any launch."""
    vp = ctypes.c_void_p
    size = ctypes.c_size_t()
    assert lib.slista_kkt(None, vp(16), 4, ctypes.c_float(0.1), vp(16), vp(16), None, None) == -1
    assert lib.slista_lambda_max_workspace_size(None, 4, ctypes.byref(size)) == -1
    assert lib.slista_lambda_max(None, vp(16), 4, vp(16), None, vp(256), ctypes.c_size_t(1 << 20), None) == -1
    assert lib.slista_batched_workspace_size(None, 1, 5, 0, 1, ctypes.byref(size)) == -1
    assert lib.slista_batched_fwd_bwd(None, 1, 5, 0, 1, vp(256), ctypes.c_size_t(1 << 20), None, 0) == -1
    assert lib.slista_batched_release() == 0
    assert lib.slista_set_option(3, 2) == -1
    assert lib.slista_set_option(3, 0) == 0
    assert lib.slista_status_string(-6) == b"non-finite values (NaN or Inf) found by the finite-value check"


def test_precision_schedule_is_checked_on_the_host(lib):
    """SLISTA_BF16_FP32_TAIL(k) = 1 | k << 8: the tail must not exceed T, needs
    BF16 layers before it, and with checkpoints its first layer must be a
    checkpoint. A batch of problems takes the same encoding."""
    import re
    text = open(HEADER).read()
    assert re.search(r"#define SLISTA_BF16_FP32_TAIL\(tail\) \(SLISTA_BF16 \| \(\(tail\) << 8\)\)", text)

    class P(ctypes.Structure):
        _fields_ = [("dict", ctypes.c_void_p), ("X", ctypes.c_void_p), ("N", ctypes.c_int),
                    ("lam", ctypes.c_float), ("alpha", ctypes.c_void_p), ("Z", ctypes.c_void_p),
                    ("F", ctypes.c_void_p), ("loss", ctypes.c_void_p), ("dalpha", ctypes.c_void_p)]
    arr = (P * 1)()
    out = ctypes.c_void_p()
    for prec, T, k, frag in [((1 | (6 << 8)), 5, 1, b"longer than T"), ((0 | (2 << 8)), 5, 1, b"needs SLISTA_BF16"),
                             ((1 | (3 << 8)), 10, 2, b"checkpoint"), (7, 5, 1, b"unknown precision")]:
        # the schedule is parsed before the problems are looked at
        assert lib.slista_batch_create(ctypes.cast(arr, ctypes.c_void_p), 1, T, prec, k, ctypes.byref(out)) == -1
        assert frag in lib.slista_last_error(), (prec, lib.slista_last_error())


def test_f64_forward_rejects_bad_arguments(lib):
    vp = ctypes.c_void_p
    n = ctypes.c_size_t()
    assert lib.slista_forward_f64_workspace_size(None, 4, ctypes.byref(n)) == -1
    st = lib.slista_forward_f64(None, vp(256), 4, 0.1, vp(256), 3, vp(256), None, 0, None, None, 0, None)
    assert st == -1 and b"dict" in lib.slista_last_error()
