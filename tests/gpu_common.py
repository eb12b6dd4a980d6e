"""Shared helpers for the GPU parity tests (the oracle is the reference)."""
from __future__ import annotations

import numpy as np

import oracle

U32 = 2.0 ** -24   # unit roundoff of FP32
U16 = 2.0 ** -8    # unit roundoff of BF16 (8-bit significand)

# Objective-gap tolerances: relative error of the mean gap
# mean_i (F_i(z_i^T) - F_i*), both F evaluated in FP64 from the returned codes.
GAP_TOL = {"fp32": 1e-5, "bf16": 2e-2}
# Step-size gradient tolerance, relative to max |dalpha| of the oracle.
DALPHA_TOL = {"fp32": 1e-5, "bf16": 2e-2}


def z_tolerance(D, X, alpha, iterates) -> float:
    """Forward-error bound for FP32 layers, elementwise (absolute).

    With alpha_t <= 2/L every layer is non-expansive in l2, so the rounding
    errors of the T layers add up at most linearly. Per sample, layer t
    rounds one length-m dot product per coordinate of G z (|error| <=
    (m+1) u (|G||z|)_j: Higham's gamma_m plus the rounding of G to FP32),
    reads c = D^T x, itself a length-n FP32 dot product (|error| <=
    n u (|D|^T |x|)_j), and does a few elementwise operations. Its error
    vector therefore has l2 norm at most
        alpha_t ((m+1) u || |G| ||_2 ||z^t||_2 + n u || |D|^T |x| ||_2)
        + 4 u (||z^t||_2 + alpha_t ||c||_2).
    Summed over layers with the largest sample norms; an elementwise error
    is at most the l2 norm of the error vector."""
    D = np.asarray(D, np.float64)
    X = np.asarray(X, np.float64)
    n, m = D.shape
    g2 = float(np.linalg.norm(np.abs(D.T @ D), 2))
    cabs = float(np.max(np.linalg.norm(np.abs(X) @ np.abs(D), axis=1))) if X.size else 0.0
    cmax = float(np.max(np.linalg.norm(X @ D, axis=1))) if X.size else 0.0
    tol = 0.0
    for a, Zt in zip(np.asarray(alpha, np.float64), iterates[:-1]):
        zn = float(np.max(np.linalg.norm(Zt, axis=1))) if Zt.size else 0.0
        tol += a * ((m + 1) * U32 * g2 * zn + n * U32 * cabs) + 4.0 * U32 * (zn + a * cmax)
    return tol + 1e-30


def mean_gap_rel_error(D, X, lam, Z_gpu, Z_orc, Zstar):
    Fs = oracle.objective(D, X, Zstar, lam)
    g_gpu = float(np.mean(oracle.objective(D, X, Z_gpu, lam) - Fs))
    g_orc = float(np.mean(oracle.objective(D, X, Z_orc, lam) - Fs))
    return abs(g_gpu - g_orc) / g_orc, g_gpu, g_orc


def round_to_bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)

