"""The kernels evaluate the soft threshold ST(u, t) = sign(u) max(|u| - t, 0)
(Section 1, after Eq. (2)) as u - clamp(u, -t, t) (one median-of-three and
one subtraction). In FP32 the two forms give the same bits for every finite
u and t > 0 (the threshold lambda alpha_t is positive by the library's
preconditions): both round only |u| - t (u - t or u + t on the other side),
rounding to nearest is symmetric, and inside [-t, t] both give +0. Checked
here with numpy float32 arithmetic (each operation rounded to FP32) on random
values and on the boundary cases."""
import numpy as np

F32 = np.float32


def st_sign_max(u, t):
    au = np.abs(u) - t
    return np.where(au > 0, np.copysign(au, u), F32(0.0)).astype(F32)


def st_clamp(u, t):
    return (u - np.minimum(np.maximum(u, -t), t)).astype(F32)


def _same_bits(a, b):
    return np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_forms_agree_bitwise_on_random_values():
    rng = np.random.default_rng(7)
    for scale in (1e-30, 1e-6, 1.0, 1e6, 1e30):
        u = (rng.standard_normal(200_000) * scale).astype(F32)
        for t in (F32(scale * 1e-3), F32(scale * 0.5), F32(scale * 3.0), F32(1e-45)):
            assert _same_bits(st_sign_max(u, t), st_clamp(u, t)), (scale, t)


def test_forms_agree_on_boundaries():
    t = F32(0.375)
    edge = np.array([0.0, -0.0, t, -t, np.nextafter(t, F32(1)), np.nextafter(-t, F32(-1)),
                     np.nextafter(t, F32(0)), np.nextafter(-t, F32(0)), 1e-45, -1e-45,
                     np.finfo(F32).max, -np.finfo(F32).max, np.finfo(F32).tiny], dtype=F32)
    a, b = st_sign_max(edge, t), st_clamp(edge, t)
    assert _same_bits(a, b)
    # inside the band the result is +0 (not -0) in both forms
    assert np.all(a[[0, 1, 2, 3, 6, 7, 8, 9, 12]].view(np.uint32) == 0)
    # the smallest positive threshold: only values inside [-t, t] change
    z = np.array([-2.5, -0.0, 0.0, 1e-45, -1e-45, 1e-38, 3.0], dtype=F32)
    tt = F32(1e-45)
    assert _same_bits(st_clamp(z, tt), st_sign_max(z, tt))
