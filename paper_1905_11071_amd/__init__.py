"""MI355X (gfx950) library for batched unfolded ISTA / Step-LISTA.

The computation lives in libslista.so (HIP kernels behind the C ABI of
include/slista.h); this package is its thin PyTorch binding.
"""
from .ops import (  # noqa: F401
    PRECISIONS,
    Batch,
    BatchedCall,
    batched_release,
    bf16_fp32_tail,
    kkt,
    lambda_max,
    set_check_finite,
    Dictionary,
    SlistaError,
    autotune,
    tune_load,
    tune_save,
    train,
    fista,
    oista,
    lista,
    lista_backward,
    lista_forward,
    lista_forward_backward,
    lista_workspace,
    ListaFunction,
    backward,
    forward,
    forward_backward,
    objective,
    profile_begin,
    profile_end,
    set_kernel_family,
    set_tile_variant,
    slista,
    SlistaFunction,
)
