"""Plain FP64 CPU oracle for unfolded ISTA / Step-LISTA.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
link this package: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it. It shares no code with the HIP library.
"""
from .slista import (  # noqa: F401
    soft_threshold,
    lipschitz,
    lambda_max,
    objective,
    forward,
    forward_backward,
    adjoint,
    kkt_residual,
    lasso_solution,
    brute_force_lasso,
    train_steps,
    support_lipschitz,
    fista_momentum,
    fista,
    oista,
    lista_layer,
    lista_forward,
    lista_forward_backward,
)
