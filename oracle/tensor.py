"""mu-mode product, Tucker operator and Kronecker-sum action (FP64).

Test infrastructure only (see the package docstring).

Tensors are numpy arrays of shape (n_1, ..., n_d); axis mu-1 is direction mu.
The flat (vec) form is the Fortran-order ravel, which stacks by columns as in
Section 2.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np


def mode_product(T: np.ndarray, L: np.ndarray, mu: int) -> np.ndarray:
    """S = T x_mu L  (mu is 1-based), the definition of Section 2:
    s_{i_1..i_d} = sum_j t_{i_1..j..i_d} l_{i_mu j}, i.e. L applied to every
    mu-fiber.  The contraction is numpy's tensordot (a library matmul)."""
    ax = mu - 1
    if L.shape != (T.shape[ax], T.shape[ax]):
        raise ValueError("matrix size does not match the tensor along mode %d" % mu)
    S = np.tensordot(L, T, axes=([1], [ax]))     # S[i_mu, rest...]
    return np.moveaxis(S, 0, ax)


def tucker(T: np.ndarray, Ls: Sequence[Optional[np.ndarray]]) -> np.ndarray:
    """T x_1 L_1 x_2 ... x_d L_d (Section 2); None stands for the identity.
    Modes are applied in the order 1..d."""
    if len(Ls) != T.ndim:
        raise ValueError("one matrix per mode")
    S = T
    for mu, L in enumerate(Ls, start=1):
        if L is not None:
            S = mode_product(S, L, mu)
    return S


def kron_sum_action(T: np.ndarray, As: Sequence[np.ndarray]) -> np.ndarray:
    """K t in tensor form, eq. (kronsumv): sum_mu T x_mu A_mu."""
    S = np.zeros_like(T)
    for mu, A in enumerate(As, start=1):
        S = S + mode_product(T, A, mu)
    return S
