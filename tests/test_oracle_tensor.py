"""Pins for the oracle's mu-mode product, Tucker operator and K action.

* brute force with explicit loops on tiny tensors (the elementwise definition
  of the mu-mode product, Section 2);
* the Kronecker identity eq. (krontomu): (L_d x ... x L_1) vec(T) = vec(T x_1 L_1 ... x_d L_d),
  with the Kronecker product built by numpy.kron;
* the 2-D case is L_1 V L_2^T (eq. exp2d);
* K vec(T) for the dense Kronecker sum K = sum_mu I x .. x A_mu x .. x I
  (eq. kronsum) equals eq. (kronsumv).
"""
import itertools
from functools import reduce

import numpy as np
import pytest

from oracle import tensor
from workloads import random_matrix, random_tensor


def _vec(T):
    return T.ravel(order="F")


def _kron_chain(Ls):
    """L_d x ... x L_1 for the list [L_1, ..., L_d]."""
    return reduce(np.kron, Ls[::-1])


def test_mode_product_elementwise_loops():
    dims = (3, 4, 2)
    T = random_tensor(dims, 11)
    for mu in (1, 2, 3):
        n = dims[mu - 1]
        L = random_matrix(n, 20 + mu)
        S = tensor.mode_product(T, L, mu)
        for idx in itertools.product(*[range(m) for m in dims]):
            acc = 0.0
            for j in range(n):
                src = list(idx)
                src[mu - 1] = j
                acc += T[tuple(src)] * L[idx[mu - 1], j]
            assert abs(S[idx] - acc) < 1e-14


@pytest.mark.parametrize("dims", [(3, 4, 5), (6, 7), (2, 3, 2, 3), (5,)])
def test_tucker_matches_kronecker(dims):
    T = random_tensor(dims, 3)
    Ls = [random_matrix(n, 100 + k) for k, n in enumerate(dims)]
    lhs = _kron_chain(Ls) @ _vec(T)
    rhs = _vec(tensor.tucker(T, Ls))
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(lhs))


def test_tucker_identity_entries():
    T = random_tensor((4, 5, 6), 5)
    L2 = random_matrix(5, 8)
    a = tensor.tucker(T, [None, L2, None])
    b = tensor.mode_product(T, L2, 2)
    assert np.array_equal(a, b)


def test_two_d_is_matrix_sandwich():
    V = random_tensor((6, 9), 4)
    L1, L2 = random_matrix(6, 1), random_matrix(9, 2)
    assert np.allclose(tensor.tucker(V, [L1, L2]), L1 @ V @ L2.T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dims", [(3, 4, 5), (5, 6)])
def test_kron_sum_action_dense(dims):
    T = random_tensor(dims, 9)
    As = [random_matrix(n, 50 + k) for k, n in enumerate(dims)]
    K = np.zeros((T.size, T.size))
    for mu in range(len(dims)):
        mats = [np.eye(n) for n in dims]
        mats[mu] = As[mu]
        K += _kron_chain(mats)
    lhs = K @ _vec(T)
    rhs = _vec(tensor.kron_sum_action(T, As))
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(lhs))


def test_mode_product_rejects_bad_shape():
    with pytest.raises(ValueError):
        tensor.mode_product(np.zeros((3, 4)), np.zeros((3, 3)), 2)
