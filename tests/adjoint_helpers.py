"""Test helpers for adjoints: brute-force core adjoints of a linear
functional of a TT."""
import numpy as np


def full_vjp(cores, t):
    """Core adjoints of f = <full(cores), t> by brute-force contraction of
    each core's left and right environments with the dense tensor t."""
    d = len(cores)
    out = []
    for k in range(d):
        left = np.ones((1, 1))
        for j in range(k):
            left = np.einsum("xa,aib->xib", left, cores[j]).reshape(-1, cores[j].shape[2])
        right = np.ones((1, 1))
        for j in range(d - 1, k, -1):
            right = np.einsum("aib,bx->aix", cores[j], right).reshape(cores[j].shape[0], -1)
        tk = t.reshape(left.shape[0], cores[k].shape[1], right.shape[1])
        out.append(np.einsum("la,lir,br->aib", left, tk, right))
    return out
