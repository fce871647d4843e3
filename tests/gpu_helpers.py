"""Shared helpers of the GPU tests (not collected)."""
import numpy as np

from oracle import tt as ttm


def rand_pos_tt(rng, n, r):
    rk = [1] + list(r) + [1]
    return [np.abs(rng.standard_normal((rk[k], n[k], rk[k + 1]))) + 0.05 for k in range(len(n))]


def caps_of(cores, extra=0):
    return [1] + [g.shape[2] + extra for g in cores[:-1]] + [1]


def to_dev(B, cores, dtype, cap=None, log_scale=0.0):
    n = [g.shape[1] for g in cores]
    t = B.DeviceTT(n, cap or caps_of(cores), dtype)
    t.load(cores, log_scale)
    return t


def fetch_full(t):
    cores, st = t.fetch_scaled()
    return ttm.full(cores), cores, st
