"""Thin ctypes binding of libttgbf.so (include/ttgbf.h).

Argument marshalling only: every numerical step runs in the HIP library.
PyTorch supplies device memory and the stream.  Importing this module loads
the library and raises if it is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttgbf.so")

MAXD = 16
F64, F32 = 0, 1
OK, ERR_ARG, ERR_SHAPE, ERR_WORKSPACE, ERR_HIP = 0, 1, 2, 3, 4
STATUS_NONPOSITIVE, STATUS_NONFINITE, STATUS_CAPACITY = 1, 2, 4
STATE_SAVE, STATE_LOAD = 0, 1


class Grid(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int32 * MAXD), ("lo", C.c_double * MAXD),
                ("hi", C.c_double * MAXD)]


class Train(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int32 * MAXD), ("cap", C.c_int32 * (MAXD + 1)),
                ("dtype", C.c_int32), ("cores", C.c_void_p), ("ranks", C.c_void_p),
                ("log_scale", C.c_void_p), ("status", C.c_void_p)]


class Meas(C.Structure):
    _fields_ = [("kind", C.c_int32), ("sensor", C.c_double * 2), ("sigma_r", C.c_double),
                ("sigma_lin", C.c_double), ("lik_tol", C.c_double), ("lik_max_rank", C.c_int32)]


class FilterSpec(C.Structure):
    _fields_ = [("grid", Grid), ("meas", Meas), ("m0", C.c_double * MAXD),
                ("p0_diag", C.c_double * MAXD), ("cap", C.c_int32), ("eps", C.c_double),
                ("kernel_index", C.c_int32), ("kernel_cap", C.c_int32),
                ("lik_rank_cap", C.c_int32)]


class Monitor(C.Structure):
    _fields_ = [("marg_min_dev", C.c_void_p), ("tail_dev", C.c_void_p)]


class GradSpec(C.Structure):
    _fields_ = [("f", FilterSpec), ("q", C.c_double * (MAXD * MAXD)), ("halfwidths", C.c_int32 * MAXD),
                ("kernel_tol", C.c_double)]


class RoundTapeStruct(C.Structure):
    _fields_ = [("g", C.c_void_p * MAXD), ("f", C.c_void_p * MAXD), ("v", C.c_void_p * MAXD),
                ("s", C.c_void_p * MAXD), ("valid", C.c_void_p), ("rank", C.c_void_p)]


class TTError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2501_07942_amd.build`")
    # torch first: the library then binds to the HIP runtime torch already
    # loaded, so both see the same devices and streams whatever the caller's
    # import order (loaded the other way round, the library's runtime found
    # no device)
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, S, I, D = C.c_void_p, C.c_size_t, C.c_int32, C.c_double
    sigs = {
        "tt_train_elems": (S, [I, P, P]),
        "tt_last_error": (C.c_char_p, []),
        "tt_version": (C.c_char_p, []),
        "tt_kernel_build_workspace": (S, [P, P, P]),
        "tt_kernel_build": (I, [P, P, P, D, P, P, S, P]),
        "tt_predict_workspace": (S, [I]),
        "tt_predict": (I, [I, P, P, P, P, S, P]),
        "tt_update_workspace": (S, [I, P, P, P, P, I]),
        "tt_update": (I, [I, P, P, P, I, P, P, I, P, P, S, P]),
        "tt_round_workspace": (S, [I, P, P]),
        "tt_round": (I, [I, P, P, D, I, P, S, P]),
        "tt_normalize_moments_workspace": (S, [I, P]),
        "tt_normalize_moments": (I, [I, P, P, P, P, P, P, S, P]),
        "tt_filter_run_workspace": (S, [I, P, P, I, I]),
        "tt_profile_begin": (None, [I]),
        "tt_set_predict_mode": (I, [I]),
        "tt_get_predict_mode": (I, []),
        "tt_profile_end": (I, [P, P, P, P, I]),
        "tt_filter_run": (I, [I, P, P, I, P, I, I, I, I, I, P, P, P, P, P, P, P, P, P, P, P, S, P]),
        "tt_filter_run_monitored": (I, [I, P, P, I, P, I, I, I, I, I, P, P, P, P, P, P, P, P, P, P, P, P, S, P]),
        "tt_marginal_min_workspace": (S, [I, P]),
        "tt_normalize_moments_adjoint_workspace": (S, [I, P]),
        "tt_update_adjoint_workspace": (S, [I, P, P, P, P, I]),
        "tt_update_adjoint": (I, [I, P, P, P, I, P, P, P, P, I, P, P, P, S, P]),
        "tt_normalize_moments_adjoint": (I, [I, P, P, P, P, P, P, P, P, S, P]),
        "tt_marginal_min": (I, [I, P, P, P, S, P]),
        "tt_filter_graph_create": (I, [I, P, P, I, P, I, I, I, I, I, P, P, P, P, P, P, P, P, P, P, P, S, P,
                                       C.POINTER(C.c_void_p)]),
        "tt_filter_graph_launch": (I, [P, P]),
        "tt_adjoint_workspace": (S, [I, I, I]),
        "tt_round_adjoint_workspace": (S, [I, P, P]),
        "tt_round_adjoint": (I, [I, P, P, P, P, P, P, S, P]),
        "tt_round_taped": (I, [I, P, P, D, I, P, P, S, P]),
        "tt_predict_einsum_workspace": (S, [I, P, P]),
        "tt_predict_einsum": (I, [I, P, P, P, P, S, P]),
        "tt_grid_redesign_workspace": (S, [I, I]),
        "tt_grid_redesign": (I, [I, I, P, P, D, P, P, P, P, P, S, P]),
        "tt_interpolate_workspace": (S, [I]),
        "tt_interpolate": (I, [I, P, P, P, P, P, S, P]),
        "tt_prior": (I, [I, P, P, P, P, P, S, P]),
        "tt_likelihood": (I, [I, P, P, P, I, P, I, P, S, P]),
        "tt_kernel_build_batch_workspace": (S, [I, P, P, P]),
        "tt_kernel_build_batch": (I, [I, P, P, P, D, P, P, S, P]),
        "tt_likelihood_dense": (I, [I, P, P, P, I, P, P, S, P]),
        "tt_likelihood_adjoint_workspace": (S, [I, P, P, P]),
        "tt_likelihood_adjoint": (I, [I, P, P, P, P, P, P, S, P]),
        "tt_adjoint_axpy": (I, [I, D, P, P, P, S, P]),
        "tt_adjoint_inner": (I, [I, P, P, P, P, S, P]),
        "tt_align_signs": (I, [I, P, P, P, S, P]),
        "tt_predict_adjoint": (I, [I, P, P, P, P, P, P, S, P]),
        "tt_hadamard_adjoint": (I, [I, P, P, P, P, P, P, S, P]),
        "tt_normalize_adjoint": (I, [I, P, P, P, P, P, S, P]),
        "tt_autotune_prediction": (I, [I, P, P, I, P, I, I, I, P, P, P, P, P, S, P, I, I, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_float)]),
        "tt_filter_graph_destroy": (None, [P]),
        "tt_filter_state": (I, [I, P, P, I, I, I, P, P, S, P]),
        "tt_normalize_moments_noalloc": (I, [I, P, P, P, P, P, P]),
        "tt_kernel_build_cross_workspace": (S, [I, P, P, P]),
        "tt_kernel_build_cross": (I, [I, P, P, P, D, I, P, P, S, P]),
        "tt_interpolate_lattice_workspace": (S, [I, P, P, I]),
        "tt_interpolate_lattice": (I, [I, P, P, P, P, D, I, P, P, S, P]),
        "tt_filter_run_linear_workspace": (S, [I, P, I]),
        "tt_filter_run_linear": (I, [I, P, P, P, D, D, D, P, I, I, P, P, P, P, P, P, P, P, S, P]),
        "tt_filter_grad_workspace": (S, [I, P, I, I]),
        "tt_filter_run_taped": (I, [I, P, P, I, I, I, P, P, P, S, P]),
        "tt_filter_run_adjoint": (I, [I, P, P, I, I, I, P, P, P, P, S, P]),
        "tt_autotune_save": (I, [C.c_char_p]),
        "tt_autotune_load": (I, [C.c_char_p, C.POINTER(C.c_int32)]),
        "tt_status_string": (C.c_char_p, [I]),
        "tt_device_status_string": (C.c_char_p, [I]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()
EXPORTED = ("tt_train_elems", "tt_last_error", "tt_version", "tt_kernel_build_workspace",
            "tt_kernel_build", "tt_predict_workspace", "tt_predict", "tt_update_workspace",
            "tt_update", "tt_round_workspace", "tt_round", "tt_normalize_moments_workspace",
            "tt_normalize_moments", "tt_filter_run_workspace", "tt_filter_run", "tt_profile_begin",
            "tt_profile_end", "tt_set_predict_mode", "tt_get_predict_mode", "tt_filter_graph_create",
            "tt_filter_graph_launch", "tt_filter_graph_destroy", "tt_autotune_prediction",
            "tt_adjoint_workspace", "tt_predict_adjoint", "tt_hadamard_adjoint", "tt_normalize_adjoint",
            "tt_round_adjoint_workspace", "tt_round_adjoint", "tt_prior", "tt_likelihood", "tt_likelihood_dense",
            "tt_kernel_build_batch_workspace", "tt_kernel_build_batch",
            "tt_likelihood_adjoint_workspace", "tt_likelihood_adjoint", "tt_adjoint_axpy",
            "tt_adjoint_inner", "tt_align_signs", "tt_round_taped", "tt_predict_einsum_workspace",
            "tt_predict_einsum", "tt_grid_redesign_workspace", "tt_grid_redesign", "tt_interpolate_workspace",
            "tt_interpolate", "tt_filter_state", "tt_status_string", "tt_device_status_string",
            "tt_normalize_moments_noalloc", "tt_autotune_save", "tt_autotune_load", "tt_filter_grad_workspace",
            "tt_filter_run_taped", "tt_filter_run_adjoint", "tt_kernel_build_cross_workspace",
            "tt_kernel_build_cross", "tt_interpolate_lattice_workspace", "tt_interpolate_lattice",
            "tt_filter_run_linear_workspace", "tt_filter_run_linear", "tt_filter_run_monitored",
            "tt_marginal_min_workspace", "tt_marginal_min", "tt_normalize_moments_adjoint_workspace",
            "tt_normalize_moments_adjoint", "tt_update_adjoint_workspace", "tt_update_adjoint")

PREDICT_DIRECT, PREDICT_FFT, PREDICT_UNFUSED, PREDICT_DIRECT_VALU = 0, 1, 2, 3


def filter_run_linear(fspecs: Sequence[FilterSpec], f: np.ndarray, q: np.ndarray, z, nsigma: float = 4.0,
                      kernel_nsigma: float = 4.0, kernel_tol: float = 1e-12) -> dict:
    """tt_filter_run_linear over a batch (z: float64 device [B, K, zdim]);
    returns device tensors loglik, log_c, log_mpred, mean, cov, status and
    the host array grids [B, K, 2d] (lo, hi of each step's grid)."""
    torch = _torch()
    B = len(fspecs)
    K, zdim = int(z.shape[1]), int(z.shape[2])
    d = fspecs[0].grid.d
    arr = (FilterSpec * B)(*fspecs)
    nbytes = LIB.tt_filter_run_linear_workspace(B, arr, K)
    if nbytes == 0:
        _check(ERR_ARG, "tt_filter_run_linear_workspace")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dev = lambda *shape: torch.zeros(*shape, dtype=torch.float64, device="cuda")  # noqa: E731
    out = {"loglik": dev(B), "log_c": dev(B, K), "log_mpred": dev(B, K), "mean": dev(B, K, d), "cov": dev(B, K, d, d),
           "status": torch.zeros(B, dtype=torch.int32, device="cuda")}
    grids = np.zeros((B, K, 2 * d))
    ff = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
    qq = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
    _check(LIB.tt_filter_run_linear(B, arr, ff.ctypes.data_as(C.c_void_p), qq.ctypes.data_as(C.c_void_p),
                                    float(nsigma), float(kernel_nsigma), float(kernel_tol), z.data_ptr(), zdim, K,
                                    out["loglik"].data_ptr(), out["log_c"].data_ptr(), out["log_mpred"].data_ptr(),
                                    out["mean"].data_ptr(), out["cov"].data_ptr(), grids.ctypes.data_as(C.c_void_p),
                                    out["status"].data_ptr(), ws.data_ptr(), ws.numel(), _stream()),
           "tt_filter_run_linear")
    out["grids"] = grids
    return out


class FilterGrad:
    """tt_filter_run_taped / tt_filter_run_adjoint for a batch of GradSpec:
    the workspace (kernels, tape or checkpoints, temporaries) lives as long
    as this object.  z: float64 device tensor [B, K, zdim]."""

    def __init__(self, gspecs: Sequence[GradSpec], z, ckpt_every: int = 1):
        torch = _torch()
        self.B = len(gspecs)
        self.specs = (GradSpec * self.B)(*gspecs)
        self.z = z
        self.K, self.zdim = int(z.shape[1]), int(z.shape[2])
        self.C = int(ckpt_every)
        d = gspecs[0].f.grid.d
        self.n_theta = d + 4 if gspecs[0].f.meas.kind == 1 else d + 1
        nbytes = LIB.tt_filter_grad_workspace(self.B, self.specs, self.K, self.C)
        if nbytes == 0:
            _check(ERR_ARG, "tt_filter_grad_workspace")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.loglik = torch.zeros(self.B, dtype=torch.float64, device="cuda")
        self.theta_bar = torch.zeros(self.B, self.n_theta, dtype=torch.float64, device="cuda")
        self.status = torch.zeros(self.B, dtype=torch.int32, device="cuda")

    def forward(self):
        """LL [B] (device); keeps what the reverse sweep needs."""
        self.status.zero_()
        _check(LIB.tt_filter_run_taped(self.B, self.specs, self.z.data_ptr(), self.zdim, self.K, self.C,
                                       self.loglik.data_ptr(), self.status.data_ptr(), self.ws.data_ptr(),
                                       self.ws.numel(), _stream()), "tt_filter_run_taped")
        return self.loglik

    def backward(self, loglik_bar):
        """theta_bar [B, n_theta] = loglik_bar[b] * dLL_b/dtheta (device)."""
        lb = loglik_bar.to(dtype=_torch().float64).contiguous()
        _check(LIB.tt_filter_run_adjoint(self.B, self.specs, self.z.data_ptr(), self.zdim, self.K, self.C,
                                         lb.data_ptr(), self.theta_bar.data_ptr(), self.status.data_ptr(),
                                         self.ws.data_ptr(), self.ws.numel(), _stream()), "tt_filter_run_adjoint")
        return self.theta_bar


def autotune_save(path: str):
    """tt_autotune_save: the tuned launch shapes of this process as JSON."""
    _check(LIB.tt_autotune_save(os.fsencode(path)), "tt_autotune_save")


def autotune_load(path: str) -> int:
    """tt_autotune_load: adopt the shapes a previous run saved for this
    device's architecture; returns how many were adopted."""
    n = C.c_int32(0)
    _check(LIB.tt_autotune_load(os.fsencode(path), C.byref(n)), "tt_autotune_load")
    return int(n.value)


def set_predict_mode(mode: int):
    _check(LIB.tt_set_predict_mode(int(mode)), "tt_set_predict_mode")

PROFILE_CLASSES = ("conv", "hadamard", "gram", "pchol", "jacobi", "trsm", "gemm", "lik", "contract", "pred",
                   "einsum", "interp")


def profile_begin(classes=PROFILE_CLASSES):
    mask = 0
    for c in classes:
        mask |= 1 << PROFILE_CLASSES.index(c)
    LIB.tt_profile_begin(mask)


def profile_end():
    """{class: (total ms, launches, algorithmic flops, algorithmic bytes)} of
    the launches since profile_begin (work is 0 for classes without a model)."""
    n = len(PROFILE_CLASSES)
    ms = (C.c_double * n)()
    cnt = (C.c_int32 * n)()
    fl = (C.c_double * n)()
    by = (C.c_double * n)()
    if LIB.tt_profile_end(ms, cnt, fl, by, n) < 0:
        raise TTError(LIB.tt_last_error().decode())
    return {PROFILE_CLASSES[i]: (ms[i], cnt[i], fl[i], by[i]) for i in range(n)}


def _check(st: int, what: str):
    if st != OK:
        raise TTError(f"{what} failed ({LIB.tt_status_string(st).decode()}): {LIB.tt_last_error().decode()}")


def status_string(code: int) -> str:
    return LIB.tt_status_string(int(code)).decode()


def device_status_string(bits: int) -> str:
    return LIB.tt_device_status_string(int(bits)).decode()


def _torch():
    import torch  # imported lazily so that the CPU-only symbol test needs no GPU
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _arr(structs):
    arr_t = type(structs[0]) * len(structs)
    return arr_t(*structs)


def make_grid(d: int, n: Sequence[int], lo: Sequence[float], hi: Sequence[float]) -> Grid:
    g = Grid()
    g.d = d
    for l in range(d):
        g.n[l] = int(n[l])
        g.lo[l] = float(lo[l])
        g.hi[l] = float(hi[l])
    return g


def make_meas(kind: int, sensor=(0.0, 0.0), sigma_r=1.0, sigma_lin=1.0, lik_tol=1e-12,
              lik_max_rank=0) -> Meas:
    m = Meas()
    m.kind = kind
    m.sensor[0], m.sensor[1] = float(sensor[0]), float(sensor[1])
    m.sigma_r = float(sigma_r)
    m.sigma_lin = float(sigma_lin)
    m.lik_tol = float(lik_tol)
    m.lik_max_rank = int(lik_max_rank)
    return m


class DeviceTT:
    """A TT whose cores, ranks, log-scale and status live in torch device
    tensors.  Layout of core k: [r_{k-1}][n_k][r_k] packed with the current
    ranks at offset sum_{j<k} cap[j]*n[j]*cap[j+1]."""

    def __init__(self, n: Sequence[int], cap: Sequence[int], dtype: int = F64, device="cuda"):
        torch = _torch()
        total = self._layout(n, cap, dtype)
        tdt = torch.float64 if dtype == F64 else torch.float32
        self.cores = torch.zeros(total, dtype=tdt, device=device)
        self.ranks = torch.ones(self.d + 1, dtype=torch.int32, device=device)
        self.log_scale = torch.zeros(1, dtype=torch.float64, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)

    def _layout(self, n: Sequence[int], cap: Sequence[int], dtype: int) -> int:
        self.d = len(n)
        self.n = [int(x) for x in n]
        self.cap = [int(x) for x in cap]
        assert len(self.cap) == self.d + 1 and self.cap[0] == 1 and self.cap[-1] == 1
        self.dtype = dtype
        self.offsets = []
        off = 0
        for k in range(self.d):
            self.offsets.append(off)
            off += self.cap[k] * self.n[k] * self.cap[k + 1]
        return max(off, 1)

    @classmethod
    def batch(cls, ns: Sequence[Sequence[int]], caps: Sequence[Sequence[int]], dtype: int = F64,
              device="cuda") -> List["DeviceTT"]:
        """Several TTs whose cores, ranks, log-scales and statuses are views of
        four shared allocations (each core buffer starts 512-byte aligned)."""
        torch = _torch()
        objs = [cls.__new__(cls) for _ in ns]
        totals = [o._layout(n, c, dtype) for o, n, c in zip(objs, ns, caps)]
        starts, pos = [], 0
        for t in totals:
            starts.append(pos)
            pos += (t + 127) // 128 * 128
        tdt = torch.float64 if dtype == F64 else torch.float32
        cores = torch.zeros(max(pos, 1), dtype=tdt, device=device)
        dmax = max(o.d for o in objs) + 1
        ranks = torch.ones((len(objs), dmax), dtype=torch.int32, device=device)
        logs = torch.zeros(len(objs), dtype=torch.float64, device=device)
        status = torch.zeros(len(objs), dtype=torch.int32, device=device)
        for b, (o, st, t) in enumerate(zip(objs, starts, totals)):
            o.cores = cores[st:st + t]
            o.ranks = ranks[b, :o.d + 1]
            o.log_scale = logs[b:b + 1]
            o.status = status[b:b + 1]
        return objs

    def struct(self) -> Train:
        t = Train()
        t.d = self.d
        for k in range(self.d):
            t.n[k] = self.n[k]
        for j in range(self.d + 1):
            t.cap[j] = self.cap[j]
        t.dtype = self.dtype
        t.cores = self.cores.data_ptr()
        t.ranks = self.ranks.data_ptr()
        t.log_scale = self.log_scale.data_ptr()
        t.status = self.status.data_ptr()
        return t

    def load(self, cores: List[np.ndarray], log_scale: float = 0.0):
        """Copy host cores (list of (r0, n, r1) arrays) into the device TT."""
        torch = _torch()
        host = torch.zeros_like(self.cores, device="cpu")
        for k, g in enumerate(cores):
            r0, n, r1 = g.shape
            if r0 > self.cap[k] or r1 > self.cap[k + 1] or n != self.n[k]:
                raise ValueError(f"core {k} {g.shape} exceeds capacity {self.cap[k]}x{self.n[k]}x{self.cap[k+1]}")
            flat = torch.from_numpy(np.ascontiguousarray(g).ravel()).to(host.dtype)
            host[self.offsets[k]:self.offsets[k] + flat.numel()] = flat
        self.cores.copy_(host)
        rk = [1] + [g.shape[2] for g in cores]
        self.ranks.copy_(torch.tensor(rk, dtype=torch.int32))
        self.log_scale.fill_(float(log_scale))
        self.status.zero_()

    def fetch(self):
        """(cores, log_scale, status) as host FP64 arrays."""
        rk = self.ranks.cpu().numpy().tolist()
        data = self.cores.cpu().double().numpy()
        cores = []
        for k in range(self.d):
            r0, r1 = rk[k], rk[k + 1]
            sz = r0 * self.n[k] * r1
            cores.append(data[self.offsets[k]:self.offsets[k] + sz].reshape(r0, self.n[k], r1).copy())
        return cores, float(self.log_scale.cpu().item()), int(self.status.cpu().item())

    def fetch_scaled(self):
        """Cores with exp(log_scale) folded into the first core."""
        cores, ls, st = self.fetch()
        cores[0] = cores[0] * math.exp(ls)
        return cores, st


def _ws(nbytes: int):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def tt_kernel_build(grid: Grid, q: np.ndarray, halfwidths: Sequence[int], svd_tol: float, out: DeviceTT):
    d = grid.d
    hw = (C.c_int32 * d)(*[int(h) for h in halfwidths])
    qq = (C.c_double * (d * d))(*np.asarray(q, dtype=np.float64).ravel().tolist())
    capa = (C.c_int32 * (d + 1))(*out.cap)
    nbytes = LIB.tt_kernel_build_workspace(C.byref(grid), hw, capa)
    if nbytes == 0:
        _check(ERR_ARG, "tt_kernel_build_workspace")
    ws = _ws(nbytes)
    t = out.struct()
    _check(LIB.tt_kernel_build(C.byref(grid), qq, hw, float(svd_tol), C.byref(t), ws.data_ptr(),
                               ws.numel(), _stream()), "tt_kernel_build")
    return out


def tt_kernel_build_batch(grids: Sequence[Grid], qs: Sequence[np.ndarray], halfwidths: Sequence[int],
                          svd_tol: float, outs: Sequence[DeviceTT]):
    """tt_kernel_build for several kernels sharing d and the offset box."""
    B = len(outs)
    d = grids[0].d
    hw = (C.c_int32 * d)(*[int(h) for h in halfwidths])
    qq = np.ascontiguousarray(np.stack([np.asarray(q, dtype=np.float64).reshape(d, d) for q in qs]))
    caps = (C.c_int32 * (B * (d + 1)))(*[int(c) for o in outs for c in o.cap])
    g = _arr(list(grids))
    nbytes = LIB.tt_kernel_build_batch_workspace(B, g, hw, caps)
    if nbytes == 0:
        _check(ERR_ARG, "tt_kernel_build_batch_workspace")
    ws = _ws(nbytes)
    _check(LIB.tt_kernel_build_batch(B, g, qq.ctypes.data_as(C.c_void_p), hw, float(svd_tol),
                                     _arr([o.struct() for o in outs]), ws.data_ptr(), ws.numel(), _stream()),
           "tt_kernel_build_batch")
    return outs


def tt_predict(kernels: Sequence[DeviceTT], p_in: Sequence[DeviceTT], p_out: Sequence[DeviceTT]):
    B = len(p_in)
    ks, ps, xs = _arr([k.struct() for k in kernels]), _arr([p.struct() for p in p_in]), _arr([x.struct() for x in p_out])
    ws = _ws(LIB.tt_predict_workspace(B))
    _check(LIB.tt_predict(B, ks, ps, xs, ws.data_ptr(), ws.numel(), _stream()), "tt_predict")


def tt_kernel_build_cross(grids: Sequence[Grid], qs: Sequence[np.ndarray], halfwidths: Sequence[int],
                          svd_tol: float, outs: Sequence[DeviceTT], max_rank: int = 64):
    """The kernel TT by deterministic TT-cross from point values (any d)."""
    B = len(outs)
    d = grids[0].d
    hw = (C.c_int32 * d)(*[int(h) for h in halfwidths])
    qq = np.ascontiguousarray(np.stack([np.asarray(q, dtype=np.float64).reshape(d, d) for q in qs]))
    g, o = _arr(list(grids)), _arr([t.struct() for t in outs])
    nbytes = LIB.tt_kernel_build_cross_workspace(B, g, hw, o)
    if nbytes == 0:
        _check(ERR_ARG, "tt_kernel_build_cross_workspace")
    ws = _ws(nbytes)
    _check(LIB.tt_kernel_build_cross(B, g, qq.ctypes.data_as(C.c_void_p), hw, float(svd_tol), int(max_rank), o,
                                     ws.data_ptr(), ws.numel(), _stream()), "tt_kernel_build_cross")


def tt_interpolate_lattice(f: np.ndarray, lattice: Sequence[Grid], to: Sequence[Grid], t_in: Sequence[DeviceTT],
                           t_out: Sequence[DeviceTT], tol: float = 1e-12, max_rank: int = 64):
    """Weights on the lattice F xi(lattice) interpolated onto the grids `to`."""
    B = len(t_in)
    ff = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
    tg, o = _arr(list(to)), _arr([t.struct() for t in t_out])
    nbytes = LIB.tt_interpolate_lattice_workspace(B, tg, o, int(max_rank))
    if nbytes == 0:
        _check(ERR_ARG, "tt_interpolate_lattice_workspace")
    ws = _ws(nbytes)
    _check(LIB.tt_interpolate_lattice(B, ff.ctypes.data_as(C.c_void_p), _arr(list(lattice)), tg,
                                      _arr([t.struct() for t in t_in]), float(tol), int(max_rank), o, ws.data_ptr(),
                                      ws.numel(), _stream()), "tt_interpolate_lattice")


def tt_update(grids: Sequence[Grid], meas: Sequence[Meas], z, p_pred: Sequence[DeviceTT],
              h_out: Sequence[DeviceTT], lik_rank_cap: int, log_c):
    """z: torch float64 device tensor [B, zdim]; log_c: torch float64 device [B]."""
    B = len(p_pred)
    g, m = _arr(list(grids)), _arr(list(meas))
    ps, hs = _arr([p.struct() for p in p_pred]), _arr([h.struct() for h in h_out])
    nbytes = LIB.tt_update_workspace(B, g, m, ps, hs, int(lik_rank_cap))
    if nbytes == 0:
        _check(ERR_ARG, "tt_update_workspace")
    ws = _ws(nbytes)
    _check(LIB.tt_update(B, g, m, z.data_ptr(), int(z.shape[1]), ps, hs, int(lik_rank_cap),
                         log_c.data_ptr(), ws.data_ptr(), ws.numel(), _stream()), "tt_update")


class RoundTape:
    """Record of an FP64 rounding's sweeps, one per filter: for each bond j
    the right-part Gram and its pivoted Cholesky factor, the singular vectors
    of the left-to-right step ending there (c_j x c_j doubles each, c_j the
    input's cap[j], min(cap[1], n[0]) for bond 1) and its singular values, a
    flag set and the factor's rank per bond, all in device memory."""

    def __init__(self, t_in: Sequence[DeviceTT]):
        torch = _torch()
        self.d = t_in[0].d
        # bond 1 of rank above n[0] is folded with the first core: its record
        # is n[0] x n[0] at most
        caps = [[(min(t.cap[1], t.n[0]) if j == 1 else t.cap[j]) if 1 <= j < self.d else 0 for j in range(self.d)]
                for t in t_in]
        self.sizes = [[c * c for c in cc] for cc in caps]
        per = [3 * sum(sz) + sum(c) for sz, c in zip(self.sizes, caps)]
        self.buf = torch.zeros(max(sum(per), 1), dtype=torch.float64, device="cuda")
        self.valid = torch.zeros((len(t_in), self.d + 1), dtype=torch.int32, device="cuda")
        self.rank = torch.zeros((len(t_in), self.d + 1), dtype=torch.int32, device="cuda")
        self.structs = []
        off = 0
        for b, sz in enumerate(self.sizes):
            st = RoundTapeStruct()
            for j in range(1, self.d):
                st.g[j] = self.buf.data_ptr() + 8 * off
                off += sz[j]
                st.f[j] = self.buf.data_ptr() + 8 * off
                off += sz[j]
                st.v[j] = self.buf.data_ptr() + 8 * off
                off += sz[j]
                st.s[j] = self.buf.data_ptr() + 8 * off
                off += caps[b][j]
            st.valid = self.valid.data_ptr() + 4 * b * (self.d + 1)
            st.rank = self.rank.data_ptr() + 4 * b * (self.d + 1)
            self.structs.append(st)

    def select(self, idx: Sequence[int]):
        return [self.structs[i] for i in idx]


def tt_round(t_in: Sequence[DeviceTT], t_out: Sequence[DeviceTT], eps: float, max_rank: int, tape=None):
    """tape: None, or a list of RoundTapeStruct (one per filter, FP64 only)
    that receives the right-to-left record for tt_round_adjoint."""
    B = len(t_in)
    a, b = _arr([t.struct() for t in t_in]), _arr([t.struct() for t in t_out])
    nbytes = LIB.tt_round_workspace(B, a, b)
    if nbytes == 0:
        _check(ERR_ARG, "tt_round_workspace")
    ws = _ws(nbytes)
    if tape is None:
        _check(LIB.tt_round(B, a, b, float(eps), int(max_rank), ws.data_ptr(), ws.numel(), _stream()), "tt_round")
    else:
        assert len(tape) == B
        _check(LIB.tt_round_taped(B, a, b, float(eps), int(max_rank), _arr(list(tape)), ws.data_ptr(), ws.numel(),
                                  _stream()), "tt_round_taped")


def tt_predict_einsum(tpm: Sequence[DeviceTT], p_in: Sequence[DeviceTT], p_out: Sequence[DeviceTT]):
    """P' = sum_j T(i, j) P(j) with T a 2d-core transition train (Alg. 1)."""
    B = len(p_in)
    tt, pp = _arr([t.struct() for t in tpm]), _arr([p.struct() for p in p_in])
    nbytes = LIB.tt_predict_einsum_workspace(B, tt, pp)
    if nbytes == 0:
        _check(ERR_ARG, "tt_predict_einsum_workspace")
    ws = _ws(nbytes)
    _check(LIB.tt_predict_einsum(B, tt, pp, _arr([o.struct() for o in p_out]), ws.data_ptr(), ws.numel(),
                                 _stream()), "tt_predict_einsum")


def tt_grid_redesign(old_grids: Sequence[Grid], f, q, nsigma: float, mean, cov) -> List[Grid]:
    """New filtering grids by Alg. 4.  f, q: host (d, d) float64 arrays;
    mean [B, d], cov [B, d, d]: torch float64 device tensors."""
    B = len(old_grids)
    d = old_grids[0].d
    fa = np.ascontiguousarray(f, dtype=np.float64)
    qa = np.ascontiguousarray(q, dtype=np.float64)
    out = (Grid * B)()
    ws = _ws(LIB.tt_grid_redesign_workspace(B, d))
    _check(LIB.tt_grid_redesign(B, d, fa.ctypes.data, qa.ctypes.data, float(nsigma), mean.data_ptr(), cov.data_ptr(),
                                _arr(list(old_grids)), out, ws.data_ptr(), ws.numel(), _stream()), "tt_grid_redesign")
    return list(out)


def tt_interpolate(from_grids: Sequence[Grid], to_grids: Sequence[Grid], t_in: Sequence[DeviceTT],
                   t_out: Sequence[DeviceTT]):
    B = len(t_in)
    ws = _ws(LIB.tt_interpolate_workspace(B))
    _check(LIB.tt_interpolate(B, _arr(list(from_grids)), _arr(list(to_grids)), _arr([t.struct() for t in t_in]),
                              _arr([t.struct() for t in t_out]), ws.data_ptr(), ws.numel(), _stream()),
           "tt_interpolate")


def tt_normalize_moments(grids: Sequence[Grid], tts: Sequence[DeviceTT], log_mass, mean=None, cov=None):
    B = len(tts)
    g, a = _arr(list(grids)), _arr([t.struct() for t in tts])
    ws = _ws(LIB.tt_normalize_moments_workspace(B, a))
    _check(LIB.tt_normalize_moments(B, g, a, log_mass.data_ptr(), mean.data_ptr() if mean is not None else None,
                                    cov.data_ptr() if cov is not None else None, ws.data_ptr(), ws.numel(),
                                    _stream()), "tt_normalize_moments")


def tt_normalize_moments_noalloc(grids: Sequence[Grid], tts: Sequence[DeviceTT], log_mass, mean=None, cov=None):
    """tt_normalize_moments on the library's static scratch (allocates nothing)."""
    B = len(tts)
    g, a = _arr(list(grids)), _arr([t.struct() for t in tts])
    _check(LIB.tt_normalize_moments_noalloc(B, g, a, log_mass.data_ptr(),
                                            mean.data_ptr() if mean is not None else None,
                                            cov.data_ptr() if cov is not None else None, _stream()),
           "tt_normalize_moments_noalloc")


def _adj_ws(tts):
    B = len(tts)
    d = tts[0].d
    rcap = max(max(t.cap) for t in tts)
    return _ws(LIB.tt_adjoint_workspace(B, d, rcap))


def tt_predict_adjoint(kernels: Sequence[DeviceTT], p_in: Sequence[DeviceTT], c_bar: Sequence[DeviceTT],
                       p_bar: Sequence[DeviceTT], k_bar: Sequence[DeviceTT]):
    B = len(p_in)
    ws = _adj_ws(list(p_in) + list(c_bar) + list(kernels))
    _check(LIB.tt_predict_adjoint(B, _arr([k.struct() for k in kernels]), _arr([p.struct() for p in p_in]),
                                  _arr([c.struct() for c in c_bar]), _arr([p.struct() for p in p_bar]),
                                  _arr([k.struct() for k in k_bar]), ws.data_ptr(), ws.numel(), _stream()),
           "tt_predict_adjoint")


def tt_hadamard_adjoint(a: Sequence[DeviceTT], b: Sequence[DeviceTT], h_bar: Sequence[DeviceTT],
                        a_bar: Optional[Sequence[DeviceTT]], b_bar: Optional[Sequence[DeviceTT]]):
    B = len(b)
    ws = _adj_ws(list(a) + list(b) + list(h_bar))
    _check(LIB.tt_hadamard_adjoint(B, _arr([t.struct() for t in a]), _arr([t.struct() for t in b]),
                                   _arr([t.struct() for t in h_bar]),
                                   _arr([t.struct() for t in a_bar]) if a_bar else None,
                                   _arr([t.struct() for t in b_bar]) if b_bar else None,
                                   ws.data_ptr(), ws.numel(), _stream()), "tt_hadamard_adjoint")


def tt_normalize_adjoint(x: Sequence[DeviceTT], p_bar: Sequence[DeviceTT], log_mass_bar, x_bar: Sequence[DeviceTT]):
    """log_mass_bar: torch float64 device tensor [B] or None."""
    B = len(x)
    ws = _adj_ws(list(x))
    _check(LIB.tt_normalize_adjoint(B, _arr([t.struct() for t in x]), _arr([t.struct() for t in p_bar]),
                                    log_mass_bar.data_ptr() if log_mass_bar is not None else None,
                                    _arr([t.struct() for t in x_bar]), ws.data_ptr(), ws.numel(), _stream()),
           "tt_normalize_adjoint")


def tt_round_adjoint(a: Sequence[DeviceTT], y: Sequence[DeviceTT], y_bar: Sequence[DeviceTT],
                     a_bar: Sequence[DeviceTT], tape=None):
    """tape: None, or the RoundTapeStruct list tt_round filled for this rounding."""
    B = len(a)
    aa, yy = _arr([t.struct() for t in a]), _arr([t.struct() for t in y])
    nbytes = LIB.tt_round_adjoint_workspace(B, aa, yy)
    if nbytes == 0:
        _check(ERR_ARG, "tt_round_adjoint_workspace")
    ws = _ws(nbytes)
    _check(LIB.tt_round_adjoint(B, aa, yy, _arr([t.struct() for t in y_bar]), _arr([t.struct() for t in a_bar]),
                                _arr(list(tape)) if tape is not None else None, ws.data_ptr(), ws.numel(),
                                _stream()), "tt_round_adjoint")


def tt_prior(grids: Sequence[Grid], m0: np.ndarray, p0_diag: np.ndarray, out: Sequence[DeviceTT]):
    B = len(out)
    d = out[0].d
    m = np.ascontiguousarray(np.asarray(m0, dtype=np.float64).reshape(B * d))
    p = np.ascontiguousarray(np.asarray(p0_diag, dtype=np.float64).reshape(B * d))
    ws = _ws(2 * B * 4096 + 4096)
    _check(LIB.tt_prior(B, _arr(list(grids)), m.ctypes.data_as(C.c_void_p), p.ctypes.data_as(C.c_void_p),
                        _arr([t.struct() for t in out]), ws.data_ptr(), ws.numel(), _stream()), "tt_prior")


def tt_likelihood(grids: Sequence[Grid], meas: Sequence[Meas], z, l_out: Sequence[DeviceTT], lik_rank_cap: int):
    """z: float64 device tensor [B, zdim]."""
    B = len(l_out)
    g, m = _arr(list(grids)), _arr(list(meas))
    ls = _arr([t.struct() for t in l_out])
    nbytes = LIB.tt_update_workspace(B, g, m, ls, ls, int(lik_rank_cap))
    if nbytes == 0:
        _check(ERR_ARG, "tt_update_workspace")
    ws = _ws(nbytes)
    _check(LIB.tt_likelihood(B, g, m, z.data_ptr(), int(z.shape[1]), ls, int(lik_rank_cap), ws.data_ptr(),
                             ws.numel(), _stream()), "tt_likelihood")


def tt_normalize_moments_adjoint(grids: Sequence[Grid], x: Sequence[DeviceTT], p_bar: Sequence[DeviceTT],
                                 log_mass_bar, x_bar: Sequence[DeviceTT], mean_bar=None, cov_bar=None):
    """log_mass_bar [B], mean_bar [B, d], cov_bar [B, d, d]: float64 device tensors (the last two nullable)."""
    B = len(x)
    xs = _arr([t.struct() for t in x])
    ws = _ws(LIB.tt_normalize_moments_adjoint_workspace(B, xs))
    _check(LIB.tt_normalize_moments_adjoint(B, _arr(list(grids)), xs, _arr([t.struct() for t in p_bar]),
                                            log_mass_bar.data_ptr() if log_mass_bar is not None else None,
                                            mean_bar.data_ptr() if mean_bar is not None else None,
                                            cov_bar.data_ptr() if cov_bar is not None else None,
                                            _arr([t.struct() for t in x_bar]), ws.data_ptr(), ws.numel(),
                                            _stream()), "tt_normalize_moments_adjoint")


def tt_update_adjoint(grids: Sequence[Grid], meas: Sequence[Meas], z, p_pred: Sequence[DeviceTT],
                      h: Sequence[DeviceTT], h_bar, log_c_bar, lik_rank_cap: int, p_pred_bar: Sequence[DeviceTT],
                      theta_bar):
    """z: float64 device tensor [B, zdim]; h_bar: list of DeviceTT or None;
    log_c_bar [B] (or None) and theta_bar [B, n_theta] float64 device tensors
    (theta_bar is accumulated into)."""
    B = len(p_pred)
    g, m = _arr(list(grids)), _arr(list(meas))
    ps, hs = _arr([t.struct() for t in p_pred]), _arr([t.struct() for t in h])
    nbytes = LIB.tt_update_adjoint_workspace(B, g, m, ps, hs, int(lik_rank_cap))
    if nbytes == 0:
        _check(ERR_ARG, "tt_update_adjoint_workspace")
    ws = _ws(nbytes)
    _check(LIB.tt_update_adjoint(B, g, m, z.data_ptr(), int(z.shape[1]), ps, hs,
                                 _arr([t.struct() for t in h_bar]) if h_bar is not None else None,
                                 log_c_bar.data_ptr() if log_c_bar is not None else None, int(lik_rank_cap),
                                 _arr([t.struct() for t in p_pred_bar]), theta_bar.data_ptr(), ws.data_ptr(),
                                 ws.numel(), _stream()), "tt_update_adjoint")


def tt_marginal_min(tts: Sequence[DeviceTT], out):
    """out: float64 device tensor [B] <- the smallest 1-D marginal value of each TT."""
    B = len(tts)
    a = _arr([t.struct() for t in tts])
    ws = _ws(LIB.tt_marginal_min_workspace(B, a))
    _check(LIB.tt_marginal_min(B, a, out.data_ptr(), ws.data_ptr(), ws.numel(), _stream()), "tt_marginal_min")


def tt_likelihood_dense(grids: Sequence[Grid], meas: Sequence[Meas], z, p_out: Sequence[DeviceTT]):
    """The likelihood before the range block's SVD (bond 1 of full rank n[1]
    for the range model).  z: float64 device tensor [B, zdim]."""
    B = len(p_out)
    g, m = _arr(list(grids)), _arr(list(meas))
    ps = _arr([t.struct() for t in p_out])
    nbytes = LIB.tt_update_workspace(B, g, m, ps, ps, 1)
    if nbytes == 0:
        _check(ERR_ARG, "tt_update_workspace")
    ws = _ws(nbytes)
    _check(LIB.tt_likelihood_dense(B, g, m, z.data_ptr(), int(z.shape[1]), ps, ws.data_ptr(), ws.numel(),
                                   _stream()), "tt_likelihood_dense")


def tt_likelihood_adjoint(meas: Sequence[Meas], p: Sequence[DeviceTT], l: Sequence[DeviceTT],
                          l_bar: Sequence[DeviceTT], p_bar: Sequence[DeviceTT]):
    B = len(p)
    m = _arr(list(meas))
    pp, ll = _arr([t.struct() for t in p]), _arr([t.struct() for t in l])
    nbytes = LIB.tt_likelihood_adjoint_workspace(B, m, pp, ll)
    if nbytes == 0:
        _check(ERR_ARG, "tt_likelihood_adjoint_workspace")
    ws = _ws(nbytes)
    _check(LIB.tt_likelihood_adjoint(B, m, pp, ll, _arr([t.struct() for t in l_bar]),
                                     _arr([t.struct() for t in p_bar]), ws.data_ptr(), ws.numel(), _stream()),
           "tt_likelihood_adjoint")


def tt_adjoint_axpy(alpha: float, x: Sequence[DeviceTT], y: Sequence[DeviceTT]):
    ws = _adj_ws(list(x))
    _check(LIB.tt_adjoint_axpy(len(x), float(alpha), _arr([t.struct() for t in x]), _arr([t.struct() for t in y]),
                               ws.data_ptr(), ws.numel(), _stream()), "tt_adjoint_axpy")


def tt_adjoint_inner(a_bar: Sequence[DeviceTT], b: Sequence[DeviceTT], out):
    """out: float64 device tensor [B]."""
    ws = _adj_ws(list(a_bar))
    _check(LIB.tt_adjoint_inner(len(b), _arr([t.struct() for t in a_bar]), _arr([t.struct() for t in b]),
                                out.data_ptr(), ws.data_ptr(), ws.numel(), _stream()), "tt_adjoint_inner")


def tt_align_signs(ref: Sequence[DeviceTT], t: Sequence[DeviceTT]):
    ws = _adj_ws(list(ref))
    _check(LIB.tt_align_signs(len(t), _arr([x.struct() for x in ref]), _arr([x.struct() for x in t]),
                              ws.data_ptr(), ws.numel(), _stream()), "tt_align_signs")


def workspace_bytes(specs: Sequence[FilterSpec], kernels: Sequence[DeviceTT], precision: int) -> int:
    """tt_filter_run_workspace for a list of specs (no allocation)."""
    n = LIB.tt_filter_run_workspace(len(specs), _arr(list(specs)), _arr([k.struct() for k in kernels]),
                                    len(kernels), precision)
    if n == 0:
        _check(ERR_ARG, "tt_filter_run_workspace")
    return int(n)


class FilterRun:
    """Device buffers and workspace of one batched tt_filter_run call."""

    def __init__(self, specs: Sequence[FilterSpec], kernels: Sequence[DeviceTT], K: int, zdim: int,
                 precision: int, monitor: bool = False):
        """monitor: also record per step the smallest 1-D marginal value of
        the filtering density (marg_min [B, K]) and the relative error bounds
        of both roundings (tails [B, K, 2]) by tt_filter_run_monitored."""
        torch = _torch()
        self.B = len(specs)
        self.K = K
        self.zdim = zdim
        self.precision = precision
        self.specs = _arr(list(specs))
        self.kernels = kernels
        self.karr = _arr([k.struct() for k in kernels])
        d = specs[0].grid.d
        self.d = d
        dev = "cuda"
        self.loglik = torch.zeros(self.B, dtype=torch.float64, device=dev)
        self.log_c = torch.zeros(self.B, K, dtype=torch.float64, device=dev)
        self.log_mpred = torch.zeros(self.B, K, dtype=torch.float64, device=dev)
        self.mean = torch.zeros(self.B, K, d, dtype=torch.float64, device=dev)
        self.cov = torch.zeros(self.B, K, d, d, dtype=torch.float64, device=dev)
        self.ranks = torch.zeros(self.B, K, d + 1, dtype=torch.int32, device=dev)
        self.ranks_pred = torch.zeros(self.B, K, d + 1, dtype=torch.int32, device=dev)
        self.status = torch.zeros(self.B, dtype=torch.int32, device=dev)
        self.monitor = None
        if monitor:
            self.marg_min = torch.zeros(self.B, K, dtype=torch.float64, device=dev)
            self.tails = torch.zeros(self.B, K, 2, dtype=torch.float64, device=dev)
            self.monitor = Monitor(self.marg_min.data_ptr(), self.tails.data_ptr())
        nbytes = LIB.tt_filter_run_workspace(self.B, self.specs, self.karr, len(kernels), precision)
        if nbytes == 0:
            _check(ERR_ARG, "tt_filter_run_workspace")
        self.ws = _ws(nbytes)

    def __call__(self, z, moments: bool = True, k_begin: int = 0, k_count: Optional[int] = None,
                 replay=None):
        """z: float64 device tensor [B, K, zdim].  Runs steps k_begin ..
        k_begin+k_count-1 (all K by default); k_begin > 0 resumes from the
        state the previous call left in this object's workspace.  replay =
        (ranks_pred, ranks) int32 device tensors [B, K, d+1] fixes the ranks
        of every rounding (rank replay)."""
        if k_count is None:
            k_count = self.K - k_begin
        rp = rf = None
        if replay is not None:
            rp, rf = replay
            for t in (rp, rf):
                if tuple(t.shape) != (self.B, self.K, self.d + 1) or t.dtype != _torch().int32 or not t.is_contiguous():
                    raise TTError("replay ranks must be contiguous int32 [B, K, d+1]")
        args = (self.B, self.specs, self.karr, len(self.kernels), z.data_ptr(), self.zdim,
                self.K, int(k_begin), int(k_count), self.precision, self.loglik.data_ptr(),
                self.log_c.data_ptr(), self.log_mpred.data_ptr(),
                self.mean.data_ptr() if moments else None, self.cov.data_ptr() if moments else None,
                self.ranks.data_ptr(), self.status.data_ptr(), self.ranks_pred.data_ptr(),
                rp.data_ptr() if rp is not None else None, rf.data_ptr() if rf is not None else None)
        if self.monitor is not None:
            st = LIB.tt_filter_run_monitored(*args, C.byref(self.monitor), self.ws.data_ptr(), self.ws.numel(),
                                             _stream())
        else:
            st = LIB.tt_filter_run(*args, self.ws.data_ptr(), self.ws.numel(), _stream())
        _check(st, "tt_filter_run")

    def _state(self, trains: Sequence[DeviceTT], direction: int):
        if len(trains) != self.B:
            raise TTError("one train per filter")
        _check(LIB.tt_filter_state(self.B, self.specs, self.karr, len(self.kernels), self.precision, direction,
                                   _arr([t.struct() for t in trains]), self.ws.data_ptr(), self.ws.numel(),
                                   _stream()), "tt_filter_state")

    def state_trains(self) -> List[DeviceTT]:
        """Trains that can hold every filter's state (the run's rank caps)."""
        specs = list(self.specs)
        return DeviceTT.batch([[s.grid.n[k] for k in range(self.d)] for s in specs],
                              [[1] + [int(s.cap)] * (self.d - 1) + [1] for s in specs], self.precision)

    def save_state(self, trains: Optional[Sequence[DeviceTT]] = None) -> List[DeviceTT]:
        """tt_filter_state(SAVE): the filtering densities after the last step
        run, one train per filter."""
        trains = list(trains) if trains is not None else self.state_trains()
        self._state(trains, STATE_SAVE)
        return trains

    def load_state(self, trains: Sequence[DeviceTT]):
        """tt_filter_state(LOAD): make this workspace continue from the given
        filtering densities (then call with k_begin = the next step)."""
        self._state(list(trains), STATE_LOAD)

    def autotune(self, z, warmup_steps: int = 3, rounds: int = 2) -> dict:
        """tt_autotune_prediction on this batch: times each prediction launch
        shape (one step per candidate per round after the warm-up) and keeps
        the fastest for later runs of the same shape.  The workspace state
        afterwards is the tuner's: rerun from k_begin = 0."""
        best = C.c_int32(0)
        ms = (C.c_float * 4)()
        st = LIB.tt_autotune_prediction(self.B, self.specs, self.karr, len(self.kernels), z.data_ptr(), self.zdim,
                                        self.K, self.precision, self.loglik.data_ptr(), self.log_c.data_ptr(),
                                        self.log_mpred.data_ptr(), self.status.data_ptr(), self.ws.data_ptr(),
                                        self.ws.numel(), _stream(), int(warmup_steps), int(rounds), C.byref(best),
                                        ms)
        _check(st, "tt_autotune_prediction")
        return {"best_bb": int(best.value), "ms_per_step": {bb: round(float(m), 3) for bb, m in zip((2, 4, 8, 16), ms)}}

    def graph(self, z, k_begin: int, k_count: int = 1, moments: bool = True) -> "FilterGraph":
        """Record steps k_begin .. k_begin+k_count-1 (k_begin >= 1) as a HIP
        graph over this object's buffers (tt_filter_graph_create).  Each
        launch() continues from the current workspace state; ``z`` must stay
        alive and may be rewritten in place between launches."""
        if self.precision not in (F32, F64):
            raise TTError("bad precision")
        h = C.c_void_p()
        st = LIB.tt_filter_graph_create(self.B, self.specs, self.karr, len(self.kernels), z.data_ptr(), self.zdim,
                                        self.K, int(k_begin), int(k_count), self.precision,
                                        self.loglik.data_ptr(), self.log_c.data_ptr(), self.log_mpred.data_ptr(),
                                        self.mean.data_ptr() if moments else None,
                                        self.cov.data_ptr() if moments else None,
                                        self.ranks.data_ptr(), self.status.data_ptr(), self.ranks_pred.data_ptr(),
                                        None, None, self.ws.data_ptr(), self.ws.numel(), _stream(), C.byref(h))
        _check(st, "tt_filter_graph_create")
        return FilterGraph(h, (self, z))


class FilterGraph:
    """A recorded HIP graph of filter steps (tt_filter_graph_*); keeps the
    buffers it was recorded over alive."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    def launch(self):
        if self._h is None:
            raise TTError("graph destroyed")
        _check(LIB.tt_filter_graph_launch(self._h, _stream()), "tt_filter_graph_launch")

    def destroy(self):
        if self._h is not None:
            LIB.tt_filter_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
