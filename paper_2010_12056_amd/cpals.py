"""ctypes binding of libcpals.so (declared in include/cpals.h).

Argument marshalling only: PyTorch supplies device memory (the workspace,
tensors, factors) and the HIP stream; every step of the computation runs in
the HIP library.  There is no fallback: if the library is missing or no GPU
is present, the calls raise.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpals.so")

CP_OK, CP_ERR_ARG, CP_ERR_STATE, CP_ERR_UNSUPPORTED, CP_ERR_HIP, CP_ERR_NOT_SPD, CP_ERR_NUMERIC = range(7)
CP_F64, CP_F32, CP_BF16, CP_BF16X2, CP_FP8, CP_FP8X2, CP_F32X3, CP_FP8F8 = 0, 1, 2, 3, 4, 5, 6, 7
CP_TREE_DT, CP_TREE_DT_COMBINED, CP_TREE_MSDT = 0, 1, 2
CP_PP_AUTO, CP_PP_FORCE_EXACT, CP_PP_FORCE_APPROX, CP_PP_FORCE_REINIT, CP_PP_LEARNED = range(5)
KIND_NAMES = {0: "exact", 1: "init", 2: "approx"}
PHASES = ["ttm", "mttv", "update", "pp", "other"]

PRECS = {"f64": CP_F64, "f32": CP_F32, "bf16": CP_BF16, "bf16x2": CP_BF16X2, "fp8": CP_FP8, "fp8x2": CP_FP8X2,
         "f32x3": CP_F32X3, "fp8f8": CP_FP8F8}
TREES = {"dt": CP_TREE_DT, "dt_combined": CP_TREE_DT_COMBINED, "msdt": CP_TREE_MSDT}
PP_MODES = {"auto": CP_PP_AUTO, "exact": CP_PP_FORCE_EXACT, "approx": CP_PP_FORCE_APPROX,
            "init": CP_PP_FORCE_REINIT, "learned": CP_PP_LEARNED}
TORCH_DTYPE = {CP_F64: torch.float64, CP_F32: torch.float32, CP_BF16: torch.bfloat16, CP_BF16X2: torch.bfloat16,
               CP_FP8: torch.float8_e4m3fn, CP_FP8X2: torch.float8_e4m3fn, CP_F32X3: torch.float32,
               CP_FP8F8: torch.float8_e4m3fn}


class SweepInfo(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("fitness_is_exact", ctypes.c_int),
        ("fitness", ctypes.c_double),
        ("r", ctypes.c_double),
        ("dA_rel", ctypes.c_double * 8),
        ("ttm_count", ctypes.c_int),
        ("pinv_updates", ctypes.c_int),
        ("rolled_back", ctypes.c_int),
        ("r_clamped", ctypes.c_int),
    ]

    def as_dict(self, order):
        return {
            "kind": KIND_NAMES[self.kind],
            "fitness_is_exact": bool(self.fitness_is_exact),
            "fitness": self.fitness,
            "r": self.r,
            "dA_rel": [self.dA_rel[i] for i in range(order)],
            "ttm_count": self.ttm_count,
            "pinv_updates": self.pinv_updates,
            "rolled_back": bool(self.rolled_back),
            "r_clamped": bool(self.r_clamped),
        }


class CpalsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"cpals status {status}: {msg}")
        self.status = status


_lib = None

EXPORTS = {
    "cp_plan_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "cp_plan_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "cp_plan_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "cp_set_tensor": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "cp_mttkrp": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p]),
    "cp_mttkrp_static": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "cp_mttkrp_rooted": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                        ctypes.c_int, ctypes.c_void_p]),
    "cp_als_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(SweepInfo)]),
    "cp_pp_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_double,
                                   ctypes.c_int, ctypes.POINTER(SweepInfo)]),
    "cp_reset": (ctypes.c_int, [ctypes.c_void_p]),
    "cp_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "cp_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "cp_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "cp_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]),
    "cp_fitness": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double)]),
    "cp_pp_set_switch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_double]),
    "cp_pp_last_decision": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]),
    "cp_mlp_param_count": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "cp_mlp_scratch_floats": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "cp_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "cp_mlp_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cp_mlp_adam": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_void_p]),
    "cp_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int), ctypes.c_void_p]),
    "cp_batch_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "cp_batch_set_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "cp_batch_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "cp_batch_set_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "cp_batch_sweeps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "cp_batch_tick_rate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "cp_batch_destroy": (None, [ctypes.c_void_p]),
    "cp_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "cp_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
}


def lib():
    """Load libcpals.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run paper_2010_12056_amd.build_lib.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptrs(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else ctypes.c_void_p(t.data_ptr())
    return arr


def mttkrp_static(T, A, mode, rank, prec="f32", out=None):
    """M = MTTKRP of `mode` through cp_mttkrp_static (no plan, no workspace:
    the library's static device scratch holds the intermediates).  T: device
    tensor in `prec`; A: list of FP64 device factors (A[mode] may be None)."""
    L = lib()
    dims = tuple(int(d) for d in T.shape)
    N = len(dims)
    M = out if out is not None else torch.empty((dims[mode], rank), dtype=torch.float64, device=T.device)
    d = (ctypes.c_int64 * N)(*dims)
    st = torch.cuda.current_stream(T.device).cuda_stream
    s = L.cp_mttkrp_static(N, d, int(rank), PRECS[prec], ctypes.c_void_p(T.data_ptr()), _ptrs(A), int(mode),
                           ctypes.c_void_p(M.data_ptr()), ctypes.c_void_p(st))
    if s != CP_OK:
        raise CpalsError(s, L.cp_last_error(None).decode())
    return M


class Plan:
    """A CP-ALS plan: tensor dims, rank, precision ("f64" / "f32" / "f32x3" (an
    FP32 tensor, first contraction as three-part BF16 products) / "bf16" /
    "bf16x2" / "fp8" / "fp8x2" / "fp8f8", the last three an E4M3 tensor) and tree ("dt" / "dt_combined" / "msdt"), bound to the current
    HIP stream of `device`."""

    def __init__(self, dims, rank, prec="f32", tree="dt", device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("cpals needs a GPU; none is visible")
        self.L = lib()
        self.dims = tuple(int(d) for d in dims)
        self.order = len(self.dims)
        self.rank = int(rank)
        self.prec = PRECS[prec]
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        d = (ctypes.c_int64 * self.order)(*self.dims)
        self._check(self.L.cp_plan_create(ctypes.byref(h), self.order, d, self.rank, self.prec,
                                          TREES[tree], ctypes.c_void_p(self.stream.cuda_stream)), None)
        self.h = h
        nbytes = ctypes.c_size_t()
        self._check(self.L.cp_plan_workspace_size(self.h, ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self.ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._check(self.L.cp_plan_set_workspace(self.h, ctypes.c_void_p(aligned), self.workspace_bytes))
        self.T = None

    def _check(self, status, h="self"):
        if status != CP_OK:
            hh = self.h if h == "self" else h
            msg = self.L.cp_last_error(hh) if hh else b""
            base = self.L.cp_status_str(status)
            raise CpalsError(status, (base or b"").decode() + ": " + (msg or b"").decode())

    def set_tensor(self, T):
        if T.dtype != TORCH_DTYPE[self.prec] or tuple(T.shape) != self.dims or not T.is_contiguous():
            raise ValueError("tensor must be contiguous with the plan's dims and precision")
        if T.device != self.device and not (T.is_cuda and self.device.type == "cuda"):
            raise ValueError("tensor must be on the plan's device")
        self.T = T
        self._check(self.L.cp_set_tensor(self.h, ctypes.c_void_p(T.data_ptr())))

    def _factors(self, A, allow_none=None):
        if len(A) != self.order:
            raise ValueError("need one factor per mode")
        for i, a in enumerate(A):
            if a is None and i == allow_none:
                continue
            if a.dtype != torch.float64 or tuple(a.shape) != (self.dims[i], self.rank) or not a.is_contiguous() \
                    or not a.is_cuda:
                raise ValueError(f"factor {i} must be a contiguous FP64 CUDA tensor of shape "
                                 f"({self.dims[i]}, {self.rank})")
        return _ptrs(A)

    def mttkrp(self, A, mode, root=None, out=None):
        M = out if out is not None else torch.empty((self.dims[mode], self.rank), dtype=torch.float64,
                                                   device=self.device)
        p = self._factors(A, allow_none=mode)
        if root is None:
            self._check(self.L.cp_mttkrp(self.h, p, int(mode), ctypes.c_void_p(M.data_ptr())))
        else:
            self._check(self.L.cp_mttkrp_rooted(self.h, p, int(mode), int(root), ctypes.c_void_p(M.data_ptr())))
        return M

    def als_sweep(self, A, info=True):
        p = self._factors(A)
        if info:
            si = SweepInfo()
            self._check(self.L.cp_als_sweep(self.h, p, ctypes.byref(si)))
            return si.as_dict(self.order)
        self._check(self.L.cp_als_sweep(self.h, p, None))
        return None

    def pp_sweep(self, A, tol=0.2, mode="auto", info=True):
        p = self._factors(A)
        if info:
            si = SweepInfo()
            self._check(self.L.cp_pp_sweep(self.h, p, float(tol), PP_MODES[mode], ctypes.byref(si)))
            return si.as_dict(self.order)
        self._check(self.L.cp_pp_sweep(self.h, p, float(tol), PP_MODES[mode], None))
        return None

    def fitness(self, A):
        """Exact fitness of the given factors (audit of approximated sweeps)."""
        f = ctypes.c_double()
        self._check(self.L.cp_fitness(self.h, self._factors(A), ctypes.byref(f)))
        return f.value

    def set_switch(self, theta, hidden, shift, scale, threshold=0.5):
        """Attach the learned PP switch (theta: FP32 device tensor, kept alive)."""
        if theta is None:
            self._switch = None
            self._check(self.L.cp_pp_set_switch(self.h, None, 0, None, None, 0.0))
            return
        D = self.order + 3
        sh = (ctypes.c_double * D)(*[float(x) for x in shift])
        sc = (ctypes.c_double * D)(*[float(x) for x in scale])
        self._switch = theta
        self._check(self.L.cp_pp_set_switch(self.h, ctypes.c_void_p(theta.data_ptr()), int(hidden), sh, sc,
                                            float(threshold)))

    def last_decision(self):
        D = self.order + 3
        f = (ctypes.c_double * D)()
        pr = ctypes.c_double()
        self._check(self.L.cp_pp_last_decision(self.h, f, ctypes.byref(pr)))
        return [f[i] for i in range(D)], pr.value

    def profile(self, on=True, phases=None):
        """Time the given phases (names from PHASES; all when None) from now on,
        or none when `on` is false."""
        mask = 0
        if on:
            mask = (1 << len(PHASES)) - 1 if phases is None else sum(1 << PHASES.index(ph) for ph in phases)
        self._check(self.L.cp_profile_enable(self.h, mask))

    def profile_read(self):
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_int64 * 5)()
        self._check(self.L.cp_profile_read(self.h, ms, cnt))
        return {PHASES[i]: (ms[i], int(cnt[i])) for i in range(5)}

    def reset(self):
        self._check(self.L.cp_reset(self.h))

    def sync(self):
        self._check(self.L.cp_sync(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.L.cp_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _mlp_check(status):
    if status != CP_OK:
        raise CpalsError(status, (lib().cp_status_str(status) or b"").decode())


def mlp_param_count(D, H):
    return int(lib().cp_mlp_param_count(D, H))


def mlp_forward(X, theta, H, stream=None):
    """Probabilities of the switch network for the rows of X (FP32 CUDA tensors)."""
    B, D = X.shape
    p = torch.empty(B, dtype=torch.float32, device=X.device)
    st = (stream or torch.cuda.current_stream(X.device)).cuda_stream
    _mlp_check(lib().cp_mlp_forward(ctypes.c_void_p(X.data_ptr()), B, D, H, ctypes.c_void_p(theta.data_ptr()),
                                    ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(st)))
    return p


def mlp_grad(X, y, theta, H, scratch=None, out=None, stream=None):
    """Gradient of the mean BCE (out[:n]) and the loss (out[n])."""
    B, D = X.shape
    n = mlp_param_count(D, H)
    if out is None:
        out = torch.empty(n + 1, dtype=torch.float32, device=X.device)
    if scratch is None:
        scratch = torch.empty(int(lib().cp_mlp_scratch_floats(B, H)), dtype=torch.float32, device=X.device)
    st = (stream or torch.cuda.current_stream(X.device)).cuda_stream
    _mlp_check(lib().cp_mlp_grad(ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(y.data_ptr()), B, D, H,
                                 ctypes.c_void_p(theta.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(scratch.data_ptr()), ctypes.c_void_p(st)))
    return out


def mlp_adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    st = (stream or torch.cuda.current_stream(theta.device)).cuda_stream
    _mlp_check(lib().cp_mlp_adam(ctypes.c_void_p(theta.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                                 ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(v.data_ptr()), theta.numel(), int(t),
                                 float(lr), float(beta1), float(beta2), float(eps), ctypes.c_void_p(st)))


class Batch:
    """Many small order-3 FP32 tensors decomposed in one persistent launch
    (cp_batch_* in include/cpals.h).  dims: list of (s0, s1, s2); ranks: list
    of R.  Packs tensors and factors into the library's layout on the device."""

    def __init__(self, dims, ranks, device="cuda", waves=4, groups_per_cu=2):
        if not torch.cuda.is_available():
            raise RuntimeError("cpals needs a GPU; none is visible")
        self.L = lib()
        self.count = len(dims)
        self.dims = [tuple(int(x) for x in d) for d in dims]
        self.ranks = [int(r) for r in ranks]
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        flat = (ctypes.c_int64 * (3 * self.count))(*[x for d in self.dims for x in d])
        rk = (ctypes.c_int * self.count)(*self.ranks)
        h = ctypes.c_void_p()
        _mlp_check(self.L.cp_batch_create(ctypes.byref(h), self.count, flat, rk,
                                          ctypes.c_void_p(self.stream.cuda_stream)))
        self.h = h
        _mlp_check(self.L.cp_batch_set_launch(self.h, int(waves), int(groups_per_cu)))
        toff = (ctypes.c_int64 * self.count)()
        aoff = (ctypes.c_int64 * (3 * self.count))()
        tt, at = ctypes.c_int64(), ctypes.c_int64()
        _mlp_check(self.L.cp_batch_layout(self.h, toff, aoff, ctypes.byref(tt), ctypes.byref(at)))
        self.t_off = [toff[i] for i in range(self.count)]
        self.a_off = [[aoff[3 * i + m] for m in range(3)] for i in range(self.count)]
        self.t_total, self.a_total = tt.value, at.value
        nbytes = ctypes.c_size_t()
        _mlp_check(self.L.cp_batch_workspace_size(self.h, ctypes.byref(nbytes)))
        self.ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.ws.data_ptr() + 255) // 256 * 256
        _mlp_check(self.L.cp_batch_set_workspace(self.h, ctypes.c_void_p(aligned), int(nbytes.value)))

    def pack_tensors(self, tensors):
        """One FP32 device array holding every tensor at its offset."""
        T = torch.zeros(self.t_total, dtype=torch.float32, device=self.device)
        for i, t in enumerate(tensors):
            src = torch.as_tensor(t, dtype=torch.float32).reshape(-1)
            T[self.t_off[i]:self.t_off[i] + src.numel()].copy_(src)
        return T

    def pack_factors(self, factors):
        """factors[i] = [A0, A1, A2] (FP64): one FP64 device array."""
        A = torch.zeros(self.a_total, dtype=torch.float64, device=self.device)
        for i, fs in enumerate(factors):
            for m in range(3):
                src = torch.as_tensor(fs[m], dtype=torch.float64).reshape(-1)
                A[self.a_off[i][m]:self.a_off[i][m] + src.numel()].copy_(src)
        return A

    def unpack_factors(self, A, i):
        out = []
        for m in range(3):
            n = self.dims[i][m] * self.ranks[i]
            out.append(A[self.a_off[i][m]:self.a_off[i][m] + n].reshape(self.dims[i][m], self.ranks[i]))
        return out

    def sweeps(self, T, A, sweeps, fitness=None, status=None, ticks=None):
        """Enqueue `sweeps` sweeps of every tensor (no synchronization)."""
        if fitness is None:
            fitness = torch.empty((self.count, sweeps), dtype=torch.float64, device=self.device)
        if status is None:
            status = torch.empty(self.count, dtype=torch.int32, device=self.device)
        tp = ctypes.c_void_p(ticks.data_ptr()) if ticks is not None else None
        _mlp_check(self.L.cp_batch_sweeps(self.h, ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(A.data_ptr()),
                                          int(sweeps), ctypes.c_void_p(fitness.data_ptr()),
                                          ctypes.c_void_p(status.data_ptr()), tp))
        return fitness, status

    def tick_rate(self):
        hz = ctypes.c_double()
        _mlp_check(self.L.cp_batch_tick_rate(self.h, ctypes.byref(hz)))
        return hz.value

    def close(self):
        if getattr(self, "h", None):
            self.L.cp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

