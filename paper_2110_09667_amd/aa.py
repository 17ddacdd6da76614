"""ctypes binding of ``libaa.so`` (``include/aa.h``): argument marshalling only.

Every function named ``aa_*`` here calls the C entry point of the same name
with raw device pointers (``tensor.data_ptr()``) and the HIP stream of the
current torch stream.  Errors come back as ``AAError`` carrying the status.
Torch is used for device memory and streams only.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaa.so")

MGS, CGS2, DCGS2, ICWY, DCGS2_LAG = 0, 1, 2, 3, 4
VARIANTS = {"mgs": MGS, "cgs2": CGS2, "dcgs2": DCGS2, "icwy": ICWY, "dcgs2_lag": DCGS2_LAG}
DCGS2_LITERAL = 1 << 1
ICWY_T_TRANSFORM = 1 << 2
DCGS2_GUARD_GE3 = 1 << 4
FUSE_RHS = 1 << 3
FUSE_DELETE = 1 << 5
QR_ONLY = 1 << 8
MAX_COLS = 65

STATUS = {0: "AA_OK", -1: "AA_EINVAL", -2: "AA_EHIP", -3: "AA_EBREAKDOWN",
          -4: "AA_ESTATE", -5: "AA_ENOSPACE"}

SYMBOLS = [
    "aa_workspace_size", "aa_init", "aa_set_stream", "aa_step", "aa_get_info",
    "aa_qr_add", "aa_qr_delete", "aa_qr_solve", "aa_get_qr", "aa_qr_basis",
    "aa_qr_load", "aa_reset", "aa_destroy", "aa_sync_counts", "aa_problem_apply",
    "aa_fill_uniform", "aa_fill_normal", "aa_version", "aa_profile_enable",
    "aa_profile_read", "aa_profile_reset", "aa_set_grid", "aa_set_fused_threshold", "aa_set_graph",
    "aa_batch_workspace_size", "aa_batch_init", "aa_batch_run", "aa_batch_read",
    "aa_batch_set_schedule", "aa_batch_autotune", "aa_batch_destroy", "aa_mlp_param_count",
    "aa_mlp_workspace_size", "aa_mlp_init", "aa_mlp_reseed", "aa_mlp_set_params",
    "aa_mlp_get_params", "aa_mlp_get_grads", "aa_mlp_forward", "aa_mlp_backward",
    "aa_mlp_adam", "aa_mlp_destroy", "aa_batch_run_learned", "aa_batch_train",
    "aa_batch_read_learning", "aa_qr_solve_noalloc", "aa_bandwidth_probe", "aa_em_apply",
    "aa_set_stop", "aa_batch_set_tiles", "aa_batch_set_split",
    "aa_batch_split_count", "aa_pde2d_workspace_size", "aa_pde2d_init", "aa_pde2d_apply",
    "aa_pde2d_solve", "aa_pde2d_vcycle", "aa_pde2d_set_iters", "aa_pde2d_last",
    "aa_pde2d_set_stream", "aa_pde2d_destroy",
]
PDE_HEAT_NL1, PDE_HEAT_NL2, PDE_BRATU = 1, 2, 3
EM_WORK_DOUBLES = 6144

BATCH_LEARNED = 1 << 9

KERNEL_KINDS = ["dots", "update", "cgs2b", "givens", "rotate", "scale", "history", "xupdate",
                "fused", "finalize"]


class AAError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}")
        self.status = status


class Info(C.Structure):
    _fields_ = [("iter", C.c_int64), ("m_i", C.c_int), ("k", C.c_int),
                ("res_norm", C.c_double), ("res0_norm", C.c_double),
                ("step_norm", C.c_double), ("status", C.c_int), ("stopped", C.c_int),
                ("stop_iter", C.c_int64)]


RUNNING, STOPPED_TEST, STOPPED_BREAKDOWN, STOPPED_CAP = 0, 1, 2, 3
STOP_RESIDUAL, STOP_STEP = 0, 1


class BatchInstance(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int), ("dim", C.c_int), ("s", C.c_int64),
                ("h", C.c_double), ("omega", C.c_double), ("c", C.c_double),
                ("d_f", C.c_void_p), ("d_x", C.c_void_p)]


class EmMixture(C.Structure):
    _fields_ = [("alpha", C.c_double * 3), ("sigma", C.c_double * 3)]


class BatchSchedule(C.Structure):
    _fields_ = [("grid", C.c_int), ("order", C.c_int), ("ms_per_iter", C.c_double),
                ("trials", C.c_int), ("pairs", C.c_int)]


class BatchState(C.Structure):
    _fields_ = [("iter", C.c_int64), ("stop_iter", C.c_int64), ("k", C.c_int),
                ("m_i", C.c_int), ("active", C.c_int), ("status", C.c_int),
                ("res_norm", C.c_double), ("res0_norm", C.c_double),
                ("g_evals", C.c_int64), ("accepted", C.c_int64), ("loss", C.c_double),
                ("pending", C.c_int), ("g_valid", C.c_int)]


_lib = None


def lib():
    """Load ``libaa.so``; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    P, I64, I, U, D, U64 = C.c_void_p, C.c_int64, C.c_int, C.c_uint, C.c_double, C.c_uint64
    sig = {
        "aa_workspace_size": [I64, I, I, U, C.POINTER(C.c_size_t)],
        "aa_init": [C.POINTER(P), I64, I, I, U, P, C.c_size_t, P],
        "aa_set_stream": [P, P],
        "aa_step": [P, P, P, P],
        "aa_get_info": [P, C.POINTER(Info)],
        "aa_set_stop": [P, D, I64, I],
        "aa_batch_set_tiles": [P, I],
        "aa_batch_set_split": [P, I64, I],
        "aa_batch_split_count": [P, C.POINTER(I)],
        "aa_qr_add": [P, P],
        "aa_qr_delete": [P],
        "aa_qr_solve": [P, P, P],
        "aa_qr_solve_noalloc": [P, I64, I64, I, P, I, P, P, P],
        "aa_bandwidth_probe": [I, I, P, I64, P, I64, P, P],
        "aa_em_apply": [C.POINTER(EmMixture), P, I64, P, P, I64, P, P],
        "aa_get_qr": [P, P, P, C.POINTER(C.c_int)],
        "aa_qr_basis": [P, C.POINTER(P), C.POINTER(I64)],
        "aa_qr_load": [P, I, P, I64, P, P],
        "aa_reset": [P],
        "aa_destroy": [P],
        "aa_sync_counts": [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)],
        "aa_problem_apply": [I, I64, D, D, D, P, P, P, P],
        "aa_fill_uniform": [P, I64, U64, U64, U64, D, D, P],
        "aa_fill_normal": [P, I64, U64, U64, U64, P],
        "aa_profile_enable": [P, I],
        "aa_profile_read": [P, I, C.POINTER(D), C.POINTER(I64), C.POINTER(D)],
        "aa_profile_reset": [P],
        "aa_set_grid": [P, I, I],
        "aa_set_fused_threshold": [P, I64],
        "aa_set_graph": [P, I],
        "aa_batch_workspace_size": [I, C.POINTER(BatchInstance), I, U, C.POINTER(C.c_size_t)],
        "aa_batch_init": [C.POINTER(P), I, C.POINTER(BatchInstance), I, U, D, I64, P,
                          C.c_size_t, P],
        "aa_batch_run": [P, I],
        "aa_batch_read": [P, C.POINTER(BatchState), C.POINTER(I)],
        "aa_batch_set_schedule": [P, I, I, I],
        "aa_batch_autotune": [P, I, C.c_char_p, C.POINTER(BatchSchedule)],
        "aa_batch_destroy": [P],
        "aa_mlp_workspace_size": [I, C.POINTER(C.c_size_t)],
        "aa_mlp_init": [C.POINTER(P), I, U64, P, C.c_size_t, P],
        "aa_mlp_reseed": [P, U64],
        "aa_mlp_set_params": [P, P],
        "aa_mlp_get_params": [P, P],
        "aa_mlp_get_grads": [P, P],
        "aa_mlp_forward": [P, I, P, P],
        "aa_mlp_backward": [P, I, P],
        "aa_mlp_adam": [P, C.c_float, C.c_float, C.c_float, C.c_float],
        "aa_mlp_destroy": [P],
        "aa_batch_run_learned": [P, P, I],
        "aa_batch_train": [P, P, I, C.c_float],
        "aa_batch_read_learning": [P, P, P, P],
        "aa_pde2d_workspace_size": [I64, I, C.POINTER(C.c_size_t)],
        "aa_pde2d_init": [C.POINTER(P), I64, I, D, D, I, P, C.c_size_t, P],
        "aa_pde2d_apply": [P, P, P, P],
        "aa_pde2d_solve": [P, P, P],
        "aa_pde2d_vcycle": [P, P, P],
        "aa_pde2d_set_iters": [P, I],
        "aa_pde2d_last": [P, C.POINTER(I), C.POINTER(I)],
        "aa_pde2d_set_stream": [P, P],
        "aa_pde2d_destroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.aa_mlp_param_count.argtypes = []
    L.aa_mlp_param_count.restype = C.c_int64
    L.aa_version.argtypes = []
    L.aa_version.restype = C.c_char_p
    _lib = L
    return L


def _check(st: int, where: str):
    if st != 0:
        raise AAError(st, where)


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


# ---- thin wrappers with the C names -----------------------------------------

def aa_workspace_size(n: int, m: int, variant: int, flags: int = 0) -> int:
    b = C.c_size_t(0)
    _check(lib().aa_workspace_size(n, m, variant, flags, C.byref(b)), "aa_workspace_size")
    return b.value


def aa_init(n, m, variant, flags, workspace, stream=None):
    ctx = C.c_void_p()
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().aa_init(C.byref(ctx), n, m, variant, flags, workspace.data_ptr(), nbytes,
                         _stream(stream)), "aa_init")
    return ctx


def aa_step(ctx, x, g, x_next):
    _check(lib().aa_step(ctx, _ptr(x), _ptr(g), _ptr(x_next)), "aa_step")


def aa_get_info(ctx) -> Info:
    info = Info()
    _check(lib().aa_get_info(ctx, C.byref(info)), "aa_get_info")
    return info


def aa_qr_add(ctx, v):
    _check(lib().aa_qr_add(ctx, _ptr(v)), "aa_qr_add")


def aa_qr_delete(ctx):
    _check(lib().aa_qr_delete(ctx), "aa_qr_delete")


def aa_qr_solve(ctx, f, gamma):
    _check(lib().aa_qr_solve(ctx, _ptr(f), _ptr(gamma)), "aa_qr_solve")


def aa_bandwidth_probe(reads, writes, src, ld, dst, n, sink, stream=None):
    _check(lib().aa_bandwidth_probe(reads, writes, _ptr(src), ld, _ptr(dst), n, _ptr(sink),
                                    _stream(stream)), "aa_bandwidth_probe")


def aa_pde2d_workspace_size(N: int, max_iter: int) -> int:
    b = C.c_size_t(0)
    _check(lib().aa_pde2d_workspace_size(N, max_iter, C.byref(b)), "aa_pde2d_workspace_size")
    return b.value


def aa_pde2d_init(N, problem, lam, tol, max_iter, workspace, stream=None):
    ctx = C.c_void_p()
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().aa_pde2d_init(C.byref(ctx), N, problem, lam, tol, max_iter,
                               workspace.data_ptr(), nbytes, _stream(stream)), "aa_pde2d_init")
    return ctx


def aa_pde2d_apply(ctx, b, u, out):
    _check(lib().aa_pde2d_apply(ctx, _ptr(b), _ptr(u), _ptr(out)), "aa_pde2d_apply")


def aa_pde2d_solve(ctx, rhs, x):
    _check(lib().aa_pde2d_solve(ctx, _ptr(rhs), _ptr(x)), "aa_pde2d_solve")


def aa_pde2d_vcycle(ctx, r, z):
    _check(lib().aa_pde2d_vcycle(ctx, _ptr(r), _ptr(z)), "aa_pde2d_vcycle")


def aa_pde2d_set_iters(ctx, iters: int):
    _check(lib().aa_pde2d_set_iters(ctx, iters), "aa_pde2d_set_iters")


def aa_pde2d_last(ctx):
    it, conv = C.c_int(0), C.c_int(0)
    _check(lib().aa_pde2d_last(ctx, C.byref(it), C.byref(conv)), "aa_pde2d_last")
    return it.value, bool(conv.value)


def aa_pde2d_set_stream(ctx, stream=None):
    _check(lib().aa_pde2d_set_stream(ctx, _stream(stream)), "aa_pde2d_set_stream")


def aa_pde2d_destroy(ctx):
    _check(lib().aa_pde2d_destroy(ctx), "aa_pde2d_destroy")


def aa_em_apply(alpha, sigma, x, u, out, work, stream=None):
    mix = EmMixture((C.c_double * 3)(*alpha), (C.c_double * 3)(*sigma))
    _check(lib().aa_em_apply(C.byref(mix), _ptr(x), x.numel(), _ptr(u), _ptr(out), u.numel(),
                             _ptr(work), _stream(stream)), "aa_em_apply")


def aa_qr_solve_noalloc(Q, ldq, n, k, R, ldr, f, gamma, stream=None):
    _check(lib().aa_qr_solve_noalloc(_ptr(Q), ldq, n, k, _ptr(R), ldr, _ptr(f), _ptr(gamma),
                                     _stream(stream)), "aa_qr_solve_noalloc")


def aa_get_qr(ctx, cap: int):
    import numpy as np
    R = np.zeros(cap * cap)
    T = np.zeros(cap * cap)
    k = C.c_int(0)
    _check(lib().aa_get_qr(ctx, R.ctypes.data, T.ctypes.data, C.byref(k)), "aa_get_qr")
    kk = k.value
    return (R[: kk * kk].reshape(kk, kk, order="F").copy(),
            T[: kk * kk].reshape(kk, kk, order="F").copy(), kk)


def aa_qr_basis(ctx):
    p = C.c_void_p()
    ld = C.c_int64(0)
    _check(lib().aa_qr_basis(ctx, C.byref(p), C.byref(ld)), "aa_qr_basis")
    return p.value, ld.value


def aa_qr_load(ctx, k, Q_ptr, ldq, R, T=None):
    import numpy as np
    Rf = np.asfortranarray(R, dtype=np.float64)
    Tf = None if T is None else np.asfortranarray(T, dtype=np.float64)
    _check(lib().aa_qr_load(ctx, k, Q_ptr, ldq, Rf.ctypes.data,
                            None if Tf is None else Tf.ctypes.data), "aa_qr_load")


def aa_reset(ctx):
    _check(lib().aa_reset(ctx), "aa_reset")


def aa_destroy(ctx):
    _check(lib().aa_destroy(ctx), "aa_destroy")


def aa_sync_counts(ctx):
    a, d, r = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().aa_sync_counts(ctx, C.byref(a), C.byref(d), C.byref(r)), "aa_sync_counts")
    return a.value, d.value, r.value


def aa_problem_apply(dim, s, h, omega, c, f, u, out, stream=None):
    _check(lib().aa_problem_apply(dim, s, h, omega, c, _ptr(f), _ptr(u), _ptr(out),
                                  _stream(stream)), "aa_problem_apply")


def aa_fill_uniform(out, seed, stream_id, offset=0, lo=0.0, hi=1.0, stream=None):
    _check(lib().aa_fill_uniform(_ptr(out), out.numel(), seed, stream_id, offset, lo, hi,
                                 _stream(stream)), "aa_fill_uniform")


def aa_fill_normal(out, seed, stream_id, offset=0, stream=None):
    _check(lib().aa_fill_normal(_ptr(out), out.numel(), seed, stream_id, offset,
                                _stream(stream)), "aa_fill_normal")


def aa_profile_enable(ctx, enable=True):
    _check(lib().aa_profile_enable(ctx, 1 if enable else 0), "aa_profile_enable")


def aa_profile_read(ctx, kind: int):
    ms, n, b = C.c_double(), C.c_int64(), C.c_double()
    _check(lib().aa_profile_read(ctx, kind, C.byref(ms), C.byref(n), C.byref(b)),
           "aa_profile_read")
    return ms.value, n.value, b.value


def aa_profile_reset(ctx):
    _check(lib().aa_profile_reset(ctx), "aa_profile_reset")


def aa_set_grid(ctx, stream_max: int, gram_max: int):
    _check(lib().aa_set_grid(ctx, stream_max, gram_max), "aa_set_grid")


def aa_set_fused_threshold(ctx, n_max: int):
    _check(lib().aa_set_fused_threshold(ctx, n_max), "aa_set_fused_threshold")


def aa_batch_workspace_size(insts, variant: int, flags: int = 0) -> int:
    arr = (BatchInstance * len(insts))(*insts)
    b = C.c_size_t(0)
    _check(lib().aa_batch_workspace_size(len(insts), arr, variant, flags, C.byref(b)),
           "aa_batch_workspace_size")
    return b.value


def aa_batch_init(insts, variant, flags, tol, max_iter, workspace, stream=None):
    arr = (BatchInstance * len(insts))(*insts)
    b = C.c_void_p()
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().aa_batch_init(C.byref(b), len(insts), arr, variant, flags, tol, max_iter,
                               workspace.data_ptr(), nbytes, _stream(stream)), "aa_batch_init")
    return b


def aa_batch_run(b, iters: int):
    _check(lib().aa_batch_run(b, iters), "aa_batch_run")


def aa_batch_read(b, count: int):
    states = (BatchState * count)()
    active = C.c_int(0)
    _check(lib().aa_batch_read(b, states, C.byref(active)), "aa_batch_read")
    return list(states), active.value


def aa_batch_set_schedule(b, grid: int = 0, order: int = 0, use_graph: bool = True):
    _check(lib().aa_batch_set_schedule(b, grid, order, 1 if use_graph else 0),
           "aa_batch_set_schedule")


def aa_batch_destroy(b):
    _check(lib().aa_batch_destroy(b), "aa_batch_destroy")


def aa_version() -> str:
    return lib().aa_version().decode()


# ---- convenience context ------------------------------------------------------

class AAContext:
    """Owns a torch workspace and a library context for vectors of length n."""

    def __init__(self, n: int, m: int, variant="mgs", flags: int = 0, device="cuda",
                 stream=None):
        import torch
        self.n, self.m = int(n), int(m)
        self.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self.flags = int(flags)
        nbytes = aa_workspace_size(self.n, self.m, self.variant, self.flags)
        # 256-byte aligned: torch's caching allocator aligns blocks to >= 512 B
        self.workspace = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device)
        assert self.workspace.data_ptr() % 256 == 0
        self.ctx = aa_init(self.n, self.m, self.variant, self.flags, self.workspace, stream)

    def step(self, x, g, x_next):
        aa_step(self.ctx, x, g, x_next)

    def info(self) -> Info:
        return aa_get_info(self.ctx)

    def qr_add(self, v):
        aa_qr_add(self.ctx, v)

    def qr_delete(self):
        aa_qr_delete(self.ctx)

    def qr_solve(self, f, gamma):
        aa_qr_solve(self.ctx, f, gamma)

    def get_qr(self):
        return aa_get_qr(self.ctx, self.m)

    def basis(self, k: int | None = None):
        """Torch view of Q's first k columns as an (n, k) column-major tensor."""
        import torch
        ptr, ld = aa_qr_basis(self.ctx)
        if k is None:
            k = aa_get_qr(self.ctx, self.m)[2]
        ws = self.workspace
        off = (ptr - ws.data_ptr()) // 8
        return ws.as_strided((self.n, k), (1, ld), off)

    def profile(self, enable=True):
        aa_profile_enable(self.ctx, enable)

    def profile_read(self):
        """{kind: (ms, launches, algorithmic bytes)} since the last reset."""
        return {name: aa_profile_read(self.ctx, i) for i, name in enumerate(KERNEL_KINDS)}

    def set_grid(self, stream_max: int, gram_max: int):
        aa_set_grid(self.ctx, stream_max, gram_max)

    def set_graph(self, enable: bool = True):
        """Replay steady-state iterations from HIP graphs (see aa_set_graph)."""
        _check(lib().aa_set_graph(self.ctx, 1 if enable else 0), "aa_set_graph")

    def set_stop(self, tol: float, max_iter: int = 0, mode: int = 0):
        """Stopping rule evaluated on the device (see aa_set_stop)."""
        _check(lib().aa_set_stop(self.ctx, tol, max_iter, mode), "aa_set_stop")

    def set_fused_threshold(self, n_max: int):
        aa_set_fused_threshold(self.ctx, n_max)

    def sync_counts(self):
        return aa_sync_counts(self.ctx)

    def reset(self):
        aa_reset(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            aa_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AABatch:
    """Owns the workspace of a batch of model-map instances (2D/3D stencils)."""

    def __init__(self, problems, ms, variant="icwy", flags: int = 0, tol: float = 1e-8,
                 max_iter: int = 5000, x0=None, stream=None, device="cuda"):
        import torch
        self.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self.count = len(problems)
        self.f = []
        self.x = []
        insts = []
        for j, (p, m) in enumerate(zip(problems, ms)):
            fj = p.f if hasattr(p.f, "data_ptr") else torch.from_numpy(p.f).to(device)
            xj = torch.zeros(p.n, dtype=torch.float64, device=device) if x0 is None else \
                x0[j].clone()
            self.f.append(fj)
            self.x.append(xj)
            insts.append(BatchInstance(p.n, int(m), p.d, p.s, p.h, p.omega, p.c,
                                       fj.data_ptr(), xj.data_ptr()))
        nbytes = aa_batch_workspace_size(insts, self.variant, flags)
        self.workspace = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device)
        self.b = aa_batch_init(insts, self.variant, flags, tol, max_iter, self.workspace, stream)

    def run(self, iters: int):
        aa_batch_run(self.b, iters)

    def read(self):
        return aa_batch_read(self.b, self.count)

    def set_schedule(self, grid: int = 0, order: int = 0, use_graph: bool = True):
        aa_batch_set_schedule(self.b, grid, order, use_graph)

    def set_tiles(self, pairs: int):
        """Row pairs per lane of the persistent kernel's tiles (2 or 4)."""
        _check(lib().aa_batch_set_tiles(self.b, pairs), "aa_batch_set_tiles")

    def set_split(self, min_n: int = 65536, active_max: int = 0):
        """Move active instances with n >= min_n onto the grid-wide passes
        once at most active_max are active (0: one per compute unit; min_n
        = 0 never)."""
        _check(lib().aa_batch_set_split(self.b, min_n, active_max), "aa_batch_set_split")

    def split_count(self) -> int:
        """Instances on the split path as of the last run."""
        c = C.c_int(0)
        _check(lib().aa_batch_split_count(self.b, C.byref(c)), "aa_batch_split_count")
        return c.value

    def autotune(self, iters: int = 3, cache_path: str | None = None) -> "BatchSchedule":
        """Pick the persistent grid and instance order by timing real
        iterations (see aa_batch_autotune); returns the chosen schedule."""
        best = BatchSchedule()
        _check(lib().aa_batch_autotune(self.b, iters,
                                       cache_path.encode() if cache_path else None,
                                       C.byref(best)), "aa_batch_autotune")
        return best

    def run_learned(self, net, iters: int):
        _check(lib().aa_batch_run_learned(self.b, net.net, iters), "aa_batch_run_learned")

    def train(self, net, iters: int, lr: float = 1e-3):
        _check(lib().aa_batch_train(self.b, net.net, iters, lr), "aa_batch_train")

    def read_learning(self):
        """(features [count x 230], outputs [count x 21], dL/doutputs [count x 21])."""
        import numpy as np
        f = np.empty((self.count, 230), dtype=np.float32)
        o = np.empty((self.count, 21), dtype=np.float32)
        d = np.empty((self.count, 21), dtype=np.float32)
        _check(lib().aa_batch_read_learning(self.b, f.ctypes.data, o.ctypes.data, d.ctypes.data),
               "aa_batch_read_learning")
        return f, o, d

    def close(self):
        if getattr(self, "b", None) is not None:
            aa_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_FEATURES, MLP_OUTPUTS = 230, 21


class AAMlp:
    """The mixing-weight network (BF16 MFMA kernels) with its own workspace."""

    def __init__(self, max_batch: int, seed: int = 0, stream=None, device="cuda"):
        import torch
        b = C.c_size_t(0)
        _check(lib().aa_mlp_workspace_size(max_batch, C.byref(b)), "aa_mlp_workspace_size")
        self.workspace = torch.empty((b.value + 7) // 8, dtype=torch.float64, device=device)
        self.net = C.c_void_p()
        _check(lib().aa_mlp_init(C.byref(self.net), max_batch, seed, self.workspace.data_ptr(),
                                 b.value, _stream(stream)), "aa_mlp_init")
        self.P = lib().aa_mlp_param_count()

    def set_params(self, params):
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32)
        assert a.size == self.P
        _check(lib().aa_mlp_set_params(self.net, a.ctypes.data), "aa_mlp_set_params")

    def get_params(self):
        import numpy as np
        a = np.empty(self.P, dtype=np.float32)
        _check(lib().aa_mlp_get_params(self.net, a.ctypes.data), "aa_mlp_get_params")
        return a

    def get_grads(self):
        import numpy as np
        a = np.empty(self.P, dtype=np.float32)
        _check(lib().aa_mlp_get_grads(self.net, a.ctypes.data), "aa_mlp_get_grads")
        return a

    def forward(self, x, out=None):
        _check(lib().aa_mlp_forward(self.net, x.shape[0], x.data_ptr(), _ptr(out)),
               "aa_mlp_forward")

    def backward(self, dout):
        _check(lib().aa_mlp_backward(self.net, dout.shape[0], dout.data_ptr()), "aa_mlp_backward")

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        _check(lib().aa_mlp_adam(self.net, lr, b1, b2, eps), "aa_mlp_adam")

    def reseed(self, seed: int):
        _check(lib().aa_mlp_reseed(self.net, seed), "aa_mlp_reseed")

    def close(self):
        if getattr(self, "net", None) is not None and self.net.value:
            _check(lib().aa_mlp_destroy(self.net), "aa_mlp_destroy")
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

class PDE2D:
    """Owns a torch workspace and a library context of the 2D test problems'
    map (Sec. 5.1, 5.2): G(u) by PCG with the library's multigrid cycle."""

    def __init__(self, N: int, problem: int, lam: float = 6.7, tol: float = 1e-10,
                 max_iter: int = 200, device="cuda", stream=None):
        import torch
        self.N, self.problem = int(N), int(problem)
        nbytes = aa_pde2d_workspace_size(self.N, max_iter)
        self.workspace = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device)
        assert self.workspace.data_ptr() % 256 == 0
        self.ctx = aa_pde2d_init(self.N, self.problem, lam, tol, max_iter, self.workspace, stream)

    def apply(self, b, u, out):
        aa_pde2d_apply(self.ctx, b, u, out)

    def solve(self, rhs, x):
        aa_pde2d_solve(self.ctx, rhs, x)

    def vcycle(self, r, z):
        aa_pde2d_vcycle(self.ctx, r, z)

    def set_iters(self, iters: int):
        aa_pde2d_set_iters(self.ctx, iters)

    def last(self):
        return aa_pde2d_last(self.ctx)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and _lib is not None:
            _lib.aa_pde2d_destroy(ctx)
            self.ctx = None
