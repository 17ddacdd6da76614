"""FP64 CPU oracle for Anderson acceleration with windowed QR updates.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product path (the HIP library
and its binding) never imports this package, and this package never imports
the product.  The arithmetic lives in ``aa_oracle.c`` (plain C, FP64, no FMA
contraction, compensated dot products); this module only marshals numpy
arrays and adds the "definition" least-squares solve used as a second,
independent route to the same answer.

Parity pins for every function here are the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "aa_oracle.c")

MGS, CGS2, DCGS2, ICWY, DCGS2_LAG = 0, 1, 2, 3, 4
VARIANTS = {"mgs": MGS, "cgs2": CGS2, "dcgs2": DCGS2, "icwy": ICWY, "dcgs2_lag": DCGS2_LAG}
DCGS2_LITERAL = 1 << 1
ICWY_T_TRANSFORM = 1 << 2
DCGS2_GUARD_GE3 = 1 << 4
OK, EINVAL, EBREAKDOWN, ESTATE = 0, -1, -3, -4


OMP_LIB_PATH = os.path.join(HERE, "liboracle_omp.so")


def build(force: bool = True) -> str:
    """Compile ``aa_oracle.c`` into ``liboracle.so`` with gcc (FP64, no
    contraction), and the same source with OpenMP into ``liboracle_omp.so``
    (the CPU baseline: fixed row blocks, so the results are bitwise those of
    the single-threaded build for any thread count)."""
    for path, extra in ((LIB_PATH, []), (OMP_LIB_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call([
                "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                "-fPIC", "-shared", "-Wall", *extra, "-o", tmp, SRC_PATH, "-lm"])
            os.replace(tmp, path)
    return LIB_PATH


def use_openmp(threads: int) -> int:
    """Switch this process to the OpenMP build with ``threads`` threads (the
    CPU baseline); returns the thread count in effect."""
    global _lib, _lib_omp
    if _lib_omp is None:
        if not os.path.exists(OMP_LIB_PATH):
            build(force=False)
        saved, real = _lib, LIB_PATH
        try:
            _lib = None
            globals()["LIB_PATH"] = OMP_LIB_PATH
            _lib_omp = lib()
        finally:
            globals()["LIB_PATH"] = real
    _lib = _lib_omp
    return int(_lib.or_set_threads(int(threads)))


_lib = None
_lib_omp = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.or_qr_add.argtypes = [C.POINTER(_QR), C.c_int, C.c_uint, P]
        L.or_qr_delete.argtypes = [C.POINTER(_QR), C.c_int, C.c_uint]
        L.or_qr_flush.argtypes = [C.POINTER(_QR), C.c_int]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_qr_rhs.argtypes = [C.POINTER(_QR), P, P]
        L.or_qr_rhs.restype = None
        L.or_backsolve.argtypes = [C.c_int, C.c_int, P, P, P]
        L.or_aa_step.argtypes = [C.POINTER(_AA), P, P, P]
        L.or_G_stencil.argtypes = [C.c_int, C.c_int64, C.c_double, C.c_double,
                                   C.c_double, P, P, P]
        L.or_G_stencil.restype = None
        L.or_G_em.argtypes = [C.c_int64, P, P, C.c_int64, P, P, P]
        L.or_G_em.restype = None
        L.or_laplacian.argtypes = [C.c_int, C.c_int64, C.c_double, P, P]
        L.or_laplacian.restype = None
        L.or_gmres.argtypes = [C.c_int64, P, C.c_int, C.c_int64, C.c_double,
                               P, P, C.c_int, P]
        _lib = L
    return _lib


class _QR(C.Structure):
    _fields_ = [("n", C.c_int64), ("ld", C.c_int64), ("cap", C.c_int),
                ("k", C.c_int), ("Q", C.c_void_p), ("R", C.c_void_p),
                ("T", C.c_void_p), ("work", C.c_void_p),
                ("syncs_add", C.c_int64), ("syncs_delete", C.c_int64),
                ("syncs_rhs", C.c_int64)]


class _AA(C.Structure):
    _fields_ = [("qr", _QR), ("m", C.c_int), ("variant", C.c_int),
                ("flags", C.c_uint), ("i", C.c_int64), ("m_i", C.c_int),
                ("f_prev", C.c_void_p), ("g_prev", C.c_void_p),
                ("dG", C.c_void_p), ("dF", C.c_void_p),
                ("gamma", C.c_void_p), ("c", C.c_void_p), ("f", C.c_void_p),
                ("res_norm", C.c_double), ("res0_norm", C.c_double),
                ("step_norm", C.c_double), ("status", C.c_int)]


def _ptr(a: np.ndarray) -> int:
    assert a.dtype == np.float64 and (a.flags.c_contiguous or a.flags.f_contiguous)
    return a.ctypes.data


def _variant(v) -> int:
    return VARIANTS[v] if isinstance(v, str) else int(v)


class QR:
    """Windowed QR factorization F = Q R held in numpy arrays (Alg. 2)."""

    def __init__(self, n: int, cap: int, variant="mgs", flags: int = 0):
        self.n, self.cap = int(n), int(cap)
        self.variant, self.flags = _variant(variant), int(flags)
        self.Q = np.zeros((self.n, self.cap), order="F")
        self.R = np.zeros((self.cap, self.cap), order="F")
        self.T = np.zeros((self.cap, self.cap), order="F")
        self.work = np.zeros(2 * self.n)
        self.s = _QR(self.n, self.n, self.cap, 0, _ptr(self.Q), _ptr(self.R),
                     _ptr(self.T), _ptr(self.work), 0, 0, 0)

    @property
    def k(self) -> int:
        return self.s.k

    @property
    def syncs(self) -> tuple[int, int, int]:
        """(reductions in QRAdd, in QRDelete, in Q^T f) so far."""
        return self.s.syncs_add, self.s.syncs_delete, self.s.syncs_rhs

    def add(self, v) -> int:
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert v.shape == (self.n,)
        return lib().or_qr_add(C.byref(self.s), self.variant, self.flags, _ptr(v))

    def delete(self) -> int:
        return lib().or_qr_delete(C.byref(self.s), self.variant, self.flags)

    def flush(self) -> int:
        """The lagged DCGS-2's final reorthogonalization and normalization of
        the newest column (one reduction); other variants: EINVAL."""
        return lib().or_qr_flush(C.byref(self.s), self.variant)

    def rhs(self, f) -> np.ndarray:
        f = np.ascontiguousarray(f, dtype=np.float64)
        c = np.zeros(max(self.k, 1))
        lib().or_qr_rhs(C.byref(self.s), _ptr(f), _ptr(c))
        return c[: self.k]

    def solve(self, f) -> np.ndarray:
        c = np.zeros(max(self.k, 1))
        c[: self.k] = self.rhs(f)
        g = np.zeros(max(self.k, 1))
        st = lib().or_backsolve(self.k, self.cap, _ptr(self.R), _ptr(c), _ptr(g))
        if st != OK:
            raise FloatingPointError("breakdown in back substitution")
        return g[: self.k]

    def Qk(self) -> np.ndarray:
        return self.Q[:, : self.k].copy()

    def Rk(self) -> np.ndarray:
        return self.R[: self.k, : self.k].copy()

    def Tk(self) -> np.ndarray:
        return self.T[: self.k, : self.k].copy()


class AA:
    """Anderson acceleration state stepped one iteration at a time (Alg. 1)."""

    def __init__(self, n: int, m: int, variant="mgs", flags: int = 0):
        self.n, self.m = int(n), int(m)
        self.qr = QR(n, m, variant, flags)
        z = lambda *shape: np.zeros(shape, order="F")
        self.f_prev, self.g_prev, self.f = z(n), z(n), z(n)
        self.dG, self.dF = z(n, m), z(n, m)
        self.gamma, self.c = z(m), z(m)
        self.s = _AA(self.qr.s, self.m, self.qr.variant, self.qr.flags, 0, 0,
                     _ptr(self.f_prev), _ptr(self.g_prev), _ptr(self.dG),
                     _ptr(self.dF), _ptr(self.gamma), _ptr(self.c), _ptr(self.f),
                     0.0, 0.0, 0.0, 0)
        # the embedded QR struct is a copy: point the QR view at it
        self.qr.s = self.s.qr

    def step(self, x, g) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        out = np.empty(self.n)
        st = lib().or_aa_step(C.byref(self.s), _ptr(x), _ptr(g), _ptr(out))
        if st != OK:
            raise FloatingPointError(f"oracle AA step status {st}")
        return out

    @property
    def i(self) -> int:
        return self.s.i

    @property
    def m_i(self) -> int:
        return self.s.m_i

    @property
    def k(self) -> int:
        return self.s.qr.k

    @property
    def res_norm(self) -> float:
        return self.s.res_norm

    @property
    def res0_norm(self) -> float:
        return self.s.res0_norm

    @property
    def step_norm(self) -> float:
        return self.s.step_norm

    @property
    def syncs(self):
        q = self.s.qr
        return q.syncs_add, q.syncs_delete, q.syncs_rhs

    def F(self) -> np.ndarray:
        """F_i = [Delta f_{i-m_i} .. Delta f_{i-1}] in window order (oracle only)."""
        i, mi = self.s.i - 1, self.s.m_i
        return np.stack([self.dF[:, (i - mi + j) % self.m] for j in range(mi)], 1)

    def Gmat(self) -> np.ndarray:
        i, mi = self.s.i - 1, self.s.m_i
        return np.stack([self.dG[:, (i - mi + j) % self.m] for j in range(mi)], 1)

    def Qk(self):
        return self.qr.Q[:, : self.k].copy()

    def Rk(self):
        return self.qr.R[: self.k, : self.k].copy()

    def Tk(self):
        return self.qr.T[: self.k, : self.k].copy()

    def gamma_k(self):
        return self.gamma[: self.m_i].copy()


# --------------------------------------------------------------------------
# model problems, GMRES and the definition LSP
# --------------------------------------------------------------------------

def G_stencil(prob, u) -> np.ndarray:
    """G(u) = u - omega (A u + c u^3 - f) for an ``aa_workloads.StencilProblem``."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.ascontiguousarray(prob.f, dtype=np.float64)
    out = np.empty_like(u)
    lib().or_G_stencil(prob.d, prob.s, prob.h, prob.omega, prob.c, _ptr(f),
                       _ptr(u), _ptr(out))
    return out


def G_em(prob, u) -> np.ndarray:
    """The EM map of Sec. 5.3 for an ``aa_workloads.EMProblem``: the means in
    u[0:3] updated from the samples, written to every replica."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    x = np.ascontiguousarray(prob.samples, dtype=np.float64)
    a = np.ascontiguousarray(prob.alpha, dtype=np.float64)
    sg = np.ascontiguousarray(prob.sigma, dtype=np.float64)
    out = np.empty_like(u)
    lib().or_G_em(u.shape[0], _ptr(u), _ptr(x), x.shape[0], _ptr(a), _ptr(sg), _ptr(out))
    return out


def laplacian(d: int, s: int, h: float, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    y = np.empty_like(u)
    lib().or_laplacian(d, s, h, _ptr(u), _ptr(y))
    return y


def gmres(b, x0, K: int, A=None, d: int = 1, s: int = 0, h: float = 1.0) -> np.ndarray:
    """GMRES iterates x_0..x_K (columns) for A x = b; A dense or the Laplacian."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    n = b.shape[0]
    X = np.zeros((n, K + 1), order="F")
    Ad = None if A is None else np.asfortranarray(A, dtype=np.float64)
    done = lib().or_gmres(n, None if Ad is None else _ptr(Ad), d, s, h, _ptr(b),
                          _ptr(x0), K, _ptr(X))
    return X[:, : done + 1]


def lsp_definition(F: np.ndarray, f: np.ndarray) -> np.ndarray:
    """gamma = argmin ||f - F gamma||_2 by Householder QR of the explicit F
    (Alg. 1's least-squares problem by its definition, not by the update)."""
    Qh, Rh = np.linalg.qr(F, mode="reduced")
    return np.linalg.solve(np.triu(Rh), Qh.T @ f)


def run_aa(G, x0, m: int, variant="mgs", iters: int = 20, flags: int = 0,
           tol: float = 0.0, record=True):
    """Drive Alg. 1 for ``iters`` iterations (or until ||f_i|| <= tol ||f_0||).

    Returns (list of iterates x_0..x_I, AA state, list of ||f_i||)."""
    st = AA(x0.shape[0], m, variant, flags)
    xs, res = [x0.copy()], []
    x = x0.copy()
    for _ in range(iters + 1):
        g = G(x)
        if st.i >= 1 and tol > 0.0:
            f_norm = np.linalg.norm(g - x)
            if f_norm <= tol * st.res0_norm:
                res.append(f_norm)
                break
        x = st.step(x, g)
        res.append(st.res_norm)
        if record:
            xs.append(x.copy())
    return xs, st, res


# --------------------------------------------------------------------------
# learned-guarded step (an addition to the paper's method, used to pin the
# GPU training gradient): candidate and one-step loss from the oracle's state
# --------------------------------------------------------------------------

def learned_candidate(st: "AA", g: np.ndarray, dgamma: np.ndarray, beta: float) -> np.ndarray:
    """x_c = G(x_i) - G_i gamma' - (1 - beta)(f_i - Q R gamma'), gamma' = gamma +
    dgamma, from the state right after the oracle's step i (its gamma, Q, R,
    window of Delta g and f_i)."""
    gp = st.gamma_k() + dgamma[: st.m_i]
    Fg = st.Qk() @ (st.Rk() @ gp)
    return g - st.Gmat() @ gp - (1.0 - beta) * (st.f - Fg)


def learned_loss(prob, st: "AA", g: np.ndarray, outputs: np.ndarray) -> float:
    """log(||G(x_c) - x_c||^2 / ||f_i||^2) for network outputs (delta gamma in
    outputs[:20] masked to m_i, beta = sigmoid(outputs[20]))."""
    dg = np.zeros(20)
    dg[: st.m_i] = outputs[: st.m_i]
    beta = 1.0 / (1.0 + np.exp(-outputs[20]))
    xc = learned_candidate(st, g, dg, beta)
    r = G_stencil(prob, xc) - xc
    return float(np.log(np.dot(r, r) / np.dot(st.f, st.f)))
