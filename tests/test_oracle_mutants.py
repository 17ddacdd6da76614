"""The oracle's pins have teeth: plant plausible mistakes in a copy of the
oracle source (a dropped term, a flipped sign, a wrong index, a transposed
operand), compile the copy on the CPU, and check that the pins reject it.

The real oracle is never modified; each mutant lives in a temporary directory.
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle as O

SRC = O.SRC_PATH

# (name, exact text in aa_oracle.c, replacement)
MUTANTS = [
    ("icwy_solve_sign", "acc -= TM(s, a, b) * rc[b];", "acc += TM(s, a, b) * rc[b];"),
    ("icwy_T_transposed", "acc -= TM(s, a, b) * rc[b];", "acc -= TM(s, b, a) * rc[b];"),
    ("cgs2_drop_z", "RM(s, j, k) = sc[j] + zc[j];", "RM(s, j, k) = sc[j];"),
    ("dcgs2_unscaled", "double scale = (flags & OR_DCGS2_LITERAL) ? 1.0 : RM(s, p, p);",
     "double scale = 1.0;"),
    ("givens_sign", "qb[r] = -sn * x + c * y;", "qb[r] = sn * x + c * y;"),
    ("givens_R_row", "RM(s, j + 1, col) = -sn * hj + c * hj1;", "RM(s, j + 1, col) = -sn * hj1 + c * hj;"),
    ("ring_index", "int64_t col = (i - m_i + j) % m;", "int64_t col = (i - m_i + j + 1) % m;"),
    ("backsolve_index", "acc -= R[a + (int64_t)b * cap] * gamma[b];",
     "acc -= R[b + (int64_t)a * cap] * gamma[b];"),
    ("mgs_stale_update", "axmy(s->n, rj, QCOL(s, j), v);", "(void)0;"),
    # ICWY's T after QRDelete by rotating the old Gram matrix
    ("T_transform_row_sign", "SM(j + 1, r) = -sn * x + c * y;", "SM(j + 1, r) = sn * x + c * y;"),
    ("T_transform_no_row_rotation", "SM(j, r) = c * x + sn * y;", "(void)x;"),
    # DCGS-2 with the normalization lagged
    ("lag_R_unscaled", "RM(s, j, p) = RM(s, j, p) + rpp * sc[j];",
     "RM(s, j, p) = RM(s, j, p) + sc[j];"),
    ("lag_rpk_no_correction", "double rpk = (beta - sz) / rho;", "double rpk = beta / rho;"),
    ("lag_norm_sign", "double rho2 = alpha - ss;", "double rho2 = alpha + ss;"),
]


def _compile(tmpdir, text):
    src = os.path.join(tmpdir, "m.c")
    so = os.path.join(tmpdir, "m.so")
    open(src, "w").write(text)
    subprocess.check_call(["gcc", "-O1", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", so, src, "-lm"])
    return so


def _run_pins(so):
    """A compact subset of the pins, run against the library at ``so``.
    Returns True when every pin passes."""
    saved = O._lib
    try:
        O._lib = None
        L = C.CDLL(so)
        real = O.LIB_PATH
        O.LIB_PATH = so
        try:
            lib = O.lib()
        finally:
            O.LIB_PATH = real
        del L
        rng = np.random.default_rng(0)
        n, m = 60, 5
        U, _ = np.linalg.qr(rng.standard_normal((n, m)))
        V, _ = np.linalg.qr(rng.standard_normal((m, m)))
        F = (U * np.logspace(0, -5, m)) @ V.T * 3.0
        for v in ["mgs", "cgs2", "dcgs2", "icwy"]:
            q = O.QR(n, m, v)
            for j in range(m):
                if q.add(F[:, j]) != 0:
                    return False
            Q, R = q.Qk(), q.Rk()
            if np.linalg.norm(F - Q @ R) > 1e-13 * np.linalg.norm(F):
                return False
            if q.delete() != 0:
                return False
            Q, R = q.Qk(), q.Rk()
            if np.linalg.norm(F[:, 1:] - Q @ R) > 1e-13 * np.linalg.norm(F):
                return False
            if np.linalg.norm(np.eye(m - 1) - Q.T @ Q) > 1e-9:
                return False
            # ICWY's next add uses the refreshed T
            w = rng.standard_normal(n)
            if q.add(w) != 0:
                return False
            Fn = np.column_stack([F[:, 1:], w])
            if np.linalg.norm(Fn - q.Qk() @ q.Rk()) > 1e-13 * np.linalg.norm(Fn):
                return False
        # ICWY's T solve reproduces MGS's coefficients on an ill-conditioned
        # MGS basis (entries of L ~ 1e-5, so the check has teeth)
        U2, _ = np.linalg.qr(rng.standard_normal((n, 6)))
        V2, _ = np.linalg.qr(rng.standard_normal((6, 6)))
        F2 = (U2 * np.logspace(0, -12, 6)) @ V2.T
        base = O.QR(n, 6, "mgs")
        for j in range(6):
            base.add(F2[:, j])
        Qb = base.Qk()
        w = rng.standard_normal(n)
        cols = {}
        for v in ("mgs", "icwy"):
            q = O.QR(n, 7, v)
            q.Q[:, :6] = Qb
            q.R[:6, :6] = base.Rk()
            q.T[:6, :6] = np.eye(6) + np.tril(Qb.T @ Qb, -1)
            q.s.k = 6
            if q.add(w) != 0:
                return False
            cols[v] = q.R[:6, 6].copy()
        if np.abs(cols["mgs"] - cols["icwy"]).max() > 1e-13 * np.linalg.norm(w):
            return False
        # Q R = F is an identity of every update, even on this non-orthonormal basis
        for v in ("mgs", "cgs2", "dcgs2", "icwy"):
            q = O.QR(n, 7, v)
            q.Q[:, :6] = Qb
            q.R[:6, :6] = base.Rk()
            q.T[:6, :6] = np.eye(6) + np.tril(Qb.T @ Qb, -1)
            q.s.k = 6
            if q.add(w) != 0:
                return False
            Fn = np.column_stack([Qb @ base.Rk(), w])
            if np.linalg.norm(Fn - q.Qk() @ q.Rk()) > 1e-13 * np.linalg.norm(Fn):
                return False
        # ICWY with T rotated after QRDelete: T stays the Gram of the basis
        q = O.QR(n, 6, "icwy", O.ICWY_T_TRANSFORM)
        for j in range(6):
            if q.add(F2[:, j]) != 0:
                return False
        if q.delete() != 0:
            return False
        Gq = q.Qk().T @ q.Qk()
        Tq = q.Tk()
        for a in range(1, 4):
            if np.abs(Tq[a, :a] - Gq[a, :a]).max() > 1e-13:
                return False
        # lagged DCGS-2 on the same non-orthonormal basis (its delayed
        # corrections s ~ 1e-4 are large here): Q R = F, the reorthogonalized
        # previous column has unit norm, the new column is orthogonal to it
        q = O.QR(n, 7, "dcgs2_lag")
        q.Q[:, :6] = Qb
        q.R[:6, :6] = base.Rk()
        q.s.k = 6
        if q.add(w) != 0:
            return False
        Fn = np.column_stack([Qb @ base.Rk(), w])
        if np.linalg.norm(Fn - q.Qk() @ q.Rk()) > 1e-13 * np.linalg.norm(Fn):
            return False
        if abs(np.linalg.norm(q.Q[:, 5]) - 1.0) > 1e-10 or abs(q.Q[:, 5] @ q.Q[:, 6]) > 1e-6:
            return False
        # lagged DCGS-2: Q R = F after each add, orthonormal after the last step
        q = O.QR(n, m, "dcgs2_lag")
        for j in range(m):
            if q.add(F[:, j]) != 0:
                return False
            if np.linalg.norm(F[:, : j + 1] - q.Qk() @ q.Rk()) > 1e-13 * np.linalg.norm(F):
                return False
        if q.flush() != 0 or np.linalg.norm(np.eye(m) - q.Qk().T @ q.Qk()) > 1e-13:
            return False
        # whole loop: AA == GMRES on a small SPD system
        A = rng.standard_normal((20, 20))
        A = A @ A.T / 20 + np.eye(20)
        b = rng.standard_normal(20)
        om = 0.9 / np.linalg.eigvalsh(A).max()
        G = lambda x: x - om * (A @ x - b)
        X = O.gmres(b, np.zeros(20), 8, A=A)
        for v in ["mgs", "icwy"]:
            xs, _, _ = O.run_aa(G, np.zeros(20), m=3, variant=v, iters=8)
            xs2, _, _ = O.run_aa(G, np.zeros(20), m=12, variant=v, iters=8)
            for k in range(8):
                if np.linalg.norm(xs2[k + 1] - G(X[:, k])) > 1e-10 * np.linalg.norm(xs2[k + 1]):
                    return False
            # truncated window: compare against the definition LSP
            st = O.AA(20, 3, v)
            x = np.zeros(20)
            hist_x, hist_g = [], []
            for i in range(8):
                g = G(x)
                hist_x.append(x); hist_g.append(g)
                xn = st.step(x, g)
                if i >= 1:
                    mi = min(3, i)
                    fs = [hist_g[j] - hist_x[j] for j in range(i + 1)]
                    Fm = np.stack([fs[j + 1] - fs[j] for j in range(i - mi, i)], 1)
                    Gm = np.stack([hist_g[j + 1] - hist_g[j] for j in range(i - mi, i)], 1)
                    ref = g - Gm @ O.lsp_definition(Fm, fs[i])
                    if np.linalg.norm(xn - ref) > 1e-9 * np.linalg.norm(ref):
                        return False
                x = xn
        return True
    finally:
        O._lib = saved


def test_unmutated_copy_passes(tmp_path):
    so = _compile(str(tmp_path), open(SRC).read())
    assert _run_pins(so)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    text = open(SRC).read()
    assert old in text, f"mutation anchor for {name} not found"
    so = _compile(str(tmp_path), text.replace(old, new, 1))
    assert not _run_pins(so), f"mutant {name} survived the pins"
