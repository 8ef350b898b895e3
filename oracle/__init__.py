"""ctypes wrapper of the FP64 CPU oracle (``omg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark. The GPU library never imports, links or
calls it, and it never imports the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "omg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAXLEV = 16

OK, EINVAL, ENOMEM, ENOTSPD, ENOCONV, EUNSUPPORTED = 0, -1, -2, -4, -5, -7


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Opts(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int), ("coarse_sync", ctypes.c_int), ("s_pre", ctypes.c_int),
        ("s_post", ctypes.c_int), ("n_s", ctypes.c_int), ("max_iter", ctypes.c_int),
        ("precision", ctypes.c_int), ("gs", ctypes.c_int), ("alpha_mode", ctypes.c_int),
        ("m_max", ctypes.c_int), ("max_outer", ctypes.c_int), ("n_crit", ctypes.c_int),
        ("smoother", ctypes.c_int), ("pad_smoother", ctypes.c_int),
        ("omega", ctypes.c_double), ("inner_tol", ctypes.c_double), ("breakdown", ctypes.c_double),
        ("crit_rel", ctypes.c_double * MAXLEV), ("crit_max", ctypes.c_int * MAXLEV),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("iters_fine", ctypes.c_int), ("n_dirs_fine", ctypes.c_int),
        ("n_breakdowns", ctypes.c_int), ("outer_iters", ctypes.c_int), ("n_visits", ctypes.c_int),
        ("n_trace", ctypes.c_int), ("n_vnorm", ctypes.c_int),
        ("rel_res_rec", ctypes.c_double), ("rel_res_true", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        # OMG_ORACLE_LIB: another build of the same source (the sanitizer
        # test loads an AddressSanitizer/UBSan build this way)
        path = os.environ.get("OMG_ORACLE_LIB")
        if not path:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            path = _LIB
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i, d, i64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
        L.oracle_setup.argtypes = [P, P, P, i64, i, i, i, i, i, P, ctypes.POINTER(P)]
        L.oracle_setup_sip.argtypes = [i, i, i, i, d, d, P, i, P, ctypes.POINTER(P)]
        L.oracle_setup_h.argtypes = [P, P, P, i64, i, i, P, P, P, P, P, ctypes.POINTER(P)]
        L.oracle_solve.argtypes = [P, P, P, d, P]
        L.oracle_grad.argtypes = [P, P, P, P, P, d, P]
        L.oracle_destroy.argtypes = [P]
        L.oracle_destroy.restype = None
        L.oracle_level_info.argtypes = [P, i, P, P, P]
        L.oracle_get_matrix.argtypes = [P, i, P, P, P]
        L.oracle_get_embedding.argtypes = [P, P]
        L.oracle_embedding_p.argtypes = [i, P]
        L.oracle_get_dirs.argtypes = [P, i, P, P]
        L.oracle_get_residual.argtypes = [P, i, P]
        L.oracle_get_visits.argtypes = [P, P]
        L.oracle_set_step_schedule.argtypes = [P, P, i]
        L.oracle_get_trace.argtypes = [P, P]
        L.oracle_get_visit_norms.argtypes = [P, P]
        L.oracle_spmv32.argtypes = [P, i, P, P, P]
        L.oracle_restrict32.argtypes = [P, i, P, P]
        L.oracle_prolong32.argtypes = [P, i, P, P]
        L.oracle_spmv.argtypes = [P, i, P, P, P]
        L.oracle_smoother.argtypes = [P, i, P, i, P]
        L.oracle_smoother32.argtypes = [P, i, P, i, P]
        L.oracle_restrict.argtypes = [P, i, P, P]
        L.oracle_prolong.argtypes = [P, i, P, P]
        L.oracle_coarse_solve.argtypes = [P, P, P]
        L.oracle_get_dinv.argtypes = [P, i, P]
        L.oracle_element.argtypes = [i, d, d, P, P, P]
        L.oracle_default_opts.argtypes = [P]
        L.oracle_default_opts.restype = None
        L.oracle_nbasis.argtypes = [i]
        L.oracle_num_threads.argtypes = []
        L.oracle_set_threads.argtypes = [i]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_opts(**kw) -> Opts:
    """Options: variant ('sync'|'overlap'|'hybrid'|'add_sync' or 0|1|2|3), smoother ('bj'|'schwarz'),
    s_pre, s_post, n_s, omega,
    max_iter, precision ('fp64'|'mixed_ir'|'mixed_flex' or 0|1|2), gs
    ('mgs'|'mgs2'), alpha_mode, m_max, inner_tol, max_outer, breakdown,
    coarse_sync, crit (list of (rel, max) for levels 1, 2, ...)."""
    o = Opts()
    lib().oracle_default_opts(ctypes.byref(o))
    names = {"sync": 0, "overlap": 1, "hybrid": 2, "add_sync": 3, "bj": 0, "schwarz": 1, "fp64": 0, "mixed_ir": 1, "mixed_flex": 2, "mgs": 0, "mgs2": 1}
    crit = kw.pop("crit", None)
    for k, v in kw.items():
        if isinstance(v, str):
            v = names[v]
        setattr(o, k, v)
    if crit is not None:
        for l in range(MAXLEV):
            rel, mx = crit[l] if l < len(crit) else (-1.0, 1)
            o.crit_rel[l] = rel
            o.crit_max[l] = mx
    return o


class Oracle:
    """Owns one oracle solver (hierarchy + coarse factor)."""

    def __init__(self, handle, n_cells, bs, n_levels, nu=None):
        self._h = handle
        self.n_cells = n_cells
        self.bs = bs
        self.n = n_cells * bs
        self.n_levels = n_levels
        self.nu = nu
        self.last_report = None

    @classmethod
    def from_sip(cls, prob, nu, **opts):
        nu = np.ascontiguousarray(nu, dtype=np.float64)
        h = ctypes.c_void_p()
        o = make_opts(**opts)
        st = lib().oracle_setup_sip(prob.nx, prob.ny, prob.nz, prob.p, prob.h, prob.penalty_c, _p(nu),
                                    prob.n_levels, ctypes.byref(o), ctypes.byref(h))
        if st != OK:
            raise OracleError(st)
        return cls(h, prob.n_cells, prob.bs, prob.n_levels, nu)

    @classmethod
    def from_bsr(cls, row_ptr, col_idx, val, nx, ny, nz, p, n_levels, **opts):
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        h = ctypes.c_void_p()
        o = make_opts(**opts)
        st = lib().oracle_setup(_p(row_ptr), _p(col_idx), _p(val), len(col_idx), nx, ny, nz, p, n_levels,
                                ctypes.byref(o), ctypes.byref(h))
        if st != OK:
            raise OracleError(st)
        bs = lib().oracle_nbasis(p)
        return cls(h, nx * ny * nz, bs, n_levels)

    @classmethod
    def from_bsr_hierarchy(cls, row_ptr, col_idx, val, n_cells, parents, slots, embed, **opts):
        """Setup with a caller-supplied agglomeration hierarchy: level sizes
        n_cells[0..L-1], per level l < L-1 the parent (int) and slot (0..7) of
        every cell, and the embedding blocks embed[8][bs][bs]."""
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        nc = np.ascontiguousarray(n_cells, dtype=np.int32)
        par = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.int32) for p in parents])
                                   if len(parents) else np.zeros(1, np.int32))
        sl = np.ascontiguousarray(np.concatenate([np.asarray(q, dtype=np.uint8) for q in slots])
                                  if len(slots) else np.zeros(1, np.uint8))
        E = np.ascontiguousarray(embed, dtype=np.float64)
        bs = val.shape[1]
        h = ctypes.c_void_p()
        o = make_opts(**opts)
        st = lib().oracle_setup_h(_p(row_ptr), _p(col_idx), _p(val), len(col_idx), bs, len(nc), _p(nc), _p(par),
                                  _p(sl), _p(E), ctypes.byref(o), ctypes.byref(h))
        if st != OK:
            raise OracleError(st)
        return cls(h, int(nc[0]), bs, len(nc))

    def close(self):
        if self._h:
            lib().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, x0=None, tol=1e-10, check=True):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        rep = Report()
        st = lib().oracle_solve(self._h, _p(b), _p(x), tol, ctypes.byref(rep))
        self.last_report = rep.as_dict()
        if check and st not in (OK,):
            raise OracleError(st, x=x, report=self.last_report)
        return x

    def grad(self, u, g_u, tol=1e-10):
        u = np.ascontiguousarray(u, dtype=np.float64)
        g_u = np.ascontiguousarray(g_u, dtype=np.float64)
        g_f = np.zeros(self.n)
        g_nu = np.zeros(self.n_cells)
        rep = Report()
        st = lib().oracle_grad(self._h, _p(u), _p(g_u), _p(g_f), _p(g_nu), tol, ctypes.byref(rep))
        self.last_report = rep.as_dict()
        if st != OK:
            raise OracleError(st, report=self.last_report)
        return g_f, g_nu

    def level_info(self, l):
        n = ctypes.c_int()
        nnzb = ctypes.c_int64()
        k = ctypes.c_int()
        lib().oracle_level_info(self._h, l, ctypes.byref(n), ctypes.byref(nnzb), ctypes.byref(k))
        return n.value, nnzb.value, k.value

    def matrix(self, l=0):
        n, nnzb, _ = self.level_info(l)
        rp = np.zeros(n + 1, dtype=np.int32)
        ci = np.zeros(nnzb, dtype=np.int32)
        v = np.zeros((nnzb, self.bs, self.bs))
        lib().oracle_get_matrix(self._h, l, _p(rp), _p(ci), _p(v))
        return rp, ci, v

    def scipy_matrix(self, l=0):
        import scipy.sparse as sp
        rp, ci, v = self.matrix(l)
        return sp.bsr_matrix((v, ci, rp), shape=(len(rp) - 1) * np.array([self.bs, self.bs])).tocsr()

    def embedding(self):
        E = np.zeros((8, self.bs, self.bs))
        lib().oracle_get_embedding(self._h, _p(E))
        return E

    def dirs(self, l=0):
        n, _, k = self.level_info(l)
        N = n * self.bs
        W = np.zeros((k, N))
        Z = np.zeros((k, N))
        lib().oracle_get_dirs(self._h, l, _p(W), _p(Z))
        return W, Z

    def residual(self, l=0):
        n, _, _ = self.level_info(l)
        r = np.zeros(n * self.bs)
        lib().oracle_get_residual(self._h, l, _p(r))
        return r

    def visits(self):
        cnt = self.last_report["n_visits"]
        out = np.zeros(2 * max(cnt, 1), dtype=np.int32)
        m = lib().oracle_get_visits(self._h, _p(out))
        return out[: 2 * m].reshape(m, 2)

    def set_step_schedule(self, counts):
        """Smoother-step counts per cycle of the forking level for the next
        solves (replay of a timing-adaptive run); empty clears."""
        c = np.ascontiguousarray(counts, dtype=np.int32)
        st = lib().oracle_set_step_schedule(self._h, _p(c) if len(c) else None, len(c))
        if st != OK:
            raise OracleError(st)

    def trace(self):
        cnt = self.last_report["n_trace"]
        out = np.zeros(3 * max(cnt, 1))
        m = lib().oracle_get_trace(self._h, _p(out))
        return out[: 3 * m].reshape(m, 3)

    def visit_norms(self):
        """Per-visit residual log of the last solve, in completion order: a list
        of (level, iterations, ||r0||, array of ||r|| after each iteration)."""
        cnt = self.last_report["n_vnorm"]
        out = np.zeros(max(cnt, 1))
        m = lib().oracle_get_visit_norms(self._h, _p(out))
        return parse_visit_norms(out[:m])

    def spmv(self, x, l=0, b=None, fp32=False):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
        f = lib().oracle_spmv32 if fp32 else lib().oracle_spmv
        st = f(self._h, l, _p(x), None if bb is None else _p(bb), _p(y))
        if st != OK:
            raise OracleError(st)
        return y

    def smoother(self, r, s, l=0, fp32=False):
        r = np.ascontiguousarray(r, dtype=np.float64)
        out = np.zeros_like(r)
        st = (lib().oracle_smoother32 if fp32 else lib().oracle_smoother)(self._h, l, _p(r), s, _p(out))
        if st != OK:
            raise OracleError(st)
        return out

    def restrict(self, r, l=0, fp32=False):
        r = np.ascontiguousarray(r, dtype=np.float64)
        nc, _, _ = self.level_info(l + 1)
        rc = np.zeros(nc * self.bs)
        st = (lib().oracle_restrict32 if fp32 else lib().oracle_restrict)(self._h, l, _p(r), _p(rc))
        if st != OK:
            raise OracleError(st)
        return rc

    def prolong(self, zc, l=0, fp32=False):
        zc = np.ascontiguousarray(zc, dtype=np.float64)
        n, _, _ = self.level_info(l)
        z = np.zeros(n * self.bs)
        st = (lib().oracle_prolong32 if fp32 else lib().oracle_prolong)(self._h, l, _p(zc), _p(z))
        if st != OK:
            raise OracleError(st)
        return z

    def coarse_solve(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        lib().oracle_coarse_solve(self._h, _p(b), _p(x))
        return x

    def dinv(self, l=0):
        n, _, _ = self.level_info(l)
        D = np.zeros((n, self.bs, self.bs))
        st = lib().oracle_get_dinv(self._h, l, _p(D))
        if st != OK:
            raise OracleError(st)
        return D


def parse_visit_norms(v):
    """Split a flat per-visit log (level, iterations, ||r0||, ||r||...) into
    (level, iterations, r0, array of ||r|| per iteration) tuples."""
    out, i = [], 0
    v = np.asarray(v, dtype=np.float64)
    while i < len(v):
        l, it = int(v[i]), int(v[i + 1])
        out.append((l, it, float(v[i + 2]), v[i + 3:i + 3 + it].copy()))
        i += 3 + it
    return out


class OracleError(RuntimeError):
    def __init__(self, status, x=None, report=None):
        super().__init__(f"oracle status {status}")
        self.status = status
        self.x = x
        self.report = report


def embedding(p: int) -> np.ndarray:
    bs = lib().oracle_nbasis(p)
    E = np.zeros((8, bs, bs))
    st = lib().oracle_embedding_p(p, _p(E))
    if st != OK:
        raise OracleError(st)
    return E


def element(p: int, h: float, penalty_c: float = 4.0):
    """Unit-coefficient element matrices: S, F[d][X][Y], B[d][side]."""
    bs = lib().oracle_nbasis(p)
    S = np.zeros((bs, bs))
    F = np.zeros((3, 2, 2, bs, bs))
    B = np.zeros((3, 2, bs, bs))
    lib().oracle_element(p, h, penalty_c, _p(S), _p(F), _p(B))
    return S, F, B


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's row-parallel loops from now on."""
    lib().oracle_set_threads(int(n))
