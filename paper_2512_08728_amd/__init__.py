"""Python binding of the MI355X OrthoMG library (``libomg.so``).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels. torch supplies device memory (tensor ``data_ptr()``) and the current
HIP stream. Importing this module does not load the library; the first use
does, and raises if the built library is missing (no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libomg.so")
# the persistent RM kernel's launch configurations chosen per device kind and
# level size (read by the library; sizes not listed are tuned and appended)
TUNE_FILE = os.path.join(_HERE, "rm_tuning.jsonl")
MAX_LEVELS = 16

OK, EINVAL, ENOMEM, EHIP, ENOTSPD, ENOCONV, EBREAKDOWN, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
SYNC_MULT, OVERLAP_DET, HYBRID, ADD_SYNC = 0, 1, 2, 3
FP64, MIXED_IR, MIXED_FLEX = 0, 1, 2
SMOOTH_BJ, SMOOTH_AS = 0, 1


class OmgError(RuntimeError):
    def __init__(self, status, what=""):
        msg = lib().omg_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("p", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("pad", ctypes.c_int32), ("h", ctypes.c_double),
                ("penalty_c", ctypes.c_double)]


class Bsr(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32), ("bs", ctypes.c_int32), ("nnzb", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class HierarchyC(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("pad", ctypes.c_int32), ("n_cells", ctypes.c_void_p),
                ("parent", ctypes.c_void_p), ("slot", ctypes.c_void_p), ("embed", ctypes.c_void_p)]


class Hierarchy:
    """An agglomeration hierarchy for omg_setup / omg_setup_sip (host arrays):
    level sizes ``n_cells``, per level l < L-1 the ``parents[l]`` (int32) and
    ``slots[l]`` (uint8, 0..7) of its cells, and the eight embedding blocks
    ``embed`` [8][bs][bs] (None: the library's basis, omg_setup_sip only)."""

    def __init__(self, n_cells, parents, slots, embed=None):
        self.n_cells = np.ascontiguousarray(n_cells, dtype=np.int32)
        self.parents = [np.ascontiguousarray(p, dtype=np.int32) for p in parents]
        self.slots = [np.ascontiguousarray(q, dtype=np.uint8) for q in slots]
        self.embed = None if embed is None else np.ascontiguousarray(embed, dtype=np.float64)
        self._pp = (ctypes.c_void_p * max(len(self.parents), 1))(*[a.ctypes.data for a in self.parents])
        self._sp = (ctypes.c_void_p * max(len(self.slots), 1))(*[a.ctypes.data for a in self.slots])
        self.c = HierarchyC(len(self.n_cells), 0, self.n_cells.ctypes.data,
                            ctypes.cast(self._pp, ctypes.c_void_p) if self.parents else None,
                            ctypes.cast(self._sp, ctypes.c_void_p) if self.slots else None,
                            None if self.embed is None else self.embed.ctypes.data)

    @property
    def n_levels(self):
        return len(self.n_cells)

    @classmethod
    def of_grid(cls, grid: "Grid"):
        """The 2x2x2 agglomeration of a Cartesian grid (omg_grid_hierarchy) with
        the library's embedding blocks (omg_embedding)."""
        L = lib()
        n_cells = [(grid.nx >> l) * (grid.ny >> l) * (grid.nz >> l) for l in range(grid.n_levels)]
        parents, slots = [], []
        for l in range(grid.n_levels - 1):
            par = np.zeros(n_cells[l], dtype=np.int32)
            sl = np.zeros(n_cells[l], dtype=np.uint8)
            _check(L.omg_grid_hierarchy(ctypes.byref(grid), l, par.ctypes.data, sl.ctypes.data), "grid_hierarchy")
            parents.append(par)
            slots.append(sl)
        bs = (grid.p + 1) * (grid.p + 2) * (grid.p + 3) // 6
        E = np.zeros((8, bs, bs))
        _check(L.omg_embedding(grid.p, E.ctypes.data), "embedding")
        return cls(n_cells, parents, slots, E)


class Options(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("coarse_sync", ctypes.c_int32), ("s_pre", ctypes.c_int32),
                ("s_post", ctypes.c_int32), ("n_s", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("overlap_streams", ctypes.c_int32), ("trace", ctypes.c_int32),
                ("n_s_max", ctypes.c_int32), ("smoother", ctypes.c_int32), ("m_max", ctypes.c_int32),
                ("pad1", ctypes.c_int32),
                ("omega", ctypes.c_double), ("inner_tol", ctypes.c_double), ("breakdown", ctypes.c_double),
                ("crit_rel", ctypes.c_double * MAX_LEVELS), ("crit_max", ctypes.c_int32 * MAX_LEVELS)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters_fine", ctypes.c_int32), ("n_dirs_fine", ctypes.c_int32),
                ("n_breakdowns", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("n_visits", ctypes.c_int32),
                ("n_trace", ctypes.c_int32), ("pad", ctypes.c_int32), ("rel_res_rec", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("t_solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


_lib = None
EXPORTS = ["omg_default_options", "omg_grid_hierarchy", "omg_embedding", "omg_get_visit_norms",
           "omg_setup", "omg_setup_sip", "omg_solve", "omg_solve_batched",
           "omg_solve_backward", "omg_destroy", "omg_strerror", "omg_level_info", "omg_level_matrix",
           "omg_level_spmv", "omg_level_smoother", "omg_level_restrict", "omg_level_prolong", "omg_coarse_solve",
           "omg_get_dirs", "omg_get_visits", "omg_get_trace", "omg_get_step_counts", "omg_set_replay", "omg_bench_kernel",
           "omg_get_kernel_counts", "omg_probe_kernel", "omg_probe_result", "omg_level_multi",
           "omg_level_tuning", "omg_level_rm_step", "omg_level_rm_configs", "omg_rm_step_noalloc",
           "omg_level_set_rm_config"]
MR_SPMV, MR_SMOOTHER, MR_COARSE = 0, 1, 2
K_SPMV, K_SPMV32, K_BJ, K_BJ32, K_MGS, K_RESTRICT, K_PROLONG, K_COARSE, K_RMFIN, K_BJFIRST, K_RMP, K_COPY = range(12)
K_NAMES = ["spmv", "spmv32", "bj_sweep", "bj_sweep32", "mgs_step", "restrict", "prolong", "coarse_gemv",
           "rm_finish", "bj_first", "rm_persistent", "copy"]


def lib():
    """Load libomg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2512_08728_amd/build.py "
                              "(no CPU fallback exists)")
        os.environ.setdefault("OMG_RM_TUNE_FILE", TUNE_FILE)
        L = ctypes.CDLL(LIB_PATH)
        P, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.omg_default_options.argtypes = [P]
        L.omg_default_options.restype = None
        L.omg_grid_hierarchy.argtypes = [P, i32, P, P]
        L.omg_embedding.argtypes = [i32, P]
        L.omg_get_visit_norms.argtypes = [P, P, i32, P]
        L.omg_setup.argtypes = [P, P, P, P, ctypes.POINTER(P)]
        L.omg_setup_sip.argtypes = [P, P, P, P, P, ctypes.POINTER(P)]
        L.omg_solve.argtypes = [P, P, P, d, P, P]
        L.omg_solve_batched.argtypes = [P, i32, i32, P, P, d, P]
        L.omg_solve_backward.argtypes = [P, P, P, P, P, d, P]
        L.omg_destroy.argtypes = [P]
        L.omg_destroy.restype = None
        L.omg_strerror.argtypes = [ctypes.c_int]
        L.omg_strerror.restype = ctypes.c_char_p
        L.omg_level_info.argtypes = [P, i32, P, P, P]
        L.omg_level_matrix.argtypes = [P, i32, P, P, P, P]
        L.omg_level_spmv.argtypes = [P, i32, i32, P, P, P]
        L.omg_level_smoother.argtypes = [P, i32, i32, P, i32, P]
        L.omg_level_restrict.argtypes = [P, i32, i32, P, P]
        L.omg_level_prolong.argtypes = [P, i32, i32, P, P]
        L.omg_coarse_solve.argtypes = [P, P, P]
        L.omg_get_dirs.argtypes = [P, i32, P, P]
        L.omg_get_visits.argtypes = [P, P, i32, P]
        L.omg_get_trace.argtypes = [P, P, i32, P]
        L.omg_get_step_counts.argtypes = [P, P, i32, P]
        L.omg_set_replay.argtypes = [P, P, i32]
        L.omg_bench_kernel.argtypes = [P, i32, i32, i32, P, P]
        L.omg_get_kernel_counts.argtypes = [P, P]
        L.omg_probe_kernel.argtypes = [P, i32, i32, i32]
        L.omg_probe_result.argtypes = [P, P, P, P]
        L.omg_level_multi.argtypes = [P, i32, i32, i32, i32, i32, P, P, P]
        L.omg_level_tuning.argtypes = [P, i32, P]
        L.omg_level_rm_step.argtypes = [P, i32, i32, P, P, P, P, P, P, P, P]
        L.omg_level_rm_configs.argtypes = [P, i32, P, i32, P]
        L.omg_level_set_rm_config.argtypes = [P, i32, P]
        L.omg_rm_step_noalloc.argtypes = [ctypes.c_int64, i32, P, P, P, P, d, P, P, P, P]
        for name in EXPORTS:
            if name not in ("omg_default_options", "omg_destroy", "omg_strerror"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st, what):
    if st != OK:
        raise OmgError(st, what)


def options(**kw) -> Options:
    """omg_options with defaults; keyword names as in the struct. ``variant``
    accepts 'sync'/'overlap'/'hybrid'/'add_sync', ``smoother`` 'bj'/'schwarz', ``precision``
    'fp64'/'mixed_ir'/'mixed_flex', and
    ``crit`` a list of (rel, max) pairs for levels 1, 2, ..."""
    o = Options()
    lib().omg_default_options(ctypes.byref(o))
    names = {"sync": SYNC_MULT, "overlap": OVERLAP_DET, "hybrid": HYBRID, "add_sync": ADD_SYNC,
             "bj": SMOOTH_BJ, "schwarz": SMOOTH_AS, "fp64": FP64, "mixed_ir": MIXED_IR,
             "mixed_flex": MIXED_FLEX}
    crit = kw.pop("crit", None)
    for k, v in kw.items():
        if isinstance(v, str):
            v = names[v]
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    if crit is not None:
        for l in range(MAX_LEVELS):
            rel, mx = crit[l] if l < len(crit) else (-1.0, 1)
            o.crit_rel[l] = rel
            o.crit_max[l] = mx
    return o


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """Owns one library solver (hierarchy, factors, workspaces) on cuda:0."""

    def __init__(self, handle, bs: int, n_cells: int, has_sip: bool, grid: Grid = None):
        self._h = handle
        self.grid = grid
        self.bs = bs
        self.n_cells = n_cells
        self.n = self.n_cells * self.bs
        self.has_sip = has_sip
        self.last_report = None

    @staticmethod
    def make_grid(nx, ny, nz, p, n_levels, h=None, penalty_c=4.0) -> Grid:
        return Grid(nx, ny, nz, p, n_levels, 0, 1.0 / nx if h is None else h, penalty_c)

    @classmethod
    def from_bsr(cls, row_ptr, col_idx, val, hierarchy, **opts):
        """omg_setup on a host BSR matrix. ``hierarchy`` is a Hierarchy, or a
        Grid whose 2x2x2 agglomeration is taken."""
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        H = Hierarchy.of_grid(hierarchy) if isinstance(hierarchy, Grid) else hierarchy
        bs = val.shape[1]
        A = Bsr(len(row_ptr) - 1, bs, len(col_idx), row_ptr.ctypes.data, col_idx.ctypes.data, val.ctypes.data)
        h = ctypes.c_void_p()
        o = options(**opts)
        _check(lib().omg_setup(ctypes.byref(A), ctypes.byref(H.c), ctypes.byref(o), _stream(), ctypes.byref(h)),
               "omg_setup")
        return cls(h, bs, len(row_ptr) - 1, False, hierarchy if isinstance(hierarchy, Grid) else None)

    @classmethod
    def from_sip(cls, grid: Grid, nu, hierarchy: Hierarchy = None, **opts):
        import torch
        nu = torch.as_tensor(nu, dtype=torch.float64, device="cuda").contiguous()
        h = ctypes.c_void_p()
        o = options(**opts)
        _check(lib().omg_setup_sip(ctypes.byref(grid), _ptr(nu), None if hierarchy is None else ctypes.byref(hierarchy.c),
                                   ctypes.byref(o), _stream(), ctypes.byref(h)), "omg_setup_sip")
        bs = (grid.p + 1) * (grid.p + 2) * (grid.p + 3) // 6
        return cls(h, bs, grid.nx * grid.ny * grid.nz, True, grid)

    def close(self):
        if self._h:
            lib().omg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, x=None, tol=1e-10, check=True, r_out=None):
        import torch
        b = torch.as_tensor(b, dtype=torch.float64, device="cuda").contiguous()
        x = torch.zeros_like(b) if x is None else torch.as_tensor(x, dtype=torch.float64, device="cuda").clone()
        rep = Report()
        st = lib().omg_solve(self._h, _ptr(b), _ptr(x), tol, None if r_out is None else _ptr(r_out),
                             ctypes.byref(rep))
        self.last_report = rep.as_dict()
        if check and st != OK:
            raise OmgError(st, "omg_solve")
        return x

    def backward(self, u, g_u, tol=1e-10, want_nu=True):
        import torch
        u = torch.as_tensor(u, dtype=torch.float64, device="cuda").contiguous()
        g_u = torch.as_tensor(g_u, dtype=torch.float64, device="cuda").contiguous()
        g_f = torch.empty_like(u)
        g_nu = torch.empty(self.n_cells, dtype=torch.float64, device="cuda") if want_nu else None
        rep = Report()
        st = lib().omg_solve_backward(self._h, _ptr(u), _ptr(g_u), _ptr(g_f), None if g_nu is None else _ptr(g_nu),
                                      tol, ctypes.byref(rep))
        self.last_report = rep.as_dict()
        if st != OK:  # gradients exist only for a converged adjoint solve
            raise OmgError(st, "omg_solve_backward")
        return g_f, g_nu

    # ---- inspection -------------------------------------------------------
    def level_info(self, l):
        n, w, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().omg_level_info(self._h, l, ctypes.byref(n), ctypes.byref(w), ctypes.byref(k)), "level_info")
        return n.value, w.value, k.value

    def level_matrix(self, l):
        n, w, _ = self.level_info(l)
        rp = np.zeros(n + 1, dtype=np.int32)
        ci = np.zeros(n * w, dtype=np.int32)
        v = np.zeros((n * w, self.bs, self.bs))
        nnzb = ctypes.c_int64()
        _check(lib().omg_level_matrix(self._h, l, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, ctypes.byref(nnzb)),
               "level_matrix")
        return rp, ci[:nnzb.value], v[:nnzb.value]

    def level_spmv(self, l, x, b=None, fp32=False):
        import torch
        y = torch.empty_like(x)
        _check(lib().omg_level_spmv(self._h, l, int(fp32), _ptr(x), None if b is None else _ptr(b), _ptr(y)),
               "level_spmv")
        return y

    def level_smoother(self, l, r, sweeps, fp32=False):
        import torch
        out = torch.empty_like(r)
        _check(lib().omg_level_smoother(self._h, l, int(fp32), _ptr(r), sweeps, _ptr(out)), "level_smoother")
        return out

    def level_restrict(self, l, r, fp32=False):
        import torch
        nc, _, _ = self.level_info(l + 1)
        rc = torch.empty(nc * self.bs, dtype=torch.float64, device="cuda")
        _check(lib().omg_level_restrict(self._h, l, int(fp32), _ptr(r), _ptr(rc)), "level_restrict")
        return rc

    def level_prolong(self, l, zc, fp32=False):
        import torch
        nf, _, _ = self.level_info(l)
        z = torch.empty(nf * self.bs, dtype=torch.float64, device="cuda")
        _check(lib().omg_level_prolong(self._h, l, int(fp32), _ptr(zc), _ptr(z)), "level_prolong")
        return z

    def coarse_solve(self, b):
        import torch
        x = torch.empty_like(b)
        _check(lib().omg_coarse_solve(self._h, _ptr(b), _ptr(x)), "coarse_solve")
        return x

    def level_multi(self, l, op, X, B=None, sweeps=1, fp32=False):
        """Multi-right-hand-side level operation (as inside batched solves):
        X, B are (N_l, nrhs) CUDA tensors, RHS index fastest."""
        import torch
        X = X.contiguous()
        Y = torch.empty_like(X)
        nrhs = X.shape[1]
        _check(lib().omg_level_multi(self._h, l, op, nrhs, sweeps, int(fp32), _ptr(X),
                                     None if B is None else _ptr(B.contiguous()), _ptr(Y)), "level_multi")
        return Y

    def level_tuning(self, l):
        """Autotuned launch configurations of level l: (multi-RHS shapes
        [op][fp32][two tiles], (RM blocks, entries per thread, MGS block, leader exchange,
        compute waves of the exchange-wave form or 0, exchanges in flight of the lagged form or 0))."""
        out = np.zeros(19, dtype=np.int32)
        _check(lib().omg_level_tuning(self._h, l, out.ctypes.data), "level_tuning")
        return out[:12].reshape(3, 2, 2), tuple(int(v) for v in out[12:18])

    def rm_dropped(self, l):
        """RM launch configurations the tuner dropped on level l because a
        bounded wait expired (their grid was not resident at once)."""
        out = np.zeros(19, dtype=np.int32)
        _check(lib().omg_level_tuning(self._h, l, out.ctypes.data), "level_tuning")
        return int(out[18])

    def rm_configs(self, l=0):
        """Co-resident launch configurations of level l's persistent RM kernel."""
        n = ctypes.c_int32()
        _check(lib().omg_level_rm_configs(self._h, l, None, 0, ctypes.byref(n)), "rm_configs")
        out = np.zeros(6 * max(n.value, 1), dtype=np.int32)
        _check(lib().omg_level_rm_configs(self._h, l, out.ctypes.data, n.value, ctypes.byref(n)), "rm_configs")
        return [tuple(int(v) for v in out[6 * i:6 * i + 6]) for i in range(n.value)]

    def set_rm_config(self, l, cfg):
        """Use this co-resident RM configuration (a tuple from rm_configs) on level l."""
        c = np.ascontiguousarray(np.asarray(cfg, dtype=np.int32))
        _check(lib().omg_level_set_rm_config(self._h, l, c.ctypes.data), "set_rm_config")

    def rm_step(self, l, W, w, z, r, cfg=None):
        """One RM step on flat vectors (see omg_level_rm_step): returns
        (Wk, r_new, betas, gamma, alpha)."""
        import torch
        k = 0 if W is None else W.shape[0]
        Wk = torch.empty_like(w)
        rn = torch.empty_like(w)
        coeff = np.zeros(k + 2)
        c = None if cfg is None else np.ascontiguousarray(np.asarray(cfg, dtype=np.int32))
        _check(lib().omg_level_rm_step(self._h, l, k, None if W is None else _ptr(W.contiguous()), _ptr(w), _ptr(z),
                                       _ptr(r), None if c is None else c.ctypes.data, _ptr(Wk), _ptr(rn),
                                       coeff.ctypes.data), "rm_step")
        return Wk, rn, coeff[:k], coeff[k], coeff[k + 1]

    def dirs(self, l=0):
        import torch
        n, _, k = self.level_info(l)
        W = torch.empty((k, n * self.bs), dtype=torch.float64, device="cuda")
        Z = torch.empty_like(W)
        _check(lib().omg_get_dirs(self._h, l, _ptr(W), _ptr(Z)), "get_dirs")
        return W, Z

    def visits(self):
        n = ctypes.c_int32()
        lib().omg_get_visits(self._h, None, 0, ctypes.byref(n))
        out = np.zeros(2 * max(n.value, 1), dtype=np.int32)
        lib().omg_get_visits(self._h, out.ctypes.data, n.value, ctypes.byref(n))
        return out[: 2 * n.value].reshape(-1, 2)

    def visit_norms(self):
        """Per-visit residual log of the last solve: (level, iterations, ||r0||,
        array of ||r|| after each iteration) in completion order."""
        n = ctypes.c_int32()
        lib().omg_get_visit_norms(self._h, None, 0, ctypes.byref(n))
        out = np.zeros(max(n.value, 1))
        lib().omg_get_visit_norms(self._h, out.ctypes.data, n.value, ctypes.byref(n))
        res, i = [], 0
        while i < n.value:
            l, it = int(out[i]), int(out[i + 1])
            res.append((l, it, float(out[i + 2]), out[i + 3:i + 3 + it].copy()))
            i += 3 + it
        return res

    def step_counts(self):
        """Smoother+RM steps per cycle of the forking level in the last solve."""
        n = ctypes.c_int32()
        lib().omg_get_step_counts(self._h, None, 0, ctypes.byref(n))
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        lib().omg_get_step_counts(self._h, out.ctypes.data, n.value, ctypes.byref(n))
        return out[: n.value]

    def trace(self):
        n = ctypes.c_int32()
        lib().omg_get_trace(self._h, None, 0, ctypes.byref(n))
        out = np.zeros(3 * max(n.value, 1))
        lib().omg_get_trace(self._h, out.ctypes.data, n.value, ctypes.byref(n))
        return out[: 3 * n.value].reshape(-1, 3)

    def bench_kernel(self, kind, level, reps=20):
        """(average ms per launch, algorithmic bytes per launch) of one kernel,
        timed with HIP events on the solver's stream."""
        ms, by = ctypes.c_double(), ctypes.c_double()
        _check(lib().omg_bench_kernel(self._h, kind, level, reps, ctypes.byref(ms), ctypes.byref(by)),
               "bench_kernel")
        return ms.value, by.value

    def probe(self, kind, level, max_launches=100000):
        _check(lib().omg_probe_kernel(self._h, kind, level, max_launches), "probe_kernel")

    def probe_result(self):
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(lib().omg_probe_result(self._h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)), "probe_result")
        return n.value, ms.value, by.value

    def kernel_counts(self):
        out = np.zeros((12, MAX_LEVELS), dtype=np.int64)
        _check(lib().omg_get_kernel_counts(self._h, out.ctypes.data), "kernel_counts")
        return out

    def set_replay(self, visits):
        v = np.ascontiguousarray(np.asarray(visits, dtype=np.int32).reshape(-1))
        _check(lib().omg_set_replay(self._h, v.ctypes.data if len(v) else None, len(v) // 2), "set_replay")


def rm_step_noalloc(W, w, z, r, breakdown=1e-14, r_new=None):
    """omg_rm_step_noalloc: one RM step on caller arrays with the library's
    fixed scratch (no device allocation by the library). W: (k, N) CUDA
    tensor or None; returns (Wk, r_new, betas, gamma, alpha)."""
    import torch
    k = 0 if W is None else W.shape[0]
    N = w.shape[0]
    Wk = torch.empty_like(w)
    rn = torch.empty_like(w) if r_new is None else r_new
    coeff = np.zeros(k + 2)
    _check(lib().omg_rm_step_noalloc(N, k, None if W is None else _ptr(W), _ptr(w), _ptr(z), _ptr(r), breakdown,
                                     _stream(), _ptr(Wk), _ptr(rn), coeff.ctypes.data), "rm_step_noalloc")
    return Wk, rn, coeff[:k], coeff[k], coeff[k + 1]


def solve_batched(solvers, bs_list, xs_list=None, tol=1e-10, nrhs=1):
    """Batched solve: ``bs_list[i]`` is an (N_i, nrhs) CUDA tensor (RHS index
    fastest) for solver i. Returns the solutions and the per-column reports."""
    import torch
    n = len(solvers)
    bs_list = [torch.as_tensor(b, dtype=torch.float64, device="cuda").contiguous() for b in bs_list]
    xs = [torch.zeros_like(b) for b in bs_list] if xs_list is None else [x.clone() for x in xs_list]
    harr = (ctypes.c_void_p * n)(*[s._h.value for s in solvers])
    barr = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs_list])
    xarr = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    reps = (Report * (n * nrhs))()
    st = lib().omg_solve_batched(harr, n, nrhs, barr, xarr, tol, reps)
    if st not in (OK,):
        raise OmgError(st, "omg_solve_batched")
    return xs, [r.as_dict() for r in reps]


def _autograd():
    import torch

    class SolveFn(torch.autograd.Function):
        """u = A(exp(log_nu))^-1 f on the SIP operator. Forward: omg_setup_sip +
        omg_solve; backward: omg_solve_backward (adjoint solve + per-cell
        contraction). Only (f, log_nu) are saved; the hierarchy is rebuilt in
        backward (checkpointed forward state)."""

        @staticmethod
        def forward(ctx, f, log_nu, grid, tol, opts):
            nu = torch.exp(log_nu.detach()).to(torch.float64).contiguous()
            s = Solver.from_sip(grid, nu, **(opts or {}))
            u = s.solve(f.detach(), tol=tol)
            s.close()
            ctx.save_for_backward(f, log_nu, u)
            ctx.grid, ctx.tol, ctx.opts = grid, tol, opts
            return u

        @staticmethod
        def backward(ctx, g_u):
            f, log_nu, u = ctx.saved_tensors
            nu = torch.exp(log_nu.detach()).to(torch.float64).contiguous()
            s = Solver.from_sip(ctx.grid, nu, **(ctx.opts or {}))
            g_f, g_nu = s.backward(u, g_u.contiguous(), tol=ctx.tol)
            s.close()
            return g_f, g_nu * nu, None, None, None

    return SolveFn


def solve_fn():
    """The torch.autograd.Function wrapping the differentiable solve."""
    return _autograd()
