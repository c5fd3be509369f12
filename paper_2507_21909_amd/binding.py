"""ctypes binding of libtrg.so (argument marshalling only).

The names follow the C ABI of include/trg.h: ``Solver.tensor_init``,
``Solver.atrg_step``, ``Solver.triad_atrg_step``, ``Solver.log_z_per_site``.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrg.so")

FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
SVD_SKETCH, SVD_EXACT = 0, 1
TAN_BETA, TAN_H = 1, 2
MODEL_ISING = 0
T_PHI, T_PSI, T_SIGMA, T_RESPLIT = 0, 1, 2, 3
METHOD_ATRG, METHOD_TRIAD = 0, 1


class Options(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("r", ctypes.c_int),
        ("sketch_mult", ctypes.c_int),
        ("power_iters", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("instance", ctypes.c_uint32),
        ("precision", ctypes.c_int),
        ("bond_svd", ctypes.c_int),
        ("max_sweeps", ctypes.c_int),
        ("workspace_cap", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("device", ctypes.c_int),
        ("tau_deg", ctypes.c_double),
        ("tangents", ctypes.c_int),
        ("r_bond", ctypes.c_int),
    ]


class TrgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("trg error %d: %s" % (code, msg))
        self.code = code


_LIB = None
_DP = ctypes.POINTER(ctypes.c_double)


def load_library(path=None):
    """Load libtrg.so (raises FileNotFoundError if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise FileNotFoundError("libtrg.so not built: run paper_2507_21909_amd/build.py (%s)" % path)
    # torch ships its own HIP runtime under the same soname: loaded first, it
    # is the one libtrg.so binds to, so the process holds a single runtime and
    # torch's device pointers are valid in the library (loaded the other way
    # round, two runtimes would each claim the GPU and torch's fails to start)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    st = ctypes.c_void_p
    lib.trg_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.trg_default_options.restype = None
    lib.trg_create.argtypes = [ctypes.POINTER(Options), ctypes.POINTER(st)]
    lib.trg_destroy.argtypes = [st]
    lib.tensor_init.argtypes = [st, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.atrg_step.argtypes = [st, ctypes.c_int]
    lib.triad_atrg_step.argtypes = [st, ctypes.c_int]
    lib.log_z_per_site.argtypes = [st, _DP]
    lib.gu_wen_x.argtypes = [st, ctypes.c_int, _DP]
    lib.impurity_derivatives.argtypes = [st, _DP, _DP]
    lib.trg_shape.argtypes = [st, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_int)]
    lib.trg_export.argtypes = [st, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t]
    lib.trg_export_size.argtypes = [st, ctypes.c_int]
    lib.trg_export_size.restype = ctypes.c_size_t
    lib.trg_set_timing.argtypes = [st, ctypes.c_int]
    lib.trg_kernel_time.argtypes = [st, _DP, _DP, ctypes.POINTER(ctypes.c_int)]
    lib.trg_strerror.argtypes = [ctypes.c_int]
    lib.trg_strerror.restype = ctypes.c_char_p
    lib.trg_last_error.argtypes = [st]
    lib.trg_last_error.restype = ctypes.c_char_p
    lib.trg_selftest_gemm.argtypes = [ctypes.c_int] * 7 + [_DP, _DP, _DP]
    lib.trg_selftest_tsqr.argtypes = [ctypes.c_int, ctypes.c_int, _DP, _DP, _DP]
    _IP = ctypes.POINTER(ctypes.c_int)
    lib.trg_selftest_permute.argtypes = [ctypes.c_int, _IP, _IP, _DP, _DP]
    lib.trg_selftest_svd.argtypes = [ctypes.c_int, ctypes.c_int, _DP, _DP, _DP, _DP, ctypes.POINTER(ctypes.c_int)]
    lib.trg_selftest_eigh.argtypes = [ctypes.c_int, ctypes.c_int, _DP, _DP, _DP, ctypes.POINTER(ctypes.c_int)]
    lib.trg_selftest_pchol.argtypes = [ctypes.c_int, ctypes.c_int, _DP, ctypes.c_double, _DP,
                                       ctypes.POINTER(ctypes.c_int)]
    lib.trg_selftest_gram_eig.argtypes = [ctypes.c_int, ctypes.c_int, _DP, _DP, _DP, ctypes.POINTER(ctypes.c_int)]
    lib.trg_selftest_sketch.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32] + [ctypes.c_int] * 5 + [_DP]
    lib.trg_batch_create.argtypes = [ctypes.c_int, _DP, _DP, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_void_p)]
    lib.trg_batch_run.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.trg_batch_run_graphs.argtypes = lib.trg_batch_run.argtypes
    lib.trg_batch_run_graphs.restype = ctypes.c_int
    lib.trg_batch_log_z.argtypes = [ctypes.c_void_p, _DP]
    lib.trg_batch_size.argtypes = [ctypes.c_void_p]
    lib.trg_batch_last_error.argtypes = [ctypes.c_void_p]
    lib.trg_batch_last_error.restype = ctypes.c_char_p
    lib.trg_batch_destroy.argtypes = [ctypes.c_void_p]
    lib.trg_qr.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_void_p]
    lib.trg_qr.restype = ctypes.c_int
    lib.trg_qr_noalloc.argtypes = lib.trg_qr.argtypes
    lib.trg_qr_noalloc.restype = ctypes.c_int
    lib.trg_release_workspace.argtypes = [st]
    lib.trg_release_workspace.restype = ctypes.c_int
    lib.trg_graph_capture.argtypes = [st, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    lib.trg_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.trg_graph_destroy.argtypes = [ctypes.c_void_p]
    for f in ("trg_graph_capture", "trg_graph_launch", "trg_graph_destroy"):
        getattr(lib, f).restype = ctypes.c_int
    for f in ("trg_batch_create", "trg_batch_run", "trg_batch_log_z", "trg_batch_size", "trg_batch_destroy"):
        getattr(lib, f).restype = ctypes.c_int
    for f in ("trg_create", "trg_destroy", "tensor_init", "atrg_step", "triad_atrg_step", "log_z_per_site", "gu_wen_x",
              "impurity_derivatives",
              "trg_shape", "trg_export", "trg_set_timing", "trg_kernel_time", "trg_selftest_gemm",
              "trg_selftest_tsqr", "trg_selftest_svd", "trg_selftest_eigh", "trg_selftest_pchol",
              "trg_selftest_gram_eig", "trg_selftest_sketch", "trg_selftest_permute"):
        getattr(lib, f).restype = ctypes.c_int
    _LIB = lib
    return lib


def _p(a):
    return a.ctypes.data_as(_DP)


def _check(rc, state=None):
    if rc != 0:
        lib = load_library()
        msg = lib.trg_last_error(state).decode() if state is not None else lib.trg_last_error(None).decode()
        raise TrgError(rc, "%s (%s)" % (lib.trg_strerror(rc).decode(), msg))


class Solver:
    """One ATRG / triad-ATRG solve on one GPU (a trg_state)."""

    def __init__(self, dim=4, r=7, sketch_mult=2, power_iters=1, seed=0, instance=0, precision=FP64,
                 bond_svd=SVD_SKETCH, max_sweeps=0, workspace_cap=0, stream=None, device=0, tau_deg=0.0,
                 r_bond=1, tangents=0):
        lib = load_library()
        o = Options()
        lib.trg_default_options(ctypes.byref(o))
        o.dim, o.r, o.sketch_mult, o.power_iters = dim, r, sketch_mult, power_iters
        o.seed, o.instance, o.precision, o.bond_svd = seed, instance, precision, bond_svd
        o.max_sweeps, o.workspace_cap, o.device = max_sweeps, workspace_cap, device
        o.stream = stream
        o.tau_deg = tau_deg
        o.r_bond = r_bond
        o.tangents = tangents
        self._lib = lib
        self._s = ctypes.c_void_p()
        _check(lib.trg_create(ctypes.byref(o), ctypes.byref(self._s)))
        self.dim = dim

    def close(self):
        if self._s:
            self._lib.trg_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tensor_init(self, model, beta, h, D):
        _check(self._lib.tensor_init(self._s, model, beta, h, D), self._s)

    def atrg_step(self, axis):
        _check(self._lib.atrg_step(self._s, axis), self._s)

    def triad_atrg_step(self, axis):
        _check(self._lib.triad_atrg_step(self._s, axis), self._s)

    def log_z_per_site(self):
        out = ctypes.c_double()
        _check(self._lib.log_z_per_site(self._s, ctypes.byref(out)), self._s)
        return out.value

    def impurity_derivatives(self):
        """(d(log Z/V)/d(beta), d(log Z/V)/dh) by the impurity-tensor method (Sec. III D); NaN for a
        tangent the solver does not carry.  u = -first, m = second."""
        db, dh = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.impurity_derivatives(self._s, ctypes.byref(db), ctypes.byref(dh)), self._s)
        return db.value, dh.value

    def gu_wen_x(self, axis=3):
        """X = (Tr A)^2 / Tr(A A) of the current coarse tensor, A open along ``axis`` (Sec. III D)."""
        out = ctypes.c_double()
        _check(self._lib.gu_wen_x(self._s, axis, ctypes.byref(out)), self._s)
        return out.value

    def shape(self):
        dims = (ctypes.c_int * self.dim)()
        chi, steps = ctypes.c_int(), ctypes.c_int()
        _check(self._lib.trg_shape(self._s, dims, ctypes.byref(chi), ctypes.byref(steps)), self._s)
        return tuple(dims), chi.value, steps.value

    def export(self, which):
        n = self._lib.trg_export_size(self._s, which)
        out = np.empty(n // 8, dtype=np.float64)
        _check(self._lib.trg_export(self._s, which, out.ctypes.data_as(ctypes.c_void_p), n), self._s)
        if which in (T_PHI, T_PSI):
            dims, chi, _ = self.shape()
            out = out.reshape(tuple(dims) + (chi,))
        return out

    def set_timing(self, on=True):
        _check(self._lib.trg_set_timing(self._s, 1 if on else 0), self._s)

    def release_workspace(self):
        """Free the step workspace (trg_release_workspace); recorded graphs of this state retire."""
        _check(self._lib.trg_release_workspace(self._s), self._s)

    def capture(self, axis, method=METHOD_TRIAD):
        """Record one step along ``axis`` at the current shapes as a HIP graph (trg_graph_capture)."""
        g = ctypes.c_void_p()
        _check(self._lib.trg_graph_capture(self._s, method, axis, ctypes.byref(g)), self._s)
        return Graph(self, g)

    def kernel_time(self):
        ms, fl, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(self._lib.trg_kernel_time(self._s, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(n)), self._s)
        return ms.value, fl.value, n.value


class Graph:
    """A recorded RG step (trg_graph); ``launch()`` replays it on the solver's stream."""

    def __init__(self, solver, handle):
        self._solver = solver   # destroyed before the solver: keep it alive
        self._g = handle

    def launch(self, check=False):
        """Replay the step (trg_graph_launch); check=True waits, and rolls a failed step back."""
        _check(self._solver._lib.trg_graph_launch(self._g, 1 if check else 0), self._solver._s)

    def close(self):
        if self._g:
            self._solver._lib.trg_graph_destroy(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many (beta, h, D) triad-ATRG solves driven together (trg_batch)."""

    def __init__(self, betas, hs, Ds, r=7, sketch_mult=2, power_iters=1, seed=0, instance=0, precision=FP64,
                 max_sweeps=0, device=0, tau_deg=0.0):
        lib = load_library()
        n = len(betas)
        if len(hs) != n or len(Ds) != n:
            raise ValueError("betas, hs and Ds must have the same length")
        o = Options()
        lib.trg_default_options(ctypes.byref(o))
        o.r, o.sketch_mult, o.power_iters = r, sketch_mult, power_iters
        o.seed, o.instance, o.precision, o.max_sweeps, o.device = seed, instance, precision, max_sweeps, device
        o.tau_deg = tau_deg
        b = np.ascontiguousarray(betas, dtype=np.float64)
        h = np.ascontiguousarray(hs, dtype=np.float64)
        d = (ctypes.c_int * n)(*[int(x) for x in Ds])
        self._lib = lib
        self._b = ctypes.c_void_p()
        self.n = n
        rc = lib.trg_batch_create(n, _p(b), _p(h), d, ctypes.byref(o), ctypes.byref(self._b))
        if rc != 0:
            raise TrgError(rc, "%s (%s)" % (lib.trg_strerror(rc).decode(), lib.trg_last_error(None).decode()))

    def _check(self, rc):
        if rc != 0:
            raise TrgError(rc, "%s (%s)" % (self._lib.trg_strerror(rc).decode(),
                                            self._lib.trg_batch_last_error(self._b).decode()))

    def run(self, nsteps, axes=None, graphs=False):
        """nsteps steps of every instance (trg_batch_run, or trg_batch_run_graphs with graphs=True)."""
        ax = None if axes is None else (ctypes.c_int * len(axes))(*axes)
        if axes is not None and len(axes) != nsteps:
            raise ValueError("axes must list one axis per step")
        f = self._lib.trg_batch_run_graphs if graphs else self._lib.trg_batch_run
        self._check(f(self._b, nsteps, ax))

    def log_z_per_site(self):
        out = np.empty(self.n)
        self._check(self._lib.trg_batch_log_z(self._b, _p(out)))
        return out

    def close(self):
        if self._b:
            self._lib.trg_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def selftest_gemm(a, b, ta=False, tb=False, precision=FP64):
    """C[b] = op(A[b]) op(B[b]) on the GPU; a: (batch, M, K) or (batch, K, M) if ta."""
    lib = load_library()
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    batch = a.shape[0]
    m, k = (a.shape[2], a.shape[1]) if ta else (a.shape[1], a.shape[2])
    n = b.shape[1] if tb else b.shape[2]
    c = np.empty((batch, m, n))
    _check(lib.trg_selftest_gemm(precision, int(ta), int(tb), m, n, k, batch, _p(a), _p(b), _p(c)))
    return c


def selftest_permute(a, perm):
    """np.transpose(a, perm) computed by the library's permute."""
    lib = load_library()
    a = np.ascontiguousarray(a, dtype=np.float64)
    nd = a.ndim
    dims = (ctypes.c_int * nd)(*a.shape)
    pm = (ctypes.c_int * nd)(*perm)
    out = np.empty(a.size)
    _check(lib.trg_selftest_permute(nd, dims, pm, _p(a), _p(out)))
    return out.reshape(tuple(a.shape[p] for p in perm))


def selftest_tsqr(a):
    lib = load_library()
    a = np.ascontiguousarray(a, dtype=np.float64)
    m, n = a.shape
    q = np.empty((m, n))
    r = np.empty((n, n))
    _check(lib.trg_selftest_tsqr(m, n, _p(a), _p(q), _p(r)))
    return q, r


def selftest_svd(a):
    lib = load_library()
    a = np.ascontiguousarray(a, dtype=np.float64)
    m, n = a.shape
    u, s, v = np.empty((m, n)), np.empty(n), np.empty((n, n))
    sw = ctypes.c_int()
    _check(lib.trg_selftest_svd(m, n, _p(a), _p(u), _p(s), _p(v), ctypes.byref(sw)))
    return u, s, v, sw.value


def selftest_eigh(k):
    """Eigen-decomposition of symmetric matrices k (n x n or count x n x n)."""
    lib = load_library()
    k = np.ascontiguousarray(k, dtype=np.float64)
    single = k.ndim == 2
    kb = k[None] if single else k
    count, n = kb.shape[0], kb.shape[1]
    if kb.shape[2] != n:
        raise ValueError("square matrices required")
    lam = np.empty((count, n))
    v = np.empty((count, n, n))
    sw = ctypes.c_int(0)
    _check(lib.trg_selftest_eigh(count, n, _p(kb), _p(lam), _p(v), ctypes.byref(sw)))
    return (lam[0], v[0], sw.value) if single else (lam, v, sw.value)


def _square_batch(k):
    k = np.ascontiguousarray(k, dtype=np.float64)
    single = k.ndim == 2
    kb = k[None] if single else k
    if kb.ndim != 3 or kb.shape[2] != kb.shape[1]:
        raise ValueError("square matrices required")
    return kb, single


def selftest_pchol(k, tol=0.0):
    """Pivoted Cholesky factors X (K = X X^T, X = P L) and ranks of PSD matrices k."""
    lib = load_library()
    kb, single = _square_batch(k)
    count, n = kb.shape[0], kb.shape[1]
    x = np.empty((count, n, n))
    rank = (ctypes.c_int * count)()
    _check(lib.trg_selftest_pchol(count, n, _p(kb), float(tol), _p(x), rank))
    rk = list(rank)
    return (x[0], rk[0]) if single else (x, rk)


def selftest_gram_eig(k):
    """Eigen-decomposition of PSD Grams k through their pivoted Cholesky factors."""
    lib = load_library()
    kb, single = _square_batch(k)
    count, n = kb.shape[0], kb.shape[1]
    lam = np.empty((count, n))
    v = np.empty((count, n, n))
    sw = ctypes.c_int(0)
    _check(lib.trg_selftest_gram_eig(count, n, _p(kb), _p(lam), _p(v), ctypes.byref(sw)))
    return (lam[0], v[0], sw.value) if single else (lam, v, sw.value)


def selftest_sketch(seed, step, instance, chi, jdims, m):
    lib = load_library()
    jd = list(jdims) + [1] * (3 - len(jdims))
    out = np.empty((chi, jd[0], jd[1], jd[2], m))
    _check(lib.trg_selftest_sketch(seed, step, instance, chi, jd[0], jd[1], jd[2], m, _p(out)))
    return out.reshape([chi] + list(jdims) + [m])


def _device_args(a, n_max=64):
    """Checks a torch float64 CUDA matrix and returns (m, n, stream handle)."""
    import torch
    if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64 and a.dim() == 2
            and a.is_contiguous()):
        raise ValueError("a contiguous float64 CUDA matrix is required")
    m, n = a.shape
    if not (1 <= n <= n_max and m >= n):
        raise ValueError("needs 1 <= n <= %d and m >= n (got %d x %d)" % (n_max, m, n))
    return m, n, torch.cuda.current_stream(a.device).cuda_stream


def qr(a):
    """Thin QR of a float64 CUDA matrix (trg_qr) on torch's current stream: (Q, R) CUDA tensors."""
    import torch
    lib = load_library()
    m, n, st = _device_args(a)
    q = torch.empty((m, n), dtype=torch.float64, device=a.device)
    r = torch.empty((n, n), dtype=torch.float64, device=a.device)
    with torch.cuda.device(a.device):
        _check(lib.trg_qr(a.data_ptr(), m, n, q.data_ptr(), r.data_ptr(), st))
    return q, r


def qr_noalloc(a, q=None, r=None):
    """trg_qr_noalloc: thin QR of a float64 CUDA matrix into caller-provided (or new) Q and R, enqueued
    on torch's current stream without any device allocation by the library (no synchronisation)."""
    import torch
    lib = load_library()
    m, n, st = _device_args(a)
    if q is None:
        q = torch.empty((m, n), dtype=torch.float64, device=a.device)
    if r is None:
        r = torch.empty((n, n), dtype=torch.float64, device=a.device)
    for t, shp in ((q, (m, n)), (r, (n, n))):
        if not (t.is_cuda and t.dtype == torch.float64 and tuple(t.shape) == shp and t.is_contiguous()):
            raise ValueError("Q and R must be contiguous float64 CUDA tensors of shapes %s and %s" % ((m, n), (n, n)))
    with torch.cuda.device(a.device):
        _check(lib.trg_qr_noalloc(a.data_ptr(), m, n, q.data_ptr(), r.data_ptr(), st))
    return q, r
