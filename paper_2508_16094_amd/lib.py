"""ctypes binding of ``include/pdipm.h`` (same names; argument marshalling
only — every step of the interior-point hot path runs in the HIP library).

The shared library must have been built (``python -m
paper_2508_16094_amd.build``); loading fails loudly otherwise.  PyTorch
provides device memory (the workspace tensor) and the stream.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libpdipm.so")

PDIPM_OK, PDIPM_MAX_ITER, PDIPM_TIME_LIMIT, PDIPM_STALLED = 0, 1, 2, 3
PDIPM_ERR_INVALID_ARG, PDIPM_ERR_OUT_OF_MEMORY, PDIPM_ERR_NOT_PD = -1, -2, -3
PDIPM_ERR_NUMERICAL, PDIPM_ERR_DEVICE, PDIPM_ERR_NOT_ANALYZED = -4, -5, -6
PDIPM_FP64, PDIPM_FP32, PDIPM_PRECISION_AUTO = 0, 1, 2
PDIPM_HOST, PDIPM_DEVICE = 0, 1
PDIPM_KKT_PRIMAL, PDIPM_KKT_DUAL, PDIPM_KKT_AUGMENTED, PDIPM_KKT_AUTO = 0, 1, 2, 3
PDIPM_ORDER_LEVELS, PDIPM_ORDER_MULTILEVEL = 0, 1

_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f64 = ctypes.c_double


class pdipm_csr(ctypes.Structure):
    _fields_ = [("nrows", _i64), ("ncols", _i64), ("rowptr", _p), ("colind", _p), ("val", _p)]


class ipm_problem_desc(ctypes.Structure):
    _fields_ = [("n", _i64), ("m", _i64), ("c", _p), ("b", _p), ("A", pdipm_csr), ("W", pdipm_csr),
                ("Q", pdipm_csr), ("q4", _p), ("xl", _p), ("xu", _p)]


class ipm_options(ctypes.Structure):
    _fields_ = [("tol", _f64), ("max_iter", _i32), ("max_wall_time", _f64), ("delta_p", _f64),
                ("delta_d", _f64), ("precision", _i32), ("ir_max", _i32), ("ir_tol", _f64),
                ("nd_leaf", _i32), ("amalg_menu", _i32), ("print_level", _i32),
                ("fp64_fallback", _i32), ("use_graphs", _i32), ("graph_iters", _i32), ("kkt_form", _i32),
                ("ordering", _i32)]


class kkt_symbolic_stats(ctypes.Structure):
    _fields_ = [("n", _i64), ("nnz_K", _i64), ("nnz_L", _i64), ("nnz_L_stored", _i64),
                ("n_super", _i64), ("max_front", _i64), ("n_levels", _i64), ("n_triples", _i64),
                ("flops", _f64), ("update_bytes", _f64), ("kkt_form", _i32), ("precision", _i32)]


class kkt_factor_info(ctypes.Structure):
    _fields_ = [("status", _i32), ("first_bad_col", _i64), ("ms", _f64), ("flops", _f64)]


class kkt_solve_info(ctypes.Structure):
    _fields_ = [("ir_steps", _i32), ("residual", _f64), ("fallback", _i32), ("ms", _f64)]


class ipm_profile(ctypes.Structure):
    _fields_ = [("gemm32_launches", _i64), ("gemm32_ms", _f64), ("gemm32_flops", _f64),
                ("gemm64_launches", _i64), ("gemm64_ms", _f64), ("gemm64_flops", _f64),
                ("factorizations32", _i64), ("factorizations64", _i64), ("factor_ms", _f64),
                ("factor_flops", _f64), ("solves", _i64), ("solve_bytes", _f64), ("gemm32_bytes", _f64),
                ("gemm64_bytes", _f64)]


class ipm_start(ctypes.Structure):
    _fields_ = [("x", _p), ("lam", _p), ("memspace", _i32)]


class ipm_result(ctypes.Structure):
    _fields_ = [("status", _i32), ("iterations", _i32), ("f", _f64), ("P", _f64), ("D", _f64),
                ("C", _f64), ("mu", _f64), ("ms_total", _f64), ("ms_eval", _f64),
                ("ms_assemble", _f64), ("ms_factor", _f64), ("ms_solve", _f64), ("ir_steps", _i32),
                ("fp64_refactors", _i32), ("inertia_corrections", _i32), ("max_ir_residual", _f64)]


class ipm_batch_info(ctypes.Structure):
    _fields_ = [("iterations", _i32), ("solved", _i32), ("graph_launches", _i32), ("fp64_from", _i32),
                ("factor_failures", _i32), ("refine_misses", _i32), ("blocking", _i32), ("pad", _i32),
                ("ms_total", _f64), ("ms_capture", _f64)]


_SIGS = {
    "ipm_default_options": (None, [_p]),
    "ipm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ipm_last_error": (ctypes.c_char_p, [_p]),
    "ipm_create": (ctypes.c_int, [_p, _p, _p]),
    "kkt_create_csr": (ctypes.c_int, [_i64, _p, _p, _p, _p]),
    "kkt_analyze": (ctypes.c_int, [_p, _p]),
    "kkt_get_symbolic": (ctypes.c_int, [_p, _p, _p, _p, _p, _p, _p]),
    "kkt_get_pattern": (ctypes.c_int, [_p, _p, _p]),
    "ipm_workspace_query": (ctypes.c_int, [_p, _p]),
    "ipm_set_workspace": (ctypes.c_int, [_p, _p, ctypes.c_size_t]),
    "ipm_set_stream": (ctypes.c_int, [_p, _p]),
    "kkt_set_values": (ctypes.c_int, [_p, _p]),
    "kkt_assemble": (ctypes.c_int, [_p, _p, _p, _p, _p, ctypes.c_int]),
    "kkt_get_values": (ctypes.c_int, [_p, _p]),
    "kkt_factor": (ctypes.c_int, [_p, ctypes.c_int, _p]),
    "kkt_get_factor": (ctypes.c_int, [_p, _p]),
    "kkt_solve": (ctypes.c_int, [_p, _p, _p, _p]),
    "ipm_evaluate": (ctypes.c_int, [_p, _p, _p, _p, _p, _p, _p, _p]),
    "ipm_pattern_sizes": (ctypes.c_int, [_p, _p, _p]),
    "ipm_get_patterns": (ctypes.c_int, [_p, _p, _p, _p, _p]),
    "ipm_solve": (ctypes.c_int, [_p, _p, _p]),
    "ipm_set_precision": (ctypes.c_int, [_p, ctypes.c_int]),
    "ipm_solve_static": (ctypes.c_int, [_p, _p, _p]),
    "ipm_get_solution": (ctypes.c_int, [_p, _p, _p, _p, _p, _p, ctypes.c_int]),
    "ipm_set_profiling": (ctypes.c_int, [_p, ctypes.c_int]),
    "ipm_get_profile": (ctypes.c_int, [_p, _p]),
    "ipm_destroy": (None, [_p]),
    "ipm_batch_create": (ctypes.c_int, [_i32, _p, _p, _p]),
    "ipm_batch_analyze": (ctypes.c_int, [_p, _p]),
    "ipm_batch_offsets": (ctypes.c_int, [_p, _p, _p]),
    "ipm_batch_workspace_query": (ctypes.c_int, [_p, _p]),
    "ipm_batch_set_workspace": (ctypes.c_int, [_p, _p, ctypes.c_size_t]),
    "ipm_batch_set_stream": (ctypes.c_int, [_p, _p]),
    "ipm_batch_blockings": (ctypes.c_int, [_p, _p, _p, _p]),
    "ipm_batch_set_blocking": (ctypes.c_int, [_p, _i32]),
    "ipm_batch_autotune": (ctypes.c_int, [_p, _i32, _p, _p]),
    "ipm_batch_solve": (ctypes.c_int, [_p, _p, _p, _p]),
    "ipm_batch_get_solution": (ctypes.c_int, [_p, _p, _p, _p, _p, _p, ctypes.c_int]),
    "ipm_batch_set_b": (ctypes.c_int, [_p, _p]),
    "ipm_batch_last_error": (ctypes.c_char_p, [_p]),
    "ipm_batch_destroy": (None, [_p]),
    "mlp_create": (ctypes.c_int, [_i32, _p, _i32, _f64, _f64, _i32, _p]),
    "mlp_num_params": (ctypes.c_int, [_p, _p]),
    "mlp_workspace_query": (ctypes.c_int, [_p, _p]),
    "mlp_set_workspace": (ctypes.c_int, [_p, _p, ctypes.c_size_t]),
    "mlp_set_stream": (ctypes.c_int, [_p, _p]),
    "mlp_set_params": (ctypes.c_int, [_p, _p]),
    "mlp_get_params": (ctypes.c_int, [_p, _p]),
    "mlp_forward": (ctypes.c_int, [_p, _p, _p, _i32]),
    "mlp_gradients": (ctypes.c_int, [_p, _p, _p, _i32, _p, _p]),
    "mlp_train_step": (ctypes.c_int, [_p, _p, _p, _i32, ctypes.c_float, _p]),
    "mlp_flops": (ctypes.c_double, [_p, _i32, _i32]),
    "mlp_last_error": (ctypes.c_char_p, [_p]),
    "mlp_destroy": (None, [_p]),
}

_lib = None


def lib():
    """Load libpdipm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is missing: build it with "
                               "`python -m paper_2508_16094_amd.build` (no CPU fallback exists)")
        # torch ships its own HIP runtime: load it first so that the library
        # binds to the same runtime instead of a second copy that would then
        # hide the devices from torch
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(SO_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


class PdipmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def _ptr(a):
    return ctypes.c_void_p(0) if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def default_options(**kw):
    o = ipm_options()
    lib().ipm_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _csr(mat, nrows, ncols, keep):
    c = pdipm_csr()
    c.nrows, c.ncols = nrows, ncols
    if mat is None:
        return c
    rp = np.ascontiguousarray(mat.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(mat.colind, dtype=np.int32)
    va = np.ascontiguousarray(mat.val, dtype=np.float64)
    keep += [rp, ci, va]
    c.rowptr, c.colind, c.val = _ptr(rp), _ptr(ci), _ptr(va)
    return c


def _desc(problem, keep):
    """ipm_problem_desc viewing the problem's arrays (kept alive in keep)."""
    d = ipm_problem_desc()
    d.n, d.m = problem.n, problem.m

    def vec(a, n):
        if a is None:
            return ctypes.c_void_p(0)
        arr = np.ascontiguousarray(a, np.float64)
        assert arr.shape == (n,)
        keep.append(arr)
        return _ptr(arr)

    d.c = vec(problem.c, problem.n)
    d.b = vec(problem.b if problem.m else None, problem.m)
    d.A = _csr(problem.A, problem.m, problem.n, keep)
    d.W = _csr(problem.W, problem.m, problem.n, keep)
    d.Q = _csr(problem.Q, problem.n, problem.n, keep)
    d.q4 = vec(problem.q4, problem.n)
    d.xl = vec(problem.xl, problem.n)
    d.xu = vec(problem.xu, problem.n)
    return d


class _Handle:
    def __init__(self):
        self.h = ctypes.c_void_p()
        self.ws = None

    def _check(self, rc, what):
        if rc < 0:
            msg = lib().ipm_last_error(self.h).decode()
            raise PdipmError(rc, f"{what}: {msg}")
        return rc

    def __del__(self):
        try:
            if self.h:
                lib().ipm_destroy(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass

    def stats(self):
        s = kkt_symbolic_stats()
        self._check(lib().kkt_analyze(self.h, ctypes.byref(s)), "kkt_analyze")
        return {k: getattr(s, k) for k, _ in s._fields_}

    def symbolic(self):
        s = self.stats()
        n, ns = s["n"], s["n_super"]
        perm = np.empty(n, np.int32); et = np.empty(n, np.int32); cc = np.empty(n, np.int64)
        st = np.empty(ns + 1, np.int32); rp = np.empty(ns + 1, np.int64)
        self._check(lib().kkt_get_symbolic(self.h, _ptr(perm), _ptr(et), _ptr(cc), _ptr(st), _ptr(rp),
                                           ctypes.c_void_p(0)), "kkt_get_symbolic")
        rows = np.empty(int(rp[-1]), np.int32)
        self._check(lib().kkt_get_symbolic(self.h, None, None, None, None, None, _ptr(rows)),
                    "kkt_get_symbolic")
        return dict(perm=perm, etree=et, colcount=cc, sn_start=st, sn_rowptr=rp, sn_rows=rows)

    def k_pattern(self):
        s = self.stats()
        rp = np.empty(s["n"] + 1, np.int64); ci = np.empty(s["nnz_K"], np.int32)
        self._check(lib().kkt_get_pattern(self.h, _ptr(rp), _ptr(ci)), "kkt_get_pattern")
        return rp, ci

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        self._check(lib().ipm_workspace_query(self.h, ctypes.byref(b)), "ipm_workspace_query")
        return b.value

    def bind(self, device="cuda:0", workspace=None, stream=None):
        """Give the handle a torch-owned workspace and the current stream."""
        import torch
        nbytes = self.workspace_bytes()
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = workspace.data_ptr()
        off = (-base) % 256
        self.ws = workspace
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._check(lib().ipm_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)), "ipm_set_stream")
        self._check(lib().ipm_set_workspace(self.h, ctypes.c_void_p(base + off), nbytes),
                    "ipm_set_workspace")
        return self

    def set_profiling(self, enable=True):
        self._check(lib().ipm_set_profiling(self.h, int(enable)), "ipm_set_profiling")

    def profile(self):
        p = ipm_profile()
        self._check(lib().ipm_get_profile(self.h, ctypes.byref(p)), "ipm_get_profile")
        return {k: getattr(p, k) for k, _ in p._fields_}

    def factor(self, precision=PDIPM_FP64):
        info = kkt_factor_info()
        rc = lib().kkt_factor(self.h, precision, ctypes.byref(info))
        if rc == PDIPM_ERR_NOT_PD:
            return dict(status=rc, first_bad_col=info.first_bad_col, ms=info.ms)
        self._check(rc, "kkt_factor")
        return dict(status=rc, first_bad_col=info.first_bad_col, ms=info.ms, flops=info.flops)

    def solve_kkt(self, rhs, out=None):
        import torch
        if out is None:
            out = torch.empty_like(rhs)
        info = kkt_solve_info()
        self._check(lib().kkt_solve(self.h, _dptr(rhs), _dptr(out), ctypes.byref(info)), "kkt_solve")
        return out, dict(ir_steps=info.ir_steps, residual=info.residual, fallback=info.fallback, ms=info.ms)

    def factor_values(self):
        s = self.stats()
        out = np.empty(s["nnz_L_stored"], np.float64)
        self._check(lib().kkt_get_factor(self.h, _ptr(out)), "kkt_get_factor")
        return out


class KktSolver(_Handle):
    """Standalone KKT factor/solve for an explicit SPD matrix (lower CSR)."""

    def __init__(self, n, rowptr, colind, options=None):
        super().__init__()
        self.rowptr = np.ascontiguousarray(rowptr, np.int64)
        self.colind = np.ascontiguousarray(colind, np.int32)
        opts = options if options is not None else default_options()
        rc = lib().kkt_create_csr(n, _ptr(self.rowptr), _ptr(self.colind), ctypes.byref(opts),
                                  ctypes.byref(self.h))
        if rc < 0:
            raise PdipmError(rc, "kkt_create_csr: " + lib().ipm_last_error(None).decode())

    def set_values(self, kval):
        self._check(lib().kkt_set_values(self.h, _dptr(kval)), "kkt_set_values")


class IpmSolver(_Handle):
    """Interior-point solver for a problem object with attributes n, m, c, b,
    A, W, Q, q4, xl, xu (CSR parts rowptr/colind/val)."""

    def __init__(self, problem, options=None, **kw):
        super().__init__()
        keep = []
        d = _desc(problem, keep)
        opts = options if options is not None else default_options(**kw)
        self.options = opts
        self.n, self.m = problem.n, problem.m
        rc = lib().ipm_create(ctypes.byref(d), ctypes.byref(opts), ctypes.byref(self.h))
        if rc < 0:
            raise PdipmError(rc, "ipm_create: " + lib().ipm_last_error(None).decode())

    def patterns(self):
        nj, nh = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().ipm_pattern_sizes(self.h, ctypes.byref(nj), ctypes.byref(nh)), "sizes")
        jrp = np.empty(self.m + 1, np.int64); jci = np.empty(nj.value, np.int32)
        hrp = np.empty(self.n + 1, np.int64); hci = np.empty(nh.value, np.int32)
        self._check(lib().ipm_get_patterns(self.h, _ptr(jrp), _ptr(jci), _ptr(hrp), _ptr(hci)), "patterns")
        return (jrp, jci), (hrp, hci)

    def evaluate(self, x, lam):
        import torch
        (jrp, jci), (hrp, hci) = self.patterns()
        grad = torch.empty(self.n, dtype=torch.float64, device=x.device)
        g = torch.empty(max(self.m, 1), dtype=torch.float64, device=x.device)
        jv = torch.empty(max(len(jci), 1), dtype=torch.float64, device=x.device)
        hv = torch.empty(max(len(hci), 1), dtype=torch.float64, device=x.device)
        f = ctypes.c_double()
        self._check(lib().ipm_evaluate(self.h, _dptr(x), _dptr(lam), ctypes.byref(f), _dptr(grad),
                                       _dptr(g), _dptr(jv), _dptr(hv)), "ipm_evaluate")
        return f.value, grad, g[:self.m], jv[:len(jci)], hv[:len(hci)]

    def assemble(self, x, lam, sig_s, sig_x, precision=PDIPM_FP64):
        self._check(lib().kkt_assemble(self.h, _dptr(x), _dptr(lam), _dptr(sig_s), _dptr(sig_x),
                                       precision), "kkt_assemble")

    def k_values(self):
        out = np.empty(self.stats()["nnz_K"], np.float64)
        self._check(lib().kkt_get_values(self.h, _ptr(out)), "kkt_get_values")
        return out

    def solve_static(self, start=None):
        """ipm_solve_static: solve in the library's static device array (no
        workspace tensor); start as in solve()."""
        res = ipm_result()
        st = self._start(start)
        rc = lib().ipm_solve_static(self.h, ctypes.byref(st) if st is not None else None, ctypes.byref(res))
        self._check(rc, "ipm_solve_static")
        return {k: getattr(res, k) for k, _ in res._fields_}

    def set_precision(self, precision):
        self._check(lib().ipm_set_precision(self.h, int(precision)), "ipm_set_precision")

    def _start(self, start):
        if start is None:
            return None
        xs, ls = start
        st = ipm_start()
        if hasattr(xs, "data_ptr"):
            st.x, st.lam, st.memspace = _dptr(xs), _dptr(ls), PDIPM_DEVICE
        else:
            self._start_keep = (np.ascontiguousarray(xs, np.float64), np.ascontiguousarray(ls, np.float64))
            st.x, st.lam, st.memspace = _ptr(self._start_keep[0]), _ptr(self._start_keep[1]), PDIPM_HOST
        return st

    def solve(self, start=None):
        res = ipm_result()
        st = self._start(start)
        rc = lib().ipm_solve(self.h, ctypes.byref(st) if st is not None else None, ctypes.byref(res))
        self._check(rc, "ipm_solve")
        return {k: getattr(res, k) for k, _ in res._fields_}

    def solution(self):
        x = np.empty(self.n); s = np.empty(self.m); lam = np.empty(self.m)
        zl = np.empty(self.n); zu = np.empty(self.n)
        self._check(lib().ipm_get_solution(self.h, _ptr(x), _ptr(s) if self.m else None,
                                           _ptr(lam) if self.m else None, _ptr(zl), _ptr(zu),
                                           PDIPM_HOST), "ipm_get_solution")
        return dict(x=x, s=s, lam=lam, zl=zl, zu=zu)


class BatchSolver:
    """Batched interior-point solve of many LP/QP problem objects."""

    def __init__(self, problems, options=None, **kw):
        self.h = ctypes.c_void_p()
        self.ws = None
        keep = []
        descs = (ipm_problem_desc * len(problems))()
        for i, p in enumerate(problems):
            descs[i] = _desc(p, keep)
        opts = options if options is not None else default_options(**kw)
        self.options = opts
        self.count = len(problems)
        rc = lib().ipm_batch_create(self.count, descs, ctypes.byref(opts), ctypes.byref(self.h))
        if rc < 0:
            raise PdipmError(rc, "ipm_batch_create: " + lib().ipm_batch_last_error(None).decode())
        self.xoff = np.empty(self.count + 1, np.int64)
        self.roff = np.empty(self.count + 1, np.int64)
        self._check(lib().ipm_batch_offsets(self.h, _ptr(self.xoff), _ptr(self.roff)), "ipm_batch_offsets")

    def _check(self, rc, what):
        if rc < 0:
            raise PdipmError(rc, f"{what}: " + lib().ipm_batch_last_error(self.h).decode())
        return rc

    def __del__(self):
        try:
            if self.h:
                lib().ipm_batch_destroy(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass

    def stats(self):
        s = kkt_symbolic_stats()
        self._check(lib().ipm_batch_analyze(self.h, ctypes.byref(s)), "ipm_batch_analyze")
        return {k: getattr(s, k) for k, _ in s._fields_}

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        self._check(lib().ipm_batch_workspace_query(self.h, ctypes.byref(b)), "ipm_batch_workspace_query")
        return b.value

    def bind(self, device="cuda:0", workspace=None, stream=None):
        import torch
        nbytes = self.workspace_bytes()
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = workspace.data_ptr()
        off = (-base) % 256
        self.ws = workspace
        if stream is None:
            stream = torch.cuda.current_stream(device)
        torch.cuda.synchronize(device)
        self._check(lib().ipm_batch_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)),
                    "ipm_batch_set_stream")
        self._check(lib().ipm_batch_set_workspace(self.h, ctypes.c_void_p(base + off), nbytes),
                    "ipm_batch_set_workspace")
        return self

    def blockings(self):
        c = ctypes.c_int32()
        self._check(lib().ipm_batch_blockings(self.h, ctypes.byref(c), None, None), "ipm_batch_blockings")
        sh = np.empty(c.value, np.int32); ob = np.empty(c.value, np.int32)
        self._check(lib().ipm_batch_blockings(self.h, ctypes.byref(c), _ptr(sh), _ptr(ob)), "ipm_batch_blockings")
        return list(zip(sh.tolist(), ob.tolist()))

    def set_blocking(self, index):
        self._check(lib().ipm_batch_set_blocking(self.h, index), "ipm_batch_set_blocking")

    def autotune(self, reps=2):
        n = len(self.blockings())
        ms = np.empty(n, np.float64)
        chosen = ctypes.c_int32()
        self._check(lib().ipm_batch_autotune(self.h, reps, ctypes.byref(chosen), _ptr(ms)), "ipm_batch_autotune")
        return chosen.value, ms

    def set_b(self, b):
        self._b_keep = np.ascontiguousarray(b, np.float64)
        assert self._b_keep.shape == (int(self.roff[-1]),)
        self._check(lib().ipm_batch_set_b(self.h, _ptr(self._b_keep)), "ipm_batch_set_b")

    def solve(self, start=None):
        res = (ipm_result * self.count)()
        info = ipm_batch_info()
        st = None
        if start is not None:
            xs, ls = start
            st = ipm_start()
            if hasattr(xs, "data_ptr"):
                st.x, st.lam, st.memspace = _dptr(xs), _dptr(ls), PDIPM_DEVICE
            else:
                self._start_keep = (np.ascontiguousarray(xs, np.float64), np.ascontiguousarray(ls, np.float64))
                st.x, st.lam, st.memspace = _ptr(self._start_keep[0]), _ptr(self._start_keep[1]), PDIPM_HOST
        rc = lib().ipm_batch_solve(self.h, ctypes.byref(st) if st is not None else None, res, ctypes.byref(info))
        self._check(rc, "ipm_batch_solve")
        results = [{k: getattr(r, k) for k in ("status", "iterations", "f", "P", "D", "C", "mu")} for r in res]
        return results, {k: getattr(info, k) for k, _ in info._fields_ if k != "pad"}

    def solution(self):
        N, M = int(self.xoff[-1]), int(self.roff[-1])
        x = np.empty(N); s = np.empty(max(M, 1)); lam = np.empty(max(M, 1))
        zl = np.empty(N); zu = np.empty(N)
        self._check(lib().ipm_batch_get_solution(self.h, _ptr(x), _ptr(s) if M else None,
                                                 _ptr(lam) if M else None, _ptr(zl), _ptr(zu), PDIPM_HOST),
                    "ipm_batch_get_solution")
        out = []
        for i in range(self.count):
            a, b = int(self.xoff[i]), int(self.xoff[i + 1])
            r0, r1 = int(self.roff[i]), int(self.roff[i + 1])
            out.append(dict(x=x[a:b], s=s[r0:r1], lam=lam[r0:r1], zl=zl[a:b], zu=zu[a:b]))
        return out


class MlpModel:
    """Warm-start MLP (pdipm_mlp.h): dims[0] -> ... -> dims[-1], the first n_x
    outputs are x in (0, x_scale), the rest lambda > 0."""

    def __init__(self, dims, n_x, x_scale=10.0, max_batch=256, x_weight=1.0):
        self.h = ctypes.c_void_p()
        self.ws = None
        self.dims = [int(d) for d in dims]
        self.n_x = int(n_x)
        d = np.asarray(self.dims, np.int32)
        rc = lib().mlp_create(len(self.dims) - 1, _ptr(d), self.n_x, float(x_scale), float(x_weight),
                              int(max_batch), ctypes.byref(self.h))
        if rc < 0:
            raise PdipmError(rc, "mlp_create: " + lib().mlp_last_error(None).decode())
        c = ctypes.c_int64()
        self._check(lib().mlp_num_params(self.h, ctypes.byref(c)), "mlp_num_params")
        self.num_params = c.value
        self.max_batch = int(max_batch)

    def _check(self, rc, what):
        if rc < 0:
            raise PdipmError(rc, f"{what}: " + lib().mlp_last_error(self.h).decode())
        return rc

    def __del__(self):
        try:
            if self.h:
                lib().mlp_destroy(self.h)
                self.h = ctypes.c_void_p()
        except Exception:
            pass

    def bind(self, device="cuda:0", stream=None):
        import torch
        b = ctypes.c_size_t()
        self._check(lib().mlp_workspace_query(self.h, ctypes.byref(b)), "mlp_workspace_query")
        self.ws = torch.empty(b.value + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._check(lib().mlp_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)), "mlp_set_stream")
        self._check(lib().mlp_set_workspace(self.h, ctypes.c_void_p(base + (-base) % 256), b.value),
                    "mlp_set_workspace")
        return self

    @staticmethod
    def flatten(params):
        return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)

    def unflatten(self, flat):
        out, o = [], 0
        for a, b in zip(self.dims[:-1], self.dims[1:]):
            W = flat[o:o + a * b].reshape(b, a); o += a * b
            bb = flat[o:o + b]; o += b
            out.append((W, bb))
        return out

    def set_params(self, params):
        flat = np.ascontiguousarray(self.flatten(params), np.float32)
        assert flat.size == self.num_params
        self._check(lib().mlp_set_params(self.h, _ptr(flat)), "mlp_set_params")

    def get_params(self):
        flat = np.empty(self.num_params, np.float32)
        self._check(lib().mlp_get_params(self.h, _ptr(flat)), "mlp_get_params")
        return self.unflatten(flat)

    def forward(self, theta, out=None):
        import torch
        B = theta.shape[0]
        if out is None:
            out = torch.empty((B, self.dims[-1]), dtype=torch.float32, device=theta.device)
        self._check(lib().mlp_forward(self.h, _dptr(theta), _dptr(out), B), "mlp_forward")
        return out

    def gradients(self, theta, target):
        loss = ctypes.c_float()
        g = np.empty(self.num_params, np.float32)
        self._check(lib().mlp_gradients(self.h, _dptr(theta), _dptr(target), theta.shape[0], ctypes.byref(loss),
                                        _ptr(g)), "mlp_gradients")
        return loss.value, self.unflatten(g)

    def train_step(self, theta, target, lr, want_loss=True):
        loss = ctypes.c_float()
        self._check(lib().mlp_train_step(self.h, _dptr(theta), _dptr(target), theta.shape[0], float(lr),
                                         ctypes.byref(loss) if want_loss else None), "mlp_train_step")
        return loss.value if want_loss else None

    def flops(self, B, training):
        return lib().mlp_flops(self.h, int(B), int(training))
