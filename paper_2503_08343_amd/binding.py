"""Thin ctypes binding of libgmrf.so (C ABI in include/gmrf.h).

Argument marshalling only: every step of the posterior path runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  The library must exist
(built by ``paper_2503_08343_amd.build``); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmrf.so")

GMRF_OK = 0
GMRF_ERR_ARG = -1
GMRF_ERR_STATE = -2
GMRF_ERR_NOT_SPD = -3
GMRF_ERR_PATTERN = -4
GMRF_ERR_HIP = -5
GMRF_ERR_OOM = -6
GMRF_ERR_NOT_CONVERGED = -7
GMRF_FP64 = 0
GMRF_FP32_REFINE = 1

EXPORTS = ["gmrf_create", "gmrf_destroy", "gmrf_assemble", "gmrf_update_values", "gmrf_analyze",
           "gmrf_factor", "gmrf_logdet", "gmrf_solve", "gmrf_sample", "gmrf_selinv", "gmrf_selinv_submit",
           "gmrf_selinv_wait", "gmrf_dot",
           "gmrf_stats", "gmrf_pivot_order", "gmrf_phase_ms", "gmrf_last_error",
           "gmrf_symbolic_host", "gmrf_profile", "gmrf_kernel_stats", "gmrf_matern_values",
           "gmrf_spmv", "gmrf_misfit", "gmrf_solve_rhs", "gmrf_gn_burgers", "gmrf_launch_records",
           "gmrf_logdet_noalloc", "gmrf_lml_gradient", "gmrf_gn_pointwise", "gmrf_pcg", "gmrf_sample_cg",
           "gmrf_rbmc_variances"]


class gmrf_options(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("relax_small", ctypes.c_int32),
                ("relax_mid", ctypes.c_int32), ("relax_big", ctypes.c_int32)]


class gmrf_stats_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz_q", ctypes.c_int64), ("m", ctypes.c_int64),
                ("nnz_a", ctypes.c_int64), ("nnz_l", ctypes.c_int64), ("stored_l", ctypes.c_int64),
                ("n_super", ctypes.c_int64), ("tree_depth", ctypes.c_int64),
                ("max_front", ctypes.c_int64), ("flops_factor", ctypes.c_double),
                ("flops_selinv", ctypes.c_double), ("flops_solve", ctypes.c_double),
                ("bytes_front_ws", ctypes.c_double), ("bytes_factor", ctypes.c_double),
                ("failed_index", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("refine_resid", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


KERNEL_CLASSES = ["assemble", "equilibrate", "front_zero", "front_scatter", "extend_add",
                  "potrf_diag", "trsm_panel", "update_panel", "syrk_update", "copy_L", "logdet",
                  "solve_fwd", "solve_bwd", "residual", "permute", "sel_gather", "sel_Y",
                  "sel_gemm", "sel_diag", "sel_extract", "sel_reduce", "sel_gemm_small", "syrk_small"]


class gmrf_kernel_stat_t(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class GmrfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gmrf error {code}: {msg}")
        self.code = code


class NotSPDError(GmrfError):
    pass


class NotConvergedError(GmrfError):
    pass


_lib = None


def load():
    """Load libgmrf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2503_08343_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, d = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "gmrf_create": ([ctypes.POINTER(P), ctypes.c_int, P], i32),
        "gmrf_destroy": ([P], i32),
        "gmrf_assemble": ([P, i64, P, P, P, i64, P, P, P, P, P, P, P, i64, P], i32),
        "gmrf_update_values": ([P, P, P, P, P, P], i32),
        "gmrf_analyze": ([P, P, ctypes.c_int, P], i32),
        "gmrf_factor": ([P, ctypes.c_int], i32),
        "gmrf_logdet": ([P, P], i32),
        "gmrf_solve": ([P, P, ctypes.c_int, d, P, P], i32),
        "gmrf_sample": ([P, i64, P, P], i32),
        "gmrf_selinv": ([P, P, P], i32),
        "gmrf_selinv_submit": ([P, P, P], i32),
        "gmrf_selinv_wait": ([P], i32),
        "gmrf_dot": ([P, i64, P, P, P], i32),
        "gmrf_stats": ([P, P], i32),
        "gmrf_pivot_order": ([P, P], i32),
        "gmrf_phase_ms": ([P, P], i32),
        "gmrf_last_error": ([P], ctypes.c_char_p),
        "gmrf_symbolic_host": ([i64, P, P, P, ctypes.c_int, P, P, P, P, P], i32),
        "gmrf_profile": ([P, ctypes.c_int], i32),
        "gmrf_matern_values": ([P, i64, P, P, P, d, d, P, P], i32),
        "gmrf_spmv": ([P, P, P, P], i32),
        "gmrf_misfit": ([P, P, P], i32),
        "gmrf_solve_rhs": ([P, P, P], i32),
        "gmrf_gn_burgers": ([P, i64, i64, d, d, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d,
                             ctypes.c_int, P, P], i32),
        "gmrf_kernel_stats": ([P, P, ctypes.c_int, P], i32),
        "gmrf_logdet_noalloc": ([P, P], i32),
        "gmrf_lml_gradient": ([P, P, ctypes.c_int, P, P, P, ctypes.c_int, d, P, P], i32),
        "gmrf_gn_pointwise": ([P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d,
                               ctypes.c_int, P, P], i32),
        "gmrf_pcg": ([P, i64, P, P, P, ctypes.c_int, ctypes.c_int, d, P, P], i32),
        "gmrf_sample_cg": ([P, i64, i64, P, P, P, P, P, P, ctypes.c_int, ctypes.c_int, d, P], i32),
        "gmrf_rbmc_variances": ([P, i64, P, P], i32),
        "gmrf_launch_records": ([P, P, ctypes.c_int64, P], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _np_ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _t_ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _opts(opts):
    if opts is None:
        return None
    o = gmrf_options()
    for k, v in opts.items():
        setattr(o, k, int(v))
    return ctypes.byref(o)


def symbolic_host(indptr, indices, coords=None, opts=None, perm_in=None):
    """Host-only analysis (no device): returns (perm, colcount, stats dict); perm_in: an
    ordering to analyse instead of the library's nested dissection."""
    lib = load()
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    n = indptr.size - 1
    perm = np.empty(n, dtype=np.int32)
    cc = np.empty(n, dtype=np.int64)
    st = gmrf_stats_t()
    dim = 0
    if coords is not None:
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        dim = coords.shape[1]
    pin = None if perm_in is None else np.ascontiguousarray(perm_in, dtype=np.int32)
    rc = lib.gmrf_symbolic_host(n, _np_ptr(indptr), _np_ptr(indices), _np_ptr(coords), dim,
                                _opts(opts), _np_ptr(pin), _np_ptr(perm), _np_ptr(cc), ctypes.byref(st))
    if rc != GMRF_OK:
        raise GmrfError(rc, "symbolic analysis failed")
    return perm, cc, st.as_dict()


class Context:
    """One library context on a device; every array argument is a torch CUDA tensor."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = device
        self.h = ctypes.c_void_p()
        s = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        self._stream = stream
        rc = self.lib.gmrf_create(ctypes.byref(self.h), device, s)
        if rc != GMRF_OK:
            raise GmrfError(rc, "gmrf_create failed")
        self.n = 0
        self.nblocks = 1

    def close(self):
        if self.h:
            self.lib.gmrf_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc == GMRF_OK:
            return
        msg = self.lib.gmrf_last_error(self.h).decode()
        if rc == GMRF_ERR_NOT_SPD:
            raise NotSPDError(rc, msg)
        if rc == GMRF_ERR_NOT_CONVERGED:
            raise NotConvergedError(rc, msg)
        raise GmrfError(rc, msg)

    def _dev(self, t, dtype):
        if t is None:
            return None
        assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), (t.device, t.dtype)
        return t

    def assemble(self, q_indptr, q_indices, q_data, a_indptr, a_indices, a_data, q_eps, y,
                 b=None, mu=None, block_ptr=None):
        T = self.torch
        n = q_indptr.numel() - 1
        m = 0 if a_indptr is None else a_indptr.numel() - 1
        self.n = n
        bp = None
        nb = 0
        if block_ptr is not None:
            bp = np.ascontiguousarray(block_ptr, dtype=np.int64)
            nb = bp.size - 1
            self.nblocks = nb
        self._keep = [q_indptr, q_indices, q_data, a_indptr, a_indices, a_data, q_eps, y, b, mu]
        rc = self.lib.gmrf_assemble(
            self.h, n, _t_ptr(self._dev(q_indptr, T.int64)), _t_ptr(self._dev(q_indices, T.int32)),
            _t_ptr(self._dev(q_data, T.float64)), m,
            _t_ptr(self._dev(a_indptr, T.int64)), _t_ptr(self._dev(a_indices, T.int32)),
            _t_ptr(self._dev(a_data, T.float64)), _t_ptr(self._dev(q_eps, T.float64)),
            _t_ptr(self._dev(y, T.float64)), _t_ptr(self._dev(b, T.float64)),
            _t_ptr(self._dev(mu, T.float64)), nb, _np_ptr(bp))
        self._check(rc)

    def update_values(self, q_data=None, a_data=None, q_eps=None, y=None, b=None):
        rc = self.lib.gmrf_update_values(self.h, _t_ptr(q_data), _t_ptr(a_data), _t_ptr(q_eps),
                                         _t_ptr(y), _t_ptr(b))
        self._check(rc)

    def analyze(self, coords=None, opts=None):
        dim = 0
        c = None
        if coords is not None:
            c = np.ascontiguousarray(coords, dtype=np.float64)
            dim = c.shape[1]
        self._check(self.lib.gmrf_analyze(self.h, _np_ptr(c), dim, _opts(opts)))

    def factor(self, precision=GMRF_FP64):
        self._check(self.lib.gmrf_factor(self.h, int(precision)))

    def logdet(self):
        out = np.zeros(self.nblocks)
        self._check(self.lib.gmrf_logdet(self.h, _np_ptr(out)))
        return out

    def logdet_noalloc(self, out):
        """Log-determinant per block into the device tensor `out` (float64, n_blocks),
        asynchronous, through the library's fixed workspace (no allocation)."""
        self._check(self.lib.gmrf_logdet_noalloc(self.h, _t_ptr(out)))
        return out

    def solve(self, max_refine=0, tol=0.0, out=None, raise_not_converged=True):
        T = self.torch
        mu = out if out is not None else T.empty(self.n, dtype=T.float64, device=f"cuda:{self.device}")
        it = ctypes.c_int(0)
        res = ctypes.c_double(0.0)
        rc = self.lib.gmrf_solve(self.h, _t_ptr(mu), int(max_refine), float(tol), ctypes.byref(it),
                                 ctypes.byref(res))
        if rc == GMRF_ERR_NOT_CONVERGED and not raise_not_converged:
            return mu, it.value, res.value
        self._check(rc)
        return mu, it.value, res.value

    def sample(self, z_kn):
        """z_kn: (k, n) float32 CUDA tensor, row r = r-th standard-normal vector in pivot
        order (its memory is the n x k column-major block of the C ABI).  Returns the
        (k, n) float64 samples, row r in original order."""
        T = self.torch
        z_kn = self._dev(z_kn, T.float32)
        if z_kn.dim() == 1:
            z_kn = z_kn.unsqueeze(0)
        k = z_kn.shape[0]
        x = T.empty((k, self.n), dtype=T.float64, device=z_kn.device)
        self._check(self.lib.gmrf_sample(self.h, k, _t_ptr(z_kn), _t_ptr(x)))
        return x

    def selinv(self, with_pattern=False, nnzq=None):
        T = self.torch
        var = T.empty(self.n, dtype=T.float64, device=f"cuda:{self.device}")
        sq = None
        if with_pattern:
            sq = T.empty(int(nnzq), dtype=T.float64, device=f"cuda:{self.device}")
        self._check(self.lib.gmrf_selinv(self.h, _t_ptr(var), _t_ptr(sq)))
        return var if sq is None else (var, sq)

    def selinv_submit(self, with_pattern=False, nnzq=None):
        """Start the selected inversion on the library's second stream; the returned
        tensors are valid after selinv_wait().  Solves, samples and log-determinants of
        the same factor may be called meanwhile."""
        T = self.torch
        var = T.empty(self.n, dtype=T.float64, device=f"cuda:{self.device}")
        sq = None
        if with_pattern:
            sq = T.empty(int(nnzq), dtype=T.float64, device=f"cuda:{self.device}")
        self._check(self.lib.gmrf_selinv_submit(self.h, _t_ptr(var), _t_ptr(sq)))
        self._sel_pending = (var, sq)
        return var if sq is None else (var, sq)

    def selinv_wait(self):
        self._check(self.lib.gmrf_selinv_wait(self.h))
        self._sel_pending = None

    def dot(self, a, b):
        out = np.zeros(1)
        self._check(self.lib.gmrf_dot(self.h, a.numel(), _t_ptr(a), _t_ptr(b), _np_ptr(out)))
        return float(out[0])

    def matern_values(self, m_on_q, s_on_q, sms_on_q, kappa, tau, q_out, dq_out=None):
        self._check(self.lib.gmrf_matern_values(self.h, m_on_q.numel(), _t_ptr(m_on_q), _t_ptr(s_on_q),
                                                _t_ptr(sms_on_q), float(kappa), float(tau), _t_ptr(q_out),
                                                _t_ptr(dq_out)))

    def spmv(self, v_val, x, y):
        self._check(self.lib.gmrf_spmv(self.h, _t_ptr(v_val), _t_ptr(x), _t_ptr(y)))
        return y

    def lml_gradient(self, prior, dq=None, da=None, dqeps=None, max_refine=0, tol=0.0, mu_out=None):
        """(LML, gradient) of gmrf_lml_gradient; this context holds the posterior, `prior`
        the prior alone; dq / da / dqeps: device tensors (k, nnz_q) / (k, nnz_a) /
        (k, m) or None; mu_out: device tensor (n) receiving the posterior mean, or None."""
        k = 0 if dq is None else int(dq.shape[0])
        out = np.zeros(1 + k)
        rc = self.lib.gmrf_lml_gradient(self.h, prior.h, k, _t_ptr(dq), _t_ptr(da), _t_ptr(dqeps),
                                        int(max_refine), float(tol), _np_ptr(out), _t_ptr(mu_out))
        if rc != GMRF_ERR_NOT_CONVERGED:
            self._check(rc)
        return float(out[0]), out[1:].copy()

    def solve_rhs(self, rhs, out=None):
        T = self.torch
        x = out if out is not None else T.empty_like(rhs)
        self._check(self.lib.gmrf_solve_rhs(self.h, _t_ptr(rhs), _t_ptr(x)))
        return x

    def gn_burgers(self, nx, nt, dt, nu, mass, stiff3, u, iters=10, precision=GMRF_FP64, refine=2,
                   use_graph=True, refine_tol=0.0, decrement_tol=0.0):
        """Gauss-Newton iterations on the assembled Burgers problem; u (device) is updated in
        place.  Returns the per-iteration records (objective, step, decrement, slope,
        relative residual of the linearised solve, corrections applied; NaN rows for the
        iterations a decrement_tol > 0 stopping rule skipped)."""
        rec = np.zeros(6 * iters)
        self._check(self.lib.gmrf_gn_burgers(self.h, int(nx), int(nt), float(dt), float(nu), _t_ptr(mass),
                                             _t_ptr(stiff3), int(iters), int(precision), int(refine),
                                             float(refine_tol), float(decrement_tol), 1 if use_graph else 0,
                                             _t_ptr(u), _np_ptr(rec)))
        return rec.reshape(iters, 6)

    def gn_pointwise(self, lin_val, nl_col, nl_coef, power, u, iters=10, precision=GMRF_FP64, refine=2,
                     use_graph=True, refine_tol=0.0, decrement_tol=0.0):
        """Gauss-Newton for residuals with a pointwise power nonlinearity (gmrf_gn_pointwise);
        u (device) is updated in place; returns the per-iteration records like gn_burgers."""
        rec = np.zeros(6 * iters)
        self._check(self.lib.gmrf_gn_pointwise(self.h, _t_ptr(lin_val), _t_ptr(nl_col), _t_ptr(nl_coef),
                                               int(power), int(iters), int(precision), int(refine),
                                               float(refine_tol), float(decrement_tol), 1 if use_graph else 0,
                                               _t_ptr(u), _np_ptr(rec)))
        return rec.reshape(iters, 6)

    def pcg(self, rhs=None, x0=None, precond=1, maxit=1000, tol=1e-12, raise_not_converged=True):
        """Preconditioned CG (gmrf_pcg): rhs (device, n or n x k as (k, n)) or None for the
        posterior mean; returns (x, iterations, relative residuals)."""
        T = self.torch
        k = 1 if rhs is None or rhs.dim() == 1 else int(rhs.shape[0])
        x = T.empty((k, self.n), dtype=T.float64, device="cuda")
        its = np.zeros(k, dtype=np.int32)
        res = np.zeros(k)
        rc = self.lib.gmrf_pcg(self.h, k, _t_ptr(rhs), _t_ptr(x0), _t_ptr(x), int(precond), int(maxit), float(tol),
                               _np_ptr(its), _np_ptr(res))
        if rc != GMRF_ERR_NOT_CONVERGED or raise_not_converged:
            self._check(rc)
        return (x[0] if k == 1 and (rhs is None or rhs.dim() == 1) else x), its, res

    def sample_cg(self, r_indptr, r_indices, r_data, w1, w2, precond=1, maxit=1000, tol=1e-12):
        """CG sampling (gmrf_sample_cg): R as device CSR tensors (n x r), w1 (k, r), w2 (k, m);
        returns (x (k, n), iterations)."""
        T = self.torch
        k, r = int(w1.shape[0]), int(w1.shape[1])
        x = T.empty((k, self.n), dtype=T.float64, device="cuda")
        its = np.zeros(k, dtype=np.int32)
        self._check(self.lib.gmrf_sample_cg(self.h, k, r, _t_ptr(r_indptr), _t_ptr(r_indices), _t_ptr(r_data),
                                            _t_ptr(w1), _t_ptr(w2), _t_ptr(x), int(precond), int(maxit),
                                            float(tol), _np_ptr(its)))
        return x, its

    def rbmc_variances(self, xs):
        """Rao-Blackwellised variances from centred draws xs (k, n) (gmrf_rbmc_variances)."""
        T = self.torch
        var = T.empty(self.n, dtype=T.float64, device="cuda")
        self._check(self.lib.gmrf_rbmc_variances(self.h, int(xs.shape[0]), _t_ptr(xs.contiguous()), _t_ptr(var)))
        return var

    def misfit(self, x):
        out = np.zeros(1)
        self._check(self.lib.gmrf_misfit(self.h, _t_ptr(x), _np_ptr(out)))
        return float(out[0])

    def stats(self):
        st = gmrf_stats_t()
        rc = self.lib.gmrf_stats(self.h, ctypes.byref(st))
        self._check(rc)
        return st.as_dict()

    def pivot_order(self):
        p = np.empty(self.n, dtype=np.int32)
        self._check(self.lib.gmrf_pivot_order(self.h, _np_ptr(p)))
        return p

    def profile(self, enable=True, classes=None):
        """enable: switch per-launch events on/off; classes: optional list of kernel-class
        names (as reported by kernel_stats) restricting the events to those classes."""
        val = 1 if enable else 0
        if enable and classes:
            names = KERNEL_CLASSES
            val = 0
            for c in classes:
                val |= 1 << names.index(c)
            if val == 1:   # class 0 alone would read as "all"; widen by an unused bit
                val |= 1 << 31
        self._check(self.lib.gmrf_profile(self.h, val))

    def kernel_stats(self):
        cnt = ctypes.c_int(0)
        self._check(self.lib.gmrf_kernel_stats(self.h, None, 0, ctypes.byref(cnt)))
        arr = (gmrf_kernel_stat_t * cnt.value)()
        self._check(self.lib.gmrf_kernel_stats(self.h, arr, cnt.value, ctypes.byref(cnt)))
        return {a.name.decode(): dict(launches=a.launches, ms=a.ms, flops=a.flops, bytes=a.bytes)
                for a in arr}

    def launch_records(self):
        """Per-launch profile records since the last profile() call: structured array
        with fields cls (class name), flops, bytes, ms."""
        cnt = ctypes.c_int64(0)
        self._check(self.lib.gmrf_launch_records(self.h, None, 0, ctypes.byref(cnt)))
        raw = np.zeros(cnt.value, dtype=[("cls", np.int32), ("reserved", np.int32), ("flops", np.float64),
                                         ("bytes", np.float64), ("ms", np.float64)])
        if cnt.value:
            self._check(self.lib.gmrf_launch_records(self.h, _np_ptr(raw), cnt.value, ctypes.byref(cnt)))
        names = np.array(KERNEL_CLASSES)
        out = np.zeros(len(raw), dtype=[("cls", "U16"), ("flops", np.float64), ("bytes", np.float64),
                                        ("ms", np.float64)])
        out["cls"] = names[raw["cls"]] if len(raw) else []
        for f in ("flops", "bytes", "ms"):
            out[f] = raw[f]
        return out

    def phase_ms(self):
        out = np.zeros(3)
        self._check(self.lib.gmrf_phase_ms(self.h, _np_ptr(out)))
        return dict(factor=out[0], solve=out[1], selinv=out[2])


def problem_to_device(problem, device="cuda:0"):
    """Upload a gmrf_inputs.Problem's arrays as torch tensors (plumbing only)."""
    import torch
    qi, qj, qv = problem.csr("Q")
    ai, aj, av = problem.csr("A")

    def t(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
    d = dict(q_indptr=t(qi, torch.int64), q_indices=t(qj, torch.int32), q_data=t(qv, torch.float64),
             a_indptr=t(ai, torch.int64), a_indices=t(aj, torch.int32), a_data=t(av, torch.float64),
             q_eps=t(problem.q_eps, torch.float64), y=t(problem.y, torch.float64),
             b=t(problem.b, torch.float64) if problem.b is not None else None,
             mu=t(problem.mu, torch.float64) if problem.mu is not None else None)
    return d


def posterior_context(problem, precision=GMRF_FP64, device=0, opts=None, use_coords=True):
    """assemble -> analyze -> factor for a Problem; returns the Context."""
    ctx = Context(device)
    d = problem_to_device(problem, f"cuda:{device}")
    ctx.assemble(**d, block_ptr=problem.block_ptr)
    ctx.analyze(problem.coords if use_coords else None, opts)
    ctx.factor(precision)
    return ctx
