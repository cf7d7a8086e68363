"""ctypes binding of libpfmm.so: argument marshalling only.

Device vectors are torch tensors (float64, on the tree's GPU); their data
pointers and the current HIP stream are handed to the C ABI.  Every step of
the computation runs in the library's kernels.  Loading fails loudly when the
library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STATUS_NAMES = {0: "PFMM_OK", -1: "PFMM_EINVAL", -2: "PFMM_ENOMEM", -3: "PFMM_EDEVICE",
                -4: "PFMM_ENOTCONV", -5: "PFMM_ENONFINITE", -6: "PFMM_EUNSUPPORTED"}
PROFILE_STAGES = ["permute", "s2m", "m2m", "m2l", "l2l", "l2t", "nearfield", "unpermute"]
OP_V, OP_K, OP_K1 = 1, 2, 4
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
NF_STORED, NF_TOEPLITZ = 0, 1


class PfmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("m_t", ctypes.c_int32), ("m_x", ctypes.c_int32),
                ("n_max", ctypes.c_int32), ("c_st", ctypes.c_double), ("n_tr", ctypes.c_int32),
                ("q_reg", ctypes.c_int32), ("q_sing", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("operators", ctypes.c_int32), ("check_finite", ctypes.c_int32), ("nearfield_mode", ctypes.c_int32),
                ("nearfield_gemm", ctypes.c_int32), ("device_mem_budget", ctypes.c_uint64)]


class Stats(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("n_levels_far", ctypes.c_int32), ("boxes", ctypes.c_int64),
                ("leaves", ctypes.c_int64), ("near_entries", ctypes.c_int64), ("m2l_pairs", ctypes.c_int64),
                ("near_row_groups", ctypes.c_int64), ("distinct_integrals", ctypes.c_int64),
                ("device_bytes", ctypes.c_uint64), ("m2l_matrix_cores", ctypes.c_int32),
                ("near_gemm_groups", ctypes.c_int32), ("n_time_classes", ctypes.c_int32),
                ("near_entries_V", ctypes.c_int64), ("near_entries_K", ctypes.c_int64),
                ("near_nonzero_K", ctypes.c_int64), ("near_entries_K1", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("inner_precision", ctypes.c_int32),
                ("x0_dev", ctypes.c_void_p), ("precond", ctypes.c_void_p), ("precond_path", ctypes.c_char_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("true_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int32),
                ("history_len", ctypes.c_int32), ("outer", ctypes.c_int32), ("precond_fallback", ctypes.c_int32)]


def lib_path():
    return os.path.join(_HERE, "libpfmm.so")


def load_library():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(python paper_2106_15911_amd/build.py)")
    lib = ctypes.CDLL(path)
    P, I64, I32, VP = ctypes.POINTER, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    dp, ip = P(ctypes.c_double), P(ctypes.c_int32)
    sig = {
        "pfmm_default_params": ([P(Params)], I32),
        "pfmm_build_tree": ([dp, I64, ip, I64, dp, I64, P(Params), I32, VP, P(VP)], I32),
        "pfmm_apply_V": ([VP, VP, VP, VP], I32),
        "pfmm_apply_K": ([VP, VP, VP, VP], I32),
        "pfmm_apply_K1": ([VP, VP, VP, VP], I32),
        "pfmm_dirichlet_rhs_p1": ([VP, VP, VP, VP], I32),
        "pfmm_solve_dirichlet_p1": ([VP, VP, VP, P(SolveOpts), P(SolveInfo), VP], I32),
        "pfmm_tree_stats": ([VP, P(Stats)], I32),
        "pfmm_autotune": ([VP, ctypes.c_char_p, VP, P(I32), P(I32)], I32),
        "pfmm_representation": ([VP, VP, VP, VP, I64, I32, VP, VP], I32),
        "pfmm_plan_stats": ([dp, I64, ip, I64, dp, I64, P(Params), P(Stats)], I32),
        "pfmm_profile_enable": ([VP, I32], I32),
        "pfmm_set_precision": ([VP, I32], I32),
        "pfmm_profile_read": ([VP, dp, P(I64), P(I32)], I32),
        "pfmm_default_solve_opts": ([P(SolveOpts)], I32),
        "pfmm_solve_V": ([VP, VP, VP, P(SolveOpts), P(SolveInfo), VP], I32),
        "pfmm_solve_dirichlet": ([VP, VP, VP, P(SolveOpts), P(SolveInfo), VP], I32),
        "pfmm_dirichlet_rhs": ([VP, VP, VP, VP], I32),
        "pfmm_destroy": ([VP], None),
        "pfmm_batch_create": ([P(VP), I32, P(VP)], I32),
        "pfmm_apply_V_batch": ([VP, P(VP), P(VP), VP], I32),
        "pfmm_batch_destroy": ([VP], None),
        "pfmm_batch_set_cross_m2l": ([VP, I32], I32),
        "pfmm_precond_create": ([I32, I32, I32, ctypes.c_uint64, P(VP)], I32),
        "pfmm_precond_train": ([VP, VP, VP, I32, I32, I32, ctypes.c_float, ctypes.c_uint64,
                                P(ctypes.c_float), VP], I32),
        "pfmm_precond_apply": ([VP, VP, VP, VP, VP], I32),
        "pfmm_precond_apply_noalloc": ([VP, VP, VP, VP, VP], I32),
        "pfmm_precond_save": ([VP, ctypes.c_char_p], I32),
        "pfmm_precond_load": ([ctypes.c_char_p, I32, P(VP)], I32),
        "pfmm_precond_destroy": ([VP], None),
        "pfmm_solve_V_precond": ([VP, VP, I32, VP, VP, P(SolveOpts), P(SolveInfo), VP], I32),
        "pfmm_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = lib
    return lib


def _check(status):
    if status != 0:
        raise PfmmError(status, load_library().pfmm_last_error().decode())


def default_params(**kw):
    p = Params()
    _check(load_library().pfmm_default_params(ctypes.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _mesh_args(vertices, triangles, time_nodes):
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    t = np.ascontiguousarray(triangles, dtype=np.int32)
    tn = np.ascontiguousarray(time_nodes, dtype=np.float64)
    if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3 or tn.ndim != 1:
        raise ValueError("vertices (n,3), triangles (m,3), time_nodes (E_t+1,)")
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    return (v, t, tn), (v.ctypes.data_as(dp), v.shape[0], t.ctypes.data_as(ip), t.shape[0],
                        tn.ctypes.data_as(dp), tn.shape[0] - 1)


def plan_stats(vertices, triangles, time_nodes, params=None):
    """Host-only planning (no GPU): counts of the tree and its lists."""
    keep, args = _mesh_args(vertices, triangles, time_nodes)
    st = Stats()
    _check(load_library().pfmm_plan_stats(*args, ctypes.byref(params) if params is not None else None,
                                          ctypes.byref(st)))
    return st.as_dict()


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Tree:
    """A built tree on one GPU; apply_V / apply_K take and return torch tensors."""

    def __init__(self, vertices, triangles, time_nodes, params=None, device=0, stream=None):
        import torch
        self.lib = load_library()
        keep, args = _mesh_args(vertices, triangles, time_nodes)
        self.n_dofs = int(args[3]) * int(args[5])
        self.n_vertex_dofs = int(args[1]) * int(args[5])    # p1 vectors: steps x vertices
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.pfmm_build_tree(*args, ctypes.byref(params) if params is not None else None,
                                            device, _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def _apply(self, fn, x, out, stream, n_in=None):
        import torch
        n_in = self.n_dofs if n_in is None else n_in
        if x.dtype != torch.float64 or x.device != self.device or x.numel() != n_in:
            raise ValueError(f"expected a float64 tensor of {n_in} entries on {self.device}")
        x = x.contiguous()
        if out is None:
            out = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        _check(fn(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def apply_V(self, w, out=None, stream=None):
        return self._apply(self.lib.pfmm_apply_V, w, out, stream)

    def apply_K(self, u, out=None, stream=None):
        return self._apply(self.lib.pfmm_apply_K, u, out, stream)

    def apply_K1(self, u, out=None, stream=None):
        """The double layer with p1-continuous trial functions: u per (step, vertex), time-major."""
        return self._apply(self.lib.pfmm_apply_K1, u, out, stream, n_in=self.n_vertex_dofs)

    def dirichlet_rhs_p1(self, g, out=None, stream=None):
        """(1/2 M_h + K_h) g for a p1 datum g (steps x vertices); needs OP_K1."""
        return self._apply(self.lib.pfmm_dirichlet_rhs_p1, g, out, stream, n_in=self.n_vertex_dofs)

    def _solve(self, fn, rhs, out, rtol, max_iter, stream, raise_on_notconv, x0=None, precond=None,
               precond_path=None, inner_precision=FP64, n_rhs=None):
        import torch
        for v, n in ((rhs, self.n_dofs if n_rhs is None else n_rhs), (x0, self.n_dofs)):
            if v is not None and (v.dtype != torch.float64 or v.device != self.device or v.numel() != n
                                  or not v.is_contiguous()):
                raise ValueError(f"expected a contiguous float64 tensor of {n} entries on {self.device}")
        if out is None:
            out = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        o = SolveOpts()
        _check(self.lib.pfmm_default_solve_opts(ctypes.byref(o)))
        o.rtol, o.max_iter, o.inner_precision = rtol, max_iter, int(inner_precision)
        o.x0_dev = x0.data_ptr() if x0 is not None else None
        o.precond = precond.handle.value if precond is not None else None
        o.precond_path = str(precond_path).encode() if precond_path is not None else None
        hist = (ctypes.c_double * (max_iter + 1))()
        info = SolveInfo()
        info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        info.history_cap = max_iter + 1
        st = fn(self.handle, ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(out.data_ptr()), ctypes.byref(o),
                ctypes.byref(info), _stream_ptr(stream))
        d = {"iters": info.iters, "converged": bool(info.converged), "rel_residual": info.rel_residual,
             "true_rel_residual": info.true_rel_residual, "seconds": info.seconds,
             "history": list(hist[:info.history_len]), "outer": info.outer,
             "precond_fallback": bool(info.precond_fallback)}
        if st != 0 and not (st == -4 and not raise_on_notconv):
            _check(st)
        return out, d

    def solve_V_precond(self, b, precond=None, inner_precision=FP64, out=None, rtol=1e-8, max_iter=200, stream=None,
                        raise_on_notconv=True, x0=None):
        """FP64 iterative refinement around flexible GMRES with the learned preconditioner
        (None: no preconditioner) and inner applies in `inner_precision`; returns (w, info)."""
        h = precond.handle if precond is not None else None
        fn = lambda tree, rhs, x, o, info, st: self.lib.pfmm_solve_V_precond(tree, h, int(inner_precision), rhs, x, o,
                                                                             info, st)
        return self._solve(fn, b, out, rtol, max_iter, stream, raise_on_notconv, x0=x0)

    def solve_V(self, b, out=None, rtol=1e-8, max_iter=200, stream=None, raise_on_notconv=True, x0=None,
                precond=None, precond_path=None, inner_precision=FP64):
        """Solve V_h w = b (device tensors, natural order): GMRES from x0 (None: 0), or the
        refinement solve when a preconditioner or a reduced inner precision is given;
        returns (w, info)."""
        return self._solve(self.lib.pfmm_solve_V, b, out, rtol, max_iter, stream, raise_on_notconv, x0, precond,
                           precond_path, inner_precision)

    def dirichlet_rhs(self, g, out=None, stream=None):
        """(1/2 M_h + K_h) g on the device (needs K_h)."""
        return self._apply(self.lib.pfmm_dirichlet_rhs, g, out, stream)

    def solve_dirichlet(self, g, out=None, rtol=1e-8, max_iter=200, stream=None, raise_on_notconv=True, x0=None,
                        precond=None, precond_path=None, inner_precision=FP64):
        """Solve V_h w = (1/2 M_h + K_h) g, options as solve_V; returns (w, info)."""
        return self._solve(self.lib.pfmm_solve_dirichlet, g, out, rtol, max_iter, stream, raise_on_notconv, x0,
                           precond, precond_path, inner_precision)

    def solve_dirichlet_p1(self, g, out=None, rtol=1e-8, max_iter=200, stream=None, raise_on_notconv=True, x0=None,
                           precond=None, precond_path=None, inner_precision=FP64):
        """Solve V_h w = (1/2 M_h + K_h) g for a p1 datum g (steps x vertices); options as solve_V."""
        return self._solve(self.lib.pfmm_solve_dirichlet_p1, g, out, rtol, max_iter, stream, raise_on_notconv, x0,
                           precond, precond_path, inner_precision, n_rhs=self.n_vertex_dofs)

    def representation(self, w, u, xt, q=4, out=None, stream=None):
        """(V~ w - W u)(x_i, t_i) at the rows (x, y, z, t) of xt (float64 device tensor, M x 4);
        w or u may be None."""
        import torch
        for v in (w, u):
            if v is not None and (v.dtype != torch.float64 or v.device != self.device or v.numel() != self.n_dofs
                                  or not v.is_contiguous()):
                raise ValueError(f"expected a contiguous float64 tensor of {self.n_dofs} entries on {self.device}")
        if xt.dtype != torch.float64 or xt.device != self.device or xt.dim() != 2 or xt.shape[1] != 4:
            raise ValueError("xt must be a float64 (M, 4) tensor on the tree's device")
        xt = xt.contiguous()
        if out is None:
            out = torch.empty(xt.shape[0], dtype=torch.float64, device=self.device)
        _check(self.lib.pfmm_representation(self.handle, ctypes.c_void_p(w.data_ptr()) if w is not None else None,
                                            ctypes.c_void_p(u.data_ptr()) if u is not None else None,
                                            ctypes.c_void_p(xt.data_ptr()), xt.shape[0], int(q),
                                            ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def autotune(self, cache_path=None, stream=None):
        """Time the M2L launch choices per level and precision (cached in cache_path);
        returns (levels timed, levels taken from the cache)."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.pfmm_autotune(self.handle, str(cache_path).encode() if cache_path else None,
                                      _stream_ptr(stream), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def stats(self):
        st = Stats()
        _check(self.lib.pfmm_tree_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def set_precision(self, precision):
        """Farfield precision of the following applies: FP64 or MIXED_FP32 (tree built in MIXED_FP32)."""
        _check(self.lib.pfmm_set_precision(self.handle, int(precision)))

    def profile_enable(self, on=True):
        _check(self.lib.pfmm_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self):
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_int64 * 8)()
        n = ctypes.c_int32()
        _check(self.lib.pfmm_profile_read(self.handle, ms, cnt, ctypes.byref(n)))
        return {PROFILE_STAGES[i]: (ms[i], cnt[i]) for i in range(n.value)}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pfmm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent trees (same device) applied together: apply_V(ws) returns
    [V_h^(i) w_i]; the applies run as one captured HIP graph (re-captured when
    the output/input tensors change)."""

    def __init__(self, trees):
        self.lib = load_library()
        self.trees = list(trees)
        arr = (ctypes.c_void_p * len(self.trees))(*[t.handle.value for t in self.trees])
        h = ctypes.c_void_p()
        _check(self.lib.pfmm_batch_create(arr, len(self.trees), ctypes.byref(h)))
        self.handle = h

    def apply_V(self, ws, outs=None, stream=None):
        import torch
        if len(ws) != len(self.trees):
            raise ValueError("one density per tree")
        for t, x in zip(self.trees, ws):
            if x.dtype != torch.float64 or x.device != t.device or x.numel() != t.n_dofs or not x.is_contiguous():
                raise ValueError(f"expected a contiguous float64 tensor of {t.n_dofs} entries on {t.device}")
        if outs is None:
            outs = [torch.empty_like(x) for x in ws]
        wp = (ctypes.c_void_p * len(ws))(*[x.data_ptr() for x in ws])
        fp = (ctypes.c_void_p * len(ws))(*[y.data_ptr() for y in outs])
        _check(self.lib.pfmm_apply_V_batch(self.handle, wp, fp, _stream_ptr(stream)))
        return outs

    def set_cross_m2l(self, enable):
        """One M2L launch across the trees (levels with unequal intervals) or whole applies per tree."""
        _check(self.lib.pfmm_batch_set_cross_m2l(self.handle, 1 if enable else 0))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pfmm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Precond:
    """The learned temporal-block preconditioner (FP32 perceptron on the GPU)."""

    def __init__(self, device=0, features=8, hidden=256, seed=1, path=None):
        self.lib = load_library()
        h = ctypes.c_void_p()
        if path is not None:
            _check(self.lib.pfmm_precond_load(str(path).encode(), device, ctypes.byref(h)))
        else:
            _check(self.lib.pfmm_precond_create(device, features, hidden, seed, ctypes.byref(h)))
        self.handle = h

    def train(self, tree, b, n_snap=8, steps=1500, batch=4096, lr=1e-3, seed=7, stream=None):
        """Fit on pairs from FP64 GMRES solves of tree's V_h x = b (device tensor); returns the last loss."""
        loss = ctypes.c_float()
        _check(self.lib.pfmm_precond_train(self.handle, tree.handle, ctypes.c_void_p(b.data_ptr()), n_snap, steps,
                                           batch, lr, seed, ctypes.byref(loss), _stream_ptr(stream)))
        return float(loss.value)

    def apply(self, tree, v, out=None, stream=None):
        """z = s N(x(v)) on tree's mesh (float64 device tensors in the natural order)."""
        import torch
        if v.dtype != torch.float64 or v.device != tree.device or v.numel() != tree.n_dofs:
            raise ValueError(f"expected a float64 tensor of {tree.n_dofs} entries on {tree.device}")
        v = v.contiguous()
        if out is None:
            out = torch.empty_like(v)
        _check(self.lib.pfmm_precond_apply(self.handle, tree.handle, ctypes.c_void_p(v.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def apply_noalloc(self, tree, v, out, stream=None):
        """As apply, through the entry point that allocates no device memory
        (library-held scratch; stream-ordered, no synchronisation); `out` is
        required."""
        import torch
        for x in (v, out):
            if (x.dtype != torch.float64 or x.device != tree.device or x.numel() != tree.n_dofs
                    or not x.is_contiguous()):
                raise ValueError(f"expected contiguous float64 tensors of {tree.n_dofs} entries on {tree.device}")
        _check(self.lib.pfmm_precond_apply_noalloc(self.handle, tree.handle, ctypes.c_void_p(v.data_ptr()),
                                                   ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def save(self, path):
        _check(self.lib.pfmm_precond_save(self.handle, str(path).encode()))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pfmm_precond_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
