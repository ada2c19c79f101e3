"""ctypes binding of libhss.so (include/hss.h). Argument marshalling only:
every step of the factorization, apply and GMRES runs in the library.

Device vectors are torch tensors (float64 or complex128, on the GPU); torch is
used for device memory and streams only. The library must have been built
(``python -m paper_1508_07798_amd.build``); nothing here falls back to any
other implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhss.so")

HSS_OK, HSS_EINVAL, HSS_ENOMEM, HSS_ESINGULAR, HSS_ENOCONV, HSS_EDEVICE, HSS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
HSS_R64, HSS_C128 = 0, 1
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
MLP_NPARAMS = 4801

EXPORTS = ["hss_default_opts", "hss_factor", "hss_factor_batched", "hss_apply", "gmres_solve", "hss_query",
           "hss_destroy", "hss_last_error", "hss_plan_create", "hss_plan_query", "hss_plan_destroy",
           "hss_mlp_forward", "hss_mlp_grad", "hss_mlp_train", "hss_mlp_grad_noalloc", "hss_rank_model_train",
           "hss_tuning_load", "hss_tuning_set", "hss_tuning_clear", "hss_tuning_candidates"]


class BlockOp(C.Structure):
    _fields_ = [("n_el", C.c_int32), ("q", C.c_int32), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("vals", C.c_void_p), ("dtype", C.c_int), ("vals_on_device", C.c_int32)]


class TreeC(C.Structure):
    _fields_ = [("n_leaves", C.c_int32), ("leaf_node", C.c_void_p), ("leaf_ptr", C.c_void_p),
                ("leaf_elems", C.c_void_p), ("elem_xy", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("prec", C.c_int), ("p_os", C.c_int32), ("l0", C.c_int32), ("max_attempts", C.c_int32),
                ("seed", C.c_uint64), ("rank_model", C.c_void_p), ("kappa_h", C.c_double),
                ("hip_stream", C.c_void_p), ("profile", C.c_int32), ("apply_graph", C.c_int32),
                ("hss_leaf_elems", C.c_int32), ("rank_model_path", C.c_char_p), ("keep_box", C.c_int32),
                ("ldu", C.c_int32), ("model_margin", C.c_double)]


class GmresInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("true_relres", C.c_double),
                ("status", C.c_int32)]


class HssError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1508_07798_amd.build`")
        L = C.CDLL(LIB_PATH)
        L.hss_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("hss_last_error", "hss_default_opts", "hss_destroy", "hss_plan_destroy",
                            "hss_tuning_clear"):
                getattr(L, name).restype = C.c_int
        L.hss_factor.argtypes = [C.POINTER(BlockOp), C.POINTER(TreeC), C.c_double, C.POINTER(Opts),
                                 C.POINTER(C.c_void_p)]
        L.hss_factor_batched.argtypes = [C.c_int32, C.POINTER(BlockOp), C.POINTER(TreeC), C.c_double,
                                         C.POINTER(Opts), C.POINTER(C.c_void_p)]
        L.hss_apply.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32]
        L.gmres_solve.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_double,
                                  C.c_int32, C.c_int32, C.c_int32, C.POINTER(GmresInfo)]
        L.hss_query.argtypes = [C.c_void_p, C.c_char_p, C.POINTER(C.c_double), C.c_int64,
                                C.POINTER(C.c_int64)]
        L.hss_destroy.argtypes = [C.c_void_p]
        L.hss_destroy.restype = None
        L.hss_default_opts.argtypes = [C.POINTER(Opts)]
        L.hss_default_opts.restype = None
        L.hss_plan_create.argtypes = [C.POINTER(BlockOp), C.POINTER(TreeC), C.c_int32, C.POINTER(C.c_void_p)]
        L.hss_rank_model_train.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_char_p, C.c_uint64]
        L.hss_plan_query.argtypes = [C.c_void_p, C.c_char_p, C.c_int32, C.POINTER(C.c_int64), C.c_int64,
                                     C.POINTER(C.c_int64)]
        L.hss_tuning_load.argtypes = [C.c_char_p]
        L.hss_tuning_set.argtypes = [C.c_int32] * 6
        L.hss_tuning_clear.argtypes = []
        L.hss_tuning_clear.restype = None
        L.hss_tuning_candidates.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
        L.hss_plan_destroy.argtypes = [C.c_void_p]
        L.hss_plan_destroy.restype = None
        L.hss_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        L.hss_mlp_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                   C.POINTER(C.c_double), C.c_void_p]
        L.hss_mlp_grad_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                           C.POINTER(C.c_double), C.c_void_p]
        L.hss_mlp_train.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_float,
                                    C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _check(status):
    if status != HSS_OK:
        raise HssError(status, lib().hss_last_error().decode())


class _Keep:
    """Holds numpy arrays alive while their pointers are in a C struct."""

    def __init__(self):
        self.items = []

    def arr(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.items.append(a)
        return a.ctypes.data


def _op_struct(op, keep: _Keep, vals_dev=None):
    s = BlockOp()
    s.n_el = op.n_el
    s.q = op.q
    s.row_ptr = keep.arr(op.row_ptr, np.int32)
    s.col_idx = keep.arr(op.col_idx, np.int32)
    if vals_dev is not None:
        keep.items.append(vals_dev)
        s.vals = vals_dev.data_ptr()
        s.vals_on_device = 1
    else:
        s.vals = keep.arr(op.vals, np.complex128 if op.is_complex else np.float64)
        s.vals_on_device = 0
    s.dtype = HSS_C128 if op.is_complex else HSS_R64
    return s


def _tree_struct(tree, keep: _Keep):
    t = TreeC()
    t.n_leaves = int(tree.leaf_node.size)
    t.leaf_node = keep.arr(tree.leaf_node, np.int32)
    t.leaf_ptr = keep.arr(tree.leaf_ptr, np.int32)
    t.leaf_elems = keep.arr(tree.leaf_elems, np.int32)
    t.elem_xy = keep.arr(tree.elem_xy.reshape(-1), np.int32)
    return t


def default_opts() -> Opts:
    o = Opts()
    lib().hss_default_opts(C.byref(o))
    return o


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream


class Handle:
    def __init__(self, ptr, ndof, cplx, stream, keep):
        self.ptr = ptr
        self.ndof = ndof
        self.cplx = cplx
        self.stream = stream
        self._keep = keep

    def close(self):
        if self.ptr:
            lib().hss_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, x):
        import torch
        want = torch.complex128 if self.cplx else torch.float64
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == want):
            raise TypeError(f"expected a CUDA tensor of {want}")
        if x.dim() == 1:
            x = x[:, None]
        if x.shape[0] != self.ndof:
            raise ValueError(f"vector length {x.shape[0]} != {self.ndof}")
        return x.t().contiguous().t() if x.stride(0) != 1 else x

    def kept_schur(self):
        """(S, S~) of the box named by factor(..., keep_box=heap id): its Schur complement
        (symmetrized, before compression) and the compressed form, n x n over the box's
        boundary dofs in the planner's order."""
        n = int(self.query("kept_n")[0])
        out = []
        for key in ("kept_S", "kept_St"):
            v = np.asarray(self.query(key))
            if self.cplx:
                v = v[0::2] + 1j * v[1::2]
            out.append(v.reshape((n, n), order="F"))
        return out[0], out[1]

    def _host(self, x):
        want = np.complex128 if self.cplx else np.float64
        x = np.asarray(x)
        if x.dtype != want:
            raise TypeError(f"expected a host array of {want}")
        if x.ndim == 1:
            x = x[:, None]
        if x.shape[0] != self.ndof:
            raise ValueError(f"vector length {x.shape[0]} != {self.ndof}")
        return np.asfortranarray(x)

    def apply(self, x):
        """y = M^{-t} D^{-1} L^{-1} x for a [n] or [n, k] CUDA tensor, or a host
        numpy array (on_device = 0: the library copies it to the device and back)."""
        if isinstance(x, np.ndarray):
            squeeze = x.ndim == 1
            xx = self._host(x)
            y = np.empty_like(xx, order="F")
            _check(lib().hss_apply(self.ptr, xx.shape[1], xx.ctypes.data, self.ndof, y.ctypes.data, self.ndof, 0))
            return y[:, 0] if squeeze else y
        import torch
        squeeze = x.dim() == 1
        xx = self._vec(x)
        y = torch.empty_like(xx).t().contiguous().t()
        ld_x = xx.stride(1) if xx.shape[1] > 1 else self.ndof
        ld_y = y.stride(1) if y.shape[1] > 1 else self.ndof
        _check(lib().hss_apply(self.ptr, xx.shape[1], xx.data_ptr(), ld_x, y.data_ptr(), ld_y, 1))
        return y[:, 0] if squeeze else y

    def gmres(self, b, x0=None, tol=1e-8, restart=30, maxit=1000, nprob=1, raise_on_noconv=True):
        """gmres_solve for a CUDA tensor b (device vectors) or a host numpy array
        (on_device = 0)."""
        if isinstance(b, np.ndarray):
            squeeze = b.ndim == 1
            bb = self._host(b)
            x = np.zeros_like(bb, order="F") if x0 is None else np.array(self._host(x0), order="F")
            k = bb.shape[1]
            info = (GmresInfo * (nprob * k))()
            st = lib().gmres_solve(self.ptr, k, bb.ctypes.data, x.ctypes.data, self.ndof, tol, restart, maxit, 0,
                                   info)
            if st != HSS_OK and not (st == HSS_ENOCONV and not raise_on_noconv):
                _check(st)
            out = [dict(iters=i.iters, restarts=i.restarts, true_relres=i.true_relres, status=i.status)
                   for i in info]
            return (x[:, 0] if squeeze else x), out
        import torch
        squeeze = b.dim() == 1
        bb = self._vec(b).t().contiguous().t()
        x = torch.zeros_like(bb) if x0 is None else self._vec(x0).t().contiguous().t().clone()
        k = bb.shape[1]
        info = (GmresInfo * (nprob * k))()
        st = lib().gmres_solve(self.ptr, k, bb.data_ptr(), x.data_ptr(), self.ndof, tol, restart, maxit, 1, info)
        if st != HSS_OK and not (st == HSS_ENOCONV and not raise_on_noconv):
            _check(st)
        out = [dict(iters=i.iters, restarts=i.restarts, true_relres=i.true_relres, status=i.status) for i in info]
        return (x[:, 0] if squeeze else x), out

    def query(self, key):
        n = C.c_int64(0)
        _check(lib().hss_query(self.ptr, key.encode(), None, 0, C.byref(n)))
        buf = (C.c_double * max(n.value, 1))()
        _check(lib().hss_query(self.ptr, key.encode(), buf, n.value, C.byref(n)))
        v = np.frombuffer(buf, dtype=np.float64, count=n.value).copy()
        return v


def factor(op, tree, tol, prec="fp32", seed=1508, stream=None, l0=32, p_os=10, max_attempts=8,
           rank_model=None, kappa_h=0.0, profile=False, vals_dev=None, apply_graph=True, hss_leaf_elems=4,
           rank_model_path=None, keep_box=0, ldu=2, model_margin=0.0):
    """hss_factor: build the preconditioner of one operator (see include/hss.h)."""
    return factor_batched([op], [tree], tol, prec=prec, seed=seed, stream=stream, l0=l0, p_os=p_os,
                          max_attempts=max_attempts, rank_model=rank_model, kappa_h=kappa_h,
                          profile=profile, vals_dev=None if vals_dev is None else [vals_dev],
                          apply_graph=apply_graph, hss_leaf_elems=hss_leaf_elems,
                          rank_model_path=rank_model_path, keep_box=keep_box, ldu=ldu,
                          model_margin=model_margin)


def factor_batched(ops, trees, tol, prec="fp32", seed=1508, stream=None, l0=32, p_os=10, max_attempts=8,
                   rank_model=None, kappa_h=0.0, profile=False, vals_dev=None, apply_graph=True, hss_leaf_elems=4,
                   rank_model_path=None, keep_box=0, ldu=2, model_margin=0.0):
    keep = _Keep()
    n = len(ops)
    A = (BlockOp * n)(*[_op_struct(op, keep, None if vals_dev is None else vals_dev[i])
                        for i, op in enumerate(ops)])
    T = (TreeC * n)(*[_tree_struct(t, keep) for t in trees])
    o = default_opts()
    o.prec = PREC[prec]
    o.seed = seed
    o.l0 = l0
    o.p_os = p_os
    o.max_attempts = max_attempts
    o.kappa_h = kappa_h
    # True: every kernel class; an int: the class bit mask (bit c + 1 for class c)
    o.profile = (1 if profile else 0) if isinstance(profile, bool) else int(profile)
    o.apply_graph = 1 if apply_graph else 0
    o.hss_leaf_elems = int(hss_leaf_elems)
    o.keep_box = int(keep_box)
    o.ldu = int(ldu)
    o.model_margin = float(model_margin)
    if rank_model_path is not None:
        o.rank_model_path = os.fsencode(rank_model_path)
        keep.items.append(o.rank_model_path)
    o.hip_stream = _stream_ptr(stream)
    if rank_model is not None:
        o.rank_model = keep.arr(rank_model, np.float32)
    h = C.c_void_p()
    _check(lib().hss_factor_batched(n, A, T, tol, C.byref(o), C.byref(h)))
    ndof = sum(op.ndof for op in ops)
    return Handle(h.value, ndof, ops[0].is_complex, o.hip_stream, keep)


class Plan:
    """Host-only planner output (hss_plan_create)."""

    def __init__(self, op, tree, hss_leaf_elems=0):
        keep = _Keep()
        A = _op_struct(op, keep)
        T = _tree_struct(tree, keep)
        p = C.c_void_p()
        _check(lib().hss_plan_create(C.byref(A), C.byref(T), int(hss_leaf_elems), C.byref(p)))
        self.ptr = p.value

    def query(self, key, node=1):
        n = C.c_int64(0)
        _check(lib().hss_plan_query(self.ptr, key.encode(), node, None, 0, C.byref(n)))
        buf = (C.c_int64 * max(n.value, 1))()
        _check(lib().hss_plan_query(self.ptr, key.encode(), node, buf, n.value, C.byref(n)))
        return np.frombuffer(buf, dtype=np.int64, count=n.value).copy()

    def close(self):
        if self.ptr:
            lib().hss_plan_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_forward(w, x, stream=None):
    import torch
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    _check(lib().hss_mlp_forward(w.data_ptr(), x.contiguous().data_ptr(), x.shape[0], y.data_ptr(),
                                 _stream_ptr(stream)))
    return y


def mlp_grad(w, x, t, stream=None):
    import torch
    g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=x.device)
    loss = C.c_double(0)
    _check(lib().hss_mlp_grad(w.data_ptr(), x.contiguous().data_ptr(), t.contiguous().data_ptr(), x.shape[0],
                              g.data_ptr(), C.byref(loss), _stream_ptr(stream)))
    return g, loss.value


def rank_model_train(features, ranks, out_path, seed=0):
    """hss_rank_model_train: train on host (features [n, 8], ranks [n]) and write the
    weights file that factor(..., rank_model_path=...) reads."""
    f = np.ascontiguousarray(features, dtype=np.float32)
    r = np.ascontiguousarray(ranks, dtype=np.float32)
    if f.ndim != 2 or f.shape[1] != 8 or r.shape != (f.shape[0],):
        raise ValueError("features must be [n, 8] and ranks [n]")
    _check(lib().hss_rank_model_train(f.ctypes.data, r.ctypes.data, f.shape[0], os.fsencode(out_path),
                                      C.c_uint64(seed)))


MLP_NOALLOC_MAX_N = 8192


def mlp_grad_noalloc(w, x, t, grad, stream=None):
    """hss_mlp_grad_noalloc: the gradient into the caller's tensor ``grad``
    (MLP_NPARAMS floats on the device); the library allocates nothing. Returns the loss."""
    loss = C.c_double(0)
    _check(lib().hss_mlp_grad_noalloc(w.data_ptr(), x.contiguous().data_ptr(), t.contiguous().data_ptr(),
                                      x.shape[0], grad.data_ptr(), C.byref(loss), _stream_ptr(stream)))
    return loss.value


def mlp_train(w, x, t, steps, lr=1e-2, stream=None):
    import torch
    hist = torch.empty(max(steps, 1), dtype=torch.float32, device=x.device)
    _check(lib().hss_mlp_train(w.data_ptr(), x.contiguous().data_ptr(), t.contiguous().data_ptr(), x.shape[0],
                               steps, lr, hist.data_ptr(), _stream_ptr(stream)))
    return hist[:steps]


# ---- kernel-level diagnostics (include/hss_debug.h) ----
_SCALAR = {"float32": 0, "float64": 1, "complex64": 2, "complex128": 3}


def _scalar_code(t):
    return _SCALAR[str(t.dtype).replace("torch.", "")]


def debug_gemm(As, Bs, Cs, alpha=1.0, beta=0.0, stream=None, bf16x3=False, big=False):
    """C_b = alpha A_b B_b + beta C_b in place (column-major views of CUDA tensors:
    pass tensors shaped [cols, rows] in row-major storage, i.e. X.T of the matrix).
    bf16x3: float32 or complex64 operands on the BF16 matrix cores (hi / lo split, three
    products per real product). big: float32 operands on the 128 x 128-tile kernel."""
    L = lib()
    L.hss_debug_gemm.restype = C.c_int
    n = len(As)
    P = C.c_void_p * n
    I = C.c_int32 * n
    code = _scalar_code(As[0])
    if bf16x3:
        if code not in (0, 2):
            raise ValueError("bf16x3 takes float32 or complex64 operands")
        code = 4 if code == 0 else 5
    elif big:
        if code != 0:
            raise ValueError("big tiles take float32 operands")
        code = 6
    M = I(*[c.shape[1] for c in Cs])
    N = I(*[c.shape[0] for c in Cs])
    K = I(*[a.shape[0] for a in As])
    al = (C.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (C.c_double * 2)(complex(beta).real, complex(beta).imag)
    _check(L.hss_debug_gemm(code, n, P(*[a.data_ptr() for a in As]), P(*[b.data_ptr() for b in Bs]),
                            P(*[c.data_ptr() for c in Cs]), M, N, K, I(*[a.shape[1] for a in As]),
                            I(*[b.shape[1] for b in Bs]), I(*[c.shape[1] for c in Cs]), al, be,
                            C.c_void_p(_stream_ptr(stream))))


def debug_gj(mats, ns, ms, block=0, stream=None):
    """In-place blocked Gauss-Jordan on column-major [A | B] blocks (tensors shaped
    [n + m, n] row-major = the transposed view). block > 0 forces second-level
    blocks of that many pivot columns. Returns the singular flag."""
    L = lib()
    L.hss_debug_gj.restype = C.c_int
    k = len(mats)
    sing = C.c_int32(0)
    _check(L.hss_debug_gj(_scalar_code(mats[0]), k, (C.c_void_p * k)(*[m.data_ptr() for m in mats]),
                          (C.c_int32 * k)(*ns), (C.c_int32 * k)(*ms), int(block), C.byref(sing),
                          C.c_void_p(_stream_ptr(stream))))
    return sing.value


def debug_row_id(Z, thresh, p_os=10, stream=None):
    """Row ID of a CUDA tensor Z (m x l, row-major) as the compression computes it
    for one HSS node. Returns (k, skeleton indices, U (m x k, numpy), max |T|)."""
    import torch
    L = lib()
    L.hss_debug_row_id.restype = C.c_int
    m, l = Z.shape
    Zc = Z.contiguous()
    kc = min(l, m)
    U = torch.empty((kc, m), dtype=Z.dtype, device=Z.device)  # column-major m x kc
    k = C.c_int32(0)
    skel = (C.c_int32 * m)()
    tm = C.c_float(0)
    _check(L.hss_debug_row_id(_scalar_code(Z), C.c_void_p(Zc.data_ptr()), m, l, C.c_double(thresh), p_os,
                              C.byref(k), skel, C.c_void_p(U.data_ptr()), C.byref(tm),
                              C.c_void_p(_stream_ptr(stream))))
    kk = k.value
    return kk, np.array(skel[:kk], dtype=np.int64), U.cpu().numpy().T[:, :kk], tm.value


SCALAR_CODE = {"float32": 0, "float64": 1, "complex64": 2, "complex128": 3}


def tuning_load(path):
    """hss_tuning_load: read an autotuner JSON file into the process-wide table."""
    _check(lib().hss_tuning_load(os.fsencode(path)))


def tuning_set(scalar, rows_class, nb=0, rpt=0, nt=0, block=-1):
    """hss_tuning_set: one entry of the table (scalar: a SCALAR_CODE key)."""
    _check(lib().hss_tuning_set(SCALAR_CODE[scalar], rows_class, nb, rpt, nt, block))


def tuning_clear():
    lib().hss_tuning_clear()


def tuning_candidates(scalar, rows):
    """Compiled compact panel shapes (nb, rpt, nt) that hold `rows` rows."""
    n = C.c_int32(0)
    _check(lib().hss_tuning_candidates(SCALAR_CODE[scalar], rows, None, 0, C.byref(n)))
    buf = (C.c_int32 * max(3 * n.value, 1))()
    _check(lib().hss_tuning_candidates(SCALAR_CODE[scalar], rows, buf, n.value, C.byref(n)))
    return [tuple(buf[3 * i:3 * i + 3]) for i in range(n.value)]

