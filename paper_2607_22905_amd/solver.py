"""Python binding of the AlgMortar-PCG library: argument marshalling only.

Every step of the method runs in the HIP library (libalgmortar.so); torch is
used for device memory and the current stream.  Device vectors are float64
CUDA tensors in original ordering: shape ``(n,)`` for one right-hand side or
``(k, n)`` for ``k`` right-hand sides (row c = column c of the C-ABI's
column-major block, leading dimension n).
"""
import ctypes
from ctypes import byref, c_int32, c_int64, c_void_p

import numpy as np

from . import _lib
from ._lib import AmCsr, AmFaces, AmInfo, AmOptions, check, load

__all__ = ["AlgMortar", "Tpfa", "partition_blocks", "partition_bisect", "structure", "interface_nd",
           "structure_sizes"]


def _np(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a):
    return c_void_p(a.ctypes.data) if a is not None else c_void_p(0)


def _csr(A):
    """Build an am_csr for an object with n, row_ptr, col, val (host arrays, or
    a float64 CUDA tensor for val).  Returns (struct, keep-alive tuple)."""
    rp = _np(A.row_ptr, np.int64)
    ci = _np(A.col, np.int32)
    val = A.val
    on_dev = 0
    if hasattr(val, "is_cuda") and val.is_cuda:
        import torch
        assert val.dtype == torch.float64 and val.is_contiguous()
        vptr = c_void_p(val.data_ptr())
        keep = (rp, ci, val)
        on_dev = 1
    else:
        v = _np(val, np.float64)
        vptr = _ptr(v)
        keep = (rp, ci, v)
    s = AmCsr(n=int(A.n), nnz=int(rp[-1]), row_ptr=_ptr(rp), col_idx=_ptr(ci), val=vptr,
              values_on_device=on_dev)
    return s, keep


def partition_blocks(dims, block):
    nx, ny, nz = dims
    bx, by, bz = block
    part = np.empty(nx * ny * nz, dtype=np.int32)
    m = c_int32()
    check(load().am_partition_blocks(nx, ny, nz, bx, by, bz, _ptr(part), byref(m)))
    return part, m.value


def partition_bisect(A, lo=200, hi=800, seed=0):
    s, keep = _csr(A)
    part = np.empty(int(A.n), dtype=np.int32)
    m = c_int32()
    check(load().am_partition_bisect(byref(s), lo, hi, seed, _ptr(part), byref(m)))
    return part, m.value


def structure_sizes(A, part, nparts, mortar="interface"):
    s, keep = _csr(A)
    p = _np(part, np.int32)
    nl, ne = c_int64(), c_int64()
    check(load().am_structure_sizes(byref(s), _ptr(p), nparts, _lib.MORTAR[mortar], byref(nl), byref(ne)))
    return nl.value, ne.value


def interface_nd(A, part, nparts, max_nrhs=1):
    """Host-only nested-dissection order of the interface system:
    (order, blk_off, ntop) -- ND position -> basis function, the block
    boundaries, the number of separator rows last in the order."""
    NL, _ = structure_sizes(A, part, nparts)
    s, keep = _csr(A)
    p = _np(part, np.int32)
    order = np.empty(NL, dtype=np.int32)
    blk = np.empty(NL + 1, dtype=np.int64)
    nb, nt = c_int32(), c_int64()
    check(load().am_interface_nd(byref(s), _ptr(p), int(nparts), int(max_nrhs), _ptr(order),
                                 _ptr(blk), byref(nb), byref(nt)))
    return order, blk[:nb.value + 1].copy(), nt.value


def structure(A, part, nparts, mortar="interface"):
    """Host-only interface structure (perm, sub_ptr, iface_ptr, iface_ij, edge_k, edge_l)."""
    NL, NE = structure_sizes(A, part, nparts, mortar)
    s, keep = _csr(A)
    p = _np(part, np.int32)
    n = int(A.n)
    out = dict(perm=np.empty(n, np.int32), sub_ptr=np.empty(nparts + 1, np.int64),
               iface_ptr=np.empty(NL + 1, np.int64), iface_ij=np.empty((NL, 2), np.int32),
               edge_k=np.empty(NE, np.int32), edge_l=np.empty(NE, np.int32))
    check(load().am_structure(byref(s), _ptr(p), nparts, _lib.MORTAR[mortar], _ptr(out["perm"]),
                              _ptr(out["sub_ptr"]), _ptr(out["iface_ptr"]), _ptr(out["iface_ij"]),
                              _ptr(out["edge_k"]), _ptr(out["edge_l"])))
    return out


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def _vec(x, n):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64):
        raise TypeError("expected a float64 CUDA tensor")
    if not x.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if x.dim() == 1:
        if x.shape[0] != n:
            raise ValueError("length mismatch")
        return 1
    if x.dim() == 2 and x.shape[1] == n:
        return x.shape[0]
    raise ValueError("expected shape (n,) or (k, n)")


class AlgMortar:
    """Handle of a set-up AlgMortar preconditioner (Algorithm 1) on one GPU."""

    def __init__(self, A, part, nparts, prec="fp64", mortar="interface", max_nrhs=1, device=0,
                 graph=True, stream=None, separate_iface=False, dense_iface=False,
                 inexact_iface=False, bf16_products=False):
        lib = load()
        s, keep = _csr(A)
        p = _np(part, np.int32)
        opt = AmOptions(local_prec=_lib.PREC[prec], mortar=_lib.MORTAR[mortar],
                        max_nrhs=int(max_nrhs), device=int(device),
                        flags=(0 if graph else _lib.AM_FLAG_NO_GRAPH)
                        | (_lib.AM_FLAG_SEPARATE_IFACE if separate_iface else 0)
                        | (_lib.AM_FLAG_DENSE_IFACE if dense_iface else 0)
                        | (_lib.AM_FLAG_INEXACT_IFACE if inexact_iface else 0)
                        | (_lib.AM_FLAG_BF16_PRODUCTS if bf16_products else 0))
        h = c_void_p()
        st = c_void_p(0) if stream is False else _stream(stream)
        check(lib.algmortar_setup(byref(s), _ptr(p), int(nparts), byref(opt), st, byref(h)))
        self._h = h
        self.n = int(A.n)
        self.nparts = int(nparts)
        self.prec = prec
        n, m, nl, ne = c_int64(), c_int64(), c_int64(), c_int64()
        check(lib.algmortar_sizes(h, byref(n), byref(m), byref(nl), byref(ne)), h)
        self.n_iface, self.n_edges = nl.value, ne.value

    def close(self):
        if getattr(self, "_h", None):
            load().algmortar_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_values(self, A, stream=None):
        """New values for the matrix (same pattern as at set-up; ``A.val`` on
        the host or a float64 CUDA tensor): Algorithm 1's numeric part is
        redone, the structure and layout are kept."""
        s, keep = _csr(A)
        check(load().algmortar_update_values(self._h, byref(s), _stream(stream)), self._h)

    def set_smoother(self, blocks, nblocks, steps, stream=None):
        """Block-Jacobi pre/post smoothing (Sec. 5.4) on the blocks of the
        host partition ``blocks`` (int32[n]), ``steps`` before and after the
        correction; steps = 0 removes it."""
        b = _np(blocks, np.int32)
        if b.shape != (self.n,):
            raise ValueError("blocks must have one entry per unknown")
        check(load().algmortar_set_smoother(self._h, _ptr(b), int(nblocks), int(steps),
                                            _stream(stream)), self._h)
        self.smooth_steps = int(steps)

    def apply(self, r, out=None, stream=None):
        """z = Mcal^{-1} r (Algorithm 2), smoothed when a smoother is set."""
        import torch
        k = _vec(r, self.n)
        z = torch.empty_like(r) if out is None else out
        check(load().algmortar_apply(self._h, c_void_p(r.data_ptr()), c_void_p(z.data_ptr()), k,
                                     self.n, _stream(stream)), self._h)
        return z

    def set_inexact(self, rtol=1e-2, maxit=50):
        """Tolerance and iteration cap of the inexact interface solve (handles
        set up with inexact_iface=True)."""
        check(load().algmortar_set_inexact(self._h, float(rtol), int(maxit)), self._h)

    def apply_static(self, r, out=None, stream=None):
        """The allocation-free form of ``apply``: the same result, with the
        library's work buffers in its static device scratch."""
        import torch
        k = _vec(r, self.n)
        z = torch.empty_like(r) if out is None else out
        check(load().algmortar_apply_static(self._h, c_void_p(r.data_ptr()), c_void_p(z.data_ptr()),
                                            k, self.n, _stream(stream)), self._h)
        return z

    def local_solve(self, r, stream=None):
        import torch
        _vec(r, self.n)
        z = torch.empty_like(r)
        check(load().algmortar_local_solve(self._h, c_void_p(r.data_ptr()), c_void_p(z.data_ptr()),
                                           _stream(stream)), self._h)
        return z

    def pcg(self, b, tol, maxit=10000, out=None, stream=None, raise_on_error=True):
        """Solve A x = b (x0 = 0); returns (x, [info dict per column], status)."""
        import torch
        k = _vec(b, self.n)
        x = torch.empty_like(b) if out is None else out
        infos = (AmInfo * k)()
        status = load().algmortar_pcg(self._h, c_void_p(b.data_ptr()), c_void_p(x.data_ptr()), k,
                                      self.n, float(tol), int(maxit), ctypes.cast(infos, c_void_p),
                                      _stream(stream))
        if raise_on_error:
            check(status, self._h)
        return x, [infos[i].as_dict() for i in range(k)], status

    def pcg_profile(self, b, tol, maxit=10000, out=None):
        """PCG with plain launches, each timed with HIP events.  Returns
        (x, info dicts, {kernel: (summed ms, launches)})."""
        import torch
        k = _vec(b, self.n)
        x = torch.empty_like(b) if out is None else out
        infos = (AmInfo * k)()
        ms = (ctypes.c_double * 5)()
        cnt = (c_int64 * 5)()
        torch.cuda.synchronize()
        check(load().algmortar_pcg_profile(self._h, c_void_p(b.data_ptr()), c_void_p(x.data_ptr()), k,
                                           self.n, float(tol), int(maxit), ctypes.cast(infos, c_void_p),
                                           ms, cnt, c_void_p(0)), self._h)
        names = {0: "local", 1: "gemv", 3: "spmv", 4: "update"}
        return x, [infos[i].as_dict() for i in range(k)], {v: (ms[i], cnt[i]) for i, v in names.items()}

    def tile_choice(self, nrhs=1):
        """(chosen candidate, [average launch us of each candidate]) of the
        local kernel's wave layout for nrhs right-hand sides (autotuned)."""
        ch, nc = c_int32(), c_int32()
        us = (ctypes.c_double * 4)()
        check(load().algmortar_tile_choice(self._h, int(nrhs), byref(ch), byref(nc), us), self._h)
        return ch.value, [us[i] for i in range(nc.value)]

    def time_kernel(self, kernel, nrhs=1, reps=20):
        """(average launch ms, algorithmic bytes per launch) of an apply kernel:
        "local" (band sweeps + reconstruction), "gemv", "bpart"."""
        kid = {"local": 0, "gemv": 1, "bpart": 2, "spmv": 3, "update": 4, "smooth_block": 5}[kernel]
        ms, by = ctypes.c_double(), ctypes.c_double()
        check(load().algmortar_time_kernel(self._h, kid, int(nrhs), int(reps), byref(ms), byref(by)), self._h)
        return ms.value, by.value

    def interfaces(self):
        out = dict(perm=np.empty(self.n, np.int32), sub_ptr=np.empty(self.nparts + 1, np.int64),
                   iface_ptr=np.empty(self.n_iface + 1, np.int64),
                   iface_ij=np.empty((self.n_iface, 2), np.int32),
                   edge_k=np.empty(self.n_edges, np.int32), edge_l=np.empty(self.n_edges, np.int32))
        check(load().algmortar_interfaces(self._h, _ptr(out["perm"]), _ptr(out["sub_ptr"]),
                                          _ptr(out["iface_ptr"]), _ptr(out["iface_ij"]),
                                          _ptr(out["edge_k"]), _ptr(out["edge_l"])), self._h)
        return out

    def export_interface(self, which="S"):
        out = np.empty((self.n_iface, self.n_iface), np.float64)
        check(load().algmortar_export_interface(self._h, 0 if which == "S" else 1, _ptr(out)), self._h)
        return out

    def export_mbf(self, iface, sub, size):
        out = np.empty(size, np.float64)
        check(load().algmortar_export_mbf(self._h, int(iface), int(sub), _ptr(out)), self._h)
        return out


class Tpfa:
    """Device TPFA assembler for a face list (differentiation form)."""

    def __init__(self, faces, n, device=0):
        lib = load()
        self._keep = [_np(faces.k, np.int64), _np(faces.l, np.int64), _np(faces.gk, np.float64),
                      _np(faces.gl, np.float64), _np(faces.pD, np.float64)]
        k, l, gk, gl, pD = self._keep
        f = AmFaces(n_faces=k.size, k=_ptr(k), l=_ptr(l), gk=_ptr(gk), gl=_ptr(gl), pD=_ptr(pD))
        t = c_void_p()
        nnz = c_int64()
        check(lib.am_tpfa_create(byref(f), int(n), int(device), byref(t), byref(nnz)))
        self._t = t
        self.n = int(n)
        self.nnz = nnz.value
        self.row_ptr = np.empty(self.n + 1, np.int64)
        self.col = np.empty(self.nnz, np.int32)
        check(lib.am_tpfa_pattern(t, _ptr(self.row_ptr), _ptr(self.col)))

    def close(self):
        if getattr(self, "_t", None):
            load().am_tpfa_destroy(self._t)
            self._t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def assemble(self, logK, stream=None):
        """(val, f) on the device for log-permeability ``logK`` (float64 CUDA)."""
        import torch
        _vec(logK, self.n)
        val = torch.empty(self.nnz, dtype=torch.float64, device=logK.device)
        f = torch.empty(self.n, dtype=torch.float64, device=logK.device)
        check(load().am_tpfa_assemble(self._t, c_void_p(logK.data_ptr()), c_void_p(val.data_ptr()),
                                      c_void_p(f.data_ptr()), _stream(stream)))
        return val, f

    def face_grad(self, logK, p, lam, stream=None):
        import torch
        g = torch.empty_like(p)
        check(load().am_tpfa_face_grad(self._t, c_void_p(logK.data_ptr()), c_void_p(p.data_ptr()),
                                       c_void_p(lam.data_ptr()), c_void_p(g.data_ptr()), _stream(stream)))
        return g

    class _Mat:
        def __init__(self, n, rp, ci, val):
            self.n, self.row_ptr, self.col, self.val = n, rp, ci, val

    def matrix(self, val):
        return Tpfa._Mat(self.n, self.row_ptr, self.col, val)


def adjoint_grad(handle, tpfa, logK, p, dJdp, tol=1e-12, maxit=10000, stream=None):
    """(grad, lambda, info) of J through A(logK) p = f (adjoint PCG + face scatter)."""
    import torch
    lam = torch.empty_like(p)
    grad = torch.empty_like(p)
    info = AmInfo()
    check(load().algmortar_adjoint_grad(handle._h, tpfa._t, c_void_p(logK.data_ptr()),
                                        c_void_p(p.data_ptr()), c_void_p(dJdp.data_ptr()), float(tol),
                                        int(maxit), c_void_p(lam.data_ptr()), c_void_p(grad.data_ptr()),
                                        byref(info), _stream(stream)), handle._h)
    return grad, lam, info.as_dict()
