"""Argument marshalling between torch/numpy and the C ABI of libfracctl.

Device buffers are torch CUDA (HIP) tensors; their data pointers are handed to
the library as-is.  Every step of the method runs in the library."""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np

from ._lib import Info, SetupParams, check, lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    return int(stream.cuda_stream)


def _host_array(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


class Plan:
    """One setup (fc_setup_ex): spectra, operator and preconditioner factors,
    workspace.  Release with close() (also on garbage collection)."""

    def __init__(self, n: int, a: Sequence[np.ndarray], alpha: float, beta: float,
                 gamma: float = 1.0, eps: float = 1e-6, tol: float = 0.0,
                 op_accuracy: float = 0.0, max_iter: int = 0, max_rank: int = 0,
                 precond_rank: int = 0, precision: int = 0, stream=None, precond: int = 0,
                 precond_b0: Optional[Sequence[float]] = None, dims: int = 3):
        if dims not in (2, 3):
            raise ValueError("dims must be 2 or 3")
        self._a = [_host_array(x) for x in a[:dims]]
        if len(self._a) != dims:
            raise ValueError(f"need {dims} coefficient arrays")
        for x in self._a:
            if x.shape != (n + 1,):
                raise ValueError("each coefficient needs n+1 midpoint samples")
        p = SetupParams()
        p.n = n
        for l in range(dims):
            p.a[l] = self._a[l].ctypes.data_as(C.POINTER(C.c_double))
        p.dims = dims
        p.alpha, p.beta, p.gamma, p.eps, p.tol = alpha, beta, gamma, eps, tol
        p.op_accuracy = op_accuracy
        p.max_iter, p.max_rank, p.precond_rank, p.precision = (max_iter, max_rank, precond_rank,
                                                                precision)
        p.precond = precond
        if precond_b0 is not None:
            for l in range(3):
                p.precond_b0[l] = float(precond_b0[l])
        h = C.c_void_p()
        check(lib().fc_setup_ex(C.byref(p), _stream_ptr(stream), C.byref(h)), "fc_setup_ex")
        self.handle = h
        self.n = n
        self.alpha, self.beta, self.gamma, self.eps = alpha, beta, gamma, eps

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().fc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- introspection -------------------------------------------------
    def spectrum(self, with_vectors: bool = False):
        n = self.n
        lam = np.zeros(3 * n)
        V = np.zeros(3 * n * n) if with_vectors else None
        check(lib().fc_plan_spectrum(self.handle, lam.ctypes.data_as(C.POINTER(C.c_double)),
                                     V.ctypes.data_as(C.POINTER(C.c_double)) if V is not None else None),
              "fc_plan_spectrum")
        lam = lam.reshape(3, n)
        if V is None:
            return lam
        return lam, [V[l * n * n:(l + 1) * n * n].reshape(n, n, order="F") for l in range(3)]

    def separable(self, which: int):
        rank = C.c_int()
        lib().fc_plan_separable(self.handle, which, 0, C.byref(rank), None, None)
        cap = rank.value
        n = self.n
        w = np.zeros(cap)
        F = np.zeros(3 * n * cap)
        check(lib().fc_plan_separable(self.handle, which, cap, C.byref(rank),
                                      w.ctypes.data_as(C.POINTER(C.c_double)),
                                      F.ctypes.data_as(C.POINTER(C.c_double))), "fc_plan_separable")
        return w, [F[l * n * cap:(l + 1) * n * cap].reshape(n, cap, order="F") for l in range(3)]

    def tuning(self):
        """The autotuner's choices for this plan and the measured candidate
        times (fc_plan_tuning)."""
        ch = (C.c_int * 6)()
        us = (C.c_double * 10)()
        check(lib().fc_plan_tuning(self.handle, ch, us), "fc_plan_tuning")
        names = ("gram_batched_waves", "gram_single_waves", "kron_waves", "stream_kc", "panel_b")
        out = {k: ch[i] for i, k in enumerate(names)}
        out["tuned"] = bool(ch[5])
        out["candidate_us"] = [us[i] for i in range(10)]
        return out

    # ---- solve -----------------------------------------------------------
    def solve(self, w_y, Y: Sequence, cap_u: int = 4096, stream=None, out=None):
        """Y: three (n, rank) column-major device tensors (float64), i.e.
        tensors whose transpose is contiguous.  Returns (w_u, [U1, U2, U3], info)."""
        import torch
        n = self.n
        Yc = [_colmajor(y) for y in Y]
        rank_y = Yc[0].shape[1]
        dev = Yc[0].device
        if out is None:
            w_u = torch.empty(cap_u, dtype=torch.float64, device=dev)
            U = [torch.empty((cap_u, n), dtype=torch.float64, device=dev).t() for _ in range(3)]
        else:
            w_u, U = out
        info = Info()
        rank_u = C.c_int()
        st = lib().fc_solve(self.handle, rank_y, _ptr(w_y), _ptr(Yc[0]), _ptr(Yc[1]), _ptr(Yc[2]),
                            cap_u, C.byref(rank_u), _ptr(w_u), _ptr(U[0]), _ptr(U[1]), _ptr(U[2]),
                            C.byref(info), _stream_ptr(stream))
        check(st, "fc_solve")
        k = rank_u.value
        return w_u[:k], [u[:, :k] for u in U], info.as_dict()

    def solve2d(self, w_y, Y: Sequence, cap_u: int = 256, stream=None):
        """fc_solve2d on a dims=2 plan.  Y: two (n, rank) column-major device
        tensors.  Returns (w_u, [U1, U2], info)."""
        import torch
        n = self.n
        Yc = [_colmajor(y) for y in Y]
        dev = Yc[0].device
        w_u = torch.empty(cap_u, dtype=torch.float64, device=dev)
        U = [torch.empty((cap_u, n), dtype=torch.float64, device=dev).t() for _ in range(2)]
        info = Info()
        rank_u = C.c_int()
        st = lib().fc_solve2d(self.handle, Yc[0].shape[1], _ptr(w_y), _ptr(Yc[0]), _ptr(Yc[1]),
                              cap_u, C.byref(rank_u), _ptr(w_u), _ptr(U[0]), _ptr(U[1]),
                              C.byref(info), _stream_ptr(stream))
        check(st, "fc_solve2d")
        k = rank_u.value
        return w_u[:k], [u[:, :k] for u in U], info.as_dict()

    def solve_state(self, w_y, Y: Sequence, cap_u: int = 4096, cap_s: int = 4096, stream=None):
        """fc_solve_state: the control u, the state y = beta A^-alpha u and the
        cost J.  Returns (w_u, [U1, U2, U3], w_s, [S1, S2, S3], J, info)."""
        import torch
        n = self.n
        Yc = [_colmajor(y) for y in Y]
        dev = Yc[0].device
        w_u = torch.empty(cap_u, dtype=torch.float64, device=dev)
        U = [torch.empty((cap_u, n), dtype=torch.float64, device=dev).t() for _ in range(3)]
        w_s = torch.empty(cap_s, dtype=torch.float64, device=dev)
        S = [torch.empty((cap_s, n), dtype=torch.float64, device=dev).t() for _ in range(3)]
        info = Info()
        rank_u, rank_s, J = C.c_int(), C.c_int(), C.c_double()
        st = lib().fc_solve_state(self.handle, Yc[0].shape[1], _ptr(w_y), *[_ptr(y) for y in Yc],
                                  cap_u, C.byref(rank_u), _ptr(w_u), *[_ptr(u) for u in U],
                                  cap_s, C.byref(rank_s), _ptr(w_s), *[_ptr(x) for x in S],
                                  C.byref(J), C.byref(info), _stream_ptr(stream))
        check(st, "fc_solve_state")
        k, ks = rank_u.value, rank_s.value
        return (w_u[:k], [u[:, :k] for u in U], w_s[:ks], [x[:, :ks] for x in S], J.value,
                info.as_dict())

    def mode_transform(self, mode: int, transpose: bool, X, stream=None):
        import torch
        Xc = _colmajor(X)
        out = torch.empty((Xc.shape[1], self.n), dtype=torch.float64, device=Xc.device).t()
        check(lib().fc_mode_transform(self.handle, mode, int(transpose), Xc.shape[1], _ptr(Xc),
                                      _ptr(out), _stream_ptr(stream)), "fc_mode_transform")
        return out

    def cp_inner(self, wa, A, wb, B, stream=None) -> float:
        Ac = [_colmajor(x) for x in A]
        Bc = [_colmajor(x) for x in B]
        out = C.c_double()
        check(lib().fc_cp_inner(self.handle, Ac[0].shape[1], _ptr(wa), *[_ptr(x) for x in Ac],
                                Bc[0].shape[1], _ptr(wb), *[_ptr(x) for x in Bc], C.byref(out),
                                _stream_ptr(stream)), "fc_cp_inner")
        return out.value

    def _canon_call(self, fn, name, pre, w, X, eps, cap, stream):
        import torch
        Xc = [_colmajor(x) for x in X]
        dev = Xc[0].device
        w_o = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        O = [torch.empty((max(cap, 1), self.n), dtype=torch.float64, device=dev).t() for _ in range(3)]
        rank = C.c_int()
        check(fn(self.handle, *pre, Xc[0].shape[1], _ptr(w), *[_ptr(x) for x in Xc], eps, cap,
                 C.byref(rank), _ptr(w_o), *[_ptr(o) for o in O], _stream_ptr(stream)), name)
        k = rank.value
        return w_o[:k], [o[:, :k] for o in O]

    def cp_truncate(self, w, X, eps, cap=4096, stream=None):
        return self._canon_call(lib().fc_cp_truncate, "fc_cp_truncate", (), w, X, eps, cap, stream)

    def apply_separable(self, which, w, X, eps, cap=4096, stream=None):
        return self._canon_call(lib().fc_apply_separable, "fc_apply_separable", (which,), w, X, eps,
                                cap, stream)


def solve_batched(plans: Sequence["Plan"], problems: Sequence, cap_u: int = 4096, stream=None,
                  outs=None, raise_on_error: bool = True):
    """Concurrent solves (fc_solve_batched): problems[i] = (w_y, [Y1, Y2, Y3]) on
    plans[i] ([Y1, Y2] for a dims=2 plan).  Returns a list of
    (w_u, [U1, U2, U3] or [U1, U2], info, status)."""
    import torch
    from ._lib import Info, STATUS
    count = len(plans)
    VP = C.c_void_p
    arr = lambda xs: (VP * count)(*xs)
    Ys = [[_colmajor(y) for y in p[1]] for p in problems]
    if outs is None:
        outs = []
        for i in range(count):
            dev = Ys[i][0].device
            n = plans[i].n
            outs.append((torch.empty(cap_u, dtype=torch.float64, device=dev),
                         [torch.empty((cap_u, n), dtype=torch.float64, device=dev).t()
                          for _ in range(len(Ys[i]))]))
    rank_y = (C.c_int * count)(*[Ys[i][0].shape[1] for i in range(count)])
    capa = (C.c_int * count)(*[outs[i][0].shape[0] for i in range(count)])
    rank_u = (C.c_int * count)()
    status = (C.c_int * count)()
    infos = (Info * count)()
    st = lib().fc_solve_batched(
        count, arr([p.handle.value for p in plans]), rank_y,
        arr([_ptr(p[0]) for p in problems]),
        arr([_ptr(Ys[i][0]) for i in range(count)]), arr([_ptr(Ys[i][1]) for i in range(count)]),
        arr([_ptr(Ys[i][2]) if len(Ys[i]) > 2 else None for i in range(count)]), capa, rank_u,
        arr([_ptr(o[0]) for o in outs]), arr([_ptr(o[1][0]) for o in outs]),
        arr([_ptr(o[1][1]) for o in outs]),
        arr([_ptr(o[1][2]) if len(o[1]) > 2 else None for o in outs]),
        status, infos, _stream_ptr(stream))
    res = []
    for i in range(count):
        k = rank_u[i]
        w_u, U = outs[i]
        res.append((w_u[:k], [u[:, :k] for u in U], infos[i].as_dict(), STATUS.get(status[i])))
    if st != 0 and raise_on_error:
        check(st, "fc_solve_batched")
    return res


def _colmajor(t):
    """A (rows, cols) tensor laid out column-major (its transpose contiguous)."""
    if t.dim() != 2:
        raise ValueError("factor matrices must be 2-D")
    if t.t().is_contiguous():
        return t
    return t.t().contiguous().t()


def to_device_colmajor(M: np.ndarray, device="cuda"):
    import torch
    A = np.asfortranarray(np.asarray(M, dtype=np.float64))
    return torch.from_numpy(np.ascontiguousarray(A.T)).to(device).t()


def host_fd_eigen(a_mid: np.ndarray, vectors: bool = True):
    a = _host_array(a_mid)
    n = a.shape[0] - 1
    lam = np.zeros(n)
    V = np.zeros(n * n) if vectors else None
    check(lib().fc_host_fd_eigen(n, a.ctypes.data_as(C.POINTER(C.c_double)),
                                 lam.ctypes.data_as(C.POINTER(C.c_double)),
                                 V.ctypes.data_as(C.POINTER(C.c_double)) if vectors else None),
          "fc_host_fd_eigen")
    return lam, (V.reshape(n, n, order="F") if vectors else None)


def host_expsum(kind: int, p1: float, p2: float, p3: float, s_min: float, s_max: float,
                terms: int):
    t = np.zeros(terms)
    c = np.zeros(terms)
    e = C.c_double()
    check(lib().fc_host_expsum(kind, p1, p2, p3, s_min, s_max, terms,
                               t.ctypes.data_as(C.POINTER(C.c_double)),
                               c.ctypes.data_as(C.POINTER(C.c_double)), C.byref(e)),
          "fc_host_expsum")
    return t, c, e.value
