"""Python binding of libdp (distance-preconditioned Wilson-clover inversion on
MI355X).  Argument marshalling only: every step of the computation runs in
the HIP kernels of ``libdp.so``.  Host arrays are numpy complex128 in the
layouts of ``include/dp.h``; device arrays are torch CUDA (HIP) tensors of
complex128 (or float64 with a trailing 2) in the same layout.
"""
import ctypes

import numpy as np

from . import _lib as L
from ._lib import DPError  # noqa: F401

__all__ = ["Lattice", "Batch", "DPError", "footprint_bytes"]


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def footprint_bytes(dims, nrhs, precision="f64", new_masses=1):
    d = (ctypes.c_int * 4)(*dims)
    return int(L.lib().dp_footprint_bytes(d, int(nrhs), L.DP_PREC[precision], int(new_masses)))


class Lattice:
    """One lattice with a resident gauge field on one GPU (a dp_ctx)."""

    def __init__(self, dims, bc_t=-1, device=0):
        self.dims = tuple(int(d) for d in dims)
        self.T = self.dims[0]
        self.V = int(np.prod(self.dims))
        self._L = L.lib()
        h = ctypes.c_void_p()
        rc = self._L.dp_create((ctypes.c_int * 4)(*self.dims), int(bc_t), int(device), ctypes.byref(h))
        if rc != L.DP_OK:
            raise DPError(rc, "dp_create failed")
        self._h = h

    # ------------------------------------------------------------ plumbing
    def _check(self, rc, allow=()):
        if rc != L.DP_OK and rc not in allow:
            raise DPError(rc, self._L.dp_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            self._L.dp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ state
    def set_gauge(self, U):
        if hasattr(U, "is_cuda") and U.is_cuda:
            import torch
            stream = torch.cuda.current_stream(U.device).cuda_stream
            self._check(self._L.dp_set_gauge_dev(self._h, ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(stream)))
            return
        U = _c128(U)
        assert U.size == self.V * 36, "gauge field must have T*L1*L2*L3*4*9 entries"
        self._check(self._L.dp_set_gauge(self._h, _ptr(U)))

    def set_gauge_sf(self, U_ext, ct_tilde=1.0):
        """Schroedinger-functional links: U_ext of shape (T+2, L1, L2, L3, 4, 3, 3),
        the boundary timeslices first and last (ctx created with bc_t = 0)."""
        U_ext = _c128(U_ext)
        assert U_ext.size == (self.T + 2) * (self.V // self.T) * 36
        self._check(self._L.dp_set_gauge_sf(self._h, _ptr(U_ext), float(ct_tilde)))

    def sf_wall_sources(self, c0=0, ncols=12, out=None, side=0):
        """The boundary sources of the x0 = 0 boundary (side 0: U_0(0, xs)^+ P+ e_c
        on the first interior timeslice) or the x0 = T + 1 one (side 1:
        U_0(T, xs) P- e_c on the last), as a complex128 CUDA tensor [ncols, V*12]."""
        import torch
        if out is None:
            out = torch.empty((ncols, self.V * 12), dtype=torch.complex128, device="cuda")
        assert out.is_cuda and out.is_contiguous() and out.numel() == ncols * self.V * 12
        stream = torch.cuda.current_stream(out.device).cuda_stream
        self._check(self._L.dp_sf_wall_sources(self._h, int(side), int(c0), int(ncols),
                                               ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)))
        return out

    def set_clover(self, csw):
        self._check(self._L.dp_set_clover(self._h, float(csw)))

    def set_clover_field(self, C):
        C = _c128(C)
        assert C.size == self.V * 144
        self._check(self._L.dp_set_clover_field(self._h, _ptr(C)))

    def set_mass(self, M):
        self._check(self._L.dp_set_mass(self._h, float(M)))

    def set_kappa(self, kappa):
        self._check(self._L.dp_set_kappa(self._h, float(kappa)))

    def set_alpha(self, alpha):
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        assert a.shape == (self.T,)
        self._check(self._L.dp_set_alpha(self._h, _ptr(a)))

    def set_alpha_space(self, a1=None, a2=None, a3=None):
        """Spatial profiles of the light-quark factorisation (None: ones)."""
        arrs = []
        for a, L in ((a1, self.dims[1]), (a2, self.dims[2]), (a3, self.dims[3])):
            if a is None:
                arrs.append(None)
            else:
                a = np.ascontiguousarray(a, dtype=np.float64)
                assert a.shape == (L,)
                arrs.append(a)
        self._check(self._L.dp_set_alpha_space(self._h, *[_ptr(a) if a is not None else None for a in arrs]))

    def set_beta(self, beta):
        """beta(y) = prod_mu a_mu(y_mu) from four profiles (None: ones)."""
        self.set_alpha(np.ones(self.T) if beta[0] is None else beta[0])
        self.set_alpha_space(*beta[1:])

    # ------------------------------------------------------------ operator
    def apply(self, psi, precond=False, dagger=False, hop_only=False, schur=False, precision="f64"):
        psi = _c128(psi)
        assert psi.size == self.V * 12
        out = np.zeros_like(psi)
        flags = (L.DP_PRECOND if precond else 0) | (L.DP_DAGGER if dagger else 0)
        flags |= (L.DP_HOP_ONLY if hop_only else 0) | (L.DP_APPLY_SCHUR if schur else 0)
        flags |= {"f64": 0, "f32": L.DP_APPLY_F32, "f16": L.DP_APPLY_F16}[precision]
        self._check(self._L.dp_apply(self._h, _ptr(psi), _ptr(out), flags))
        return out

    def apply_dev(self, in_t, out_t, precond=False, dagger=False, hop_only=False, schur=False, precision="f64",
                  masses=None, alphas=None):
        """dp_apply on torch CUDA tensors holding nrhs spinors in host layout
        (complex128, contiguous); every right-hand side is a slot of the
        multi-RHS kernels.  masses (nrhs values) and alphas ([nrhs, T]) give
        each slot its own mass and time profile (dp_apply_dev_slots)."""
        import torch
        assert in_t.is_cuda and out_t.is_cuda and in_t.is_contiguous() and out_t.is_contiguous()
        assert in_t.dtype == torch.complex128 and out_t.dtype == torch.complex128
        n = in_t.numel() // (self.V * 12)
        assert n * self.V * 12 == in_t.numel() and out_t.numel() == in_t.numel()
        flags = (L.DP_PRECOND if precond else 0) | (L.DP_DAGGER if dagger else 0)
        flags |= (L.DP_HOP_ONLY if hop_only else 0) | (L.DP_APPLY_SCHUR if schur else 0)
        flags |= {"f64": 0, "f32": L.DP_APPLY_F32, "f16": L.DP_APPLY_F16}[precision]
        stream = torch.cuda.current_stream(in_t.device).cuda_stream
        if masses is None and alphas is None:
            self._check(self._L.dp_apply_dev(self._h, ctypes.c_void_p(in_t.data_ptr()),
                                             ctypes.c_void_p(out_t.data_ptr()), n, flags, ctypes.c_void_p(stream)))
            return
        m = None if masses is None else np.ascontiguousarray(masses, dtype=np.float64)
        a = None if alphas is None else np.ascontiguousarray(alphas, dtype=np.float64)
        assert m is None or m.shape == (n,)
        assert a is None or a.shape == (n, self.T)
        self._check(self._L.dp_apply_dev_slots(self._h, ctypes.c_void_p(in_t.data_ptr()),
                                               ctypes.c_void_p(out_t.data_ptr()), n, flags,
                                               _ptr(m) if m is not None else None, _ptr(a) if a is not None else None,
                                               ctypes.c_void_p(stream)))

    def apply_dev_noalloc(self, in_t, out_t, precond=False, dagger=False, hop_only=False, schur=False,
                          precision="f64"):
        """apply_dev through dp_apply_dev_noalloc: the library allocates nothing
        (its temporaries live in a static device scratch array per GPU)."""
        import torch
        assert in_t.is_cuda and out_t.is_cuda and in_t.is_contiguous() and out_t.is_contiguous()
        assert in_t.dtype == torch.complex128 and out_t.dtype == torch.complex128
        n = in_t.numel() // (self.V * 12)
        assert n * self.V * 12 == in_t.numel() and out_t.numel() == in_t.numel()
        flags = (L.DP_PRECOND if precond else 0) | (L.DP_DAGGER if dagger else 0)
        flags |= (L.DP_HOP_ONLY if hop_only else 0) | (L.DP_APPLY_SCHUR if schur else 0)
        flags |= {"f64": 0, "f32": L.DP_APPLY_F32, "f16": L.DP_APPLY_F16}[precision]
        stream = torch.cuda.current_stream(in_t.device).cuda_stream
        self._check(self._L.dp_apply_dev_noalloc(self._h, ctypes.c_void_p(in_t.data_ptr()),
                                                 ctypes.c_void_p(out_t.data_ptr()), n, flags,
                                                 ctypes.c_void_p(stream)))

    def point_sources(self, site, c0=0, ncols=12, out=None):
        """Unit point sources at `site` in spin-colour components c0 .. c0+ncols-1,
        written by dp_point_sources into a complex128 CUDA tensor [ncols, V*12]
        (or into `out`)."""
        import torch
        if out is None:
            out = torch.empty((ncols, self.V * 12), dtype=torch.complex128, device="cuda")
        assert out.is_cuda and out.is_contiguous() and out.dtype == torch.complex128
        assert out.numel() == ncols * self.V * 12
        stream = torch.cuda.current_stream(out.device).cuda_stream
        self._check(self._L.dp_point_sources(self._h, (ctypes.c_int * 4)(*[int(v) for v in site]), int(c0),
                                             int(ncols), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)))
        return out

    # ------------------------------------------------------------ timing
    def set_timing(self, enable=True):
        self._check(self._L.dp_set_timing(self._h, int(bool(enable))))

    def timing(self):
        """Per-kernel statistics: {name: dict(launches, ms, bytes, flops)}."""
        n = ctypes.c_int(0)
        self._check(self._L.dp_get_timing(self._h, None, 0, ctypes.byref(n)))
        arr = (L.dp_kernel_stat * max(n.value, 1))()
        self._check(self._L.dp_get_timing(self._h, arr, n.value, ctypes.byref(n)))
        return {a.name.decode(): dict(launches=a.launches, ms=a.ms, bytes=a.bytes, flops=a.flops)
                for a in arr[:n.value]}

    def timing_samples(self, name):
        """Per-launch durations (ms) of one timed kernel variant, in launch order."""
        n = ctypes.c_int(0)
        self._check(self._L.dp_get_timing_samples(self._h, name.encode(), None, 0, ctypes.byref(n)))
        arr = (ctypes.c_float * max(n.value, 1))()
        self._check(self._L.dp_get_timing_samples(self._h, name.encode(), arr, n.value, ctypes.byref(n)))
        return np.array(arr[:n.value], dtype=np.float64)

    # ------------------------------------------------------------ solves
    @staticmethod
    def _params(r, solver, precision, max_iter, delta, x0_src, ncols_group):
        return L.dp_params(float(r), L.DP_SOLVER[solver], L.DP_PREC[precision], int(max_iter), float(delta),
                           int(x0_src), int(ncols_group))

    @staticmethod
    def _infos(info):
        return [dict(status=i.status, iters=i.iters, outer=i.outer, hop_calls=i.hop_calls,
                     restarts=i.restarts, true_res=i.true_res, seconds=i.seconds, fallback=i.fallback)
                for i in info]

    def solve(self, eta, r=1e-11, solver="bicgstab", precision="f64", max_iter=10000, delta=0.0, x0_src=0,
              ncols_group=0, want_S=True, allow_unconverged=False, allow=()):
        """Solve (D+M) S = eta for eta of shape ([nrhs,] T, L1, L2, L3, 4, 3).
        precision: "f64", "f32", "f16" (inner precision under FP64 defect
        correction) or "f32single" (one FP32 solve, no correction).
        Returns (S, cpp, info); `allow` lists further return codes that do not raise."""
        eta = _c128(eta)
        if eta.ndim == 6:
            eta = eta[None]
        n = eta.shape[0]
        S = np.zeros_like(eta) if want_S else None
        grp = ncols_group if ncols_group > 0 else 1
        cpp = np.zeros((n // grp, self.T))
        info = (L.dp_info * n)()
        p = self._params(r, solver, precision, max_iter, delta, x0_src, ncols_group)
        rc = self._L.dp_solve(self._h, _ptr(eta), n, ctypes.byref(p), _ptr(S) if want_S else None, _ptr(cpp),
                              info)
        self._check(rc, allow=((L.DP_ERR_NOT_CONVERGED,) if allow_unconverged else ()) + tuple(allow))
        return S, cpp, self._infos(info)

    def solve_sap(self, eta, block, r=1e-10, ncy=5, nmr=4, nkv=16, precision="f32", max_iter=1000,
                  allow_unconverged=False):
        """SAP+GCR for one right-hand side (host layout) with Schwarz blocks of
        extents `block`; returns (S, cpp, info)."""
        eta = _c128(eta)
        assert eta.size == self.V * 12
        S = np.zeros_like(eta)
        cpp = np.zeros(self.T)
        info = L.dp_info()
        p = L.dp_sap_params(float(r), (ctypes.c_int * 4)(*[int(b) for b in block]), int(ncy), int(nmr), int(nkv),
                            L.DP_PREC[precision], int(max_iter))
        rc = self._L.dp_solve_sap(self._h, _ptr(eta), ctypes.byref(p), _ptr(S), _ptr(cpp), ctypes.byref(info))
        self._check(rc, allow=(L.DP_ERR_NOT_CONVERGED,) if allow_unconverged else ())
        return S, cpp, self._infos([info])[0]

    def solve_sap_dev(self, eta_t, S_t=None, block=(4, 4, 4, 4), r=1e-10, ncy=5, nmr=4, nkv=16, precision="f32",
                      max_iter=1000, allow_unconverged=False):
        """SAP+GCR with eta_t (and S_t) torch CUDA tensors in host layout;
        returns (cpp, info)."""
        import torch
        assert eta_t.is_cuda and eta_t.is_contiguous() and eta_t.numel() * eta_t.element_size() == self.V * 12 * 16
        cpp = np.zeros(self.T)
        info = L.dp_info()
        p = L.dp_sap_params(float(r), (ctypes.c_int * 4)(*[int(b) for b in block]), int(ncy), int(nmr), int(nkv),
                            L.DP_PREC[precision], int(max_iter))
        stream = torch.cuda.current_stream(eta_t.device).cuda_stream
        rc = self._L.dp_solve_sap_dev(self._h, ctypes.c_void_p(eta_t.data_ptr()), ctypes.byref(p),
                                      ctypes.c_void_p(S_t.data_ptr()) if S_t is not None else None, _ptr(cpp),
                                      ctypes.byref(info), ctypes.c_void_p(stream))
        self._check(rc, allow=(L.DP_ERR_NOT_CONVERGED,) if allow_unconverged else ())
        return cpp, self._infos([info])[0]

    def sap_precondition(self, r, block, ncy=5, nmr=4, precision="f32"):
        """One application psi = M r of the SAP preconditioner (host layout,
        preconditioned variables)."""
        r = _c128(r)
        assert r.size == self.V * 12
        psi = np.zeros_like(r)
        p = L.dp_sap_params(1.0, (ctypes.c_int * 4)(*[int(b) for b in block]), int(ncy), int(nmr), 1,
                            L.DP_PREC[precision], 1)
        self._check(self._L.dp_sap_precondition(self._h, _ptr(r), ctypes.byref(p), _ptr(psi)))
        return psi

    def solve_dev(self, eta_t, S_t=None, r=1e-11, solver="bicgstab", precision="f64", max_iter=10000, delta=0.0,
                  x0_src=0, ncols_group=0, allow_unconverged=False, allow=()):
        """Device variant: eta_t (and S_t) are torch CUDA tensors in host layout."""
        import torch
        assert eta_t.is_cuda and eta_t.is_contiguous()
        n = eta_t.numel() * eta_t.element_size() // (self.V * 12 * 16)
        grp = ncols_group if ncols_group > 0 else 1
        cpp = np.zeros((n // grp, self.T))
        info = (L.dp_info * n)()
        p = self._params(r, solver, precision, max_iter, delta, x0_src, ncols_group)
        stream = torch.cuda.current_stream(eta_t.device).cuda_stream
        rc = self._L.dp_solve_dev(self._h, ctypes.c_void_p(eta_t.data_ptr()), n, ctypes.byref(p),
                                  ctypes.c_void_p(S_t.data_ptr()) if S_t is not None else None, _ptr(cpp), info,
                                  ctypes.c_void_p(stream))
        self._check(rc, allow=((L.DP_ERR_NOT_CONVERGED,) if allow_unconverged else ()) + tuple(allow))
        return cpp, self._infos(info)


class Batch:
    """A set of slots on one Lattice that solve right-hand sides entering and
    leaving independently (continuous batching).  Sources and solutions are
    torch CUDA tensors in host layout; results come back with their tag."""

    def __init__(self, lattice, nslots, precision="f32", solver="bicgstab"):
        self.L = lattice
        self.nslots = int(nslots)
        h = ctypes.c_void_p()
        lattice._check(lattice._L.dp_batch_open(lattice._h, self.nslots, L.DP_PREC[precision],
                                                L.DP_SOLVER[solver], ctypes.byref(h)))
        self._h = h
        self._keep = {}  # tag -> tensors that must stay alive until harvested

    def close(self):
        if getattr(self, "_h", None):
            self.L._L.dp_batch_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def status(self):
        f, r, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self.L._check(self.L._L.dp_batch_status(self._h, ctypes.byref(f), ctypes.byref(r), ctypes.byref(d)))
        return dict(free=f.value, running=r.value, done=d.value)

    def device_bytes(self):
        return int(self.L._L.dp_batch_device_bytes(self._h))

    def admit(self, eta_t, S_t=None, M=0.0, alpha=None, r=1e-10, max_iter=10000, delta=0.0, x0_src=0, tag=0):
        """Admit the columns of eta_t ([ncols, ...] complex128 CUDA tensor).
        Returns the slot indices, or None when the batch has too few free slots."""
        import torch
        assert eta_t.is_cuda and eta_t.is_contiguous()
        ncols = eta_t.numel() * eta_t.element_size() // (self.L.V * 12 * 16)
        a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
        torch.cuda.current_stream(eta_t.device).synchronize()  # the library runs on its own stream
        slots = (ctypes.c_int * ncols)()
        rc = self.L._L.dp_batch_admit(self._h, ncols, ctypes.c_void_p(eta_t.data_ptr()),
                                      ctypes.c_void_p(S_t.data_ptr()) if S_t is not None else None, float(M),
                                      _ptr(a) if a is not None else None, float(r), int(max_iter), float(delta),
                                      int(x0_src), int(tag), slots)
        if rc == L.DP_ERR_FULL:
            return None
        self.L._check(rc)
        if S_t is not None:  # written when the columns finish
            self._keep.setdefault(int(tag), []).append(S_t)
        return list(slots)

    def step(self, k=4):
        n = ctypes.c_int(0)
        self.L._check(self.L._L.dp_batch_step(self._h, int(k), ctypes.byref(n)))
        return n.value

    def harvest(self, max_results=None):
        """Finished right-hand sides: list of dict(tag, slot, info, cpp)."""
        m = self.nslots if max_results is None else int(max_results)
        out = (L.dp_batch_result * m)()
        cpp = np.zeros((m, self.L.T))
        n = ctypes.c_int(0)
        self.L._check(self.L._L.dp_batch_harvest(self._h, out, _ptr(cpp), m, ctypes.byref(n)))
        res = []
        for k in range(n.value):
            o = out[k]
            i = o.info
            res.append(dict(tag=o.tag, slot=o.slot, cpp=cpp[k].copy(),
                            info=dict(status=i.status, iters=i.iters, outer=i.outer, hop_calls=i.hop_calls,
                                      restarts=i.restarts, true_res=i.true_res, seconds=i.seconds,
                                      fallback=i.fallback)))
        return res

    def release(self, tag):
        """Drop the references kept for a finished request."""
        self._keep.pop(int(tag), None)
