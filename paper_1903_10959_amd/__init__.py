"""MI355X (gfx950) Chebyshev-filtered subspace iteration for the spectral
finite-element Kohn-Sham operator -- Python binding of libchfsi.so.

Every numerical step runs in the HIP library (include/chfsi.h); this module
only marshals arguments: torch tensors on the GPU supply device pointers and
the current HIP stream.  Blocks X are float64, DoF-major (row = degree of
freedom, column = vector), row stride ``X.stride(0)``.

There is no CPU fallback: if the library is not built, construction raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import PRECISIONS, Opts, Report

__all__ = ["Context", "ChfsiError", "footprint_bytes", "batch_footprint_bytes", "solve_batch", "BatchSession", "PRECISIONS", "library_path"]


class ChfsiError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


def library_path() -> str:
    return _lib.LIB_PATH


def footprint_bytes(n_el: int, p: int, nblock: int, block_width: int = 0, prec: str = "fp64") -> int:
    return int(_lib.load().chfsi_footprint_bytes(n_el, p, nblock, block_width, PRECISIONS[prec]))


def batch_footprint_bytes(n_el: int, p: int, nblock: int) -> int:
    """Device bytes of a context in a batch session (without the caller's block)."""
    return int(_lib.load().chfsi_batch_footprint_bytes(n_el, p, nblock))


def fermi_level(evals_fr, n_oc: int, n_electrons: float, sigma: float) -> float:
    """Fermi energy of Alg. 5 step 1: 2 (n_oc + sum_k f(e_k, mu)) = n_electrons."""
    ev = np.ascontiguousarray(np.asarray(evals_fr, dtype=np.float64))
    mu = C.c_double(0.0)
    st = _lib.load().chfsi_fermi_level(ev.ctypes.data_as(C.c_void_p), int(ev.size), int(n_oc), float(n_electrons),
                                       float(sigma), C.byref(mu))
    if st != 0:
        raise ChfsiError(st, "fermi_level", "n_electrons outside (2 n_oc, 2 (n_oc + n_fr)), or bad input")
    return float(mu.value)


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _opts(nstates, nblock, degree, tol, max_iter, block_width=0, ladder=("fp64",), ladder_tol=None,
          mixed_cholgs=False) -> Opts:
    o = Opts()
    o.nstates, o.nblock, o.degree, o.max_iter, o.block_width = int(nstates), int(nblock), int(degree), \
        int(max_iter), int(block_width)
    o.tol = float(tol)
    lad = [_prec(x) for x in ladder][:4]
    for i, v in enumerate(lad):
        o.ladder[i] = v
    o.n_ladder = len(lad)
    for k, v in enumerate(list(ladder_tol or [])[:4]):
        o.ladder_tol[k] = float(v)
    o.mixed_cholgs = 1 if mixed_cholgs else 0
    return o


def _report(rep: Report, st: int) -> dict:
    return dict(status=st, converged=(st == 0), iters=rep.iters, rung=rep.rung, t_filter=rep.t_filter,
                t_cholgs=rep.t_cholgs, t_rr=rep.t_rr, max_resid=rep.max_resid, dofvecs=rep.dofvecs)


class BatchSession:
    """chfsi_batch_*: problems join (add) and leave (when converged) between
    passes; every pass runs their filters in shared graph-captured sweeps."""

    def __init__(self, device: int = 0):
        self._lib = _lib.load()
        h = C.c_void_p()
        st = self._lib.chfsi_batch_create(C.byref(h), device)
        if st != 0:
            raise ChfsiError(st, "chfsi_batch_create", "invalid device or no GPU")
        self._h = h
        self._keep = {}     # id -> (opts, evals, resid, X, ctx): alive while in the session
        self._done = (C.c_int * 4096)()

    def add(self, ctx, X, nstates: int, degree: int, tol: float, max_iter: int = 200, ladder=("fp32", "fp64"),
            mixed_cholgs: bool = False, ladder_tol=None) -> int:
        px, ld, nb = Context._block(X)
        o = _opts(nstates, nb, degree, tol, max_iter, 0, ladder, ladder_tol, mixed_cholgs)
        ev, rs = np.empty(nb), np.empty(nb)
        pid = self._lib.chfsi_batch_add(self._h, ctx._h, C.byref(o), px, ld, ev.ctypes.data_as(C.c_void_p),
                                       rs.ctypes.data_as(C.c_void_p))
        if pid < 0:
            msg = self._lib.chfsi_batch_last_error(self._h)
            raise ChfsiError(pid, "chfsi_batch_add", msg.decode() if msg else "")
        self._keep[pid] = (o, ev, rs, X, ctx)
        return pid

    def set_threads(self, threads: int):
        """Host threads for the per-problem CholGS / Rayleigh-Ritz steps."""
        st = self._lib.chfsi_batch_set_threads(self._h, int(threads))
        if st != 0:
            raise ChfsiError(st, "chfsi_batch_set_threads", "threads must be in 1..256")
        return self

    def step(self):
        """One pass; returns (remaining, [(id, result dict), ...] of problems that
        left).  A problem that failed on its own has status < 0 in its dict."""
        nd = C.c_int()
        rem = self._lib.chfsi_batch_pass(self._h, self._done, C.byref(nd), len(self._done))
        if rem < 0:
            msg = self._lib.chfsi_batch_last_error(self._h)
            raise ChfsiError(rem, "chfsi_batch_pass", msg.decode() if msg else "")
        out = []
        for k in range(nd.value):
            pid = int(self._done[k])
            rep = Report()
            self._lib.chfsi_batch_report(self._h, pid, C.byref(rep))
            o, ev, rs, X, ctx = self._keep.pop(pid)
            d = _report(rep, rep.status)
            d.update(evals=ev, resid=rs)
            out.append((pid, d))
        return rem, out

    def run(self):
        """Passes until no problem remains; returns {id: result dict} of every
        problem that left during them."""
        out = {}
        while True:
            rem, done = self.step()
            out.update(done)
            if rem == 0:
                while True:                 # ids the last pass could not report at once
                    rem, done = self.step()
                    if not done:
                        return out
                    out.update(done)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.chfsi_batch_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(contexts, blocks, nstates, degree: int, tol: float, max_iter: int = 200, prec: str = "fp32",
                mixed_cholgs: bool = False, ladder=None):
    """chfsi_solve_batch over problems i (context contexts[i], block blocks[i],
    nstates[i] wanted states), every problem on the filter precision prec or,
    when given, on the precision ladder (e.g. ("bf16", "fp32", "fp64")).
    Returns a list of per-problem result dicts."""
    lib = _lib.load()
    n = len(contexts)
    if len(blocks) != n or len(nstates) != n:
        raise ValueError("contexts, blocks and nstates must have the same length")
    opts = (Opts * n)()
    ctxs = (C.c_void_p * n)()
    xs = (C.c_void_p * n)()
    lds = (C.c_int64 * n)()
    evs = [np.empty(int(b.shape[1])) for b in blocks]
    rss = [np.empty(int(b.shape[1])) for b in blocks]
    evp = (C.c_void_p * n)(*[e.ctypes.data for e in evs])
    rsp = (C.c_void_p * n)(*[r.ctypes.data for r in rss])
    reps = (Report * n)()
    for i, (c, X, N) in enumerate(zip(contexts, blocks, nstates)):
        px, ld, nb = Context._block(X)
        opts[i] = _opts(N, nb, degree, tol, max_iter, 0, tuple(ladder) if ladder else (prec,), None, mixed_cholgs)
        ctxs[i] = c._h.value
        xs[i] = px.value
        lds[i] = ld
    st = lib.chfsi_solve_batch(ctxs, n, opts, xs, lds, evp, rsp, reps)
    if st not in (0, _lib.WARN_NOT_CONVERGED):
        msg = lib.chfsi_last_error(contexts[0]._h)
        raise ChfsiError(st, "solve_batch", msg.decode() if msg else "")
    out = []
    for i in range(n):
        d = _report(reps[i], reps[i].status)
        d.update(evals=evs[i], resid=rss[i])
        out.append(d)
    return out


class Context:
    """One library context: mesh tables, potential and workspaces on one GPU.
    Work is enqueued on ``stream`` (default: torch's current stream).
    ``device=-1`` gives a host-only context (tables and bound, no device work)."""

    def __init__(self, device: int = 0, stream=None):
        self._lib = _lib.load()
        self.device = device
        handle = None
        if device >= 0:
            import torch

            if stream is None:
                stream = torch.cuda.current_stream(device)
            handle = stream.cuda_stream
        self.stream = stream
        h = C.c_void_p()
        st = self._lib.chfsi_create(C.byref(h), device, C.c_void_p(handle))
        if st != 0:
            raise ChfsiError(st, "chfsi_create", "invalid device or no GPU")
        self._h = h
        self.n_dof = self.n_cells = self.n_loc = 0

    # ---- helpers ---------------------------------------------------------
    def _check(self, st: int, where: str, ok=(0,)):
        if st not in ok:
            msg = self._lib.chfsi_last_error(self._h)
            raise ChfsiError(st, where, msg.decode() if msg else "")
        return st

    @staticmethod
    def _block(X):
        import torch

        if not isinstance(X, torch.Tensor) or X.dtype != torch.float64 or not X.is_cuda or X.dim() != 2:
            raise TypeError("expected a 2-D float64 CUDA tensor [n_dof, ncols]")
        if X.shape[1] > 1 and X.stride(1) != 1:
            raise ValueError("columns must be contiguous (stride(1) == 1)")
        return C.c_void_p(X.data_ptr()), int(X.stride(0)), int(X.shape[1])

    def close(self):
        if getattr(self, "_h", None):
            self._lib.chfsi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- setMesh ---------------------------------------------------------
    def set_mesh(self, L: float, n_el: int, p: int, periodic: bool = False):
        """Dirichlet cube [0, L]^3 (default) or the periodic cell [0, L)^3 (n_el even)."""
        if periodic:
            self._check(self._lib.chfsi_set_mesh_periodic(self._h, float(L), int(n_el), int(p)), "set_mesh_periodic")
        else:
            self._check(self._lib.chfsi_set_mesh(self._h, float(L), int(n_el), int(p)), "set_mesh")
        self.periodic = bool(periodic)
        nd, nc, nl = C.c_int64(), C.c_int64(), C.c_int()
        self._check(self._lib.chfsi_get_sizes(self._h, C.byref(nd), C.byref(nc), C.byref(nl)), "get_sizes")
        self.n_dof, self.n_cells, self.n_loc = nd.value, nc.value, nl.value
        self.L, self.n_el, self.p = float(L), int(n_el), int(p)
        return self

    def cell_dof_map(self) -> np.ndarray:
        out = np.empty((self.n_cells, self.n_loc), dtype=np.int32)
        self._check(self._lib.chfsi_get_cell_dof_map(self._h, out.ctypes.data_as(C.c_void_p)), "get_cell_dof_map")
        return out

    def cell_colors(self) -> np.ndarray:
        out = np.empty(self.n_cells, dtype=np.uint8)
        self._check(self._lib.chfsi_get_cell_colors(self._h, out.ctypes.data_as(C.c_void_p)), "get_cell_colors")
        return out

    def dof_coords(self) -> np.ndarray:
        out = np.empty((self.n_dof, 3), dtype=np.float64)
        self._check(self._lib.chfsi_get_dof_coords(self._h, out.ctypes.data_as(C.c_void_p)), "get_dof_coords")
        return out

    def mass(self) -> np.ndarray:
        out = np.empty(self.n_dof, dtype=np.float64)
        self._check(self._lib.chfsi_get_mass(self._h, out.ctypes.data_as(C.c_void_p)), "get_mass")
        return out

    def cell_matrix(self) -> np.ndarray:
        out = np.empty((self.n_loc, self.n_loc), dtype=np.float64)
        self._check(self._lib.chfsi_get_cell_matrix(self._h, out.ctypes.data_as(C.c_void_p)), "get_cell_matrix")
        return out

    # ---- setPotential ----------------------------------------------------
    def set_potential(self, V):
        import torch

        if isinstance(V, torch.Tensor):
            if V.dtype != torch.float64 or V.numel() != self.n_dof:
                raise ValueError("V must be float64 with n_dof entries")
            V = V.contiguous()
            st = self._lib.chfsi_set_potential(self._h, C.c_void_p(V.data_ptr()), self.n_dof, 1 if V.is_cuda else 0)
        else:
            v = np.ascontiguousarray(V, dtype=np.float64)
            if v.size != self.n_dof:
                raise ValueError("V must have n_dof entries")
            st = self._lib.chfsi_set_potential(self._h, v.ctypes.data_as(C.c_void_p), self.n_dof, 0)
        self._check(st, "set_potential")
        return self

    @property
    def upper_bound(self) -> float:
        b = C.c_double()
        self._check(self._lib.chfsi_get_upper_bound(self._h, C.byref(b)), "get_upper_bound")
        return b.value

    # ---- operator --------------------------------------------------------
    def apply(self, X, Y=None, prec="fp64"):
        import torch

        if Y is None:
            Y = torch.empty_strided(tuple(X.shape), tuple(X.stride()), dtype=X.dtype, device=X.device)
        px, ld, n = self._block(X)
        py, ldy, ny = self._block(Y)
        if ldy != ld or ny != n:
            raise ValueError("X and Y must have the same shape and row stride")
        self._check(self._lib.chfsi_apply(self._h, px, py, ld, n, _prec(prec)), "apply")
        return Y

    def set_kpoint(self, k):
        """Bloch wave vector (kx, ky, kz) of the complex operator (periodic mesh)."""
        kx, ky, kz = (float(v) for v in k)
        self._check(self._lib.chfsi_set_kpoint(self._h, kx, ky, kz), "set_kpoint")
        return self

    def poisson_apply(self, x, y=None):
        """y = A x, A = 1/(4 pi) int grad N_i . grad N_j (Dirichlet mesh)."""
        import torch

        if y is None:
            y = torch.empty_like(x)
        for t in (x, y):
            if t.dtype != torch.float64 or not t.is_cuda or t.numel() != self.n_dof or not t.is_contiguous():
                raise TypeError("x, y: contiguous float64 CUDA tensors of n_dof values")
        self._check(self._lib.chfsi_poisson_apply(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())),
                    "poisson_apply")
        return y

    def poisson_solve(self, rho, phi=None, charges=(), tol: float = 1e-10, max_iter: int = 10000):
        """Electrostatic potential of the nodal density rho plus point charges
        [(dof, q), ...] (Jacobi-PCG).  Returns dict(phi, iters, rel_resid, converged)."""
        import torch

        if phi is None:
            phi = torch.zeros_like(rho)
        for t in (rho, phi):
            if t.dtype != torch.float64 or not t.is_cuda or t.numel() != self.n_dof or not t.is_contiguous():
                raise TypeError("rho, phi: contiguous float64 CUDA tensors of n_dof values")
        cd = np.ascontiguousarray(np.array([int(d) for d, _ in charges], dtype=np.int64))
        cq = np.ascontiguousarray(np.array([float(q) for _, q in charges], dtype=np.float64))
        it, rr = C.c_int(0), C.c_double(0.0)
        st = self._lib.chfsi_poisson_solve(self._h, C.c_void_p(rho.data_ptr()), int(cd.size),
                                           cd.ctypes.data_as(C.c_void_p), cq.ctypes.data_as(C.c_void_p),
                                           C.c_void_p(phi.data_ptr()), float(tol), int(max_iter), C.byref(it),
                                           C.byref(rr))
        self._check(st, "poisson_solve", ok=(0, _lib.WARN_NOT_CONVERGED))
        return dict(phi=phi, iters=it.value, rel_resid=rr.value, converged=(st == 0))

    def set_kpoints(self, ks):
        """A group of wave vectors [[kx, ky, kz], ...] for apply_complex_kpoints."""
        k = np.ascontiguousarray(np.asarray(ks, dtype=np.float64).reshape(-1, 3))
        self._check(self._lib.chfsi_set_kpoints(self._h, int(k.shape[0]), k.ctypes.data_as(C.c_void_p)),
                    "set_kpoints")
        self.nk = int(k.shape[0])
        return self

    def apply_complex_kpoints(self, X, Y=None):
        """Y[g] = Htilde_{k_g} X[g] for a complex128 CUDA tensor [nk, n_dof, ncols]."""
        import torch

        if not isinstance(X, torch.Tensor) or X.dtype != torch.complex128 or not X.is_cuda or X.dim() != 3:
            raise TypeError("expected a 3-D complex128 CUDA tensor [nk, n_dof, ncols]")
        if X.shape[0] != self.nk or X.shape[1] != self.n_dof or (X.shape[2] > 1 and X.stride(2) != 1):
            raise ValueError("X must be [nk, n_dof, ncols] with contiguous columns")
        if Y is None:
            Y = torch.empty_strided(tuple(X.shape), tuple(X.stride()), dtype=X.dtype, device=X.device)
        if Y.dtype != torch.complex128 or tuple(Y.shape) != tuple(X.shape) or Y.stride() != X.stride():
            raise ValueError("Y must match X in shape, dtype and strides")
        self._check(self._lib.chfsi_apply_complex_kpoints(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                                                          int(X.stride(1)), int(X.shape[2]), int(X.stride(0))),
                    "apply_complex_kpoints")
        return Y

    def apply_complex(self, X, Y=None):
        """Y = Htilde_k X for a complex128 CUDA tensor [n_dof, ncols] (periodic mesh)."""
        import torch

        if not isinstance(X, torch.Tensor) or X.dtype != torch.complex128 or not X.is_cuda or X.dim() != 2:
            raise TypeError("expected a 2-D complex128 CUDA tensor [n_dof, ncols]")
        if X.shape[1] > 1 and X.stride(1) != 1:
            raise ValueError("columns must be contiguous (stride(1) == 1)")
        if Y is None:
            Y = torch.empty_strided(tuple(X.shape), tuple(X.stride()), dtype=X.dtype, device=X.device)
        if Y.dtype != torch.complex128 or tuple(Y.shape) != tuple(X.shape) or Y.stride() != X.stride():
            raise ValueError("Y must match X in shape, dtype and strides")
        self._check(self._lib.chfsi_apply_complex(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()),
                                                  int(X.stride(0)), int(X.shape[1])), "apply_complex")
        return Y

    # ---- ChFSI at the k-point (complex Hermitian operator) -------------------
    @staticmethod
    def _cblock(X):
        import torch

        if not isinstance(X, torch.Tensor) or X.dtype != torch.complex128 or not X.is_cuda or X.dim() != 2:
            raise TypeError("expected a 2-D complex128 CUDA tensor [n_dof, ncols]")
        if X.shape[1] > 1 and X.stride(1) != 1:
            raise ValueError("columns must be contiguous (stride(1) == 1)")
        return C.c_void_p(X.data_ptr()), int(X.stride(0)), int(X.shape[1])

    @property
    def upper_bound_k(self) -> float:
        b = C.c_double()
        self._check(self._lib.chfsi_get_upper_bound_k(self._h, C.byref(b)), "get_upper_bound_k")
        return b.value

    def chebyshev_filter_complex(self, X, degree: int, a: float, b: float, a0: float, block_width: int = 0):
        px, ld, n = self._cblock(X)
        self._check(self._lib.chfsi_chebyshev_filter_complex(self._h, px, ld, n, int(degree), float(a), float(b),
                                                             float(a0), int(block_width)), "chebyshev_filter_complex")
        return X

    def orthonormalize_complex(self, X):
        px, ld, n = self._cblock(X)
        self._check(self._lib.chfsi_orthonormalize_complex(self._h, px, ld, n), "orthonormalize_complex")
        return X

    def rayleigh_ritz_complex(self, X, HX_out=None):
        px, ld, n = self._cblock(X)
        ev, rs = np.empty(n), np.empty(n)
        ph = C.c_void_p(0)
        if HX_out is not None:
            ph, ldh, nh = self._cblock(HX_out)
            if ldh != ld or nh != n:
                raise ValueError("HX_out must match X")
        st = self._check(self._lib.chfsi_rayleigh_ritz_complex(self._h, px, ld, n, ev.ctypes.data_as(C.c_void_p),
                                                               rs.ctypes.data_as(C.c_void_p), ph),
                         "rayleigh_ritz_complex", ok=(0, _lib.WARN_NOT_CONVERGED))
        self.last_eigensolve_converged = st == 0
        return ev, rs

    def solve_complex(self, X, nstates: int, degree: int, tol: float, max_iter: int = 200, block_width: int = 0):
        px, ld, nb = self._cblock(X)
        o = _opts(nstates, nb, degree, tol, max_iter, block_width, ("fp64",), None, False)
        ev, rs = np.empty(nb), np.empty(nb)
        rep = Report()
        st = self._lib.chfsi_solve_complex(self._h, C.byref(o), px, ld, ev.ctypes.data_as(C.c_void_p),
                                           rs.ctypes.data_as(C.c_void_p), C.byref(rep))
        self._check(st, "solve_complex", ok=(0, _lib.WARN_NOT_CONVERGED))
        return dict(evals=ev, resid=rs, status=st, converged=(st == 0), iters=rep.iters, t_filter=rep.t_filter,
                    t_cholgs=rep.t_cholgs, t_rr=rep.t_rr, max_resid=rep.max_resid, dofvecs=rep.dofvecs)

    def cheb_step(self, X, Xprev, Y, s1: float, s2: float, shift: float):
        px, ld, n = self._block(X)
        py, ldy, _ = self._block(Y)
        pp = C.c_void_p(0)
        if Xprev is not None:
            pp, ldp, _ = self._block(Xprev)
            if ldp != ld:
                raise ValueError("row strides differ")
        if ldy != ld:
            raise ValueError("row strides differ")
        self._check(self._lib.chfsi_cheb_step(self._h, px, pp, py, ld, n, float(s1), float(s2), float(shift)),
                    "cheb_step")
        return Y

    # ---- chebyshevFilter -------------------------------------------------
    def chebyshev_filter(self, X, degree: int, a: float, b: float, a0: float, prec="fp64", block_width: int = 0):
        px, ld, n = self._block(X)
        self._check(self._lib.chfsi_chebyshev_filter(self._h, px, ld, n, int(degree), float(a), float(b), float(a0),
                                                     _prec(prec), int(block_width)), "chebyshev_filter")
        return X

    # ---- orthonormalize --------------------------------------------------
    def orthonormalize(self, X, mixed: bool = False):
        px, ld, n = self._block(X)
        self._check(self._lib.chfsi_orthonormalize(self._h, px, ld, n, 1 if mixed else 0), "orthonormalize")
        return X

    # ---- rayleighRitz ----------------------------------------------------
    def rayleigh_ritz(self, X, HX_out=None):
        px, ld, n = self._block(X)
        ev = np.empty(n)
        rs = np.empty(n)
        ph = C.c_void_p(0)
        if HX_out is not None:
            ph, ldh, nh = self._block(HX_out)
            if ldh != ld or nh != n:
                raise ValueError("HX_out must match X")
        st = self._check(self._lib.chfsi_rayleigh_ritz(self._h, px, ld, n, ev.ctypes.data_as(C.c_void_p),
                                                       rs.ctypes.data_as(C.c_void_p), ph), "rayleigh_ritz",
                         ok=(0, _lib.WARN_NOT_CONVERGED))
        self.last_eigensolve_converged = st == 0
        return ev, rs

    def rayleigh_ritz_split(self, X, n_fr: int, mixed: bool = True, Xfr=None):
        """Spectrum-splitting Rayleigh-Ritz (Alg. 4): Ritz values and residuals of
        the n_fr largest pairs.  The rotated vectors X Q_fr go to Xfr (a float64
        CUDA tensor [n_dof, >= n_fr], X left unchanged) or, with Xfr None, over
        the trailing n_fr columns of X."""
        px, ld, n = self._block(X)
        pf, ldf = C.c_void_p(0), 0
        if Xfr is not None:
            pf, ldf, nf = self._block(Xfr)
            if nf < n_fr:
                raise ValueError("Xfr needs at least n_fr columns")
        ev = np.empty(int(n_fr))
        rs = np.empty(int(n_fr))
        st = self._check(self._lib.chfsi_rayleigh_ritz_split(self._h, px, ld, n, int(n_fr), 1 if mixed else 0, pf,
                                                             ldf, ev.ctypes.data_as(C.c_void_p),
                                                             rs.ctypes.data_as(C.c_void_p)),
                         "rayleigh_ritz_split", ok=(0, _lib.WARN_NOT_CONVERGED))
        self.last_eigensolve_converged = st == 0
        return ev, rs

    def density(self, X, Xfr=None, evals_fr=None, mu: float = 0.0, sigma: float = 0.0, rho=None):
        """Nodal electron density (Alg. 5, eq. elecDensSP) from the orthonormal
        basis X and the rotated fractionally occupied vectors Xfr with Ritz
        values evals_fr; returns rho (float64 CUDA tensor [n_dof])."""
        import torch

        px, ld, n = self._block(X)
        pf, ldf, nfr = C.c_void_p(0), 0, 0
        ev = None
        if Xfr is not None:
            pf, ldf, nfr = self._block(Xfr)
            ev = np.ascontiguousarray(np.asarray(evals_fr, dtype=np.float64))
            if ev.shape != (nfr,):
                raise ValueError("evals_fr must have one value per column of Xfr")
        if rho is None:
            rho = torch.empty(self.n_dof, dtype=torch.float64, device=X.device)
        if rho.dtype != torch.float64 or not rho.is_cuda or rho.numel() != self.n_dof or not rho.is_contiguous():
            raise TypeError("rho must be a contiguous float64 CUDA tensor of n_dof values")
        self._check(self._lib.chfsi_density(self._h, px, ld, n, pf, ldf, nfr,
                                            ev.ctypes.data_as(C.c_void_p) if ev is not None else None,
                                            float(mu), float(sigma), C.c_void_p(rho.data_ptr())), "density")
        return rho

    # ---- solve -----------------------------------------------------------
    def solve(self, X, nstates: int, degree: int, tol: float, max_iter: int = 200, block_width: int = 0,
              ladder=("fp64",), ladder_tol=None, mixed_cholgs: bool = False):
        px, ld, nb = self._block(X)
        o = _opts(nstates, nb, degree, tol, max_iter, block_width, ladder, ladder_tol, mixed_cholgs)
        ev = np.empty(nb)
        rs = np.empty(nb)
        rep = Report()
        st = self._lib.chfsi_solve(self._h, C.byref(o), px, ld, ev.ctypes.data_as(C.c_void_p),
                                   rs.ctypes.data_as(C.c_void_p), C.byref(rep))
        self._check(st, "solve", ok=(0, _lib.WARN_NOT_CONVERGED))
        return dict(evals=ev, resid=rs, status=st, converged=(st == 0), iters=rep.iters, rung=rep.rung,
                    t_filter=rep.t_filter, t_cholgs=rep.t_cholgs, t_rr=rep.t_rr, max_resid=rep.max_resid,
                    dofvecs=rep.dofvecs)

    # ---- timing of the cell-product kernel ---------------------------------
    def set_tile_variant(self, variant: int = -1):
        """Cell-kernel tile configuration: -1 built-in, 0 four-wave, 1 eight-wave."""
        self._check(self._lib.chfsi_set_tile_variant(self._h, int(variant)), "set_tile_variant")
        self.tile_variant = int(variant)
        return self

    def set_jacobi_sweeps(self, max_sweeps: int = 40):
        """Cap on the Jacobi sweeps of the projected eigensolve."""
        self._check(self._lib.chfsi_set_jacobi_sweeps(self._h, int(max_sweeps)), "set_jacobi_sweeps")
        return self

    def device_bytes(self) -> int:
        """Device bytes the context holds now."""
        b = C.c_size_t()
        self._check(self._lib.chfsi_device_bytes(self._h, C.byref(b)), "device_bytes")
        return int(b.value)

    def set_cells_per_tile(self, cpt: int = 0):
        """Cells per work-group of the cell kernel: 0 chosen from the column count, or 1, 2, 4."""
        self._check(self._lib.chfsi_set_cells_per_tile(self._h, int(cpt)), "set_cells_per_tile")
        self.cells_per_tile = int(cpt)
        return self

    def set_rr_residual(self, mode: int = 0):
        """Ritz residuals: 0 cost model, 1 rotate HX with X, 2 apply Htilde again."""
        self._check(self._lib.chfsi_set_rr_residual(self._h, int(mode)), "set_rr_residual")
        return self

    def set_timing(self, enable: bool = True):
        self._check(self._lib.chfsi_set_timing(self._h, 1 if enable else 0), "set_timing")

    def reset_timing(self):
        self._check(self._lib.chfsi_reset_timing(self._h), "reset_timing")

    def filter_timing(self):
        ms, n, cv = C.c_double(), C.c_int(), C.c_int64()
        self._check(self._lib.chfsi_last_filter_timing(self._h, C.byref(ms), C.byref(n), C.byref(cv)),
                    "last_filter_timing")
        return dict(ms=ms.value, launches=n.value, cell_vecs=cv.value)
