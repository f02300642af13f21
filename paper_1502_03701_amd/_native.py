"""ctypes binding of libsa (include/sa.h).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  PyTorch provides
device memory (tensors) and the stream.

The library must have been built (``python -m paper_1502_03701_amd.build``);
loading fails loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsa.so")

SA_OK = 0
SA_NOT_CONVERGED = 1
SA_EINVAL = -1
SA_ENOMEM = -2
SA_EDEVICE = -3
SA_ESINGULAR = -4
SA_ENONFINITE = -5
SA_ESTATE = -6

SA_F64, SA_F32, SA_MIXED = 0, 1, 2
SA_BC_PERIODIC, SA_BC_WALL = 0, 1

EXPORTED = ["sa_create", "sa_destroy", "sa_last_error", "sa_version", "sa_base_set",
            "sa_op_apply", "sa_precond_setup", "sa_precond_apply", "sa_gmres_solve",
            "sa_arnoldi_eigs", "sa_set_jv_variant", "sa_get_jv_variant", "sa_gmres_solve_noalloc"]

# bytes of the device scratch array behind sa_gmres_solve_noalloc
NOALLOC_SCRATCH_BYTES = 64 << 20

# operator kernel variants (sa_jv_variant)
JV_VARIANTS = ["prefetch_z32", "prefetch_z16", "stage_z16", "stage_z32", "prefetch_z4", "prefetch_z1", "stage_z4",
               "stage_z1", "iso_z32", "iso_z16", "iso_z4", "iso_z1"]


class Problem(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("len", C.c_double * 3),
                ("bc_y", C.c_int), ("mach", C.c_double), ("re", C.c_double),
                ("pr", C.c_double), ("gamma", C.c_double), ("sutherland", C.c_double),
                ("scheme", C.c_int), ("stretch", C.c_double)]


class GmresOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("tol", C.c_double), ("max_matvec", C.c_long),
                ("use_precond", C.c_int), ("prec", C.c_int), ("inner_tol", C.c_double),
                ("max_outer", C.c_int), ("use_graph", C.c_int), ("augment", C.c_int)]


class GmresInfo(C.Structure):
    _fields_ = [("iters", C.c_long), ("matvecs", C.c_long), ("precond_applies", C.c_long),
                ("cycles", C.c_int), ("outer", C.c_int), ("relres", C.c_double),
                ("status", C.c_int)]


SA_PC_BLOCK_JACOBI, SA_PC_MEAN_FLOW = 0, 1


class PrecondOpts(C.Structure):
    _fields_ = [("bx", C.c_int), ("by", C.c_int), ("bz", C.c_int), ("diag_add", C.c_double),
                ("noise_std", C.c_double), ("seed", C.c_ulonglong), ("factor_prec", C.c_int),
                ("kind", C.c_int)]


class EigOpts(C.Structure):
    _fields_ = [("nev", C.c_int), ("ncv", C.c_int), ("sigma", C.c_double), ("mu", C.c_double),
                ("tol", C.c_double), ("max_restarts", C.c_int), ("lin", GmresOpts)]


class EigResult(C.Structure):
    _fields_ = [("nconv", C.c_int), ("restarts", C.c_int), ("n_cayley", C.c_long),
                ("n_matvec", C.c_long), ("n_precond", C.c_long),
                ("lam_re", C.c_double * 32), ("lam_im", C.c_double * 32),
                ("theta_re", C.c_double * 32), ("theta_im", C.c_double * 32),
                ("ritz_est", C.c_double * 32), ("resid", C.c_double * 32),
                ("evec_re_dev", C.c_void_p), ("evec_im_dev", C.c_void_p),
                ("wall_seconds", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libsa.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libsa.so is not built (%s); run python -m paper_1502_03701_amd.build" % path)
    lib = C.CDLL(path)
    vp, ip, dp = C.c_void_p, C.c_int, C.c_double
    lib.sa_create.argtypes = [C.POINTER(vp), vp]
    lib.sa_create.restype = ip
    lib.sa_destroy.argtypes = [vp]
    lib.sa_destroy.restype = None
    lib.sa_last_error.argtypes = [vp]
    lib.sa_last_error.restype = C.c_char_p
    lib.sa_version.argtypes = []
    lib.sa_version.restype = C.c_char_p
    lib.sa_base_set.argtypes = [vp, C.POINTER(Problem), vp]
    lib.sa_base_set.restype = ip
    lib.sa_op_apply.argtypes = [vp, ip, ip, vp, vp, dp]
    lib.sa_op_apply.restype = ip
    lib.sa_precond_setup.argtypes = [vp, C.POINTER(PrecondOpts), ip, C.POINTER(dp)]
    lib.sa_precond_setup.restype = ip
    lib.sa_precond_apply.argtypes = [vp, ip, ip, ip, vp, vp]
    lib.sa_precond_apply.restype = ip
    lib.sa_gmres_solve.argtypes = [vp, C.POINTER(GmresOpts), ip, C.POINTER(dp), vp, vp,
                                   C.POINTER(GmresInfo)]
    lib.sa_gmres_solve.restype = ip
    lib.sa_gmres_solve_noalloc.argtypes = lib.sa_gmres_solve.argtypes
    lib.sa_gmres_solve_noalloc.restype = ip
    lib.sa_arnoldi_eigs.argtypes = [C.POINTER(vp), ip, C.POINTER(EigOpts), C.POINTER(vp),
                                    C.POINTER(EigResult)]
    lib.sa_arnoldi_eigs.restype = ip
    lib.sa_set_jv_variant.argtypes = [vp, ip, ip]
    lib.sa_set_jv_variant.restype = ip
    lib.sa_get_jv_variant.argtypes = [vp, ip, C.POINTER(C.c_float)]
    lib.sa_get_jv_variant.restype = ip
    _lib = lib
    return lib


class SAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libsa error %d: %s" % (code, msg))
        self.code = code


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _check_dev(t, dtype=None, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected dtype %s, got %s" % (dtype, t.dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("tensor too small: %d < %d" % (t.numel(), numel))


def make_problem(prob) -> Problem:
    """From a synth.Problem-like object (ndim, n, length, bc, mach, re, pr,
    gamma, sutherland, optional scheme)."""
    p = Problem()
    p.ndim = prob.ndim
    for a in range(3):
        p.n[a] = prob.n[a]
        p.len[a] = prob.length[a]
    p.bc_y = prob.bc[1]
    p.mach, p.re, p.pr = prob.mach, prob.re, prob.pr
    p.gamma, p.sutherland = prob.gamma, prob.sutherland
    p.scheme = getattr(prob, "scheme", 0)
    p.stretch = float(getattr(prob, "stretch", 0.0))
    return p


class Context:
    """One libsa context bound to a torch stream (default: the current one)."""

    def __init__(self, stream=None):
        import torch
        self.lib = load()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = self.lib.sa_create(C.byref(h), C.c_void_p(self.stream.cuda_stream))
        if rc != SA_OK:
            raise SAError(rc, "sa_create failed")
        self.h = h
        self.prob = None
        self._pc = False

    def close(self):
        if getattr(self, "h", None):
            self.lib.sa_destroy(self.h)
            self.h = None

    __del__ = close

    def _err(self, rc):
        if rc < 0:
            raise SAError(rc, self.lib.sa_last_error(self.h).decode())
        return rc

    @property
    def ndof(self):
        return self.prob.ndof

    def base_set(self, prob, q0):
        import torch
        _check_dev(q0, torch.float64, prob.ndof)
        self.prob = prob
        self._p = make_problem(prob)
        self._pc = False
        return self._err(self.lib.sa_base_set(self.h, C.byref(self._p), _ptr(q0)))

    def has_precond(self):
        """Whether block-Jacobi factors are set up for the current base state."""
        return self._pc

    def op_apply(self, x, y, shift=0.0, nrhs=1):
        import torch
        prec = SA_F64 if x.dtype == torch.float64 else SA_F32
        _check_dev(x, x.dtype, nrhs * self.ndof)
        _check_dev(y, x.dtype, nrhs * self.ndof)
        return self._err(self.lib.sa_op_apply(self.h, prec, nrhs, _ptr(x), _ptr(y), float(shift)))

    def set_jv_variant(self, prec, variant):
        """Pin the operator kernel variant of a precision (-1: unpin)."""
        return self._err(self.lib.sa_set_jv_variant(self.h, prec, variant))

    def jv_variant(self, prec=SA_F64):
        """(variant in use, {variant name: measured us per launch})."""
        t = (C.c_float * len(JV_VARIANTS))()
        v = self.lib.sa_get_jv_variant(self.h, prec, t)
        return v, {n: float(t[i]) for i, n in enumerate(JV_VARIANTS)}

    def precond_setup(self, shifts, bx=4, by=4, bz=1, diag_add=0.1, noise_std=0.01, seed=3,
                      factor_prec=SA_F32, kind=SA_PC_BLOCK_JACOBI):
        """kind: SA_PC_BLOCK_JACOBI (the block fields apply) or SA_PC_MEAN_FLOW."""
        o = PrecondOpts(bx, by, bz, diag_add, noise_std, seed, factor_prec, kind)
        arr = (C.c_double * len(shifts))(*shifts)
        self._pc = False
        rc = self._err(self.lib.sa_precond_setup(self.h, C.byref(o), len(shifts), arr))
        self._pc = True
        return rc

    def precond_apply(self, ishift, r, z, nrhs=1):
        import torch
        prec = SA_F64 if r.dtype == torch.float64 else SA_F32
        _check_dev(r, r.dtype, nrhs * self.ndof)
        _check_dev(z, r.dtype, nrhs * self.ndof)
        return self._err(self.lib.sa_precond_apply(self.h, prec, ishift, nrhs, _ptr(r), _ptr(z)))

    def gmres_solve(self, sigmas, b, x, restart=40, tol=1e-10, max_matvec=10 ** 6,
                    use_precond=False, prec=SA_F64, inner_tol=1e-4, max_outer=10, use_graph=True, augment=0,
                    noalloc=False):
        """augment = k > 0: LGMRES(restart, k).  noalloc: call
        sa_gmres_solve_noalloc (workspace in the library's static scratch,
        no device allocation; use_graph is then ignored)."""
        import torch
        ns = len(sigmas)
        dt = torch.float32 if prec == SA_F32 else torch.float64
        _check_dev(b, dt, ns * self.ndof)
        _check_dev(x, dt, ns * self.ndof)
        o = GmresOpts(restart, tol, max_matvec, 1 if use_precond else 0, prec, inner_tol, max_outer,
                      1 if use_graph else 0, augment)
        infos = (GmresInfo * ns)()
        arr = (C.c_double * ns)(*sigmas)
        fn = self.lib.sa_gmres_solve_noalloc if noalloc else self.lib.sa_gmres_solve
        rc = self._err(fn(self.h, C.byref(o), ns, arr, _ptr(b), _ptr(x), infos))
        return rc, [dict(iters=i.iters, matvecs=i.matvecs, precond_applies=i.precond_applies,
                         cycles=i.cycles, outer=i.outer, relres=i.relres, status=i.status)
                    for i in infos]


def arnoldi_eigs(ctxs, v0s, nev=6, ncv=30, sigma=0.2, mu=-0.2, tol=1e-10, max_restarts=500,
                 restart=40, lin_tol=1e-12, max_matvec=10 ** 7, use_precond=False, prec=SA_F64,
                 inner_tol=1e-4, max_outer=10, evecs=None, use_graph=True, augment=0):
    """Leading eigenpairs for several problems (one context each).  evecs: optional
    list of (re, im) device float64 tensors of nev*n entries per problem.
    Contexts on one shared stream run in turn; contexts on pairwise distinct
    streams run concurrently."""
    import torch
    lib = load()
    npb = len(ctxs)
    o = EigOpts(nev, ncv, sigma, mu, tol, max_restarts,
                GmresOpts(restart, lin_tol, max_matvec, 1 if use_precond else 0, prec, inner_tol,
                          max_outer, 1 if use_graph else 0, augment))
    hs = (C.c_void_p * npb)(*[c.h for c in ctxs])
    for c, v in zip(ctxs, v0s):
        _check_dev(v, torch.float64, c.ndof)
    vs = (C.c_void_p * npb)(*[v.data_ptr() for v in v0s])
    res = (EigResult * npb)()
    if evecs is not None:
        for r, (re, im) in zip(res, evecs):
            r.evec_re_dev = re.data_ptr()
            r.evec_im_dev = im.data_ptr()
    rc = lib.sa_arnoldi_eigs(hs, npb, C.byref(o), vs, res)
    if rc < 0:
        raise SAError(rc, lib.sa_last_error(ctxs[0].h).decode())
    out = []
    for r in res:
        k = nev
        out.append(dict(nconv=r.nconv, restarts=r.restarts, n_cayley=r.n_cayley,
                        n_matvec=r.n_matvec, n_precond=r.n_precond,
                        lam=[complex(r.lam_re[i], r.lam_im[i]) for i in range(k)],
                        theta=[complex(r.theta_re[i], r.theta_im[i]) for i in range(k)],
                        ritz_est=[r.ritz_est[i] for i in range(k)],
                        resid=[r.resid[i] for i in range(k)], seconds=r.wall_seconds))
    return rc, out
