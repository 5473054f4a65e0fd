"""ctypes binding of libtmamg.so (the C ABI in include/tmamg.h).

Argument marshalling only: device buffers are torch tensors (complex128,
canonical layouts), streams are torch streams; every computation runs in
the HIP library.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
# TMAMG_LIB selects another build of the library (same ABI)
LIB_PATH = os.environ.get("TMAMG_LIB", os.path.join(HERE, "libtmamg.so"))

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, ENUMERIC, ESTATE = 0, 1, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
STORE_FP64, STORE_FP32, STORE_BF16, STORE_FP16 = 0, 1, 2, 3
(OP_D64, OP_D32, OP_PROLONG, OP_RESTRICT, OP_DC, OP_SAP, OP_PREC, OP_COARSEST, OP_SCHUR64, OP_SCHUR32, OP_DDAG64,
 OP_DDAG32, OP_DCND, OP_SAPND) = range(14)

EXPORTS = [
    "tmamg_default_params", "tmamg_create", "tmamg_setup", "tmamg_setup_update", "tmamg_solve",
    "tmamg_solve_shifted", "tmamg_force", "tmamg_force_from_fields", "tmamg_apply",
    "tmamg_debug_set_test_vectors", "tmamg_debug_export", "tmamg_level_info", "tmamg_destroy",
    "tmamg_time_kernel", "tmamg_last_error", "tmamg_autotune", "tmamg_tune_load", "tmamg_tune_save",
    "tmamg_tune_set", "tmamg_tune_get", "tmamg_tune_entries", "tmamg_tune_clear", "tmamg_force_link_gradient",
    "tmamg_solve_nd", "tmamg_solve_guess", "tmamg_debug_inject", "tmamg_solve_multishift", "tmamg_force_at",
    "tmamg_gauge_force", "tmamg_md_update_links", "tmamg_md_update_momenta", "tmamg_md_kinetic", "tmamg_solve_eo", "tmamg_force_from_fields_noalloc",
]
K_DSLASH32, K_DSLASH64, K_SAP0, K_RESTRICT0, K_PROLONG0, K_DC1, K_DC2, K_SAP1, K_COPY, K_SCHUR32 = range(10)
TUNE_COARSE_APPLY, TUNE_SAP1, TUNE_RESTRICT0, TUNE_PROLONG0, TUNE_SAP0 = range(5)


class Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("t_antiperiodic", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [
        ("nlevels", ctypes.c_int),
        ("agg", (ctypes.c_int * 4) * 2),
        ("nv", ctypes.c_int * 2),
        ("setup_iters", ctypes.c_int),
        ("init_smooth", ctypes.c_int),
        ("sap_block1", ctypes.c_int * 4),
        ("sap_sweeps", ctypes.c_int * 2),
        ("mr_steps", ctypes.c_int),
        ("l2_iters", ctypes.c_int),
        ("l2_tol", ctypes.c_double),
        ("coarsest_iters", ctypes.c_int),
        ("coarsest_tol", ctypes.c_double),
        ("restart", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("storage", ctypes.c_int),
        ("inner_tol", ctypes.c_double),
        ("seed", ctypes.c_ulonglong),
        ("use_graph", ctypes.c_int),
        ("nd_coarse_coupling", ctypes.c_int),
        ("setup_chunk", ctypes.c_int),
        ("keep_test_vectors", ctypes.c_int),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("outer_iters", ctypes.c_int),
        ("cycles", ctypes.c_int),
        ("true_rel_resid", ctypes.c_double),
        ("t_setup_s", ctypes.c_double),
        ("t_solve_s", ctypes.c_double),
        ("l2_iters_total", ctypes.c_longlong),
        ("coarsest_iters_total", ctypes.c_longlong),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libtmamg.so; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run paper_1710_06198_amd.build (or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    lib.tmamg_default_params.argtypes = [P(Params)]
    lib.tmamg_create.argtypes = [P(vp), P(Lattice), P(Params), vp, P(Allocator)]
    lib.tmamg_setup.argtypes = [vp, vp, d, d, d]
    lib.tmamg_setup_update.argtypes = [vp, vp, i]
    lib.tmamg_solve.argtypes = [vp, vp, vp, i, P(d), d, P(Info)]
    lib.tmamg_solve_guess.argtypes = [vp, vp, vp, i, P(d), d, P(Info)]
    lib.tmamg_solve_shifted.argtypes = [vp, vp, vp, i, P(d), d, P(Info)]
    lib.tmamg_solve_multishift.argtypes = [vp, vp, vp, i, P(d), d, P(Info)]
    lib.tmamg_solve_eo.argtypes = [vp, vp, vp, i, P(d), d, P(Info)]
    lib.tmamg_debug_inject.argtypes = [vp, i]
    lib.tmamg_force.argtypes = [vp, vp, vp, P(d), d, P(Info)]
    lib.tmamg_force_at.argtypes = [vp, vp, d, vp, P(d), d, P(Info)]
    lib.tmamg_gauge_force.argtypes = [vp, vp, d, vp, P(d)]
    lib.tmamg_md_update_links.argtypes = [vp, vp, vp, d]
    lib.tmamg_md_update_momenta.argtypes = [vp, vp, vp, d]
    lib.tmamg_md_kinetic.argtypes = [vp, vp, P(d)]
    lib.tmamg_solve_nd.argtypes = [vp, vp, vp, d, d, d, P(Info)]
    lib.tmamg_force_from_fields.argtypes = [vp, vp, vp, vp]
    lib.tmamg_force_from_fields_noalloc.argtypes = [vp, vp, vp, vp]
    lib.tmamg_force_link_gradient.argtypes = [vp, vp, vp, d]
    lib.tmamg_apply.argtypes = [vp, i, i, vp, vp, i, P(d)]
    lib.tmamg_debug_set_test_vectors.argtypes = [vp, i, vp]
    lib.tmamg_debug_export.argtypes = [vp, i, i, vp]
    lib.tmamg_level_info.argtypes = [vp, i, P(ctypes.c_long), P(i)]
    lib.tmamg_time_kernel.argtypes = [vp, i, i, i, P(d)]
    lib.tmamg_destroy.argtypes = [vp]
    lib.tmamg_destroy.restype = None
    lib.tmamg_last_error.restype = ctypes.c_char_p
    cs, lg = ctypes.c_char_p, ctypes.c_long
    lib.tmamg_autotune.argtypes = [vp, P(i), i, i, cs]
    lib.tmamg_tune_load.argtypes = [cs, P(i)]
    lib.tmamg_tune_save.argtypes = [cs]
    lib.tmamg_tune_set.argtypes = [i, lg, lg, lg, i]
    lib.tmamg_tune_get.argtypes = [i, lg, lg, lg]
    lib.tmamg_tune_entries.argtypes = []
    lib.tmamg_tune_clear.argtypes = []
    lib.tmamg_tune_clear.restype = None
    for nm in EXPORTS:
        if nm not in ("tmamg_destroy", "tmamg_last_error", "tmamg_tune_clear"):
            getattr(lib, nm).restype = ctypes.c_int
    _lib = lib
    return lib


class TmamgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tmamg status {status}: {msg}")
        self.status = status


def _check(status):
    if status < 0:
        raise TmamgError(status, load().tmamg_last_error().decode())
    return status


def default_params(**kw) -> Params:
    p = Params()
    _check(load().tmamg_default_params(ctypes.byref(p)))
    for k, v in kw.items():
        if k == "agg":
            for l, a in enumerate(v):
                for m in range(4):
                    p.agg[l][m] = a[m]
        elif k in ("nv", "sap_sweeps", "sap_block1"):
            arr = getattr(p, k)
            for j, x in enumerate(v):
                arr[j] = x
        else:
            setattr(p, k, v)
    return p


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dvec(vals):
    if vals is None:
        return None
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr


def check_field(name, t, count, device):
    """Validate a buffer handed to the library: a complex128, contiguous
    tensor of `count` elements on `device`.  The C ABI takes raw pointers, so
    a wrong dtype or size would be read or written out of bounds there."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != torch.complex128:
        raise ValueError(f"{name}: dtype must be complex128, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.numel() != count:
        raise ValueError(f"{name}: expected {count} complex elements, got {t.numel()} (shape {tuple(t.shape)})")
    if device is not None and t.device != device:
        raise ValueError(f"{name}: must be on {device}, found {t.device}")


def check_values(name, vals, n):
    if vals is None:
        return
    if len(vals) != n:
        raise ValueError(f"{name}: expected {n} values (one per right-hand side), got {len(vals)}")


# live contexts, closed at interpreter exit before any module is torn down:
# the library's buffers may belong to torch's caching allocator, and no
# device memory is released after the runtimes start finalising
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for s in list(_live):
        try:
            s.close()
        except Exception:
            pass


def torch_allocator(device, stream):
    """A tmamg_allocator backed by torch's caching allocator on `device`,
    stream-ordered on `stream` (device memory then shows up in
    torch.cuda.memory_allocated and is reused by torch after close)."""
    import torch
    dev_index = torch.device(device).index or 0

    def _alloc(nbytes, hip_stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev_index, stream=int(hip_stream or 0))
        except Exception:
            return None

    def _free(ptr, hip_stream, user):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    a = Allocator()
    a.alloc = ALLOC_FN(_alloc)
    a.free = FREE_FN(_free)
    a.user = None
    return a


class Solver:
    """One context of the library.  Buffers are torch complex128 CUDA tensors.

    allocator: "torch" (default) lets torch's caching allocator back every
    internal device buffer; None uses hipMalloc/hipFree inside the library."""

    def __init__(self, dims, params: Params = None, antiperiodic: bool = True, stream=None, allocator="torch"):
        import torch
        lib = load()
        self.lib = lib
        self.dims = tuple(int(d) for d in dims)
        self.params = params if params is not None else default_params()
        lat = Lattice()
        for m in range(4):
            lat.dims[m] = int(dims[m])
        lat.t_antiperiodic = 1 if antiperiodic else 0
        s = stream if stream is not None else torch.cuda.current_stream()
        self._stream = s
        self.device = torch.device("cuda", s.device.index if s.device.index is not None else 0)
        self._alloc = None
        if allocator == "torch":
            self._alloc = torch_allocator(self.device, s)
        elif allocator is not None:
            raise ValueError('allocator must be "torch" or None')
        h = ctypes.c_void_p()
        _check(lib.tmamg_create(ctypes.byref(h), ctypes.byref(lat), ctypes.byref(self.params),
                                ctypes.c_void_p(s.cuda_stream),
                                ctypes.byref(self._alloc) if self._alloc is not None else None))
        self.h = h
        _live.add(self)

    def _ordered(self, fn):
        """fn with the library's stream ordered after the caller's current
        stream (the inputs written there are complete before the library
        reads them) and the caller's stream after the library's (the outputs
        are complete before the caller's next work reads them)."""
        import torch

        def call(*args):
            cur = torch.cuda.current_stream(self.device)
            other = cur.cuda_stream != self._stream.cuda_stream
            if other:
                self._stream.wait_stream(cur)
            try:
                return fn(*args)
            finally:
                if other:
                    cur.wait_stream(self._stream)
        return call

    @property
    def volume(self):
        v = 1
        for d in self.dims:
            v *= d
        return v

    def _spinors(self, name, t, n=None):
        if n is None:
            n = t.shape[0] if hasattr(t, "shape") and len(t.shape) > 0 else 0
        if n < 1:
            raise ValueError(f"{name}: needs a leading right-hand-side axis")
        check_field(name, t, n * self.volume * 12, getattr(self, "device", None))
        return n

    def _links(self, name, t):
        check_field(name, t, 4 * self.volume * 9, getattr(self, "device", None))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.tmamg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # links_version counts the link fields loaded (setup or setup_update),
    # so a gradient can check that the links are still those of its action
    links_version = 0

    def setup(self, U, kappa, csw, mu):
        self._links("U", U)
        _check(self._ordered(self.lib.tmamg_setup)(self.h, _ptr(U), float(kappa), float(csw), float(mu)))
        self.links_version += 1

    def setup_update(self, U, iters=1):
        self._links("U", U)
        _check(self._ordered(self.lib.tmamg_setup_update)(self.h, _ptr(U), int(iters)))
        self.links_version += 1

    def solve(self, b, x, mu_rhs=None, tol=1e-10, guess=False):
        """D(mu_r) x_r = b_r; guess=True starts from the x passed in."""
        n = self._spinors("b", b)
        self._spinors("x", x, n)
        check_values("mu_rhs", mu_rhs, n)
        info = Info()
        fn = self._ordered(self.lib.tmamg_solve_guess if guess else self.lib.tmamg_solve)
        st = fn(self.h, _ptr(b), _ptr(x), n, _dvec(mu_rhs), float(tol), ctypes.byref(info))
        _check(st)
        return info

    def solve_eo(self, b, x, mu_rhs=None, tol=1e-10):
        """Even-odd reduced D_hat x_e = b_e (even sites; odd entries of b
        ignored, odd entries of x set to 0)."""
        n = self._spinors("b", b)
        self._spinors("x", x, n)
        check_values("mu_rhs", mu_rhs, n)
        info = Info()
        st = self._ordered(self.lib.tmamg_solve_eo)(self.h, _ptr(b), _ptr(x), n, _dvec(mu_rhs), float(tol),
                                                     ctypes.byref(info))
        _check(st)
        return info

    def solve_shifted(self, b, x, sigma, tol=1e-10):
        n = self._spinors("b", b)
        self._spinors("x", x, n)
        if sigma is None:
            raise ValueError("sigma: one shift per right-hand side is required")
        check_values("sigma", sigma, n)
        info = Info()
        st = self._ordered(self.lib.tmamg_solve_shifted)(self.h, _ptr(b), _ptr(x), n, _dvec(sigma), float(tol),
                                                          ctypes.byref(info))
        _check(st)
        return info

    def solve_multishift(self, b, x, sigma, tol=1e-10):
        """(D D^dag + sigma_k) x_k = b for one source b [1] and x [len(sigma)],
        with first-order initial guesses around the smallest shift (Sec. 3)."""
        self._spinors("b", b, 1)
        n = self._spinors("x", x)
        if sigma is None:
            raise ValueError("sigma: one shift per solution is required")
        check_values("sigma", sigma, n)
        info = Info()
        fn = self._ordered(self.lib.tmamg_solve_multishift)
        st = fn(self.h, _ptr(b), _ptr(x), n, _dvec(sigma), float(tol), ctypes.byref(info))
        _check(st)
        return info

    def solve_nd(self, b, x, mubar, epsbar, tol=1e-10):
        """Doublet D_ND(mubar, epsbar) x = b (Eq. 2); b, x: complex128 [2][T][Z][Y][X][4][3]."""
        if b.shape[0] != 2 or x.shape[0] != 2:
            raise ValueError("a doublet has two flavours: b and x need a leading axis of 2")
        self._spinors("b", b, 2)
        self._spinors("x", x, 2)
        info = Info()
        fn = self._ordered(self.lib.tmamg_solve_nd)
        st = fn(self.h, _ptr(b), _ptr(x), float(mubar), float(epsbar), float(tol), ctypes.byref(info))
        _check(st)
        return info

    def force(self, phi, F, tol=1e-12):
        self._spinors("phi", phi, 1)
        self._links("F", F)
        info = Info()
        S = ctypes.c_double()
        _check(self._ordered(self.lib.tmamg_force)(self.h, _ptr(phi), _ptr(F), ctypes.byref(S), float(tol),
                                                    ctypes.byref(info)))
        return S.value, info

    def force_at(self, phi, mu, F, tol=1e-12):
        """tmamg_force at twisted mass mu: S_f = phi^dag (D(mu) D(mu)^dag)^-1 phi and its force."""
        self._spinors("phi", phi, 1)
        self._links("F", F)
        info = Info()
        S = ctypes.c_double()
        fn = self._ordered(self.lib.tmamg_force_at)
        _check(fn(self.h, _ptr(phi), float(mu), _ptr(F), ctypes.byref(S), float(tol), ctypes.byref(info)))
        return S.value, info

    def gauge_force(self, U, beta, F):
        """Wilson plaquette action S_g (returned) and its force into F."""
        self._links("U", U)
        self._links("F", F)
        S = ctypes.c_double()
        _check(self._ordered(self.lib.tmamg_gauge_force)(self.h, _ptr(U), float(beta), _ptr(F), ctypes.byref(S)))
        return S.value

    def md_update_links(self, U, P, eps):
        self._links("U", U)
        self._links("P", P)
        _check(self._ordered(self.lib.tmamg_md_update_links)(self.h, _ptr(U), _ptr(P), float(eps)))

    def md_update_momenta(self, P, F, coef):
        self._links("P", P)
        self._links("F", F)
        _check(self._ordered(self.lib.tmamg_md_update_momenta)(self.h, _ptr(P), _ptr(F), float(coef)))

    def md_kinetic(self, P):
        self._links("P", P)
        K = ctypes.c_double()
        _check(self._ordered(self.lib.tmamg_md_kinetic)(self.h, _ptr(P), ctypes.byref(K)))
        return K.value

    def force_from_fields(self, X, Y, F):
        self._spinors("X", X, 1)
        self._spinors("Y", Y, 1)
        self._links("F", F)
        _check(self._ordered(self.lib.tmamg_force_from_fields)(self.h, _ptr(X), _ptr(Y), _ptr(F)))

    def force_from_fields_noalloc(self, X, Y, F):
        """force_from_fields without any device allocation: the library's
        static per-GPU scratch array (at most 134,432 sites; calls that
        overlap on one GPU race)."""
        self._spinors("X", X, 1)
        self._spinors("Y", Y, 1)
        self._links("F", F)
        _check(self._ordered(self.lib.tmamg_force_from_fields_noalloc)(self.h, _ptr(X), _ptr(Y), _ptr(F)))

    def force_link_gradient(self, F, G, scale=1.0):
        self._links("F", F)
        self._links("G", G)
        _check(self._ordered(self.lib.tmamg_force_link_gradient)(self.h, _ptr(F), _ptr(G), float(scale)))

    def apply(self, op, level, inp, out, mu_rhs=None):
        n = inp.shape[0]
        lin = lout = int(level)
        if op == OP_PROLONG:
            lout = lin - 1
        elif op == OP_RESTRICT:
            lout = lin + 1
        sin, din = self.level_info(lin)
        sout, dout = self.level_info(lout)
        check_field("in", inp, n * sin * din, self.device)
        check_field("out", out, n * sout * dout, self.device)
        if op not in (OP_DCND, OP_SAPND):
            check_values("mu_rhs", mu_rhs, n)
        elif mu_rhs is None or len(mu_rhs) != 2 or n != 2:
            raise ValueError("doublet operators: two flavours and mu_rhs = (mubar, epsbar)")
        _check(self._ordered(self.lib.tmamg_apply)(self.h, int(op), int(level), _ptr(inp), _ptr(out), n, _dvec(mu_rhs)))

    def set_test_vectors(self, level, v):
        if level == 0:
            check_field("v", v, self.params.nv[0] * self.volume * 12, self.device)
        else:
            s1, d1 = self.level_info(1)
            check_field("v", v, self.params.nv[1] * s1 * d1, self.device)
        _check(self._ordered(self.lib.tmamg_debug_set_test_vectors)(self.h, int(level), _ptr(v)))

    def export(self, what, level, out):
        if what == 0:
            sf, df = self.level_info(level)
            check_field("out", out, self.params.nv[level] * sf * df, self.device)
        else:
            sc, dc = self.level_info(level)
            check_field("out", out, sc * 9 * dc * dc, self.device)
        _check(self._ordered(self.lib.tmamg_debug_export)(self.h, int(what), int(level), _ptr(out)))

    def inject_barrier_timeout(self):
        """Failure-path hook: the next solve reports TMAMG_EHIP and the
        context falls back to the generic coarse kernels."""
        _check(self._ordered(self.lib.tmamg_debug_inject)(self.h, 0))

    def time_kernel(self, kernel, nrhs=1, reps=20):
        ms = ctypes.c_double()
        _check(self._ordered(self.lib.tmamg_time_kernel)(self.h, int(kernel), int(nrhs), int(reps), ctypes.byref(ms)))
        return ms.value

    def autotune(self, nrhs_list, reps=5, json_path=None):
        """Time both variants of every tunable kernel family at these
        right-hand-side counts and keep the faster in the variant table."""
        arr = (ctypes.c_int * len(nrhs_list))(*[int(n) for n in nrhs_list])
        fn = self._ordered(self.lib.tmamg_autotune)
        _check(fn(self.h, arr, len(nrhs_list), int(reps), None if json_path is None else os.fsencode(json_path)))

    def level_info(self, level):
        s, d = ctypes.c_long(), ctypes.c_int()
        _check(self.lib.tmamg_level_info(self.h, int(level), ctypes.byref(s), ctypes.byref(d)))
        return s.value, d.value


# ---- process-wide kernel variant table (see tmamg_tune_* in include/tmamg.h)
def tune_load(path) -> int:
    n = ctypes.c_int()
    _check(load().tmamg_tune_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def tune_save(path):
    _check(load().tmamg_tune_save(os.fsencode(path)))


def tune_set(family, a, b, nrhs, variant):
    _check(load().tmamg_tune_set(int(family), int(a), int(b), int(nrhs), int(variant)))


def tune_get(family, a, b, nrhs) -> int:
    return load().tmamg_tune_get(int(family), int(a), int(b), int(nrhs))


def tune_entries() -> int:
    return load().tmamg_tune_entries()


def tune_clear():
    load().tmamg_tune_clear()
