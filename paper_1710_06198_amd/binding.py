"""ctypes binding of libtmamg.so (the C ABI in include/tmamg.h).

Argument marshalling only: device buffers are torch tensors (complex128,
canonical layouts), streams are torch streams; every computation runs in
the HIP library.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TMAMG_LIB selects another build of the library (same ABI)
LIB_PATH = os.environ.get("TMAMG_LIB", os.path.join(HERE, "libtmamg.so"))

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, ENUMERIC, ESTATE = 0, 1, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
STORE_FP64, STORE_FP32, STORE_BF16, STORE_FP16 = 0, 1, 2, 3
OP_D64, OP_D32, OP_PROLONG, OP_RESTRICT, OP_DC, OP_SAP, OP_PREC, OP_COARSEST, OP_SCHUR64, OP_SCHUR32 = range(10)

EXPORTS = [
    "tmamg_default_params", "tmamg_create", "tmamg_setup", "tmamg_setup_update", "tmamg_solve",
    "tmamg_solve_shifted", "tmamg_force", "tmamg_force_from_fields", "tmamg_apply",
    "tmamg_debug_set_test_vectors", "tmamg_debug_export", "tmamg_level_info", "tmamg_destroy",
    "tmamg_time_kernel", "tmamg_last_error", "tmamg_autotune", "tmamg_tune_load", "tmamg_tune_save",
    "tmamg_tune_set", "tmamg_tune_get", "tmamg_tune_entries", "tmamg_tune_clear", "tmamg_force_link_gradient",
    "tmamg_solve_nd",
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
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("outer_iters", ctypes.c_int),
        ("cycles", ctypes.c_int),
        ("true_rel_resid", ctypes.c_double),
        ("t_setup_s", ctypes.c_double),
        ("t_solve_s", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


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
    lib.tmamg_create.argtypes = [P(vp), P(Lattice), P(Params), vp]
    lib.tmamg_setup.argtypes = [vp, vp, d, d, d]
    lib.tmamg_setup_update.argtypes = [vp, vp, i]
    lib.tmamg_solve.argtypes = [vp, vp, vp, i, P(d), d, P(Info)]
    lib.tmamg_solve_shifted.argtypes = [vp, vp, vp, i, P(d), d, P(Info)]
    lib.tmamg_force.argtypes = [vp, vp, vp, P(d), d, P(Info)]
    lib.tmamg_solve_nd.argtypes = [vp, vp, vp, d, d, d, P(Info)]
    lib.tmamg_force_from_fields.argtypes = [vp, vp, vp, vp]
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


class Solver:
    """One context of the library.  Buffers are torch complex128 CUDA tensors."""

    def __init__(self, dims, params: Params = None, antiperiodic: bool = True, stream=None):
        import torch
        lib = load()
        self.lib = lib
        self.dims = tuple(dims)
        self.params = params if params is not None else default_params()
        lat = Lattice()
        for m in range(4):
            lat.dims[m] = int(dims[m])
        lat.t_antiperiodic = 1 if antiperiodic else 0
        s = stream if stream is not None else torch.cuda.current_stream()
        self._stream = s
        h = ctypes.c_void_p()
        _check(lib.tmamg_create(ctypes.byref(h), ctypes.byref(lat), ctypes.byref(self.params),
                                ctypes.c_void_p(s.cuda_stream)))
        self.h = h

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
        _check(self.lib.tmamg_setup(self.h, _ptr(U), float(kappa), float(csw), float(mu)))
        self.links_version += 1

    def setup_update(self, U, iters=1):
        _check(self.lib.tmamg_setup_update(self.h, _ptr(U), int(iters)))
        self.links_version += 1

    def solve(self, b, x, mu_rhs=None, tol=1e-10):
        info = Info()
        n = b.shape[0]
        st = self.lib.tmamg_solve(self.h, _ptr(b), _ptr(x), n, _dvec(mu_rhs), float(tol), ctypes.byref(info))
        _check(st)
        return info

    def solve_shifted(self, b, x, sigma, tol=1e-10):
        info = Info()
        st = self.lib.tmamg_solve_shifted(self.h, _ptr(b), _ptr(x), b.shape[0], _dvec(sigma), float(tol),
                                          ctypes.byref(info))
        _check(st)
        return info

    def solve_nd(self, b, x, mubar, epsbar, tol=1e-10):
        """Doublet D_ND(mubar, epsbar) x = b (Eq. 2); b, x: complex128 [2][T][Z][Y][X][4][3]."""
        if b.shape[0] != 2 or x.shape[0] != 2:
            raise ValueError("a doublet has two flavours: b and x need a leading axis of 2")
        info = Info()
        st = self.lib.tmamg_solve_nd(self.h, _ptr(b), _ptr(x), float(mubar), float(epsbar), float(tol),
                                     ctypes.byref(info))
        _check(st)
        return info

    def force(self, phi, F, tol=1e-12):
        info = Info()
        S = ctypes.c_double()
        _check(self.lib.tmamg_force(self.h, _ptr(phi), _ptr(F), ctypes.byref(S), float(tol), ctypes.byref(info)))
        return S.value, info

    def force_from_fields(self, X, Y, F):
        _check(self.lib.tmamg_force_from_fields(self.h, _ptr(X), _ptr(Y), _ptr(F)))

    def force_link_gradient(self, F, G, scale=1.0):
        _check(self.lib.tmamg_force_link_gradient(self.h, _ptr(F), _ptr(G), float(scale)))

    def apply(self, op, level, inp, out, mu_rhs=None):
        _check(self.lib.tmamg_apply(self.h, int(op), int(level), _ptr(inp), _ptr(out), inp.shape[0],
                                    _dvec(mu_rhs)))

    def set_test_vectors(self, level, v):
        _check(self.lib.tmamg_debug_set_test_vectors(self.h, int(level), _ptr(v)))

    def export(self, what, level, out):
        _check(self.lib.tmamg_debug_export(self.h, int(what), int(level), _ptr(out)))

    def time_kernel(self, kernel, nrhs=1, reps=20):
        ms = ctypes.c_double()
        _check(self.lib.tmamg_time_kernel(self.h, int(kernel), int(nrhs), int(reps), ctypes.byref(ms)))
        return ms.value

    def autotune(self, nrhs_list, reps=5, json_path=None):
        """Time both variants of every tunable kernel family at these
        right-hand-side counts and keep the faster in the variant table."""
        arr = (ctypes.c_int * len(nrhs_list))(*[int(n) for n in nrhs_list])
        _check(self.lib.tmamg_autotune(self.h, arr, len(nrhs_list), int(reps),
                                       None if json_path is None else os.fsencode(json_path)))

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
