"""ctypes binding of libpbcjk.so (include/pbcjk.h): argument marshalling only.

Every step of a build runs in the HIP library; this module only converts
numpy arrays and torch device tensors into pointers.  Loading fails loudly
when the built library is missing (run __graft_entry__.build()).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_long, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbcjk.so")

PBC_JK_OK = 0
PBC_JK_EINVAL = -1
PBC_JK_ENOMEM = -2
PBC_JK_EDEVICE = -3
PBC_JK_ENOTSUP = -4
PBC_JK_ECANCELED = -5
PBC_JK_EBUSY = -6
PART_SR, PART_LR, PART_SELF = 1, 2, 4
SERVE_ARRIVAL, SERVE_DEADLINE = 0, 1
LR_AUTO, LR_DENSE = 0, 1

# every symbol the header declares
EXPORTS = ["pbc_jk_create", "pbc_jk_build", "pbc_jk_build_device", "pbc_jk_build_device_static",
           "pbc_jk_one_electron", "pbc_jk_destroy",
           "pbc_jk_nbf", "pbc_jk_stats", "pbc_jk_set_graph", "pbc_jk_set_parts", "pbc_jk_set_sr_classes", "pbc_jk_set_lr", "pbc_jk_last_error",
           "pbc_jk_server_create", "pbc_jk_server_submit", "pbc_jk_server_wait", "pbc_jk_server_cancel",
           "pbc_jk_server_stats", "pbc_jk_server_destroy"]


class pbc_cell(ctypes.Structure):
    _fields_ = [("a", c_double * 9)]


class pbc_atoms(ctypes.Structure):
    _fields_ = [("natom", c_int), ("xyz", POINTER(c_double)), ("charge", POINTER(c_double))]


class pbc_basis(ctypes.Structure):
    _fields_ = [("nshell", c_int), ("atom", POINTER(c_int)), ("l", POINTER(c_int)),
                ("pure", POINTER(c_int)), ("nprim", POINTER(c_int)),
                ("exps", POINTER(c_double)), ("coefs", POINTER(c_double))]


class pbc_jk_thresholds(ctypes.Structure):
    _fields_ = [("pair_R", c_double), ("pair_cs", c_double), ("ewald_R", c_double),
                ("ewald_K", c_double), ("schwarz", c_double), ("fp32_below", c_double),
                ("r_cut", c_double), ("g_cut", c_double)]


class pbc_jk_counters(ctypes.Structure):
    _fields_ = [("nbf", c_int), ("nbf_cart", c_int), ("n_pairs", c_long), ("n_groups", c_long),
                ("n_gvec", c_int), ("omega", c_double), ("quartets", c_double),
                ("terms", c_double), ("terms_fp32", c_double), ("t_setup_ms", c_double),
                ("t_build_ms", c_double), ("t_sr_ms", c_double), ("t_lr_ms", c_double),
                ("t_other_ms", c_double), ("t_gemm_ms", c_double), ("gemm_flops", c_double),
                ("n_gemm", c_int), ("t_sfac_ms", c_double), ("terms_class", c_double * 21),
                ("n_group_pairs", c_double), ("lr_rank", c_double), ("t_chol_ms", c_double),
                ("gemm_kernel", c_int), ("t_sr_class_ms", c_double * 21), ("t_y_ms", c_double),
                ("y_flops", c_double), ("n_y", c_int), ("sr_fold_mask", c_int),
                ("sr_kernel_mask", c_int), ("sr_jengine_mask", c_int), ("y_kernel", c_int)]


class pbc_jk_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("slots", c_int), ("cache_cells", c_int),
                ("lr_budget_mb", c_double), ("use_graphs", c_int), ("policy", c_int)]


class pbc_jk_request_info(ctypes.Structure):
    _fields_ = [("status", c_int), ("cache_hit", c_int), ("retries", c_int), ("nbf", c_int),
                ("queue_ms", c_double), ("setup_ms", c_double), ("build_ms", c_double),
                ("latency_ms", c_double), ("device_bytes", ctypes.c_size_t), ("error", ctypes.c_char * 160)]


class pbc_jk_server_counters(ctypes.Structure):
    _fields_ = [("submitted", c_long), ("completed", c_long), ("failed", c_long), ("cancelled", c_long),
                ("cache_hits", c_long), ("evictions", c_long), ("retries", c_long), ("slots", c_int),
                ("peak_running", c_int), ("budget", ctypes.c_size_t), ("in_use", ctypes.c_size_t),
                ("peak_in_use", ctypes.c_size_t)]


class PbcJkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pbcjk error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Loads libpbcjk.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    lib.pbc_jk_create.argtypes = [POINTER(pbc_cell), POINTER(pbc_atoms), POINTER(pbc_basis), c_double,
                                  POINTER(pbc_jk_thresholds), POINTER(c_void_p)]
    lib.pbc_jk_create.restype = c_int
    lib.pbc_jk_build.argtypes = [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                 POINTER(c_double), POINTER(c_double)]
    lib.pbc_jk_build.restype = c_int
    lib.pbc_jk_build_device.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double),
                                        POINTER(c_double), c_void_p]
    lib.pbc_jk_build_device.restype = c_int
    lib.pbc_jk_build_device_static.argtypes = lib.pbc_jk_build_device.argtypes
    lib.pbc_jk_build_device_static.restype = c_int
    lib.pbc_jk_one_electron.argtypes = [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                        POINTER(c_double)]
    lib.pbc_jk_one_electron.restype = c_int
    lib.pbc_jk_destroy.argtypes = [c_void_p]
    lib.pbc_jk_destroy.restype = None
    lib.pbc_jk_nbf.argtypes = [c_void_p]
    lib.pbc_jk_nbf.restype = c_int
    lib.pbc_jk_stats.argtypes = [c_void_p, POINTER(pbc_jk_counters)]
    lib.pbc_jk_stats.restype = c_int
    lib.pbc_jk_set_graph.argtypes = [c_void_p, c_int]
    lib.pbc_jk_set_graph.restype = c_int
    lib.pbc_jk_set_parts.argtypes = [c_void_p, c_int]
    lib.pbc_jk_set_parts.restype = c_int
    lib.pbc_jk_set_sr_classes.argtypes = [c_void_p, c_int]
    lib.pbc_jk_set_sr_classes.restype = c_int
    lib.pbc_jk_set_lr.argtypes = [c_void_p, c_int, c_double]
    lib.pbc_jk_set_lr.restype = c_int
    lib.pbc_jk_server_create.argtypes = [POINTER(pbc_jk_server_config), POINTER(c_void_p)]
    lib.pbc_jk_server_create.restype = c_int
    lib.pbc_jk_server_submit.argtypes = [c_void_p, POINTER(pbc_cell), POINTER(pbc_atoms), POINTER(pbc_basis),
                                         c_double, POINTER(pbc_jk_thresholds), POINTER(c_double),
                                         POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                         POINTER(c_double), POINTER(ctypes.c_ulonglong)]
    lib.pbc_jk_server_submit.restype = c_int
    lib.pbc_jk_server_wait.argtypes = [c_void_p, ctypes.c_ulonglong, POINTER(pbc_jk_request_info)]
    lib.pbc_jk_server_wait.restype = c_int
    lib.pbc_jk_server_cancel.argtypes = [c_void_p, ctypes.c_ulonglong]
    lib.pbc_jk_server_cancel.restype = c_int
    lib.pbc_jk_server_stats.argtypes = [c_void_p, POINTER(pbc_jk_server_counters)]
    lib.pbc_jk_server_stats.restype = c_int
    lib.pbc_jk_server_destroy.argtypes = [c_void_p]
    lib.pbc_jk_server_destroy.restype = None
    lib.pbc_jk_last_error.argtypes = []
    lib.pbc_jk_last_error.restype = c_char_p
    lib.pbc_becke_create.argtypes = [POINTER(pbc_cell), c_int, POINTER(c_double), c_double, c_double,
                                     POINTER(c_void_p)]
    lib.pbc_becke_create.restype = c_int
    lib.pbc_becke_weights.argtypes = [c_void_p, ctypes.c_long, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.pbc_becke_weights.restype = c_int
    lib.pbc_becke_info.argtypes = [c_void_p, POINTER(c_int), POINTER(ctypes.c_long)]
    lib.pbc_becke_info.restype = c_int
    lib.pbc_becke_evaluations.argtypes = [c_void_p, POINTER(c_double)]
    lib.pbc_becke_evaluations.restype = c_int
    lib.pbc_becke_destroy.argtypes = [c_void_p]
    lib.pbc_becke_destroy.restype = None
    _lib = lib
    return lib


def pbc_jk_last_error() -> str:
    return load().pbc_jk_last_error().decode()


def _check(rc: int):
    if rc != PBC_JK_OK:
        raise PbcJkError(rc, pbc_jk_last_error())


def _dp(a):
    return a.ctypes.data_as(POINTER(c_double))


def _ip(a):
    return a.ctypes.data_as(POINTER(c_int))


def _inputs(cell, xyz, shell_atom, shell_l, shell_pure, shell_nprim, exps, coefs, thr, charge=None):
    """C structs for one cell; `keep` owns the arrays the structs point into."""
    c = pbc_cell()
    c.a[:] = [float(x) for x in np.asarray(cell, dtype=np.float64).ravel()]
    keep = [np.ascontiguousarray(xyz, dtype=np.float64),
            np.ascontiguousarray(shell_atom, dtype=np.int32),
            np.ascontiguousarray(shell_l, dtype=np.int32),
            np.ascontiguousarray(shell_pure, dtype=np.int32),
            np.ascontiguousarray(shell_nprim, dtype=np.int32),
            np.ascontiguousarray(exps, dtype=np.float64),
            np.ascontiguousarray(coefs, dtype=np.float64)]
    if charge is not None:
        keep.append(np.ascontiguousarray(charge, dtype=np.float64))
    at = pbc_atoms(keep[0].shape[0], _dp(keep[0]), _dp(keep[7]) if len(keep) > 7 else None)
    bs = pbc_basis(keep[1].shape[0], _ip(keep[1]), _ip(keep[2]), _ip(keep[3]), _ip(keep[4]),
                   _dp(keep[5]), _dp(keep[6]))
    th = None
    if thr is not None:
        th = pbc_jk_thresholds(thr.pair_R, thr.pair_cs, thr.ewald_R, thr.ewald_K, thr.schwarz,
                               thr.fp32_below, thr.r_cut, thr.g_cut)
    return c, at, bs, th, keep


def pbc_jk_create(cell, xyz, shell_atom, shell_l, shell_pure, shell_nprim, exps, coefs,
                  omega: float, thr=None, charge=None) -> int:
    """Returns the opaque handle (an integer address)."""
    lib = load()
    c, at, bs, th, keep = _inputs(cell, xyz, shell_atom, shell_l, shell_pure, shell_nprim, exps, coefs, thr,
                                  charge)
    h = c_void_p()
    rc = lib.pbc_jk_create(byref(c), byref(at), byref(bs), float(omega),
                           byref(th) if th is not None else None, byref(h))
    _check(rc)
    return h.value


def _square(n: int, what: str, shape):
    if tuple(shape) != (n, n):
        raise ValueError(f"{what} must be {n} x {n} (the handle's AO count), got {tuple(shape)}")


def pbc_jk_build(h: int, D, want_J: bool = True, want_K: bool = True):
    """Host-memory build: returns (J, K, E_J, E_K)."""
    lib = load()
    n = pbc_jk_nbf(h)
    _check(n if n < 0 else 0)
    D = np.ascontiguousarray(D, dtype=np.float64)
    _square(n, "D", D.shape)
    J = np.empty((n, n)) if want_J else None
    K = np.empty((n, n)) if want_K else None
    ej, ek = c_double(), c_double()
    # E_K is asked for only with K: without it the library runs the J-engine
    rc = lib.pbc_jk_build(c_void_p(h), _dp(D), _dp(J) if J is not None else None,
                          _dp(K) if K is not None else None, byref(ej), byref(ek) if want_K else None)
    _check(rc)
    return J, K, ej.value, (ek.value if want_K else None)


def _stream_ptr(stream):
    """hipStream_t of a torch stream (or an integer handle); None means
    torch's current stream on the current device."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check_device_buffers(h: int, **bufs):
    import torch
    n = pbc_jk_nbf(h)
    _check(n if n < 0 else 0)
    for name, t in bufs.items():
        if t is None:
            continue
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 cuda tensor")
        _square(n, name, t.shape)


def pbc_jk_build_device(h: int, dD, dJ=None, dK=None, energies: bool = True, stream=None):
    """Device-memory build on torch tensors (float64, cuda, contiguous,
    nbf x nbf), queued on `stream` (default: torch's current stream).
    Returns (E_J, E_K) when energies (E_K None without dK: a J-only build
    runs the J-engine), else None (asynchronous)."""
    lib = load()
    _check_device_buffers(h, dD=dD, dJ=dJ, dK=dK)
    ej, ek = c_double(), c_double()
    want_ek = energies and dK is not None
    rc = lib.pbc_jk_build_device(c_void_p(h), c_void_p(dD.data_ptr()),
                                 c_void_p(dJ.data_ptr()) if dJ is not None else None,
                                 c_void_p(dK.data_ptr()) if dK is not None else None,
                                 byref(ej) if energies else None, byref(ek) if want_ek else None,
                                 _stream_ptr(stream))
    _check(rc)
    return (ej.value, ek.value if want_ek else None) if energies else None


def pbc_jk_build_device_static(h: int, dD, dJ=None, dK=None, energies: bool = True, stream=None):
    """pbc_jk_build_device with the work buffers in the library's static
    device array (no device allocation); same arguments and results."""
    lib = load()
    _check_device_buffers(h, dD=dD, dJ=dJ, dK=dK)
    ej, ek = c_double(), c_double()
    want_ek = energies and dK is not None
    rc = lib.pbc_jk_build_device_static(c_void_p(h), c_void_p(dD.data_ptr()),
                                        c_void_p(dJ.data_ptr()) if dJ is not None else None,
                                        c_void_p(dK.data_ptr()) if dK is not None else None,
                                        byref(ej) if energies else None, byref(ek) if want_ek else None,
                                        _stream_ptr(stream))
    _check(rc)
    return (ej.value, ek.value if want_ek else None) if energies else None


def pbc_jk_one_electron(h: int, want_S=True, want_T=True, want_V=True, want_E_nuc=True):
    """Returns (S, T, V, E_nuc) of the handle's cell (None for what was not
    asked for)."""
    lib = load()
    n = pbc_jk_nbf(h)
    _check(n if n < 0 else 0)
    S = np.empty((n, n)) if want_S else None
    T = np.empty((n, n)) if want_T else None
    V = np.empty((n, n)) if want_V else None
    e = c_double()
    rc = lib.pbc_jk_one_electron(c_void_p(h), _dp(S) if S is not None else None, _dp(T) if T is not None else None,
                                 _dp(V) if V is not None else None, byref(e) if want_E_nuc else None)
    _check(rc)
    return S, T, V, (e.value if want_E_nuc else None)


def pbc_jk_destroy(h: int):
    if h:
        load().pbc_jk_destroy(c_void_p(h))


def pbc_jk_nbf(h: int) -> int:
    return load().pbc_jk_nbf(c_void_p(h))


def pbc_jk_stats(h: int) -> dict:
    s = pbc_jk_counters()
    _check(load().pbc_jk_stats(c_void_p(h), byref(s)))
    out = {k: getattr(s, k) for k, _ in s._fields_}
    out["terms_class"] = list(s.terms_class)
    out["t_sr_class_ms"] = list(s.t_sr_class_ms)
    return out


def pbc_jk_set_parts(h: int, mask: int):
    _check(load().pbc_jk_set_parts(c_void_p(h), int(mask)))


def pbc_jk_set_lr(h: int, mode: int, tol: float = 0.0):
    _check(load().pbc_jk_set_lr(c_void_p(h), int(mode), float(tol)))


class Handle:
    """Owns one library handle for a System from paper_2410_22278_amd.inputs."""

    def __init__(self, system, omega=None, thr=None):
        t = thr if thr is not None else system.thr
        self.h = pbc_jk_create(system.cell, system.xyz, system.shell_atom, system.shell_l,
                               system.shell_pure, system.shell_nprim, system.exps, system.coefs,
                               system.omega if omega is None else omega, t, getattr(system, "charge", None))
        self.nbf = pbc_jk_nbf(self.h)

    def build(self, D, want_J=True, want_K=True):
        return pbc_jk_build(self.h, D, want_J, want_K)

    def build_device(self, dD, dJ=None, dK=None, energies=True, stream=None):
        return pbc_jk_build_device(self.h, dD, dJ, dK, energies, stream)

    def build_device_static(self, dD, dJ=None, dK=None, energies=True, stream=None):
        return pbc_jk_build_device_static(self.h, dD, dJ, dK, energies, stream)

    def stats(self):
        return pbc_jk_stats(self.h)

    def one_electron(self, **kw):
        return pbc_jk_one_electron(self.h, **kw)

    def set_parts(self, mask):
        pbc_jk_set_parts(self.h, mask)

    def set_graph(self, enable=True):
        _check(load().pbc_jk_set_graph(c_void_p(self.h), 1 if enable else 0))

    def set_sr_classes(self, mask21):
        _check(load().pbc_jk_set_sr_classes(c_void_p(self.h), int(mask21)))

    def set_lr(self, mode, tol=0.0):
        pbc_jk_set_lr(self.h, mode, tol)

    def close(self):
        if self.h:
            pbc_jk_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The library's request server (pbc_jk_server_*): submit builds for any
    System, wait for them in any order.  Output arrays are owned here until
    the ticket is waited for."""

    def __init__(self, hbm_budget: int = 0, slots: int = 4, cache_cells: bool = True,
                 lr_budget_mb: float = 0.0, use_graphs: bool = False, policy: str = "arrival"):
        lib = load()
        pol = {"arrival": SERVE_ARRIVAL, "deadline": SERVE_DEADLINE}[policy]
        cfg = pbc_jk_server_config(int(hbm_budget), int(slots), 1 if cache_cells else 0, float(lr_budget_mb),
                                   1 if use_graphs else 0, pol)
        s = c_void_p()
        _check(lib.pbc_jk_server_create(byref(cfg), byref(s)))
        self.s = s.value
        self._live = {}

    def submit(self, system, D=None, want_J=True, want_K=True) -> int:
        lib = load()
        c, at, bs, th, keep = _inputs(system.cell, system.xyz, system.shell_atom, system.shell_l,
                                      system.shell_pure, system.shell_nprim, system.exps, system.coefs,
                                      system.thr)
        D = np.ascontiguousarray(system.D if D is None else D, dtype=np.float64)
        n = int(system.nbf)
        _square(n, "D", D.shape)
        J = np.empty((n, n)) if want_J else None
        K = np.empty((n, n)) if want_K else None
        ej, ek = c_double(), c_double()
        t = ctypes.c_ulonglong()
        rc = lib.pbc_jk_server_submit(c_void_p(self.s), byref(c), byref(at), byref(bs), float(system.omega),
                                      byref(th), _dp(D), _dp(J) if J is not None else None,
                                      _dp(K) if K is not None else None, byref(ej), byref(ek), byref(t))
        _check(rc)
        self._live[t.value] = (J, K, ej, ek)
        return t.value

    def wait(self, ticket: int) -> dict:
        """Returns {"status", "J", "K", "E_J", "E_K", and the request info}."""
        info = pbc_jk_request_info()
        rc = load().pbc_jk_server_wait(c_void_p(self.s), ctypes.c_ulonglong(ticket), byref(info))
        J, K, ej, ek = self._live.pop(ticket, (None, None, c_double(), c_double()))
        out = {k: getattr(info, k) for k, _ in info._fields_ if k != "error"}
        out.update(status=rc, error=info.error.decode(errors="replace"), J=J, K=K, E_J=ej.value, E_K=ek.value)
        return out

    def cancel(self, ticket: int) -> int:
        return load().pbc_jk_server_cancel(c_void_p(self.s), ctypes.c_ulonglong(ticket))

    def stats(self) -> dict:
        c = pbc_jk_server_counters()
        _check(load().pbc_jk_server_stats(c_void_p(self.s), byref(c)))
        return {k: getattr(c, k) for k, _ in c._fields_}

    def close(self):
        if getattr(self, "s", None):
            load().pbc_jk_server_destroy(c_void_p(self.s))
            self.s = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Becke:
    """The library's periodic Becke-weight plan (pbc_becke_*) for one cell:
    weights(pts, origin) on torch cuda tensors (float64 N x 3, int32 N)."""

    def __init__(self, cell, xyz, rcut: float = 17.0, delta: float = 1e-14):
        lib = load()
        c = pbc_cell()
        c.a[:] = [float(v) for v in np.asarray(cell, float).ravel()]
        x = np.ascontiguousarray(np.asarray(xyz, float).reshape(-1, 3))
        self.natom = len(x)
        out = c_void_p()
        _check(lib.pbc_becke_create(byref(c), self.natom, x.ctypes.data_as(POINTER(c_double)), float(rcut),
                                    float(delta), byref(out)))
        self.b = out.value

    def info(self):
        m, t = c_int(), ctypes.c_long()
        _check(load().pbc_becke_info(c_void_p(self.b), byref(m), byref(t)))
        return {"max_images": m.value, "total_images": t.value}

    def evaluations(self) -> float:
        """Switching factors evaluated by the last weights() call (waits for it)."""
        e = c_double()
        _check(load().pbc_becke_evaluations(c_void_p(self.b), byref(e)))
        return e.value

    def weights(self, pts, origin, out=None, stream=None):
        """Queues the weights of the points on `stream` (default: torch's
        current stream) and returns the output tensor (not synchronised)."""
        import torch
        if pts.dtype != torch.float64 or not pts.is_cuda or not pts.is_contiguous() or pts.dim() != 2 \
                or pts.shape[1] != 3:
            raise ValueError("pts must be a contiguous float64 cuda tensor of shape (N, 3)")
        if origin.dtype != torch.int32 or not origin.is_cuda or not origin.is_contiguous() \
                or origin.shape != (pts.shape[0],):
            raise ValueError("origin must be a contiguous int32 cuda tensor of shape (N,)")
        n = pts.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=pts.device)
        elif out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.shape != (n,):
            raise ValueError("out must be a contiguous float64 cuda tensor of shape (N,)")
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(load().pbc_becke_weights(c_void_p(self.b), n, c_void_p(pts.data_ptr()),
                                        c_void_p(origin.data_ptr()), c_void_p(out.data_ptr()),
                                        c_void_p(stream.cuda_stream)))
        return out

    def close(self):
        if getattr(self, "b", None):
            load().pbc_becke_destroy(c_void_p(self.b))
            self.b = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
