"""Thin Python binding of libpod.so (C ABI in include/pod.h).

Argument marshalling only: every step of the POD path runs in the HIP
library.  Tensors are torch CUDA (HIP) tensors; the library works on their
data pointers on the current torch stream.  There is no CPU fallback: if the
library is missing or no GPU is present the calls raise.

Function names mirror the C entry points (pod_init, pod_descriptors,
pod_energy_forces, ...); ``PodModel`` bundles a handle with its parameters.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpod.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "pod.h")

POD_F64, POD_F32 = 0, 1
POD_MAX_L, POD_MAX_K, POD_MAX_P, POD_MAX_P4 = 16, 12, 10, 6
POD_MLP_HIDDEN, POD_MLP_MAX_IN = 64, 64
ERRORS = {0: "POD_OK", -1: "POD_EINVAL", -2: "POD_ERANGE", -3: "POD_ENONFINITE", -4: "POD_ENOMEM",
          -5: "POD_EHIP", -6: "POD_ENOTSUP", -7: "POD_ENEIGH", -8: "POD_ESINGULAR", -9: "POD_ETOOBIG"}
POD_STATIC_SCRATCH_BYTES = 64 << 20

_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class PodParamsC(ctypes.Structure):
    _fields_ = [
        ("rin", ctypes.c_double), ("rcut", ctypes.c_double), ("L", ctypes.c_int),
        ("alpha", _dp), ("beta", _dp), ("gamma", _dp), ("kappa", _dp),
        ("K2", ctypes.c_int), ("K3", ctypes.c_int), ("K4", ctypes.c_int),
        ("P3", ctypes.c_int), ("P4", ctypes.c_int), ("dtype", ctypes.c_int),
        ("Q", _dp), ("n_quad", ctypes.c_int),
    ]


class PodTuneC(ctypes.Structure):
    _fields_ = [("cw", ctypes.c_int), ("nblocks", ctypes.c_int), ("threads", ctypes.c_int)]


class PodError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({_strerror(code)})")


_lib = None


def header_symbols():
    """Names of the functions declared in include/pod.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pod_[a-z0-9_]+)\s*\(", txt)))


def lib():
    """Load libpod.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2212_14446_amd.build_lib")
    L = ctypes.CDLL(LIB_PATH)
    i, P = ctypes.c_int, ctypes.POINTER
    L.pod_init.argtypes = [P(PodParamsC), _vp, P(_vp)]
    L.pod_compute_basis.argtypes = [P(PodParamsC), _dp, _dp]
    L.pod_num_descriptors.argtypes = [_vp, P(i), P(i)]
    L.pod_get_basis.argtypes = [_vp, _dp, _dp]
    L.pod_descriptors.argtypes = [_vp, i, i, _vp, _dp, _vp, _vp, _vp, _vp]
    L.pod_energy_forces.argtypes = [_vp, i, i, _vp, _dp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.pod_energy_forces_noalloc.argtypes = [_vp, i, i, _vp, _dp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.pod_neighbor_reverse.argtypes = [_vp, i, i, _vp, _vp, _vp, _vp]
    L.pod_batch_assemble.argtypes = [_vp, i, i, i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, P(PodTuneC)]
    lg, f = ctypes.c_long, ctypes.c_float
    L.pod_build_neighbors.argtypes = [_vp, i, _vp, _dp, ctypes.c_double, _vp, _vp, _vp, lg, P(lg)]
    d = ctypes.c_double
    L.pod_fit_gram.argtypes = [_vp, i, i, _vp, _vp, d, lg, _vp, _vp, d, i, _vp]
    L.pod_fit_solve.argtypes = [_vp, i, _vp, d, _vp, _vp]
    L.pod_opod_descriptors.argtypes = [_vp, i, i, _vp, _dp, _vp, _vp, _vp, _vp]
    L.pod_md_verlet.argtypes = [_vp, i, i, _vp, _vp, _vp, _dp, _vp, _vp, _vp, _vp, _vp, d, d, i, _vp, _vp, _vp, _vp]
    L.pod_md_max_displacement.argtypes = [_vp, i, _vp, _vp, _vp]
    L.pod_opod_energy_forces.argtypes = [_vp, i, i, _vp, _dp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.pod_mlp_num_params.argtypes = [i]
    L.pod_mlp_forward.argtypes = [_vp, i, i, _vp, lg, _vp, _vp, _vp, _vp, _vp]
    L.pod_mlp_train_step.argtypes = [_vp, i, i, _vp, lg, _vp, _vp, _vp, _vp, _vp, _vp, i, f, f, f, f, _vp]
    L.pod_energy_forces_surrogate.argtypes = [_vp, i, i, _vp, _dp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                              _vp, _vp, _vp]
    L.pod_five_body_count.argtypes = [i, P(i)]
    L.pod_five_body_descriptors.argtypes = [_vp, i, i, _vp, _dp, _vp, _vp, _vp, i, i, _vp]
    L.pod_five_body_energy_forces.argtypes = [_vp, i, i, _vp, _dp, _vp, _vp, _vp, _vp, i, i, _vp, _vp, _vp]
    L.pod_acsf_create.argtypes = [_vp, i, _dp, i, _dp, i, _dp, P(_vp)]
    L.pod_acsf_num_functions.argtypes = [_vp, P(i), P(i)]
    L.pod_acsf_descriptors.argtypes = [_vp, _vp, i, i, _vp, _dp, _vp, _vp, _vp, _vp]
    L.pod_acsf_forces.argtypes = [_vp, _vp, i, i, _vp, _dp, _vp, _vp, _vp, _vp, _vp, lg, _vp, _vp]
    L.pod_acsf_free.argtypes = [_vp]
    L.pod_acsf_free.restype = None
    L.pod_check.argtypes = [_vp]
    L.pod_set_kernel_timing.argtypes = [_vp, i]
    L.pod_get_kernel_time.argtypes = [_vp, i, _dp, P(i)]
    L.pod_strerror.argtypes = [i]
    L.pod_strerror.restype = ctypes.c_char_p
    L.pod_free.argtypes = [_vp]
    L.pod_free.restype = None
    for name in ("pod_init", "pod_compute_basis", "pod_num_descriptors", "pod_get_basis", "pod_descriptors",
                 "pod_energy_forces", "pod_energy_forces_noalloc", "pod_check", "pod_set_kernel_timing",
                 "pod_get_kernel_time",
                 "pod_neighbor_reverse", "pod_batch_assemble", "pod_mlp_num_params", "pod_mlp_forward",
                 "pod_mlp_train_step", "pod_energy_forces_surrogate", "pod_build_neighbors", "pod_fit_gram",
                 "pod_fit_solve", "pod_opod_descriptors", "pod_opod_energy_forces", "pod_md_verlet",
                 "pod_md_max_displacement", "pod_acsf_create", "pod_acsf_num_functions", "pod_acsf_descriptors",
                 "pod_acsf_forces", "pod_five_body_count", "pod_five_body_descriptors",
                 "pod_five_body_energy_forces"):
        getattr(L, name).restype = i
    _lib = L
    return L


def pod_strerror(code: int) -> str:
    """Static description of an error code."""
    return lib().pod_strerror(int(code)).decode()


def _strerror(code):
    try:
        return lib().pod_strerror(int(code)).decode()
    except Exception:  # library not loadable: still produce a message
        return ERRORS.get(code, "unknown")


def _ok(rc, where):
    if rc != 0:
        raise PodError(rc, where)


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _ptr_at(t, elem_offset):
    """Device pointer of element `elem_offset` of a contiguous tensor."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if not 0 <= elem_offset < max(t.numel(), 1):
        raise ValueError("offset outside the tensor")
    return ctypes.c_void_p(t.data_ptr() + int(elem_offset) * t.element_size())


def _cell_ptr(cell):
    if cell is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(9))
    return arr, arr.ctypes.data_as(_dp)


@dataclass
class Setup:
    rin: float
    rcut: float
    alpha: np.ndarray
    beta: np.ndarray
    gamma: np.ndarray
    kappa: np.ndarray
    K2: int
    K3: int
    K4: int
    P3: int
    P4: int


def _params(s: Setup, dtype_code: int, Q=None, n_quad=0):
    keep = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (s.alpha, s.beta, s.gamma, s.kappa)]
    qarr = None if Q is None else np.ascontiguousarray(np.asarray(Q, dtype=np.float64))
    p = PodParamsC(float(s.rin), float(s.rcut), len(keep[0]),
                   *[k.ctypes.data_as(_dp) for k in keep],
                   int(s.K2), int(s.K3), int(s.K4), int(s.P3), int(s.P4), int(dtype_code),
                   qarr.ctypes.data_as(_dp) if qarr is not None else None, int(n_quad))
    return p, (keep, qarr)


def pod_compute_basis(setup: Setup, n_quad: int = 0):
    """Host-only POD basis (no device call): (Q [L, L], eigenvalues [L])."""
    p, keep = _params(setup, POD_F64, None, n_quad)
    L = p.L
    Q = np.zeros((L, L))
    e = np.zeros(L)
    _ok(lib().pod_compute_basis(ctypes.byref(p), Q.ctypes.data_as(_dp), e.ctypes.data_as(_dp)), "pod_compute_basis")
    return Q, e


class Handle:
    def __init__(self, ptr, dtype_code, M, K, L):
        self.ptr = ptr
        self.dtype_code = dtype_code
        self.M = M
        self.K = K
        self.L = L

    def __del__(self):
        try:
            pod_free(self)
        except Exception:
            pass


def pod_init(setup: Setup, dtype: str = "f64", Q=None, n_quad: int = 0, stream=None) -> Handle:
    import torch
    code = POD_F64 if dtype in ("f64", "float64") else POD_F32
    p, keep = _params(setup, code, Q, n_quad)
    if stream is None:
        stream = torch.cuda.current_stream()
    h = ctypes.c_void_p()
    _ok(lib().pod_init(ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)), "pod_init")
    M = ctypes.c_int()
    _ok(lib().pod_num_descriptors(h, ctypes.byref(M), None), "pod_num_descriptors")
    return Handle(h, code, M.value, max(setup.K2, setup.K3, setup.K4), p.L)


def pod_num_descriptors(h: Handle):
    M = ctypes.c_int()
    by = (ctypes.c_int * 4)()
    _ok(lib().pod_num_descriptors(h.ptr, ctypes.byref(M), by), "pod_num_descriptors")
    return M.value, list(by)


def pod_get_basis(h: Handle):
    Q = np.zeros((h.L, h.K))
    e = np.zeros(h.L)
    _ok(lib().pod_get_basis(h.ptr, Q.ctypes.data_as(_dp), e.ctypes.data_as(_dp)), "pod_get_basis")
    return Q, e


def pod_descriptors(h: Handle, N, P, pos, cell, offsets, nbr_j, shift, D):
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_descriptors(h.ptr, int(N), int(P), _ptr(pos), cp, _ptr(offsets), _ptr(nbr_j), _ptr(shift),
                              _ptr(D)), "pod_descriptors")


def pod_neighbor_reverse(h: Handle, N, P, offsets, nbr_j, shift, rev):
    _ok(lib().pod_neighbor_reverse(h.ptr, int(N), int(P), _ptr(offsets), _ptr(nbr_j), _ptr(shift), _ptr(rev)),
        "pod_neighbor_reverse")


def pod_build_neighbors(h: Handle, N, pos, cell, rlist, offsets, nbr_j=None, shift=None, capacity=0):
    """Returns the number of directed pairs; the list is written when capacity >= it."""
    arr, cp = _cell_ptr(cell)
    n = ctypes.c_long()
    _ok(lib().pod_build_neighbors(h.ptr, int(N), _ptr(pos), cp, float(rlist), _ptr(offsets), _ptr(nbr_j),
                                  _ptr(shift), int(capacity), ctypes.byref(n)), "pod_build_neighbors")
    return n.value


def pod_opod_descriptors(h: Handle, N, P, pos, cell, offsets, nbr_j, shift, D):
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_opod_descriptors(h.ptr, int(N), int(P), _ptr(pos), cp, _ptr(offsets), _ptr(nbr_j), _ptr(shift),
                                   _ptr(D)), "pod_opod_descriptors")


def pod_opod_energy_forces(h: Handle, N, P, pos, cell, offsets, nbr_j, shift, c, E_atom=None, E=None, F=None,
                           W=None):
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_opod_energy_forces(h.ptr, int(N), int(P), _ptr(pos), cp, _ptr(offsets), _ptr(nbr_j),
                                     _ptr(shift), _ptr(c), _ptr(E_atom), _ptr(E), _ptr(F), _ptr(W)),
        "pod_opod_energy_forces")


def pod_md_verlet(h: Handle, N, P, pos, vel, F, cell, offsets, nbr_j, shift, rev, c, mass, dt, nsteps, E_pot=None,
                  E_kin=None, pos_ref=None, max_disp=None):
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_md_verlet(h.ptr, int(N), int(P), _ptr(pos), _ptr(vel), _ptr(F), cp, _ptr(offsets), _ptr(nbr_j),
                            _ptr(shift), _ptr(rev), _ptr(c), float(mass), float(dt), int(nsteps), _ptr(E_pot),
                            _ptr(E_kin), _ptr(pos_ref), _ptr(max_disp)), "pod_md_verlet")


def pod_md_max_displacement(h: Handle, N, pos, pos_ref, out):
    _ok(lib().pod_md_max_displacement(h.ptr, int(N), _ptr(pos), _ptr(pos_ref), _ptr(out)), "pod_md_max_displacement")


def pod_fit_gram(h: Handle, M, n_cfg, G, E_ref, w_e, n_frows, dGdR, F_ref, w_f, Z, accumulate=False):
    _ok(lib().pod_fit_gram(h.ptr, int(M), int(n_cfg), _ptr(G), _ptr(E_ref), float(w_e), int(n_frows), _ptr(dGdR),
                           _ptr(F_ref), float(w_f), 1 if accumulate else 0, _ptr(Z)), "pod_fit_gram")


def pod_fit_solve(h: Handle, M, Z, gamma, c, loss=None):
    _ok(lib().pod_fit_solve(h.ptr, int(M), _ptr(Z), float(gamma), _ptr(c), _ptr(loss)), "pod_fit_solve")


def pod_energy_forces(h: Handle, N, P, pos, cell, offsets, nbr_j, shift, c, E_atom=None, E=None, F=None, W=None,
                      G=None, rev=None):
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_energy_forces(h.ptr, int(N), int(P), _ptr(pos), cp, _ptr(offsets), _ptr(nbr_j), _ptr(shift),
                                _ptr(rev), _ptr(c), _ptr(E_atom), _ptr(E), _ptr(F), _ptr(W), _ptr(G)),
        "pod_energy_forces")


def pod_energy_forces_noalloc(h: Handle, N, P, pos, cell, offsets, nbr_j, shift, c, E_atom=None, E=None, F=None,
                              W=None, G=None, rev=None):
    """pod_energy_forces on the library's static scratch (no allocation)."""
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_energy_forces_noalloc(h.ptr, int(N), int(P), _ptr(pos), cp, _ptr(offsets), _ptr(nbr_j),
                                        _ptr(shift), _ptr(rev), _ptr(c), _ptr(E_atom), _ptr(E), _ptr(F), _ptr(W),
                                        _ptr(G)),
        "pod_energy_forces_noalloc")


def pod_batch_assemble(h: Handle, n_cfg, N, P, cfg_atom_off, pos, cells, offsets, nbr_j, shift, D=None, G=None,
                       dGdR=None, tune=None):
    """tune: None (library defaults) or a (cw, nblocks, threads) triple."""
    t = None
    if tune is not None:
        t = ctypes.byref(PodTuneC(int(tune[0]), int(tune[1]), int(tune[2])))
    _ok(lib().pod_batch_assemble(h.ptr, int(n_cfg), int(N), int(P), _ptr(cfg_atom_off), _ptr(pos), _ptr(cells),
                                 _ptr(offsets), _ptr(nbr_j), _ptr(shift), _ptr(D), _ptr(G), _ptr(dGdR), t),
        "pod_batch_assemble")


def pod_mlp_num_params(n_in):
    rc = lib().pod_mlp_num_params(int(n_in))
    if rc < 0:
        raise PodError(rc, "pod_mlp_num_params")
    return rc


def pod_mlp_forward(h: Handle, n, n_in, X, ldx, theta, mu, inv_sigma, y=None, dydx=None, x_col=0):
    """X: contiguous device tensor in the handle dtype; the network reads
    X.flat[i * ldx + x_col + k]."""
    xp = _ptr_at(X, x_col) if n > 0 else _ptr(X)
    _ok(lib().pod_mlp_forward(h.ptr, int(n), int(n_in), xp, int(ldx), _ptr(theta), _ptr(mu), _ptr(inv_sigma),
                              _ptr(y), _ptr(dydx)), "pod_mlp_forward")


def pod_mlp_train_step(h: Handle, n, n_in, X, ldx, target, mu, inv_sigma, theta, m, v, step, lr, beta1=0.9,
                       beta2=0.999, eps=1e-8, loss=None):
    _ok(lib().pod_mlp_train_step(h.ptr, int(n), int(n_in), _ptr(X), int(ldx), _ptr(target), _ptr(mu),
                                 _ptr(inv_sigma), _ptr(theta), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                                 float(beta2), float(eps), _ptr(loss)), "pod_mlp_train_step")


def pod_energy_forces_surrogate(h: Handle, N, P, pos, cell, offsets, nbr_j, shift, c, theta, mu, inv_sigma,
                                E_atom=None, E=None, F=None, W=None, rev=None):
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_energy_forces_surrogate(h.ptr, int(N), int(P), _ptr(pos), cp, _ptr(offsets), _ptr(nbr_j),
                                          _ptr(shift), _ptr(rev), _ptr(c), _ptr(theta), _ptr(mu), _ptr(inv_sigma),
                                          _ptr(E_atom), _ptr(E), _ptr(F), _ptr(W)),
        "pod_energy_forces_surrogate")


def pod_check(h: Handle):
    _ok(lib().pod_check(h.ptr), "pod_check")


def pod_set_kernel_timing(h: Handle, n: int):
    _ok(lib().pod_set_kernel_timing(h.ptr, int(n)), "pod_set_kernel_timing")


def pod_get_kernel_time(h: Handle, kind: int = 1):
    """(total ms, launches) of kernel `kind` (0 finalize, 1 per-atom, 2 network,
    3 fit Gram, 4 pair gradients)."""
    ms = ctypes.c_double()
    n = ctypes.c_int()
    _ok(lib().pod_get_kernel_time(h.ptr, int(kind), ctypes.byref(ms), ctypes.byref(n)), "pod_get_kernel_time")
    return ms.value, n.value


def pod_free(h: Handle):
    if h is not None and h.ptr:
        lib().pod_free(h.ptr)
        h.ptr = None


def pod_five_body_count(P5: int) -> int:
    n = ctypes.c_int()
    _ok(lib().pod_five_body_count(int(P5), ctypes.byref(n)), "pod_five_body_count")
    return n.value


def pod_five_body_descriptors(h: Handle, N, P, pos, cell, offsets, nbr_j, shift, K5, P5, D5):
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_five_body_descriptors(h.ptr, int(N), int(P), _ptr(pos), cp, _ptr(offsets), _ptr(nbr_j),
                                        _ptr(shift), int(K5), int(P5), _ptr(D5)), "pod_five_body_descriptors")


def pod_five_body_energy_forces(h: Handle, N, P, pos, cell, offsets, nbr_j, shift, rev, K5, P5, c5, E_atom=None,
                                F=None):
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_five_body_energy_forces(h.ptr, int(N), int(P), _ptr(pos), cp, _ptr(offsets), _ptr(nbr_j),
                                          _ptr(shift), _ptr(rev), int(K5), int(P5), _ptr(c5), _ptr(E_atom), _ptr(F)),
        "pod_five_body_energy_forces")


class AcsfSet:
    """A set of symmetry functions created on the device for one handle."""

    def __init__(self, ptr, h: Handle, n_functions: int, n_channels: int):
        self.ptr = ptr
        self.h = h            # keeps the handle alive as long as the set
        self.n = n_functions
        self.n_channels = n_channels

    def __del__(self):
        try:
            pod_acsf_free(self)
        except Exception:
            pass


def _acsf_rows(rows, width):
    arr = np.ascontiguousarray(np.asarray(rows, dtype=np.float64).reshape(-1, width))
    return arr, (arr.ctypes.data_as(_dp) if arr.size else None)


def pod_acsf_create(h: Handle, g2=(), g3=(), g4=()) -> AcsfSet:
    a2, p2 = _acsf_rows(g2, 2)
    a3, p3 = _acsf_rows(g3, 3)
    a4, p4 = _acsf_rows(g4, 7)
    out = ctypes.c_void_p()
    _ok(lib().pod_acsf_create(h.ptr, a2.shape[0], p2, a3.shape[0], p3, a4.shape[0], p4, ctypes.byref(out)),
        "pod_acsf_create")
    n, nc = ctypes.c_int(), ctypes.c_int()
    _ok(lib().pod_acsf_num_functions(out, ctypes.byref(n), ctypes.byref(nc)), "pod_acsf_num_functions")
    return AcsfSet(out, h, n.value, nc.value)


def pod_acsf_num_functions(a: AcsfSet):
    """(number of functions, number of radial channels) of a set."""
    n, nc = ctypes.c_int(), ctypes.c_int()
    _ok(lib().pod_acsf_num_functions(a.ptr, ctypes.byref(n), ctypes.byref(nc)), "pod_acsf_num_functions")
    return n.value, nc.value


def pod_acsf_descriptors(h: Handle, a: AcsfSet, N, P, pos, cell, offsets, nbr_j, shift, G):
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_acsf_descriptors(h.ptr, a.ptr, int(N), int(P), _ptr(pos), cp, _ptr(offsets), _ptr(nbr_j),
                                   _ptr(shift), _ptr(G)), "pod_acsf_descriptors")


def pod_acsf_forces(h: Handle, a: AcsfSet, N, P, pos, cell, offsets, nbr_j, shift, rev, W, ldw, F, G=None):
    arr, cp = _cell_ptr(cell)
    _ok(lib().pod_acsf_forces(h.ptr, a.ptr, int(N), int(P), _ptr(pos), cp, _ptr(offsets), _ptr(nbr_j),
                              _ptr(shift), _ptr(rev), _ptr(W), int(ldw), _ptr(G), _ptr(F)), "pod_acsf_forces")


def pod_acsf_free(a: AcsfSet):
    if a.ptr:
        lib().pod_acsf_free(a.ptr)
        a.ptr = None


# --------------------------------------------------------------------------
# Convenience wrapper
# --------------------------------------------------------------------------
class DeviceNeighbors:
    """CSR neighbour list resident on the device (int32)."""

    def __init__(self, offsets, nbr_j, shift, device="cuda"):
        import torch
        self.offsets = torch.as_tensor(np.asarray(offsets, dtype=np.int32), device=device)
        self.nbr_j = torch.as_tensor(np.asarray(nbr_j, dtype=np.int32), device=device)
        self.shift = torch.as_tensor(np.asarray(shift, dtype=np.int32), device=device)
        self.N = int(self.offsets.numel()) - 1
        self.P = int(self.nbr_j.numel())
        self.rev = None

    def build_reverse(self, model: "PodModel", check=True):
        """Reverse-pair index on the device (once per list)."""
        import torch
        self.rev = torch.empty(max(self.P, 1), dtype=torch.int32, device=self.offsets.device)
        pod_neighbor_reverse(model.h, self.N, self.P, self.offsets, self.nbr_j, self.shift, self.rev)
        if check:
            pod_check(model.h)
        return self.rev

    @classmethod
    def from_list(cls, nl, device="cuda"):
        return cls(nl.offsets, nl.nbr_j, nl.shift, device)

    @classmethod
    def build(cls, model: "PodModel", pos, cell, rlist=0.0, capacity=None, check=True):
        """Build the list on the device (pod_build_neighbors): one call when
        `capacity` pairs suffice, else a second call sized from the count."""
        import torch
        pos = model._pos(pos)
        N = int(pos.shape[0])
        dev = model.device
        offsets = torch.empty(N + 1, dtype=torch.int32, device=dev)
        cap = int(capacity) if capacity is not None else 64 * N
        for _ in range(2):
            nbr_j = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            shift = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            P = pod_build_neighbors(model.h, N, pos, cell, rlist, offsets, nbr_j, shift, cap)
            if P <= cap:
                break
            cap = P
        if check:
            pod_check(model.h)
        self = cls.__new__(cls)
        self.offsets, self.nbr_j, self.shift = offsets, nbr_j[:P], shift[:P]
        self.N, self.P, self.rev = N, P, None
        return self


class PodModel:
    """A POD handle plus its parameters; tensors in and out live on the GPU."""

    def __init__(self, setup: Setup, dtype: str = "f64", Q=None, n_quad: int = 0, device="cuda"):
        import torch
        self.setup = setup
        self.device = torch.device(device)
        self.torch_dtype = torch.float64 if dtype in ("f64", "float64") else torch.float32
        self.h = pod_init(setup, dtype, Q, n_quad)
        self.M, self.M_by_order = pod_num_descriptors(self.h)

    def basis(self):
        return pod_get_basis(self.h)

    def _pos(self, pos):
        import torch
        return torch.as_tensor(pos, dtype=self.torch_dtype, device=self.device).contiguous()

    def descriptors(self, pos, cell, nbrs: DeviceNeighbors, check=True):
        import torch
        pos = self._pos(pos)
        D = torch.empty((nbrs.N, self.M), dtype=self.torch_dtype, device=self.device)
        pod_descriptors(self.h, nbrs.N, nbrs.P, pos, cell, nbrs.offsets, nbrs.nbr_j, nbrs.shift, D)
        if check:
            pod_check(self.h)
        return D

    def energy_forces(self, pos, cell, nbrs: DeviceNeighbors, c, forces=True, virial=True, global_desc=True,
                      per_atom=True, check=True, out=None):
        import torch
        pos = self._pos(pos)
        c = torch.as_tensor(c, dtype=self.torch_dtype, device=self.device).contiguous()
        if c.numel() != self.M:
            raise ValueError(f"expected {self.M} coefficients, got {c.numel()}")
        N = nbrs.N
        o = out if out is not None else {
            "E": torch.empty(1, dtype=torch.float64, device=self.device),
            "E_atom": torch.empty(N, dtype=self.torch_dtype, device=self.device) if per_atom else None,
            "F": torch.empty((N, 3), dtype=self.torch_dtype, device=self.device) if forces else None,
            "W": torch.empty((3, 3), dtype=torch.float64, device=self.device) if virial else None,
            "G": torch.empty(self.M, dtype=torch.float64, device=self.device) if global_desc else None,
        }
        pod_energy_forces(self.h, N, nbrs.P, pos, cell, nbrs.offsets, nbrs.nbr_j, nbrs.shift, c,
                          o["E_atom"], o["E"], o["F"], o["W"], o["G"], rev=nbrs.rev)
        if check:
            pod_check(self.h)
        return o

    def opod_descriptors(self, pos, cell, nbrs: DeviceNeighbors, check=True):
        """Exclusive-sum descriptors (eqs. (15b), (20a)), FP64 handles."""
        import torch
        pos = self._pos(pos)
        D = torch.empty((nbrs.N, self.M), dtype=self.torch_dtype, device=self.device)
        pod_opod_descriptors(self.h, nbrs.N, nbrs.P, pos, cell, nbrs.offsets, nbrs.nbr_j, nbrs.shift, D)
        if check:
            pod_check(self.h)
        return D

    def opod_energy_forces(self, pos, cell, nbrs: DeviceNeighbors, c, check=True, out=None):
        """Energy, forces and virial of the 2/3-body exclusive model (K4 = 0, FP64)."""
        import torch
        pos = self._pos(pos)
        c = torch.as_tensor(c, dtype=self.torch_dtype, device=self.device).contiguous()
        N = nbrs.N
        o = out if out is not None else {
            "E": torch.empty(1, dtype=torch.float64, device=self.device),
            "E_atom": torch.empty(N, dtype=self.torch_dtype, device=self.device),
            "F": torch.empty((N, 3), dtype=self.torch_dtype, device=self.device),
            "W": torch.empty((3, 3), dtype=torch.float64, device=self.device),
        }
        pod_opod_energy_forces(self.h, N, nbrs.P, pos, cell, nbrs.offsets, nbrs.nbr_j, nbrs.shift, c,
                               o["E_atom"], o["E"], o["F"], o["W"])
        if check:
            pod_check(self.h)
        return o

    def five_body_descriptors(self, pos, cell, nbrs: DeviceNeighbors, K5: int, P5: int, check=True):
        """[N, K5 * pod_five_body_count(P5)] five-body descriptors (m-major)."""
        import torch
        pos = self._pos(pos)
        n = pod_five_body_count(P5)
        D5 = torch.empty((nbrs.N, K5 * n), dtype=self.torch_dtype, device=self.device)
        pod_five_body_descriptors(self.h, nbrs.N, nbrs.P, pos, cell, nbrs.offsets, nbrs.nbr_j, nbrs.shift, K5, P5,
                                  D5)
        if check:
            pod_check(self.h)
        return D5

    def five_body_energy_forces(self, pos, cell, nbrs: DeviceNeighbors, K5: int, P5: int, c5, check=True):
        """Per-atom energies and forces of the linear five-body term c5 . D5."""
        import torch
        pos = self._pos(pos)
        c5 = torch.as_tensor(c5, dtype=self.torch_dtype, device=self.device).contiguous()
        if c5.numel() != K5 * pod_five_body_count(P5):
            raise ValueError("expected K5 x pod_five_body_count(P5) coefficients")
        if nbrs.rev is None:
            nbrs.build_reverse(self, check=check)
        o = {"E_atom": torch.empty(nbrs.N, dtype=self.torch_dtype, device=self.device),
             "F": torch.empty((nbrs.N, 3), dtype=self.torch_dtype, device=self.device)}
        pod_five_body_energy_forces(self.h, nbrs.N, nbrs.P, pos, cell, nbrs.offsets, nbrs.nbr_j, nbrs.shift, nbrs.rev,
                                    K5, P5, c5, o["E_atom"], o["F"])
        if check:
            pod_check(self.h)
        return o

    def acsf(self, spec) -> AcsfSet:
        """A symmetry-function set (workloads.AcsfSpec or anything with g2,
        g3, g4) on this handle: its rin, rcut, dtype and stream."""
        return pod_acsf_create(self.h, spec.g2, spec.g3, spec.g4)

    def acsf_descriptors(self, a: AcsfSet, pos, cell, nbrs: DeviceNeighbors, check=True):
        import torch
        pos = self._pos(pos)
        G = torch.empty((nbrs.N, a.n), dtype=self.torch_dtype, device=self.device)
        pod_acsf_descriptors(self.h, a, nbrs.N, nbrs.P, pos, cell, nbrs.offsets, nbrs.nbr_j, nbrs.shift, G)
        if check:
            pod_check(self.h)
        return G

    def acsf_forces(self, a: AcsfSet, pos, cell, nbrs: DeviceNeighbors, W, with_G=False, check=True):
        """F = -d(sum_i W_i . G_i)/dx; W is [n] (shared) or [N, n]."""
        import torch
        pos = self._pos(pos)
        W = torch.as_tensor(W, dtype=self.torch_dtype, device=self.device).contiguous()
        ldw = 0 if W.dim() == 1 else int(W.shape[1])
        if nbrs.rev is None:
            nbrs.build_reverse(self, check=check)
        F = torch.empty((nbrs.N, 3), dtype=self.torch_dtype, device=self.device)
        G = torch.empty((nbrs.N, a.n), dtype=self.torch_dtype, device=self.device) if with_G else None
        pod_acsf_forces(self.h, a, nbrs.N, nbrs.P, pos, cell, nbrs.offsets, nbrs.nbr_j, nbrs.shift, nbrs.rev, W,
                        ldw, F, G)
        if check:
            pod_check(self.h)
        return (F, G) if with_G else F

    def energy_forces_surrogate(self, pos, cell, nbrs: DeviceNeighbors, c, net, forces=True, virial=True,
                                per_atom=True, check=True, out=None):
        """Energy and forces with the network `net` (surrogate.Network) in
        place of the 4-body term; this model must have K4 = 0."""
        import torch
        pos = self._pos(pos)
        c = torch.as_tensor(c, dtype=self.torch_dtype, device=self.device).contiguous()
        N = nbrs.N
        o = out if out is not None else {
            "E": torch.empty(1, dtype=torch.float64, device=self.device),
            "E_atom": torch.empty(N, dtype=self.torch_dtype, device=self.device) if per_atom else None,
            "F": torch.empty((N, 3), dtype=self.torch_dtype, device=self.device) if forces else None,
            "W": torch.empty((3, 3), dtype=torch.float64, device=self.device) if virial else None,
        }
        pod_energy_forces_surrogate(self.h, N, nbrs.P, pos, cell, nbrs.offsets, nbrs.nbr_j, nbrs.shift, c,
                                    net.theta, net.mu, net.inv_sigma, o["E_atom"], o["E"], o["F"], o["W"],
                                    rev=nbrs.rev)
        if check:
            pod_check(self.h)
        return o

    def check(self):
        pod_check(self.h)


class DeviceBatch:
    """Many cells stacked for pod_batch_assemble: atom offsets per cell, the
    stacked positions, the cells (n_cfg x 3 x 3) and one stacked CSR list."""

    def __init__(self, cfg_atom_off, pos, cells, offsets, nbr_j, shift, device="cuda"):
        import torch
        self.cfg_atom_off = torch.as_tensor(np.asarray(cfg_atom_off, dtype=np.int32), device=device)
        self.pos = torch.as_tensor(np.asarray(pos, dtype=np.float64), device=device).contiguous()
        self.cells = torch.as_tensor(np.asarray(cells, dtype=np.float64).reshape(-1, 9), device=device).contiguous()
        self.nbrs = DeviceNeighbors(offsets, nbr_j, shift, device)
        self.n_cfg = int(self.cfg_atom_off.numel()) - 1
        self.N = self.nbrs.N
        self.P = self.nbrs.P

    @classmethod
    def from_batch(cls, b, device="cuda"):
        """From a workloads.Batch."""
        return cls(b.cfg_atom_off, b.pos, b.cells, b.nl.offsets, b.nl.nbr_j, b.nl.shift, device)


def batch_assemble(model: PodModel, batch: DeviceBatch, D=True, G=True, dGdR=True, tune=None, check=True,
                   out=None):
    """D (N x M), G (n_cfg x M) and dG/dR (3N x M) of every cell, FP64."""
    import torch
    dev, M = model.device, model.M
    o = out if out is not None else {
        "D": torch.empty((batch.N, M), dtype=torch.float64, device=dev) if D else None,
        "G": torch.empty((batch.n_cfg, M), dtype=torch.float64, device=dev) if G else None,
        "dGdR": torch.empty((3 * batch.N, M), dtype=torch.float64, device=dev) if dGdR else None,
    }
    nb = batch.nbrs
    pod_batch_assemble(model.h, batch.n_cfg, batch.N, batch.P, batch.cfg_atom_off, batch.pos, batch.cells,
                       nb.offsets, nb.nbr_j, nb.shift, o["D"], o["G"], o["dGdR"], tune)
    if check:
        pod_check(model.h)
    return o


def setup_from_workload(s) -> Setup:
    """Setup of a workloads.PodSetup (snapshot family included)."""
    a, b, g, k = s.snapshot_family()
    return Setup(s.rin, s.rcut, a, b, g, k, s.K2, s.K3, s.K4, s.P3, s.P4)
