"""Python binding of libmbstokes (ctypes): argument marshalling only.

Every call goes through the C ABI declared in include/mbstokes.h; the arithmetic runs in the
library's HIP kernels. Tensors are torch float64 CUDA tensors (device memory of the context's
GPU); the current torch stream is passed to the library. If the shared library is missing or
no GPU is present, the calls raise instead of computing anything elsewhere.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbstokes.so")

MBS_OK, MBS_EINVAL, MBS_ENOCONV, MBS_EOVERLAP, MBS_EUNSUPPORTED, MBS_ENOMEM, MBS_EHIP = 0, -1, -2, -3, -4, -5, -6
ERROR_NAMES = {MBS_EINVAL: "MBS_EINVAL", MBS_ENOCONV: "MBS_ENOCONV", MBS_EOVERLAP: "MBS_EOVERLAP",
               MBS_EUNSUPPORTED: "MBS_EUNSUPPORTED", MBS_ENOMEM: "MBS_ENOMEM", MBS_EHIP: "MBS_EHIP"}
MBS_FP64, MBS_MIXED, MBS_FP32 = 0, 1, 1
MBS_GUESS_ZERO, MBS_GUESS_DIAG, MBS_GUESS_LEARNED, MBS_GUESS_USER = 0, 1, 2, 3

EXPORTS = ("mbs_default_params", "mbs_create", "mbs_destroy", "mbs_set_params", "mbs_last_error",
           "mbs_solve", "mbs_matvec", "mbs_rhs", "mbs_outputs", "mbs_flow", "mbs_step", "mbs_solve_batched",
           "mbs_autotune", "mbs_autotune_batched", "mbs_features", "mbs_warmstart_init", "mbs_warmstart_set", "mbs_warmstart_get",
           "mbs_warmstart_forward", "mbs_warmstart_grad", "mbs_warmstart_train", "mbs_warmstart_save",
           "mbs_warmstart_load", "mbs_warmstart_target", "mbs_initial_guess", "mbs_precond_apply",
           "mbs_solve_ex", "mbs_rhs_ex", "mbs_outputs_ex", "mbs_flow_ex", "mbs_matvec_static",
           "mbs_warmstart_features", "mbs_features_ex", "mbs_matvec_r3", "mbs_rhs_r3", "mbs_outputs_r3",
           "mbs_solve_r3", "mbs_precond_apply_r3")
R3_DIM = 20  # unknowns per sphere at traction ranks <= 3: Sigma (5), X^gam (7), X^psi (5), X^d (3)
MLP_NPARAM, MLP_NFEAT = 27525, 80
MLP_NPARAM_RHS, MLP_NFEAT_RHS = 37765, 160
MBS_FEATURES_GEOMETRY, MBS_FEATURES_GEOMETRY_RHS = 0, 1
_MLP_SIZES = {MBS_FEATURES_GEOMETRY: (MLP_NFEAT, MLP_NPARAM), MBS_FEATURES_GEOMETRY_RHS: (MLP_NFEAT_RHS, MLP_NPARAM_RHS)}


class MbsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("a", ctypes.c_double), ("tol", ctypes.c_double),
                ("self_slip_c", ctypes.c_double), ("inner_tol", ctypes.c_double),
                ("near_cutoff", ctypes.c_double),
                ("lmax", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("guess", ctypes.c_int32),
                ("check_overlap", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("batch_item", ctypes.c_int32), ("superposition", ctypes.c_int32),
                ("near_order", ctypes.c_int32), ("spatial_order", ctypes.c_int32),
                ("plane", ctypes.c_int32), ("ewald_mesh", ctypes.c_int32), ("plane_z", ctypes.c_double),
                ("box", ctypes.c_double), ("ewald_xi", ctypes.c_double)]


class SlipEx(ctypes.Structure):
    """mbs_slip_ex: septlet gamma [n, 10], vortlet psi [n, 5], spinlet lambda [n, 10] (NULL = zero)."""
    _fields_ = [("gam", ctypes.c_void_p), ("psi", ctypes.c_void_p), ("lam", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("fp64_matvecs", ctypes.c_int32), ("fp32_matvecs", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("t_rhs_ms", ctypes.c_double), ("t_iter_ms", ctypes.c_double),
                ("t_out_ms", ctypes.c_double), ("pair_blocks", ctypes.c_double),
                ("t_op64_ms", ctypes.c_double), ("t_op32_ms", ctypes.c_double),
                ("out_fused", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmbstokes.so not found at {path}: build it with "
                           "`python -m paper_1411_0278_amd.build` (no fallback path exists)")
    lib = ctypes.CDLL(path)
    P, D, I32, I64, VP = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.mbs_default_params.argtypes = [ctypes.POINTER(Params)]
    lib.mbs_default_params.restype = None
    lib.mbs_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(Params)]
    lib.mbs_create.restype = ctypes.c_int
    lib.mbs_destroy.argtypes = [P]
    lib.mbs_destroy.restype = None
    lib.mbs_set_params.argtypes = [P, ctypes.POINTER(Params)]
    lib.mbs_set_params.restype = ctypes.c_int
    lib.mbs_last_error.argtypes = [P]
    lib.mbs_last_error.restype = ctypes.c_char_p
    lib.mbs_solve.argtypes = [P, I64] + [P] * 12 + [ctypes.POINTER(Stats), VP]
    lib.mbs_solve.restype = ctypes.c_int
    lib.mbs_matvec.argtypes = [P, I64, P, P, P, ctypes.c_int, VP]
    lib.mbs_matvec.restype = ctypes.c_int
    lib.mbs_matvec_static.argtypes = [P, I64, P, P, P, ctypes.c_int, VP]
    lib.mbs_matvec_static.restype = ctypes.c_int
    lib.mbs_rhs.argtypes = [P, I64, P, P, P, P, P, P, VP]
    lib.mbs_rhs.restype = ctypes.c_int
    lib.mbs_outputs.argtypes = [P, I64] + [P] * 10 + [VP]
    lib.mbs_outputs.restype = ctypes.c_int
    lib.mbs_flow.argtypes = [P, I64, P, I64, P, P, P, P, P, P, VP]
    lib.mbs_flow.restype = ctypes.c_int
    lib.mbs_step.argtypes = [P, I64, P, P, D, ctypes.POINTER(ctypes.c_double), D, I32, I32, P, I32,
                             ctypes.POINTER(Stats), ctypes.POINTER(ctypes.c_double), VP]
    lib.mbs_step.restype = ctypes.c_int
    lib.mbs_solve_batched.argtypes = [P, I32, ctypes.POINTER(ctypes.c_int64)] + [P] * 10 + [
        ctypes.POINTER(Stats), ctypes.POINTER(ctypes.c_double), VP]
    lib.mbs_solve_batched.restype = ctypes.c_int
    lib.mbs_autotune.argtypes = [P, I64, P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32), VP]
    lib.mbs_autotune.restype = ctypes.c_int
    lib.mbs_autotune_batched.argtypes = [P, I32, ctypes.POINTER(ctypes.c_int64), P, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_double), VP]
    lib.mbs_autotune_batched.restype = ctypes.c_int
    FP = ctypes.POINTER(ctypes.c_float)
    lib.mbs_features.argtypes = [P, I64, P, P, P, P, VP]
    lib.mbs_features_ex.argtypes = [P, I64, P, P, P, P, P, VP]
    lib.mbs_warmstart_features.argtypes = [P, I32]
    lib.mbs_warmstart_init.argtypes = [P, ctypes.c_uint64]
    lib.mbs_warmstart_set.argtypes = [P, FP]
    lib.mbs_warmstart_get.argtypes = [P, FP]
    lib.mbs_warmstart_forward.argtypes = [P, I64, P, P, VP]
    lib.mbs_warmstart_grad.argtypes = [P, I64, P, P, FP, ctypes.POINTER(ctypes.c_double), VP]
    lib.mbs_warmstart_train.argtypes = [P, I64, P, P, I32, I32, D, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_double), VP]
    lib.mbs_warmstart_save.argtypes = [P, ctypes.c_char_p]
    lib.mbs_warmstart_load.argtypes = [P, ctypes.c_char_p]
    lib.mbs_warmstart_target.argtypes = [P, I64] + [P] * 7 + [VP]
    lib.mbs_precond_apply.argtypes = [P, I64, P, P, P, VP]
    lib.mbs_precond_apply.restype = ctypes.c_int
    lib.mbs_initial_guess.argtypes = [P, I64] + [P] * 6 + [I32, P, VP]
    EX = ctypes.POINTER(SlipEx)
    lib.mbs_solve_ex.argtypes = [P, I64] + [P] * 5 + [EX] + [P] * 7 + [ctypes.POINTER(Stats), VP]
    lib.mbs_rhs_ex.argtypes = [P, I64, P, P, P, EX, P, P, P, VP]
    lib.mbs_outputs_ex.argtypes = [P, I64, P, P, P, P, EX] + [P] * 6 + [VP]
    lib.mbs_flow_ex.argtypes = [P, I64, P, I64, P, P, P, P, P, EX, P, VP]
    lib.mbs_matvec_r3.argtypes = [P, I64, P, P, P, VP]
    lib.mbs_rhs_r3.argtypes = [P, I64, P, P, P, EX, P, P, P, VP]
    lib.mbs_outputs_r3.argtypes = [P, I64, P, P, P, EX] + [P] * 6 + [VP]
    lib.mbs_solve_r3.argtypes = [P, I64] + [P] * 4 + [EX] + [P] * 7 + [ctypes.POINTER(Stats), VP]
    lib.mbs_precond_apply_r3.argtypes = [P, I64, P, P, P, VP]
    for name in ("mbs_solve_ex", "mbs_rhs_ex", "mbs_outputs_ex", "mbs_flow_ex", "mbs_matvec_r3", "mbs_rhs_r3",
                 "mbs_outputs_r3", "mbs_solve_r3", "mbs_precond_apply_r3"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("mbs_warmstart_target", "mbs_initial_guess", "mbs_features", "mbs_features_ex",
                 "mbs_warmstart_features", "mbs_warmstart_init", "mbs_warmstart_set", "mbs_warmstart_get",
                 "mbs_warmstart_forward", "mbs_warmstart_grad", "mbs_warmstart_train", "mbs_warmstart_save",
                 "mbs_warmstart_load"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def default_params(**kw) -> Params:
    lib = load()
    p = Params()
    lib.mbs_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _ptr(t, n=None, width=None, name="array", dtype=None):
    """Device pointer of a CUDA tensor (None -> NULL), with dtype and shape checks (float64 default)."""
    if t is None:
        return None
    import torch
    dtype = dtype or torch.float64
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda:
        raise TypeError(f"{name}: expected a {dtype} CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if n is not None and width is not None and tuple(t.shape) != (n, width):
        raise ValueError(f"{name}: expected shape ({n}, {width}), got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A solver context on one GPU (wraps mbs_create / mbs_destroy)."""

    def __init__(self, device: int = 0, **params):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libmbstokes runs only on the device")
        self.lib = load()
        self.device = device
        self.params = default_params(**params)
        h = ctypes.c_void_p()
        torch.cuda.set_device(device)
        rc = self.lib.mbs_create(ctypes.byref(h), device, ctypes.byref(self.params))
        if rc != MBS_OK:
            raise MbsError(rc, self.lib.mbs_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.mbs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != MBS_OK and rc not in allow:
            raise MbsError(rc, self.lib.mbs_last_error(self.h).decode())
        return rc

    def set_params(self, **kw):
        for k, v in kw.items():
            if not hasattr(self.params, k):
                raise AttributeError(k)
            setattr(self.params, k, v)
        self._check(self.lib.mbs_set_params(self.h, ctypes.byref(self.params)))

    # ------------------------------------------------------------------ entry points
    def mbs_solve(self, R, p=None, v1s=None, v2s=None, v3t=None, Fe=None, Te=None, sigma0=None,
                  V=None, W=None, S=None, Sigma=None, allow_noconv=False):
        import torch
        n = R.shape[0]
        V = torch.empty((n, 3), dtype=torch.float64, device=R.device) if V is None else V
        W = torch.empty((n, 3), dtype=torch.float64, device=R.device) if W is None else W
        S = torch.empty((n, 5), dtype=torch.float64, device=R.device) if S is None else S
        st = Stats()
        rc = self.lib.mbs_solve(self.h, n, _ptr(R, n, 3, "R"), _ptr(p, n, 3, "p"), _ptr(v1s, n, 3, "v1s"),
                                _ptr(v2s, n, 5, "v2s"), _ptr(v3t, n, 3, "v3t"), _ptr(Fe, n, 3, "Fe"),
                                _ptr(Te, n, 3, "Te"), _ptr(sigma0, n, 5, "sigma0"), _ptr(V, n, 3, "V"),
                                _ptr(W, n, 3, "W"), _ptr(S, n, 5, "S"), _ptr(Sigma, n, 5, "Sigma"),
                                ctypes.byref(st), _stream())
        self._check(rc, (MBS_ENOCONV,) if allow_noconv else ())
        return V, W, S, st.as_dict()

    def mbs_matvec(self, R, x, y=None, precision=MBS_FP64):
        import torch
        n = R.shape[0]
        y = torch.empty((n, 5), dtype=torch.float64, device=R.device) if y is None else y
        self._check(self.lib.mbs_matvec(self.h, n, _ptr(R, n, 3, "R"), _ptr(x, n, 5, "x"),
                                        _ptr(y, n, 5, "y"), precision, _stream()))
        return y

    def mbs_matvec_static(self, R, x, y, precision=MBS_FP64):
        """The operator with the library's static scratch (no device allocation); y is required."""
        n = R.shape[0]
        self._check(self.lib.mbs_matvec_static(self.h, n, _ptr(R, n, 3, "R"), _ptr(x, n, 5, "x"),
                                               _ptr(y, n, 5, "y"), precision, _stream()))
        return y

    def mbs_rhs(self, R, v2s=None, v3t=None, Fe=None, Te=None, b=None):
        import torch
        n = R.shape[0]
        b = torch.empty((n, 5), dtype=torch.float64, device=R.device) if b is None else b
        self._check(self.lib.mbs_rhs(self.h, n, _ptr(R, n, 3, "R"), _ptr(v2s, n, 5, "v2s"),
                                     _ptr(v3t, n, 3, "v3t"), _ptr(Fe, n, 3, "Fe"), _ptr(Te, n, 3, "Te"),
                                     _ptr(b, n, 5, "b"), _stream()))
        return b

    def mbs_outputs(self, R, Sigma, v1s=None, v2s=None, v3t=None, Fe=None, Te=None, V=None, W=None, S=None):
        import torch
        n = R.shape[0]
        V = torch.empty((n, 3), dtype=torch.float64, device=R.device) if V is None else V
        W = torch.empty((n, 3), dtype=torch.float64, device=R.device) if W is None else W
        S = torch.empty((n, 5), dtype=torch.float64, device=R.device) if S is None else S
        self._check(self.lib.mbs_outputs(self.h, n, _ptr(R, n, 3, "R"), _ptr(v1s, n, 3, "v1s"),
                                         _ptr(v2s, n, 5, "v2s"), _ptr(v3t, n, 3, "v3t"), _ptr(Fe, n, 3, "Fe"),
                                         _ptr(Te, n, 3, "Te"), _ptr(Sigma, n, 5, "Sigma"), _ptr(V, n, 3, "V"),
                                         _ptr(W, n, 3, "W"), _ptr(S, n, 5, "S"), _stream()))
        return V, W, S

    def mbs_flow(self, X, R, Sigma, Fe=None, Te=None, v3t=None, U=None):
        import torch
        m, n = X.shape[0], R.shape[0]
        U = torch.empty((m, 3), dtype=torch.float64, device=X.device) if U is None else U
        self._check(self.lib.mbs_flow(self.h, m, _ptr(X, m, 3, "X"), n, _ptr(R, n, 3, "R"), _ptr(Fe, n, 3, "Fe"),
                                      _ptr(Te, n, 3, "Te"), _ptr(Sigma, n, 5, "Sigma"), _ptr(v3t, n, 3, "v3t"),
                                      _ptr(U, m, 3, "U"), _stream()))
        return U

    # ---- the higher slip modes (septlet gam [n, 10], vortlet psi [n, 5], spinlet lam [n, 10])
    @staticmethod
    def _slip_ex(n, gam, psi, lam):
        ex = SlipEx()
        ex.gam = _ptr(gam, n, 10, "gam")
        ex.psi = _ptr(psi, n, 5, "psi")
        ex.lam = _ptr(lam, n, 10, "lam")
        return ex

    def mbs_solve_ex(self, R, p=None, v1s=None, v2s=None, v3t=None, gam=None, psi=None, lam=None, Fe=None,
                     Te=None, sigma0=None, V=None, W=None, S=None, Sigma=None, allow_noconv=False):
        import torch
        n = R.shape[0]
        V = torch.empty((n, 3), dtype=torch.float64, device=R.device) if V is None else V
        W = torch.empty((n, 3), dtype=torch.float64, device=R.device) if W is None else W
        S = torch.empty((n, 5), dtype=torch.float64, device=R.device) if S is None else S
        ex = self._slip_ex(n, gam, psi, lam)
        st = Stats()
        rc = self.lib.mbs_solve_ex(self.h, n, _ptr(R, n, 3, "R"), _ptr(p, n, 3, "p"), _ptr(v1s, n, 3, "v1s"),
                                   _ptr(v2s, n, 5, "v2s"), _ptr(v3t, n, 3, "v3t"), ctypes.byref(ex),
                                   _ptr(Fe, n, 3, "Fe"), _ptr(Te, n, 3, "Te"), _ptr(sigma0, n, 5, "sigma0"),
                                   _ptr(V, n, 3, "V"), _ptr(W, n, 3, "W"), _ptr(S, n, 5, "S"),
                                   _ptr(Sigma, n, 5, "Sigma"), ctypes.byref(st), _stream())
        self._check(rc, (MBS_ENOCONV,) if allow_noconv else ())
        return V, W, S, st.as_dict()

    def mbs_rhs_ex(self, R, v2s=None, v3t=None, gam=None, psi=None, lam=None, Fe=None, Te=None, b=None):
        import torch
        n = R.shape[0]
        b = torch.empty((n, 5), dtype=torch.float64, device=R.device) if b is None else b
        ex = self._slip_ex(n, gam, psi, lam)
        self._check(self.lib.mbs_rhs_ex(self.h, n, _ptr(R, n, 3, "R"), _ptr(v2s, n, 5, "v2s"), _ptr(v3t, n, 3, "v3t"),
                                        ctypes.byref(ex), _ptr(Fe, n, 3, "Fe"), _ptr(Te, n, 3, "Te"),
                                        _ptr(b, n, 5, "b"), _stream()))
        return b

    def mbs_outputs_ex(self, R, Sigma, v1s=None, v2s=None, v3t=None, gam=None, psi=None, lam=None, Fe=None,
                       Te=None, V=None, W=None, S=None):
        import torch
        n = R.shape[0]
        V = torch.empty((n, 3), dtype=torch.float64, device=R.device) if V is None else V
        W = torch.empty((n, 3), dtype=torch.float64, device=R.device) if W is None else W
        S = torch.empty((n, 5), dtype=torch.float64, device=R.device) if S is None else S
        ex = self._slip_ex(n, gam, psi, lam)
        self._check(self.lib.mbs_outputs_ex(self.h, n, _ptr(R, n, 3, "R"), _ptr(v1s, n, 3, "v1s"),
                                            _ptr(v2s, n, 5, "v2s"), _ptr(v3t, n, 3, "v3t"), ctypes.byref(ex),
                                            _ptr(Fe, n, 3, "Fe"), _ptr(Te, n, 3, "Te"), _ptr(Sigma, n, 5, "Sigma"),
                                            _ptr(V, n, 3, "V"), _ptr(W, n, 3, "W"), _ptr(S, n, 5, "S"), _stream()))
        return V, W, S

    def mbs_flow_ex(self, X, R, Sigma, Fe=None, Te=None, v3t=None, gam=None, psi=None, lam=None, U=None):
        import torch
        m, n = X.shape[0], R.shape[0]
        U = torch.empty((m, 3), dtype=torch.float64, device=X.device) if U is None else U
        ex = self._slip_ex(n, gam, psi, lam)
        self._check(self.lib.mbs_flow_ex(self.h, m, _ptr(X, m, 3, "X"), n, _ptr(R, n, 3, "R"), _ptr(Fe, n, 3, "Fe"),
                                         _ptr(Te, n, 3, "Te"), _ptr(Sigma, n, 5, "Sigma"), _ptr(v3t, n, 3, "v3t"),
                                         ctypes.byref(ex), _ptr(U, m, 3, "U"), _stream()))
        return U

    # ---- traction ranks <= 3: unknowns x [n, 20] = [Sigma (5-basis), X^gam (7-basis), X^psi, X^d]
    def mbs_matvec_r3(self, R, x, y=None):
        import torch
        n = R.shape[0]
        y = torch.empty((n, R3_DIM), dtype=torch.float64, device=R.device) if y is None else y
        self._check(self.lib.mbs_matvec_r3(self.h, n, _ptr(R, n, 3, "R"), _ptr(x, n, R3_DIM, "x"),
                                           _ptr(y, n, R3_DIM, "y"), _stream()))
        return y

    def mbs_rhs_r3(self, R, v2s=None, v3t=None, gam=None, psi=None, lam=None, Fe=None, Te=None, b=None):
        import torch
        n = R.shape[0]
        b = torch.empty((n, R3_DIM), dtype=torch.float64, device=R.device) if b is None else b
        ex = self._slip_ex(n, gam, psi, lam)
        self._check(self.lib.mbs_rhs_r3(self.h, n, _ptr(R, n, 3, "R"), _ptr(v2s, n, 5, "v2s"), _ptr(v3t, n, 3, "v3t"),
                                        ctypes.byref(ex), _ptr(Fe, n, 3, "Fe"), _ptr(Te, n, 3, "Te"),
                                        _ptr(b, n, R3_DIM, "b"), _stream()))
        return b

    def mbs_outputs_r3(self, R, x, v1s=None, v2s=None, lam=None, Fe=None, Te=None, V=None, W=None, S=None):
        import torch
        n = R.shape[0]
        V = torch.empty((n, 3), dtype=torch.float64, device=R.device) if V is None else V
        W = torch.empty((n, 3), dtype=torch.float64, device=R.device) if W is None else W
        S = torch.empty((n, 5), dtype=torch.float64, device=R.device) if S is None else S
        ex = self._slip_ex(n, None, None, lam)
        self._check(self.lib.mbs_outputs_r3(self.h, n, _ptr(R, n, 3, "R"), _ptr(v1s, n, 3, "v1s"),
                                            _ptr(v2s, n, 5, "v2s"), ctypes.byref(ex), _ptr(Fe, n, 3, "Fe"),
                                            _ptr(Te, n, 3, "Te"), _ptr(x, n, R3_DIM, "x"), _ptr(V, n, 3, "V"),
                                            _ptr(W, n, 3, "W"), _ptr(S, n, 5, "S"), _stream()))
        return V, W, S

    def mbs_precond_apply_r3(self, R, x, y=None):
        import torch
        n = R.shape[0]
        y = torch.empty((n, R3_DIM), dtype=torch.float64, device=R.device) if y is None else y
        self._check(self.lib.mbs_precond_apply_r3(self.h, n, _ptr(R, n, 3, "R"), _ptr(x, n, R3_DIM, "x"),
                                                  _ptr(y, n, R3_DIM, "y"), _stream()))
        return y

    def mbs_solve_r3(self, R, v1s=None, v2s=None, v3t=None, gam=None, psi=None, lam=None, Fe=None, Te=None,
                     x0=None, V=None, W=None, S=None, x=None, allow_noconv=False):
        """Returns V, W, S, x [n, 20] and the stats."""
        import torch
        n = R.shape[0]
        V = torch.empty((n, 3), dtype=torch.float64, device=R.device) if V is None else V
        W = torch.empty((n, 3), dtype=torch.float64, device=R.device) if W is None else W
        S = torch.empty((n, 5), dtype=torch.float64, device=R.device) if S is None else S
        x = torch.empty((n, R3_DIM), dtype=torch.float64, device=R.device) if x is None else x
        ex = self._slip_ex(n, gam, psi, lam)
        st = Stats()
        rc = self.lib.mbs_solve_r3(self.h, n, _ptr(R, n, 3, "R"), _ptr(v1s, n, 3, "v1s"), _ptr(v2s, n, 5, "v2s"),
                                   _ptr(v3t, n, 3, "v3t"), ctypes.byref(ex), _ptr(Fe, n, 3, "Fe"),
                                   _ptr(Te, n, 3, "Te"), _ptr(x0, n, R3_DIM, "x0"), _ptr(V, n, 3, "V"),
                                   _ptr(W, n, 3, "W"), _ptr(S, n, 5, "S"), _ptr(x, n, R3_DIM, "x"),
                                   ctypes.byref(st), _stream())
        self._check(rc, (MBS_ENOCONV,) if allow_noconv else ())
        return V, W, S, x, st.as_dict()

    def mbs_step(self, R, p, k_trap, slip_coef, dt, nsteps, order=2, want_min_dist=False,
                 allow_noconv=False, hist=None, hist_valid=False):
        """hist: float64 device tensor [11 n] (V, Omega x p, Sigma of the previous step) or None."""
        n = R.shape[0]
        coef = (ctypes.c_double * 3)(*slip_coef)
        stats = (Stats * max(nsteps, 1))()
        md = (ctypes.c_double * max(nsteps, 1))() if want_min_dist else None
        rc = self.lib.mbs_step(self.h, n, _ptr(R, n, 3, "R"), _ptr(p, n, 3, "p"), float(k_trap), coef,
                               float(dt), int(nsteps), int(order), _ptr(hist.reshape(11 * n, 1) if hist is not None else None, 11 * n, 1, "hist"),
                               int(bool(hist_valid)), stats, md, _stream())
        self._check(rc, (MBS_ENOCONV,) if allow_noconv else ())
        return [stats[k].as_dict() for k in range(nsteps)], (list(md)[:nsteps] if md is not None else None)

    def mbs_solve_batched(self, offsets, R, v1s=None, v2s=None, v3t=None, Fe=None, Te=None,
                          V=None, W=None, S=None, Sigma=None):
        import torch
        nconf = len(offsets) - 1
        ntot = int(offsets[-1])
        off = (ctypes.c_int64 * (nconf + 1))(*[int(o) for o in offsets])
        V = torch.empty((ntot, 3), dtype=torch.float64, device=R.device) if V is None else V
        W = torch.empty((ntot, 3), dtype=torch.float64, device=R.device) if W is None else W
        S = torch.empty((ntot, 5), dtype=torch.float64, device=R.device) if S is None else S
        stats = (Stats * nconf)()
        lat = (ctypes.c_double * nconf)()
        rc = self.lib.mbs_solve_batched(self.h, nconf, off, _ptr(R, ntot, 3, "R"), _ptr(v1s, ntot, 3, "v1s"),
                                        _ptr(v2s, ntot, 5, "v2s"), _ptr(v3t, ntot, 3, "v3t"),
                                        _ptr(Fe, ntot, 3, "Fe"), _ptr(Te, ntot, 3, "Te"), _ptr(V, ntot, 3, "V"),
                                        _ptr(W, ntot, 3, "W"), _ptr(S, ntot, 5, "S"),
                                        _ptr(Sigma, ntot, 5, "Sigma"), stats, lat, _stream())
        self._check(rc)
        return V, W, S, [stats[b].as_dict() for b in range(nconf)], list(lat)


def _autotune_batched(self, offsets, R):
    nconf = len(offsets) - 1
    off = (ctypes.c_int64 * (nconf + 1))(*[int(o) for o in offsets])
    chosen = ctypes.c_int32()
    ms = (ctypes.c_double * 3)()
    self._check(self.lib.mbs_autotune_batched(self.h, nconf, off, _ptr(R, int(offsets[-1]), 3, "R"),
                                              ctypes.byref(chosen), ms, _stream()))
    return int(chosen.value), {64: ms[0], 128: ms[1], 256: ms[2]}


Context.mbs_autotune_batched = _autotune_batched


def _autotune(self, R, cache_json=None):
    n = R.shape[0]
    chosen = (ctypes.c_int32 * 2)()
    self._check(self.lib.mbs_autotune(self.h, n, _ptr(R, n, 3, "R"),
                                      cache_json.encode() if cache_json else None, chosen, _stream()))
    return int(chosen[0]), int(chosen[1])


Context.mbs_autotune = _autotune


def _features(self, R, p, want_nbr=False):
    import torch
    n = R.shape[0]
    feat = torch.empty((n, MLP_NFEAT), dtype=torch.float32, device=R.device)
    nbr = torch.empty((n, 16), dtype=torch.int32, device=R.device) if want_nbr else None
    self._check(self.lib.mbs_features(self.h, n, _ptr(R, n, 3, "R"), _ptr(p, n, 3, "p"),
                                      _ptr(feat, n, MLP_NFEAT, "feat", torch.float32),
                                      _ptr(nbr, n, 16, "nbr", torch.int32), _stream()))
    return (feat, nbr) if want_nbr else feat


def _mlp_sizes(self):
    """(input width, parameter count) of the context's feature set."""
    return _MLP_SIZES[getattr(self, "_mlp_set", MBS_FEATURES_GEOMETRY)]


def _ws_features(self, feature_set):
    self._check(self.lib.mbs_warmstart_features(self.h, int(feature_set)))
    self._mlp_set = int(feature_set)


def _features_ex(self, R, p, b=None, want_nbr=False):
    """Features of the context's feature set (b: the right-hand side [n, 5], needed by the wider set)."""
    import torch
    n = R.shape[0]
    width = _mlp_sizes(self)[0]
    feat = torch.empty((n, width), dtype=torch.float32, device=R.device)
    nbr = torch.empty((n, 16), dtype=torch.int32, device=R.device) if want_nbr else None
    self._check(self.lib.mbs_features_ex(self.h, n, _ptr(R, n, 3, "R"), _ptr(p, n, 3, "p"), _ptr(b, n, 5, "b"),
                                         _ptr(feat, n, width, "feat", torch.float32),
                                         _ptr(nbr, n, 16, "nbr", torch.int32), _stream()))
    return (feat, nbr) if want_nbr else feat


def _ws_init(self, seed=0):
    self._check(self.lib.mbs_warmstart_init(self.h, int(seed)))


def _ws_set(self, params):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    npar = _mlp_sizes(self)[1]
    if a.size != npar:
        raise ValueError(f"expected {npar} parameters")
    self._check(self.lib.mbs_warmstart_set(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))


def _ws_get(self):
    import numpy as np
    a = np.empty(_mlp_sizes(self)[1], dtype=np.float32)
    self._check(self.lib.mbs_warmstart_get(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return a


def _ws_forward(self, feat):
    import torch
    m = feat.shape[0]
    out = torch.empty((m, 5), dtype=torch.float32, device=feat.device)
    self._check(self.lib.mbs_warmstart_forward(self.h, m, _ptr(feat, m, _mlp_sizes(self)[0], "feat", torch.float32),
                                               _ptr(out, m, 5, "out", torch.float32), _stream()))
    return out


def _ws_grad(self, feat, target):
    import numpy as np
    import torch
    m = feat.shape[0]
    g = np.empty(_mlp_sizes(self)[1], dtype=np.float32)
    loss = ctypes.c_double()
    self._check(self.lib.mbs_warmstart_grad(self.h, m, _ptr(feat, m, _mlp_sizes(self)[0], "feat", torch.float32),
                                            _ptr(target, m, 5, "target", torch.float32),
                                            g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                            ctypes.byref(loss), _stream()))
    return loss.value, g


def _ws_train(self, feat, target, epochs, batch=4096, lr=1e-3, seed=0):
    import torch
    m = feat.shape[0]
    hist = (ctypes.c_double * max(epochs, 1))()
    self._check(self.lib.mbs_warmstart_train(self.h, m, _ptr(feat, m, _mlp_sizes(self)[0], "feat", torch.float32),
                                             _ptr(target, m, 5, "target", torch.float32), int(epochs),
                                             int(batch), float(lr), int(seed), hist, _stream()))
    return list(hist)[:epochs]


def _ws_save(self, path):
    self._check(self.lib.mbs_warmstart_save(self.h, str(path).encode()))


def _ws_load(self, path):
    import struct
    self._check(self.lib.mbs_warmstart_load(self.h, str(path).encode()))
    with open(path, "rb") as f:  # the library selected the file's feature set: follow it
        magic, version, _ = struct.unpack("<III", f.read(12))
        self._mlp_set = struct.unpack("<I", f.read(4))[0] if version == 2 else MBS_FEATURES_GEOMETRY


def _ws_target(self, R, Sigma, v2s=None, v3t=None, Fe=None, Te=None):
    import torch
    n = R.shape[0]
    t = torch.empty((n, 5), dtype=torch.float32, device=R.device)
    self._check(self.lib.mbs_warmstart_target(self.h, n, _ptr(R, n, 3, "R"), _ptr(v2s, n, 5, "v2s"),
                                              _ptr(v3t, n, 3, "v3t"), _ptr(Fe, n, 3, "Fe"), _ptr(Te, n, 3, "Te"),
                                              _ptr(Sigma, n, 5, "Sigma"), _ptr(t, n, 5, "target", torch.float32),
                                              _stream()))
    return t


def _initial_guess(self, R, guess, p=None, v2s=None, v3t=None, Fe=None, Te=None):
    import torch
    n = R.shape[0]
    out = torch.empty((n, 5), dtype=torch.float64, device=R.device)
    self._check(self.lib.mbs_initial_guess(self.h, n, _ptr(R, n, 3, "R"), _ptr(p, n, 3, "p"),
                                           _ptr(v2s, n, 5, "v2s"), _ptr(v3t, n, 3, "v3t"), _ptr(Fe, n, 3, "Fe"),
                                           _ptr(Te, n, 3, "Te"), int(guess), _ptr(out, n, 5, "sigma0"),
                                           _stream()))
    return out


def _precond_apply(self, R, x):
    import torch
    n = R.shape[0]
    y = torch.empty((n, 5), dtype=torch.float64, device=R.device)
    self._check(self.lib.mbs_precond_apply(self.h, n, _ptr(R, n, 3, "R"), _ptr(x, n, 5, "x"),
                                           _ptr(y, n, 5, "y"), _stream()))
    return y


Context.mbs_precond_apply = _precond_apply
Context.mbs_warmstart_target = _ws_target
Context.mbs_initial_guess = _initial_guess
Context.mbs_features = _features
Context.mbs_features_ex = _features_ex
Context.mbs_warmstart_features = _ws_features
Context.mbs_warmstart_init = _ws_init
Context.mbs_warmstart_set = _ws_set
Context.mbs_warmstart_get = _ws_get
Context.mbs_warmstart_forward = _ws_forward
Context.mbs_warmstart_grad = _ws_grad
Context.mbs_warmstart_train = _ws_train
Context.mbs_warmstart_save = _ws_save
Context.mbs_warmstart_load = _ws_load


def to_device(w, device="cuda"):
    """Copy a paper_1411_0278_amd.inputs.Workload's arrays to float64 device tensors."""
    import torch
    f = lambda a: torch.as_tensor(a, dtype=torch.float64).contiguous().to(device)
    d = dict(R=f(w.R), p=f(w.p), v1s=f(w.v1s), v2s=f(w.v2s), v3t=f(w.v3t), Fe=f(w.Fe), Te=f(w.Te))
    for k in ("gam", "psi", "lam"):  # the higher slip modes, when the workload has them
        if getattr(w, k, None) is not None:
            d[k] = f(getattr(w, k))
    return d
