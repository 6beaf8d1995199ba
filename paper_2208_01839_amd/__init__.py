"""Python binding of libseird (the SEIRD implicit-step library for MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libseird.so`` behind the C ABI declared in ``include/seird.h``.
PyTorch supplies device memory (float64 CUDA tensors) and the current HIP
stream.  If the shared library is missing, every entry point raises; there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Mesh", "Problem", "Precond", "PicardGS", "Batch", "workspace_bytes", "create_in_workspace", "SeirdError", "autotune", "tune_cache_clear", "gmres", "gmres_noalloc", "step",
           "forward_record", "adjoint", "SEIRDRun", "lib", "library_path"]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libseird.so")
_lib = None


class SeirdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libseird error {code}: {msg}")
        self.code = code


STATUS = {0: "OK", -1: "ARG", -2: "MESH", -3: "HIP", -4: "NONFINITE",
          -5: "BREAKDOWN", -6: "DIVERGED", -7: "NOT_CONVERGED", -8: "WORKSPACE", -9: "STATE"}


class _Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("sigma", "gamma_E", "gamma_R", "gamma_D", "A", "alpha", "mu",
                 "beta_I", "beta_E")] + [("nu", ctypes.c_double * 5)]


class _Schwarz(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("factor_prec", ctypes.c_int32),
                ("n_ref", ctypes.c_int32),
                ("level_n", ctypes.POINTER(ctypes.c_int64)),
                ("parents", ctypes.POINTER(ctypes.c_int32))]


class _Krylov(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_it", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("dtol", ctypes.c_double), ("graphs", ctypes.c_int32)]


class _KStats(ctypes.Structure):
    _fields_ = [("its", ctypes.c_int32), ("reason", ctypes.c_int32),
                ("resid", ctypes.c_double), ("bnorm", ctypes.c_double)]


class _Newton(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_it", ctypes.c_int32), ("pc_reuse", ctypes.c_int32),
                ("strict_linear", ctypes.c_int32), ("pc_keep_steps", ctypes.c_int32)]


MAX_NEWTON = 32


class _SStats(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int32), ("gmres_its_total", ctypes.c_int32),
                ("gmres_its", ctypes.c_int32 * MAX_NEWTON),
                ("res_hist", ctypes.c_double * (MAX_NEWTON + 1)),
                ("eps", ctypes.c_double), ("reason", ctypes.c_int32),
                ("pc_setups", ctypes.c_int32), ("t_residual_ms", ctypes.c_double), ("t_jacobian_ms", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_gmres_ms", ctypes.c_double),
                ("t_ras_kernel_ms", ctypes.c_double), ("n_ras_launches", ctypes.c_int32),
                ("ras_bytes_per_launch", ctypes.c_double), ("backtracks", ctypes.c_int32),
                ("inexact_solves", ctypes.c_int32)]


class _SInfo(ctypes.Structure):
    _fields_ = [("factor_entries", ctypes.c_int64), ("local_unknowns", ctypes.c_int64),
                ("max_local_nodes", ctypes.c_int32), ("max_bandwidth", ctypes.c_int32),
                ("mean_bandwidth", ctypes.c_double), ("coarse_n", ctypes.c_int64),
                ("coarse_bandwidth", ctypes.c_int32), ("lu_mfma_flops", ctypes.c_double),
                ("lu_useful_flops", ctypes.c_double)]


class _PerfReport(ctypes.Structure):
    _fields_ = [("lu_mfma_flops", ctypes.c_double), ("lu_useful_flops", ctypes.c_double),
                ("factor_bytes", ctypes.c_double), ("solve_bytes", ctypes.c_double),
                ("setups", ctypes.c_int32), ("t_extract_ms", ctypes.c_double), ("t_lu_ms", ctypes.c_double)]


class _CoarseKrylovOpts(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int32), ("overlap", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("max_it", ctypes.c_int32), ("rtol", ctypes.c_double), ("atol", ctypes.c_double)]


class _CoarseKrylovStats(ctypes.Structure):
    _fields_ = [("solves", ctypes.c_int64), ("its", ctypes.c_int64), ("its_max", ctypes.c_int64),
                ("unconverged", ctypes.c_int64), ("coarse_subdomains", ctypes.c_int32),
                ("coarse_local_unknowns", ctypes.c_int64), ("amg_levels", ctypes.c_int32),
                ("amg_last_nodes", ctypes.c_int64)]


class _CoarseAmgOpts(ctypes.Structure):
    _fields_ = [("max_coarse", ctypes.c_int32), ("nu", ctypes.c_int32), ("omega", ctypes.c_double),
                ("restart", ctypes.c_int32), ("max_it", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("atol", ctypes.c_double)]


MAX_PGS = 64
NC22 = 22
_P22_FIELDS = ["beta_A", "beta_F", "beta_B", "beta_C", "r_V", "delta_S", "delta_V",
               "gamma_A", "gamma_C", "gamma_DA", "gamma_DM", "gamma_E", "gamma_I", "gamma_L",
               "gamma_M", "gamma_P", "gamma_R", "gamma_S1", "gamma_S2", "gamma_T", "gamma_V",
               "sigma_A", "sigma_C", "sigma_H", "sigma_S", "pi_A", "pi_B", "pi_C", "pi_H",
               "phi_C", "phi_M", "phi_S", "phi_P", "kappa_H", "kappa_I", "kappa_N", "kappa_P"]


class _Params22(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in _P22_FIELDS] + [("nu", ctypes.c_double * 10)]


class _Stats22(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("gmres_its", ctypes.c_int32 * 22),
                ("eps_hist", ctypes.c_double * 64), ("res_scaled", ctypes.c_double),
                ("pc_setups", ctypes.c_int32), ("inexact_solves", ctypes.c_int32),
                ("reason", ctypes.c_int32), ("t_setup_ms", ctypes.c_double),
                ("t_gmres_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double)]


class _PgsOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_sweeps", ctypes.c_int32), ("strict_linear", ctypes.c_int32),
                ("pc_lag", ctypes.c_int32)]


class _PgsStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("gmres_its", ctypes.c_int32 * 5),
                ("eps_hist", ctypes.c_double * MAX_PGS), ("res_scaled", ctypes.c_double),
                ("pc_setups", ctypes.c_int32), ("inexact_solves", ctypes.c_int32), ("reason", ctypes.c_int32),
                ("t_setup_ms", ctypes.c_double), ("t_gmres_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double)]


class _WsOpts(ctypes.Structure):
    _fields_ = [("restart_max", ctypes.c_int32), ("tape_states", ctypes.c_int32),
                ("n_regions_max", ctypes.c_int32), ("csr_pattern", ctypes.c_int32)]


class _AStats(ctypes.Structure):
    _fields_ = [("gmres_its_total", ctypes.c_int32), ("recomputed_steps", ctypes.c_int32),
                ("t_forward_ms", ctypes.c_double), ("t_reverse_ms", ctypes.c_double),
                ("setups", ctypes.c_int32)]


class _TuneCand(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("solve_threads", ctypes.c_int32), ("status", ctypes.c_int32),
                ("setup_ms", ctypes.c_double), ("apply_ms", ctypes.c_double), ("score_ms", ctypes.c_double)]


TUNE_MAX = 8


class _TuneReport(ctypes.Structure):
    _fields_ = [("best_tile", ctypes.c_int32), ("best_solve_threads", ctypes.c_int32),
                ("n_candidates", ctypes.c_int32), ("cand", _TuneCand * TUNE_MAX),
                ("from_cache", ctypes.c_int32)]


_P = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)
_SIGS = {
    "seird_last_error": ([], ctypes.c_char_p),
    "seird_version": ([], ctypes.c_char_p),
    "seird_device_allocations": ([_I64P, _I64P], ctypes.c_int),
    "seird_problem_create": ([ctypes.c_int64, _P, ctypes.c_int64, _P,
                              ctypes.POINTER(_Params), ctypes.POINTER(_P)], ctypes.c_int),
    "seird_problem_destroy": ([_P], None),
    "seird_mesh_create": ([ctypes.c_int64, _P, ctypes.c_int64, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "seird_mesh_destroy": ([_P], None),
    "seird_mesh_info": ([_P, _I64P, _I64P], ctypes.c_int),
    "seird_problem_create_from_mesh": ([_P, ctypes.POINTER(_Params), ctypes.POINTER(_P)], ctypes.c_int),
    "seird_workspace_bytes": ([_P, ctypes.POINTER(_Schwarz), _P, ctypes.POINTER(_WsOpts), _I64P], ctypes.c_int),
    "seird_create_in_workspace": ([_P, ctypes.POINTER(_Params), ctypes.POINTER(_Schwarz), _P,
                                   ctypes.POINTER(_WsOpts), _P, ctypes.c_int64, ctypes.POINTER(_P),
                                   ctypes.POINTER(_P)], ctypes.c_int),
    "seird_csr": ([_P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), _I64P, _I64P],
                  ctypes.c_int),
    "seird_csr_values": ([_P, _P, _P, _P], ctypes.c_int),
    "seird_set_params": ([_P, ctypes.POINTER(_Params)], ctypes.c_int),
    "seird_set_beta_field": ([_P, _P, _P], ctypes.c_int),
    "seird_set_beta_schedule": ([_P, _P], ctypes.c_int),
    "seird_set_time": ([_P, ctypes.c_double], ctypes.c_int),
    "seird_get_time": ([_P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "seird_set_beta_regional": ([_P] + [ctypes.c_double] * 7 + [_P], ctypes.c_int),
    "seird_set_mass": ([_P, ctypes.c_int32], ctypes.c_int),
    "seird_set_boundary_flux": ([_P, _P, _P], ctypes.c_int),
    "seird_problem_info": ([_P, _I64P, _I64P], ctypes.c_int),
    "seird_pattern": ([_P, _P, _P], ctypes.c_int),
    "seird_lumped_mass": ([_P, _P, _P], ctypes.c_int),
    "seird_residual": ([_P, _P, _P, ctypes.c_double, _P, _P, _P], ctypes.c_int),
    "seird_jacobian_size": ([_P, _I64P], ctypes.c_int),
    "seird_jacobian": ([_P, _P, ctypes.c_double, _P, _P], ctypes.c_int),
    "seird_spmv": ([_P, _P, _P, _P, ctypes.c_int, _P], ctypes.c_int),
    "seird_precond_create": ([_P, ctypes.POINTER(_Schwarz), _P, ctypes.POINTER(_P)], ctypes.c_int),
    "seird_precond_destroy": ([_P], None),
    "seird_precond_info": ([_P, _I64P, _I64P, _I32P, _I32P], ctypes.c_int),
    "seird_precond_setup": ([_P, _P, _P], ctypes.c_int),
    "seird_precond_setup_scalar": ([_P, _P, _P, _P], ctypes.c_int),
    "seird_precond_timing": ([_P, ctypes.c_int], ctypes.c_int),
    "seird_precond_perf": ([_P, ctypes.POINTER(_PerfReport), ctypes.c_int], ctypes.c_int),
    "seird_precond_set_solve_threads": ([_P, ctypes.c_int32], ctypes.c_int),
    "seird_precond_set_coarse_solver": ([_P, ctypes.c_int32], ctypes.c_int),
    "seird_precond_set_coarse_block": ([_P, ctypes.c_int32], ctypes.c_int),
    "seird22_create": ([_P, ctypes.POINTER(_Params22), ctypes.POINTER(_Schwarz), _P, ctypes.POINTER(_P)],
                       ctypes.c_int),
    "seird22_destroy": ([_P], None),
    "seird22_set_params": ([_P, ctypes.POINTER(_Params22)], ctypes.c_int),
    "seird22_residual": ([_P, _P, _P, ctypes.c_double, _P, _P], ctypes.c_int),
    "seird22_step": ([_P, _P, ctypes.c_double, ctypes.POINTER(_PgsOpts), ctypes.POINTER(_Krylov),
                      ctypes.POINTER(_Stats22), _P], ctypes.c_int),
    "seird_precond_set_coarse_krylov": ([_P, ctypes.POINTER(_CoarseKrylovOpts)], ctypes.c_int),
    "seird_precond_coarse_krylov_stats": ([_P, ctypes.POINTER(_CoarseKrylovStats), ctypes.c_int], ctypes.c_int),
    "seird_precond_set_coarse_amg": ([_P, ctypes.POINTER(_CoarseAmgOpts)], ctypes.c_int),
    "seird_autotune_schwarz": ([_P, ctypes.POINTER(_Schwarz), _P, _P, ctypes.c_int32, ctypes.c_int32,
                                ctypes.POINTER(_TuneReport), _P], ctypes.c_int),
    "seird_tune_cache_clear": ([], ctypes.c_int),
    "seird_batch_autotune": ([_P, ctypes.c_int32, ctypes.POINTER(_TuneReport), _P], ctypes.c_int),
    "seird_analyze_schwarz": ([ctypes.c_int64, _P, ctypes.c_int64, _P, ctypes.POINTER(_Schwarz), _P,
                               ctypes.POINTER(_SInfo), _P, _P], ctypes.c_int),
    "seird_precond_apply": ([_P, _P, _P, ctypes.c_int, _P], ctypes.c_int),
    "seird_gmres": ([_P, _P, _P, _P, _P, ctypes.POINTER(_Krylov),
                     ctypes.POINTER(_KStats), ctypes.c_int, _P], ctypes.c_int),
    "seird_gmres_noalloc": ([_P, _P, _P, _P, _P, ctypes.POINTER(_Krylov),
                             ctypes.POINTER(_KStats), ctypes.c_int, _P], ctypes.c_int),
    "seird_step": ([_P, _P, _P, ctypes.c_double, _P, ctypes.POINTER(_Newton),
                    ctypes.POINTER(_Krylov), ctypes.POINTER(_SStats), _P], ctypes.c_int),
    "seird_forward_record": ([_P, _P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _P,
                              ctypes.c_int32, _P, ctypes.POINTER(_Newton), ctypes.POINTER(_Krylov), _P],
                             ctypes.c_int),
    "seird_adjoint": ([_P, _P, _P, _P, _P, ctypes.POINTER(_Krylov), ctypes.POINTER(_AStats), _P],
                      ctypes.c_int),
    "seird_pgs_create": ([_P, ctypes.POINTER(_Schwarz), _P, ctypes.POINTER(_P)], ctypes.c_int),
    "seird_pgs_destroy": ([_P], None),
    "seird_pgs_precond": ([_P, _P], ctypes.c_int),
    "seird_pgs_step": ([_P, _P, ctypes.c_double, ctypes.POINTER(_PgsOpts), ctypes.POINTER(_Krylov),
                        ctypes.POINTER(_PgsStats), _P], ctypes.c_int),
    "seird_batch_create": ([ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_int32, ctypes.POINTER(_P)], ctypes.c_int),
    "seird_batch_destroy": ([_P], None),
    "seird_batch_info": ([_P, _P], ctypes.c_int),
    "seird_batch_precond": ([_P, _P], ctypes.c_int),
    "seird_batch_step": ([_P, _P, ctypes.c_double, ctypes.POINTER(_Newton), ctypes.POINTER(_Krylov),
                          _P, _P], ctypes.c_int),
}


def lib():
    """Load libseird.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise RuntimeError(f"libseird.so not built ({library_path}); run "
                               "paper_2208_01839_amd/build.py")
        L = ctypes.CDLL(library_path)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        msg = lib().seird_last_error().decode()
        raise SeirdError(code, f"{STATUS.get(code, code)}: {msg}")


def _torch():
    import torch
    return torch


def _dptr(t, n=None, name="tensor"):
    """Device pointer of a contiguous float64 CUDA tensor."""
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _params(p) -> _Params:
    c = _Params()
    for k in ("sigma", "gamma_E", "gamma_R", "gamma_D", "A", "alpha", "mu",
              "beta_I", "beta_E"):
        setattr(c, k, float(getattr(p, k)))
    for k in range(5):
        c.nu[k] = float(p.nu[k])
    return c


def _krylov(restart=30, max_it=200, rtol=1e-5, atol=1e-50, dtol=1e5, graphs=0):
    return _Krylov(int(restart), int(max_it), float(rtol), float(atol), float(dtol), int(bool(graphs)))


class Mesh:
    """A validated triangle mesh held on the host (node graph, element
    incidence, lumped mass); problems are created from it."""

    def __init__(self, xy, tri):
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().seird_mesh_create(len(xy), xy.ctypes.data, len(tri), tri.ctypes.data, ctypes.byref(h)))
        self.h = h
        n, ns = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().seird_mesh_info(self.h, ctypes.byref(n), ctypes.byref(ns)))
        self.n, self.nslots = n.value, ns.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.seird_mesh_destroy(self.h)
            self.h = None


def device_allocations():
    """(count, bytes) of the device allocations the library has made."""
    c, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().seird_device_allocations(ctypes.byref(c), ctypes.byref(b)))
    return c.value, b.value


def _ws_opts(restart_max=30, tape_states=0, n_regions_max=0, csr_pattern=False):
    return _WsOpts(int(restart_max), int(tape_states), int(n_regions_max), int(bool(csr_pattern)))


def workspace_bytes(mesh: Mesh, part=None, n_sub=0, overlap=0, tile=32, factor_prec=0, coarse=None, **ws):
    """Bytes of device workspace for a problem on ``mesh`` and (with a
    partition) its Schwarz preconditioner; ``ws``: restart_max, tape_states,
    n_regions_max, csr_pattern (see seird_workspace_opts)."""
    wo = _ws_opts(**ws)
    b = ctypes.c_int64()
    if part is None:
        _check(lib().seird_workspace_bytes(mesh.h, None, None, ctypes.byref(wo), ctypes.byref(b)))
    else:
        part = np.ascontiguousarray(part, dtype=np.int32)
        o, keep = _schwarz_opts(n_sub, overlap, tile, factor_prec, coarse)
        _check(lib().seird_workspace_bytes(mesh.h, ctypes.byref(o), part.ctypes.data, ctypes.byref(wo),
                                           ctypes.byref(b)))
        del keep
    return b.value


def create_in_workspace(mesh: Mesh, params, workspace, part=None, n_sub=0, overlap=0, tile=32, factor_prec=0,
                        coarse=None, **ws):
    """(Problem, Precond or None) whose device arrays all live in
    ``workspace`` (a CUDA uint8 tensor of at least workspace_bytes(...)
    bytes, kept alive by the returned handles)."""
    torch = _torch()
    if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or workspace.dtype != torch.uint8:
        raise TypeError("workspace must be a CUDA uint8 tensor")
    wo = _ws_opts(**ws)
    pr = _params(params)
    hp, hc = ctypes.c_void_p(), ctypes.c_void_p()
    if part is None:
        _check(lib().seird_create_in_workspace(mesh.h, ctypes.byref(pr), None, None, ctypes.byref(wo),
                                               ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                               ctypes.byref(hp), None))
    else:
        part = np.ascontiguousarray(part, dtype=np.int32)
        o, keep = _schwarz_opts(n_sub, overlap, tile, factor_prec, coarse)
        _check(lib().seird_create_in_workspace(mesh.h, ctypes.byref(pr), ctypes.byref(o), part.ctypes.data,
                                               ctypes.byref(wo), ctypes.c_void_p(workspace.data_ptr()),
                                               workspace.numel(), ctypes.byref(hp), ctypes.byref(hc)))
        del keep
    prob = Problem._from_handle(hp, params, workspace)
    pc = Precond._from_handle(hc, prob, workspace) if part is not None else None
    return prob, pc


class Problem:
    """A SEIRD problem on a triangle mesh (host arrays are copied)."""

    def __init__(self, xy, tri, params):
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        h = ctypes.c_void_p()
        self._params = _params(params)
        _check(lib().seird_problem_create(len(xy), xy.ctypes.data, len(tri),
                                          tri.ctypes.data, ctypes.byref(self._params),
                                          ctypes.byref(h)))
        self._init_handle(h)

    @classmethod
    def from_mesh(cls, mesh: Mesh, params):
        h = ctypes.c_void_p()
        pr = _params(params)
        _check(lib().seird_problem_create_from_mesh(mesh.h, ctypes.byref(pr), ctypes.byref(h)))
        obj = cls.__new__(cls)
        obj._params = pr
        obj._init_handle(h)
        return obj

    @classmethod
    def _from_handle(cls, h, params, workspace):
        obj = cls.__new__(cls)
        obj._params = _params(params)
        obj._workspace = workspace  # keeps the device memory alive
        obj._init_handle(h)
        return obj

    def _init_handle(self, h):
        self.h = h
        ni = ctypes.c_int64()
        _check(lib().seird_problem_info(self.h, ctypes.byref(ni), None))
        self.n = ni.value
        self.N = 5 * self.n
        nv = ctypes.c_int64()
        _check(lib().seird_jacobian_size(self.h, ctypes.byref(nv)))
        self.nvals = nv.value
        ns = ctypes.c_int64()
        _check(lib().seird_problem_info(self.h, None, ctypes.byref(ns)))
        self.nslots = ns.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.seird_problem_destroy(self.h)
            self.h = None

    def set_params(self, params):
        self._params = _params(params)
        _check(lib().seird_set_params(self.h, ctypes.byref(self._params)))

    def set_beta_field(self, g):
        _check(lib().seird_set_beta_field(self.h, _dptr(g, self.n, "g"), _stream()))

    def set_beta_schedule(self, a=None, b=0.0, k=1.0, tc=0.0):
        """Time profile of the transmission rate (Eq. beta_ie): beta times
        a - b / (1 + exp(k (tc - t))); a=None removes it."""
        if a is None:
            _check(lib().seird_set_beta_schedule(self.h, None))
            return
        arr = (ctypes.c_double * 4)(float(a), float(b), float(k), float(tc))
        _check(lib().seird_set_beta_schedule(self.h, ctypes.cast(arr, ctypes.c_void_p)))

    def set_time(self, t):
        _check(lib().seird_set_time(self.h, float(t)))

    def get_time(self):
        t = ctypes.c_double()
        _check(lib().seird_get_time(self.h, ctypes.byref(t)))
        return t.value

    def set_beta_regional(self, beta_c, beta_e, beta_w, x_e, x_w, k_e=5.0, k_w=10.0):
        """Regional transmission field along x (Eq. beta_x)."""
        _check(lib().seird_set_beta_regional(self.h, float(beta_c), float(beta_e), float(beta_w), float(x_e),
                                             float(x_w), float(k_e), float(k_w), _stream()))

    def set_mass(self, consistent):
        """Mass of the time-derivative term: lumped (False) or consistent."""
        _check(lib().seird_set_mass(self.h, int(bool(consistent))))

    def set_boundary_flux(self, q):
        """Neumann data: flux vectors [n, 5, 2] (float64 CUDA); None: zero."""
        _check(lib().seird_set_boundary_flux(self.h, _dptr(q, 10 * self.n, "q") if q is not None else None,
                                             _stream()))

    def pattern(self):
        rp = np.zeros(self.n + 1, dtype=np.int64)
        col = np.zeros(self.nslots, dtype=np.int32)
        _check(lib().seird_pattern(self.h, rp.ctypes.data, col.ctypes.data))
        return rp, col

    def lumped_mass(self, out=None):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.float64, device="cuda") if out is None else out
        _check(lib().seird_lumped_mass(self.h, _dptr(out, self.n, "out"), _stream()))
        return out

    def residual(self, u, u_prev, dt, src=None, out=None):
        torch = _torch()
        out = torch.empty_like(u) if out is None else out
        _check(lib().seird_residual(self.h, _dptr(u, self.N, "u"), _dptr(u_prev, self.N, "u_prev"),
                                    float(dt), _dptr(src, self.N, "src"), _dptr(out, self.N, "F"),
                                    _stream()))
        return out

    def jacobian(self, u, dt, out=None):
        torch = _torch()
        out = torch.empty(self.nvals, dtype=torch.float64, device=u.device) if out is None else out
        _check(lib().seird_jacobian(self.h, _dptr(u, self.N, "u"), float(dt),
                                    _dptr(out, self.nvals, "vals"), _stream()))
        return out

    def csr(self):
        """(rowptr, col) device tensors of the Jacobian's scalar CSR pattern
        (copies) and nnz; see seird_csr."""
        torch = _torch()
        rp, col = ctypes.c_void_p(), ctypes.c_void_p()
        nnz, nrows = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().seird_csr(self.h, ctypes.byref(rp), ctypes.byref(col), ctypes.byref(nnz), ctypes.byref(nrows)))
        self.csr_nnz = nnz.value
        hr = np.zeros(nrows.value + 1, dtype=np.int64)
        hc = np.zeros(nnz.value, dtype=np.int32)
        import ctypes as _c
        torch.cuda.synchronize()
        lib_hip = _hip()
        lib_hip.hipMemcpy(_c.c_void_p(hr.ctypes.data), rp, _c.c_size_t(hr.nbytes), 2)
        lib_hip.hipMemcpy(_c.c_void_p(hc.ctypes.data), col, _c.c_size_t(hc.nbytes), 2)
        return hr, hc

    def csr_values(self, vals, out=None):
        torch = _torch()
        if not hasattr(self, "csr_nnz"):
            self.csr()
        out = torch.empty(self.csr_nnz, dtype=torch.float64, device=vals.device) if out is None else out
        _check(lib().seird_csr_values(self.h, _dptr(vals, self.nvals, "vals"), _dptr(out, self.csr_nnz, "out"),
                                      _stream()))
        return out

    def spmv(self, vals, x, transpose=False, out=None):
        torch = _torch()
        out = torch.empty_like(x) if out is None else out
        _check(lib().seird_spmv(self.h, _dptr(vals, self.nvals, "vals"), _dptr(x, self.N, "x"),
                                _dptr(out, self.N, "y"), int(bool(transpose)), _stream()))
        return out


def _schwarz_opts(n_sub, overlap, tile, factor_prec, coarse):
    o = _Schwarz()
    o.n_sub, o.overlap, o.tile, o.factor_prec = int(n_sub), int(overlap), int(tile), int(factor_prec)
    keep = []
    if coarse is not None:
        parents, n_coarse = coarse
        level_n = np.array([n_coarse] + [len(p) for p in parents], dtype=np.int64)
        par = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.int32).reshape(-1)
                                                   for p in parents]), dtype=np.int32)
        keep = [level_n, par]
        o.n_ref = len(parents)
        o.level_n = level_n.ctypes.data_as(_I64P)
        o.parents = par.ctypes.data_as(_I32P)
    else:
        o.n_ref = 0
    return o, keep


def analyze_schwarz(xy, tri, part, n_sub, overlap, tile=32, coarse=None, maps=False):
    """Host-only decomposition analysis (no GPU needed).  Returns a dict of
    sizes; with maps=True also the local->global unknown map and owner flags
    of every subdomain, concatenated in subdomain order."""
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    part = np.ascontiguousarray(part, dtype=np.int32)
    o, keep = _schwarz_opts(n_sub, overlap, tile, 0, coarse)
    info = _SInfo()
    _check(lib().seird_analyze_schwarz(len(xy), xy.ctypes.data, len(tri), tri.ctypes.data,
                                       ctypes.byref(o), part.ctypes.data, ctypes.byref(info),
                                       None, None))
    out = {k: getattr(info, k) for k, _ in _SInfo._fields_}
    if maps:
        l2g = np.zeros(info.local_unknowns, dtype=np.int32)
        owned = np.zeros(info.local_unknowns, dtype=np.uint8)
        _check(lib().seird_analyze_schwarz(len(xy), xy.ctypes.data, len(tri), tri.ctypes.data,
                                           ctypes.byref(o), part.ctypes.data, ctypes.byref(info),
                                           l2g.ctypes.data, owned.ctypes.data))
        out["l2g"], out["owned"] = l2g, owned
    del keep
    return out


_hip_lib = None


def _hip():
    """The HIP runtime (for reading back library-owned device arrays)."""
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = ctypes.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip_lib.hipMemcpy.restype = ctypes.c_int
    return _hip_lib


class Precond:
    """Restricted additive Schwarz (one-level, or multiplicative two-grid
    when ``coarse = (parents_list, n_coarse)`` is given)."""

    @classmethod
    def _from_handle(cls, h, problem, workspace):
        obj = cls.__new__(cls)
        obj.problem = problem
        obj.h = h
        obj._vals = None
        obj._workspace = workspace
        return obj

    def __init__(self, problem: Problem, part, n_sub, overlap, tile=32,
                 factor_prec=0, coarse=None, solve_threads=256):
        self.problem = problem
        part = np.ascontiguousarray(part, dtype=np.int32)
        if len(part) != problem.n:
            raise ValueError("partition length must equal the node count")
        o, keep = _schwarz_opts(n_sub, overlap, tile, factor_prec, coarse)
        h = ctypes.c_void_p()
        _check(lib().seird_precond_create(problem.h, ctypes.byref(o), part.ctypes.data,
                                          ctypes.byref(h)))
        del keep
        self.h = h
        self._vals = None
        if solve_threads != 256:
            self.set_solve_threads(solve_threads)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.seird_precond_destroy(self.h)
            self.h = None

    def info(self):
        fe, cn = ctypes.c_int64(), ctypes.c_int64()
        mn, mb = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().seird_precond_info(self.h, ctypes.byref(fe), ctypes.byref(cn),
                                        ctypes.byref(mn), ctypes.byref(mb)))
        return dict(factor_entries=fe.value, coarse_n=cn.value,
                    max_local_nodes=mn.value, max_bandwidth=mb.value)

    def enable_timing(self, on=True):
        _check(lib().seird_precond_timing(self.h, int(bool(on))))

    def perf(self, reset=False):
        """Factorisation flop counts, factor bytes and (timing on) the
        HIP-event times of the setups since the last reset."""
        r = _PerfReport()
        _check(lib().seird_precond_perf(self.h, ctypes.byref(r), int(bool(reset))))
        return {k: getattr(r, k) for k, _ in _PerfReport._fields_}

    def set_solve_threads(self, threads):
        """Workgroup size of the subdomain solves (256; 128, 512 or 1024 with tile 32)."""
        _check(lib().seird_precond_set_solve_threads(self.h, int(threads)))

    def set_coarse_solver(self, solver):
        """1: block sweep over inverted diagonal super-blocks of the coarse
        factors; 0: band sweeps; 2: the Krylov coarse solver (after
        set_coarse_krylov)."""
        _check(lib().seird_precond_set_coarse_solver(self.h, int(solver)))

    def set_coarse_krylov(self, n_sub=0, overlap=1, restart=30, max_it=100, rtol=1e-5, atol=1e-50):
        """Two-grid RAS-V2: the coarse system solved by inner GMRES with RAS
        on the coarse graph (selects coarse solver 2; set up again before
        applying)."""
        o = _CoarseKrylovOpts(int(n_sub), int(overlap), int(restart), int(max_it), float(rtol), float(atol))
        _check(lib().seird_precond_set_coarse_krylov(self.h, ctypes.byref(o)))

    def set_coarse_amg(self, max_coarse=40, nu=1, omega=2.0 / 3.0, restart=30, max_it=100, rtol=1e-5,
                       atol=1e-50):
        """Two-grid RAS-V3: the coarse system solved by inner GMRES with an
        aggregation-AMG V-cycle (selects coarse solver 3; set up again
        before applying)."""
        o = _CoarseAmgOpts(int(max_coarse), int(nu), float(omega), int(restart), int(max_it), float(rtol),
                           float(atol))
        _check(lib().seird_precond_set_coarse_amg(self.h, ctypes.byref(o)))

    def coarse_krylov_stats(self, reset=False):
        r = _CoarseKrylovStats()
        _check(lib().seird_precond_coarse_krylov_stats(self.h, ctypes.byref(r), int(bool(reset))))
        return {k: getattr(r, k) for k, _ in _CoarseKrylovStats._fields_}

    def set_coarse_block(self, tiles):
        """Super-block size of the coarse inverses in tile rows (0: full
        inverses); takes effect at the next setup."""
        _check(lib().seird_precond_set_coarse_block(self.h, int(tiles)))

    def setup(self, vals):
        _check(lib().seird_precond_setup(self.h, _dptr(vals, self.problem.nvals, "vals"), _stream()))
        self._vals = vals  # the two-grid apply reads it

    def apply(self, r, transpose=False, out=None):
        out = _torch().empty_like(r) if out is None else out
        N = self.problem.N
        _check(lib().seird_precond_apply(self.h, _dptr(r, N, "r"), _dptr(out, N, "z"),
                                         int(bool(transpose)), _stream()))
        return out


def autotune(problem: Problem, part, n_sub, overlap, vals, factor_prec=0, coarse=None,
             applies_per_setup=15, reps=3):
    """Choose the tile size and the subdomain-solve workgroup size for this
    problem by timing every candidate on the Jacobian ``vals`` (see
    seird_autotune_schwarz).  Returns dict(tile, solve_threads, candidates)."""
    part = np.ascontiguousarray(part, dtype=np.int32)
    o, keep = _schwarz_opts(n_sub, overlap, 32, factor_prec, coarse)
    rep = _TuneReport()
    _check(lib().seird_autotune_schwarz(problem.h, ctypes.byref(o), part.ctypes.data,
                                        _dptr(vals, problem.nvals, "vals"), int(applies_per_setup),
                                        int(reps), ctypes.byref(rep), _stream()))
    del keep
    return _tune_dict(rep)


def _tune_dict(rep):
    cands = [dict(tile=c.tile, solve_threads=c.solve_threads, status=c.status, setup_ms=c.setup_ms,
                  apply_ms=c.apply_ms, score_ms=c.score_ms) for c in rep.cand[:rep.n_candidates]]
    return dict(tile=rep.best_tile, solve_threads=rep.best_solve_threads, candidates=cands,
                from_cache=bool(rep.from_cache))


def tune_cache_clear():
    """Empty the autotuner's in-process cache."""
    _check(lib().seird_tune_cache_clear())


def gmres(problem: Problem, pc, vals, b, transpose=False, x=None, **kw):
    """Solve J x = b (or J^T x = b).  Returns (x, stats dict)."""
    x = _torch().empty_like(b) if x is None else x
    o = _krylov(**kw)
    s = _KStats()
    code = lib().seird_gmres(problem.h, pc.h if pc is not None else None,
                             _dptr(vals, problem.nvals, "vals"), _dptr(b, problem.N, "b"),
                             _dptr(x, problem.N, "x"), ctypes.byref(o), ctypes.byref(s),
                             int(bool(transpose)), _stream())
    stats = dict(its=s.its, reason=s.reason, resid=s.resid, bnorm=s.bnorm, status=code)
    if code not in (0, -7):
        _check(code)
    return x, stats


STATIC_SCRATCH_BYTES = 64 << 20


def gmres_noalloc(problem: Problem, pc, vals, b, x, transpose=False, **kw):
    """seird_gmres_noalloc: the solve of ``gmres`` with its Krylov scratch in
    the library's fixed per-GPU array (no device allocation in the call).
    ``x`` (the output) must be given.  Returns the stats dict."""
    o = _krylov(**kw)
    s = _KStats()
    code = lib().seird_gmres_noalloc(problem.h, pc.h if pc is not None else None,
                                     _dptr(vals, problem.nvals, "vals"), _dptr(b, problem.N, "b"),
                                     _dptr(x, problem.N, "x"), ctypes.byref(o), ctypes.byref(s),
                                     int(bool(transpose)), _stream())
    stats = dict(its=s.its, reason=s.reason, resid=s.resid, bnorm=s.bnorm, status=code)
    if code not in (0, -7):
        _check(code)
    return stats


def step(problem: Problem, pc, u, dt, src=None, tol=1e-10, max_it=20, pc_reuse=0, strict_linear=False,
         gmres_max_it=200, pc_keep_steps=0, **kw):
    """One implicit step in place on u (float64 CUDA [n,5]).  Returns stats.
    max_it: Newton iterations; gmres_max_it: iterations of each GMRES solve.
    strict_linear: fail (NOT_CONVERGED) when a GMRES solve inside Newton
    stops at its max_it, instead of taking the inexact update.
    pc_keep_steps: a step's setup may serve this many later steps."""
    n = _Newton(float(tol), int(max_it), int(pc_reuse), int(bool(strict_linear)), int(pc_keep_steps))
    o = _krylov(max_it=gmres_max_it, **kw)
    s = _SStats()
    code = lib().seird_step(problem.h, pc.h if pc is not None else None,
                            _dptr(u, problem.N, "u"), float(dt), _dptr(src, problem.N, "src"),
                            ctypes.byref(n), ctypes.byref(o), ctypes.byref(s), _stream())
    k = s.newton_its
    stats = dict(newton_its=k, gmres_its=list(s.gmres_its[:k]), gmres_its_total=s.gmres_its_total,
                 res_hist=list(s.res_hist[:k + 1]), eps=s.eps, reason=s.reason, pc_setups=s.pc_setups,
                 t_residual_ms=s.t_residual_ms, t_jacobian_ms=s.t_jacobian_ms,
                 t_setup_ms=s.t_setup_ms, t_gmres_ms=s.t_gmres_ms,
                 t_ras_kernel_ms=s.t_ras_kernel_ms, n_ras_launches=s.n_ras_launches,
                 ras_bytes_per_launch=s.ras_bytes_per_launch, backtracks=s.backtracks,
                 inexact_solves=s.inexact_solves)
    _check(code)
    return stats


def forward_record(problem: Problem, pc, u, n_steps, dt, region, n_regions, ckpt_every=10,
                   tol=1e-10, max_it=20, pc_reuse=0, pc_keep_steps=0, **kw):
    """Run n_steps implicit steps in place on u, recording checkpoints for
    ``adjoint``; returns the counts [n_steps, n_regions] (CUDA float64).
    pc_keep_steps > 0 keeps a step's preconditioner setup for that many
    further steps within each checkpoint segment, and ``adjoint`` then keeps
    its transposed-solve setups the same way."""
    torch = _torch()
    region = np.ascontiguousarray(region, dtype=np.int32)
    if len(region) != problem.n:
        raise ValueError("region must have one entry per node")
    counts = torch.empty((int(n_steps), int(n_regions)), dtype=torch.float64, device=u.device)
    nopt = _Newton(float(tol), int(max_it), int(pc_reuse), 0, int(pc_keep_steps))
    kopt = _krylov(**kw)
    # a new record replaces the problem's previous one (the library keeps one)
    problem.record_generation = getattr(problem, "record_generation", 0) + 1
    _check(lib().seird_forward_record(problem.h, pc.h if pc is not None else None,
                                      _dptr(u, problem.N, "u"), int(n_steps), float(dt),
                                      int(ckpt_every), region.ctypes.data, int(n_regions),
                                      _dptr(counts, None, "counts"), ctypes.byref(nopt),
                                      ctypes.byref(kopt), _stream()))
    return counts


def adjoint(problem: Problem, pc, grad_counts, **kw):
    """Reverse sweep of the last forward_record.  grad_counts: dL/dcounts
    [n_steps, n_regions].  Returns (grad_g [n] CUDA, grad_nu [5] numpy,
    stats)."""
    torch = _torch()
    gc = grad_counts.contiguous().to(torch.float64)
    grad_g = torch.empty(problem.n, dtype=torch.float64, device=gc.device)
    grad_nu = np.zeros(5, dtype=np.float64)
    kopt = _krylov(**kw)
    st = _AStats()
    _check(lib().seird_adjoint(problem.h, pc.h if pc is not None else None, _dptr(gc, None, "grad_counts"),
                               _dptr(grad_g, problem.n, "grad_g"), grad_nu.ctypes.data,
                               ctypes.byref(kopt), ctypes.byref(st), _stream()))
    return grad_g, grad_nu, dict(gmres_its_total=st.gmres_its_total,
                                 recomputed_steps=st.recomputed_steps,
                                 setups=st.setups, t_reverse_ms=st.t_reverse_ms)


def _make_run_function():
    torch = _torch()

    class SEIRDRun(torch.autograd.Function):
        """counts = SEIRDRun.apply(g, nu, problem, pc, u0, n_steps, dt,
        region, n_regions, options) -- the infected counts of every region
        at every step of an implicit run, differentiable with respect to the
        transmission field g [n] and the diffusion coefficients nu [5]
        through the library's discrete adjoint (reverse sweep with
        checkpoints).  ``options`` is a dict with base_params (rates),
        ckpt_every, tol, pc_reuse, pc_keep_steps and the forward/adjoint
        Krylov settings."""

        @staticmethod
        def _record(problem, pc, g, nu, u0, n_steps, dt, region, n_regions, options):
            import copy
            base = copy.copy(options["base_params"])
            base.nu = tuple(float(x) for x in nu.tolist())
            problem.set_params(base)
            problem.set_beta_field(g)
            u = u0.clone()
            return forward_record(problem, pc, u, n_steps, dt, region, n_regions,
                                  ckpt_every=options.get("ckpt_every", 10),
                                  tol=options.get("tol", 1e-10), pc_reuse=options.get("pc_reuse", 0),
                                  pc_keep_steps=options.get("pc_keep_steps", 0),
                                  **options.get("krylov", {}))

        @staticmethod
        def forward(ctx, g, nu, problem, pc, u0, n_steps, dt, region, n_regions, options):
            # the inputs of this record are kept in ctx: the problem holds
            # one record and one parameter set, which a later forward replaces
            gd = g.detach().contiguous().to(torch.float64).clone()
            nud = nu.detach().to(torch.float64).cpu().clone()
            ud = u0.detach().clone()
            counts = SEIRDRun._record(problem, pc, gd, nud, ud, n_steps, dt, region, n_regions, options)
            ctx.problem, ctx.pc, ctx.options = problem, pc, options
            ctx.inputs = (gd, nud, ud, n_steps, dt, region, n_regions)
            ctx.generation = problem.record_generation
            ctx.nu_device = nu.device
            return counts

        @staticmethod
        def backward(ctx, grad_counts):
            problem, pc, options = ctx.problem, ctx.pc, ctx.options
            gd, nud, ud, n_steps, dt, region, n_regions = ctx.inputs
            if getattr(problem, "record_generation", None) != ctx.generation:
                # another forward replaced this run's record: record it again
                # from the saved inputs (same parameters, same states)
                SEIRDRun._record(problem, pc, gd, nud, ud, n_steps, dt, region, n_regions, options)
                ctx.generation = problem.record_generation
            else:
                import copy
                base = copy.copy(options["base_params"])
                base.nu = tuple(float(x) for x in nud.tolist())
                problem.set_params(base)
                problem.set_beta_field(gd)
            grad_g, grad_nu, _ = adjoint(problem, pc, grad_counts,
                                         **options.get("adjoint_krylov", {"rtol": 1e-10}))
            gnu = torch.as_tensor(grad_nu, dtype=torch.float64, device=ctx.nu_device)
            return grad_g, gnu, None, None, None, None, None, None, None, None

    return SEIRDRun


class _LazyRun:
    _cls = None

    def __getattr__(self, name):
        if _LazyRun._cls is None:
            _LazyRun._cls = _make_run_function()
        return getattr(_LazyRun._cls, name)


SEIRDRun = _LazyRun()


class _BorrowedPrecond:
    """A preconditioner owned by another handle (timing and info only)."""

    def __init__(self, h, owner):
        self.h = h
        self._owner = owner

    def info(self):
        return Precond.info(self)

    def enable_timing(self, on=True):
        Precond.enable_timing(self, on)

    def perf(self, reset=False):
        return Precond.perf(self, reset)

    def set_solve_threads(self, threads):
        Precond.set_solve_threads(self, threads)

    def setup_scalar(self, diag, off):
        """Scalar preconditioners: factor the subdomain matrices of the
        scalar matrix (diag [n], off [n_slots] on the node graph)."""
        prob = self._owner.problem
        _check(lib().seird_precond_setup_scalar(self.h, _dptr(diag, prob.n, "diag"),
                                                _dptr(off, prob.nslots, "off"), _stream()))

    def apply(self, r, transpose=False, out=None):
        out = _torch().empty_like(r) if out is None else out
        _check(lib().seird_precond_apply(self.h, _dptr(r, None, "r"), _dptr(out, r.numel(), "z"),
                                         int(bool(transpose)), _stream()))
        return out


class PicardGS:
    """The paper's decoupled Picard-Gauss-Seidel solver (Appendix A): one
    implicit step is a sequence of sweeps over the compartments, each a
    scalar system solved by GMRES with a one-level RAS of scalar subdomains
    (the partition and overlap given here)."""

    def __init__(self, problem: Problem, part, n_sub, overlap, tile=32, factor_prec=0):
        self.problem = problem
        part = np.ascontiguousarray(part, dtype=np.int32)
        if len(part) != problem.n:
            raise ValueError("partition length must equal the node count")
        o, keep = _schwarz_opts(n_sub, overlap, tile, factor_prec, None)
        h = ctypes.c_void_p()
        _check(lib().seird_pgs_create(problem.h, ctypes.byref(o), part.ctypes.data, ctypes.byref(h)))
        del keep
        self.h = h
        ph = ctypes.c_void_p()
        _check(lib().seird_pgs_precond(self.h, ctypes.byref(ph)))
        self.precond = _BorrowedPrecond(ph, self)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.seird_pgs_destroy(self.h)
            self.h = None

    def step(self, u, dt, tol=1e-10, max_sweeps=50, strict_linear=False, gmres_max_it=200, pc_lag=False, **kw):
        """One implicit step in place on u (float64 CUDA [n, 5]); sweeps
        until epsilon (Eq. picardtol) <= tol.  pc_lag: set each diffusing
        compartment's preconditioner up at the first sweep only.  Returns
        the statistics."""
        po = _PgsOpts(float(tol), int(max_sweeps), int(bool(strict_linear)), int(bool(pc_lag)))
        o = _krylov(max_it=gmres_max_it, **kw)
        s = _PgsStats()
        code = lib().seird_pgs_step(self.h, _dptr(u, self.problem.N, "u"), float(dt), ctypes.byref(po),
                                    ctypes.byref(o), ctypes.byref(s), _stream())
        k = s.sweeps
        stats = dict(sweeps=k, gmres_its=list(s.gmres_its), eps_hist=list(s.eps_hist[:k]),
                     res_scaled=s.res_scaled, pc_setups=s.pc_setups, inexact_solves=s.inexact_solves,
                     reason=s.reason, t_setup_ms=s.t_setup_ms, t_gmres_ms=s.t_gmres_ms,
                     t_total_ms=s.t_total_ms)
        _check(code)
        return stats


def _params22(p) -> _Params22:
    c = _Params22()
    for f in _P22_FIELDS:
        setattr(c, f, float(getattr(p, f)))
    if len(p.nu) != 10:
        raise ValueError("nu holds the 10 diffusion coefficients of S V E A F B C P R1 R2")
    for k in range(10):
        c.nu[k] = float(p.nu[k])
    return c


class Model22:
    """The 22-compartment model of Appendix C on a mesh (state: float64 CUDA
    [n, 22], compartments S V E Q A W F B C X Y Z G N H H1 I H2 R1 R2 P D),
    stepped by compartment-wise Picard-Gauss-Seidel sweeps with one-level
    scalar RAS + GMRES for the ten diffusing compartments.  ``p`` has the
    fields of the parameter table (see seird22_params)."""

    def __init__(self, mesh: Mesh, p, part, n_sub, overlap, tile=32):
        self.mesh = mesh
        self.n = mesh.n
        part = np.ascontiguousarray(part, dtype=np.int32)
        if len(part) != mesh.n:
            raise ValueError("partition length must equal the node count")
        o, keep = _schwarz_opts(n_sub, overlap, tile, 0, None)
        c = _params22(p)
        h = ctypes.c_void_p()
        _check(lib().seird22_create(mesh.h, ctypes.byref(c), ctypes.byref(o), part.ctypes.data, ctypes.byref(h)))
        del keep
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.seird22_destroy(self.h)
            self.h = None

    def set_params(self, p):
        c = _params22(p)
        _check(lib().seird22_set_params(self.h, ctypes.byref(c)))

    def residual(self, u, u_prev, dt, out=None):
        out = _torch().empty_like(u) if out is None else out
        N = NC22 * self.n
        _check(lib().seird22_residual(self.h, _dptr(u, N, "u"), _dptr(u_prev, N, "u_prev"), float(dt),
                                      _dptr(out, N, "F"), _stream()))
        return out

    def step(self, u, dt, tol=1e-10, max_sweeps=64, strict_linear=False, gmres_max_it=200, **kw):
        """One implicit step in place on u; sweeps until epsilon <= tol.
        Returns the statistics."""
        po = _PgsOpts(float(tol), int(max_sweeps), int(bool(strict_linear)))
        o = _krylov(max_it=gmres_max_it, **kw)
        s = _Stats22()
        code = lib().seird22_step(self.h, _dptr(u, NC22 * self.n, "u"), float(dt), ctypes.byref(po),
                                  ctypes.byref(o), ctypes.byref(s), _stream())
        k = s.sweeps
        stats = dict(sweeps=k, gmres_its=list(s.gmres_its), eps_hist=list(s.eps_hist[:k]),
                     res_scaled=s.res_scaled, pc_setups=s.pc_setups, inexact_solves=s.inexact_solves,
                     reason=s.reason, t_setup_ms=s.t_setup_ms, t_gmres_ms=s.t_gmres_ms,
                     t_total_ms=s.t_total_ms)
        _check(code)
        return stats


class Batch:
    """Independent problems stepped together (one-level RAS).  instances: a
    list of (xy, tri, params, part, n_sub).  The batch state is the
    concatenation of the instances' [n_k, 5] states."""

    def __init__(self, instances, overlap=2, tile=32, factor_prec=0):
        K = len(instances)
        keep = []
        nn = np.array([len(x[0]) for x in instances], dtype=np.int64)
        nt = np.array([len(x[1]) for x in instances], dtype=np.int64)
        xys = [np.ascontiguousarray(x[0], dtype=np.float64) for x in instances]
        tris = [np.ascontiguousarray(x[1], dtype=np.int32) for x in instances]
        parts = [np.ascontiguousarray(x[3], dtype=np.int32) for x in instances]
        keep += xys + tris + parts
        P = (_Params * K)(*[_params(x[2]) for x in instances])
        xyp = (ctypes.c_void_p * K)(*[a.ctypes.data for a in xys])
        trp = (ctypes.c_void_p * K)(*[a.ctypes.data for a in tris])
        pap = (ctypes.c_void_p * K)(*[a.ctypes.data for a in parts])
        nsub = np.array([x[4] for x in instances], dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().seird_batch_create(K, nn.ctypes.data, ctypes.cast(xyp, ctypes.c_void_p),
                                        nt.ctypes.data, ctypes.cast(trp, ctypes.c_void_p),
                                        ctypes.cast(P, ctypes.c_void_p), ctypes.cast(pap, ctypes.c_void_p),
                                        nsub.ctypes.data, int(overlap), int(tile), int(factor_prec),
                                        ctypes.byref(h)))
        del keep
        self.h = h
        self.K = K
        off = np.zeros(K + 1, dtype=np.int64)
        _check(lib().seird_batch_info(self.h, off.ctypes.data))
        self.node_offsets = off
        self.n = int(off[-1])
        ph = ctypes.c_void_p()
        _check(lib().seird_batch_precond(self.h, ctypes.byref(ph)))
        self.precond = _BorrowedPrecond(ph, self)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.seird_batch_destroy(self.h)
            self.h = None

    def autotune(self, reps=3):
        """Choose the subdomain-solve width on the ensemble itself (after a
        step, so that the factors exist); see seird_batch_autotune."""
        rep = _TuneReport()
        _check(lib().seird_batch_autotune(self.h, int(reps), ctypes.byref(rep), _stream()))
        return _tune_dict(rep)

    def step(self, u, dt, tol=1e-10, max_it=20, pc_reuse=0, **kw):
        """One implicit step of every instance, in place on u [n_total, 5].
        Returns a list of per-instance statistics."""
        n = _Newton(float(tol), int(max_it), int(pc_reuse), 0)
        o = _krylov(**kw)
        st = (_SStats * self.K)()
        code = lib().seird_batch_step(self.h, _dptr(u, 5 * self.n, "u"), float(dt), ctypes.byref(n),
                                      ctypes.byref(o), ctypes.cast(st, ctypes.c_void_p), _stream())
        _check(code)
        out = []
        for s in st:
            k = s.newton_its
            out.append(dict(newton_its=k, gmres_its=list(s.gmres_its[:k]),
                            res_hist=list(s.res_hist[:k + 1]), eps=s.eps, pc_setups=s.pc_setups,
                            t_residual_ms=s.t_residual_ms, t_jacobian_ms=s.t_jacobian_ms,
                            t_setup_ms=s.t_setup_ms, t_gmres_ms=s.t_gmres_ms,
                            t_ras_kernel_ms=s.t_ras_kernel_ms, n_ras_launches=s.n_ras_launches,
                            ras_bytes_per_launch=s.ras_bytes_per_launch, backtracks=s.backtracks,
                            inexact_solves=s.inexact_solves))
        return out
