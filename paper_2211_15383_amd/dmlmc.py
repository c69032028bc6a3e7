"""ctypes binding of libdmlmc.so (include/dmlmc.h).  Argument marshalling only.

Device vectors are torch tensors on the GPU (complex128 for FP64, complex64 for the
complex-FP32 operators); the library enqueues on torch's current HIP stream.  Every
wrapper raises DmlmcError on a non-zero status.  There is no fallback: if the shared
library is missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdmlmc.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ENUMERIC, ESTATE = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
DIRECT_OFF, DIRECT_FP32, DIRECT_FP16, DIRECT_FP8 = 0, 1, 2, 3
OP_D, OP_RESTRICT, OP_PROLONG, OP_SMOOTH, OP_VCYCLE, OP_DEFL_C, OP_DEFL_P, OP_GAMMA5_D = 0, 1, 2, 3, 4, 6, 7, 8
# launch-variant autotuner kernel ids (dmlmc_tune_kernels)
(KV_WILSON_RB, KV_COARSE_SPLIT, KV_SAP_RB, KV_GS_SPLIT, KV_RESTRICT_UT, KV_PROLONG_MT, KV_PROLONG_STAGED,
 KV_RESTRICT_STAGED) = range(8)
KV_COUNT = 8
KV_NAMES = ("wilson_rb", "coarse_split", "sap_rb", "gs_split", "restrict_ut", "prolong_mt", "prolong_staged",
            "restrict_staged")

EXPORTED = [
    "dmlmc_create", "dmlmc_destroy", "dmlmc_last_error", "dmlmc_version", "dmlmc_build_hierarchy",
    "dmlmc_free_hierarchy", "dmlmc_level_info", "dmlmc_work_stride", "dmlmc_apply_strided", "dmlmc_export_level", "dmlmc_deflate", "dmlmc_deflate_difference",
    "dmlmc_free_deflation", "dmlmc_deflation_info", "dmlmc_export_deflation", "dmlmc_solve_multi_rhs", "dmlmc_mlmc_trace",
    "dmlmc_hutchinson_trace",
    "dmlmc_apply", "dmlmc_set_deflation", "dmlmc_z2_noise", "dmlmc_set_solver_params",
    "dmlmc_get_solver_params", "dmlmc_timing_enable", "dmlmc_timing_select", "dmlmc_tune_rhs_block",
    "dmlmc_coarsest_direct", "dmlmc_deflate_project_noalloc",
    "dmlmc_timing_reset", "dmlmc_timing_get", "dmlmc_tune_kernels", "dmlmc_set_kernel_variant",
    "dmlmc_get_kernel_variant", "dmlmc_set_verbose",
]


class DmlmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dmlmc status {status}: {msg}")
        self.status = status


class Lattice(C.Structure):
    _fields_ = [("Lx", C.c_int), ("Lt", C.c_int), ("m0", C.c_double), ("antiperiodic_t", C.c_int),
                ("theta", C.POINTER(C.c_double))]


class MGParams(C.Structure):
    _fields_ = [("nlevels", C.c_int), ("agg", (C.c_int * 2) * 7), ("ntv", C.c_int * 7), ("n_inv", C.c_int),
                ("seed", C.c_uint64), ("import_tv", C.POINTER(C.c_void_p))]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("ir_steps", C.c_int), ("converged", C.c_int), ("relres_max", C.c_double)]


class SolverParams(C.Structure):
    _fields_ = [("sap_mr_iters", C.c_int), ("nu_pre", C.c_int), ("nu_post", C.c_int), ("coarsest_iters", C.c_int),
                ("coarsest_iters_defl", C.c_int), ("restart", C.c_int), ("use_graphs", C.c_int),
                ("nu_post_coarse", C.c_int), ("inner_rtol", C.c_double), ("smoother_half", C.c_int)]


class MLMCParams(C.Structure):
    _fields_ = [("eps", C.c_double), ("noise_seed", C.c_uint64), ("n0", C.c_int * 8),
                ("max_samples", C.c_int64 * 8), ("rhs_block", C.c_int), ("prec", C.c_int), ("rtol", C.c_double),
                ("fixed_counts", C.c_int), ("maxiter", C.c_int), ("samples_out", C.POINTER(C.c_double) * 8),
                ("skip", C.c_int * 8), ("term_defl", C.c_void_p * 8)]


class TraceResult(C.Structure):
    _fields_ = [("trace", C.c_double), ("trace_imag", C.c_double), ("rel_err", C.c_double),
                ("N", C.c_int64 * 8), ("mean_re", C.c_double * 8), ("mean_im", C.c_double * 8),
                ("var", C.c_double * 8), ("cost_s", C.c_double * 8), ("tr_defl", C.c_double),
                ("t_trace_s", C.c_double), ("iters", C.c_int64 * 8)]


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2211_15383_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "dmlmc_create": (i32, [C.POINTER(vp), i32, vp]),
        "dmlmc_destroy": (None, [vp]),
        "dmlmc_last_error": (C.c_char_p, [vp]),
        "dmlmc_version": (C.c_char_p, []),
        "dmlmc_build_hierarchy": (i32, [vp, C.POINTER(Lattice), C.POINTER(MGParams), C.POINTER(vp)]),
        "dmlmc_free_hierarchy": (None, [vp]),
        "dmlmc_level_info": (i32, [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "dmlmc_export_level": (i32, [vp, vp, i32, vp, vp, vp]),
        "dmlmc_deflate": (i32, [vp, vp, i32, i32, dbl, vp, C.POINTER(dbl), C.POINTER(vp), C.POINTER(dbl)]),
        "dmlmc_deflate_difference": (i32, [vp, vp, i32, i32, i32, dbl, dbl, i32, vp, C.POINTER(dbl), dbl,
                                           C.POINTER(vp), C.POINTER(dbl)]),
        "dmlmc_free_deflation": (None, [vp]),
        "dmlmc_deflation_info": (i32, [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(dbl)]),
        "dmlmc_export_deflation": (i32, [vp, vp, vp, C.POINTER(dbl)]),
        "dmlmc_solve_multi_rhs": (i32, [vp, vp, i32, vp, vp, vp, i32, i64, i32, dbl, i32, C.POINTER(SolveStats)]),
        "dmlmc_mlmc_trace": (i32, [vp, vp, vp, C.POINTER(MLMCParams), C.POINTER(TraceResult)]),
        "dmlmc_hutchinson_trace": (i32, [vp, vp, vp, vp, C.POINTER(MLMCParams), C.POINTER(TraceResult)]),
        "dmlmc_apply": (i32, [vp, vp, i32, i32, vp, vp, i32, i32, u64]),
        "dmlmc_apply_strided": (i32, [vp, vp, i32, i32, vp, i64, vp, i64, i32, i32, u64]),
        "dmlmc_work_stride": (i32, [vp, i32, C.POINTER(i64)]),
        "dmlmc_set_deflation": (i32, [vp, vp]),
        "dmlmc_z2_noise": (i32, [vp, i64, u64, i32, i64, i32, vp, i32]),
        "dmlmc_set_solver_params": (i32, [vp, C.POINTER(SolverParams)]),
        "dmlmc_get_solver_params": (i32, [vp, C.POINTER(SolverParams)]),
        "dmlmc_timing_enable": (i32, [vp, i32]),
        "dmlmc_timing_reset": (i32, [vp]),
        "dmlmc_timing_select": (i32, [vp, C.c_char_p]),
        "dmlmc_coarsest_direct": (i32, [vp, vp, vp, i32]),
        "dmlmc_deflate_project_noalloc": (i32, [vp, vp, vp, vp, i32]),
        "dmlmc_tune_rhs_block": (i32, [vp, vp, vp, C.POINTER(i32), i32, i32, dbl, C.c_uint64, C.POINTER(i32),
                                       C.POINTER(dbl)]),
        "dmlmc_timing_get": (i32, [vp, C.c_char_p, C.POINTER(i64), C.POINTER(dbl), C.POINTER(dbl)]),
        "dmlmc_tune_kernels": (i32, [vp, vp, i32, i32, C.c_char_p, C.POINTER(i32), C.POINTER(dbl), C.POINTER(dbl)]),
        "dmlmc_set_kernel_variant": (i32, [vp, i32, i32, i32]),
        "dmlmc_set_verbose": (i32, [vp, i32]),
        "dmlmc_get_kernel_variant": (i32, [vp, i32, i32, C.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def _ptr(t) -> int:
    """Device address of a tensor handed to the library.  The library enqueues on its own
    stream when torch runs on the default one, so torch's pending work on t's device (which
    may still be writing t) is waited for before the address is passed on."""
    if t.is_cuda:
        import torch

        torch.cuda.current_stream(t.device).synchronize()
    return t.data_ptr()


# Library objects still alive at interpreter exit are released child-first (deflations,
# hierarchies, then contexts) before the HIP runtime shuts down.
_LIVE = {"defl": weakref.WeakSet(), "hier": weakref.WeakSet(), "ctx": weakref.WeakSet()}


@atexit.register
def _release_all():
    for kind in ("defl", "hier", "ctx"):
        for obj in list(_LIVE[kind]):
            try:
                obj.close()
            except Exception:
                pass


class Context:
    """A library context bound to a GPU and a HIP stream (torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        handle = C.c_void_p()
        st = lib().dmlmc_create(C.byref(handle), device, C.c_void_p(stream.cuda_stream))
        if st != OK:
            raise DmlmcError(st, lib().dmlmc_last_error(None).decode())
        self.h = handle
        self.device = device
        self.stream = stream
        _LIVE["ctx"].add(self)

    def check(self, st: int):
        if st != OK:
            raise DmlmcError(st, lib().dmlmc_last_error(self.h).decode())

    def close(self):
        if self.h:
            lib().dmlmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- timing
    def verbose(self, level: int = 1):
        """Progress lines of long phases (eigensolver iterations) on stderr (see dmlmc_set_verbose)."""
        self.check(lib().dmlmc_set_verbose(self.h, level))

    def timing(self, enable: bool):
        self.check(lib().dmlmc_timing_enable(self.h, 1 if enable else 0))

    def timing_select(self, classes=None):
        """Restricts timing to the given class names (iterable of str); None = all."""
        arg = None if not classes else ",".join(classes).encode()
        self.check(lib().dmlmc_timing_select(self.h, arg))

    def timing_reset(self):
        self.check(lib().dmlmc_timing_reset(self.h))

    def timing_get(self, cls: str):
        n, ms, b = C.c_int64(), C.c_double(), C.c_double()
        self.check(lib().dmlmc_timing_get(self.h, cls.encode(), C.byref(n), C.byref(ms), C.byref(b)))
        return n.value, ms.value, b.value

    # ---------------------------------------------------------------- noise
    def z2_noise(self, n: int, seed: int, level: int, sample0: int, nrhs: int, prec: int = FP64):
        dt = self.torch.complex128 if prec == FP64 else self.torch.complex64
        out = self.torch.empty((nrhs, n), dtype=dt, device=f"cuda:{self.device}")
        self.check(lib().dmlmc_z2_noise(self.h, n, seed, level, sample0, nrhs, C.c_void_p(_ptr(out)), prec))
        return out


class Hierarchy:
    """Multigrid hierarchy of one gauge field (built on the device)."""

    def __init__(self, ctx: Context, theta: np.ndarray, m0: float, aggs: Sequence[Sequence[int]],
                 ntv: Sequence[int], n_inv: int = 3, seed: int = 7, antiperiodic: bool = True,
                 import_tv: Optional[List[np.ndarray]] = None):
        self.ctx = ctx
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        _, Lt, Lx = theta.shape
        lat = Lattice(Lx, Lt, float(m0), 1 if antiperiodic else 0, theta.ctypes.data_as(C.POINTER(C.c_double)))
        mgp = MGParams()
        mgp.nlevels = len(aggs) + 1
        for i, (a, n) in enumerate(zip(aggs, ntv)):
            mgp.agg[i][0], mgp.agg[i][1] = int(a[0]), int(a[1])
            mgp.ntv[i] = int(n)
        mgp.n_inv = n_inv
        mgp.seed = seed
        keep = []
        if import_tv is not None:
            arr = (C.c_void_p * len(import_tv))()
            for i, V in enumerate(import_tv):
                Vc = np.ascontiguousarray(np.asarray(V, dtype=np.complex128).T)  # [ntv][n]
                keep.append(Vc)
                arr[i] = Vc.ctypes.data
            mgp.import_tv = C.cast(arr, C.POINTER(C.c_void_p))
            keep.append(arr)
        handle = C.c_void_p()
        ctx.check(lib().dmlmc_build_hierarchy(ctx.h, C.byref(lat), C.byref(mgp), C.byref(handle)))
        self.h = handle
        self.nlevels = mgp.nlevels
        self.theta = theta
        _LIVE["hier"].add(self)

    def close(self):
        if self.h:
            lib().dmlmc_free_hierarchy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level: int):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        st = lib().dmlmc_level_info(self.h, level, C.byref(a), C.byref(b), C.byref(c))
        if st != OK:
            raise DmlmcError(st, "level_info")
        return a.value, b.value, c.value

    def n(self, level: int) -> int:
        Lx, Lt, d = self.level_info(level)
        return Lx * Lt * d

    def export(self, level: int, P: bool = False, Dc: bool = False, tv: bool = False):
        out = {}
        pP = pD = pT = None
        if P:
            out["P"] = np.zeros((self.n(level), self.n(level + 1)), dtype=np.complex128)
            pP = out["P"].ctypes.data
        if Dc:
            Lx, Lt, d = self.level_info(level)
            out["Dc"] = np.zeros((Lx * Lt, 5, d, d), dtype=np.complex128)
            pD = out["Dc"].ctypes.data
        if tv:
            ntv = self._ntv(level)
            out["tv"] = np.zeros((ntv, self.n(level)), dtype=np.complex128)
            pT = out["tv"].ctypes.data
        self.ctx.check(lib().dmlmc_export_level(self.ctx.h, self.h, level, pP, pD, pT))
        return out

    def _ntv(self, level: int) -> int:
        _, _, dc = self.level_info(level + 1)
        return dc // 2

    # ---------------------------------------------------------------- operators
    def apply(self, op: int, level: int, x, out, prec: int = FP64, arg: int = 0, ld_in: int = 0, ld_out: int = 0):
        """ld_in / ld_out: strides between the RHS of x / out in complex entries (0: the
        vector's level size); with both 0 this is dmlmc_apply, else dmlmc_apply_strided."""
        nrhs = x.shape[0] if op != OP_PROLONG else out.shape[0]
        if ld_in == 0 and ld_out == 0:
            self.ctx.check(lib().dmlmc_apply(self.ctx.h, self.h, op, level, C.c_void_p(_ptr(x)),
                                             C.c_void_p(_ptr(out)), nrhs, prec, arg))
        else:
            self.ctx.check(lib().dmlmc_apply_strided(self.ctx.h, self.h, op, level, C.c_void_p(_ptr(x)), ld_in,
                                                     C.c_void_p(_ptr(out)), ld_out, nrhs, prec, arg))
        return out

    def work_stride(self, level: int) -> int:
        """Stride between RHS of the solver's internal work vectors on `level`."""
        ld = C.c_int64()
        st = lib().dmlmc_work_stride(self.h, level, C.byref(ld))
        if st != OK:
            raise DmlmcError(st, "dmlmc_work_stride failed")
        return ld.value

    def solve(self, level: int, B, prec: int = FP64, rtol: float = 1e-10, maxiter: int = 2000, proj=None):
        torch = self.ctx.torch
        X = torch.empty_like(B)
        stats = SolveStats()
        st = lib().dmlmc_solve_multi_rhs(self.ctx.h, self.h, level, proj.h if proj is not None else None,
                                         C.c_void_p(_ptr(B)), C.c_void_p(_ptr(X)), B.shape[0], B.shape[1], prec,
                                         rtol, maxiter, C.byref(stats))
        if st not in (OK,):
            raise DmlmcError(st, lib().dmlmc_last_error(self.ctx.h).decode())
        return X, stats

    def solver_params(self, **kw):
        """Sets the given solver parameters (see dmlmc_solver_params); returns all of them."""
        p = SolverParams(*([-1] * len(SolverParams._fields_)))
        for key, v in kw.items():
            setattr(p, key, float(v) if key == "inner_rtol" else int(v))
        st = lib().dmlmc_set_solver_params(self.h, C.byref(p))
        if st != OK:
            raise DmlmcError(st, f"invalid solver parameters {kw}")
        q = SolverParams()
        lib().dmlmc_get_solver_params(self.h, C.byref(q))
        return {f: getattr(q, f) for f, _ in SolverParams._fields_}

    def tune_rhs_block(self, defl: Optional["Deflation"], candidates=(16, 32, 64), prec: int = FP64,
                       rtol: float = 1e-10, noise_seed: int = 0):
        """Times one block of samples per level for each candidate block size (see
        dmlmc_tune_rhs_block); returns (best, {candidate: seconds per sample})."""
        cand = (C.c_int32 * len(candidates))(*candidates)
        secs = (C.c_double * len(candidates))()
        best = C.c_int32()
        self.ctx.check(lib().dmlmc_tune_rhs_block(self.ctx.h, self.h, defl.h if defl is not None else None, cand,
                                                  len(candidates), prec, rtol, noise_seed, C.byref(best), secs))
        return best.value, {c: secs[i] for i, c in enumerate(candidates)}

    def tune_kernels(self, nrhs: int, reps: int = 10, cache_path: Optional[str] = None):
        """Launch-variant autotuner (see dmlmc_tune_kernels); returns {(level, kernel name):
        (choice, us of the choice, us of the built-in rule)} for the kernels run on each level."""
        L = self.nlevels
        picks = (C.c_int32 * (L * KV_COUNT))()
        best = (C.c_double * (L * KV_COUNT))()
        dflt = (C.c_double * (L * KV_COUNT))()
        path = cache_path.encode() if cache_path else None
        self.ctx.check(lib().dmlmc_tune_kernels(self.ctx.h, self.h, nrhs, reps, path, picks, best, dflt))
        out = {}
        for l in range(L):
            for k, name in enumerate(KV_NAMES):
                i = l * KV_COUNT + k
                if picks[i] >= 0:
                    out[(l + 1, name)] = (picks[i], best[i], dflt[i])
        return out

    def set_kernel_variant(self, level: int, kernel: int, value: int):
        st = lib().dmlmc_set_kernel_variant(self.h, level, kernel, value)
        if st != OK:
            raise DmlmcError(st, f"set_kernel_variant({level}, {kernel}, {value})")

    def kernel_variant(self, level: int, kernel: int) -> int:
        v = C.c_int32()
        st = lib().dmlmc_get_kernel_variant(self.h, level, kernel, C.byref(v))
        if st != OK:
            raise DmlmcError(st, f"kernel_variant({level}, {kernel})")
        return v.value

    def coarsest_direct(self, defl: Optional["Deflation"] = None, enable=True):
        """Explicit-inverse coarsest solve (computed on first use): enable True or
        DIRECT_FP32, DIRECT_FP16, DIRECT_FP8, or False / DIRECT_OFF (see dmlmc_coarsest_direct)."""
        mode = DIRECT_FP32 if enable is True else (DIRECT_OFF if enable is False else int(enable))
        self.ctx.check(lib().dmlmc_coarsest_direct(self.ctx.h, self.h, defl.h if defl is not None else None, mode))

    def set_deflation(self, d: Optional["Deflation"]):
        st = lib().dmlmc_set_deflation(self.h, d.h if d is not None else None)
        if st != OK:
            raise DmlmcError(st, "set_deflation")


class Deflation:
    """Exact deflation of the coarsest term (dmlmc_deflate) or, with `level_b`, of the
    difference term (level, level_b) (dmlmc_deflate_difference)."""

    def __init__(self, hier: Hierarchy, level: int, k: int, eig_rtol: float = 1e-12,
                 import_X: Optional[np.ndarray] = None, import_lambda: Optional[np.ndarray] = None,
                 level_b: int = 0, solve_rtol: float = 1e-12, prec: int = MIXED, corr_rtol: float = 0.0):
        self.hier = hier
        ctx = hier.ctx
        handle = C.c_void_p()
        tr = C.c_double()
        pX = plam = None
        keep = []
        if import_X is not None:
            Xc = np.ascontiguousarray(np.asarray(import_X, dtype=np.complex128).T)  # [k][n]
            lam = np.ascontiguousarray(import_lambda, dtype=np.float64)
            keep += [Xc, lam]
            pX = Xc.ctypes.data
            plam = lam.ctypes.data_as(C.POINTER(C.c_double))
        if level_b:
            st = lib().dmlmc_deflate_difference(ctx.h, hier.h, level, level_b, k, eig_rtol, solve_rtol, prec, pX, plam,
                                                corr_rtol, C.byref(handle), C.byref(tr))
        else:
            st = lib().dmlmc_deflate(ctx.h, hier.h, level, k, eig_rtol, pX, plam, C.byref(handle), C.byref(tr))
        self.level_b = level_b
        self.status = st
        if st not in (OK, ENOCONV):
            raise DmlmcError(st, lib().dmlmc_last_error(ctx.h).decode())
        self.h = handle
        self.tr_defl = tr.value
        self.k = k
        self.level = level
        _LIVE["defl"].add(self)

    def info(self):
        it, deg, res = C.c_int(), C.c_int64(), C.c_double()
        st = lib().dmlmc_deflation_info(self.h, C.byref(it), C.byref(deg), C.byref(res))
        if st != OK:
            raise DmlmcError(st, "deflation_info")
        return {"iters": it.value, "degree_sum": deg.value, "max_residual": res.value}

    def project_noalloc(self, x, out):
        """out = x - W (W^H x) through dmlmc_deflate_project_noalloc (complex128 [nrhs][n]
        tensors on the device; the library allocates nothing for it)."""
        self.hier.ctx.check(lib().dmlmc_deflate_project_noalloc(self.hier.ctx.h, self.h, C.c_void_p(_ptr(x)),
                                                                C.c_void_p(_ptr(out)), x.shape[0]))
        return out

    def export(self):
        n = self.hier.n(self.level)
        X = np.zeros((self.k, n), dtype=np.complex128)
        lam = np.zeros(self.k, dtype=np.float64)
        self.hier.ctx.check(lib().dmlmc_export_deflation(self.hier.ctx.h, self.h, X.ctypes.data,
                                                         lam.ctypes.data_as(C.POINTER(C.c_double))))
        return X, lam

    def close(self):
        if self.h:
            lib().dmlmc_free_deflation(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class TraceEstimate:
    trace: float
    trace_imag: float
    rel_err: float
    N: List[int]
    mean: List[complex]
    var: List[float]
    cost_s: List[float]
    iters: List[int]
    tr_defl: float
    seconds: float
    samples: Optional[List[np.ndarray]] = None


def mlmc_trace(hier: Hierarchy, defl: Optional[Deflation], eps: float, noise_seed: int, n0: Sequence[int],
               rhs_block: int, prec: int = FP64, rtol: float = 1e-10, fixed_counts: bool = False,
               max_samples: Optional[Sequence[int]] = None, keep_samples: bool = False,
               maxiter: int = 2000, skip: Sequence[int] = (),
               term_defl: Optional[Sequence[Optional[Deflation]]] = None) -> TraceEstimate:
    """skip: hierarchy levels left out of the telescoping sum (eq. 12); term_defl[a-1]:
    deflation of the difference term starting at level a, or None."""
    L = hier.nlevels
    p = MLMCParams()
    p.eps = eps
    p.noise_seed = noise_seed
    for l in range(L):
        p.n0[l] = int(n0[l])
        p.max_samples[l] = int(max_samples[l]) if max_samples is not None else 0
    p.rhs_block = rhs_block
    p.prec = prec
    p.rtol = rtol
    p.fixed_counts = 1 if fixed_counts else 0
    p.maxiter = maxiter
    for l in skip:
        p.skip[l - 1] = 1
    if term_defl is not None:
        for l, d in enumerate(term_defl):
            p.term_defl[l] = d.h.value if d is not None else None
    bufs = []
    if keep_samples:
        if max_samples is None:
            raise ValueError("keep_samples needs max_samples")
        for l in range(L):
            b = np.zeros(2 * int(max_samples[l]), dtype=np.float64)
            bufs.append(b)
            p.samples_out[l] = b.ctypes.data_as(C.POINTER(C.c_double))
    r = TraceResult()
    hier.ctx.check(lib().dmlmc_mlmc_trace(hier.ctx.h, hier.h, defl.h if defl is not None else None,
                                          C.byref(p), C.byref(r)))
    out = TraceEstimate(r.trace, r.trace_imag, r.rel_err, [r.N[l] for l in range(L)],
                        [complex(r.mean_re[l], r.mean_im[l]) for l in range(L)], [r.var[l] for l in range(L)],
                        [r.cost_s[l] for l in range(L)], [r.iters[l] for l in range(L)], r.tr_defl, r.t_trace_s)
    if keep_samples:
        out.samples = [bufs[l][: 2 * r.N[l]].view(np.complex128) for l in range(L)]
    return out


def hutchinson_trace(hier: Hierarchy, fine: Optional[Deflation], eps: float, noise_seed: int, n0: int,
                     rhs_block: int, prec: int = FP64, rtol: float = 1e-10, fixed_counts: bool = False,
                     max_samples: int = 0, keep_samples: bool = False, maxiter: int = 2000,
                     coarsest: Optional[Deflation] = None) -> TraceEstimate:
    """Deflated plain Hutchinson at the fine level (see dmlmc_hutchinson_trace); fine: a
    Deflation of level 1 or None; the result lists have one entry."""
    p = MLMCParams()
    p.eps = eps
    p.noise_seed = noise_seed
    p.n0[0] = int(n0)
    p.max_samples[0] = int(max_samples)
    p.rhs_block = rhs_block
    p.prec = prec
    p.rtol = rtol
    p.fixed_counts = 1 if fixed_counts else 0
    p.maxiter = maxiter
    buf = None
    if keep_samples:
        if max_samples <= 0:
            raise ValueError("keep_samples needs max_samples")
        buf = np.zeros(2 * int(max_samples), dtype=np.float64)
        p.samples_out[0] = buf.ctypes.data_as(C.POINTER(C.c_double))
    r = TraceResult()
    hier.ctx.check(lib().dmlmc_hutchinson_trace(hier.ctx.h, hier.h, fine.h if fine is not None else None,
                                                coarsest.h if coarsest is not None else None, C.byref(p),
                                                C.byref(r)))
    out = TraceEstimate(r.trace, r.trace_imag, r.rel_err, [r.N[0]], [complex(r.mean_re[0], r.mean_im[0])],
                        [r.var[0]], [r.cost_s[0]], [r.iters[0]], r.tr_defl, r.t_trace_s)
    if keep_samples:
        out.samples = [buf[: 2 * r.N[0]].view(np.complex128)]
    return out
