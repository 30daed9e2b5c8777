"""Thin ctypes binding of libshg.so (C ABI in include/shg.h).

Argument marshalling only: torch supplies device memory and the stream, every
step of the integral path runs in the library's HIP kernels. There is no CPU
fallback: if the library or a GPU is missing, construction raises.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshg.so")

OPS = {"overlap": 0, "coulomb": 1, "erf": 2, "erfc": 3, "gauss": 4, "gcoulomb": 5}
ERRORS = {-1: "SHG_EINVAL", -2: "SHG_ENOMEM", -3: "SHG_EDEVICE"}
EXPORTS = ("shg_create", "shg_destroy", "shg_last_error", "shg_pairs", "shg_pairs_deriv", "shg_aab",
           "shg_set_tile_shape", "shg_get_tile_shape", "shg_autotune", "shg_tuning_save", "shg_tuning_load",
           "shg_profile_enable", "shg_profile_read", "shg_plan_create", "shg_plan_execute",
           "shg_plan_autotune", "shg_plan_set_mode", "shg_plan_mode", "shg_plan_destroy",
           "shg_plan_stats", "shg_plan_kernel_ms", "shg_plan_skipped", "shg_plan_tile_order", "shg_pairs_noalloc", "shg_set_aab_chunk", "shg_plan_time_kernels", "shg_plan_kernel_time", "shg_plan_set_tile_order", "shg_set_pairs",
           "shg_plan_create_screened", "shg_mlp_create", "shg_mlp_destroy", "shg_mlp_params", "shg_mlp_set_norm",
           "shg_mlp_set_margin", "shg_mlp_set_scope", "shg_mlp_train_step", "shg_mlp_grad", "shg_mlp_predict", "shg_mlp_save",
           "shg_mlp_load", "shg_screen_features", "shg_block_logmax")


class ShgShells(C.Structure):
    _fields_ = [("nshell", C.c_int32), ("nprim_total", C.c_int64), ("center", C.c_void_p),
                ("l", C.c_void_p), ("nprim", C.c_void_p), ("prim_off", C.c_void_p),
                ("exps", C.c_void_p), ("coefs", C.c_void_p)]


class ShgSets(C.Structure):
    _fields_ = [("nset", C.c_int32), ("nexp_total", C.c_int64), ("nfun_total", C.c_int64),
                ("ncoef_total", C.c_int64), ("center", C.c_void_p), ("nexp", C.c_void_p), ("exp_off", C.c_void_p),
                ("exps", C.c_void_p), ("nfun", C.c_void_p), ("fun_off", C.c_void_p), ("fun_l", C.c_void_p),
                ("coef_off", C.c_void_p), ("coefs", C.c_void_p)]


class ShgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libshg.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1701_06588_amd/build.py")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.shg_create.argtypes = [C.POINTER(C.c_void_p), P]
    lib.shg_create.restype = C.c_int
    lib.shg_destroy.argtypes = [P]
    lib.shg_destroy.restype = None
    lib.shg_last_error.argtypes = [P]
    lib.shg_last_error.restype = C.c_char_p
    lib.shg_pairs.argtypes = [P, C.POINTER(ShgShells), C.c_int, C.c_double, P, C.c_int64, P, P]
    lib.shg_pairs.restype = C.c_int
    lib.shg_pairs_deriv.argtypes = [P, C.POINTER(ShgShells), C.c_int, C.c_double, P, C.c_int64, P, P, P]
    lib.shg_pairs_deriv.restype = C.c_int
    lib.shg_aab.argtypes = [P, C.POINTER(ShgShells), C.POINTER(ShgShells), P, C.c_int64, P, P, P]
    lib.shg_aab.restype = C.c_int
    lib.shg_pairs_noalloc.argtypes = [P, C.POINTER(ShgShells), C.c_int, C.c_double, P, C.c_int64, P, P, P]
    lib.shg_pairs_noalloc.restype = C.c_int
    lib.shg_set_pairs.argtypes = [P, C.POINTER(ShgSets), C.c_int, C.c_double, P, C.c_int64, P, P, P]
    lib.shg_set_pairs.restype = C.c_int
    lib.shg_set_aab_chunk.argtypes = [P, C.c_int64]
    lib.shg_set_aab_chunk.restype = C.c_int
    lib.shg_pairs_r2n.argtypes = [P, C.POINTER(ShgShells), C.c_int, P, C.c_int64, P, P, P]
    lib.shg_pairs_r2n.restype = C.c_int
    lib.shg_pairs_swap.argtypes = [P, C.POINTER(ShgShells), P, C.c_int64, P, P, P, P]
    lib.shg_pairs_swap.restype = C.c_int
    lib.shg_pairs_swap_check.argtypes = [P]
    lib.shg_pairs_swap_check.restype = C.c_int
    lib.shg_fp64_ceiling.argtypes = [P, C.c_int64, C.c_int, P, C.POINTER(C.c_double)]
    lib.shg_fp64_ceiling.restype = C.c_int
    I = C.c_int
    lib.shg_set_tile_shape.argtypes = [P, I, I, I, I, I, I]
    lib.shg_get_tile_shape.argtypes = [P, I, I, I, I, C.POINTER(I), C.POINTER(I)]
    lib.shg_autotune.argtypes = [P, C.POINTER(ShgShells), I, C.c_double, P, C.c_int64, P, P, P, I]
    lib.shg_tuning_save.argtypes = [P, C.c_char_p]
    lib.shg_tuning_load.argtypes = [P, C.c_char_p]
    lib.shg_profile_enable.argtypes = [P, I]
    lib.shg_profile_read.argtypes = [P, I, I, I, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64)]
    lib.shg_plan_create.argtypes = [P, C.POINTER(ShgShells), I, C.c_double, P, C.c_int64, P, P, P, C.c_uint,
                                    C.POINTER(C.c_void_p)]
    lib.shg_plan_create_r2n.argtypes = [P, C.POINTER(ShgShells), I, P, C.c_int64, P, P, P, C.c_uint,
                                        C.POINTER(C.c_void_p)]
    lib.shg_plan_create_r2n.restype = C.c_int
    lib.shg_plan_execute.argtypes = [P]
    lib.shg_plan_autotune.argtypes = [P, I, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.shg_plan_set_mode.argtypes = [P, I]
    lib.shg_plan_mode.argtypes = [P]
    lib.shg_plan_tile_order.argtypes = [P]
    lib.shg_plan_set_tile_order.argtypes = [P, I]
    lib.shg_plan_destroy.argtypes = [P]
    lib.shg_plan_destroy.restype = None
    lib.shg_plan_stats.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.shg_plan_kernel_ms.argtypes = [P, I, C.POINTER(C.c_double)]
    lib.shg_plan_time_kernels.argtypes = [P, I]
    lib.shg_plan_kernel_time.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.shg_plan_skipped.argtypes = [P, P, C.c_int64]
    lib.shg_plan_skipped.restype = C.c_int64
    lib.shg_plan_create_screened.argtypes = [P, C.POINTER(ShgShells), I, C.c_double, P, C.c_int64, P, P, P,
                                             C.c_uint, C.c_double, P, C.POINTER(C.c_void_p),
                                             C.POINTER(C.c_int64)]
    lib.shg_mlp_create.argtypes = [P, C.c_uint64, C.POINTER(C.c_void_p)]
    lib.shg_mlp_destroy.argtypes = [P]
    lib.shg_mlp_destroy.restype = None
    lib.shg_mlp_params.argtypes = [P, P, P]
    lib.shg_mlp_set_norm.argtypes = [P, P, P, P, P]
    lib.shg_mlp_set_margin.argtypes = [P, C.c_float]
    lib.shg_mlp_set_scope.argtypes = [P, C.c_uint32, I]
    lib.shg_mlp_train_step.argtypes = [P, P, P, I, C.c_float, C.c_float, P]
    lib.shg_mlp_grad.argtypes = [P, P, P, I, C.c_float, P, P]
    lib.shg_mlp_predict.argtypes = [P, P, C.c_int64, P, P]
    lib.shg_mlp_save.argtypes = [P, C.c_char_p]
    lib.shg_mlp_load.argtypes = [P, C.c_char_p]
    lib.shg_screen_features.argtypes = [P, C.POINTER(ShgShells), I, C.c_double, P, C.c_int64, I, P, P]
    lib.shg_block_logmax.argtypes = [P, C.POINTER(ShgShells), P, C.c_int64, P, P, P, P]
    _lib = lib
    return lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class DeviceShells:
    """A shell table resident in device memory (torch tensors) plus its C view."""

    def __init__(self, sh, device):
        import torch
        self.center = torch.as_tensor(np.ascontiguousarray(sh.center, np.float64), device=device)
        self.l = torch.as_tensor(np.ascontiguousarray(sh.l, np.int32), device=device)
        self.nprim = torch.as_tensor(np.ascontiguousarray(sh.nprim, np.int32), device=device)
        self.prim_off = torch.as_tensor(np.ascontiguousarray(sh.prim_off, np.int64), device=device)
        self.exps = torch.as_tensor(np.ascontiguousarray(sh.exps, np.float64), device=device)
        self.coefs = torch.as_tensor(np.ascontiguousarray(sh.coefs, np.float64), device=device)
        self.host = sh
        self.c = ShgShells(int(sh.n), int(len(sh.exps)), _ptr(self.center), _ptr(self.l), _ptr(self.nprim),
                           _ptr(self.prim_off), _ptr(self.exps), _ptr(self.coefs))


class DeviceSets:
    """A family-set table resident in device memory plus its C view."""

    def __init__(self, st, device):
        import torch
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a, dt), device=device)
        self.center = t(st.center, np.float64)
        self.nexp = t(st.nexp, np.int32)
        self.exp_off = t(st.exp_off, np.int64)
        self.exps = t(st.exps, np.float64)
        self.nfun = t(st.nfun, np.int32)
        self.fun_off = t(st.fun_off, np.int64)
        self.fun_l = t(st.fun_l, np.int32)
        self.coef_off = t(st.coef_off, np.int64)
        self.coefs = t(st.coefs, np.float64)
        self.host = st
        self.c = ShgSets(int(st.n), int(len(st.exps)), int(len(st.fun_l)), int(len(st.coefs)), _ptr(self.center),
                         _ptr(self.nexp), _ptr(self.exp_off), _ptr(self.exps), _ptr(self.nfun), _ptr(self.fun_off),
                         _ptr(self.fun_l), _ptr(self.coef_off), _ptr(self.coefs))


class Engine:
    """One shg_ctx bound to the current device and a torch stream."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libshg needs a ROCm GPU; none is visible")
        self.lib = load_library()
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = self.lib.shg_create(C.byref(h), C.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise ShgError(rc, self.lib.shg_last_error(None).decode())
        self.ctx = h
        # plans and models made on this context; closed before the context is
        self._children = weakref.WeakSet()

    def _adopt(self, obj):
        self._children.add(obj)

    def close(self):
        if getattr(self, "ctx", None):
            for ch in list(getattr(self, "_children", ())):
                ch.close()
            self.lib.shg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise ShgError(rc, self.lib.shg_last_error(self.ctx).decode())

    def set_tile_shape(self, op, la, lb, deriv, tp, rows_pp):
        self._check(self.lib.shg_set_tile_shape(self.ctx, OPS[op], la, lb, int(deriv), tp, rows_pp))

    def get_tile_shape(self, op, la, lb, deriv):
        tp, rows = C.c_int(), C.c_int()
        self._check(self.lib.shg_get_tile_shape(self.ctx, OPS[op], la, lb, int(deriv), C.byref(tp),
                                                C.byref(rows)))
        return tp.value, rows.value

    def autotune(self, dsh, op, omega, pairs, out_off, out, dout=None, reps=3):
        self._check(self.lib.shg_autotune(self.ctx, C.byref(dsh.c), OPS[op], float(omega), _ptr(pairs),
                                          int(pairs.shape[0]), _ptr(out_off), _ptr(out), _ptr(dout), reps))

    def tuning_save(self, path):
        self._check(self.lib.shg_tuning_save(self.ctx, path.encode()))

    def tuning_load(self, path) -> int:
        rc = self.lib.shg_tuning_load(self.ctx, path.encode())
        if rc < 0:
            self._check(rc)
        return rc

    def profile_enable(self, on=True):
        self._check(self.lib.shg_profile_enable(self.ctx, int(on)))

    def profile_read(self, la, lb, deriv):
        """(ms, launches, pairs) accumulated for class (la, lb, deriv); la < 0: binning."""
        ms, nl, npairs = C.c_double(), C.c_int64(), C.c_int64()
        self._check(self.lib.shg_profile_read(self.ctx, la, lb, int(deriv), C.byref(ms), C.byref(nl),
                                              C.byref(npairs)))
        return ms.value, nl.value, npairs.value

    def shells(self, sh) -> DeviceShells:
        return DeviceShells(sh, self.torch.device("cuda", self.torch.cuda.current_device()))

    def pairs(self, dsh: DeviceShells, op: str, omega: float, pairs, out_off, out, dout=None):
        """shg_pairs / shg_pairs_deriv on device tensors (pairs int32 [n,2], out_off int64 [n])."""
        n = int(pairs.shape[0])
        if dout is None:
            rc = self.lib.shg_pairs(self.ctx, C.byref(dsh.c), OPS[op], float(omega), _ptr(pairs), n,
                                    _ptr(out_off), _ptr(out))
        else:
            rc = self.lib.shg_pairs_deriv(self.ctx, C.byref(dsh.c), OPS[op], float(omega), _ptr(pairs), n,
                                          _ptr(out_off), _ptr(out), _ptr(dout))
        self._check(rc)

    def sets(self, st) -> DeviceSets:
        return DeviceSets(st, self.torch.device("cuda", self.torch.cuda.current_device()))

    def set_pairs(self, dst: DeviceSets, op: str, omega: float, set_pairs, out_off, out, dout=None):
        """shg_set_pairs: family-set pair blocks (and d/dR_A with `dout`) on device tensors."""
        n = int(set_pairs.shape[0])
        self._check(self.lib.shg_set_pairs(self.ctx, C.byref(dst.c), OPS[op], float(omega), _ptr(set_pairs), n,
                                           _ptr(out_off), _ptr(out), _ptr(dout)))

    def pairs_noalloc(self, dsh: DeviceShells, op: str, omega: float, pairs, out_off, out, dout=None):
        """shg_pairs_noalloc: shg_pairs / shg_pairs_deriv with the library's fixed
        scratch (no allocation in the call)."""
        n = int(pairs.shape[0])
        self._check(self.lib.shg_pairs_noalloc(self.ctx, C.byref(dsh.c), OPS[op], float(omega), _ptr(pairs), n,
                                               _ptr(out_off), _ptr(out), _ptr(dout)))

    def pairs_r2n(self, dsh: DeviceShells, nr: int, pairs, out_off, out, dout=None):
        """shg_pairs_r2n: (a|r_a^{2n}|b) (and d/dR_a with `dout`) on device tensors."""
        n = int(pairs.shape[0])
        rc = self.lib.shg_pairs_r2n(self.ctx, C.byref(dsh.c), int(nr), _ptr(pairs), n, _ptr(out_off), _ptr(out),
                                    _ptr(dout))
        self._check(rc)

    def pairs_swap(self, dsh: DeviceShells, pairs, src_off, dst_off, out, dout=None, check=False):
        """shg_pairs_swap: blocks of the swapped pairs (b, a) from those of pairs (a, b)."""
        n = int(pairs.shape[0])
        self._check(self.lib.shg_pairs_swap(self.ctx, C.byref(dsh.c), _ptr(pairs), n, _ptr(src_off), _ptr(dst_off),
                                            _ptr(out), _ptr(dout)))
        if check:
            self._check(self.lib.shg_pairs_swap_check(self.ctx))

    def fp64_ceiling(self, iters: int, blocks: int, out) -> float:
        """shg_fp64_ceiling: launch the FMA-chain kernel; returns its flop count."""
        fl = C.c_double()
        self._check(self.lib.shg_fp64_ceiling(self.ctx, int(iters), int(blocks), _ptr(out), C.byref(fl)))
        return fl.value

    def set_aab_chunk(self, chunk: int):
        """shg_set_aab_chunk: triples per (class, chunk) work item of shg_aab"""
        self._check(self.lib.shg_set_aab_chunk(self.ctx, int(chunk)))

    def aab(self, orb: DeviceShells, aux: DeviceShells, triples, out_off, out, dout=None):
        n = int(triples.shape[0])
        rc = self.lib.shg_aab(self.ctx, C.byref(orb.c), C.byref(aux.c), _ptr(triples), n, _ptr(out_off),
                              _ptr(out), _ptr(dout))
        self._check(rc)


PLAN_PERSISTENT = 1
NOALLOC_MAX_PAIRS = 1 << 20     # SHG_NOALLOC_MAX_PAIRS
PLAN_NO_GRAPH = 2
PLAN_COMPACT = 4


class Plan:
    """A recorded evaluation (shg_plan_*): fixed shells, operator, pairs and outputs.
    With `tau` the plan is screened (shg_plan_create_screened): pairs whose analytic
    bound, or (with `mlp`) learned prediction plus margin, is below tau are skipped."""

    def __init__(self, engine: "Engine", dsh: DeviceShells, op: str, omega: float, pairs, out_off, out, dout=None,
                 flags: int = 0, tau: float | None = None, mlp: "Mlp | None" = None, nr: int | None = None):
        """op "r2n" with `nr` records (a|r_a^{2n}|b) (shg_plan_create_r2n; omega ignored)."""
        self.engine = engine
        self.keep = (dsh, pairs, out_off, out, dout, mlp)   # the plan references these buffers
        h = C.c_void_p()
        self.n_skipped = 0
        if op == "r2n":
            engine._check(engine.lib.shg_plan_create_r2n(engine.ctx, C.byref(dsh.c), int(nr), _ptr(pairs),
                                                         int(pairs.shape[0]), _ptr(out_off), _ptr(out), _ptr(dout),
                                                         int(flags), C.byref(h)))
        elif tau is None:
            engine._check(engine.lib.shg_plan_create(engine.ctx, C.byref(dsh.c), OPS[op], float(omega),
                                                     _ptr(pairs), int(pairs.shape[0]), _ptr(out_off), _ptr(out),
                                                     _ptr(dout), int(flags), C.byref(h)))
        else:
            ns = C.c_int64()
            engine._check(engine.lib.shg_plan_create_screened(
                engine.ctx, C.byref(dsh.c), OPS[op], float(omega), _ptr(pairs), int(pairs.shape[0]),
                _ptr(out_off), _ptr(out), _ptr(dout), int(flags), float(tau), mlp.h if mlp else None, C.byref(h),
                C.byref(ns)))
            self.n_skipped = ns.value
        self.h = h
        engine._adopt(self)

    def execute(self):
        self.engine._check(self.engine.lib.shg_plan_execute(self.h))

    def autotune(self, reps=3):
        a, b = C.c_double(), C.c_double()
        self.engine._check(self.engine.lib.shg_plan_autotune(self.h, reps, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_mode(self, persistent: bool):
        self.engine._check(self.engine.lib.shg_plan_set_mode(self.h, int(persistent)))

    def stats(self):
        """(pairs evaluated, their algorithmic bytes)"""
        k, b = C.c_int64(), C.c_int64()
        self.engine._check(self.engine.lib.shg_plan_stats(self.h, C.byref(k), C.byref(b)))
        return k.value, b.value

    def skipped(self) -> np.ndarray:
        n = self.engine.lib.shg_plan_skipped(self.h, None, 0)
        ids = np.zeros(max(n, 0), np.int32)
        if n > 0:
            self.engine.lib.shg_plan_skipped(self.h, ids.ctypes.data_as(C.c_void_p), n)
        return ids

    def kernel_ms(self, reps=3) -> float:
        ms = C.c_double()
        self.engine._check(self.engine.lib.shg_plan_kernel_ms(self.h, reps, C.byref(ms)))
        return ms.value

    def time_kernels(self, on: bool = True):
        """record HIP events around the evaluation kernels of every later execute"""
        self.engine._check(self.engine.lib.shg_plan_time_kernels(self.h, int(on)))

    def kernel_time(self):
        """(summed kernel ms, timed executions) since the last call; synchronises"""
        ms, k = C.c_double(), C.c_int64()
        self.engine._check(self.engine.lib.shg_plan_kernel_time(self.h, C.byref(ms), C.byref(k)))
        return ms.value, k.value

    def set_tile_order(self, order: str):
        """fix the persistent queue's tile order without timing the alternatives"""
        code = {"heaviest-first": 0, "alternating": 1, "round-robin": 2}[order]
        self.engine._check(self.engine.lib.shg_plan_set_tile_order(self.h, code))

    @property
    def tile_order(self) -> str:
        return {0: "heaviest-first", 1: "alternating", 2: "round-robin"}.get(
            self.engine.lib.shg_plan_tile_order(self.h), "?")

    @property
    def mode(self) -> str:
        return {0: "per-class", 1: "persistent"}.get(self.engine.lib.shg_plan_mode(self.h), "?")

    def close(self):
        if getattr(self, "h", None):
            self.engine.lib.shg_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NPARAM = 9217
NFEAT = 12


class Mlp:
    """The learned prescreener (shg_mlp_*); device buffers are torch tensors."""

    def __init__(self, engine: "Engine", seed: int = 0):
        self.engine = engine
        h = C.c_void_p()
        engine._check(engine.lib.shg_mlp_create(engine.ctx, C.c_uint64(seed), C.byref(h)))
        self.h = h
        engine._adopt(self)

    def close(self):
        if getattr(self, "h", None):
            self.engine.lib.shg_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.zeros(NPARAM, np.float32)
        self.engine._check(self.engine.lib.shg_mlp_params(self.h, out.ctypes.data_as(C.c_void_p), None))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        self.engine._check(self.engine.lib.shg_mlp_params(self.h, None, p.ctypes.data_as(C.c_void_p)))

    def set_norm(self, mean, std, lo=None, hi=None):
        arrs = [np.ascontiguousarray(x, np.float32) if x is not None else None for x in (mean, std, lo, hi)]
        ptrs = [a.ctypes.data_as(C.c_void_p) if a is not None else None for a in arrs]
        self.engine._check(self.engine.lib.shg_mlp_set_norm(self.h, *ptrs))

    def set_margin(self, m: float):
        self.engine._check(self.engine.lib.shg_mlp_set_margin(self.h, float(m)))

    def set_scope(self, ops, deriv_targets: bool):
        """operators (names) the model predicts, and whether its targets include d/dR_a"""
        mask = 0
        for o in ops:
            mask |= 1 << OPS[o]
        self.engine._check(self.engine.lib.shg_mlp_set_scope(self.h, mask, int(deriv_targets)))

    def train_step(self, X, y, lr, quantile, loss_out=None):
        self.engine._check(self.engine.lib.shg_mlp_train_step(self.h, _ptr(X), _ptr(y), int(X.shape[0]), float(lr),
                                                              float(quantile), _ptr(loss_out)))

    def grad(self, X, y, quantile, grad_out, loss_out=None):
        self.engine._check(self.engine.lib.shg_mlp_grad(self.h, _ptr(X), _ptr(y), int(X.shape[0]), float(quantile),
                                                        _ptr(grad_out), _ptr(loss_out)))

    def predict(self, X, pred, in_range):
        self.engine._check(self.engine.lib.shg_mlp_predict(self.h, _ptr(X), int(X.shape[0]), _ptr(pred),
                                                           _ptr(in_range)))

    def save(self, path):
        self.engine._check(self.engine.lib.shg_mlp_save(self.h, path.encode()))

    def load(self, path):
        self.engine._check(self.engine.lib.shg_mlp_load(self.h, path.encode()))


def screen_features(engine: Engine, dsh: DeviceShells, op: str, omega: float, pairs, deriv: bool = False):
    """(features [n,12] fp32, log10 analytic bound [n] fp32) on the device; with
    `deriv` the bound also covers the d/dR_a elements."""
    torch = engine.torch
    n = int(pairs.shape[0])
    feat = torch.empty((max(n, 1), NFEAT), dtype=torch.float32, device=pairs.device)
    logb = torch.empty(max(n, 1), dtype=torch.float32, device=pairs.device)
    engine._check(engine.lib.shg_screen_features(engine.ctx, C.byref(dsh.c), OPS[op], float(omega), _ptr(pairs), n,
                                                 int(deriv), _ptr(feat), _ptr(logb)))
    return feat[:n], logb[:n]


def block_logmax(engine: Engine, dsh: DeviceShells, pairs, out_off, out, dout=None):
    """log10 max|element| per block (values, and with `dout` the d/dR_a blocks too)"""
    torch = engine.torch
    n = int(pairs.shape[0])
    y = torch.empty(max(n, 1), dtype=torch.float32, device=pairs.device)
    engine._check(engine.lib.shg_block_logmax(engine.ctx, C.byref(dsh.c), _ptr(pairs), n, _ptr(out_off), _ptr(out),
                                              _ptr(dout), _ptr(y)))
    return y[:n]


def run_workload_pairs(engine: Engine, w, op: str, deriv: bool):
    """Upload a workload, evaluate one operator, return host numpy (out, dout)."""
    torch = engine.torch
    dev = torch.device("cuda", torch.cuda.current_device())
    dsh = engine.shells(w.shells)
    off, tot = w.out_offsets()
    pairs = torch.as_tensor(np.ascontiguousarray(w.pairs, np.int32), device=dev)
    out_off = torch.as_tensor(off, device=dev)
    out = torch.full((max(tot, 1),), float("nan"), dtype=torch.float64, device=dev)
    dout = torch.full((max(3 * tot, 1),), float("nan"), dtype=torch.float64, device=dev) if deriv else None
    engine.pairs(dsh, op, w.omega.get(op, 0.0), pairs, out_off, out, dout)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:tot], (dout.cpu().numpy()[:3 * tot] if deriv else None)
