"""Python binding of libhbj, the MI355X block-Jacobi sweeping Helmholtz solver.

Argument marshalling only: every computation runs in the HIP library behind the C
ABI of ``include/hbj.h``.  torch supplies device memory (tensors on ``cuda``) and
the stream.  Importing this package fails loudly when the library is not built.

    import paper_2209_10886_amd as hbj
    ctx = hbj.setup(nx=1024, ny=1024, k=k, n1=8, n2=8, c=c_tensor)
    ctx.factor()
    u, stats = ctx.solve(f, tol=1e-6)
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhbj.so")

if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2209_10886_amd.build` "
                      "(or __graft_entry__.build()); there is no fallback implementation")

_lib = ctypes.CDLL(_LIB_PATH)

FP64, MIXED = 0, 1
PC_NONE, PC_SGS, PC_BJ = 0, 1, 2
BJ_RESTRICTED, BJ_ADDITIVE = 0, 1
BJ_PRODUCT, BJ_RESIDUAL = 0, 1
OP_BANDED, OP_DENSE = 0, 1
SWEEP_STEPPED, SWEEP_DATAFLOW = 0, 1
ORTH_CGS2, ORTH_DCGS2, ORTH_SSTEP, ORTH_AUTO = 0, 1, 2, 3  # Gram-Schmidt variant of the Arnoldi steps
MSOLVE_CHAINS, MSOLVE_MFMA = 0, 1  # banded solves of many right-hand sides per subdomain
OK, EINVAL, ESTATE, EHIP, ENOMEM, EWAIT, EIO, ZERO_PIVOT, NOT_CONVERGED = 0, -1, -2, -3, -4, -5, -6, 1, 2
# launch shapes of the banded solve batches (hbj_set_solve_tuning): one workgroup per solve at three
# register prefetch depths, 16 right-hand sides per workgroup on MFMA, or each solve split over
# several workgroups (runs of column blocks, hbj_set_solve_partitions)
SOLVE_SHAPES = ("workgroup per solve, depth 0", "workgroup per solve, depth 1", "workgroup per solve, depth 2",
                "MFMA tiles of 16 right-hand sides", "split over runs of column blocks")
SOLVE_SHAPE_MFMA = 3
SOLVE_SHAPE_SPLIT = 4
VR_NOALLOC_MAX_RHS = 64  # right-hand sides the allocation-free residual's static scratch holds
K_FWD, K_BWD, K_FACTOR, K_KRYLOV, K_SCATTER, K_SWEEP, K_LIFT, K_OPERATOR = 0, 1, 2, 3, 4, 5, 6, 7


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("h", ctypes.c_double), ("k", ctypes.c_double),
                ("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("bj_width", ctypes.c_int32), ("bj_combine", ctypes.c_int32),
                ("bj_compose", ctypes.c_int32), ("operator_form", ctypes.c_int32), ("sweep_exec", ctypes.c_int32),
                ("transmission", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("flexible", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("steps_per_pc", ctypes.c_int32), ("local_ir_max", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("relres", ctypes.c_double), ("seconds", ctypes.c_double),
                ("local_solves", ctypes.c_int64), ("res_hist", ctypes.POINTER(ctypes.c_double)),
                ("res_hist_len", ctypes.c_int32), ("local_ir_resid", ctypes.c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I32 = ctypes.c_int32
_SIGS = {
    "hbj_setup": (_I, [ctypes.POINTER(Problem), _P, _P, ctypes.POINTER(_P)]),
    "hbj_set_slowness2": (_I, [_P, _P]),
    "hbj_factor": (_I, [_P]),
    "hbj_zero_pivot": (_I, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "hbj_apply_operator": (_I, [_P, _P, _P, _I32]),
    "hbj_apply_preconditioner": (_I, [_P, _P, _P, _I32]),
    "hbj_lifting": (_I, [_P, _P, _P, _I32]),
    "hbj_reconstruct": (_I, [_P, _P, _P, _P, _I32]),
    "hbj_solve": (_I, [_P, _P, _P, _I32, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)]),
    "hbj_gradient": (_I, [_P, _P, _I32, _P, _I32, _P, _P, ctypes.POINTER(ctypes.c_double), _P,
                          ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats)]),
    "hbj_volume_residual": (_I, [_P, _P, _P, _I32, ctypes.POINTER(ctypes.c_double)]),
    "hbj_volume_residual_noalloc": (_I, [_P, _P, _P, _I32, _P]),
    "hbj_local_solve": (_I, [_P, _I32, ctypes.POINTER(_I32), _P, _P, _I32]),
    "hbj_band_factors": (_I, [_P, _I32, _P, _P]),
    "hbj_interface_len": (_I32, [_P]),
    "hbj_sizes": (_I, [_P] + [ctypes.POINTER(_I32)] * 5),
    "hbj_steps_per_preconditioner": (_I32, [_P]),
    "hbj_set_profiling": (_I, [_P, _I32]),
    "hbj_kernel_stats": (_I, [_P, _I32, ctypes.POINTER(KernelStat)]),
    "hbj_reset_kernel_stats": (_I, [_P]),
    "hbj_set_sweep_wait": (_I, [_P, _I32, _I32]),
    "hbj_get_tuning": (_I, [_P, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_float)]),
    "hbj_set_tuning": (_I, [_P, ctypes.POINTER(_I32)]),
    "hbj_set_solve_tuning": (_I, [_P, _I32]),
    "hbj_set_solve_partitions": (_I, [_P, _I32]),
    "hbj_set_operator_overlap": (_I, [_P, _I32]),
    "hbj_get_solve_tuning": (_I, [_P, ctypes.POINTER(_I32), ctypes.c_char_p, ctypes.POINTER(_I32),
                                  ctypes.POINTER(ctypes.c_float)]),
    "hbj_tune_cache_path": (ctypes.c_char_p, []),
    "hbj_tune_cache_set_path": (_I, [ctypes.c_char_p]),
    "hbj_tune_cache_lookup": (_I, [ctypes.c_char_p, ctypes.POINTER(_I32)]),
    "hbj_tune_cache_store": (_I, [ctypes.c_char_p, _I32, ctypes.POINTER(ctypes.c_float), _I32]),
    "hbj_tune_cache_size": (_I32, []),
    "hbj_set_graphs": (_I, [_P, _I32]),
    "hbj_set_orthogonalization": (_I, [_P, _I32]),
    "hbj_set_sstep_block": (_I, [_P, _I32]),
    "hbj_set_step_chaining": (_I, [_P, _I32]),
    "hbj_set_multi_solve": (_I, [_P, _I32]),
    "hbj_strerror": (ctypes.c_char_p, [_I]),
    "hbj_last_error": (ctypes.c_char_p, []),
    "hbj_destroy": (None, [_P]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


class HbjError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_lib.hbj_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _check(code, allow=()):
    if code != OK and code not in allow:
        raise HbjError(code, _lib.hbj_last_error().decode())
    return code


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return _P(t.data_ptr())


@dataclasses.dataclass
class Stats:
    iters: int
    steps_per_pc: int
    local_ir_max: int
    converged: int
    relres: float
    seconds: float
    local_solves: int
    history: list
    code: int
    local_ir_resid: float = 0.0


def _stats(st: SolveStats, hist, code) -> Stats:
    return Stats(st.iters, st.steps_per_pc, st.local_ir_max, st.converged, st.relres, st.seconds, st.local_solves,
                 list(hist[: st.res_hist_len]), code, st.local_ir_resid)


class Context:
    """One problem on one stream (hbj_ctx)."""

    def __init__(self, prob: Problem, c: torch.Tensor, stream=None):
        self.nx, self.ny = prob.nx, prob.ny
        self.device = c.device
        s = torch.cuda.current_stream(c.device) if stream is None else stream
        self._stream = s
        h = _P()
        _check(_lib.hbj_setup(ctypes.byref(prob), _dev(c, torch.float64, "c"), _P(s.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.prob = prob
        self.nif = int(_lib.hbj_interface_len(h))
        a = [_I32() for _ in range(5)]
        _check(_lib.hbj_sizes(h, *[ctypes.byref(x) for x in a]))
        self.sub_nx, self.sub_ny, self.n_loc, self.kl, self.ndom = (int(x.value) for x in a)

    # -- lifecycle -------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.hbj_destroy(self._h)
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

    # -- operations --------------------------------------------------------
    def set_slowness2(self, m: torch.Tensor):
        _check(_lib.hbj_set_slowness2(self._h, _dev(m, torch.float64, "m")))

    def factor(self):
        code = _lib.hbj_factor(self._h)
        if code == ZERO_PIVOT:
            s, r = _I32(), _I32()
            _lib.hbj_zero_pivot(self._h, ctypes.byref(s), ctypes.byref(r))
            raise HbjError(code, f"subdomain {s.value} row {r.value}")
        _check(code)

    def _vec(self, nrhs):
        return torch.empty((nrhs, self.nif), dtype=torch.complex128, device=self.device)

    def _field(self, nrhs):
        return torch.empty((nrhs, self.ny, self.nx), dtype=torch.complex128, device=self.device)

    @staticmethod
    def _nrhs(t, trailing):
        return 1 if t.dim() == trailing else t.shape[0]

    def apply_operator(self, g, out=None):
        n = self._nrhs(g, 1)
        out = self._vec(n).view(g.shape) if out is None else out
        _check(_lib.hbj_apply_operator(self._h, _dev(g, torch.complex128, "g"), _dev(out, torch.complex128, "out"), n))
        return out

    def apply_preconditioner(self, r, out=None):
        n = self._nrhs(r, 1)
        out = self._vec(n).view(r.shape) if out is None else out
        _check(_lib.hbj_apply_preconditioner(self._h, _dev(r, torch.complex128, "r"),
                                             _dev(out, torch.complex128, "z"), n))
        return out

    def lifting(self, f, out=None):
        n = self._nrhs(f, 2)
        out = (self._vec(n) if f.dim() == 3 else self._vec(1)[0]) if out is None else out
        _check(_lib.hbj_lifting(self._h, _dev(f, torch.complex128, "f"), _dev(out, torch.complex128, "b"), n))
        return out

    def reconstruct(self, f, g, out=None):
        n = self._nrhs(f, 2)
        out = torch.empty_like(f) if out is None else out
        gp = _dev(g, torch.complex128, "g") if self.nif else _P(0)
        _check(_lib.hbj_reconstruct(self._h, _dev(f, torch.complex128, "f"), gp, _dev(out, torch.complex128, "u"), n))
        return out

    def solve(self, f, tol=1e-6, restart=50, maxit=1000, flexible=True, out=None, hist_len=4096, check=True):
        n = self._nrhs(f, 2)
        out = torch.empty_like(f) if out is None else out
        opts = SolveOpts(tol, restart, maxit, 1 if flexible else 0)
        hist = (ctypes.c_double * hist_len)()
        st = SolveStats()
        st.res_hist = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        st.res_hist_len = hist_len
        code = _lib.hbj_solve(self._h, _dev(f, torch.complex128, "f"), _dev(out, torch.complex128, "u"), n,
                              ctypes.byref(opts), ctypes.byref(st))
        _check(code, allow=() if check else (NOT_CONVERGED,))
        return out, _stats(st, hist, code)

    def gradient(self, f, rec_idx, d, tol=1e-10, restart=50, maxit=2000, flexible=True, return_u=False):
        """(loss, dL/dm [ny, nx] float64[, u]) by forward + adjoint solves."""
        n = self._nrhs(f, 2)
        grad = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        u = torch.empty_like(f) if return_u else None
        loss = ctypes.c_double()
        opts = SolveOpts(tol, restart, maxit, 1 if flexible else 0)
        st = SolveStats()
        _check(_lib.hbj_gradient(self._h, _dev(f, torch.complex128, "f"), n, _dev(rec_idx, torch.int32, "rec_idx"),
                                 rec_idx.numel(), _dev(d, torch.complex128, "d"), _dev(grad, torch.float64, "grad"),
                                 ctypes.byref(loss), _dev(u, torch.complex128, "u") if u is not None else _P(0),
                                 ctypes.byref(opts), ctypes.byref(st)))
        return (loss.value, grad, u) if return_u else (loss.value, grad)

    def volume_residual(self, f, u):
        """||f - A u|| / ||f|| of the global discrete problem per right-hand side (list of floats)."""
        n = self._nrhs(f, 2)
        if u.shape != f.shape:
            raise ValueError("f and u must have the same shape")
        out = (ctypes.c_double * n)()
        _check(_lib.hbj_volume_residual(self._h, _dev(f, torch.complex128, "f"), _dev(u, torch.complex128, "u"), n,
                                        out))
        return [float(x) for x in out]

    def volume_residual_noalloc(self, f, u, out):
        """The same residuals into the caller's device tensor out [nrhs] float64, through the
        library's static scratch (no allocation, no host synchronisation)."""
        n = self._nrhs(f, 2)
        if u.shape != f.shape:
            raise ValueError("f and u must have the same shape")
        if out.numel() < n:
            raise ValueError("out holds fewer than nrhs entries")
        _check(_lib.hbj_volume_residual_noalloc(self._h, _dev(f, torch.complex128, "f"), _dev(u, torch.complex128, "u"),
                                                n, _dev(out, torch.float64, "relres")))
        return out

    def local_solve(self, subs, rhs, precision=FP64, out=None):
        subs = [int(s) for s in subs]
        arr = (_I32 * len(subs))(*subs)
        out = torch.empty_like(rhs) if out is None else out
        _check(_lib.hbj_local_solve(self._h, len(subs), arr, _dev(rhs, torch.complex128, "rhs"),
                                    _dev(out, torch.complex128, "x"), precision))
        return out

    def band_factors(self, s):
        ldab = 3 * self.kl + 1
        ab = torch.empty((self.n_loc, ldab), dtype=torch.complex128, device=self.device)
        ip = torch.empty(self.n_loc, dtype=torch.int32, device=self.device)
        _check(_lib.hbj_band_factors(self._h, s, _dev(ab, torch.complex128, "ab"), _dev(ip, torch.int32, "ipiv")))
        return ab, ip

    def steps_per_preconditioner(self):
        return int(_lib.hbj_steps_per_preconditioner(self._h))

    def set_profiling(self, on=True):
        _check(_lib.hbj_set_profiling(self._h, 1 if on else 0))

    def kernel_stats(self, kclass):
        ks = KernelStat()
        _check(_lib.hbj_kernel_stats(self._h, kclass, ctypes.byref(ks)))
        return {"launches": ks.launches, "ms": ks.ms, "bytes": ks.bytes, "flops": ks.flops}

    def reset_kernel_stats(self):
        _check(_lib.hbj_reset_kernel_stats(self._h))

    def set_graphs(self, on=True):
        """Replay GMRES iterations as HIP graphs (default off: one-by-one launches are faster once
        the next step is queued ahead)."""
        _check(_lib.hbj_set_graphs(self._h, 1 if on else 0))

    def set_orthogonalization(self, mode):
        """ORTH_CGS2 (classical Gram-Schmidt twice), ORTH_DCGS2 (delayed reorthogonalisation),
        ORTH_SSTEP (s-step cycles: blocks of s steps orthogonalised together) or ORTH_AUTO (s-step
        cycles for large blocks of Krylov vectors, delayed reorthogonalisation otherwise; default)
        for the Arnoldi steps."""
        _check(_lib.hbj_set_orthogonalization(self._h, int(mode)))

    def set_step_chaining(self, on=True):
        """Chained sweep steps on the many-right-hand-side path (default on): each step writes the
        next step's gathered tile; the same results bit for bit."""
        _check(_lib.hbj_set_step_chaining(self._h, 1 if on else 0))

    def set_sstep_block(self, s):
        """Steps per block of the ORTH_SSTEP cycles (1..8, default 8)."""
        _check(_lib.hbj_set_sstep_block(self._h, int(s)))

    def set_multi_solve(self, mode):
        """MSOLVE_CHAINS (one workgroup per subdomain and right-hand side) or MSOLVE_MFMA (16
        right-hand sides of one subdomain per workgroup on the matrix cores, default) for batches
        of banded solves with many right-hand sides per subdomain."""
        _check(_lib.hbj_set_multi_solve(self._h, int(mode)))

    def tuning(self):
        """Autotuned variants of the many-RHS operator kernel with the measured us per launch of every
        variant. Variants 0-11: batches of 2, 4 or 8 k-steps, the incoming data gathered into tiles
        first or read from the interface vector, one or two wavefront groups sharing the right-hand
        sides; 12-15: a register ring of 4 or 8 k-steps over all faces, gathered or direct, two groups;
        16, 17: gathered/4 and direct/2 with two groups; 12-17 place the tiles of a subdomain on one XCD;
        18-21: eight wavefronts splitting the k range (one group), 2 or 4 k-steps, gathered or direct."""
        nv = MM_VARIANTS
        v = (_I32 * 4)()
        us = (ctypes.c_float * (4 * nv))()
        _check(_lib.hbj_get_tuning(self._h, v, us))
        kinds = ("c128 steps", "c128 operator", "c64 steps", "c64 operator")
        label = [mm_variant_label(j) for j in range(nv)]
        out = {}
        for i, k in enumerate(kinds):
            j = v[i]
            if j < 0:
                out[k] = {"k_steps_per_batch": None, "incoming": None, "wave_groups": None, "k_waves": None,
                          "ring": None, "xcd_order": None, "us": None}
                continue
            d = mm_variant_fields(j)
            d["us"] = {label[q]: round(us[i * nv + q], 2) for q in range(nv)}
            out[k] = d
        return out

    def set_tuning(self, variants):
        """Fix the many-RHS operator kernel's variant per kind (c128 steps, c128 operator, c64 steps,
        c64 operator): 0-21, or -1 to let the autotuner choose."""
        v = (_I32 * 4)(*[int(x) for x in variants])
        _check(_lib.hbj_set_tuning(self._h, v))

    def set_operator_overlap(self, on):
        """Apply the operator to the preconditioned vector beside the backward pass, or after it (default)."""
        _check(_lib.hbj_set_operator_overlap(self._h, 1 if on else 0))

    def set_solve_tuning(self, shape):
        """Fix the launch shape of every banded solve batch (0-2: one workgroup per solve at the three
        prefetch depths, 3: MFMA tiles where they apply, 4: each solve split over runs of column
        blocks), or -1 to choose per batch class by timing."""
        _check(_lib.hbj_set_solve_tuning(self._h, int(shape)))

    def set_solve_partitions(self, np_runs=0):
        """Runs per local solve of the split launch shape (2..4096; 0: the default, 16)."""
        _check(_lib.hbj_set_solve_partitions(self._h, int(np_runs)))

    def solve_tuning(self):
        """The launch shapes chosen so far, per batch class: {key: {"shape": s, "us": [per shape]}}
        (us 0: not timed here, the choice came from the tuning cache file or was fixed)."""
        n = _I32(0)
        _check(_lib.hbj_get_solve_tuning(self._h, ctypes.byref(n), None, None, None))
        cap = n.value
        if cap == 0:
            return {}
        keys = ctypes.create_string_buffer(96 * cap)
        shapes = (_I32 * cap)()
        ns = len(SOLVE_SHAPES)
        us = (ctypes.c_float * (ns * cap))()
        n = _I32(cap)
        _check(_lib.hbj_get_solve_tuning(self._h, ctypes.byref(n), keys, shapes, us))
        out = {}
        for i in range(min(cap, n.value)):
            key = keys.raw[96 * i:96 * (i + 1)].split(b"\0", 1)[0].decode()
            out[key] = {"shape": int(shapes[i]), "us": [round(us[ns * i + j], 2) for j in range(ns)]}
        return out

    def set_sweep_wait(self, max_polls=0, stall_task=-1):
        """Bounds of the dataflow sweeps' dependency waits (error-path tests)."""
        _check(_lib.hbj_set_sweep_wait(self._h, max_polls, stall_task))


MM_VARIANTS = 22  # variants of the many-right-hand-side operator kernel (hbj_set_tuning)


def mm_variant_fields(v):
    """What variant v of the many-right-hand-side operator kernel is (see Context.tuning)."""
    if v < 12:
        return {"k_steps_per_batch": (2, 4, 8)[v % 3], "incoming": "gathered" if v % 6 < 3 else "direct",
                "wave_groups": (1, 2)[v // 6], "k_waves": 4, "ring": False, "xcd_order": False}
    if v < 16:
        return {"k_steps_per_batch": (4, 8)[v % 2], "incoming": "gathered" if v < 14 else "direct",
                "wave_groups": 2, "k_waves": 4, "ring": True, "xcd_order": True}
    if v < 18:
        return {"k_steps_per_batch": 4 if v == 16 else 2, "incoming": "gathered" if v == 16 else "direct",
                "wave_groups": 2, "k_waves": 4, "ring": False, "xcd_order": True}
    return {"k_steps_per_batch": (2, 4)[v % 2], "incoming": "gathered" if v < 20 else "direct",
            "wave_groups": 1, "k_waves": 8, "ring": False, "xcd_order": False}


def mm_variant_label(v):
    d = mm_variant_fields(v)
    return (f"{d['incoming']}/{'ring' if d['ring'] else ''}{d['k_steps_per_batch']}/{d['wave_groups']}"
            f"{'/k8' if d['k_waves'] == 8 else ''}{'/xcd' if d['xcd_order'] else ''}")


def tune_cache_path():
    """The tuning cache file in use ("" = none)."""
    return _lib.hbj_tune_cache_path().decode()


def set_tune_cache_path(path):
    """Use `path` as the tuning cache file (None: the default rule, "": no file) and read it."""
    _check(_lib.hbj_tune_cache_set_path(None if path is None else str(path).encode()))


def tune_cache_lookup(key):
    """The cached variant for `key`, or None."""
    v = _I32(0)
    r = _lib.hbj_tune_cache_lookup(key.encode(), ctypes.byref(v))
    if r < 0:
        raise HbjError(r, f"tuning cache lookup {key!r}")
    return int(v.value) if r == 1 else None


def tune_cache_store(key, variant, us=()):
    """Record key -> (variant, us) in the tuning cache and rewrite its file."""
    arr = (ctypes.c_float * max(1, len(us)))(*[float(x) for x in us])
    r = _lib.hbj_tune_cache_store(key.encode(), int(variant), arr, len(us))
    if r != OK:
        raise HbjError(r, f"tuning cache entry {key!r}")


def tune_cache_size():
    return int(_lib.hbj_tune_cache_size())


def setup(nx, ny, k, n1, n2, c=None, m=None, h=0.0, precision=FP64, precond=PC_BJ, bj_width=0,
          bj_combine=BJ_RESTRICTED, bj_compose=BJ_PRODUCT, operator_form=OP_BANDED, sweep_exec=SWEEP_STEPPED,
          transmission=1, device="cuda", stream=None) -> Context:
    """hbj_setup with a wave speed c (or squared slowness m) given as a [ny, nx] float64 tensor.
    transmission: 1 (Robin) or 2 (second-order condition on interface faces), in either operator form;
    3 (the Pade condition with 8 auxiliary fields and branch rotation pi/3) in the dense form."""
    prob = Problem(nx, ny, h, k, n1, n2, precision, precond, bj_width, bj_combine, bj_compose, operator_form,
                   sweep_exec, transmission)
    if c is None and m is None:
        raise ValueError("give c or m")
    if c is None:
        m = m.to(device=device, dtype=torch.float64).contiguous()
        ctx = Context(prob, torch.ones_like(m), stream)
        ctx.set_slowness2(m)
        return ctx
    return Context(prob, c.to(device=device, dtype=torch.float64).contiguous(), stream)
