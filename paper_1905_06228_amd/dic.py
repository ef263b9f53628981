"""ctypes binding of libdic.so.

Argument marshalling only: every step of the correlation runs in the HIP
library.  Tensors must be CUDA tensors on the plan's device; the calls are
asynchronous on the current torch stream.  There is no fallback: a missing
library or a non-GPU tensor raises.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdic.so")

FP32_BATCHED = 0
FP64_PLAIN = 1
FLAG_USE_GRAPH = 1
FLAG_CACHE_REF_PREP = 2
FLAG_DETERMINISTIC_BWD = 4
FLAG_REFINE_NR = 8
FLAG_INTERP_BILINEAR = 16   # IC-GN / Newton-Raphson with Eq. (5) bilinear interpolation
FLAG_BICUBIC_LUT = 32       # IC-GN / Newton-Raphson from the per-cell bicubic coefficient table
FLAG_INTERP_BSPLINE = 64    # IC-GN / Newton-Raphson with cubic B-spline interpolation

POI_OK = 0
POI_NOT_CONVERGED = 1
POI_OUT_OF_BOUNDS = 2
POI_ZERO_VARIANCE = 3
POI_SINGULAR_HESSIAN = 4
POI_NO_VALID_CANDIDATE = 5
POI_NAN_INPUT = 6
STATUS_NAMES = {POI_OK: "OK", POI_NOT_CONVERGED: "NOT_CONVERGED",
                POI_OUT_OF_BOUNDS: "OUT_OF_BOUNDS", POI_ZERO_VARIANCE: "ZERO_VARIANCE",
                POI_SINGULAR_HESSIAN: "SINGULAR_HESSIAN",
                POI_NO_VALID_CANDIDATE: "NO_VALID_CANDIDATE", POI_NAN_INPUT: "NAN_INPUT"}


def status_histogram(status) -> dict:
    """Count of every per-POI status code in ``status`` (a tensor or array of
    codes), by name; a code outside the table is counted as ``UNKNOWN_<code>``."""
    import numpy as np
    a = status.detach().cpu().numpy() if isinstance(status, torch.Tensor) else np.asarray(status)
    codes, counts = np.unique(a.astype(np.int64).ravel(), return_counts=True)
    return {STATUS_NAMES.get(int(c), f"UNKNOWN_{int(c)}"): int(n) for c, n in zip(codes, counts)}


class PairDesc(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("subset_radius", ctypes.c_int32), ("search_radius", ctypes.c_int32),
                ("ref_offset", ctypes.c_int64), ("def_offset", ctypes.c_int64),
                ("poi_offset", ctypes.c_int64), ("poi_count", ctypes.c_int64)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("num_pairs", ctypes.c_int32), ("pairs", ctypes.POINTER(PairDesc)),
                ("precision", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("conv_tol", ctypes.c_double), ("flags", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    _fields_ = [("search_block", ctypes.c_int32), ("search_occupancy", ctypes.c_int32),
                ("icgn_waves", ctypes.c_int32), ("icgn_slack", ctypes.c_int32)]


PSO_PARTICLES = 50      # swarm size of dic_pso_search
PSO_GENERATIONS = 5     # its maximum number of generations

EXPORTS = [
    "dic_plan_create", "dic_plan_workspace_size", "dic_plan_bind", "dic_plan_get_tuning",
    "dic_plan_set_tuning", "dic_plan_autotune", "dic_plan_invalidate_reference",
    "dic_prepare_reference", "dic_prepare_deformed", "dic_integer_search", "dic_pso_search",
    "dic_icgn_refine", "dic_nr_refine", "dic_correlate", "dic_correlate_noalloc",
    "dic_znssd_backward", "dic_seed_update", "dic_poi_grid", "dic_plan_destroy",
    "dic_status_string", "dic_last_error",
]

_lib = None


class DicError(RuntimeError):
    pass


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise DicError(f"{path} is missing: build it with __graft_entry__.build() "
                       "or python paper_1905_06228_amd/build.py")
    L = ctypes.CDLL(path)
    P, V, I32, I64 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.dic_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(P)]
    L.dic_plan_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    L.dic_plan_bind.argtypes = [P, V, ctypes.c_size_t, V]
    L.dic_plan_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    L.dic_plan_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    L.dic_plan_autotune.argtypes = [P, V, V, V, V, V, V, V, V]
    L.dic_plan_invalidate_reference.argtypes = [P]
    L.dic_prepare_reference.argtypes = [P, V, V, V]
    L.dic_prepare_deformed.argtypes = [P, V, V]
    L.dic_integer_search.argtypes = [P, V, V, V, V, V, V, V, V]
    L.dic_pso_search.argtypes = [P, V, V, V, V, V, I32, V, V, V, V, V, V]
    L.dic_icgn_refine.argtypes = [P, V, V, V, V, V, V, V, V, V, V, V]
    L.dic_nr_refine.argtypes = [P, V, V, V, V, V, V, V, V, V, V, V]
    L.dic_correlate.argtypes = [P, V, V, V, V, V, V, V, V, V, V, V, V, V]
    L.dic_correlate_noalloc.argtypes = [P, V, V, V, V, V, V, V, V, V, V, V, V, V]
    L.dic_znssd_backward.argtypes = [P, V, V, V, V, V, V, V, V, V]
    L.dic_seed_update.argtypes = [P, V, V, V, V, V]
    L.dic_poi_grid.argtypes = [I32, I32, I32, I32, I32, V, I64, ctypes.POINTER(I64)]
    L.dic_plan_destroy.argtypes = [P]
    L.dic_plan_destroy.restype = None
    L.dic_status_string.argtypes = [I32]
    L.dic_status_string.restype = ctypes.c_char_p
    L.dic_last_error.argtypes = []
    L.dic_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in ("dic_plan_destroy", "dic_status_string", "dic_last_error"):
            fn.restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int) -> None:
    if rc != 0:
        L = load_library()
        raise DicError(f"{L.dic_status_string(rc).decode()} ({rc}): "
                       f"{L.dic_last_error().decode()}")


def _ptr(t: Optional[torch.Tensor], dtype: torch.dtype, device: torch.device,
         name: str) -> Optional[int]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise DicError(f"{name} must be a CUDA tensor on {device}")
    if t.device != device:
        raise DicError(f"{name} is on {t.device}, plan on {device}")
    if t.dtype != dtype:
        raise DicError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise DicError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def poi_grid(width: int, height: int, M: int, S: int, step: int) -> torch.Tensor:
    """Host POI grid from the library (x0 = m + k step, m = M+S+2), int32 [N, 2]."""
    L = load_library()
    cnt = ctypes.c_int64(0)
    _check(L.dic_poi_grid(width, height, M, S, step, None, 0, ctypes.byref(cnt)))
    out = torch.empty((cnt.value, 2), dtype=torch.int32)
    _check(L.dic_poi_grid(width, height, M, S, step, ctypes.c_void_p(out.data_ptr()),
                          cnt.value, ctypes.byref(cnt)))
    return out


@dataclass
class PairSpec:
    width: int
    height: int
    M: int
    S: int
    ref_offset: int = 0
    def_offset: int = 0
    poi_offset: int = 0
    poi_count: int = 0


class Plan:
    """A bound plan: the library's host plan plus a torch-owned workspace."""

    def __init__(self, pairs: Sequence[PairSpec], precision: int = FP32_BATCHED,
                 max_iters: int = 20, conv_tol: float = 1e-3, flags: int = 0,
                 device: Optional[torch.device] = None, bind: bool = True):
        """``bind=False`` leaves the plan without a workspace (no device
        allocation): only ``correlate_noalloc`` can run it then."""
        self.L = load_library()
        dev = torch.device(device) if device is not None else torch.device("cuda")
        if dev.type != "cuda":
            raise DicError("the library runs on a GPU; device must be cuda")
        self.device = dev if dev.index is not None else torch.device("cuda", torch.cuda.current_device())
        arr = (PairDesc * len(pairs))()
        for k, q in enumerate(pairs):
            arr[k] = PairDesc(q.width, q.height, q.M, q.S, q.ref_offset, q.def_offset,
                              q.poi_offset, q.poi_count)
        desc = PlanDesc(len(pairs), arr, precision, max_iters, conv_tol, flags)
        self._h = ctypes.c_void_p()
        _check(self.L.dic_plan_create(ctypes.byref(desc), ctypes.byref(self._h)))
        self.pairs = list(pairs)
        self.N = sum(q.poi_count for q in pairs)
        self.precision = precision
        self.flags = flags
        nbytes = ctypes.c_size_t(0)
        _check(self.L.dic_plan_workspace_size(self._h, ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self.workspace = None
        if not bind:
            return
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8,
                                         device=self.device)
            _check(self.L.dic_plan_bind(self._h, self.workspace.data_ptr(),
                                        self.workspace.numel(), _stream()))

    # -- lifetime ------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            self.L.dic_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tuning --------------------------------------------------------------
    @property
    def tuning(self) -> Tuple[int, int, int, int]:
        t = Tuning()
        _check(self.L.dic_plan_get_tuning(self._h, ctypes.byref(t)))
        return (t.search_block, t.search_occupancy, t.icgn_waves, t.icgn_slack)

    @tuning.setter
    def tuning(self, v: Tuple[int, int, int, int]) -> None:
        t = Tuning(*v)
        _check(self.L.dic_plan_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, ref: torch.Tensor, defm: torch.Tensor, pois: torch.Tensor) -> Tuple:
        d = self.device
        uv = torch.empty((self.N, 2), dtype=torch.int32, device=d)
        fs = torch.empty(self.N, dtype=torch.float32, device=d)
        is_ = torch.empty(2 * self.N, dtype=torch.int32, device=d)
        ps = torch.empty((self.N, 6), dtype=torch.float64, device=d)
        _check(self.L.dic_plan_autotune(
            self._h, _ptr(ref, torch.float32, d, "ref"), _ptr(defm, torch.float32, d, "def"),
            _ptr(pois, torch.int32, d, "pois"), uv.data_ptr(), fs.data_ptr(), is_.data_ptr(),
            ps.data_ptr(), _stream()))
        return self.tuning

    def invalidate_reference(self) -> None:
        _check(self.L.dic_plan_invalidate_reference(self._h))

    # -- the hot path ----------------------------------------------------------
    def prepare_reference(self, ref: torch.Tensor, pois: torch.Tensor) -> None:
        d = self.device
        _check(self.L.dic_prepare_reference(self._h, _ptr(ref, torch.float32, d, "ref"),
                                            _ptr(pois, torch.int32, d, "pois"), _stream()))

    def prepare_deformed(self, defm: torch.Tensor) -> None:
        _check(self.L.dic_prepare_deformed(self._h, _ptr(defm, torch.float32, self.device, "def"),
                                           _stream()))

    def integer_search(self, ref, defm, pois, seed=None, out=None):
        d, N = self.device, self.N
        uv, zn, st = out if out is not None else (
            torch.empty((N, 2), dtype=torch.int32, device=d),
            torch.empty(N, dtype=torch.float32, device=d),
            torch.empty(N, dtype=torch.int32, device=d))
        _check(self.L.dic_integer_search(
            self._h, _ptr(ref, torch.float32, d, "ref"), _ptr(defm, torch.float32, d, "def"),
            _ptr(pois, torch.int32, d, "pois"), _ptr(seed, torch.int32, d, "seed"),
            _ptr(uv, torch.int32, d, "uv"), _ptr(zn, torch.float32, d, "zncc"),
            _ptr(st, torch.int32, d, "status"), _stream()))
        return uv, zn, st

    def pso_search(self, ref, defm, pois, swarm_random, modified=False, seed=None, out=None):
        """Particle swarm integer search (modified=True: with the star step).
        swarm_random: float32 [N, 5, 50, 4] uniforms in [0, 1).  Returns
        (uv, zncc, status, generations, evaluations)."""
        d, N = self.device, self.N
        if tuple(swarm_random.shape) != (N, PSO_GENERATIONS, PSO_PARTICLES, 4):
            raise DicError(f"swarm_random must have shape {(N, PSO_GENERATIONS, PSO_PARTICLES, 4)}")
        uv, zn, st, gen, ev = out if out is not None else (
            torch.empty((N, 2), dtype=torch.int32, device=d),
            torch.empty(N, dtype=torch.float32, device=d),
            torch.empty(N, dtype=torch.int32, device=d),
            torch.empty(N, dtype=torch.int32, device=d),
            torch.empty(N, dtype=torch.int32, device=d))
        _check(self.L.dic_pso_search(
            self._h, _ptr(ref, torch.float32, d, "ref"), _ptr(defm, torch.float32, d, "def"),
            _ptr(pois, torch.int32, d, "pois"), _ptr(seed, torch.int32, d, "seed"),
            _ptr(swarm_random, torch.float32, d, "swarm_random"), 1 if modified else 0,
            _ptr(uv, torch.int32, d, "uv"), _ptr(zn, torch.float32, d, "zncc"),
            _ptr(st, torch.int32, d, "status"), _ptr(gen, torch.int32, d, "generations"),
            _ptr(ev, torch.int32, d, "evaluations"), _stream()))
        return uv, zn, st, gen, ev

    def icgn_refine(self, ref, defm, pois, uv, status_in=None, p_init=None, out=None):
        return self._refine(self.L.dic_icgn_refine, ref, defm, pois, uv, status_in, p_init, out)

    def nr_refine(self, ref, defm, pois, uv, status_in=None, p_init=None, out=None):
        """Newton-Raphson refinement (same arguments and outputs as icgn_refine)."""
        return self._refine(self.L.dic_nr_refine, ref, defm, pois, uv, status_in, p_init, out)

    def _refine(self, fn, ref, defm, pois, uv, status_in, p_init, out):
        d, N = self.device, self.N
        p, zn, it, st = out if out is not None else (
            torch.empty((N, 6), dtype=torch.float64, device=d),
            torch.empty(N, dtype=torch.float32, device=d),
            torch.empty(N, dtype=torch.int32, device=d),
            torch.empty(N, dtype=torch.int32, device=d))
        _check(fn(
            self._h, _ptr(ref, torch.float32, d, "ref"), _ptr(defm, torch.float32, d, "def"),
            _ptr(pois, torch.int32, d, "pois"), _ptr(uv, torch.int32, d, "uv"),
            _ptr(status_in, torch.int32, d, "status_in"),
            _ptr(p_init, torch.float64, d, "p_init"), _ptr(p, torch.float64, d, "p"),
            _ptr(zn, torch.float32, d, "zncc"), _ptr(it, torch.int32, d, "iters"),
            _ptr(st, torch.int32, d, "status"), _stream()))
        return p, zn, it, st

    def new_outputs(self) -> dict:
        d, N = self.device, self.N
        return dict(uv=torch.empty((N, 2), dtype=torch.int32, device=d),
                    zncc_int=torch.empty(N, dtype=torch.float32, device=d),
                    status_int=torch.empty(N, dtype=torch.int32, device=d),
                    p=torch.empty((N, 6), dtype=torch.float64, device=d),
                    zncc=torch.empty(N, dtype=torch.float32, device=d),
                    iters=torch.empty(N, dtype=torch.int32, device=d),
                    status=torch.empty(N, dtype=torch.int32, device=d))

    def correlate(self, ref, defm, pois, seed=None, p_init=None, out: Optional[dict] = None) -> dict:
        """Search then refine (graph-replayed when the plan has FLAG_USE_GRAPH)."""
        return self._correlate(self.L.dic_correlate, ref, defm, pois, seed, p_init, out)

    def correlate_noalloc(self, ref, defm, pois, seed=None, p_init=None,
                          out: Optional[dict] = None) -> dict:
        """dic_correlate_noalloc: the same call run in the library's static
        device scratch (plans up to 64 MiB of workspace; no binding needed)."""
        return self._correlate(self.L.dic_correlate_noalloc, ref, defm, pois, seed, p_init, out)

    def _correlate(self, fn, ref, defm, pois, seed, p_init, out) -> dict:
        d = self.device
        o = out if out is not None else self.new_outputs()
        _check(fn(
            self._h, _ptr(ref, torch.float32, d, "ref"), _ptr(defm, torch.float32, d, "def"),
            _ptr(pois, torch.int32, d, "pois"), _ptr(seed, torch.int32, d, "seed"),
            _ptr(p_init, torch.float64, d, "p_init"), _ptr(o["uv"], torch.int32, d, "uv"),
            _ptr(o["zncc_int"], torch.float32, d, "zncc_int"),
            _ptr(o["status_int"], torch.int32, d, "status_int"),
            _ptr(o["p"], torch.float64, d, "p"), _ptr(o["zncc"], torch.float32, d, "zncc"),
            _ptr(o["iters"], torch.int32, d, "iters"), _ptr(o["status"], torch.int32, d, "status"),
            _stream()))
        return o

    def znssd(self, ref, defm, pois, p, grad_c=None, c_out=None, grad_p=None, grad_def=None):
        d = self.device
        _check(self.L.dic_znssd_backward(
            self._h, _ptr(ref, torch.float32, d, "ref"), _ptr(defm, torch.float32, d, "def"),
            _ptr(pois, torch.int32, d, "pois"), _ptr(p, torch.float64, d, "p"),
            _ptr(grad_c, torch.float32, d, "grad_c"), _ptr(c_out, torch.float32, d, "c_out"),
            _ptr(grad_p, torch.float64, d, "grad_p"),
            _ptr(grad_def, torch.float32, d, "grad_def"), _stream()))

    def seed_update(self, p, status, seed_uv, p_seed) -> None:
        d = self.device
        _check(self.L.dic_seed_update(
            self._h, _ptr(p, torch.float64, d, "p"), _ptr(status, torch.int32, d, "status"),
            _ptr(seed_uv, torch.int32, d, "seed_uv"), _ptr(p_seed, torch.float64, d, "p_seed"),
            _stream()))


# ---------------------------------------------------------------------------
# convenience front ends
# ---------------------------------------------------------------------------

def single_pair_plan(width: int, height: int, M: int, S: int, n_pois: int,
                     precision: int = FP32_BATCHED, **kw) -> Plan:
    return Plan([PairSpec(width, height, M, S, 0, 0, 0, n_pois)], precision, **kw)


def correlate(ref: torch.Tensor, defm: torch.Tensor, pois: torch.Tensor, M: int, S: int,
              precision: int = FP32_BATCHED, seed=None, p_init=None, **kw) -> dict:
    """Integer search + IC-GN for one pair of [H, W] float32 CUDA images."""
    H, W = ref.shape
    plan = single_pair_plan(W, H, M, S, pois.shape[0], precision, **kw)
    out = plan.correlate(ref, defm, pois, seed, p_init)
    out["plan"] = plan
    return out


def batch_layout(pairs: Sequence[Tuple[torch.Tensor, torch.Tensor, torch.Tensor, int, int]],
                 device) -> Tuple[List[PairSpec], torch.Tensor, torch.Tensor, torch.Tensor]:
    """Packs (ref, def, pois, M, S) tuples into two image arenas and one POI array."""
    specs, refs, defs, pts = [], [], [], []
    roff = doff = poff = 0
    for f, g, q, M, S in pairs:
        H, W = f.shape
        specs.append(PairSpec(W, H, M, S, roff, doff, poff, q.shape[0]))
        refs.append(f.reshape(-1))
        defs.append(g.reshape(-1))
        pts.append(q)
        roff += H * W
        doff += H * W
        poff += q.shape[0]
    ref = torch.cat(refs).to(device).contiguous()
    defm = torch.cat(defs).to(device).contiguous()
    pois = torch.cat(pts).to(device).contiguous()
    return specs, ref, defm, pois


def correlate_batch(pairs, precision: int = FP32_BATCHED, **kw) -> dict:
    """Many independent pairs (mixed sizes and subset radii) in one plan."""
    device = pairs[0][0].device
    specs, ref, defm, pois = batch_layout(pairs, device)
    plan = Plan(specs, precision, **kw)
    out = plan.correlate(ref, defm, pois)
    out.update(plan=plan, ref=ref, defm=defm, pois=pois)
    return out


class _FrameRing:
    """A ring of device frame buffers for the sequence drivers.  Host frames go
    through two pinned staging buffers and are copied on a side stream, so the
    copy of the next frame overlaps the current pair's kernels; a slot is
    overwritten only after the work that last read it (``release``).  Frames
    already on the device as contiguous float32 are used in place unless
    ``copy_device`` (a caller that may reuse its buffer)."""

    def __init__(self, shape, slots: int, device: torch.device, copy_device: bool = False):
        self.shape = tuple(shape)
        self.device = device
        self.copy_device = copy_device
        self.bufs = [torch.empty(self.shape, dtype=torch.float32, device=device)
                     for _ in range(slots)]
        self.pinned = [torch.empty(self.shape, dtype=torch.float32).pin_memory()
                       for _ in range(2)]
        self.copy = torch.cuda.Stream(device=device)
        self.ready = [torch.cuda.Event() for _ in range(slots)]
        self.released = [torch.cuda.Event() for _ in range(slots)]
        self.copied = [torch.cuda.Event() for _ in range(2)]
        for e in self.released + self.copied:
            e.record()
        self.views: List[Optional[torch.Tensor]] = [None] * slots
        self.staged = 0

    def stage(self, slot: int, frame) -> None:
        if (not self.copy_device and isinstance(frame, torch.Tensor)
                and frame.device == self.device and frame.dtype == torch.float32
                and frame.is_contiguous()):
            if tuple(frame.shape) != self.shape:
                raise DicError(f"frame shape {tuple(frame.shape)} != {self.shape}")
            self.views[slot] = frame
            self.ready[slot].record()
            return
        src = torch.as_tensor(frame, dtype=torch.float32)
        if tuple(src.shape) != self.shape:
            raise DicError(f"frame shape {tuple(src.shape)} != {self.shape}")
        if src.device.type == "cuda":
            self.bufs[slot].copy_(src)
            self.ready[slot].record()
        else:
            k = self.staged % 2
            self.copied[k].synchronize()          # the pinned buffer's last copy is done
            self.pinned[k].copy_(src)
            with torch.cuda.stream(self.copy):
                self.copy.wait_event(self.released[slot])
                self.bufs[slot].copy_(self.pinned[k], non_blocking=True)
                self.ready[slot].record(self.copy)
                self.copied[k].record(self.copy)
            self.staged += 1
        self.views[slot] = self.bufs[slot]

    def acquire(self, slot: int) -> torch.Tensor:
        torch.cuda.current_stream().wait_event(self.ready[slot])
        return self.views[slot]

    def release(self, slot: int) -> None:
        self.released[slot].record()


class SequenceCheckpoint:
    """The state a frame sequence carries from one pair to the next, on disk.
    After pair k (frame k against its reference) ``save`` writes
    ``<directory>/frame_<k>.npz`` holding the seeds of the next pair (integer
    displacement and warp of every POI), pair k's warp and statuses, the
    reference policy and the POI count.  A file is written under a temporary
    name and renamed, so one that exists is whole.  To resume after pair k,
    the reference side is prepared again (a deterministic computation) and
    the seeds are read back, so the pairs after k come out bit-identical to an
    uninterrupted run."""

    def __init__(self, directory: str):
        self.directory = directory

    def path(self, k: int) -> str:
        return os.path.join(self.directory, f"frame_{k:06d}.npz")

    def frames(self) -> List[int]:
        """Pairs with a saved state, ascending."""
        if not os.path.isdir(self.directory):
            return []
        out = []
        for name in os.listdir(self.directory):
            if name.startswith("frame_") and name.endswith(".npz"):
                try:
                    out.append(int(name[6:-4]))
                except ValueError:
                    pass
        return sorted(out)

    def save(self, k: int, reference: str, seed, p_seed, p, status) -> None:
        import numpy as np
        os.makedirs(self.directory, exist_ok=True)
        host = {name: (t.detach().cpu().numpy() if isinstance(t, torch.Tensor) else np.asarray(t))
                for name, t in (("seed", seed), ("p_seed", p_seed), ("p", p), ("status", status))}
        tmp = self.path(k) + ".tmp"
        with open(tmp, "wb") as fh:
            np.savez(fh, frame=np.int64(k), reference=np.array(reference),
                     n=np.int64(host["seed"].shape[0]), **host)
        os.replace(tmp, self.path(k))

    def load(self, k: Optional[int] = None) -> Tuple[int, dict]:
        """The state saved after pair k (the latest if None)."""
        import numpy as np
        if k is None:
            have = self.frames()
            if not have:
                raise DicError(f"no sequence checkpoint in {self.directory}")
            k = have[-1]
        if not os.path.exists(self.path(k)):
            raise DicError(f"no sequence checkpoint for pair {k} in {self.directory}")
        with np.load(self.path(k), allow_pickle=False) as z:
            st = {name: z[name] for name in z.files}
        if int(st["frame"]) != k:
            raise DicError(f"checkpoint {self.path(k)} holds pair {int(st['frame'])}")
        return k, st


def correlate_sequence(frames: Sequence, pois: torch.Tensor, M: int, S: int,
                       precision: int = FP32_BATCHED, device=None, reference: str = "first",
                       checkpoint: Optional[str] = None, resume=False,
                       **kw) -> List[dict]:
    """A frame sequence, each pair seeded by the last OK result of its POI
    (search centred on its rounded displacement, refinement starting from its
    gradient terms).

    reference="first": every frame k >= 1 against frame 0, whose reference
    record is computed once.  reference="previous": frame k against frame
    k - 1 (the reference updated after every evaluation, Sec. 3): the POIs
    are the same pixel positions of every reference and each result is the
    increment between the two frames.  Host frames are copied through pinned
    memory on a side stream, one frame ahead of the kernels.

    checkpoint: a directory where the state after every pair is saved
    (SequenceCheckpoint; each save waits for its pair's results).  resume: True (the latest saved pair) or a pair
    index k: continue after pair k from its saved state; the list then holds
    the pairs after k only."""
    if reference not in ("first", "previous"):
        raise DicError("reference must be 'first' or 'previous'")
    if resume is not False and resume is not None and checkpoint is None:
        raise DicError("resume needs a checkpoint directory")
    device = torch.device(device if device is not None else "cuda")
    if device.index is None:
        device = torch.device("cuda", torch.cuda.current_device())
    shape = tuple(torch.as_tensor(frames[0]).shape) if not isinstance(frames[0], torch.Tensor) \
        else tuple(frames[0].shape)
    H, W = shape
    N = pois.shape[0]
    flags = kw.pop("flags", 0)
    # "first": the reference never changes, so its record is cached; "previous":
    # buffers are reused for other frames, so nothing may be cached by pointer
    flags = flags | FLAG_CACHE_REF_PREP if reference == "first" else flags & ~FLAG_CACHE_REF_PREP
    plan = single_pair_plan(W, H, M, S, N, precision, flags=flags, device=device, **kw)
    seed = torch.zeros((N, 2), dtype=torch.int32, device=device)
    p_seed = torch.zeros((N, 6), dtype=torch.float64, device=device)
    ring = _FrameRing(shape, 3, device)
    if reference == "first":
        def slot(k: int) -> int:
            return 0 if k == 0 else 1 + (k - 1) % 2
    else:
        def slot(k: int) -> int:
            return k % 3
    ckpt = SequenceCheckpoint(checkpoint) if checkpoint is not None else None
    start = 1
    if resume is not False and resume is not None:
        k0, st = ckpt.load(None if resume is True else int(resume))
        if str(st["reference"]) != reference or int(st["n"]) != N:
            raise DicError(f"checkpoint of pair {k0} is for reference={str(st['reference'])!r}, "
                           f"{int(st['n'])} POIs, not {reference!r}, {N}")
        if not 1 <= k0 < len(frames):
            raise DicError(f"checkpoint of pair {k0} is outside a sequence of {len(frames)} frames")
        seed.copy_(torch.from_numpy(st["seed"]).to(device))
        p_seed.copy_(torch.from_numpy(st["p_seed"]).to(device))
        start = k0 + 1
    results = []
    out = plan.new_outputs()          # fixed buffers: graph replays keep their key
    r0 = 0 if reference == "first" else start - 1     # the first pair's reference frame
    ring.stage(slot(r0), frames[r0])
    if start < len(frames):
        ring.stage(slot(start), frames[start])
    for k in range(start, len(frames)):
        ref = ring.acquire(slot(0) if reference == "first" else slot(k - 1))
        cur = ring.acquire(slot(k))
        if reference == "first":
            # the deformed frames reuse ring slots, so a pointer comes back with
            # new pixels: its preparation (box sums, interpolation table) is
            # redone here, and only the reference side stays cached
            plan.prepare_deformed(cur)
        o = plan.correlate(ref, cur, pois, seed, p_seed, out=out)
        plan.seed_update(o["p"], o["status"], seed, p_seed)
        if ckpt is not None:
            ckpt.save(k, reference, seed, p_seed, o["p"], o["status"])
        ring.release(slot(k) if reference == "first" else slot(k - 1))
        if k + 1 < len(frames):
            ring.stage(slot(k + 1), frames[k + 1])
        results.append({key: v.clone() for key, v in o.items()})
    return results


class LatestFrame:
    """One-frame mailbox between a camera (producer) and the correlator
    (consumer): ``put`` replaces a frame that was not taken yet (counted in
    ``skipped``), ``take`` returns the newest frame and its sequence number
    and empties the box.  Thread-safe.  The box holds the caller's object, not
    a copy: a frame must stay unchanged until it is taken or replaced."""

    def __init__(self):
        self._lock = threading.Lock()
        self._frame = None
        self._seq = -1
        self._pending = False
        self.received = 0
        self.skipped = 0

    def put(self, frame) -> int:
        with self._lock:
            if self._pending:
                self.skipped += 1
            self._frame = frame
            self._seq += 1
            self._pending = True
            self.received += 1
            return self._seq

    def take(self):
        with self._lock:
            if not self._pending:
                return None, -1
            frame, seq = self._frame, self._seq
            self._frame = None
            self._pending = False
            return frame, seq


class LiveCorrelator:
    """Live pipelining (Sec. 6): each ``step`` correlates the most recent
    frame against the previously used target, which it replaces as the
    reference, so frames that arrive faster than they are processed are
    skipped instead of queued.  The copy of a step's frame to the device runs
    on a side stream and overlaps the previous step's kernels.  A step returns
    None until a reference exists or when no new frame arrived; otherwise the
    pair's outputs (device tensors, not synchronised) with the sequence
    numbers of the frame and its reference.  Seeding as in
    ``correlate_sequence(reference="previous")``."""

    def __init__(self, height: int, width: int, pois: torch.Tensor, M: int, S: int,
                 precision: int = FP32_BATCHED, device=None, **kw):
        device = torch.device(device if device is not None else "cuda")
        if device.index is None:
            device = torch.device("cuda", torch.cuda.current_device())
        flags = kw.pop("flags", 0) & ~(FLAG_CACHE_REF_PREP | FLAG_USE_GRAPH)
        self.pois = pois
        self.plan = single_pair_plan(width, height, M, S, pois.shape[0], precision, flags=flags,
                                     device=device, **kw)
        N = pois.shape[0]
        self.seed = torch.zeros((N, 2), dtype=torch.int32, device=device)
        self.p_seed = torch.zeros((N, 6), dtype=torch.float64, device=device)
        self.ring = _FrameRing((height, width), 3, device, copy_device=True)
        self.mailbox = LatestFrame()
        self.ref_slot: Optional[int] = None
        self.ref_seq = -1
        self.pairs = 0

    def put(self, frame) -> int:
        return self.mailbox.put(frame)

    def step(self) -> Optional[dict]:
        frame, seq = self.mailbox.take()
        if frame is None:
            return None
        slot = 0 if self.ref_slot is None else (self.ref_slot + 1) % 3
        self.ring.stage(slot, frame)
        if self.ref_slot is None:
            self.ref_slot, self.ref_seq = slot, seq
            return None
        ref = self.ring.acquire(self.ref_slot)
        cur = self.ring.acquire(slot)
        o = self.plan.correlate(ref, cur, self.pois, self.seed, self.p_seed)
        self.plan.seed_update(o["p"], o["status"], self.seed, self.p_seed)
        self.ring.release(self.ref_slot)
        o.update(frame=seq, reference=self.ref_seq)
        self.ref_slot, self.ref_seq = slot, seq
        self.pairs += 1
        return o


class ZNSSD(torch.autograd.Function):
    """C[i] = sum over POI i's subset of (fhat - ghat)^2 as a differentiable
    function of the warp parameters p [N, 6] (float64) and the deformed image
    g (float32, the plan's deformed arena)."""

    @staticmethod
    def forward(ctx, p, g, plan: Plan, ref, pois):
        c = torch.empty(plan.N, dtype=torch.float32, device=p.device)
        plan.znssd(ref, g.detach().contiguous(), pois, p.detach().contiguous(), c_out=c)
        ctx.plan = plan
        ctx.save_for_backward(p, g, ref, pois)
        return c

    @staticmethod
    def backward(ctx, grad_c):
        p, g, ref, pois = ctx.saved_tensors
        plan = ctx.plan
        gp = torch.zeros_like(p) if ctx.needs_input_grad[0] else None
        gg = torch.zeros_like(g) if ctx.needs_input_grad[1] else None
        plan.znssd(ref, g.detach().contiguous(), pois, p.detach().contiguous(),
                   grad_c=grad_c.to(torch.float32).contiguous(), grad_p=gp, grad_def=gg)
        return gp, gg, None, None, None
