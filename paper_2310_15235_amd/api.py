"""Python binding of the C ABI in include/trevr2.h (argument marshalling only).

Every step of the computation runs in the HIP library ``libtrevr2.so``; this
module only passes device pointers of torch tensors and the current HIP
stream.  There is no fallback: if the library is missing or no GPU is
present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libtrevr2.so")

# status codes and flags (include/trevr2.h)
OK, E_INVALID, E_CAPACITY, E_HIP, E_STATE, E_DATA = range(6)
THICK_CORR, NEAR_FIELD, BACKGROUND, ABSORPTION_AVG, KEEP_DEPTHS, DIRECTED, COMPLEX_SOURCE = \
    1, 2, 4, 8, 16, 32, 64

EXPORTED = ("trevr_workspace_bytes", "trevr_build_tree", "trevr_compute_J",
            "trevr_compute_J_backward", "trevr_tree_tune",
            "trevr_scratch_needed", "trevr_get_counters", "trevr_check", "trevr_tree_destroy",
            "trevr_tree_info", "trevr_tree_export", "trevr_profile_enable",
            "trevr_profile_read", "trevr_status_string", "trevr_last_error",
            "trevr_forest_workspace_bytes", "trevr_build_forest", "trevr_forest_plan_bytes",
            "trevr_forest_plan", "trevr_forest_scratch_bytes", "trevr_compute_J_batched",
            "trevr_compute_J_backward_batched", "trevr_forest_check",
            "trevr_forest_get_counters", "trevr_forest_scene", "trevr_forest_destroy",
            "trevr_forest_autotune", "trevr_forest_set_config", "trevr_forest_get_config",
            "trevr_compute_J_noalloc", "trevr_forest_profile_enable",
            "trevr_forest_profile_read", "trevr_forest_job_log")
NOALLOC_SCRATCH_BYTES = 64 << 20   # the fixed device array of trevr_compute_J_noalloc
TUNE_STACK, TUNE_CUT, TUNE_STAGE = 0, 1, 2
CONFIGS = 8          # launch configurations of the forest autotuner
PROF_NAMES = ("setup", "walk", "reduce", "near", "adj_reduce", "adj_near", "adj_tree", "pp_src",
              "adj_pp_src")
PROF_SLOTS = len(PROF_NAMES)


class TrevrError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
                ("n_bands", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("theta", ctypes.c_double), ("rpp_min", ctypes.c_double),
                ("box", ctypes.c_double * 4), ("target", ctypes.c_double * 3)]


class Counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("buckets", "cells", "absorber_entries", "source_entries", "segments",
                 "near_pairs", "max_near", "nodes", "src_pairs", "near_src_triples", "max_cut",
                 "max_stack", "near_src_hits", "pp_log_entries")]


_lib = None


def lib():
    """Load libtrevr2.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is missing: build it with "
                               "`python paper_2310_15235_amd/build.py`")
        L = ctypes.CDLL(SO_PATH)
        vp, sz, i64, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int32
        L.trevr_workspace_bytes.argtypes = [ctypes.POINTER(Params), i64, ctypes.POINTER(sz),
                                            ctypes.POINTER(sz)]
        L.trevr_build_tree.argtypes = [ctypes.POINTER(Params), i64] + [vp] * 8 + [sz, vp,
                                                                                   ctypes.POINTER(vp)]
        L.trevr_compute_J.argtypes = [vp, vp, vp, vp, vp, sz, vp]
        L.trevr_compute_J_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.trevr_tree_tune.argtypes = [vp, ctypes.c_int, i64]
        L.trevr_scratch_needed.argtypes = [vp, ctypes.POINTER(sz)]
        L.trevr_get_counters.argtypes = [vp, ctypes.POINTER(Counters)]
        L.trevr_check.argtypes = [vp]
        L.trevr_tree_destroy.argtypes = [vp]
        L.trevr_tree_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                      ctypes.POINTER(i32), vp]
        L.trevr_tree_export.argtypes = [vp] * 12
        L.trevr_profile_enable.argtypes = [vp, ctypes.c_int]
        L.trevr_profile_read.argtypes = [vp, vp, vp]
        L.trevr_forest_workspace_bytes.argtypes = [ctypes.POINTER(Params), i32, vp,
                                                   ctypes.POINTER(sz)]
        L.trevr_build_forest.argtypes = [ctypes.POINTER(Params), i32, vp] + [vp] * 8 + \
            [sz, vp, ctypes.POINTER(vp)]
        L.trevr_forest_plan_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.trevr_forest_plan.argtypes = [vp, vp, sz, vp]
        L.trevr_forest_scratch_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.trevr_compute_J_batched.argtypes = [vp, vp, vp, vp, vp, sz, vp]
        L.trevr_compute_J_backward_batched.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.trevr_forest_check.argtypes = [vp]
        L.trevr_forest_get_counters.argtypes = [vp, i32, ctypes.POINTER(Counters)]
        L.trevr_forest_scene.argtypes = [vp, i32, ctypes.POINTER(vp)]
        L.trevr_forest_destroy.argtypes = [vp]
        L.trevr_forest_autotune.argtypes = [vp] * 9 + [sz, vp, i32, vp]
        L.trevr_forest_set_config.argtypes = [vp, i32]
        L.trevr_forest_get_config.argtypes = [vp, ctypes.POINTER(i32)]
        L.trevr_forest_profile_enable.argtypes = [vp, ctypes.c_int]
        L.trevr_forest_profile_read.argtypes = [vp, vp, vp]
        L.trevr_compute_J_noalloc.argtypes = [vp, vp, vp, vp, vp]
        L.trevr_forest_job_log.argtypes = [vp, sz]
        L.trevr_status_string.restype = ctypes.c_char_p
        L.trevr_status_string.argtypes = [ctypes.c_int]
        L.trevr_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("trevr_status_string", "trevr_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != OK:
        raise TrevrError(status, where, lib().trevr_last_error().decode())


def make_params(nside=2, leaf_size=8, n_bands=1, flags=THICK_CORR | NEAR_FIELD, theta=0.75,
                rpp_min=0.0, box=None, target=None) -> Params:
    p = Params()
    p.nside, p.leaf_size, p.n_bands, p.flags = int(nside), int(leaf_size), int(n_bands), int(flags)
    p.theta, p.rpp_min = float(theta), float(rpp_min)
    b = (0.0, 0.0, 0.0, 0.0) if box is None else box
    for a in range(4):
        p.box[a] = float(b[a])
    for a in range(3):
        p.target[a] = 0.0 if target is None else float(target[a])
    return p


def workspace_bytes(params: Params, n: int):
    tb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().trevr_workspace_bytes(ctypes.byref(params), int(n), ctypes.byref(tb),
                                       ctypes.byref(sb)), "trevr_workspace_bytes")
    return tb.value, sb.value


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


class Tree:
    """A radiation tree built on the GPU; owns its workspace tensor."""

    def __init__(self, x, y, z, m, rho, kappa, lum, *, nside=2, leaf_size=8, theta=0.75,
                 flags=THICK_CORR | NEAR_FIELD, rpp_min=0.0, box=None, scratch=None,
                 target=None):
        """``scratch`` (optional): a uint8 device tensor to use as the
        compute scratch, e.g. ``previous_tree.scratch`` when stepping through
        scenes of similar size; it is replaced by a larger one when a call
        needs more (``self.scratch`` is always the current one)."""
        torch = _torch()
        n = int(x.shape[0])
        B = int(kappa.shape[0])
        self.n, self.B, self.nside = n, B, int(nside)
        self.params = make_params(nside, leaf_size, B, flags, theta, rpp_min, box, target)
        tb, sb = workspace_bytes(self.params, n)
        self.device = x.device
        self.ws = torch.empty(tb, dtype=torch.uint8, device=x.device)
        if scratch is not None and scratch.numel() >= sb:
            self._scratch = scratch
        else:
            self._scratch = torch.empty(sb, dtype=torch.uint8, device=x.device)
        f = torch.float32
        h = ctypes.c_void_p()
        _check(lib().trevr_build_tree(ctypes.byref(self.params), n, _dev(x, f), _dev(y, f),
                                      _dev(z, f), _dev(m, f), _dev(rho, f), _dev(kappa, f),
                                      _dev(lum, f), ctypes.c_void_p(self.ws.data_ptr()), tb,
                                      _stream_ptr(), ctypes.byref(h)), "trevr_build_tree")
        self.handle = h

    @classmethod
    def from_scene(cls, scene, device="cuda", extra_flags=0):
        """The tree of a scene; extra_flags (e.g. KEEP_DEPTHS) are or-ed into
        the scene's own option flags."""
        torch = _torch()
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)
        flags = scene_flags(scene) | int(extra_flags)
        return cls(t(scene.x), t(scene.y), t(scene.z), t(scene.m), t(scene.rho), t(scene.kappa),
                   t(scene.lum), nside=scene.nside, leaf_size=scene.leaf_size, theta=scene.theta,
                   flags=flags, rpp_min=scene.rpp_min, box=scene.box,
                   target=getattr(scene, "directed", None))

    def compute_J(self, active=None, bg=None, out=None):
        """J [B, n] float64 on the device (rows of inactive elements keep
        `out`'s values, zeros by default)."""
        torch = _torch()
        if out is None:
            out = torch.zeros((self.B, self.n), dtype=torch.float64, device=self.device)
        a = None if active is None else _dev(active, torch.uint8)
        g = None if bg is None else _dev(bg, torch.float32)
        self._call_with_scratch(
            lambda sp, sb: lib().trevr_compute_J(self.handle, a, g, _dev(out, torch.float64), sp,
                                                 sb, _stream_ptr()), "trevr_compute_J")
        return out

    def compute_J_noalloc(self, active=None, bg=None, out=None):
        """compute_J through trevr_compute_J_noalloc: the library's fixed
        per-GPU scratch array instead of this tree's scratch tensor."""
        torch = _torch()
        if out is None:
            out = torch.zeros((self.B, self.n), dtype=torch.float64, device=self.device)
        a = None if active is None else _dev(active, torch.uint8)
        g = None if bg is None else _dev(bg, torch.float32)
        _check(lib().trevr_compute_J_noalloc(self.handle, a, g, _dev(out, torch.float64),
                                             _stream_ptr()), "trevr_compute_J_noalloc")
        return out

    def _call_with_scratch(self, fn, where):
        """Run fn(scratch_ptr, scratch_bytes); on TREVR_E_CAPACITY grow the
        scratch to the size the library reports and run once more."""
        torch = _torch()
        for _ in range(2):
            st = fn(ctypes.c_void_p(self._scratch.data_ptr()), self._scratch.numel())
            if st != E_CAPACITY:
                break
            need = ctypes.c_size_t()
            _check(lib().trevr_scratch_needed(self.handle, ctypes.byref(need)),
                   "trevr_scratch_needed")
            if need.value <= self._scratch.numel():
                break
            self._scratch = torch.empty(int(need.value * 1.1) + 4096, dtype=torch.uint8,
                                        device=self.device)
        _check(st, where)

    def compute_J_backward(self, gJ, active=None, bg=None, out=None):
        """Adjoint of compute_J: (dE/dL [B, n], dE/dkappa [B, n], dE/drho [n])
        as float64 device tensors, given gJ = dE/dJ [B, n] float64."""
        torch = _torch()
        if out is None:
            out = (torch.empty((self.B, self.n), dtype=torch.float64, device=self.device),
                   torch.empty((self.B, self.n), dtype=torch.float64, device=self.device),
                   torch.empty((self.n,), dtype=torch.float64, device=self.device))
        gL, gk, gr = out
        a = None if active is None else _dev(active, torch.uint8)
        g = None if bg is None else _dev(bg, torch.float32)
        f64 = torch.float64
        self._call_with_scratch(
            lambda sp, sb: lib().trevr_compute_J_backward(
                self.handle, a, g, _dev(gJ, f64), _dev(gL, f64), _dev(gk, f64), _dev(gr, f64),
                sp, sb, _stream_ptr()), "trevr_compute_J_backward")
        return gL, gk, gr

    @property
    def scratch(self):
        return self._scratch

    def tune(self, key: int, value: int):
        _check(lib().trevr_tree_tune(self.handle, int(key), int(value)), "trevr_tree_tune")

    def check(self):
        _check(lib().trevr_check(self.handle), "trevr_check")

    def counters(self) -> dict:
        c = Counters()
        _check(lib().trevr_get_counters(self.handle, ctypes.byref(c)), "trevr_get_counters")
        return {k: int(getattr(c, k)) for k, _ in Counters._fields_}

    def profile(self, on: bool = True):
        _check(lib().trevr_profile_enable(self.handle, int(on)), "trevr_profile_enable")

    def profile_read(self):
        ms = np.zeros(PROF_SLOTS)
        calls = np.zeros(PROF_SLOTS, np.int64)
        _check(lib().trevr_profile_read(self.handle, ms.ctypes.data_as(ctypes.c_void_p),
                                        calls.ctypes.data_as(ctypes.c_void_p)),
               "trevr_profile_read")
        return {nm: (float(ms[i]), int(calls[i])) for i, nm in enumerate(PROF_NAMES)}

    def info(self):
        nn, nc, dp = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        box = np.zeros(4)
        _check(lib().trevr_tree_info(self.handle, ctypes.byref(nn), ctypes.byref(nc),
                                     ctypes.byref(dp), box.ctypes.data_as(ctypes.c_void_p)),
               "trevr_tree_info")
        return dict(num_nodes=nn.value, num_classes=nc.value, depth=dp.value, root_box=box)

    def export(self) -> dict:
        inf = self.info()
        nn, C, B = inf["num_nodes"], inf["num_classes"], self.B
        perm = np.zeros(self.n, np.int64)
        ints = np.zeros((nn, 7), np.int64)
        box = np.zeros((nn, 6))
        cen = np.zeros((nn, 3))
        Lb = np.zeros((nn, B))
        Lbol = np.zeros(nn)
        alpha = np.zeros((nn, C, B), np.float32)
        K = 12 * self.nside ** 2
        rc = np.zeros(K, np.int32)
        kmass = np.zeros(nn)
        cplx = bool(self.params.flags & COMPLEX_SOURCE)
        cd = np.zeros((nn, K)) if cplx else None
        ca = np.zeros((nn, K, B)) if cplx else None
        p = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().trevr_tree_export(self.handle, p(perm), p(ints), p(box), p(cen), p(Lb),
                                       p(Lbol), p(alpha), p(rc), p(kmass), p(cd), p(ca)),
               "trevr_tree_export")
        return dict(perm=perm, first=ints[:, 0], count=ints[:, 1], lown=ints[:, 2],
                    split=ints[:, 3], child0=ints[:, 4], child1=ints[:, 5], next=ints[:, 6],
                    lo=box[:, :3], hi=box[:, 3:], cen=cen, Lb=Lb, Lbol=Lbol, alpha=alpha,
                    ray_class=rc, kmass=kmass, csrc_d=cd, csrc_a=ca, **inf)

    def close(self):
        if getattr(self, "_owned", True) and getattr(self, "handle", None) is not None and \
                self.handle.value:
            lib().trevr_tree_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def compute_J(scene, active=None, device="cuda"):
    """Build the tree of a scene and return (J as numpy [B, n], counters)."""
    torch = _torch()
    T = Tree.from_scene(scene, device=device)
    act = scene.active if active is None else active
    a = None if act is None else torch.as_tensor(np.ascontiguousarray(act, np.uint8), device=device)
    bg = None
    if scene.background and scene.bg is not None:
        bg = torch.as_tensor(np.ascontiguousarray(scene.bg, np.float32), device=device)
    J = T.compute_J(a, bg)
    T.check()
    out = J.cpu().numpy()
    cnt = T.counters()
    T.close()
    return out, cnt


def compute_J_backward(scene, gJ, active=None, device="cuda", extra_flags=0):
    """Build the tree of a scene, run the adjoint of compute_J for
    gJ = dE/dJ [B, n]; returns numpy (gL [B, n], gkappa [B, n], grho [n])."""
    torch = _torch()
    T = Tree.from_scene(scene, device=device, extra_flags=extra_flags)
    act = scene.active if active is None else active
    a = None if act is None else torch.as_tensor(np.ascontiguousarray(act, np.uint8), device=device)
    bg = None
    if scene.background and scene.bg is not None:
        bg = torch.as_tensor(np.ascontiguousarray(scene.bg, np.float32), device=device)
    g = torch.as_tensor(np.ascontiguousarray(gJ, np.float64), device=device)
    gL, gk, gr = T.compute_J_backward(g, a, bg)
    T.check()
    out = (gL.cpu().numpy(), gk.cpu().numpy(), gr.cpu().numpy())
    T.close()
    return out

def scene_flags(scene) -> int:
    return (THICK_CORR if scene.thick_corr else 0) | (NEAR_FIELD if scene.near_field else 0) | \
        (BACKGROUND if scene.background else 0) | \
        (ABSORPTION_AVG if getattr(scene, "absorption_avg", False) else 0) | \
        (DIRECTED if getattr(scene, "directed", None) is not None else 0) | \
        (COMPLEX_SOURCE if getattr(scene, "complex_source", False) else 0)


class Forest:
    """Independent scenes computed together (trevr_build_forest and the
    batched calls of include/trevr2.h).  Element arrays are concatenated
    over scenes, band arrays as per-scene [B_s, n_s] blocks; ``split``
    cuts such a flat array back into per-scene views.

    Construction builds every scene's tree and plans the forest (sizes of
    every later call); ``compute_J`` and ``compute_J_backward`` then only
    enqueue kernels on torch's current stream, so they can be captured in a
    ``torch.cuda.CUDAGraph``."""

    def __init__(self, scenes, device="cuda"):
        torch = _torch()
        self.device = torch.device(device)
        self.S = len(scenes)
        self.n = [int(s.n) for s in scenes]
        self.B = [int(s.n_bands) for s in scenes]
        self.offsets = np.zeros(self.S + 1, np.int64)
        self.offsets[1:] = np.cumsum(self.n)
        self.boff = np.zeros(self.S + 1, np.int64)
        self.boff[1:] = np.cumsum([b * n for b, n in zip(self.B, self.n)])
        self.bgoff = np.zeros(self.S + 1, np.int64)
        self.bgoff[1:] = np.cumsum(self.B)
        params = (Params * self.S)()
        for i, s in enumerate(scenes):
            params[i] = make_params(s.nside, s.leaf_size, s.n_bands, scene_flags(s), s.theta,
                                    s.rpp_min, s.box, getattr(s, "directed", None))
        self.params = params
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=self.device)
        cat = lambda name: f32(np.concatenate([getattr(s, name) for s in scenes]))
        catb = lambda name: f32(np.concatenate([np.asarray(getattr(s, name)).ravel()
                                                for s in scenes]))
        x, y, z, m, rho = (cat(k) for k in ("x", "y", "z", "m", "rho"))
        kappa, lum = catb("kappa"), catb("lum")
        off_p = self.offsets.ctypes.data_as(ctypes.c_void_p)
        wb = ctypes.c_size_t()
        _check(lib().trevr_forest_workspace_bytes(params, self.S, off_p, ctypes.byref(wb)),
               "trevr_forest_workspace_bytes")
        self.ws = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        f = torch.float32
        _check(lib().trevr_build_forest(params, self.S, off_p, _dev(x, f), _dev(y, f), _dev(z, f),
                                        _dev(m, f), _dev(rho, f), _dev(kappa, f), _dev(lum, f),
                                        ctypes.c_void_p(self.ws.data_ptr()), wb.value,
                                        _stream_ptr(), ctypes.byref(h)), "trevr_build_forest")
        self.handle = h
        pb = ctypes.c_size_t()
        _check(lib().trevr_forest_plan_bytes(h, ctypes.byref(pb)), "trevr_forest_plan_bytes")
        plan_scratch = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
        _check(lib().trevr_forest_plan(h, ctypes.c_void_p(plan_scratch.data_ptr()), pb.value,
                                       _stream_ptr()), "trevr_forest_plan")
        del plan_scratch
        sb = ctypes.c_size_t()
        _check(lib().trevr_forest_scratch_bytes(h, ctypes.byref(sb)), "trevr_forest_scratch_bytes")
        self.scratch = torch.empty(sb.value, dtype=torch.uint8, device=self.device)
        self.job_log_bytes = 0
        self.bg_default = None
        if any(s.background for s in scenes):
            self.bg_default = f32(np.concatenate([
                np.asarray(s.bg if s.bg is not None else np.zeros(s.n_bands), np.float32)
                for s in scenes]))

    def set_job_log(self, nbytes):
        """Size of the p-p job log the forward keeps for the adjoint
        (trevr_forest_job_log; 0 turns it off).  Reallocates the scratch, so
        the next backward recomputes the forward state unless a forward runs
        first."""
        torch = _torch()
        _check(lib().trevr_forest_job_log(self.handle, int(nbytes)), "trevr_forest_job_log")
        sb = ctypes.c_size_t()
        _check(lib().trevr_forest_scratch_bytes(self.handle, ctypes.byref(sb)),
               "trevr_forest_scratch_bytes")
        self.scratch = None
        self.scratch = torch.empty(sb.value, dtype=torch.uint8, device=self.device)
        self.job_log_bytes = int(nbytes)

    def flat_active(self, actives):
        """uint8 device tensor [sum n] from per-scene flags (None = all)."""
        torch = _torch()
        a = np.concatenate([np.ones(n, np.uint8) if v is None else np.asarray(v, np.uint8)
                            for v, n in zip(actives, self.n)])
        return torch.as_tensor(a, device=self.device)

    def split(self, flat):
        """Per-scene [B_s, n_s] views of a band-major flat array, or [n_s]
        views of an element array."""
        if flat.numel() == int(self.boff[-1]):
            return [flat[self.boff[s]:self.boff[s + 1]].view(self.B[s], self.n[s])
                    for s in range(self.S)]
        return [flat[self.offsets[s]:self.offsets[s + 1]] for s in range(self.S)]

    def new_J(self):
        torch = _torch()
        return torch.zeros(int(self.boff[-1]), dtype=torch.float64, device=self.device)

    def compute_J(self, active=None, bg=None, out=None):
        torch = _torch()
        if out is None:
            out = self.new_J()
        bg = self.bg_default if bg is None else bg
        a = None if active is None else _dev(active, torch.uint8)
        g = None if bg is None else _dev(bg, torch.float32)
        _check(lib().trevr_compute_J_batched(self.handle, a, g, _dev(out, torch.float64),
                                             ctypes.c_void_p(self.scratch.data_ptr()),
                                             self.scratch.numel(), _stream_ptr()),
               "trevr_compute_J_batched")
        return out

    def compute_J_backward(self, gJ, active=None, bg=None, out=None):
        torch = _torch()
        f64 = torch.float64
        if out is None:
            out = (torch.empty(int(self.boff[-1]), dtype=f64, device=self.device),
                   torch.empty(int(self.boff[-1]), dtype=f64, device=self.device),
                   torch.empty(int(self.offsets[-1]), dtype=f64, device=self.device))
        gL, gk, gr = out
        bg = self.bg_default if bg is None else bg
        a = None if active is None else _dev(active, torch.uint8)
        g = None if bg is None else _dev(bg, torch.float32)
        _check(lib().trevr_compute_J_backward_batched(
            self.handle, a, g, _dev(gJ, f64), _dev(gL, f64), _dev(gk, f64), _dev(gr, f64),
            ctypes.c_void_p(self.scratch.data_ptr()), self.scratch.numel(), _stream_ptr()),
            "trevr_compute_J_backward_batched")
        return gL, gk, gr

    def autotune(self, active=None, bg=None, gJ=None, reps=2):
        """Time the batched calls under every launch configuration, keep the
        fastest; returns (chosen configuration, ms per candidate)."""
        torch = _torch()
        f64 = torch.float64
        J = self.new_J()
        bg = self.bg_default if bg is None else bg
        a = None if active is None else _dev(active, torch.uint8)
        g = None if bg is None else _dev(bg, torch.float32)
        grads = [None, None, None]
        gj = None
        if gJ is not None:
            gj = _dev(gJ, f64)
            bufs = (torch.empty_like(J), torch.empty_like(J),
                    torch.empty(int(self.offsets[-1]), dtype=f64, device=self.device))
            grads = [_dev(t, f64) for t in bufs]
        times = np.zeros(CONFIGS)
        _check(lib().trevr_forest_autotune(
            self.handle, a, g, _dev(J, f64), gj, grads[0], grads[1], grads[2],
            ctypes.c_void_p(self.scratch.data_ptr()), self.scratch.numel(), _stream_ptr(),
            int(reps), times.ctypes.data_as(ctypes.c_void_p)), "trevr_forest_autotune")
        return self.config(), times

    def config(self) -> int:
        v = ctypes.c_int32()
        _check(lib().trevr_forest_get_config(self.handle, ctypes.byref(v)),
               "trevr_forest_get_config")
        return int(v.value)

    def set_config(self, k: int):
        _check(lib().trevr_forest_set_config(self.handle, int(k)), "trevr_forest_set_config")

    def check(self):
        _check(lib().trevr_forest_check(self.handle), "trevr_forest_check")

    def counters(self, scene=-1) -> dict:
        c = Counters()
        _check(lib().trevr_forest_get_counters(self.handle, int(scene), ctypes.byref(c)),
               "trevr_forest_get_counters")
        return {k: int(getattr(c, k)) for k, _ in Counters._fields_}

    def profile(self, on: bool = True):
        _check(lib().trevr_forest_profile_enable(self.handle, int(on)),
               "trevr_forest_profile_enable")

    def profile_read(self):
        """{phase: (milliseconds, launches)} recorded since profile(True)."""
        ms = np.zeros(PROF_SLOTS)
        calls = np.zeros(PROF_SLOTS, np.int64)
        _check(lib().trevr_forest_profile_read(self.handle, ms.ctypes.data_as(ctypes.c_void_p),
                                               calls.ctypes.data_as(ctypes.c_void_p)),
               "trevr_forest_profile_read")
        return {nm: (float(ms[i]), int(calls[i])) for i, nm in enumerate(PROF_NAMES)}

    def scene_tree(self, s: int) -> "Tree":
        """The tree of scene s as a Tree (owned by the forest) for the
        single-tree calls."""
        torch = _torch()
        h = ctypes.c_void_p()
        _check(lib().trevr_forest_scene(self.handle, int(s), ctypes.byref(h)), "trevr_forest_scene")
        t = Tree.__new__(Tree)
        t.n, t.B, t.nside = self.n[s], self.B[s], int(self.params[s].nside)
        t.params = self.params[s]
        t.device = self.device
        t.ws = self.ws
        t.handle = h
        t._owned = False
        tb, sb = workspace_bytes(self.params[s], self.n[s])
        t._scratch = torch.empty(sb, dtype=torch.uint8, device=self.device)
        return t

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().trevr_forest_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TrevrJ:
    """J as a differentiable torch function of (kappa, lum, rho).

    ``TrevrJ.apply(x, y, z, m, rho, kappa, lum, active, bg, opts)`` builds the
    tree and returns J [B, n] (float64).  The backward pass calls
    trevr_compute_J_backward on the same tree; positions, masses, the active
    set and bg get no gradient.  ``opts`` holds the Tree keyword arguments
    (nside, leaf_size, theta, flags, rpp_min, box)."""

    _fn = None

    @classmethod
    def apply(cls, *args):
        if cls._fn is None:
            torch = _torch()

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, x, y, z, m, rho, kappa, lum, active, bg, opts):
                    T = Tree(x.detach(), y.detach(), z.detach(), m.detach(), rho.detach(),
                             kappa.detach(), lum.detach(), **opts)
                    J = T.compute_J(active, bg)
                    ctx.tree, ctx.active, ctx.bg = T, active, bg
                    ctx.dtypes = (rho.dtype, kappa.dtype, lum.dtype)
                    return J

                @staticmethod
                def backward(ctx, gJ):
                    gL, gk, gr = ctx.tree.compute_J_backward(gJ.contiguous().to(torch.float64),
                                                             ctx.active, ctx.bg)
                    dr, dk, dl = ctx.dtypes
                    return (None, None, None, None, gr.to(dr), gk.to(dk), gL.to(dl), None, None,
                            None)

            cls._fn = _F
        return cls._fn.apply(*args)
