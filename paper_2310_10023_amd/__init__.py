"""Python binding of libbbs: 3D-BBS batched branch-and-bound scan matching on
AMD Instinct MI355X (gfx950).

Argument marshalling only: every step of the search runs in the HIP library
(`_lib/libbbs.so`, built by `python -m paper_2310_10023_amd.build`).  Inputs may
be numpy arrays (host) or torch tensors on the GPU (device pointers are passed
straight through, with torch's current stream).  There is no CPU fallback:
if the library is missing, importing the library functions raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = ["LibraryMissing", "BbsError", "Map", "Workspace", "localize", "localize_noalloc", "score_nodes", "serve", "lib",
           "library_path", "preprocess_scan", "rotation_margins", "EXPORTED_SYMBOLS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_lib", "libbbs.so")
MAX_LEVELS = 16

EXPORTED_SYMBOLS = (
    "bbs_default_options", "bbs_abi_version", "bbs_last_error", "bbs_build_map", "bbs_free_map", "bbs_map_info",
    "bbs_map_layout", "bbs_map_dump_level", "bbs_map_contains", "bbs_workspace_create", "bbs_workspace_free", "bbs_localize", "bbs_localize_noalloc",
    "bbs_score_nodes", "bbs_serve", "bbs_net_param_count", "bbs_net_create", "bbs_net_free", "bbs_net_set_params",
    "bbs_net_get_params", "bbs_net_forward", "bbs_net_prior", "bbs_net_train_step", "bbs_bev_image", "bbs_autotune",
    "bbs_bandwidth_probe", "bbs_preprocess_scan", "bbs_build_map_margins", "bbs_rotation_margins",
    "bbs_gicp_target_create", "bbs_gicp_target_free", "bbs_gicp_default_options", "bbs_gicp_refine",
    "bbs_gicp_linearize",
)

STRATEGIES = {"best_first": 0, "depth_first": 1}
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "OOM", -3: "DEVICE", -4: "QUEUE_OVERFLOW", -5: "INTERNAL"}


class LibraryMissing(ImportError):
    pass


class BbsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class SearchRange(C.Structure):
    _fields_ = [("min", C.c_float * 6), ("max", C.c_float * 6)]


class Options(C.Structure):
    _fields_ = [("batch_size", C.c_int32), ("translation_only", C.c_int32), ("profile", C.c_int32),
                ("seed_beam", C.c_int32), ("stream", C.c_void_p), ("prior", C.c_void_p),
                ("persistent", C.c_int32), ("score_items", C.c_int32), ("graph", C.c_int32),
                ("hist_min_level", C.c_int32), ("strategy", C.c_int32), ("rot_exact", C.c_int32),
                ("nested_angles", C.c_int32), ("reserved3", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("found", C.c_int32), ("score", C.c_int32), ("leaf", C.c_int32 * 6), ("pose", C.c_float * 6),
                ("nodes_expanded", C.c_int64), ("nodes_scored", C.c_int64), ("flushes", C.c_int64),
                ("leaves_accepted", C.c_int64), ("initial_size", C.c_int64), ("initial_kept", C.c_int64),
                ("score_kernel_ms", C.c_double), ("score_launches", C.c_int64), ("score_pairs", C.c_int64),
                ("score_groups", C.c_int64), ("phase_ms", C.c_double * 4), ("prior_used", C.c_int32),
                ("seeded", C.c_int32), ("seed_score", C.c_int32), ("persistent_used", C.c_int32),
                ("seed_beam_used", C.c_int32), ("reserved_r", C.c_int32), ("serial_ms", C.c_double * 4),
                ("level_groups", C.c_int64 * MAX_LEVELS), ("hist_groups", C.c_int64), ("hist_items", C.c_int64),
                ("hist_fallbacks", C.c_int32), ("hist_off", C.c_int32)]

    def as_dict(self):
        return {"found": self.found, "score": self.score, "leaf": list(self.leaf), "pose": list(self.pose),
                "nodes_expanded": self.nodes_expanded, "nodes_scored": self.nodes_scored, "flushes": self.flushes,
                "leaves_accepted": self.leaves_accepted, "initial_size": self.initial_size,
                "initial_kept": self.initial_kept, "score_kernel_ms": self.score_kernel_ms,
                "score_launches": self.score_launches, "score_pairs": self.score_pairs,
                "score_groups": self.score_groups,
                "phase_ms": list(self.phase_ms), "prior_used": self.prior_used, "seeded": self.seeded,
                "seed_score": self.seed_score, "persistent_used": self.persistent_used,
                "seed_beam_used": self.seed_beam_used, "serial_ms": list(self.serial_ms),
                "level_groups": list(self.level_groups), "hist_groups": self.hist_groups,
                "hist_items": self.hist_items, "hist_fallbacks": self.hist_fallbacks, "hist_off": self.hist_off}


class TuneEntry(C.Structure):
    _fields_ = [("batch_size", C.c_int32), ("score_items", C.c_int32), ("ms", C.c_double)]


class GicpOptions(C.Structure):
    _fields_ = [("max_iterations", C.c_int32), ("min_points", C.c_int32), ("eps_rot", C.c_double),
                ("eps_trans", C.c_double)]


class GicpResult(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("cost", C.c_double), ("pairs", C.c_int64),
                ("iterations", C.c_int32), ("converged", C.c_int32)]


class PreprocessOptions(C.Structure):
    _fields_ = [("gravity", C.c_float * 3), ("leaf", C.c_float), ("target_points", C.c_int64)]


class Query(C.Structure):
    _fields_ = [("scan_xyz", C.c_void_p), ("k", C.c_int64), ("scan_on_device", C.c_int32),
                ("score_threshold", C.c_int32), ("range", SearchRange), ("arrival_s", C.c_double),
                ("prior", C.c_void_p)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded libbbs (raises LibraryMissing if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise LibraryMissing(f"libbbs is not built ({_LIB_PATH}); run python -m paper_2310_10023_amd.build")
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes libbbs bind to that one, so the process holds a single
        # HIP runtime (a second one, loaded first, leaves torch without devices)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(_LIB_PATH)
        P, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        L.bbs_default_options.argtypes = [C.POINTER(Options)]
        L.bbs_abi_version.restype = I32
        L.bbs_last_error.restype = C.c_char_p
        L.bbs_build_map.argtypes = [P, I64, I32, F, I32, I32, P, C.POINTER(P)]
        L.bbs_build_map.restype = C.c_int
        L.bbs_build_map_margins.argtypes = [P, I64, I32, F, I32, I32, P, P, C.POINTER(P)]
        L.bbs_build_map_margins.restype = C.c_int
        L.bbs_rotation_margins.argtypes = [F, I32, C.c_double, C.POINTER(SearchRange), I32, P]
        L.bbs_rotation_margins.restype = C.c_int
        D = C.c_double
        L.bbs_gicp_target_create.argtypes = [P, I64, I32, D, I32, P, C.POINTER(P)]
        L.bbs_gicp_target_create.restype = C.c_int
        L.bbs_gicp_target_free.argtypes = [P]
        L.bbs_gicp_default_options.argtypes = [C.POINTER(GicpOptions)]
        L.bbs_gicp_refine.argtypes = [P, P, I64, I32, P, P, C.POINTER(GicpOptions), P, C.POINTER(GicpResult)]
        L.bbs_gicp_refine.restype = C.c_int
        L.bbs_gicp_linearize.argtypes = [P, P, I64, I32, P, P, I32, P, P, P, C.POINTER(D), C.POINTER(I64)]
        L.bbs_gicp_linearize.restype = C.c_int
        L.bbs_free_map.argtypes = [P]
        L.bbs_map_info.argtypes = [P, C.POINTER(I32), C.POINTER(F), P, P, P]
        L.bbs_map_info.restype = C.c_int
        L.bbs_map_layout.argtypes = [P, I32, C.POINTER(I32), C.POINTER(I64)]
        L.bbs_map_layout.restype = C.c_int
        L.bbs_map_dump_level.argtypes = [P, I32, P, I64, C.POINTER(I64)]
        L.bbs_map_dump_level.restype = C.c_int
        L.bbs_map_contains.argtypes = [P, I32, P, I64, P]
        L.bbs_map_contains.restype = C.c_int
        L.bbs_workspace_create.argtypes = [I64, C.POINTER(P)]
        L.bbs_workspace_create.restype = C.c_int
        L.bbs_workspace_free.argtypes = [P]
        L.bbs_localize.argtypes = [P, P, P, I64, I32, C.POINTER(SearchRange), I32, C.POINTER(Options),
                                   C.POINTER(Result)]
        L.bbs_localize.restype = C.c_int
        L.bbs_localize_noalloc.argtypes = [P, P, I64, I32, C.POINTER(SearchRange), I32, C.POINTER(Options),
                                           C.POINTER(Result)]
        L.bbs_localize_noalloc.restype = C.c_int
        L.bbs_score_nodes.argtypes = [P, P, I64, C.POINTER(SearchRange), I32, P, I64, P]
        L.bbs_score_nodes.restype = C.c_int
        L.bbs_serve.argtypes = [P, C.POINTER(Query), I64, I32, C.POINTER(Options), C.POINTER(Result), P, P]
        L.bbs_serve.restype = C.c_int
        L.bbs_autotune.argtypes = [P, C.POINTER(Query), I64, P, I32, P, I32, C.POINTER(Options),
                                   C.POINTER(TuneEntry), P]
        L.bbs_autotune.restype = C.c_int
        L.bbs_bandwidth_probe.argtypes = [I32, I64, I64, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.bbs_bandwidth_probe.restype = C.c_int
        L.bbs_preprocess_scan.argtypes = [P, I64, I32, C.POINTER(PreprocessOptions), P, I64, C.POINTER(I64),
                                          C.POINTER(F), P]
        L.bbs_preprocess_scan.restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise BbsError(rc, lib().bbs_last_error().decode())


def _points(x, name):
    """(pointer, count, on_device, keepalive) of an n x 3 float32 point array."""
    try:
        import torch
        if isinstance(x, torch.Tensor):
            if x.dtype != torch.float32 or x.dim() != 2 or x.shape[1] != 3:
                raise ValueError(f"{name} must be an (n, 3) float32 tensor")
            if x.is_cuda:
                x = x.contiguous()
                return x.data_ptr(), x.shape[0], 1, x
            x = x.numpy()
    except ImportError:
        pass
    a = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)
    return a.ctypes.data, a.shape[0], 0, a


def _stream(stream):
    if stream is not None:
        return stream
    try:
        import torch
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            return torch.cuda.current_stream().cuda_stream
    except ImportError:
        pass
    return None


def _range(rmin, rmax):
    r = SearchRange()
    lo = np.asarray(rmin, dtype=np.float32).reshape(6)
    hi = np.asarray(rmax, dtype=np.float32).reshape(6)
    for i in range(6):
        r.min[i] = float(lo[i])
        r.max[i] = float(hi[i])
    return r


class Map:
    """Sparse multi-resolution voxel map (Sec. III-C) resident on the GPU."""

    def __init__(self, points, min_res: float, levels: int, dilate_leaf: bool = True, stream=None, margins=None):
        """margins: None, or levels + 1 box margins of the grown tables that the
        exact rotational bound (localize(rot_exact=True)) reads; see
        rotation_margins()."""
        ptr, n, dev, keep = _points(points, "points")
        h = C.c_void_p()
        mg = None if margins is None else np.ascontiguousarray(margins, dtype=np.int32).reshape(-1)
        if mg is not None and len(mg) != int(levels) + 1:
            raise ValueError("margins needs levels + 1 entries")
        _check(lib().bbs_build_map_margins(ptr, n, dev, float(min_res), int(levels), int(dilate_leaf),
                                           None if mg is None else mg.ctypes.data, _stream(stream), C.byref(h)))
        del keep
        self.margins = [0] * (int(levels) + 1) if mg is None else [int(v) for v in mg]
        self._h = h
        self.min_res = float(np.float32(min_res))
        self.levels = int(levels)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().bbs_free_map(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        lv = C.c_int32()
        r = C.c_float()
        vox = np.zeros(MAX_LEVELS, np.int64)
        slots = np.zeros(MAX_LEVELS, np.int64)
        bricks = np.zeros(MAX_LEVELS, np.int64)
        _check(lib().bbs_map_info(self._h, C.byref(lv), C.byref(r), vox.ctypes.data, slots.ctypes.data,
                                  bricks.ctypes.data))
        n = lv.value + 1
        dense, dense_n = [], []
        for l in range(n):
            d = C.c_int32()
            e = C.c_int64()
            _check(lib().bbs_map_layout(self._h, l, C.byref(d), C.byref(e)))
            dense.append(bool(d.value))
            dense_n.append(e.value)
        return {"levels": lv.value, "min_res": r.value, "voxels": vox[:n].tolist(), "slots": slots[:n].tolist(),
                "bricks": bricks[:n].tolist(), "dense": dense, "dense_entries": dense_n}

    def dump_level(self, level: int) -> np.ndarray:
        """Voxels of D_level as an (m, 3) int32 array, sorted lexicographically."""
        cnt = C.c_int64()
        _check(lib().bbs_map_dump_level(self._h, level, None, 0, C.byref(cnt)))
        out = np.zeros((max(cnt.value, 1), 3), np.int32)
        _check(lib().bbs_map_dump_level(self._h, level, out.ctypes.data, cnt.value, C.byref(cnt)))
        out = out[:cnt.value]
        return out[np.lexsort((out[:, 2], out[:, 1], out[:, 0]))]

    def contains(self, level: int, voxels) -> np.ndarray:
        v = np.ascontiguousarray(voxels, dtype=np.int32).reshape(-1, 3)
        out = np.zeros(len(v), np.uint8)
        _check(lib().bbs_map_contains(self._h, level, v.ctypes.data, len(v), out.ctypes.data))
        return out.astype(bool)


class Workspace:
    """Device node queue and buffers for one search at a time."""

    def __init__(self, max_queue_nodes: int = 0):
        h = C.c_void_p()
        _check(lib().bbs_workspace_create(int(max_queue_nodes), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().bbs_workspace_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def localize(bmap: Map, scan, rmin, rmax, score_threshold: int, *, batch_size: int = 10000,
             translation_only: bool = False, profile: int = 0, workspace: Workspace | None = None,
             stream=None, prior=None, seed_beam: int = 0, persistent: bool = False,
             score_items: int = 0, graph: bool = False, hist_min_level: int = 0,
             strategy: str = "best_first", rot_exact: bool = False, nested_angles: bool = False) -> dict:
    """Global localization of one scan (Alg. 2 on the GPU).  Returns the result
    fields as a dict (found, score, leaf, pose, node counters, timings).
    prior: optional 1088 logits of the proposal network."""
    ptr, k, dev, keep = _points(scan, "scan")
    opt = Options()
    lib().bbs_default_options(C.byref(opt))
    opt.batch_size = int(batch_size)
    opt.translation_only = int(translation_only)
    opt.profile = int(profile)
    opt.seed_beam = int(seed_beam)
    opt.persistent = int(persistent)
    opt.score_items = int(score_items)
    opt.graph = int(graph)
    opt.hist_min_level = int(hist_min_level)
    opt.strategy = STRATEGIES[strategy]
    opt.rot_exact = int(rot_exact)
    opt.nested_angles = int(nested_angles)
    pr = None
    if prior is not None:
        pr = np.ascontiguousarray(prior, dtype=np.float32).reshape(1088)
        opt.prior = pr.ctypes.data
    st = _stream(stream)
    opt.stream = st
    rng = _range(rmin, rmax)
    res = Result()
    _check(lib().bbs_localize(bmap.handle, workspace.handle if workspace else None, ptr, k, dev, C.byref(rng),
                              int(score_threshold), C.byref(opt), C.byref(res)))
    del keep, pr
    return res.as_dict()


def localize_noalloc(bmap: Map, scan, rmin, rmax, score_threshold: int, *, batch_size: int = 10000,
                     translation_only: bool = False, stream=None, prior=None, seed_beam: int = 0,
                     persistent: bool = False, score_items: int = 0) -> dict:
    """localize() through bbs_localize_noalloc: no device allocation, every
    buffer comes from the library's static per-GPU scratch."""
    ptr, k, dev, keep = _points(scan, "scan")
    opt = Options()
    lib().bbs_default_options(C.byref(opt))
    opt.batch_size = int(batch_size)
    opt.translation_only = int(translation_only)
    opt.seed_beam = int(seed_beam)
    opt.persistent = int(persistent)
    opt.score_items = int(score_items)
    pr = None
    if prior is not None:
        pr = np.ascontiguousarray(prior, dtype=np.float32).reshape(1088)
        opt.prior = pr.ctypes.data
    opt.stream = _stream(stream)
    rng = _range(rmin, rmax)
    res = Result()
    _check(lib().bbs_localize_noalloc(bmap.handle, ptr, k, dev, C.byref(rng), int(score_threshold), C.byref(opt),
                                      C.byref(res)))
    del keep, pr
    return res.as_dict()


def score_nodes(bmap: Map, scan, rmin, rmax, nodes, translation_only: bool = False,
                rot_exact: bool = False, nested_angles: bool = False) -> np.ndarray:
    """Scores of arbitrary nodes (rows level, x, y, z, i_roll, i_pitch, i_yaw)
    computed by the device scoring kernel."""
    s = np.ascontiguousarray(scan, dtype=np.float32).reshape(-1, 3)
    nd = np.ascontiguousarray(nodes, dtype=np.int32).reshape(-1, 7)
    out = np.zeros(len(nd), np.int32)
    rng = _range(rmin, rmax)
    _check(lib().bbs_score_nodes(bmap.handle, s.ctypes.data, len(s), C.byref(rng),
                                 int(bool(translation_only)) | (2 if rot_exact else 0) | (4 if nested_angles else 0),
                                 nd.ctypes.data, len(nd), out.ctypes.data))
    return out


def _queries(scans, ranges, thresholds, arrivals, priors=None):
    n = len(scans)
    qs = (Query * max(n, 1))()
    keep = []
    for i in range(n):
        ptr, k, dev, kp = _points(scans[i], "scan")
        keep.append(kp)
        if priors is not None and priors[i] is not None:
            pr = np.ascontiguousarray(priors[i], np.float32).reshape(1088)
            keep.append(pr)
            qs[i].prior = pr.ctypes.data
        qs[i].scan_xyz = ptr
        qs[i].k = k
        qs[i].scan_on_device = dev
        qs[i].score_threshold = int(thresholds[i])
        qs[i].range = _range(*ranges[i])
        qs[i].arrival_s = float(arrivals[i])
    return qs, keep


def autotune(bmap: Map, scans, rmin, rmax, thresholds, batch_sizes, score_items, *, persistent: bool = False,
             prior=None, seed_beam: int = 0):
    """Fastest (batch_size, score_items) on the sample scans; returns
    (best dict, list of all measured entries)."""
    qs, keep = _queries(scans, [(rmin, rmax)] * len(scans), thresholds, [0.0] * len(scans))
    bs = np.ascontiguousarray(batch_sizes, np.int32)
    it = np.ascontiguousarray(score_items, np.int32)
    opt = Options()
    lib().bbs_default_options(C.byref(opt))
    opt.persistent = int(persistent)
    pr = None
    if prior is not None:
        pr = np.ascontiguousarray(prior, np.float32).reshape(1088)
        opt.prior = pr.ctypes.data
        opt.seed_beam = int(seed_beam)
    best = TuneEntry()
    allv = (TuneEntry * (len(bs) * len(it)))()
    _check(lib().bbs_autotune(bmap.handle, qs, len(scans), bs.ctypes.data, len(bs), it.ctypes.data, len(it),
                              C.byref(opt), C.byref(best), allv))
    del keep, pr
    conv = lambda e: {"batch_size": e.batch_size, "score_items": e.score_items, "ms": e.ms}
    return conv(best), [conv(e) for e in allv]


def serve(bmap: Map, scans, ranges, thresholds, arrivals, *, workers: int = 4, batch_size: int = 10000,
          translation_only: bool = False, persistent: bool = False, priors=None,
          seed_beam: int = 0) -> tuple[list, "np.ndarray", "np.ndarray"]:
    """Serve a stream of queries (sorted by arrival time, seconds from the
    start) with `workers` concurrent searches.  priors: optional per-query
    1088 proposal logits (None entries run plain).  Returns (results,
    start_s, end_s)."""
    n = len(scans)
    qs, keep = _queries(scans, ranges, thresholds, arrivals, priors)
    opt = Options()
    lib().bbs_default_options(C.byref(opt))
    opt.batch_size = int(batch_size)
    opt.translation_only = int(translation_only)
    opt.persistent = int(persistent)
    opt.seed_beam = int(seed_beam)
    res = (Result * max(n, 1))()
    t_start = np.zeros(max(n, 1), np.float64)
    t_end = np.zeros(max(n, 1), np.float64)
    _check(lib().bbs_serve(bmap.handle, qs, n, int(workers), C.byref(opt), res, t_start.ctypes.data,
                           t_end.ctypes.data))
    del keep
    return [res[i].as_dict() for i in range(n)], t_start[:n], t_end[:n]


def bandwidth_probe(kind: str, table_bytes: int, loads: int = 1 << 26) -> dict:
    """Achievable memory rate of the GPU: kind "stream" (coalesced read of the
    whole table) or "gather" (random 8-byte loads into the table).  Returns
    {"gbs": useful GB/s, "ms": kernel time, "table_bytes": ...}."""
    gbs, ms = C.c_double(), C.c_double()
    k = {"stream": 0, "gather": 1}[kind]
    _check(lib().bbs_bandwidth_probe(k, int(table_bytes), int(loads), C.byref(gbs), C.byref(ms)))
    return {"kind": kind, "gbs": gbs.value, "ms": ms.value, "table_bytes": int(table_bytes),
            "loads": int(loads) if k == 1 else None}


def preprocess_scan(points, gravity=None, leaf: float = 0.0, target_points: int = 0, stream=None):
    """Gravity alignment and voxel-grid filter of one scan (bbs_preprocess_scan).
    `points`: an (n, 3) float32 numpy array or device tensor; the result is
    of the same kind.  Returns (points, leaf used or 0.0)."""
    ptr, n, dev, keep = _points(points, "points")
    opt = PreprocessOptions()
    if gravity is not None:
        for i, v in enumerate(np.asarray(gravity, np.float32).reshape(3)):
            opt.gravity[i] = float(v)
    opt.leaf = float(leaf)
    opt.target_points = int(target_points)
    out_n, used = C.c_int64(), C.c_float()
    if dev:
        import torch
        out = torch.empty((max(n, 1), 3), dtype=torch.float32, device=keep.device)
        optr = out.data_ptr()
    else:
        out = np.empty((max(n, 1), 3), np.float32)
        optr = out.ctypes.data
    _check(lib().bbs_preprocess_scan(ptr, n, dev, C.byref(opt), optr, n, C.byref(out_n), C.byref(used),
                                      C.c_void_p(_stream(stream))))
    del keep
    return out[:out_n.value], float(used.value)


def rotation_margins(min_res: float, levels: int, d_max: float, rmin, rmax, nested_angles: bool = False) -> list:
    """Box margins e_l ([0] = 0) that the exact rotational bound needs for
    scans of largest range d_max over the search range (bbs_rotation_margins)."""
    out = np.zeros(int(levels) + 1, np.int32)
    rng = _range(rmin, rmax)
    _check(lib().bbs_rotation_margins(float(min_res), int(levels), float(d_max), C.byref(rng), int(nested_angles),
                                      out.ctypes.data))
    return [int(v) for v in out]


class GicpTarget:
    """The voxel distributions of a map for pose refinement (bbs_gicp_target_create)."""

    def __init__(self, points, voxel: float = 1.0, min_points: int = 5, stream=None):
        ptr, n, dev, keep = _points(points, "points")
        h = C.c_void_p()
        _check(lib().bbs_gicp_target_create(ptr, n, dev, float(voxel), int(min_points), _stream(stream),
                                            C.byref(h)))
        del keep
        self._h = h
        self.voxel = float(voxel)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().bbs_gicp_target_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refine(self, scan, R0, t0, max_iterations: int = 20, min_points: int = 5, eps_rot: float = 1e-6,
               eps_trans: float = 1e-5, stream=None):
        """GICP from (R0, t0): returns (R 3x3, t 3, info dict)."""
        ptr, k, dev, keep = _points(scan, "scan")
        opt = GicpOptions()
        lib().bbs_gicp_default_options(C.byref(opt))
        opt.max_iterations, opt.min_points = int(max_iterations), int(min_points)
        opt.eps_rot, opt.eps_trans = float(eps_rot), float(eps_trans)
        R = np.ascontiguousarray(R0, np.float64).reshape(9)
        t = np.ascontiguousarray(t0, np.float64).reshape(3)
        res = GicpResult()
        _check(lib().bbs_gicp_refine(self._h, ptr, k, dev, R.ctypes.data, t.ctypes.data, C.byref(opt),
                                     _stream(stream), C.byref(res)))
        del keep
        return (np.array(res.R).reshape(3, 3), np.array(res.t),
                {"cost": res.cost, "pairs": res.pairs, "iterations": res.iterations,
                 "converged": bool(res.converged)})

    def linearize(self, scan, R, t, min_points: int = 5, stream=None):
        """(H 6x6, g 6, cost, pairs) of one Gauss-Newton step at (R, t)."""
        ptr, k, dev, keep = _points(scan, "scan")
        Rr = np.ascontiguousarray(R, np.float64).reshape(9)
        tt = np.ascontiguousarray(t, np.float64).reshape(3)
        H = np.zeros(36)
        g = np.zeros(6)
        cost, pairs = C.c_double(), C.c_int64()
        _check(lib().bbs_gicp_linearize(self._h, ptr, k, dev, Rr.ctypes.data, tt.ctypes.data, int(min_points),
                                        _stream(stream), H.ctypes.data, g.ctypes.data, C.byref(cost),
                                        C.byref(pairs)))
        del keep
        return H.reshape(6, 6), g, cost.value, pairs.value
