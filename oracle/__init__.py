"""CPU oracle for 3D-BBS (arXiv 2310.10023): Python loader for `bbs_oracle.c`.

TEST INFRASTRUCTURE ONLY.  The oracle is the plain reference that the HIP
library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the library itself
never does, and the two share no code.

Parity pins for each function live in `tests/test_oracle_*.py`: the node
counters and pop order of the search schedule are pinned by hand-traced
instances (`tests/golden/schedule_hand.json`).  The learned prior's trained
weights are the one part with no pin ("parity unpinned": any weights are
valid; only the ordering rules that use them are pinned).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bbs_oracle.c")
# BBS_ORACLE_LIB names another build of this source to load instead (the
# mutation tests load deliberately broken copies this way, in a subprocess)
_LIB_OVERRIDE = os.environ.get("BBS_ORACLE_LIB")
_LIB = _LIB_OVERRIDE or os.path.join(_HERE, "liboracle_bbs.so")

MAX_LEVELS = 16


def compile_source(src: str, out: str) -> str:
    """Compile an oracle source file with gcc (-O2, no FP contraction, no fast math)."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle in place."""
    if _LIB_OVERRIDE:
        return _LIB
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


class Grid(C.Structure):
    _fields_ = [("levels", C.c_int32), ("translation_only", C.c_int32), ("r", C.c_float),
                ("dmax", C.c_double), ("delta", C.c_double * MAX_LEVELS),
                ("n", (C.c_int32 * MAX_LEVELS) * 3), ("dprime", (C.c_double * MAX_LEVELS) * 3),
                ("a", (C.c_int32 * MAX_LEVELS) * 3), ("wmin", C.c_double * 3), ("wmax", C.c_double * 3),
                ("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3), ("tmin", C.c_double * 3), ("tmax", C.c_double * 3),
                ("rot_exact", C.c_int32), ("pad", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("found", C.c_int32), ("score", C.c_int32), ("leaf", C.c_int32 * 6),
                ("pose", C.c_double * 6), ("nodes_expanded", C.c_int64), ("nodes_scored", C.c_int64),
                ("flushes", C.c_int64), ("leaves_accepted", C.c_int64), ("initial_size", C.c_int64),
                ("initial_kept", C.c_int64), ("bound_checks", C.c_int64), ("bound_violations", C.c_int64),
                ("violation_excess_sum", C.c_double), ("prior_used", C.c_int32), ("seeded", C.c_int32),
                ("seed_score", C.c_int32), ("pad", C.c_int32), ("events", C.c_int64)]

    def as_dict(self):
        return {"found": self.found, "score": self.score, "leaf": list(self.leaf),
                "pose": list(self.pose), "nodes_expanded": self.nodes_expanded,
                "nodes_scored": self.nodes_scored, "flushes": self.flushes,
                "leaves_accepted": self.leaves_accepted, "initial_size": self.initial_size,
                "initial_kept": self.initial_kept, "bound_checks": self.bound_checks,
                "bound_violations": self.bound_violations,
                "violation_excess_sum": self.violation_excess_sum, "prior_used": self.prior_used,
                "seeded": self.seeded, "seed_score": self.seed_score}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _LIB_OVERRIDE and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = C.CDLL(_LIB)
        P, I32, I64, F = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        L.orc_build_map.argtypes = [P, I64, F, I32, I32, C.POINTER(P)]
        L.orc_build_map.restype = C.c_int
        L.orc_build_map_margins.argtypes = [P, I64, F, I32, I32, P, C.POINTER(P)]
        L.orc_build_map_margins.restype = C.c_int
        L.orc_map_contains_rot.argtypes = [P, I32, I32, I32, I32]
        L.orc_map_contains_rot.restype = I32
        L.orc_rotation_margins.argtypes = [C.POINTER(Grid), P]
        L.orc_grid_nest.argtypes = [C.POINTER(Grid)]
        L.orc_grid_nest.restype = C.c_int
        L.orc_free_map.argtypes = [P]
        L.orc_map_level_size.argtypes = [P, I32]
        L.orc_map_level_size.restype = I64
        L.orc_map_level_keys.argtypes = [P, I32, P, I64]
        L.orc_map_level_keys.restype = I64
        L.orc_map_contains.argtypes = [P, I32, I32, I32, I32]
        L.orc_map_contains.restype = I32
        L.orc_setup.argtypes = [P, I64, P, P, F, I32, I32, C.POINTER(Grid)]
        L.orc_setup.restype = C.c_int
        L.orc_rotation.argtypes = [C.POINTER(Grid), I32, I32, I32, I32, P]
        L.orc_score.argtypes = [P, P, I64, C.POINTER(Grid), I32, I32, I32, I32, I32, I32, I32]
        L.orc_score.restype = I32
        L.orc_score_nodes.argtypes = [P, P, I64, C.POINTER(Grid), P, I64, P, I32]
        L.orc_localize.argtypes = [P, P, I64, C.POINTER(Grid), I32, I64, I32, I64, C.POINTER(Result), P, I64, P, I32,
                                   P, I64, I32]
        L.orc_localize.restype = C.c_int
        L.orc_bruteforce.argtypes = [P, P, I64, C.POINTER(Grid), I32, I32, C.POINTER(Result)]
        L.orc_bruteforce.restype = C.c_int
        L.orc_all_leaf_scores.argtypes = [P, P, I64, C.POINTER(Grid), P, I64, I32]
        L.orc_all_leaf_scores.restype = I64
        L.orc_children.argtypes = [C.POINTER(Grid), P, P, I64]
        L.orc_children.restype = I64
        L.orc_prior_key.argtypes = [C.POINTER(Grid), P, P]
        L.orc_prior_key.restype = C.c_double
        L.orc_sizeof_grid.restype = I64
        L.orc_sizeof_result.restype = I64
        assert L.orc_sizeof_grid() == C.sizeof(Grid), "oracle Grid layout mismatch"
        assert L.orc_sizeof_result() == C.sizeof(Result), "oracle Result layout mismatch"
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleError(RuntimeError):
    pass


class Map:
    """The dilated multi-resolution voxel sets D_0 .. D_levels (Sec. III-C)."""

    def __init__(self, points, r: float, levels: int, dilate_leaf: bool = True, margins=None):
        """margins: None, or levels + 1 ints ([0] unused); M_l > 0 also builds
        D_l grown by the box [-M_l, M_l]^3, the table of the exact rotational
        bound at level l."""
        pts = _f32(points).reshape(-1, 3)
        h = C.c_void_p()
        mg = None if margins is None else _i32(margins).reshape(-1)
        if mg is not None and len(mg) != int(levels) + 1:
            raise ValueError("margins needs levels + 1 entries")
        rc = lib().orc_build_map_margins(pts.ctypes.data, len(pts), float(r), int(levels), int(dilate_leaf),
                                         None if mg is None else mg.ctypes.data, C.byref(h))
        if rc != 0:
            raise OracleError(f"orc_build_map failed ({rc})")
        self._h = h
        self.r = float(np.float32(r))
        self.levels = int(levels)
        self.margins = [0] * (int(levels) + 1) if mg is None else [int(v) for v in mg]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_free_map(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def level_size(self, l: int) -> int:
        return int(lib().orc_map_level_size(self._h, l))

    def level_keys(self, l: int) -> np.ndarray:
        n = self.level_size(l)
        out = np.zeros((max(n, 1), 3), dtype=np.int32)
        lib().orc_map_level_keys(self._h, l, out.ctypes.data, n)
        return out[:n]

    def contains(self, l: int, x: int, y: int, z: int) -> bool:
        return bool(lib().orc_map_contains(self._h, l, int(x), int(y), int(z)))

    def contains_grown(self, l: int, x: int, y: int, z: int) -> bool:
        """Membership in the grown table of level l >= 1 (rot_margin > 0)."""
        v = lib().orc_map_contains_rot(self._h, l, int(x), int(y), int(z))
        if v < 0:
            raise OracleError("no grown table at this level")
        return bool(v)


class Search:
    """A scan plus its search ranges: the angular/translational grid and the
    oracle's score, branching and search."""

    def __init__(self, omap: Map, scan, rmin, rmax, translation_only: bool = False, rot_exact: bool = False,
                 nested: bool = False):
        """rot_exact: inner nodes are scored against the map's grown tables
        (the exact rotational bound); the map's margins must cover
        margins_needed().  nested: the angular grid is built top down so that
        every cell splits into equal children (orc_grid_nest)."""
        self.map = omap
        self.scan = _f32(scan).reshape(-1, 3)
        self.rmin = _f32(rmin)
        self.rmax = _f32(rmax)
        self.grid = Grid()
        rc = lib().orc_setup(self.scan.ctypes.data, len(self.scan), self.rmin.ctypes.data, self.rmax.ctypes.data,
                             omap.r, omap.levels, int(translation_only), C.byref(self.grid))
        if rc != 0:
            raise OracleError(f"orc_setup failed ({rc})")
        if nested and lib().orc_grid_nest(C.byref(self.grid)) != 0:
            raise OracleError("orc_grid_nest failed")
        self.grid.rot_exact = int(bool(rot_exact))
        if rot_exact and any(e > m for e, m in zip(self.margins_needed(), omap.margins)):
            raise OracleError(f"the map's rotation margins {omap.margins} are below the {self.margins_needed()} "
                              f"this search needs")

    def margins_needed(self) -> list:
        """Per-level box margins e_l of the exact rotational bound ([0] = 0)."""
        out = np.zeros(MAX_LEVELS, dtype=np.int32)
        lib().orc_rotation_margins(C.byref(self.grid), out.ctypes.data)
        return [int(v) for v in out[: self.map.levels + 1]]

    # grid accessors
    @property
    def k(self):
        return len(self.scan)

    def n(self, ax: int, l: int) -> int:
        return int(self.grid.n[ax][l])

    def a(self, ax: int, l: int) -> int:
        return int(self.grid.a[ax][l])

    def delta(self, l: int) -> float:
        return float(self.grid.delta[l])

    def dprime(self, ax: int, l: int) -> float:
        return float(self.grid.dprime[ax][l])

    @property
    def lo(self):
        return tuple(self.grid.lo)

    @property
    def hi(self):
        return tuple(self.grid.hi)

    def rotation(self, level, ia, ib, ig) -> np.ndarray:
        R = np.zeros(9, dtype=np.float32)
        lib().orc_rotation(C.byref(self.grid), level, ia, ib, ig, R.ctypes.data)
        return R.reshape(3, 3)

    def score(self, level, x, y, z, ia, ib, ig) -> int:
        return int(lib().orc_score(self.map.handle, self.scan.ctypes.data, self.k, C.byref(self.grid),
                                   level, x, y, z, ia, ib, ig))

    def score_nodes(self, nodes, threads: int = 1) -> np.ndarray:
        """nodes: (n, 7) int32 rows (level, x, y, z, roll, pitch, yaw)."""
        nodes = _i32(nodes).reshape(-1, 7)
        out = np.zeros(len(nodes), dtype=np.int32)
        lib().orc_score_nodes(self.map.handle, self.scan.ctypes.data, self.k, C.byref(self.grid),
                              nodes.ctypes.data, len(nodes), out.ctypes.data, threads)
        return out

    def children(self, node) -> np.ndarray:
        node = _i32(node)
        cap = 8 * 64 * 8
        out = np.zeros((cap, 7), dtype=np.int32)
        n = lib().orc_children(C.byref(self.grid), node.ctypes.data, out.ctypes.data, cap)
        return out[:n]

    def prior_key(self, prior, node) -> float:
        """Ordering key of a node (level, x, y, z, roll, pitch, yaw) under a
        1088-logit prior: best yaw-bin logit plus best cell logit over the
        leaves below the node."""
        pr = np.ascontiguousarray(prior, dtype=np.float32).reshape(1088)
        nd = _i32(node).reshape(7)
        return float(lib().orc_prior_key(C.byref(self.grid), pr.ctypes.data, nd.ctypes.data))

    EVENT_KINDS = ("prune", "leaf", "branch", "flush")

    STRATEGIES = {"best_first": 0, "depth_first": 1}

    def localize(self, threshold: int, batch: int = 10000, threads: int = 1, max_scored: int = 0,
                 trace_cap: int = 0, prior=None, seed_beam: int = 0, events_cap: int = 0,
                 strategy: str = "best_first") -> dict:
        """Alg. 2 (strategy "best_first"), or the same batched search in the
        queue order of Alg. 1 (strategy "depth_first": deeper levels first,
        then higher score).  prior: optional 1088 float logits (64 yaw bins, then 32 x 32
        translation cells) that order the initial set; a seed beam of width
        `seed_beam` ranked by (score, prior key) may seed the incumbent.
        trace_cap > 0 adds the flush sizes; events_cap > 0 adds the search
        loop's events in order: ("prune" | "leaf" | "branch", node, score) for
        every pop, node = (level, x, y, z, roll, pitch, yaw), and ("flush",
        number of nodes scored)."""
        res = Result()
        tr = np.zeros(max(trace_cap, 1), dtype=np.int64)
        ev = np.zeros((max(events_cap, 1), 9), dtype=np.int32)
        pr = None if prior is None else np.ascontiguousarray(prior, dtype=np.float32).reshape(1088)
        rc = lib().orc_localize(self.map.handle, self.scan.ctypes.data, self.k, C.byref(self.grid), int(threshold),
                                int(batch), int(threads), int(max_scored), C.byref(res),
                                tr.ctypes.data if trace_cap else None, int(trace_cap),
                                pr.ctypes.data if pr is not None else None, int(seed_beam),
                                ev.ctypes.data if events_cap else None, int(events_cap),
                                self.STRATEGIES[strategy])
        if rc != 0:
            raise OracleError(f"orc_localize failed ({rc})")
        d = res.as_dict()
        if trace_cap:
            d["flush_sizes"] = tr[:min(trace_cap, res.flushes)].tolist()
        if events_cap:
            out = []
            for e in ev[:min(events_cap, res.events)].tolist():
                kind = self.EVENT_KINDS[e[0]]
                out.append([kind, e[8]] if kind == "flush" else [kind, e[1:8], e[8]])
            d["events"] = out
            d["events_total"] = int(res.events)
        return d

    def bruteforce(self, threshold: int, threads: int = 1) -> dict:
        res = Result()
        rc = lib().orc_bruteforce(self.map.handle, self.scan.ctypes.data, self.k, C.byref(self.grid),
                                  int(threshold), int(threads), C.byref(res))
        if rc != 0:
            raise OracleError(f"orc_bruteforce failed ({rc})")
        return res.as_dict()

    def all_leaf_scores(self, threads: int = 1) -> np.ndarray:
        """Scores of every valid leaf, shaped (nx, ny, nz, n_roll, n_pitch, n_yaw)."""
        g = self.grid
        shape = tuple(int(g.hi[i] - g.lo[i] + 1) for i in range(3)) + tuple(int(g.n[i][0]) for i in range(3))
        total = int(np.prod(shape))
        out = np.zeros(total, dtype=np.int32)
        lib().orc_all_leaf_scores(self.map.handle, self.scan.ctypes.data, self.k, C.byref(self.grid),
                                  out.ctypes.data, total, threads)
        return out.reshape(shape)
