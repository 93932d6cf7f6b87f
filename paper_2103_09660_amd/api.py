"""Python binding of the HyperNetVec refinement library (include/hnv.h).

Every function here marshals arguments into one C-ABI call; the refinement
itself (projection, sweeps, residuals, reverse sweeps, reciprocals, casts)
runs in the library's HIP kernels.  PyTorch provides device memory and the
current HIP stream.  The hierarchy (coarsening, Section 3.1) is built by the
library either on the host (C++) or on the GPU (HIP), with identical maps.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L


def abi_version() -> int:
    return int(L.lib().hnv_abi_version())


def last_error() -> str:
    return L.last_error()


# ----------------------------------------------------------------------------
# host hierarchy
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class HostLevel:
    n_nodes: int
    n_edges: int
    edge_ptr: np.ndarray              # int64 [n_edges+1]  CSR: hyperedge -> members
    edge_idx: np.ndarray              # int32 [nnz]
    edge_w: Optional[np.ndarray]      # float32 [n_edges] or None
    node_ptr: Optional[np.ndarray] = None   # int64 [n_nodes+1]  CSC: node -> hyperedges, or None
    node_idx: Optional[np.ndarray] = None   # int32 [nnz]

    def __post_init__(self):
        self.edge_ptr = np.ascontiguousarray(self.edge_ptr, dtype=np.int64)
        self.edge_idx = np.ascontiguousarray(self.edge_idx, dtype=np.int32)
        if self.edge_w is not None:
            self.edge_w = np.ascontiguousarray(self.edge_w, dtype=np.float32)
        if self.node_ptr is not None:
            self.node_ptr = np.ascontiguousarray(self.node_ptr, dtype=np.int64)
        if self.node_idx is not None:
            self.node_idx = np.ascontiguousarray(self.node_idx, dtype=np.int32)

    @property
    def nnz(self) -> int:
        return int(self.edge_ptr[-1])

    @property
    def rows(self) -> int:
        return self.n_nodes + self.n_edges

    def c(self) -> L.HnvLevel:
        return L.HnvLevel(self.n_nodes, self.n_edges, self.nnz,
                          self.edge_ptr.ctypes.data_as(L.i64p), self.edge_idx.ctypes.data_as(L.i32p),
                          None if self.edge_w is None else self.edge_w.ctypes.data_as(L.f32p),
                          None if self.node_ptr is None else self.node_ptr.ctypes.data_as(L.i64p),
                          None if self.node_idx is None else self.node_idx.ctypes.data_as(L.i32p))


@dataclasses.dataclass
class HostMap:
    node_rep: np.ndarray   # int32 [n_nodes of the finer level]
    edge_rep: np.ndarray   # int32 [n_edges of the finer level], -1 = removed

    def c(self) -> L.HnvMap:
        return L.HnvMap(self.node_rep.ctypes.data_as(L.i32p), self.edge_rep.ctypes.data_as(L.i32p))


def validate_level(level: HostLevel) -> None:
    lv = level.c()
    L.call("hnv_validate_level", ctypes.byref(lv))


def coarsen_level(level: HostLevel):
    """One featureless coarsening step (library C++): returns (HostMap, coarse HostLevel)."""
    nnz = level.nnz
    node_rep = np.empty(max(level.n_nodes, 1), dtype=np.int32)
    edge_rep = np.empty(max(level.n_edges, 1), dtype=np.int32)
    c_ptr = np.empty(level.n_edges + 1, dtype=np.int64)
    c_idx = np.empty(max(nnz, 1), dtype=np.int32)
    c_w = None if level.edge_w is None else np.empty(max(level.n_edges, 1), dtype=np.float32)
    nv, ne, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    lv = level.c()
    L.call("hnv_coarsen_level", ctypes.byref(lv), node_rep.ctypes.data_as(L.i32p), edge_rep.ctypes.data_as(L.i32p),
           c_ptr.ctypes.data_as(L.i64p), c_idx.ctypes.data_as(L.i32p),
           None if c_w is None else c_w.ctypes.data_as(L.f32p), ctypes.byref(nv), ctypes.byref(ne), ctypes.byref(nz))
    coarse = HostLevel(nv.value, ne.value, c_ptr[: ne.value + 1].copy(), c_idx[: nz.value].copy(),
                       None if c_w is None else c_w[: ne.value].copy())
    return HostMap(node_rep[: level.n_nodes].copy(), edge_rep[: level.n_edges].copy()), coarse


@dataclasses.dataclass
class DeviceLevel:
    """A level in device memory: int32 offsets and members, float32 weights
    or None (torch tensors on one GPU)."""
    n_nodes: int
    n_edges: int
    nnz: int
    edge_ptr: "object"                # torch.int32 [n_edges+1]
    edge_idx: "object"                # torch.int32 [nnz]
    edge_w: "object" = None           # torch.float32 [n_edges] or None

    @classmethod
    def from_host(cls, level: HostLevel, device=None) -> "DeviceLevel":
        torch = _torch()
        dev = torch.device("cuda") if device is None else torch.device(device)
        return cls(level.n_nodes, level.n_edges, level.nnz,
                   torch.as_tensor(level.edge_ptr.astype(np.int32)).to(dev),
                   torch.as_tensor(level.edge_idx).to(dev),
                   None if level.edge_w is None else torch.as_tensor(level.edge_w).to(dev))

    def check(self):
        """Types, sizes and placement of the arrays (their contents are
        checked by the library on the device)."""
        torch = _torch()
        dev = self.edge_ptr.device
        for t, dt, n, name in ((self.edge_ptr, torch.int32, self.n_edges + 1, "edge_ptr"),
                               (self.edge_idx, torch.int32, self.nnz, "edge_idx"),
                               (self.edge_w, torch.float32, self.n_edges, "edge_w")):
            if t is not None and (t.dtype != dt or not t.is_contiguous() or t.device != dev or t.numel() < n
                                  or dev.type != "cuda"):
                raise ValueError(f"{name}: expected a contiguous {dt} GPU tensor of at least {n} elements on "
                                 f"{dev}, got {t.dtype} {tuple(t.shape)} on {t.device}")
        if min(self.n_nodes, self.n_edges, self.nnz) < 0:
            raise ValueError("negative size")

    def to_host(self) -> HostLevel:
        return HostLevel(self.n_nodes, self.n_edges, self.edge_ptr.cpu().numpy().astype(np.int64),
                         self.edge_idx.cpu().numpy(), None if self.edge_w is None else self.edge_w.cpu().numpy())


def coarsen_workspace_bytes(n_nodes: int, n_edges: int, nnz: int) -> int:
    out = ctypes.c_size_t()
    L.call("hnv_coarsen_workspace_bytes", n_nodes, n_edges, nnz, ctypes.byref(out))
    return int(out.value)


def coarsen_level_device(level: DeviceLevel, workspace=None):
    """One featureless coarsening step on the GPU (library HIP): returns
    (node_rep, edge_rep, coarse DeviceLevel), all on the level's device.
    The call waits for the coarse sizes; ``workspace`` (a uint8 tensor of at
    least :func:`coarsen_workspace_bytes`) may be reused between calls."""
    torch = _torch()
    level.check()
    need = coarsen_workspace_bytes(level.n_nodes, level.n_edges, level.nnz)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=level.edge_ptr.device)
    return _coarsen_step(level, workspace)


def _coarsen_step(level: DeviceLevel, workspace):
    """coarsen_level_device with a workspace taken as is (the library
    returns HNV_EWORKSPACE if it is too small)."""
    torch = _torch()
    dev = level.edge_ptr.device
    # the four int32 outputs carved from one allocation, each on a 256-byte boundary
    lens = (max(level.n_nodes, 1), max(level.n_edges, 1), level.n_edges + 1, max(level.nnz, 1))
    offs = [0]
    for n in lens:
        offs.append(offs[-1] + (n + 63) // 64 * 64)
    block = torch.empty(offs[-1], dtype=torch.int32, device=dev)
    node_rep, edge_rep, c_ptr, c_idx = (block[o:o + n] for o, n in zip(offs, lens))
    c_w = None if level.edge_w is None else torch.empty(max(level.n_edges, 1), dtype=torch.float32, device=dev)
    sizes = (ctypes.c_int64 * 3)()
    with torch.cuda.device(dev):
        L.call("hnv_coarsen_level_device", level.n_nodes, level.n_edges, level.nnz, _ptr(level.edge_ptr),
               _ptr(level.edge_idx), _ptr(level.edge_w), _ptr(node_rep), _ptr(edge_rep), _ptr(c_ptr), _ptr(c_idx),
               _ptr(c_w), ctypes.cast(sizes, L.i64p), _ptr(workspace), workspace.numel(), _stream(dev))
    nv, ne, nz = int(sizes[0]), int(sizes[1]), int(sizes[2])
    coarse = DeviceLevel(nv, ne, nz, c_ptr[: ne + 1], c_idx[:nz], None if c_w is None else c_w[:ne])
    return node_rep[: level.n_nodes], edge_rep[: level.n_edges], coarse


def coarsen_features_workspace_bytes(n_nodes: int, n_edges: int, nnz: int, k: int) -> int:
    out = ctypes.c_size_t()
    L.call("hnv_coarsen_features_workspace_bytes", n_nodes, n_edges, nnz, k, ctypes.byref(out))
    return int(out.value)


def coarsen_level_features_device(level: DeviceLevel, x, workspace=None):
    """One coarsening step on the GPU driven by node features (bag-of-words
    counts, int32 [n_nodes x k], k a multiple of 4): returns (node_rep,
    edge_rep, coarse DeviceLevel, coarse features int32 [coarse n_nodes x k])."""
    torch = _torch()
    dev = level.edge_ptr.device
    level.check()
    if x.dtype != torch.int32 or x.dim() != 2 or x.shape[0] != level.n_nodes or not x.is_contiguous() \
            or x.device != dev:
        raise ValueError("x must be a contiguous int32 [n_nodes x k] tensor on the level's device")
    k = int(x.shape[1])
    need = coarsen_features_workspace_bytes(level.n_nodes, level.n_edges, level.nnz, k)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    node_rep = torch.empty(max(level.n_nodes, 1), **i32)
    edge_rep = torch.empty(max(level.n_edges, 1), **i32)
    c_ptr = torch.empty(level.n_edges + 1, **i32)
    c_idx = torch.empty(max(level.nnz, 1), **i32)
    c_w = None if level.edge_w is None else torch.empty(max(level.n_edges, 1), dtype=torch.float32, device=dev)
    c_x = torch.empty((max(level.n_nodes, 1), k), **i32)
    sizes = (ctypes.c_int64 * 3)()
    with torch.cuda.device(dev):
        L.call("hnv_coarsen_level_features_device", level.n_nodes, level.n_edges, level.nnz, _ptr(level.edge_ptr),
               _ptr(level.edge_idx), _ptr(level.edge_w), _ptr(x), k, _ptr(node_rep), _ptr(edge_rep), _ptr(c_ptr),
               _ptr(c_idx), _ptr(c_w), _ptr(c_x), ctypes.cast(sizes, L.i64p), _ptr(workspace), workspace.numel(),
               _stream(dev))
    nv, ne, nz = int(sizes[0]), int(sizes[1]), int(sizes[2])
    coarse = DeviceLevel(nv, ne, nz, c_ptr[: ne + 1], c_idx[:nz], None if c_w is None else c_w[:ne])
    return node_rep[: level.n_nodes], edge_rep[: level.n_edges], coarse, c_x[:nv]


def coarsen_hierarchy_features_device(level: DeviceLevel, x, n_coarsen: int):
    """n_coarsen feature-driven GPU coarsening steps, one shared workspace:
    returns (device levels, [(node_rep, edge_rep)], feature matrices)."""
    torch = _torch()
    ws = torch.empty(coarsen_features_workspace_bytes(level.n_nodes, level.n_edges, level.nnz, int(x.shape[1])),
                     dtype=torch.uint8, device=level.edge_ptr.device)
    levels, maps, feats = [level], [], [x]
    for _ in range(n_coarsen):
        nrep, erep, coarse, xc = coarsen_level_features_device(levels[-1], feats[-1], ws)
        maps.append((nrep, erep))
        levels.append(coarse)
        feats.append(xc)
    return levels, maps, feats


def _stop(rows_fine: int, rows_coarse: Optional[int], min_rows: int) -> bool:
    """Depth rule (Section 3.1, Algorithm 1's depth K): with min_rows > 0,
    coarsening stops once a level has at most min_rows star-expansion rows,
    or when a step no longer shrinks the level."""
    if min_rows <= 0:
        return False
    return rows_fine <= min_rows or (rows_coarse is not None and rows_coarse >= rows_fine)


def coarsen_hierarchy_device(level: DeviceLevel, n_coarsen: int, min_rows: int = 0):
    """Up to n_coarsen GPU coarsening steps from ``level`` (fewer when
    min_rows > 0 stops them, see :func:`_stop`), one shared workspace:
    returns (device levels, [(node_rep, edge_rep)] per step)."""
    torch = _torch()
    level.check()
    # the finest level's workspace serves every step: no step's workspace is
    # larger, since a coarse level is never larger than the fine one
    ws = torch.empty(coarsen_workspace_bytes(level.n_nodes, level.n_edges, level.nnz), dtype=torch.uint8,
                     device=level.edge_ptr.device)
    levels, maps = [level], []
    for _ in range(n_coarsen):
        fine = levels[-1]
        if _stop(fine.n_nodes + fine.n_edges, None, min_rows):
            break
        nrep, erep, coarse = _coarsen_step(fine, ws)
        if _stop(fine.n_nodes + fine.n_edges, coarse.n_nodes + coarse.n_edges, min_rows):
            break
        maps.append((nrep, erep))
        levels.append(coarse)
    return levels, maps


class Hierarchy:
    """Levels 0 (finest) .. L (coarsest) and the maps between them."""

    def __init__(self, levels: List[HostLevel], maps: List[HostMap]):
        assert len(maps) == len(levels) - 1
        self.levels = levels
        self.maps = maps

    @classmethod
    def build(cls, n_nodes, n_edges, edge_ptr, edge_idx, edge_w, n_coarsen: int, device=None,
              min_rows: int = 0) -> "Hierarchy":
        """Coarsens up to n_coarsen times (fewer when min_rows > 0 stops
        them: a level of at most min_rows rows, or a step that no longer
        shrinks the level), on the host, or on ``device`` (a GPU) with the
        result copied back."""
        levels = [HostLevel(n_nodes, n_edges, edge_ptr, edge_idx, edge_w)]
        maps = []
        if device is not None:
            dl, dm = coarsen_hierarchy_device(DeviceLevel.from_host(levels[0], device), n_coarsen, min_rows)
            levels += [x.to_host() for x in dl[1:]]
            maps = [HostMap(a.cpu().numpy(), b.cpu().numpy()) for a, b in dm]
            return cls(levels, maps)
        for _ in range(n_coarsen):
            if _stop(levels[-1].rows, None, min_rows):
                break
            m, c = coarsen_level(levels[-1])
            if _stop(levels[-1].rows, c.rows, min_rows):
                break
            maps.append(m)
            levels.append(c)
        return cls(levels, maps)

    def coarsest_edgelist(self):
        """The coarsest level's star expansion as an edge list for an
        external initial embedder (Section 3.2): see :func:`star_edgelist`."""
        return star_edgelist(self.levels[-1])

    @property
    def n_levels(self) -> int:
        return len(self.levels)

    def c_arrays(self):
        lv = (L.HnvLevel * self.n_levels)(*[x.c() for x in self.levels])
        mp = (L.HnvMap * max(len(self.maps), 1))(*[m.c() for m in self.maps]) if self.maps else None
        return lv, mp


def star_edgelist(level: HostLevel):
    """The star expansion H* of a level (Section 1.1) as an edge list in the
    library's row numbering (node v -> row v, hyperedge e -> row n_nodes + e):
    returns (src int64 [nnz], dst int64 [nnz], weight float32 [nnz]) with
    one edge per incidence, node row first, weighted by w_e (1 without
    weights).  This is the graph an initial embedder such as node2vec or
    DeepWalk takes for the coarsest level; its output rows map one to one
    onto the coarsest embedding the refinement starts from."""
    counts = np.diff(level.edge_ptr)
    edges = np.repeat(np.arange(level.n_edges, dtype=np.int64), counts)
    src = level.edge_idx.astype(np.int64)
    dst = level.n_nodes + edges
    w = np.ones(level.nnz, dtype=np.float32) if level.edge_w is None else level.edge_w[edges].astype(np.float32)
    return src, dst, w


def _options(options) -> Optional[L.HnvOptions]:
    if options is None:
        return None
    if isinstance(options, L.HnvOptions):
        return options
    order = options.get("order", 0)
    if isinstance(order, str):
        order = {"jacobi": L.HNV_ORDER_JACOBI, "edge_first": L.HNV_ORDER_EDGE_FIRST}[order]
    return L.HnvOptions(int(options.get("panel_cols", 0)), int(options.get("small_max", 0)),
                        int(options.get("chunk", 0)), int(order))


def plan_workspace_bytes(hier: Hierarchy, d: int, dtype: str = "f32", options=None) -> int:
    lv, mp = hier.c_arrays()
    out = ctypes.c_size_t()
    o = _options(options)
    L.call("hnv_plan_workspace_bytes", lv, mp, hier.n_levels, d, _dt(dtype),
           None if o is None else ctypes.byref(o), ctypes.byref(out))
    return int(out.value)


def _dt(dtype: str) -> int:
    if dtype in ("f32", "float32"):
        return L.HNV_F32
    if dtype in ("bf16", "bfloat16"):
        return L.HNV_BF16
    raise ValueError(dtype)


# ----------------------------------------------------------------------------
# device plan
# ----------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream(device=None) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_vec(t, n: int, dtype, name: str):
    """A device vector the kernels read or write n entries of (None passes)."""
    if t is None:
        return
    if t.dtype != dtype or not t.is_contiguous() or t.device.type != "cuda" or t.numel() < n:
        raise ValueError(f"{name}: expected a contiguous {dtype} GPU tensor of at least {n} elements, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")


def _check_sweeps(sweeps, n_levels: int) -> np.ndarray:
    sw = np.ascontiguousarray(sweeps, dtype=np.int32)
    if sw.ndim != 1 or len(sw) != n_levels:
        raise ValueError(f"sweeps: one count per level expected ({n_levels}), got {len(np.atleast_1d(sw))}")
    return sw


class Plan:
    """A device plan over a hierarchy: the workspace (a torch uint8 tensor)
    holds every level's adjacency, work lists, maps and reciprocals."""

    def __init__(self, hier: Hierarchy, d: int, dtype: str = "f32", options=None, device=None,
                 validate: bool = True, build: str = "host"):
        """build="host" builds the plan from the host arrays (hnv_plan_create);
        build="device" uploads the levels and builds the identical plan on
        the GPU (hnv_plan_create_device), much faster for large hierarchies."""
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required for a device plan")
        if build == "device":
            dev = torch.device("cuda" if device is None else device)
            levels = [DeviceLevel.from_host(lv, dev) for lv in hier.levels]
            maps = [(torch.as_tensor(m.node_rep).to(dev), torch.as_tensor(m.edge_rep).to(dev)) for m in hier.maps]
            other = Plan.from_device(levels, maps, d, dtype, options, validate)
            self.__dict__.update(other.__dict__)
            other._h = None
            self.hier = hier
            return
        if build != "host":
            raise ValueError("build must be 'host' or 'device'")
        self.device = torch.device("cuda" if device is None else device)
        self.hier = hier
        self.d = int(d)
        self.dtype = dtype
        self.torch_dtype = torch.float32 if _dt(dtype) == L.HNV_F32 else torch.bfloat16
        self.n_levels = hier.n_levels
        nbytes = plan_workspace_bytes(hier, d, dtype, options)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace is not 256-byte aligned")
        lv, mp = hier.c_arrays()
        o = _options(options)
        handle = ctypes.c_void_p()
        L.call("hnv_plan_create", lv, mp, self.n_levels, self.d, _dt(dtype), None if o is None else ctypes.byref(o),
               1 if validate else 0, self.workspace.data_ptr(), nbytes, _stream(self.device), ctypes.byref(handle))
        self._h = handle

    @classmethod
    def from_device(cls, levels: Sequence[DeviceLevel], maps: Sequence, d: int, dtype: str = "f32", options=None,
                    validate: bool = True) -> "Plan":
        """A plan built on the GPU from device levels (finest first, e.g. from
        :func:`coarsen_hierarchy_device`) and device maps [(node_rep,
        edge_rep)]: identical to the plan built from host copies."""
        torch = _torch()
        self = cls.__new__(cls)
        self.device = levels[0].edge_ptr.device
        self.hier = None
        self.d = int(d)
        self.dtype = dtype
        self.torch_dtype = torch.float32 if _dt(dtype) == L.HNV_F32 else torch.bfloat16
        self.n_levels = len(levels)
        if len(maps) != self.n_levels - 1:
            raise ValueError("need one map per coarsening step")
        for x in levels:
            x.check()
        for l, (a, b) in enumerate(maps):
            _check_vec(a, levels[l].n_nodes, torch.int32, f"node_rep of map {l}")
            _check_vec(b, levels[l].n_edges, torch.int32, f"edge_rep of map {l}")
        lv = (L.HnvLevelDev * self.n_levels)(*[L.HnvLevelDev(x.n_nodes, x.n_edges, x.nnz, _ptr(x.edge_ptr),
                                                             _ptr(x.edge_idx), _ptr(x.edge_w)) for x in levels])
        mp = (L.HnvMapDev * max(len(maps), 1))(*[L.HnvMapDev(_ptr(a), _ptr(b)) for a, b in maps])
        o = _options(options)
        ob = None if o is None else ctypes.byref(o)
        nbytes = ctypes.c_size_t()
        with torch.cuda.device(self.device):
            L.call("hnv_plan_workspace_bytes_device", lv, mp, self.n_levels, self.d, _dt(dtype), ob,
                   ctypes.byref(nbytes))
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            handle = ctypes.c_void_p()
            L.call("hnv_plan_create_device", lv, mp, self.n_levels, self.d, _dt(dtype), ob, 1 if validate else 0,
                   self.workspace.data_ptr(), int(nbytes.value), _stream(self.device), ctypes.byref(handle))
        self._h = handle
        return self

    def close(self):
        if getattr(self, "_h", None):
            L.lib().hnv_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # sizes -----------------------------------------------------------------
    def level_info(self, level: int):
        nv, ne, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        L.call("hnv_plan_level_info", self._h, level, ctypes.byref(nv), ctypes.byref(ne), ctypes.byref(nz))
        return nv.value, ne.value, nz.value

    def rows(self, level: int) -> int:
        nv, ne, _ = self.level_info(level)
        return nv + ne

    def empty(self, level: int):
        return _torch().empty((self.rows(level), self.d), dtype=self.torch_dtype, device=self.device)

    def _check(self, t, level: int, name: str):
        if t.dtype != self.torch_dtype or not t.is_contiguous() or t.device.type != "cuda" or \
                tuple(t.shape) != (self.rows(level), self.d):
            raise ValueError(f"{name}: expected contiguous {self.torch_dtype} [{self.rows(level)} x {self.d}] "
                             f"on the GPU, got {t.dtype} {tuple(t.shape)} on {t.device}")

    # kernel timing ---------------------------------------------------------
    def set_profiling(self, enable: bool):
        L.call("hnv_plan_set_profiling", self._h, 1 if enable else 0)
        self._profiling = bool(enable)

    def profile_read(self, kind: int, level: int = -1):
        """(launches, total milliseconds) of one kernel kind (see hnv.h)."""
        n, ms = ctypes.c_int64(), ctypes.c_double()
        L.call("hnv_plan_profile_read", self._h, int(kind), int(level), ctypes.byref(n), ctypes.byref(ms))
        return n.value, ms.value

    # weights ---------------------------------------------------------------
    def _check_edge_vec(self, level: int, t, name: str):
        _check_vec(t, self.level_info(level)[1], _torch().float32, name)

    def set_edge_weights(self, level: int, w):
        self._check_edge_vec(level, w, "w")
        L.call("hnv_set_edge_weights", self._h, level, _ptr(w), _stream(self.device))

    def set_edge_logweights(self, level: int, theta, w_out=None):
        self._check_edge_vec(level, theta, "theta")
        self._check_edge_vec(level, w_out, "w_out")
        L.call("hnv_set_edge_logweights", self._h, level, _ptr(theta), _ptr(w_out), _stream(self.device))

    def logweight_grad(self, level: int, dw, dtheta=None):
        out = dw if dtheta is None else dtheta
        self._check_edge_vec(level, dw, "dw")
        self._check_edge_vec(level, out, "dtheta")
        L.call("hnv_logweight_grad", self._h, level, _ptr(dw), _ptr(out), _stream(self.device))
        return out

    # forward ---------------------------------------------------------------
    def refine(self, z_coarsest, sweeps: Sequence[int], omega: float = 0.5, tol: float = 0.0,
               residuals: bool = False, out=None):
        """Multi-level refinement.  Returns (z_finest, residuals or None, sweeps_done)."""
        torch = _torch()
        self._check(z_coarsest, self.n_levels - 1, "z_coarsest")
        z_out = self.empty(0) if out is None else out
        self._check(z_out, 0, "out")
        sw = _check_sweeps(sweeps, self.n_levels)
        res = torch.zeros(max(int(sw.sum()), 1), dtype=torch.float64, device=self.device) if residuals else None
        done = np.zeros(self.n_levels, dtype=np.int32)
        L.call("hnv_refine", self._h, z_coarsest.data_ptr(), z_out.data_ptr(), sw.ctypes.data_as(L.i32p),
               float(omega), float(tol), _ptr(res), done.ctypes.data_as(L.i32p), _stream(self.device))
        return z_out, res, done

    def capture_refine(self, z_coarsest, sweeps: Sequence[int], omega: float = 0.5, residuals: bool = False,
                       tol: float = 0.0):
        """Captures one refinement into a HIP graph (through
        torch.cuda.CUDAGraph) for launch-bound sizes: returns a RefineGraph
        whose replay() reruns every launch on the current stream, reading
        ``z_coarsest`` (the same tensor, refill it in place) and writing
        its ``out`` (and ``residuals``) tensors.  With ``tol`` > 0 the
        early stop is decided on the device at every replay."""
        return RefineGraph(self, z_coarsest, sweeps, omega, residuals, tol)

    def sweep(self, level: int, z_in, omega: float = 0.5, from_coarse: bool = False, out=None, resid=None):
        """One sweep; ``out`` may be ``z_in`` itself for an edge-first plan."""
        self._check(z_in, level + 1 if from_coarse else level, "z_in")
        z_out = self.empty(level) if out is None else out
        self._check(z_out, level, "out")
        _check_vec(resid, 1, _torch().float64, "resid")
        L.call("hnv_sweep", self._h, level, z_in.data_ptr(), z_out.data_ptr(), float(omega), 1 if from_coarse else 0,
               _ptr(resid), _stream(self.device))
        return z_out

    def sweep_noalloc(self, level: int, z_in, omega: float = 0.5, from_coarse: bool = False, out=None, resid=None):
        """The same sweep through hnv_sweep_noalloc (scratch in the library's
        static device array, no allocation by the call itself; ``out`` should
        be passed by callers that must not allocate)."""
        self._check(z_in, level + 1 if from_coarse else level, "z_in")
        z_out = self.empty(level) if out is None else out
        self._check(z_out, level, "out")
        _check_vec(resid, 1, _torch().float64, "resid")
        L.call("hnv_sweep_noalloc", self._h, level, z_in.data_ptr(), z_out.data_ptr(), float(omega),
               1 if from_coarse else 0, _ptr(resid), _stream(self.device))
        return z_out

    def project(self, level: int, z_coarse, out=None):
        self._check(z_coarse, level + 1, "z_coarse")
        z_out = self.empty(level) if out is None else out
        self._check(z_out, level, "out")
        L.call("hnv_project", self._h, level, z_coarse.data_ptr(), z_out.data_ptr(), _stream(self.device))
        return z_out

    # reverse ---------------------------------------------------------------
    def sweep_adjoint(self, level: int, g_in, z_prev, z_cur, omega: float = 0.5, dw=None, out=None,
                      node_acc=None):
        """Reverse mode of one sweep, in the plan's sweep order (Jacobi or
        edge-first).  With ``dw`` the weight gradient is added
        to it; with ``node_acc`` too (float32 [n_nodes], zeroed before the
        first of several sweeps) it is split, and :meth:`weight_grad_finish`
        completes ``dw`` after the last sweep."""
        for t, n in ((g_in, "g_in"), (z_prev, "z_prev"), (z_cur, "z_cur")):
            self._check(t, level, n)
        g_out = self.empty(level) if out is None else out
        self._check(g_out, level, "out")
        self._check_edge_vec(level, dw, "dw")
        if node_acc is None:
            L.call("hnv_sweep_adjoint", self._h, level, g_in.data_ptr(), g_out.data_ptr(), z_prev.data_ptr(),
                   z_cur.data_ptr(), _ptr(dw), float(omega), _stream(self.device))
        else:
            if dw is None:
                raise ValueError("node_acc needs dw")
            _check_vec(node_acc, self.level_info(level)[0], _torch().float32, "node_acc")
            L.call("hnv_sweep_adjoint_split", self._h, level, g_in.data_ptr(), g_out.data_ptr(), z_prev.data_ptr(),
                   z_cur.data_ptr(), _ptr(dw), _ptr(node_acc), float(omega), _stream(self.device))
        return g_out

    def weight_grad_finish(self, level: int, node_acc, dw):
        """dw[e] -= sum of node_acc over the members of e (completes a split weight gradient)."""
        _check_vec(node_acc, self.level_info(level)[0], _torch().float32, "node_acc")
        self._check_edge_vec(level, dw, "dw")
        L.call("hnv_weight_grad_finish", self._h, level, _ptr(node_acc), _ptr(dw), _stream(self.device))
        return dw

    def project_adjoint(self, level: int, g_fine, out=None):
        self._check(g_fine, level, "g_fine")
        g_out = self.empty(level + 1) if out is None else out
        self._check(g_out, level + 1, "out")
        L.call("hnv_project_adjoint", self._h, level, g_fine.data_ptr(), g_out.data_ptr(), _stream(self.device))
        return g_out


_SCORE_OPS = {"variance": L.HNV_SCORE_VARIANCE, "mean": L.HNV_SCORE_MEAN, "min": L.HNV_SCORE_MIN,
              "max": L.HNV_SCORE_MAX}


class RefineGraph:
    """A refinement captured into a HIP graph (see Plan.capture_refine).
    Kernel profiling records host-side events and is not captured."""

    def __init__(self, plan: "Plan", z_coarsest, sweeps: Sequence[int], omega: float, residuals: bool,
                 tol: float = 0.0):
        torch = _torch()
        if getattr(plan, "_profiling", False):
            raise RuntimeError("turn kernel profiling off before capturing a refinement")
        plan._check(z_coarsest, plan.n_levels - 1, "z_coarsest")
        self.plan, self.z_coarsest, self.omega, self.tol = plan, z_coarsest, float(omega), float(tol)
        self.sweeps = _check_sweeps(sweeps, plan.n_levels)
        self.out = plan.empty(0)
        self.residuals = (torch.zeros(max(int(self.sweeps.sum()), 1), dtype=torch.float64, device=plan.device)
                          if residuals else None)
        self._done = np.zeros(plan.n_levels, dtype=np.int32)
        side = torch.cuda.Stream(device=plan.device)
        side.wait_stream(torch.cuda.current_stream(plan.device))
        with torch.cuda.stream(side):                 # first run outside the graph
            self._launch(self._done.ctypes.data_as(L.i32p))
        torch.cuda.current_stream(plan.device).wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            # no sweep counts: with tol they would be read back on the host
            self._launch(None)

    def _launch(self, done):
        L.call("hnv_refine", self.plan._h, self.z_coarsest.data_ptr(), self.out.data_ptr(),
               self.sweeps.ctypes.data_as(L.i32p), self.omega, self.tol,
               _ptr(self.residuals), done, _stream(self.plan.device))

    def replay(self):
        """Reruns the captured refinement; returns (out, residuals)."""
        self.graph.replay()
        return self.out, self.residuals


class ScorePlan:
    """Candidate node sets for hyperedge-prediction features (Section 4),
    planned once on the host (``cand_ptr`` / ``cand_idx``: CSR of member node
    ids) or on the GPU (:meth:`from_device`) and kept in a device workspace."""

    def __init__(self, cand_ptr, cand_idx, z_rows: int, d: int, dtype: str = "f32", device=None):
        torch = _torch()
        self.device = torch.device("cuda" if device is None else device)
        ptr = np.ascontiguousarray(np.asarray(cand_ptr), dtype=np.int64)
        idx = np.ascontiguousarray(np.asarray(cand_idx), dtype=np.int32)
        self.n_cand = len(ptr) - 1
        self.z_rows = int(z_rows)
        self.d = int(d)
        self.dtype = dtype
        dt = _dt(dtype)
        need = ctypes.c_size_t()
        L.call("hnv_score_workspace_bytes", ptr.ctypes.data_as(L.i64p), self.n_cand, self.d, dt, ctypes.byref(need))
        self.workspace = torch.empty(max(need.value, 256), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        L.call("hnv_score_plan_create", ptr.ctypes.data_as(L.i64p), idx.ctypes.data_as(L.i32p), self.n_cand,
               int(z_rows), self.d, dt, self.workspace.data_ptr(), self.workspace.numel(), _stream(self.device),
               ctypes.byref(h))
        self._h = h

    @classmethod
    def from_device(cls, cand_ptr, cand_idx, z_rows: int, d: int, dtype: str = "f32") -> "ScorePlan":
        """The same plan built on the GPU from device tensors (int32
        ``cand_ptr`` [n_cand+1] and ``cand_idx`` [n_members])."""
        torch = _torch()
        for t in (cand_ptr, cand_idx):
            if t.dtype != torch.int32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("cand_ptr / cand_idx: contiguous int32 device tensors expected")
        self = cls.__new__(cls)
        self.device = cand_ptr.device
        self.n_cand = int(cand_ptr.numel()) - 1
        self.z_rows = int(z_rows)
        n_members = int(cand_idx.numel())
        self.d = int(d)
        self.dtype = dtype
        dt = _dt(dtype)
        need = ctypes.c_size_t()
        with torch.cuda.device(self.device):
            L.call("hnv_score_workspace_bytes_device", self.n_cand, n_members, self.d, dt, ctypes.byref(need))
            self.workspace = torch.empty(need.value, dtype=torch.uint8, device=self.device)
            h = ctypes.c_void_p()
            L.call("hnv_score_plan_create_device", cand_ptr.data_ptr(), _ptr(cand_idx) if n_members else None,
                   self.n_cand, n_members, int(z_rows), self.d, dt, self.workspace.data_ptr(), self.workspace.numel(),
                   _stream(self.device), ctypes.byref(h))
        self._h = h
        return self

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                L.lib().hnv_score_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def score(self, z_nodes, op: str = "variance", out=None):
        torch = _torch()
        want = torch.float32 if _dt(self.dtype) == L.HNV_F32 else torch.bfloat16
        if z_nodes.dtype != want or not z_nodes.is_contiguous() or z_nodes.dim() != 2 or \
                z_nodes.shape[1] != self.d or z_nodes.shape[0] < self.z_rows or z_nodes.device.type != "cuda":
            raise ValueError(f"z_nodes: contiguous {want} [>= {self.z_rows} x {self.d}] GPU tensor expected, got "
                             f"{z_nodes.dtype} {tuple(z_nodes.shape)} on {z_nodes.device}")
        if out is None:
            out = torch.empty((self.n_cand, self.d), dtype=torch.float32, device=self.device)
        _check_vec(out, self.n_cand * self.d, torch.float32, "out")
        L.call("hnv_score_candidates", self._h, z_nodes.data_ptr(), _SCORE_OPS[op], out.data_ptr(),
               _stream(self.device))
        return out


def score_candidates(z_nodes, cand_ptr, cand_idx, op: str = "variance"):
    """One-shot hyperedge-prediction features (plans, then scores)."""
    torch = _torch()
    dtype = "f32" if z_nodes.dtype == torch.float32 else "bf16"
    plan = ScorePlan(cand_ptr, cand_idx, z_nodes.shape[0], z_nodes.shape[1], dtype, z_nodes.device)
    return plan.score(z_nodes, op)


def cast(src, dst_dtype: str):
    """Storage conversion on the device (FP32 -> BF16 rounds to nearest even)."""
    torch = _torch()
    sdt = L.HNV_F32 if src.dtype == torch.float32 else L.HNV_BF16 if src.dtype == torch.bfloat16 else None
    if sdt is None or not src.is_contiguous():
        raise ValueError("cast: contiguous float32 or bfloat16 tensor expected")
    ddt = _dt(dst_dtype)
    out = torch.empty(src.shape, dtype=torch.float32 if ddt == L.HNV_F32 else torch.bfloat16, device=src.device)
    L.call("hnv_cast", src.data_ptr(), sdt, out.data_ptr(), ddt, src.numel(), _stream(src.device))
    return out


# ----------------------------------------------------------------------------
# autograd
# ----------------------------------------------------------------------------

def _refine_function():
    torch = _torch()

    class RefineFunction(torch.autograd.Function):
        """K sweeps at one level with learnable log-weights theta (w = exp theta),
        starting from the coarser level's embedding (from_coarse, the first
        sweep fused with the projection) or from this level's own.  The
        forward keeps every ckpt_every-th state; the backward recomputes each
        segment from its checkpoint and runs the reverse sweeps."""

        @staticmethod
        def forward(ctx, z_start, theta, plan, level, sweeps, omega, from_coarse, ckpt_every):
            if theta is not None:
                plan.set_edge_logweights(level, theta.detach())
            ck = max(1, int(ckpt_every))
            K = int(sweeps)
            saved = {0: z_start.detach()}
            cur = z_start.detach()
            for i in range(1, K + 1):
                nxt = plan.sweep(level, cur, omega, from_coarse=(from_coarse and i == 1))
                if i % ck == 0 or i == K:
                    saved[i] = nxt
                cur = nxt
            if K == 0:
                cur = plan.project(level, z_start.detach()) if from_coarse else z_start.detach().clone()
            ctx.plan, ctx.level, ctx.K, ctx.omega, ctx.from_coarse, ctx.ck = plan, level, K, omega, from_coarse, ck
            ctx.ckpt_keys = sorted(saved)
            ctx.save_for_backward(*(saved[k] for k in ctx.ckpt_keys), *(() if theta is None else (theta.detach(),)))
            ctx.has_theta = theta is not None
            return cur

        @staticmethod
        def backward(ctx, g_out):
            torch = _torch()
            plan, level, K, omega = ctx.plan, ctx.level, ctx.K, ctx.omega
            tensors = ctx.saved_tensors
            n_ck = len(ctx.ckpt_keys)
            ckpts = dict(zip(ctx.ckpt_keys, tensors[:n_ck]))
            theta = tensors[n_ck] if ctx.has_theta else None
            if theta is not None:
                plan.set_edge_logweights(level, theta)
            g = g_out.contiguous().to(plan.torch_dtype)
            n_nodes, n_edges, _ = plan.level_info(level)
            dw = torch.zeros(max(n_edges, 1), dtype=torch.float32, device=plan.device) if theta is not None else None
            # the weight gradient of all K reverse sweeps, split: the per-node
            # part is summed over the sweeps and gathered per hyperedge once
            nacc = torch.zeros(max(n_nodes, 1), dtype=torch.float32, device=plan.device) if theta is not None \
                else None
            bounds = ctx.ckpt_keys
            for si in range(len(bounds) - 1, 0, -1):
                s0, s1 = bounds[si - 1], bounds[si]
                states = {}
                start = ckpts[s0]
                if ctx.from_coarse and s0 == 0:
                    states[0] = plan.project(level, start)
                else:
                    states[s0] = start
                for i in range(s0 + 1, s1):
                    states[i] = plan.sweep(level, states[i - 1], omega)
                states[s1] = ckpts[s1]
                for i in range(s1, s0, -1):
                    g = plan.sweep_adjoint(level, g, states[i - 1], states[i], omega, dw=dw, node_acc=nacc)
            if K == 0 and not ctx.from_coarse:
                gz = g
            elif ctx.from_coarse:
                gz = plan.project_adjoint(level, g)
            else:
                gz = g
            if theta is not None:
                plan.weight_grad_finish(level, nacc, dw)
            gtheta = plan.logweight_grad(level, dw)[:n_edges] if theta is not None else None
            return gz, gtheta, None, None, None, None, None, None

    return RefineFunction


_RF = None


def refine_level(z_start, theta, plan: Plan, level: int, sweeps: int, omega: float = 0.5,
                 from_coarse: bool = True, ckpt_every: int = 5):
    """Differentiable refinement of one level (see RefineFunction)."""
    global _RF
    if _RF is None:
        _RF = _refine_function()
    return _RF.apply(z_start, theta, plan, level, sweeps, omega, from_coarse, ckpt_every)


def refine_hierarchy(z_coarsest, thetas, plan: Plan, sweeps: Sequence[int], omega: float = 0.5,
                     ckpt_every: int = 5):
    """Differentiable multi-level refinement (Section 3.3): the sweeps of the
    coarsest level, then projection and sweeps at each finer level, one
    :func:`refine_level` per level.  ``thetas[l]`` are level l's learnable
    log-weights (or None to keep the plan's weights); gradients reach
    ``z_coarsest`` and every ``thetas[l]``.  Returns the finest embedding."""
    L = plan.n_levels - 1
    if len(thetas) != plan.n_levels:
        raise ValueError(f"thetas: one entry per level expected ({plan.n_levels})")
    sw = _check_sweeps(sweeps, plan.n_levels)
    z = refine_level(z_coarsest, thetas[L], plan, L, int(sw[L]), omega, from_coarse=False, ckpt_every=ckpt_every)
    for lvl in range(L - 1, -1, -1):
        z = refine_level(z, thetas[lvl], plan, lvl, int(sw[lvl]), omega, from_coarse=True, ckpt_every=ckpt_every)
    return z
