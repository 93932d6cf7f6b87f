"""Seeded synthetic hypergraphs shaped like the paper's workloads.

The paper evaluates on citation / co-authorship hypergraphs (Table 1) and on
large social hypergraphs such as Friendster (Table 3, Table 5).  None of those
datasets is available here, so every input is synthetic and seeded:

* hyperedge sizes are drawn from a uniform range or from a truncated power law
  P(k) proportional to k^-a on the support [2, N];
* members are drawn without replacement, either uniformly over the nodes or in
  proportion to a node popularity p_v = rank_v^-b (rank = seeded permutation);
* hyperedge weights are unit or uniform in [lo, hi] (float32);
* coarsest-level embeddings are N(0, 1) float32;
* node features, where a workload has them, are bag-of-words counts (the
  paper's citation datasets encode each document that way, Section 3.1 and
  Section 4): each node holds a few distinct words drawn by a Zipf word
  popularity over a k-word vocabulary, each with a small count; some nodes
  are empty documents and some repeat another node's document exactly.

A hypergraph is returned in canonical form: each hyperedge row lists its
members in ascending order without duplicates (hyperedges are sets of nodes,
Section 1), offsets are int64 and member ids int32.

Each named configuration carries a seed k: structure k, weights 100+k,
embeddings 200+k, labels / head / cotangent 300+k, features 400+k.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    seed: int
    n_nodes: int
    n_edges: int
    sizes: tuple            # ("uniform", lo, hi) or ("zipf", a, N)
    members: tuple          # ("uniform",) or ("popularity", b)
    weights: tuple          # ("unit",) or ("uniform", lo, hi)
    d: int
    levels: int             # number of coarsening steps L (L+1 levels)
    sweeps: tuple           # sweeps per level, index = level (0 = finest)
    dtypes: tuple = ("f32",)
    adjoint_sweeps: int = 0
    label_frac: float = 0.0
    n_classes: int = 0
    checkpoint_every: int = 0
    features: tuple = ()    # ("bow", k, words_lo, words_hi) or ()


def _sweeps(levels: int, k: int) -> tuple:
    return tuple([k] * (levels + 1))


CONFIGS = {
    # tiny: Citeseer-scale (Table 1), correctness only
    "tiny-2k": Config("tiny-2k", 1, 2_000, 1_000, ("uniform", 2, 8), ("uniform",), ("unit",),
                      32, 3, _sweeps(3, 10)),
    # medium, hub-heavy node side (DBLP / Wordnet scale, Tables 1 and 3)
    "hub-200k": Config("hub-200k", 2, 200_000, 100_000, ("zipf", 2.1, 500), ("popularity", 1.5),
                       ("uniform", 0.5, 2.0), 64, 5, _sweeps(5, 20)),
    # BF16 vs FP32 refinement at millions of rows
    "zipf-2m": Config("zipf-2m", 3, 2_000_000, 1_500_000, ("zipf", 2.1, 2_000), ("uniform",), ("unit",),
                      128, 8, _sweeps(8, 20), dtypes=("bf16", "f32")),
    # differentiable refinement: one coarsening step, 10 sweeps at the finest level only
    "grad-500k": Config("grad-500k", 4, 500_000, 300_000, ("zipf", 2.1, 1_000), ("uniform",), ("unit",),
                        128, 1, (10, 0), adjoint_sweeps=10, label_frac=0.10, n_classes=16,
                        checkpoint_every=5),
    # feature-driven coarsening: Pubmed-sized (Table 1), k = 500 words
    "bow-20k": Config("bow-20k", 6, 19_717, 7_963, ("zipf", 2.1, 171), ("uniform",), ("unit",),
                      32, 4, _sweeps(4, 10), features=("bow", 500, 5, 50)),
    # feature-driven coarsening at a million nodes, k = 512 words
    "bow-1m": Config("bow-1m", 7, 1_000_000, 600_000, ("zipf", 2.1, 500), ("uniform",), ("unit",),
                     64, 6, _sweeps(6, 10), features=("bow", 512, 5, 40)),
    # Friendster-scale BF16 refinement + adjoint (Table 3 / Table 5 scale)
    "zipf-8m": Config("zipf-8m", 5, 8_000_000, 10_000_000, ("zipf", 2.0, 5_000), ("uniform",), ("unit",),
                      128, 10, _sweeps(10, 20), dtypes=("bf16",), adjoint_sweeps=5),
}


@dataclasses.dataclass
class Hypergraph:
    n_nodes: int
    n_edges: int
    edge_ptr: np.ndarray           # int64 [n_edges + 1]
    edge_idx: np.ndarray           # int32 [nnz], each row ascending, unique
    edge_w: Optional[np.ndarray]   # float32 [n_edges] or None (unit)

    @property
    def nnz(self) -> int:
        return int(self.edge_ptr[-1])


# ----------------------------------------------------------------------------
# size and member sampling
# ----------------------------------------------------------------------------

def _draw_sizes(rng: np.random.Generator, n_edges: int, spec: tuple, n_nodes: int,
                size_mode: str = "truncate") -> np.ndarray:
    kind = spec[0]
    if kind == "uniform":
        lo, hi = int(spec[1]), int(spec[2])
        return rng.integers(lo, hi + 1, size=n_edges, dtype=np.int64)
    if kind == "zipf":
        a, cap = float(spec[1]), int(spec[2])
        cap = min(cap, n_nodes)
        if size_mode == "truncate":
            k = np.arange(2, cap + 1, dtype=np.float64)
            cdf = np.cumsum(k ** (-a))
            cdf /= cdf[-1]
            u = rng.random(n_edges)
            return 2 + np.searchsorted(cdf, u, side="right").astype(np.int64).clip(0, cap - 2)
        if size_mode == "clamp":
            return np.clip(rng.zipf(a, size=n_edges), 2, cap).astype(np.int64)
        raise ValueError(f"unknown size_mode {size_mode!r}")
    raise ValueError(f"unknown size distribution {spec!r}")


def _segment_positions(starts: np.ndarray, lens: np.ndarray) -> np.ndarray:
    """Concatenation of the ranges [starts[i], starts[i] + lens[i])."""
    total = int(lens.sum())
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    seg = np.repeat(np.arange(len(lens), dtype=np.int64), lens)
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    return starts[seg] + (np.arange(total, dtype=np.int64) - offs[seg])


def _fill_members(rng: np.random.Generator, sizes: np.ndarray, n_nodes: int, draw) -> tuple:
    """Draw each hyperedge's members without replacement.

    All slots are drawn at once; then, repeatedly, the rows that still hold a
    repeated member are sorted and every repeat is redrawn, until every row
    is a set.  A row that comes out of a round with no repeat is left sorted.
    """
    n_edges = len(sizes)
    ptr = np.zeros(n_edges + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    idx = draw(int(ptr[-1]))
    active = np.arange(n_edges, dtype=np.int64)
    while active.size:
        lens = sizes[active]
        pos = _segment_positions(ptr[active], lens)
        rid = np.repeat(np.arange(active.size, dtype=np.int64), lens)
        key = rid * np.int64(n_nodes) + idx[pos]
        key.sort()                       # sorts within each row (rows are key-disjoint)
        sub = key - rid * np.int64(n_nodes)
        same = sub[1:] == sub[:-1]
        same &= rid[1:] == rid[:-1]
        dpos = np.nonzero(same)[0] + 1
        if dpos.size:
            sub[dpos] = draw(dpos.size)
        idx[pos] = sub
        active = active[np.unique(rid[dpos])]
    return ptr, idx.astype(np.int32)


def _uniform_draw(rng, n_nodes):
    return lambda n: rng.integers(0, n_nodes, size=n, dtype=np.int64)


def _popularity_draw(rng, n_nodes, b):
    perm = rng.permutation(n_nodes)              # perm[r-1] = node of rank r
    cdf = np.cumsum(np.arange(1, n_nodes + 1, dtype=np.float64) ** (-b))
    cdf /= cdf[-1]

    def draw(n):
        r = np.searchsorted(cdf, rng.random(n), side="right").clip(0, n_nodes - 1)
        return perm[r].astype(np.int64)
    return draw


def make_hypergraph(cfg: Config, size_mode: str = "truncate") -> Hypergraph:
    """The finest-level hypergraph of a named configuration."""
    rng = np.random.default_rng(cfg.seed)
    sizes = _draw_sizes(rng, cfg.n_edges, cfg.sizes, cfg.n_nodes, size_mode)
    if cfg.members[0] == "uniform":
        draw = _uniform_draw(rng, cfg.n_nodes)
    elif cfg.members[0] == "popularity":
        draw = _popularity_draw(rng, cfg.n_nodes, float(cfg.members[1]))
    else:
        raise ValueError(cfg.members)
    ptr, idx = _fill_members(rng, sizes, cfg.n_nodes, draw)
    w = None
    if cfg.weights[0] == "uniform":
        wr = np.random.default_rng(100 + cfg.seed)
        w = wr.uniform(cfg.weights[1], cfg.weights[2], size=cfg.n_edges).astype(np.float32)
    return Hypergraph(cfg.n_nodes, cfg.n_edges, ptr, idx, w)


def random_hypergraph(seed: int, n_nodes: int, n_edges: int, size_lo: int = 1, size_hi: int = 5,
                      weighted: bool = True, w_lo: float = 0.5, w_hi: float = 2.0,
                      integer_weights: bool = False) -> Hypergraph:
    """A small random hypergraph for property tests (isolated nodes and
    singleton hyperedges occur on purpose)."""
    rng = np.random.default_rng(seed)
    size_hi = min(size_hi, n_nodes)
    size_lo = min(size_lo, size_hi)
    sizes = rng.integers(size_lo, size_hi + 1, size=n_edges, dtype=np.int64)
    ptr, idx = _fill_members(rng, sizes, n_nodes, _uniform_draw(rng, n_nodes))
    w = None
    if weighted:
        if integer_weights:
            w = rng.integers(1, 4, size=n_edges).astype(np.float32)
        else:
            w = rng.uniform(w_lo, w_hi, size=n_edges).astype(np.float32)
    return Hypergraph(n_nodes, n_edges, ptr, idx, w)


# ----------------------------------------------------------------------------
# embeddings, labels, heads, cotangents
# ----------------------------------------------------------------------------

def coarsest_embedding(cfg_or_seed, n_rows: int, d: int, columns: Optional[Sequence[int]] = None) -> np.ndarray:
    """N(0,1) float32 [n_rows x d].  With ``columns``, only those columns of
    the same matrix are returned (the draw is column-major by construction, so
    a column subset is cheap and identical to slicing the full matrix)."""
    seed = cfg_or_seed.seed if isinstance(cfg_or_seed, Config) else int(cfg_or_seed)
    cols = range(d) if columns is None else list(columns)
    out = np.empty((n_rows, len(cols)), dtype=np.float32)
    for j, c in enumerate(cols):
        rng = np.random.default_rng([200 + seed, int(c)])
        out[:, j] = rng.standard_normal(n_rows, dtype=np.float32)
    return out


def drop_isolated_and_singletons(hg: Hypergraph) -> tuple:
    """The paper's dataset cleaning (Section 4): hyperedges with one member
    are dropped, then nodes left without hyperedges, and the remaining nodes
    are renumbered in order.  Returns (pruned Hypergraph, kept node ids of
    the input)."""
    sizes = np.diff(hg.edge_ptr)
    keep_e = np.nonzero(sizes >= 2)[0]
    seg = np.repeat(np.arange(hg.n_edges), sizes)
    keep_inc = np.isin(seg, keep_e)
    members = hg.edge_idx[keep_inc]
    used = np.zeros(hg.n_nodes, dtype=bool)
    used[members] = True
    kept_nodes = np.nonzero(used)[0]
    new_id = np.full(hg.n_nodes, -1, dtype=np.int64)
    new_id[kept_nodes] = np.arange(len(kept_nodes))
    ptr = np.zeros(len(keep_e) + 1, dtype=np.int64)
    np.cumsum(sizes[keep_e], out=ptr[1:])
    idx = new_id[members].astype(np.int32)     # renumbering keeps each row ascending
    w = None if hg.edge_w is None else hg.edge_w[keep_e].copy()
    return Hypergraph(len(kept_nodes), len(keep_e), ptr, idx, w), kept_nodes


def bag_of_words(seed: int, n_nodes: int, k: int, words_lo: int, words_hi: int, zipf_a: float = 1.1,
                 max_count: int = 3, empty_frac: float = 0.02, repeat_frac: float = 0.05) -> np.ndarray:
    """int32 [n_nodes x k] word counts: words_lo..words_hi distinct words per
    node (word rank r drawn with probability proportional to r^-zipf_a),
    counts uniform on 1..max_count, a fraction of empty rows and a fraction
    of rows copied from a random other row."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(k)
    cdf = np.cumsum(np.arange(1, k + 1, dtype=np.float64) ** (-zipf_a))
    cdf /= cdf[-1]
    x = np.zeros((n_nodes, k), dtype=np.int32)
    n_words = rng.integers(words_lo, min(words_hi, k) + 1, size=n_nodes)
    total = int(n_words.sum())
    rows = np.repeat(np.arange(n_nodes, dtype=np.int64), n_words)
    cols = perm[np.searchsorted(cdf, rng.random(total), side="right").clip(0, k - 1)]
    counts = rng.integers(1, max_count + 1, size=total).astype(np.int32)
    x[rows, cols] = counts                      # a repeated word keeps one count
    empty = rng.random(n_nodes) < empty_frac
    x[empty] = 0
    rep = np.nonzero(rng.random(n_nodes) < repeat_frac)[0]
    if rep.size and n_nodes > 1:
        x[rep] = x[rng.integers(0, n_nodes, size=rep.size)]
    return x


def node_features(cfg: Config) -> np.ndarray:
    """The bag-of-words matrix of a named configuration that has features."""
    kind, k, lo, hi = cfg.features
    assert kind == "bow"
    return bag_of_words(400 + cfg.seed, cfg.n_nodes, k, lo, hi)


def labelled_nodes(cfg: Config) -> tuple:
    """(node ids ascending int64, labels int64) for the classification head."""
    rng = np.random.default_rng(300 + cfg.seed)
    n_lab = int(round(cfg.label_frac * cfg.n_nodes))
    nodes = np.sort(rng.choice(cfg.n_nodes, size=n_lab, replace=False)).astype(np.int64)
    labels = rng.integers(0, cfg.n_classes, size=n_lab, dtype=np.int64)
    return nodes, labels


def linear_head(cfg: Config) -> tuple:
    """(W [C x d] ~ N(0, 1/d) float32, b = 0 [C])."""
    rng = np.random.default_rng([300 + cfg.seed, 1])
    W = (rng.standard_normal((cfg.n_classes, cfg.d)) / np.sqrt(cfg.d)).astype(np.float32)
    return W, np.zeros(cfg.n_classes, dtype=np.float32)


def cotangent(cfg_or_seed, n_rows: int, d: int, columns: Optional[Sequence[int]] = None) -> np.ndarray:
    """N(0,1) float32 cotangent for an adjoint run, same column convention as
    :func:`coarsest_embedding`."""
    seed = cfg_or_seed.seed if isinstance(cfg_or_seed, Config) else int(cfg_or_seed)
    cols = range(d) if columns is None else list(columns)
    out = np.empty((n_rows, len(cols)), dtype=np.float32)
    for j, c in enumerate(cols):
        rng = np.random.default_rng([300 + seed, 2, int(c)])
        out[:, j] = rng.standard_normal(n_rows, dtype=np.float32)
    return out
