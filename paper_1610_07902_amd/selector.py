"""Learned schedule selector: training data from the library's own timings,
training with the library's MLP kernels, evaluation helpers.

The selector replaces the fixed bucket count the paper uses on CPUs (4t
buckets, "Performance optimizations") by a per-call choice among ten
classes: push (Algorithm 1) with 2^(c+4) buckets for c = 0..8, or the pull
direction (c = 9).  Its six inputs are quantities the work-estimation scan
already has: nnz(x), the products W (the sum of the selected column lengths,
the paper's work bound), the longest selected column, n, nnz(A) / n and the
number of unvisited vertices (n outside a BFS), each as log2(1 + v).

Everything here drives the C library: the timings are the library's own
calls (HIP events on the launch stream), the network is trained by
spmspv_mlp_train_step and evaluated by spmspv_mlp_forward on the device.
PyTorch only holds device buffers and builds index / mask arrays.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import (MIN_SELECT2ND_I32, OR_AND_BOOL, PLUS_TIMES_F32, PULL_ROWWISE, X_ALL_TRUE, X_VAL_IS_INDEX,
               MLP_PARAMS, NUM_CLASSES, Schedule, spmspv_class_schedule, spmspv_mlp_forward, spmspv_mlp_train_step,
               spmspv_run_masked)

IN, H1, H2, OUT = 6, 64, 64, NUM_CLASSES
WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.json")


def kernel_digest() -> str:
    """Digest of the library's device sources (every .hip and .h under
    csrc/, the one build.py compiles into the library).  Weights are trained
    on timings of these kernels; a weights file whose digest differs was
    trained on other kernels and is stale."""
    from .build import source_digest
    return source_digest()


def weights_current(meta: dict) -> bool:
    """True when weights (their meta) were trained on the current kernels."""
    return meta.get("kernel_digest") == kernel_digest()


def encode(raw: np.ndarray) -> np.ndarray:
    """log2(1 + v) of the six raw features (what the device computes)."""
    return np.log2(1.0 + np.asarray(raw, np.float64))


def raw_features(f, W, maxlen, n, nnz, unvisited) -> np.ndarray:
    return np.array([f, W, maxlen, n, nnz / n, unvisited], np.float64)


@dataclass
class Samples:
    raw: List[np.ndarray] = field(default_factory=list)      # [6] each
    times: List[np.ndarray] = field(default_factory=list)    # [10] microseconds (inf = unavailable)
    tags: List[str] = field(default_factory=list)

    def add(self, raw, times, tag):
        self.raw.append(np.asarray(raw, np.float64))
        self.times.append(np.asarray(times, np.float64))
        self.tags.append(tag)

    def extend(self, other: "Samples"):
        self.raw += other.raw
        self.times += other.times
        self.tags += other.tags

    def subset(self, keep) -> "Samples":
        out = Samples()
        for r, t, g, k in zip(self.raw, self.times, self.tags, keep):
            if k:
                out.add(r, t, g)
        return out

    @property
    def bfs_steps(self) -> np.ndarray:
        """Samples taken inside a BFS: fewer unvisited vertices than n."""
        X = self.X
        return X[:, 5] < X[:, 3]

    @property
    def X(self) -> np.ndarray:
        return np.array(self.raw).reshape(-1, IN)

    @property
    def T(self) -> np.ndarray:
        return np.array(self.times).reshape(-1, OUT)

    def save(self, path):
        np.savez(path, raw=self.X, times=self.T, tags=np.array(self.tags))

    @classmethod
    def load(cls, path):
        z = np.load(path, allow_pickle=False)
        s = cls()
        for r, t, g in zip(z["raw"], z["times"], z["tags"]):
            s.add(r, t, str(g))
        return s


def class_schedule(M, c: int, semiring: int = MIN_SELECT2ND_I32) -> Schedule:
    """The library's schedule for class c (push tile and merge variant, or pull)."""
    return spmspv_class_schedule(M.handle, semiring, c)


def time_classes(M, semiring: int, x_idx, x_val, flags: int, mask, reps: int = 3, bfs_step: bool = False):
    """Microseconds per call of every class on one input (inf when a class
    is unavailable), plus the scan's statistics (W, max column length)."""
    import torch
    stream = torch.cuda.current_stream()
    f = int(x_idx.numel())
    cap = M.m
    vdt = {PLUS_TIMES_F32: torch.float32, MIN_SELECT2ND_I32: torch.int32, OR_AND_BOOL: torch.uint8}[semiring]
    y_idx = torch.empty(max(cap, 1), dtype=torch.int32, device=x_idx.device)
    y_val = torch.empty(max(cap, 1), dtype=vdt, device=x_idx.device)
    times = np.full(OUT, np.inf)
    stats = None
    for c in range(OUT):
        try:
            M.schedule = class_schedule(M, c, semiring)
        except Exception:   # the handle has no row form: pull unavailable
            continue
        fl = flags | (PULL_ROWWISE if (c == OUT - 1 and bfs_step) else 0)
        spmspv_run_masked(M.handle, semiring, fl, f, x_idx, x_val, mask, y_idx, y_val, cap, sync=False)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            spmspv_run_masked(M.handle, semiring, fl, f, x_idx, x_val, mask, y_idx, y_val, cap, sync=False)
        e1.record(stream)
        torch.cuda.synchronize()
        times[c] = e0.elapsed_time(e1) * 1e3 / reps
        if stats is None and c < OUT - 1:
            stats = M.last_stats()
    M.schedule = None
    return times, stats


def visited_words(level, upto: int):
    """Bitmap (int32 words) of vertices with 0 <= level <= upto."""
    import torch
    n = level.numel()
    bits = ((level >= 0) & (level <= upto)).to(torch.int64)
    pad = (-n) % 32
    if pad:
        bits = torch.cat([bits, torch.zeros(pad, dtype=torch.int64, device=level.device)])
    w = (bits.view(-1, 32) << torch.arange(32, device=level.device, dtype=torch.int64)).sum(1)
    return torch.where(w >= (1 << 31), w - (1 << 32), w).to(torch.int32)


def bfs_samples(M, nnz: int, roots, semiring: int = MIN_SELECT2ND_I32, reps: int = 3, tag: str = "",
                max_levels: int = 64) -> Samples:
    """One sample per BFS level: the frontier of level L expanded with the
    vertices of levels <= L masked, as a BFS step runs it."""
    import torch
    out = Samples()
    n = M.n
    for r in roots:
        level, _, nl = M.bfs(int(r), semiring=semiring, parents=False)
        levels = range(nl) if nl <= max_levels else np.unique(np.linspace(0, nl - 1, max_levels).astype(int))
        for L in levels:
            L = int(L)
            front = torch.nonzero(level == L).flatten().to(torch.int32)
            if front.numel() == 0:
                continue
            mask = visited_words(level, L)
            unvisited = n - int(((level >= 0) & (level <= L)).sum().item())
            flags = X_VAL_IS_INDEX if semiring == MIN_SELECT2ND_I32 else X_ALL_TRUE
            t, st = time_classes(M, semiring, front, None, flags, mask, reps=reps, bfs_step=True)
            out.add(raw_features(front.numel(), st["W"], st["maxlen"], n, nnz, unvisited), t, f"{tag}/r{r}/L{L}")
    return out


def random_samples(M, nnz: int, densities, semiring: int = PLUS_TIMES_F32, reps: int = 3, seed: int = 0,
                   tag: str = "") -> Samples:
    """Standalone multiplies with x of the given densities (uniform indices)."""
    import torch
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    out = Samples()
    n = M.n
    for d in densities:
        f = max(1, int(round(d * n)))
        idx = torch.randperm(n, generator=g)[:f].sort().values.to(torch.int32).cuda()
        val = ((torch.randint(0, 1 << 24, (f,), generator=g) + 1).float() / float(1 << 24)).cuda()
        if semiring == PLUS_TIMES_F32:
            t, st = time_classes(M, semiring, idx, val, 0, None, reps=reps)
        else:
            t, st = time_classes(M, semiring, idx, None, X_VAL_IS_INDEX, None, reps=reps)
        out.add(raw_features(f, st["W"], st["maxlen"], n, nnz, n), t, f"{tag}/d{d:g}")
    return out


# ----------------------------------------------------------------- training
def init_params(rng) -> np.ndarray:
    parts = [rng.normal(0, np.sqrt(2.0 / IN), H1 * IN), np.zeros(H1),
             rng.normal(0, np.sqrt(2.0 / H1), H2 * H1), np.zeros(H2),
             rng.normal(0, np.sqrt(1.0 / H2), OUT * H2), np.zeros(OUT)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == MLP_PARAMS
    return p


def labels(T: np.ndarray, tie: float = 0.03) -> np.ndarray:
    """Fastest class per sample; classes within `tie` of the fastest count as
    tied and the tie goes to the class that is fastest most often overall, so
    near-equal timings give consistent labels."""
    best = T.min(1, keepdims=True)
    prior = np.bincount(T.argmin(1), minlength=OUT).astype(np.float64)
    ok = T <= best * (1 + tie)
    score = np.where(ok, prior[None, :] + 1e-9 * (OUT - np.arange(OUT))[None, :], -1.0)
    return score.argmax(1).astype(np.int32)


# Scale augmentation of BFS steps: every sample taken inside a BFS (fewer
# unvisited vertices than n) also enters with its size features (f, W,
# longest column, n, unvisited) multiplied by these factors and nnz/n kept,
# with the same timings.  A BFS step's direction choice depends on ratios of
# these quantities (frontier edges against unexplored edges; the pull step
# probes only a bitmap of the frontier), so the copies carry the training
# graphs' decisions to graphs several times larger than any of them, where
# the network would otherwise extrapolate.  Standalone multiplies are not
# copied: a plus-times pull step reads a dense value array of n entries,
# which stops fitting in cache as n grows, so their choice does not carry
# over to larger graphs.
AUGMENT_SCALES = (2.0, 4.0)
SIZE_FEATURES = np.array([1.0, 1.0, 1.0, 1.0, 0.0, 1.0])


def augmented(raw: np.ndarray, times: np.ndarray, scales=AUGMENT_SCALES):
    """The samples and the scaled copies of the BFS-step samples (raw
    features, times)."""
    bfs = raw[:, 5] < raw[:, 3]
    Xs, Ts = [raw], [times]
    for sc in scales:
        Xs.append(raw[bfs] * np.where(SIZE_FEATURES > 0, sc, 1.0)[None, :])
        Ts.append(times[bfs])
    return np.concatenate(Xs), np.concatenate(Ts)


def train(samples: Samples, epochs: int = 300, lr: float = 1e-3, batch: int = 128, seed: int = 0,
          scales=AUGMENT_SCALES):
    """Adam on softmax cross-entropy towards the fastest class, on the GPU,
    over the samples and their scaled copies.  Returns (params, mean, std,
    loss history)."""
    import torch
    raw, T = augmented(samples.X, samples.T, scales)
    X = encode(raw)
    y = labels(T)
    mean = X.mean(0)
    std = X.std(0)
    std[std < 1e-3] = 1.0
    # Cost-sensitive: a sample is repeated in proportion to its best time (in
    # 100 us units, 1..16 copies), so mistakes on expensive steps weigh more.
    reps = np.clip(np.ceil(T.min(1) / 100.0), 1, 16).astype(int)
    keep = np.repeat(np.arange(T.shape[0]), reps)
    X, y = X[keep], y[keep]
    Z = ((X - mean) / std).astype(np.float32)
    rng = np.random.default_rng(seed)
    p = torch.as_tensor(init_params(rng)).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    Zd = torch.as_tensor(Z).cuda()
    yd = torch.as_tensor(y).cuda()
    N = Z.shape[0]
    step = 0
    hist = []
    for ep in range(epochs):
        order = torch.as_tensor(rng.permutation(N)).cuda()
        tot = 0.0
        for b0 in range(0, N, batch):
            sel = order[b0:b0 + batch]
            step += 1
            spmspv_mlp_train_step(p, m, v, step, lr, Zd[sel].contiguous(), yd[sel].contiguous(), loss=loss)
            tot += float(loss.item()) * sel.numel()
        hist.append(tot / N)
    return p.cpu().numpy(), mean.astype(np.float32), std.astype(np.float32), hist


def predict(params, mean, std, raw: np.ndarray) -> np.ndarray:
    import torch
    Z = ((encode(raw) - mean) / std).astype(np.float32)
    logits = torch.empty((Z.shape[0], OUT), dtype=torch.float32, device="cuda")
    spmspv_mlp_forward(torch.as_tensor(np.ascontiguousarray(params)).cuda(), torch.as_tensor(Z).cuda(), logits)
    return logits.argmax(1).cpu().numpy()


def regret(times: np.ndarray, choice: np.ndarray) -> float:
    """Sum of the chosen classes' times over the sum of the best times."""
    best = times.min(1)
    return float(times[np.arange(times.shape[0]), choice].sum() / best.sum())


def save_weights(params, mean, std, meta: Optional[dict] = None, path: str = WEIGHTS_PATH, multiply=None):
    """The BFS-step network at the top level; `multiply` = (params, mean,
    std) of the network for standalone multiplies (PageRank's steps)."""
    meta = dict(meta or {})
    meta["kernel_digest"] = kernel_digest()
    d = {"params": [float(v) for v in params], "mean": [float(v) for v in mean],
         "std": [float(v) for v in std], "meta": meta}
    if multiply is not None:
        mp, mm, ms = multiply
        d["multiply"] = {"params": [float(v) for v in mp], "mean": [float(v) for v in mm],
                         "std": [float(v) for v in ms]}
    with open(path, "w") as fh:
        json.dump(d, fh)


def load_weights(path: str = WEIGHTS_PATH, kind: str = "bfs"):
    """(params, mean, std, meta) of the BFS-step network (kind "bfs") or of
    the standalone-multiply network (kind "multiply"; the BFS one when the
    file has no second network).  The same six inputs and ten classes: a BFS
    step is a masked multiply whose pull step stops at the first frontier
    neighbour, a standalone plus-times multiply reads every stored entry in
    the pull direction, and the inputs cannot tell the two apart."""
    with open(path) as fh:
        d = json.load(fh)
    net = d["multiply"] if kind == "multiply" and "multiply" in d else d
    return (np.array(net["params"], np.float32), np.array(net["mean"], np.float32),
            np.array(net["std"], np.float32), d.get("meta", {}))
