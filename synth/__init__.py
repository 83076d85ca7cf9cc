"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module only draws random numbers and arranges them into arrays.  It holds
none of the method's arithmetic, so both the oracle and the HIP path may use it
without sharing any computation.

Every workload stands in for the paper's own neuron placements, which are not
public (the evaluation section uses networks of an existing simulator).  The
draws follow one fixed order per workload: positions (float64, then rounded to
float32), then vacant axon counts, then vacant dendrite counts, each count an
integer in 0..5.

Units: micrometres for positions and for sigma.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2301105700


@dataclass
class Workload:
    """One attraction-sum problem.

    x, y, z   float32 positions of all neurons (one union point set)
    a         float32 vacant axon counts; a neuron with a > 0 is a target
    w         float32 vacant dendrite counts; the weight of the neuron as a source
    sigma     kernel width of exp(-d^2 / sigma^2)
    p         expansion terms per axis
    leaf_max  octree leaf capacity
    """
    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    a: np.ndarray
    w: np.ndarray
    sigma: float
    p: int = 8
    leaf_max: int = 64
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def is_target(self) -> np.ndarray:
        return (self.a > 0).astype(np.uint8)

    def pos64(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1).astype(np.float64)


def _counts(rng: np.random.Generator, n: int) -> tuple[np.ndarray, np.ndarray]:
    a = rng.integers(0, 6, size=n).astype(np.float32)
    w = rng.integers(0, 6, size=n).astype(np.float32)
    return a, w


def _finish(name, pos64, rng, sigma, p=8, leaf_max=64, **extra) -> Workload:
    pos = pos64.astype(np.float32)
    a, w = _counts(rng, pos.shape[0])
    return Workload(name, np.ascontiguousarray(pos[:, 0]), np.ascontiguousarray(pos[:, 1]),
                    np.ascontiguousarray(pos[:, 2]), a, w, float(sigma), p, leaf_max, dict(extra))


def uniform_box(n: int, extent=(1000.0, 1000.0, 1000.0), sigma=100.0, seed=0, p=8,
                leaf_max=64, name=None) -> Workload:
    """n neurons uniform in [0, ex) x [0, ey) x [0, ez)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    ext = np.asarray(extent, dtype=np.float64)
    pos = rng.random((n, 3)) * ext
    return _finish(name or f"uniform{n}", pos, rng, sigma, p, leaf_max)


def blobs(n_blobs: int, per_blob: int, extent=4000.0, std=50.0, sigma=200.0, seed=0, p=8,
          leaf_max=64, name=None) -> Workload:
    """Gaussian clusters: centres uniform in a cube, per-axis normal offsets, no clipping."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    centres = rng.random((n_blobs, 3)) * extent
    off = rng.normal(0.0, std, size=(n_blobs, per_blob, 3))
    pos = (centres[:, None, :] + off).reshape(-1, 3)
    return _finish(name or f"blobs{n_blobs}x{per_blob}", pos, rng, sigma, p, leaf_max)


def _workload(idx: int, scale: float = 1.0) -> Workload:
    """The workloads below by their stream number (which fixes their seed).

    scale < 1 shrinks the neuron counts (and nothing else) for quick tests.
    1: 4,096 neurons uniform in a 1000 um cube, sigma 100, p 8
    2: 262,144 neurons in 64 Gaussian blobs (centres uniform in a 4 mm cube,
       per-axis std 50 um), sigma 200, p 8
    3: 4,194,304 neurons uniform in a 10 x 10 x 2 mm slab, sigma 750, p 8
    4: 1,048,576 weighted sources and 1,048,576 separate targets uniform in a
       2 mm cube, sigma 200 (sources have w in 0..5 and a = 0, targets w = 0 and
       a = 1); extra["g"] holds upstream gradients drawn from U(0.5, 1.5)
    5: the 256 populations of populations()
    """
    seed = SEED_BASE + idx
    rng = np.random.default_rng(np.random.PCG64(seed))
    if idx == 1:
        n = max(1, int(round(4096 * scale)))
        pos = rng.random((n, 3)) * 1000.0
        return _finish("uniform4k", pos, rng, 100.0)
    if idx == 2:
        per = max(1, int(round(4096 * scale)))
        centres = rng.random((64, 3)) * 4000.0
        off = rng.normal(0.0, 50.0, size=(64, per, 3))
        pos = (centres[:, None, :] + off).reshape(-1, 3)
        return _finish("blobs262k", pos, rng, 200.0)
    if idx == 3:
        n = max(1, int(round(4194304 * scale)))
        pos = rng.random((n, 3)) * np.array([10000.0, 10000.0, 2000.0])
        return _finish("slab4M", pos, rng, 750.0)
    if idx == 4:
        m = max(1, int(round(1048576 * scale)))
        src = rng.random((m, 3)) * 2000.0
        tgt = rng.random((m, 3)) * 2000.0
        w = rng.integers(0, 6, size=m).astype(np.float32)
        g = rng.uniform(0.5, 1.5, size=m).astype(np.float32)
        pos = np.concatenate([src, tgt]).astype(np.float32)
        a = np.concatenate([np.zeros(m, np.float32), np.ones(m, np.float32)])
        ww = np.concatenate([w, np.zeros(m, np.float32)])
        return Workload("sources_targets_1M", np.ascontiguousarray(pos[:, 0]),
                        np.ascontiguousarray(pos[:, 1]), np.ascontiguousarray(pos[:, 2]),
                        a, ww, 200.0, 8, 64, {"g": np.concatenate([np.zeros(m, np.float32), g])})
    raise ValueError(f"unknown workload {idx}")


def uniform4k(scale: float = 1.0) -> Workload:
    """4,096 neurons uniform in a 1000 um cube, sigma 100 um."""
    return _workload(1, scale)


def blobs262k(scale: float = 1.0) -> Workload:
    """262,144 neurons in 64 Gaussian blobs (4 mm cube, std 50 um), sigma 200 um."""
    return _workload(2, scale)


def slab4m(scale: float = 1.0) -> Workload:
    """4,194,304 neurons uniform in a 10 x 10 x 2 mm slab, sigma 750 um."""
    return _workload(3, scale)


def sources_targets_1m(scale: float = 1.0) -> Workload:
    """1,048,576 sources and 1,048,576 targets uniform in a 2 mm cube, sigma 200 um,
    with upstream gradients in extra["g"]."""
    return _workload(4, scale)


def populations(count: int = 256, scale: float = 1.0, seed: int | None = None) -> list[Workload]:
    """Independent populations with log-uniform sizes in [1024, 65536]
    and log-uniform sigma in [50, 300] um, each uniform in its own 1 mm cube."""
    rng = np.random.default_rng(np.random.PCG64(SEED_BASE + 5 if seed is None else seed))
    sizes = np.rint(np.exp(rng.uniform(math.log(1024), math.log(65536), size=count))).astype(np.int64)
    sigmas = np.exp(rng.uniform(math.log(50.0), math.log(300.0), size=count))
    out = []
    for k in range(count):
        n = max(1, int(round(int(sizes[k]) * scale)))
        pos = rng.random((n, 3)) * 1000.0
        out.append(_finish(f"population{k}", pos, rng, float(sigmas[k])))
    return out


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices from range(n), sorted (seeded, without replacement)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def uniforms(k: int, seed: int) -> np.ndarray:
    """k float32 draws from [0, 1) for proportional child choice."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    return rng.random(k, dtype=np.float32)


def boundary_sample(wl: Workload, targets: np.ndarray, reach: float, k_face: int, seed: int) -> dict:
    """Targets near the edges of the point cloud's bounding box, where the sums
    are smallest: every target within `reach` of one of the box's eight corners,
    and k_face targets (seeded) among the others within `reach` of an x or y face.
    Returns {"corner": indices, "face": indices} (input indices, sorted)."""
    pos = np.stack([wl.x, wl.y, wl.z], axis=1).astype(np.float64)[targets]
    lo = np.array([wl.x.min(), wl.y.min(), wl.z.min()], np.float64)
    hi = np.array([wl.x.max(), wl.y.max(), wl.z.max()], np.float64)
    corner = np.zeros(targets.size, bool)
    for c in range(8):
        vert = np.where([(c >> 2) & 1, (c >> 1) & 1, c & 1], hi, lo)
        corner |= np.sum((pos - vert) ** 2, axis=1) <= reach * reach
    edge = np.minimum(np.minimum(pos[:, 0] - lo[0], hi[0] - pos[:, 0]),
                      np.minimum(pos[:, 1] - lo[1], hi[1] - pos[:, 1]))
    face_pool = np.nonzero((edge <= reach) & ~corner)[0]
    face = face_pool[sample_indices(face_pool.size, k_face, seed)]
    return {"corner": np.sort(targets[corner]), "face": np.sort(targets[face])}
