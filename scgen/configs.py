"""The five benchmark workloads as seeded synthetic subdomain batches.

  1  one 2D heat subdomain, 16x16 Q1 elements on the unit square (289 DOFs),
     64 multipliers (all boundary nodes)
  2  1024 identical 3D heat subdomains, 12^3 hex8 elements on the unit cube
     (2197 DOFs), 866 multipliers (all surface nodes); own signs each
  3  512 uneven 3D elasticity boxes, elements per axis drawn from U{6..16}
     independently per axis, h = 1/16, multipliers = all surface DOFs
  4  the batch of workload 3 (mixed precision + dual PCPG)
  5  64 elasticity boxes of 20^3 hex8 elements (27783 DOFs), h = 1/20,
     multipliers per face (6 * 21^2 * 3 = 7938; edge and corner DOFs repeated)
Workload k uses base seed BASE_SEED + k; subdomain i draws its signs from the
SplitMix64 stream seeded with base + i * 0x9E3779B97F4A7C15; the per-axis
element counts of workloads 3/4 come from the stream seeded with
base ^ SIZE_SALT, three outputs per subdomain (x, y, z), count = 6 + out % 11.
"""
from typing import List, Optional

import numpy as np

from .mesh import Subdomain, box_subdomain
from .rng import splitmix64, stream_seed

BASE_SEED = 250921037
SIZE_SALT = 0xD1B54A32D192ED03

CONFIG_NAMES = {
    1: "heat2d_q1_16x16_x1",
    2: "heat3d_hex8_12cube_x1024",
    3: "elast3d_hex8_uneven6to16_x512_fp64",
    4: "elast3d_hex8_uneven6to16_x512_mixed_pcpg100",
    5: "elast3d_hex8_20cube_perface_x64",
}

CONFIG_BATCH = {1: 1, 2: 1024, 3: 512, 4: 512, 5: 64}


# The paper's own workloads (Sec. 4): heat transfer on P1 triangles (2D) and
# tetrahedra (3D), subdomain sizes from its figures (nodes per side), batches
# of about the paper's total problem size (8.4 M unknowns in 2D, 1.1 M in 3D)
# between 16 and 512 subdomains.  Subdomain i of the (dim, nodes) batch draws
# its signs from the stream seeded with
# stream_seed(BASE_SEED + 100 * dim + nodes, i).
PAPER_NODES = {2: (7, 33, 129, 257, 513, 725), 3: (4, 9, 14, 21, 33, 41)}
PAPER_TOTAL_DOFS = {2: 8.4e6, 3: 1.1e6}


def paper_batch_size(dim: int, nodes: int) -> int:
    n = nodes ** dim
    return int(min(512, max(16, round(PAPER_TOTAL_DOFS[dim] / n))))


def paper_subdomains(dim: int, nodes: int, count: Optional[int] = None, start: int = 0) -> List[Subdomain]:
    """P1 heat subdomains (triangles for dim 2, tetrahedra for dim 3) with
    `nodes` nodes per side on the unit square / cube, multipliers on every
    boundary node; subdomains start .. start + count - 1 of the batch."""
    from .simplex import simplex_subdomain
    if count is None:
        count = paper_batch_size(dim, nodes) - start
    base = BASE_SEED + 100 * dim + nodes
    out = [simplex_subdomain(dim, nodes - 1, stream_seed(base, i)) for i in range(start, start + count)]
    for s in out:
        s.meta["paper"] = (dim, nodes)
    return out


def config_description(cfg: int) -> str:
    return CONFIG_NAMES[cfg]


def uneven_sizes(base_seed: int, count: int, start: int = 0) -> np.ndarray:
    z = splitmix64(base_seed ^ SIZE_SALT, 3 * count, start=3 * start)
    return (6 + (z % np.uint64(11)).astype(np.int64)).reshape(count, 3)


def config_subdomains(cfg: int, count: Optional[int] = None, start: int = 0) -> List[Subdomain]:
    """Subdomains start .. start+count-1 of workload `cfg` (default: the whole batch)."""
    total = CONFIG_BATCH[cfg]
    if count is None:
        count = total - start
    base = BASE_SEED + cfg
    out = []
    if cfg == 1:
        for i in range(start, start + count):
            out.append(box_subdomain("heat", (16, 16), 1.0 / 16, stream_seed(base, i)))
    elif cfg == 2:
        for i in range(start, start + count):
            out.append(box_subdomain("heat", (12, 12, 12), 1.0 / 12, stream_seed(base, i)))
    elif cfg in (3, 4):
        base = BASE_SEED + 3          # workload 4 reuses the batch of workload 3
        sizes = uneven_sizes(base, count, start)
        for k, i in enumerate(range(start, start + count)):
            out.append(box_subdomain("elasticity", tuple(int(v) for v in sizes[k]), 1.0 / 16,
                                     stream_seed(base, i)))
    elif cfg == 5:
        for i in range(start, start + count):
            out.append(box_subdomain("elasticity", (20, 20, 20), 1.0 / 20, stream_seed(base, i),
                                     gluing="per_face"))
    else:
        raise ValueError(cfg)
    for s in out:
        s.meta["config"] = cfg
    return out
