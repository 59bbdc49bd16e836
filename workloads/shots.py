"""Source and receiver positions and the batched shot list.

* Single-shot source: an explosive point source at (5.1, 4.9, 9.1), a generic
  position in the top layer of the [0, 10]^3 box.
* Receivers: 64 points on the free surface z = 10 at
  (0.662 + 1.25 i, 0.584 + 1.25 j), i, j = 0..7.  The offsets keep them off
  the cell diagonals of meshes with 16 and 24 cells per side.
* Batched shots: 32 source positions drawn uniformly in
  [0.5, 9.5] x [0.5, 9.5] x [5.0, 9.5] and 32 lengths drawn uniformly from
  500..2000 steps, both from one generator seeded 11052.
"""

import numpy as np

SHOT_SEED = 11052
ricker_f0 = 1.0


def default_source():
    return np.array([5.1, 4.9, 9.1], dtype=np.float64)


def default_receivers(nx=8, z=10.0):
    i, j = np.meshgrid(np.arange(nx), np.arange(nx), indexing="ij")
    x = 0.662 + 1.25 * i.ravel()
    y = 0.584 + 1.25 * j.ravel()
    return np.stack([x, y, np.full_like(x, z)], axis=1)


def batched_shots(nshots=32, min_steps=500, max_steps=2000):
    rng = np.random.default_rng(SHOT_SEED)
    pos = rng.uniform([0.5, 0.5, 5.0], [9.5, 9.5, 9.5], (nshots, 3))
    lengths = rng.integers(min_steps, max_steps + 1, nshots)
    return pos, lengths.astype(np.int64)
