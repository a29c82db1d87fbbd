"""Shared test inputs: adversarial clouds for nearest-neighbour selection and
pose-error helpers.  Inputs only: no registration arithmetic here."""
import math

import numpy as np


def adversarial_sets():
    """(name, src, tgt, r) tuples that stress the selection rule."""
    rng = np.random.default_rng(3)
    sets = []
    tgt = rng.uniform(0, 1, (300, 3)).astype(np.float32)
    src = rng.uniform(-0.1, 1.1, (200, 3)).astype(np.float32)
    sets.append(("random", src, tgt, 0.08))
    base = rng.uniform(0, 1, (40, 3)).astype(np.float32)
    tgt = np.concatenate([base, base, base[::-1]])
    src = (base + rng.normal(0, 0.01, base.shape)).astype(np.float32)
    sets.append(("duplicates", src, tgt, 0.05))
    src = np.array([[0.5, 0.5, 0.5], [0.25, 0.25, 0.25]], np.float32)
    tgt = np.array([[0.5 + 0.125, 0.5, 0.5], [0.5, 0.5 - 0.125, 0.5],
                    [0.25, 0.25, 0.25 + 0.125 + 2**-20]], np.float32)
    sets.append(("boundary", src, tgt, 0.125))
    tgt = rng.uniform(0, 1, (100, 3)).astype(np.float32)
    src = rng.uniform(5, 6, (50, 3)).astype(np.float32)
    sets.append(("outside", src, tgt, 0.1))
    tgt = rng.uniform(0, 0.01, (150, 3)).astype(np.float32)
    src = rng.uniform(0, 0.01, (60, 3)).astype(np.float32)
    sets.append(("one_cell", src, tgt, 0.05))
    tgt = rng.uniform(0, 1, (200, 3)).astype(np.float32)
    src = rng.uniform(0, 1, (100, 3)).astype(np.float32)
    sets.append(("r_small", src, tgt, 0.005))
    sets.append(("r_large", src, tgt, 3.0))
    # points sitting exactly on cell faces of a grid with edge ~r
    g = np.arange(0.0, 1.0, 0.0625, dtype=np.float32)
    tgt = np.stack(np.meshgrid(g, g, g[:4], indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    src = (tgt[::7] + np.float32(0.03125)).astype(np.float32)
    sets.append(("lattice_faces", src, tgt, 0.0625))
    return sets


def pose_error(Ta, Tb):
    """(rotation angle between the two rotations in rad, translation distance)."""
    dR = np.linalg.norm(Ta[:3, :3] - Tb[:3, :3])
    ang = 2.0 * math.asin(min(1.0, dR / (2.0 * math.sqrt(2.0))))
    return ang, float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3]))
