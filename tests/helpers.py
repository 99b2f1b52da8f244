"""Shared helpers of the test-suite: input marshalling for both sides and the
tolerance rules.  Nothing here computes any part of the docking method."""
import numpy as np


def box32(box):
    """The box as the library sees it (float32 fields), in the oracle's dict form."""
    return {"centre": np.asarray(box["centre"], dtype=np.float32).astype(np.float64),
            "size": np.broadcast_to(np.asarray(box["size"], dtype=np.float32), (3,)).astype(np.float64),
            "spacing": float(np.float32(box["spacing"]))}


def random_poses(n_tors, n, lo, hi, rng, margin=0.0):
    """float32 poses [p(3), q(4), theta]: position uniform in [lo - margin, hi + margin]."""
    P = np.zeros((n, 7 + n_tors), dtype=np.float32)
    P[:, :3] = rng.uniform(lo - margin, hi + margin, size=(n, 3))
    q = rng.normal(size=(n, 4))
    P[:, 3:7] = q / np.linalg.norm(q, axis=1, keepdims=True)
    P[:, 7:] = rng.uniform(-np.pi, np.pi, size=(n, n_tors))
    return P


def rmsd(a, b):
    return float(np.sqrt(np.mean(np.sum((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2, axis=-1))))
