"""Shared test helpers (no method arithmetic)."""
import numpy as np


def to_dev(wl):
    import torch
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return {"x": t(wl.x), "y": t(wl.y), "z": t(wl.z), "w": t(wl.w),
            "tgt": t((wl.a > 0).astype(np.uint8))}


def rel_err(u, ref):
    u = np.asarray(u, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(u - ref) / np.abs(ref)


def paper_parameters():
    """name -> value of tests/golden/paper_parameters.txt (values the paper prints)."""
    import os
    out = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            name, value = line.split()[:2]
            out[name] = float(value)
    return out
