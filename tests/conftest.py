import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU-side oracle work")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a visible device; without one they are skipped rather than failed,
    # so that `-m gpu` on a CPU-only host reports skips instead of errors.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session")
def slab_reference():
    """The slab workload (4,194,304 neurons in 10 x 10 x 2 mm, sigma 750 um) with
    FP64 oracle sums at 65,536 seeded targets plus every target within one cell of
    the p = 8 expansion level (625 um) of a corner of the slab and 8,192 seeded
    targets within that reach of an x or y face.  Computed once per session (about
    a minute and a half of CPU on 16 threads)."""
    import time

    import numpy as np

    import oracle
    import synth
    wl = synth.slab4m()
    tgt = np.nonzero(wl.a > 0)[0]
    groups = {"uniform": tgt[synth.sample_indices(tgt.size, 65536, seed=303)]}
    reach = float(max(np.ptp(wl.x), np.ptp(wl.y), np.ptp(wl.z))) / 16.0
    groups.update(synth.boundary_sample(wl, tgt, reach, 8192, seed=304))
    sel = np.unique(np.concatenate(list(groups.values())))
    t0 = time.time()
    print(f"slab reference: FP64 oracle at {sel.size} targets ...", flush=True)
    ref = oracle.attraction(wl, sel)
    print(f"slab reference: done in {time.time() - t0:.1f} s", flush=True)
    where = {g: np.searchsorted(sel, idx) for g, idx in groups.items()}
    return wl, sel, ref, where
