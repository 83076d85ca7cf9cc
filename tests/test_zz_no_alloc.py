"""msp_fgt_forward_noalloc (per-call buffers in the library's fixed per-device
scratch, no allocation) gives the bits of msp_fgt_forward, on two calls in a row
with the second on a smaller input, on both routes; a call that needs more than
the scratch holds is refused before any work."""
import numpy as np
import pytest

import synth
from tests.helpers import to_dev

pytestmark = pytest.mark.gpu


def _pair(wl, route, **kw):
    import paper_2301_10570_amd as msp
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max)
    ref = tree.forward(d["w"], d["tgt"], sigma=wl.sigma, p=wl.p, route=route, **kw).cpu().numpy()
    return tree, d, ref


@pytest.mark.parametrize("route", ["fgt", "direct"])
def test_noalloc_matches_forward_on_two_calls(route):
    import torch
    big = synth.slab4m(0.25) if route == "fgt" else synth.blobs262k()
    small = synth.uniform4k()
    print(f"no-alloc forward, route={route}: {big.n} then {small.n} points", flush=True)
    t_big, d_big, ref_big = _pair(big, route)
    t_small, d_small, ref_small = _pair(small, route)
    # the first call leaves the larger problem's data in the scratch; the second,
    # smaller call must not depend on it
    out_big = torch.full_like(d_big["w"], float("nan"))
    t_big.forward_noalloc(d_big["w"], d_big["tgt"], sigma=big.sigma, p=big.p, route=route, out=out_big)
    out_small = torch.full_like(d_small["w"], float("nan"))
    t_small.forward_noalloc(d_small["w"], d_small["tgt"], sigma=small.sigma, p=small.p, route=route,
                            out=out_small)
    got_big = out_big.cpu().numpy()
    got_small = out_small.cpu().numpy()
    assert np.array_equal(got_big.view(np.uint32), ref_big.view(np.uint32))
    assert np.array_equal(got_small.view(np.uint32), ref_small.view(np.uint32))
    # and the larger one again after the smaller one
    t_big.forward_noalloc(d_big["w"], d_big["tgt"], sigma=big.sigma, p=big.p, route=route, out=out_big)
    assert np.array_equal(out_big.cpu().numpy().view(np.uint32), ref_big.view(np.uint32))


def test_noalloc_refuses_beyond_its_scratch():
    import paper_2301_10570_amd as msp
    wl = synth.slab4m(0.25)
    d = to_dev(wl)
    tree = msp.build_tree(d["x"], d["y"], d["z"], leaf_max=wl.leaf_max)
    # p = 16 at level 6: about 0.9 GB per expansion grid
    need = tree.forward_query(wl.sigma, p=16, level=6, route="fgt")
    assert need > 64 << 20
    with pytest.raises(msp.MspError) as e:
        tree.forward_noalloc(d["w"], d["tgt"], sigma=wl.sigma, p=16, level=6, route="fgt")
    assert e.value.code == msp.MSP_ENOSPC
    assert "scratch" in str(e.value)
