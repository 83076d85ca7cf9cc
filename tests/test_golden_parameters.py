"""The workloads use the parameters the paper prints (tests/golden/paper_parameters.txt)."""
import synth
from tests.helpers import paper_parameters


def test_fixture_complete():
    g = paper_parameters()
    assert set(g) == {"sigma_um", "c1", "c2"}
    assert g["c1"] == g["c2"]


def test_slab_uses_the_papers_sigma():
    """The 4M-neuron slab is the paper's setting: sigma 750 um (model parameter table)."""
    g = paper_parameters()
    assert synth.slab4m(0.01).sigma == g["sigma_um"]
