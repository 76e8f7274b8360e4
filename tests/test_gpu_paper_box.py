"""The paper's own geometry (Results section) at zero and strong shear, as a
physics regression of the whole step: after a short start-up, the ring
average of S(q) at rest has its minimum near the first-shell wavenumber
q lambda = 2.3 that the paper reports, and the intensity at small q in the
flow-gradient plane is several times larger at kappa tau = 0.5 than at
rest (the paper reports about 20x after its longer runs), and the
neighbours under shear sit more often in quadrants 2 and 4 of the
flow-gradient plane than in 1 and 3.  Seeds are fixed
and the GPU path is deterministic, so the numbers are reproducible; the
bounds leave room for changes of summation order."""
import pytest

from paper_1808_06381_amd import paper_runs

pytestmark = pytest.mark.gpu


def test_paper_box_structure_and_shear_growth():
    res = paper_runs.run(steps=3000, discard=1000, every=100, noise="paper", shears=(0.0, 0.5))
    assert res["samples"] == 20
    assert 1.9 <= res["zero_shear_min_q"] <= 2.7
    assert res["small_q_window_growth"][1] > 3.0
    # the pair correlation skewed backwards under shear: more neighbours in
    # quadrants 2 and 4 of the flow-gradient plane, none preferred at rest
    assert abs(res["quadrant_asymmetry"][0]) < 0.005
    assert res["quadrant_asymmetry"][1] > 0.01
    # the velocity correlation at alpha = 4 decays but persists over several lambda
    vv0 = res["vv_corr"][0]
    assert vv0[0] > 0.5 and 0.05 < vv0[10] < vv0[0] and vv0[-1] < 0.05
