"""The paper's fixed-opacity tests (Sections 3.3, 3.4) on the HIP path: J on
the measuring shell against the oracle element by element (1e-4, counters
exact), with transmission averaging and with linear absorption averaging,
and the escape fractions and covering factors that follow from it."""
import numpy as np
import pytest

import oracle
from paper_2310_15235_amd import scenes
from tests.escape_metrics import escape_covering
from tests.test_gpu_parity import compare_J

pytestmark = pytest.mark.gpu

MAKERS = {
    "source+none": lambda avg: scenes.source_features_scene("none", avg=avg),
    "source+clouds": lambda avg: scenes.source_features_scene("clouds", avg=avg),
    "source+wall": lambda avg: scenes.source_features_scene("wall", avg=avg),
    "two sources+cloud": lambda avg: scenes.two_sources_cloud_scene(avg=avg),
}


@pytest.mark.parametrize("test", list(MAKERS))
@pytest.mark.parametrize("avg", [False, True], ids=["transmission", "absorption_average"])
def test_escape_scene_parity(test, avg):
    import torch
    from paper_2310_15235_amd import api
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sc = MAKERS[test](avg)
    act = scenes.shell_active(sc)
    print(f"[escape] {sc.name}: n {sc.n}, shell {int(act.sum())}", flush=True)
    compare_J(sc, active=act)
    Jg, _ = api.compute_J(sc, active=act)
    Jo, _ = oracle.OracleTree(sc).compute_J(act)
    eg, cg = escape_covering(sc, Jg, act)
    eo, co = escape_covering(sc, Jo, act)
    assert eg == pytest.approx(eo, rel=1e-5)
    assert cg == co
