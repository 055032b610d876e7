"""The paper's fixed-opacity single-step tests (Sections 3.3, 3.4, Table
'escape') on the oracle.

The glass initial conditions are not available; jittered lattices with the
same spacings stand in for them (`scenes.source_features_scene`,
`scenes.two_sources_cloud_scene`).  Pins:
  * exact: a lone source in a uniform alpha = 1 medium lets e^-2 = 13.53% of
    its flux reach r = 2 (the table's 'Exact (no clouds)' row); the method's
    own discretisation (beam directions, p-p columns of discrete elements)
    stays within 6% of it;
  * loose: the escape fractions and covering factors of TREVR2 with
    transmission averaging and with linear absorption averaging are compared
    with the table's printed values (escape within 10% relative, covering
    within 0.12), and the qualitative findings are asserted: linear averaging
    loses most of the flux of the two-sources test once the sources and the
    cloud merge into one cell, transmission averaging does not; the wall's
    shadow is too wide with either, wider with linear averaging."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2310_15235_amd import scenes
from tests.escape_metrics import escape_covering

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TABLE = {(r["test"], r["method"]): r
         for r in json.load(open(os.path.join(GOLD, "escape_table.json")))["rows"]}


def _run(sc):
    act = scenes.shell_active(sc)
    J, c = oracle.OracleTree(sc).compute_J(act)
    return escape_covering(sc, J, act), act, J


def test_lone_source_escape_is_e_minus_2():
    g = json.load(open(os.path.join(GOLD, "escape_closed_form.json")))
    sc = scenes.source_features_scene("none")
    (esc, cov), act, J = _run(sc)
    exact = np.exp(-g["alpha"] * g["radius"])
    assert 100 * exact == pytest.approx(g["escape_percent"], abs=0.005)
    assert esc == pytest.approx(exact, rel=0.06)
    assert cov == 0.0
    assert act.sum() > 10000


MAKERS = {
    "source+clouds": lambda avg: scenes.source_features_scene("clouds", avg=avg),
    "source+wall": lambda avg: scenes.source_features_scene("wall", avg=avg),
    "two sources+cloud": lambda avg: scenes.two_sources_cloud_scene(avg=avg),
}


@pytest.mark.parametrize("test", list(MAKERS))
@pytest.mark.parametrize("avg", [False, True], ids=["transmission", "absorption_average"])
def test_escape_table_loose(test, avg):
    (esc, cov), _, _ = _run(MAKERS[test](avg))
    row = TABLE[(test, "absorption_average" if avg else "trevr2")]
    assert 100 * esc == pytest.approx(row["escape_percent"], rel=0.10), (test, avg, esc, cov)
    assert cov == pytest.approx(row["covering"], abs=0.12), (test, avg, esc, cov)


def test_linear_average_catastrophe_and_wall_shadow():
    """Section 3.3: with linear absorption averaging the two sources and the
    dense cloud merge into one opaque cell and most of the flux is lost;
    transmission averaging keeps most of it.  Section 3.4.2: both averages
    overestimate the wall's shadow, linear averaging more."""
    (e_t, _), _, _ = _run(MAKERS["two sources+cloud"](False))
    (e_a, c_a), _, _ = _run(MAKERS["two sources+cloud"](True))
    assert e_t > 0.85 and e_a < 0.5 and c_a > 0.4
    (w_t, wc_t), _, _ = _run(MAKERS["source+wall"](False))
    (w_a, wc_a), _, _ = _run(MAKERS["source+wall"](True))
    exact = TABLE[("source+wall", "exact")]
    assert w_a < w_t < exact["escape_percent"] / 100
    assert exact["covering"] < wc_t < wc_a


@pytest.mark.parametrize("test", ["source+clouds", "source+wall"])
def test_directed_rays_table_loose(test):
    """Sections 3.4.1-3.4.2, the 'Directed' rows: aiming each bucket's ray
    at the source moves the escape fraction toward the exact value (the wall
    test: 5.42% -> 6.16% in the table, exact 7.61%)."""
    sc = MAKERS[test](False)
    (e0, c0), _, _ = _run(sc)
    (ed, cd), _, _ = _run(sc.with_(directed=tuple(sc.meta["src_pos"][0])))
    row = TABLE[(test, "directed")]
    assert 100 * ed == pytest.approx(row["escape_percent"], rel=0.10), (test, ed, cd)
    assert cd == pytest.approx(row["covering"], abs=0.12), (test, ed, cd)
    exact = TABLE[(test, "exact")]["escape_percent"] / 100
    assert abs(ed - exact) < abs(e0 - exact)


@pytest.mark.parametrize("test", list(MAKERS))
def test_complex_source_table_loose(test):
    """Section 2.7 and the 'Complex Source' rows of the escape table: the
    per-direction absorption around merged sources moves the escape
    fraction of every test toward the exact value (or past TREVR2's)."""
    sc = MAKERS[test](False)
    (e0, _), _, _ = _run(sc)
    (ec, cc), _, _ = _run(sc.with_(complex_source=True))
    row = TABLE[(test, "complex_source")]
    assert 100 * ec == pytest.approx(row["escape_percent"], rel=0.12), (test, ec, cc)
    assert cc == pytest.approx(row["covering"], abs=0.12), (test, ec, cc)
    if test != "two sources+cloud":
        exact = TABLE[(test, "exact")]["escape_percent"] / 100
        assert abs(ec - exact) < abs(e0 - exact)
    else:
        assert ec > e0
