"""The lattice facts the paper prints (tests/golden/lattice_facts.json, each
entry with where it is printed) against the oracle's lattices and the
library's own lattice table: the temperature T0, the order of isotropy 2N
and the default Hermite truncation K."""
import json
import os
from fractions import Fraction

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
FACTS = json.load(open(os.path.join(HERE, "golden", "lattice_facts.json")))


@pytest.mark.parametrize("name", sorted(FACTS["T0"]))
def test_printed_temperature(name):
    want = Fraction(*FACTS["T0"][name]["value"])
    assert abs(oracle.lattice(name)["T0"] - float(want)) < 1e-15


@pytest.mark.parametrize("name", sorted(FACTS["two_n"]))
def test_printed_order_of_isotropy(name):
    assert oracle.lattice(name)["two_n"] == FACTS["two_n"][name]["value"]


def test_library_table_agrees_with_the_printed_facts():
    """The library's lattice descriptor (host-side, no GPU needed)."""
    from paper_2002_02503_amd import lbm

    try:
        lbm.load_library()
    except ImportError:
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    for name, fact in FACTS["two_n"].items():
        assert lbm.lattice_table(name)["two_n"] == fact["value"], name
    for name, fact in FACTS["T0"].items():
        assert abs(lbm.lattice_table(name)["T0"] - float(Fraction(*fact["value"]))) < 1e-15, name


@pytest.mark.parametrize("name", sorted(FACTS["hermite_order"]))
def test_default_hermite_order_follows_the_printed_truncation(name):
    """The oracle's default K is the printed truncation: 2N - 1 on the 2N = 4
    lattices, the u^2 terms of eq. filter-2nd on D3Q39."""
    sim = oracle.Sim(name, (2, 2, 1 if name == "D2Q9" else 2), 0.7)
    assert sim.K == FACTS["hermite_order"][name]["value"]


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(FACTS["hermite_order"]))
def test_library_default_hermite_order(name):
    from paper_2002_02503_amd import lbm

    with lbm.Simulation(name, (4, 4, 1 if name == "D2Q9" else 4), 0.7) as sim:
        assert sim.info()["K"] == FACTS["hermite_order"][name]["value"]
