"""The oracle on the constructed edge box (``tests/edge_cases.py``): the closed-form
outcomes of eq. (detect1/detect2) hold for pairs embedded in a dense polydisperse box
(a contact exactly at dt kept and one ulp later rejected, a tangent contact at its
closed-form time, touching, overlapping, b = 0 and a = 0 pairs without a collision,
exact three-sphere ties, inside the box, through the periodic face and across the
split's two layers, going to the smaller index), and the grazing and slow-approach
families fall on both sides of the contact distance and of the end of the step."""
import math

import oracle
from tests.edge_cases import DT, check_designed as _check_designed, edge_box


def test_oracle_edge_box_designed_outcomes():
    box, groups = edge_box()
    res = oracle.step(box)
    _check_designed(groups, res.partner, res.tcoll)
    b = box.copy()
    b.dt = math.nextafter(DT, 0.0)
    res = oracle.step(b)
    _check_designed(groups, res.partner, res.tcoll, dt=b.dt)
    g = next(g for g in groups if g.name == "t_eq_dt")
    assert res.partner[g.first] == -1
