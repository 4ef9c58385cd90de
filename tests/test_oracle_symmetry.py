"""Fine cells at offsets +d and -d from a coarse centre have conjugate fine
phasors (eq. (44): the fine phase is linear in the offsets, and the offsets
run over [-R/2, R - R/2) on every axis).  The conjugate-pair form of the fine
search rests on this; cells with an offset of -R/2 on some axis (even R) have
no partner."""
import numpy as np
import pytest

from cases import CASES
from oracle import transforms as OT
from oracle.grid import Axis, Radar, make_grid


def _grid(name):
    c = CASES[name]
    return make_grid(Radar(c["fc"], c["fs"], c["prf"]), c["M"], c["N"], c["order"],
                     [Axis(*a) for a in c["axes"]])


@pytest.mark.parametrize("name", list(CASES))
def test_fine_phasors_conjugate_in_pairs(name):
    g = _grid(name)
    F = OT.fine_matrix(g)
    fo = g.fine_offsets()
    index = {tuple(o): i for i, o in enumerate(fo)}
    unpaired = 0
    for i, o in enumerate(fo):
        j = index.get(tuple(-o))
        if j is None:
            assert (o[:g.order] == -g.h).any() and g.R % 2 == 0, (name, o)
            unpaired += 1
            continue
        assert np.abs(F[:, j] - np.conj(F[:, i])).max() <= 1e-12, (name, o)
    # an odd R pairs every cell; an even R leaves R^P - (R - 1)^P alone
    assert unpaired == (g.R ** g.order - (g.R - 1) ** g.order if g.R % 2 == 0 else 0)
