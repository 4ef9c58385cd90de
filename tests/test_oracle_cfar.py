"""Pins of the oracle's cell-averaging CFAR (a detector beside the paper's
LRT threshold): a hand-worked map, the textbook false-alarm rate for
exponential power, scale invariance and the edges."""
import numpy as np

from oracle import detect as OD


def test_hand_worked_map():
    # rows 0..8 of one cell; guard 1, train 2: training rows of r are
    # r-3, r-2, r+2, r+3 inside [0, 9)
    P = np.array([[1, 1, 1, 1, 10, 1, 1, 1, 2]], dtype=np.float32)
    # alpha 3: row 4 (10 vs mean of rows 1, 2, 6, 7 = 1) only; row 8 has
    # training rows 5, 6 only (mean 1), 2 < 3
    assert np.nonzero(OD.ca_cfar(P, 1, 2, 3.0)[0])[0].tolist() == [4]
    # alpha 1.5: row 8 now passes (2 > 1.5); row 5 (training 2, 3, 7, 8:
    # mean 1.25) does not (1 < 1.875); row 6 (3, 4, 8: mean 13/3) does not
    assert np.nonzero(OD.ca_cfar(P, 1, 2, 1.5)[0])[0].tolist() == [4, 8]


def test_no_training_entry_no_detection():
    P = np.array([[5.0], [7.0]])
    assert not OD.ca_cfar(P, 0, 3, 0.0).any()
    # two rows, guard 1: the other row is a guard row
    P = np.array([[1.0, 100.0]])
    assert not OD.ca_cfar(P, 1, 4, 0.5).any()
    assert OD.ca_cfar(P, 0, 4, 0.5)[0].tolist() == [False, True]


def test_exponential_false_alarm_rate():
    """i.i.d. exponential power: P_FA = (1 + alpha/N)^-N for N training
    entries (interior rows)."""
    rng = np.random.default_rng(77)
    n, rows, guard, train = 2000, 400, 2, 8
    P = rng.exponential(1.0, size=(n, rows))
    pfa = 1e-2
    alpha = OD.cfar_alpha(2 * train, pfa)
    hit = OD.ca_cfar(P, guard, train, alpha)
    inner = hit[:, guard + train: rows - guard - train]
    est = inner.mean()
    sd = np.sqrt(pfa * (1 - pfa) / inner.size)
    assert abs(est - pfa) < 5 * sd, (est, pfa, sd)


def test_scale_invariance_and_cells_independent():
    rng = np.random.default_rng(5)
    P = rng.exponential(1.0, size=(6, 50)).astype(np.float32)
    h = OD.ca_cfar(P, 1, 4, 2.5)
    assert np.array_equal(h, OD.ca_cfar(P * np.float32(8.0), 1, 4, 2.5))
    # each cell is decided from its own rows only
    Q = P.copy()
    Q[3] *= 1000.0
    h2 = OD.ca_cfar(Q, 1, 4, 2.5)
    assert np.array_equal(np.delete(h, 3, 0), np.delete(h2, 3, 0))
