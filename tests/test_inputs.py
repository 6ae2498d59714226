"""CPU checks of the input generators against numbers the paper or the literature fix."""
import math

import numpy as np
import pytest

from paper_1511_00242_amd import inputs as I


def test_tanh_mesh_ratio_and_cavity_parameters():
    w = I.cavity(256)
    d = np.diff(w.xf)
    assert np.max(np.maximum(d[1:] / d[:-1], d[:-1] / d[1:])) == pytest.approx(1.05, abs=1e-9)
    assert w.tau == pytest.approx(3e-4) and w.meta["re"] == 1000.0


def test_boundary_layer_paper_mesh_matches_the_printed_stations():
    """Sec. 3.3: Delta x_min = 0.1 at the leading edge, 80 plate cells growing by 1.05,
    40 upstream cells growing by 1.1, y growing by 1.1 to just past 50.  The printed
    profile stations 6.4381 and 21.5082 and the plate length 94.76 are then cell centres
    of the plate (cells 29, 50 and 79)."""
    for dy, ny in ((0.1, 42), (0.05, 49), (0.02, 58)):
        w = I.boundary_layer_paper(dy)
        assert (w.nx, w.ny) == (120, ny)
        assert w.yf[-1] > 50.0 and w.yf[-2] <= 50.0
        xc = 0.5 * (w.xf[1:] + w.xf[:-1])
        assert round(w.meta["stations"]["x1"], 4) == 6.4381
        assert round(w.meta["stations"]["x2"], 4) == 21.5082
        assert round(xc[40 + 79], 2) == 94.76
        assert min(np.diff(w.xf)) == pytest.approx(0.1) and w.xf[40] == 0.0
        assert w.meta["nu"] == pytest.approx(0.1 * 94.76 / 1e5)


def test_blasius_solution():
    """Blasius (1908): F''(0) = 0.33206 and, far from the wall, eta F' - F -> 1.7208."""
    eta, u, v, fpp0 = I.blasius()
    assert fpp0 == pytest.approx(0.332057, abs=2e-6)
    assert u[-1] == pytest.approx(1.0, abs=1e-9)
    assert v[-1] == pytest.approx(1.7208, abs=1e-4)
    # 99 % thickness near eta = 4.9
    assert eta[np.argmax(u >= 0.99)] == pytest.approx(4.91, abs=0.02)


def test_splitmix64_reference_values():
    """SplitMix64 with seed 0: the first outputs of the published generator."""
    g = I.SplitMix64(0)
    assert [g.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
