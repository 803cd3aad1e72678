"""Host-side pieces of the warm-start pipeline (CPU only)."""
import numpy as np

from oracle import cnn_oracle as co
from paper_1303_0625_amd import warmstart as ws


def test_init_params_layout_matches_the_network():
    p = ws.init_params(0)
    assert p.dtype == np.float32 and p.size == co.param_count(ws.CH)
    layers = co.unpack(p.astype(np.float64), ws.CH)
    for k, (W, b) in enumerate(layers):
        assert (b == 0).all()
        ci = W.shape[3]
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if k == len(layers) - 1 else 1.0)
        assert abs(W.std() / std - 1.0) < 0.2, k


def test_steady_time_picks_the_first_check_that_stays_within_tolerance():
    d_inf = [1.0, 2.0]
    hist = [(0.1, 100, [0.5, 2.0], [1e-3, 1e-3]), (0.2, 200, [0.99995, 2.1], [1e-7, 1e-4]),
            (0.3, 300, [1.00002, 2.00001], [1e-9, 1e-9]), (0.4, 400, [1.0, 2.0], [-1.0, 1e-12])]
    st = ws.steady_time(hist, d_inf)
    assert st[0] == (200, 0.2) and st[1] == (300, 0.3)
    assert ws.steady_time(hist[:2], [1.0, 3.0])[1] is None


def test_first_below_reads_the_residual_history():
    hist = [(0.1, 100, [0.5, 2.0], [1e-3, 1e-3]), (0.2, 200, [0.99995, 2.1], [1e-7, 1e-4]),
            (0.3, 300, [1.00002, 2.00001], [1e-9, 1e-9])]
    assert ws.first_below(hist, 0, 1e-8) == (300, 0.3)
    assert ws.first_below(hist, 1, 1e-3) == (200, 0.2)
    assert ws.first_below(hist, 1, 1e-10) is None
