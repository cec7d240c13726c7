"""The seeded input generators (no scheme arithmetic) produce what their
docstrings promise: periodic data where the problem is periodic."""
import numpy as np
import pytest

from paper_2411_11229_amd import workloads as WL


@pytest.mark.parametrize("n,ny", [(70, 36), (64, 50), (48, 40), (96, 72), (61, 37), (128, 128)])
def test_smooth_2d_data_are_periodic(n, ny):
    """Across each periodic seam the data change no more than between
    neighbouring interior rows / columns (a seam jump would stand out), and
    the analytic derivatives match centred differences of the data."""
    w = WL.euler2d_smooth(n, seed=3101, ny=ny)
    for ax, D, h in ((-1, w.V, w.dx), (-2, w.W, w.dy)):
        inner = np.max(np.abs(np.diff(w.U, axis=ax)))
        seam = np.max(np.abs(np.take(w.U, 0, axis=ax) - np.take(w.U, -1, axis=ax)))
        assert seam <= 1.5 * inner, (ax, seam, inner)
        # 4th-order centred difference with periodic wrap ~ the exact derivative
        d = (8 * (np.roll(w.U, -1, ax) - np.roll(w.U, 1, ax))
             - (np.roll(w.U, -2, ax) - np.roll(w.U, 2, ax))) / (12 * h)
        assert np.max(np.abs(d - D)) <= 0.05 * np.max(np.abs(D)), ax
