"""Host side of the horizon runs: the fragment count of a periodic field."""
import numpy as np

from paper_2407_12263_amd.runs import _crossing, fragments


def _ball(shape, c, r):
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    d = [x - c[0], y - c[1], z - c[2]]
    n = [shape[2], shape[1], shape[0]]
    d = [a - n_ * np.round(a / n_) for a, n_ in zip(d, n)]
    return (d[0] ** 2 + d[1] ** 2 + d[2] ** 2 <= r * r).astype(float)


def test_fragments_counts_separate_balls():
    shape = (32, 32, 32)
    phi = np.maximum(_ball(shape, (8, 8, 8), 3), _ball(shape, (24, 20, 16), 4))
    assert fragments(phi) == 2
    assert fragments(np.zeros(shape)) == 0


def test_fragments_joins_across_periodic_faces():
    shape = (16, 16, 16)
    phi = _ball(shape, (0, 8, 8), 3)          # cut in two by the x faces
    assert fragments(phi) == 1
    assert fragments(phi, periodic=(False, True, True)) == 2
    phi = _ball(shape, (0, 0, 0), 3)          # split over all eight corners
    assert fragments(phi) == 1
    assert fragments(phi, periodic=(False, False, False)) == 8


def test_fragments_diagonal_contact_is_not_a_connection():
    phi = np.zeros((4, 4, 4))
    phi[1, 1, 1] = phi[2, 2, 2] = 1.0
    assert fragments(phi, periodic=(False, False, False)) == 2


def test_front_crossings():
    y = np.arange(64, dtype=float)
    col = 0.5 * (1 + np.tanh(2 * (y - 40.3) / 4))   # heavy above 40.3
    assert abs(_crossing(col, True) - 40.3) < 0.05
    assert abs(_crossing(col, False) - 40.3) < 0.05
    assert np.isnan(_crossing(np.ones(8), True))


def test_fragment_sizes_count_nodes_across_faces():
    from paper_2407_12263_amd.runs import fragment_sizes
    phi = np.zeros((8, 8, 8))
    phi[0, 0, 0] = phi[0, 0, 7] = 1.0          # one fragment of 2 nodes across x
    phi[4, 4, 3:6] = 1.0                         # one of 3
    assert fragment_sizes(phi).tolist() == [3, 2]
    assert fragment_sizes(phi, periodic=(False, True, True)).tolist() == [3, 1, 1]
