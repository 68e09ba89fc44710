"""The parity measures themselves (CPU): a single wrong, dropped or swapped
16-point tile is invisible in the whole-vector relative error at the
workload's size but of order one in the per-tile measure."""
import numpy as np

from tests.parity import rel, tile_err


def _noisy(ref, eps, rng):
    return ref * (1.0 + eps * rng.standard_normal(ref.shape))


def test_one_bad_tile_is_seen_per_tile_not_globally():
    rng = np.random.default_rng(0)
    N = 65536
    ref = rng.standard_normal((3, N))
    got = _noisy(ref, 5e-3, rng)  # BF16-like noise everywhere
    assert tile_err(got, ref) < 0.1
    bad = got.copy()
    bad[:, 16 * 100:16 * 101] = ref[:, 16 * 200:16 * 201]  # one tile holds another tile's values
    assert rel(bad, ref) < 3e-2  # of the order of a 16-bit whole-vector bar
    assert tile_err(bad, ref) > 0.9
    dropped = got.copy()
    dropped[:, 16 * 7:16 * 8] = 0.0
    assert tile_err(dropped, ref) > 0.5


def test_channels_are_measured_separately():
    rng = np.random.default_rng(1)
    N = 4096
    ref = rng.standard_normal((2, 3, N)) * np.array([1.0, 1e3, 1e-3])[None, :, None]
    got = ref.copy()
    got[:, 2, 16 * 5:16 * 6] *= -1.0  # wrong sign on one tile of the smallest channel
    assert rel(got, ref) < 1e-6
    assert tile_err(got, ref) > 1.0


def test_ragged_tail_and_exact_match():
    rng = np.random.default_rng(2)
    ref = rng.standard_normal((1, 1000))
    assert tile_err(ref, ref) == 0.0
    got = ref.copy()
    got[0, 995:] += 10.0  # the 8-point tail tile
    assert tile_err(got, ref) > 1.0
