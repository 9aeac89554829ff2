"""The tiled whole-grid oracle gradient (tests/oracle_tiles.py) equals the
oracle's own whole-grid gradient on small grids: the partition of the sum
over samples, the pruning of primitives outside a tile's reach and the cut of
the z layers change nothing beyond FP64 rounding."""
import numpy as np
import pytest

from oracle import scene as S
from paper_2311_05646_amd import workloads as W
from tests.oracle_tiles import tiled_grad


@pytest.mark.parametrize("name,tile", [("c3_small", (16, 8)), ("c4_small", (10, 12)), ("psgc3_small", (8, 9)),
                                       ("taper3_sine_small", (13, 7))])
def test_tiled_equals_whole(name, tile):
    cfg = W.CONFIGS[name]()
    E, A = cfg["E"].astype(np.complex64), cfg["A"].astype(np.complex64)
    full = S.grad_analytic(cfg["scene"], cfg["p"], S.sensitivity(E, A, cfg["omega"]))
    got = tiled_grad(cfg["scene"], cfg["p"], E, A, cfg["omega"], tile=tile, workers=1)
    assert np.count_nonzero(full) > 0.8 * full.size
    assert np.linalg.norm(got - full) / np.linalg.norm(full) < 1e-13
