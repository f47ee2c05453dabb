"""Operator shapes for tiling (Appendix B): host logic only."""
from paper_2606_05297_amd import tiling
import workload as W


def test_ring_distance_shapes_are_translation_invariant():
    # on a ring of 5 the pairs (0, 1), (1, 2), ..., (0, 4) are all nearest neighbours
    nn = [("HR", i, (i + 1) % 5) for i in range(5)]
    nn = [(t, min(i, j), max(i, j)) for t, i, j in nn]
    assert {tiling.shape_of(op, 5) for op in nn} == {("HR", 1)}
    assert {tiling.shape_of(op) for op in nn} == {("HR", 1), ("HR", 4)}  # open chain: index distance
    assert tiling.shape_of(("PI", 0, 3), 5) == ("PI", 2) and tiling.shape_of(("SR", 2, -1), 5) == ("SR", None)


def test_tile_pool_keeps_order_and_learned_shapes():
    full = W.pool(5, "all", True, ("HR", "PR")) + W.site_ops(5, ("SR", "ROT"))
    shapes = {("HR", 1), ("PR", 2), ("SR", None)}
    tiled = tiling.tile_pool(full, shapes, 5)
    assert tiled == [op for op in full if op in tiled]  # pool order
    assert len(tiled) == 5 + 5 + 5
    assert all(tiling.shape_of(op, 5) in shapes for op in tiled)
