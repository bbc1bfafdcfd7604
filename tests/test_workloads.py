"""The seeded input generators: node counts, order and layouts."""
import numpy as np

import workloads as W


def test_node_counts():
    assert len(W.interface_nodes(2, 1, 32)) == 31
    assert len(W.interface_nodes(4, 4, 256)) == 1521
    assert len(W.interface_nodes(8, 8, 768)) == 10689
    assert len(W.STATIC_BUMP_31.nodes()) == 31 and len(W.MOVING_BUMP_1521.nodes()) == 1521


def test_canonical_order_and_uniqueness():
    p = W.interface_nodes(4, 4, 256)
    assert len({(round(a * 256), round(b * 256)) for a, b in p}) == len(p)
    assert np.all((p > 0) & (p < 1))
    # vertical lines first, ascending y on each
    assert np.all(p[:255, 0] == 0.25) and np.all(np.diff(p[:255, 1]) > 0)
    assert np.all(p[765:, 1] == 0.25) or p[765, 1] == 0.25


def test_layouts_are_seeded():
    a = W.random_layouts(64)
    assert a == W.random_layouts(64)
    assert all(2 <= px <= 8 and 2 <= py <= 8 for px, py in a)
    lv = W.batched_levels(64)
    sizes = [len(n) for _, _, _, n in lv]
    assert min(sizes) >= 253 and max(sizes) <= 1729
    assert [round(t, 10) for t, *_ in lv[:3]] == [0.01, 0.02, 0.03]
