"""The order index of the collective study (Fig. 5C): the length of the
mean unit persistence direction over the cells whose direction is set."""
import numpy as np
import torch

from paper_2312_09317_amd import collective


class _Sim:
    def __init__(self, dirs):
        self.dirs = np.asarray(dirs, dtype=np.int32)

    def persistence(self):
        return torch.as_tensor(self.dirs)


def test_aligned_cells_have_order_one():
    d = np.zeros((11, 3), np.int32)
    d[1:] = (0, 16384, 0)
    d[5] = (0, 4000, 0)  # length does not matter, only the direction
    assert abs(collective.order_index(_Sim(d)) - 1.0) < 1e-12


def test_opposed_pairs_cancel_and_unset_cells_are_ignored():
    d = np.zeros((9, 3), np.int32)
    d[1], d[2] = (16384, 0, 0), (-16384, 0, 0)
    d[3], d[4] = (0, 0, 9000), (0, 0, -9000)
    # rows 5-8 (and the medium, row 0) have no direction yet
    assert collective.order_index(_Sim(d)) == 0.0


def test_random_directions_give_small_order():
    rng = np.random.default_rng(3)
    v = rng.normal(size=(20000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    d = np.zeros((20001, 3), np.int32)
    d[1:] = np.round(v * 16384).astype(np.int32)
    o = collective.order_index(_Sim(d))
    assert o < 5.0 / np.sqrt(20000)


def test_no_cell_with_a_direction():
    assert collective.order_index(_Sim(np.zeros((4, 3), np.int32))) == 0.0
