"""Pins the branching rules of the branch-and-bound loops on hand examples:
the ReLU split takes the best-scoring unsplit unstable neuron, the children
carry the parent's splits plus one branch each, and the input split halves
the dimension with the largest width times plane weight."""
import numpy as np

from oracle import bab


def test_relu_branch_and_children():
    l = np.array([[-1.0, -2.0, 0.5, -1.0], [1.0, 1.0, 1.0, 1.0]])
    u = np.array([[1.0, 2.0, 1.0, 3.0], [2.0, 2.0, 2.0, 2.0]])
    w = np.array([1.0, 1.0, 5.0, 1.0])
    # scores row 0: 0.5, 1.0, 0 (stable), 0.75; neuron 1 is already split
    neuron = np.array([[1, 0], [0, 0]])
    sign = np.array([[1, 0], [0, 0]], np.int8)
    count = np.array([1, 0])
    ch = bab.branch_relu(l, u, w, neuron, sign, count)
    assert ch.tolist() == [3, -1]            # row 1: nothing unstable
    lo = np.zeros((2, 3))
    hi = np.ones((2, 3))
    n2, s2, c2, lo2, hi2 = bab.children_relu(neuron, sign, count, lo, hi, ch)
    assert n2.shape == (4, 3) and c2.tolist() == [2, 2, 0, 0]
    assert n2[0, :2].tolist() == [1, 3] and s2[0, :2].tolist() == [1, -1]
    assert n2[1, :2].tolist() == [1, 3] and s2[1, :2].tolist() == [1, 1]
    assert np.array_equal(lo2, np.zeros((4, 3)))


def test_relu_branch_ties_go_to_lower_index():
    l = np.array([[-1.0, -1.0, -1.0]])
    u = np.array([[1.0, 1.0, 1.0]])
    ch = bab.branch_relu(l, u, np.array([2.0, 3.0, 3.0]), np.zeros((1, 1), int),
                         np.zeros((1, 1), np.int8), np.array([0]))
    assert ch.tolist() == [1]


def test_input_branch_and_children_cover_the_parent():
    lo = np.array([[0.0, 0.0, -1.0]], np.float32)
    hi = np.array([[1.0, 0.5, 1.0]], np.float32)
    A = np.array([[[1.0, 4.0, 0.5], [-1.0, 0.0, 0.25]]])
    # (hi - lo) * sum |A|: 2, 2, 1.5 -> dimension 0 (tie with 1, lower index)
    d = bab.branch_input(lo, hi, A)
    assert d.tolist() == [0]
    lo2, hi2 = bab.children_input(lo, hi, d)
    assert hi2[0, 0] == 0.5 and lo2[1, 0] == 0.5
    assert np.array_equal(lo2[0], lo[0]) and np.array_equal(hi2[1], hi[0])
    assert np.array_equal(lo2[:, 1:], np.repeat(lo[:, 1:], 2, 0))
