"""Host-side comparison helpers used to report the FP32 density variant."""
import numpy as np

from paper_1001_3411_amd.report import group_change_fraction, max_rel_error


def test_identical_labellings_do_not_change():
    a = np.array([0, 0, 1, -1, 2, 2])
    assert group_change_fraction(a, a) == 0.0


def test_relabelled_groups_do_not_change():
    a = np.array([0, 0, 1, 1, -1, 2])
    b = np.array([7, 7, 3, 3, -1, 0])
    assert group_change_fraction(a, b) == 0.0


def test_merged_and_dropped_groups_change():
    # groups 0 and 1 merge: the smaller side (group 1, 2 particles) changed;
    # group 2 vanished (1 particle); a -1 particle joined a group (1)
    a = np.array([0, 0, 0, 1, 1, 2, -1, -1])
    b = np.array([4, 4, 4, 4, 4, -1, 4, -1])
    assert group_change_fraction(a, b) == 4 / 8


def test_split_group_changes_the_minority():
    a = np.array([0, 0, 0, 0, 0])
    b = np.array([1, 1, 1, 2, 2])
    assert group_change_fraction(a, b) == 2 / 5


def test_max_rel_error():
    ref = np.array([1.0, 2.0, 0.0, 4.0])
    val = np.array([1.0, 2.002, 5.0, 3.996])
    assert abs(max_rel_error(ref, val) - 1e-3) < 1e-12
