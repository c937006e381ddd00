"""Device data checks of the index build (Sec. 3.4: trajectories are sorted
along time): a time that decreases within a trajectory gives TNN_E_UNSORTED,
a NaN or infinite coordinate TNN_E_NONFINITE; equal times and a time that
drops from one trajectory to the next are valid."""
import numpy as np
import pytest
import torch

from gpu_util import say
from paper_2112_10408_amd import capi, synth
from paper_2112_10408_amd import tnn as T

pytestmark = pytest.mark.gpu
K = 8


def _base():
    return synth.trajectories(6, 40, 200.0, 3600.0, seed=41)


def _build_status(ps):
    x, y, z, t = T.to_device(ps.x, ps.y, ps.z, ps.t)
    try:
        T.tnn_build_segments(x, y, z, t, ps.offsets, K, synth.SCALE)
    except capi.TnnError as e:
        return e.code
    finally:
        torch.cuda.synchronize()
    return capi.TNN_OK


def test_sorted_input_builds():
    assert _build_status(_base()) == capi.TNN_OK


def test_equal_times_and_drops_between_trajectories_are_valid():
    ps = _base()
    o = ps.offsets
    ps.t[o[2] + 3] = ps.t[o[2] + 2]                    # repeated timestamp
    ps.t[o[3]:o[4]] -= np.float32(3000.0)               # next trajectory starts earlier
    assert ps.t[o[3]] < ps.t[o[3] - 1]
    assert _build_status(ps) == capi.TNN_OK


@pytest.mark.parametrize("where", ["inside_a_segment", "across_a_segment_boundary",
                                   "last_point", "first_trajectory_start"])
def test_decreasing_time_is_rejected(where):
    ps = _base()
    o = ps.offsets
    if where == "inside_a_segment":
        i = o[1] + 3                                    # 4th point of a segment of 8
    elif where == "across_a_segment_boundary":
        i = o[1] + K                                    # first point of the 2nd segment
    elif where == "last_point":
        i = o[6] - 1
    else:
        i = 1
    ps.t[i] = ps.t[i - 1] - np.float32(1.0)
    say("unsorted", where, i)
    assert _build_status(ps) == capi.TNN_E_UNSORTED


@pytest.mark.parametrize("coord", ["x", "y", "z", "t"])
@pytest.mark.parametrize("value", [np.nan, np.inf, -np.inf])
def test_non_finite_coordinate_is_rejected(coord, value):
    ps = _base()
    i = int(ps.offsets[3] + 5)
    getattr(ps, coord)[i] = np.float32(value)
    say("non-finite", coord, value)
    assert _build_status(ps) == capi.TNN_E_NONFINITE
