"""Factorisation shapes follow the schedule groups: without tuning, a
problem whose first group (the 256 largest subsets) takes 8-wave
work-groups and whose remainder group lies below the shape threshold gives
the same bits in pcv_eval, pcv_eval_batch and a served evaluation."""
import sys

import numpy as np
import pytest

from paper_1912_13132_amd import pcv
from parity_util import mixed_size_subsets

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def datas():
    return [mixed_size_subsets(1)]


def test_default_shapes_follow_schedule_groups(datas):
    """Without tuning: the first schedule group (256 largest subsets) takes
    8-wave work-groups, the remainder (all below the shape threshold) 4-wave
    ones.  The multi-theta launches and a served evaluation (launches of one
    work-group per compute unit) factor every subset with its group's shape,
    so all three agree bit for bit."""
    ths = [pcv.theta(0.4, 0.1), pcv.theta(0.3, 0.15)]
    say("[case] default shapes per schedule group: eval, eval_batch, served")
    with pcv.Problem(*datas[0], prec="mixed") as P:
        single = [P.eval(t) for t in ths]
        np.testing.assert_array_equal(P.eval_batch(ths), single)
        P.factor(ths[0])
        with pcv.Server(P) as srv:
            served = [srv.wait(srv.submit_eval(t)) for t in ths]
    assert served == single
