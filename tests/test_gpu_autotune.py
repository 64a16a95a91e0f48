"""An autotuner (timing the FP32 factorisation shape threshold and the
sharing of large subsets per problem, with a cache file of choices) was
built and taken out again: its first two GPU runs ended in host
segmentation faults inside the tuning call, on the third problem tuned in
the process each time, and the cause was not found.  These tests stay as
the record of that case and are skipped; the library keeps its measured
default launch configuration."""
import pytest

pytestmark = pytest.mark.gpu

REASON = ("autotuner taken out: host segmentation faults inside the tuning call on its first two GPU "
          "runs, cause not found")


@pytest.mark.skip(reason=REASON)
def test_autotune_mixed_candidates_agree_and_cache():
    pass


@pytest.mark.skip(reason=REASON)
def test_autotune_fp64_candidates():
    pass
