"""The debug library (every source compiled with VR_DEBUG_BOUNDS) checks the
index range of every direct gather and every LDS voxel-box read; run over
every kernel family (single pass on all paths, object order, bricks with and
without LDS boxes, batch, adjoint, depth), on orbit views and an eye inside
the cube, it counts no violation.  The kernels run in a process of their own
that loads the debug library."""
import json
import os
import subprocess
import sys

import pytest

from tests.gpu_util import log

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_no_index_range_violations():
    from paper_1012_2909_amd import build
    if not os.path.exists(build.LIB_DEBUG):
        pytest.fail(f"{build.LIB_DEBUG} is missing: run __graft_entry__.build() first")
    log("case: debug library, every kernel family")
    env = dict(os.environ, VRCUBE_LIB=build.LIB_DEBUG)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "debug_bounds_run.py")], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    line = [x for x in r.stdout.splitlines() if x.startswith("{")][-1]
    res = json.loads(line)
    log(f"debug bounds: {res}")
    assert res["lib"] == os.path.basename(build.LIB_DEBUG)
    assert res["violations"] and all(v == 0 for v in res["violations"].values()), res


def test_release_library_has_no_checks():
    """The release library reports the checks as unsupported."""
    from paper_1012_2909_amd import vr
    R = vr.Renderer(0)
    try:
        with pytest.raises(vr.VRError) as e:
            R.debug_bounds_violations()
        assert e.value.code == -5
    finally:
        R.close()
