"""The bounds-checked build (liblpgpu_checked.so): the same solves in a process that loads it
(every entry point returned without a check failure, the device check word is 0 at the end)
give, bit for bit, the points of the plain build, which this process loads."""
import os
import subprocess
import sys

import numpy as np
import pytest

import paper_2604_23951_amd as lpg

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_checked_build_runs_clean_and_equals_plain(tmp_path):
    lib = os.path.join(ROOT, "paper_2604_23951_amd", "_lib", "liblpgpu_checked.so")
    if not os.path.exists(lib):
        pytest.skip("checked build not compiled (run __graft_entry__.build())")
    out = tmp_path / "checked.npz"
    env = dict(os.environ, LPGPU_CHECKED="1", PYTHONPATH=os.pathsep.join([ROOT, HERE]))
    env.pop("LPGPU_LIB_OVERRIDE", None)
    print("checked build: child process", flush=True)
    r = subprocess.run([sys.executable, os.path.join(HERE, "checked_child.py"), str(out)], env=env,
                       capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    got = np.load(out)
    assert int(got["checked"]) == 1 and int(got["word"]) == 0
    sys.path.insert(0, HERE)
    import checked_child

    word, checked = lpg.lp_check_word(0)
    assert (word, checked) == (0, False)
    ref = checked_child.solves()
    assert len(ref) == len(got.files) - 2
    for name, x in ref:
        np.testing.assert_array_equal(got[name], x, err_msg=name)
