"""The checked build (libsf_checked.so: the kernels' index checks compiled in,
recording instead of trapping) on the library's data-dependent paths: no check
fails, the self-test shows that a failing check is recorded, and every output
equals the normal library's."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECKED = os.path.join(ROOT, "paper_1801_04720_amd", "libsf_checked.so")
NORMAL = os.path.join(ROOT, "paper_1801_04720_amd", "libsf.so")


def run_with(lib, out):
    env = dict(os.environ, SF_LIB_PATH=lib)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "checked_run.py"), out],
                       capture_output=True, text=True, env=env, timeout=280)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_checked_build_records_nothing_and_matches(tmp_path):
    if not os.path.exists(CHECKED):
        pytest.fail("libsf_checked.so is not built (run __graft_entry__.build())")
    print("checked library run", flush=True)
    rc = run_with(CHECKED, str(tmp_path / "checked.npz"))
    print(rc, flush=True)
    assert rc["checked"] == 1
    assert rc["before"] == 0
    assert rc["selftest"] == 1 << 31 and rc["after_clear"] == 0
    assert rc["workloads"] == 0, f"index checks failed at sites {rc['workloads']:#x}"
    print("normal library run", flush=True)
    rn = run_with(NORMAL, str(tmp_path / "normal.npz"))
    assert rn["checked"] == 0 and rn["selftest"] == 0 and rn["workloads"] == 0
    with np.load(str(tmp_path / "checked.npz")) as a, np.load(str(tmp_path / "normal.npz")) as b:
        assert sorted(a.files) == sorted(b.files)
        for k in a.files:
            assert np.array_equal(a[k], b[k], equal_nan=True), k
