"""All-points and serving parity with the library's per-launch synchronisation off, as the
benchmark and a serving process run: the calls' launches are all queued at once, cached
workspace blocks move between streams behind events, and the serving slots' batches are in
flight on the device together (shown by their device-side spans).  The flag is read once per
process and this suite's process sets it, so the cases run in one child process."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_async_pipeline_matches_oracle():
    env = dict(os.environ)
    env.pop("RPF_SYNC_CHECK", None)
    print("[async] child process: tests/async_cases.py", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "async_cases.py")], env=env,
                       capture_output=True, text=True, timeout=600)
    print(r.stdout[-4000:], flush=True)
    print(r.stderr[-4000:], flush=True)
    assert r.returncode == 0 and "async cases ok" in r.stdout
