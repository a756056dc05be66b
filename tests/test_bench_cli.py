"""bench.py's host-side contract, checked without a GPU: more than one GPU
is refused with a message and exit status 2 before anything touches a
device, and every workload the help lists is one the script dispatches."""

import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_every_listed_workload_is_dispatched():
    src = open(os.path.join(ROOT, "bench.py")).read()
    listed = re.search(r'"--workload", default="room", choices=\[([^\]]*)\]', src).group(1)
    names = re.findall(r'"(\w+)"', listed)
    assert {"room", "rgb", "devox", "batched", "diff", "precision"} <= set(names)
    for n in names:
        assert re.search(r'"%s": run_%s\b' % (n, n), src), n
