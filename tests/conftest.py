import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_sessionfinish(session, exitstatus):
    """Writes the argmax agreement of every GPU comparison of the session, if any,
    to gpurun_out/argmax_agreement.json (the GPU runs' output folder)."""
    try:
        from tests import refpath
    except Exception:
        return
    if not refpath.ARGMAX_LOG:
        return
    out = os.path.join(ROOT, "gpurun_out")
    try:
        import json
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "argmax_agreement.json"), "w") as f:
            json.dump([{"label": l, "identical": s, "frames": n} for l, s, n in
                       refpath.ARGMAX_LOG], f, indent=0)
    except OSError:
        pass
