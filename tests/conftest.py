import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Measured errors of the parity checks of this session, with their gates
# (written out at the end of the session, so the margins survive a quiet run).
_MARGINS = []


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture
def margin(request):
    """check(what, err, bound): assert err < bound and record both.

    The records go to $LGT_MARGINS_FILE, else parity_margins.json at the
    repository root (not tracked), at the end of the session."""
    def check(what, err, bound):
        err = float(err)
        _MARGINS.append({"test": request.node.nodeid, "what": what, "err": err, "gate": float(bound),
                         "ratio": err / float(bound), "pass": bool(err < bound)})
        print(f"margin {request.node.nodeid} {what}: {err:.3e} (gate {bound:.0e})", file=sys.stderr, flush=True)
        assert err < bound, f"{what}: {err:.3e} is not below {bound:.1e}"
    return check


def pytest_sessionfinish(session, exitstatus):
    if not _MARGINS:
        return
    path = os.environ.get("LGT_MARGINS_FILE") or os.path.join(ROOT, "parity_margins.json")
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        worst = max(_MARGINS, key=lambda m: m["ratio"])
        with open(path, "w") as f:
            json.dump({"checks": len(_MARGINS), "worst": worst, "margins": _MARGINS}, f, indent=1)
    except OSError as e:
        print(f"could not write the parity margins to {path}: {e}", file=sys.stderr)
