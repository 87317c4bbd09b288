import json
import math
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs through the C-ABI")
    config.addinivalue_line("markers", "slow: long-running test (large inputs)")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; fails loudly if not built."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    import paper_2106_03219_amd as omprt
    omprt.load()          # raises if libomprt.so is missing
    return omprt


def pytest_terminal_summary(terminalreporter):
    """Per-result error report of the floating sums the GPU tests checked: the worst
    relative error against the oracle per test, with its kappa."""
    mod = sys.modules.get("gpu_util")
    errs = getattr(mod, "ERRORS", None) if mod else None
    if not errs:
        return
    worst = {}
    for e in errs:
        w = worst.get(e["test"])
        if w is None or e["rel"] > w["rel"]:
            worst[e["test"]] = e
    tr = terminalreporter
    tr.write_sep("-", f"floating sums vs the FP64 oracle: {len(errs)} results, worst per test")
    for t, e in sorted(worst.items(), key=lambda kv: -kv[1]["rel"]):
        k = "inf" if math.isinf(e["kappa"]) else f"{e['kappa']:.3g}"
        tr.write_line(f"rel {e['rel']:.3e}  kappa {k:>9}  {e['dtype']:>4}  {t}  {e['what']}")
    path = os.environ.get("OMPRT_ERROR_REPORT")
    if path:
        with open(path, "w") as fh:
            json.dump([{**e, "kappa": None if math.isinf(e["kappa"]) else e["kappa"]}
                       for e in errs], fh)
