"""The load-balance diagnostic (CPU only): its summary of per-wave records,
and which build exports its entry point."""
import ctypes
import os
import re

import numpy as np

from paper_2507_15121_amd import api, build, queue_balance

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_summary_of_synthetic_records():
    # 2 workgroups x 2 waves: [chunks, nonzeros, first pop, exit]
    rec = np.array([[3, 300, 100, 400], [1, 100, 110, 300],
                    [2, 250, 100, 500], [0, 0, 0, 120]], dtype=np.uint64)
    s = queue_balance.summarize(rec, 2, 1e6)
    assert s["blocks"] == 2 and s["chunks"] == (2, 3.0, 4) and s["nnz"] == (250, 325.0, 400)
    # the launch spans first pop 100 .. last exit 500; a wave with no chunk
    # does not count as a start
    assert abs(s["span_us"] - 400.0) < 1e-9
    assert abs(s["exit_spread"] - 100 / 400) < 1e-12
    assert abs(s["start_spread"] - 0.0) < 1e-12
    assert abs(s["busy_spread"] - 100 / 400) < 1e-12
    assert abs(s["idle_share"] - (1 - (300 + 400) / 800)) < 1e-12


def test_diagnostic_entry_point_only_in_the_diagnostic_build():
    text = open(os.path.join(ROOT, "include", "amped_diag.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    decl = sorted(set(re.findall(r"\b(amped_[a-z0-9_]+)\s*\(", text)))
    assert decl == ["amped_queue_stats"]
    assert not hasattr(api.lib(), "amped_queue_stats")
    if os.path.exists(build.QSTATS_LIB):
        L = ctypes.CDLL(build.QSTATS_LIB)
        for name in decl + api.EXPORTED:
            assert hasattr(L, name), name
