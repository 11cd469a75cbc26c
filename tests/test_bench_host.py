"""Host-side logic of bench.py: the traffic record is keyed by the code that
sets the field kernel's traffic, so comments do not invalidate it, code
changes do, and a stale record reads as no measurement."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_only_drops_comments_and_blank_lines():
    a = "int x = 1;  // one\n\n/* block\n comment */\nint y = 2;\n"
    b = "int x = 1;\n// a different comment\nint y = 2;\n\n"
    assert bench._code_only(a) == bench._code_only(b) == "int x = 1;\nint y = 2;"
    assert bench._code_only(a) != bench._code_only(a.replace("2", "3"))



def test_traffic_is_reported_only_for_the_recorded_sources(monkeypatch):
    (key, rec), = [(k, v) for k, v in bench.MEASURED_TRAFFIC.items() if k[0] == "translation"]
    monkeypatch.setattr(bench, "_sources_sha", lambda algo: rec[0])
    assert bench._traffic(key[1], key[2], "translation") == rec[1]
    monkeypatch.setattr(bench, "_sources_sha", lambda algo: "0" * 40)
    assert bench._traffic(key[1], key[2], "translation") is None
    assert bench._traffic("no_such_workload", key[2], "translation") is None
