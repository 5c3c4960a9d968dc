"""The persistent sweep-shape cache: the shipped file's format (CPU) and a
choice measured in one process found, not measured again, in the next (GPU,
two child processes sharing one PAMC_TUNE_CACHE file)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIPPED = os.path.join(ROOT, "paper_1710_09025_amd", "tune_cache.jsonl")
FIELDS = ["device", "variant", "dim", "L", "sweeps", "cap_log2", "packed", "tile_rows", "group_quads",
          "ns_per_attempt"]


def test_shipped_cache_lines_are_complete_choices():
    if not os.path.exists(SHIPPED):
        pytest.skip("no tuning cache shipped beside the library")
    keys = set()
    with open(SHIPPED) as f:
        lines = [line for line in f if line.strip()]
    assert lines
    for line in lines:
        d = json.loads(line)
        assert list(d) == FIELDS  # the library reads the fields in this order
        assert d["device"].startswith("gfx950")
        assert d["dim"] in (2, 3) and 2 <= d["L"] <= 64 and d["sweeps"] >= 1
        assert d["tile_rows"] >= 1 and d["group_quads"] >= 0 and d["ns_per_attempt"] > 0
        key = (d["device"], d["variant"], d["dim"], d["L"], d["sweeps"], d["cap_log2"], d["packed"])
        assert key not in keys, key
        keys.add(key)


CHILD = """
import json, sys
sys.path.insert(0, {root!r})
from paper_1710_09025_amd import autotune
print(json.dumps(autotune(7, 3000, 3, torch_stream=False)), flush=True)
"""


@pytest.mark.gpu
def test_tuned_choice_persists_across_processes(tmp_path):
    path = tmp_path / "cache.jsonl"
    env = dict(os.environ, PAMC_TUNE_CACHE=str(path))
    code = CHILD.format(root=ROOT)

    def child():
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    # L = 7 with three sweeps per step is in no shipped file: measured here
    tr1, gr1, ns1 = child()
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    d = json.loads(lines[0])
    assert (d["L"], d["sweeps"], d["tile_rows"], 4 * d["group_quads"]) == (7, 3, tr1, gr1)
    # the second process takes the stored choice (its figure is the file's,
    # six decimals) and appends nothing
    tr2, gr2, ns2 = child()
    assert (tr2, gr2) == (tr1, gr1)
    assert ns2 == d["ns_per_attempt"]
    assert len(path.read_text().splitlines()) == 1
