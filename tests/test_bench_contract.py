"""Host-side contract of bench.py (no GPU): more than one GPU is refused with a
message before anything touches a device, and the query's HBM traffic is
reported only while the query sources hash to the committed counter summary."""
import importlib.util
import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_contract", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "error" in line and line["n_gpus"] == 2


def test_traffic_follows_the_query_sources(tmp_path):
    """A counter summary is used only while its recorded source hash matches
    the query sources; one changed byte turns the traffic off."""
    import hashlib
    b = _bench()
    for rel in ("paper_2511_07418_amd/csrc/query.hip", "paper_2511_07418_amd/csrc/lg_internal.h"):
        os.makedirs(tmp_path / os.path.dirname(rel), exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), tmp_path / rel)
    h = hashlib.sha256()
    for rel in ("paper_2511_07418_amd/csrc/query.hip", "paper_2511_07418_amd/csrc/lg_internal.h"):
        h.update((tmp_path / rel).read_bytes())
    os.makedirs(tmp_path / "profiles", exist_ok=True)
    (tmp_path / "profiles/k_query_c3_counters.md").write_text(
        f"HBM traffic per launch (bytes): 123456789\nsource sha256: {h.hexdigest()}\n")
    b.ROOT = str(tmp_path)
    assert b.query_traffic() == 123456789
    q = tmp_path / "paper_2511_07418_amd/csrc/query.hip"
    q.write_bytes(q.read_bytes() + b"\n")
    assert b.query_traffic() is None
