"""CPU checks of bench.py's command line: more than one GPU is refused with a
message before anything touches a GPU, and the counter summary it reads is
keyed to the kernel sources it was taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_summary_names_its_source_hash():
    """The committed FETCH_SIZE / WRITE_SIZE summary records the hash of the
    kernel sources it was taken on; bench.py reports its traffic only while
    the sources still hash to that value."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    with open(b.TRAFFIC_FILE) as fh:
        d = json.load(fh)
    for k in ("k_predictor<7", "k_corrector<7"):
        assert d[k]["traffic_bytes"] > d[k]["algorithmic_bytes"] * 0.9
    got = b.measured_traffic("k_predictor<7")
    if d["source_hash"] == b.kernel_source_hash():
        assert got == d["k_predictor<7"]["traffic_bytes"]
    else:
        assert got is None
