"""Host-side pieces of bench.py (no GPU): the one-GPU guard and the traffic
record computed from rocprofv3 counter CSVs."""
import importlib.util
import json
import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_record_scaling(tmp_path, monkeypatch):
    b = _bench()
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(b, "PROFILE_TRAFFIC", str(out))
    hdr = "Kernel_Name,Counter_Name,Counter_Value\n"
    # k_batch reads 1000 KiB and writes 300 KiB per launch; the 1 GiB copy reads as 512 Ki / 1 Mi KiB
    (tmp_path / "f.csv").write_text(hdr + "void k_batch<float>,FETCH_SIZE,900\nvoid k_batch<float>,FETCH_SIZE,1100\n"
                                    "__amd_rocclr_copyBuffer,FETCH_SIZE,524288\n")
    (tmp_path / "w.csv").write_text(hdr + "void k_batch<float>,WRITE_SIZE,300\ncopyBuffer,WRITE_SIZE,1048576\n")
    args = types.SimpleNamespace(config=2, dtype="f32", mode="fixed")
    b.write_traffic(args, str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    rec = json.loads(out.read_text())
    assert rec["factor_fetch"] == 2.0 and rec["factor_write"] == 1.0
    assert rec["bytes_per_launch"] == int(1000 * 1024 * 2.0 + 300 * 1024 * 1.0)
    assert rec["kernel_hash"] == b.kernel_source_hash()
